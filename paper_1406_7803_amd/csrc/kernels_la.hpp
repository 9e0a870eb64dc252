// Band-solver kernels: Gram matrices, the FP64 Rayleigh-Ritz solve
// (Cholesky with column dropping, reduction, Jacobi eigensolver), rotations,
// residual + Teter-Payne-Allan preconditioner, occupations.
#pragma once

#include "common.hpp"

namespace fde {

constexpr int kLBlk = 256;
constexpr double kInactiveDiag = 1.0e6;

// ---------------------------------------------------------------------------
// Gram partials: part[chunk][0][i][j] = sum_{G in chunk} conj(V_i) V_j,
//                part[chunk][1][i][j] = sum_{G in chunk} conj(V_i) HV_j.
// grid (nchunk, ceil(m/TI), ceil(m/TI)); chunk = 2048 plane waves.
// ---------------------------------------------------------------------------
template <typename T>
struct KGram {
  static constexpr int CH = 2048, TG = 32, TI = 32;
  static size_t lds_bytes() { return sizeof(cplx<T>) * 3 * TI * TG + sizeof(cplx<double>) * 2 * TI * TI; }
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const cplx<T>* __restrict__ v, const cplx<T>* __restrict__ hv,
                         int npw, int m, cplx<double>* __restrict__ part) {
    const int g0 = c.bx() * CH;
    const int i0 = c.by() * TI, j0 = c.bz() * TI;
    cplx<T>* sA = (cplx<T>*)lds;   // V_i   [TI][TG]
    cplx<T>* sB = sA + TI * TG;    // V_j   [TI][TG]
    cplx<T>* sH = sB + TI * TG;    // HV_j  [TI][TG]
    cplx<double>* accS = (cplx<double>*)(sH + TI * TG);
    cplx<double>* accA = accS + TI * TI;
    for (int o = c.tid(); o < TI * TI; o += c.nthr()) {
      accS[o] = mk<double>(0, 0);
      accA[o] = mk<double>(0, 0);
    }
    const int gend = (g0 + CH) < npw ? (g0 + CH) : npw;
    for (int gs = g0; gs < gend; gs += TG) {
      for (int idx = c.tid(); idx < TI * TG; idx += c.nthr()) {
        const int r = idx / TG, g = gs + (idx - r * TG);
        const bool gi = g < gend;
        sA[idx] = (i0 + r < m && gi) ? v[(size_t)(i0 + r) * npw + g] : mk<T>(0, 0);
        sB[idx] = (j0 + r < m && gi) ? v[(size_t)(j0 + r) * npw + g] : mk<T>(0, 0);
        sH[idx] = (j0 + r < m && gi) ? hv[(size_t)(j0 + r) * npw + g] : mk<T>(0, 0);
      }
      c.sync();
      for (int o = c.tid(); o < TI * TI; o += c.nthr()) {
        const int i = o / TI, j = o - i * TI;
        double sx = 0, sy = 0, ax = 0, ay = 0;
        for (int g = 0; g < TG; ++g) {
          const cplx<T> a = sA[i * TG + g];
          const cplx<T> b = sB[j * TG + g];
          const cplx<T> h = sH[j * TG + g];
          sx += (double)a.x * b.x + (double)a.y * b.y;
          sy += (double)a.x * b.y - (double)a.y * b.x;
          ax += (double)a.x * h.x + (double)a.y * h.y;
          ay += (double)a.x * h.y - (double)a.y * h.x;
        }
        accS[o].x += sx;
        accS[o].y += sy;
        accA[o].x += ax;
        accA[o].y += ay;
      }
      c.sync();
    }
    const size_t mm = (size_t)m * m;
    for (int o = c.tid(); o < TI * TI; o += c.nthr()) {
      const int i = o / TI, j = o - i * TI;
      if (i0 + i < m && j0 + j < m) {
        const size_t e = (size_t)(i0 + i) * m + j0 + j;
        part[(size_t)c.bx() * 2 * mm + e] = accS[o];
        part[(size_t)c.bx() * 2 * mm + mm + e] = accA[o];
      }
    }
  }
};

// S, A = sum over chunks (fixed order). grid ceil(2*m*m/256)
struct KGramReduce {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const cplx<double>* __restrict__ part, int nchunk, int m,
                         cplx<double>* __restrict__ S, cplx<double>* __restrict__ A) {
    const size_t mm = (size_t)m * m;
    for (int l = c.tid(); l < kLBlk; l += c.nthr()) {
      const size_t o = (size_t)c.bx() * kLBlk + l;
      if (o >= 2 * mm) break;
      double sx = 0, sy = 0;
      for (int k = 0; k < nchunk; ++k) {
        const cplx<double> v = part[(size_t)k * 2 * mm + o];
        sx += v.x;
        sy += v.y;
      }
      if (o < mm) S[o] = mk<double>(sx, sy);
      else A[o - mm] = mk<double>(sx, sy);
    }
  }
};

// ---------------------------------------------------------------------------
// Single-workgroup FP64 Rayleigh-Ritz solve. Matrices row-major [i][j] in
// global memory (L2 resident at these sizes). Uses LDS for: reduction scratch
// (17 doubles), rotation parameters (3*mp/2 + 2 doubles), flags.
//   In:  S, A (overwritten), active[m] (nullable), nb, drop_tol
//   Out: eval[nb], Cd[m][nb] (FP64), Ct[m][nb] (plan precision), info
// ---------------------------------------------------------------------------
struct RRArgs {
  cplx<double>*S, *A, *L, *B, *W;
  const uint8_t* active;
  int m, nb;
  double drop_tol;
  double* eval;
  cplx<double>* Cd;
  void* Ct;
  int ct_double;
  int* info;
  int* order;      // [m] scratch
  double* theta;   // [m] scratch
  int* masked;     // [m] scratch
};

FDE_HD cplx<double> cdiv_real(cplx<double> a, double d) { return mk<double>(a.x / d, a.y / d); }

struct KRRSolve {
  static size_t lds_bytes(int m) { return sizeof(double) * (32 + 4 * ((m + 2) / 2 + 1)); }

  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, RRArgs a) {
    double* red = (double*)lds;            // 17 used
    double* rot = red + 32;                // [4][mp/2]
    const int m = a.m, nb = a.nb;
    const int tid = c.tid(), nt = c.nthr();
    cplx<double>*S = a.S, *A = a.A, *L = a.L, *B = a.B, *W = a.W;
    if (tid == 0) a.info[0] = 0;
    // ---- masks
    for (int j = tid; j < m; j += nt) a.masked[j] = (a.active && !a.active[j]) ? 1 : 0;
    c.sync();
    for (int e = tid; e < m * m; e += nt) {
      const int i = e / m, j = e - i * m;
      if (a.masked[i] || a.masked[j]) {
        S[e] = mk<double>(i == j ? 1.0 : 0.0, 0.0);
        A[e] = mk<double>(i == j ? kInactiveDiag : 0.0, 0.0);
      }
      L[e] = mk<double>(0, 0);
    }
    c.sync();
    // ---- Cholesky, column by column, dropping near-dependent columns j >= nb
    for (int j = 0; j < m; ++j) {
      double part = 0.0;
      for (int k = tid; k < j; k += nt) part += norm2(L[(size_t)j * m + k]);
      const double sjj = S[(size_t)j * m + j].x;
      const double d = sjj - c.sum(part, red);
      const bool drop = (j >= nb) && !(d >= a.drop_tol * sjj);
      if (drop) {
        for (int k = tid; k < j; k += nt) L[(size_t)j * m + k] = mk<double>(0, 0);
        for (int i = tid; i < m; i += nt) {
          if (i != j) {
            A[(size_t)i * m + j] = mk<double>(0, 0);
            A[(size_t)j * m + i] = mk<double>(0, 0);
          }
        }
        if (tid == 0) {
          L[(size_t)j * m + j] = mk<double>(1.0, 0.0);
          A[(size_t)j * m + j] = mk<double>(kInactiveDiag, 0.0);
          a.masked[j] = 1;
        }
        c.sync();
        continue;
      }
      if (!(d > 0.0)) {
        // not positive definite: report, and leave X = the first nb columns of V
        if (tid == 0) a.info[0] = j + 1;
        for (int e = tid; e < m * nb; e += nt) {
          const int i = e / nb, n = e - i * nb;
          const cplx<double> v = mk<double>(i == n ? 1.0 : 0.0, 0.0);
          a.Cd[e] = v;
          if (a.ct_double) ((cplx<double>*)a.Ct)[e] = v;
          else ((cplx<float>*)a.Ct)[e] = mk<float>((float)v.x, 0.0f);
        }
        for (int n = tid; n < nb; n += nt) a.eval[n] = 0.0 / 0.0;
        c.sync();
        return;  // uniform: every thread saw the same d
      }
      const double ljj = sqrt(d);
      if (tid == 0) L[(size_t)j * m + j] = mk<double>(ljj, 0.0);
      for (int i = j + 1 + tid; i < m; i += nt) {
        cplx<double> acc = S[(size_t)i * m + j];
        for (int k = 0; k < j; ++k) {
          const cplx<double> lik = L[(size_t)i * m + k], ljk = L[(size_t)j * m + k];
          // acc -= L_ik conj(L_jk)
          acc.x -= lik.x * ljk.x + lik.y * ljk.y;
          acc.y -= lik.y * ljk.x - lik.x * ljk.y;
        }
        L[(size_t)i * m + j] = cdiv_real(acc, ljj);
      }
      c.sync();
    }
    // ---- B = L^{-1} A (column per thread), then A~ = L^{-1} B^H into A
    for (int col = tid; col < m; col += nt) {
      for (int i = 0; i < m; ++i) {
        cplx<double> acc = A[(size_t)i * m + col];
        for (int k = 0; k < i; ++k) acc = acc - L[(size_t)i * m + k] * B[(size_t)k * m + col];
        B[(size_t)i * m + col] = cdiv_real(acc, L[(size_t)i * m + i].x);
      }
    }
    c.sync();
    for (int col = tid; col < m; col += nt) {
      for (int i = 0; i < m; ++i) {
        cplx<double> acc = conj(B[(size_t)col * m + i]);
        for (int k = 0; k < i; ++k) acc = acc - L[(size_t)i * m + k] * A[(size_t)k * m + col];
        A[(size_t)i * m + col] = cdiv_real(acc, L[(size_t)i * m + i].x);
      }
    }
    c.sync();
    // hermitise: A~ <- (A~ + A~^H)/2
    for (int e = tid; e < m * m; e += nt) {
      const int i = e / m, j = e - i * m;
      if (i < j) {
        const cplx<double> u = A[(size_t)i * m + j], l = A[(size_t)j * m + i];
        const cplx<double> h = mk<double>(0.5 * (u.x + l.x), 0.5 * (u.y - l.y));
        A[(size_t)i * m + j] = h;
        A[(size_t)j * m + i] = conj(h);
      } else if (i == j) {
        A[e].y = 0.0;
      }
      W[e] = mk<double>(i == j ? 1.0 : 0.0, 0.0);
    }
    c.sync();
    // ---- cyclic parallel Jacobi (round-robin pairs), W accumulates U
    const int mp = m + (m & 1);
    const int npair = mp / 2;
    double* rc = rot;
    double* rs = rot + npair;
    double* rex = rot + 2 * npair;
    double* rey = rot + 3 * npair;
    bool conv = false;
    double prev_off = 1e300;
    for (int sweep = 0; sweep < 40 && !conv; ++sweep) {
      for (int r = 0; r < mp - 1; ++r) {
        for (int k = tid; k < npair; k += nt) {
          int p, q;
          if (k == 0) {
            p = r;
            q = mp - 1;
          } else {
            p = (r + k) % (mp - 1);
            q = (r - k + (mp - 1)) % (mp - 1);
          }
          double cc = 1.0, ss = 0.0, ex = 1.0, ey = 0.0;
          if (p < m && q < m) {
            const cplx<double> bpq = A[(size_t)p * m + q];
            const double ab = sqrt(norm2(bpq));
            if (ab > 1e-300) {
              const double app = A[(size_t)p * m + p].x, aqq = A[(size_t)q * m + q].x;
              const double th = (aqq - app) / (2.0 * ab);
              const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
              cc = 1.0 / sqrt(t * t + 1.0);
              ss = t * cc;
              ex = bpq.x / ab;
              ey = bpq.y / ab;
            }
          }
          rc[k] = cc;
          rs[k] = ss;
          rex[k] = ex;
          rey[k] = ey;
        }
        c.sync();
        // columns: X[:,p] = c X_p - s e^{-i phi} X_q ; X[:,q] = s X_p + c e^{-i phi} X_q  (X = A and W)
        for (int e = tid; e < npair * m; e += nt) {
          const int k = e / m, i = e - k * m;
          int p, q;
          if (k == 0) {
            p = r;
            q = mp - 1;
          } else {
            p = (r + k) % (mp - 1);
            q = (r - k + (mp - 1)) % (mp - 1);
          }
          if (p >= m || q >= m || rs[k] == 0.0) continue;
          const double cc = rc[k], ss = rs[k];
          const cplx<double> em = mk<double>(rex[k], -rey[k]);  // e^{-i phi}
          for (int which = 0; which < 2; ++which) {
            cplx<double>* X = which ? W : A;
            const cplx<double> xp = X[(size_t)i * m + p], xq = X[(size_t)i * m + q];
            const cplx<double> emq = em * xq;
            X[(size_t)i * m + p] = mk<double>(cc * xp.x - ss * emq.x, cc * xp.y - ss * emq.y);
            X[(size_t)i * m + q] = mk<double>(ss * xp.x + cc * emq.x, ss * xp.y + cc * emq.y);
          }
        }
        c.sync();
        // rows: A[p,:] = c A_p - s e^{i phi} A_q ; A[q,:] = s A_p + c e^{i phi} A_q
        for (int e = tid; e < npair * m; e += nt) {
          const int k = e / m, j = e - k * m;
          int p, q;
          if (k == 0) {
            p = r;
            q = mp - 1;
          } else {
            p = (r + k) % (mp - 1);
            q = (r - k + (mp - 1)) % (mp - 1);
          }
          if (p >= m || q >= m || rs[k] == 0.0) continue;
          const double cc = rc[k], ss = rs[k];
          const cplx<double> ep = mk<double>(rex[k], rey[k]);
          const cplx<double> ap = A[(size_t)p * m + j], aq = A[(size_t)q * m + j];
          const cplx<double> epq = ep * aq;
          A[(size_t)p * m + j] = mk<double>(cc * ap.x - ss * epq.x, cc * ap.y - ss * epq.y);
          A[(size_t)q * m + j] = mk<double>(ss * ap.x + cc * epq.x, ss * ap.y + cc * epq.y);
        }
        c.sync();
      }
      // convergence: max |A_ij|, i != j, among unmasked, vs max |A_ii| among unmasked
      double off = 0.0, dia = 0.0;
      for (int e = tid; e < m * m; e += nt) {
        const int i = e / m, j = e - i * m;
        if (a.masked[i] || a.masked[j]) continue;
        const double v = sqrt(norm2(A[e]));
        if (i == j) dia = dia > v ? dia : v;
        else off = off > v ? off : v;
      }
      off = c.max(off, red);
      dia = c.max(dia, red);
      const double scale = dia > 1e-300 ? dia : 1e-300;
      // converged at a few ulps, or once rounding stops the decrease
      conv = off <= 1e-14 * scale || (off <= 1e-12 * scale && off > 0.5 * prev_off);
      prev_off = off;
      if (sweep == 39 && !conv && tid == 0) a.info[0] = -1;
    }
    // ---- ascending order of eigenvalues, ties by index
    for (int i = tid; i < m; i += nt) a.theta[i] = A[(size_t)i * m + i].x;
    c.sync();
    for (int i = tid; i < m; i += nt) {
      const double ti = a.theta[i];
      int rank = 0;
      for (int j = 0; j < m; ++j) {
        const double tj = a.theta[j];
        if (tj < ti || (tj == ti && j < i)) ++rank;
      }
      a.order[rank] = i;
    }
    c.sync();
    // ---- C = L^{-H} W[:, order[:nb]]  (back substitution, column per thread)
    for (int n = tid; n < nb; n += nt) {
      const int col = a.order[n];
      a.eval[n] = a.theta[col];
      for (int i = m - 1; i >= 0; --i) {
        cplx<double> acc = W[(size_t)i * m + col];
        for (int k = i + 1; k < m; ++k) acc = acc - conj(L[(size_t)k * m + i]) * a.Cd[(size_t)k * nb + n];
        a.Cd[(size_t)i * nb + n] = cdiv_real(acc, L[(size_t)i * m + i].x);
      }
    }
    c.sync();
    for (int e = tid; e < m * nb; e += nt) {
      const cplx<double> v = a.Cd[e];
      if (a.ct_double) ((cplx<double>*)a.Ct)[e] = v;
      else ((cplx<float>*)a.Ct)[e] = mk<float>((float)v.x, (float)v.y);
    }
  }
};

// ---------------------------------------------------------------------------
// Rotation X[n][G] = sum_j C[j][n] V[j][G]; grid (ceil(npw/256), ceil(nb/16)).
// C chunk of JC rows staged in LDS.
// ---------------------------------------------------------------------------
template <typename T>
struct KRotate {
  static constexpr int NT = 16, JC = 64;
  static size_t lds_bytes() { return sizeof(cplx<T>) * JC * NT; }
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const cplx<T>* __restrict__ v, const cplx<T>* __restrict__ C,
                         cplx<T>* __restrict__ x, int npw, int m, int nb) {
    cplx<T>* sC = (cplx<T>*)lds;
    const int n0 = c.by() * NT;
    // each thread owns G = bx*256 + l for l = tid, tid + nthr, ...; partial sums kept in x
    for (int j0 = 0; j0 < m; j0 += JC) {
      const int jc = (m - j0) < JC ? (m - j0) : JC;
      for (int idx = c.tid(); idx < JC * NT; idx += c.nthr()) {
        const int j = idx / NT, q = idx - j * NT;
        sC[idx] = (j < jc && n0 + q < nb) ? C[(size_t)(j0 + j) * nb + n0 + q] : mk<T>(0, 0);
      }
      c.sync();
      for (int l = c.tid(); l < kLBlk; l += c.nthr()) {
        const int g = c.bx() * kLBlk + l;
        if (g >= npw) break;
        cplx<T> acc[NT];
        for (int q = 0; q < NT; ++q) acc[q] = (j0 == 0 || n0 + q >= nb) ? mk<T>(0, 0) : x[(size_t)(n0 + q) * npw + g];
        for (int j = 0; j < jc; ++j) {
          const cplx<T> vv = v[(size_t)(j0 + j) * npw + g];
          for (int q = 0; q < NT; ++q) acc[q] = acc[q] + vv * sC[j * NT + q];
        }
        for (int q = 0; q < NT && n0 + q < nb; ++q) x[(size_t)(n0 + q) * npw + g] = acc[q];
      }
      c.sync();
    }
  }
};

// ---------------------------------------------------------------------------
// Residual + TPA preconditioner, one block per band.
// ---------------------------------------------------------------------------
template <typename T>
struct KPrecond {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const cplx<T>* __restrict__ x, const cplx<T>* __restrict__ hx,
                         const double* __restrict__ eval, cplx<T>* __restrict__ t, uint8_t* __restrict__ active,
                         double* __restrict__ rnorm, const int* __restrict__ millp, int npw, double kf0, double kf1,
                         double kf2, double b0, double b1, double b2) {
    double* red = (double*)lds;
    const int n = c.bx();
    const double lam = eval[n];
    const cplx<T>* xn = x + (size_t)n * npw;
    const cplx<T>* hn = hx + (size_t)n * npw;
    cplx<T>* tn = t + (size_t)n * npw;
    double r2 = 0.0, tk = 0.0;
    for (int g = c.tid(); g < npw; g += c.nthr()) {
      const cplx<T> xv = xn[g], hv = hn[g];
      const double rx = (double)hv.x - lam * xv.x, ry = (double)hv.y - lam * xv.y;
      r2 += rx * rx + ry * ry;
      const int p = millp[g];
      const double q1 = (((p & 1023) - 512) + kf0) * b0;
      const double q2 = ((((p >> 10) & 1023) - 512) + kf1) * b1;
      const double q3 = ((((p >> 20) & 1023) - 512) + kf2) * b2;
      tk += 0.5 * (q1 * q1 + q2 * q2 + q3 * q3) * ((double)xv.x * xv.x + (double)xv.y * xv.y);
    }
    r2 = c.sum(r2, red);
    tk = c.sum(tk, red);
    const double rn = sqrt(r2);
    const bool act = rn > 1e-10;
    double t2 = 0.0;
    for (int g = c.tid(); g < npw; g += c.nthr()) {
      const cplx<T> xv = xn[g], hv = hn[g];
      const double rx = (double)hv.x - lam * xv.x, ry = (double)hv.y - lam * xv.y;
      const int p = millp[g];
      const double q1 = (((p & 1023) - 512) + kf0) * b0;
      const double q2 = ((((p >> 10) & 1023) - 512) + kf1) * b1;
      const double q3 = ((((p >> 20) & 1023) - 512) + kf2) * b2;
      const double xx = 0.5 * (q1 * q1 + q2 * q2 + q3 * q3) / tk;
      const double pp = 27.0 + xx * (18.0 + xx * (12.0 + 8.0 * xx));
      const double K = pp / (pp + 16.0 * xx * xx * xx * xx);
      const double ux = K * rx, uy = K * ry;
      t2 += ux * ux + uy * uy;
      tn[g] = mk<T>((T)ux, (T)uy);
    }
    t2 = c.sum(t2, red);
    const double sc = (act && t2 > 0.0) ? 1.0 / sqrt(t2) : 0.0;
    for (int g = c.tid(); g < npw; g += c.nthr()) {
      const cplx<T> v = tn[g];
      tn[g] = mk<T>((T)(sc * v.x), (T)(sc * v.y));
    }
    if (c.tid() == 0) {
      active[n] = act ? 1 : 0;
      rnorm[n] = rn;
    }
  }
};

// ---------------------------------------------------------------------------
// Occupations of one subsystem (single block).
// ---------------------------------------------------------------------------
struct KOccupations {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const double* __restrict__ eval, const double* __restrict__ wk,
                         int nk, int nb, double nelec, int mode, double sigma, double* __restrict__ occw,
                         double* __restrict__ mu, int* __restrict__ info) {
    double* red = (double*)lds;
    const int tot = nk * nb;
    if (mode == 0) {
      const int nocc = (int)floor(nelec / 2.0 + 0.5);
      double emx = -1e300;
      for (int e = c.tid(); e < tot; e += c.nthr()) {
        const int k = e / nb, n = e - k * nb;
        occw[e] = n < nocc ? 2.0 * wk[k] : 0.0;
        if (n == nocc - 1) emx = emx > eval[e] ? emx : eval[e];
      }
      emx = c.max(emx, red);
      if (c.tid() == 0) {
        info[0] = nocc > nb ? 1 : 0;
        mu[0] = emx;
      }
      return;
    }
    double lo = 1e300, hi = -1e300;
    for (int e = c.tid(); e < tot; e += c.nthr()) {
      lo = lo < eval[e] ? lo : eval[e];
      hi = hi > eval[e] ? hi : eval[e];
    }
    lo = -c.max(-lo, red) - 20.0 * sigma;
    hi = c.max(hi, red) + 20.0 * sigma;
    double m = 0.5 * (lo + hi);
    for (int it = 0; it < 200; ++it) {
      m = 0.5 * (lo + hi);
      double s = 0.0;
      for (int e = c.tid(); e < tot; e += c.nthr()) s += wk[e / nb] * (1.0 - tanh((eval[e] - m) / (2.0 * sigma)));
      s = c.sum(s, red);
      if (fabs(s - nelec) < 1e-13) break;
      if (s < nelec) lo = m;
      else hi = m;
    }
    for (int e = c.tid(); e < tot; e += c.nthr())
      occw[e] = wk[e / nb] * (1.0 - tanh((eval[e] - m) / (2.0 * sigma)));
    if (c.tid() == 0) {
      mu[0] = m;
      info[0] = 0;
    }
  }
};

}  // namespace fde
