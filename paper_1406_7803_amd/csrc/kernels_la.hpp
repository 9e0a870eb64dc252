// Band-solver kernels: Gram matrices, the FP64 Rayleigh-Ritz solve
// (Cholesky with column dropping, reduction, Jacobi eigensolver), rotations,
// residual + Teter-Payne-Allan preconditioner, occupations.
#pragma once

#include "common.hpp"

namespace fde {

constexpr int kLBlk = 256;
constexpr double kInactiveDiag = 1.0e6;


constexpr int kMaxBatch = 16;   // problems per batched launch (descriptors travel as kernel arguments)
constexpr int kMaxChunks = 64;  // plane-wave chunks of a Gram product

// One band block of the solver: a (subsystem, k-point) pair. Rows 0..nb-1 of
// v/hv are X/HX, rows nb..m-1 the correction vectors T/HT.
template <typename T>
struct Prob {
  cplx<T>* v;
  cplx<T>* hv;
  cplx<T>* sv;             // [m][npw] S v of the generalised problem, or null (S = 1)
  cplx<T>* t;              // [nb][npw] preconditioner output (rows nb.. of v in a block)
  const uint8_t* active;   // [m] or null (Rayleigh-Ritz input)
  uint8_t* act_out;        // [nb] (preconditioner output, the T rows' flags)
  double* eval;            // [nb]
  double* rnorm;           // [nb]
  int* info;
  const int* millp;        // packed Miller indices [npw]
  double kf[3];
  int npw, m, nb, nchunk, chunk;
  // per-problem scratch
  cplx<double>* part;      // Gram partials [nchunk][2][m][m]
  cplx<double>*S, *A, *L, *B, *W, *Cd;
  void* Ct;                // C in plan precision [m][nb]
  double* theta;
  int* order;
  int* masked;
};

template <typename T>
struct ProbSet {
  int n;
  double b[3];
  double drop_tol;
  Prob<T> p[kMaxBatch];
};

// S, A = sum over chunks (fixed order). grid (ceil(2 m^2/256), n)
template <typename T>
struct KGramReduce {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const ProbSet<T> ps) {
    const Prob<T>& P = ps.p[c.by()];
    const size_t mm = (size_t)P.m * P.m;
    for (int l = c.tid(); l < kLBlk; l += c.nthr()) {
      const size_t o = (size_t)c.bx() * kLBlk + l;
      if (o >= 2 * mm) break;
      double sx = 0, sy = 0;
      for (int k = 0; k < P.nchunk; ++k) {
        const cplx<double> v = P.part[(size_t)k * 2 * mm + o];
        sx += v.x;
        sy += v.y;
      }
      if (o < mm) P.S[o] = mk<double>(sx, sy);
      else P.A[o - mm] = mk<double>(sx, sy);
    }
  }
};

FDE_HD cplx<double> cdiv_real(cplx<double> a, double d) { return mk<double>(a.x / d, a.y / d); }

// One column of X = L^{-1} R (L lower triangular, row-major, ld m; forward substitution) or,
// with `upper`, of X = L^{-H} R (backward substitution). Rows go in blocks of 8: each x_k
// loaded serves the 8 rows of a block, whose L entries are the same for every column (one
// column per thread), then the block's own triangle is solved in registers. R(i) is
// conj(r[i * rs]) when `rconj`; x_k lives at x[k * xs].
FDE_HD inline void tri_solve_col(const cplx<double>* L, int m, const cplx<double>* r, size_t rs, bool rconj,
                                 cplx<double>* x, size_t xs, bool upper) {
  constexpr int RB = 8;
  for (int b0 = 0; b0 < m; b0 += RB) {
    const int nr = m - b0 < RB ? m - b0 : RB;
    // rows of the block: i_q = b0 + q (forward) or m - 1 - b0 - q (backward)
    double ax[RB], ay[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) ax[q] = ay[q] = 0.0;
    // rows beyond the last (q >= nr) repeat row nr - 1: every load stays unconditional (and in
    // bounds), so the block's loads issue together; their sums are not used
    for (int t = 0; t < b0; ++t) {  // the rows already solved
      const int k = upper ? m - 1 - t : t;
      const cplx<double> xk = x[(size_t)k * xs];
      cplx<double> l[RB];
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const int qq = q < nr ? q : nr - 1;
        const int i = upper ? m - 1 - b0 - qq : b0 + qq;
        l[q] = upper ? L[(size_t)k * m + i] : L[(size_t)i * m + k];
      }
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        // forward: L_ik x_k; backward: conj(L_ki) x_k
        const double ly = upper ? -l[q].y : l[q].y;
        ax[q] += l[q].x * xk.x - ly * xk.y;
        ay[q] += l[q].x * xk.y + ly * xk.x;
      }
    }
    cplx<double> xb[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) {
      if (q < nr) {
        const int i = upper ? m - 1 - b0 - q : b0 + q;
        double sx = ax[q], sy = ay[q];
#pragma unroll
        for (int p = 0; p < q; ++p) {
          const int k = upper ? m - 1 - b0 - p : b0 + p;
          const cplx<double> l = upper ? L[(size_t)k * m + i] : L[(size_t)i * m + k];
          const double ly = upper ? -l.y : l.y;
          sx += l.x * xb[p].x - ly * xb[p].y;
          sy += l.x * xb[p].y + ly * xb[p].x;
        }
        const cplx<double> ri = r[(size_t)i * rs];
        const double rix = ri.x, riy = rconj ? -ri.y : ri.y;
        xb[q] = cdiv_real(mk<double>(rix - sx, riy - sy), L[(size_t)i * m + i].x);
        x[(size_t)i * xs] = xb[q];
      }
    }
  }
}

template <typename T>
struct KRRSolve {
  // reduction scratch + rotation parameters; the Jacobi matrices A~ and W are
  // staged in LDS when they fit in `lds_mats` bytes (A~ first, then W).
  FDE_HD static size_t lds_fixed(int m) { return sizeof(double) * (32 + 4 * ((m + 2) / 2 + 1)); }

  // Masks, Cholesky with dropping, B = L^{-1} A, A~ = L^{-1} B^H (in a.A), all in global memory.
  // Returns false, with C = I, NaN eigenvalues and info written, when a band column has no
  // positive pivot.
  template <class Ctx>
  FDE_HD static bool front(const Ctx& c, double* red, const Prob<T>& a, double drop_tol) {
    if (!front_chol(c, red, a, drop_tol)) return false;
    const int m = a.m, tid = c.tid(), nt = c.nthr();
    cplx<double>*A = a.A, *L = a.L, *B = a.B;
    // ---- B = L^{-1} A, then A~ = L^{-1} B^H into A: column per thread
    for (int col = tid; col < m; col += nt) tri_solve_col(L, m, A + col, m, false, B + col, m, false);
    c.sync();
    for (int col = tid; col < m; col += nt) tri_solve_col(L, m, B + (size_t)col * m, 1, true, A + col, m, false);
    c.sync();
    return true;
  }

  // Masks and the Cholesky factor with dropping (the first part of front).
  template <class Ctx>
  FDE_HD static bool front_chol(const Ctx& c, double* red, const Prob<T>& a, double drop_tol) {
    const int m = a.m, nb = a.nb;
    const int tid = c.tid(), nt = c.nthr();
#if defined(__HIP_DEVICE_COMPILE__)
    constexpr int GL = 16;
#else
    constexpr int GL = 1;
#endif
    const int gl = tid % GL, grp = tid / GL, ng = nt / GL;
    cplx<double>*S = a.S, *A = a.A, *L = a.L, *B = a.B;
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
      const bool drop = (j >= nb) && !(d >= drop_tol * sjj);
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
      if (!(d >= drop_tol * sjj) || !(d > 0.0)) {
        // a band column (j < nb) that is (numerically) dependent: report, and
        // leave X = the first nb columns of V
        if (tid == 0) a.info[0] = j + 1;
        for (int e = tid; e < m * nb; e += nt) {
          const int i = e / nb, n = e - i * nb;
          const cplx<double> v = mk<double>(i == n ? 1.0 : 0.0, 0.0);
          a.Cd[e] = v;
          ((cplx<T>*)a.Ct)[e] = mk<T>((T)v.x, (T)v.y);
        }
        for (int n = tid; n < nb; n += nt) a.eval[n] = 0.0 / 0.0;
        c.sync();
        return false;  // uniform: every thread saw the same d
      }
      const double ljj = sqrt(d);
      if (tid == 0) L[(size_t)j * m + j] = mk<double>(ljj, 0.0);
      // row i by a lane group, lane g summing the terms k = g (mod GL)
      for (int i = j + 1 + grp; i < m; i += ng) {
        const cplx<double>*li = L + (size_t)i * m, *lj = L + (size_t)j * m;
        double ax = 0.0, ay = 0.0;  // sum_k L_ik conj(L_jk)
        for (int k = gl; k < j; k += GL) {
          const cplx<double> lik = li[k], ljk = lj[k];
          ax += lik.x * ljk.x + lik.y * ljk.y;
          ay += lik.y * ljk.x - lik.x * ljk.y;
        }
        ax = c.template gsum<GL>(ax);
        ay = c.template gsum<GL>(ay);
        if (gl == 0) {
          const cplx<double> sij = S[(size_t)i * m + j];
          L[(size_t)i * m + j] = cdiv_real(mk<double>(sij.x - ax, sij.y - ay), ljj);
        }
      }
      c.sync();
    }
    (void)B;
    return true;
  }

  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps, size_t lds_mats) {
    const Prob<T>& a = ps.p[c.bx()];
    double* red = (double*)lds;            // 17 used
    double* rot = red + 32;                // [4][mp/2]
    const int m = a.m, nb = a.nb;
    const int tid = c.tid(), nt = c.nthr();
    cplx<double>*S = a.S, *A = a.A, *L = a.L, *B = a.B, *W = a.W;
    const double drop_tol = ps.drop_tol;
    char* mats = lds + ((lds_fixed(m) + 15) & ~(size_t)15);
    const size_t mbytes = (size_t)m * m * sizeof(cplx<double>);
    if (!front(c, red, a, drop_tol)) return;
    // hermitise: A~ <- (A~ + A~^H)/2, staged into LDS when it fits
    cplx<double>* Aj = (mbytes <= lds_mats) ? (cplx<double>*)mats : A;
    cplx<double>* Wj = (2 * mbytes <= lds_mats) ? (cplx<double>*)(mats + mbytes) : W;
    for (int e = tid; e < m * m; e += nt) {
      const int i = e / m, j = e - i * m;
      if (i < j) {
        const cplx<double> u = A[(size_t)i * m + j], l = A[(size_t)j * m + i];
        const cplx<double> h = mk<double>(0.5 * (u.x + l.x), 0.5 * (u.y - l.y));
        Aj[(size_t)i * m + j] = h;
        Aj[(size_t)j * m + i] = conj(h);
      } else if (i == j) {
        Aj[e] = mk<double>(A[e].x, 0.0);
      }
      Wj[e] = mk<double>(i == j ? 1.0 : 0.0, 0.0);
    }
    c.sync();
    A = Aj;
    W = Wj;
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
      ((cplx<T>*)a.Ct)[e] = mk<T>((T)v.x, (T)v.y);
    }
  }
};

// ---------------------------------------------------------------------------
// In-place rotation of every problem: rows 0..nb-1 of V (grid.y = 0) or HV
// (grid.y = 1) become sum_j C[j][n] V_j. Each block stages its plane-wave
// chunk of all m rows in LDS first, so overwriting rows 0..nb-1 is safe.
// grid (ceil(npw_max/GC), 2, n)
// ---------------------------------------------------------------------------
template <typename T>
struct KRotate {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps, int GC, int c_in_lds) {
    const Prob<T>& P = ps.p[c.bz()];
    const int m = P.m, nb = P.nb, npw = P.npw;
    const int g0 = c.bx() * GC;
    if (g0 >= npw) return;  // uniform per block
    const int gc = (npw - g0) < GC ? (npw - g0) : GC;
    cplx<T>* M = c.by() == 0 ? P.v : (c.by() == 1 ? P.hv : P.sv);
    if (!M) return;  // no S v rows in this problem (uniform per block)
    const cplx<T>* Cg = (const cplx<T>*)P.Ct;
    cplx<T>* sV = (cplx<T>*)lds;               // [m][GC]
    cplx<T>* sC = sV + (size_t)m * GC;         // [m][nb] when staged
    for (int idx = c.tid(); idx < m * GC; idx += c.nthr()) {
      const int j = idx / GC, g = idx - j * GC;
      sV[idx] = g < gc ? M[(size_t)j * npw + g0 + g] : mk<T>(0, 0);
    }
    if (c_in_lds)
      for (int idx = c.tid(); idx < m * nb; idx += c.nthr()) sC[idx] = Cg[idx];
    c.sync();
    const cplx<T>* Cs = c_in_lds ? sC : Cg;
#if defined(__HIP_DEVICE_COMPILE__)
    if (GC == 64 && c_in_lds && c.nthr() == 256 && nb <= 64) {
      // matrix cores: wave w owns plane-wave columns 16 w .. 16 w + 15 and every 16-band tile;
      // X = C^T V as four real products per complex one (Re = CrVr - CiVi, Im = CrVi + CiVr)
      const int lane = c.tid() & 63, w = c.tid() >> 6;
      const int col = lane & 15, kq = lane >> 4;
      constexpr int MT = 4;  // up to 64 bands per block
      typedef T v4 __attribute__((ext_vector_type(4)));
      v4 re[MT], im[MT];
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        re[t] = v4{0, 0, 0, 0};
        im[t] = v4{0, 0, 0, 0};
      }
      const int nmt = (nb + 15) / 16;
      for (int k0 = 0; k0 < m; k0 += 4) {
        const int k = k0 + kq;
        const cplx<T> b = k < m ? sV[k * GC + 16 * w + col] : mk<T>(0, 0);
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          if (t >= nmt) break;
          const int n = 16 * t + col;
          const cplx<T> a_ = (k < m && n < nb) ? sC[(size_t)k * nb + n] : mk<T>(0, 0);
          if constexpr (sizeof(T) == 8) {
            re[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_.x, b.x, re[t], 0, 0, 0);
            re[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a_.y, b.y, re[t], 0, 0, 0);
            im[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_.x, b.y, im[t], 0, 0, 0);
            im[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_.y, b.x, im[t], 0, 0, 0);
          } else {
            re[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_.x, b.x, re[t], 0, 0, 0);
            re[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a_.y, b.y, re[t], 0, 0, 0);
            im[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_.x, b.y, im[t], 0, 0, 0);
            im[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_.y, b.x, im[t], 0, 0, 0);
          }
        }
      }
      const int g = 16 * w + col;
      if (g < gc) {
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          if (t >= nmt) break;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            // output row of register r: FP64 MFMA 4 r + l/16, FP32 MFMA 4 (l/16) + r
            const int n = 16 * t + (sizeof(T) == 8 ? 4 * r + kq : 4 * kq + r);
            if (n < nb) M[(size_t)n * npw + g0 + g] = mk<T>(re[t][r], im[t][r]);
          }
        }
      }
      return;
    }
#endif
    for (int o = c.tid(); o < nb * GC; o += c.nthr()) {
      const int n = o / GC, g = o - n * GC;
      if (g >= gc) continue;
      cplx<T> acc = mk<T>(0, 0);
      for (int j = 0; j < m; ++j) acc = acc + sV[j * GC + g] * Cs[(size_t)j * nb + n];
      M[(size_t)n * npw + g0 + g] = acc;
    }
  }
};

// ---------------------------------------------------------------------------
// The same rotation for any m and 64 < nb <= 128 on the matrix cores: a workgroup of four
// wavefronts takes 64 plane-wave columns (16 per wavefront, read straight from global memory
// into registers, four k-steps of 4 rows at a time) and every band tile; C passes through
// LDS in chunks of kRotChunk rows shared by the four wavefronts. Each wavefront writes its
// nb output rows after it has read all m rows of its columns. grid (ceil(npw / 64), 2, n).
// ---------------------------------------------------------------------------
constexpr int kRotChunk = 16;

template <typename T>
struct KRotateChunk {
  static constexpr int MT = 8;  // band tiles: nb <= 128
  FDE_HD static size_t lds_bytes(int nb) { return sizeof(cplx<T>) * (size_t)kRotChunk * nb; }
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps) {
    const Prob<T>& P = ps.p[c.bz()];
    const int m = P.m, nb = P.nb, npw = P.npw;
    const int g0 = c.bx() * 64;
    if (g0 >= npw) return;  // uniform per block
    cplx<T>* M = c.by() == 0 ? P.v : (c.by() == 1 ? P.hv : P.sv);
    if (!M) return;  // no S v rows in this problem (uniform per block)
    const cplx<T>* Cg = (const cplx<T>*)P.Ct;
    cplx<T>* sC = (cplx<T>*)lds;  // [kRotChunk][nb]
#if defined(__HIP_DEVICE_COMPILE__)
    const int lane = c.tid() & 63, w = c.tid() >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int g = g0 + 16 * w + col;
    const bool gin = g < npw;
    typedef T v4 __attribute__((ext_vector_type(4)));
    v4 re[MT], im[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      re[t] = v4{0, 0, 0, 0};
      im[t] = v4{0, 0, 0, 0};
    }
    const int nmt = (nb + 15) / 16;
    for (int k0 = 0; k0 < m; k0 += kRotChunk) {
      const int kc = (m - k0) < kRotChunk ? (m - k0) : kRotChunk;
      c.sync();  // the previous chunk is consumed
      for (int idx = c.tid(); idx < kRotChunk * nb; idx += c.nthr())
        sC[idx] = idx < kc * nb ? Cg[(size_t)k0 * nb + idx] : mk<T>(0, 0);
      // V rows k0 + 4 s + kq of this lane's column, all loads of the chunk issued together
      cplx<T> b[kRotChunk / 4];
#pragma unroll
      for (int s4 = 0; s4 < kRotChunk / 4; ++s4) {
        const int k = k0 + 4 * s4 + kq;
        b[s4] = (gin && k < m) ? M[(size_t)k * npw + g] : mk<T>(0, 0);
      }
      c.sync();
#pragma unroll
      for (int s4 = 0; s4 < kRotChunk / 4; ++s4) {
        const int kl = 4 * s4 + kq;  // row within the chunk (zero beyond kc)
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          if (t >= nmt) break;
          const int n = 16 * t + col;
          const cplx<T> a_ = n < nb ? sC[kl * nb + n] : mk<T>(0, 0);
          if constexpr (sizeof(T) == 8) {
            re[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_.x, b[s4].x, re[t], 0, 0, 0);
            re[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a_.y, b[s4].y, re[t], 0, 0, 0);
            im[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_.x, b[s4].y, im[t], 0, 0, 0);
            im[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_.y, b[s4].x, im[t], 0, 0, 0);
          } else {
            re[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_.x, b[s4].x, re[t], 0, 0, 0);
            re[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a_.y, b[s4].y, re[t], 0, 0, 0);
            im[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_.x, b[s4].y, im[t], 0, 0, 0);
            im[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_.y, b[s4].x, im[t], 0, 0, 0);
          }
        }
      }
    }
    if (gin) {
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        if (t >= nmt) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // output row of register r: FP64 MFMA 4 r + l/16, FP32 MFMA 4 (l/16) + r
          const int n = 16 * t + (sizeof(T) == 8 ? 4 * r + kq : 4 * kq + r);
          if (n < nb) M[(size_t)n * npw + g] = mk<T>(re[t][r], im[t][r]);
        }
      }
    }
#else
    // host: column by column, all m rows read before the nb rows are written
    for (int gg = g0; gg < g0 + 64 && gg < npw; ++gg) {
      cplx<T>* v = new cplx<T>[m];
      for (int k = 0; k < m; ++k) v[k] = M[(size_t)k * npw + gg];
      for (int n = 0; n < nb; ++n) {
        cplx<T> acc = mk<T>(0, 0);
        for (int k = 0; k < m; ++k) acc = acc + v[k] * Cg[(size_t)k * nb + n];
        M[(size_t)n * npw + gg] = acc;
      }
      delete[] v;
    }
    (void)sC;
#endif
  }
};

// ---------------------------------------------------------------------------
// The same rotation for any m and nb > 128 on the matrix cores. A workgroup of
// four wavefronts takes 16 CG plane-wave columns. Only the rows 0..nb-1 of V are
// overwritten, so only those (the X rows of the columns) are staged in LDS
// before any output is written; the rows nb..m-1 are read straight from global
// memory. Wavefront w accumulates the band tiles w, w + 4, ... (16 bands each,
// at most kRotWideTiles per wavefront) over all m rows, then writes them.
// grid (ceil(npw / (16 CG)), number of rotated matrices, n).
// ---------------------------------------------------------------------------
constexpr int kRotWideTiles = 8;  // per wavefront: nb <= 4 * 8 * 16 = 512

// CG groups of 16 plane-wave columns per workgroup (1 or 2): with two, every C element
// loaded feeds twice the matrix-core work and C is read half as often over the grid.
template <typename T, int CG = 1>
struct KRotateWide {
  static constexpr int NC = 16 * CG;  // plane-wave columns per workgroup
  FDE_HD static size_t lds_bytes(int nb) { return sizeof(cplx<T>) * (size_t)nb * NC; }
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps) {
    const Prob<T>& P = ps.p[c.bz()];
    const int m = P.m, nb = P.nb, npw = P.npw;
    const int g0 = c.bx() * NC;
    if (g0 >= npw) return;  // uniform per block
    cplx<T>* M = c.by() == 0 ? P.v : (c.by() == 1 ? P.hv : P.sv);
    if (!M) return;  // no S v rows in this problem (uniform per block)
    const cplx<T>* Cg = (const cplx<T>*)P.Ct;
    cplx<T>* sX = (cplx<T>*)lds;  // [nb][NC]
    for (int idx = c.tid(); idx < nb * NC; idx += c.nthr()) {
      const int j = idx / NC, g = g0 + (idx % NC);
      sX[idx] = g < npw ? M[(size_t)j * npw + g] : mk<T>(0, 0);
    }
    c.sync();
#if defined(__HIP_DEVICE_COMPILE__)
    const int lane = c.tid() & 63, w = c.tid() >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int ntile = (nb + 15) / 16;
    typedef T v4 __attribute__((ext_vector_type(4)));
    v4 re[kRotWideTiles][CG], im[kRotWideTiles][CG];
#pragma unroll
    for (int t = 0; t < kRotWideTiles; ++t)
#pragma unroll
      for (int h = 0; h < CG; ++h) {
        re[t][h] = v4{0, 0, 0, 0};
        im[t][h] = v4{0, 0, 0, 0};
      }
    // operands of step k0 + 4 are loaded while the matrix cores work on step k0
    auto load = [&](int k0, cplx<T>* b, cplx<T>* a) {
      const int k = k0 + kq;
#pragma unroll
      for (int h = 0; h < CG; ++h) {
        const int g = g0 + 16 * h + col;
        b[h] = mk<T>(0, 0);
        if (k < nb) b[h] = sX[k * NC + 16 * h + col];
        else if (k < m && g < npw) b[h] = M[(size_t)k * npw + g];
      }
#pragma unroll
      for (int i = 0; i < kRotWideTiles; ++i) {
        const int n = 16 * (w + 4 * i) + col;
        a[i] = (k < m && n < nb) ? Cg[(size_t)k * nb + n] : mk<T>(0, 0);
      }
    };
    cplx<T> bc[CG], ac[kRotWideTiles], bn[CG], an[kRotWideTiles];
    load(0, bc, ac);
    for (int k0 = 0; k0 < m; k0 += 4) {
      if (k0 + 4 < m) load(k0 + 4, bn, an);
#pragma unroll
      for (int i = 0; i < kRotWideTiles; ++i) {
        const int t = w + 4 * i;
        if (t >= ntile) break;
        const cplx<T> a_ = ac[i];
#pragma unroll
        for (int h = 0; h < CG; ++h) {
          const cplx<T> b = bc[h];
          if constexpr (sizeof(T) == 8) {
            re[i][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_.x, b.x, re[i][h], 0, 0, 0);
            re[i][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a_.y, b.y, re[i][h], 0, 0, 0);
            im[i][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_.x, b.y, im[i][h], 0, 0, 0);
            im[i][h] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_.y, b.x, im[i][h], 0, 0, 0);
          } else {
            re[i][h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_.x, b.x, re[i][h], 0, 0, 0);
            re[i][h] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a_.y, b.y, re[i][h], 0, 0, 0);
            im[i][h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_.x, b.y, im[i][h], 0, 0, 0);
            im[i][h] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_.y, b.x, im[i][h], 0, 0, 0);
          }
        }
      }
#pragma unroll
      for (int h = 0; h < CG; ++h) bc[h] = bn[h];
#pragma unroll
      for (int i = 0; i < kRotWideTiles; ++i) ac[i] = an[i];
    }
#pragma unroll
    for (int h = 0; h < CG; ++h) {
      const int g = g0 + 16 * h + col;
      if (g >= npw) continue;
#pragma unroll
      for (int i = 0; i < kRotWideTiles; ++i) {
        const int t = w + 4 * i;
        if (t >= ntile) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // output row of register r: FP64 MFMA 4 r + l/16, FP32 MFMA 4 (l/16) + r
          const int n = 16 * t + (sizeof(T) == 8 ? 4 * r + kq : 4 * kq + r);
          if (n < nb) M[(size_t)n * npw + g] = mk<T>(re[i][h][r], im[i][h][r]);
        }
      }
    }
#else
    // host: the X rows come from LDS, the rest from global memory (never written)
    for (int gg = g0; gg < g0 + NC && gg < npw; ++gg) {
      for (int n = 0; n < nb; ++n) {
        cplx<T> acc = mk<T>(0, 0);
        for (int k = 0; k < m; ++k) {
          const cplx<T> v = k < nb ? sX[k * NC + (gg - g0)] : M[(size_t)k * npw + gg];
          acc = acc + v * Cg[(size_t)k * nb + n];
        }
        M[(size_t)n * npw + gg] = acc;
      }
    }
#endif
  }
};

// ---------------------------------------------------------------------------
// The same rotation streamed (m <= 4 kRotSteps, nb <= 64): C staged once per
// workgroup in LDS; each wavefront takes groups of 16 plane-wave columns in turn,
// loads all m rows of its group straight into registers (no LDS staging of V),
// multiplies on the matrix cores and writes the nb rows back in place (every row
// of the group was read first). grid (gx, 2, n); gx workgroups share the groups.
// ---------------------------------------------------------------------------
constexpr int kRotSteps = 20;  // k-steps of 4 rows held in registers: m <= 80

template <typename T>
struct KRotateStream {
  FDE_HD static size_t lds_bytes(int m, int nb) { return sizeof(cplx<T>) * (size_t)m * nb; }
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps, int gx) {
    const Prob<T>& P = ps.p[c.bz()];
    const int m = P.m, nb = P.nb, npw = P.npw;
    cplx<T>* M = c.by() == 0 ? P.v : (c.by() == 1 ? P.hv : P.sv);
    if (!M) return;  // no S v rows in this problem (uniform per block)
    const cplx<T>* Cg = (const cplx<T>*)P.Ct;
    cplx<T>* sC = (cplx<T>*)lds;
    for (int idx = c.tid(); idx < m * nb; idx += c.nthr()) sC[idx] = Cg[idx];
    c.sync();
    const int ngroups = (npw + 15) / 16;
#if defined(__HIP_DEVICE_COMPILE__)
    const int lane = c.tid() & 63, w = c.tid() >> 6, nw = c.nthr() >> 6;
    const int col = lane & 15, kq = lane >> 4;
    constexpr int MT = 4;
    typedef T v4 __attribute__((ext_vector_type(4)));
    const int nmt = (nb + 15) / 16;
    for (int grp = c.bx() * nw + w; grp < ngroups; grp += gx * nw) {  // uniform per wavefront
      const int g = 16 * grp + col;
      v4 re[MT], im[MT];
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        re[t] = v4{0, 0, 0, 0};
        im[t] = v4{0, 0, 0, 0};
      }
      // the group's rows in two halves of kRotSteps / 2 k-steps (fewer live registers)
#pragma unroll
      for (int hf = 0; hf < 2; ++hf) {
      constexpr int HS = kRotSteps / 2;
      cplx<T> b[HS];
#pragma unroll
      for (int u = 0; u < HS; ++u) {
        const int k = 4 * (HS * hf + u) + kq;
        b[u] = (k < m && g < npw) ? M[(size_t)k * npw + g] : mk<T>(0, 0);
      }
#pragma unroll
      for (int u = 0; u < HS; ++u) {
        const int st = HS * hf + u;
        if (4 * st >= m) break;  // uniform
        const int k = 4 * st + kq;
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          if (t >= nmt) break;
          const int n = 16 * t + col;
          const cplx<T> a_ = (k < m && n < nb) ? sC[(size_t)k * nb + n] : mk<T>(0, 0);
          if constexpr (sizeof(T) == 8) {
            re[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_.x, b[u].x, re[t], 0, 0, 0);
            re[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a_.y, b[u].y, re[t], 0, 0, 0);
            im[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_.x, b[u].y, im[t], 0, 0, 0);
            im[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_.y, b[u].x, im[t], 0, 0, 0);
          } else {
            re[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_.x, b[u].x, re[t], 0, 0, 0);
            re[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(-a_.y, b[u].y, re[t], 0, 0, 0);
            im[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_.x, b[u].y, im[t], 0, 0, 0);
            im[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a_.y, b[u].x, im[t], 0, 0, 0);
          }
        }
      }
      }
      if (g < npw) {
#pragma unroll
        for (int t = 0; t < MT; ++t) {
          if (t >= nmt) break;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            // output row of register r: FP64 MFMA 4 r + l/16, FP32 MFMA 4 (l/16) + r
            const int n = 16 * t + (sizeof(T) == 8 ? 4 * r + kq : 4 * kq + r);
            if (n < nb) M[(size_t)n * npw + g] = mk<T>(re[t][r], im[t][r]);
          }
        }
      }
    }
#else
    for (int grp = c.bx(); grp < ngroups; grp += gx) {
      const int gend = 16 * grp + 16 < npw ? 16 * grp + 16 : npw;
      for (int g = 16 * grp; g < gend; ++g) {
        cplx<T> col[4 * kRotSteps];
        for (int k = 0; k < m; ++k) col[k] = M[(size_t)k * npw + g];
        for (int n = 0; n < nb; ++n) {
          cplx<T> acc = mk<T>(0, 0);
          for (int k = 0; k < m; ++k) acc = acc + col[k] * sC[(size_t)k * nb + n];
          M[(size_t)n * npw + g] = acc;
        }
      }
    }
#endif
  }
};

// ---------------------------------------------------------------------------
// Residual + Teter-Payne-Allan preconditioner of every problem; block (n, p)
// handles band n of problem p and writes the correction T_n into row n of its
// t (rows nb.. of V in a band block). grid (nb_max, n)
// ---------------------------------------------------------------------------
template <typename T>
struct KPrecond {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps) {
    const Prob<T>& P = ps.p[c.by()];
    const int n = c.bx();
    if (n >= P.nb) return;  // uniform per block
    double* red = (double*)lds;
    const int npw = P.npw;
    const double lam = P.eval[n];
    const cplx<T>* xn = P.v + (size_t)n * npw;
    const cplx<T>* hn = P.hv + (size_t)n * npw;
    const cplx<T>* sn = P.sv ? P.sv + (size_t)n * npw : xn;  // residual H x - lambda S x
    cplx<T>* tn = P.t + (size_t)n * npw;
    const double kf0 = P.kf[0], kf1 = P.kf[1], kf2 = P.kf[2];
    const double b0 = ps.b[0], b1 = ps.b[1], b2 = ps.b[2];
    double r2 = 0.0, tk = 0.0;
    for (int g = c.tid(); g < npw; g += c.nthr()) {
      const cplx<T> xv = xn[g], hv = hn[g], sv = sn[g];
      const double rx = (double)hv.x - lam * sv.x, ry = (double)hv.y - lam * sv.y;
      r2 += rx * rx + ry * ry;
      const int p = P.millp[g];
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
      const cplx<T> hv = hn[g], sv = sn[g];
      const double rx = (double)hv.x - lam * sv.x, ry = (double)hv.y - lam * sv.y;
      const int p = P.millp[g];
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
      P.act_out[n] = act ? 1 : 0;
      P.rnorm[n] = rn;
    }
  }
};

// The same preconditioner spread over plane-wave chunks (kPcChunks blocks per
// band), in three passes with fixed-order reductions of per-chunk partials
// (kept in the problem's Gram-partial scratch, free between Rayleigh-Ritz
// steps): (A) |R|^2 and T_n^kin, (B) T = K R unnormalised and |T|^2, (C) the
// normalisation, the active flag and ||R||. grid (kPcChunks, nb_max, nprob).
constexpr int kPcChunks = 16;

template <typename T>
struct KPcBase {
  FDE_HD static double kin_of_g(const Prob<T>& P, const ProbSet<T>& ps, int g) {
    const int p = P.millp[g];
    const double q1 = (((p & 1023) - 512) + P.kf[0]) * ps.b[0];
    const double q2 = ((((p >> 10) & 1023) - 512) + P.kf[1]) * ps.b[1];
    const double q3 = ((((p >> 20) & 1023) - 512) + P.kf[2]) * ps.b[2];
    return 0.5 * (q1 * q1 + q2 * q2 + q3 * q3);
  }
  FDE_HD static void range(const Prob<T>& P, int ch, int& g0, int& g1) {
    const int len = (P.npw + kPcChunks - 1) / kPcChunks;
    g0 = ch * len;
    g1 = (g0 + len) < P.npw ? (g0 + len) : P.npw;
  }
  FDE_HD static double* part(const Prob<T>& P, int n) { return (double*)P.part + (size_t)n * kPcChunks * 3; }
};

template <typename T>
struct KPrecondA : KPcBase<T> {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps) {
    const Prob<T>& P = ps.p[c.bz()];
    const int n = c.by(), ch = c.bx();
    if (n >= P.nb) return;  // uniform per block
    int g0, g1;
    KPcBase<T>::range(P, ch, g0, g1);
    const double lam = P.eval[n];
    const cplx<T>* xn = P.v + (size_t)n * P.npw;
    const cplx<T>* hn = P.hv + (size_t)n * P.npw;
    const cplx<T>* sn = P.sv ? P.sv + (size_t)n * P.npw : xn;  // residual H x - lambda S x
    double r2 = 0.0, tk = 0.0;
    for (int g = g0 + c.tid(); g < g1; g += c.nthr()) {
      const cplx<T> xv = xn[g], hv = hn[g], sv = sn[g];
      const double rx = (double)hv.x - lam * sv.x, ry = (double)hv.y - lam * sv.y;
      r2 += rx * rx + ry * ry;
      tk += KPcBase<T>::kin_of_g(P, ps, g) * ((double)xv.x * xv.x + (double)xv.y * xv.y);
    }
    r2 = c.sum(r2, (double*)lds);
    tk = c.sum(tk, (double*)lds);
    if (c.tid() == 0) {
      double* pt = KPcBase<T>::part(P, n);
      pt[ch] = r2;
      pt[kPcChunks + ch] = tk;
    }
  }
};

template <typename T>
struct KPrecondB : KPcBase<T> {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps) {
    const Prob<T>& P = ps.p[c.bz()];
    const int n = c.by(), ch = c.bx();
    if (n >= P.nb) return;
    int g0, g1;
    KPcBase<T>::range(P, ch, g0, g1);
    double* pt = KPcBase<T>::part(P, n);
    double tk = 0.0;
    for (int k = 0; k < kPcChunks; ++k) tk += pt[kPcChunks + k];
    const double lam = P.eval[n];
    const cplx<T>* xn = P.v + (size_t)n * P.npw;
    const cplx<T>* hn = P.hv + (size_t)n * P.npw;
    const cplx<T>* sn = P.sv ? P.sv + (size_t)n * P.npw : xn;  // residual H x - lambda S x
    cplx<T>* tn = P.t + (size_t)n * P.npw;
    double t2 = 0.0;
    for (int g = g0 + c.tid(); g < g1; g += c.nthr()) {
      const cplx<T> hv = hn[g], sv = sn[g];
      const double rx = (double)hv.x - lam * sv.x, ry = (double)hv.y - lam * sv.y;
      const double xx = KPcBase<T>::kin_of_g(P, ps, g) / tk;
      const double pp = 27.0 + xx * (18.0 + xx * (12.0 + 8.0 * xx));
      const double K = pp / (pp + 16.0 * xx * xx * xx * xx);
      const double ux = K * rx, uy = K * ry;
      t2 += ux * ux + uy * uy;
      tn[g] = mk<T>((T)ux, (T)uy);
    }
    t2 = c.sum(t2, (double*)lds);
    if (c.tid() == 0) pt[2 * kPcChunks + ch] = t2;
  }
};

template <typename T>
struct KPrecondC : KPcBase<T> {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const ProbSet<T> ps) {
    const Prob<T>& P = ps.p[c.bz()];
    const int n = c.by(), ch = c.bx();
    if (n >= P.nb) return;
    int g0, g1;
    KPcBase<T>::range(P, ch, g0, g1);
    const double* pt = KPcBase<T>::part(P, n);
    double r2 = 0.0, t2 = 0.0;
    for (int k = 0; k < kPcChunks; ++k) {
      r2 += pt[k];
      t2 += pt[2 * kPcChunks + k];
    }
    const double rn = sqrt(r2);
    const bool act = rn > 1e-10;
    const double sc = (act && t2 > 0.0) ? 1.0 / sqrt(t2) : 0.0;
    cplx<T>* tn = P.t + (size_t)n * P.npw;
    for (int g = g0 + c.tid(); g < g1; g += c.nthr()) {
      const cplx<T> v = tn[g];
      tn[g] = mk<T>((T)(sc * v.x), (T)(sc * v.y));
    }
    if (ch == 0 && c.tid() == 0) {
      P.act_out[n] = act ? 1 : 0;
      P.rnorm[n] = rn;
    }
  }
};

// ---------------------------------------------------------------------------
// Occupations of one subsystem (single block).
// ---------------------------------------------------------------------------
// occupation (f in [0, 2]) of a level eps at Fermi level mu: Fermi-Dirac (mode 1) or
// first-order Methfessel-Paxton (mode 2)
FDE_HD double smear(int mode, double eps, double mu, double sigma) {
  if (mode == 2) {
    const double x = (eps - mu) / sigma;
    return erfc(x) - x * exp(-x * x) * 0.56418958354775628695;  // 1/sqrt(pi)
  }
  return 1.0 - tanh((eps - mu) / (2.0 * sigma));
}

struct KOccupations {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const double* __restrict__ eval, const double* __restrict__ wk,
                         int nk, int nb, double nelec, int mode, double sigma, double* __restrict__ occw,
                         double* __restrict__ mu, int* __restrict__ info) {
    double* red = (double*)lds;
    const int tot = nk * nb;
    if (mode == 0) {
      const int nocc = (int)(nelec / 2.0);  // nelec even and whole (checked on the host)
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
      for (int e = c.tid(); e < tot; e += c.nthr()) s += wk[e / nb] * smear(mode, eval[e], m, sigma);
      s = c.sum(s, red);
      if (fabs(s - nelec) < 1e-13) break;
      if (s < nelec) lo = m;
      else hi = m;
    }
    for (int e = c.tid(); e < tot; e += c.nthr())
      occw[e] = wk[e / nb] * smear(mode, eval[e], m, sigma);
    if (c.tid() == 0) {
      mu[0] = m;
      info[0] = 0;
    }
  }
};

}  // namespace fde
