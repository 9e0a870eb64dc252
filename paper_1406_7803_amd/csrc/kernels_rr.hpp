// Rayleigh-Ritz solve of one band block held entirely in LDS (m <= kRRLdsMax),
// one workgroup per problem:
//   1. Cholesky S = L L^H, right-looking (one barrier per column), dropping
//      dependent correction columns as the global-memory solver does;
//   2. A~ = L^{-1} A L^{-H} by right-looking forward substitutions on the rows
//      (B = L^{-1} A) and on the columns (E = B L^{-H}), then made Hermitian;
//   3. cyclic parallel Jacobi on the packed Hermitian A~ (round-robin pairing,
//      m/2 disjoint rotations per round, two barriers per round), with the
//      rotations accumulated in W^T;
//   4. ascending order (ties by index), C = L^{-H} W[:, order[:nb]] by a
//      right-looking back substitution.
// KRRSolveTri (below) keeps steps 1, 2 and 4 and solves step 3 through a tridiagonal
// reduction instead of Jacobi sweeps.
// LDS: packed triangle U (m(m+1)/2 complex: L, then A~), a full work matrix M
// (m rows, padded stride m+1: the lower triangle of S during the Cholesky,
// then B/E, then W^T), and small per-pair / per-column arrays. While the
// packed triangle holds A~, the factor is parked in the problem's global L.
#pragma once

#include "kernels_la.hpp"

namespace fde {

constexpr int kRRLdsMax = 80;
// smallest m of a batch that takes the split multi-workgroup eigensolver
constexpr int kRRSplitMin = 256;
constexpr int kWRows = 15;  // row groups of the eigenvector update items

FDE_HD int tri(int i, int j) { return i * (i + 1) / 2 + j; }  // j <= i
// by-value select (a conditional between two lvalues would give v0 an address)
FDE_HD cplx<double> pick(bool c, cplx<double> a, cplx<double> b) { return c ? a : b; }

// Hermitian packed access: entries (r, c) with r >= c are stored at tri(r, c).
FDE_HD cplx<double> hget(const cplx<double>* U, int i, int j) {
  return i >= j ? U[tri(i, j)] : conj(U[tri(j, i)]);
}
FDE_HD void hset(cplx<double>* U, int i, int j, cplx<double> v) {
  if (i >= j) U[tri(i, j)] = v;
  else U[tri(j, i)] = conj(v);
}

// Round-robin schedule on mp (even) indices: in round r, pair k is (p, q).
// Over rounds 0..mp-2 every unordered pair occurs exactly once.
FDE_HD void rr_pair(int r, int k, int mp, int& p, int& q) {
  if (k == 0) {
    p = r;
    q = mp - 1;
  } else {
    p = (r + k) % (mp - 1);
    q = (r - k + (mp - 1)) % (mp - 1);
  }
}

// e / n for 0 <= e < 2^16, 1 <= n <= 2^8 through a float reciprocal:
// (e + 1/2) / n lies at least 1/(2n) from an integer, and the float product is
// within 2^-22 relative (< 0.008/n absolute) of it, so truncation is exact.
FDE_HD int qdiv(int e, float inv_n) { return (int)(((float)e + 0.5f) * inv_n); }

// Steps 1-2, shared by the LDS solvers: masks, Cholesky with dropping, A~ into the packed
// triangle U (Hermitian, lower storage); L parked in the problem's global L and its diagonal in
// sdiag. Returns false, with C = I, NaN eigenvalues and info = j + 1 written, when band column j
// has no positive pivot (uniform over the workgroup).
#if defined(__HIP_DEVICE_COMPILE__)
// Forward substitution in place on the m x m matrix M (ld = m + 1) with the packed lower
// triangle L in U: columns of B = L^{-1} M (ROWS false) or rows of E = M L^{-H} (ROWS true).
// A column (row) belongs to a group of 8 lanes; lane g keeps entries i = g + 8 s in
// registers; step i divides entry i by L_ii on its owner, broadcasts it within the group and
// removes it from the entries below. Needs 8 m threads; m <= kRRLdsMax.
template <bool ROWS>
__device__ void tri_lanes(const DevCtx& c, const cplx<double>* U, cplx<double>* M, int m) {
  constexpr int R = (kRRLdsMax + 7) / 8;
  const int ld = m + 1, g = c.tid() & 7, grp = c.tid() >> 3;
  if (grp >= m) return;  // uniform per group; no barrier inside
  cplx<double> z[R];
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const int r = g + 8 * s;
    z[s] = r < m ? M[ROWS ? (size_t)grp * ld + r : (size_t)r * ld + grp] : mk<double>(0.0, 0.0);
  }
#pragma unroll
  for (int s = 0; s < R; ++s) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int i = 8 * s + q;
      if (i >= m) break;  // uniform
      const double inv = 1.0 / U[tri(i, i)].x;
      const cplx<double> val = mk<double>(z[s].x * inv, z[s].y * inv);
      const cplx<double> bi = mk<double>(__shfl(val.x, q, 8), __shfl(val.y, q, 8));
      if (g == q) z[s] = bi;
#pragma unroll
      for (int t = s; t < R; ++t) {
        const int r = g + 8 * t;
        const bool below = r > i && r < m;
        const int rc = r < m ? r : m - 1;  // in bounds for every lane
        const cplx<double> u = U[tri(rc, i)];
        const double ly = ROWS ? -u.y : u.y;  // E: conj(L_ri)
        const double lx = below ? u.x : 0.0, lyy = below ? ly : 0.0;
        z[t].x -= lx * bi.x - lyy * bi.y;
        z[t].y -= lx * bi.y + lyy * bi.x;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const int r = g + 8 * s;
    if (r < m) M[ROWS ? (size_t)grp * ld + r : (size_t)r * ld + grp] = z[s];
  }
}

// Backward substitution C = L^{-H} W in place on the rows order[n] (n < nb) of M: a row
// belongs to a group of 8 lanes holding entries i = g + 8 s; step i (descending) divides
// entry i by L_ii on its owner, broadcasts it and removes it from the entries above.
__device__ void tri_lanes_back(const DevCtx& c, const cplx<double>* U, cplx<double>* M, int m, int nb,
                               const int* order) {
  constexpr int R = (kRRLdsMax + 7) / 8;
  const int ld = m + 1, g = c.tid() & 7, grp = c.tid() >> 3;
  if (grp >= nb) return;  // uniform per group; no barrier inside
  cplx<double>* row = M + (size_t)order[grp] * ld;
  cplx<double> z[R];
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const int r = g + 8 * s;
    z[s] = r < m ? row[r] : mk<double>(0.0, 0.0);
  }
#pragma unroll
  for (int s = R - 1; s >= 0; --s) {
#pragma unroll
    for (int q = 7; q >= 0; --q) {
      const int i = 8 * s + q;
      if (i >= m) continue;  // uniform
      const double inv = 1.0 / U[tri(i, i)].x;
      const cplx<double> val = mk<double>(z[s].x * inv, z[s].y * inv);
      const cplx<double> ci = mk<double>(__shfl(val.x, q, 8), __shfl(val.y, q, 8));
      if (g == q) z[s] = ci;
#pragma unroll
      for (int t = 0; t <= s; ++t) {
        const int r = g + 8 * t;
        const bool above = r < i;
        const cplx<double> u = U[tri(i, above ? r : i)];  // L_ir, in bounds for every lane
        const double lx = above ? u.x : 0.0, ly = above ? -u.y : 0.0;  // conj(L_ir)
        z[t].x -= lx * ci.x - ly * ci.y;
        z[t].y -= lx * ci.y + ly * ci.x;
      }
    }
  }
#pragma unroll
  for (int s = 0; s < R; ++s) {
    const int r = g + 8 * s;
    if (r < m) row[r] = z[s];
  }
}
#endif

template <typename T, class Ctx>
FDE_HD bool rr_front(const Ctx& c, const Prob<T>& a, double drop_tol, cplx<double>* U, cplx<double>* M,
                     double* sdiag, int* masked) {
  const int m = a.m, nb = a.nb, tid = c.tid(), nt = c.nthr(), ld = m + 1;
  const float inv_m = 1.0f / (float)m;
  if (tid == 0) a.info[0] = 0;
  for (int j = tid; j < m; j += nt) masked[j] = (a.active && !a.active[j]) ? 1 : 0;
  c.sync();
  // ---- lower triangle of S into M (masked columns -> e_j)
  for (int e = tid; e < m * m; e += nt) {
    const int i = qdiv(e, inv_m), j = e - i * m;
    if (j > i) continue;
    const cplx<double> v = (masked[i] || masked[j]) ? mk<double>(i == j ? 1.0 : 0.0, 0.0) : a.S[e];
    M[(size_t)i * ld + j] = v;
    if (i == j) sdiag[i] = v.x;
  }
  // ---- right-looking Cholesky into U
  for (int j = 0; j < m; ++j) {
    c.sync();
    const double d = M[(size_t)j * ld + j].x;  // S_jj - sum_k<j |L_jk|^2
    const double sjj = sdiag[j];
    if (j >= nb && !(d >= drop_tol * sjj)) {
      // dependent correction column: L column j = e_j, basis vector j dropped
      for (int k = tid; k < j; k += nt) U[tri(j, k)] = mk<double>(0, 0);
      for (int i = j + 1 + tid; i < m; i += nt) U[tri(i, j)] = mk<double>(0, 0);
      if (tid == 0) {
        U[tri(j, j)] = mk<double>(1.0, 0.0);
        masked[j] = 1;
      }
      continue;
    }
    if (!(d >= drop_tol * sjj) || !(d > 0.0)) {
      // a band column (or a non-positive pivot): report, C = identity
      if (tid == 0) a.info[0] = j + 1;
      for (int e = tid; e < m * nb; e += nt) {
        const int i = e / nb, n = e - i * nb;
        const cplx<double> v = mk<double>(i == n ? 1.0 : 0.0, 0.0);
        a.Cd[e] = v;
        ((cplx<T>*)a.Ct)[e] = mk<T>((T)v.x, (T)v.y);
      }
      for (int n = tid; n < nb; n += nt) a.eval[n] = 0.0 / 0.0;
      return false;  // uniform: every thread read the same d
    }
    const double ljj = sqrt(d), inv_d = 1.0 / d;
    if (tid == 0) U[tri(j, j)] = mk<double>(ljj, 0.0);
    for (int i = j + 1 + tid; i < m; i += nt) U[tri(i, j)] = cdiv_real(M[(size_t)i * ld + j], ljj);
    // trailing update of the lower triangle: M_ik -= M_ij conj(M_kj) / d, j < k <= i
    const int n = m - 1 - j;
    const float inv_n = 1.0f / (float)(n > 0 ? n : 1);
    for (int e = tid; e < n * n; e += nt) {
      const int ii = qdiv(e, inv_n), kk = e - ii * n;
      if (kk > ii) continue;
      const int i = j + 1 + ii, k = j + 1 + kk;
      const cplx<double> lij = M[(size_t)i * ld + j], lkj = M[(size_t)k * ld + j];
      cplx<double>& t = M[(size_t)i * ld + k];
      t.x -= (lij.x * lkj.x + lij.y * lkj.y) * inv_d;
      t.y -= (lij.y * lkj.x - lij.x * lkj.y) * inv_d;
    }
  }
  c.sync();
  // ---- A into M (masked / dropped columns -> 1e6 e_j)
  for (int e = tid; e < m * m; e += nt) {
    const int i = qdiv(e, inv_m), j = e - i * m;
    M[(size_t)i * ld + j] = (masked[i] || masked[j]) ? mk<double>(i == j ? kInactiveDiag : 0.0, 0.0) : a.A[e];
  }
#if defined(__HIP_DEVICE_COMPILE__)
  // ---- B = L^{-1} A by columns, then E = B L^{-H} by rows, each in registers of 8-lane groups
  c.sync();
  tri_lanes<false>(c, U, M, m);
  c.sync();
  tri_lanes<true>(c, U, M, m);
  c.sync();
#else
  // ---- B = L^{-1} A: step i removes row i's contribution from the rows below
  for (int i = 0; i < m; ++i) {
    c.sync();
    const double inv_lii = 1.0 / U[tri(i, i)].x;
    const int n = m - 1 - i;
    for (int e = tid; e < n * m; e += nt) {
      const int rr = qdiv(e, inv_m), col = e - rr * m;
      const int r = i + 1 + rr;
      const cplx<double> l = U[tri(r, i)];
      const cplx<double> bi = M[(size_t)i * ld + col];
      cplx<double>& t = M[(size_t)r * ld + col];
      t = t - (inv_lii * l) * bi;
    }
  }
  c.sync();
  for (int e = tid; e < m * m; e += nt) {
    const int i = qdiv(e, inv_m), j = e - i * m;
    M[(size_t)i * ld + j] = cdiv_real(M[(size_t)i * ld + j], U[tri(i, i)].x);
  }
  // ---- E = B L^{-H}: step j removes column j's contribution from the columns right of it
  for (int j = 0; j < m; ++j) {
    c.sync();
    const double inv_ljj = 1.0 / U[tri(j, j)].x;
    const int n = m - 1 - j;
    const float inv_n = 1.0f / (float)(n > 0 ? n : 1);
    for (int e = tid; e < n * m; e += nt) {
      const int r = qdiv(e, inv_n), kk = e - r * n;
      const int k = j + 1 + kk;
      const cplx<double> l = conj(U[tri(k, j)]);
      const cplx<double> ej = M[(size_t)r * ld + j];
      cplx<double>& t = M[(size_t)r * ld + k];
      t = t - (inv_ljj * ej) * l;
    }
  }
  c.sync();
  for (int e = tid; e < m * m; e += nt) {  // E_ij = M_ij / L_jj
    const int i = qdiv(e, inv_m), j = e - i * m;
    M[(size_t)i * ld + j] = cdiv_real(M[(size_t)i * ld + j], U[tri(j, j)].x);
  }
  c.sync();
#endif
  // ---- park L in global memory (its diagonal also in sdiag); A~ = (E + E^H)/2 into U
  for (int e = tid; e < m * (m + 1) / 2; e += nt) a.L[e] = U[e];
  for (int i = tid; i < m; i += nt) sdiag[i] = U[tri(i, i)].x;
  c.sync();
  for (int e = tid; e < m * m; e += nt) {
    const int i = qdiv(e, inv_m), j = e - i * m;
    if (j > i) continue;
    const cplx<double> eij = M[(size_t)i * ld + j];
    const cplx<double> eji = M[(size_t)j * ld + i];
    U[tri(i, j)] = i == j ? mk<double>(eij.x, 0.0) : mk<double>(0.5 * (eji.x + eij.x), 0.5 * (eij.y - eji.y));
  }
  c.sync();
  return true;
}

// Step 4, shared by the LDS solvers: eigenvalues theta[order[n]] and C = L^{-H} W[:, order[:nb]]
// by a right-looking back substitution in place in the W^T rows of M (stride m + 1); L is
// restored from the problem's global L into U.
template <typename T, class Ctx>
FDE_HD void rr_tail(const Ctx& c, const Prob<T>& a, cplx<double>* U, cplx<double>* M, const double* sdiag,
                    const int* order) {
  const int m = a.m, nb = a.nb, tid = c.tid(), nt = c.nthr(), ld = m + 1;
  c.sync();
  // ---- restore L; C = L^{-H} W[:, order[:nb]] in place in the W^T rows
  for (int e = tid; e < m * (m + 1) / 2; e += nt) U[e] = a.L[e];
  for (int n = tid; n < nb; n += nt) a.eval[n] = a.theta[order[n]];
  const float inv_nb = 1.0f / (float)nb;
#if defined(__HIP_DEVICE_COMPILE__)
  c.sync();
  tri_lanes_back(c, U, M, m, nb, order);  // C rows divided by L_ii
  c.sync();
  for (int e = tid; e < m * nb; e += nt) {
    const int i = qdiv(e, inv_nb), n = e - i * nb;
    const cplx<double> v = M[(size_t)order[n] * ld + i];
#else
  for (int i = m - 1; i >= 0; --i) {
    c.sync();
    // row i of C is final: C_i = W_i / L_ii; remove it from the rows above
    const double inv_lii = 1.0 / sdiag[i];
    for (int e = tid; e < i * nb; e += nt) {
      const int r = qdiv(e, inv_nb), n = e - r * nb;
      const int col = order[n];
      const cplx<double> l = conj(U[tri(i, r)]);
      const cplx<double> ci = M[(size_t)col * ld + i];
      cplx<double>& t = M[(size_t)col * ld + r];
      t = t - (inv_lii * l) * ci;
    }
  }
  c.sync();
  for (int e = tid; e < m * nb; e += nt) {
    const int i = qdiv(e, inv_nb), n = e - i * nb;
    const cplx<double> v = cdiv_real(M[(size_t)order[n] * ld + i], sdiag[i]);
#endif
    a.Cd[e] = v;
    ((cplx<T>*)a.Ct)[e] = mk<T>((T)v.x, (T)v.y);
  }
}

template <typename T>
struct KRRSolveLds {
  FDE_HD static size_t lds_bytes(int m) {
    const int mp = m + (m & 1), npair = mp / 2;
    const int nblk = npair * (npair - 1) / 2;
    size_t b = sizeof(cplx<double>) * ((size_t)m * (m + 1) / 2 + (size_t)m * (m + 1));
    b += sizeof(double) * (32 + 8 * (size_t)npair + m);   // red, rotations (two rounds), diag of S
    b += sizeof(int) * (2 * (size_t)m + 4 * (size_t)npair);  // masked, order, pair tables (two rounds)
    b += sizeof(unsigned short) * ((size_t)nblk + 2);
    return b + 64;
  }

  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps) {
    const Prob<T>& a = ps.p[c.bx()];
    const int m = a.m, nb = a.nb;
    const int mp = m + (m & 1), npair = mp / 2;
    const int nblk = npair * (npair - 1) / 2;
    const int tid = c.tid(), nt = c.nthr();
    const double drop_tol = ps.drop_tol;
    const int ld = m + 1;  // padded row stride of M
    cplx<double>* U = (cplx<double>*)lds;
    cplx<double>* M = U + (size_t)m * (m + 1) / 2;
    double* red = (double*)(M + (size_t)m * ld);
    double* rot = red + 32;          // [2 rounds][4][npair]: c, s, Re e^{i phi}, Im e^{i phi}
    double* sdiag = rot + 8 * npair; // S_jj after masking
    int* masked = (int*)(sdiag + m);
    int* order = masked + m;
    int* ptab = order + m;           // [2 rounds][2][npair]: the pairs (p, q)
    unsigned short* blk = (unsigned short*)(ptab + 4 * npair);  // block item -> K | Q << 8
    const float inv_m = 1.0f / (float)m;

    if (!rr_front<T>(c, a, drop_tol, U, M, sdiag, masked)) return;
    // ---- W^T = I in M; block-item table
    for (int e = tid; e < m * m; e += nt) {
      const int i = qdiv(e, inv_m), j = e - i * m;
      M[(size_t)i * ld + j] = mk<double>(i == j ? 1.0 : 0.0, 0.0);
    }
    for (int it = tid; it < nblk; it += nt) {
      // row K of the strictly upper pair triangle starts at K (2 npair - K - 1) / 2
      int K = 0;
      while ((K + 1) * (2 * npair - K - 2) / 2 <= it) ++K;
      const int Q = K + 1 + (it - K * (2 * npair - K - 1) / 2);
      blk[it] = (unsigned short)(K | (Q << 8));
    }
    c.sync();
    // ---- cyclic parallel Jacobi on the packed Hermitian A~. Round r's rotations are computed by
    //      the first wavefront while the others apply round r-1's rotations to the W^T rows
    //      (rotation parameters double-buffered by round parity); then the 2 x 2 blocks.
    bool conv = false;
    double prev_off = 1e300;
    int rg = 0;  // rounds done
    const int wbase = nt > 64 ? 64 : 0, wstride = nt > 64 ? nt - 64 : nt;
    auto w_update = [&](int buf) {  // W^T rows p, q of every pair, rotated by round `buf`'s parameters
      const double* rc = rot + buf * 4 * npair;
      const double* rs = rc + npair;
      const double* rex = rs + npair;
      const double* rey = rex + npair;
      const int* pp = ptab + buf * 2 * npair;
      const int* pq = pp + npair;
      for (int e = tid - wbase; e >= 0 && e < npair * kWRows; e += wstride) {
        const int K = e / kWRows, i0 = e - K * kWRows;
        if (rs[K] == 0.0) continue;
        const int p = pp[K], q = pq[K];
        const double cc = rc[K], ss = rs[K];
        const cplx<double> em = mk<double>(rex[K], -rey[K]);
        cplx<double>* wpr = M + (size_t)p * ld;
        cplx<double>* wqr = M + (size_t)q * ld;
        for (int ib = i0; ib < m; ib += 4 * kWRows) {
          cplx<double> xp[4], xq[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = ib + u * kWRows;
            if (i < m) {
              xp[u] = wpr[i];
              xq[u] = wqr[i];
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int i = ib + u * kWRows;
            if (i < m) {
              const cplx<double> emq = em * xq[u];
              wpr[i] = mk<double>(cc * xp[u].x - ss * emq.x, cc * xp[u].y - ss * emq.y);
              wqr[i] = mk<double>(ss * xp[u].x + cc * emq.x, ss * xp[u].y + cc * emq.y);
            }
          }
        }
      }
    };
    for (int sweep = 0; sweep < 40 && !conv; ++sweep) {
      for (int r = 0; r < mp - 1; ++r, ++rg) {
        const int buf = rg & 1;
        double* rc = rot + buf * 4 * npair;
        double* rs = rc + npair;
        double* rex = rs + npair;
        double* rey = rex + npair;
        int* pp = ptab + buf * 2 * npair;
        int* pq = pp + npair;
        // rotation of each pair; the pair's own 2 x 2 block is updated here
        if (tid < 64) {
          for (int k = tid; k < npair; k += (nt < 64 ? nt : 64)) {
            int p, q;
            rr_pair(r, k, mp, p, q);
            pp[k] = p;
            pq[k] = q;
            double cc = 1.0, ss = 0.0, ex = 1.0, ey = 0.0;
            if (p < m && q < m) {
              const cplx<double> bpq = hget(U, p, q);
              const double app = U[tri(p, p)].x, aqq = U[tri(q, q)].x;
              const double ab = sqrt(norm2(bpq));
              if (ab > 1e-300) {
                const double th = (aqq - app) / (2.0 * ab);
                const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                cc = 1.0 / sqrt(t * t + 1.0);
                ss = t * cc;
                ex = bpq.x / ab;
                ey = bpq.y / ab;
                U[tri(p, p)] = mk<double>(app - t * ab, 0.0);
                U[tri(q, q)] = mk<double>(aqq + t * ab, 0.0);
                hset(U, p, q, mk<double>(0.0, 0.0));
              }
            }
            rc[k] = cc;
            rs[k] = ss;
            rex[k] = ex;
            rey[k] = ey;
          }
        }
        if (rg > 0) w_update(buf ^ 1);
        c.sync();
        // off-diagonal 2 x 2 blocks (pairs K < Q): B' = G_K^H B G_Q
        for (int it = tid; it < nblk; it += nt) {
          const int K = blk[it] & 255, Q = blk[it] >> 8;
          const bool rotK = rs[K] != 0.0, rotQ = rs[Q] != 0.0;
          if (!rotK && !rotQ) continue;
          const int p = pp[K], q = pq[K], p2 = pp[Q], q2 = pq[Q];
          // rows {p, q} (one may be the dummy index m when m is odd), cols {p2, q2}
          cplx<double> b00 = (p < m && p2 < m) ? hget(U, p, p2) : mk<double>(0, 0);
          cplx<double> b01 = (p < m && q2 < m) ? hget(U, p, q2) : mk<double>(0, 0);
          cplx<double> b10 = (q < m && p2 < m) ? hget(U, q, p2) : mk<double>(0, 0);
          cplx<double> b11 = (q < m && q2 < m) ? hget(U, q, q2) : mk<double>(0, 0);
          if (rotK) {  // rows: [c, -s e^{i phi}; s, c e^{i phi}]
            const double c1 = rc[K], s1 = rs[K];
            const cplx<double> ep = mk<double>(rex[K], rey[K]);
            const cplx<double> e10 = ep * b10, e11 = ep * b11;
            const cplx<double> n00 = mk<double>(c1 * b00.x - s1 * e10.x, c1 * b00.y - s1 * e10.y);
            const cplx<double> n01 = mk<double>(c1 * b01.x - s1 * e11.x, c1 * b01.y - s1 * e11.y);
            const cplx<double> n10 = mk<double>(s1 * b00.x + c1 * e10.x, s1 * b00.y + c1 * e10.y);
            const cplx<double> n11 = mk<double>(s1 * b01.x + c1 * e11.x, s1 * b01.y + c1 * e11.y);
            b00 = n00;
            b01 = n01;
            b10 = n10;
            b11 = n11;
          }
          if (rotQ) {  // columns: [c, s; -s e^{-i phi}, c e^{-i phi}]
            const double c2 = rc[Q], s2 = rs[Q];
            const cplx<double> em = mk<double>(rex[Q], -rey[Q]);
            const cplx<double> f01 = em * b01, f11 = em * b11;
            const cplx<double> n00 = mk<double>(c2 * b00.x - s2 * f01.x, c2 * b00.y - s2 * f01.y);
            const cplx<double> n01 = mk<double>(s2 * b00.x + c2 * f01.x, s2 * b00.y + c2 * f01.y);
            const cplx<double> n10 = mk<double>(c2 * b10.x - s2 * f11.x, c2 * b10.y - s2 * f11.y);
            const cplx<double> n11 = mk<double>(s2 * b10.x + c2 * f11.x, s2 * b10.y + c2 * f11.y);
            b00 = n00;
            b01 = n01;
            b10 = n10;
            b11 = n11;
          }
          if (p < m && p2 < m) hset(U, p, p2, b00);
          if (p < m && q2 < m) hset(U, p, q2, b01);
          if (q < m && p2 < m) hset(U, q, p2, b10);
          if (q < m && q2 < m) hset(U, q, q2, b11);
        }
        c.sync();
      }
      double off = 0.0, dia = 0.0;
      for (int e = tid; e < m * m; e += nt) {
        const int i = qdiv(e, inv_m), j = e - i * m;
        if (j > i || masked[i] || masked[j]) continue;
        const double v = sqrt(norm2(U[tri(i, j)]));
        if (i == j) dia = dia > v ? dia : v;
        else off = off > v ? off : v;
      }
      off = c.max(off, red);
      dia = c.max(dia, red);
      const double scale = dia > 1e-300 ? dia : 1e-300;
      conv = off <= 1e-14 * scale || (off <= 1e-12 * scale && off > 0.5 * prev_off);
      prev_off = off;
      if (sweep == 39 && !conv && tid == 0) a.info[0] = -1;
    }
    if (rg > 0) w_update((rg - 1) & 1);  // the last round's rotations
    c.sync();
    // ---- eigenvalues, ascending order (ties by index)
    for (int i = tid; i < m; i += nt) a.theta[i] = U[tri(i, i)].x;
    c.sync();
    for (int i = tid; i < m; i += nt) {
      const double ti = a.theta[i];
      int rank = 0;
      for (int j = 0; j < m; ++j) {
        const double tj = a.theta[j];
        if (tj < ti || (tj == ti && j < i)) ++rank;
      }
      order[rank] = i;
    }
    rr_tail<T>(c, a, U, M, sdiag, order);
  }
};

// Rayleigh-Ritz solve of one band block in LDS with the eigenproblem of A~ reduced to a real
// tridiagonal (used when the block fits; steps 1, 2 and 4 as in KRRSolveLds):
//   3a. the active part of A~ (masked indices dropped) compacted into U; Householder reduction
//       with reflectors H_k = I - beta_k v_k v_k^H kept in place below the subdiagonal, two
//       barriers per column;
//   3b. the complex subdiagonal alpha made real by a diagonal phase D;
//   3c. the nw lowest eigenvalues by multisection on Sturm counts (nt / nw points per
//       eigenvalue and step);
//   3d. their eigenvectors by inverse iteration (partial-pivoting LU of T - lambda I, three
//       solves from a fixed pseudo-random start), one wavefront per cluster of close
//       eigenvalues, each solve orthogonalised against the cluster's earlier vectors;
//   3e. back-transformation W = Q D Y by groups of 16 lanes, one eigenvector per group, and
//       the rows scattered back to the physical indices.
// Inside M once A~ is reduced: region R1 (compaction buffer, then Sturm counts, then the
// per-wavefront LU factors, then the W^T rows), the tridiagonal eigenvectors Y [nw][ma], and the
// per-column arrays.
template <typename T>
struct KRRSolveTri {
  static constexpr int kThreads = 1024;
  static constexpr int kWaves = kThreads / 64;
  static constexpr int kGroup = 16;
  static constexpr int kInvIt = 3;
  static constexpr int kBigCluster = 16;  // larger clusters: vectors in parallel, then orthonormalised
  static constexpr int kMsPoints = 7;  // multisection points per eigenvalue and step

  FDE_HD static size_t lu_stride(int m) { return ((size_t)m * (4 * sizeof(double) + 1) + 15) & ~(size_t)15; }
  FDE_HD static size_t r1_bytes(int m, int nb) {
    size_t r = (size_t)nb * (m + 1) * sizeof(cplx<double>);
    const size_t lu = (size_t)kWaves * lu_stride(m), cnt = (size_t)kThreads * sizeof(int);
    const size_t pk = (size_t)m * (m + 1) / 2 * sizeof(cplx<double>);
    r = r > lu ? r : lu;
    r = r > cnt ? r : cnt;
    r = r > pk ? r : pk;
    return (r + 255) & ~(size_t)255;
  }
  FDE_HD static size_t y_bytes(int m, int nb) { return ((size_t)m * nb * sizeof(double) + 15) & ~(size_t)15; }
  FDE_HD static size_t small_bytes(int m) { return (size_t)m * (17 * sizeof(double) + 2 * sizeof(int)) + 64; }
  // column-packed offset of the reflector vector v_k (ma - k - 1 entries) in U
  FDE_HD static int voff(int k, int ma) { return k * (ma - 1) - k * (k - 1) / 2; }
  FDE_HD static size_t mspan(int m, int nb) {
    const size_t mb = (size_t)m * (m + 1) * sizeof(cplx<double>);
    const size_t need = r1_bytes(m, nb) + y_bytes(m, nb) + small_bytes(m);
    return ((mb > need ? mb : need) + 15) & ~(size_t)15;
  }
  FDE_HD static size_t lds_bytes(int m, int nb) {
    return sizeof(cplx<double>) * ((size_t)m * (m + 1) / 2) + mspan(m, nb) + sizeof(double) * (32 + (size_t)m) +
           sizeof(int) * 2 * (size_t)m + 64;
  }

  // fixed pseudo-random start vector entry in [-1, 1)
  FDE_HD static double start_value(int i, int j) {
    unsigned h = (unsigned)i * 73856093u ^ (unsigned)j * 19349663u ^ 0x9e3779b9u;
    h ^= h >> 16;
    h *= 0x7feb352du;
    h ^= h >> 15;
    h *= 0x846ca68bu;
    h ^= h >> 16;
    return (double)(h >> 8) * (2.0 / 16777216.0) - 1.0;
  }

  // LU with partial pivoting of the n x n tridiagonal T - lam I (diagonal dg, off-diagonal ea):
  // reciprocal pivots, the two superdiagonals of U, the multipliers and the interchange flags.
  // Pivots below tiny in magnitude are replaced by +-tiny. The running row stays in registers.
  template <class Ctx>
  FDE_HD static void lu_factor(int n, const double* dg, const double* ea, double lam, double tiny, double* lu,
                               unsigned char* piv) {
    double *ru0 = lu, *u1 = lu + n, *u2 = lu + 2 * n, *ml = lu + 3 * n;
    double cd = dg[0] - lam, cs = n > 1 ? ea[0] : 0.0;  // current row: (i, i), (i, i + 1)
#pragma unroll 4
    for (int i = 0; i < n - 1; ++i) {
      const double sub = ea[i], dn = dg[i + 1] - lam, sn = i + 2 < n ? ea[i + 1] : 0.0;
      if (fabs(cd) >= fabs(sub)) {
        const double pv = fabs(cd) < tiny ? (cd < 0.0 ? -tiny : tiny) : cd;
        const double rp = Ctx::rcp(pv);
        const double l = sub * rp;
        ru0[i] = rp;
        u1[i] = cs;
        u2[i] = 0.0;
        ml[i] = l;
        piv[i] = 0;
        cd = dn - l * cs;
        cs = sn;
      } else {
        const double rp = Ctx::rcp(sub);
        const double l = cd * rp;
        ru0[i] = rp;
        u1[i] = dn;
        u2[i] = sn;
        ml[i] = l;
        piv[i] = 1;
        cd = cs - l * dn;
        cs = -l * sn;
      }
    }
    ru0[n - 1] = Ctx::rcp(fabs(cd) < tiny ? (cd < 0.0 ? -tiny : tiny) : cd);
  }

  // b <- (T - lam I)^{-1} b with the factors of lu_factor (running values in registers). Each
  // pass loads kC entries of b and the factors ahead of the stores they precede (a store to b
  // could otherwise alias the next loads and serialise them); every load reads the value the
  // entry held before this pass stored to it, as a one-at-a-time order would.
  FDE_HD static void lu_solve(int n, const double* lu, const unsigned char* piv, double* b) {
    constexpr int kC = 8;
    const double *ru0 = lu, *u1 = lu + n, *u2 = lu + 2 * n, *ml = lu + 3 * n;
    double cur = b[0];
    for (int i0 = 0; i0 < n - 1; i0 += kC) {
      double nx[kC], mc[kC];
      bool pc[kC];
#pragma unroll
      for (int t = 0; t < kC; ++t) {
        const int i = i0 + t < n - 1 ? i0 + t : n - 2;
        nx[t] = b[i + 1];
        mc[t] = ml[i];
        pc[t] = piv[i] != 0;
      }
#pragma unroll
      for (int t = 0; t < kC; ++t) {
        const int i = i0 + t;
        if (i >= n - 1) break;
        if (pc[t]) {
          b[i] = nx[t];
          cur = cur - mc[t] * nx[t];
        } else {
          b[i] = cur;
          cur = nx[t] - mc[t] * cur;
        }
      }
    }
    double x1 = cur * ru0[n - 1], x2 = 0.0;  // x_{i+1}, x_{i+2}
    b[n - 1] = x1;
    for (int i0 = n - 2; i0 >= 0; i0 -= kC) {
      double bc[kC], a1[kC], a2[kC], rc[kC];
#pragma unroll
      for (int t = 0; t < kC; ++t) {
        const int i = i0 - t > 0 ? i0 - t : 0;
        bc[t] = b[i];
        a1[t] = u1[i];
        a2[t] = u2[i];
        rc[t] = ru0[i];
      }
#pragma unroll
      for (int t = 0; t < kC; ++t) {
        const int i = i0 - t;
        if (i < 0) break;
        const double x = (bc[t] - a1[t] * x1 - a2[t] * x2) * rc[t];
        b[i] = x;
        x2 = x1;
        x1 = x;
      }
    }
  }

  // Householder reduction in LDS (host twin of house_regs): the active part compacted into U
  // (logical index i <-> physical act[i]), reduced in place, then the reflector vectors moved to
  // their column-packed slots voff(k) and the diagonal into dg.
  template <class Ctx>
  FDE_HD static void house_lds(const Ctx& c, cplx<double>* U, char* r1, int m, int ma, const int* act, double* dg,
                               double* beta, double* ar, double* ai, double* pbx, double* pby) {
    const int tid = c.tid(), nt = c.nthr();
    const int lane = c.lane(), wl = c.wlanes(), wv = c.wave(), nwv = c.nwave();
    if (ma < m) {
      cplx<double>* P = (cplx<double>*)r1;
      for (int e = tid; e < ma * (ma + 1) / 2; e += nt) {
        int i = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
        if ((i + 1) * (i + 2) / 2 <= e) ++i;
        if (i * (i + 1) / 2 > e) --i;
        P[e] = U[tri(act[i], act[e - i * (i + 1) / 2])];
      }
      c.sync();
      for (int e = tid; e < ma * (ma + 1) / 2; e += nt) U[e] = P[e];
      c.sync();
    }
    // column k: x = A~(k+1.., k); H_k x = alpha e_1
    for (int k = 0; k + 1 < ma; ++k) {
      const int n1 = ma - k - 1;
      const cplx<double>* xc = U + tri(k + 1, k);  // x_r at xc[tri(k + 1 + r, k) - tri(k + 1, k)]
      double s2 = 0.0;
      for (int r = lane; r < n1; r += wl) s2 += norm2(U[tri(k + 1 + r, k)]);
      s2 = c.template gsum<64>(s2);
      const cplx<double> x0 = xc[0];
      double bt = 0.0;
      cplx<double> alpha = x0, v0 = x0;
      if (n1 > 1 && s2 > norm2(x0)) {
        const double ax0 = sqrt(norm2(x0)), sg = sqrt(s2);
        const cplx<double> ph = ax0 > 0.0 ? mk<double>(x0.x / ax0, x0.y / ax0) : mk<double>(1.0, 0.0);
        alpha = mk<double>(-ph.x * sg, -ph.y * sg);
        v0 = mk<double>(x0.x + ph.x * sg, x0.y + ph.y * sg);
        bt = 1.0 / (sg * (sg + ax0));
      }
      if (tid == 0) {
        beta[k] = bt;
        ar[k] = alpha.x;
        ai[k] = alpha.y;
      }
      if (bt != 0.0) {  // uniform: every wavefront summed in the same order
        // p = beta A' v over the trailing block, one row per wavefront at a time
        for (int r = wv; r < n1; r += nwv) {
          const int ir = k + 1 + r;
          double sx = 0.0, sy = 0.0;
          for (int j = lane; j < n1; j += wl) {
            const int ij = k + 1 + j;
            const cplx<double> vj = pick(j == 0, v0, U[tri(ij, k)]);
            const cplx<double> arj = ir >= ij ? U[tri(ir, ij)] : conj(U[tri(ij, ir)]);
            sx += arj.x * vj.x - arj.y * vj.y;
            sy += arj.x * vj.y + arj.y * vj.x;
          }
          sx = c.template gsum<64>(sx);
          sy = c.template gsum<64>(sy);
          if (lane == 0) {
            pbx[r] = bt * sx;
            pby[r] = bt * sy;
          }
        }
        c.sync();
        // K = beta/2 v^H p (real), then A' -= v w^H + w v^H with w = p - K v, lower triangle
        double kk = 0.0;
        for (int r = lane; r < n1; r += wl) {
          const cplx<double> vr = pick(r == 0, v0, U[tri(k + 1 + r, k)]);
          kk += vr.x * pbx[r] + vr.y * pby[r];
        }
        kk = 0.5 * bt * c.template gsum<64>(kk);
        const int ntri = n1 * (n1 + 1) / 2;
        for (int e = tid; e < ntri; e += nt) {
          int r = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
          if ((r + 1) * (r + 2) / 2 <= e) ++r;
          if (r * (r + 1) / 2 > e) --r;
          const int j = e - r * (r + 1) / 2;
          const cplx<double> vr = pick(r == 0, v0, U[tri(k + 1 + r, k)]);
          const cplx<double> vj = pick(j == 0, v0, U[tri(k + 1 + j, k)]);
          const double wrx = pbx[r] - kk * vr.x, wry = pby[r] - kk * vr.y;
          const double wjx = pbx[j] - kk * vj.x, wjy = pby[j] - kk * vj.y;
          cplx<double>& t = U[tri(k + 1 + r, k + 1 + j)];
          t.x -= (vr.x * wjx + vr.y * wjy) + (wrx * vj.x + wry * vj.y);
          t.y -= (vr.y * wjx - vr.x * wjy) + (wry * vj.x - wrx * vj.y);
        }
        if (tid == 0) U[tri(k + 1, k)] = v0;
      }
      c.sync();
    }
    // reflector vectors to their column-packed slots (through r1), diagonal to dg
    cplx<double>* P = (cplx<double>*)r1;
    for (int k = wv; k + 1 < ma; k += nwv)
      for (int r = lane; r < ma - k - 1; r += wl) P[voff(k, ma) + r] = U[tri(k + 1 + r, k)];
    for (int k = tid; k < ma; k += nt) dg[k] = U[tri(k, k)].x;
    c.sync();
    for (int e = tid; e < ma * (ma - 1) / 2; e += nt) U[e] = P[e];
    c.sync();
  }

#if defined(__HIP_DEVICE_COMPILE__)
  // Householder reduction with the active block in registers (1024 threads): row i on lane
  // i % 64 (slot i / 64), column j on wavefront j / kCPW (slot j % kCPW). Step k: every
  // wavefront forms partial sums of A' v over its columns (LDS, [wavefront][row]); the rows'
  // sums in a fixed order give p = beta A' v and the wavefront sums of Re(v^H p) give K; every
  // wavefront applies A' -= v w^H + w v^H to its columns; the owner of column k + 1 then forms
  // the next reflector (v through LDS, double-buffered). Three barriers per column.
  static constexpr int kRT = (kRRLdsMax + 63) / 64;                // row slots per lane
  static constexpr int kCPW = (kRRLdsMax + kWaves - 1) / kWaves;    // columns per wavefront
  __device__ static void house_regs(const DevCtx& c, cplx<double>* U, char* r1, int m, int ma, const int* act,
                                    double* dg, double* beta, double* ar, double* ai, cplx<double>* xb,
                                    double* pbx, double* pby) {
    const int tid = c.tid(), lane = c.lane(), wv = c.wave();
    cplx<double>* part = (cplx<double>*)r1;  // [kWaves][m]
    double* kpart = (double*)(part + (size_t)kWaves * m);  // [2]
    cplx<double> A[kRT][kCPW];
#pragma unroll
    for (int t = 0; t < kRT; ++t)
#pragma unroll
      for (int s = 0; s < kCPW; ++s) {
        const int i = lane + 64 * t, j = kCPW * wv + s;
        A[t][s] = (i < ma && j < ma) ? hget(U, act[i], act[j]) : mk<double>(0.0, 0.0);
      }
    c.sync();  // U is free from here on: it receives the reflector vectors
    // the owner of column k: diagonal entry, reflector of the column below it into xv and U
    auto gen = [&](int k, cplx<double>* xv) {
#pragma unroll
      for (int s = 0; s < kCPW; ++s) {
        if (kCPW * wv + s != k) continue;  // uniform
        double loc = 0.0;
#pragma unroll
        for (int t = 0; t < kRT; ++t) {
          const int i = lane + 64 * t;
          if (i == k) dg[k] = A[t][s].x;
          if (i > k && i < ma) loc += norm2(A[t][s]);
        }
        if (k + 1 >= ma) return;
        const double s2 = c.gsum<64>(loc);
        cplx<double> x0 = mk<double>(0.0, 0.0);
#pragma unroll
        for (int t = 0; t < kRT; ++t)
          if ((k + 1) / 64 == t) x0 = mk<double>(DevCtx::rdlane(A[t][s].x, (k + 1) & 63),
                                                 DevCtx::rdlane(A[t][s].y, (k + 1) & 63));
        double bt = 0.0;
        cplx<double> alpha = x0, v0 = x0;
        const double n0 = norm2(x0);
        if (k + 2 < ma && s2 > n0) {
          // |x0|, sigma and beta from reciprocal square roots / reciprocals with Newton steps
          const double r0 = n0 > 0.0 ? DevCtx::rsq(n0) : 0.0, rs = DevCtx::rsq(s2);
          const double ax0 = n0 * r0, sg = s2 * rs;
          const cplx<double> ph = n0 > 0.0 ? mk<double>(x0.x * r0, x0.y * r0) : mk<double>(1.0, 0.0);
          alpha = mk<double>(-ph.x * sg, -ph.y * sg);
          v0 = mk<double>(x0.x + ph.x * sg, x0.y + ph.y * sg);
          bt = DevCtx::rcp(sg * (sg + ax0));
        }
        const int vo = voff(k, ma) - (k + 1);
#pragma unroll
        for (int t = 0; t < kRT; ++t) {
          const int i = lane + 64 * t;
          if (i > k && i < ma) {
            const cplx<double> v = pick(i == k + 1, v0, A[t][s]);
            xv[i] = v;
            U[vo + i] = v;
          }
        }
        if (lane == 0) {
          beta[k] = bt;
          ar[k] = alpha.x;
          ai[k] = alpha.y;
        }
      }
    };
    gen(0, xb);
    c.sync();
    for (int k = 0; k + 1 < ma; ++k) {
      const cplx<double>* xk = xb + (k & 1) * m;
      cplx<double>* xn = xb + ((k + 1) & 1) * m;
      const double bt = beta[k];
      if (bt != 0.0) {  // uniform
        // partial sums of A' v over this wavefront's columns
        // columns of this wavefront inside the trailing block: j in [jlo, jhi) (uniform)
        const int jlo = kCPW * wv > k + 1 ? kCPW * wv : k + 1;
        const int jhi = kCPW * wv + kCPW < ma ? kCPW * wv + kCPW : ma;
        cplx<double> vs[kCPW];
#pragma unroll
        for (int s = 0; s < kCPW; ++s) {
          const int j = kCPW * wv + s;
          vs[s] = (j >= jlo && j < jhi) ? xk[j] : mk<double>(0.0, 0.0);
        }
#pragma unroll
        for (int t = 0; t < kRT; ++t) {
          if (64 * t >= ma || 64 * t + 63 <= k) continue;  // no trailing row in this slot (uniform)
          const int i = lane + 64 * t;
          double sx = 0.0, sy = 0.0;
#pragma unroll
          for (int s = 0; s < kCPW; ++s) {
            const int j = kCPW * wv + s;
            if (j >= jlo && j < jhi) {  // uniform
              sx += A[t][s].x * vs[s].x - A[t][s].y * vs[s].y;
              sy += A[t][s].x * vs[s].y + A[t][s].y * vs[s].x;
            }
          }
          if (i > k && i < ma) part[(size_t)wv * m + i] = mk<double>(sx, sy);
        }
        c.sync();
        // p_i = beta sum_w part[w][i]; K partials Re(conj(v_i) p_i) summed per wavefront
        if (wv < kRT) {  // threads tid < 64 kRT cover every row
          double kv = 0.0;
          const int i = tid;
          if (i > k && i < ma) {
            double sx = 0.0, sy = 0.0;
            for (int w = 0; w < kWaves; ++w) {
              const cplx<double> q = part[(size_t)w * m + i];
              sx += q.x;
              sy += q.y;
            }
            sx *= bt;
            sy *= bt;
            pbx[i] = sx;
            pby[i] = sy;
            const cplx<double> vi = xk[i];
            kv = vi.x * sx + vi.y * sy;
          }
          kv = c.gsum<64>(kv);
          if (lane == 0) kpart[wv] = kv;
        }
        c.sync();
        double kk = 0.0;
        for (int w = 0; w < kRT; ++w) kk += kpart[w];
        kk *= 0.5 * bt;
        if (jlo < jhi) {  // uniform: this wavefront has trailing columns
          cplx<double> ws[kCPW];
#pragma unroll
          for (int s = 0; s < kCPW; ++s) {
            const int j = kCPW * wv + s;
            ws[s] = (j >= jlo && j < jhi) ? mk<double>(pbx[j] - kk * vs[s].x, pby[j] - kk * vs[s].y)
                                          : mk<double>(0.0, 0.0);
          }
#pragma unroll
          for (int t = 0; t < kRT; ++t) {
            if (64 * t >= ma || 64 * t + 63 <= k) continue;  // uniform
            const int i = lane + 64 * t;
            const cplx<double> vi = (i > k && i < ma) ? xk[i] : mk<double>(0.0, 0.0);
            const double wix = (i > k && i < ma) ? pbx[i] - kk * vi.x : 0.0;
            const double wiy = (i > k && i < ma) ? pby[i] - kk * vi.y : 0.0;
#pragma unroll
            for (int s = 0; s < kCPW; ++s) {
              const int j = kCPW * wv + s;
              if (j >= jlo && j < jhi) {  // uniform; rows outside the block have v = w = 0
                // A_ij -= v_i conj(w_j) + w_i conj(v_j)
                A[t][s].x -= (vi.x * ws[s].x + vi.y * ws[s].y) + (wix * vs[s].x + wiy * vs[s].y);
                A[t][s].y -= (vi.y * ws[s].x - vi.x * ws[s].y) + (wiy * vs[s].x - wix * vs[s].y);
              }
            }
          }
        }
      }
      gen(k + 1, xn);
      c.sync();
    }
  }
#endif

  // Work areas of the eigen phases (tri_eigen): per-column arrays, the active-index map and
  // cluster list, Sturm counts, a scratch area for the twisted factorisations and then the
  // per-wavefront LU factors (stride lus), the tridiagonal eigenvectors Y [nw][ma], the
  // column-packed reflectors V, the W^T rows out (stride ld) and the eigenvalues out.
  struct TriWork {
    double *dg, *e2, *ea, *beta, *ar, *ai, *dre, *dim, *lam, *lo, *hi;
    int *act, *cls, *masked, *cnt;
    char* lu;
    size_t lus;
    double* Y;
    const cplx<double>* V;
    cplx<double>* Wt;
    int ld;
    double* theta;
    // optional: per-wavefront LDS slots (factors, pivots, working vector) of luls bytes for
    // the first nlw wavefronts, which then take every cluster's inverse iteration
    char* lul = nullptr;
    size_t luls = 0;
    int nlw = 0;
    double* tn = nullptr;  // optional: receives |T| (the scale of the pivot floor)
  };
  // bytes of one wavefront's LDS slot for the inverse iteration of an m-row problem
  FDE_HD static size_t lul_stride(int m) {
    return ((((size_t)m * (4 * sizeof(double) + 1) + 15) & ~(size_t)15) + (size_t)m * sizeof(double) + 15) &
           ~(size_t)15;
  }

  // Back-transformation of NV eigenvectors at a time per group of GL lanes: z = D y in
  // registers (rows i = gl + GL s), then H_k z for k = ma - 2 .. 0; each reflector's entries
  // are loaded once for the NV vectors. Slots whose rows all lie outside k + 1 .. ma - 1 are
  // skipped by the whole group.
  template <int GL, int ZR, int NV, class Ctx>
  FDE_HD static void back_transform(const Ctx& c, const TriWork& w, int m, int ma, int nw, int g0 = 0,
                                    int gstride = 0) {
    const int tid = c.tid(), nt = c.nthr();
    const int gl = tid % GL, ngrp = nt / GL;
    // vector groups g0 + tid/GL, advancing by gstride groups (default: this workgroup's groups)
    const int gs = gstride > 0 ? gstride : ngrp;
    for (int n0 = (g0 + tid / GL) * NV; n0 < nw; n0 += gs * NV) {
      cplx<double> z[NV][ZR];
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const double* y = w.Y + (size_t)(n0 + q) * ma;
#pragma unroll
        for (int s = 0; s < ZR; ++s) {
          const int i = gl + GL * s;
          z[q][s] = (n0 + q < nw && i < ma) ? mk<double>(w.dre[i] * y[i], w.dim[i] * y[i]) : mk<double>(0.0, 0.0);
        }
      }
      for (int k = ma - 2; k >= 0; --k) {
        const double bt = w.beta[k];
        if (bt == 0.0) continue;
        const int vo = voff(k, ma) - (k + 1);  // V[vo + i] = v_k for rows i = k + 1 .. ma - 1
        // a short reflector slice stays in registers for the update; a long one is loaded again
        constexpr bool kKeep = ZR <= 8;
        cplx<double> v[kKeep ? ZR : 1];
        double sx[NV], sy[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) sx[q] = sy[q] = 0.0;
#pragma unroll
        for (int s = 0; s < ZR; ++s) {
          const int i = gl + GL * s;
          if (GL * s < ma && GL * s + GL - 1 > k) {
            const cplx<double> vi = (i > k && i < ma) ? w.V[vo + i] : mk<double>(0.0, 0.0);
            if constexpr (kKeep) v[s] = vi;
#pragma unroll
            for (int q = 0; q < NV; ++q) {
              sx[q] += vi.x * z[q][s].x + vi.y * z[q][s].y;
              sy[q] += vi.x * z[q][s].y - vi.y * z[q][s].x;
            }
          }
        }
#pragma unroll
        for (int q = 0; q < NV; ++q) {
          sx[q] = bt * c.template gsum<GL>(sx[q]);
          sy[q] = bt * c.template gsum<GL>(sy[q]);
        }
#pragma unroll
        for (int s = 0; s < ZR; ++s) {
          if (GL * s < ma && GL * s + GL - 1 > k) {
            const int i = gl + GL * s;
            cplx<double> vi;
            if constexpr (kKeep)
              vi = v[s];
            else
              vi = (i > k && i < ma) ? w.V[vo + i] : mk<double>(0.0, 0.0);
#pragma unroll
            for (int q = 0; q < NV; ++q) {
              z[q][s].x -= vi.x * sx[q] - vi.y * sy[q];
              z[q][s].y -= vi.x * sy[q] + vi.y * sx[q];
            }
          }
        }
      }
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        if (n0 + q >= nw) break;
        cplx<double>* wr = w.Wt + (size_t)(n0 + q) * w.ld;
#pragma unroll
        for (int s = 0; s < ZR; ++s) {
          const int i = gl + GL * s;
          if (i < ma) wr[w.act[i]] = z[q][s];
        }
        for (int p = gl; p < m; p += GL)
          if (w.masked[p]) wr[p] = mk<double>(0.0, 0.0);
      }
    }
  }

  // Orthonormalisation of the cluster j0 .. j1 - 1 of unit vectors in Y (rows of ma), in index
  // order by the whole workgroup: classical Gram-Schmidt of vector j against all earlier ones
  // at once (their projections in dq), repeated once when the pass removed more than half of
  // the norm, then normalisation. red: block-sum scratch.
  template <class Ctx>
  FDE_HD static void cluster_orth(const Ctx& c, double* Y, int ma, int j0, int j1, double* dq, double* red) {
    const int tid = c.tid(), nt = c.nthr();
    const int lane = c.lane(), wl = c.wlanes(), wv = c.wave(), nwv = c.nwave();
    for (int j = j0 + 1; j < j1; ++j) {
      double* y = Y + (size_t)j * ma;
      for (int pass = 0; pass < 2; ++pass) {
        constexpr int QB = 4;  // earlier vectors per wavefront step, loaded together
        for (int q = j0 + wv * QB; q < j; q += nwv * QB) {
          double sq[QB];
#pragma unroll
          for (int t = 0; t < QB; ++t) sq[t] = 0.0;
          for (int i = lane; i < ma; i += wl) {
            const double yi = y[i];
#pragma unroll
            for (int t = 0; t < QB; ++t) {
              const int qq = q + t < j ? q + t : q;
              sq[t] += Y[(size_t)qq * ma + i] * yi;
            }
          }
#pragma unroll
          for (int t = 0; t < QB; ++t) {
            const double v = c.template gsum<64>(sq[t]);
            if (lane == 0 && q + t < j) dq[q + t - j0] = v;
          }
        }
        c.sync();
        double nr = 0.0;
        for (int i = tid; i < ma; i += nt) {
          double acc = 0.0;
          for (int q = j0; q < j; ++q) acc += dq[q - j0] * Y[(size_t)q * ma + i];
          const double v = y[i] - acc;
          y[i] = v;
          nr += v * v;
        }
        nr = c.sum(nr, red);
        const bool again = pass == 0 && !(nr >= 0.25);  // the vector entered with unit norm
        if (nr > 0.0) {
          const double sc = 1.0 / sqrt(nr);
          for (int i = tid; i < ma; i += nt) y[i] *= sc;
        } else {
          for (int i = tid; i < ma; i += nt) y[i] = i == j % ma ? 1.0 : 0.0;
        }
        c.sync();
        if (!again) break;
      }
    }
  }

  // The same orthonormalisation by blocks of kOrthBlock vectors (block classical Gram-Schmidt,
  // applied twice): a block, staged in LDS (YB, kOrthBlock x ma), is projected against all
  // earlier vectors of the cluster at once (projections in D, [nq][kOrthBlock]), each
  // earlier vector read once per block; then its vectors are orthonormalised among
  // themselves in order (a projection repeated once when it removed more than three
  // quarters of the squared norm); then both steps once more. red: 32 doubles of LDS.
  static constexpr int kOrthBlock = 8;
  template <class Ctx>
  FDE_HD static void cluster_orth_block(const Ctx& c, double* Y, int ma, int j0, int j1, double* YB, double* D,
                                        double* red) {
    constexpr int QB = kOrthBlock;
    const int tid = c.tid(), nt = c.nthr();
    const int lane = c.lane(), wl = c.wlanes(), wv = c.wave(), nwv = c.nwave();
    double* d2 = red + 20;  // projections on the block's earlier vectors (< QB)
    for (int b0 = j0; b0 < j1; b0 += QB) {
      const int nbk = j1 - b0 < QB ? j1 - b0 : QB;
      for (int e = tid; e < QB * ma; e += nt) {
        const int r = e / ma, i = e - r * ma;
        YB[e] = r < nbk ? Y[(size_t)(b0 + r) * ma + i] : 0.0;
      }
      c.sync();
      for (int pass = 0; pass < 2; ++pass) {
        const int nq = b0 - j0;
        if (nq > 0) {
          for (int q = wv; q < nq; q += nwv) {
            const double* yq = Y + (size_t)(j0 + q) * ma;
            double sq[QB];
#pragma unroll
            for (int r = 0; r < QB; ++r) sq[r] = 0.0;
            for (int i = lane; i < ma; i += wl) {
              const double v = yq[i];
#pragma unroll
              for (int r = 0; r < QB; ++r) sq[r] += v * YB[r * ma + i];
            }
#pragma unroll
            for (int r = 0; r < QB; ++r) {
              const double t = c.template gsum<64>(sq[r]);
              if (lane == 0) D[q * QB + r] = t;
            }
          }
          c.sync();
          for (int i = tid; i < ma; i += nt) {
            double acc[QB];
#pragma unroll
            for (int r = 0; r < QB; ++r) acc[r] = 0.0;
            for (int q = 0; q < nq; ++q) {
              const double v = Y[(size_t)(j0 + q) * ma + i];
#pragma unroll
              for (int r = 0; r < QB; ++r) acc[r] += D[q * QB + r] * v;
            }
#pragma unroll
            for (int r = 0; r < QB; ++r) YB[r * ma + i] -= acc[r];
          }
          c.sync();
        }
        for (int r = 0; r < nbk; ++r) {
          double* y = YB + r * ma;
          double n0 = 0.0;
          for (int i = tid; i < ma; i += nt) n0 += y[i] * y[i];
          n0 = c.sum(n0, red);
          double nr = n0;
          for (int rep = 0; rep < 2 && r > 0; ++rep) {
            for (int rp = wv; rp < r; rp += nwv) {
              double t = 0.0;
              for (int i = lane; i < ma; i += wl) t += YB[rp * ma + i] * y[i];
              t = c.template gsum<64>(t);
              if (lane == 0) d2[rp] = t;
            }
            c.sync();
            double part = 0.0;
            for (int i = tid; i < ma; i += nt) {
              double v = y[i];
              for (int rp = 0; rp < r; ++rp) v -= d2[rp] * YB[rp * ma + i];
              y[i] = v;
              part += v * v;
            }
            const double n1 = c.sum(part, red);
            const bool again = !(n1 >= 0.25 * nr);
            nr = n1;
            if (!again) break;
          }
          if (nr > 0.0) {
            const double sc = 1.0 / sqrt(nr);
            for (int i = tid; i < ma; i += nt) y[i] *= sc;
          } else {
            for (int i = tid; i < ma; i += nt) y[i] = i == (b0 + r) % ma ? 1.0 : 0.0;
          }
          c.sync();
        }
      }
      for (int e = tid; e < nbk * ma; e += nt) Y[(size_t)b0 * ma + e] = YB[e];
      c.sync();
    }
  }

  // Steps 3b-3e on the reduced active block (ma rows; dg, beta and alpha from the reduction):
  // eigenvalues and eigenvectors of the lowest nb, W^T rows n < nb with physical row indices,
  // masked rows zero, masked eigenpairs after the active ones. ZMAX bounds m.
  // DEFER: every vector that needs inverse iteration (clusters, failed singles) gets its shift
  // in hi but neither its iteration nor its orthonormalisation, which separate launches do.
  template <int ZMAX, bool BACK = true, bool DEFER = false, class Ctx>
  FDE_HD static void tri_eigen(const Ctx& c, const TriWork& w, int m, int nb, int ma) {
    const int tid = c.tid(), nt = c.nthr();
    const int lane = c.lane(), wl = c.wlanes(), wv = c.wave(), nwv = c.nwave();
    const int nw = nb < ma ? nb : ma;
    double *dg = w.dg, *e2 = w.e2, *ea = w.ea, *beta = w.beta, *ar = w.ar, *ai = w.ai, *dre = w.dre, *dim = w.dim;
    double *lam = w.lam, *lo = w.lo, *hi = w.hi, *Y = w.Y;
    int *act = w.act, *cls = w.cls, *masked = w.masked, *cnt = w.cnt;
    // ---- 3b. real tridiagonal (dg, ea) and the phases D
    for (int k = tid; k + 1 < ma; k += nt) {
      e2[k] = ar[k] * ar[k] + ai[k] * ai[k];
      ea[k] = sqrt(e2[k]);
    }
    if (tid == 0 && ma > 0) {
      double px = 1.0, py = 0.0;
      dre[0] = 1.0;
      dim[0] = 0.0;
      for (int k = 0; k + 1 < ma; ++k) {
        const double ab = sqrt(ar[k] * ar[k] + ai[k] * ai[k]);
        if (ab > 0.0) {
          const double ux = ar[k] / ab, uy = ai[k] / ab;
          const double qx = px * ux - py * uy, qy = px * uy + py * ux;
          px = qx;
          py = qy;
        }
        dre[k + 1] = px;
        dim[k + 1] = py;
      }
    }
    c.sync();

    if (nw > 0) {
      // ---- 3c. multisection for the nw lowest eigenvalues
      double glo = 1e300, ghi = -1e300, emax2 = 0.0;
      for (int i = 0; i < ma; ++i) {
        const double rad = (i > 0 ? ea[i - 1] : 0.0) + (i + 1 < ma ? ea[i] : 0.0);
        glo = fmin(glo, dg[i] - rad);
        ghi = fmax(ghi, dg[i] + rad);
        if (i + 1 < ma) emax2 = fmax(emax2, e2[i]);
      }
      const double eps = 2.220446049250313e-16;
      const double tnorm = fmax(fmax(fabs(glo), fabs(ghi)), 1e-300);
      const double pivmin = 2.2250738585072014e-308 * fmax(1.0, emax2);
      glo -= 4.0 * eps * tnorm + 2.0 * pivmin;
      ghi += 4.0 * eps * tnorm + 2.0 * pivmin;
      const int G = nt >= nw ? (nt / nw < kMsPoints ? nt / nw : kMsPoints) : 1;
      int niter = 1;
      for (double w = ghi - glo; w > 2.0 * eps * tnorm; w /= (double)(G + 1)) ++niter;
      auto sturm = [&](double x) {  // number of eigenvalues below x
        double q = dg[0] - x;
        if (fabs(q) < pivmin) q = -pivmin;
        int n = q < 0.0 ? 1 : 0;
#pragma unroll 8
        for (int i = 1; i < ma; ++i) {
          q = (dg[i] - x) - e2[i - 1] * Ctx::rcp(q);
          if (fabs(q) < pivmin) q = -pivmin;
          n += q < 0.0 ? 1 : 0;
        }
        return n;
      };
      for (int j = tid; j < nw; j += nt) {
        lo[j] = glo;
        hi[j] = ghi;
      }
      c.sync();
      for (int it = 0; it < niter; ++it) {
        for (int vt = tid; vt < nw * G; vt += nt) {
          const int j = vt / G, g = vt - j * G;
          const double l = lo[j], step = (hi[j] - l) / (double)(G + 1);
          cnt[vt] = sturm(l + (double)(g + 1) * step);
        }
        c.sync();
        for (int j = tid; j < nw; j += nt) {
          const double l0 = lo[j], step = (hi[j] - l0) / (double)(G + 1);
          double l = l0, h = hi[j];
          for (int g = 0; g < G; ++g) {
            const double x = l0 + (double)(g + 1) * step;
            if (cnt[j * G + g] <= j) {
              l = x;
            } else {
              h = x;
              break;
            }
          }
          lo[j] = l;
          hi[j] = h;
        }
        c.sync();
      }
      for (int j = tid; j < nw; j += nt) lam[j] = 0.5 * (lo[j] + hi[j]);
      c.sync();
      // clusters: neighbours closer than 1e-3 |T| share one wavefront
      const double ortol = 1e-3 * tnorm, pertol = 10.0 * eps * tnorm;
      if (tid == 0) {
        int ncl = 0;
        for (int j = 0; j < nw; ++j)
          if (j == 0 || lam[j] - lam[j - 1] > ortol) cls[ncl++] = j;
        cls[ncl] = nw;
        cls[m + 2] = ncl;
      }
      c.sync();
      // ---- 3d. eigenvectors. An eigenvalue farther than ortol from its neighbours: one thread,
      //      twisted factorisation N_r D N_r^T of T - lambda I (forward pivots D+, backward D-,
      //      twist r at the smallest |gamma_r|), x_r = 1 and the two recurrences outward.
      //      Clusters, and any vector that came out non-finite: inverse iteration below.
      auto single = [&](int j) {
        return (j == 0 || lam[j] - lam[j - 1] > ortol) && (j + 1 == nw || lam[j + 1] - lam[j] > ortol);
      };
      for (int j = tid; j < nw; j += nt) {
        lo[j] = 1.0;  // 1: needs inverse iteration
        if (!single(j)) continue;
        double* rp = (double*)w.lu + (size_t)j * 2 * ma;  // 1 / D+_i
        double* rm = rp + ma;                            // 1 / D-_i
        // The recurrences carry their previous pivot in a register; where a pass reads back
        // stored pivots, it loads kC of them before its stores (the stores could otherwise
        // alias the loads and serialise them).
        constexpr int kC = 8;
        const double lj = lam[j];
        double q = dg[0] - lj;
        if (fabs(q) < pivmin) q = -pivmin;
        double rprev = Ctx::rcp(q);
        rp[0] = rprev;
        for (int i = 1; i < ma; ++i) {
          q = (dg[i] - lj) - e2[i - 1] * rprev;
          if (fabs(q) < pivmin) q = -pivmin;
          rprev = Ctx::rcp(q);
          rp[i] = rprev;
        }
        double best = fabs(q);  // gamma_{ma-1} = D+_{ma-1}
        int r = ma - 1;
        q = dg[ma - 1] - lj;
        if (fabs(q) < pivmin) q = -pivmin;
        double rnext = Ctx::rcp(q);
        rm[ma - 1] = rnext;
        for (int i0 = ma - 2; i0 >= 0; i0 -= kC) {
          double rpc[kC];  // rp[i - 1] for i = i0 - t
#pragma unroll
          for (int t = 0; t < kC; ++t) rpc[t] = rp[i0 - t - 1 > 0 ? i0 - t - 1 : 0];
#pragma unroll
          for (int t = 0; t < kC; ++t) {
            const int i = i0 - t;
            if (i < 0) break;
            const double dpi = (dg[i] - lj) - (i > 0 ? e2[i - 1] * rpc[t] : 0.0);  // D+_i
            const double gam = dpi - e2[i] * rnext;
            if (fabs(gam) < best) {
              best = fabs(gam);
              r = i;
            }
            q = (dg[i] - lj) - e2[i] * rnext;
            if (fabs(q) < pivmin) q = -pivmin;
            rnext = Ctx::rcp(q);
            rm[i] = rnext;
          }
        }
        double* y = Y + (size_t)j * ma;
        double x = 1.0, nr = 1.0;
        y[r] = 1.0;
        for (int i0 = r - 1; i0 >= 0; i0 -= kC) {
          double rc[kC];
#pragma unroll
          for (int t = 0; t < kC; ++t) rc[t] = rp[i0 - t > 0 ? i0 - t : 0];
#pragma unroll
          for (int t = 0; t < kC; ++t) {
            const int i = i0 - t;
            if (i < 0) break;
            x = -(ea[i] * rc[t]) * x;
            y[i] = x;
            nr += x * x;
          }
        }
        x = 1.0;
        for (int i0 = r + 1; i0 < ma; i0 += kC) {
          double rc[kC];
#pragma unroll
          for (int t = 0; t < kC; ++t) rc[t] = rm[i0 + t < ma ? i0 + t : ma - 1];
#pragma unroll
          for (int t = 0; t < kC; ++t) {
            const int i = i0 + t;
            if (i >= ma) break;
            x = -(ea[i - 1] * rc[t]) * x;
            y[i] = x;
            nr += x * x;
          }
        }
        if (nr > 0.0 && nr < 1e300) {
          const double sc = 1.0 / sqrt(nr);
          for (int i0 = 0; i0 < ma; i0 += kC) {
            double yc[kC];
#pragma unroll
            for (int t = 0; t < kC; ++t) yc[t] = y[i0 + t < ma ? i0 + t : ma - 1];
#pragma unroll
            for (int t = 0; t < kC; ++t)
              if (i0 + t < ma) y[i0 + t] = yc[t] * sc;
          }
          lo[j] = 0.0;
        }
      }
      c.sync();
      // inverse iteration, one cluster (or failed single) per wavefront
      const int ncl = cls[m + 2];
      // factors and the working vector in LDS when the problem has per-wavefront slots there
      // (the serial LU passes then wait on LDS, not global memory); results go to Y either way
      const bool lds_it = w.lul != nullptr;
      const int nit = lds_it && w.nlw < nwv ? w.nlw : nwv;  // wavefronts taking clusters
      double* lu = lds_it ? (double*)(w.lul + (size_t)wv * w.luls) : (double*)(w.lu + (size_t)wv * w.lus);
      unsigned char* piv = (unsigned char*)(lu + 4 * ma);
      double* yl = lds_it ? (double*)((char*)lu + (((size_t)ma * (4 * sizeof(double) + 1) + 15) & ~(size_t)15))
                          : nullptr;
      // one vector on one wavefront: shift lj, start vector, kInvIt solves, each followed by
      // modified Gram-Schmidt against the vectors q0 .. j - 1 (none when q0 = j) and normalisation
      auto inv_iter = [&](int j, double lj, int q0) {
        double* const yout = Y + (size_t)j * ma;
        double* y = lds_it ? yl : yout;
        for (int i = lane; i < ma; i += wl) y[i] = start_value(i, j);
        if (lane == 0) lu_factor<Ctx>(ma, dg, ea, lj, eps * tnorm, lu, piv);
        c.wsync();
        for (int it = 0; it < kInvIt; ++it) {
          if (lane == 0) lu_solve(ma, lu, piv, y);
          c.wsync();
          for (int q = q0; q < j; ++q) {
            const double* yq = Y + (size_t)q * ma;
            double d = 0.0;
            for (int i = lane; i < ma; i += wl) d += yq[i] * y[i];
            d = c.template gsum<64>(d);
            for (int i = lane; i < ma; i += wl) y[i] -= d * yq[i];
          }
          double nr = 0.0;
          for (int i = lane; i < ma; i += wl) nr += y[i] * y[i];
          nr = c.template gsum<64>(nr);
          if (nr > 0.0) {
            const double sc = 1.0 / sqrt(nr);
            for (int i = lane; i < ma; i += wl) y[i] *= sc;
          } else {
            for (int i = lane; i < ma; i += wl) y[i] = i == j % ma ? 1.0 : 0.0;
          }
          c.wsync();
        }
        if (lds_it) {
          for (int i = lane; i < ma; i += wl) yout[i] = y[i];
          c.wsync();
        }
      };
      // clusters of up to kBigCluster vectors: one wavefront each, its vectors in turn
      for (int ci = wv; !DEFER && wv < nit && ci < ncl; ci += nit) {
        const int j0 = cls[ci], j1 = cls[ci + 1];
        if (j1 - j0 == 1 && lo[j0] == 0.0) continue;
        if (j1 - j0 > kBigCluster) continue;
        double lprev = 0.0;
        for (int j = j0; j < j1; ++j) {
          double lj = lam[j];
          if (j > j0 && lj - lprev < pertol) lj = lprev + pertol;
          lprev = lj;
          inv_iter(j, lj, j0);
        }
      }
      // Larger clusters: the shifts (same perturbation rule) into hi, every vector iterated on
      // its own with the wavefronts taking vectors in turn, then each cluster orthonormalised by
      // the whole workgroup in index order: classical Gram-Schmidt against the earlier vectors
      // (the projections summed over all of them at once), repeated once when the first pass
      // removed more than half of the norm. The iterates of distinct shifts are already close to
      // orthogonal, so one pass is the rule and the repeat covers near-degenerate pairs.
      if (tid == 0) {
        for (int ci = 0; ci < ncl; ++ci) {
          const int j0 = cls[ci], j1 = cls[ci + 1];
          if (j1 - j0 <= (DEFER ? 0 : kBigCluster)) continue;
          double lprev = 0.0;
          for (int j = j0; j < j1; ++j) {
            double lj = lam[j];
            if (j > j0 && lj - lprev < pertol) lj = lprev + pertol;
            lprev = lj;
            hi[j] = lj;
          }
        }
      }
      c.sync();
      if constexpr (!DEFER)
        for (int ci = 0; ci < ncl; ++ci) {
          const int j0 = cls[ci], j1 = cls[ci + 1];
          if (j1 - j0 <= kBigCluster) continue;
          for (int j = j0 + wv; wv < nit && j < j1; j += nit) inv_iter(j, hi[j], j);
        }
      if (w.tn && tid == 0) *w.tn = tnorm;
      c.sync();
      // projections in e2 and the block sums in lo (both free once the vectors are computed)
      if constexpr (!DEFER)
        for (int ci = 0; ci < ncl; ++ci) {
          const int j0 = cls[ci], j1 = cls[ci + 1];
          if (j1 - j0 > kBigCluster) cluster_orth(c, Y, ma, j0, j1, e2, lo);
        }
      c.sync();
      // ---- 3e. W^T rows n < nw: z = D y, H_k z for k = ma - 2 .. 0, written to the physical
      //      indices act[i], masked rows zero (BACK false: left to a separate launch)
      if constexpr (!BACK) {
      } else
#if defined(__HIP_DEVICE_COMPILE__)
      if constexpr (ZMAX > 16 * kGroup) {  // a whole wavefront per vector
        if (ma <= 256)
          back_transform<64, 4, 2>(c, w, m, ma, nw);
        else
          back_transform<64, (ZMAX + 63) / 64, 1>(c, w, m, ma, nw);
      } else {
        back_transform<kGroup, (ZMAX + kGroup - 1) / kGroup, 1>(c, w, m, ma, nw);
      }
#else
      {
        back_transform<1, ZMAX, 1>(c, w, m, ma, nw);
      }
#endif
    }
    // masked eigenpairs (A~ = kInactiveDiag e_p e_p^H) fill the columns beyond the active count
    for (int n = nw + tid; n < nb; n += nt) {
      int left = n - nw, p = 0;
      for (; p < m; ++p)
        if (masked[p] && left-- == 0) break;
      cplx<double>* z = w.Wt + (size_t)n * w.ld;
      for (int i = 0; i < m; ++i) z[i] = mk<double>(i == p ? 1.0 : 0.0, 0.0);
      w.theta[n] = kInactiveDiag;
    }
    for (int n = tid; n < nw; n += nt) w.theta[n] = lam[n];
  }

  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps) {
    const Prob<T>& a = ps.p[c.bx()];
    const int m = a.m, nb = a.nb, ld = m + 1;
    const int tid = c.tid(), nt = c.nthr();
    const int lane = c.lane(), wl = c.wlanes(), wv = c.wave(), nwv = c.nwave();
    cplx<double>* U = (cplx<double>*)lds;
    cplx<double>* M = U + (size_t)m * (m + 1) / 2;
    double* red = (double*)((char*)M + mspan(m, nb));
    double* sdiag = red + 32;
    int* masked = (int*)(sdiag + m);
    int* order = masked + m;
    char* r1 = (char*)M;
    double* Y = (double*)(r1 + r1_bytes(m, nb));
    double* dg = (double*)((char*)Y + y_bytes(m, nb));
    double *e2 = dg + m, *ea = e2 + m, *beta = ea + m, *ar = beta + m, *ai = ar + m, *dre = ai + m, *dim = dre + m;
    double *lam = dim + m, *lo = lam + m, *hi = lo + m, *pbx = hi + m, *pby = pbx + m;
    cplx<double>* xb = (cplx<double>*)(pby + m);  // [2][m]: the current column, double-buffered
    int* act = (int*)(xb + 2 * m);
    int* cls = act + m;  // cluster starts (m + 1 entries), then the active count and the cluster count
    int* cnt = (int*)r1;

    if (!rr_front<T>(c, a, ps.drop_tol, U, M, sdiag, masked)) return;
    if (tid == 0) {
      int k = 0;
      for (int j = 0; j < m; ++j)
        if (!masked[j]) act[k++] = j;
      cls[m + 1] = k;
    }
    c.sync();
    const int ma = cls[m + 1];
    const int nw = nb < ma ? nb : ma;
    // ---- 3a. Householder reduction of the active part
#if defined(__HIP_DEVICE_COMPILE__)
    house_regs(c, U, r1, m, ma, act, dg, beta, ar, ai, xb, pbx, pby);
#else
    house_lds(c, U, r1, m, ma, act, dg, beta, ar, ai, pbx, pby);
#endif
    // ---- 3b-3e. tridiagonal eigenproblem and back-transformation
    const TriWork tw{dg, e2, ea, beta, ar, ai, dre, dim, lam, lo, hi, act, cls, masked, cnt, r1, lu_stride(m), Y, U, M,
                     ld, a.theta};
    tri_eigen<kRRLdsMax>(c, tw, m, nb, ma);
    for (int n = tid; n < nb; n += nt) order[n] = n;
    rr_tail<T>(c, a, U, M, sdiag, order);
  }
};

// Rayleigh-Ritz solve of one band block too large for the LDS solvers (kRRLdsMax < m <=
// kRRTriMax), matrices in global memory: the front end of KRRSolve (Cholesky, A~), then the
// Householder reduction of (A~ + A~^H)/2 on the active rows and columns, held with both
// triangles in the problem's W buffer, and the tridiagonal route of KRRSolveTri (per-column
// arrays in LDS; B holds the twisted factorisations and, when no LDS slots fit, the LU
// factors; S the tridiagonal eigenvectors and, behind them, the reflectors; A the W^T rows),
// and C = L^{-H} W one column per thread in blocks of 8 rows.
constexpr int kRRTriMax = 768;

template <typename T>
struct KRRSolveTriG {
  using Tri = KRRSolveTri<T>;
  static constexpr int kThreads = Tri::kThreads;
  FDE_HD static size_t base_bytes(int m) {
    return sizeof(double) * (32 + 15 * (size_t)m) + sizeof(int) * (2 * (size_t)m + 3 + kThreads) + 64;
  }
  // wavefronts with an LDS slot for the inverse iteration: as many as fit 160 KiB, none
  // below four (the factors then stay in global memory)
  FDE_HD static int lds_waves(int m) {
    const size_t base = (base_bytes(m) + 15) & ~(size_t)15, lim = 160 * 1024;
    const int n = base < lim ? (int)((lim - base) / Tri::lul_stride(m)) : 0;
    return n < 4 ? 0 : (n < Tri::kWaves ? n : Tri::kWaves);
  }
  FDE_HD static size_t lds_bytes(int m) {
    return ((base_bytes(m) + 15) & ~(size_t)15) + (size_t)lds_waves(m) * Tri::lul_stride(m);
  }

  // Householder reduction of the active block held with both triangles in G (row-major, ld ma,
  // logical indices): step k reads row k (conjugate of column k), stages v in LDS (vl), forms
  // p = beta G' v one row per wavefront and applies the rank-2 update to the whole trailing
  // block. v_k goes to V[voff(k) ..], the diagonal to dg.
  template <class Ctx>
  FDE_HD static void house_full(const Ctx& c, cplx<double>* G, cplx<double>* V, cplx<double>* vl, int ma,
                                double* dg, double* beta, double* ar, double* ai, double* pbx, double* pby) {
    const int tid = c.tid(), nt = c.nthr();
    const int lane = c.lane(), wl = c.wlanes(), wv = c.wave(), nwv = c.nwave();
    for (int k = 0; k + 1 < ma; ++k) {
      const int n1 = ma - k - 1;
      const cplx<double>* gk = G + (size_t)k * ma + k + 1;  // x_r = conj(gk[r])
      double s2 = 0.0;
      for (int r = lane; r < n1; r += wl) s2 += norm2(gk[r]);
      s2 = c.template gsum<64>(s2);
      const cplx<double> x0 = conj(gk[0]);
      double bt = 0.0;
      cplx<double> alpha = x0, v0 = x0;
      if (n1 > 1 && s2 > norm2(x0)) {
        const double ax0 = sqrt(norm2(x0)), sg = sqrt(s2);
        const cplx<double> ph = ax0 > 0.0 ? mk<double>(x0.x / ax0, x0.y / ax0) : mk<double>(1.0, 0.0);
        alpha = mk<double>(-ph.x * sg, -ph.y * sg);
        v0 = mk<double>(x0.x + ph.x * sg, x0.y + ph.y * sg);
        bt = 1.0 / (sg * (sg + ax0));
      }
      if (tid == 0) {
        beta[k] = bt;
        ar[k] = alpha.x;
        ai[k] = alpha.y;
        dg[k] = G[(size_t)k * ma + k].x;
      }
      cplx<double>* vk = V + Tri::voff(k, ma);
      for (int r = tid; r < n1; r += nt) {
        const cplx<double> v = r == 0 ? v0 : conj(gk[r]);
        vl[r] = v;
        vk[r] = v;
      }
      c.sync();
      if (bt != 0.0) {  // uniform: every wavefront summed in the same order
        // rows r0 + q nwv (q < RB) of a wavefront together, so their loads are in flight at once
        constexpr int RB = 4;
        for (int r0 = wv; r0 < n1; r0 += RB * nwv) {
          double sx[RB], sy[RB];
#pragma unroll
          for (int q = 0; q < RB; ++q) sx[q] = sy[q] = 0.0;
          for (int j = lane; j < n1; j += wl) {
            const cplx<double> v = vl[j];
            cplx<double> g[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) {  // rows past the end repeat row r0: loads unconditional
              const int r = r0 + q * nwv < n1 ? r0 + q * nwv : r0;
              g[q] = G[(size_t)(k + 1 + r) * ma + k + 1 + j];
            }
#pragma unroll
            for (int q = 0; q < RB; ++q) {
              sx[q] += g[q].x * v.x - g[q].y * v.y;
              sy[q] += g[q].x * v.y + g[q].y * v.x;
            }
          }
#pragma unroll
          for (int q = 0; q < RB; ++q) {
            const int r = r0 + q * nwv;
            if (r < n1) {
              const double tx = c.template gsum<64>(sx[q]), ty = c.template gsum<64>(sy[q]);
              if (lane == 0) {
                pbx[r] = bt * tx;
                pby[r] = bt * ty;
              }
            }
          }
        }
        c.sync();
        // K = beta/2 v^H p (real); G' -= v w^H + w v^H with w = p - K v
        double kk = 0.0;
        for (int r = lane; r < n1; r += wl) kk += vl[r].x * pbx[r] + vl[r].y * pby[r];
        kk = 0.5 * bt * c.template gsum<64>(kk);
        for (int r0 = wv; r0 < n1; r0 += RB * nwv) {
          for (int j = lane; j < n1; j += wl) {
            const cplx<double> vj = vl[j];
            const double wjx = pbx[j] - kk * vj.x, wjy = pby[j] - kk * vj.y;
            cplx<double> t[RB];
#pragma unroll
            for (int q = 0; q < RB; ++q) {
              const int r = r0 + q * nwv < n1 ? r0 + q * nwv : r0;
              t[q] = G[(size_t)(k + 1 + r) * ma + k + 1 + j];
            }
#pragma unroll
            for (int q = 0; q < RB; ++q) {
              const int r = r0 + q * nwv;
              if (r < n1) {
                const cplx<double> vr = vl[r];
                const double wrx = pbx[r] - kk * vr.x, wry = pby[r] - kk * vr.y;
                t[q].x -= (vr.x * wjx + vr.y * wjy) + (wrx * vj.x + wry * vj.y);
                t[q].y -= (vr.y * wjx - vr.x * wjy) + (wry * vj.x - wrx * vj.y);
                G[(size_t)(k + 1 + r) * ma + k + 1 + j] = t[q];
              }
            }
          }
        }
        c.sync();
      }
    }
    if (tid == 0 && ma > 0) dg[ma - 1] = G[(size_t)(ma - 1) * ma + ma - 1].x;
    c.sync();
  }

  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps) {
    const Prob<T>& a = ps.p[c.bx()];
    const int m = a.m, nb = a.nb;
    const int tid = c.tid(), nt = c.nthr();
    double* red = (double*)lds;
    double* dg = red + 32;
    double *e2 = dg + m, *ea = e2 + m, *beta = ea + m, *ar = beta + m, *ai = ar + m, *dre = ai + m, *dim = dre + m;
    double *lam = dim + m, *lo = lam + m, *hi = lo + m, *pbx = hi + m, *pby = pbx + m;
    cplx<double>* vl = (cplx<double>*)(((size_t)(pby + m) + 15) & ~(size_t)15);  // 16-byte aligned
    int* act = (int*)(vl + m);
    int* cls = act + m;      // cluster starts (m + 1), the active count, the cluster count
    int* cnt = cls + m + 3;  // Sturm counts, one per thread
    if (!KRRSolve<T>::front(c, red, a, ps.drop_tol)) return;
    if (tid == 0) {
      int k = 0;
      for (int j = 0; j < m; ++j)
        if (!a.masked[j]) act[k++] = j;
      cls[m + 1] = k;
    }
    c.sync();
    const int ma = cls[m + 1];
    // (A~ + A~^H)/2 on the active rows and columns, both triangles, into G
    cplx<double>* G = a.W;
    for (int e = tid; e < ma * ma; e += nt) {
      const int i = e / ma, j = e - i * ma;
      const cplx<double> l = a.A[(size_t)act[i] * m + act[j]], u = a.A[(size_t)act[j] * m + act[i]];
      G[e] = mk<double>(0.5 * (l.x + u.x), 0.5 * (l.y - u.y));
    }
    c.sync();
    // reflectors behind the inverse-iteration vectors (which take at most m * m doubles of S)
    cplx<double>* V = (cplx<double>*)((double*)a.S + (size_t)m * m);
    house_full(c, G, V, vl, ma, dg, beta, ar, ai, pbx, pby);
    typename Tri::TriWork tw{dg,  e2,     ea,       beta, ar, ai,    dre,  dim,     lam,
                             lo,  hi,     act,      cls,  a.masked, cnt, (char*)a.B,
                             Tri::lu_stride(m), (double*)a.S, V,  a.A,  m,       a.theta};
    // the launch sized LDS for the batch's largest m: slots of that size
    int mmax = 0;
    for (int q = 0; q < ps.n; ++q) mmax = ps.p[q].m > mmax ? ps.p[q].m : mmax;
    if (lds_waves(mmax) > 0) {
      tw.lul = lds + ((base_bytes(mmax) + 15) & ~(size_t)15);
      tw.luls = Tri::lul_stride(mmax);
      tw.nlw = lds_waves(mmax);
    }
    Tri::template tri_eigen<kRRTriMax>(c, tw, m, nb, ma);
    c.sync();
    // C = L^{-H} W[:, :nb], W^T rows in A (stride m): column n per thread
    for (int n = tid; n < nb; n += nt) {
      a.eval[n] = a.theta[n];
      tri_solve_col(a.L, m, a.A + (size_t)n * m, 1, false, a.Cd + n, nb, true);
    }
    c.sync();
    for (int e = tid; e < m * nb; e += nt) {
      const cplx<double> v = a.Cd[e];
      ((cplx<T>*)a.Ct)[e] = mk<T>((T)v.x, (T)v.y);
    }
  }
};

// ---------------------------------------------------------------------------
// The same solve for large m split over launches so that most of it runs on many
// workgroups (the single-workgroup solver above is latency-bound on one CU):
//   KRRChol*      blocked Cholesky with dropping (below);
//   KRRBigTrsm    B = L^{-1} A, A~ = L^{-1} B^H and, at the end, C = L^{-H} W, by column strips;
//   KRRBigPrep    the active indices, (A~ + A~^H)/2 on them into W, the first reflector;
//   KRRBigHhP(0)  p_0 = beta_0 G' v_0, rows of the trailing block over many workgroups;
//   KRRBigHh(k)   one launch per Householder column: the rank-2 update G' -= v w^H + w v^H
//                 (w = p - K v, K = beta/2 v^H p) on rows over many workgroups, reflector
//                 k + 1 formed by every workgroup from the updated row k + 1, and p_{k+1};
//   KRRBigTri     real tridiagonal, multisection, twisted factorisations of isolated eigenvalues
//                 and the shifts of the rest (one workgroup per problem);
//   KRRBigInv     inverse iteration of the clustered eigenvalues' vectors, one per wavefront;
//   KRRBigOrth    their orthonormalisation per cluster (one workgroup per problem);
//   KRRBigBack    back-transformation W = Q D Y, one wavefront per eigenvector, many workgroups.
// A problem whose Cholesky reported a dependent band column (info > 0) is skipped by every
// later launch. Per-problem vectors live in the Gram-partial area, free after the Gram sums.
// ---------------------------------------------------------------------------
struct BigWs {
  cplx<double>* v[2];  // reflector v_k, double-buffered by k parity
  cplx<double>* pp[2];  // beta_k G' v_k, double-buffered by k parity
  double *dg, *beta, *ar, *ai, *dre, *dim, *ea, *shift, *sdiag, *tnorm;
  int *act, *nact;     // active indices and their count
  int *cls, *ncl;      // cluster starts (ncl + 1) and the cluster count
  int *bigv, *nbig;    // the vectors that need inverse iteration, in order, and their count
  template <typename T>
  FDE_HD explicit BigWs(const Prob<T>& a) {
    double* b = (double*)a.part;
    const size_t m = (size_t)a.m;
    v[0] = (cplx<double>*)b;
    v[1] = (cplx<double>*)(b + 2 * m);
    pp[0] = (cplx<double>*)(b + 4 * m);
    pp[1] = (cplx<double>*)(b + 6 * m);
    double* q = b + 8 * m;
    dg = q;
    beta = q + m;
    ar = q + 2 * m;
    ai = q + 3 * m;
    dre = q + 4 * m;
    dim = q + 5 * m;
    ea = q + 6 * m;
    shift = q + 7 * m;
    sdiag = q + 8 * m;
    tnorm = q + 9 * m;
    act = (int*)(q + 9 * m + 2);
    nact = act + m;
    cls = nact + 1;
    ncl = cls + m + 1;
    bigv = ncl + 1;
    nbig = bigv + m;
  }
};

// reflector k of the active block G (ld ma) from row k (one workgroup): v into vbuf and
// V's column-packed slot, beta, alpha, the diagonal G_kk
template <class Ctx>
FDE_HD void big_reflector(const Ctx& c, double* red, const cplx<double>* G, int ma, int k, cplx<double>* V,
                          cplx<double>* vbuf, const BigWs& w) {
  const int tid = c.tid(), nt = c.nthr();
  const int n1 = ma - k - 1;
  const cplx<double>* gk = G + (size_t)k * ma + k + 1;  // x_r = conj(gk[r])
  double s2 = 0.0;
  for (int r = tid; r < n1; r += nt) s2 += norm2(gk[r]);
  s2 = c.sum(s2, red);
  const cplx<double> x0 = conj(gk[0]);
  double bt = 0.0;
  cplx<double> alpha = x0, v0 = x0;
  if (n1 > 1 && s2 > norm2(x0)) {
    const double ax0 = sqrt(norm2(x0)), sg = sqrt(s2);
    const cplx<double> ph = ax0 > 0.0 ? mk<double>(x0.x / ax0, x0.y / ax0) : mk<double>(1.0, 0.0);
    alpha = mk<double>(-ph.x * sg, -ph.y * sg);
    v0 = mk<double>(x0.x + ph.x * sg, x0.y + ph.y * sg);
    bt = 1.0 / (sg * (sg + ax0));
  }
  if (tid == 0) {
    w.beta[k] = bt;
    w.ar[k] = alpha.x;
    w.ai[k] = alpha.y;
    w.dg[k] = G[(size_t)k * ma + k].x;
  }
  cplx<double>* vk = V + KRRSolveTri<double>::voff(k, ma);
  for (int r = tid; r < n1; r += nt) {
    const cplx<double> v = r == 0 ? v0 : conj(gk[r]);
    vbuf[r] = v;
    vk[r] = v;
  }
}

FDE_HD cplx<double>* big_reflectors(const cplx<double>* S, int m) {
  return (cplx<double>*)((double*)S + (size_t)m * m);  // behind the eigenvectors Y in S
}

// Blocked right-looking Cholesky with dropping (the same decisions as KRRSolve::front_chol: a
// correction column j >= nb whose pivot d = S_jj - sum_k |L_jk|^2 falls below drop_tol S_jj is
// dropped, a band column with such a pivot is an error), in column blocks of kCholB:
//   KRRCholInit    masks, S and A of masked columns, L = 0, the diagonal of S kept;
//   KRRCholDiag    the block's columns in turn on one wavefront (S' holds S minus the earlier
//                  blocks' terms), drop decisions, the block's own rows of L;
//   KRRCholPanel   L for the rows below the block, one row per thread (zero in dropped columns);
//   KRRCholUpdate  S'_il -= sum over the block L_ip conj(L_lp) on the trailing lower triangle,
//                  32 x 32 tiles over many workgroups.
constexpr int kCholB = 32;

template <typename T>
struct KRRCholInit {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const ProbSet<T> ps) {
    const Prob<T>& a = ps.p[c.by()];
    const int m = a.m;
    const BigWs w(a);
    const size_t mm = (size_t)m * m;
    for (int l = c.tid(); l < 1024; l += c.nthr()) {
      const size_t e = (size_t)c.bx() * 1024 + l;
      if (e >= mm) break;
      const int i = (int)(e / m), j = (int)(e - (size_t)i * m);
      const bool mi = a.active && !a.active[i], mj = a.active && !a.active[j];
      if (mi || mj) {
        a.S[e] = mk<double>(i == j ? 1.0 : 0.0, 0.0);
        a.A[e] = mk<double>(i == j ? kInactiveDiag : 0.0, 0.0);
      }
      a.L[e] = mk<double>(0.0, 0.0);
      if (i == j) {
        a.masked[j] = mi ? 1 : 0;
        w.sdiag[j] = mi ? 1.0 : a.S[e].x;
      }
      if (e == 0) a.info[0] = 0;
    }
  }
};

template <typename T>
struct KRRCholDiag {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps, int j0) {
    const Prob<T>& a = ps.p[c.bx()];
    const int m = a.m, nb = a.nb;
    if (a.info[0] > 0 || j0 >= m) return;
    const int j1 = j0 + kCholB < m ? j0 + kCholB : m;
    const int tid = c.tid(), nt = c.nthr();
    double* red = (double*)lds;
    const BigWs w(a);
    cplx<double>*S = a.S, *L = a.L, *A = a.A;
    const double drop_tol = ps.drop_tol;
    for (int j = j0; j < j1; ++j) {
      double part = 0.0;
      for (int k = j0 + tid; k < j; k += nt) part += norm2(L[(size_t)j * m + k]);
      const double sjj = w.sdiag[j];
      const double d = S[(size_t)j * m + j].x - c.sum(part, red);
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
        // a dependent band column: report, C = I, NaN eigenvalues; later launches skip
        if (tid == 0) a.info[0] = j + 1;
        for (int e = tid; e < m * nb; e += nt) {
          const int i = e / nb, n = e - i * nb;
          const cplx<double> v = mk<double>(i == n ? 1.0 : 0.0, 0.0);
          a.Cd[e] = v;
          ((cplx<T>*)a.Ct)[e] = mk<T>((T)v.x, (T)v.y);
        }
        for (int n = tid; n < nb; n += nt) a.eval[n] = 0.0 / 0.0;
        return;  // uniform
      }
      const double ljj = sqrt(d);
      if (tid == 0) L[(size_t)j * m + j] = mk<double>(ljj, 0.0);
      for (int i = j + 1 + tid; i < j1; i += nt) {
        double ax = 0.0, ay = 0.0;  // sum over the block's earlier columns of L_ip conj(L_jp)
        for (int p = j0; p < j; ++p) {
          const cplx<double> lip = L[(size_t)i * m + p], ljp = L[(size_t)j * m + p];
          ax += lip.x * ljp.x + lip.y * ljp.y;
          ay += lip.y * ljp.x - lip.x * ljp.y;
        }
        const cplx<double> sij = S[(size_t)i * m + j];
        L[(size_t)i * m + j] = cdiv_real(mk<double>(sij.x - ax, sij.y - ay), ljj);
      }
      c.sync();
    }
  }
};

// rows j1 .. m - 1 of L in the block's columns; grid (ceil((m - j1) / 64), n), 64 threads
template <typename T>
struct KRRCholPanel {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps, int j0) {
    const Prob<T>& a = ps.p[c.by()];
    const int m = a.m;
    if (a.info[0] > 0 || j0 >= m) return;
    const int j1 = j0 + kCholB < m ? j0 + kCholB : m, nbk = j1 - j0;
    cplx<double>* Lb = (cplx<double>*)lds;  // the block's diagonal tile [nbk][nbk]
    for (int e = c.tid(); e < nbk * nbk; e += c.nthr()) {
      const int r = e / nbk, q = e - r * nbk;
      Lb[e] = a.L[(size_t)(j0 + r) * m + j0 + q];
    }
    c.sync();
    for (int l = c.tid(); l < 64; l += c.nthr()) {
      const int i = j1 + c.bx() * 64 + l;
      if (i >= m) break;
      cplx<double>* li = a.L + (size_t)i * m;
      const cplx<double>* si = a.S + (size_t)i * m;
      for (int j = j0; j < j1; ++j) {
        const int q = j - j0;
        if (a.masked[j]) {
          li[j] = mk<double>(0.0, 0.0);
          continue;
        }
        double ax = 0.0, ay = 0.0;
        for (int p = 0; p < q; ++p) {
          const cplx<double> lip = li[j0 + p], ljp = Lb[q * nbk + p];
          ax += lip.x * ljp.x + lip.y * ljp.y;
          ay += lip.y * ljp.x - lip.x * ljp.y;
        }
        li[j] = cdiv_real(mk<double>(si[j].x - ax, si[j].y - ay), Lb[q * nbk + q].x);
      }
    }
  }
};

// S'_il -= sum_{p in block} L_ip conj(L_lp), j1 <= l <= i < m; one 32 x 32 tile of the trailing
// lower triangle per workgroup (tile index over the triangle), 256 threads
template <typename T>
struct KRRCholUpdate {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps, int j0) {
    const Prob<T>& a = ps.p[c.by()];
    const int m = a.m;
    if (a.info[0] > 0) return;
    const int j1 = j0 + kCholB;
    if (j1 >= m) return;
    const int ntile = (m - j1 + 31) / 32;
    // tile (ti, tl), tl <= ti, from the workgroup index
    int t = c.bx(), ti = 0;
    while (ti < ntile && t > ti) {
      t -= ti + 1;
      ++ti;
    }
    if (ti >= ntile) return;
    const int tl = t;
    cplx<double>* Li = (cplx<double>*)lds;  // [32][kCholB] rows i of the block's columns
    cplx<double>* Ll = Li + 32 * kCholB;     // [32][kCholB] rows l
    const int i0 = j1 + ti * 32, l0 = j1 + tl * 32;
    for (int e = c.tid(); e < 32 * kCholB; e += c.nthr()) {
      const int r = e / kCholB, p = e - r * kCholB;
      Li[e] = i0 + r < m ? a.L[(size_t)(i0 + r) * m + j0 + p] : mk<double>(0.0, 0.0);
      Ll[e] = l0 + r < m ? a.L[(size_t)(l0 + r) * m + j0 + p] : mk<double>(0.0, 0.0);
    }
    c.sync();
    for (int e = c.tid(); e < 32 * 32; e += c.nthr()) {
      const int r = e / 32, q = e - r * 32;
      const int i = i0 + r, l = l0 + q;
      if (i >= m || l > i) continue;
      double ax = 0.0, ay = 0.0;
      for (int p = 0; p < kCholB; ++p) {
        const cplx<double> x = Li[r * kCholB + p], y = Ll[q * kCholB + p];
        ax += x.x * y.x + x.y * y.y;
        ay += x.y * y.x - x.x * y.y;
      }
      cplx<double>& s = a.S[(size_t)i * m + l];
      s.x -= ax;
      s.y -= ay;
    }
  }
};

template <typename T>
struct KRRBigPrep {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps) {
    const Prob<T>& a = ps.p[c.bx()];
    if (a.info[0] > 0) return;
    const int m = a.m, tid = c.tid(), nt = c.nthr();
    double* red = (double*)lds;
    int* sh = (int*)(red + 32);
    const BigWs w(a);
    if (tid == 0) {
      int k = 0;
      for (int j = 0; j < m; ++j)
        if (!a.masked[j]) w.act[k++] = j;
      w.nact[0] = k;
      sh[0] = k;
    }
    c.sync();
    const int ma = sh[0];
    cplx<double>* G = a.W;
    for (int e = tid; e < ma * ma; e += nt) {
      const int i = e / ma, j = e - i * ma;
      const int ai = w.act[i], aj = w.act[j];
      const cplx<double> l = a.A[(size_t)ai * m + aj], u = a.A[(size_t)aj * m + ai];
      G[e] = mk<double>(0.5 * (l.x + u.x), 0.5 * (l.y - u.y));
    }
    c.sync();
    if (ma >= 2)
      big_reflector(c, red, G, ma, 0, big_reflectors(a.S, m), w.v[0], w);
    else if (tid == 0 && ma == 1)
      w.dg[0] = G[0].x;
  }
};

// rows per workgroup of the Householder launches, lanes per row
constexpr int kHhRows = 16;

template <typename T>
struct KRRBigHhP {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const ProbSet<T> ps, int k) {
    const Prob<T>& a = ps.p[c.by()];
    if (a.info[0] > 0) return;
    const BigWs w(a);
    const int ma = w.nact[0];
    if (!(k + 1 < ma)) return;
    const double bt = w.beta[k];
    if (bt == 0.0) return;
    const int n1 = ma - k - 1;
#if defined(__HIP_DEVICE_COMPILE__)
    constexpr int GL = 16;
#else
    constexpr int GL = 1;
#endif
    const cplx<double>* G = a.W;
    const cplx<double>* v = w.v[k & 1];
    const int tid = c.tid(), nt = c.nthr();
    const int gl = tid % GL, grp = tid / GL, ng = nt / GL;
    for (int rl = grp; rl < kHhRows; rl += ng) {
      const int r = c.bx() * kHhRows + rl;
      if (r >= n1) break;  // uniform per lane group
      const cplx<double>* g = G + (size_t)(k + 1 + r) * ma + k + 1;
      double sx = 0.0, sy = 0.0;
      for (int j = gl; j < n1; j += GL) {
        const cplx<double> gj = g[j], vj = v[j];
        sx += gj.x * vj.x - gj.y * vj.y;
        sy += gj.x * vj.y + gj.y * vj.x;
      }
      sx = c.template gsum<GL>(sx);
      sy = c.template gsum<GL>(sy);
      if (gl == 0) w.pp[k & 1][r] = mk<double>(bt * sx, bt * sy);
    }
  }
};

// One Householder column k as one launch: with v_k, beta_k and p_k = beta_k G' v_k from the
// previous launch, every workgroup forms K = beta_k/2 v_k^H p_k and w = p_k - K v_k, the
// updated row k + 1 (in LDS; that row is read by all and written by none), and from it
// reflector k + 1 (all identically; workgroup 0 stores it, with the diagonal). Then it
// applies the rank-2 update to its own rows below row k + 1 and, in the same pass, forms
// their entries of p_{k+1} = beta_{k+1} G'' v_{k+1}. grid (max(1, ceil((m - k - 2) / 16)), n),
// 256 threads (16 rows of 16 lanes).
template <typename T>
struct KRRBigHh {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps, int k) {
    const Prob<T>& a = ps.p[c.by()];
    if (a.info[0] > 0) return;
    const BigWs w(a);
    const int ma = w.nact[0];
    if (!(k + 1 < ma)) return;
    const int n1 = ma - k - 1, m = a.m;
    const int tid = c.tid(), nt = c.nthr();
#if defined(__HIP_DEVICE_COMPILE__)
    constexpr int GL = 16;
#else
    constexpr int GL = 1;
#endif
    const int gl = tid % GL, grp = tid / GL, ng = nt / GL;
    double* red = (double*)lds;
    cplx<double>* row = (cplx<double>*)(red + 32);  // updated row k + 1, trailing columns [n1]
    cplx<double>* vn = row + n1;                    // v_{k+1} [n1 - 1]
    cplx<double>* G = a.W;
    const cplx<double>* v = w.v[k & 1];
    const cplx<double>* p = w.pp[k & 1];
    const double bt = w.beta[k];
    double kk = 0.0;
    if (bt != 0.0) {  // uniform per problem
      for (int r = tid; r < n1; r += nt) kk += v[r].x * p[r].x + v[r].y * p[r].y;
      kk = 0.5 * bt * c.sum(kk, red);
    }
    // updated row k + 1: t_j - (v_0 conj(w_j) + w_0 conj(v_j))
    const cplx<double>* g1 = G + (size_t)(k + 1) * ma + k + 1;
    {
      const cplx<double> v0 = v[0];
      const double w0x = p[0].x - kk * v0.x, w0y = p[0].y - kk * v0.y;
      for (int j = tid; j < n1; j += nt) {
        cplx<double> t = g1[j];
        if (bt != 0.0) {
          const cplx<double> vj = v[j];
          const double wjx = p[j].x - kk * vj.x, wjy = p[j].y - kk * vj.y;
          t.x -= (v0.x * wjx + v0.y * wjy) + (w0x * vj.x + w0y * vj.y);
          t.y -= (v0.y * wjx - v0.x * wjy) + (w0y * vj.x - w0x * vj.y);
        }
        row[j] = t;
      }
    }
    c.sync();
    // reflector k + 1 from the row (x_r = conj(row[1 + r])), as big_reflector does
    const int n2 = n1 - 1;
    double bt1 = 0.0;
    if (n2 >= 1) {
      double s2 = 0.0;
      for (int r = tid; r < n2; r += nt) s2 += norm2(row[1 + r]);
      s2 = c.sum(s2, red);
      const cplx<double> x0 = conj(row[1]);
      cplx<double> alpha = x0, v0 = x0;
      if (n2 > 1 && s2 > norm2(x0)) {
        const double ax0 = sqrt(norm2(x0)), sg = sqrt(s2);
        const cplx<double> ph = ax0 > 0.0 ? mk<double>(x0.x / ax0, x0.y / ax0) : mk<double>(1.0, 0.0);
        alpha = mk<double>(-ph.x * sg, -ph.y * sg);
        v0 = mk<double>(x0.x + ph.x * sg, x0.y + ph.y * sg);
        bt1 = 1.0 / (sg * (sg + ax0));
      }
      cplx<double>* vk = big_reflectors(a.S, m) + KRRSolveTri<double>::voff(k + 1, ma);
      for (int r = tid; r < n2; r += nt) {
        const cplx<double> vr = r == 0 ? v0 : conj(row[1 + r]);
        vn[r] = vr;
        if (c.bx() == 0) {
          w.v[(k + 1) & 1][r] = vr;
          vk[r] = vr;
        }
      }
      if (c.bx() == 0 && tid == 0) {
        w.beta[k + 1] = bt1;
        w.ar[k + 1] = alpha.x;
        w.ai[k + 1] = alpha.y;
      }
    }
    if (c.bx() == 0 && tid == 0) w.dg[k + 1] = row[0].x;
    c.sync();
    // own rows k + 2 + r (r < n2): rank-2 update of columns k + 2 .. ma - 1, and p_{k+1}
    for (int rl = grp; rl < kHhRows; rl += ng) {
      const int r = c.bx() * kHhRows + rl;
      if (r >= n2) break;  // uniform per lane group
      cplx<double>* g = G + (size_t)(k + 2 + r) * ma + k + 2;
      const cplx<double> vr = v[1 + r];
      const double wrx = p[1 + r].x - kk * vr.x, wry = p[1 + r].y - kk * vr.y;
      double sx = 0.0, sy = 0.0;
      for (int j = gl; j < n2; j += GL) {
        cplx<double> t = g[j];
        if (bt != 0.0) {
          const cplx<double> vj = v[1 + j];
          const double wjx = p[1 + j].x - kk * vj.x, wjy = p[1 + j].y - kk * vj.y;
          t.x -= (vr.x * wjx + vr.y * wjy) + (wrx * vj.x + wry * vj.y);
          t.y -= (vr.y * wjx - vr.x * wjy) + (wry * vj.x - wrx * vj.y);
          g[j] = t;
        }
        const cplx<double> u = vn[j];
        sx += t.x * u.x - t.y * u.y;
        sy += t.x * u.y + t.y * u.x;
      }
      sx = c.template gsum<GL>(sx);
      sy = c.template gsum<GL>(sy);
      if (gl == 0) w.pp[(k + 1) & 1][r] = mk<double>(bt1 * sx, bt1 * sy);
    }
  }
};

template <typename T>
struct KRRBigTri {
  using Tri = KRRSolveTri<T>;
  using TriG = KRRSolveTriG<T>;
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps) {
    const Prob<T>& a = ps.p[c.bx()];
    if (a.info[0] > 0) return;
    const int m = a.m, nb = a.nb;
    const int tid = c.tid(), nt = c.nthr();
    double* red = (double*)lds;
    double* dg = red + 32;
    double *e2 = dg + m, *ea = e2 + m, *beta = ea + m, *ar = beta + m, *ai = ar + m, *dre = ai + m, *dim = dre + m;
    double *lam = dim + m, *lo = lam + m, *hi = lo + m, *pbx = hi + m, *pby = pbx + m;
    cplx<double>* vl = (cplx<double>*)(((size_t)(pby + m) + 15) & ~(size_t)15);
    int* act = (int*)(vl + m);
    int* cls = act + m;
    int* cnt = cls + m + 3;
    const BigWs w(a);
    const int ma = w.nact[0];
    for (int i = tid; i < m; i += nt) {
      dg[i] = i < ma ? w.dg[i] : 0.0;
      beta[i] = i + 1 < ma ? w.beta[i] : 0.0;
      ar[i] = i + 1 < ma ? w.ar[i] : 0.0;
      ai[i] = i + 1 < ma ? w.ai[i] : 0.0;
      act[i] = i < ma ? w.act[i] : 0;
    }
    if (tid == 0) cls[m + 1] = ma;
    c.sync();
    typename Tri::TriWork tw{dg,  e2,     ea,       beta, ar, ai,    dre,  dim,     lam,
                             lo,  hi,     act,      cls,  a.masked, cnt, (char*)a.B,
                             Tri::lu_stride(m), (double*)a.S, big_reflectors(a.S, m), a.A, m, a.theta};
    int mmax = 0;
    for (int q = 0; q < ps.n; ++q) mmax = ps.p[q].m > mmax ? ps.p[q].m : mmax;
    if (TriG::lds_waves(mmax) > 0) {
      tw.lul = lds + ((TriG::base_bytes(mmax) + 15) & ~(size_t)15);
      tw.luls = Tri::lul_stride(mmax);
      tw.nlw = TriG::lds_waves(mmax);
    }
    tw.tn = w.tnorm;
    Tri::template tri_eigen<kRRTriMax, false, true>(c, tw, m, nb, ma);
    c.sync();
    // the phases of the later launches: D, the off-diagonal, the shifts and the vectors that
    // need inverse iteration (clusters and failed singles)
    const int nw = nb < ma ? nb : ma;
    for (int i = tid; i < ma; i += nt) {
      w.dre[i] = dre[i];
      w.dim[i] = dim[i];
      w.ea[i] = ea[i];
    }
    for (int j = tid; j < nw; j += nt) w.shift[j] = hi[j];
    if (tid == 0) {
      const int ncl = nw > 0 ? cls[m + 2] : 0;
      int nbig = 0;
      for (int ci = 0; ci <= ncl; ++ci) w.cls[ci] = cls[ci];
      for (int ci = 0; ci < ncl; ++ci)
        if (cls[ci + 1] - cls[ci] > 1 || lo[cls[ci]] != 0.0)
          for (int j = cls[ci]; j < cls[ci + 1]; ++j) w.bigv[nbig++] = j;
      w.ncl[0] = ncl;
      w.nbig[0] = nbig;
    }
  }
};

// Inverse iteration of the vectors of clusters (and of failed singles), each on its own
// wavefront with its factors and working vector in LDS (the tridiagonal in LDS too), no
// orthogonalisation.
// grid (ceil(max nbig / 4), n), 256 threads.
template <typename T>
struct KRRBigInv {
  using Tri = KRRSolveTri<T>;
  static constexpr int kVec = 4;  // vectors (wavefronts) per workgroup
  FDE_HD static size_t slot_bytes(int m) { return Tri::lul_stride(m); }
  FDE_HD static size_t lds_bytes(int m) { return 2 * (size_t)m * sizeof(double) + kVec * slot_bytes(m); }
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps, int mmax) {
    const Prob<T>& a = ps.p[c.by()];
    if (a.info[0] > 0) return;
    const BigWs w(a);
    const int nbig = w.nbig[0];
    if (c.bx() * kVec >= nbig) return;
    const int ma = w.nact[0];
    const int tid = c.tid(), nt = c.nthr(), lane = c.lane(), wl = c.wlanes();
    double* dgl = (double*)lds;
    double* eal = dgl + mmax;
    for (int i = tid; i < ma; i += nt) {
      dgl[i] = w.dg[i];
      eal[i] = w.ea[i];
    }
    c.sync();
    const double tiny = 2.220446049250313e-16 * w.tnorm[0];
    double* Y = (double*)a.S;
    for (int v = c.wave(); v < kVec; v += c.nwave()) {
      const int k = c.bx() * kVec + v;
      if (k >= nbig) break;  // wavefront-uniform
      const int j = w.bigv[k];
      double* lu = (double*)(lds + 2 * (size_t)mmax * sizeof(double) + (size_t)v * slot_bytes(mmax));
      unsigned char* piv = (unsigned char*)(lu + 4 * ma);
      double* y = (double*)((char*)lu + Tri::lu_stride(ma));
      for (int i = lane; i < ma; i += wl) y[i] = Tri::start_value(i, j);
      if (lane == 0) Tri::template lu_factor<Ctx>(ma, dgl, eal, w.shift[j], tiny, lu, piv);
      c.wsync();
      for (int it = 0; it < Tri::kInvIt; ++it) {
        if (lane == 0) Tri::lu_solve(ma, lu, piv, y);
        c.wsync();
        double nr = 0.0;
        for (int i = lane; i < ma; i += wl) nr += y[i] * y[i];
        nr = c.template gsum<64>(nr);
        if (nr > 0.0) {
          const double sc = 1.0 / sqrt(nr);
          for (int i = lane; i < ma; i += wl) y[i] *= sc;
        } else {
          for (int i = lane; i < ma; i += wl) y[i] = i == j % ma ? 1.0 : 0.0;
        }
        c.wsync();
      }
      double* yout = Y + (size_t)j * ma;
      for (int i = lane; i < ma; i += wl) yout[i] = y[i];
    }
  }
};

// Orthonormalisation of every cluster (one workgroup per problem, block Gram-Schmidt).
// LDS: 32 + 2 kOrthBlock mmax doubles.
template <typename T>
struct KRRBigOrth {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps) {
    const Prob<T>& a = ps.p[c.bx()];
    if (a.info[0] > 0) return;
    const BigWs w(a);
    if (w.nbig[0] == 0) return;
    const int ma = w.nact[0], ncl = w.ncl[0];
    double* red = (double*)lds;
    double* YB = red + 32;                                   // [kOrthBlock][ma]
    double* D = YB + (size_t)KRRSolveTri<T>::kOrthBlock * ma;  // [ma][kOrthBlock]
    for (int ci = 0; ci < ncl; ++ci) {
      const int j0 = w.cls[ci], j1 = w.cls[ci + 1];
      if (j1 - j0 > 1) KRRSolveTri<T>::cluster_orth_block(c, (double*)a.S, ma, j0, j1, YB, D, red);
    }
  }
};

// back-transformation: one wavefront (host: one thread) per eigenvector.
// grid (nwg, n), 256 threads.
template <typename T>
struct KRRBigBack {
  using Tri = KRRSolveTri<T>;
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const ProbSet<T> ps) {
    const Prob<T>& a = ps.p[c.by()];
    if (a.info[0] > 0) return;
    const BigWs w(a);
    const int m = a.m, nb = a.nb, ma = w.nact[0];
    const int nw = nb < ma ? nb : ma;
    typename Tri::TriWork tw{w.dg, nullptr, nullptr, w.beta, w.ar, w.ai, w.dre, w.dim, nullptr,
                             nullptr, nullptr, w.act, nullptr, a.masked, nullptr, nullptr,
                             0, (double*)a.S, big_reflectors(a.S, m), a.A, m, a.theta};
#if defined(__HIP_DEVICE_COMPILE__)
    const int gpb = c.nthr() / 64;  // vector groups per workgroup
    Tri::template back_transform<64, (kRRTriMax + 63) / 64, 1>(c, tw, m, ma, nw, c.bx() * gpb, gpb * gridDim.x);
#else
    (void)tw;
    if (c.bx() == 0) Tri::template back_transform<1, kRRTriMax, 1>(c, tw, m, ma, nw);
#endif
  }
};

// Triangular solves of the split path by column strips: a workgroup of 32 x 8 threads takes
// 8 columns, keeps them in LDS, and walks the rows in blocks of 32 (forward, or backward for
// L^H): thread (r, q) first subtracts from row r of the block the terms of every row already
// solved (a dot product over them, the rows of the block in parallel), then the first
// wavefront solves the block's own triangle, all its rows and columns in parallel per step.
//   MODE 0: B = L^{-1} A;  MODE 1: A~ = L^{-1} B^H (into A);
//   MODE 2: C = L^{-H} W[:, :nb] (W^T rows in A) into Cd and, in plan precision, Ct, and the
//           eigenvalues.
// grid (ceil(ncols / 8), n), 256 threads, LDS m x 8 complex doubles.
template <typename T, int MODE>
struct KRRBigTrsm {
  static constexpr int RB = 32, CB = 8;
  FDE_HD static size_t lds_bytes(int m) { return ((size_t)m * CB + RB * RB) * sizeof(cplx<double>); }
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps) {
    const Prob<T>& a = ps.p[c.by()];
    if (a.info[0] > 0) return;
    const int m = a.m, nb = a.nb;
    const int ncols = MODE == 2 ? nb : m;
    const int c0 = c.bx() * CB;
    if (c0 >= ncols) return;
    const int tid = c.tid(), nt = c.nthr();
    constexpr bool up = MODE == 2;
    const cplx<double>* L = a.L;
    cplx<double>* X = (cplx<double>*)lds;  // [m][CB]
    cplx<double>* Ld = X + (size_t)m * CB;  // the block's own factors [RB][RB] (diagonal: real)
    for (int e = tid; e < m * CB; e += nt) {
      const int i = e / CB, q = e - i * CB, col = c0 + q;
      cplx<double> v = mk<double>(0.0, 0.0);
      if (col < ncols) {
        if (MODE == 0) v = a.A[(size_t)i * m + col];
        if (MODE == 1) v = conj(a.B[(size_t)col * m + i]);
        if (MODE == 2) v = a.A[(size_t)col * m + i];
      }
      X[e] = v;
    }
    c.sync();
    // logical row t in solve order <-> physical row
    auto row = [&](int t) { return up ? m - 1 - t : t; };
    // factor of row i against solved row k: L_ik (forward), conj(L_ki) (backward)
    auto lf = [&](int i, int k) {
      const cplx<double> l = up ? L[(size_t)k * m + i] : L[(size_t)i * m + k];
      return up ? conj(l) : l;
    };
    for (int b0 = 0; b0 < m; b0 += RB) {
      const int nr = m - b0 < RB ? m - b0 : RB;
      for (int e = tid; e < RB * CB; e += nt) {
        const int r = e % RB, q = e / RB;
        if (r >= nr) continue;
        const int i = row(b0 + r);
        double ax = 0.0, ay = 0.0;
        for (int t = 0; t < b0; ++t) {
          const int k = row(t);
          const cplx<double> l = lf(i, k), xk = X[k * CB + q];
          ax += l.x * xk.x - l.y * xk.y;
          ay += l.x * xk.y + l.y * xk.x;
        }
        X[i * CB + q].x -= ax;
        X[i * CB + q].y -= ay;
      }
      for (int e = tid; e < nr * nr; e += nt) {
        const int r = e / nr, p = e - r * nr;
        if (p > r) continue;
        const int i = row(b0 + r);
        Ld[r * RB + p] = p < r ? lf(i, row(b0 + p)) : mk<double>(L[(size_t)i * m + i].x, 0.0);
      }
      c.sync();
      // the block's own triangle by the first wavefront, row by row: row p is final once
      // divided by its diagonal, then every row below subtracts its term of row p (the same
      // terms in the same order as a row-by-row dot product)
      if (c.wave() == 0) {
        for (int p = 0; p < nr; ++p) {
          const int ip = row(b0 + p);
          for (int q = c.lane(); q < CB; q += c.wlanes()) X[ip * CB + q] = cdiv_real(X[ip * CB + q], Ld[p * RB + p].x);
          c.wsync();
          for (int e = c.lane(); e < (nr - 1 - p) * CB; e += c.wlanes()) {
            const int r = p + 1 + e / CB, q = e % CB;
            const int i = row(b0 + r);
            const cplx<double> l = Ld[r * RB + p], xk = X[ip * CB + q];
            X[i * CB + q].x -= l.x * xk.x - l.y * xk.y;
            X[i * CB + q].y -= l.x * xk.y + l.y * xk.x;
          }
          c.wsync();
        }
      }
      c.sync();
    }
    for (int e = tid; e < m * CB; e += nt) {
      const int i = e / CB, q = e - i * CB, col = c0 + q;
      if (col >= ncols) continue;
      const cplx<double> v = X[e];
      if (MODE == 0) a.B[(size_t)i * m + col] = v;
      if (MODE == 1) a.A[(size_t)i * m + col] = v;
      if (MODE == 2) {
        a.Cd[(size_t)i * nb + col] = v;
        ((cplx<T>*)a.Ct)[(size_t)i * nb + col] = mk<T>((T)v.x, (T)v.y);
      }
    }
    if (MODE == 2)
      for (int q = tid; q < CB; q += nt)
        if (c0 + q < nb) a.eval[c0 + q] = a.theta[c0 + q];
  }
};

}  // namespace fde
