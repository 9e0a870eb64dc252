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
// LDS: packed triangle U (m(m+1)/2 complex: L, then A~), a full work matrix M
// (m rows, padded stride m+1: the lower triangle of S during the Cholesky,
// then B/E, then W^T), and small per-pair / per-column arrays. While the
// packed triangle holds A~, the factor is parked in the problem's global L.
#pragma once

#include "kernels_la.hpp"

namespace fde {

constexpr int kRRLdsMax = 80;
constexpr int kWRows = 15;  // row groups of the eigenvector update items

FDE_HD int tri(int i, int j) { return i * (i + 1) / 2 + j; }  // j <= i

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
        return;  // uniform: every thread read the same d
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
    // ---- park L in global memory (its diagonal also in sdiag); A~ = (E + E^H)/2 into U,
    //      with E_ij = M_ij / L_jj (the column scaling of the last substitution)
    for (int e = tid; e < m * (m + 1) / 2; e += nt) a.L[e] = U[e];
    for (int i = tid; i < m; i += nt) sdiag[i] = U[tri(i, i)].x;
    c.sync();
    for (int e = tid; e < m * m; e += nt) {
      const int i = qdiv(e, inv_m), j = e - i * m;
      if (j > i) continue;
      const cplx<double> eij = cdiv_real(M[(size_t)i * ld + j], sdiag[j]);
      const cplx<double> eji = cdiv_real(M[(size_t)j * ld + i], sdiag[i]);
      U[tri(i, j)] = i == j ? mk<double>(eij.x, 0.0) : mk<double>(0.5 * (eji.x + eij.x), 0.5 * (eij.y - eji.y));
    }
    c.sync();
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
    // ---- restore L; C = L^{-H} W[:, order[:nb]] in place in the W^T rows
    for (int e = tid; e < m * (m + 1) / 2; e += nt) U[e] = a.L[e];
    for (int n = tid; n < nb; n += nt) a.eval[n] = a.theta[order[n]];
    const float inv_nb = 1.0f / (float)nb;
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
      a.Cd[e] = v;
      ((cplx<T>*)a.Ct)[e] = mk<T>((T)v.x, (T)v.y);
    }
  }
};

}  // namespace fde
