// Rayleigh-Ritz solve of one band block held entirely in LDS (m <= kRRLdsMax):
//   Cholesky of S (packed lower factor, column dropping as in KRRSolve),
//   A~ = L^{-1} A L^{-H} in place (columns: B = L^{-1} A; rows: E = B L^{-H};
//   A~ = E^H made Hermitian), cyclic parallel Jacobi on the packed Hermitian
//   A~ with 2 x 2 block rotations (two barriers per round), ascending order,
//   C = L^{-H} W[:, order[:nb]].
// LDS: packed triangle (m(m+1)/2), full m x m work matrix, rotation and
// diagonal arrays. The factor is parked in the problem's global L while the
// packed triangle holds A~.
#pragma once

#include "kernels_la.hpp"

namespace fde {

constexpr int kRRLdsMax = 80;

FDE_HD int tri(int i, int j) { return i * (i + 1) / 2 + j; }  // j <= i

// Hermitian packed access: element (i, j) of a matrix whose (r, c) entries with
// r >= c are stored at tri(r, c).
FDE_HD cplx<double> hget(const cplx<double>* U, int i, int j) {
  return i >= j ? U[tri(i, j)] : conj(U[tri(j, i)]);
}
FDE_HD void hset(cplx<double>* U, int i, int j, cplx<double> v) {
  if (i >= j) U[tri(i, j)] = v;
  else U[tri(j, i)] = conj(v);
}

FDE_HD void rr_pair(int r, int k, int mp, int& p, int& q) {
  if (k == 0) {
    p = r;
    q = mp - 1;
  } else {
    p = (r + k) % (mp - 1);
    q = (r - k + (mp - 1)) % (mp - 1);
  }
}

template <typename T>
struct KRRSolveLds {
  FDE_HD static size_t lds_bytes(int m) {
    const int mp = m + (m & 1);
    return sizeof(cplx<double>) * ((size_t)m * (m + 1) / 2 + (size_t)m * (m + 1)) +
           sizeof(double) * (32 + 6 * (mp / 2 + 1)) + sizeof(int) * 2 * (size_t)m + 64;
  }

  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps) {
    const Prob<T>& a = ps.p[c.bx()];
    const int m = a.m, nb = a.nb;
    const int mp = m + (m & 1), npair = mp / 2;
    const int tid = c.tid(), nt = c.nthr();
    const double drop_tol = ps.drop_tol;
    cplx<double>* U = (cplx<double>*)lds;             // packed triangle
    const int ld = m + 1;                              // padded row stride of M (no bank conflicts)
    cplx<double>* M = U + (size_t)m * (m + 1) / 2;     // full work matrix
    double* red = (double*)(M + (size_t)m * ld);
    double* rc = red + 32;
    double* rs = rc + npair;
    double* rex = rs + npair;
    double* rey = rex + npair;
    double* dp_ = rey + npair;   // new diagonal values of each pair
    double* dq_ = dp_ + npair;
    int* masked = (int*)(dq_ + npair);
    int* order = masked + m;
    if (tid == 0) a.info[0] = 0;
    for (int j = tid; j < m; j += nt) masked[j] = (a.active && !a.active[j]) ? 1 : 0;
    c.sync();
    // ---- S into M (masked columns -> e_j)
    for (int e = tid; e < m * m; e += nt) {
      const int i = e / m, j = e - i * m;
      M[(size_t)i * ld + j] = (masked[i] || masked[j]) ? mk<double>(i == j ? 1.0 : 0.0, 0.0) : a.S[e];
    }
    c.sync();
    // ---- Cholesky into U (lower, packed), dropping dependent correction columns
    for (int j = 0; j < m; ++j) {
      double part = 0.0;
      for (int k = tid; k < j; k += nt) part += norm2(U[tri(j, k)]);
      const double sjj = M[(size_t)j * ld + j].x;
      const double d = sjj - c.sum(part, red);
      if (j >= nb && !(d >= drop_tol * sjj)) {
        for (int k = tid; k < j; k += nt) U[tri(j, k)] = mk<double>(0, 0);
        for (int i = j + 1 + tid; i < m; i += nt) U[tri(i, j)] = mk<double>(0, 0);
        if (tid == 0) {
          U[tri(j, j)] = mk<double>(1.0, 0.0);
          masked[j] = 1;
        }
        c.sync();
        continue;
      }
      if (!(d >= drop_tol * sjj) || !(d > 0.0)) {
        if (tid == 0) a.info[0] = j + 1;
        for (int e = tid; e < m * nb; e += nt) {
          const int i = e / nb, n = e - i * nb;
          const cplx<double> v = mk<double>(i == n ? 1.0 : 0.0, 0.0);
          a.Cd[e] = v;
          ((cplx<T>*)a.Ct)[e] = mk<T>((T)v.x, (T)v.y);
        }
        for (int n = tid; n < nb; n += nt) a.eval[n] = 0.0 / 0.0;
        c.sync();
        return;  // uniform: every thread saw the same d
      }
      const double ljj = sqrt(d);
      if (tid == 0) U[tri(j, j)] = mk<double>(ljj, 0.0);
      for (int i = j + 1 + tid; i < m; i += nt) {
        cplx<double> acc = M[(size_t)i * ld + j];
        for (int k = 0; k < j; ++k) {
          const cplx<double> lik = U[tri(i, k)], ljk = U[tri(j, k)];
          acc.x -= lik.x * ljk.x + lik.y * ljk.y;
          acc.y -= lik.y * ljk.x - lik.x * ljk.y;
        }
        U[tri(i, j)] = cdiv_real(acc, ljj);
      }
      c.sync();
    }
    // ---- A into M (masked / dropped columns -> 1e6 e_j)
    for (int e = tid; e < m * m; e += nt) {
      const int i = e / m, j = e - i * m;
      M[(size_t)i * ld + j] = (masked[i] || masked[j]) ? mk<double>(i == j ? kInactiveDiag : 0.0, 0.0) : a.A[e];
    }
    c.sync();
    // ---- B = L^{-1} A, one column per thread, in place
    for (int col = tid; col < m; col += nt) {
      for (int i = 0; i < m; ++i) {
        const cplx<double>* Li = U + tri(i, 0);
        cplx<double> a0 = M[(size_t)i * ld + col], a1 = mk<double>(0, 0), a2 = a1, a3 = a1;
        int k = 0;
        for (; k + 4 <= i; k += 4) {
          a0 = a0 - Li[k] * M[(size_t)k * ld + col];
          a1 = a1 - Li[k + 1] * M[(size_t)(k + 1) * ld + col];
          a2 = a2 - Li[k + 2] * M[(size_t)(k + 2) * ld + col];
          a3 = a3 - Li[k + 3] * M[(size_t)(k + 3) * ld + col];
        }
        for (; k < i; ++k) a0 = a0 - Li[k] * M[(size_t)k * ld + col];
        M[(size_t)i * ld + col] = cdiv_real((a0 + a1) + (a2 + a3), Li[i].x);
      }
    }
    c.sync();
    // ---- E = B L^{-H}, one row per thread, in place: E_rj = (B_rj - sum_{k<j} E_rk conj(L_jk)) / L_jj
    for (int r = tid; r < m; r += nt) {
      cplx<double>* Mr = M + (size_t)r * ld;
      for (int j = 0; j < m; ++j) {
        const cplx<double>* Lj = U + tri(j, 0);
        cplx<double> a0 = Mr[j], a1 = mk<double>(0, 0), a2 = a1, a3 = a1;
        int k = 0;
        for (; k + 4 <= j; k += 4) {
          a0 = a0 - Mr[k] * conj(Lj[k]);
          a1 = a1 - Mr[k + 1] * conj(Lj[k + 1]);
          a2 = a2 - Mr[k + 2] * conj(Lj[k + 2]);
          a3 = a3 - Mr[k + 3] * conj(Lj[k + 3]);
        }
        for (; k < j; ++k) a0 = a0 - Mr[k] * conj(Lj[k]);
        Mr[j] = cdiv_real((a0 + a1) + (a2 + a3), Lj[j].x);
      }
    }
    c.sync();
    // ---- park L in global memory, A~ = (E^H + E)/2 into the packed triangle, W = I into M
    for (int e = tid; e < m * (m + 1) / 2; e += nt) a.L[e] = U[e];
    c.sync();
    for (int i = tid; i < m; i += nt) {
      for (int j = 0; j <= i; ++j) {
        const cplx<double> eij = M[(size_t)i * ld + j], eji = M[(size_t)j * ld + i];
        // A~_ij = conj(E_ji); Hermitian part: (conj(E_ji) + E_ij)/2
        U[tri(i, j)] = i == j ? mk<double>(eij.x, 0.0) : mk<double>(0.5 * (eji.x + eij.x), 0.5 * (eij.y - eji.y));
      }
    }
    c.sync();
    for (int e = tid; e < m * m; e += nt) {
      const int i = e / m, j = e - i * m;
      M[(size_t)i * ld + j] = mk<double>(i == j ? 1.0 : 0.0, 0.0);
    }
    c.sync();
    // ---- cyclic parallel Jacobi on the packed Hermitian A~, W (= M) accumulates U
    bool conv = false;
    double prev_off = 1e300;
    const int nblk = npair * (npair - 1) / 2;
    for (int sweep = 0; sweep < 40 && !conv; ++sweep) {
      for (int r = 0; r < mp - 1; ++r) {
        for (int k = tid; k < npair; k += nt) {
          int p, q;
          rr_pair(r, k, mp, p, q);
          double cc = 1.0, ss = 0.0, ex = 1.0, ey = 0.0, np_ = 0.0, nq_ = 0.0;
          if (p < m && q < m) {
            const cplx<double> bpq = hget(U, p, q);
            const double app = U[tri(p, p)].x, aqq = U[tri(q, q)].x;
            np_ = app;
            nq_ = aqq;
            const double ab = sqrt(norm2(bpq));
            if (ab > 1e-300) {
              const double th = (aqq - app) / (2.0 * ab);
              const double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
              cc = 1.0 / sqrt(t * t + 1.0);
              ss = t * cc;
              ex = bpq.x / ab;
              ey = bpq.y / ab;
              np_ = app - t * ab;
              nq_ = aqq + t * ab;
            }
          }
          rc[k] = cc;
          rs[k] = ss;
          rex[k] = ex;
          rey[k] = ey;
          dp_[k] = np_;
          dq_[k] = nq_;
        }
        c.sync();
        // off-diagonal 2x2 blocks (pairs K < Q): B' = U_K^H B U_Q ; diagonal blocks; W columns
        const int items = nblk + npair + npair * m;
        for (int it = tid; it < items; it += nt) {
          if (it < nblk) {
            // decode (K, Q), K < Q, from the linear index: row K starts at
            // K (2 npair - K - 1) / 2
            const double tt = 2.0 * npair - 1.0;
            int K = (int)floor(0.5 * (tt - sqrt(tt * tt - 8.0 * it)));
            if (K < 0) K = 0;
            while (K > 0 && K * (2 * npair - K - 1) / 2 > it) --K;
            while ((K + 1) * (2 * npair - K - 2) / 2 <= it) ++K;
            const int Q = K + 1 + (it - K * (2 * npair - K - 1) / 2);
            int p, q, pp, qq;
            rr_pair(r, K, mp, p, q);
            rr_pair(r, Q, mp, pp, qq);
            const bool rowK = p < m && q < m, colQ = pp < m && qq < m;
            if ((!rowK || rs[K] == 0.0) && (!colQ || rs[Q] == 0.0)) continue;
            // rows {p, q} (may include the dummy index when m is odd), cols {pp, qq}
            cplx<double> b00 = (p < m && pp < m) ? hget(U, p, pp) : mk<double>(0, 0);
            cplx<double> b01 = (p < m && qq < m) ? hget(U, p, qq) : mk<double>(0, 0);
            cplx<double> b10 = (q < m && pp < m) ? hget(U, q, pp) : mk<double>(0, 0);
            cplx<double> b11 = (q < m && qq < m) ? hget(U, q, qq) : mk<double>(0, 0);
            if (rowK && rs[K] != 0.0) {  // rows: [c, -s e^{i phi}; s, c e^{i phi}]
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
            if (colQ && rs[Q] != 0.0) {  // columns: [c, s; -s e^{-i phi}, c e^{-i phi}]
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
            if (p < m && pp < m) hset(U, p, pp, b00);
            if (p < m && qq < m) hset(U, p, qq, b01);
            if (q < m && pp < m) hset(U, q, pp, b10);
            if (q < m && qq < m) hset(U, q, qq, b11);
          } else if (it < nblk + npair) {
            const int K = it - nblk;
            int p, q;
            rr_pair(r, K, mp, p, q);
            if (p >= m || q >= m || rs[K] == 0.0) continue;
            U[tri(p, p)] = mk<double>(dp_[K], 0.0);
            U[tri(q, q)] = mk<double>(dq_[K], 0.0);
            hset(U, p, q, mk<double>(0.0, 0.0));
          } else {
            const int e = it - nblk - npair;
            const int K = e / m, i = e - K * m;
            int p, q;
            rr_pair(r, K, mp, p, q);
            if (p >= m || q >= m || rs[K] == 0.0) continue;
            const double cc = rc[K], ss = rs[K];
            const cplx<double> em = mk<double>(rex[K], -rey[K]);
            const cplx<double> xp = M[(size_t)i * ld + p], xq = M[(size_t)i * ld + q];
            const cplx<double> emq = em * xq;
            M[(size_t)i * ld + p] = mk<double>(cc * xp.x - ss * emq.x, cc * xp.y - ss * emq.y);
            M[(size_t)i * ld + q] = mk<double>(ss * xp.x + cc * emq.x, ss * xp.y + cc * emq.y);
          }
        }
        c.sync();
      }
      double off = 0.0, dia = 0.0;
      for (int e = tid; e < m * (m + 1) / 2; e += nt) {
        int i = 0;
        while (tri(i + 1, 0) <= e) ++i;
        const int j = e - tri(i, 0);
        if (masked[i] || masked[j]) continue;
        const double v = sqrt(norm2(U[e]));
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
    // ---- restore L; C = L^{-H} W[:, order[:nb]] (one column per thread)
    for (int e = tid; e < m * (m + 1) / 2; e += nt) U[e] = a.L[e];
    c.sync();
    // in place in column order[n] of W (distinct columns per thread)
    for (int n = tid; n < nb; n += nt) {
      const int col = order[n];
      a.eval[n] = a.theta[col];
      for (int i = m - 1; i >= 0; --i) {
        cplx<double> acc = M[(size_t)i * ld + col];
        for (int k = i + 1; k < m; ++k) acc = acc - conj(U[tri(k, i)]) * M[(size_t)k * ld + col];
        M[(size_t)i * ld + col] = cdiv_real(acc, U[tri(i, i)].x);
      }
    }
    c.sync();
    for (int e = tid; e < m * nb; e += nt) {
      const int i = e / nb, n = e - i * nb;
      const cplx<double> v = M[(size_t)i * ld + order[n]];
      a.Cd[e] = v;
      ((cplx<T>*)a.Ct)[e] = mk<T>((T)v.x, (T)v.y);
    }
  }
};

}  // namespace fde
