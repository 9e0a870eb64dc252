// Plane pass of the H application and of the density with two-factor FFTs in
// LDS: every in-plane line of length N = P Q is transformed in place in two
// steps, a Q-point register DFT over the strided elements a + P b followed by
// a P-point register DFT over the contiguous block a + P k (and the mirror
// image for the forward direction), so a line is spread over P or Q lanes and
// every lane holds at most 16 complex values. The inverse column transform
// leaves the rows in "slot" order (slot k1 + P k2 holds y = Q k1 + k2), the
// row pass works on the rows in that order, and the forward column transform
// takes slot order back to natural order, so no reordering pass is needed.
//
// LDS layout against bank conflicts: in the row buffer element e = a + P k of
// a line sits at a + (P + 1) k, so the lanes of the strided steps (a fixed,
// k = lane) hit distinct banks as well as those of the contiguous ones; the
// twiddles of each step are stored in the order its lanes read them (lane
// index fastest).
//
// Rows are private to wavefronts: each of the four wavefronts owns RW rows of
// the row buffer and takes its rows of every batch through the three row steps
// with wavefront-level ordering only, so no workgroup barrier separates them.
//
// Per band and z-plane (workgroup of 256 threads; one z-plane, BPW bands):
//   1. compact plane P[y][xa] (only the nxa active x-columns) = zeros, then the
//      ncol sticks of the band at their positions
//   2. inverse y-FFT of the active columns (two steps, one barrier between)
//   3. rows, RB at a time through a row buffer R[RB][N1]:
//        step 1: Q1-point inverse DFT of the active inputs of each row
//        step 2: P1-point inverse DFT, times V_eff (or |u|^2 into the density),
//                P1-point forward DFT and twiddle, in registers
//        step 3: Q1-point forward DFT; only the active outputs are kept
//   4. forward y-FFT of the active columns
//   5. sticks = compact plane at their positions
#pragma once

#include "common.hpp"

namespace fde {

// N = P Q of the in-plane lengths this pass supports (every factor a product
// of 2, 3, 4, 5 and 8 up to 16, so both register DFTs are compile-time codelets).
struct Split2 {
  int p, q;
};
FDE_HD constexpr Split2 split2(int n) {
  switch (n) {
    case 24: return {4, 6};
    case 30: return {5, 6};
    case 36: return {6, 6};
    case 40: return {5, 8};
    case 48: return {6, 8};
    case 60: return {6, 10};
    case 72: return {8, 9};
    case 80: return {8, 10};
    case 90: return {9, 10};
    case 96: return {8, 12};
    case 120: return {10, 12};
    case 144: return {12, 12};
    case 160: return {10, 16};
    case 180: return {12, 15};
    case 240: return {15, 16};
    default: return {0, 0};
  }
}
inline bool plane4_len_ok(int n) { return split2(n).p > 0; }

// Twiddle tables of one line length N = P Q (w = exp(-2 pi i / N)):
// ta[k P + a] = w^{a k} (a < P, k < Q) for the steps whose lane is a, and
// tb[m Q + k2] = w^{k2 m} (k2 < Q, m < P) for those whose lane is k2.

// Inverse, step 1 (lane a < P): Q-point DFT over positions a + P b, twiddle
// w^{a k}, back to positions a + P k. L: line base, es: element stride.
template <typename T, int N>
FDE_HD void inv_step1(cplx<T>* L, int es, int a, const cplx<T>* ta) {
  constexpr int P = split2(N).p, Q = split2(N).q;
  cplx<T> v[Q];
#pragma unroll
  for (int b = 0; b < Q; ++b) v[b] = L[(a + P * b) * es];
  reg_fft<T, true, Q>(v, nullptr);
#pragma unroll
  for (int k = 1; k < Q; ++k) v[k] = cmulc(ta[k * P + a], v[k]);
#pragma unroll
  for (int k = 0; k < Q; ++k) L[(a + P * k) * es] = v[k];
}

// Inverse, step 2: lane k2 < Q, P-point DFT over the contiguous block k2 P + a;
// output y = Q k1 + k2 lands in slot k1 + P k2.
template <typename T, int N>
FDE_HD void inv_step2(cplx<T>* L, int es, int k2) {
  constexpr int P = split2(N).p;
  cplx<T> v[P];
#pragma unroll
  for (int a = 0; a < P; ++a) v[a] = L[(a + P * k2) * es];
  reg_fft<T, true, P>(v, nullptr);
#pragma unroll
  for (int k1 = 0; k1 < P; ++k1) L[(k1 + P * k2) * es] = v[k1];
}

// Forward, step 1: lane k2 < Q, P-point DFT over slots k1 + P k2 (values at
// y = Q k1 + k2), twiddle w^{-k2 m1}, back to slots m1 + P k2.
template <typename T, int N>
FDE_HD void fwd_step1(cplx<T>* L, int es, int k2, const cplx<T>* tb) {
  constexpr int P = split2(N).p, Q = split2(N).q;
  cplx<T> v[P];
#pragma unroll
  for (int k1 = 0; k1 < P; ++k1) v[k1] = L[(k1 + P * k2) * es];
  reg_fft<T, false, P>(v, nullptr);
#pragma unroll
  for (int m1 = 1; m1 < P; ++m1) v[m1] = tb[m1 * Q + k2] * v[m1];
#pragma unroll
  for (int m1 = 0; m1 < P; ++m1) L[(m1 + P * k2) * es] = v[m1];
}

// Forward, step 2: lane m1 < P, Q-point DFT over slots m1 + P k2; the result
// F[m1 + P m2] lands in slot m1 + P m2 (natural order).
template <typename T, int N>
FDE_HD void fwd_step2(cplx<T>* L, int es, int m1) {
  constexpr int P = split2(N).p, Q = split2(N).q;
  cplx<T> v[Q];
#pragma unroll
  for (int k2 = 0; k2 < Q; ++k2) v[k2] = L[(m1 + P * k2) * es];
  reg_fft<T, false, Q>(v, nullptr);
#pragma unroll
  for (int m2 = 0; m2 < Q; ++m2) L[(m1 + P * m2) * es] = v[m2];
}

// Dispatch over the supported lengths (runtime n, compile-time codelets).
#define FDE_SPLIT2_CASES(X) \
  X(24) X(30) X(36) X(40) X(48) X(60) X(72) X(80) X(90) X(96) X(120) X(144) X(160) X(180) X(240)

// Column passes of the compact plane: the nxa lines are columns xa (element
// stride nxa). Lanes run with xa fastest, so neighbouring lanes touch
// neighbouring LDS words.
template <typename T, bool INV, class Ctx>
FDE_HD void plane4_columns(const Ctx& c, cplx<T>* P, int N2, int nxa, const cplx<T>* ta2, const cplx<T>* tb2) {
  const Split2 sp = split2(N2);
  const int n1 = INV ? sp.p : sp.q;  // lanes per line in the first step
  const int n2 = INV ? sp.q : sp.p;
  for (int q = c.tid(); q < nxa * n1; q += c.nthr()) {
    const int j = q / nxa, xa = q - j * nxa;
    switch (N2) {
#define FDE_C1(NN) \
  case NN:         \
    if (INV) inv_step1<T, NN>(P + xa, nxa, j, ta2); else fwd_step1<T, NN>(P + xa, nxa, j, tb2); break;
      FDE_SPLIT2_CASES(FDE_C1)
#undef FDE_C1
      default: break;
    }
  }
  c.sync();
  for (int q = c.tid(); q < nxa * n2; q += c.nthr()) {
    const int j = q / nxa, xa = q - j * nxa;
    switch (N2) {
#define FDE_C2(NN) \
  case NN:         \
    if (INV) inv_step2<T, NN>(P + xa, nxa, j); else fwd_step2<T, NN>(P + xa, nxa, j); break;
      FDE_SPLIT2_CASES(FDE_C2)
#undef FDE_C2
      default: break;
    }
  }
  c.sync();
}

// Row-buffer length of a line of N = P Q points (element a + P k at a + (P + 1) k).
FDE_HD constexpr int rrow_len(int n) { return n + split2(n).q; }

// Row step 1 for row r of the batch (plane slot s): lane a gathers the active
// inputs e = a + P1 b (centred index of e in [mlo, mlo + nxa)), Q1-point
// inverse DFT, twiddle, into R[r] at element a + P1 k.
template <typename T, int N>
FDE_HD void row_step1(const cplx<T>* Prow, cplx<T>* Rr, int a, int nxa, int mlo, const cplx<T>* ta) {
  constexpr int P = split2(N).p, Q = split2(N).q;
  cplx<T> v[Q];
#pragma unroll
  for (int b = 0; b < Q; ++b) {
    const int e = a + P * b;
    const int xa = (e <= N / 2 ? e : e - N) - mlo;
    const bool ok = (unsigned)xa < (unsigned)nxa;
    const cplx<T> val = Prow[ok ? xa : 0];
    v[b] = ok ? val : mk<T>(0, 0);
  }
  reg_fft<T, true, Q>(v, nullptr);
#pragma unroll
  for (int k = 1; k < Q; ++k) v[k] = cmulc(ta[k * P + a], v[k]);
#pragma unroll
  for (int k = 0; k < Q; ++k) Rr[a + (P + 1) * k] = v[k];
}

// Row step 2 of the H application (lane k2): inverse P1-point DFT gives u at
// x = Q1 k1 + k2; times V_eff (vv[k1], loaded beforehand); forward P1-point DFT
// over k1 and twiddle.
template <typename T, int N>
FDE_HD void row_step2_hv(cplx<T>* Rr, int k2, const T* vv, const cplx<T>* tb) {
  constexpr int P = split2(N).p, Q = split2(N).q;
  cplx<T> v[P];
#pragma unroll
  for (int a = 0; a < P; ++a) v[a] = Rr[a + (P + 1) * k2];
  reg_fft<T, true, P>(v, nullptr);
#pragma unroll
  for (int k1 = 0; k1 < P; ++k1) v[k1] = mk<T>(vv[k1] * v[k1].x, vv[k1] * v[k1].y);
  reg_fft<T, false, P>(v, nullptr);
#pragma unroll
  for (int m1 = 1; m1 < P; ++m1) v[m1] = tb[m1 * Q + k2] * v[m1];
#pragma unroll
  for (int m1 = 0; m1 < P; ++m1) Rr[m1 + (P + 1) * k2] = v[m1];
}

// Row step 2 of the density (lane k2): acc[x] += wgt |u(x)|^2, x = Q1 k1 + k2.
template <typename T, int N>
FDE_HD void row_step2_rho(const cplx<T>* Rr, int k2, T* __restrict__ arow, T wgt) {
  constexpr int P = split2(N).p, Q = split2(N).q;
  cplx<T> v[P];
#pragma unroll
  for (int a = 0; a < P; ++a) v[a] = Rr[a + (P + 1) * k2];
  reg_fft<T, true, P>(v, nullptr);
#pragma unroll
  for (int k1 = 0; k1 < P; ++k1) arow[Q * k1 + k2] += wgt * norm2(v[k1]);
}

// Row step 3 (lane m1): forward Q1-point DFT; the active outputs go back to the
// compact plane row.
template <typename T, int N>
FDE_HD void row_step3(const cplx<T>* Rr, cplx<T>* Prow, int m1, int nxa, int mlo) {
  constexpr int P = split2(N).p, Q = split2(N).q;
  cplx<T> v[Q];
#pragma unroll
  for (int k2 = 0; k2 < Q; ++k2) v[k2] = Rr[m1 + (P + 1) * k2];
  reg_fft<T, false, Q>(v, nullptr);
#pragma unroll
  for (int m2 = 0; m2 < Q; ++m2) {
    const int e = m1 + P * m2;
    const int xa = (e <= N / 2 ? e : e - N) - mlo;
    if ((unsigned)xa < (unsigned)nxa) Prow[xa] = v[m2];
  }
}

// Plane slot s -> row y after the inverse column transform (N2 = P2 Q2).
FDE_HD int plane4_row_of_slot(int s, int P2, int Q2) { return Q2 * (s % P2) + s / P2; }

// Wavefronts per workgroup of the pass; the row buffer holds RB = kPlane4Waves RW rows.
constexpr int kPlane4Waves = 4;

// LDS of the pass: compact plane [N2][nxa], row buffer [RB][rrow_len(N1)], the
// twiddle tables ta, tb of N1 and (when N2 differs) of N2.
template <typename T>
FDE_HD size_t plane4_lds(int N1, int N2, int nxa, int RB) {
  const size_t ntw = (size_t)2 * N1 + (N2 == N1 ? 0 : (size_t)2 * N2);
  return sizeof(cplx<T>) * ((size_t)N2 * nxa + (size_t)RB * rrow_len(N1) + ntw) + 64;
}

template <typename T>
struct Plane4Lds {
  cplx<T>*P, *R, *ta1, *tb1, *ta2, *tb2;
  FDE_HD Plane4Lds(char* lds, int N1, int N2, int nxa, int RB) {
    P = (cplx<T>*)lds;
    R = P + (size_t)N2 * nxa;
    ta1 = R + (size_t)RB * rrow_len(N1);
    tb1 = ta1 + N1;
    ta2 = N2 == N1 ? ta1 : tb1 + N1;
    tb2 = N2 == N1 ? tb1 : ta2 + N2;
  }
};

// Compact-plane position of stick i (packed x-slot | y << 16 in the stick table).
FDE_HD int plane4_pos(const int4* __restrict__ sticks, int i, int nxa) {
  const int w = sticks[i].w;
  return (w >> 16) * nxa + (w & 0xffff);
}

// Sticks of one band into / out of the compact plane, kStickBatch per thread at a time so
// that the global loads of a batch are in flight together.
constexpr int kStickBatch = 8;
template <typename T, class Ctx>
FDE_HD void plane4_scatter(const Ctx& c, cplx<T>* P, const cplx<T>* __restrict__ row,
                           const int4* __restrict__ sticks, int ncol, int nxa) {
  for (int i0 = c.tid(); i0 < ncol; i0 += kStickBatch * c.nthr()) {
    int ps[kStickBatch];
    cplx<T> v[kStickBatch];
#pragma unroll
    for (int j = 0; j < kStickBatch; ++j) {
      const int i = i0 + j * c.nthr();
      if (i < ncol) {
        ps[j] = plane4_pos(sticks, i, nxa);
        v[j] = row[i];
      }
    }
#pragma unroll
    for (int j = 0; j < kStickBatch; ++j)
      if (i0 + j * c.nthr() < ncol) P[ps[j]] = v[j];
  }
}
template <typename T, class Ctx>
FDE_HD void plane4_gather(const Ctx& c, const cplx<T>* P, cplx<T>* __restrict__ row,
                          const int4* __restrict__ sticks, int ncol, int nxa) {
  for (int i0 = c.tid(); i0 < ncol; i0 += kStickBatch * c.nthr()) {
    int ps[kStickBatch];
#pragma unroll
    for (int j = 0; j < kStickBatch; ++j) {
      const int i = i0 + j * c.nthr();
      if (i < ncol) ps[j] = plane4_pos(sticks, i, nxa);
    }
#pragma unroll
    for (int j = 0; j < kStickBatch; ++j) {
      const int i = i0 + j * c.nthr();
      if (i < ncol) row[i] = P[ps[j]];
    }
  }
}

// ta[k P + a] = w^{a k}, tb[m Q + k2] = w^{k2 m} from the natural table tw[m] = w^m.
template <typename T, class Ctx>
FDE_HD void plane4_twiddles(const Ctx& c, cplx<T>* ta, cplx<T>* tb, const cplx<T>* __restrict__ tw, int N) {
  const Split2 s = split2(N);
  for (int i = c.tid(); i < N; i += c.nthr()) {
    const int k = i / s.p, a = i - k * s.p;
    ta[i] = tw[(a * k) % N];
    const int m = i / s.q, k2 = i - m * s.q;
    tb[i] = tw[(k2 * m) % N];
  }
}

template <typename T, class Ctx>
FDE_HD void plane4_setup(const Ctx& c, Plane4Lds<T>& L, const cplx<T>* __restrict__ tw1,
                         const cplx<T>* __restrict__ tw2, int N1, int N2) {
  plane4_twiddles<T>(c, L.ta1, L.tb1, tw1, N1);
  if (N2 != N1) plane4_twiddles<T>(c, L.ta2, L.tb2, tw2, N2);
  c.sync();
}

// compact plane = zeros, then the sticks of one band; inverse y-FFT
template <typename T, class Ctx>
FDE_HD void plane4_load(const Ctx& c, Plane4Lds<T>& L, const cplx<T>* __restrict__ row,
                        const int4* __restrict__ sticks, int ncol, int nxa, int N2) {
  const int n = N2 * nxa;
  for (int i = c.tid(); i < n; i += c.nthr()) L.P[i] = mk<T>(0, 0);
  c.sync();
  plane4_scatter<T>(c, L.P, row, sticks, ncol, nxa);
  c.sync();
  plane4_columns<T, true>(c, L.P, N2, nxa, L.ta2, L.tb2);
}

// The row steps of the H application for one band: wavefront w takes rows y0 + w RW + r
// (r < RW) of each batch into row-buffer rows w RW + r. Each lane's V_eff values for step 2
// are loaded at the start of step 1, so their latency is spent on step 1's arithmetic.
template <typename T, int N1, class Ctx>
FDE_HD void plane4_rows_h(const Ctx& c, Plane4Lds<T>& L, int N2, int nxa, int mlo, int RB, const T* __restrict__ vz,
                          Split2 s2) {
  constexpr int P = split2(N1).p, Q = split2(N1).q, RS = rrow_len(N1);
  const int RW = RB / kPlane4Waves;
#if defined(__HIP_DEVICE_COMPILE__)
  constexpr int NL = 1;
#else
  constexpr int NL = 64 * kPlane4Waves;  // the serial host run keeps every lane's values
#endif
  T vv[NL][P];
  for (int y0 = 0; y0 < N2; y0 += RB) {
    for (int q = c.tid(); q < 64 * kPlane4Waves; q += c.nthr()) {
      const int w = q >> 6, l = q & 63;
      const int r2 = l / Q, k2 = l - r2 * Q, y2 = y0 + w * RW + r2;
      if (r2 < RW && y2 < N2) {
        const T* vrow = vz + (size_t)plane4_row_of_slot(y2, s2.p, s2.q) * N1;
#pragma unroll
        for (int k1 = 0; k1 < P; ++k1) vv[NL == 1 ? 0 : q][k1] = vrow[Q * k1 + k2];
      }
      const int r = l / P, a = l - r * P, y = y0 + w * RW + r;
      if (r >= RW || y >= N2) continue;
      row_step1<T, N1>(L.P + (size_t)y * nxa, L.R + (size_t)(w * RW + r) * RS, a, nxa, mlo, L.ta1);
    }
    c.wsync();
    for (int q = c.tid(); q < 64 * kPlane4Waves; q += c.nthr()) {
      const int w = q >> 6, l = q & 63, r = l / Q, k2 = l - r * Q, y = y0 + w * RW + r;
      if (r >= RW || y >= N2) continue;
      row_step2_hv<T, N1>(L.R + (size_t)(w * RW + r) * RS, k2, vv[NL == 1 ? 0 : q], L.tb1);
    }
    c.wsync();
    for (int q = c.tid(); q < 64 * kPlane4Waves; q += c.nthr()) {
      const int w = q >> 6, l = q & 63, r = l / P, m1 = l - r * P, y = y0 + w * RW + r;
      if (r >= RW || y >= N2) continue;
      row_step3<T, N1>(L.R + (size_t)(w * RW + r) * RS, L.P + (size_t)y * nxa, m1, nxa, mlo);
    }
    c.wsync();
  }
}

// H application plane pass; grid (N3, ceil(nb / BPW)), 64 kPlane4Waves threads.
template <typename T>
struct KPlaneH4 {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, cplx<T>* __restrict__ sb, int nbands, int BPW,
                         const int4* __restrict__ sticks, int ncol, int nxa, int mlo, int N1, int N2, int N3, int RB,
                         const cplx<T>* __restrict__ tw1, const cplx<T>* __restrict__ tw2,
                         const T* __restrict__ veff) {
    // the band groups of one plane run on one XCD, so its V_eff plane is read from that L2
    int z, grp;
    c.template xcd_tile<true>(z, grp);
    Plane4Lds<T> L(lds, N1, N2, nxa, RB);
    plane4_setup<T>(c, L, tw1, tw2, N1, N2);
    const Split2 s2 = split2(N2);
    const T* vz = veff + (size_t)z * N1 * N2;
    const int b0 = grp * BPW;
    for (int band = b0; band < b0 + BPW && band < nbands; ++band) {
      cplx<T>* row = sb + ((size_t)band * N3 + z) * stick_stride(ncol);
      plane4_load<T>(c, L, row, sticks, ncol, nxa, N2);
      switch (N1) {
#define FDE_RH(NN) case NN: plane4_rows_h<T, NN>(c, L, N2, nxa, mlo, RB, vz, s2); break;
        FDE_SPLIT2_CASES(FDE_RH)
#undef FDE_RH
        default: break;
      }
      c.sync();
      plane4_columns<T, false>(c, L.P, N2, nxa, L.ta2, L.tb2);
      plane4_gather<T>(c, L.P, row, sticks, ncol, nxa);
      c.sync();
    }
  }
};

// Density plane pass: out[group][z] = scale sum_n occw_n |u_n|^2 over the
// workgroup's bands, accumulated in place in the output plane (zeroed first).
template <typename T>
struct KPlaneRho4 {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const cplx<T>* __restrict__ sb, int nbands, int BPW,
                         const double* __restrict__ occw, const int4* __restrict__ sticks, int ncol, int nxa, int mlo,
                         int N1, int N2, int N3, int RB, const cplx<T>* __restrict__ tw1,
                         const cplx<T>* __restrict__ tw2, T* __restrict__ out, double scale) {
    const int z = c.bx();
    Plane4Lds<T> L(lds, N1, N2, nxa, RB);
    plane4_setup<T>(c, L, tw1, tw2, N1, N2);
    const Split2 s1 = split2(N1), s2 = split2(N2);
    const int RS = rrow_len(N1), RW = RB / kPlane4Waves;
    T* o = out + ((size_t)c.by() * N3 + z) * N1 * N2;
    for (int i = c.tid(); i < N1 * N2; i += c.nthr()) o[i] = T(0);
    const int b0 = c.by() * BPW;
    for (int band = b0; band < b0 + BPW && band < nbands; ++band) {
      const T wgt = (T)(occw[band] * scale);
      const cplx<T>* row = sb + ((size_t)band * N3 + z) * stick_stride(ncol);
      plane4_load<T>(c, L, row, sticks, ncol, nxa, N2);
      // wavefront w owns rows y0 + w RW + r of each batch, in every band, so its
      // accumulation into those output rows is never shared
      for (int y0 = 0; y0 < N2; y0 += RB) {
        for (int q = c.tid(); q < 64 * kPlane4Waves; q += c.nthr()) {
          const int w = q >> 6, l = q & 63, r = l / s1.p, a = l - r * s1.p, y = y0 + w * RW + r;
          if (r >= RW || y >= N2) continue;
          const cplx<T>* Prow = L.P + (size_t)y * nxa;
          cplx<T>* Rr = L.R + (size_t)(w * RW + r) * RS;
          switch (N1) {
#define FDE_R1(NN) case NN: row_step1<T, NN>(Prow, Rr, a, nxa, mlo, L.ta1); break;
            FDE_SPLIT2_CASES(FDE_R1)
#undef FDE_R1
            default: break;
          }
        }
        c.wsync();
        for (int q = c.tid(); q < 64 * kPlane4Waves; q += c.nthr()) {
          const int w = q >> 6, l = q & 63, r = l / s1.q, k2 = l - r * s1.q, y = y0 + w * RW + r;
          if (r >= RW || y >= N2) continue;
          T* arow = o + (size_t)plane4_row_of_slot(y, s2.p, s2.q) * N1;
          const cplx<T>* Rr = L.R + (size_t)(w * RW + r) * RS;
          switch (N1) {
#define FDE_R2(NN) case NN: row_step2_rho<T, NN>(Rr, k2, arow, wgt); break;
            FDE_SPLIT2_CASES(FDE_R2)
#undef FDE_R2
            default: break;
          }
        }
        c.wsync();
      }
      c.sync();
    }
  }
};

}  // namespace fde
