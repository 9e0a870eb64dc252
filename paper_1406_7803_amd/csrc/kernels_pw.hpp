// Plane-wave kernels: the H|psi> FFT sandwich, the density, and the
// Kleinman-Bylander projector products.
//
// Data flow of one band-apply (Eq. KS; coefficients on the sphere S_k):
//   psi [nb][npw] --KZInv--> sticks [nb][N3][ncs] (inverse z-FFT of each
//   z-stick of the sphere) --KPlaneH--> same layout (per z-plane: inverse y-FFT
//   on the active x-columns, inverse x-FFT per row, times V_eff, forward x-FFT,
//   forward y-FFT, keep the sticks) --KZFwd--> hpsi [nb][npw] (forward z-FFT,
//   1/N, plus |k+G|^2/2 psi).
// The sticks buffer holds, for every z-plane, the ncol sticks contiguously
// (row stride ncs = stick_stride(ncol), 128-byte aligned rows) so both the
// z-passes and the plane pass read and write it coalesced.
#pragma once

#include "common.hpp"

namespace fde {

constexpr int kBlk = 256;  // nominal threads per block of element-wise kernels

struct KVec {
  double kf[3];
  double b[3];
};

// |k+G|^2 / 2 for G = (m1, m2, m3), evaluated exactly as the plan's sphere test.
FDE_HD double kin_of(const KVec& k, int m1, int m2, int m3) {
  const double q1 = (m1 + k.kf[0]) * k.b[0];
  const double q2 = (m2 + k.kf[1]) * k.b[1];
  const double q3 = (m3 + k.kf[2]) * k.b[2];
  return 0.5 * (q1 * q1 + q2 * q2 + q3 * q3);
}

FDE_HD void unpack_mill(int p, int& m1, int& m2, int& m3) {
  m1 = (p & 1023) - 512;
  m2 = ((p >> 10) & 1023) - 512;
  m3 = ((p >> 20) & 1023) - 512;
}

// ---------------------------------------------------------------------------
// Inverse z-FFT of SZ sticks of one band: grid (ceil(ncol/SZ), nb).
// LDS: 2*N3*SZ + N3 complex.
// ---------------------------------------------------------------------------
template <typename T>
struct KZInv {
  // LDS: two buffers of N3 x (SZ + 1) (padded stride against bank conflicts) + N3 twiddles
  FDE_HD static size_t lds_bytes(int N3, int SZ) { return sizeof(cplx<T>) * ((size_t)2 * N3 * (SZ + 1) + N3); }
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const cplx<T>* __restrict__ psi, int npw,
                         const int4* __restrict__ sticks, int ncol, Radix r3, const cplx<T>* __restrict__ tw,
                         cplx<T>* __restrict__ sb, int SZ) {
    const int N3 = r3.n;
    const int ES = SZ + 1;
    // neighbouring stick groups of a band on one XCD (their row segments share cache lines)
    int grp, band;
    c.template xcd_tile<false>(grp, band);
    const int c0 = grp * SZ;
    const int nsz = (ncol - c0) < SZ ? (ncol - c0) : SZ;
    cplx<T>* a = (cplx<T>*)lds;
    cplx<T>* b = a + N3 * ES;
    cplx<T>* twl = b + N3 * ES;
    for (int i = c.tid(); i < N3; i += c.nthr()) twl[i] = tw[i];
    for (int i = c.tid(); i < N3 * ES; i += c.nthr()) a[i] = mk<T>(0, 0);
    c.sync();
    const cplx<T>* pb = psi + (size_t)band * npw;
    for (int idx = c.tid(); idx < SZ * N3; idx += c.nthr()) {
      const int s = idx / N3, t = idx - s * N3;
      if (s < nsz) {
        const int4 st = sticks[c0 + s];
        if (t < st.y) a[imod(st.z + t, N3) * ES + s] = pb[st.x + t];
      }
    }
    c.sync();
    cplx<T>* r = lds_fft_any<T, true>(c, a, b, SZ, 1, ES, r3, twl);
    const int ncs = stick_stride(ncol);
    cplx<T>* ob = sb + (size_t)band * N3 * ncs;
    for (int idx = c.tid(); idx < N3 * SZ; idx += c.nthr()) {
      const int z = idx / SZ, s = idx - z * SZ;
      if (s < nsz) ob[(size_t)z * ncs + c0 + s] = r[z * ES + s];
    }
  }
};

// ---------------------------------------------------------------------------
// Forward z-FFT of SZ sticks, gather of the sphere, 1/N and kinetic term:
//   hpsi(G) = (1/N) FFT_z(...)(G) + |k+G|^2/2 psi(G).   grid (ceil(ncol/SZ), nb)
// ---------------------------------------------------------------------------
template <typename T>
struct KZFwd {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const cplx<T>* __restrict__ sb, const cplx<T>* __restrict__ psi,
                         cplx<T>* __restrict__ hpsi, int npw, const int4* __restrict__ sticks,
                         const int* __restrict__ xlist, int ncol, int N1, int N2, Radix r3,
                         const cplx<T>* __restrict__ tw, KVec kv, double invN, int SZ) {
    const int N3 = r3.n;
    const int ES = SZ + 1;
    // neighbouring stick groups of a band on one XCD: row segments narrower than a cache
    // line are then fetched once, not once per XCD
    int grp, band;
    c.template xcd_tile<false>(grp, band);
    const int c0 = grp * SZ;
    const int nsz = (ncol - c0) < SZ ? (ncol - c0) : SZ;
    cplx<T>* a = (cplx<T>*)lds;
    cplx<T>* b = a + N3 * ES;
    cplx<T>* twl = b + N3 * ES;
    for (int i = c.tid(); i < N3; i += c.nthr()) twl[i] = tw[i];
    const int ncs = stick_stride(ncol);
    const cplx<T>* ib = sb + (size_t)band * N3 * ncs;
    for (int idx = c.tid(); idx < N3 * SZ; idx += c.nthr()) {
      const int z = idx / SZ, s = idx - z * SZ;
      a[z * ES + s] = s < nsz ? ib[(size_t)z * ncs + c0 + s] : mk<T>(0, 0);
    }
    c.sync();
    cplx<T>* r = lds_fft_any<T, false>(c, a, b, SZ, 1, ES, r3, twl);
    const cplx<T>* pb = psi + (size_t)band * npw;
    cplx<T>* hb = hpsi + (size_t)band * npw;
    for (int idx = c.tid(); idx < SZ * N3; idx += c.nthr()) {
      const int s = idx / N3, t = idx - s * N3;
      if (s < nsz) {
        const int4 st = sticks[c0 + s];
        if (t < st.y) {
          const int g = st.x + t;
          const int m1 = centred(xlist[st.w & 0xffff], N1);
          const int m2 = centred(st.w >> 16, N2);
          const T kin = (T)kin_of(kv, m1, m2, st.z + t);
          const cplx<T> v = r[imod(st.z + t, N3) * ES + s];
          const cplx<T> p = pb[g];
          hb[g] = mk<T>((T)invN * v.x + kin * p.x, (T)invN * v.y + kin * p.y);
        }
      }
    }
  }
};

// ---------------------------------------------------------------------------
// z-FFTs of length N3 = P Q in registers (four-step): the P threads of a stick each
// transform the Q elements z = P n1 + n2 (own n2) in registers, apply the twiddle
// W^{n2 k1}, exchange through LDS inside their wavefront, and transform the P values
// of each row k1 (result X[k1 + Q k2]). 64 / P sticks per wavefront, four wavefronts per
// workgroup; no workgroup barrier. grid (ceil(ncol / (256 / P)), nb). tw: the N3 twiddles.
// In the exchange buffer of a stick, row k1 starts at k1 (P + 1): the step-2 lanes (one
// row each) then read distinct banks; stick buffers start 8 banks apart.
// ---------------------------------------------------------------------------
template <typename T, int P, int Q>
struct ZReg {
  // sticks per wavefront, rows per thread in step 2, wavefronts per block (the block's
  // 4 SPW consecutive sticks share cache lines of the stick buffer, so they stay on one CU)
  static constexpr int N = P * Q, SPW = 64 / P, RPT = (Q + P - 1) / P, WPB = 4, SPB = WPB * SPW;
  static constexpr int RS = P + 1;  // row stride of the exchange buffer
  // complex values per stick buffer: at least Q RS (and N), 32-bit word count = 8 mod 32
  static constexpr int SB = [] {
    constexpr int w = (int)(sizeof(cplx<T>) / 4);
    int s = Q * RS > N ? Q * RS : N;
    while ((s * w) % 32 != 8) ++s;
    return s;
  }();
  FDE_HD static size_t lds_bytes() { return sizeof(cplx<T>) * (size_t)SPB * SB; }
  // step 1 for lane l: v = the stick's elements P n1 + n2 (filled by the caller), transformed,
  // twiddled, written to buf [stick][k1][n2]
  template <bool INV>
  FDE_HD static void step1(cplx<T>* v, const cplx<T>* __restrict__ tw, cplx<T>* sbuf, int n2) {
    reg_fft<T, INV, Q>(v, nullptr);
#pragma unroll
    for (int k1 = 1; k1 < Q; ++k1) {
      const cplx<T> w = tw[(n2 * k1) % N];
      v[k1] = INV ? cmulc(w, v[k1]) : w * v[k1];
    }
#pragma unroll
    for (int k1 = 0; k1 < Q; ++k1) sbuf[k1 * RS + n2] = v[k1];
  }
  // step 2 for lane l: rows k1 = r, r + P, ... of the stick: u[j][k2] = X[k1 + Q k2]
  template <bool INV>
  FDE_HD static void step2(cplx<T> (&u)[RPT][P], const cplx<T>* sbuf, int r) {
#pragma unroll
    for (int j = 0; j < RPT; ++j) {
      const int k1 = r + P * j;
      if (k1 < Q) {
#pragma unroll
        for (int n2 = 0; n2 < P; ++n2) u[j][n2] = sbuf[k1 * RS + n2];
        reg_fft<T, INV, P>(u[j], nullptr);
      }
    }
  }
};

template <typename T, int P, int Q>
struct KZInvReg {
  using Z = ZReg<T, P, Q>;
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const cplx<T>* __restrict__ psi, int npw,
                         const int4* __restrict__ sticks, int ncol, const cplx<T>* __restrict__ tw,
                         cplx<T>* __restrict__ sb) {
    constexpr int N = Z::N;
    const int band = c.by();
    const cplx<T>* pb = psi + (size_t)band * npw;
    const int ncs = stick_stride(ncol);
    cplx<T>* ob = sb + (size_t)band * N * ncs;
    cplx<T>* buf = (cplx<T>*)lds;
    for (int q = c.tid(); q < 64 * Z::WPB; q += c.nthr()) {
      const int w = q >> 6, l = q & 63;
      const int s0 = (c.bx() * Z::WPB + w) * Z::SPW;  // this wavefront's first stick
      const int s = s0 + l / P, n2 = l % P;
      if (s >= ncol) continue;
      const int4 st = sticks[s];
      cplx<T> v[Q];
#pragma unroll
      for (int n1 = 0; n1 < Q; ++n1) {
        const int t = imod(P * n1 + n2 - st.z, N);
        v[n1] = t < st.y ? pb[st.x + t] : mk<T>(0, 0);
      }
      Z::template step1<true>(v, tw, buf + (w * Z::SPW + l / P) * Z::SB, n2);
    }
    c.wsync();
    // sticks fastest along the lanes for the stores (adjacent lanes write one row segment)
    for (int q = c.tid(); q < 64 * Z::WPB; q += c.nthr()) {
      const int w = q >> 6, l = q & 63;
      const int sl = l % Z::SPW, r = l / Z::SPW;
      const int s = (c.bx() * Z::WPB + w) * Z::SPW + sl;
      if (s >= ncol || r >= Q) continue;
      cplx<T> u[Z::RPT][P];
      Z::template step2<true>(u, buf + (w * Z::SPW + sl) * Z::SB, r);
#pragma unroll
      for (int j = 0; j < Z::RPT; ++j) {
        const int k1 = r + P * j;
        if (k1 < Q) {
#pragma unroll
          for (int k2 = 0; k2 < P; ++k2) ob[(size_t)(k1 + Q * k2) * ncs + s] = u[j][k2];
        }
      }
    }
  }
};

template <typename T, int P, int Q>
struct KZFwdReg {
  using Z = ZReg<T, P, Q>;
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const cplx<T>* __restrict__ sb, const cplx<T>* __restrict__ psi,
                         cplx<T>* __restrict__ hpsi, int npw, const int4* __restrict__ sticks,
                         const int* __restrict__ xlist, int ncol, int N1, int N2, const cplx<T>* __restrict__ tw,
                         KVec kv, double invN) {
    constexpr int N = Z::N;
    const int band = c.by();
    const int ncs = stick_stride(ncol);
    const cplx<T>* ib = sb + (size_t)band * N * ncs;
    cplx<T>* buf = (cplx<T>*)lds;
    // sticks fastest along the lanes: lanes reading one stick row are adjacent, so a load
    // instruction fetches whole row segments of the wavefront's sticks
    for (int q = c.tid(); q < 64 * Z::WPB; q += c.nthr()) {
      const int w = q >> 6, l = q & 63;
      const int sl = l % Z::SPW, n2 = l / Z::SPW;
      const int s = (c.bx() * Z::WPB + w) * Z::SPW + sl;
      if (s >= ncol) continue;
      cplx<T> v[Q];
#pragma unroll
      for (int n1 = 0; n1 < Q; ++n1) v[n1] = ib[(size_t)(P * n1 + n2) * ncs + s];
      Z::template step1<false>(v, tw, buf + (w * Z::SPW + sl) * Z::SB, n2);
    }
    c.wsync();
    // every row of a stick is read before any lane of that stick overwrites the buffer
    // (the serial host run keeps all lanes' rows)
#if defined(__HIP_DEVICE_COMPILE__)
    constexpr int NL = 1;
#else
    constexpr int NL = 64 * Z::WPB;
#endif
    cplx<T> u[NL][Z::RPT][P];
    for (int q = c.tid(); q < 64 * Z::WPB; q += c.nthr()) {
      const int w = q >> 6, l = q & 63;
      const int s = (c.bx() * Z::WPB + w) * Z::SPW + l / P, r = l % P;
      if (s >= ncol || r >= Q) continue;
      Z::template step2<false>(u[NL == 1 ? 0 : q], buf + (w * Z::SPW + l / P) * Z::SB, r);
    }
    c.wsync();
    for (int q = c.tid(); q < 64 * Z::WPB; q += c.nthr()) {
      const int w = q >> 6, l = q & 63;
      const int s = (c.bx() * Z::WPB + w) * Z::SPW + l / P, r = l % P;
      if (s >= ncol || r >= Q) continue;
      cplx<T>* sbuf = buf + (w * Z::SPW + l / P) * Z::SB;
#pragma unroll
      for (int j = 0; j < Z::RPT; ++j) {
        const int k1 = r + P * j;
        if (k1 < Q) {
#pragma unroll
          for (int k2 = 0; k2 < P; ++k2) sbuf[k1 + Q * k2] = u[NL == 1 ? 0 : q][j][k2];
        }
      }
    }
    c.wsync();
    // gather of the sphere, 1/N and the kinetic term
    const cplx<T>* pb = psi + (size_t)band * npw;
    cplx<T>* hb = hpsi + (size_t)band * npw;
    for (int q = c.tid(); q < 64 * Z::WPB; q += c.nthr()) {
      const int w = q >> 6, l = q & 63;
      const int s = (c.bx() * Z::WPB + w) * Z::SPW + l / P, n2 = l % P;
      if (s >= ncol) continue;
      const int4 st = sticks[s];
      const cplx<T>* sbuf = buf + (w * Z::SPW + l / P) * Z::SB;
      const int m1 = centred(xlist[st.w & 0xffff], N1);
      const int m2 = centred(st.w >> 16, N2);
      for (int t = n2; t < st.y; t += P) {
        const int g = st.x + t;
        const T kin = (T)kin_of(kv, m1, m2, st.z + t);
        const cplx<T> v = sbuf[imod(st.z + t, N)];
        const cplx<T> p = pb[g];
        hb[g] = mk<T>((T)invN * v.x + kin * p.x, (T)invN * v.y + kin * p.y);
      }
    }
  }
};

// ---------------------------------------------------------------------------
// Plane pass, shared by H application and density. Layout in LDS:
//   P0, P1 : [N2][nxa]   the active x-columns of the plane (ping-pong)
//   R0, R1 : [RB][N1]    a batch of full rows (ping-pong)
//   tw1[N1], tw2[N2], stk[ncol] (packed xa | iy << 16)
// ---------------------------------------------------------------------------
template <typename T>
struct PlaneLds {
  cplx<T>*P0, *P1, *R0, *R1, *tw1, *tw2;
  int* stk;
  T* acc;  // density accumulator [N2][N1] (density pass only)
  FDE_HD static size_t bytes(int N1, int N2, int nxa, int RB, int ncol, bool with_acc) {
    size_t s = sizeof(cplx<T>) * ((size_t)2 * N2 * nxa + (size_t)2 * RB * N1 + N1 + N2);
    s += sizeof(int) * (size_t)ncol;
    s = (s + 15) & ~(size_t)15;
    if (with_acc) s += sizeof(T) * (size_t)N1 * N2;
    return s;
  }
  FDE_HD PlaneLds(char* lds, int N1, int N2, int nxa, int RB, int ncol) {
    P0 = (cplx<T>*)lds;
    P1 = P0 + (size_t)N2 * nxa;
    R0 = P1 + (size_t)N2 * nxa;
    R1 = R0 + (size_t)RB * N1;
    tw1 = R1 + (size_t)RB * N1;
    tw2 = tw1 + N1;
    stk = (int*)(tw2 + N2);
    size_t off = sizeof(cplx<T>) * ((size_t)2 * N2 * nxa + (size_t)2 * RB * N1 + N1 + N2) + sizeof(int) * (size_t)ncol;
    off = (off + 15) & ~(size_t)15;
    acc = (T*)(lds + off);
  }
};

template <typename T, class Ctx>
FDE_HD void plane_load_tables(const Ctx& c, PlaneLds<T>& L, const int4* __restrict__ sticks, int ncol,
                              const cplx<T>* __restrict__ tw1, const cplx<T>* __restrict__ tw2, int N1, int N2) {
  for (int i = c.tid(); i < N1; i += c.nthr()) L.tw1[i] = tw1[i];
  for (int i = c.tid(); i < N2; i += c.nthr()) L.tw2[i] = tw2[i];
  for (int i = c.tid(); i < ncol; i += c.nthr()) L.stk[i] = sticks[i].w;
}

// Scatter the ncol sticks of one plane into P0 (zeroed first); inverse y-FFT
// of the nxa active columns. Returns the buffer holding the result.
template <typename T, class Ctx>
FDE_HD cplx<T>* plane_inverse_y(const Ctx& c, PlaneLds<T>& L, const cplx<T>* __restrict__ row, int ncol, int nxa,
                                Radix r2) {
  const int N2 = r2.n;
  for (int i = c.tid(); i < N2 * nxa; i += c.nthr()) L.P0[i] = mk<T>(0, 0);
  c.sync();
  for (int i = c.tid(); i < ncol; i += c.nthr()) {
    const int w = L.stk[i];
    L.P0[(w >> 16) * nxa + (w & 0xffff)] = row[i];
  }
  c.sync();
  return lds_fft_any<T, true>(c, L.P0, L.P1, nxa, 1, nxa, r2, L.tw2);
}

template <typename T>
struct KPlaneH {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, cplx<T>* __restrict__ sb, int nbands, int BPW,
                         const int4* __restrict__ sticks, const int* __restrict__ xlist, int ncol, int nxa,
                         Radix r1, Radix r2, int N3, const cplx<T>* __restrict__ tw1,
                         const cplx<T>* __restrict__ tw2, const T* __restrict__ veff, int RB) {
    const int N1 = r1.n, N2 = r2.n;
    const int z = c.bx();
    PlaneLds<T> L(lds, N1, N2, nxa, RB, ncol);
    plane_load_tables<T>(c, L, sticks, ncol, tw1, tw2, N1, N2);
    c.sync();
    const T* vz = veff + (size_t)z * N1 * N2;
    const int b0 = c.by() * BPW;
    for (int band = b0; band < b0 + BPW && band < nbands; ++band) {
      cplx<T>* row = sb + ((size_t)band * N3 + z) * stick_stride(ncol);
      cplx<T>* P = plane_inverse_y<T>(c, L, row, ncol, nxa, r2);
      for (int y0 = 0; y0 < N2; y0 += RB) {
        const int rb = (N2 - y0) < RB ? (N2 - y0) : RB;
        for (int i = c.tid(); i < rb * N1; i += c.nthr()) L.R0[i] = mk<T>(0, 0);
        c.sync();
        for (int i = c.tid(); i < rb * nxa; i += c.nthr()) {
          const int r = i / nxa, xa = i - r * nxa;
          L.R0[r * N1 + xlist[xa]] = P[(y0 + r) * nxa + xa];
        }
        c.sync();
        cplx<T>* R = lds_fft_any<T, true>(c, L.R0, L.R1, rb, N1, 1, r1, L.tw1);
        for (int i = c.tid(); i < rb * N1; i += c.nthr()) {
          const T v = vz[(size_t)y0 * N1 + i];
          R[i] = mk<T>(v * R[i].x, v * R[i].y);
        }
        c.sync();
        cplx<T>* Rf = lds_fft_any<T, false>(c, R, R == L.R0 ? L.R1 : L.R0, rb, N1, 1, r1, L.tw1);
        for (int i = c.tid(); i < rb * nxa; i += c.nthr()) {
          const int r = i / nxa, xa = i - r * nxa;
          P[(y0 + r) * nxa + xa] = Rf[r * N1 + xlist[xa]];
        }
        c.sync();
      }
      cplx<T>* Pf = lds_fft_any<T, false>(c, P, P == L.P0 ? L.P1 : L.P0, nxa, 1, nxa, r2, L.tw2);
      for (int i = c.tid(); i < ncol; i += c.nthr()) {
        const int w = L.stk[i];
        row[i] = Pf[(w >> 16) * nxa + (w & 0xffff)];
      }
      c.sync();
    }
  }
};

// Density plane pass: acc(r) = sum_n occw_n |u_n(r)|^2 over the WG's bands;
// out[group][z][y][x] = acc * scale (scale = 1/Omega). grid (N3, ngroups)
template <typename T>
struct KPlaneRho {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const cplx<T>* __restrict__ sb, int nbands, int BPW,
                         const double* __restrict__ occw, const int4* __restrict__ sticks,
                         const int* __restrict__ xlist, int ncol, int nxa, Radix r1, Radix r2, int N3,
                         const cplx<T>* __restrict__ tw1, const cplx<T>* __restrict__ tw2, T* __restrict__ out,
                         double scale, int RB) {
    const int N1 = r1.n, N2 = r2.n;
    const int z = c.bx();
    PlaneLds<T> L(lds, N1, N2, nxa, RB, ncol);
    plane_load_tables<T>(c, L, sticks, ncol, tw1, tw2, N1, N2);
    for (int i = c.tid(); i < N1 * N2; i += c.nthr()) L.acc[i] = T(0);
    c.sync();
    const int b0 = c.by() * BPW;
    for (int band = b0; band < b0 + BPW && band < nbands; ++band) {
      const T w = (T)occw[band];
      const cplx<T>* row = sb + ((size_t)band * N3 + z) * stick_stride(ncol);
      cplx<T>* P = plane_inverse_y<T>(c, L, row, ncol, nxa, r2);
      for (int y0 = 0; y0 < N2; y0 += RB) {
        const int rb = (N2 - y0) < RB ? (N2 - y0) : RB;
        for (int i = c.tid(); i < rb * N1; i += c.nthr()) L.R0[i] = mk<T>(0, 0);
        c.sync();
        for (int i = c.tid(); i < rb * nxa; i += c.nthr()) {
          const int r = i / nxa, xa = i - r * nxa;
          L.R0[r * N1 + xlist[xa]] = P[(y0 + r) * nxa + xa];
        }
        c.sync();
        cplx<T>* R = lds_fft_any<T, true>(c, L.R0, L.R1, rb, N1, 1, r1, L.tw1);
        for (int i = c.tid(); i < rb * N1; i += c.nthr()) L.acc[y0 * N1 + i] += w * norm2(R[i]);
        c.sync();
      }
    }
    T* o = out + ((size_t)c.by() * N3 + z) * N1 * N2;
    for (int i = c.tid(); i < N1 * N2; i += c.nthr()) o[i] = (T)scale * L.acc[i];
  }
};

// rho[p] += sum_g part[g][p]
template <typename T>
struct KRhoReduce {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const T* __restrict__ part, int ngroups, size_t n, T* __restrict__ rho) {
    for (int l = c.tid(); l < kBlk; l += c.nthr()) {
      const size_t i = (size_t)c.bx() * kBlk + l;
      if (i >= n) break;
      T s = rho[i];
      for (int g = 0; g < ngroups; ++g) s += part[(size_t)g * n + i];
      rho[i] = s;
    }
  }
};

// ---------------------------------------------------------------------------
// Kleinman-Bylander products (the projections <beta_i|psi_n> come from KAhB).
// ---------------------------------------------------------------------------
// dp[o] = D_i * sum_chunk part[chunk][o], o = i nb + n. grid ceil(nproj nb / 64), 256
// threads: four chunk classes (k mod 4) of 64 consecutive outputs each, so every
// read of a chunk row is one contiguous 64-element segment; the four partial
// sums are added in a fixed order.
template <typename T>
struct KKbReduce {
  static constexpr int NO = 16, NG = 16;  // outputs per block, chunk groups per output
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const cplx<double>* __restrict__ part, int nchunk, int nproj, int nb,
                         const double* __restrict__ dkb, cplx<T>* __restrict__ dp) {
    cplx<double>* red = (cplx<double>*)lds;  // [NG][NO]
    const int nout = nproj * nb;
    for (int idx = c.tid(); idx < NG * NO; idx += c.nthr()) {
      const int w = idx / NO, l = idx - w * NO;
      const int o = c.bx() * NO + l;
      double sx = 0, sy = 0;
      if (o < nout)
        for (int k = w; k < nchunk; k += NG) {
          const cplx<double> v = part[(size_t)k * nout + o];
          sx += v.x;
          sy += v.y;
        }
      red[idx] = mk<double>(sx, sy);
    }
    c.sync();
    for (int l = c.tid(); l < NO; l += c.nthr()) {
      const int o = c.bx() * NO + l;
      if (o >= nout) continue;
      double sx = 0, sy = 0;
      for (int w = 0; w < NG; ++w) {
        sx += red[w * NO + l].x;
        sy += red[w * NO + l].y;
      }
      const double d = dkb[o / nb];
      dp[o] = mk<T>((T)(d * sx), (T)(d * sy));
    }
  }
};

// hpsi[n][G] += sum_i beta_i(G) dp[i][n]. grid ceil(npw / 64), 256 threads.
// Per block: a tile of 64 plane waves; bands in chunks of 64, each chunk's sums over
// all projectors kept in registers so that every hpsi element is read and written
// once; projectors in chunks of PC, beta and dp staged in LDS per chunk. A thread
// item is a quarter of the band chunk at one G (lanes run along G), with its 16
// sums in registers.
template <typename T>
struct KKbAdd {
  static constexpr int TG = 64, PC = sizeof(T) == 4 ? 40 : 20, NBC = 64, NQ = NBC / 4;
  static size_t lds_bytes() { return sizeof(cplx<T>) * (size_t)PC * (TG + NBC); }
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const cplx<T>* __restrict__ beta, const cplx<T>* __restrict__ dp,
                         cplx<T>* __restrict__ hpsi, int npw, int nproj, int nb) {
    cplx<T>* sB = (cplx<T>*)lds;   // [PC][TG]
    cplx<T>* sD = sB + PC * TG;    // [PC][NBC]
    const int g0 = c.bx() * TG;
    // the thread items of one pass; the host runs them one after another
    constexpr int kItems = 4 * TG;
    for (int n0 = 0; n0 < nb; n0 += NBC) {
      const int nbc = (nb - n0) < NBC ? (nb - n0) : NBC;
      for (int it0 = 0; it0 < kItems; it0 += c.nthr()) {
        const int idx = it0 + c.tid();
        const int w = idx / TG, g = idx - w * TG;
        const int qa = w * NQ, qn = (nbc - qa) < NQ ? (nbc - qa) : NQ;
        const bool live = idx < kItems && g0 + g < npw && qn > 0;
        cplx<T> acc[NQ];  // compile-time indices only: stays in registers
#pragma unroll
        for (int q = 0; q < NQ; ++q) acc[q] = mk<T>(0, 0);
        for (int i0 = 0; i0 < nproj; i0 += PC) {
          const int np = (nproj - i0) < PC ? (nproj - i0) : PC;
          c.sync();
          for (int e = c.tid(); e < np * TG; e += c.nthr()) {
            const int i = e / TG, gg = e - i * TG;
            sB[e] = (g0 + gg < npw) ? beta[(size_t)(i0 + i) * npw + g0 + gg] : mk<T>(0, 0);
          }
          for (int e = c.tid(); e < np * nbc; e += c.nthr()) {
            const int i = e / nbc, q = e - i * nbc;
            sD[i * NBC + q] = dp[(size_t)(i0 + i) * nb + n0 + q];
          }
          c.sync();
          if (live)
            for (int i = 0; i < np; ++i) {
              const cplx<T> b = sB[i * TG + g];
              const cplx<T>* d = sD + i * NBC + qa;
#pragma unroll
              for (int q = 0; q < NQ; ++q) acc[q] = acc[q] + b * d[q];
            }
        }
        if (live) {
#pragma unroll
          for (int q = 0; q < NQ; ++q) {
            if (q < qn) {
              cplx<T>& h = hpsi[(size_t)(n0 + qa + q) * npw + g0 + g];
              h = h + acc[q];
            }
          }
        }
      }
    }
  }
};

// The same add on the matrix cores (up to 512 bands): a workgroup of four wavefronts takes
// 16 CG plane waves; wavefront w accumulates the band tiles w, w + 4, ... (16 bands each)
// over all projectors, four per step (A = dp^T tile, B = beta rows of the plane waves), then
// adds the tiles into hpsi, each element read and written once. With CG = 2 every dp element
// loaded feeds two column groups. grid ceil(npw / (16 CG)).
constexpr int kKbAddTiles = 8;  // per wavefront: nb <= 4 * 8 * 16 = 512

template <typename T, int CG = 1>
struct KKbAddMfma {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const cplx<T>* __restrict__ beta, const cplx<T>* __restrict__ dp,
                         cplx<T>* __restrict__ hpsi, int npw, int nproj, int nb) {
    const int g0 = c.bx() * 16 * CG;
    if (g0 >= npw) return;
#if defined(__HIP_DEVICE_COMPILE__)
    const int lane = c.tid() & 63, w = c.tid() >> 6;
    const int col = lane & 15, kq = lane >> 4;
    const int ntile = (nb + 15) / 16;
    typedef T v4 __attribute__((ext_vector_type(4)));
    v4 re[kKbAddTiles][CG], im[kKbAddTiles][CG];
#pragma unroll
    for (int t = 0; t < kKbAddTiles; ++t)
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
        b[h] = (k < nproj && g < npw) ? beta[(size_t)k * npw + g] : mk<T>(0, 0);
      }
#pragma unroll
      for (int i = 0; i < kKbAddTiles; ++i) {
        const int n = 16 * (w + 4 * i) + col;
        a[i] = (k < nproj && n < nb) ? dp[(size_t)k * nb + n] : mk<T>(0, 0);
      }
    };
    cplx<T> bc[CG], ac[kKbAddTiles], bn[CG], an[kKbAddTiles];
    load(0, bc, ac);
    for (int k0 = 0; k0 < nproj; k0 += 4) {
      if (k0 + 4 < nproj) load(k0 + 4, bn, an);
#pragma unroll
      for (int i = 0; i < kKbAddTiles; ++i) {
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
      for (int i = 0; i < kKbAddTiles; ++i) ac[i] = an[i];
    }
#pragma unroll
    for (int h = 0; h < CG; ++h) {
      const int g = g0 + 16 * h + col;
      if (g >= npw) continue;
#pragma unroll
      for (int i = 0; i < kKbAddTiles; ++i) {
        const int t = w + 4 * i;
        if (t >= ntile) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // output row of register r: FP64 MFMA 4 r + l/16, FP32 MFMA 4 (l/16) + r
          const int n = 16 * t + (sizeof(T) == 8 ? 4 * r + kq : 4 * kq + r);
          if (n < nb) {
            cplx<T>& hv = hpsi[(size_t)n * npw + g];
            hv = mk<T>(hv.x + re[i][h][r], hv.y + im[i][h][r]);
          }
        }
      }
    }
#else
    for (int gg = g0; gg < g0 + 16 * CG && gg < npw; ++gg)
      for (int n = 0; n < nb; ++n) {
        cplx<T> acc = mk<T>(0, 0);
        for (int k = 0; k < nproj; ++k) acc = acc + beta[(size_t)k * npw + gg] * dp[(size_t)k * nb + n];
        cplx<T>& h = hpsi[(size_t)n * npw + gg];
        h = h + acc;
      }
#endif
  }
};

}  // namespace fde
