// Batched complex C = A^H B over the plane-wave index on matrix cores.
//
// A [ma][npw] and B [mb][npw] are band-major complex arrays (row = band or
// projector, contiguous plane waves). For every chunk of plane waves the
// kernel writes FP64 partial sums part[chunk][prod][ma][mb] with
//   prod 0: sum_G conj(A_i(G)) B0_j(G),   prod 1 (optional): ... B1_j(G),
// which a second pass sums over chunks in a fixed order (deterministic).
//
// On the device the products run on v_mfma_f64_16x16x4f64 (inputs of either
// plan precision are widened to FP64, so the Gram matrices keep FP64
// accumulation): a complex product is four real MFMAs,
//   Re += Ar Br + Ai Bi,   Im += Ar Bi - Ai Br.
// Operand layout (wave64): lane l holds A[l%16][k0 + l/16] and
// B[k0 + l/16][l%16]; result register r holds C[4r + l/16][l%16].
// The host-emulation build computes the same tiles with plain loops.
#pragma once

#include "common.hpp"
#include "launch.hpp"

namespace fde {

template <typename T>
struct AhBProb {
  const cplx<T>* A;
  const cplx<T>* B0;
  const cplx<T>* B1;  // may be null
  int ma, mb, npw, nchunk, chunk;
  cplx<double>* part;  // [nchunk][nprod][ma][mb]
};

constexpr int kMaxAhB = 16;

template <typename T>
struct AhBSet {
  int n;
  AhBProb<T> p[kMaxAhB];
};

#if defined(__HIP_DEVICE_COMPILE__)
typedef double fde_d4 __attribute__((ext_vector_type(4)));
#endif

// Tile of TS x TS outputs per workgroup (TS = 32 or 64), four wavefronts in a 2 x 2 grid,
// each holding (TS/32)^2 16 x 16 sub-tiles; k chunks of KT plane waves staged in LDS.
// The 64 tile reads every operand row half as often per output as the 32 tile.
template <typename T, int TS = 32>
struct KAhB {
  static constexpr int TI = TS, TJ = TS, KT = TS == 32 ? 64 : 32, LD = KT + 1, SW = TS / 32;
  static size_t lds_bytes() {
    size_t s = sizeof(cplx<T>) * LD * (TI + 2 * TJ);
#ifdef FDE_EMULATE
    s += sizeof(cplx<double>) * 2 * TI * TJ;
#endif
    return s;
  }
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const AhBSet<T> set) {
    const AhBProb<T>& P = set.p[c.bz()];
    const int ntj = (P.mb + TJ - 1) / TJ;
    const int nti = (P.ma + TI - 1) / TI;
    if (c.bx() >= P.nchunk || c.by() >= nti * ntj) return;  // uniform per block
    // Gram products (A = B0, square): lower tiles only, written with their mirror
    const bool herm = P.B1 != nullptr && P.A == P.B0 && P.ma == P.mb;
    if (herm && c.by() % ntj > c.by() / ntj) return;  // uniform per block
    const int i0 = (c.by() / ntj) * TI, j0 = (c.by() % ntj) * TJ;
    const int g0 = c.bx() * P.chunk;
    const int gend = (g0 + P.chunk) < P.npw ? (g0 + P.chunk) : P.npw;
    const bool two = P.B1 != nullptr;
    const int npw = P.npw;
    cplx<T>* sA = (cplx<T>*)lds;
    cplx<T>* sB0 = sA + TI * LD;
    cplx<T>* sB1 = sB0 + TJ * LD;
#if defined(__HIP_DEVICE_COMPILE__)
    const int lane = c.tid() & 63, wave = c.tid() >> 6;
    const int wi = wave >> 1, wj = wave & 1;  // 4 waves: a 2 x 2 grid of (TS/2) x (TS/2) blocks
    fde_d4 re0[SW][SW], im0[SW][SW], re1[SW][SW], im1[SW][SW];
#pragma unroll
    for (int s = 0; s < SW; ++s)
#pragma unroll
      for (int u = 0; u < SW; ++u) {
        re0[s][u] = fde_d4{0, 0, 0, 0};
        im0[s][u] = fde_d4{0, 0, 0, 0};
        re1[s][u] = fde_d4{0, 0, 0, 0};
        im1[s][u] = fde_d4{0, 0, 0, 0};
      }
#else
    cplx<double>* acc = (cplx<double>*)(sB1 + TJ * LD);  // [2][TI][TJ]
    for (int o = c.tid(); o < 2 * TI * TJ; o += c.nthr()) acc[o] = mk<double>(0, 0);
#endif
    for (int gs = g0; gs < gend; gs += KT) {
      for (int idx = c.tid(); idx < TI * KT; idx += c.nthr()) {
        const int r = idx / KT, k = idx - r * KT;
        const int g = gs + k;
        const bool ok = g < gend;
        sA[r * LD + k] = (i0 + r < P.ma && ok) ? P.A[(size_t)(i0 + r) * npw + g] : mk<T>(0, 0);
        sB0[r * LD + k] = (j0 + r < P.mb && ok) ? P.B0[(size_t)(j0 + r) * npw + g] : mk<T>(0, 0);
        if (two) sB1[r * LD + k] = (j0 + r < P.mb && ok) ? P.B1[(size_t)(j0 + r) * npw + g] : mk<T>(0, 0);
      }
      c.sync();
#if defined(__HIP_DEVICE_COMPILE__)
      const int ra = (wi * (TS / 2) + (lane & 15)) * LD + (lane >> 4);
      const int rb = (wj * (TS / 2) + (lane & 15)) * LD + (lane >> 4);
#pragma unroll 4
      for (int k0 = 0; k0 < KT; k0 += 4) {
        double ax[SW], ay[SW], bx[SW], by[SW], hx[SW], hy[SW];
#pragma unroll
        for (int s = 0; s < SW; ++s) {
          const cplx<T> a = sA[ra + s * 16 * LD + k0];
          const cplx<T> b = sB0[rb + s * 16 * LD + k0];
          ax[s] = a.x;
          ay[s] = a.y;
          bx[s] = b.x;
          by[s] = b.y;
          if (two) {
            const cplx<T> h = sB1[rb + s * 16 * LD + k0];
            hx[s] = h.x;
            hy[s] = h.y;
          }
        }
#pragma unroll
        for (int s = 0; s < SW; ++s)
#pragma unroll
          for (int u = 0; u < SW; ++u) {
            re0[s][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[s], bx[u], re0[s][u], 0, 0, 0);
            re0[s][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ay[s], by[u], re0[s][u], 0, 0, 0);
            im0[s][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[s], by[u], im0[s][u], 0, 0, 0);
            im0[s][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ay[s], bx[u], im0[s][u], 0, 0, 0);
            if (two) {
              re1[s][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[s], hx[u], re1[s][u], 0, 0, 0);
              re1[s][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ay[s], hy[u], re1[s][u], 0, 0, 0);
              im1[s][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[s], hy[u], im1[s][u], 0, 0, 0);
              im1[s][u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ay[s], hx[u], im1[s][u], 0, 0, 0);
            }
          }
      }
#else
      for (int o = c.tid(); o < TI * TJ; o += c.nthr()) {
        const int i = o / TJ, j = o - i * TJ;
        double sx = 0, sy = 0, hx = 0, hy = 0;
        for (int k = 0; k < KT; ++k) {
          const cplx<T> a = sA[i * LD + k], b = sB0[j * LD + k];
          sx += (double)a.x * b.x + (double)a.y * b.y;
          sy += (double)a.x * b.y - (double)a.y * b.x;
          if (two) {
            const cplx<T> h = sB1[j * LD + k];
            hx += (double)a.x * h.x + (double)a.y * h.y;
            hy += (double)a.x * h.y - (double)a.y * h.x;
          }
        }
        acc[o].x += sx;
        acc[o].y += sy;
        acc[TI * TJ + o].x += hx;
        acc[TI * TJ + o].y += hy;
      }
#endif
      c.sync();
    }
    const int nprod = two ? 2 : 1;
    const size_t mab = (size_t)P.ma * P.mb;
    cplx<double>* out = P.part + (size_t)c.bx() * nprod * mab;
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
    for (int s = 0; s < SW; ++s)
#pragma unroll
      for (int u = 0; u < SW; ++u) {
        const int j = j0 + wj * (TS / 2) + u * 16 + (lane & 15);
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + wi * (TS / 2) + s * 16 + 4 * r + (lane >> 4);
          if (i < P.ma && j < P.mb && (!herm || j <= i)) {
            out[(size_t)i * P.mb + j] = mk<double>(re0[s][u][r], im0[s][u][r]);
            if (two) out[mab + (size_t)i * P.mb + j] = mk<double>(re1[s][u][r], im1[s][u][r]);
            if (herm && j < i) {
              out[(size_t)j * P.mb + i] = mk<double>(re0[s][u][r], -im0[s][u][r]);
              out[mab + (size_t)j * P.mb + i] = mk<double>(re1[s][u][r], -im1[s][u][r]);
            }
          }
        }
      }
#else
    for (int o = c.tid(); o < TI * TJ; o += c.nthr()) {
      const int i = i0 + o / TJ, j = j0 + o % TJ;
      if (i < P.ma && j < P.mb && (!herm || j <= i)) {
        out[(size_t)i * P.mb + j] = acc[o];
        if (two) out[mab + (size_t)i * P.mb + j] = acc[TI * TJ + o];
        if (herm && j < i) {
          out[(size_t)j * P.mb + i] = conj(acc[o]);
          out[mab + (size_t)j * P.mb + i] = conj(acc[TI * TJ + o]);
        }
      }
    }
#endif
  }
};

// Launch of KAhB over grid (nchunk, tiles, nz): the 64 tile for FP32 operands when both
// product dimensions reach 128 (fewer operand reads per output; its FP64 staging would
// not leave room for a second workgroup per CU), else the 32 tile.
template <typename T>
inline int ahb_tile(int ma, int mb) {
  return sizeof(T) == 4 && ma >= 128 && mb >= 128 ? 64 : 32;
}
template <typename T>
inline fde_status launch_ahb(unsigned nchunk, int ma, int mb, unsigned nz, const AhBSet<T>& set, hipStream_t s) {
  if (ahb_tile<T>(ma, mb) == 64) {
    using K = KAhB<T, 64>;
    const unsigned nt = (unsigned)(((ma + K::TI - 1) / K::TI) * ((mb + K::TJ - 1) / K::TJ));
    return launch<K, 256, 2>(dim3(nchunk, nt, nz), kBlock, K::lds_bytes(), s, set);
  }
  using K = KAhB<T>;
  const unsigned nt = (unsigned)(((ma + K::TI - 1) / K::TI) * ((mb + K::TJ - 1) / K::TJ));
  return launch<K>(dim3(nchunk, nt, nz), kBlock, K::lds_bytes(), s, set);
}

// ---------------------------------------------------------------------------
// The same products from FP32 inputs on BF16 matrix cores (FP32 plans only).
// Every real component x is split into NS BF16 terms, x = x_0 + x_1 (+ x_2),
// x_s = bf16(x - x_0 - ... - x_{s-1}); a real product keeps the term pairs
// (s, t) with s + t < NS: (0,0), (0,1), (1,0) for NS = 2 ("BF16x3", about 16
// significant bits) and additionally (1,1), (0,2), (2,0) for NS = 3 ("BF16x6",
// about FP32). Products of BF16 terms are exact in FP32; v_mfma_f32_16x16x16bf16_1k
// accumulates a 32-wide k tile in FP32, which is then added to FP64 sums.
// Operand layout (wave64): a[i] = A[l%16][4(l/16)+i], b[i] = B[4(l/16)+i][l%16],
// c[r] = C[4(l/16)+r][l%16]. The split terms are formed once when a tile is
// staged in LDS: planes [term][re|im][row][k] of BF16.
// ---------------------------------------------------------------------------
template <int NS>
struct KAhBSplit {
  static constexpr int TI = 32, TJ = 32, KT = 32, LDK = KT + 4;
  static constexpr int PLANE = 32 * LDK;             // one [row][k] plane (BF16)
  static constexpr int MAT = NS * 2 * PLANE;         // one matrix: NS terms x (re, im)
  static size_t lds_bytes() {
    size_t s = sizeof(unsigned short) * 3 * MAT;
#ifdef FDE_EMULATE
    s += sizeof(double) * 4 * TI * TJ;
#endif
    return s;
  }
  FDE_HD static unsigned short bf(float x) {
    unsigned u = __builtin_bit_cast(unsigned, x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
  }
  FDE_HD static float fb(unsigned short h) { return __builtin_bit_cast(float, (unsigned)h << 16); }
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const AhBSet<float> set) {
    const AhBProb<float>& P = set.p[c.bz()];
    const int ntj = (P.mb + TJ - 1) / TJ;
    const int nti = (P.ma + TI - 1) / TI;
    if (c.bx() >= P.nchunk || c.by() >= nti * ntj) return;  // uniform per block
    const int i0 = (c.by() / ntj) * TI, j0 = (c.by() % ntj) * TJ;
    const int g0 = c.bx() * P.chunk;
    const int gend = (g0 + P.chunk) < P.npw ? (g0 + P.chunk) : P.npw;
    const bool two = P.B1 != nullptr;
    const int npw = P.npw;
    unsigned short* sA = (unsigned short*)lds;
    unsigned short* sB0 = sA + MAT;
    unsigned short* sB1 = sB0 + MAT;
#if defined(__HIP_DEVICE_COMPILE__)
    typedef short s4 __attribute__((ext_vector_type(4)));
    typedef float f4 __attribute__((ext_vector_type(4)));
    const int lane = c.tid() & 63, wave = c.tid() >> 6;
    const int wi = wave >> 1, wj = wave & 1;
    double dre0[4] = {0, 0, 0, 0}, dim0[4] = {0, 0, 0, 0}, dre1[4] = {0, 0, 0, 0}, dim1[4] = {0, 0, 0, 0};
    auto ld4 = [&](const unsigned short* base, int term, int ri, int row, int k) {
      const uint2 v = *(const uint2*)(base + (term * 2 + ri) * PLANE + row * LDK + k);
      s4 r;
      r[0] = (short)(v.x & 0xffff);
      r[1] = (short)(v.x >> 16);
      r[2] = (short)(v.y & 0xffff);
      r[3] = (short)(v.y >> 16);
      return r;
    };
    auto neg = [](s4 v) {
      s4 r;
      for (int i = 0; i < 4; ++i) r[i] = (short)(v[i] ^ (short)0x8000);
      return r;
    };
#else
    double* acc = (double*)(sB1 + MAT);  // [4][TI][TJ]: re0, im0, re1, im1
    for (int o = c.tid(); o < 4 * TI * TJ; o += c.nthr()) acc[o] = 0.0;
#endif
    for (int gs = g0; gs < gend; gs += KT) {
      // one item: 4 consecutive k of one row of one matrix -> NS x 2 packed 8-byte stores
      const int nmat = two ? 3 : 2;
      for (int idx = c.tid(); idx < nmat * TI * (KT / 4); idx += c.nthr()) {
        const int mat = idx / (TI * (KT / 4)), rem = idx - mat * (TI * (KT / 4));
        const int r = rem / (KT / 4), k = 4 * (rem - r * (KT / 4));
        const cplx<float>* src = mat == 0 ? P.A : (mat == 1 ? P.B0 : P.B1);
        const int row = (mat == 0 ? i0 : j0) + r;
        const bool rok = row < (mat == 0 ? P.ma : P.mb);
        unsigned short* dst = (mat == 0 ? sA : (mat == 1 ? sB0 : sB1)) + r * LDK + k;
        float vx[4], vy[4];
        for (int q = 0; q < 4; ++q) {
          const int g = gs + k + q;
          const cplx<float> v = (rok && g < gend) ? src[(size_t)row * npw + g] : mk<float>(0, 0);
          vx[q] = v.x;
          vy[q] = v.y;
        }
        for (int t = 0; t < NS; ++t) {
          unsigned short hx[4], hy[4];
          for (int q = 0; q < 4; ++q) {
            hx[q] = bf(vx[q]);
            hy[q] = bf(vy[q]);
            vx[q] -= fb(hx[q]);
            vy[q] -= fb(hy[q]);
          }
          uint2 px, py;
          px.x = (unsigned)hx[0] | ((unsigned)hx[1] << 16);
          px.y = (unsigned)hx[2] | ((unsigned)hx[3] << 16);
          py.x = (unsigned)hy[0] | ((unsigned)hy[1] << 16);
          py.y = (unsigned)hy[2] | ((unsigned)hy[3] << 16);
          *(uint2*)(dst + (t * 2) * PLANE) = px;
          *(uint2*)(dst + (t * 2 + 1) * PLANE) = py;
        }
      }
      c.sync();
#if defined(__HIP_DEVICE_COMPILE__)
      f4 re0 = {0, 0, 0, 0}, im0 = {0, 0, 0, 0}, re1 = {0, 0, 0, 0}, im1 = {0, 0, 0, 0};
      const int ra = wi * 16 + (lane & 15), rb = wj * 16 + (lane & 15);
#pragma unroll
      for (int k0 = 0; k0 < KT; k0 += 16) {
        const int kk = k0 + 4 * (lane >> 4);
        s4 ar[NS], ai[NS], nai[NS], br[NS], bi[NS], hr[NS], hi[NS];
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          ar[t] = ld4(sA, t, 0, ra, kk);
          ai[t] = ld4(sA, t, 1, ra, kk);
          nai[t] = neg(ai[t]);
          br[t] = ld4(sB0, t, 0, rb, kk);
          bi[t] = ld4(sB0, t, 1, rb, kk);
          if (two) {
            hr[t] = ld4(sB1, t, 0, rb, kk);
            hi[t] = ld4(sB1, t, 1, rb, kk);
          }
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
#pragma unroll
          for (int t = 0; t < NS; ++t) {
            if (s + t >= NS) continue;
            re0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar[s], br[t], re0, 0, 0, 0);
            re0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ai[s], bi[t], re0, 0, 0, 0);
            im0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar[s], bi[t], im0, 0, 0, 0);
            im0 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(nai[s], br[t], im0, 0, 0, 0);
            if (two) {
              re1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar[s], hr[t], re1, 0, 0, 0);
              re1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ai[s], hi[t], re1, 0, 0, 0);
              im1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ar[s], hi[t], im1, 0, 0, 0);
              im1 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(nai[s], hr[t], im1, 0, 0, 0);
            }
          }
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        dre0[r] += re0[r];
        dim0[r] += im0[r];
        dre1[r] += re1[r];
        dim1[r] += im1[r];
      }
#else
      for (int o = c.tid(); o < TI * TJ; o += c.nthr()) {
        const int i = o / TJ, j = o - i * TJ;
        float sx = 0, sy = 0, tx = 0, ty = 0;
        for (int k = 0; k < KT; ++k)
          for (int s = 0; s < NS; ++s)
            for (int t = 0; t + s < NS; ++t) {
              const float ar = fb(sA[(s * 2) * PLANE + i * LDK + k]), ai = fb(sA[(s * 2 + 1) * PLANE + i * LDK + k]);
              const float br = fb(sB0[(t * 2) * PLANE + j * LDK + k]), bi = fb(sB0[(t * 2 + 1) * PLANE + j * LDK + k]);
              sx += ar * br + ai * bi;
              sy += ar * bi - ai * br;
              if (two) {
                const float hr = fb(sB1[(t * 2) * PLANE + j * LDK + k]), hi = fb(sB1[(t * 2 + 1) * PLANE + j * LDK + k]);
                tx += ar * hr + ai * hi;
                ty += ar * hi - ai * hr;
              }
            }
        acc[o] += sx;
        acc[TI * TJ + o] += sy;
        acc[2 * TI * TJ + o] += tx;
        acc[3 * TI * TJ + o] += ty;
      }
#endif
      c.sync();
    }
    const int nprod = two ? 2 : 1;
    const size_t mab = (size_t)P.ma * P.mb;
    cplx<double>* out = P.part + (size_t)c.bx() * nprod * mab;
#if defined(__HIP_DEVICE_COMPILE__)
    const int j = j0 + wj * 16 + (lane & 15);
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + wi * 16 + 4 * (lane >> 4) + r;
      if (i < P.ma && j < P.mb) {
        out[(size_t)i * P.mb + j] = mk<double>(dre0[r], dim0[r]);
        if (two) out[mab + (size_t)i * P.mb + j] = mk<double>(dre1[r], dim1[r]);
      }
    }
#else
    for (int o = c.tid(); o < TI * TJ; o += c.nthr()) {
      const int i = i0 + o / TJ, j = j0 + o % TJ;
      if (i < P.ma && j < P.mb) {
        out[(size_t)i * P.mb + j] = mk<double>(acc[o], acc[TI * TJ + o]);
        if (two) out[mab + (size_t)i * P.mb + j] = mk<double>(acc[2 * TI * TJ + o], acc[3 * TI * TJ + o]);
      }
    }
#endif
  }
};

// ---------------------------------------------------------------------------
// Both Gram products of a Rayleigh-Ritz problem in one pass over the plane
// waves: S = V^H V and A = V^H HV for V, HV [m][npw] (m <= 16 kGramTiles).
// One workgroup per (chunk, problem) stages all m rows of V and HV for a
// 32-wide k tile, so every input element is read from HBM once; only the
// lower-triangular 16 x 16 tiles are computed (both products are Hermitian) and
// written with their mirror. FP64 matrix cores (inputs widened), FP64 partial
// sums per chunk: part[chunk][prod][m][m].
// ---------------------------------------------------------------------------
constexpr int kGramTiles = 6;  // up to m = 96

template <typename T>
struct KGram {
  static constexpr int KT = 32, LD = KT + 1, NW = 8;
  static constexpr int MAXTP = (kGramTiles * (kGramTiles + 1) + NW - 1) / NW;  // tile-products per wave
  static constexpr int MAXLD = (2 * 16 * kGramTiles * KT + NW * 64 - 1) / (NW * 64);  // staged values per thread
  static size_t lds_bytes(int m) { return sizeof(cplx<T>) * 2 * (size_t)m * LD; }
  FDE_HD static void tile_of(int tp, int& I, int& J, int& prod) {
    prod = tp & 1;  // S and A interleaved
    int t = tp >> 1, i = 0;
    while ((i + 1) * (i + 2) / 2 <= t) ++i;
    I = i;
    J = t - i * (i + 1) / 2;
  }
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const AhBSet<T> set) {
    const AhBProb<T>& P = set.p[c.by()];
    const int m = P.ma, npw = P.npw;
    if (c.bx() >= P.nchunk) return;  // uniform per block
    const int g0 = c.bx() * P.chunk;
    const int gend = (g0 + P.chunk) < npw ? (g0 + P.chunk) : npw;
    const int nt = (m + 15) / 16, ntp = nt * (nt + 1);  // lower tiles x 2 products
    cplx<T>* sV = (cplx<T>*)lds;
    cplx<T>* sH = sV + (size_t)m * LD;
    const size_t mm = (size_t)m * m;
    cplx<double>* out = P.part + (size_t)c.bx() * 2 * mm;
#if defined(__HIP_DEVICE_COMPILE__)
    const int lane = c.tid() & 63, wave = c.tid() >> 6;
    const int col = lane & 15, kq = lane >> 4;
    fde_d4 re[MAXTP], im[MAXTP];
#pragma unroll
    for (int u = 0; u < MAXTP; ++u) {
      re[u] = fde_d4{0, 0, 0, 0};
      im[u] = fde_d4{0, 0, 0, 0};
    }
#else
    cplx<double>* acc = out;  // the chunk's own partials serve as the accumulator
    for (size_t o = c.tid(); o < 2 * mm; o += c.nthr()) acc[o] = mk<double>(0, 0);
#endif
#if defined(__HIP_DEVICE_COMPILE__)
    // the next stage's rows are fetched into registers while the current one is multiplied
    cplx<T> pre[MAXLD];
    auto fetch = [&](int gs) {
#pragma unroll
      for (int u = 0; u < MAXLD; ++u) {
        const int idx = c.tid() + NW * 64 * u;
        if (idx < 2 * m * KT) {
          const int h = idx / (m * KT), rem = idx - h * (m * KT);
          const int r = rem / KT, k = rem - r * KT;
          const int g = gs + k;
          const cplx<T>* src = h ? P.B1 : P.A;
          pre[u] = g < gend ? src[(size_t)r * npw + g] : mk<T>(0, 0);
        }
      }
    };
    auto stage = [&]() {
#pragma unroll
      for (int u = 0; u < MAXLD; ++u) {
        const int idx = c.tid() + NW * 64 * u;
        if (idx < 2 * m * KT) {
          const int h = idx / (m * KT), rem = idx - h * (m * KT);
          const int r = rem / KT, k = rem - r * KT;
          (h ? sH : sV)[r * LD + k] = pre[u];
        }
      }
    };
    fetch(g0);
    stage();
    c.sync();
#endif
    for (int gs = g0; gs < gend; gs += KT) {
#if defined(__HIP_DEVICE_COMPILE__)
      if (gs + KT < gend) fetch(gs + KT);
#pragma unroll
      for (int u = 0; u < MAXTP; ++u) {
        const int tp = wave + NW * u;
        if (tp >= ntp) break;
        int I, J, prod;
        tile_of(tp, I, J, prod);
        const int ra = 16 * I + col, rb = 16 * J + col;
        const cplx<T>* sB = prod ? sH : sV;
        for (int k0 = 0; k0 < KT; k0 += 4) {
          const cplx<T> a = ra < m ? sV[ra * LD + k0 + kq] : mk<T>(0, 0);
          const cplx<T> b = rb < m ? sB[rb * LD + k0 + kq] : mk<T>(0, 0);
          const double ax = a.x, ay = a.y, bx = b.x, by = b.y;
          re[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, bx, re[u], 0, 0, 0);
          re[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ay, by, re[u], 0, 0, 0);
          im[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, by, im[u], 0, 0, 0);
          im[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ay, bx, im[u], 0, 0, 0);
        }
      }
      c.sync();
      if (gs + KT < gend) stage();
#else
      for (int idx = c.tid(); idx < 2 * m * KT; idx += c.nthr()) {
        const int h = idx / (m * KT), rem = idx - h * (m * KT);
        const int r = rem / KT, k = rem - r * KT;
        const int g = gs + k;
        const cplx<T>* src = h ? P.B1 : P.A;
        (h ? sH : sV)[r * LD + k] = g < gend ? src[(size_t)r * npw + g] : mk<T>(0, 0);
      }
      c.sync();
      for (size_t o = c.tid(); o < 2 * mm; o += c.nthr()) {
        const int prod = (int)(o / mm), e = (int)(o - prod * mm);
        const int i = e / m, j = e - i * m;
        if (j > i) continue;
        const cplx<T>* sB = prod ? sH : sV;
        double sx = 0, sy = 0;
        for (int k = 0; k < KT; ++k) {
          const cplx<T> a = sV[i * LD + k], b = sB[j * LD + k];
          sx += (double)a.x * b.x + (double)a.y * b.y;
          sy += (double)a.x * b.y - (double)a.y * b.x;
        }
        acc[o].x += sx;
        acc[o].y += sy;
      }
#endif
      c.sync();
    }
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
    for (int u = 0; u < MAXTP; ++u) {
      const int tp = wave + NW * u;
      if (tp >= ntp) break;
      int I, J, prod;
      tile_of(tp, I, J, prod);
      cplx<double>* o = out + (size_t)prod * mm;
      const int j = 16 * J + col;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * I + 4 * r + kq;  // FP64 MFMA result layout
        if (i < m && j < m) {
          o[(size_t)i * m + j] = mk<double>(re[u][r], im[u][r]);
          if (I != J) o[(size_t)j * m + i] = mk<double>(re[u][r], -im[u][r]);
        }
      }
    }
#else
    for (size_t o = c.tid(); o < 2 * mm; o += c.nthr()) {  // mirror the lower triangle
      const int prod = (int)(o / mm), e = (int)(o - prod * mm);
      const int i = e / m, j = e - i * m;
      if (j > i) out[o] = conj(acc[(size_t)prod * mm + (size_t)j * m + i]);
    }
#endif
  }
};

// ---------------------------------------------------------------------------
// part[chunk][i][j] = sum_{G in chunk} conj(A_i(G)) B_j(G) for small ma, mb
// (<= 64 each, e.g. projectors x bands): one workgroup per chunk stages all rows
// of A and B for a 32-wide k tile, so each input element is read once; the
// 16 x 16 output tiles are spread over eight wavefronts. FP64 matrix cores.
// grid (nchunk), 512 threads.
// ---------------------------------------------------------------------------
template <typename T>
struct KAhBAll {
  static constexpr int KT = 32, LD = KT + 1, NW = 8, MAXT = 2;  // 16 tiles over 8 waves
  static size_t lds_bytes(int ma, int mb) { return sizeof(cplx<T>) * (size_t)(ma + mb) * LD; }
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const AhBProb<T> P) {
    const int ma = P.ma, mb = P.mb, npw = P.npw;
    if (c.bx() >= P.nchunk) return;
    const int g0 = c.bx() * P.chunk;
    const int gend = (g0 + P.chunk) < npw ? (g0 + P.chunk) : npw;
    const int ti = (ma + 15) / 16, tj = (mb + 15) / 16, ntl = ti * tj;
    cplx<T>* sA = (cplx<T>*)lds;
    cplx<T>* sB = sA + (size_t)ma * LD;
    cplx<double>* out = P.part + (size_t)c.bx() * ma * mb;
#if defined(__HIP_DEVICE_COMPILE__)
    const int lane = c.tid() & 63, wave = c.tid() >> 6;
    const int col = lane & 15, kq = lane >> 4;
    fde_d4 re[MAXT], im[MAXT];
#pragma unroll
    for (int u = 0; u < MAXT; ++u) {
      re[u] = fde_d4{0, 0, 0, 0};
      im[u] = fde_d4{0, 0, 0, 0};
    }
#else
    for (int o = c.tid(); o < ma * mb; o += c.nthr()) out[o] = mk<double>(0, 0);
#endif
    for (int gs = g0; gs < gend; gs += KT) {
      for (int idx = c.tid(); idx < (ma + mb) * KT; idx += c.nthr()) {
        const int r = idx / KT, k = idx - r * KT;
        const int g = gs + k;
        const cplx<T>* src = r < ma ? P.A + (size_t)r * npw : P.B0 + (size_t)(r - ma) * npw;
        sA[r * LD + k] = g < gend ? src[g] : mk<T>(0, 0);
      }
      c.sync();
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
      for (int u = 0; u < MAXT; ++u) {
        const int t = wave + NW * u;
        if (t >= ntl) break;
        const int I = t / tj, J = t - I * tj;
        const int ra = 16 * I + col, rb = 16 * J + col;
        for (int k0 = 0; k0 < KT; k0 += 4) {
          const cplx<T> a = ra < ma ? sA[ra * LD + k0 + kq] : mk<T>(0, 0);
          const cplx<T> b = rb < mb ? sB[rb * LD + k0 + kq] : mk<T>(0, 0);
          const double ax = a.x, ay = a.y, bx = b.x, by = b.y;
          re[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, bx, re[u], 0, 0, 0);
          re[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ay, by, re[u], 0, 0, 0);
          im[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, by, im[u], 0, 0, 0);
          im[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-ay, bx, im[u], 0, 0, 0);
        }
      }
#else
      for (int o = c.tid(); o < ma * mb; o += c.nthr()) {
        const int i = o / mb, j = o - i * mb;
        double sx = 0, sy = 0;
        for (int k = 0; k < KT; ++k) {
          const cplx<T> a = sA[i * LD + k], b = sB[j * LD + k];
          sx += (double)a.x * b.x + (double)a.y * b.y;
          sy += (double)a.x * b.y - (double)a.y * b.x;
        }
        out[o].x += sx;
        out[o].y += sy;
      }
#endif
      c.sync();
    }
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
    for (int u = 0; u < MAXT; ++u) {
      const int t = wave + NW * u;
      if (t >= ntl) break;
      const int I = t / tj, J = t - I * tj;
      const int j = 16 * J + col;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = 16 * I + 4 * r + kq;  // FP64 MFMA result layout
        if (i < ma && j < mb) out[(size_t)i * mb + j] = mk<double>(re[u][r], im[u][r]);
      }
    }
#endif
  }
};

}  // namespace fde
