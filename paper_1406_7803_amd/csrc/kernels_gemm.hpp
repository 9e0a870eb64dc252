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

template <typename T>
struct KAhB {
  static constexpr int TI = 32, TJ = 32, KT = 64, LD = KT + 1;
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
    const int wi = wave >> 1, wj = wave & 1;  // 4 waves: a 2 x 2 grid of 16 x 16 sub-tiles
    fde_d4 re0 = {0, 0, 0, 0}, im0 = {0, 0, 0, 0}, re1 = {0, 0, 0, 0}, im1 = {0, 0, 0, 0};
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
      const int ra = (wi * 16 + (lane & 15)) * LD + (lane >> 4);
      const int rb = (wj * 16 + (lane & 15)) * LD + (lane >> 4);
#pragma unroll 4
      for (int k0 = 0; k0 < KT; k0 += 4) {
        const cplx<T> a = sA[ra + k0];
        const cplx<T> b = sB0[rb + k0];
        const double ax = a.x, ay = a.y, bx = b.x, by = b.y;
        re0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, bx, re0, 0, 0, 0);
        re0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ay, by, re0, 0, 0, 0);
        im0 = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, by, im0, 0, 0, 0);
        im0 = __builtin_amdgcn_mfma_f64_16x16x4f64(-ay, bx, im0, 0, 0, 0);
        if (two) {
          const cplx<T> h = sB1[rb + k0];
          const double hx = h.x, hy = h.y;
          re1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, hx, re1, 0, 0, 0);
          re1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ay, hy, re1, 0, 0, 0);
          im1 = __builtin_amdgcn_mfma_f64_16x16x4f64(ax, hy, im1, 0, 0, 0);
          im1 = __builtin_amdgcn_mfma_f64_16x16x4f64(-ay, hx, im1, 0, 0, 0);
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
    const int j = j0 + wj * 16 + (lane & 15);
    for (int r = 0; r < 4; ++r) {
      const int i = i0 + wi * 16 + 4 * r + (lane >> 4);
      if (i < P.ma && j < P.mb) {
        out[(size_t)i * P.mb + j] = mk<double>(re0[r], im0[r]);
        if (two) out[mab + (size_t)i * P.mb + j] = mk<double>(re1[r], im1[r]);
      }
    }
#else
    for (int o = c.tid(); o < TI * TJ; o += c.nthr()) {
      const int i = i0 + o / TJ, j = j0 + o % TJ;
      if (i < P.ma && j < P.mb) {
        out[(size_t)i * P.mb + j] = acc[o];
        if (two) out[mab + (size_t)i * P.mb + j] = acc[TI * TJ + o];
      }
    }
#endif
  }
};

}  // namespace fde
