// Plane pass of the H application and of the density with whole-line FFTs
// in registers: one thread transforms one column or one row of a z-plane, so
// a band-plane needs five barriers. Used when both in-plane lengths are
// specialised (reg_plane_ok); otherwise the LDS Stockham plane pass runs.
//
// Per band and z-plane (LDS plane [N2][N1], plane position of every stick,
// V_eff plane staged once per workgroup; twiddles are compile-time constants):
//   1. plane = zeros, then the sticks at their positions
//   2. inverse y-FFT of each active x-column
//   3. per row: inverse x-FFT, times V_eff (or accumulate occw |u|^2), forward x-FFT
//   4. forward y-FFT of each active x-column
//   5. sticks = plane at their positions
#pragma once

#include "common.hpp"

namespace fde {

// Lengths with whole-line register FFTs, grouped in classes so that a kernel
// instantiation only holds codelets of similar register footprint (at most
// 256 VGPRs, two waves per SIMD, no spills):
//   FP32: class 0 = 24, 48, 60; class 1 = 72.   FP64: class 0 = 24.
inline int reg_len_class(int n, bool fp64) {
  if (fp64) return n == 24 ? 0 : -1;
  switch (n) {
    case 24: case 48: case 60: return 0;
    case 72: return 1;
    default: return -1;
  }
}

template <typename T, int CLS, int N>
FDE_HD constexpr bool reg_has() {
  if (sizeof(T) == 8) return CLS == 0 && N == 24;
  if (CLS == 0) return N == 24 || N == 48 || N == 60;
  return N == 72;
}

// Compact plane layout P[y][xa]: only the nxa active x-columns are stored.
// The active columns of a sphere form one range of centred Miller indices
// m1 in [mlo, mlo + nxa), and xa = m1 - mlo (the plan checks this).

// Column xa of the compact plane, element e (row y) at xa + y*nxa.
template <typename T, bool INV, int N>
FDE_HD void col_fft(cplx<T>* P, int xa, int nxa) {
  cplx<T> v[N];
#pragma unroll
  for (int e = 0; e < N; ++e) v[e] = P[xa + e * nxa];
  reg_fft<T, INV, N>(v, nullptr);
#pragma unroll
  for (int e = 0; e < N; ++e) P[xa + e * nxa] = v[e];
}

template <typename T, bool INV, int CLS, class Ctx>
FDE_HD void columns_fft(const Ctx& c, cplx<T>* P, int N2, int nxa) {
  for (int xa = c.tid(); xa < nxa; xa += c.nthr()) {
    switch (N2) {
      case 24: if constexpr (reg_has<T, CLS, 24>()) col_fft<T, INV, 24>(P, xa, nxa); break;
      case 48: if constexpr (reg_has<T, CLS, 48>()) col_fft<T, INV, 48>(P, xa, nxa); break;
      case 60: if constexpr (reg_has<T, CLS, 60>()) col_fft<T, INV, 60>(P, xa, nxa); break;
      case 72: if constexpr (reg_has<T, CLS, 72>()) col_fft<T, INV, 72>(P, xa, nxa); break;
      default: break;
    }
  }
}

// Expand row y of the compact plane into a full row of N (zeros outside the
// range). Branch-free: out-of-range elements load a valid slot and select 0,
// and store into the junk slot P[N2*nxa] (`junk`).
template <typename T, int N>
FDE_HD void row_load(const cplx<T>* P, int y, int nxa, int mlo, cplx<T>* v) {
  const cplx<T>* p = P + (size_t)y * nxa;
#pragma unroll
  for (int e = 0; e < N; ++e) {
    const int xa = (e <= N / 2 ? e : e - N) - mlo;
    const bool ok = (unsigned)xa < (unsigned)nxa;
    const cplx<T> val = p[ok ? xa : 0];
    v[e] = ok ? val : mk<T>(0, 0);
  }
}

template <typename T, int N>
FDE_HD void row_store(cplx<T>* P, cplx<T>* junk, int y, int nxa, int mlo, const cplx<T>* v) {
  cplx<T>* p = P + (size_t)y * nxa;
#pragma unroll
  for (int e = 0; e < N; ++e) {
    const int xa = (e <= N / 2 ? e : e - N) - mlo;
    const bool ok = (unsigned)xa < (unsigned)nxa;
    *(ok ? p + xa : junk) = v[e];
  }
}

// Row pass of the H application: inverse x-FFT, times V (from global memory), forward x-FFT.
template <typename T, int N>
FDE_HD void row_h(cplx<T>* P, cplx<T>* junk, const T* __restrict__ vrow, int y, int nxa, int mlo) {
  cplx<T> v[N];
  row_load<T, N>(P, y, nxa, mlo, v);
  reg_fft<T, true, N>(v, nullptr);
#pragma unroll
  for (int e = 0; e < N; ++e) {
    const T w = vrow[e];
    v[e] = mk<T>(w * v[e].x, w * v[e].y);
  }
  reg_fft<T, false, N>(v, nullptr);
  row_store<T, N>(P, junk, y, nxa, mlo, v);
}

// Row pass of the density: inverse x-FFT, acc += w |u|^2 (acc: full row in global scratch).
template <typename T, int N>
FDE_HD void row_rho(const cplx<T>* P, T* __restrict__ arow, int y, int nxa, int mlo, T wgt) {
  cplx<T> v[N];
  row_load<T, N>(P, y, nxa, mlo, v);
  reg_fft<T, true, N>(v, nullptr);
#pragma unroll
  for (int e = 0; e < N; ++e) arow[e] += wgt * norm2(v[e]);
}

template <typename T, int CLS, int N>
FDE_HD void row_any(cplx<T>* P, cplx<T>* junk, T* row_g, int y, int nxa, int mlo, bool dens, T w) {
  if constexpr (reg_has<T, CLS, N>()) {
    if (dens) row_rho<T, N>(P, row_g, y, nxa, mlo, w);
    else row_h<T, N>(P, junk, row_g, y, nxa, mlo);
  }
}

// rows: for the H pass row_g = V_eff plane, for the density the accumulator plane
template <typename T, int CLS, class Ctx>
FDE_HD void reg_rows(const Ctx& c, cplx<T>* P, T* plane_g, int N1, int N2, int nxa, int mlo, bool dens, T w) {
  cplx<T>* junk = P + (size_t)N2 * nxa;
  for (int y = c.tid(); y < N2; y += c.nthr()) {
    T* rg = plane_g + (size_t)y * N1;
    switch (N1) {
      case 24: row_any<T, CLS, 24>(P, junk, rg, y, nxa, mlo, dens, w); break;
      case 48: row_any<T, CLS, 48>(P, junk, rg, y, nxa, mlo, dens, w); break;
      case 60: row_any<T, CLS, 60>(P, junk, rg, y, nxa, mlo, dens, w); break;
      case 72: row_any<T, CLS, 72>(P, junk, rg, y, nxa, mlo, dens, w); break;
      default: break;
    }
  }
}

// LDS: the compact plane P [N2][nxa], one junk slot, the compact position of every stick.
template <typename T>
FDE_HD size_t reg_plane_lds(int N2, int nxa, int ncol) {
  return sizeof(cplx<T>) * ((size_t)N2 * nxa + 1) + sizeof(int) * (size_t)ncol + 64;
}

// plane <- zeros, then the sticks of one band at their compact positions (w & 0xffff = xa, w >> 16 = y)
template <typename T, class Ctx>
FDE_HD void reg_scatter(const Ctx& c, cplx<T>* P, const int* cpos, const cplx<T>* __restrict__ row, int ncol, int n) {
  for (int i = c.tid(); i < n; i += c.nthr()) P[i] = mk<T>(0, 0);
  c.sync();
  for (int i = c.tid(); i < ncol; i += c.nthr()) P[cpos[i]] = row[i];
  c.sync();
}

template <class Ctx>
FDE_HD void reg_setup(const Ctx& c, int* cpos, const int4* __restrict__ sticks, int ncol, int nxa) {
  for (int i = c.tid(); i < ncol; i += c.nthr()) {
    const int w = sticks[i].w;
    cpos[i] = (w >> 16) * nxa + (w & 0xffff);
  }
  c.sync();
}

// H application plane pass; grid (N3, ceil(nb/BPW)), one wavefront per block.
template <typename T, int CLS>
struct KPlaneHReg {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, cplx<T>* __restrict__ sb, int nbands, int BPW,
                         const int4* __restrict__ sticks, int ncol, int nxa, int mlo, int N1, int N2, int N3,
                         const T* __restrict__ veff) {
    const int z = c.bx();
    cplx<T>* P = (cplx<T>*)lds;
    int* cpos = (int*)(P + (size_t)N2 * nxa + 1);
    reg_setup(c, cpos, sticks, ncol, nxa);
    T* vz = const_cast<T*>(veff) + (size_t)z * N1 * N2;
    const int b0 = c.by() * BPW;
    for (int band = b0; band < b0 + BPW && band < nbands; ++band) {
      cplx<T>* row = sb + ((size_t)band * N3 + z) * stick_stride(ncol);
      reg_scatter<T>(c, P, cpos, row, ncol, N2 * nxa);
      columns_fft<T, true, CLS>(c, P, N2, nxa);
      c.sync();
      reg_rows<T, CLS>(c, P, vz, N1, N2, nxa, mlo, false, T(0));
      c.sync();
      columns_fft<T, false, CLS>(c, P, N2, nxa);
      c.sync();
      for (int i = c.tid(); i < ncol; i += c.nthr()) row[i] = P[cpos[i]];
      c.sync();
    }
  }
};

// Density plane pass: acc[group][z] = scale * sum_n occw_n |u_n|^2 over the block's
// bands, accumulated in place in the output plane (zeroed by the block first).
template <typename T, int CLS>
struct KPlaneRhoReg {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const cplx<T>* __restrict__ sb, int nbands, int BPW,
                         const double* __restrict__ occw, const int4* __restrict__ sticks, int ncol, int nxa,
                         int mlo, int N1, int N2, int N3, T* __restrict__ out, double scale) {
    const int z = c.bx();
    const int n = N1 * N2;
    cplx<T>* P = (cplx<T>*)lds;
    int* cpos = (int*)(P + (size_t)N2 * nxa + 1);
    reg_setup(c, cpos, sticks, ncol, nxa);
    T* o = out + ((size_t)c.by() * N3 + z) * n;
    for (int i = c.tid(); i < n; i += c.nthr()) o[i] = T(0);
    const int b0 = c.by() * BPW;
    for (int band = b0; band < b0 + BPW && band < nbands; ++band) {
      const cplx<T>* row = sb + ((size_t)band * N3 + z) * stick_stride(ncol);
      reg_scatter<T>(c, P, cpos, row, ncol, N2 * nxa);
      columns_fft<T, true, CLS>(c, P, N2, nxa);
      c.sync();
      reg_rows<T, CLS>(c, P, o, N1, N2, nxa, mlo, true, (T)(occw[band] * scale));
      c.sync();
    }
  }
};

}  // namespace fde
