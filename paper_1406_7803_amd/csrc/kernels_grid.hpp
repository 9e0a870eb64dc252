// Grid kernels of the embedding potential: batched 3-D FFT passes,
// reciprocal-space operators on the density sphere D, pointwise functionals
// and deterministic reductions.
#pragma once

#include "common.hpp"

namespace fde {

constexpr int kGBlk = 256;   // nominal threads per block of grid kernels
constexpr int kRedBlocks = 1024;
constexpr int kNQ = 8;       // quantities reduced per pointwise kernel

struct GridGeo {
  int N1, N2, N3;
  double b1, b2, b3;
  double gd2;     // |G|^2 bound of the density sphere D (8 E_cut)
  size_t n;
};

FDE_HD void grid_g(const GridGeo& g, size_t i, double& gx, double& gy, double& gz) {
  const int x = (int)(i % g.N1);
  const int y = (int)((i / g.N1) % g.N2);
  const int z = (int)(i / ((size_t)g.N1 * g.N2));
  gx = centred(x, g.N1) * g.b1;
  gy = centred(y, g.N2) * g.b2;
  gz = centred(z, g.N3) * g.b3;
}

// ---------------------------------------------------------------------------
// One batched pass of a 3-D FFT along `axis` (0: x, 1: y, 2: z) over complex
// grids [N3][N2][N1] in place, grid z of them gstride elements apart. L lines per
// workgroup.
//   axis 0: grid (ceil(N2*N3/L), 1, count);  axis 1: grid (ceil(N1/L), N3, count);
//   axis 2: grid (ceil(N1/L), N2, count)
// ---------------------------------------------------------------------------
template <typename T, bool INV>
struct KFftAxis {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, cplx<T>* __restrict__ data, size_t gstride, int N1, int N2, int N3,
                         int axis, Radix r, const cplx<T>* __restrict__ tw, int L) {
    data += (size_t)c.bz() * gstride;
    const int n = r.n;
    cplx<T>* a = (cplx<T>*)lds;
    cplx<T>* b = a + (size_t)L * n;
    cplx<T>* twl = b + (size_t)L * n;
    for (int i = c.tid(); i < n; i += c.nthr()) twl[i] = tw[i];
    if (axis == 0) {
      const int nrows = N2 * N3;
      const int r0 = c.bx() * L;
      const int nl = (nrows - r0) < L ? (nrows - r0) : L;
      for (int idx = c.tid(); idx < nl * n; idx += c.nthr()) a[idx] = data[(size_t)r0 * N1 + idx];
      c.sync();
      cplx<T>* res = lds_fft_any<T, INV>(c, a, b, nl, n, 1, r, twl);
      for (int idx = c.tid(); idx < nl * n; idx += c.nthr()) data[(size_t)r0 * N1 + idx] = res[idx];
      return;
    }
    const int x0 = c.bx() * L;
    const int nl = (N1 - x0) < L ? (N1 - x0) : L;
    const size_t estride = axis == 1 ? (size_t)N1 : (size_t)N1 * N2;
    const size_t base = axis == 1 ? (size_t)c.by() * N1 * N2 + x0 : (size_t)c.by() * N1 + x0;
    for (int idx = c.tid(); idx < n * L; idx += c.nthr()) {
      const int e = idx / L, l = idx - e * L;
      if (l < nl) a[idx] = data[base + e * estride + l];
      else a[idx] = mk<T>(0, 0);
    }
    c.sync();
    cplx<T>* res = lds_fft_any<T, INV>(c, a, b, L, 1, L, r, twl);
    for (int idx = c.tid(); idx < n * L; idx += c.nthr()) {
      const int e = idx / L, l = idx - e * L;
      if (l < nl) data[base + e * estride + l] = res[idx];
    }
  }
};

// Per-block sums of kNQ quantities -> part[block][kNQ]
template <class Ctx>
FDE_HD void block_store(const Ctx& c, double* red, const double* acc, double* part) {
  for (int q = 0; q < kNQ; ++q) {
    const double s = c.sum(acc[q], red);
    if (c.tid() == 0) part[(size_t)c.bx() * kNQ + q] = s;
  }
}

// out[row*ne + slot[q]] = scale * sum_blocks part[b][q] for q with slot[q] >= 0 (single block)
struct KRedFinal {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const double* __restrict__ part, int nblk, double scale,
                         double* __restrict__ out, int s0, int s1, int s2, int s3, int s4, int s5, int s6, int s7) {
    const int slot[kNQ] = {s0, s1, s2, s3, s4, s5, s6, s7};
    for (int q = 0; q < kNQ; ++q) {
      double acc = 0.0;
      for (int b = c.tid(); b < nblk; b += c.nthr()) acc += part[(size_t)b * kNQ + q];
      acc = c.sum(acc, (double*)lds);
      if (c.tid() == 0 && slot[q] >= 0) out[slot[q]] = scale * acc;
    }
  }
};

// ---------------------------------------------------------------------------
// Pointwise functionals (double precision arithmetic for both plan precisions)
// ---------------------------------------------------------------------------
// Slater exchange + Perdew-Zunger 1981 correlation (unpolarised): energy per
// volume e = rho eps_xc and potential v = d(rho eps)/drho.
FDE_HD void lda_point(double rho, double& e, double& v) {
  const double pi = 3.14159265358979323846;
  const double cx = 0.75 * cbrt(3.0 / pi);
  const double r13 = cbrt(rho);
  const double ex = -cx * r13;
  const double vx = (4.0 / 3.0) * ex;
  const double rs = cbrt(3.0 / (4.0 * pi * rho));
  double ec, vc;
  if (rs >= 1.0) {
    const double g = -0.1423, b1 = 1.0529, b2 = 0.3334;
    const double sq = sqrt(rs);
    const double den = 1.0 + b1 * sq + b2 * rs;
    ec = g / den;
    vc = ec * (1.0 + (7.0 / 6.0) * b1 * sq + (4.0 / 3.0) * b2 * rs) / den;
  } else {
    const double A = 0.0311, B = -0.048, C = 0.0020, D = -0.0116;
    const double lr = log(rs);
    ec = A * lr + B + C * rs * lr + D * rs;
    vc = A * lr + (B - A / 3.0) + (2.0 / 3.0) * C * rs * lr + (2.0 * D - C) * rs / 3.0;
  }
  e = rho * (ex + ec);
  v = vx + vc;
}

struct KinConst {
  double ctf, cs;
};

// LC94 enhancement: F(s) = 1 + Delta/den with
//   Delta = (a3 - a4 e^{-alpha s^2}) s^2 - a5 s^4,  den = 1 + a1 s asinh(a2 s) + a5 s^4,
// and F'/s = (Delta'/s)/den - (Delta/s) den'/den^2, which has no 0/0 at s = 0.
FDE_HD void lc94(double s, double& F, double& dFs) {
  const double a1 = 0.093907, a2 = 76.32, a3 = 0.26608, a4 = 0.0809615, a5 = 5.7767e-5, al = 100.0;
  const double s2 = s * s;
  const double ex = exp(-al * s2);
  const double c = a3 - a4 * ex;
  const double as = asinh(a2 * s);
  const double den = 1.0 + a1 * s * as + a5 * s2 * s2;
  const double delta = c * s2 - a5 * s2 * s2;
  const double dden = a1 * as + a1 * a2 * s / sqrt(1.0 + a2 * a2 * s2) + 4.0 * a5 * s2 * s;
  const double dDs = 2.0 * c + 2.0 * al * a4 * s2 * ex - 4.0 * a5 * s2;
  const double Ds = c * s - a5 * s2 * s;
  F = 1.0 + delta / den;
  dFs = dDs / den - Ds * dden / (den * den);
}

}  // namespace fde
