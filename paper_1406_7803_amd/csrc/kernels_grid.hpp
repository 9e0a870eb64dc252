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

// revAPBEK enhancement (APBEK's mu with revPBE's kappa): F = 1 + k - k/(1 + mu s^2/k),
// F'/s = 2 mu / (1 + mu s^2/k)^2.
FDE_HD void revapbek(double s, double& F, double& dFs) {
  const double k = 1.245, mu = 0.23889;
  const double d = 1.0 + mu * s * s / k;
  F = 1.0 + k - k / d;
  dFs = 2.0 * mu / (d * d);
}

// PBE exchange-correlation (spin-unpolarised) at one point as e(rho, sigma), sigma =
// |grad rho|^2: energy per volume e, er = de/drho, es = de/dsigma.
//   exchange: e_x = -C_X rho^{4/3} F(u), u = s^2 = C_S^2 sigma / rho^{8/3},
//             F = 1 + kappa - kappa / (1 + mu u / kappa), F_u = mu / (1 + mu u/kappa)^2;
//             er = -C_X rho^{1/3} (4/3)(F - 2 u F_u),  es = -C_X C_S^2 F_u / rho^{4/3}.
//   correlation: e_c = rho (eps + H(eps, y)), y = t^2 = c_t sigma rho^{-7/3},
//             c_t = pi / (16 (3 pi^2)^{1/3}); PW92 eps(r_s) with r_s = (3/(4 pi rho))^{1/3};
//             H = gamma ln(1 + R), R = (beta/gamma) y P/Q, P = 1 + A y, Q = P + A^2 y^2,
//             A = (beta/gamma)/(E - 1), E = exp(-eps/gamma), dA/deps = A^2 E / beta;
//             er = eps + H + rho [(1 + H_A dA/deps) deps/drho - (7/3) H_y y / rho],
//             deps/drho = -eps'(r_s) r_s / (3 rho),   es = rho H_y c_t rho^{-7/3}.
FDE_HD void pbe_point(double rho, double sigma, double& e, double& er, double& es) {
  const double pi = 3.14159265358979323846;
  const double cx = 0.75 * cbrt(3.0 / pi);
  const double cs2 = 1.0 / (4.0 * cbrt(9.0 * pi * pi * pi * pi));  // C_S^2 = 1/(4 (3 pi^2)^{2/3})
  const double kap = 0.804, beta = 0.06672455060314922, gam = (1.0 - log(2.0)) / (pi * pi);
  const double mu = beta * pi * pi / 3.0;
  const double r13 = cbrt(rho), r43 = rho * r13;
  // exchange
  const double u = cs2 * sigma / (r43 * r43);
  const double dx = 1.0 + mu * u / kap;
  const double F = 1.0 + kap - kap / dx, Fu = mu / (dx * dx);
  e = -cx * r43 * F;
  er = -cx * r13 * (4.0 / 3.0) * (F - 2.0 * u * Fu);
  es = -cx * cs2 * Fu / r43;
  // PW92 correlation energy per electron and its r_s derivative
  const double a = 0.0310907, a1 = 0.21370, b1 = 7.5957, b2 = 3.5876, b3 = 1.6382, b4 = 0.49294;
  const double rs = cbrt(3.0 / (4.0 * pi * rho)), srs = sqrt(rs);
  const double q = 2.0 * a * (b1 * srs + b2 * rs + b3 * rs * srs + b4 * rs * rs);
  const double dq = 2.0 * a * (0.5 * b1 / srs + b2 + 1.5 * b3 * srs + 2.0 * b4 * rs);
  const double lg = log(1.0 + 1.0 / q);
  const double eps = -2.0 * a * (1.0 + a1 * rs) * lg;
  const double deps_rs = -2.0 * a * a1 * lg + 2.0 * a * (1.0 + a1 * rs) * dq / (q * q + q);
  const double deps = -deps_rs * rs / (3.0 * rho);
  // gradient correction H
  const double ct = pi / (16.0 * cbrt(3.0 * pi * pi));
  const double r73 = rho * r43;  // rho^{7/3}
  const double y = ct * sigma / r73;
  const double E = exp(-eps / gam);
  const double A = (beta / gam) / (E - 1.0);
  const double P = 1.0 + A * y, Q = P + A * A * y * y;
  const double R = (beta / gam) * y * P / Q;
  const double H = gam * log1p(R);
  const double Ry = (beta / gam) * ((P + A * y) / Q - y * P * (A + 2.0 * A * A * y) / (Q * Q));
  const double RA = (beta / gam) * y * (y / Q - P * (y + 2.0 * A * y * y) / (Q * Q));
  const double Hy = gam * Ry / (1.0 + R), HA = gam * RA / (1.0 + R);
  const double dA = A * A * E / beta;
  e += rho * (eps + H);
  er += eps + H + rho * ((1.0 + HA * dA) * deps - (7.0 / 3.0) * Hy * y / rho);
  es += rho * Hy * ct / r73;
}

}  // namespace fde
