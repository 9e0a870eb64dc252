// Host entry points of the grid kernels: fde_embed_potential,
// fde_local_potential, fde_mix, fde_mix_pulay, fde_grid_dot, fde_density_l1, fde_grid_mean,
// fde_energy_total.
#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels_grid.hpp"
#include "launch.hpp"

namespace fde {

static GridGeo geo(const fde_plan* p) {
  GridGeo g;
  g.N1 = p->N[0];
  g.N2 = p->N[1];
  g.N3 = p->N[2];
  g.b1 = p->b[0];
  g.b2 = p->b[1];
  g.b3 = p->b[2];
  g.gd2 = 8.0 * p->ecut;
  g.n = p->npts();
  return g;
}

static unsigned red_blocks(size_t n) { return (unsigned)std::min<size_t>(kRedBlocks, (n + kGBlk - 1) / kGBlk); }

// ---------------------------------------------------------------------------
// Pointwise kernels. All use the grid-stride pattern
//   for i0 in [bx*256, n) step nblk*256: for l in [tid, 256) step nthr: i = i0 + l
// and reduce kNQ doubles per block into part[block][kNQ] when part != nullptr.
// ---------------------------------------------------------------------------
#define GRID_FOR(c, n, nblk)                                                           \
  for (size_t i0_ = (size_t)(c).bx() * kGBlk; i0_ < (n); i0_ += (size_t)(nblk) * kGBlk) \
    for (int l_ = (c).tid(); l_ < kGBlk; l_ += (c).nthr())

// rho = sum_I rho_sub[I]; W = (rho, 0)
template <typename T>
struct KSumSub {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const T* __restrict__ sub, int ns, size_t n, T* __restrict__ rho,
                         unsigned nblk) {
    GRID_FOR(c, n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= n) break;
      T s = 0;
      for (int I = 0; I < ns; ++I) s += sub[(size_t)I * n + i];
      rho[i] = s;
    }
  }
};

// env[I * ld + i] = sum_{J != I} rho_sub[J][i], J ascending. grid (nblk, ns)
template <typename T>
struct KEnvironment {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const T* __restrict__ sub, int ns, size_t n, T* __restrict__ env,
                         size_t ld, unsigned nblk) {
    const int I = c.by();
    GRID_FOR(c, n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= n) break;
      T s = 0;
      for (int J = 0; J < ns; ++J)
        if (J != I) s += sub[(size_t)J * n + i];
      env[(size_t)I * ld + i] = s;
    }
  }
};

template <typename T>
struct KToComplex {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const T* __restrict__ x, size_t n, cplx<T>* __restrict__ w,
                         unsigned nblk) {
    GRID_FOR(c, n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= n) break;
      w[i] = mk<T>(x[i], T(0));
    }
  }
};

// XG <- XG/N on D, 0 outside; optionally H <- 4 pi XG / G^2 (G != 0) for the
// Hartree potential. q0 = sum_{D, G!=0} 4 pi |XG|^2 / G^2 (self Hartree, x Omega/2).
template <typename T>
struct KMaskXG {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, cplx<T>* __restrict__ xg, cplx<T>* __restrict__ h, GridGeo g,
                         double invN, double* __restrict__ part, unsigned nblk) {
    const double fpi = 4.0 * 3.14159265358979323846;
    double acc[kNQ] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_FOR(c, g.n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= g.n) break;
      double gx, gy, gz;
      grid_g(g, i, gx, gy, gz);
      const double G2 = gx * gx + gy * gy + gz * gz;
      const bool inD = G2 <= g.gd2;
      const cplx<T> v = xg[i];
      const double vx = inD ? invN * v.x : 0.0, vy = inD ? invN * v.y : 0.0;
      xg[i] = mk<T>((T)vx, (T)vy);
      if (inD && G2 > 0) acc[0] += fpi * (vx * vx + vy * vy) / G2;
      if (h) {
        const double f = (inD && G2 > 0) ? fpi / G2 : 0.0;
        h[i] = mk<T>((T)(f * vx), (T)(f * vy));
      }
    }
    block_store(c, (double*)lds, acc, part);
  }
};

// W_d = i G_d XG (d = x, y, z)
template <typename T>
struct KGradPrep {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const cplx<T>* __restrict__ xg, cplx<T>* __restrict__ w1,
                         cplx<T>* __restrict__ w2, cplx<T>* __restrict__ w3, GridGeo g, unsigned nblk) {
    GRID_FOR(c, g.n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= g.n) break;
      double gx, gy, gz;
      grid_g(g, i, gx, gy, gz);
      const cplx<T> v = xg[i];
      w1[i] = mk<T>((T)(-gx * v.y), (T)(gx * v.x));
      w2[i] = mk<T>((T)(-gy * v.y), (T)(gy * v.x));
      w3[i] = mk<T>((T)(-gz * v.y), (T)(gz * v.x));
    }
  }
};

// The functionals of one density X that need its gradient, at each point: the kinetic
// functional (kin: 1 Thomas-Fermi, 2 TF x LC94, 3 TF x revAPBEK; coefficient 1) and up
// to two PBE exchange-correlation terms with coefficients ca, cb (0: energy only).
// In: X and, when grad != 0, the gradient in Re(W_d). Out: v = the sum of the local parts
// de/dX, and (grad != 0) the field h = sum of the 2 de/dsigma grad X terms in W_d (the
// kinetic one in the regular form C_TF C_s^2 (F'/s) grad X / X). q0, q1, q2 = sums of the
// energy densities of kin, a, b. Below thr every term is zero.
struct GgaSet {
  int kin;
  int xa, xb;      // FDE_XC_PBE or FDE_XC_NONE
  double ca, cb;
  int sa, sb;      // energy slots of a, b (-1: none)
};

template <typename T>
struct KGgaPoint {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const T* __restrict__ X, cplx<T>* __restrict__ w1,
                         cplx<T>* __restrict__ w2, cplx<T>* __restrict__ w3, T* __restrict__ v, size_t n, GgaSet f,
                         int grad, KinConst k, double thr, double* __restrict__ part, unsigned nblk) {
    double acc[kNQ] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_FOR(c, n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= n) break;
      const double x = X[i];
      if (!(x >= thr)) {
        v[i] = T(0);
        if (grad) {
          w1[i] = mk<T>(0, 0);
          w2[i] = mk<T>(0, 0);
          w3[i] = mk<T>(0, 0);
        }
        continue;
      }
      const double x13 = cbrt(x);
      const double x23 = x13 * x13;
      const double x53 = x * x23;
      double dx = 0.0, dy = 0.0, dz = 0.0;
      if (grad) {
        dx = w1[i].x;
        dy = w2[i].x;
        dz = w3[i].x;
      }
      const double sigma = dx * dx + dy * dy + dz * dz;
      double vl = 0.0, hf = 0.0;
      if (f.kin == FDE_KIN_TF) {
        acc[0] += k.ctf * x53;
        vl += k.ctf * (5.0 / 3.0) * x23;
      } else if (f.kin == FDE_KIN_LC94 || f.kin == FDE_KIN_REVAPBEK) {
        const double s = k.cs * sqrt(sigma) / (x * x13);
        double F, dFs;
        if (f.kin == FDE_KIN_LC94) lc94(s, F, dFs);
        else revapbek(s, F, dFs);
        acc[0] += k.ctf * x53 * F;
        vl += k.ctf * x23 * ((5.0 / 3.0) * F - (4.0 / 3.0) * s * s * dFs);
        hf += k.ctf * k.cs * k.cs * dFs / x;
      }
      if (f.xa == FDE_XC_PBE || f.xb == FDE_XC_PBE) {
        double e, er, es;
        pbe_point(x, sigma, e, er, es);
        if (f.xa == FDE_XC_PBE) {
          acc[1] += e;
          vl += f.ca * er;
          hf += 2.0 * f.ca * es;
        }
        if (f.xb == FDE_XC_PBE) {
          acc[2] += e;
          vl += f.cb * er;
          hf += 2.0 * f.cb * es;
        }
      }
      v[i] = (T)vl;
      if (grad) {
        w1[i] = mk<T>((T)(hf * dx), T(0));
        w2[i] = mk<T>((T)(hf * dy), T(0));
        w3[i] = mk<T>((T)(hf * dz), T(0));
      }
    }
    block_store(c, (double*)lds, acc, part);
  }
};

// W0 = (1/N) sum_d i G_d W_d on D (the divergence in reciprocal space)
template <typename T>
struct KDivPrep {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, cplx<T>* __restrict__ w0, const cplx<T>* __restrict__ w1,
                         const cplx<T>* __restrict__ w2, const cplx<T>* __restrict__ w3, GridGeo g, double invN,
                         unsigned nblk) {
    GRID_FOR(c, g.n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= g.n) break;
      double gx, gy, gz;
      grid_g(g, i, gx, gy, gz);
      const bool inD = gx * gx + gy * gy + gz * gz <= g.gd2;
      const cplx<T> a = w1[i], b = w2[i], d = w3[i];
      const double re = -(gx * a.y + gy * b.y + gz * d.y);
      const double im = gx * a.x + gy * b.x + gz * d.x;
      w0[i] = inD ? mk<T>((T)(invN * re), (T)(invN * im)) : mk<T>(0, 0);
    }
  }
};

// v <- v - Re(W0)
template <typename T>
struct KKinFinish {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, T* __restrict__ v, const cplx<T>* __restrict__ w0, size_t n,
                         unsigned nblk) {
    GRID_FOR(c, n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= n) break;
      v[i] = v[i] - w0[i].x;
    }
  }
};

// out = Re(W)
template <typename T>
struct KRealPart {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const cplx<T>* __restrict__ w, T* __restrict__ out, size_t n,
                         unsigned nblk) {
    GRID_FOR(c, n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= n) break;
      out[i] = w[i].x;
    }
  }
};

FDE_HD void xc_point(int kind, double rho, double thr, double& e, double& v) {
  e = 0.0;
  v = 0.0;
  if (kind == FDE_XC_LDA && rho >= thr) lda_point(rho, e, v);
}

// Total density: vxt = V~xc[rho]. q0 = E~xc[rho], q1 = E_xc[rho], q3 = int vloc rho,
// q4 = int V_H rho, q7 = int rho (sums; scaled by dV later).
template <typename T>
struct KXcTotal {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const T* __restrict__ rho, const T* __restrict__ vloc,
                         const T* __restrict__ vh, T* __restrict__ vxt, size_t n, int xc, int xc_nad, double thr,
                         double* __restrict__ part, unsigned nblk) {
    double acc[kNQ] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_FOR(c, n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= n) break;
      const double r = rho[i];
      double e, v, e2, v2;
      xc_point(xc_nad, r, thr, e, v);
      xc_point(xc, r, thr, e2, v2);
      vxt[i] = (T)v;
      acc[0] += e;
      acc[1] += e2;
      acc[3] += (double)vloc[i] * r;
      acc[4] += (double)vh[i] * r;
      acc[7] += r;
    }
    block_store(c, (double*)lds, acc, part);
  }
};

// Subsystem assembly (recast effective potential):
//   veff = vloc + V_H + v_xc[rho_I] + (V~xc[rho] - v~xc[rho_I]) + (V~kin[rho] - vk_I)
// where vk_I is read from veff on entry. q0 = E_xc[rho_I], q1 = E~xc[rho_I],
// q3 = int vloc rho_I, q4 = int V_H rho_I, q6 = -int (veff - vloc) rho_I, q7 = int rho_I.
template <typename T>
struct KAssemble {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const T* __restrict__ rhoI, const T* __restrict__ vloc,
                         const T* __restrict__ vh, const T* __restrict__ vxt, const T* __restrict__ vkt,
                         T* __restrict__ veff, size_t n, int xc, int xc_nad, double thr, double* __restrict__ part,
                         int* __restrict__ info, unsigned nblk) {
    double acc[kNQ] = {0, 0, 0, 0, 0, 0, 0, 0};
    int bad = 0;
    GRID_FOR(c, n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= n) break;
      const double r = rhoI[i];
      double e, v, et, vt;
      xc_point(xc, r, thr, e, v);
      xc_point(xc_nad, r, thr, et, vt);
      const double vl = vloc[i];
      const double out = vl + (double)vh[i] + v + ((double)vxt[i] - vt) + ((double)vkt[i] - (double)veff[i]);
      const T o = (T)out;
      veff[i] = o;
      if (!(out == out) || out > 1e300 || out < -1e300) bad = 1;
      acc[0] += e;
      acc[1] += et;
      acc[3] += vl * r;
      acc[4] += (double)vh[i] * r;
      acc[6] -= ((double)o - vl) * r;
      acc[7] += r;
    }
    if (bad) info[0] = 1;
    block_store(c, (double*)lds, acc, part);
  }
};

// 3-D FFT of `count` grids in place, gstride elements apart (one launch per axis for all)
template <typename T>
static fde_status fft3(fde_plan* p, cplx<T>* w, bool inv, hipStream_t s, int count = 1, size_t gstride = 0) {
  const int N1 = p->N[0], N2 = p->N[1], N3 = p->N[2];
  for (int axis = 0; axis < 3; ++axis) {
    const int n = p->N[axis];
    int L = 16;
    while (L > 1 && (2 * (size_t)L * n + n) * sizeof(cplx<T>) > 64 * 1024) L /= 2;
    const size_t lds = (2 * (size_t)L * n + n) * sizeof(cplx<T>);
    dim3 grid;
    if (axis == 0) grid = dim3((N2 * N3 + L - 1) / L, 1, count);
    else grid = dim3((N1 + L - 1) / L, axis == 1 ? N3 : N2, count);
    const cplx<T>* tw = (const cplx<T>*)p->d_tw[axis];
    if (inv)
      FDE_TRY(launch<KFftAxis<T, true>>(grid, kBlock, lds, s, w, gstride, N1, N2, N3, axis, p->rad[axis], tw, L));
    else
      FDE_TRY(launch<KFftAxis<T, false>>(grid, kBlock, lds, s, w, gstride, N1, N2, N3, axis, p->rad[axis], tw, L));
  }
  return FDE_OK;
}

template <typename T>
struct EmbedWs {
  cplx<T>*W0, *W1, *W2, *W3;
  T *rho, *vh, *vxt, *vkt;
  double* part;  // [kRedBlocks][kNQ]
};

template <typename T>
static EmbedWs<T> embed_ws(fde_plan* p) {
  EmbedWs<T> e;
  const size_t n = p->npts();
  char* w = p->scratch;
  size_t off = 0;
  cplx<T>** cg[4] = {&e.W0, &e.W1, &e.W2, &e.W3};
  for (int i = 0; i < 4; ++i) {
    *cg[i] = (cplx<T>*)(w + off);
    off += align256(n * sizeof(cplx<T>));
  }
  T** rg[4] = {&e.rho, &e.vh, &e.vxt, &e.vkt};
  for (int i = 0; i < 4; ++i) {
    *rg[i] = (T*)(w + off);
    off += align256(n * sizeof(T));
  }
  e.part = (double*)(w + off);
  return e;
}

// Gradient functionals of density X into vout (the kinetic one and the PBE terms of f);
// writes their energies into the row and, from the transformed density, E_H[X]. If
// vh != nullptr also returns V_H[X] (used for the total density).
template <typename T>
static fde_status kinetic_and_hartree(fde_plan* p, EmbedWs<T>& e, const T* X, T* vout, const GgaSet& f, double thr,
                                      T* vh, double* erow, hipStream_t s) {
  const GridGeo g = geo(p);
  const size_t n = g.n;
  const unsigned nb = red_blocks(n);
  const double invN = 1.0 / (double)n;
  const double dV = p->omega / (double)n;
  const KinConst kc = {0.3 * std::pow(3.0 * M_PI * M_PI, 2.0 / 3.0), 1.0 / (2.0 * std::cbrt(3.0 * M_PI * M_PI))};
  const size_t red = 17 * sizeof(double);
  // X(G) on D, self Hartree energy, optional V_H
  FDE_TRY(launch<KToComplex<T>>(dim3(nb), kBlock, 0, s, X, n, e.W0, nb));
  FDE_TRY(fft3<T>(p, e.W0, false, s));
  FDE_TRY(launch<KMaskXG<T>>(dim3(nb), kBlock, red, s, e.W0, vh ? e.W1 : (cplx<T>*)nullptr, g, invN, e.part, nb));
  FDE_TRY(launch<KRedFinal>(dim3(1), kBlock, red, s, (const double*)e.part, (int)nb, 0.5 * p->omega, erow,
                            (int)FDE_E_HSELF, -1, -1, -1, -1, -1, -1, -1));
  if (vh) {
    FDE_TRY(fft3<T>(p, e.W1, true, s));
    FDE_TRY(launch<KRealPart<T>>(dim3(nb), kBlock, 0, s, (const cplx<T>*)e.W1, vh, n, nb));
  }
  const bool pbe = f.xa == FDE_XC_PBE || f.xb == FDE_XC_PBE;
  if (f.kin == FDE_KIN_NONE && !pbe) {
    FDE_TRY(zero_bytes(vout, n * sizeof(T), s));
    FDE_TRY(zero_bytes(erow + FDE_E_KIN, sizeof(double), s));
    return FDE_OK;
  }
  const int grad = (pbe || f.kin == FDE_KIN_LC94 || f.kin == FDE_KIN_REVAPBEK) ? 1 : 0;
  const int skin = f.kin == FDE_KIN_NONE ? -1 : (int)FDE_E_KIN;
  if (f.kin == FDE_KIN_NONE) FDE_TRY(zero_bytes(erow + FDE_E_KIN, sizeof(double), s));
  if (grad) {
    FDE_TRY(launch<KGradPrep<T>>(dim3(nb), kBlock, 0, s, (const cplx<T>*)e.W0, e.W1, e.W2, e.W3, g, nb));
    FDE_TRY(fft3<T>(p, e.W1, true, s, 3, (size_t)(e.W2 - e.W1)));  // the three components, W1..W3
  }
  FDE_TRY(launch<KGgaPoint<T>>(dim3(nb), kBlock, red, s, X, e.W1, e.W2, e.W3, vout, n, f, grad, kc, thr, e.part,
                               nb));
  FDE_TRY(launch<KRedFinal>(dim3(1), kBlock, red, s, (const double*)e.part, (int)nb, dV, erow, skin, f.sa, f.sb, -1,
                            -1, -1, -1, -1));
  if (!grad) return FDE_OK;
  // divergence of h
  FDE_TRY(fft3<T>(p, e.W1, false, s, 3, (size_t)(e.W2 - e.W1)));
  FDE_TRY(launch<KDivPrep<T>>(dim3(nb), kBlock, 0, s, e.W0, (const cplx<T>*)e.W1, (const cplx<T>*)e.W2,
                              (const cplx<T>*)e.W3, g, invN, nb));
  FDE_TRY(fft3<T>(p, e.W0, true, s));
  FDE_TRY(launch<KKinFinish<T>>(dim3(nb), kBlock, 0, s, vout, (const cplx<T>*)e.W0, n, nb));
  return FDE_OK;
}

template <typename T>
static fde_status embed_t(fde_plan* p, int ns, const T* rho_sub, const T* vloc, const fde_functionals* f, T* veff,
                          double* en, int* info, hipStream_t s) {
  EmbedWs<T> e = embed_ws<T>(p);
  const size_t n = p->npts();
  const unsigned nb = red_blocks(n);
  const double dV = p->omega / (double)n;
  const size_t red = 17 * sizeof(double);
  FDE_TRY(zero_bytes(info, sizeof(int), s));
  FDE_TRY(zero_bytes(en, (size_t)(ns + 1) * FDE_NE * sizeof(double), s));
  FDE_TRY(launch<KSumSub<T>>(dim3(nb), kBlock, 0, s, rho_sub, ns, n, e.rho, nb));
  double* etot = en + (size_t)ns * FDE_NE;
  // PBE terms go with the gradient functionals; the pointwise kernels see them as "none"
  const bool xpbe = f->xc == FDE_XC_PBE, npbe = f->xc_nad == FDE_XC_PBE;
  const int xc_pt = xpbe ? FDE_XC_NONE : f->xc, nad_pt = npbe ? FDE_XC_NONE : f->xc_nad;
  // total density: V~kin[rho] + V~xc[rho] (PBE), energies E~xc[rho] and E_xc[rho] (PBE)
  const GgaSet ftot{f->kin_nad, npbe ? FDE_XC_PBE : FDE_XC_NONE, xpbe ? FDE_XC_PBE : FDE_XC_NONE, 1.0, 0.0,
                    npbe ? (int)FDE_E_XCNAD : -1, xpbe ? (int)FDE_E_XC : -1};
  FDE_TRY(kinetic_and_hartree<T>(p, e, e.rho, e.vkt, ftot, f->rho_thr, e.vh, etot, s));
  FDE_TRY(launch<KXcTotal<T>>(dim3(nb), kBlock, red, s, (const T*)e.rho, vloc, (const T*)e.vh, e.vxt, n, xc_pt,
                              nad_pt, f->rho_thr, e.part, nb));
  FDE_TRY(launch<KRedFinal>(dim3(1), kBlock, red, s, (const double*)e.part, (int)nb, dV, etot,
                            npbe ? -1 : (int)FDE_E_XCNAD, xpbe ? -1 : (int)FDE_E_XC, -1, (int)FDE_E_LOC,
                            (int)FDE_E_HEMB, -1, -1, (int)FDE_E_CHARGE));
  // subsystem I: V~kin[rho_I] - V_xc[rho_I] (PBE) + V~xc[rho_I] (PBE), subtracted in KAssemble
  const GgaSet fsub{f->kin_nad, xpbe ? FDE_XC_PBE : FDE_XC_NONE, npbe ? FDE_XC_PBE : FDE_XC_NONE, -1.0, 1.0,
                    xpbe ? (int)FDE_E_XC : -1, npbe ? (int)FDE_E_XCNAD : -1};
  for (int I = 0; I < ns; ++I) {
    const T* rI = rho_sub + (size_t)I * n;
    T* vI = veff + (size_t)I * n;
    double* erow = en + (size_t)I * FDE_NE;
    FDE_TRY(kinetic_and_hartree<T>(p, e, rI, vI, fsub, f->rho_thr, (T*)nullptr, erow, s));
    FDE_TRY(launch<KAssemble<T>>(dim3(nb), kBlock, red, s, rI, vloc, (const T*)e.vh, (const T*)e.vxt,
                                 (const T*)e.vkt, vI, n, xc_pt, nad_pt, f->rho_thr, e.part, info, nb));
    FDE_TRY(launch<KRedFinal>(dim3(1), kBlock, red, s, (const double*)e.part, (int)nb, dV, erow,
                              xpbe ? -1 : (int)FDE_E_XC, npbe ? -1 : (int)FDE_E_XCNAD, -1, (int)FDE_E_LOC,
                              (int)FDE_E_HEMB, -1, (int)FDE_E_DEBAND, (int)FDE_E_CHARGE));
  }
  return FDE_OK;
}

// ---------------------------------------------------------------------------
// Local potential of Gaussian ions
// ---------------------------------------------------------------------------
struct Ion {
  double R[3];
  double Z, w;
};

template <typename T>
struct KVlocG {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const Ion* __restrict__ ions, int nion, GridGeo g, double omega,
                         cplx<T>* __restrict__ w, unsigned nblk) {
    const double pi = 3.14159265358979323846;
    GRID_FOR(c, g.n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= g.n) break;
      double gx, gy, gz;
      grid_g(g, i, gx, gy, gz);
      const double G2 = gx * gx + gy * gy + gz * gz;
      double re = 0.0, im = 0.0;
      if (G2 <= g.gd2) {
        for (int a = 0; a < nion; ++a) {
          const Ion at = ions[a];
          if (G2 > 0) {
            const double amp = -4.0 * pi * at.Z * exp(-0.5 * G2 * at.w * at.w) / G2;
            const double ph = -(gx * at.R[0] + gy * at.R[1] + gz * at.R[2]);
            re += amp * cos(ph);
            im += amp * sin(ph);
          } else {
            re += 2.0 * pi * at.Z * at.w * at.w;
          }
        }
      }
      w[i] = mk<T>((T)(re / omega), (T)(im / omega));
    }
  }
};

// Augmentation charge in G: sum_a c_a exp(-G^2 w_a^2 / 2) e^{-iG.R_a} / Omega on the density
// sphere (atoms [natom][4] = x, y, z, w and charges c on the device).
template <typename T>
struct KAugG {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const double* __restrict__ atoms, const double* __restrict__ q,
                         int natom, GridGeo g, double omega, cplx<T>* __restrict__ w, unsigned nblk) {
    GRID_FOR(c, g.n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= g.n) break;
      double gx, gy, gz;
      grid_g(g, i, gx, gy, gz);
      const double G2 = gx * gx + gy * gy + gz * gz;
      double re = 0.0, im = 0.0;
      if (G2 <= g.gd2) {
        for (int a = 0; a < natom; ++a) {
          const double* at = atoms + 4 * a;
          const double amp = q[a] * exp(-0.5 * G2 * at[3] * at[3]);
          const double ph = -(gx * at[0] + gy * at[1] + gz * at[2]);
          re += amp * cos(ph);
          im += amp * sin(ph);
        }
      }
      w[i] = mk<T>((T)(re / omega), (T)(im / omega));
    }
  }
};

template <typename T>
static fde_status vloc_t(fde_plan* p, const std::vector<Ion>& ions, T* vloc, hipStream_t s) {
  EmbedWs<T> e = embed_ws<T>(p);
  const size_t n = p->npts();
  const unsigned nb = red_blocks(n);
  Ion* d_ions = (Ion*)e.W1;  // staged in a work grid (synchronous copy)
  FDE_TRY(stream_sync(s));
  FDE_TRY(copy_h2d_sync(d_ions, ions.data(), ions.size() * sizeof(Ion)));
  FDE_TRY(launch<KVlocG<T>>(dim3(nb), kBlock, 0, s, (const Ion*)d_ions, (int)ions.size(), geo(p), p->omega, e.W0, nb));
  FDE_TRY(fft3<T>(p, e.W0, true, s));
  FDE_TRY(launch<KRealPart<T>>(dim3(nb), kBlock, 0, s, (const cplx<T>*)e.W0, vloc, n, nb));
  return FDE_OK;
}

// ---------------------------------------------------------------------------
// Mixing and grid dot product
// ---------------------------------------------------------------------------
template <typename T>
struct KMix {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, T* __restrict__ a, const T* __restrict__ b, size_t n, double beta,
                         unsigned nblk) {
    GRID_FOR(c, n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= n) break;
      a[i] = (T)((1.0 - beta) * (double)a[i] + beta * (double)b[i]);
    }
  }
};

template <typename T>
struct KDot {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const T* __restrict__ a, const T* __restrict__ b, size_t n,
                         double* __restrict__ part, unsigned nblk) {
    double acc[kNQ] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_FOR(c, n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= n) break;
      acc[0] += b ? (double)a[i] * (double)b[i] : (double)a[i];
    }
    block_store(c, (double*)lds, acc, part);
  }
};

// |sum_{I < ns} a_I - b| per point, summed per block
template <typename T>
struct KAbsDiff {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const T* __restrict__ a, int ns, const T* __restrict__ b, size_t n,
                         double* __restrict__ part, unsigned nblk) {
    double acc[kNQ] = {0, 0, 0, 0, 0, 0, 0, 0};
    GRID_FOR(c, n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= n) break;
      double t = -(double)b[i];
      for (int I = 0; I < ns; ++I) t += (double)a[(size_t)I * n + i];
      acc[0] += fabs(t);
    }
    block_store(c, (double*)lds, acc, part);
  }
};

// out[0] += scale * sum part[b][0]   (out[0] = ... when set)
struct KRedAdd {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const double* __restrict__ part, int nblk, double scale,
                         double* __restrict__ out, int set) {
    double acc = 0.0;
    for (int b = c.tid(); b < nblk; b += c.nthr()) acc += part[(size_t)b * kNQ];
    acc = c.sum(acc, (double*)lds);
    if (c.tid() == 0) out[0] = (set ? 0.0 : out[0]) + scale * acc;
  }
};

// ---------------------------------------------------------------------------
// Pulay mixing with a Kerker preconditioner
// ---------------------------------------------------------------------------
constexpr int kPulayBlocks = 128;

// x_hist[slot] = rho_in, r_hist[slot] = rho_out - rho_in over n values
// State of the history (device ints): [0] entries filled, [1] next slot, [2] entries in use
// by the current call. x_hist[slot] = rho_in, r_hist[slot] = rho_out - rho_in over n values.
template <typename T>
struct KPulayStore {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, T* __restrict__ xh, T* __restrict__ rh, const int* __restrict__ state,
                         const T* __restrict__ rin, const T* __restrict__ rout, size_t n, unsigned nblk) {
    const size_t off = (size_t)state[1] * n;
    GRID_FOR(c, n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= n) break;
      const T a = rin[i];
      xh[off + i] = a;
      rh[off + i] = (T)((double)rout[i] - (double)a);
    }
  }
};

// part[block][pair] = partial sums of R_i R_j for the pairs i <= j < nh (packed)
template <typename T>
struct KPulayGram {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const T* __restrict__ rh, size_t n, size_t hstride,
                         const int* __restrict__ state, int nhmax, double* __restrict__ part, unsigned nblk) {
    const int nh = state[0] + 1 < nhmax ? state[0] + 1 : nhmax;
    double acc[FDE_PULAY_MAX * (FDE_PULAY_MAX + 1) / 2];
    const int npair = nh * (nh + 1) / 2;
    for (int q = 0; q < npair; ++q) acc[q] = 0.0;
    GRID_FOR(c, n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= n) break;
      double r[FDE_PULAY_MAX];
      for (int a = 0; a < nh; ++a) r[a] = (double)rh[(size_t)a * hstride + i];
      int q = 0;
      for (int a = 0; a < nh; ++a)
        for (int b = a; b < nh; ++b) acc[q++] += r[a] * r[b];
    }
    for (int q = 0; q < npair; ++q) {
      const double t = c.sum(acc[q], (double*)lds);
      if (c.tid() == 0) part[(size_t)c.bx() * npair + q] = t;
    }
  }
};

// Reduce the pair partials in a fixed order and solve [B 1; 1^T 0][a; l] = [0; 1] (one
// thread): with d_i = sqrt(B_ii) and a_i = a'_i / d_i the system is solved for the unit-
// diagonal B'_ij = B_ij / (d_i d_j), bordered by 1/d_i, by Gaussian elimination with
// partial pivoting. An exactly zero pivot or a non-finite solution (a repeated pair)
// falls back to a = e_newest, linear mixing of the new pair, with info = 1; a zero
// residual (d_i = 0) selects its own input. Nearly dependent residuals are kept (near a
// fixed point the minimising combination is such a dependency).
struct KPulaySolve {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const double* __restrict__ part, int nblk, int* __restrict__ state,
                         int nhmax, double* __restrict__ alpha, int* __restrict__ info) {
    const int nh = state[0] + 1 < nhmax ? state[0] + 1 : nhmax;
    const int newest = state[1];
    double* Bp = (double*)lds + 17;  // packed pair sums
    const int npair = nh * (nh + 1) / 2;
    for (int q = 0; q < npair; ++q) {
      double acc = 0.0;
      for (int b = c.tid(); b < nblk; b += c.nthr()) acc += part[(size_t)b * npair + q];
      acc = c.sum(acc, (double*)lds);
      if (c.tid() == 0) Bp[q] = acc;
      c.sync();
    }
    if (c.tid() != 0) return;
    constexpr int M = FDE_PULAY_MAX + 1;
    double A[M][M + 1], d[M];
    const int n = nh + 1;
    int q = 0, zero = -1;
    for (int a = 0; a < nh; ++a)
      for (int b = a; b < nh; ++b) {
        A[a][b] = A[b][a] = Bp[q++];
      }
    for (int a = 0; a < nh; ++a) {
      d[a] = sqrt(A[a][a] > 0.0 ? A[a][a] : 0.0);
      if (d[a] == 0.0 && zero < 0) zero = a;
    }
    bool ok = zero < 0;
    if (ok) {
      for (int a = 0; a < nh; ++a) {
        for (int b = 0; b < nh; ++b) A[a][b] /= d[a] * d[b];
        A[a][nh] = A[nh][a] = 1.0 / d[a];
        A[a][n] = 0.0;
      }
      A[nh][nh] = 0.0;
      A[nh][n] = 1.0;
    }
    for (int k = 0; k < n && ok; ++k) {
      int piv = k;
      for (int r = k + 1; r < n; ++r)
        if (fabs(A[r][k]) > fabs(A[piv][k])) piv = r;
      if (!(fabs(A[piv][k]) > 0.0)) ok = false;
      if (!ok) break;
      if (piv != k)
        for (int j = 0; j <= n; ++j) {
          const double t = A[k][j];
          A[k][j] = A[piv][j];
          A[piv][j] = t;
        }
      for (int r = k + 1; r < n; ++r) {
        const double f = A[r][k] / A[k][k];
        for (int j = k; j <= n; ++j) A[r][j] -= f * A[k][j];
      }
    }
    if (ok) {
      double x[M];
      for (int k = n - 1; k >= 0; --k) {
        double t = A[k][n];
        for (int j = k + 1; j < n; ++j) t -= A[k][j] * x[j];
        x[k] = t / A[k][k];
      }
      for (int a = 0; a < nh; ++a) {
        alpha[a] = x[a] / d[a];
        if (!(alpha[a] == alpha[a]) || fabs(alpha[a]) > 1e300) ok = false;
      }
      info[0] = 0;
    }
    if (!ok) {
      const int pick = zero >= 0 ? zero : newest;
      for (int a = 0; a < nh; ++a) alpha[a] = a == pick ? 1.0 : 0.0;
      info[0] = zero >= 0 ? 0 : 1;
    }
    state[2] = nh;
    state[0] = nh;
    state[1] = newest + 1 < nhmax ? newest + 1 : 0;
  }
};

// rho_in = sum a_i x_i (+ beta sum a_i R_i when kerker == 0); rbar = sum a_i R_i otherwise
template <typename T>
struct KPulayCombine {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const T* __restrict__ xh, const T* __restrict__ rh, size_t hstride,
                         const int* __restrict__ state, const double* __restrict__ alpha, double beta, int kerker,
                         T* __restrict__ rin, T* __restrict__ rbar, size_t n, unsigned nblk) {
    const int nh = state[2];
    GRID_FOR(c, n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= n) break;
      double xb = 0.0, rb = 0.0;
      for (int a = 0; a < nh; ++a) {
        xb += alpha[a] * (double)xh[(size_t)a * hstride + i];
        rb += alpha[a] * (double)rh[(size_t)a * hstride + i];
      }
      if (kerker) {
        rin[i] = (T)xb;
        rbar[i] = (T)rb;
      } else {
        rin[i] = (T)(xb + beta * rb);
      }
    }
  }
};

// W <- W |G|^2 / (|G|^2 + q0^2) / N over the whole grid (the 1/N of the forward transform)
template <typename T>
struct KKerker {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, cplx<T>* __restrict__ w, GridGeo g, double q0, double invN,
                         unsigned nblk) {
    GRID_FOR(c, g.n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= g.n) break;
      double gx, gy, gz;
      grid_g(g, i, gx, gy, gz);
      const double G2 = gx * gx + gy * gy + gz * gz;
      const double k = G2 / (G2 + q0 * q0) * invN;
      const cplx<T> v = w[i];
      w[i] = mk<T>((T)(k * (double)v.x), (T)(k * (double)v.y));
    }
  }
};

// out += beta Re(w)
template <typename T>
struct KAddReal {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const cplx<T>* __restrict__ w, double beta, T* __restrict__ out,
                         size_t n, unsigned nblk) {
    GRID_FOR(c, n, nblk) {
      const size_t i = i0_ + l_;
      if (i >= n) break;
      out[i] = (T)((double)out[i] + beta * (double)w[i].x);
    }
  }
};

template <typename T>
static fde_status pulay_t(fde_plan* p, int ns, int nhmax, int* state, T* xh, T* rh, T* rin, const T* rout,
                          double beta, double q0, int* info, hipStream_t s) {
  EmbedWs<T> e = embed_ws<T>(p);
  const size_t N = p->npts();
  const size_t n = (size_t)ns * N;
  const unsigned nb = red_blocks(n);
  const size_t red = 17 * sizeof(double);
  const int pmax = nhmax * (nhmax + 1) / 2;
  double* part = e.part;
  double* alpha = e.part + (size_t)kPulayBlocks * pmax;
  FDE_TRY(launch<KPulayStore<T>>(dim3(nb), kBlock, 0, s, xh, rh, (const int*)state, (const T*)rin, rout, n, nb));
  FDE_TRY(launch<KPulayGram<T>>(dim3(kPulayBlocks), kBlock, red, s, (const T*)rh, n, n, (const int*)state, nhmax, part,
                                (unsigned)kPulayBlocks));
  FDE_TRY(launch<KPulaySolve>(dim3(1), kBlock, red + (size_t)pmax * sizeof(double), s, (const double*)part,
                              kPulayBlocks, state, nhmax, alpha, info));
  const int kerker = q0 > 0.0 ? 1 : 0;
  if (!kerker)
    return launch<KPulayCombine<T>>(dim3(nb), kBlock, 0, s, (const T*)xh, (const T*)rh, n, (const int*)state,
                                    (const double*)alpha, beta, 0, rin, (T*)nullptr, n, nb);
  const GridGeo g = geo(p);
  const unsigned nbN = red_blocks(N);
  for (int I = 0; I < ns; ++I) {
    FDE_TRY(launch<KPulayCombine<T>>(dim3(nbN), kBlock, 0, s, (const T*)(xh + (size_t)I * N),
                                     (const T*)(rh + (size_t)I * N), n, (const int*)state, (const double*)alpha, beta,
                                     1, rin + (size_t)I * N, e.rho, N, nbN));
    FDE_TRY(launch<KToComplex<T>>(dim3(nbN), kBlock, 0, s, (const T*)e.rho, N, e.W0, nbN));
    FDE_TRY(fft3<T>(p, e.W0, false, s));
    FDE_TRY(launch<KKerker<T>>(dim3(nbN), kBlock, 0, s, e.W0, g, q0, 1.0 / (double)N, nbN));
    FDE_TRY(fft3<T>(p, e.W0, true, s));
    FDE_TRY(launch<KAddReal<T>>(dim3(nbN), kBlock, 0, s, (const cplx<T>*)e.W0, beta, rin + (size_t)I * N, N, nbN));
  }
  return FDE_OK;
}

// E_K per subsystem, the nonadditive terms and E_FDE by both routes (single thread;
// row layout of the inputs as in fde_energy_total).
struct KEnergyTotal {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, int ns, const double* __restrict__ en, const double* __restrict__ band,
                         const double* __restrict__ dots, double* __restrict__ out) {
    if (c.tid() != 0) return;
    const double* tot = en + (size_t)ns * FDE_NE;
    double tnad = tot[FDE_E_KIN], xnad = tot[FDE_E_XCNAD];
    for (int I = 0; I < ns; ++I) {
      tnad -= en[(size_t)I * FDE_NE + FDE_E_KIN];
      xnad -= en[(size_t)I * FDE_NE + FDE_E_XCNAD];
    }
    double direct = tot[FDE_E_HSELF] + tnad + xnad, frag = tnad + xnad;
    for (int I = 0; I < ns; ++I) {
      const double* e = en + (size_t)I * FDE_NE;
      const double* b = band + 3 * I;
      const double deband = -(dots[2 * I] - dots[2 * I + 1]);
      const double ek = b[2] + deband + e[FDE_E_XC] + 0.5 * e[FDE_E_HEMB];
      out[I] = ek;
      frag += ek;
      direct += b[0] + b[1] + e[FDE_E_LOC] + e[FDE_E_XC];
    }
    out[ns] = tnad;
    out[ns + 1] = xnad;
    out[ns + 2] = direct;
    out[ns + 3] = frag;
  }
};

}  // namespace fde

using namespace fde;

extern "C" {

fde_status fde_energy_total(int ns, const double* embed_energies, const double* band_terms, const double* dots,
                            double* out, hipStream_t s) {
  if (ns < 1) return fail(FDE_ERR_ARG, "ns must be >= 1");
  if (!embed_energies || !band_terms || !dots || !out) return fail(FDE_ERR_ARG, "null argument");
  return launch<KEnergyTotal>(dim3(1), 64, 0, s, ns, embed_energies, band_terms, dots, out);
}

fde_status fde_mix_pulay(fde_plan* p, int ns, int nhmax, int* state, void* x_hist, void* r_hist, void* rho_in,
                         const void* rho_out, double beta, double q0, int* info, hipStream_t s) {
  if (!p) return fail(FDE_ERR_ARG, "null plan");
  if (!p->ws) return fail(FDE_ERR_WORKSPACE, "no workspace attached (fde_plan_set_workspace)");
  if (ns < 1) return fail(FDE_ERR_ARG, "ns must be >= 1");
  if (nhmax < 1 || nhmax > FDE_PULAY_MAX) return fail(FDE_ERR_ARG, "nhmax must be in [1, FDE_PULAY_MAX]");
  if (!state || !x_hist || !r_hist || !rho_in || !rho_out || !info) return fail(FDE_ERR_ARG, "null argument");
  if (!(q0 >= 0.0) || !(beta > 0.0)) return fail(FDE_ERR_ARG, "need beta > 0 and q0 >= 0");
  if (p->prec == FDE_F64)
    return pulay_t<double>(p, ns, nhmax, state, (double*)x_hist, (double*)r_hist, (double*)rho_in,
                           (const double*)rho_out, beta, q0, info, s);
  return pulay_t<float>(p, ns, nhmax, state, (float*)x_hist, (float*)r_hist, (float*)rho_in, (const float*)rho_out,
                        beta, q0, info, s);
}

fde_status fde_embed_potential(fde_plan* p, int ns, const void* rho_sub, const void* vloc, const fde_functionals* f,
                               void* veff, double* energies, int* info, hipStream_t s) {
  if (!p) return fail(FDE_ERR_ARG, "null plan");
  if (!p->ws) return fail(FDE_ERR_WORKSPACE, "no workspace attached (fde_plan_set_workspace)");
  if (ns < 1) return fail(FDE_ERR_ARG, "ns must be >= 1");
  if (!rho_sub || !vloc || !f || !veff || !energies || !info) return fail(FDE_ERR_ARG, "null argument");
  if (f->xc < 0 || f->xc > 2 || f->xc_nad < 0 || f->xc_nad > 2 || f->kin_nad < 0 || f->kin_nad > 3)
    return fail(FDE_ERR_ARG, "unknown functional id");
  if (!(f->rho_thr >= 0)) return fail(FDE_ERR_ARG, "rho_thr must be >= 0");
  if (p->prec == FDE_F64)
    return embed_t<double>(p, ns, (const double*)rho_sub, (const double*)vloc, f, (double*)veff, energies, info, s);
  return embed_t<float>(p, ns, (const float*)rho_sub, (const float*)vloc, f, (float*)veff, energies, info, s);
}

fde_status fde_local_potential(fde_plan* p, int natoms, const double* pos, const double* Z, const double* width,
                               void* vloc, hipStream_t s) {
  if (!p) return fail(FDE_ERR_ARG, "null plan");
  if (!p->ws) return fail(FDE_ERR_WORKSPACE, "no workspace attached (fde_plan_set_workspace)");
  if (natoms < 0 || (natoms > 0 && (!pos || !Z || !width)) || !vloc) return fail(FDE_ERR_ARG, "null argument");
  if ((size_t)natoms * sizeof(Ion) > p->npts() * p->csize()) return fail(FDE_ERR_SHAPE, "too many atoms for the grid");
  std::vector<Ion> ions(natoms);
  for (int a = 0; a < natoms; ++a) {
    for (int i = 0; i < 3; ++i) ions[a].R[i] = pos[3 * a + i];
    ions[a].Z = Z[a];
    ions[a].w = width[a];
  }
  if (p->prec == FDE_F64) return vloc_t<double>(p, ions, (double*)vloc, s);
  return vloc_t<float>(p, ions, (float*)vloc, s);
}

fde_status fde_aug_density(fde_plan* p, int natom, const double* atoms, const double* charges, void* rho,
                           hipStream_t s) {
  if (!p) return fail(FDE_ERR_ARG, "null plan");
  if (!p->ws) return fail(FDE_ERR_WORKSPACE, "no workspace attached (fde_plan_set_workspace)");
  if (natom < 0 || (natom > 0 && (!atoms || !charges)) || !rho) return fail(FDE_ERR_ARG, "null argument");
  if (natom == 0) return FDE_OK;
  const size_t n = p->npts();
  const unsigned nb = red_blocks(n);
  if (p->prec == FDE_F64) {
    EmbedWs<double> e = embed_ws<double>(p);
    FDE_TRY(launch<KAugG<double>>(dim3(nb), kBlock, 0, s, atoms, charges, natom, geo(p), p->omega, e.W0, nb));
    FDE_TRY(fft3<double>(p, e.W0, true, s));
    return launch<KAddReal<double>>(dim3(nb), kBlock, 0, s, (const cplx<double>*)e.W0, 1.0, (double*)rho, n, nb);
  }
  EmbedWs<float> e = embed_ws<float>(p);
  FDE_TRY(launch<KAugG<float>>(dim3(nb), kBlock, 0, s, atoms, charges, natom, geo(p), p->omega, e.W0, nb));
  FDE_TRY(fft3<float>(p, e.W0, true, s));
  return launch<KAddReal<float>>(dim3(nb), kBlock, 0, s, (const cplx<float>*)e.W0, 1.0, (float*)rho, n, nb);
}

fde_status fde_mix(size_t n, double beta, void* rho_in, const void* rho_out, int prec, hipStream_t s) {
  if (!rho_in || !rho_out) return fail(FDE_ERR_ARG, "null argument");
  if (prec != FDE_F64 && prec != FDE_F32) return fail(FDE_ERR_ARG, "prec must be FDE_F64 or FDE_F32");
  const unsigned nb = red_blocks(n);
  if (n == 0) return FDE_OK;
  if (prec == FDE_F64) return launch<KMix<double>>(dim3(nb), kBlock, 0, s, (double*)rho_in, (const double*)rho_out, n, beta, nb);
  return launch<KMix<float>>(dim3(nb), kBlock, 0, s, (float*)rho_in, (const float*)rho_out, n, beta, nb);
}

fde_status fde_grid_dot(fde_plan* p, const void* a, const void* b, double* out, hipStream_t s) {
  if (!p) return fail(FDE_ERR_ARG, "null plan");
  if (!p->ws) return fail(FDE_ERR_WORKSPACE, "no workspace attached (fde_plan_set_workspace)");
  if (!a || !out) return fail(FDE_ERR_ARG, "null argument");
  const size_t n = p->npts();
  const unsigned nb = red_blocks(n);
  double* part = (double*)p->scratch;
  const size_t red = 17 * sizeof(double);
  if (p->prec == FDE_F64)
    FDE_TRY(launch<KDot<double>>(dim3(nb), kBlock, red, s, (const double*)a, (const double*)b, n, part, nb));
  else
    FDE_TRY(launch<KDot<float>>(dim3(nb), kBlock, red, s, (const float*)a, (const float*)b, n, part, nb));
  return launch<KRedAdd>(dim3(1), kBlock, red, s, (const double*)part, (int)nb, p->omega / (double)n, out, 0);
}

fde_status fde_density_l1(fde_plan* p, int ns, const void* rho_sub, const void* rho_ref, double* out,
                          hipStream_t s) {
  if (!p) return fail(FDE_ERR_ARG, "null plan");
  if (!p->ws) return fail(FDE_ERR_WORKSPACE, "no workspace attached (fde_plan_set_workspace)");
  if (ns < 1) return fail(FDE_ERR_ARG, "ns must be >= 1");
  if (!rho_sub || !rho_ref || !out) return fail(FDE_ERR_ARG, "null argument");
  const size_t n = p->npts();
  const unsigned nb = red_blocks(n);
  double* part = (double*)p->scratch;
  const size_t red = 17 * sizeof(double);
  if (p->prec == FDE_F64)
    FDE_TRY(launch<KAbsDiff<double>>(dim3(nb), kBlock, red, s, (const double*)rho_sub, ns, (const double*)rho_ref, n,
                                     part, nb));
  else
    FDE_TRY(launch<KAbsDiff<float>>(dim3(nb), kBlock, red, s, (const float*)rho_sub, ns, (const float*)rho_ref, n,
                                    part, nb));
  return launch<KRedAdd>(dim3(1), kBlock, red, s, (const double*)part, (int)nb, p->omega / (double)n, out, 0);
}

fde_status fde_frozen_environment(fde_plan* p, int ns, const void* rho_sub, void* env, size_t ld,
                                  hipStream_t s) {
  if (!p) return fail(FDE_ERR_ARG, "null plan");
  if (ns < 1) return fail(FDE_ERR_ARG, "ns must be >= 1");
  if (!rho_sub || !env) return fail(FDE_ERR_ARG, "null argument");
  const size_t n = p->npts();
  if (ld < n) return fail(FDE_ERR_ARG, "ld must be at least the number of grid points");
  const unsigned nb = red_blocks(n);
  if (p->prec == FDE_F64)
    return launch<KEnvironment<double>>(dim3(nb, ns), kBlock, 0, s, (const double*)rho_sub, ns, n, (double*)env, ld,
                                        nb);
  return launch<KEnvironment<float>>(dim3(nb, ns), kBlock, 0, s, (const float*)rho_sub, ns, n, (float*)env, ld, nb);
}

fde_status fde_grid_mean(fde_plan* p, const void* a, double* out, hipStream_t s) {
  if (!p) return fail(FDE_ERR_ARG, "null plan");
  if (!p->ws) return fail(FDE_ERR_WORKSPACE, "no workspace attached (fde_plan_set_workspace)");
  if (!a || !out) return fail(FDE_ERR_ARG, "null argument");
  const size_t n = p->npts();
  const unsigned nb = red_blocks(n);
  double* part = (double*)p->scratch;
  const size_t red = 17 * sizeof(double);
  if (p->prec == FDE_F64)
    FDE_TRY(launch<KDot<double>>(dim3(nb), kBlock, red, s, (const double*)a, (const double*)nullptr, n, part, nb));
  else
    FDE_TRY(launch<KDot<float>>(dim3(nb), kBlock, red, s, (const float*)a, (const float*)nullptr, n, part, nb));
  return launch<KRedAdd>(dim3(1), kBlock, red, s, (const double*)part, (int)nb, 1.0 / (double)n, out, 1);
}

}  // extern "C"
