// Host entry points of the plane-wave kernels: fde_apply_h, fde_density,
// fde_kb_projectors, fde_init_bands, fde_band_energies.
#include <algorithm>
#include <cmath>

#include "kernels_gemm.hpp"
#include "kernels_plane.hpp"
#include "kernels_plane4.hpp"
#include "kernels_pw.hpp"
#include "launch.hpp"

// register plane passes: at least two waves per SIMD
constexpr int REGW = 2;

namespace fde {

static KVec kvec(const fde_plan* p, int ik) {
  KVec k;
  for (int i = 0; i < 3; ++i) {
    k.kf[i] = p->k[ik].kf[i];
    k.b[i] = p->b[i];
  }
  return k;
}

// z-passes with the four-step register FFT where N3 = P Q is specialised (240 = 16 x 15,
// 120 = 8 x 15) and not switched off by tuning; the LDS Stockham passes otherwise.
template <typename T, int P, int Q>
static fde_status z_inv_reg(const KTables& t, int nbc, const cplx<T>* ps, const cplx<T>* tw3, cplx<T>* sb,
                            hipStream_t s) {
  using Z = ZReg<T, P, Q>;
  return launch<KZInvReg<T, P, Q>, 64 * Z::WPB>(dim3((t.ncol + Z::SPB - 1) / Z::SPB, nbc), 64 * Z::WPB,
                                                Z::lds_bytes(), s, ps, t.npw, (const int4*)t.d_sticks, t.ncol, tw3,
                                                sb);
}

template <typename T, int P, int Q>
static fde_status z_fwd_reg(const fde_plan* p, const KTables& t, int nbc, const cplx<T>* sb, const cplx<T>* ps,
                            cplx<T>* hs, const cplx<T>* tw3, KVec kv, double invN, hipStream_t s) {
  using Z = ZReg<T, P, Q>;
  return launch<KZFwdReg<T, P, Q>, 64 * Z::WPB>(dim3((t.ncol + Z::SPB - 1) / Z::SPB, nbc), 64 * Z::WPB,
                                                Z::lds_bytes(), s, sb, ps, hs, t.npw, (const int4*)t.d_sticks,
                                                (const int*)t.d_xlist, t.ncol, p->N[0], p->N[1], tw3, kv, invN);
}

// 432 = 16 x 27 holds 27 complex values per lane in the first step: FP32 only (FP64
// would spill).
static int z_reg_kind(const fde_plan* p) {
  if (p->tune_zreg == 1) return 0;
  if (p->N[2] == 432) return p->prec == FDE_F32 ? 3 : 0;
  return p->N[2] == 240 ? 1 : (p->N[2] == 120 ? 2 : 0);
}

// Threads of a z-pass workgroup: one wavefront per stick up to kBlock.
static int zthreads(int SZ) { return std::min(kBlock, 64 * SZ); }

// Sticks per z-pass workgroup: the largest power of two up to 4 (or the tuned value, at
// most 16) whose LDS fits 80 KiB. Small groups keep many workgroups resident per CU,
// which hides the latency of the scattered sphere loads.

static int stick_group(const fde_plan* p) {
  const size_t cs = p->csize();
  const int top = p->tune_sz > 0 ? std::min(16, p->tune_sz) : 4;
  for (int sz = top; sz > 1; sz /= 2)
    if ((2 * (size_t)p->N[2] * (sz + 1) + p->N[2]) * cs <= 80 * 1024) return sz;
  return 1;
}

// Rows per batch of the plane pass: as many as fit 80 KiB (two workgroups per
// CU), else 160 KiB.
template <typename T>
static int plane_rows(const fde_plan* p, int ik, bool acc, size_t* lds) {
  const KTables& t = p->k[ik];
  for (size_t budget : {(size_t)80 * 1024, kLdsMax}) {
    for (int rb = p->N[1]; rb >= 1; rb = (rb > 8 ? rb / 2 : rb - 1)) {
      size_t b = PlaneLds<T>::bytes(p->N[0], p->N[1], t.nxa, rb, t.ncol, acc);
      if (b <= budget) {
        *lds = b;
        return rb;
      }
    }
  }
  return 0;
}

// Rows of the two-factor plane pass's row buffer: kPlane4Waves RW, RW rows per wavefront
// (RW times the larger factor of N1 at most 64 lanes). The tuned value rounded down to a
// multiple of kPlane4Waves, else the largest RW whose LDS fits 80 KiB (two workgroups per
// CU; a whole CU if none does). 0 when not even one row per wavefront fits.
template <typename T>
static int plane4_rows(const fde_plan* p, int ik, size_t* lds) {
  const KTables& t = p->k[ik];
  const int N1 = p->N[0], N2 = p->N[1];
  const Split2 s1 = split2(N1);
  const int rwmax = 64 / std::max(s1.p, s1.q);
  if (p->tune_rows > 0) {
    const int rb = kPlane4Waves * std::max(1, std::min(rwmax, p->tune_rows / kPlane4Waves));
    *lds = plane4_lds<T>(N1, N2, t.nxa, rb);
    return *lds <= kLdsMax ? rb : 0;
  }
  for (size_t budget : {(size_t)80 * 1024, kLdsMax}) {
    for (int rw = rwmax; rw >= 1; --rw) {
      const size_t b = plane4_lds<T>(N1, N2, t.nxa, kPlane4Waves * rw);
      if (b <= budget) {
        *lds = b;
        return kPlane4Waves * rw;
      }
    }
  }
  return 0;
}

// Plane pass kind: the tuned one where it applies, else (FP32) the whole-line
// register pass, else the two-factor LDS pass where both in-plane lengths are
// supported, else the register pass, else the LDS Stockham pass. 0 when none
// applies.
enum { kPlaneReg = 1, kPlaneLds = 2, kPlane4 = 3 };
template <typename T>
static int plane_kind(const fde_plan* p, int ik, bool reg_ok, bool lds_ok, bool p4_ok) {
  switch (p->tune_plane) {
    case kPlaneReg: if (reg_ok) return kPlaneReg; break;
    case kPlaneLds: if (lds_ok) return kPlaneLds; break;
    case kPlane4: if (p4_ok) return kPlane4; break;
    default: break;
  }
  // FP32: the whole-line register pass is the faster where it exists (60 x 60 planes,
  // measured); FP64: the two-factor pass.
  if (reg_ok && sizeof(T) == 4) return kPlaneReg;
  if (p4_ok) return kPlane4;
  if (reg_ok) return kPlaneReg;
  if (lds_ok) return kPlaneLds;
  return 0;
}

// Plane-wave chunks of the projections: kKbChunk per workgroup for the one-block product
// (few projectors and bands); for the tiled product (tiles of launch_ahb) about 2048
// workgroups over the chip, so that each runs a long k loop and the FP64 partials stay
// small. A chunk count at most that of kKbChunk-wide chunks, which sizes the workspace.
template <typename T>
static int kb_chunk(int npw, int nproj, int nb) {
  if (nproj <= 64 && nb <= 64) return kKbChunk;
  const int ts = ahb_tile<T>(nproj, nb);
  const int tiles = ((nproj + ts - 1) / ts) * ((nb + ts - 1) / ts);
  const int nc = std::max(1, std::min((npw + kKbChunk - 1) / kKbChunk, 2048 / tiles));
  return std::max(kKbChunk, ((npw + nc - 1) / nc + 63) / 64 * 64);
}

// part[chunk][i][n] = sum_{G in chunk} conj(beta_i(G)) psi_n(G), chunks of kb_chunk plane waves
template <typename T>
static fde_status kb_project(const cplx<T>* beta, const cplx<T>* psi, int npw, int nproj, int nb, int nchunk,
                             cplx<double>* part, hipStream_t s) {
  const AhBProb<T> prob{beta, psi, nullptr, nproj, nb, npw, nchunk, kb_chunk<T>(npw, nproj, nb), part};
  if (nproj <= 64 && nb <= 64)
    return launch<KAhBAll<T>, 512>(dim3(nchunk), 512, KAhBAll<T>::lds_bytes(nproj, nb), s, prob);
  AhBSet<T> set;
  set.n = 1;
  set.p[0] = prob;
  return launch_ahb<T>(nchunk, nproj, nb, 1, set, s);
}

template <typename T>
static fde_status apply_h_t(fde_plan* p, int ik, int nb, const cplx<T>* psi, cplx<T>* hpsi, const T* veff, int nproj,
                            const cplx<T>* beta, const double* dkb, hipStream_t s) {
  const KTables& t = p->k[ik];
  const int N1 = p->N[0], N2 = p->N[1], N3 = p->N[2];
  const int SZ = stick_group(p);
  const size_t zlds = KZInv<T>::lds_bytes(N3, SZ);
  size_t plds = 0;
  const int RB = plane_rows<T>(p, ik, false, &plds);
  const bool fp64 = sizeof(T) == 8;
  const size_t rlds = reg_plane_lds<T>(N2, t.nxa, t.ncol);
  const int cls = reg_len_class(N1, fp64);
  const bool reg_plane = t.xrange && cls >= 0 && cls == reg_len_class(N2, fp64) && rlds <= kLdsMax;
  size_t lds4 = 0;
  const int RB4 = (t.xrange && plane4_len_ok(N1) && plane4_len_ok(N2)) ? plane4_rows<T>(p, ik, &lds4) : 0;
  const int kind = plane_kind<T>(p, ik, reg_plane, RB > 0, RB4 > 0);
  if (kind == 0) return fail(FDE_ERR_UNSUPPORTED, "plane does not fit in LDS");
  const double invN = 1.0 / ((double)N1 * N2 * N3);
  const KVec kv = kvec(p, ik);
  cplx<T>* sb = (cplx<T>*)p->scratch;
  size_t off = align256((size_t)p->max_nb * N3 * stick_stride(p->ncol_max) * sizeof(cplx<T>));
  cplx<double>* part = (cplx<double>*)(p->scratch + off);
  const int nchunk = (t.npw + kKbChunk - 1) / kKbChunk;
  off += align256((size_t)nchunk * p->max_nproj * p->max_nb * 16);
  cplx<T>* dp = (cplx<T>*)(p->scratch + off);
  const cplx<T>* tw1 = (const cplx<T>*)p->d_tw[0];
  const cplx<T>* tw2 = (const cplx<T>*)p->d_tw[1];
  const cplx<T>* tw3 = (const cplx<T>*)p->d_tw[2];
  for (int b0 = 0; b0 < nb; b0 += p->max_nb) {
    const int nbc = std::min(p->max_nb, nb - b0);
    const cplx<T>* ps = psi + (size_t)b0 * t.npw;
    cplx<T>* hs = hpsi + (size_t)b0 * t.npw;
    const unsigned ngz = (unsigned)((t.ncol + SZ - 1) / SZ);
    const int zk = z_reg_kind(p);
    if (zk == 1)
      FDE_TRY((z_inv_reg<T, 16, 15>(t, nbc, ps, tw3, sb, s)));
    else if (zk == 2)
      FDE_TRY((z_inv_reg<T, 8, 15>(t, nbc, ps, tw3, sb, s)));
    else if (zk == 3)
      FDE_TRY((z_inv_reg<T, 16, 27>(t, nbc, ps, tw3, sb, s)));
    else
      FDE_TRY(launch<KZInv<T>>(dim3(ngz, nbc), zthreads(SZ), zlds, s, ps, t.npw, (const int4*)t.d_sticks, t.ncol,
                               p->rad[2], tw3, sb, SZ));
    if (kind == kPlane4) {
      // at most 8 bands per workgroup, fewer where that would leave under ~8192 workgroups
      // (tail balance over 256 CUs at two workgroups each), unless tuned
      const int BPW = p->tune_bpw > 0 ? std::min(nbc, p->tune_bpw)
                                      : std::max(1, std::min(std::min(nbc, 8), (N3 * nbc) / 8192));
      FDE_TRY(launch<KPlaneH4<T>>(dim3(N3, (nbc + BPW - 1) / BPW), 64 * kPlane4Waves, lds4, s, sb, nbc, BPW,
                                  (const int4*)t.d_sticks, t.ncol, t.nxa, t.mlo, N1, N2, N3, RB4, tw1, tw2, veff));
    } else if (kind == kPlaneReg) {
      // about two workgroups (one wave each) per SIMD over the whole chip, unless tuned
      const int BPW = p->tune_bpw > 0 ? std::min(nbc, p->tune_bpw) : std::max(1, std::min(nbc, (N3 * nbc) / 4096));
      const dim3 g(N3, (nbc + BPW - 1) / BPW);
      if (cls == 0)
        FDE_TRY(launch<KPlaneHReg<T, 0>, 64, REGW>(g, 64, rlds, s, sb, nbc, BPW, (const int4*)t.d_sticks, t.ncol,
                                                   t.nxa, t.mlo, N1, N2, N3, veff));
      else
        FDE_TRY(launch<KPlaneHReg<T, 1>, 64, REGW>(g, 64, rlds, s, sb, nbc, BPW, (const int4*)t.d_sticks, t.ncol,
                                                   t.nxa, t.mlo, N1, N2, N3, veff));
    } else {
      const int BPW = p->tune_bpw > 0 ? std::min(nbc, p->tune_bpw) : std::max(1, std::min(nbc, (N3 * nbc) / 4096));
      FDE_TRY(launch<KPlaneH<T>>(dim3(N3, (nbc + BPW - 1) / BPW), kBlock, plds, s, sb, nbc, BPW,
                                 (const int4*)t.d_sticks, (const int*)t.d_xlist, t.ncol, t.nxa, p->rad[0], p->rad[1],
                                 N3, tw1, tw2, veff, RB));
    }
    if (zk == 1)
      FDE_TRY((z_fwd_reg<T, 16, 15>(p, t, nbc, sb, ps, hs, tw3, kv, invN, s)));
    else if (zk == 2)
      FDE_TRY((z_fwd_reg<T, 8, 15>(p, t, nbc, sb, ps, hs, tw3, kv, invN, s)));
    else if (zk == 3)
      FDE_TRY((z_fwd_reg<T, 16, 27>(p, t, nbc, sb, ps, hs, tw3, kv, invN, s)));
    else
      FDE_TRY(launch<KZFwd<T>>(dim3(ngz, nbc), zthreads(SZ), zlds, s, (const cplx<T>*)sb, ps, hs, t.npw,
                               (const int4*)t.d_sticks, (const int*)t.d_xlist, t.ncol, N1, N2, p->rad[2], tw3, kv,
                               invN, SZ));
    if (nproj > 0) {
      const int kc = kb_chunk<T>(t.npw, nproj, nbc), nck = (t.npw + kc - 1) / kc;
      FDE_TRY(kb_project<T>(beta, ps, t.npw, nproj, nbc, nck, part, s));
      FDE_TRY(launch<KKbReduce<T>>(dim3((nproj * nbc + KKbReduce<T>::NO - 1) / KKbReduce<T>::NO), kBlock,
                                   KKbReduce<T>::NG * KKbReduce<T>::NO * sizeof(cplx<double>), s,
                                   (const cplx<double>*)part, nck,
                                   nproj, nbc, dkb, dp));
      if (nbc <= 4 * kKbAddTiles * 16)
        // FP32: two column groups per workgroup (dp read half as often), two waves per SIMD
        if (sizeof(T) == 4)
          FDE_TRY((launch<KKbAddMfma<T, 2>, 256, 2>(dim3((t.npw + 31) / 32), kBlock, 0, s, beta, (const cplx<T>*)dp,
                                                    hs, t.npw, nproj, nbc)));
        else
          FDE_TRY(launch<KKbAddMfma<T>>(dim3((t.npw + 15) / 16), kBlock, 0, s, beta, (const cplx<T>*)dp, hs, t.npw,
                                        nproj, nbc));
      else
        FDE_TRY(launch<KKbAdd<T>>(dim3((t.npw + KKbAdd<T>::TG - 1) / KKbAdd<T>::TG), kBlock, KKbAdd<T>::lds_bytes(),
                                  s, beta, (const cplx<T>*)dp, hs, t.npw, nproj, nbc));
    }
  }
  return FDE_OK;
}

template <typename T>
static fde_status density_t(fde_plan* p, int ik, int nb, const cplx<T>* psi, const double* occw, T* rho,
                            hipStream_t s) {
  const KTables& t = p->k[ik];
  const int N3 = p->N[2];
  const int SZ = stick_group(p);
  const size_t zlds = KZInv<T>::lds_bytes(N3, SZ);
  size_t plds = 0;
  const int RB = plane_rows<T>(p, ik, true, &plds);
  const int N1 = p->N[0], N2 = p->N[1];
  const bool fp64 = sizeof(T) == 8;
  const size_t rlds = reg_plane_lds<T>(N2, t.nxa, t.ncol);
  const int cls = reg_len_class(N1, fp64);
  const bool reg_plane = t.xrange && cls >= 0 && cls == reg_len_class(N2, fp64) && rlds <= kLdsMax;
  size_t lds4 = 0;
  const int RB4 = (t.xrange && plane4_len_ok(N1) && plane4_len_ok(N2)) ? plane4_rows<T>(p, ik, &lds4) : 0;
  const int kind = plane_kind<T>(p, ik, reg_plane, RB > 0, RB4 > 0);
  if (kind == 0) return fail(FDE_ERR_UNSUPPORTED, "plane does not fit in LDS");
  cplx<T>* sb = (cplx<T>*)p->scratch;
  T* part = (T*)(p->scratch + align256((size_t)p->max_nb * N3 * stick_stride(p->ncol_max) * sizeof(cplx<T>)));
  const cplx<T>* tw1 = (const cplx<T>*)p->d_tw[0];
  const cplx<T>* tw2 = (const cplx<T>*)p->d_tw[1];
  const cplx<T>* tw3 = (const cplx<T>*)p->d_tw[2];
  const size_t n = p->npts();
  for (int b0 = 0; b0 < nb; b0 += p->max_nb) {
    const int nbc = std::min(p->max_nb, nb - b0);
    const unsigned ngz = (unsigned)((t.ncol + SZ - 1) / SZ);
    const int zk = z_reg_kind(p);
    if (zk == 1)
      FDE_TRY((z_inv_reg<T, 16, 15>(t, nbc, psi + (size_t)b0 * t.npw, tw3, sb, s)));
    else if (zk == 2)
      FDE_TRY((z_inv_reg<T, 8, 15>(t, nbc, psi + (size_t)b0 * t.npw, tw3, sb, s)));
    else if (zk == 3)
      FDE_TRY((z_inv_reg<T, 16, 27>(t, nbc, psi + (size_t)b0 * t.npw, tw3, sb, s)));
    else
      FDE_TRY(launch<KZInv<T>>(dim3(ngz, nbc), zthreads(SZ), zlds, s, psi + (size_t)b0 * t.npw, t.npw,
                               (const int4*)t.d_sticks, t.ncol, p->rad[2], tw3, sb, SZ));
    const int ngroups = std::min(kRhoGroups, nbc);
    const int BPW = (nbc + ngroups - 1) / ngroups;
    const int ng = (nbc + BPW - 1) / BPW;
    if (kind == kPlane4)
      FDE_TRY(launch<KPlaneRho4<T>>(dim3(N3, ng), 64 * kPlane4Waves, lds4, s, (const cplx<T>*)sb, nbc, BPW, occw + b0,
                                    (const int4*)t.d_sticks, t.ncol, t.nxa, t.mlo, N1, N2, N3, RB4, tw1, tw2, part,
                                    1.0 / p->omega));
    else if (kind == kPlaneReg && cls == 0)
      FDE_TRY(launch<KPlaneRhoReg<T, 0>, 64, REGW>(dim3(N3, ng), 64, rlds, s, (const cplx<T>*)sb, nbc, BPW,
                                                   occw + b0, (const int4*)t.d_sticks, t.ncol, t.nxa, t.mlo, N1, N2,
                                                   N3, part, 1.0 / p->omega));
    else if (kind == kPlaneReg)
      FDE_TRY(launch<KPlaneRhoReg<T, 1>, 64, REGW>(dim3(N3, ng), 64, rlds, s, (const cplx<T>*)sb, nbc, BPW,
                                                   occw + b0, (const int4*)t.d_sticks, t.ncol, t.nxa, t.mlo, N1, N2,
                                                   N3, part, 1.0 / p->omega));
    else
      FDE_TRY(launch<KPlaneRho<T>>(dim3(N3, ng), kBlock, plds, s, (const cplx<T>*)sb, nbc, BPW, occw + b0,
                                   (const int4*)t.d_sticks, (const int*)t.d_xlist, t.ncol, t.nxa, p->rad[0],
                                   p->rad[1], N3, tw1, tw2, part, 1.0 / p->omega, RB));
    FDE_TRY(launch<KRhoReduce<T>>(dim3((unsigned)((n + kBlk - 1) / kBlk)), kBlock, 0, s, (const T*)part, ng, n, rho));
  }
  return FDE_OK;
}

// ---------------------------------------------------------------------------
// Projectors, initial bands, band energies
// ---------------------------------------------------------------------------
struct KbAtom {
  double R[3];
  double r;
  int lmax;
  int first;  // index of its first channel
};

template <typename T>
struct KKbBuild {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const KbAtom* __restrict__ atoms, int natoms, const int* __restrict__ millp,
                         int npw, KVec kv, double omega, cplx<T>* __restrict__ beta) {
    const double pi = 3.14159265358979323846;
    for (int l = c.tid(); l < kBlk; l += c.nthr()) {
      const int g = c.bx() * kBlk + l;
      if (g >= npw) break;
      int m1, m2, m3;
      unpack_mill(millp[g], m1, m2, m3);
      const double q[3] = {(m1 + kv.kf[0]) * kv.b[0], (m2 + kv.kf[1]) * kv.b[1], (m3 + kv.kf[2]) * kv.b[2]};
      const double q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
      const double pref = 1.0 / sqrt(omega);
      for (int a = 0; a < natoms; ++a) {
        const KbAtom at = atoms[a];
        if (at.lmax < 0) continue;
        const double ph = -(q[0] * at.R[0] + q[1] * at.R[1] + q[2] * at.R[2]);
        const double cr = cos(ph), ci = sin(ph);
        const double gs = exp(-0.5 * q2 * at.r * at.r);
        const double ss = pref * 2.0 * sqrt(2.0) * pow(pi, 0.75) * pow(at.r, 1.5) * gs;
        beta[(size_t)at.first * npw + g] = mk<T>((T)(ss * cr), (T)(ss * ci));
        if (at.lmax >= 1) {
          const double sp = pref * 4.0 * pow(pi, 0.75) * pow(at.r, 2.5) * gs;
          for (int d = 0; d < 3; ++d)
            beta[(size_t)(at.first + 1 + d) * npw + g] = mk<T>((T)(sp * q[d] * cr), (T)(sp * q[d] * ci));
        }
      }
    }
  }
};

template <typename T>
struct KInitBands {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const cplx<T>* __restrict__ raw, cplx<T>* __restrict__ psi,
                         const int* __restrict__ millp, int npw, KVec kv) {
    const int n = c.by();
    for (int l = c.tid(); l < kBlk; l += c.nthr()) {
      const int g = c.bx() * kBlk + l;
      if (g >= npw) break;
      int m1, m2, m3;
      unpack_mill(millp[g], m1, m2, m3);
      const double d = 1.0 / (1.0 + 2.0 * kin_of(kv, m1, m2, m3));
      const cplx<T> r = raw[(size_t)n * npw + g];
      psi[(size_t)n * npw + g] = mk<T>((T)(d * r.x), (T)(d * r.y));
    }
  }
};

// out[0] += sum_n w_n sum_G kin |psi|^2 ; one block per band (deterministic per band), then KSum
template <typename T>
struct KBandKin {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const cplx<T>* __restrict__ psi, const double* __restrict__ occw,
                         const int* __restrict__ millp, int npw, KVec kv, double* __restrict__ per_band) {
    const int n = c.bx();
    double acc = 0.0;
    for (int g = c.tid(); g < npw; g += c.nthr()) {
      int m1, m2, m3;
      unpack_mill(millp[g], m1, m2, m3);
      const cplx<T> v = psi[(size_t)n * npw + g];
      acc += kin_of(kv, m1, m2, m3) * ((double)v.x * v.x + (double)v.y * v.y);
    }
    acc = c.sum(acc, (double*)lds);
    if (c.tid() == 0) per_band[n] = occw[n] * acc;
  }
};

// out[slot] += sum_i per_item[i]  (single block, fixed order)
struct KSumInto {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const double* __restrict__ v, int n, double* __restrict__ out) {
    double acc = 0.0;
    for (int i = c.tid(); i < n; i += c.nthr()) acc += v[i];
    acc = c.sum(acc, (double*)lds);
    if (c.tid() == 0) out[0] += acc;
  }
};

// out[0] += sum_i a_i b_i  (single block, fixed order)
struct KSumProd {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const double* __restrict__ a, const double* __restrict__ b, int n,
                         double* __restrict__ out) {
    double acc = 0.0;
    for (int i = c.tid(); i < n; i += c.nthr()) acc += a[i] * b[i];
    acc = c.sum(acc, (double*)lds);
    if (c.tid() == 0) out[0] += acc;
  }
};

// per_band[n] = occw_n sum_i D_i |dp-free projections|^2 from part (FP64) partials
struct KBandNl {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const cplx<double>* __restrict__ part, int nchunk, int nproj, int nb,
                         const double* __restrict__ dkb, const double* __restrict__ occw, double* __restrict__ per_band) {
    const int n = c.bx();
    double acc = 0.0;
    for (int i = c.tid(); i < nproj; i += c.nthr()) {
      double sx = 0, sy = 0;
      for (int k = 0; k < nchunk; ++k) {
        sx += part[((size_t)k * nproj + i) * nb + n].x;
        sy += part[((size_t)k * nproj + i) * nb + n].y;
      }
      acc += dkb[i] * (sx * sx + sy * sy);
    }
    acc = c.sum(acc, (double*)lds);
    if (c.tid() == 0) per_band[n] = occw[n] * acc;
  }
};

template <typename T>
static fde_status band_energies_t(fde_plan* p, int ik, int nb, const cplx<T>* psi, const double* occw,
                                  const double* eval, int nproj, const cplx<T>* beta, const double* dkb, double* out,
                                  hipStream_t s) {
  const KTables& t = p->k[ik];
  if (nb > p->max_nb) return fail(FDE_ERR_SHAPE, "fde_band_energies: nb exceeds the workspace's max_nb");
  if (nproj > p->max_nproj) return fail(FDE_ERR_SHAPE, "nproj exceeds the workspace's max_nproj");
  const int nchunk = (t.npw + kKbChunk - 1) / kKbChunk;
  cplx<double>* part = (cplx<double>*)(p->scratch);
  double* per_band = (double*)(p->scratch + align256((size_t)nchunk * p->max_nproj * p->max_nb * 16 + 16));
  const KVec kv = kvec(p, ik);
  FDE_TRY(launch<KBandKin<T>>(dim3(nb), kBlock, 17 * sizeof(double), s, psi, occw, (const int*)t.d_millp, t.npw, kv,
                              per_band));
  FDE_TRY(launch<KSumInto>(dim3(1), kBlock, 17 * sizeof(double), s, (const double*)per_band, nb, out));
  if (nproj > 0) {
    const int kc = kb_chunk<T>(t.npw, nproj, nb), nck = (t.npw + kc - 1) / kc;
    FDE_TRY(kb_project<T>(beta, psi, t.npw, nproj, nb, nck, part, s));
    FDE_TRY(launch<KBandNl>(dim3(nb), kBlock, 17 * sizeof(double), s, (const cplx<double>*)part, nck, nproj, nb,
                            dkb, occw, per_band));
    FDE_TRY(launch<KSumInto>(dim3(1), kBlock, 17 * sizeof(double), s, (const double*)per_band, nb, out + 1));
  }
  if (eval) FDE_TRY(launch<KSumProd>(dim3(1), kBlock, 17 * sizeof(double), s, occw, eval, nb, out + 2));
  return FDE_OK;
}

}  // namespace fde

using namespace fde;

extern "C" {

fde_status fde_apply_h(fde_plan* p, int ik, int nb, const void* psi, void* hpsi, const void* veff, int nproj,
                       const void* beta, const double* dkb, hipStream_t s) {
  FDE_TRY(check_plan(p, ik));
  if (nb < 0 || nproj < 0) return fail(FDE_ERR_ARG, "negative size");
  if (nb == 0) return FDE_OK;
  if (!psi || !hpsi || !veff) return fail(FDE_ERR_ARG, "null array");
  if (psi == hpsi) return fail(FDE_ERR_ARG, "hpsi must not alias psi");
  if (nproj > 0 && (!beta || !dkb)) return fail(FDE_ERR_ARG, "nproj > 0 needs beta and dkb");
  if (nproj > p->max_nproj) return fail(FDE_ERR_SHAPE, "nproj exceeds the workspace's max_nproj");
  if (p->prec == FDE_F64)
    return apply_h_t<double>(p, ik, nb, (const cplx<double>*)psi, (cplx<double>*)hpsi, (const double*)veff, nproj,
                             (const cplx<double>*)beta, dkb, s);
  return apply_h_t<float>(p, ik, nb, (const cplx<float>*)psi, (cplx<float>*)hpsi, (const float*)veff, nproj,
                          (const cplx<float>*)beta, dkb, s);
}

fde_status fde_density(fde_plan* p, int ik, int nb, const void* psi, const double* occw, void* rho, hipStream_t s) {
  FDE_TRY(check_plan(p, ik));
  if (nb < 0) return fail(FDE_ERR_ARG, "negative size");
  if (nb == 0) return FDE_OK;
  if (!psi || !occw || !rho) return fail(FDE_ERR_ARG, "null array");
  if (p->prec == FDE_F64)
    return density_t<double>(p, ik, nb, (const cplx<double>*)psi, occw, (double*)rho, s);
  return density_t<float>(p, ik, nb, (const cplx<float>*)psi, occw, (float*)rho, s);
}

fde_status fde_kb_projectors(fde_plan* p, int ik, int natoms, const double* pos, const int* lmax, const double* rbeta,
                             void* beta, int* nproj, hipStream_t s) {
  FDE_TRY(check_plan(p, ik));
  if (natoms < 0 || (natoms > 0 && (!pos || !lmax || !rbeta)) || !nproj) return fail(FDE_ERR_ARG, "null argument");
  std::vector<KbAtom> at(natoms);
  int np = 0;
  for (int a = 0; a < natoms; ++a) {
    for (int i = 0; i < 3; ++i) at[a].R[i] = pos[3 * a + i];
    at[a].r = rbeta[a];
    at[a].lmax = lmax[a];
    at[a].first = np;
    if (lmax[a] > 1 || lmax[a] < -1) return fail(FDE_ERR_ARG, "lmax must be -1, 0 or 1");
    if (lmax[a] >= 0) np += (lmax[a] == 0 ? 1 : 4);
  }
  *nproj = np;
  if (np == 0) return FDE_OK;
  if (!beta) return fail(FDE_ERR_ARG, "null beta");
  // atom table staged in the scratch area (synchronous copy)
  KbAtom* d_at = (KbAtom*)p->scratch;
  FDE_TRY(stream_sync(s));  // the scratch area may still be in use by earlier work on s
  FDE_TRY(copy_h2d_sync(d_at, at.data(), natoms * sizeof(KbAtom)));
  const KTables& t = p->k[ik];
  if (p->prec == FDE_F64)
    return launch<KKbBuild<double>>(dim3((t.npw + kBlk - 1) / kBlk), kBlock, 0, s, (const KbAtom*)d_at, natoms,
                                    (const int*)t.d_millp, t.npw, kvec(p, ik), p->omega, (cplx<double>*)beta);
  return launch<KKbBuild<float>>(dim3((t.npw + kBlk - 1) / kBlk), kBlock, 0, s, (const KbAtom*)d_at, natoms,
                                 (const int*)t.d_millp, t.npw, kvec(p, ik), p->omega, (cplx<float>*)beta);
}

fde_status fde_init_bands(fde_plan* p, int ik, int nb, const void* raw, void* psi, hipStream_t s) {
  FDE_TRY(check_plan(p, ik));
  if (nb < 0) return fail(FDE_ERR_ARG, "negative size");
  if (nb == 0) return FDE_OK;
  if (!raw || !psi) return fail(FDE_ERR_ARG, "null array");
  const KTables& t = p->k[ik];
  dim3 g((t.npw + kBlk - 1) / kBlk, nb);
  if (p->prec == FDE_F64)
    return launch<KInitBands<double>>(g, kBlock, 0, s, (const cplx<double>*)raw, (cplx<double>*)psi,
                                      (const int*)t.d_millp, t.npw, kvec(p, ik));
  return launch<KInitBands<float>>(g, kBlock, 0, s, (const cplx<float>*)raw, (cplx<float>*)psi, (const int*)t.d_millp,
                                   t.npw, kvec(p, ik));
}

fde_status fde_band_energies(fde_plan* p, int ik, int nb, const void* psi, const double* occw, const double* eval,
                             int nproj, const void* beta, const double* dkb, double* out, hipStream_t s) {
  FDE_TRY(check_plan(p, ik));
  if (nb < 0 || nproj < 0) return fail(FDE_ERR_ARG, "negative size");
  if (nb == 0) return FDE_OK;
  if (!psi || !occw || !out || (nproj > 0 && (!beta || !dkb))) return fail(FDE_ERR_ARG, "null array");
  if (p->prec == FDE_F64)
    return band_energies_t<double>(p, ik, nb, (const cplx<double>*)psi, occw, eval, nproj, (const cplx<double>*)beta,
                                   dkb, out, s);
  return band_energies_t<float>(p, ik, nb, (const cplx<float>*)psi, occw, eval, nproj, (const cplx<float>*)beta, dkb,
                                out, s);
}

fde_status fde_plan_set_tuning(fde_plan* p, int key, int value) {
  if (!p) return fail(FDE_ERR_ARG, "null plan");
  if (value < 0 || value > 1024) return fail(FDE_ERR_ARG, "tuning value out of range");
  switch (key) {
    case FDE_TUNE_APPLY_BPW: p->tune_bpw = value; return FDE_OK;
    case FDE_TUNE_Z_REGISTER:
      if (value > 1) return fail(FDE_ERR_ARG, "z-pass register FFT switch must be 0 or 1");
      p->tune_zreg = value;
      return FDE_OK;
    case FDE_TUNE_PLANE_KIND:
      if (value > 3) return fail(FDE_ERR_ARG, "plane pass kind must be 0..3");
      p->tune_plane = value;
      return FDE_OK;
    case FDE_TUNE_PLANE_ROWS:
      p->tune_rows = value;
      return FDE_OK;
    case FDE_TUNE_RR_SPLIT:
      p->tune_rr_split = value;
      return FDE_OK;
    case FDE_TUNE_STICK_GROUP:
      if ((value & (value - 1)) != 0) return fail(FDE_ERR_ARG, "sticks per workgroup must be 0 or a power of two");
      p->tune_sz = value;
      return FDE_OK;
    default: return fail(FDE_ERR_ARG, "unknown tuning key");
  }
}

}  // extern "C"
