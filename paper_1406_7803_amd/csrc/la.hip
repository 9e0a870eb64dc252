// Host entry points of the band-solver kernels: fde_subspace_rr(_batched),
// fde_precondition(_batched), fde_occupations.
#include <algorithm>
#include <mutex>
#include <vector>

#include "kernels_gemm.hpp"
#include "kernels_la.hpp"
#include "kernels_pw.hpp"
#include "kernels_mlp.hpp"
#include "kernels_rr.hpp"
#include "launch.hpp"

namespace fde {

// Per-problem scratch of the Rayleigh-Ritz solve, for m <= mcap.
size_t rr_problem_bytes(const fde_plan* p, int mcap, int nbcap) {
  const size_t mm = (size_t)mcap * mcap;
  size_t s = align256((size_t)kMaxChunks * 2 * mm * 16);  // Gram partials
  s += 5 * align256(mm * 16);                            // S, A, L, B, W
  s += align256((size_t)mcap * nbcap * 16);              // C (FP64)
  s += align256((size_t)mcap * nbcap * p->csize());      // C (plan precision)
  s += align256(4 * (size_t)mcap * sizeof(double) + 2 * (size_t)mcap * sizeof(int));
  return s;
}

template <typename T>
static void bind_scratch(fde_plan* p, int slot, Prob<T>& P) {
  const int mcap = 2 * p->max_nb;
  const size_t mm = (size_t)mcap * mcap;
  char* w = p->scratch + (size_t)slot * rr_problem_bytes(p, mcap, p->max_nb);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* r = w + off;
    off += align256(bytes);
    return r;
  };
  P.part = (cplx<double>*)take((size_t)kMaxChunks * 2 * mm * 16);
  P.S = (cplx<double>*)take(mm * 16);
  P.A = (cplx<double>*)take(mm * 16);
  P.L = (cplx<double>*)take(mm * 16);
  P.B = (cplx<double>*)take(mm * 16);
  P.W = (cplx<double>*)take(mm * 16);
  P.Cd = (cplx<double>*)take((size_t)mcap * p->max_nb * 16);
  P.Ct = take((size_t)mcap * p->max_nb * sizeof(cplx<T>));
  char* misc = take(4 * (size_t)mcap * sizeof(double) + 2 * (size_t)mcap * sizeof(int));
  P.theta = (double*)misc;
  P.order = (int*)(misc + (size_t)mcap * sizeof(double));
  P.masked = (int*)(misc + (size_t)mcap * (sizeof(double) + sizeof(int)));
}

static fde_status check_block(const fde_plan* p, const fde_block& b, bool rr) {
  if (b.ik < 0 || b.ik >= p->nk) return fail(FDE_ERR_ARG, "block k-point index out of range");
  if (!b.v || !b.hv || !b.eval) return fail(FDE_ERR_ARG, "block: null v, hv or eval");
  if (b.v == b.hv) return fail(FDE_ERR_ARG, "block: hv must not alias v");
  if (b.nb < 1 || b.nb > p->max_nb) return fail(FDE_ERR_SHAPE, "block: nb must be in [1, max_nb]");
  if (rr) {
    if (b.m < b.nb || b.m > 2 * p->max_nb) return fail(FDE_ERR_SHAPE, "block: need nb <= m <= 2 max_nb");
    if (!b.info) return fail(FDE_ERR_ARG, "block: null info");
  } else if (!b.rnorm || !b.t_active) {
    return fail(FDE_ERR_ARG, "block: null rnorm or t_active");
  }
  return FDE_OK;
}

template <typename T>
static Prob<T> make_prob(fde_plan* p, const fde_block& b) {
  Prob<T> P;
  const KTables& t = p->k[b.ik];
  P.v = (cplx<T>*)b.v;
  P.hv = (cplx<T>*)b.hv;
  P.sv = (cplx<T>*)b.sv;
  P.t = P.v + (size_t)b.nb * t.npw;
  P.active = b.active;
  P.act_out = b.t_active;
  P.eval = b.eval;
  P.rnorm = b.rnorm;
  P.info = b.info;
  P.millp = (const int*)t.d_millp;
  for (int i = 0; i < 3; ++i) P.kf[i] = t.kf[i];
  P.npw = t.npw;
  P.m = b.m;
  P.nb = b.nb;
  P.nchunk = std::min(kMaxChunks, (t.npw + 767) / 768);
  P.chunk = (t.npw + P.nchunk - 1) / P.nchunk;
  P.chunk = (P.chunk + 31) / 32 * 32;
  return P;
}

// The eigensolver of a batch with large m as phase launches (Cholesky, triangular solves,
// one pair of launches per Householder column, tridiagonal eigenproblem, back-transformation,
// C): most phases spread over many workgroups instead of one.
template <typename T>
static fde_status rr_split(ProbSet<T>& ps, int mmax, int nbmax, hipStream_t s) {
  constexpr int TT = KRRSolveTri<T>::kThreads;
  const size_t red = 64 * sizeof(double);
  FDE_TRY(launch<KRRCholInit<T>>(dim3((unsigned)(((size_t)mmax * mmax + 1023) / 1024), ps.n), kBlock, 0, s, ps));
  for (int j0 = 0; j0 < mmax; j0 += kCholB) {
    FDE_TRY(launch<KRRCholDiag<T>>(dim3(ps.n), 64, red, s, ps, j0));
    const int rows = mmax - j0 - kCholB;
    if (rows <= 0) continue;
    FDE_TRY(launch<KRRCholPanel<T>>(dim3((rows + 63) / 64, ps.n), 64, (size_t)kCholB * kCholB * sizeof(cplx<double>),
                                    s, ps, j0));
    const int ntile = (rows + 31) / 32;
    FDE_TRY(launch<KRRCholUpdate<T>>(dim3(ntile * (ntile + 1) / 2, ps.n), kBlock,
                                     2 * 32 * kCholB * sizeof(cplx<double>), s, ps, j0));
  }
  using S0 = KRRBigTrsm<T, 0>;
  const dim3 gstrip((mmax + S0::CB - 1) / S0::CB, ps.n), gcstrip((nbmax + S0::CB - 1) / S0::CB, ps.n);
  FDE_TRY((launch<KRRBigTrsm<T, 0>>(gstrip, S0::RB * S0::CB, S0::lds_bytes(mmax), s, ps)));
  FDE_TRY((launch<KRRBigTrsm<T, 1>>(gstrip, S0::RB * S0::CB, S0::lds_bytes(mmax), s, ps)));
  FDE_TRY(launch<KRRBigPrep<T>>(dim3(ps.n), kBlock, red, s, ps));
  // p_0, then one launch per column: the update and the next reflector and p
  FDE_TRY(launch<KRRBigHhP<T>>(dim3((mmax + kHhRows - 1) / kHhRows, ps.n), kHhRows * 16, 0, s, ps, 0));
  const size_t hlds = 32 * sizeof(double) + 2 * (size_t)mmax * sizeof(cplx<double>);
  for (int k = 0; k + 1 < mmax; ++k) {
    const dim3 g((unsigned)std::max(1, (mmax - k - 2 + kHhRows - 1) / kHhRows), ps.n);
    FDE_TRY(launch<KRRBigHh<T>>(g, kHhRows * 16, hlds, s, ps, k));
  }
  FDE_TRY((launch<KRRBigTri<T>, TT>(dim3(ps.n), TT, KRRSolveTriG<T>::lds_bytes(mmax), s, ps)));
  // the large clusters' vectors: at most nbmax per problem, four per workgroup
  FDE_TRY(launch<KRRBigInv<T>>(dim3((nbmax + KRRBigInv<T>::kVec - 1) / KRRBigInv<T>::kVec, ps.n), kBlock,
                               KRRBigInv<T>::lds_bytes(mmax), s, ps, mmax));
  FDE_TRY((launch<KRRBigOrth<T>, 1024>(dim3(ps.n), 1024,
                                       (32 + 2 * (size_t)KRRSolveTri<T>::kOrthBlock * mmax) * sizeof(double), s, ps)));
  FDE_TRY(launch<KRRBigBack<T>>(dim3((nbmax + 3) / 4, ps.n), kBlock, 0, s, ps));
  FDE_TRY((launch<KRRBigTrsm<T, 2>>(gcstrip, S0::RB * S0::CB, S0::lds_bytes(mmax), s, ps)));
  return FDE_OK;
}

template <typename T>
static fde_status rr_launch(fde_plan* p, ProbSet<T>& ps, hipStream_t s) {
  int mmax = 0, nbmax = 0, npwmax = 0;
  for (int i = 0; i < ps.n; ++i) {
    mmax = std::max(mmax, ps.p[i].m);
    nbmax = std::max(nbmax, ps.p[i].nb);
    npwmax = std::max(npwmax, ps.p[i].npw);
  }
  AhBSet<T> gs;
  gs.n = ps.n;
  bool gen = false;  // a generalised problem: S = V^H (S V), full tiles on the FP64 matrix cores
  for (int i = 0; i < ps.n; ++i) {
    const Prob<T>& P = ps.p[i];
    gs.p[i] = AhBProb<T>{P.v, P.sv ? P.sv : P.v, P.hv, P.m, P.m, P.npw, P.nchunk, P.chunk, P.part};
    gen = gen || P.sv != nullptr;
  }
  const int nt = (mmax + KAhB<T>::TI - 1) / KAhB<T>::TI;
  if (gen) {
    FDE_TRY(launch_ahb<T>(kMaxChunks, mmax, mmax, ps.n, gs, s));
  } else if constexpr (sizeof(T) == 4) {
    if (p->gemm == FDE_GEMM_BF16X3)
      FDE_TRY(launch<KAhBSplit<2>>(dim3(kMaxChunks, nt * nt, ps.n), kBlock, KAhBSplit<2>::lds_bytes(), s, gs));
    else if (p->gemm == FDE_GEMM_BF16X6)
      FDE_TRY(launch<KAhBSplit<3>>(dim3(kMaxChunks, nt * nt, ps.n), kBlock, KAhBSplit<3>::lds_bytes(), s, gs));
    else if (mmax <= 16 * kGramTiles)
      FDE_TRY((launch<KGram<T>, 512>(dim3(kMaxChunks, ps.n), 512, KGram<T>::lds_bytes(mmax), s, gs)));
    else
      FDE_TRY(launch_ahb<T>(kMaxChunks, mmax, mmax, ps.n, gs, s));
  } else {
    if (mmax <= 16 * kGramTiles)
      FDE_TRY((launch<KGram<T>, 512>(dim3(kMaxChunks, ps.n), 512, KGram<T>::lds_bytes(mmax), s, gs)));
    else
      FDE_TRY(launch_ahb<T>(kMaxChunks, mmax, mmax, ps.n, gs, s));
  }
  FDE_TRY(launch<KGramReduce<T>>(dim3((unsigned)((2 * (size_t)mmax * mmax + kLBlk - 1) / kLBlk), ps.n), kBlock, 0, s,
                                 ps));
  // LDS: fixed part + as much of the Jacobi matrices as fits in 160 KiB
  const size_t fixed = (KRRSolve<T>::lds_fixed(mmax) + 15) & ~(size_t)15;
  const size_t mbytes = (size_t)mmax * mmax * sizeof(cplx<double>);
  size_t mats = 0;
  if (fixed + 2 * mbytes <= kLdsMax) mats = 2 * mbytes;
  else if (fixed + mbytes <= kLdsMax) mats = mbytes;
  const int split_min = p->tune_rr_split > 0 ? p->tune_rr_split : kRRSplitMin;
  if (mmax >= split_min && mmax <= kRRTriMax && KRRSolveTriG<T>::lds_bytes(mmax) <= kLdsMax) {
    FDE_TRY(rr_split<T>(ps, mmax, nbmax, s));
  } else if (mmax <= kRRLdsMax && KRRSolveTri<T>::lds_bytes(mmax, nbmax) <= kLdsMax)
    FDE_TRY((launch<KRRSolveTri<T>, KRRSolveTri<T>::kThreads>(dim3(ps.n), KRRSolveTri<T>::kThreads,
                                                                KRRSolveTri<T>::lds_bytes(mmax, nbmax), s, ps)));
  else if (mmax > kRRLdsMax && mmax <= kRRTriMax && KRRSolveTriG<T>::lds_bytes(mmax) <= kLdsMax)
    FDE_TRY((launch<KRRSolveTriG<T>, KRRSolveTriG<T>::kThreads>(dim3(ps.n), KRRSolveTriG<T>::kThreads,
                                                                KRRSolveTriG<T>::lds_bytes(mmax), s, ps)));
  else if (mmax <= kRRLdsMax && KRRSolveLds<T>::lds_bytes(mmax) <= kLdsMax)
    FDE_TRY((launch<KRRSolveLds<T>, 1024>(dim3(ps.n), 1024, KRRSolveLds<T>::lds_bytes(mmax), s, ps)));
  else
    FDE_TRY((launch<KRRSolve<T>, 1024>(dim3(ps.n), 1024, fixed + mats, s, ps, mats)));
  const int nrot = gen ? 3 : 2;  // X = V C, HX = HV C (and SX = SV C)
  if (mmax <= 4 * kRotSteps && nbmax <= 64 && KRotateStream<T>::lds_bytes(mmax, nbmax) <= kLdsMax) {
    // streamed rotation: about eight workgroups of four wavefronts per CU over all problems
    const int groups = (npwmax + 15) / 16;
    const int gx = std::max(1, std::min((groups + 3) / 4, 2048 / (2 * ps.n)));
    return launch<KRotateStream<T>, 256, 3>(dim3(gx, nrot, ps.n), kBlock, KRotateStream<T>::lds_bytes(mmax, nbmax), s,
                                            ps, gx);
  }
  // matrix cores with C in chunks through LDS (up to 128 bands)
  if (nbmax <= 128)
    return launch<KRotateChunk<T>, 256>(dim3((npwmax + 63) / 64, nrot, ps.n), 256, KRotateChunk<T>::lds_bytes(nbmax), s,
                                        ps);
  // matrix cores with the X rows of 16 columns in LDS (up to 512 bands)
  // two column groups per workgroup where that still leaves two workgroups per CU
  if (nbmax <= 4 * kRotWideTiles * 16 && KRotateWide<T, 2>::lds_bytes(nbmax) <= kLdsMax / 2)
    return launch<KRotateWide<T, 2>, 256, 2>(dim3((npwmax + 31) / 32, nrot, ps.n), 256, KRotateWide<T, 2>::lds_bytes(nbmax),
                                          s, ps);
  if (nbmax <= 4 * kRotWideTiles * 16 && KRotateWide<T>::lds_bytes(nbmax) <= kLdsMax)
    return launch<KRotateWide<T>, 256>(dim3((npwmax + 15) / 16, nrot, ps.n), 256, KRotateWide<T>::lds_bytes(nbmax), s,
                                       ps);
  // in-place rotation: plane-wave chunk of all m rows (+ C when it fits) in LDS
  const size_t cs = sizeof(cplx<T>);
  int GC = 64;
  while (GC > 4 && (size_t)mmax * GC * cs > 96 * 1024) GC /= 2;
  const int c_in_lds = ((size_t)mmax * GC * cs + (size_t)mmax * nbmax * cs) <= kLdsMax ? 1 : 0;
  const size_t rl = (size_t)mmax * GC * cs + (c_in_lds ? (size_t)mmax * nbmax * cs : 0);
  FDE_TRY(launch<KRotate<T>>(dim3((npwmax + GC - 1) / GC, nrot, ps.n), kBlock, rl, s, ps, GC, c_in_lds));
  return FDE_OK;
}

template <typename T>
static fde_status rr_batched_t(fde_plan* p, int nblk, const fde_block* blk_in, double drop_tol, hipStream_t s) {
  // launches take the kernels of their largest block: blocks that fit the LDS solvers
  // (m <= kRRLdsMax) are batched apart from the larger ones, order kept within each kind
  std::vector<fde_block> sorted;
  sorted.reserve(nblk);
  for (int pass = 0; pass < 2; ++pass)
    for (int i = 0; i < nblk; ++i)
      if ((blk_in[i].m <= kRRLdsMax) == (pass == 0)) sorted.push_back(blk_in[i]);
  const fde_block* blk = sorted.data();
  const int nsmall = (int)std::count_if(blk_in, blk_in + nblk, [](const fde_block& b) { return b.m <= kRRLdsMax; });
  const int per = std::min(kMaxBatch, p->max_batch);
  for (int b0 = 0; b0 < nblk;) {
    ProbSet<T> ps;
    // a batch never mixes the two kinds
    const int kind_end = b0 < nsmall ? nsmall : nblk;
    ps.n = std::min(per, kind_end - b0);
    // the split products carry relative noise of about 2^-16 (BF16x3) or 2^-24 (BF16x6): a smaller
    // Cholesky pivot than ten times that is indistinguishable from a dependent column
    const double floor_tol = p->gemm == FDE_GEMM_BF16X3 ? 2e-4 : (p->gemm == FDE_GEMM_BF16X6 ? 1e-6 : 0.0);
    ps.drop_tol = drop_tol > floor_tol ? drop_tol : floor_tol;
    for (int i = 0; i < 3; ++i) ps.b[i] = p->b[i];
    for (int i = 0; i < ps.n; ++i) {
      ps.p[i] = make_prob<T>(p, blk[b0 + i]);
      bind_scratch<T>(p, i, ps.p[i]);
    }
    FDE_TRY(rr_launch<T>(p, ps, s));
    b0 += ps.n;
  }
  return FDE_OK;
}

template <typename T>
static fde_status precond_batched_t(fde_plan* p, int nblk, const fde_block* blk, const void* t_single,
                                    hipStream_t s) {
  // the chunked form keeps its partials in the per-problem Rayleigh-Ritz scratch slots
  const int per = t_single ? kMaxBatch : std::min(kMaxBatch, p->max_batch);
  for (int b0 = 0; b0 < nblk; b0 += per) {
    ProbSet<T> ps;
    ps.n = std::min(per, nblk - b0);
    ps.drop_tol = 0;
    for (int i = 0; i < 3; ++i) ps.b[i] = p->b[i];
    int nbmax = 0;
    for (int i = 0; i < ps.n; ++i) {
      ps.p[i] = make_prob<T>(p, blk[b0 + i]);
      if (t_single)
        ps.p[i].t = (cplx<T>*)t_single;
      else
        bind_scratch<T>(p, i, ps.p[i]);
      nbmax = std::max(nbmax, ps.p[i].nb);
    }
    if (t_single) {
      FDE_TRY(launch<KPrecond<T>>(dim3(nbmax, ps.n), kBlock, 17 * sizeof(double), s, ps));
    } else {
      const dim3 g(kPcChunks, nbmax, ps.n);
      FDE_TRY(launch<KPrecondA<T>>(g, kBlock, 17 * sizeof(double), s, ps));
      FDE_TRY(launch<KPrecondB<T>>(g, kBlock, 17 * sizeof(double), s, ps));
      FDE_TRY(launch<KPrecondC<T>>(g, kBlock, 0, s, ps));
    }
  }
  return FDE_OK;
}

template <typename T>
static fde_status precond_mlp_batched_t(fde_plan* p, int nblk, const fde_block* blk, const float* params,
                                        const double* vbar, hipStream_t s) {
  for (int b0 = 0; b0 < nblk; b0 += kMaxBatch) {
    ProbSet<T> ps;
    ps.n = std::min(kMaxBatch, nblk - b0);
    ps.drop_tol = 0;
    for (int i = 0; i < 3; ++i) ps.b[i] = p->b[i];
    int nbmax = 0;
    for (int i = 0; i < ps.n; ++i) {
      ps.p[i] = make_prob<T>(p, blk[b0 + i]);
      nbmax = std::max(nbmax, ps.p[i].nb);
    }
    for (int i = 0; i < ps.n; ++i)
      if (ps.p[i].sv) return fail(FDE_ERR_UNSUPPORTED, "the learned preconditioner takes standard problems (sv = NULL)");
    FDE_TRY(launch<KPrecondMlp<T>>(dim3(nbmax, ps.n), kBlock, KPrecondMlp<T>::lds_bytes, s, ps, params, vbar + b0));
  }
  return FDE_OK;
}

// samples per block of the loss/gradient pass: a multiple of 64, at most 1024 blocks
static int mlp_per_block(int n) { return 64 * std::max(1, (n + 64 * 1024 - 1) / (64 * 1024)); }

// ---------------------------------------------------------------------------
// Library-held scratch of fde_mlp_loss_grad_static: the per-block partial
// gradients live in a file-scope device array, one copy per GPU, for the life
// of the process. In host code `scratch` names a host-side stand-in, never the
// device memory: its device address is taken once per device with
// hipGetSymbolAddress and only that address is passed to kernels.
// ---------------------------------------------------------------------------
#ifdef FDE_EMULATE
alignas(256) static char scratch[FDE_MLP_STATIC_SCRATCH_BYTES];
static fde_status static_scratch(void** out) {
  *out = scratch;
  return FDE_OK;
}
#else
static __device__ __align__(256) char scratch[FDE_MLP_STATIC_SCRATCH_BYTES];
static fde_status static_scratch(void** out) {
  constexpr int kMaxDevices = 64;
  static void* addr[kMaxDevices] = {};
  static std::mutex mu;
  int dev = 0;
  FDE_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(FDE_ERR_DEVICE, "device index beyond the scratch table");
  std::lock_guard<std::mutex> g(mu);
  if (!addr[dev]) {
    void* a = nullptr;
    FDE_HIP(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
    if (!a) return fail(FDE_ERR_DEVICE, "no device address for the scratch array");
    addr[dev] = a;
  }
  *out = addr[dev];
  return FDE_OK;
}
#endif

}  // namespace fde

using namespace fde;


// ---------------------------------------------------------------------------
// Subsystem-specific augmentation (Appendix, non-local pseudopotentials): the
// projections P = beta^H psi in FP64, S psi = psi + beta (q P), and the atom
// charges of the augmentation density.
// ---------------------------------------------------------------------------
// P[o] = sum over the plane-wave chunks of part[chunk][o], o < nproj nb (fixed order)
struct KPReduce {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const cplx<double>* __restrict__ part, int nchunk, int nout,
                         cplx<double>* __restrict__ P) {
    for (int l = c.tid(); l < 256; l += c.nthr()) {
      const int o = c.bx() * 256 + l;
      if (o >= nout) break;
      double sx = 0.0, sy = 0.0;
      for (int k = 0; k < nchunk; ++k) {
        const cplx<double> v = part[(size_t)k * nout + o];
        sx += v.x;
        sy += v.y;
      }
      P[o] = mk<double>(sx, sy);
    }
  }
};

// dp[i][n] = sum_j q[i][j] P[j][n] (q real, [nproj][nproj]); grid ceil(nproj nb / 256)
template <typename T>
struct KQMul {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const double* __restrict__ q, const cplx<double>* __restrict__ P,
                         int nproj, int nb, cplx<T>* __restrict__ dp) {
    for (int l = c.tid(); l < 256; l += c.nthr()) {
      const int o = c.bx() * 256 + l;
      if (o >= nproj * nb) break;
      const int i = o / nb, n = o - i * nb;
      double sx = 0.0, sy = 0.0;
      for (int j = 0; j < nproj; ++j) {
        const double qij = q[(size_t)i * nproj + j];
        if (qij == 0.0) continue;
        const cplx<double> v = P[(size_t)j * nb + n];
        sx += qij * v.x;
        sy += qij * v.y;
      }
      dp[o] = mk<T>((T)sx, (T)sy);
    }
  }
};

// charges[atom_of[i]] += sum_n occw_n Re(conj(P_in) sum_j q_ij P_jn), projectors in order
// (one workgroup; t_i in LDS, then one thread adds them up in index order)
struct KAugCharges {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const double* __restrict__ q, const cplx<double>* __restrict__ P,
                         const double* __restrict__ occw, int nproj, int nb, const int* __restrict__ atom_of,
                         double* __restrict__ charges) {
    double* t = (double*)lds;
    for (int i = c.tid(); i < nproj; i += c.nthr()) {
      double acc = 0.0;
      for (int n = 0; n < nb; ++n) {
        double sx = 0.0, sy = 0.0;
        for (int j = 0; j < nproj; ++j) {
          const double qij = q[(size_t)i * nproj + j];
          if (qij == 0.0) continue;
          const cplx<double> v = P[(size_t)j * nb + n];
          sx += qij * v.x;
          sy += qij * v.y;
        }
        const cplx<double> pi = P[(size_t)i * nb + n];
        acc += occw[n] * (pi.x * sx + pi.y * sy);
      }
      t[i] = acc;
    }
    c.sync();
    if (c.tid() == 0)
      for (int i = 0; i < nproj; ++i) charges[atom_of[i]] += t[i];
  }
};

// P = beta^H psi in FP64 for one band chunk (scratch: chunk partials at off_part, P at off_p)
template <typename T>
static fde_status projections_fp64(fde_plan* p, int ik, int nbc, const cplx<T>* psi, int nproj, const cplx<T>* beta,
                                   cplx<double>* part, cplx<double>* P, hipStream_t s) {
  const KTables& t = p->k[ik];
  int chunk = kKbChunk;
  if (!(nproj <= 64 && nbc <= 64)) {
    const int tiles = ((nproj + 31) / 32) * ((nbc + 31) / 32);
    const int nc = std::max(1, std::min((t.npw + kKbChunk - 1) / kKbChunk, 2048 / tiles));
    chunk = std::max(kKbChunk, ((t.npw + nc - 1) / nc + 63) / 64 * 64);
  }
  const int nchunk = (t.npw + chunk - 1) / chunk;
  const AhBProb<T> prob{beta, psi, nullptr, nproj, nbc, t.npw, nchunk, chunk, part};
  if (nproj <= 64 && nbc <= 64) {
    FDE_TRY((launch<KAhBAll<T>, 512>(dim3(nchunk), 512, KAhBAll<T>::lds_bytes(nproj, nbc), s, prob)));
  } else {
    AhBSet<T> set;
    set.n = 1;
    set.p[0] = prob;
    FDE_TRY(launch_ahb<T>(nchunk, nproj, nbc, 1, set, s));
  }
  return launch<KPReduce>(dim3((nproj * nbc + 255) / 256), kBlock, 0, s, (const cplx<double>*)part, nchunk,
                          nproj * nbc, P);
}

// scratch of the augmentation calls: P (FP64) in the stick-buffer area, the chunk partials
// and dp where fde_apply_h keeps its own
template <typename T>
static fde_status aug_scratch(fde_plan* p, int nproj, cplx<double>** part, cplx<double>** P, cplx<T>** dp) {
  const size_t sb = align256((size_t)p->max_nb * p->N[2] * stick_stride(p->ncol_max) * p->csize());
  if ((size_t)nproj * p->max_nb * sizeof(cplx<double>) > sb)
    return fail(FDE_ERR_SHAPE, "too many projectors for the workspace's stick buffer");
  const size_t nchunk = (p->npw_max + kKbChunk - 1) / kKbChunk;
  *P = (cplx<double>*)p->scratch;
  *part = (cplx<double>*)(p->scratch + sb);
  *dp = (cplx<T>*)(p->scratch + sb + align256(nchunk * (size_t)p->max_nproj * p->max_nb * 16));
  return FDE_OK;
}

template <typename T>
static fde_status apply_s_t(fde_plan* p, int ik, int nb, const cplx<T>* psi, cplx<T>* spsi, int nproj,
                            const cplx<T>* beta, const double* q, hipStream_t s) {
  const KTables& t = p->k[ik];
  cplx<double>*part, *P;
  cplx<T>* dp;
  FDE_TRY(aug_scratch<T>(p, nproj, &part, &P, &dp));
  for (int b0 = 0; b0 < nb; b0 += p->max_nb) {
    const int nbc = std::min(p->max_nb, nb - b0);
    const cplx<T>* ps = psi + (size_t)b0 * t.npw;
    cplx<T>* ss = spsi + (size_t)b0 * t.npw;
    FDE_TRY(copy_d2d(ss, ps, (size_t)nbc * t.npw * sizeof(cplx<T>), s));
    if (nproj == 0) continue;
    FDE_TRY(projections_fp64<T>(p, ik, nbc, ps, nproj, beta, part, P, s));
    FDE_TRY(launch<KQMul<T>>(dim3((nproj * nbc + 255) / 256), kBlock, 0, s, q, (const cplx<double>*)P, nproj, nbc,
                             dp));
    if (nbc <= 4 * kKbAddTiles * 16)
      FDE_TRY(launch<KKbAddMfma<T>>(dim3((t.npw + 15) / 16), kBlock, 0, s, beta, (const cplx<T>*)dp, ss, t.npw, nproj,
                                    nbc));
    else
      FDE_TRY(launch<KKbAdd<T>>(dim3((t.npw + KKbAdd<T>::TG - 1) / KKbAdd<T>::TG), kBlock, KKbAdd<T>::lds_bytes(), s,
                                beta, (const cplx<T>*)dp, ss, t.npw, nproj, nbc));
  }
  return FDE_OK;
}

template <typename T>
static fde_status aug_charges_t(fde_plan* p, int ik, int nb, const cplx<T>* psi, const double* occw, int nproj,
                                const cplx<T>* beta, const double* q, const int* atom_of, double* charges,
                                hipStream_t s) {
  const KTables& t = p->k[ik];
  cplx<double>*part, *P;
  cplx<T>* dp;
  FDE_TRY(aug_scratch<T>(p, nproj, &part, &P, &dp));
  for (int b0 = 0; b0 < nb; b0 += p->max_nb) {
    const int nbc = std::min(p->max_nb, nb - b0);
    FDE_TRY(projections_fp64<T>(p, ik, nbc, psi + (size_t)b0 * t.npw, nproj, beta, part, P, s));
    FDE_TRY(launch<KAugCharges>(dim3(1), kBlock, (size_t)nproj * sizeof(double), s, q, (const cplx<double>*)P,
                                occw + b0, nproj, nbc, atom_of, charges));
  }
  return FDE_OK;
}

extern "C" {

fde_status fde_plan_set_gemm_mode(fde_plan* p, int mode) {
  if (!p) return fail(FDE_ERR_ARG, "null plan");
  if (mode != FDE_GEMM_FP64 && mode != FDE_GEMM_BF16X3 && mode != FDE_GEMM_BF16X6)
    return fail(FDE_ERR_ARG, "unknown GEMM mode");
  if (mode != FDE_GEMM_FP64 && p->prec != FDE_F32) return fail(FDE_ERR_UNSUPPORTED, "BF16-split products need an FP32 plan");
  p->gemm = mode;
  return FDE_OK;
}

fde_status fde_subspace_rr_batched(fde_plan* p, int nblk, const fde_block* blk, double drop_tol, hipStream_t s) {
  if (!p) return fail(FDE_ERR_ARG, "null plan");
  if (!p->ws) return fail(FDE_ERR_WORKSPACE, "no workspace attached (fde_plan_set_workspace)");
  if (nblk < 0 || (nblk > 0 && !blk)) return fail(FDE_ERR_ARG, "bad block list");
  if (!(drop_tol >= 0) || drop_tol >= 1) return fail(FDE_ERR_ARG, "drop_tol must be in [0, 1)");
  for (int i = 0; i < nblk; ++i) FDE_TRY(check_block(p, blk[i], true));
  if (p->prec == FDE_F64) return rr_batched_t<double>(p, nblk, blk, drop_tol, s);
  return rr_batched_t<float>(p, nblk, blk, drop_tol, s);
}

fde_status fde_subspace_rr(fde_plan* p, int ik, int m, int nb, void* v, void* hv, const uint8_t* active,
                           double drop_tol, double* eval, int* info, hipStream_t s) {
  FDE_TRY(check_plan(p, ik));
  if (!v || !hv || !eval || !info) return fail(FDE_ERR_ARG, "null argument");
  if (v == hv) return fail(FDE_ERR_ARG, "hv must not alias v");
  if (nb < 1 || m < nb) return fail(FDE_ERR_ARG, "need 1 <= nb <= m");
  if (nb > p->max_nb || m > 2 * p->max_nb) return fail(FDE_ERR_SHAPE, "m or nb exceeds the workspace (m <= 2 max_nb)");
  fde_block b = {};
  b.ik = ik;
  b.nb = nb;
  b.m = m;
  b.v = v;
  b.hv = hv;
  b.active = active;
  b.eval = eval;
  b.info = info;
  return fde_subspace_rr_batched(p, 1, &b, drop_tol, s);
}

fde_status fde_precondition_batched(fde_plan* p, int nblk, const fde_block* blk, hipStream_t s) {
  if (!p) return fail(FDE_ERR_ARG, "null plan");
  if (!p->ws) return fail(FDE_ERR_WORKSPACE, "no workspace attached (fde_plan_set_workspace)");
  if (nblk < 0 || (nblk > 0 && !blk)) return fail(FDE_ERR_ARG, "bad block list");
  for (int i = 0; i < nblk; ++i) FDE_TRY(check_block(p, blk[i], false));
  if (p->prec == FDE_F64) return precond_batched_t<double>(p, nblk, blk, nullptr, s);
  return precond_batched_t<float>(p, nblk, blk, nullptr, s);
}

fde_status fde_precondition(fde_plan* p, int ik, int nb, const void* x, const void* hx, const double* eval, void* t,
                            uint8_t* active, double* rnorm, hipStream_t s) {
  FDE_TRY(check_plan(p, ik));
  if (nb < 0) return fail(FDE_ERR_ARG, "negative size");
  if (nb == 0) return FDE_OK;
  if (!x || !hx || !eval || !t || !active || !rnorm) return fail(FDE_ERR_ARG, "null argument");
  if (nb > p->max_nb) return fail(FDE_ERR_SHAPE, "nb exceeds the workspace's max_nb");
  fde_block b = {};
  b.ik = ik;
  b.nb = nb;
  b.m = nb;
  b.v = (void*)x;
  b.hv = (void*)hx;
  b.eval = (double*)eval;
  b.rnorm = rnorm;
  b.t_active = active;
  if (p->prec == FDE_F64) return precond_batched_t<double>(p, 1, &b, t, s);
  return precond_batched_t<float>(p, 1, &b, t, s);
}

fde_status fde_occupations(int nk, int nb, const double* eval, const double* wk, double nelec, int mode, double sigma,
                           double* occw, double* mu, int* info, hipStream_t s) {
  if (nk < 1 || nb < 1) return fail(FDE_ERR_ARG, "nk and nb must be >= 1");
  if (!eval || !wk || !occw || !mu || !info) return fail(FDE_ERR_ARG, "null argument");
  if (mode != FDE_OCC_INTEGER && mode != FDE_OCC_FERMI_DIRAC && mode != FDE_OCC_METHFESSEL_PAXTON)
    return fail(FDE_ERR_ARG, "unknown occupation mode");
  if (mode != FDE_OCC_INTEGER && !(sigma > 0)) return fail(FDE_ERR_ARG, "sigma must be positive");
  if (!(nelec >= 0) || nelec > 2.0 * nb) return fail(FDE_ERR_ARG, "nelec must be in [0, 2 nb]");
  if (mode == FDE_OCC_INTEGER && nelec != 2.0 * std::floor(nelec / 2.0))
    return fail(FDE_ERR_ARG, "integer occupations need an even, whole electron count");
  return launch<KOccupations>(dim3(1), kBlock, 17 * sizeof(double), s, eval, wk, nk, nb, nelec, mode, sigma, occw, mu,
                              info);
}

fde_status fde_precondition_mlp_batched(fde_plan* p, int nblk, const fde_block* blk, const float* params,
                                        const double* vbar, hipStream_t s) {
  if (!p) return fail(FDE_ERR_ARG, "null plan");
  if (nblk < 0 || (nblk > 0 && (!blk || !params || !vbar))) return fail(FDE_ERR_ARG, "null argument");
  for (int i = 0; i < nblk; ++i) FDE_TRY(check_block(p, blk[i], false));
  if (p->prec == FDE_F64) return precond_mlp_batched_t<double>(p, nblk, blk, params, vbar, s);
  return precond_mlp_batched_t<float>(p, nblk, blk, params, vbar, s);
}

fde_status fde_mlp_forward(int n, const float* u, const float* params, float* y, hipStream_t s) {
  if (n < 0) return fail(FDE_ERR_ARG, "negative size");
  if (n == 0) return FDE_OK;
  if (!u || !params || !y) return fail(FDE_ERR_ARG, "null argument");
  return launch<KMlpForward>(dim3((unsigned)((n + 63) / 64)), kBlock, KMlpForward::lds_bytes, s, u, n, params, y);
}

fde_status fde_mlp_workspace_bytes(int n, size_t* bytes) {
  if (n < 1 || !bytes) return fail(FDE_ERR_ARG, "need n >= 1 and an output pointer");
  const int pb = mlp_per_block(n);
  const size_t nblk = (size_t)((n + pb - 1) / pb);
  *bytes = nblk * kMlpNPad * sizeof(float) + nblk * sizeof(double) + 256;
  return FDE_OK;
}

fde_status fde_mlp_loss_grad(int n, const float* samples, const float* params, float* grad, double* loss, void* ws,
                             size_t ws_bytes, hipStream_t s) {
  if (n < 1) return fail(FDE_ERR_ARG, "need at least one sample");
  if (!samples || !params || !grad || !loss || !ws) return fail(FDE_ERR_ARG, "null argument");
  size_t need = 0;
  FDE_TRY(fde_mlp_workspace_bytes(n, &need));
  if (ws_bytes < need) return fail(FDE_ERR_WORKSPACE, "workspace smaller than fde_mlp_workspace_bytes(n)");
  const int pb = mlp_per_block(n);
  const int nblk = (n + pb - 1) / pb;
  float* part = (float*)ws;
  double* lpart = (double*)((char*)ws + align256((size_t)nblk * kMlpNPad * sizeof(float)));  // inside `need`
  FDE_TRY(launch<KMlpLossGrad>(dim3(nblk), kBlock, KMlpLossGrad::lds_bytes, s, samples, n, pb, params, part, lpart));
  return launch<KMlpReduce>(dim3((kMlpNPad + 255) / 256), kBlock, 0, s, (const float*)part, (const double*)lpart, nblk,
                            grad, loss);
}

fde_status fde_mlp_loss_grad_static(int n, const float* samples, const float* params, float* grad, double* loss,
                                    hipStream_t s) {
  if (n < 1) return fail(FDE_ERR_ARG, "need at least one sample");
  if (n > FDE_MLP_STATIC_MAX_N) return fail(FDE_ERR_SHAPE, "n exceeds FDE_MLP_STATIC_MAX_N");
  if (!samples || !params || !grad || !loss) return fail(FDE_ERR_ARG, "null argument");
  size_t need = 0;
  FDE_TRY(fde_mlp_workspace_bytes(n, &need));
  if (need > (size_t)FDE_MLP_STATIC_SCRATCH_BYTES)
    return fail(FDE_ERR_SHAPE, "n needs more scratch than FDE_MLP_STATIC_SCRATCH_BYTES");
  void* ws = nullptr;
  FDE_TRY(static_scratch(&ws));
  // every block writes its whole partial row before the reduction reads it:
  // nothing left by an earlier call is read
  const int pb = mlp_per_block(n);
  const int nblk = (n + pb - 1) / pb;
  float* part = (float*)ws;
  double* lpart = (double*)((char*)ws + align256((size_t)nblk * kMlpNPad * sizeof(float)));
  FDE_TRY(launch<KMlpLossGrad>(dim3(nblk), kBlock, KMlpLossGrad::lds_bytes, s, samples, n, pb, params, part, lpart));
  return launch<KMlpReduce>(dim3((kMlpNPad + 255) / 256), kBlock, 0, s, (const float*)part, (const double*)lpart, nblk,
                            grad, loss);
}

fde_status fde_mlp_adam(const float* grad, float* params, float* m, float* v, int t, float lr, float beta1, float beta2,
                        float eps, hipStream_t s) {
  if (!grad || !params || !m || !v) return fail(FDE_ERR_ARG, "null argument");
  if (t < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(FDE_ERR_ARG, "bad Adam hyper-parameters");
  return launch<KMlpAdam>(dim3((kMlpNParam + 255) / 256), kBlock, 0, s, grad, params, m, v, t, lr, beta1, beta2, eps);
}


fde_status fde_apply_s(fde_plan* p, int ik, int nb, const void* psi, void* spsi, int nproj, const void* beta,
                       const double* q, hipStream_t s) {
  FDE_TRY(check_plan(p, ik));
  if (nb < 0 || nproj < 0) return fail(FDE_ERR_ARG, "negative size");
  if (nb == 0) return FDE_OK;
  if (!psi || !spsi) return fail(FDE_ERR_ARG, "null array");
  if (psi == spsi) return fail(FDE_ERR_ARG, "spsi must not alias psi");
  if (nproj > 0 && (!beta || !q)) return fail(FDE_ERR_ARG, "nproj > 0 needs beta and q");
  if (nproj > p->max_nproj) return fail(FDE_ERR_SHAPE, "nproj exceeds the workspace's max_nproj");
  if (p->prec == FDE_F64)
    return apply_s_t<double>(p, ik, nb, (const cplx<double>*)psi, (cplx<double>*)spsi, nproj,
                             (const cplx<double>*)beta, q, s);
  return apply_s_t<float>(p, ik, nb, (const cplx<float>*)psi, (cplx<float>*)spsi, nproj, (const cplx<float>*)beta, q,
                          s);
}

fde_status fde_aug_charges(fde_plan* p, int ik, int nb, const void* psi, const double* occw, int nproj,
                           const void* beta, const double* q, const int* atom_of, double* charges, hipStream_t s) {
  FDE_TRY(check_plan(p, ik));
  if (nb < 0 || nproj < 0) return fail(FDE_ERR_ARG, "negative size");
  if (nb == 0 || nproj == 0) return FDE_OK;
  if (!psi || !occw || !beta || !q || !atom_of || !charges) return fail(FDE_ERR_ARG, "null array");
  if (nproj > p->max_nproj) return fail(FDE_ERR_SHAPE, "nproj exceeds the workspace's max_nproj");
  if ((size_t)nproj * sizeof(double) > kLdsMax) return fail(FDE_ERR_SHAPE, "too many projectors");
  if (p->prec == FDE_F64)
    return aug_charges_t<double>(p, ik, nb, (const cplx<double>*)psi, occw, nproj, (const cplx<double>*)beta, q,
                                 atom_of, charges, s);
  return aug_charges_t<float>(p, ik, nb, (const cplx<float>*)psi, occw, nproj, (const cplx<float>*)beta, q, atom_of,
                              charges, s);
}

}  // extern "C"
