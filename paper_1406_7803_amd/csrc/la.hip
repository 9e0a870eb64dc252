// Host entry points of the band-solver kernels: fde_subspace_rr,
// fde_precondition, fde_occupations.
#include <algorithm>

#include "kernels_la.hpp"
#include "launch.hpp"

namespace fde {

template <typename T>
static fde_status rr_t(fde_plan* p, int ik, int m, int nb, cplx<T>* v, cplx<T>* hv, const uint8_t* active,
                       double drop_tol, double* eval, int* info, hipStream_t s) {
  const KTables& t = p->k[ik];
  const int mcap = 2 * p->max_nb;
  const size_t mm = (size_t)mcap * mcap;
  char* w = p->scratch;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* r = w + off;
    off += align256(bytes);
    return r;
  };
  RRArgs a;
  a.S = (cplx<double>*)take(mm * 16);
  a.A = (cplx<double>*)take(mm * 16);
  a.L = (cplx<double>*)take(mm * 16);
  a.B = (cplx<double>*)take(mm * 16);
  a.W = (cplx<double>*)take(mm * 16);
  a.Cd = (cplx<double>*)take((size_t)mcap * p->max_nb * 16);
  a.Ct = take((size_t)mcap * p->max_nb * p->csize());
  cplx<T>* xs = (cplx<T>*)take((size_t)p->max_nb * p->npw_max * sizeof(cplx<T>));
  cplx<T>* hxs = (cplx<T>*)take((size_t)p->max_nb * p->npw_max * sizeof(cplx<T>));
  const int nchunk = (t.npw + KGram<T>::CH - 1) / KGram<T>::CH;
  const int nchunk_cap = (p->npw_max + 2047) / 2048;
  cplx<double>* part = (cplx<double>*)take((size_t)nchunk_cap * mm * 16 * 2);
  char* misc = take(4 * (size_t)mcap * sizeof(double) + mcap * sizeof(int));
  a.theta = (double*)misc;
  a.order = (int*)(misc + (size_t)mcap * sizeof(double));
  a.masked = (int*)(misc + (size_t)mcap * (sizeof(double) + sizeof(int)));
  a.active = active;
  a.m = m;
  a.nb = nb;
  a.drop_tol = drop_tol;
  a.eval = eval;
  a.ct_double = (sizeof(T) == 8);
  a.info = info;
  const int ti = KGram<T>::TI;
  FDE_TRY(launch<KGram<T>>(dim3(nchunk, (m + ti - 1) / ti, (m + ti - 1) / ti), kBlock, KGram<T>::lds_bytes(), s,
                           (const cplx<T>*)v, (const cplx<T>*)hv, t.npw, m, part));
  FDE_TRY(launch<KGramReduce>(dim3((unsigned)((2 * (size_t)m * m + kLBlk - 1) / kLBlk)), kBlock, 0, s,
                              (const cplx<double>*)part, nchunk, m, a.S, a.A));
  FDE_TRY((launch<KRRSolve, 1024>(dim3(1), 1024, KRRSolve::lds_bytes(m), s, a)));
  const dim3 rg((t.npw + kLBlk - 1) / kLBlk, (nb + KRotate<T>::NT - 1) / KRotate<T>::NT);
  FDE_TRY(launch<KRotate<T>>(rg, kBlock, KRotate<T>::lds_bytes(), s, (const cplx<T>*)v, (const cplx<T>*)a.Ct, xs,
                             t.npw, m, nb));
  FDE_TRY(launch<KRotate<T>>(rg, kBlock, KRotate<T>::lds_bytes(), s, (const cplx<T>*)hv, (const cplx<T>*)a.Ct, hxs,
                             t.npw, m, nb));
  FDE_TRY(copy_d2d(v, xs, (size_t)nb * t.npw * sizeof(cplx<T>), s));
  FDE_TRY(copy_d2d(hv, hxs, (size_t)nb * t.npw * sizeof(cplx<T>), s));
  return FDE_OK;
}

}  // namespace fde

using namespace fde;

extern "C" {

fde_status fde_subspace_rr(fde_plan* p, int ik, int m, int nb, void* v, void* hv, const uint8_t* active,
                           double drop_tol, double* eval, int* info, hipStream_t s) {
  FDE_TRY(check_plan(p, ik));
  if (!v || !hv || !eval || !info) return fail(FDE_ERR_ARG, "null argument");
  if (v == hv) return fail(FDE_ERR_ARG, "hv must not alias v");
  if (nb < 1 || m < nb) return fail(FDE_ERR_ARG, "need 1 <= nb <= m");
  if (nb > p->max_nb || m > 2 * p->max_nb) return fail(FDE_ERR_SHAPE, "m or nb exceeds the workspace (m <= 2 max_nb)");
  if (!(drop_tol >= 0) || drop_tol >= 1) return fail(FDE_ERR_ARG, "drop_tol must be in [0, 1)");
  if (p->prec == FDE_F64)
    return rr_t<double>(p, ik, m, nb, (cplx<double>*)v, (cplx<double>*)hv, active, drop_tol, eval, info, s);
  return rr_t<float>(p, ik, m, nb, (cplx<float>*)v, (cplx<float>*)hv, active, drop_tol, eval, info, s);
}

fde_status fde_precondition(fde_plan* p, int ik, int nb, const void* x, const void* hx, const double* eval, void* t,
                            uint8_t* active, double* rnorm, hipStream_t s) {
  FDE_TRY(check_plan(p, ik));
  if (nb < 0) return fail(FDE_ERR_ARG, "negative size");
  if (nb == 0) return FDE_OK;
  if (!x || !hx || !eval || !t || !active || !rnorm) return fail(FDE_ERR_ARG, "null argument");
  const KTables& k = p->k[ik];
  const size_t red = 17 * sizeof(double);
  if (p->prec == FDE_F64)
    return launch<KPrecond<double>>(dim3(nb), kBlock, red, s, (const cplx<double>*)x, (const cplx<double>*)hx, eval,
                                    (cplx<double>*)t, active, rnorm, (const int*)k.d_millp, k.npw, k.kf[0], k.kf[1],
                                    k.kf[2], p->b[0], p->b[1], p->b[2]);
  return launch<KPrecond<float>>(dim3(nb), kBlock, red, s, (const cplx<float>*)x, (const cplx<float>*)hx, eval,
                                 (cplx<float>*)t, active, rnorm, (const int*)k.d_millp, k.npw, k.kf[0], k.kf[1],
                                 k.kf[2], p->b[0], p->b[1], p->b[2]);
}

fde_status fde_occupations(int nk, int nb, const double* eval, const double* wk, double nelec, int mode, double sigma,
                           double* occw, double* mu, int* info, hipStream_t s) {
  if (nk < 1 || nb < 1) return fail(FDE_ERR_ARG, "nk and nb must be >= 1");
  if (!eval || !wk || !occw || !mu || !info) return fail(FDE_ERR_ARG, "null argument");
  if (mode != FDE_OCC_INTEGER && mode != FDE_OCC_FERMI_DIRAC) return fail(FDE_ERR_ARG, "unknown occupation mode");
  if (mode == FDE_OCC_FERMI_DIRAC && !(sigma > 0)) return fail(FDE_ERR_ARG, "sigma must be positive");
  if (!(nelec >= 0) || nelec > 2.0 * nb) return fail(FDE_ERR_ARG, "nelec must be in [0, 2 nb]");
  return launch<KOccupations>(dim3(1), kBlock, 17 * sizeof(double), s, eval, wk, nk, nb, nelec, mode, sigma, occw, mu,
                              info);
}

}  // extern "C"
