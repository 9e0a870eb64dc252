// Plane-wave plan: G-spheres, z-stick maps, twiddle tables, workspace layout.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"
#include "launch.hpp"

namespace fde {

static thread_local std::string g_last_error = "no error";

void set_error(const std::string& msg) { g_last_error = msg; }

fde_status fail(fde_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

fde_status hip_check(hipError_t e, const char* what) {
  return fail(FDE_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

hipError_t allow_lds(const void* kernel, size_t bytes) {
#ifdef FDE_EMULATE
  (void)kernel;
  (void)bytes;
  return hipSuccess;
#else
  if (bytes <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
#endif
}

fde_status check_plan(const fde_plan* p, int ik) {
  if (!p) return fail(FDE_ERR_ARG, "null plan");
  if (ik < 0 || ik >= p->nk) return fail(FDE_ERR_ARG, "k-point index out of range");
  if (!p->ws) return fail(FDE_ERR_WORKSPACE, "no workspace attached (fde_plan_set_workspace)");
  return FDE_OK;
}

// Build S_k exactly as documented: q_i = (m_i + kf_i) * b_i,
// 0.5*(q1*q1 + q2*q2 + q3*q3) <= E_cut, lexicographic on (m1, m2, m3).
static fde_status build_k(fde_plan* p, const double kf[3], KTables& t) {
  const double gmax = std::sqrt(2.0 * p->ecut);
  int lim[3];
  for (int i = 0; i < 3; ++i) lim[i] = (int)std::ceil(gmax / p->b[i] + std::fabs(kf[i])) + 1;
  for (int i = 0; i < 3; ++i) t.kf[i] = kf[i];
  t.mill.clear();
  for (int m1 = -lim[0]; m1 <= lim[0]; ++m1) {
    const double q1 = (m1 + kf[0]) * p->b[0];
    for (int m2 = -lim[1]; m2 <= lim[1]; ++m2) {
      const double q2 = (m2 + kf[1]) * p->b[1];
      for (int m3 = -lim[2]; m3 <= lim[2]; ++m3) {
        const double q3 = (m3 + kf[2]) * p->b[2];
        if (0.5 * (q1 * q1 + q2 * q2 + q3 * q3) <= p->ecut) {
          t.mill.push_back(m1);
          t.mill.push_back(m2);
          t.mill.push_back(m3);
        }
      }
    }
  }
  t.npw = (int)(t.mill.size() / 3);
  if (t.npw == 0) return fail(FDE_ERR_ARG, "empty plane-wave sphere");
  for (int g = 0; g < t.npw; ++g)
    for (int i = 0; i < 3; ++i)
      if (2 * std::abs(t.mill[3 * g + i]) >= p->N[i]) return fail(FDE_ERR_SHAPE, "sphere does not fit the grid");
  // sticks
  t.sticks.clear();
  t.xlist.clear();
  t.millp.resize(t.npw);
  std::vector<int> xa_of(p->N[0], -1);
  int g = 0;
  while (g < t.npw) {
    const int m1 = t.mill[3 * g], m2 = t.mill[3 * g + 1];
    int e = g;
    while (e < t.npw && t.mill[3 * e] == m1 && t.mill[3 * e + 1] == m2) ++e;
    const int ix = imod(m1, p->N[0]), iy = imod(m2, p->N[1]);
    if (xa_of[ix] < 0) {
      xa_of[ix] = (int)t.xlist.size();
      t.xlist.push_back(ix);
    }
    int4 s;
    s.x = g;
    s.y = e - g;
    s.z = t.mill[3 * g + 2];
    s.w = xa_of[ix] | (iy << 16);
    t.sticks.push_back(s);
    g = e;
  }
  for (int q = 0; q < t.npw; ++q)
    t.millp[q] = (t.mill[3 * q] + 512) | ((t.mill[3 * q + 1] + 512) << 10) | ((t.mill[3 * q + 2] + 512) << 20);
  t.ncol = (int)t.sticks.size();
  t.nxa = (int)t.xlist.size();
  t.mlo = t.mill[0];
  t.xrange = true;
  for (int xa = 0; xa < t.nxa; ++xa)
    if (t.xlist[xa] != imod(t.mlo + xa, p->N[0])) t.xrange = false;
  return FDE_OK;
}

size_t scratch_apply(const fde_plan* p, int max_nb, int max_nproj) {
  size_t s = align256((size_t)max_nb * p->N[2] * stick_stride(p->ncol_max) * p->csize());
  const size_t nchunk = (p->npw_max + kKbChunk - 1) / kKbChunk;
  s += align256(nchunk * (size_t)max_nproj * max_nb * 16);
  s += align256((size_t)max_nproj * max_nb * p->csize());
  return s;
}

size_t scratch_density(const fde_plan* p, int max_nb) {
  size_t s = align256((size_t)max_nb * p->N[2] * stick_stride(p->ncol_max) * p->csize());
  s += align256((size_t)kRhoGroups * p->npts() * p->rsize());
  return s;
}

size_t scratch_embed(const fde_plan* p) {
  const size_t n = p->npts();
  size_t s = 4 * align256(n * p->csize());       // XG and three work grids
  s += 4 * align256(n * p->rsize());             // rho, V_H, V~xc[rho], V~kin[rho]
  s += align256(8192 * sizeof(double));          // reduction partials
  s += align256(64 * sizeof(double));
  return s;
}

size_t scratch_subspace(const fde_plan* p, int max_nb, int max_batch) {
  return (size_t)max_batch * rr_problem_bytes(p, 2 * max_nb, max_nb);
}

}  // namespace fde

using namespace fde;

extern "C" {

const char* fde_last_error(void) { return g_last_error.c_str(); }

fde_status fde_plan_create(const double L[3], const int grid[3], double ecut_ha, int nk, const double* kfrac,
                           int prec, fde_plan** out) {
  if (!L || !grid || !out || (nk > 0 && !kfrac)) return fail(FDE_ERR_ARG, "null argument");
  *out = nullptr;
  if (nk <= 0) return fail(FDE_ERR_ARG, "nk must be positive");
  if (prec != FDE_F64 && prec != FDE_F32) return fail(FDE_ERR_ARG, "prec must be FDE_F64 or FDE_F32");
  if (!(ecut_ha > 0)) return fail(FDE_ERR_ARG, "ecut must be positive");
  fde_plan* p = new fde_plan();
  p->prec = prec;
  p->ecut = ecut_ha;
  p->nk = nk;
  for (int i = 0; i < 3; ++i) {
    if (!(L[i] > 0)) { delete p; return fail(FDE_ERR_ARG, "cell lengths must be positive"); }
    p->L[i] = L[i];
    p->b[i] = 2.0 * M_PI / L[i];
    p->N[i] = grid[i];
    if (grid[i] < 2 || grid[i] > 512) { delete p; return fail(FDE_ERR_UNSUPPORTED, "grid length must be in [2, 512]"); }
    p->rad[i] = make_radix(grid[i]);
    if (p->rad[i].nst < 0) { delete p; return fail(FDE_ERR_UNSUPPORTED, "grid length must be a product of 2, 3, 5"); }
    const double need = 4.0 * std::sqrt(2.0 * ecut_ha) / p->b[i];
    if (!(grid[i] > need)) {
      char buf[160];
      std::snprintf(buf, sizeof buf, "grid %d too small for E_cut %.6g on axis %d (needs > %.3f)", grid[i], ecut_ha, i, need);
      delete p;
      return fail(FDE_ERR_SHAPE, buf);
    }
  }
  p->omega = L[0] * L[1] * L[2];
  p->k.resize(nk);
  for (int ik = 0; ik < nk; ++ik) {
    fde_status st = build_k(p, kfrac + 3 * ik, p->k[ik]);
    if (st != FDE_OK) { delete p; return st; }
    p->npw_max = std::max(p->npw_max, p->k[ik].npw);
    p->ncol_max = std::max(p->ncol_max, p->k[ik].ncol);
    p->nxa_max = std::max(p->nxa_max, p->k[ik].nxa);
  }
  *out = p;
  return FDE_OK;
}

void fde_plan_destroy(fde_plan* plan) { delete plan; }

fde_status fde_plan_info(const fde_plan* p, int ik, int* npw, int* ncol) {
  if (!p) return fail(FDE_ERR_ARG, "null plan");
  if (ik < 0 || ik >= p->nk) return fail(FDE_ERR_ARG, "k-point index out of range");
  if (npw) *npw = p->k[ik].npw;
  if (ncol) *ncol = p->k[ik].ncol;
  return FDE_OK;
}

fde_status fde_plan_miller(const fde_plan* p, int ik, int32_t* mill) {
  if (!p || !mill) return fail(FDE_ERR_ARG, "null argument");
  if (ik < 0 || ik >= p->nk) return fail(FDE_ERR_ARG, "k-point index out of range");
  std::memcpy(mill, p->k[ik].mill.data(), p->k[ik].mill.size() * sizeof(int32_t));
  return FDE_OK;
}

static size_t tables_bytes(const fde_plan* p) {
  size_t s = 0;
  for (const auto& t : p->k) {
    s += align256(t.ncol * sizeof(int4));
    s += align256(t.nxa * sizeof(int));
    s += align256(t.npw * sizeof(int));
  }
  for (int a = 0; a < 3; ++a) s += align256(p->N[a] * p->csize());
  return s;
}

fde_status fde_plan_workspace_bytes(const fde_plan* p, int max_nb, int max_nproj, int max_batch, size_t* bytes) {
  if (!p || !bytes) return fail(FDE_ERR_ARG, "null argument");
  if (max_nb < 1 || max_nproj < 0) return fail(FDE_ERR_ARG, "max_nb must be >= 1 and max_nproj >= 0");
  if (max_batch < 1 || max_batch > 16) return fail(FDE_ERR_ARG, "max_batch must be in [1, 16]");
  size_t s = scratch_apply(p, max_nb, max_nproj);
  s = std::max(s, scratch_density(p, max_nb));
  s = std::max(s, scratch_embed(p));
  s = std::max(s, scratch_subspace(p, max_nb, max_batch));
  *bytes = tables_bytes(p) + s;
  return FDE_OK;
}

fde_status fde_plan_set_workspace(fde_plan* p, void* d_ws, size_t bytes, int max_nb, int max_nproj, int max_batch) {
  if (!p || !d_ws) return fail(FDE_ERR_ARG, "null argument");
  if (((uintptr_t)d_ws) & 255) return fail(FDE_ERR_ARG, "workspace must be 256-byte aligned");
  size_t need = 0;
  fde_status st = fde_plan_workspace_bytes(p, max_nb, max_nproj, max_batch, &need);
  if (st != FDE_OK) return st;
  if (bytes < need) return fail(FDE_ERR_WORKSPACE, "workspace too small");
  char* w = (char*)d_ws;
  size_t off = 0;
  for (auto& t : p->k) {
    t.d_sticks = (int4*)(w + off);
    FDE_TRY(copy_h2d_sync(t.d_sticks, t.sticks.data(), t.ncol * sizeof(int4)));
    off += align256(t.ncol * sizeof(int4));
    t.d_xlist = (int*)(w + off);
    FDE_TRY(copy_h2d_sync(t.d_xlist, t.xlist.data(), t.nxa * sizeof(int)));
    off += align256(t.nxa * sizeof(int));
    t.d_millp = (int*)(w + off);
    FDE_TRY(copy_h2d_sync(t.d_millp, t.millp.data(), t.npw * sizeof(int)));
    off += align256(t.npw * sizeof(int));
  }
  for (int a = 0; a < 3; ++a) {
    const int n = p->N[a];
    p->d_tw[a] = w + off;
    if (p->prec == FDE_F64) {
      std::vector<double> tw(2 * n);
      for (int m = 0; m < n; ++m) {
        const double ang = 2.0 * M_PI * (double)m / (double)n;
        tw[2 * m] = std::cos(ang);
        tw[2 * m + 1] = -std::sin(ang);
      }
      FDE_TRY(copy_h2d_sync(p->d_tw[a], tw.data(), tw.size() * sizeof(double)));
    } else {
      std::vector<float> tw(2 * n);
      for (int m = 0; m < n; ++m) {
        const double ang = 2.0 * M_PI * (double)m / (double)n;
        tw[2 * m] = (float)std::cos(ang);
        tw[2 * m + 1] = (float)-std::sin(ang);
      }
      FDE_TRY(copy_h2d_sync(p->d_tw[a], tw.data(), tw.size() * sizeof(float)));
    }
    off += align256(n * p->csize());
  }
  p->table_bytes = off;
  p->ws = w;
  p->ws_bytes = bytes;
  p->scratch = w + off;
  p->scratch_bytes = bytes - off;
  p->max_nb = max_nb;
  p->max_nproj = max_nproj;
  p->max_batch = max_batch;
  return FDE_OK;
}

}  // extern "C"
