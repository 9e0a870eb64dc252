// Internal plan structure and helpers shared by the library's translation units.
#pragma once

#include <string>
#include <vector>

#include "../../include/fde.h"
#include "common.hpp"

namespace fde {

// Per-k device table entry of one z-stick (a column (m1, m2) of S_k):
//   x = offset of its first plane wave in band order, y = count,
//   z = m3 of the first plane wave, w = xa | (iy << 16) where xa indexes the
//   plan's list of active x-columns and iy is the y grid index.
struct KTables {
  double kf[3];
  int npw = 0, ncol = 0, nxa = 0;
  int mlo = 0;          // smallest m1 of the sphere
  bool xrange = false;  // active x-columns are exactly m1 in [mlo, mlo + nxa), xa = m1 - mlo
  std::vector<int32_t> mill;   // host [npw][3]
  std::vector<int4> sticks;    // host copy of the device table
  std::vector<int> xlist;      // host: x grid index of each active column
  std::vector<int> millp;      // host: packed Miller (m1+512) | (m2+512)<<10 | (m3+512)<<20

  // device pointers into the workspace
  int4* d_sticks = nullptr;
  int* d_xlist = nullptr;
  int* d_millp = nullptr;
};

struct Scratch {
  size_t bytes = 0;
};

}  // namespace fde

struct fde_plan {
  double L[3], b[3], omega, ecut;
  int N[3];
  int prec;
  int nk;
  std::vector<fde::KTables> k;
  int npw_max = 0, ncol_max = 0, nxa_max = 0;
  fde::Radix rad[3];
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  int max_nb = 0, max_nproj = 0, max_batch = 1;
  int gemm = 0;  // FDE_GEMM_* of the subspace products
  int tune_bpw = 0;  // bands per plane-pass workgroup of fde_apply_h (0: automatic)
  int tune_sz = 0;   // z-sticks per z-pass workgroup, power of two (0: automatic, at most 16)
  int tune_zreg = 0; // z-passes: 0 four-step register FFT where specialised, 1 LDS passes always
  int tune_plane = 0; // plane pass: 0 automatic, 1 whole-line register, 2 LDS Stockham, 3 two-factor LDS
  int tune_rows = 0;  // rows per batch of the two-factor plane pass (0: automatic)
  int tune_rr_split = 0;  // smallest m of the split Rayleigh-Ritz eigensolver (0: automatic)
  void* d_tw[3] = {nullptr, nullptr, nullptr};  // twiddles exp(-2 pi i m/N_a), plan precision
  char* scratch = nullptr;
  size_t scratch_bytes = 0;
  size_t table_bytes = 0;

  size_t npts() const { return (size_t)N[0] * N[1] * N[2]; }
  size_t csize() const { return prec == FDE_F64 ? 16 : 8; }
  size_t rsize() const { return prec == FDE_F64 ? 8 : 4; }
};

namespace fde {

void set_error(const std::string& msg);
fde_status fail(fde_status code, const std::string& msg);
fde_status hip_check(hipError_t e, const char* what);

#define FDE_HIP(call)                                     \
  do {                                                    \
    hipError_t _e = (call);                               \
    if (_e != hipSuccess) return ::fde::hip_check(_e, #call); \
  } while (0)

// Scratch layout helpers (byte offsets rounded to 256).
inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

size_t scratch_apply(const fde_plan* p, int max_nb, int max_nproj);
size_t scratch_density(const fde_plan* p, int max_nb);
size_t scratch_embed(const fde_plan* p);
size_t scratch_subspace(const fde_plan* p, int max_nb, int max_batch);
size_t rr_problem_bytes(const fde_plan* p, int mcap, int nbcap);

fde_status check_plan(const fde_plan* p, int ik);

// Dynamic LDS above the default 64 KiB needs an explicit opt-in per kernel.
hipError_t allow_lds(const void* kernel, size_t bytes);

constexpr int kBlock = 256;
// plane waves per partial-sum chunk of the projector products beta^H psi
constexpr int kKbChunk = 128;
// band groups of the density plane pass (partial density planes, summed in a fixed order)
constexpr int kRhoGroups = 8;
constexpr size_t kLdsMax = 160 * 1024;

}  // namespace fde
