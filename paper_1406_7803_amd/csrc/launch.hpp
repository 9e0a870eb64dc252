// Kernel launch and memory helpers.
//
// Every kernel is a `Body` struct with a static `run(ctx, lds, args...)`
// template. The device build wraps it in one generic __global__ entry; the
// host-emulation build (FDE_EMULATE, used only by the CPU test suite to check
// indexing and arithmetic without a GPU) runs the same body serially for every
// block with a one-thread context.
#pragma once

#include <cstring>
#include <vector>

#include "internal.hpp"

namespace fde {

#ifdef FDE_EMULATE

template <class Body, int BS = 256, int MINW = 1, class... Args>
inline fde_status launch(dim3 grid, int /*block*/, size_t lds, hipStream_t, Args... args) {
  std::vector<double> buf(lds / sizeof(double) + 2);
  for (unsigned z = 0; z < grid.z; ++z)
    for (unsigned y = 0; y < grid.y; ++y)
      for (unsigned x = 0; x < grid.x; ++x) {
        HostCtx c;
        c.x = (int)x;
        c.y = (int)y;
        c.z = (int)z;
        Body::run(c, reinterpret_cast<char*>(buf.data()), args...);
      }
  return FDE_OK;
}

inline fde_status copy_d2d(void* dst, const void* src, size_t bytes, hipStream_t) {
  if (bytes) std::memmove(dst, src, bytes);
  return FDE_OK;
}

inline fde_status copy_h2d_sync(void* dst, const void* src, size_t bytes) {
  if (bytes) std::memcpy(dst, src, bytes);
  return FDE_OK;
}

inline fde_status stream_sync(hipStream_t) { return FDE_OK; }

#else

template <class Body, int BS, int MINW, class... Args>
__global__ void __launch_bounds__(BS, MINW) kgen(Args... args) {
  extern __shared__ __align__(16) char fde_smem[];
  Body::run(DevCtx{}, fde_smem, args...);
}

// Launch Body on `grid` blocks of `block` threads (block <= BS, the kernel's
// launch bound: 256 by default, 1024 for single-workgroup solvers; MINW is the
// minimum number of waves per SIMD the register allocation must allow).
template <class Body, int BS = 256, int MINW = 1, class... Args>
inline fde_status launch(dim3 grid, int block, size_t lds, hipStream_t s, Args... args) {
  if (grid.x == 0 || grid.y == 0 || grid.z == 0) return FDE_OK;
  if (lds > kLdsMax) return fail(FDE_ERR_UNSUPPORTED, "kernel needs more LDS than a CU has");
  if (block > BS) return fail(FDE_ERR_ARG, "block larger than the kernel's launch bound");
  auto k = kgen<Body, BS, MINW, Args...>;
  if (lds > 64 * 1024) {
    static size_t opted = 0;  // per instantiation
    if (lds > opted) {
      FDE_HIP(allow_lds(reinterpret_cast<const void*>(k), lds));
      opted = lds;
    }
  }
  hipLaunchKernelGGL(k, grid, dim3(block), lds, s, args...);
  FDE_HIP(hipGetLastError());
  return FDE_OK;
}

inline fde_status copy_d2d(void* dst, const void* src, size_t bytes, hipStream_t s) {
  if (bytes) FDE_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
  return FDE_OK;
}

inline fde_status copy_h2d_sync(void* dst, const void* src, size_t bytes) {
  if (bytes) FDE_HIP(hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice));
  return FDE_OK;
}

inline fde_status stream_sync(hipStream_t s) {
  FDE_HIP(hipStreamSynchronize(s));
  return FDE_OK;
}

#endif

#define FDE_TRY(...)                     \
  do {                                   \
    fde_status _s = (__VA_ARGS__);       \
    if (_s != FDE_OK) return _s;         \
  } while (0)

// Fill kernel (used instead of hipMemsetAsync so the calls stay capturable).
struct KFill {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, uint32_t* p, size_t nwords, uint32_t value, unsigned nblk) {
    const size_t stride = (size_t)c.nthr() * nblk;
    for (size_t i = (size_t)c.bx() * c.nthr() + c.tid(); i < nwords; i += stride) p[i] = value;
  }
};

inline fde_status zero_bytes(void* p, size_t bytes, hipStream_t s) {
  if (bytes % 4) return fail(FDE_ERR_ARG, "zero_bytes: size not a multiple of 4");
  size_t nw = bytes / 4;
  unsigned nblk = (unsigned)std::min<size_t>(4096, (nw + kBlock - 1) / kBlock);
  if (nblk == 0) return FDE_OK;
  return launch<KFill>(dim3(nblk), kBlock, 0, s, (uint32_t*)p, nw, 0u, nblk);
}

}  // namespace fde
