// Common device building blocks for the frozen-density-embedding library:
// complex arithmetic, execution contexts, and LDS-resident mixed-radix FFTs.
//
// Kernel bodies are written against a context object (tid, nthr, block
// indices, barrier) so that the same body runs as a HIP kernel (DevCtx) or,
// for host-side checks of indexing and arithmetic, serially on the CPU
// (HostCtx with one thread and a no-op barrier).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define FDE_HD __host__ __device__ __forceinline__

namespace fde {

template <typename T>
struct alignas(2 * sizeof(T)) cplx {
  T x, y;
};

template <typename T> FDE_HD cplx<T> mk(T a, T b) { cplx<T> r; r.x = a; r.y = b; return r; }
template <typename T> FDE_HD cplx<T> operator+(cplx<T> a, cplx<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> FDE_HD cplx<T> operator-(cplx<T> a, cplx<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> FDE_HD cplx<T> operator*(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> FDE_HD cplx<T> operator*(T s, cplx<T> a) { return mk<T>(s * a.x, s * a.y); }
template <typename T> FDE_HD cplx<T> conj(cplx<T> a) { return mk<T>(a.x, -a.y); }
// conj(a) * b
template <typename T> FDE_HD cplx<T> cmulc(cplx<T> a, cplx<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// multiply by -i (FWD) or +i (INV)
template <typename T, bool INV> FDE_HD cplx<T> rot90(cplx<T> a) {
  return INV ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}
template <typename T> FDE_HD T norm2(cplx<T> a) { return a.x * a.x + a.y * a.y; }

// --------------------------------------------------------------------------
// Execution contexts (reductions need an LDS scratch of 17 doubles)
// --------------------------------------------------------------------------
struct DevCtx {
  __device__ __forceinline__ int tid() const { return threadIdx.x; }
  __device__ __forceinline__ int nthr() const { return blockDim.x; }
  __device__ __forceinline__ int bx() const { return blockIdx.x; }
  __device__ __forceinline__ int by() const { return blockIdx.y; }
  __device__ __forceinline__ int bz() const { return blockIdx.z; }
  __device__ __forceinline__ void sync() const { __syncthreads(); }
  // Block-wide sum in a fixed order; red: >= 16 doubles of LDS. All threads
  // receive the total. Contains barriers: call from uniform control flow.
  __device__ double sum(double v, double* red) const {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      const int nw = (blockDim.x + 63) >> 6;
      for (int i = 0; i < nw; ++i) t += red[i];
      red[16] = t;
    }
    __syncthreads();
    return red[16];
  }
  __device__ double max(double v, double* red) const {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = red[0];
      const int nw = (blockDim.x + 63) >> 6;
      for (int i = 1; i < nw; ++i) t = fmax(t, red[i]);
      red[16] = t;
    }
    __syncthreads();
    return red[16];
  }
};

struct HostCtx {
  int x = 0, y = 0, z = 0;
  int tid() const { return 0; }
  int nthr() const { return 1; }
  int bx() const { return x; }
  int by() const { return y; }
  int bz() const { return z; }
  void sync() const {}
  double sum(double v, double*) const { return v; }
  double max(double v, double*) const { return v; }
};

// --------------------------------------------------------------------------
// Radix plan of one FFT length n = prod r_s, r_s in {2,3,4,5,8}
// --------------------------------------------------------------------------
struct Radix {
  int n;
  int nst;
  int r[12];
};

inline Radix make_radix(int n) {
  Radix p;
  p.n = n;
  p.nst = 0;
  int m = n;
  while (m % 5 == 0) { p.r[p.nst++] = 5; m /= 5; }
  while (m % 3 == 0) { p.r[p.nst++] = 3; m /= 3; }
  while (m % 8 == 0 && m != 16) { p.r[p.nst++] = 8; m /= 8; }
  while (m % 4 == 0) { p.r[p.nst++] = 4; m /= 4; }
  while (m % 2 == 0) { p.r[p.nst++] = 2; m /= 2; }
  if (m != 1) p.nst = -1;  // unsupported length
  return p;
}

// --------------------------------------------------------------------------
// Small DFTs in registers. FWD: exp(-2 pi i jk/R), INV: exp(+2 pi i jk/R).
// --------------------------------------------------------------------------
template <typename T, bool INV> FDE_HD void dft2(cplx<T>* v) {
  cplx<T> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <typename T, bool INV> FDE_HD void dft3(cplx<T>* v) {
  const T h = T(0.86602540378443864676);  // sqrt(3)/2
  cplx<T> t = v[1] + v[2];
  cplx<T> d = v[1] - v[2];
  cplx<T> a = v[0] - T(0.5) * t;
  cplx<T> r = rot90<T, INV>(h * d);  // -i h d (FWD)
  v[0] = v[0] + t;
  v[1] = a + r;
  v[2] = a - r;
}

template <typename T, bool INV> FDE_HD void dft4(cplx<T>* v) {
  cplx<T> t0 = v[0] + v[2], t1 = v[0] - v[2];
  cplx<T> t2 = v[1] + v[3], t3 = rot90<T, INV>(v[1] - v[3]);
  v[0] = t0 + t2;
  v[2] = t0 - t2;
  v[1] = t1 + t3;
  v[3] = t1 - t3;
}

template <typename T, bool INV> FDE_HD void dft5(cplx<T>* v) {
  const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
  const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);
  cplx<T> t1 = v[1] + v[4], t2 = v[2] + v[3];
  cplx<T> t3 = v[1] - v[4], t4 = v[2] - v[3];
  cplx<T> b1 = v[0] + c1 * t1 + c2 * t2;
  cplx<T> b2 = v[0] + c2 * t1 + c1 * t2;
  cplx<T> e1 = rot90<T, INV>(s1 * t3 + s2 * t4);  // -i(s1 t3 + s2 t4) (FWD)
  cplx<T> e2 = rot90<T, INV>(s2 * t3 - s1 * t4);
  v[0] = v[0] + t1 + t2;
  v[1] = b1 + e1;
  v[4] = b1 - e1;
  v[2] = b2 + e2;
  v[3] = b2 - e2;
}

template <typename T, bool INV> FDE_HD void dft8(cplx<T>* v) {
  cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
  cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, INV>(e);
  dft4<T, INV>(o);
  const T r = T(0.70710678118654752440);
  // w^k o_k, w = exp(-+ 2 pi i / 8)
  cplx<T> w1 = INV ? mk<T>(r * (o[1].x - o[1].y), r * (o[1].x + o[1].y))
                   : mk<T>(r * (o[1].x + o[1].y), r * (o[1].y - o[1].x));
  cplx<T> w2 = rot90<T, INV>(o[2]);
  cplx<T> w3 = INV ? mk<T>(-r * (o[3].x + o[3].y), r * (o[3].x - o[3].y))
                   : mk<T>(r * (o[3].y - o[3].x), -r * (o[3].x + o[3].y));
  v[0] = e[0] + o[0];
  v[4] = e[0] - o[0];
  v[1] = e[1] + w1;
  v[5] = e[1] - w1;
  v[2] = e[2] + w2;
  v[6] = e[2] - w2;
  v[3] = e[3] + w3;
  v[7] = e[3] - w3;
}

// One Stockham butterfly of radix R for line `base`, butterfly j, stride Ns.
// src element e of the line is src[base + e*es]; dst likewise.
// tw[m] = exp(-2 pi i m / n) (conjugated for INV).
template <typename T, bool INV, int R>
FDE_HD void bfly(const cplx<T>* __restrict__ src, cplx<T>* __restrict__ dst, int base, int es, int n,
                 int j, int Ns, const cplx<T>* __restrict__ tw) {
  const int nbf = n / R;
  const int k = j % Ns;
  cplx<T> v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = src[base + (j + r * nbf) * es];
  if (Ns > 1) {
    const int step = n / (Ns * R);
#pragma unroll
    for (int r = 1; r < R; ++r) {
      cplx<T> w = tw[r * k * step];
      v[r] = INV ? cmulc(w, v[r]) : w * v[r];
    }
  }
  if (R == 2) dft2<T, INV>(v);
  if (R == 3) dft3<T, INV>(v);
  if (R == 4) dft4<T, INV>(v);
  if (R == 5) dft5<T, INV>(v);
  if (R == 8) dft8<T, INV>(v);
  const int d = (j / Ns) * Ns * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) dst[base + (d + r * Ns) * es] = v[r];
}

// Batched in-LDS FFT of `nl` lines of length n. Element e of line l lives at
// buf[l*ls + e*es]. Ping-pongs between a and b; returns the buffer that holds
// the result. Ends with a barrier. Unscaled in both directions.
template <typename T, bool INV, class Ctx>
FDE_HD cplx<T>* lds_fft(const Ctx& c, cplx<T>* a, cplx<T>* b, int nl, int ls, int es, const Radix& rp,
                        const cplx<T>* __restrict__ tw) {
  const int n = rp.n;
  int Ns = 1;
  for (int s = 0; s < rp.nst; ++s) {
    const int R = rp.r[s];
    const int nbf = n / R;
    const int total = nl * nbf;
    for (int idx = c.tid(); idx < total; idx += c.nthr()) {
      const int l = idx / nbf;
      const int j = idx - l * nbf;
      const int base = l * ls;
      switch (R) {
        case 2: bfly<T, INV, 2>(a, b, base, es, n, j, Ns, tw); break;
        case 3: bfly<T, INV, 3>(a, b, base, es, n, j, Ns, tw); break;
        case 4: bfly<T, INV, 4>(a, b, base, es, n, j, Ns, tw); break;
        case 5: bfly<T, INV, 5>(a, b, base, es, n, j, Ns, tw); break;
        default: bfly<T, INV, 8>(a, b, base, es, n, j, Ns, tw); break;
      }
    }
    c.sync();
    cplx<T>* t = a;
    a = b;
    b = t;
    Ns *= R;
  }
  return a;
}

FDE_HD int imod(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

FDE_HD int centred(int j, int n) { return j <= n / 2 ? j : j - n; }

}  // namespace fde
