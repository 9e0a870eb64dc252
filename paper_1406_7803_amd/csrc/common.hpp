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
  // XCD-aware tile of a 2-D grid (gx, gy). The dispatcher hands consecutive workgroups to
  // the eight XCDs in turn; this maps them so that every XCD runs one contiguous range of
  // the order "x major, y minor" (XMAJOR) or "y major, x minor": neighbouring tiles of that
  // order, which read the same data or the same cache lines, then share one XCD's L2
  // instead of fetching it once per XCD.
  template <bool XMAJOR>
  __device__ __forceinline__ void xcd_tile(int& tx, int& ty) const {
    constexpr unsigned kXcds = 8;
    const unsigned gx = gridDim.x, gy = gridDim.y, total = gx * gy;
    const unsigned L = blockIdx.x + gx * blockIdx.y;
    const unsigned k = L % kXcds, idx = L / kXcds, base = total / kXcds, rem = total % kXcds;
    const unsigned logical = k * base + (k < rem ? k : rem) + idx;
    if (XMAJOR) {
      tx = (int)(logical / gy);
      ty = (int)(logical % gy);
    } else {
      ty = (int)(logical / gx);
      tx = (int)(logical % gx);
    }
  }
  // Wavefront-level helpers: lane and wavefront index, an LDS ordering point among the lanes
  // of one wavefront, and a fixed-order sum over aligned groups of W lanes that every lane of
  // the group receives (call with all W lanes of the group active).
  __device__ __forceinline__ int lane() const { return threadIdx.x & 63; }
  __device__ __forceinline__ int wave() const { return threadIdx.x >> 6; }
  __device__ __forceinline__ int nwave() const { return (blockDim.x + 63) >> 6; }
  __device__ __forceinline__ int wlanes() const { return blockDim.x < 64 ? blockDim.x : 64; }
  __device__ __forceinline__ void wsync() const {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
  template <int CTRL>
  __device__ __forceinline__ static double dpp(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  }
  __device__ __forceinline__ static double rdlane(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, l), hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
  }
  // W = 16: butterfly of row rotations (8, 4, 2, 1) inside each row of 16 lanes; a + b = b + a
  // makes the result bit-identical in every lane of the row. W = 64: the four row sums read
  // out and added in a fixed order (a wavefront-uniform value).
  template <int W>
  __device__ __forceinline__ double gsum(double v) const {
    static_assert(W == 1 || W == 16 || W == 64, "group of 1, 16 or 64 lanes");
    if (W == 1) return v;
    v += dpp<0x128>(v);
    v += dpp<0x124>(v);
    v += dpp<0x122>(v);
    v += dpp<0x121>(v);
    if (W == 16) return v;
    return (rdlane(v, 0) + rdlane(v, 16)) + (rdlane(v, 32) + rdlane(v, 48));
  }
  // 1 / sqrt(q) from the hardware estimate and two Newton steps
  __device__ __forceinline__ static double rsq(double q) {
    double r = __builtin_amdgcn_rsq(q);
    r = r * fma(-0.5 * q * r, r, 1.5);
    return r * fma(-0.5 * q * r, r, 1.5);
  }
  // 1 / q from the hardware reciprocal and two Newton steps
  __device__ __forceinline__ static double rcp(double q) {
    double r = __builtin_amdgcn_rcp(q);
    r = fma(r, fma(-q, r, 1.0), r);
    return fma(r, fma(-q, r, 1.0), r);
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
  template <bool XMAJOR>
  void xcd_tile(int& tx, int& ty) const {
    tx = x;
    ty = y;
  }
  void sync() const {}
  double sum(double v, double*) const { return v; }
  double max(double v, double*) const { return v; }
  int lane() const { return 0; }
  int wave() const { return 0; }
  int nwave() const { return 1; }
  int wlanes() const { return 1; }
  void wsync() const {}
  template <int W>
  double gsum(double v) const { return v; }
  static double rcp(double q) { return 1.0 / q; }
  static double rsq(double q) { return 1.0 / sqrt(q); }
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
      const int l = es == 1 ? idx / nbf : idx % nl;
      const int j = es == 1 ? idx - l * nbf : idx / nl;
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


// --------------------------------------------------------------------------
// Compile-time specialised Stockham passes for the grid lengths of the
// configured cells; every index computation folds to constants.
// --------------------------------------------------------------------------
struct RadixList {
  int nst;
  int r[12];
};

constexpr RadixList radix_list(int n) {
  RadixList p{0, {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0}};
  int m = n;
  while (m % 5 == 0) { p.r[p.nst++] = 5; m /= 5; }
  while (m % 3 == 0) { p.r[p.nst++] = 3; m /= 3; }
  while (m % 8 == 0 && m != 16) { p.r[p.nst++] = 8; m /= 8; }
  while (m % 4 == 0) { p.r[p.nst++] = 4; m /= 4; }
  while (m % 2 == 0) { p.r[p.nst++] = 2; m /= 2; }
  return p;
}

template <typename T, bool INV, int N, int R, int NS>
FDE_HD void bfly_c(const cplx<T>* __restrict__ src, cplx<T>* __restrict__ dst, int base, int es, int j,
                   const cplx<T>* __restrict__ tw) {
  constexpr int nbf = N / R;
  const int k = j % NS;
  cplx<T> v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = src[base + (j + r * nbf) * es];
  if (NS > 1) {
    constexpr int step = N / (NS * R);
#pragma unroll
    for (int r = 1; r < R; ++r) {
      const cplx<T> w = tw[r * k * step];
      v[r] = INV ? cmulc(w, v[r]) : w * v[r];
    }
  }
  if (R == 2) dft2<T, INV>(v);
  if (R == 3) dft3<T, INV>(v);
  if (R == 4) dft4<T, INV>(v);
  if (R == 5) dft5<T, INV>(v);
  if (R == 8) dft8<T, INV>(v);
  const int d = (j / NS) * NS * R + k;
#pragma unroll
  for (int r = 0; r < R; ++r) dst[base + (d + r * NS) * es] = v[r];
}

template <typename T, bool INV, int N, int S, int NS>
struct FftStages {
  template <class Ctx>
  FDE_HD static cplx<T>* run(const Ctx& c, cplx<T>* a, cplx<T>* b, int nl, int ls, int es,
                             const cplx<T>* __restrict__ tw) {
    constexpr RadixList RL = radix_list(N);
    if constexpr (S >= RL.nst) {
      return a;
    } else {
      constexpr int R = RL.r[S];
      constexpr int nbf = N / R;
      const int total = nl * nbf;
      if (es == 1) {  // contiguous lines: neighbouring threads take neighbouring butterflies
        for (int idx = c.tid(); idx < total; idx += c.nthr()) {
          const int l = idx / nbf;
          const int j = idx - l * nbf;
          bfly_c<T, INV, N, R, NS>(a, b, l * ls, es, j, tw);
        }
      } else {        // strided lines: neighbouring threads take neighbouring lines (no bank conflicts)
        for (int idx = c.tid(); idx < total; idx += c.nthr()) {
          const int j = idx / nl;
          const int l = idx - j * nl;
          bfly_c<T, INV, N, R, NS>(a, b, l * ls, es, j, tw);
        }
      }
      c.sync();
      return FftStages<T, INV, N, S + 1, NS * R>::run(c, b, a, nl, ls, es, tw);
    }
  }
};

// Dispatch: specialised lengths, else the runtime-radix passes.
template <typename T, bool INV, class Ctx>
FDE_HD cplx<T>* lds_fft_any(const Ctx& c, cplx<T>* a, cplx<T>* b, int nl, int ls, int es, const Radix& rp,
                            const cplx<T>* __restrict__ tw) {
  switch (rp.n) {
    case 24: return FftStages<T, INV, 24, 0, 1>::run(c, a, b, nl, ls, es, tw);
    case 48: return FftStages<T, INV, 48, 0, 1>::run(c, a, b, nl, ls, es, tw);
    case 60: return FftStages<T, INV, 60, 0, 1>::run(c, a, b, nl, ls, es, tw);
    case 72: return FftStages<T, INV, 72, 0, 1>::run(c, a, b, nl, ls, es, tw);
    case 96: return FftStages<T, INV, 96, 0, 1>::run(c, a, b, nl, ls, es, tw);
    case 120: return FftStages<T, INV, 120, 0, 1>::run(c, a, b, nl, ls, es, tw);
    case 144: return FftStages<T, INV, 144, 0, 1>::run(c, a, b, nl, ls, es, tw);
    case 180: return FftStages<T, INV, 180, 0, 1>::run(c, a, b, nl, ls, es, tw);
    case 240: return FftStages<T, INV, 240, 0, 1>::run(c, a, b, nl, ls, es, tw);
    case 432: return FftStages<T, INV, 432, 0, 1>::run(c, a, b, nl, ls, es, tw);
    default: return lds_fft<T, INV>(c, a, b, nl, ls, es, rp, tw);
  }
}



// --------------------------------------------------------------------------
// Compile-time twiddles exp(-2 pi i m / N): the angle is reduced to [0, pi/4]
// by exact integer quadrant/octant arithmetic and evaluated with Taylor series
// (terms to x^27; error below 1e-17 there).
// --------------------------------------------------------------------------
constexpr double kPiHalf = 1.57079632679489661923;

constexpr double cx_sin(double x) {
  double t = x, s = x;
  for (int n = 1; n < 14; ++n) {
    t *= -x * x / ((2.0 * n) * (2.0 * n + 1.0));
    s += t;
  }
  return s;
}

constexpr double cx_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int n = 1; n < 14; ++n) {
    t *= -x * x / ((2.0 * n - 1.0) * (2.0 * n));
    s += t;
  }
  return s;
}

// (cos, sin) of 2 pi m / n
struct CS {
  double c, s;
};
constexpr CS cx_cossin(int m, int n) {
  m %= n;
  if (m < 0) m += n;
  const int q = (4 * m) / n;            // quadrant
  const int rem = 4 * m - q * n;        // angle within it: (pi/2) rem / n
  double c = 0, s = 0;
  if (2 * rem <= n) {
    const double phi = kPiHalf * rem / n;
    c = cx_cos(phi);
    s = cx_sin(phi);
  } else {
    const double phi = kPiHalf * (n - rem) / n;
    c = cx_sin(phi);
    s = cx_cos(phi);
  }
  for (int k = 0; k < q; ++k) {  // rotate by pi/2 per quadrant
    const double t = c;
    c = -s;
    s = t;
  }
  return CS{c, s};
}

template <int N>
struct TwTable {
  double re[N], im[N];
  constexpr TwTable() : re(), im() {
    for (int m = 0; m < N; ++m) {
      const CS v = cx_cossin(m, N);
      re[m] = v.c;
      im[m] = -v.s;
    }
  }
};

template <int N>
inline constexpr TwTable<N> kTwTable{};

template <typename T, int N>
FDE_HD cplx<T> tw_const(int m) {
  return mk<T>((T)kTwTable<N>.re[m], (T)kTwTable<N>.im[m]);
}

// v times w^m (conjugated for INV), m in [0, N): the quarter turns as swaps and sign
// flips, which unrolled code resolves at compile time.
template <typename T, bool INV, int N>
FDE_HD cplx<T> tw_mul(int m, cplx<T> v) {
  if (m == 0) return v;
  if (4 * m == N) return INV ? mk<T>(-v.y, v.x) : mk<T>(v.y, -v.x);
  if (2 * m == N) return mk<T>(-v.x, -v.y);
  if (4 * m == 3 * N) return INV ? mk<T>(v.y, -v.x) : mk<T>(-v.y, v.x);
  const cplx<T> w = tw_const<T, N>(m);
  return INV ? cmulc(w, v) : w * v;
}

// --------------------------------------------------------------------------
// Whole-line FFT in registers (one thread per line): compile-time Stockham
// stages, every index a constant after unrolling, so v[] stays in VGPRs.
// --------------------------------------------------------------------------
template <typename T, bool INV, int N, int S, int NS>
FDE_HD void reg_stage(cplx<T>* x, cplx<T>* y, const cplx<T>* __restrict__ tw) {
  constexpr RadixList RL = radix_list(N);
  if constexpr (S < RL.nst) {
    constexpr int R = RL.r[S];
    constexpr int nbf = N / R;
    constexpr int step = N / (NS * R);
#pragma unroll
    for (int j = 0; j < nbf; ++j) {
      const int k = j % NS;
      cplx<T> v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = x[j + r * nbf];
      if (k != 0) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = tw_mul<T, INV, N>(r * k * step, v[r]);
      }
      if (R == 2) dft2<T, INV>(v);
      if (R == 3) dft3<T, INV>(v);
      if (R == 4) dft4<T, INV>(v);
      if (R == 5) dft5<T, INV>(v);
      if (R == 8) dft8<T, INV>(v);
      const int d = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) y[d + r * NS] = v[r];
    }
    reg_stage<T, INV, N, S + 1, NS * R>(y, x, tw);
  }
}

template <typename T, bool INV, int N>
FDE_HD void reg_fft(cplx<T>* v, const cplx<T>* __restrict__ tw) {
  cplx<T> t[N];
  reg_stage<T, INV, N, 0, 1>(v, t, tw);
  if constexpr (radix_list(N).nst % 2 == 1) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = t[i];
  }
}

FDE_HD int imod(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

// Row stride of the z-stick buffer [band][z][stick]: ncol rounded up to 16
// complex, so every plane row starts on a 128-byte boundary.
FDE_HD constexpr int stick_stride(int ncol) { return (ncol + 15) & ~15; }

FDE_HD int centred(int j, int n) { return j <= n / 2 ? j : j - n; }

}  // namespace fde
