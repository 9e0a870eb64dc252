// Learned preconditioner network: 4 -> 64 -> 64 -> 1 with tanh hidden layers.
//
// Parameters (flat FP32, FDE_MLP_NPARAM = 4545): W1[64][4], b1[64], W2[64][64],
// b2[64], w3[64], b3. Kernels use BF16 weights (W1, W2, w3 rounded to BF16 when
// staged in LDS) with FP32 accumulation; the hidden activations that feed the
// 64 x 64 products are rounded to BF16 too. The FP32 master copy is what Adam
// updates.
//
// On the device each wavefront evaluates 16 samples at a time; the 64 x 64
// layer and both 64 x 64 backward products run on v_mfma_f32_16x16x16bf16_1k:
//   a[i] = A[l % 16][4 (l / 16) + i],  b[i] = B[4 (l / 16) + i][l % 16],
//   c[r] = C[4 (l / 16) + r][l % 16]     (l = lane, i, r = 0..3).
// So lane l computes the first layer of sample l % 16 (hidden units
// 16 ks + 4 (l / 16) + i, ks = 0..3) and receives the outputs of samples
// 4 (l / 16) + r. The host-emulation build evaluates the same arithmetic with
// the same BF16 rounding points one sample at a time.
#pragma once

#include "kernels_la.hpp"

namespace fde {

constexpr int kMlpHid = 64, kMlpIn = 4, kMlpSample = 7;
constexpr int kMlpW1 = 0, kMlpB1 = kMlpW1 + kMlpHid * kMlpIn, kMlpW2 = kMlpB1 + kMlpHid;
constexpr int kMlpB2 = kMlpW2 + kMlpHid * kMlpHid, kMlpW3 = kMlpB2 + kMlpHid, kMlpB3 = kMlpW3 + kMlpHid;
constexpr int kMlpNParam = kMlpB3 + 1;                  // 4545
constexpr int kMlpNPad = (kMlpNParam + 63) & ~63;       // per-block gradient row
constexpr double kMlpRhoFloor = 1e-6;

// ---- BF16 (round to nearest even) -------------------------------------------
FDE_HD unsigned short f2bf(float x) {
  unsigned u = __builtin_bit_cast(unsigned, x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
FDE_HD float bf2f(unsigned short h) { return __builtin_bit_cast(float, (unsigned)h << 16); }
FDE_HD float bfr(float x) { return bf2f(f2bf(x)); }

FDE_HD float mlp_tanh(float x) {
  // tanh(x) = 1 - 2 / (1 + e^{2x}); saturates cleanly for large |x|
  const float e = expf(2.0f * x);
  return 1.0f - 2.0f / (1.0f + e);
}

// Weights staged in LDS (10 KB + W2^T 8 KB).
struct MlpW {
  float* W1;            // [64][4] BF16 values
  float* b1;            // [64]
  unsigned short* W2;   // [64 out][64 in] BF16
  unsigned short* W2T;  // [64 in][64 out] BF16
  float* b2;            // [64]
  float* w3;            // [64] BF16 values
  float* b3;            // [1]
  static constexpr size_t bytes = sizeof(float) * (256 + 64 + 64 + 64 + 4) + 2 * sizeof(unsigned short) * 4096;
  FDE_HD MlpW(char* lds) {
    W1 = (float*)lds;
    b1 = W1 + 256;
    b2 = b1 + 64;
    w3 = b2 + 64;
    b3 = w3 + 64;
    W2 = (unsigned short*)(b3 + 4);
    W2T = W2 + 4096;
  }
  template <class Ctx>
  FDE_HD void load(const Ctx& c, const float* __restrict__ p) {
    for (int i = c.tid(); i < 256; i += c.nthr()) W1[i] = bfr(p[kMlpW1 + i]);
    for (int i = c.tid(); i < 64; i += c.nthr()) {
      b1[i] = p[kMlpB1 + i];
      b2[i] = p[kMlpB2 + i];
      w3[i] = bfr(p[kMlpW3 + i]);
    }
    if (c.tid() == 0) b3[0] = p[kMlpB3];
    for (int i = c.tid(); i < 4096; i += c.nthr()) {
      const unsigned short h = f2bf(p[kMlpW2 + i]);
      W2[i] = h;
      W2T[(i & 63) * 64 + (i >> 6)] = h;
    }
  }
};

// Reference (per-sample) forward with the device's rounding points; also the
// emulation path. Returns y; h1b (BF16 values of tanh(z1)) and h2 if requested.
FDE_HD float mlp_forward_one(const MlpW& W, const float* u, float* h1b, float* h2) {
  float h1[kMlpHid];
  for (int k = 0; k < kMlpHid; ++k) {
    float z = W.b1[k];
    for (int j = 0; j < kMlpIn; ++j) z += W.W1[k * 4 + j] * u[j];
    h1[k] = bfr(mlp_tanh(z));
    if (h1b) h1b[k] = h1[k];
  }
  float y = W.b3[0];
  for (int o = 0; o < kMlpHid; ++o) {
    float z = 0.0f;
    for (int k = 0; k < kMlpHid; ++k) z += bf2f(W.W2[o * 64 + k]) * h1[k];
    const float h = mlp_tanh(z + W.b2[o]);
    if (h2) h2[o] = h;
    y += W.w3[o] * h;
  }
  return y;
}

#if defined(__HIP_DEVICE_COMPILE__)
typedef short fde_bf4 __attribute__((ext_vector_type(4)));
typedef float fde_f4 __attribute__((ext_vector_type(4)));

__device__ inline fde_bf4 bf4_lds(const unsigned short* p) {  // 4 consecutive BF16 (8-byte aligned)
  const uint2 v = *(const uint2*)p;
  fde_bf4 r;
  r[0] = (short)(v.x & 0xffff);
  r[1] = (short)(v.x >> 16);
  r[2] = (short)(v.y & 0xffff);
  r[3] = (short)(v.y >> 16);
  return r;
}

// Forward of 16 samples by one wavefront. u: the features of sample l % 16.
// Out: A operands of layer 2 (BF16 h1, per K-step), h2 (C layout), y of samples 4 (l / 16) + r.
__device__ inline void mlp_wave_forward(const MlpW& W, const float* u, int lane, fde_bf4 a1[4], fde_f4 h2[4],
                                        float y[4]) {
  const int q = lane >> 4, col = lane & 15;
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = 16 * ks + 4 * q + i;
      float z = W.b1[k];
#pragma unroll
      for (int j = 0; j < 4; ++j) z += W.W1[k * 4 + j] * u[j];
      a1[ks][i] = (short)f2bf(mlp_tanh(z));
    }
  }
#pragma unroll
  for (int nt = 0; nt < 4; ++nt) {
    fde_f4 acc = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const fde_bf4 b = bf4_lds(W.W2 + (16 * nt + col) * 64 + 16 * ks + 4 * q);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1[ks], b, acc, 0, 0, 0);
    }
    const float bo = W.b2[16 * nt + col];
#pragma unroll
    for (int r = 0; r < 4; ++r) h2[nt][r] = mlp_tanh(acc[r] + bo);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    float p = 0.0f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) p += W.w3[16 * nt + col] * h2[nt][r];
    p += __shfl_xor(p, 1, 64);
    p += __shfl_xor(p, 2, 64);
    p += __shfl_xor(p, 4, 64);
    p += __shfl_xor(p, 8, 64);
    y[r] = p + W.b3[0];
  }
}
#endif

// ---------------------------------------------------------------------------
// y[s] = MLP(u[s]), u [n][4]. grid ceil(n / 64), 256 threads (16 samples per wave).
// ---------------------------------------------------------------------------
struct KMlpForward {
  static constexpr size_t lds_bytes = MlpW::bytes;
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const float* __restrict__ u, int n, const float* __restrict__ params,
                         float* __restrict__ y) {
    MlpW W(lds);
    W.load(c, params);
    c.sync();
#if defined(__HIP_DEVICE_COMPILE__)
    const int lane = c.tid() & 63, wave = c.tid() >> 6;
    const int s0 = c.bx() * 64 + wave * 16;
    const int si = s0 + (lane & 15);
    float uu[4] = {0, 0, 0, 0};
    if (si < n)
      for (int j = 0; j < 4; ++j) uu[j] = u[(size_t)si * 4 + j];
    fde_bf4 a1[4];
    fde_f4 h2[4];
    float yy[4];
    mlp_wave_forward(W, uu, lane, a1, h2, yy);
    const int col = lane & 15, q = lane >> 4;
    if (col < 4) {
      const int so = s0 + 4 * q + col;
      float v = yy[0];
      if (col == 1) v = yy[1];
      if (col == 2) v = yy[2];
      if (col == 3) v = yy[3];
      if (so < n) y[so] = v;
    }
#else
    for (int l = c.tid(); l < 64; l += c.nthr()) {
      const int s = c.bx() * 64 + l;
      if (s < n) y[s] = mlp_forward_one(W, u + (size_t)s * 4, nullptr, nullptr);
    }
#endif
  }
};

// ---------------------------------------------------------------------------
// Loss and gradient over samples [n][7] = (u1..u4, A, B, C):
//   loss = (1/n) sum_s A e^{2y} - 2 B e^y + C.
// Each block takes `per_block` samples (a multiple of 64) and writes its gradient
// sum to part[block][kMlpNPad] and its loss sum to lpart[block].
// grid nblk, 256 threads.
// ---------------------------------------------------------------------------
struct KMlpLossGrad {
  // per wave: h1 tile [16][64] FP32, dz2 tile [16][64] BF16, u tile [16][4]
  static constexpr size_t wave_bytes = sizeof(float) * 16 * 64 + sizeof(unsigned short) * 16 * 64 + sizeof(float) * 64;
  static constexpr size_t lds_bytes = MlpW::bytes + 4 * wave_bytes + sizeof(float) * 4 * kMlpNPad / 4 + 64;
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const float* __restrict__ smp, int n, int per_block,
                         const float* __restrict__ params, float* __restrict__ part, double* __restrict__ lpart) {
    MlpW W(lds);
    W.load(c, params);
    const float inv_n = 1.0f / (float)n;
    const int sb0 = c.bx() * per_block;
#if defined(__HIP_DEVICE_COMPILE__)
    const int lane = c.tid() & 63, wave = c.tid() >> 6;
    const int q = lane >> 4, col = lane & 15;
    char* wbase = lds + MlpW::bytes + wave * wave_bytes;
    float* tH1 = (float*)wbase;                                   // [16 s][64 h]
    unsigned short* tDZ = (unsigned short*)(tH1 + 16 * 64);       // [16 s][64 o]
    float* tU = (float*)(tDZ + 16 * 64);                          // [16 s][4]
    fde_f4 gW2[4][4];  // [mt = o tile][ht = h tile], C layout: o = 16 mt + 4 q + r, h = 16 ht + col
    float gW1[4][4], gb1[4], gb2[4], gw3[4], gb3 = 0.0f;  // h or o = 16 t + col
    double lsum = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        gW2[a][b] = fde_f4{0, 0, 0, 0};
        gW1[a][b] = 0.0f;
      }
      gb1[a] = gb2[a] = gw3[a] = 0.0f;
    }
    c.sync();
    for (int g0 = sb0 + wave * 16; g0 < sb0 + per_block; g0 += 64) {
      const int si = g0 + col;
      float uu[4] = {0, 0, 0, 0};
      if (si < n)
        for (int j = 0; j < 4; ++j) uu[j] = smp[(size_t)si * 7 + j];
      fde_bf4 a1[4];
      fde_f4 h2[4];
      float yy[4];
      mlp_wave_forward(W, uu, lane, a1, h2, yy);
      // this wave's h1 (BF16 values) and u tiles
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
#pragma unroll
        for (int i = 0; i < 4; ++i) tH1[col * 64 + 16 * ks + 4 * q + i] = bf2f((unsigned short)a1[ks][i]);
      if (q == 0)
        for (int j = 0; j < 4; ++j) tU[col * 4 + j] = uu[j];
      // dL/dy of samples 4 q + r
      float gy[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int s = g0 + 4 * q + r;
        gy[r] = 0.0f;
        if (s < n) {
          const float A = smp[(size_t)s * 7 + 4], B = smp[(size_t)s * 7 + 5], C = smp[(size_t)s * 7 + 6];
          const float e = expf(yy[r]);
          gy[r] = (2.0f * A * e * e - 2.0f * B * e) * inv_n;
          if (col == 0) lsum += (double)(A * e * e - 2.0f * B * e + C);
          if (col == 0) gb3 += gy[r];
        }
      }
      // dz2 = gy w3 (1 - h2^2) in C layout; gw3, gb2; dz2 tile (BF16) for the dh1 product
      fde_bf4 adz[4];
#pragma unroll
      for (int nt = 0; nt < 4; ++nt) {
        const float w = W.w3[16 * nt + col];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float h = h2[nt][r];
          const float dz = gy[r] * w * (1.0f - h * h);
          gw3[nt] += gy[r] * h;
          gb2[nt] += dz;
          const unsigned short db = f2bf(dz);
          adz[nt][r] = (short)db;
          tDZ[(4 * q + r) * 64 + 16 * nt + col] = db;
        }
      }
      c.sync();  // tiles visible to the whole wave (uniform trip count over the block)
      // dW2[o][h] += sum_s dz2[s][o] h1[s][h]: A = dz2^T (own C-layout values), B = h1 (tile)
#pragma unroll
      for (int ht = 0; ht < 4; ++ht) {
        fde_bf4 bh;
#pragma unroll
        for (int i = 0; i < 4; ++i) bh[i] = (short)f2bf(tH1[(4 * q + i) * 64 + 16 * ht + col]);
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) gW2[mt][ht] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(adz[mt], bh, gW2[mt][ht], 0, 0, 0);
      }
      // dh1[s][h] = sum_o dz2[s][o] W2[o][h]: A = dz2 (tile), B = W2 (via W2^T rows)
      fde_bf4 ad[4];
#pragma unroll
      for (int ko = 0; ko < 4; ++ko) ad[ko] = bf4_lds(tDZ + col * 64 + 16 * ko + 4 * q);
#pragma unroll
      for (int ht = 0; ht < 4; ++ht) {
        fde_f4 dh = {0, 0, 0, 0};
#pragma unroll
        for (int ko = 0; ko < 4; ++ko) {
          const fde_bf4 b = bf4_lds(W.W2T + (16 * ht + col) * 64 + 16 * ko + 4 * q);
          dh = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ad[ko], b, dh, 0, 0, 0);
        }
        // dz1 = dh1 (1 - h1^2) at (s = 4 q + r, h = 16 ht + col); gW1, gb1
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int s = 4 * q + r;
          const float h = tH1[s * 64 + 16 * ht + col];
          const float dz1 = dh[r] * (1.0f - h * h);
          gb1[ht] += dz1;
#pragma unroll
          for (int j = 0; j < 4; ++j) gW1[ht][j] += dz1 * tU[s * 4 + j];
        }
      }
      c.sync();
    }
    // ---- reduce the lane partials: sum over q (lanes col, col+16, col+32, col+48), then over waves
    float* red = (float*)(lds + MlpW::bytes + 4 * wave_bytes);  // [4 waves][kMlpNPad / 4]... reuse as [kMlpNPad]
    for (int i = c.tid(); i < kMlpNPad; i += c.nthr()) red[i] = 0.0f;
    c.sync();
    // vectors over h or o (= 16 t + col): gb1, gb2, gw3, gW1
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      float v1 = gb1[t], v2 = gb2[t], v3 = gw3[t];
      v1 += __shfl_xor(v1, 16, 64);
      v1 += __shfl_xor(v1, 32, 64);
      v2 += __shfl_xor(v2, 16, 64);
      v2 += __shfl_xor(v2, 32, 64);
      v3 += __shfl_xor(v3, 16, 64);
      v3 += __shfl_xor(v3, 32, 64);
      float w1[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        w1[j] = gW1[t][j];
        w1[j] += __shfl_xor(w1[j], 16, 64);
        w1[j] += __shfl_xor(w1[j], 32, 64);
      }
      const int h = 16 * t + col;
      for (int w = 0; w < 4; ++w) {  // fixed wave order
        if (wave == w && q == 0) {
          red[kMlpB1 + h] += v1;
          red[kMlpB2 + h] += v2;
          red[kMlpW3 + h] += v3;
#pragma unroll
          for (int j = 0; j < 4; ++j) red[kMlpW1 + h * 4 + j] += w1[j];
        }
        c.sync();
      }
    }
    // dW2: each lane owns distinct (o, h) entries
    for (int w = 0; w < 4; ++w) {
      if (wave == w) {
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
          for (int ht = 0; ht < 4; ++ht)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[kMlpW2 + (16 * mt + 4 * q + r) * 64 + 16 * ht + col] += gW2[mt][ht][r];
      }
      c.sync();
    }
    // b3 and the loss: lanes col == 0 hold them
    float b3s = gb3;
    b3s += __shfl_xor(b3s, 16, 64);
    b3s += __shfl_xor(b3s, 32, 64);
    double ls = lsum;
    ls += __shfl_xor(ls, 16, 64);
    ls += __shfl_xor(ls, 32, 64);
    double* lred = (double*)(red + kMlpNPad);
    if (lane == 0) lred[wave] = ls;
    for (int w = 0; w < 4; ++w) {
      if (wave == w && lane == 0) red[kMlpB3] += b3s;
      c.sync();
    }
    for (int i = c.tid(); i < kMlpNPad; i += c.nthr()) part[(size_t)c.bx() * kMlpNPad + i] = i < kMlpNParam ? red[i] : 0.0f;
    if (c.tid() == 0) lpart[c.bx()] = ((lred[0] + lred[1]) + (lred[2] + lred[3])) / (double)n;
#else
    // emulation: one sample at a time, same rounding points
    float* red = (float*)(lds + MlpW::bytes);
    for (int i = 0; i < kMlpNPad; ++i) red[i] = 0.0f;
    double lsum = 0.0;
    for (int s = sb0; s < sb0 + per_block && s < n; ++s) {
      const float* u = smp + (size_t)s * 7;
      float h1b[kMlpHid], h2[kMlpHid];
      const float yv = mlp_forward_one(W, u, h1b, h2);
      const float A = u[4], B = u[5], C = u[6];
      const float e = expf(yv);
      const float gy = (2.0f * A * e * e - 2.0f * B * e) * inv_n;
      lsum += (double)(A * e * e - 2.0f * B * e + C);
      red[kMlpB3] += gy;
      float dz2b[kMlpHid];
      for (int o = 0; o < kMlpHid; ++o) {
        const float dz = gy * W.w3[o] * (1.0f - h2[o] * h2[o]);
        red[kMlpW3 + o] += gy * h2[o];
        red[kMlpB2 + o] += dz;
        dz2b[o] = bfr(dz);
      }
      for (int o = 0; o < kMlpHid; ++o)
        for (int k = 0; k < kMlpHid; ++k) red[kMlpW2 + o * 64 + k] += dz2b[o] * h1b[k];
      for (int k = 0; k < kMlpHid; ++k) {
        float dh = 0.0f;
        for (int o = 0; o < kMlpHid; ++o) dh += dz2b[o] * bf2f(W.W2[o * 64 + k]);
        const float dz1 = dh * (1.0f - h1b[k] * h1b[k]);
        red[kMlpB1 + k] += dz1;
        for (int j = 0; j < 4; ++j) red[kMlpW1 + k * 4 + j] += dz1 * u[j];
      }
    }
    for (int i = 0; i < kMlpNPad; ++i) part[(size_t)c.bx() * kMlpNPad + i] = i < kMlpNParam ? red[i] : 0.0f;
    lpart[c.bx()] = lsum / (double)n;
#endif
  }
};

// grad[i] = sum_b part[b][i] (fixed order); loss = sum_b lpart[b]. grid ceil(kMlpNPad / 256)
struct KMlpReduce {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const float* __restrict__ part, const double* __restrict__ lpart, int nblk,
                         float* __restrict__ grad, double* __restrict__ loss) {
    for (int l = c.tid(); l < 256; l += c.nthr()) {
      const int i = c.bx() * 256 + l;
      if (i < kMlpNParam) {
        float s = 0.0f;
        for (int b = 0; b < nblk; ++b) s += part[(size_t)b * kMlpNPad + i];
        grad[i] = s;
      }
      if (c.bx() == 0 && l == 0) {
        double t = 0.0;
        for (int b = 0; b < nblk; ++b) t += lpart[b];
        loss[0] = t;
      }
    }
  }
};

// One Adam step on the FP32 master parameters (t counts from 1).
struct KMlpAdam {
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char*, const float* __restrict__ g, float* __restrict__ p, float* __restrict__ m,
                         float* __restrict__ v, int t, float lr, float beta1, float beta2, float eps) {
    const float c1 = 1.0f - powf(beta1, (float)t), c2 = 1.0f - powf(beta2, (float)t);
    for (int l = c.tid(); l < 256; l += c.nthr()) {
      const int i = c.bx() * 256 + l;
      if (i >= kMlpNParam) continue;
      const float gi = g[i];
      const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
      const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
      m[i] = mi;
      v[i] = vi;
      p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
  }
};

// ---------------------------------------------------------------------------
// Preconditioner with the network (batched like KPrecond): per band n,
//   R = HX - lambda X, active = ||R|| > 1e-10,
//   T_G = K_TPA(x_G) exp(y_G) R_G with y_G = MLP(u_G), x_G = kin_G / T_n,
//   u = (log(1 + x), log T_n, log max(|R_G| sqrt(npw) / ||R||, 1e-6), (lambda - vbar) / T_n),
// then T normalised (zero when inactive). grid (nb, nprob), 256 threads.
// ---------------------------------------------------------------------------
template <typename T>
struct KPrecondMlp {
  static constexpr size_t lds_bytes = MlpW::bytes + 17 * sizeof(double);
  template <class Ctx>
  FDE_HD static void run(const Ctx& c, char* lds, const ProbSet<T> ps, const float* __restrict__ params,
                         const double* __restrict__ vbar) {
    const Prob<T>& P = ps.p[c.by()];
    const int n = c.bx();
    if (n >= P.nb) return;  // uniform per block
    MlpW W(lds);
    W.load(c, params);
    double* red = (double*)(lds + MlpW::bytes);
    const int npw = P.npw;
    const double lam = P.eval[n];
    const cplx<T>* xn = P.v + (size_t)n * npw;
    const cplx<T>* hn = P.hv + (size_t)n * npw;
    cplx<T>* tn = P.t + (size_t)n * npw;
    const double kf0 = P.kf[0], kf1 = P.kf[1], kf2 = P.kf[2];
    const double b0 = ps.b[0], b1 = ps.b[1], b2 = ps.b[2];
    auto kin = [&](int g) {
      const int p = P.millp[g];
      const double q1 = (((p & 1023) - 512) + kf0) * b0;
      const double q2 = ((((p >> 10) & 1023) - 512) + kf1) * b1;
      const double q3 = ((((p >> 20) & 1023) - 512) + kf2) * b2;
      return 0.5 * (q1 * q1 + q2 * q2 + q3 * q3);
    };
    double r2 = 0.0, tk = 0.0;
    for (int g = c.tid(); g < npw; g += c.nthr()) {
      const cplx<T> xv = xn[g], hv = hn[g];
      const double rx = (double)hv.x - lam * xv.x, ry = (double)hv.y - lam * xv.y;
      r2 += rx * rx + ry * ry;
      tk += kin(g) * ((double)xv.x * xv.x + (double)xv.y * xv.y);
    }
    r2 = c.sum(r2, red);
    tk = c.sum(tk, red);
    const double rn = sqrt(r2);
    const bool act = rn > 1e-10;
    const double rsc = rn > 0.0 ? sqrt((double)npw) / rn : 0.0;
    const float u2 = (float)log(tk), u4 = (float)((lam - vbar[c.by()]) / tk);
    // features of coefficient g and its TPA factor and residual
    auto feat = [&](int g, float* u, double& K, double& rx, double& ry) {
      const cplx<T> xv = xn[g], hv = hn[g];
      rx = (double)hv.x - lam * xv.x;
      ry = (double)hv.y - lam * xv.y;
      const double xx = kin(g) / tk;
      const double pp = 27.0 + xx * (18.0 + xx * (12.0 + 8.0 * xx));
      K = pp / (pp + 16.0 * xx * xx * xx * xx);
      const double rho = sqrt(rx * rx + ry * ry) * rsc;
      u[0] = (float)log1p(xx);
      u[1] = u2;
      u[2] = (float)log(rho > kMlpRhoFloor ? rho : kMlpRhoFloor);
      u[3] = u4;
    };
    double t2 = 0.0;
#if defined(__HIP_DEVICE_COMPILE__)
    const int lane = c.tid() & 63, wave = c.tid() >> 6;
    const int q = lane >> 4, col = lane & 15;
    for (int g0 = wave * 16; g0 < npw; g0 += 64) {
      float uu[4] = {0, 0, 0, 0};
      double K, rx, ry;
      if (g0 + col < npw) feat(g0 + col, uu, K, rx, ry);
      fde_bf4 a1[4];
      fde_f4 h2[4];
      float yy[4];
      mlp_wave_forward(W, uu, lane, a1, h2, yy);
      if (col < 4 && g0 + 4 * q + col < npw) {
        const int g = g0 + 4 * q + col;
        float y = yy[0];
        if (col == 1) y = yy[1];
        if (col == 2) y = yy[2];
        if (col == 3) y = yy[3];
        float ud[4];
        feat(g, ud, K, rx, ry);
        const double f = K * exp((double)y);
        const double ux = f * rx, uy = f * ry;
        t2 += ux * ux + uy * uy;
        tn[g] = mk<T>((T)ux, (T)uy);
      }
    }
#else
    for (int g = c.tid(); g < npw; g += c.nthr()) {
      float uu[4];
      double K, rx, ry;
      feat(g, uu, K, rx, ry);
      const float y = mlp_forward_one(W, uu, nullptr, nullptr);
      const double f = K * exp((double)y);
      const double ux = f * rx, uy = f * ry;
      t2 += ux * ux + uy * uy;
      tn[g] = mk<T>((T)ux, (T)uy);
    }
#endif
    t2 = c.sum(t2, red);
    const double sc = (act && t2 > 0.0) ? 1.0 / sqrt(t2) : 0.0;
    for (int g = c.tid(); g < npw; g += c.nthr()) {
      const cplx<T> v = tn[g];
      tn[g] = mk<T>((T)(sc * v.x), (T)(sc * v.y));
    }
    if (c.tid() == 0) {
      P.act_out[n] = act ? 1 : 0;
      P.rnorm[n] = rn;
    }
  }
};

}  // namespace fde
