// mhd_mlp.hpp -- device side of the learned flux correction: a 32-64-64-8
// MLP with GELU hidden layers, bfloat16 weights and activations, FP32
// accumulation on the matrix cores (v_mfma_f32_16x16x16_bf16), plus the face
// features and the output-to-flux map shared by training and inference.
//
// Parameter vector (FP32 master, 6792 values): W1[64][32], b1[64],
// W2[64][64], b2[64], W3[8][64], b3[8].  Weights are rounded to bfloat16 when
// loaded; biases stay FP32.
//
// MFMA 16x16x16 operand layout (lane l, r = l % 16, q = l / 16):
//   A (16 x 16, M x K): lane holds A[r][4q .. 4q+3]
//   B (16 x 16, K x N): lane holds B[4q .. 4q+3][r]
//   D (16 x 16, M x N): lane holds D[4q .. 4q+3][r]
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mhd {

constexpr int kMlpIn = 32;
constexpr int kMlpHid = 64;
constexpr int kMlpOut = 8;
constexpr int kMlpParams = 6792;
constexpr int kP_W1 = 0;
constexpr int kP_B1 = kP_W1 + 64 * 32;
constexpr int kP_W2 = kP_B1 + 64;
constexpr int kP_B2 = kP_W2 + 64 * 64;
constexpr int kP_W3 = kP_B2 + 64;
constexpr int kP_B3 = kP_W3 + 8 * 64;

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16v2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ unsigned short bf16_bits(float x) {
  unsigned u = __float_as_uint(x);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf16_float(unsigned short b) {
  return __uint_as_float(((unsigned)b) << 16);
}
__device__ __forceinline__ float bf16_round(float x) { return bf16_float(bf16_bits(x)); }

// Normal CDF Phi(x) = (1 + erf(x / sqrt 2)) / 2 from the Chebyshev-fitted
// erfc of Numerical Recipes (2nd ed., section 6.2; fractional error below
// 1.2e-7 for every argument), taken at |x| so that both tails keep their
// relative accuracy: Phi = 1 - erfc(|x|/sqrt 2)/2 for x >= 0, else
// erfc(|x|/sqrt 2)/2.  About 16 vector instructions against some 50 for the
// library erff; GELU's 128 evaluations per face dominate the MLP's cost.
__device__ __forceinline__ float norm_cdf(float x) {
  const float z = fabsf(x) * 0.70710678118654752f;
  const float t = __builtin_amdgcn_rcpf(1.0f + 0.5f * z);
  float p = 0.17087277f;
  p = fmaf(p, t, -0.82215223f);
  p = fmaf(p, t, 1.48851587f);
  p = fmaf(p, t, -1.13520398f);
  p = fmaf(p, t, 0.27886807f);
  p = fmaf(p, t, -0.18628806f);
  p = fmaf(p, t, 0.09678418f);
  p = fmaf(p, t, 0.37409196f);
  p = fmaf(p, t, 1.00002368f);
  p = fmaf(p, t, -1.26551223f);
  const float e = 0.5f * t * __expf(fmaf(-z, z, p));
  return x >= 0.0f ? 1.0f - e : e;
}

// The normal CDF table of the in-step inference in LDS (kPhiN quadratic
// pieces on [-8, 8), see mhd_kernels.hpp), one array per coefficient: the
// 64 lanes of a read fetch scattered pieces, and one 4-byte word a piece
// per read spreads them over all the banks, where 16-byte pieces fall into
// eight bank groups and conflict four times as often.
struct PhiLds {
  float c0[kPhiN], c1[kPhiN], c2[kPhiN];
};

// Phi(x) from the table: interpolation error below 1e-7, three LDS reads
// and 3 FMAs where the erfc form takes 16 instructions, two of them
// quarter-rate.  Outside the table Phi is its end value (|Phi(8) - 1|,
// Phi(-8) < 1e-15); a NaN argument reads piece 0.
__device__ __forceinline__ float norm_cdf_tab(const PhiLds& tab, float x) {
  float t = fmaf(x, (float)kPhiScale, (float)(kPhiHalf * kPhiScale));
  t = fminf(fmaxf(t, 0.0f), (float)kPhiN - 0x1p-10f);
  const int i = (int)t;
  const float f = __builtin_amdgcn_fractf(t);  // t - i exactly (t >= 0)
  return fmaf(f, fmaf(f, tab.c2[i], tab.c1[i]), tab.c0[i]);
}

// GELU(x) = x Phi(x) and its derivative Phi(x) + x phi(x).
__device__ __forceinline__ float gelu(float x) { return x * norm_cdf(x); }
__device__ __forceinline__ float gelu_d(float x) {
  return norm_cdf(x) + x * __expf(-0.5f * x * x) * 0.39894228040143268f;
}

// Two values in one hardware conversion (v_cvt_pk_bf16_f32, round to
// nearest even: the same as bf16_bits for finite values), a in the low
// half, b in the high half.
__device__ __forceinline__ unsigned bf16_pair(float a, float b) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f32x2{a, b}, bf16v2));
}

__device__ __forceinline__ bf16x4 pack4(unsigned short a, unsigned short b, unsigned short c,
                                        unsigned short d) {
  bf16x4 v;
  v[0] = (short)a;
  v[1] = (short)b;
  v[2] = (short)c;
  v[3] = (short)d;
  return v;
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// B fragment of W^T for a layer y = W x (W row-major [N][K] FP32): column n,
// rows k0 .. k0+3 are W[n][k0 .. k0+3]; rows n >= nvalid are zero.
__device__ __forceinline__ bf16x4 wt_frag(const float* __restrict__ W, int K, int n, int k0,
                                          int nvalid) {
  if (n >= nvalid) return pack4(0, 0, 0, 0);
  const float* w = W + n * K + k0;
  return pack4(bf16_bits(w[0]), bf16_bits(w[1]), bf16_bits(w[2]), bf16_bits(w[3]));
}

// One dense layer for the 64 samples of a wave.  in: LDS bf16 [64][ins]
// (K inputs); W: FP32 [N][K] (first nvalid rows real, the rest zero); out:
// pre-activations + bias for D element (m, n) go to emit(m, n, value).
template <int K, int NB, class Emit>
__device__ __forceinline__ void wave_layer(const unsigned short* in, int ins,
                                           const float* __restrict__ W, const float* __restrict__ b,
                                           int nvalid, Emit emit) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, q = lane >> 4;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) {
    bf16x4 bw[K / 16];
#pragma unroll
    for (int kb = 0; kb < K / 16; ++kb) bw[kb] = wt_frag(W, K, nb * 16 + r, kb * 16 + 4 * q, nvalid);
    const int n = nb * 16 + r;
    const float bias = n < nvalid ? b[n] : 0.0f;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < K / 16; ++kb) {
        const bf16x4 a = *(const bf16x4*)(in + (mb * 16 + r) * ins + kb * 16 + 4 * q);
        acc = mfma16(a, bw[kb], acc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) emit(mb * 16 + 4 * q + i, n, acc[i] + bias);
    }
  }
}

// LDS row strides (bf16 elements), padded to spread banks.
constexpr int kXs = kMlpIn + 4;
constexpr int kHs = kMlpHid + 4;

// Forward pass of a wave's 64 samples.  X: LDS bf16 [64][kXs] (inputs,
// already rounded); H1, H2: LDS bf16 [64][kHs]; Y: LDS float [64][8].
// If a1/a2 are non-null, pre-activations are also stored there ([64][64]
// float, row = sample).  Every wave of the block must call it (it holds
// block barriers between the layers: lanes read what other lanes wrote).
__device__ __forceinline__ void wave_mlp_forward(const float* __restrict__ P,
                                                 const unsigned short* X, unsigned short* H1,
                                                 unsigned short* H2, float* Y, float* a1,
                                                 float* a2) {
  wave_layer<32, 4>(X, kXs, P + kP_W1, P + kP_B1, 64, [&](int m, int n, float v) {
    if (a1) a1[m * 64 + n] = v;
    H1[m * kHs + n] = bf16_bits(gelu(v));
  });
  __syncthreads();
  wave_layer<64, 4>(H1, kHs, P + kP_W2, P + kP_B2, 64, [&](int m, int n, float v) {
    if (a2) a2[m * 64 + n] = v;
    H2[m * kHs + n] = bf16_bits(gelu(v));
  });
  __syncthreads();
  wave_layer<64, 1>(H2, kHs, P + kP_W3, P + kP_B3, 8, [&](int m, int n, float v) {
    if (n < 8) Y[m * 8 + n] = v;
  });
  __syncthreads();
}

// ---- inference with the activations kept in registers ------------------
// Each layer is computed transposed, H^T = W X^T: the weights are the A
// operand (M = outputs, K = inputs), the samples the B operand (N).  The D
// fragment of output block mb then holds, in lane (r, q), features
// 16 mb + 4q .. 4q+3 of sample r -- exactly the B fragment of the next
// layer's input block kb = mb, so hidden activations never leave the
// registers: bias, GELU and the bf16 rounding happen in place.
//
// Weights are pre-packed (k_mlp_pack, from the FP32 master vector) as bf16
// A fragments: fragment f holds, in lane l = r + 16 q, W[16 mb + r]
// [16 kb + 4q .. 4q+3] (8 bytes), stored [f][64 lanes] so that one wave
// fetches a fragment with one coalesced 512-byte load.  Rows beyond a
// layer's outputs (W3 has 8) are zero.
constexpr int kFragW1 = 0;             // mb 0..3 x kb 0..1
constexpr int kFragW2 = kFragW1 + 8;   // mb 0..3 x kb 0..3
constexpr int kFragW3 = kFragW2 + 16;  // mb 0 x kb 0..3
constexpr int kNumFrags = kFragW3 + 4;
constexpr int kFragBytes = kNumFrags * 64 * 8;

typedef unsigned u32x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ bf16x4 frag_of(const u32x2* __restrict__ W, int f, int lane) {
  return __builtin_bit_cast(bf16x4, W[f * 64 + lane]);
}

// The biases of a lane's 4 D values (features 4q .. 4q+3 of the block),
// the accumulator's start: the matrix core adds them with the products.
__device__ __forceinline__ f32x4 bias4(const float* __restrict__ b) {
  return f32x4{b[0], b[1], b[2], b[3]};
}

// GELU (Phi from the LDS table) of the 4 D values of a lane (bias already
// in), rounded to bf16 in place.
__device__ __forceinline__ bf16x4 act4(f32x4 d, const PhiLds& tab) {
  float g[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) g[i] = d[i] * norm_cdf_tab(tab, d[i]);
  const u32x2 w = {bf16_pair(g[0], g[1]), bf16_pair(g[2], g[3])};
  return __builtin_bit_cast(bf16x4, w);
}

// y = MLP(x) for the 64 samples of a wave.  X: LDS bf16 [64][kXs] (row =
// sample); Y: LDS float [64][8]; tab: the normal CDF table in LDS.
// Wave-local: the caller orders the LDS writes of X and tab before, and the
// reads of Y after, with barriers.
__device__ __forceinline__ void wave_mlp_infer(const u32x2* __restrict__ W,
                                               const float* __restrict__ P,
                                               const unsigned short* X, float* Y,
                                               const PhiLds& tab) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, q = lane >> 4;
#pragma unroll 1
  for (int sb = 0; sb < 4; ++sb) {
    const unsigned short* xr = X + (sb * 16 + r) * kXs + 4 * q;
    const bf16x4 x0 = *(const bf16x4*)(xr), x1 = *(const bf16x4*)(xr + 16);
    bf16x4 h1[4], h2[4];
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      f32x4 acc = bias4(P + kP_B1 + 16 * mb + 4 * q);
      acc = mfma16(frag_of(W, kFragW1 + 2 * mb, lane), x0, acc);
      acc = mfma16(frag_of(W, kFragW1 + 2 * mb + 1, lane), x1, acc);
      h1[mb] = act4(acc, tab);
    }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      f32x4 acc = bias4(P + kP_B2 + 16 * mb + 4 * q);
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) acc = mfma16(frag_of(W, kFragW2 + 4 * mb + kb, lane), h1[kb], acc);
      h2[mb] = act4(acc, tab);
    }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) acc = mfma16(frag_of(W, kFragW3 + kb, lane), h2[kb], acc);
    if (q < 2) {
      float* y = Y + (sb * 16 + r) * 8 + 4 * q;
#pragma unroll
      for (int i = 0; i < 4; ++i) y[i] = acc[i] + P[kP_B3 + 4 * q + i];
    }
  }
}

// ---- face features and the output <-> flux maps ------------------------
// w8 = rho, vn, vt1, vt2, P, Bn, Bt1, Bt2 of cells i-2 .. i+1 (face i-1/2),
// cell-centred, face-normal frame.  Face means rho_m, v_m, P_m of cells i-1,
// i; c_m = sqrt(gamma P_m / rho_m).

struct FaceScale {
  float rm, cm, sr;  // rho_m, c_m, sqrt(rho_m)
  float vm[3];
};

__device__ __forceinline__ FaceScale face_scale(const float w8[32], float gam) {
  FaceScale s;
  s.rm = 0.5f * (w8[8] + w8[16]);
  for (int d = 0; d < 3; ++d) s.vm[d] = 0.5f * (w8[9 + d] + w8[17 + d]);
  s.cm = __builtin_amdgcn_sqrtf(gam * 0.5f * (w8[12] + w8[20]) / s.rm);
  s.sr = __builtin_amdgcn_sqrtf(s.rm);
  return s;
}

// x = rho/rho_m, (v - v_m)/c_m, P/(rho_m c_m^2), B/(sqrt(rho_m) c_m) per cell.
__device__ __forceinline__ void face_features(const float w8[32], const FaceScale& s,
                                              float x[32]) {
  const float ir = 1.0f / s.rm, ic = 1.0f / s.cm;
  const float ip = ir * ic * ic, ib = ic / s.sr;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const float* w = w8 + 8 * c;
    float* o = x + 8 * c;
    o[0] = w[0] * ir;
    for (int d = 0; d < 3; ++d) o[1 + d] = (w[1 + d] - s.vm[d]) * ic;
    o[4] = w[4] * ip;
    for (int d = 0; d < 3; ++d) o[5 + d] = w[5 + d] * ib;
  }
}

// y (8 outputs) -> flux correction in the face frame (rho, Mn, Mt1, Mt2, E,
// Bt1, Bt2): rho_m c_m, rho_m c_m^2, rho_m c_m^3, sqrt(rho_m) c_m^2 scales and
// the Galilean shift by v_m of the momentum and energy rows; y[5] unused.
__device__ __forceinline__ void out_to_flux(const FaceScale& s, const float y[8], float df[7]) {
  const float fr = s.rm * s.cm * y[0];
  const float k2 = s.rm * s.cm * s.cm;
  const float fm0 = k2 * y[1], fm1 = k2 * y[2], fm2 = k2 * y[3];
  const float fe = k2 * s.cm * y[4];
  const float v2 = s.vm[0] * s.vm[0] + s.vm[1] * s.vm[1] + s.vm[2] * s.vm[2];
  df[0] = fr;
  df[1] = fm0 + s.vm[0] * fr;
  df[2] = fm1 + s.vm[1] * fr;
  df[3] = fm2 + s.vm[2] * fr;
  df[4] = fe + (s.vm[0] * fm0 + s.vm[1] * fm1 + s.vm[2] * fm2) + 0.5f * v2 * fr;
  const float kb = s.sr * s.cm * s.cm;
  df[5] = kb * y[6];
  df[6] = kb * y[7];
}

__device__ __forceinline__ void flux_to_out(const FaceScale& s, const float df[7], float y[8]) {
  const float fr = df[0];
  const float fm0 = df[1] - s.vm[0] * fr, fm1 = df[2] - s.vm[1] * fr, fm2 = df[3] - s.vm[2] * fr;
  const float v2 = s.vm[0] * s.vm[0] + s.vm[1] * s.vm[1] + s.vm[2] * s.vm[2];
  const float fe = df[4] - (s.vm[0] * fm0 + s.vm[1] * fm1 + s.vm[2] * fm2) - 0.5f * v2 * fr;
  const float k2 = s.rm * s.cm * s.cm;
  y[0] = fr / (s.rm * s.cm);
  y[1] = fm0 / k2;
  y[2] = fm1 / k2;
  y[3] = fm2 / k2;
  y[4] = fe / (k2 * s.cm);
  y[5] = 0.0f;
  const float kb = s.sr * s.cm * s.cm;
  y[6] = df[5] / kb;
  y[7] = df[6] / kb;
}

}  // namespace mhd
