// mhd_mlp.hip -- training-side kernels of the learned flux correction:
// batched forward, fused MSE loss + backward on the matrix cores with
// per-block partial gradients and a fixed-order reduction, Adam, and the
// data pipeline (2x coarse-graining of a fine state, accumulation of
// time-weighted fine fluxes on coarse faces, feature/target extraction).
#include <math.h>

#include "mhd_kernels.hpp"
#include "mhd_mlp.hpp"
#include "mhd_span.hpp"

namespace mhd {

// LDS of one wave for the forward/backward kernels (one wave per block).
struct MlpLds {
  unsigned short X[64 * kXs];
  unsigned short H1[64 * kHs];
  unsigned short H2[64 * kHs];
  float Y[64 * 8];
  float A1[64 * 64];   // pre-activations, later dz1 (FP32)
  float A2[64 * 64];   // pre-activations, later dz2 (FP32)
  unsigned short D3[64 * 20];   // dz3 bf16, columns 8..15 zero
  unsigned short D2[64 * kHs];  // dz2 bf16
  unsigned short D1[64 * kHs];  // dz1 bf16
  float D3f[64 * 8];            // dz3 FP32
};

struct MlpFwdLds {
  unsigned short X[64 * kXs];
  unsigned short H1[64 * kHs];
  unsigned short H2[64 * kHs];
  float Y[64 * 8];
};

__device__ __forceinline__ void load_inputs(unsigned short* X, const float* __restrict__ x,
                                            int64_t n, int64_t base) {
  const int lane = threadIdx.x;
  const int64_t b = base + lane;
#pragma unroll
  for (int c = 0; c < 32; ++c)
    X[lane * kXs + c] = b < n ? bf16_bits(x[b * 32 + c]) : (unsigned short)0;
}

__global__ void __launch_bounds__(64) k_mlp_forward(int64_t n, const float* __restrict__ x,
                                                    const float* __restrict__ P, float* y) {
  __shared__ MlpFwdLds s;
  const int64_t base = (int64_t)blockIdx.x * 64;
  load_inputs(s.X, x, n, base);
  __syncthreads();
  wave_mlp_forward(P, s.X, s.H1, s.H2, s.Y, nullptr, nullptr);
  const int64_t b = base + threadIdx.x;
  if (b < n)
#pragma unroll
    for (int o = 0; o < 8; ++o) y[b * 8 + o] = s.Y[threadIdx.x * 8 + o];
}

// Weights of P as the bf16 A fragments of wave_mlp_infer: block f packs
// fragment f, lane l the 4 weights that lane l holds.
__global__ void __launch_bounds__(64) k_mlp_pack(const float* __restrict__ P, u32x2* W) {
  const int f = blockIdx.x, lane = threadIdx.x, r = lane & 15, q = lane >> 4;
  int off, K, M, mb, kb;
  if (f < kFragW2) {
    off = kP_W1, K = kMlpIn, M = kMlpHid, mb = f / 2, kb = f % 2;
  } else if (f < kFragW3) {
    off = kP_W2, K = kMlpHid, M = kMlpHid, mb = (f - kFragW2) / 4, kb = (f - kFragW2) % 4;
  } else {
    off = kP_W3, K = kMlpHid, M = kMlpOut, mb = 0, kb = f - kFragW3;
  }
  const int row = 16 * mb + r, col = 16 * kb + 4 * q;
  unsigned v[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) v[i] = row < M ? bf16_bits(P[off + row * K + col + i]) : 0u;
  W[f * 64 + lane] = u32x2{v[0] | (v[1] << 16), v[2] | (v[3] << 16)};
}

void launch_mlp_pack(const float* P, unsigned* frags, hipStream_t st) {
  static_assert(kMlpFragBytes == kFragBytes, "fragment buffer size");
  hipLaunchKernelGGL(k_mlp_pack, dim3(kNumFrags), dim3(64), 0, st, P, (u32x2*)frags);
}

// Sum over the 64 samples (rows) of a [64][64] FP32 LDS matrix, column =
// lane.
__device__ __forceinline__ float col_sum(const float* m, int ld) {
  float a = 0.f;
  for (int r = 0; r < 64; ++r) a += m[r * ld + threadIdx.x];
  return a;
}

// Loss L = mean over samples and the 8 outputs of (y - t)^2 and its
// gradient, for the 64 samples of this block; partial gradients (param
// order) and the partial loss go to part[block][kMlpParams + 1].
__global__ void __launch_bounds__(64) k_mlp_grad(int64_t n, const float* __restrict__ x,
                                                 const float* __restrict__ t,
                                                 const float* __restrict__ P, float* part) {
  __shared__ MlpLds s;
  const int lane = threadIdx.x;
  const int r = lane & 15, q = lane >> 4;
  const int64_t base = (int64_t)blockIdx.x * 64;
  const int64_t b = base + lane;
  float* out = part + (size_t)blockIdx.x * (kMlpParams + 1);
  load_inputs(s.X, x, n, base);
  __syncthreads();
  wave_mlp_forward(P, s.X, s.H1, s.H2, s.Y, s.A1, s.A2);
  // dL/dy
  const float scale = 2.0f / (float)(n * 8);
  float loss = 0.f;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const float e = b < n ? s.Y[lane * 8 + o] - t[b * 8 + o] : 0.f;
    loss += e * e;
    const float d = e * scale;
    s.D3f[lane * 8 + o] = d;
    s.D3[lane * 20 + o] = bf16_bits(d);
    s.D3[lane * 20 + 8 + o] = 0;
  }
  for (int o = 16; o < 20; ++o) s.D3[lane * 20 + o] = 0;
  __syncthreads();
  // db3
  if (lane < 8) {
    float a = 0.f;
    for (int rr = 0; rr < 64; ++rr) a += s.D3f[rr * 8 + lane];
    out[kP_B3 + lane] = a;
  }
  // dW3[o][j] = sum_s dz3[s][o] h2[s][j]   (M = o padded to 16, N = j, K = s)
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const int s0 = kb * 16 + 4 * q;
      const bf16x4 a = pack4(s.D3[(s0 + 0) * 20 + r], s.D3[(s0 + 1) * 20 + r],
                             s.D3[(s0 + 2) * 20 + r], s.D3[(s0 + 3) * 20 + r]);
      const int j = nb * 16 + r;
      const bf16x4 bb = pack4(s.H2[(s0 + 0) * kHs + j], s.H2[(s0 + 1) * kHs + j],
                              s.H2[(s0 + 2) * kHs + j], s.H2[(s0 + 3) * kHs + j]);
      acc = mfma16(a, bb, acc);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int o = 4 * q + i, j = nb * 16 + r;
      if (o < 8) out[kP_W3 + o * 64 + j] = acc[i];
    }
  }
  // dh2[s][j] = sum_o dz3[s][o] W3[o][j]; dz2 = dh2 gelu'(a2)
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int j = nb * 16 + r;
    bf16x4 bw;
    {
      unsigned short v[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int o = 4 * q + i;
        v[i] = o < 8 ? bf16_bits(P[kP_W3 + o * 64 + j]) : (unsigned short)0;
      }
      bw = pack4(v[0], v[1], v[2], v[3]);
    }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      const bf16x4 a = *(const bf16x4*)(s.D3 + (mb * 16 + r) * 20 + 4 * q);
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
      acc = mfma16(a, bw, acc);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int sm = mb * 16 + 4 * q + i;
        const float dz = acc[i] * gelu_d(s.A2[sm * 64 + j]);
        s.A2[sm * 64 + j] = dz;
        s.D2[sm * kHs + j] = bf16_bits(dz);
      }
    }
  }
  __syncthreads();
  out[kP_B2 + lane] = col_sum(s.A2, 64);
  // dW2[i][j] = sum_s dz2[s][i] h1[s][j]
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < 4; ++nb) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const int s0 = kb * 16 + 4 * q;
        const int i0 = mb * 16 + r, j = nb * 16 + r;
        const bf16x4 a = pack4(s.D2[(s0 + 0) * kHs + i0], s.D2[(s0 + 1) * kHs + i0],
                               s.D2[(s0 + 2) * kHs + i0], s.D2[(s0 + 3) * kHs + i0]);
        const bf16x4 bb = pack4(s.H1[(s0 + 0) * kHs + j], s.H1[(s0 + 1) * kHs + j],
                                s.H1[(s0 + 2) * kHs + j], s.H1[(s0 + 3) * kHs + j]);
        acc = mfma16(a, bb, acc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) out[kP_W2 + (mb * 16 + 4 * q + i) * 64 + nb * 16 + r] = acc[i];
    }
  // dh1[s][j] = sum_i dz2[s][i] W2[i][j]; dz1 = dh1 gelu'(a1)
#pragma unroll
  for (int nb = 0; nb < 4; ++nb) {
    const int j = nb * 16 + r;
    bf16x4 bw[4];
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
      const int i0 = kb * 16 + 4 * q;
      bw[kb] = pack4(bf16_bits(P[kP_W2 + (i0 + 0) * 64 + j]), bf16_bits(P[kP_W2 + (i0 + 1) * 64 + j]),
                     bf16_bits(P[kP_W2 + (i0 + 2) * 64 + j]), bf16_bits(P[kP_W2 + (i0 + 3) * 64 + j]));
    }
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const bf16x4 a = *(const bf16x4*)(s.D2 + (mb * 16 + r) * kHs + kb * 16 + 4 * q);
        acc = mfma16(a, bw[kb], acc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int sm = mb * 16 + 4 * q + i;
        const float dz = acc[i] * gelu_d(s.A1[sm * 64 + j]);
        s.A1[sm * 64 + j] = dz;
        s.D1[sm * kHs + j] = bf16_bits(dz);
      }
    }
  }
  __syncthreads();
  out[kP_B1 + lane] = col_sum(s.A1, 64);
  // dW1[i][c] = sum_s dz1[s][i] x[s][c]
#pragma unroll
  for (int mb = 0; mb < 4; ++mb)
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < 4; ++kb) {
        const int s0 = kb * 16 + 4 * q;
        const int i0 = mb * 16 + r, c = nb * 16 + r;
        const bf16x4 a = pack4(s.D1[(s0 + 0) * kHs + i0], s.D1[(s0 + 1) * kHs + i0],
                               s.D1[(s0 + 2) * kHs + i0], s.D1[(s0 + 3) * kHs + i0]);
        const bf16x4 bb = pack4(s.X[(s0 + 0) * kXs + c], s.X[(s0 + 1) * kXs + c],
                                s.X[(s0 + 2) * kXs + c], s.X[(s0 + 3) * kXs + c]);
        acc = mfma16(a, bb, acc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) out[kP_W1 + (mb * 16 + 4 * q + i) * 32 + nb * 16 + r] = acc[i];
    }
  // loss of this block
  __shared__ float red[64];
  red[lane] = loss;
  __syncthreads();
  if (lane == 0) {
    float a = 0.f;
    for (int i = 0; i < 64; ++i) a += red[i];
    out[kMlpParams] = a / (float)(n * 8);
  }
}

// grad[p] = sum over blocks (fixed order); loss likewise.
__global__ void k_mlp_reduce(int nblocks, const float* part, float* grad, float* loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > kMlpParams) return;
  float a = 0.f;
  for (int b = 0; b < nblocks; ++b) a += part[(size_t)b * (kMlpParams + 1) + p];
  if (p < kMlpParams)
    grad[p] = a;
  else if (loss)
    *loss = a;
}

__global__ void k_mlp_adam(float* P, float* m, float* v, const float* g, float lr, float b1,
                           float b2, float eps, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kMlpParams) return;
  const float gp = g[p];
  const float mp = b1 * m[p] + (1.f - b1) * gp;
  const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
  m[p] = mp;
  v[p] = vp;
  P[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

void launch_mlp_forward(int64_t n, const float* x, const float* P, float* y, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, st, n, x, P, y);
}

size_t mlp_grad_workspace(int64_t n) {
  return (size_t)((n + 63) / 64) * (kMlpParams + 1) * sizeof(float);
}

void launch_mlp_grad(int64_t n, const float* x, const float* t, const float* P, float* grad,
                     float* loss, float* part, hipStream_t st) {
  const int nb = (int)((n + 63) / 64);
  hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(64), 0, st, n, x, t, P, part);
  hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 1 + 255) / 256), dim3(256), 0, st, nb, part,
                     grad, loss);
}

void launch_mlp_adam(float* P, float* m, float* v, const float* g, int64_t step, double lr,
                     double b1, double b2, double eps, hipStream_t st) {
  const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
  hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, st, P, m, v, g,
                     (float)lr, (float)b1, (float)b2, (float)eps, (float)c1, (float)c2);
}

// ------------------------------------------------------------------------
// Data pipeline.
// ------------------------------------------------------------------------

__device__ __forceinline__ int pidx2(const Geo& g, int i, int j, int k) {
  return (i + NG) + g.sy * (j + NG) + g.sz * (k + NG);
}

// acc[a][m][K][J][I] += dt * mean of the 2x2 fine a-faces tiling coarse
// a-face (I, J, K), frame components m = 0..6 of the fine corrector flux:
// the faces at the lower sides of the coarse cells (on a non-periodic axis
// the last boundary face is not accumulated).
template <class T>
__global__ void k_fluxacc(Geo g, Flux<T> f, T* acc, DtRef dtr) {
  const int I = blockIdx.x * 64 + threadIdx.x;
  const int J = blockIdx.y;
  const int K = blockIdx.z;
  const int nc[3] = {g.n[0] / 2, g.n[1] / 2, g.n[2] / 2};
  if (I >= nc[0]) return;
  const T dt = (T)((dtr.ptr ? *dtr.ptr : dtr.value) * dtr.factor);
  const size_t ncell = (size_t)nc[0] * nc[1] * nc[2];
  const size_t cidx = ((size_t)K * nc[1] + J) * nc[0] + I;
  const int C[3] = {2 * I, 2 * J, 2 * K};
  const int st[3] = {1, g.sy, g.sz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int t1 = (a + 1) % 3, t2 = (a + 2) % 3;
    const int p0 = pidx2(g, C[0], C[1], C[2]);
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      const T* F = f.f[a][m];
      const T s4 = F[p0] + F[p0 + st[t1]] + F[p0 + st[t2]] + F[p0 + st[t1] + st[t2]];
      acc[((size_t)a * 7 + m) * ncell + cidx] += dt * T(0.25) * s4;
    }
  }
}

template <class T>
void launch_fluxacc(const Geo& g, Flux<T> f, T* acc, DtRef dt, hipStream_t st) {
  hipLaunchKernelGGL(k_fluxacc<T>, dim3((unsigned)((g.n[0] / 2 + 63) / 64), (unsigned)(g.n[1] / 2),
                                        (unsigned)(g.n[2] / 2)),
                     dim3(64), 0, st, g, f, acc, dt);
}

// 2x coarse-graining of the interior state into interior-layout arrays:
// cells are the means of their 2^3 fine cells, faces the means of the 2^2
// fine faces tiling them.  A non-periodic axis has n/2 + 1 coarse faces
// along it (the last one tiled by the fine boundary faces), so the launch
// covers I, J, K in 0..n/2.
template <class T>
__global__ void k_coarsen(Geo g, Cons<T> s, T* cell5, T* bx, T* by, T* bz) {
  const int I = blockIdx.x * 64 + threadIdx.x;
  const int J = blockIdx.y, K = blockIdx.z;
  const int nc[3] = {g.n[0] / 2, g.n[1] / 2, g.n[2] / 2};
  int nfc[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) nfc[a] = g.nf[a] > g.n[a] ? nc[a] + 1 : nc[a];
  if (I > nc[0]) return;
  const int C[3] = {I, J, K};
  const int p0 = pidx2(g, 2 * I, 2 * J, 2 * K);
  const int st[3] = {1, g.sy, g.sz};
  if (I < nc[0] && J < nc[1] && K < nc[2]) {
    const size_t ncell = (size_t)nc[0] * nc[1] * nc[2];
    const size_t q = ((size_t)K * nc[1] + J) * nc[0] + I;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      T a = T(0);
      for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
          for (int dx = 0; dx < 2; ++dx) a += s.u[m][p0 + dx + dy * g.sy + dz * g.sz];
      cell5[m * ncell + q] = T(0.125) * a;
    }
  }
  T* out[3] = {bx, by, bz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int t1 = (a + 1) % 3, t2 = (a + 2) % 3;
    if (C[a] >= nfc[a] || C[t1] >= nc[t1] || C[t2] >= nc[t2]) continue;
    // face array a: extents nfc[a] along a, nc across, x fastest
    int ext[3] = {nc[0], nc[1], nc[2]};
    ext[a] = nfc[a];
    const size_t q = ((size_t)K * ext[1] + J) * ext[0] + I;
    const T* B = s.b[a];
    out[a][q] = T(0.25) * (B[p0] + B[p0 + st[t1]] + B[p0 + st[t2]] + B[p0 + st[t1] + st[t2]]);
  }
}

template <class T>
void launch_coarsen(const Geo& g, Cons<T> s, T* c5, T* bx, T* by, T* bz, hipStream_t st) {
  hipLaunchKernelGGL(k_coarsen<T>, dim3((unsigned)((g.n[0] / 2 + 1 + 63) / 64),
                                        (unsigned)(g.n[1] / 2 + 1), (unsigned)(g.n[2] / 2 + 1)),
                     dim3(64), 0, st, g, s, c5, bx, by, bz);
}

// Features of the corrector state W* and targets flux_to_out(F_fine - F)
// for n faces (axis, i, j, k); mask = 1 where a face touches a shock cell.
template <class T>
__global__ void k_mlp_samples(Geo g, Prim<T> w, Flux<T> f, const uint8_t* shock, const T* acc,
                              double dt_c, float gam, int64_t n, const int32_t* faces, float* x,
                              float* t, uint8_t* mask) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n) return;
  const int a = faces[4 * b], i = faces[4 * b + 1], j = faces[4 * b + 2], k = faces[4 * b + 3];
  if (a < 0 || a > 2 || i < 0 || i >= g.n[0] || j < 0 || j >= g.n[1] || k < 0 || k >= g.n[2]) {
    // not the lower face of an interior cell: no access, flagged
    for (int c = 0; c < 32; ++c) x[b * 32 + c] = 0.f;
    for (int o = 0; o < 8; ++o) t[b * 8 + o] = 0.f;
    mask[b] = 2;
    return;
  }
  const int t1 = (a + 1) % 3, t2 = (a + 2) % 3;
  const int s = a == 0 ? 1 : (a == 1 ? g.sy : g.sz);
  const int p = pidx2(g, i, j, k);
  // cells 2 below .. 1 above the face's upper cell, wrapped onto the
  // interior images along a periodic axis (a fully periodic step leaves
  // the ghost layers unfilled)
  const int ci = a == 0 ? i : (a == 1 ? j : k);
  int so[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) so[c] = (int)axis_step(g, a, ci, c - 2) * s;
  float w8[32];
  const T* src[8] = {w.w[0], w.w[1 + a], w.w[1 + t1], w.w[1 + t2],
                     w.w[4], w.w[5 + a], w.w[5 + t1], w.w[5 + t2]};
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int v = 0; v < 8; ++v) w8[8 * c + v] = (float)src[v][p + so[c]];
  const FaceScale sc = face_scale(w8, gam);
  float xf[32];
  face_features(w8, sc, xf);
#pragma unroll
  for (int c = 0; c < 32; ++c) x[b * 32 + c] = xf[c];
  const int nc[3] = {g.n[0], g.n[1], g.n[2]};
  const size_t ncell = (size_t)nc[0] * nc[1] * nc[2];
  const size_t cidx = ((size_t)k * nc[1] + j) * nc[0] + i;
  float df[7], y[8];
#pragma unroll
  for (int m = 0; m < 7; ++m)
    df[m] = (float)((double)acc[((size_t)a * 7 + m) * ncell + cidx] / dt_c - (double)f.f[a][m][p]);
  flux_to_out(sc, df, y);
#pragma unroll
  for (int o = 0; o < 8; ++o) t[b * 8 + o] = y[o];
  mask[b] = (shock[p + so[1]] || shock[p]) ? 1 : 0;
}

template <class T>
void launch_mlp_samples(const Geo& g, Prim<T> w, Flux<T> f, const uint8_t* shock, const T* acc,
                        double dt_c, double gam, int64_t n, const int32_t* faces, float* x,
                        float* t, uint8_t* mask, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_mlp_samples<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, w,
                     f, shock, acc, dt_c, (float)gam, n, faces, x, t, mask);
}

#define MHD_MLP_INST(T)                                                                          \
  template void launch_fluxacc<T>(const Geo&, Flux<T>, T*, DtRef, hipStream_t);                 \
  template void launch_coarsen<T>(const Geo&, Cons<T>, T*, T*, T*, T*, hipStream_t);            \
  template void launch_mlp_samples<T>(const Geo&, Prim<T>, Flux<T>, const uint8_t*, const T*,   \
                                      double, double, int64_t, const int32_t*, float*, float*,  \
                                      uint8_t*, hipStream_t);

MHD_MLP_INST(double)
MHD_MLP_INST(float)

}  // namespace mhd
