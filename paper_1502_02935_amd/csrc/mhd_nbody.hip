// mhd_nbody.hip -- N-body particles of the step (section 2.1 of the paper:
// particle-in-cell dynamics with the "flip-flop" integrator, a
// mass-conserving second-order mass assignment), sharing the periodic
// potential of the self-gravity solve.
//
// Cloud in cell: a particle is a cube of one cell's size; along each axis,
// in cell-centre units s = (x - x0)/d - 1/2, it overlaps cells floor(s)
// and floor(s) + 1 (periodic) with fractions 1 - f and f, f = s - floor(s).
// The deposit adds m w_x w_y w_z / dV to each of the 8 cells (atomic adds,
// so the rounding order of a cell's sum varies from run to run); the force
// is minus the cell-centred central gradient of Psi interpolated with the
// same weights, which keeps the total momentum.
//
// One thread per particle, a grid-stride loop; positions and velocities are
// [3][n] rows, so a wave's loads of one component are contiguous.
#include <math.h>

#include "mhd_span.hpp"

namespace mhd {

constexpr int kPartThreads = 256;

static unsigned part_blocks(long long n) {
  const long long b = (n + kPartThreads - 1) / kPartThreads;
  return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

template <class T>
__device__ __forceinline__ T wrap_coord(T x, double lo, double L) {
  return (T)((double)x - L * floor(((double)x - lo) / L));
}

// Weights of one axis: cells c[0], c[1] (interior indices), fractions w.
template <class T>
__device__ __forceinline__ void cic_axis(const Geo& g, int a, T x, int c[2], T w[2]) {
  const T s = (x - (T)g.x0[a]) / (T)g.d[a] - T(0.5);
  const T fl = floor(s);
  const int n = g.n[a];
  int c0 = (int)fl % n;
  if (c0 < 0) c0 += n;
  c[0] = c0;
  c[1] = c0 + 1 < n ? c0 + 1 : 0;
  w[1] = s - fl;
  w[0] = T(1) - w[1];
}

__device__ __forceinline__ void atomic_add_t(double* p, double v) { atomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_t(float* p, float v) { atomicAdd(p, v); }

template <class T>
__global__ void __launch_bounds__(kPartThreads) k_deposit(Geo g, Parts<T> pp, DtRef hr, T* c) {
  const double h = (hr.ptr ? *hr.ptr : hr.value) * hr.factor;
  const T idv = (T)(1.0 / (g.d[0] * g.d[1] * g.d[2]));
  const long long n = pp.n;
  for (long long q = (long long)blockIdx.x * kPartThreads + threadIdx.x; q < n;
       q += (long long)gridDim.x * kPartThreads) {
    int ci[3][2];
    T w[3][2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T x = pp.x[a * n + q];
      if (h != 0.0) x = wrap_coord<T>(x + (T)h * pp.v[a * n + q], g.x0[a], g.n[a] * g.d[a]);
      cic_axis<T>(g, a, x, ci[a], w[a]);
    }
    const T m = pp.m[q];
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const long cell = ((long)ci[2][e] * g.n[1] + ci[1][b]) * g.n[0] + ci[0][a];
          atomic_add_t(c + 2 * cell, m * w[0][a] * w[1][b] * w[2][e] * idv);
        }
  }
}

template <class T>
__global__ void __launch_bounds__(kPartThreads) k_kick_drift(Geo g, Parts<T> pp, Grav<T> gr,
                                                             DtRef dtr) {
  const double dt = (dtr.ptr ? *dtr.ptr : dtr.value) * dtr.factor;
  const T hdt = (T)(0.5 * dt), Tdt = (T)dt;
  const long long n = pp.n;
  for (long long q = (long long)blockIdx.x * kPartThreads + threadIdx.x; q < n;
       q += (long long)gridDim.x * kPartThreads) {
    T xh[3];
    int ci[3][2];
    T w[3][2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      xh[a] = wrap_coord<T>(pp.x[a * n + q] + hdt * pp.v[a * n + q], g.x0[a], g.n[a] * g.d[a]);
      cic_axis<T>(g, a, xh[a], ci[a], w[a]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const T* G = gr.g[a];
      T acc = T(0);
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int i = 0; i < 2; ++i)
            acc += w[0][i] * w[1][b] * w[2][e] *
                   G[(ci[0][i] + NG) + g.sy * (ci[1][b] + NG) + g.sz * (ci[2][e] + NG)];
      const T v = pp.v[a * n + q] - Tdt * acc;
      pp.v[a * n + q] = v;
      pp.x[a * n + q] = wrap_coord<T>(xh[a] + hdt * v, g.x0[a], g.n[a] * g.d[a]);
    }
  }
}

template <class T>
__global__ void __launch_bounds__(kPartThreads) k_wrap_positions(Geo g, Parts<T> pp) {
  const long long n = pp.n;
  for (long long q = (long long)blockIdx.x * kPartThreads + threadIdx.x; q < n;
       q += (long long)gridDim.x * kPartThreads)
#pragma unroll
    for (int a = 0; a < 3; ++a)
      pp.x[a * n + q] = wrap_coord<T>(pp.x[a * n + q], g.x0[a], g.n[a] * g.d[a]);
}

// Block minimum of d_a / |v_a| over the particles into part[blockIdx.x]
// (kPartCflBlocks blocks, grid-stride).
template <class T>
__global__ void __launch_bounds__(kPartThreads) k_particle_cfl(Geo g, Parts<T> pp, double* part) {
  __shared__ double red[kPartThreads / 64];
  const long long n = pp.n;
  double r = INFINITY;
  for (long long q = (long long)blockIdx.x * kPartThreads + threadIdx.x; q < n;
       q += (long long)gridDim.x * kPartThreads)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double v = fabs((double)pp.v[a * n + q]);
      if (v > 0.0) r = fmin(r, g.d[a] / v);
    }
  for (int off = 32; off > 0; off >>= 1) r = fmin(r, __shfl_xor(r, off, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int wv = 1; wv < kPartThreads / 64; ++wv) m = fmin(m, red[wv]);
    part[blockIdx.x] = m;
  }
}

template <class T>
void launch_particle_cfl(const Geo& g, Parts<T> pp, double* part, hipStream_t st) {
  hipLaunchKernelGGL(k_particle_cfl<T>, dim3(kPartCflBlocks), dim3(kPartThreads), 0, st, g, pp,
                     part);
}

template <class T>
void launch_deposit(const Geo& g, Parts<T> pp, DtRef h, T* c, hipStream_t st) {
  if (pp.n <= 0) return;
  hipLaunchKernelGGL(k_deposit<T>, dim3(part_blocks(pp.n)), dim3(kPartThreads), 0, st, g, pp, h,
                     c);
}

template <class T>
void launch_kick_drift(const Geo& g, Parts<T> pp, Grav<T> gr, DtRef dt, hipStream_t st) {
  if (pp.n <= 0) return;
  hipLaunchKernelGGL(k_kick_drift<T>, dim3(part_blocks(pp.n)), dim3(kPartThreads), 0, st, g, pp,
                     gr, dt);
}

template <class T>
void launch_wrap_positions(const Geo& g, Parts<T> pp, hipStream_t st) {
  if (pp.n <= 0) return;
  hipLaunchKernelGGL(k_wrap_positions<T>, dim3(part_blocks(pp.n)), dim3(kPartThreads), 0, st, g,
                     pp);
}

#define MHD_NBODY_INST(T)                                                                        \
  template void launch_particle_cfl<T>(const Geo&, Parts<T>, double*, hipStream_t);             \
  template void launch_deposit<T>(const Geo&, Parts<T>, DtRef, T*, hipStream_t);                \
  template void launch_kick_drift<T>(const Geo&, Parts<T>, Grav<T>, DtRef, hipStream_t);        \
  template void launch_wrap_positions<T>(const Geo&, Parts<T>, hipStream_t);

MHD_NBODY_INST(double)
MHD_NBODY_INST(float)

}  // namespace mhd
