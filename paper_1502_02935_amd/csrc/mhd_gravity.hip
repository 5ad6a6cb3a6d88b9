// mhd_gravity.hip -- self-gravity source of the step (the paper's Poisson
// equation Lap Psi = 4 pi G rho, section 2.1, "FFT-based" solver), on a
// periodic box, where only rho - <rho> can source the potential.
//
// Per stage: the stage density goes into a complex array [nz][ny][nx];
// batched radix-2 FFTs along x, y and z; each mode is divided by the
// eigenvalue of the 7-point Laplacian (times 4 pi G / N, the mean mode set
// to zero); inverse FFTs; Psi and its central gradient (periodic wrap) land
// in padded arrays that the update reads for S = (0, -rho grad Psi,
// -rho v.grad Psi, 0).  Extents are powers of two up to 1024.
//
// FFT lines: a block takes a tile of lines of one axis into LDS, splits
// each line's n = R1 R2 points into R2 DFTs of R1 points and R1 DFTs of R2
// points done in registers (two LDS passes), and writes the result out.
// x-lines are contiguous; y- and z-lines are tiled over consecutive x, so
// each element row of a tile is one contiguous run in HBM.
#include <math.h>

#include "mhd_kernels.hpp"

namespace mhd {

constexpr int kFftThreads = 256;
constexpr int kFftTileElems = 4096;  // complex values per block tile (LDS)

template <class T>
struct Cplx {
  T re, im;
};

// Interior index of cell (i, j, k) in [nz][ny][nx].
__device__ __forceinline__ long cidx(const Geo& g, int i, int j, int k) {
  return ((long)k * g.n[1] + j) * g.n[0] + i;
}

// The source density: the stage's gas density, or zero for a gas that is
// decoupled from gravity (particles only; they are added by the deposit).
template <class T>
__global__ void __launch_bounds__(256) k_grav_load(Geo g, const T* __restrict__ rho, Cplx<T>* c,
                                                   int with_gas) {
  const long q = (long)blockIdx.x * 256 + threadIdx.x;
  const long N = (long)g.n[0] * g.n[1] * g.n[2];
  if (q >= N) return;
  const int i = (int)(q % g.n[0]);
  const int j = (int)((q / g.n[0]) % g.n[1]);
  const int k = (int)(q / ((long)g.n[0] * g.n[1]));
  c[q] = Cplx<T>{with_gas ? rho[(i + NG) + g.sy * (j + NG) + g.sz * (k + NG)] : T(0), T(0)};
}

// In-register DFT of R points (R a power of two): the radix-2
// decimation-in-time butterflies, fully unrolled.  tw: n/2 values
// exp(-2 pi i q / n) (n a multiple of R); W_R^j = tw[j n / R]; sign -1
// forward, +1 inverse (conjugate twiddles).
template <int R>
__device__ constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) r = (r << 1) | ((i & b) ? 1 : 0);
  return r;
}

template <class T, int R>
__device__ __forceinline__ void dft_reg(Cplx<T> a[R], const Cplx<T>* __restrict__ tw, int n,
                                        int sign) {
  Cplx<T> b[R];
#pragma unroll
  for (int i = 0; i < R; ++i) b[bitrev<R>(i)] = a[i];
#pragma unroll
  for (int m = 1; m < R; m <<= 1) {
#pragma unroll
    for (int j = 0; j < m; ++j) {
      Cplx<T> w{T(1), T(0)};
      if (j > 0) {
        w = tw[j * (n / (2 * m))];
        if (sign > 0) w.im = -w.im;
      }
#pragma unroll
      for (int k = j; k < R; k += 2 * m) {
        const Cplx<T> u = b[k], v = b[k + m];
        T vr = v.re, vi = v.im;
        if (j > 0) {
          vr = v.re * w.re - v.im * w.im;
          vi = v.re * w.im + v.im * w.re;
        }
        b[k] = Cplx<T>{u.re + vr, u.im + vi};
        b[k + m] = Cplx<T>{u.re - vr, u.im - vi};
      }
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) a[i] = b[i];
}

// Batched FFT of all lines along axis A of c ([nz][ny][nx]) of n = R1 R2
// points: the "four-step" split within a block.  A tile of tl lines goes
// to LDS (line stride n + 1 complex values, so lines do not share banks);
// step 1: for each n2 < R2, an R1-point DFT over x[R2 n1 + n2], times
// W_n^(n2 k1), back in place; step 2: for each k1 < R1, an R2-point DFT
// over the R2 contiguous values, written to element k1 + R1 k2 of the line
// in HBM.  Two LDS passes and two barriers instead of log2(n) radix-2
// stages.  Threads take consecutive elements of a line (x-lines) or
// consecutive lines (y-, z-lines, tiled over consecutive x), so every HBM
// access of a wave is contiguous.  sign -1 forward, +1 inverse
// (unnormalised).
template <class T, int A, int R1, int R2>
__global__ void __launch_bounds__(kFftThreads) k_fft(Geo g, Cplx<T>* c, const Cplx<T>* __restrict__ tw,
                                                     int sign, int tl) {
  extern __shared__ unsigned char lds_raw[];
  Cplx<T>* buf = (Cplx<T>*)lds_raw;
  constexpr int n = R1 * R2;
  constexpr int ls = n + 1;
  const int nx = g.n[0], ny = g.n[1];
  const long estride = A == 0 ? 1 : (A == 1 ? (long)nx : (long)nx * ny);
  const long l0 = (long)blockIdx.x * tl;
  auto base = [&](long l) -> long {
    if (A == 0) return l * nx;
    if (A == 1) return (l % nx) + (l / nx) * (long)nx * ny;
    return l;  // A == 2: l = i + nx j
  };
  const int tot = tl * n;
  for (int t = threadIdx.x; t < tot; t += kFftThreads) {
    int line, e;
    if (A == 0) {
      line = t / n;
      e = t - line * n;
    } else {
      e = t / tl;
      line = t - e * tl;
    }
    buf[line * ls + e] = c[base(l0 + line) + (long)e * estride];
  }
  __syncthreads();
  for (int jb = threadIdx.x; jb < tl * R2; jb += kFftThreads) {
    int line, n2;
    if (A == 0) {
      line = jb / R2;
      n2 = jb - line * R2;
    } else {
      n2 = jb / tl;
      line = jb - n2 * tl;
    }
    Cplx<T>* L = buf + line * ls;
    Cplx<T> a[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) a[n1] = L[R2 * n1 + n2];
    dft_reg<T, R1>(a, tw, n, sign);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      const int q = (n2 * k1) & (n - 1);  // W_n^q, q < n
      Cplx<T> w = tw[q & (n / 2 - 1)];
      if (q >= n / 2) w = Cplx<T>{-w.re, -w.im};
      if (sign > 0) w.im = -w.im;
      const Cplx<T> v = a[k1];
      L[R2 * k1 + n2] = (q == 0) ? v
                                 : Cplx<T>{v.re * w.re - v.im * w.im, v.re * w.im + v.im * w.re};
    }
  }
  __syncthreads();
  for (int jb = threadIdx.x; jb < tl * R1; jb += kFftThreads) {
    int line, k1;
    if (A == 0) {
      line = jb / R1;
      k1 = jb - line * R1;
    } else {
      k1 = jb / tl;
      line = jb - k1 * tl;
    }
    const Cplx<T>* L = buf + line * ls;
    Cplx<T> a[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) a[n2] = L[R2 * k1 + n2];
    dft_reg<T, R2>(a, tw, n, sign);
    const long b0 = base(l0 + line);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) c[b0 + (long)(k1 + R1 * k2) * estride] = a[k2];
  }
}

// Mode (i, j, k): times 4 pi G / (N lambda), lambda = lx[i] + ly[j] + lz[k];
// the mean mode is zero.
template <class T>
__global__ void __launch_bounds__(256) k_grav_kmul(Geo g, Cplx<T>* c, const T* __restrict__ lx,
                                                   const T* __restrict__ ly, const T* __restrict__ lz,
                                                   double fac) {
  const long q = (long)blockIdx.x * 256 + threadIdx.x;
  const long N = (long)g.n[0] * g.n[1] * g.n[2];
  if (q >= N) return;
  const int i = (int)(q % g.n[0]);
  const int j = (int)((q / g.n[0]) % g.n[1]);
  const int k = (int)(q / ((long)g.n[0] * g.n[1]));
  if (q == 0) {
    c[0] = Cplx<T>{T(0), T(0)};
    return;
  }
  const T s = (T)(fac / ((double)lx[i] + (double)ly[j] + (double)lz[k]));
  c[q] = Cplx<T>{c[q].re * s, c[q].im * s};
}

// Psi = Re c (already normalised) and its central gradient, periodic wrap.
template <class T>
__global__ void __launch_bounds__(256) k_grav_grad(Geo g, const Cplx<T>* __restrict__ c, Grav<T> gr) {
  const long q = (long)blockIdx.x * 256 + threadIdx.x;
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const long N = (long)nx * ny * nz;
  if (q >= N) return;
  const int i = (int)(q % nx);
  const int j = (int)((q / nx) % ny);
  const int k = (int)(q / ((long)nx * ny));
  const int p = (i + NG) + g.sy * (j + NG) + g.sz * (k + NG);
  const int ip = i + 1 < nx ? i + 1 : 0, im = i > 0 ? i - 1 : nx - 1;
  const int jp = j + 1 < ny ? j + 1 : 0, jm = j > 0 ? j - 1 : ny - 1;
  const int kp = k + 1 < nz ? k + 1 : 0, km = k > 0 ? k - 1 : nz - 1;
  gr.psi[p] = c[q].re;
  gr.g[0][p] = (c[cidx(g, ip, j, k)].re - c[cidx(g, im, j, k)].re) * (T)(0.5 / g.d[0]);
  gr.g[1][p] = (c[cidx(g, i, jp, k)].re - c[cidx(g, i, jm, k)].re) * (T)(0.5 / g.d[1]);
  gr.g[2][p] = (c[cidx(g, i, j, kp)].re - c[cidx(g, i, j, km)].re) * (T)(0.5 / g.d[2]);
}

template <class T, int A, int R1, int R2>
static void fft_launch(unsigned blocks, size_t lds, hipStream_t st, const Geo& g, Cplx<T>* c,
                       const Cplx<T>* tw, int sign, int tl) {
  hipLaunchKernelGGL((k_fft<T, A, R1, R2>), dim3(blocks), dim3(kFftThreads), lds, st, g, c, tw,
                     sign, tl);
}

template <class T, int A>
static void fft_axis(const Geo& g, Cplx<T>* c, const Cplx<T>* tw, int sign, hipStream_t st) {
  const int n = g.n[A];
  if (n == 1) return;
  const long lines = (long)g.n[0] * g.n[1] * g.n[2] / n;
  int tl = kFftTileElems / n;
  if (tl < 1) tl = 1;
  if (tl > lines) tl = (int)lines;
  if (A != 0 && tl > g.n[0]) tl = g.n[0];  // tiles of consecutive x (powers of two)
  const unsigned blocks = (unsigned)(lines / tl);
  const size_t lds = (size_t)tl * (n + 1) * sizeof(Cplx<T>);
  switch (n) {  // n = R1 R2
    case 2: fft_launch<T, A, 2, 1>(blocks, lds, st, g, c, tw, sign, tl); break;
    case 4: fft_launch<T, A, 2, 2>(blocks, lds, st, g, c, tw, sign, tl); break;
    case 8: fft_launch<T, A, 4, 2>(blocks, lds, st, g, c, tw, sign, tl); break;
    case 16: fft_launch<T, A, 4, 4>(blocks, lds, st, g, c, tw, sign, tl); break;
    case 32: fft_launch<T, A, 8, 4>(blocks, lds, st, g, c, tw, sign, tl); break;
    case 64: fft_launch<T, A, 8, 8>(blocks, lds, st, g, c, tw, sign, tl); break;
    case 128: fft_launch<T, A, 16, 8>(blocks, lds, st, g, c, tw, sign, tl); break;
    case 256: fft_launch<T, A, 16, 16>(blocks, lds, st, g, c, tw, sign, tl); break;
    case 512: fft_launch<T, A, 32, 16>(blocks, lds, st, g, c, tw, sign, tl); break;
    default: fft_launch<T, A, 32, 32>(blocks, lds, st, g, c, tw, sign, tl); break;  // 1024
  }
}

template <class T>
void launch_self_gravity(const Geo& g, const Physics& ph, const T* rho, GravFFT<T> f, Grav<T> gr,
                         Parts<T> pp, DtRef h, hipStream_t st) {
  const long N = (long)g.n[0] * g.n[1] * g.n[2];
  const unsigned blocks = (unsigned)((N + 255) / 256);
  Cplx<T>* c = (Cplx<T>*)f.c;
  const Cplx<T>* tw[3] = {(const Cplx<T>*)f.tw[0], (const Cplx<T>*)f.tw[1],
                          (const Cplx<T>*)f.tw[2]};
  hipLaunchKernelGGL(k_grav_load<T>, dim3(blocks), dim3(256), 0, st, g, rho, c,
                     ph.src[1] == 1.0 ? 0 : 1);
  if (pp.n > 0) launch_deposit<T>(g, pp, h, f.c, st);
  fft_axis<T, 0>(g, c, tw[0], -1, st);
  fft_axis<T, 1>(g, c, tw[1], -1, st);
  fft_axis<T, 2>(g, c, tw[2], -1, st);
  const double fac = 4.0 * 3.14159265358979323846 * ph.src[0] / (double)N;
  hipLaunchKernelGGL(k_grav_kmul<T>, dim3(blocks), dim3(256), 0, st, g, c, f.lam[0], f.lam[1],
                     f.lam[2], fac);
  fft_axis<T, 0>(g, c, tw[0], +1, st);
  fft_axis<T, 1>(g, c, tw[1], +1, st);
  fft_axis<T, 2>(g, c, tw[2], +1, st);
  hipLaunchKernelGGL(k_grav_grad<T>, dim3(blocks), dim3(256), 0, st, g, c, gr);
}

template void launch_self_gravity<double>(const Geo&, const Physics&, const double*,
                                          GravFFT<double>, Grav<double>, Parts<double>, DtRef,
                                          hipStream_t);
template void launch_self_gravity<float>(const Geo&, const Physics&, const float*, GravFFT<float>,
                                         Grav<float>, Parts<float>, DtRef, hipStream_t);

}  // namespace mhd
