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
// FFT lines: a block takes a tile of lines of one axis into LDS (bit-reversed
// order), runs the log2(n) butterfly stages there and writes the tile back.
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

__device__ __forceinline__ int ilog2(int n) { return 31 - __clz(n); }

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

// Batched FFT of all lines along axis A of c ([nz][ny][nx]); sign -1 forward,
// +1 inverse (unnormalised).  tw: n/2 values exp(-2 pi i q / n).  tl: lines
// per block (tl * n <= kFftTileElems; for A = 1, 2 tl divides nx).
template <class T, int A>
__global__ void __launch_bounds__(kFftThreads) k_fft(Geo g, Cplx<T>* c, const Cplx<T>* __restrict__ tw,
                                                     int sign, int tl) {
  extern __shared__ unsigned char lds_raw[];
  Cplx<T>* buf = (Cplx<T>*)lds_raw;
  const int nx = g.n[0], ny = g.n[1];
  const int n = g.n[A];
  const int lg = ilog2(n);
  const long estride = A == 0 ? 1 : (A == 1 ? (long)nx : (long)nx * ny);
  const long l0 = (long)blockIdx.x * tl;
  // line l -> offset of its element 0
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
    const int rev = (int)(__brev((unsigned)e) >> (32 - lg));
    buf[line * n + rev] = c[base(l0 + line) + (long)e * estride];
  }
  __syncthreads();
  for (int s = 1; s <= lg; ++s) {
    const int m = 1 << (s - 1);
    const int half = n >> 1;
    for (int b = threadIdx.x; b < tl * half; b += kFftThreads) {
      const int line = b / half;
      const int jj = b - line * half;
      const int r = jj & (m - 1);
      const int i0 = ((jj >> (s - 1)) << s) + r;
      const int i1 = i0 + m;
      const Cplx<T> w0 = tw[r << (lg - s)];
      const T wr = w0.re, wi = sign < 0 ? w0.im : -w0.im;
      Cplx<T>* L = buf + line * n;
      const Cplx<T> u = L[i0], v = L[i1];
      const T vr = v.re * wr - v.im * wi, vi = v.re * wi + v.im * wr;
      L[i0] = Cplx<T>{u.re + vr, u.im + vi};
      L[i1] = Cplx<T>{u.re - vr, u.im - vi};
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < tot; t += kFftThreads) {
    int line, e;
    if (A == 0) {
      line = t / n;
      e = t - line * n;
    } else {
      e = t / tl;
      line = t - e * tl;
    }
    c[base(l0 + line) + (long)e * estride] = buf[line * n + e];
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
  const size_t lds = (size_t)tl * n * sizeof(Cplx<T>);
  hipLaunchKernelGGL((k_fft<T, A>), dim3(blocks), dim3(kFftThreads), lds, st, g, c, tw, sign, tl);
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
