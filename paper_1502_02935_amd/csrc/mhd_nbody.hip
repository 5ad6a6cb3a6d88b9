// mhd_nbody.hip -- N-body particles of the step (section 2.1 of the paper:
// particle-in-cell dynamics with the "flip-flop" integrator, a
// mass-conserving second-order mass assignment), sharing the periodic
// potential of the self-gravity solve.
//
// Cloud in cell: a particle is a cube of one cell's size; along each axis,
// in cell-centre units s = (x - x0)/d - 1/2, it overlaps cells floor(s)
// and floor(s) + 1 (periodic) with fractions 1 - f and f, f = s - floor(s).
// The deposit adds m w_x w_y w_z / dV to each of the 8 cells; the force is
// minus the cell-centred central gradient of Psi interpolated with the same
// weights, which keeps the total momentum.
//
// The particles are kept sorted by tile (kTile^3 cells): every step starts
// with a counting sort by the tile of each particle's cell (counts gathered
// per block in LDS, one global atomic per distinct tile and block), and
// each tile's particles are cut into chunks of at most kChunk.  One block per chunk then works in LDS: the deposit
// adds into a private copy of the cells the tile's particles can reach (the
// tile and 2 cells around it: a particle moves at most half a cell between
// the sort and the half-step deposit under the CFL limit) and flushes it
// with one atomic per touched cell; the kick stages the potential gradient
// of the same cells.  A target outside that window (a step larger than the
// CFL limit) goes to HBM directly.  The device-scope atomics of the first
// version -- 8 per particle, piled onto the few cells of a dense core -- took
// most of the step.
#include <math.h>

#include "mhd_span.hpp"

namespace mhd {

constexpr int kPartThreads = 256;
constexpr int kWin = kTile + 5;  // LDS window per axis: tile cells -2 .. kTile + 2
constexpr int kWin3 = kWin * kWin * kWin;
constexpr int kStageMin = 256;   // particles per tile from which the kick stages in LDS

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

// Cell of a (wrapped) position along axis a.
template <class T>
__device__ __forceinline__ int cell_of(const Geo& g, int a, T x) {
  int c = (int)floor(((double)x - g.x0[a]) / g.d[a]);
  return c < 0 ? 0 : (c >= g.n[a] ? g.n[a] - 1 : c);
}

template <class T>
__device__ __forceinline__ int tile_of(const Geo& g, const Parts<T>& pp, long long q) {
  const long long n = pp.n;
  const int tx = cell_of(g, 0, pp.x[q]) / kTile;
  const int ty = cell_of(g, 1, pp.x[n + q]) / kTile;
  const int tz = cell_of(g, 2, pp.x[2 * n + q]) / kTile;
  return (tz * pp.nt[1] + ty) * pp.nt[0] + tx;
}

// Window index of global cell c along an axis whose window starts at cell
// o - 2 (periodic extent n), or -1 outside the window.
__device__ __forceinline__ int win_index(int c, int o, int n) {
  int d = c - (o - 2);
  if (d < 0) d += n;
  if (d >= n) d -= n;
  return d < kWin ? d : -1;
}

__device__ __forceinline__ void atomic_add_t(double* p, double v) { atomicAdd(p, v); }
__device__ __forceinline__ void atomic_add_t(float* p, float v) { atomicAdd(p, v); }

// ---------------------------------------------------------------------------
// Sort by tile
// ---------------------------------------------------------------------------

__global__ void __launch_bounds__(kPartThreads) k_tile_zero(int* cnt, int ntiles) {
  for (int t = blockIdx.x * kPartThreads + threadIdx.x; t < ntiles; t += gridDim.x * kPartThreads)
    cnt[t] = 0;
}

// Block-level aggregation of the sort's counters: a block takes kSortChunk
// consecutive particles -- in the order of the last sort, so a few tiles
// and their neighbours -- and gathers their per-tile counts in an LDS hash
// table (kSortSlots slots, linear probing) before one global atomic per
// distinct tile.  A key the table cannot place within kSortProbes probes
// goes to HBM directly (the first sort of particles in arbitrary order).
// (Per-wave aggregation alone still piled ~2000 atomics per step onto the
// counter of a dense core tile.)
constexpr int kSortChunk = 4096;
constexpr int kSortSlots = 512;
constexpr int kSortProbes = 32;  // a key not placed within this many probes goes to HBM

struct SortTable {
  int key[kSortSlots];
  int cnt[kSortSlots];
  int base[kSortSlots];
};

__device__ __forceinline__ void table_clear(SortTable& tb) {
  for (int i = threadIdx.x; i < kSortSlots; i += kPartThreads) {
    tb.key[i] = -1;
    tb.cnt[i] = 0;
  }
}

// Slot of key in the table (inserted if absent), or -1 if it is not found
// within kSortProbes probes.
__device__ __forceinline__ int table_find(SortTable& tb, int key, bool insert) {
  int h = (int)(((unsigned)key * 2654435761u) >> 20) & (kSortSlots - 1);
  for (int probe = 0; probe < kSortProbes; ++probe) {
    const int k = __atomic_load_n(&tb.key[h], __ATOMIC_RELAXED);
    if (k == key) return h;
    if (k == -1) {
      if (!insert) return -1;
      const int old = atomicCAS(&tb.key[h], -1, key);
      if (old == -1 || old == key) return h;
    }
    h = (h + 1) & (kSortSlots - 1);
  }
  return -1;
}

static unsigned sort_blocks(long long n) {
  return (unsigned)((n + kSortChunk - 1) / kSortChunk);
}

template <class T>
__global__ void __launch_bounds__(kPartThreads) k_tile_count(Geo g, Parts<T> pp, int* cnt) {
  __shared__ SortTable tb;
  table_clear(tb);
  __syncthreads();
  const long long n = pp.n;
  const long long q0 = (long long)blockIdx.x * kSortChunk;
  const long long q1 = q0 + kSortChunk < n ? q0 + kSortChunk : n;
  for (long long q = q0 + threadIdx.x; q < q1; q += kPartThreads) {
    const int key = tile_of(g, pp, q);
    const int h = table_find(tb, key, true);
    if (h >= 0)
      atomicAdd(&tb.cnt[h], 1);
    else
      atomicAdd(cnt + key, 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kSortSlots; i += kPartThreads)
    if (tb.cnt[i] > 0) atomicAdd(cnt + tb.key[i], tb.cnt[i]);
}

// Exclusive scan of cnt into off (ntiles + 1 entries) and, if cur, cur =
// off: one block, each thread a contiguous share.
__global__ void __launch_bounds__(1024) k_tile_scan(const int* cnt, int* off, int* cur, int ntiles) {
  __shared__ int part[1024];
  const int share = (ntiles + 1023) / 1024;
  const int lo = threadIdx.x * share, hi = min(ntiles, lo + share);
  int s = 0;
  for (int t = lo; t < hi; ++t) s += cnt[t];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {  // inclusive Hillis-Steele scan of the shares
    const int v = threadIdx.x >= (unsigned)d ? part[threadIdx.x - d] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int base = threadIdx.x ? part[threadIdx.x - 1] : 0;
  for (int t = lo; t < hi; ++t) {
    off[t] = base;
    if (cur) cur[t] = base;
    base += cnt[t];
  }
  if (threadIdx.x == 1023) off[ntiles] = part[1023];
}

// Same blocks and table: each distinct tile reserves its block's range of
// slots with one global atomic on its cursor; particles take slots from
// LDS counters (their order within a tile's range is not deterministic).
template <class T>
__global__ void __launch_bounds__(kPartThreads) k_tile_scatter(Geo g, Parts<T> pp, PartSort<T> s) {
  __shared__ SortTable tb;
  table_clear(tb);
  __syncthreads();
  const long long n = pp.n;
  const long long q0 = (long long)blockIdx.x * kSortChunk;
  const long long q1 = q0 + kSortChunk < n ? q0 + kSortChunk : n;
  for (long long q = q0 + threadIdx.x; q < q1; q += kPartThreads) {
    const int h = table_find(tb, tile_of(g, pp, q), true);
    if (h >= 0) atomicAdd(&tb.cnt[h], 1);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kSortSlots; i += kPartThreads) {
    if (tb.cnt[i] > 0) tb.base[i] = atomicAdd(s.cur + tb.key[i], tb.cnt[i]);
    tb.cnt[i] = 0;
  }
  __syncthreads();
  for (long long q = q0 + threadIdx.x; q < q1; q += kPartThreads) {
    const int key = tile_of(g, pp, q);
    const int h = table_find(tb, key, false);
    const int slot = h >= 0 ? tb.base[h] + atomicAdd(&tb.cnt[h], 1) : atomicAdd(s.cur + key, 1);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      s.x[a * n + slot] = pp.x[a * n + q];
      s.v[a * n + slot] = pp.v[a * n + q];
    }
    s.m[slot] = pp.m[q];
    s.id[slot] = pp.id[q];
  }
}

// Chunks of at most kChunk particles within each tile: per tile the chunk
// count (into cnt2), then, after its scan into coff, the list of (tile,
// first, end) and the total.
__global__ void __launch_bounds__(kPartThreads) k_chunk_count(const int* cnt, int* cnt2, int ntiles) {
  for (int t = blockIdx.x * kPartThreads + threadIdx.x; t < ntiles; t += gridDim.x * kPartThreads)
    cnt2[t] = (cnt[t] + kChunk - 1) / kChunk;
}

__global__ void __launch_bounds__(kPartThreads) k_chunk_list(const int* off, const int* coff,
                                                             int* chunk, int ntiles) {
  for (int t = blockIdx.x * kPartThreads + threadIdx.x; t < ntiles; t += gridDim.x * kPartThreads) {
    const int q0 = off[t], q1 = off[t + 1];
    int k = coff[t];
    for (int q = q0; q < q1; q += kChunk, ++k) {
      chunk[1 + 3 * k] = t;
      chunk[2 + 3 * k] = q;
      chunk[3 + 3 * k] = min(q + kChunk, q1);
    }
    if (t == ntiles - 1) chunk[0] = coff[ntiles];
  }
}

template <class T>
void launch_particle_sort(const Geo& g, Parts<T> pp, PartSort<T> s, hipStream_t st) {
  if (pp.n <= 0) return;
  const unsigned tb = (unsigned)((pp.ntiles + kPartThreads - 1) / kPartThreads);
  hipLaunchKernelGGL(k_tile_zero, dim3(tb), dim3(kPartThreads), 0, st, s.cnt, pp.ntiles);
  hipLaunchKernelGGL(k_tile_count<T>, dim3(sort_blocks(pp.n)), dim3(kPartThreads), 0, st, g, pp,
                     s.cnt);
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, st, s.cnt, s.off, s.cur, pp.ntiles);
  hipLaunchKernelGGL(k_tile_scatter<T>, dim3(sort_blocks(pp.n)), dim3(kPartThreads), 0, st, g,
                     pp, s);
  // the cursors are spent: they take the chunk counts
  hipLaunchKernelGGL(k_chunk_count, dim3(tb), dim3(kPartThreads), 0, st, s.cnt, s.cur, pp.ntiles);
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(1024), 0, st, s.cur, s.coff, (int*)nullptr,
                     pp.ntiles);
  hipLaunchKernelGGL(k_chunk_list, dim3(tb), dim3(kPartThreads), 0, st, s.off, s.coff, s.chunk,
                     pp.ntiles);
}

// ---------------------------------------------------------------------------
// Deposit, kick-drift
// ---------------------------------------------------------------------------

// One block per tile: the cloud-in-cell density of the tile's particles at
// x + h v (h = dt x factor), added to the real parts of c.
template <class T>
__global__ void __launch_bounds__(kPartThreads) k_deposit(Geo g, Parts<T> pp, DtRef hr, T* c) {
  __shared__ T acc[kWin3];
  if ((int)blockIdx.x >= pp.chunk[0]) return;
  const int t = pp.chunk[1 + 3 * blockIdx.x];
  const int q0 = pp.chunk[2 + 3 * blockIdx.x], q1 = pp.chunk[3 + 3 * blockIdx.x];
  const int tx = t % pp.nt[0], ty = (t / pp.nt[0]) % pp.nt[1], tz = t / (pp.nt[0] * pp.nt[1]);
  const int o[3] = {tx * kTile, ty * kTile, tz * kTile};
  for (int i = threadIdx.x; i < kWin3; i += kPartThreads) acc[i] = T(0);
  __syncthreads();
  const double h = (hr.ptr ? *hr.ptr : hr.value) * hr.factor;
  const T idv = (T)(1.0 / (g.d[0] * g.d[1] * g.d[2]));
  const long long n = pp.n;
  for (int q = q0 + (int)threadIdx.x; q < q1; q += kPartThreads) {
    int ci[3][2], wi[3][2];
    T w[3][2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T x = pp.x[a * n + q];
      if (h != 0.0) x = wrap_coord<T>(x + (T)h * pp.v[a * n + q], g.x0[a], g.n[a] * g.d[a]);
      cic_axis<T>(g, a, x, ci[a], w[a]);
      wi[a][0] = win_index(ci[a][0], o[a], g.n[a]);
      wi[a][1] = win_index(ci[a][1], o[a], g.n[a]);
    }
    const T m = pp.m[q];
#pragma unroll
    for (int e = 0; e < 2; ++e)
#pragma unroll
      for (int b = 0; b < 2; ++b)
#pragma unroll
        for (int a = 0; a < 2; ++a) {
          const T val = m * w[0][a] * w[1][b] * w[2][e] * idv;
          if (wi[0][a] >= 0 && wi[1][b] >= 0 && wi[2][e] >= 0)
            atomicAdd(&acc[(wi[2][e] * kWin + wi[1][b]) * kWin + wi[0][a]], val);
          else
            atomic_add_t(c + 2 * (((long)ci[2][e] * g.n[1] + ci[1][b]) * g.n[0] + ci[0][a]), val);
        }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kWin3; i += kPartThreads) {
    const T v = acc[i];
    if (v == T(0)) continue;
    const int a0 = i % kWin, a1 = (i / kWin) % kWin, a2 = i / (kWin * kWin);
    int gc[3];
    const int ai[3] = {a0, a1, a2};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      int cc = o[a] - 2 + ai[a];
      cc %= g.n[a];
      if (cc < 0) cc += g.n[a];
      gc[a] = cc;
    }
    atomic_add_t(c + 2 * (((long)gc[2] * g.n[1] + gc[1]) * g.n[0] + gc[0]), v);
  }
}

template <class T>
__device__ __forceinline__ T grad_at(const Geo& g, const Grav<T>& gr, int a, int i, int j, int k) {
  return gr.g[a][(i + NG) + g.sy * (j + NG) + g.sz * (k + NG)];
}

// One block per tile: x_h = x + dt/2 v, v -= dt grad Psi(x_h) (cloud in
// cell), x = x_h + dt/2 v; tiles with many particles stage the gradient of
// their window in LDS first.
template <class T>
__global__ void __launch_bounds__(kPartThreads) k_kick_drift(Geo g, Parts<T> pp, Grav<T> gr,
                                                             DtRef dtr) {
  __shared__ T gl[3][kWin3];
  if ((int)blockIdx.x >= pp.chunk[0]) return;
  const int t = pp.chunk[1 + 3 * blockIdx.x];
  const int q0 = pp.chunk[2 + 3 * blockIdx.x], q1 = pp.chunk[3 + 3 * blockIdx.x];
  const int tx = t % pp.nt[0], ty = (t / pp.nt[0]) % pp.nt[1], tz = t / (pp.nt[0] * pp.nt[1]);
  const int o[3] = {tx * kTile, ty * kTile, tz * kTile};
  const bool staged = q1 - q0 >= kStageMin;
  if (staged) {
    for (int i = threadIdx.x; i < kWin3; i += kPartThreads) {
      const int ai[3] = {i % kWin, (i / kWin) % kWin, i / (kWin * kWin)};
      int gc[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        int cc = (o[a] - 2 + ai[a]) % g.n[a];
        if (cc < 0) cc += g.n[a];
        gc[a] = cc;
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) gl[a][i] = grad_at(g, gr, a, gc[0], gc[1], gc[2]);
    }
  }
  __syncthreads();
  const double dt = (dtr.ptr ? *dtr.ptr : dtr.value) * dtr.factor;
  const T hdt = (T)(0.5 * dt), Tdt = (T)dt;
  const long long n = pp.n;
  for (int q = q0 + (int)threadIdx.x; q < q1; q += kPartThreads) {
    T xh[3], w[3][2];
    int ci[3][2], wi[3][2];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      xh[a] = wrap_coord<T>(pp.x[a * n + q] + hdt * pp.v[a * n + q], g.x0[a], g.n[a] * g.d[a]);
      cic_axis<T>(g, a, xh[a], ci[a], w[a]);
      wi[a][0] = win_index(ci[a][0], o[a], g.n[a]);
      wi[a][1] = win_index(ci[a][1], o[a], g.n[a]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T acc = T(0);
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            const bool in = staged && wi[0][i] >= 0 && wi[1][b] >= 0 && wi[2][e] >= 0;
            const T gv = in ? gl[a][(wi[2][e] * kWin + wi[1][b]) * kWin + wi[0][i]]
                            : grad_at(g, gr, a, ci[0][i], ci[1][b], ci[2][e]);
            acc += w[0][i] * w[1][b] * w[2][e] * gv;
          }
      const T v = pp.v[a * n + q] - Tdt * acc;
      pp.v[a * n + q] = v;
      pp.x[a * n + q] = wrap_coord<T>(xh[a] + hdt * v, g.x0[a], g.n[a] * g.d[a]);
    }
  }
}

template <class T>
__global__ void __launch_bounds__(kPartThreads) k_particles_init(Geo g, Parts<T> pp) {
  const long long n = pp.n;
  for (long long q = (long long)blockIdx.x * kPartThreads + threadIdx.x; q < n;
       q += (long long)gridDim.x * kPartThreads) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
      pp.x[a * n + q] = wrap_coord<T>(pp.x[a * n + q], g.x0[a], g.n[a] * g.d[a]);
    pp.id[q] = (int)q;
  }
}

template <class T>
__global__ void __launch_bounds__(kPartThreads) k_particles_out(Parts<T> pp, T* xo, T* vo) {
  const long long n = pp.n;
  for (long long q = (long long)blockIdx.x * kPartThreads + threadIdx.x; q < n;
       q += (long long)gridDim.x * kPartThreads) {
    const long long u = pp.id[q];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (xo) xo[a * n + u] = pp.x[a * n + q];
      if (vo) vo[a * n + u] = pp.v[a * n + q];
    }
  }
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
  hipLaunchKernelGGL(k_deposit<T>, dim3((unsigned)pp.max_chunks), dim3(kPartThreads), 0, st, g, pp,
                     h, c);
}

template <class T>
void launch_kick_drift(const Geo& g, Parts<T> pp, Grav<T> gr, DtRef dt, hipStream_t st) {
  if (pp.n <= 0) return;
  hipLaunchKernelGGL(k_kick_drift<T>, dim3((unsigned)pp.max_chunks), dim3(kPartThreads), 0, st, g,
                     pp, gr, dt);
}

template <class T>
void launch_particles_init(const Geo& g, Parts<T> pp, hipStream_t st) {
  if (pp.n <= 0) return;
  hipLaunchKernelGGL(k_particles_init<T>, dim3(part_blocks(pp.n)), dim3(kPartThreads), 0, st, g,
                     pp);
}

template <class T>
void launch_particles_out(Parts<T> pp, T* x_out, T* v_out, hipStream_t st) {
  if (pp.n <= 0) return;
  hipLaunchKernelGGL(k_particles_out<T>, dim3(part_blocks(pp.n)), dim3(kPartThreads), 0, st, pp,
                     x_out, v_out);
}

#define MHD_NBODY_INST(T)                                                                        \
  template void launch_particle_cfl<T>(const Geo&, Parts<T>, double*, hipStream_t);             \
  template void launch_deposit<T>(const Geo&, Parts<T>, DtRef, T*, hipStream_t);                \
  template void launch_kick_drift<T>(const Geo&, Parts<T>, Grav<T>, DtRef, hipStream_t);        \
  template void launch_particles_init<T>(const Geo&, Parts<T>, hipStream_t);                    \
  template void launch_particle_sort<T>(const Geo&, Parts<T>, PartSort<T>, hipStream_t);        \
  template void launch_particles_out<T>(Parts<T>, T*, T*, hipStream_t);

MHD_NBODY_INST(double)
MHD_NBODY_INST(float)

}  // namespace mhd
