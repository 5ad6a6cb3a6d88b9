// mhd_span.hpp -- sweep geometry shared by the kernels of the step: padded
// indexing, the slab/plane walk of a sweep with its XCD-aware block order,
// per-wave event counting and 32-bit-offset buffer access.
#pragma once

#include "mhd_kernels.hpp"

namespace mhd {

constexpr int BX = 64;  // block x extent = one wavefront
constexpr int BY = 4;   // waves per block

__device__ __forceinline__ int pidx(const Geo& g, int i, int j, int k) {
  return (i + NG) + g.sy * (j + NG) + g.sz * (k + NG);
}

__device__ __forceinline__ int stride_of(const Geo& g, int a) {
  return a == 0 ? 1 : (a == 1 ? g.sy : g.sz);
}

// Frame component of axis a that holds global conserved component m
// (0 rho, 1..3 momentum, 4 energy).
__device__ __forceinline__ int frame_comp(int a, int m) {
  if (m == 0 || m == 4) return m;
  const int d = m - 1;
  return d == a ? 1 : (d == (a + 1) % 3 ? 2 : 3);
}

// How many times the outer face layer copies the A-face of interior cell c
// (its periodic images: along a periodic axis a cell at index 0 reappears at
// n, one at n-1 at -1, where an A-face exists only if that index is not -1
// on A itself), plus one for the face itself: a kernel that solves only the
// interior faces counts an event on that face this many times, as solving
// the outer layer too would (faces 0..n along A, rows -1..n across).
__device__ __forceinline__ int face_copies(const Geo& g, const int c[3], int A) {
  int m = 1;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (g.nf[a] != g.n[a]) continue;  // not periodic
    int k = 1;
    if (c[a] == 0) ++k;
    if (c[a] == g.n[a] - 1 && a != A) ++k;
    m *= k;
  }
  return m;
}

// Index step from index c (-2 <= c <= n + 1) to the cell d away along axis
// a (|d| <= 2), wrapped into [0, n) on a periodic axis, as an unsigned (two's
// complement) count of that axis' points.  From 4 cells up, c + d lies
// within one period of [0, n): one add or subtract, no division.
__device__ __forceinline__ unsigned axis_step(const Geo& g, int a, int c, int d) {
  int t = c + d;
  const int n = g.n[a];
  if (g.nf[a] == n) {
    if (n >= 4)
      t = t < 0 ? t + n : (t >= n ? t - n : t);
    else
      t = (t % n + n) % n;
  }
  return (unsigned)(t - c);
}

static inline dim3 grid_for(int nx, int ny, int nz) {
  return dim3((unsigned)((nx + BX - 1) / BX), (unsigned)((ny + BY - 1) / BY), (unsigned)nz);
}

// ------------------------------------------------------------------------
// Sweep geometry.  A sweep visits the points lo..hi (inclusive, per axis) of
// the padded grid.  The rows lo_y..hi_y are cut into slabs of `rows` rows;
// each z-plane of a slab is walked as one run of whole padded x-rows (row
// stride sy), kSpanThreads points per block, so a wave's 64 lanes always
// touch 64 consecutive addresses and only the few padding columns outside
// lo_x..hi_x idle (a 64-wide tiling of the x-rows alone leaves a mostly
// empty fifth wave on every row of a 256-wide box).  Blocks are numbered
// slab by slab, plane by plane within a slab, and renumbered so that each
// XCD -- the hardware deals blocks out round-robin, block b to XCD b mod 8 --
// walks a contiguous range of them: an XCD marches through the planes of
// its own slabs, and the planes a z-stencil reaches back to (plus the
// blocks in flight) stay within its L2, which whole planes of a large box
// would not (the neighbour planes were fetched from memory again).
// ------------------------------------------------------------------------

constexpr int kSpanThreads = 256;

struct Span {
  int lo[3], hi[3];
  int nt;         // threads (points) per block
  int rows;       // rows per slab (the last slab may be shorter)
  int per_plane;  // points of one slab plane: sy * rows
  int bpp;        // blocks per slab plane
  int bps;        // blocks per slab: bpp * planes
  int nblk;
  float inv_sy, inv_bpp, inv_bps;
};

// Rows per slab: whole planes for small boxes (they fit an XCD's L2), else a
// multiple of 8 slabs of at most 36 rows, so that every XCD gets the same
// number of slabs.
static inline int slab_rows(int nrows) {
  if (nrows <= 160) return nrows;
  const int nslab = 8 * ((nrows + 8 * 36 - 1) / (8 * 36));
  return (nrows + nslab - 1) / nslab;
}

static inline Span make_span(const Geo& g, int ilo, int ihi, int jlo, int jhi, int klo, int khi,
                             int nt = kSpanThreads) {
  Span s;
  s.lo[0] = ilo, s.hi[0] = ihi, s.lo[1] = jlo, s.hi[1] = jhi, s.lo[2] = klo, s.hi[2] = khi;
  s.nt = nt;
  const int nrows = jhi - jlo + 1;
  s.rows = slab_rows(nrows);
  const int nslab = (nrows + s.rows - 1) / s.rows;
  s.per_plane = g.sy * s.rows;
  s.bpp = (s.per_plane + nt - 1) / nt;
  s.bps = s.bpp * (khi - klo + 1);
  s.nblk = s.bps * nslab;
  s.inv_sy = 1.0f / (float)g.sy;
  s.inv_bpp = 1.0f / (float)s.bpp;
  s.inv_bps = 1.0f / (float)s.bps;
  return s;
}

static inline dim3 span_grid(const Span& s) { return dim3((unsigned)s.nblk); }

// q = floor(a / d) for 0 <= a < 2^31, d > 0: a float estimate (off by at
// most one step below 2^23, a few above), corrected to exact in integers.
__device__ __forceinline__ int div_small(int a, int d, float inv_d) {
  int q = (int)(((float)a + 0.5f) * inv_d);
  while (q * d > a) --q;
  while ((q + 1) * d <= a) ++q;
  return q;
}

struct Pt {
  int i, j, k, p;
  bool valid;
};

__device__ __forceinline__ Pt span_point(const Geo& g, const Span& s) {
  const unsigned nb = (unsigned)s.nblk, b0 = blockIdx.x;
  const unsigned q = nb >> 3, r = nb & 7u, x = b0 & 7u;
  const int b = (int)(x * q + (x < r ? x : r) + (b0 >> 3));
  const int slab = div_small(b, s.bps, s.inv_bps);
  const int bs = b - slab * s.bps;
  const int plane = div_small(bs, s.bpp, s.inv_bpp);
  const int t = (bs - plane * s.bpp) * s.nt + (int)threadIdx.x;
  const int row = div_small(t, g.sy, s.inv_sy);
  Pt o;
  o.i = t - row * g.sy - NG;
  o.j = s.lo[1] + slab * s.rows + row;
  o.k = s.lo[2] + plane;
  o.valid = t < s.per_plane && o.j <= s.hi[1] && o.i >= s.lo[0] && o.i <= s.hi[0];
  o.p = pidx(g, o.i, o.j, o.k);
  return o;
}

// Count lanes with `flag` set into the counter's slot of this block, with
// one atomic per wave.  Must be reached by every lane of the wave.
__device__ __forceinline__ void wave_count(bool flag, unsigned long long* ctr) {
  const unsigned long long m = __ballot(flag);
  if (m != 0ull && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)__ballot(1)) - 1)) {
    const unsigned b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    atomicAdd(ctr + (size_t)(b % kCounterSlots) * kCounterStride,
              (unsigned long long)__popcll(m));
  }
}

// Add every lane's n into the counter's slot of this block, with one
// atomic per wave.  Must be reached by every lane of the wave.
__device__ __forceinline__ void wave_add(int n, unsigned long long* ctr) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
  if (n != 0 && (threadIdx.x & 63) == (unsigned)(__ffsll((long long)__ballot(1)) - 1)) {
    const unsigned b = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    atomicAdd(ctr + (size_t)(b % kCounterSlots) * kCounterStride, (unsigned long long)n);
  }
}

// Buffer access with a 32-bit byte offset (one per stencil point, shared by
// all arrays; no 64-bit address arithmetic per access); each resource is
// bounded by its array's size, so an offset outside it reads 0.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, unsigned bytes) {
  // word 3 0x00020000: 32-bit data format, the untyped-buffer setting of gfx9
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ float bld(float, __amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}
__device__ __forceinline__ double bld(double, __amdgpu_buffer_rsrc_t r, unsigned off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ void bst(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, 0);
}
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
// Runs of consecutive elements at a 4-byte-aligned byte offset in one
// wide load: 2 floats / 4 floats / 2 doubles (the vector memory unit takes
// about as long per instruction for 4 bytes a lane as for 16).  Elements
// are copied out of the vector before the bit cast: a bit cast of a vector
// element expression reads element 0.
__device__ __forceinline__ void bld2(float* v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  const u32x2 q = __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0);
  const unsigned e0 = q[0], e1 = q[1];
  v[0] = __builtin_bit_cast(float, e0);
  v[1] = __builtin_bit_cast(float, e1);
}
__device__ __forceinline__ void bld4(float* v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
  const unsigned e0 = q[0], e1 = q[1], e2 = q[2], e3 = q[3];
  v[0] = __builtin_bit_cast(float, e0);
  v[1] = __builtin_bit_cast(float, e1);
  v[2] = __builtin_bit_cast(float, e2);
  v[3] = __builtin_bit_cast(float, e3);
}
__device__ __forceinline__ void bld2(double* v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, 0);
  const u32x2 lo = {q[0], q[1]}, hi = {q[2], q[3]};
  v[0] = __builtin_bit_cast(double, lo);
  v[1] = __builtin_bit_cast(double, hi);
}
__device__ __forceinline__ void bld4(double* v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  bld2(v, r, off);
  bld2(v + 2, r, off + 16);
}
__device__ __forceinline__ void bst(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, 0);
}

}  // namespace mhd
