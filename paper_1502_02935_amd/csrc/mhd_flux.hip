// mhd_flux.hip -- the flux sweep of the step (section 2.1 of the paper):
// limited MUSCL reconstruction (Eq. 12-14) of the face states and the
// Riemann solver (HLLD, or HLL / HLLC) on all three face families of the
// padded grid in one launch.
#include "mhd_source.hpp"
#include "mhd_span.hpp"

namespace mhd {

// ------------------------------------------------------------------------
// Fluxes of all three face families in one sweep.  The point p of cell
// (i, j, k) carries the faces at the lower x, y and z sides of that cell;
// the sweep visits i, j, k in -1..n and computes the A-face wherever the
// A-index is >= 0 (faces 0..n along A, rows -1..n across it: the boundary
// edges' EMFs need one ghost row of transverse fluxes).  One launch instead
// of three per-axis sweeps: the A-stencils of neighbouring points overlap,
// so the primitives are fetched from HBM about once instead of three times.
// Addressing: buffer loads and stores, a 32-bit byte offset per stencil
// point shared by all arrays (no 64-bit address arithmetic per access), each
// array's resource bounded by its size.
// ------------------------------------------------------------------------

// Flux of the face states with Riemann solver RS (a template parameter: a
// run-time switch would size every kernel's registers for the largest).
template <class T, int RS>
__device__ __forceinline__ int riemann_flux(const Physics& ph, const Face<T>& L, const Face<T>& R,
                                            T bn, T F[7]) {
  if constexpr (RS == kRiemannHLL) return hll(L, R, bn, (T)ph.gamma, (T)ph.igm1, F);
  if constexpr (RS == kRiemannHLLC) return hllc(L, R, (T)ph.gamma, (T)ph.igm1, F);
  return hlld(L, R, bn, (T)ph.gamma, (T)ph.igm1, F);
}

// The stencil of the A-face at point p: the seven face variables of cells
// p - 2s .. p + s (FO: first order, only p - s and p are loaded) and the
// face-normal field.  Buffer loads: an offset outside the array (a stencil
// of a face the sweep skips) reads 0 and never faults.
template <class T>
struct Stencil {
  T v[7][4];
  T bn;
};

template <class T, int A, bool FO>
__device__ __forceinline__ Stencil<T> load_stencil(int stride, unsigned bytes, const Prim<T>& w,
                                                   const T* __restrict__ bn, int p) {
  constexpr int A1 = (A + 1) % 3, A2 = (A + 2) % 3;
  const unsigned s = (unsigned)stride * (unsigned)sizeof(T);
  const unsigned o = (unsigned)p * (unsigned)sizeof(T);
  const T* src[7] = {w.w[0], w.w[1 + A], w.w[1 + A1], w.w[1 + A2], w.w[4], w.w[5 + A1], w.w[5 + A2]};
  Stencil<T> st;
#pragma unroll
  for (int v = 0; v < 7; ++v) {
    const auto q = rsrc(src[v], bytes);
    if constexpr (A == 0) {  // the x-stencil is a run of consecutive elements
      if constexpr (FO) {
        st.v[v][0] = st.v[v][3] = T(0);
        bld2(&st.v[v][1], q, o - s);
      } else {
        bld4(st.v[v], q, o - 2 * s);
      }
    } else {
      st.v[v][0] = FO ? T(0) : bld(T(), q, o - 2 * s);
      st.v[v][1] = bld(T(), q, o - s);
      st.v[v][2] = bld(T(), q, o);
      st.v[v][3] = FO ? T(0) : bld(T(), q, o + s);
    }
  }
  st.bn = bld(T(), rsrc(bn, bytes), o);
  return st;
}

// Flux of a face from its stencil: limited reconstruction (Eq. 12-14; FO:
// first order) and the Riemann solver.  Returns the HLLD branch code (bit 0
// HLL fallback, bit 1 degenerate; 0 for the other solvers).
template <class T, int RS, bool FO>
__device__ __forceinline__ int face_solve(const Physics& ph, const Stencil<T>& st,
                                          const Muscl<T>& mu, T F[7]) {
  T l[7], r[7];
#pragma unroll
  for (int v = 0; v < 7; ++v) {
    if constexpr (FO) {
      l[v] = st.v[v][1];
      r[v] = st.v[v][2];
    } else {
      muscl_lr_limited(mu, st.v[v][0], st.v[v][1], st.v[v][2], st.v[v][3], l[v], r[v]);
    }
  }
  const Face<T> L{l[0], l[1], l[2], l[3], l[4], l[5], l[6]};
  const Face<T> R{r[0], r[1], r[2], r[3], r[4], r[5], r[6]};
  return riemann_flux<T, RS>(ph, L, R, st.bn, F);
}

// Sign of the mass flux (the upwind side of Eq. 11) of the A-face at p.
template <class T, int A>
__device__ __forceinline__ void store_sign(unsigned bytes, const Flux<T>& f, T mass, int p) {
  const int sg = mass > T(0) ? 1 : (mass < T(0) ? -1 : 0);
  __builtin_amdgcn_raw_buffer_store_b8((unsigned char)sg, rsrc(f.sg[A], bytes / sizeof(T)),
                                       (unsigned)p, 0, 0);
}

// Flux of the A-face at point p, all 7 components and the sign stored.
template <class T, int A, int RS, bool FO>
__device__ __forceinline__ int face_flux(const Physics& ph, unsigned bytes, const Stencil<T>& st,
                                         const Flux<T>& f, const Muscl<T>& mu, int p) {
  const unsigned o = (unsigned)p * (unsigned)sizeof(T);
  T F[7];
  const int code = face_solve<T, RS, FO>(ph, st, mu, F);
#pragma unroll
  for (int m = 0; m < 7; ++m) bst(F[m], rsrc(f.f[A][m], bytes), o);
  store_sign<T, A>(bytes, f, F[0], p);
  return code;
}

// FP32: the loads of all three stencils are issued before the first
// Riemann solve, so each wave keeps 84 loads in flight instead of 28 (the
// sweep waits on memory latency more than on either roof; fewer waves fit,
// 4-5 per SIMD instead of 7, and the launch is still about 10 % faster).
// FP64 holds half as many values per register file and goes face by face.
template <class T, int RS, bool FO>
__device__ __forceinline__ void flux_point(const Geo& g, const Physics& ph, int i, int j, int k,
                                           int p, const Prim<T>& w, const T* __restrict__ bx,
                                           const T* __restrict__ by, const T* __restrict__ bz,
                                           const Flux<T>& f, const Muscl<T>& mu, int& cx, int& cy,
                                           int& cz) {
  const unsigned bytes = (unsigned)g.np * (unsigned)sizeof(T);
  if constexpr (sizeof(T) == 4) {
    const Stencil<T> sx = load_stencil<T, 0, FO>(1, bytes, w, bx, p);
    const Stencil<T> sy = load_stencil<T, 1, FO>(g.sy, bytes, w, by, p);
    const Stencil<T> sz = load_stencil<T, 2, FO>(g.sz, bytes, w, bz, p);
    if (i >= 0) cx = face_flux<T, 0, RS, FO>(ph, bytes, sx, f, mu, p);
    if (j >= 0) cy = face_flux<T, 1, RS, FO>(ph, bytes, sy, f, mu, p);
    if (k >= 0) cz = face_flux<T, 2, RS, FO>(ph, bytes, sz, f, mu, p);
  } else {
    if (i >= 0)
      cx = face_flux<T, 0, RS, FO>(ph, bytes, load_stencil<T, 0, FO>(1, bytes, w, bx, p), f, mu,
                                   p);
    if (j >= 0)
      cy = face_flux<T, 1, RS, FO>(ph, bytes, load_stencil<T, 1, FO>(g.sy, bytes, w, by, p), f,
                                   mu, p);
    if (k >= 0)
      cz = face_flux<T, 2, RS, FO>(ph, bytes, load_stencil<T, 2, FO>(g.sz, bytes, w, bz, p), f,
                                   mu, p);
  }
}

__device__ __forceinline__ void count_codes(const Counters& cnt, int cx, int cy, int cz) {
  wave_count((cx & 1) != 0, cnt.hll);
  wave_count((cy & 1) != 0, cnt.hll);
  wave_count((cz & 1) != 0, cnt.hll);
  wave_count((cx & 2) != 0, cnt.deg);
  wave_count((cy & 2) != 0, cnt.deg);
  wave_count((cz & 2) != 0, cnt.deg);
}

template <class T, int RS, bool FO>
__global__ void __launch_bounds__(kSpanThreads) k_flux(Geo g, Physics ph, Span sp, Prim<T> w,
                                                       const T* __restrict__ bx,
                                                       const T* __restrict__ by,
                                                       const T* __restrict__ bz, Flux<T> f,
                                                       Muscl<T> mu, Counters cnt) {
  const Pt pt = span_point(g, sp);
  int cx = 0, cy = 0, cz = 0;
  if (pt.valid) flux_point<T, RS, FO>(g, ph, pt.i, pt.j, pt.k, pt.p, w, bx, by, bz, f, mu, cx, cy, cz);
  count_codes(cnt, cx, cy, cz);
}

// Thread t -> point c of the outer layer of the flux range, [-1, n]^3
// without [0, n-1]^3: the two z-layers as whole planes, the two y-layers
// of the inner planes as whole rows, then the two x-points at the ends of
// each inner row; false past the last one.
__device__ __forceinline__ bool flux_shell_point(const Geo& g, int t, int c[3]) {
  const int w0 = g.n[0] + 2, w1 = g.n[1] + 2;
  const int nzl = 2 * w0 * w1, nyl = 2 * w0 * g.n[2], nxl = 2 * g.n[1] * g.n[2];
  if (t < nzl) {
    const int l = t / (w0 * w1), r = t - l * w0 * w1;
    c[2] = l == 0 ? -1 : g.n[2];
    c[1] = r / w0 - 1;
    c[0] = r % w0 - 1;
  } else if (t < nzl + nyl) {
    t -= nzl;
    const int k = t / (2 * w0), r = t - k * (2 * w0), l = r / w0;
    c[2] = k;
    c[1] = l == 0 ? -1 : g.n[1];
    c[0] = r - l * w0 - 1;
  } else if (t < nzl + nyl + nxl) {
    t -= nzl + nyl;
    const int l = t & 1, r = t >> 1;
    c[2] = r / g.n[1];
    c[1] = r - c[2] * g.n[1];
    c[0] = l == 0 ? -1 : g.n[0];
  } else {
    return false;
  }
  return true;
}

static int flux_shell_points(const Geo& g) {
  const int w0 = g.n[0] + 2, w1 = g.n[1] + 2;
  return 2 * (w0 * w1 + w0 * g.n[2] + g.n[1] * g.n[2]);
}

// A point of the outer layer whose out-of-range coordinates all lie on
// periodic axes is the periodic image of an interior point, whose faces the
// sweep has solved from the same stencil values: its faces are copied from
// there (bitwise what solving them would give; the sweep counted their
// solver events, face_copies).  Elsewhere (an outflow or inflow side) they
// are solved.  Runs after the sweep.
template <class T, int RS, bool FO>
__global__ void __launch_bounds__(256) k_flux_shell(Geo g, Physics ph, Prim<T> w,
                                                    const T* __restrict__ bx,
                                                    const T* __restrict__ by,
                                                    const T* __restrict__ bz, Flux<T> f,
                                                    Muscl<T> mu, Counters cnt) {
  int c[3];
  int cx = 0, cy = 0, cz = 0;
  if (flux_shell_point(g, (int)(blockIdx.x * 256u + threadIdx.x), c)) {
    const int p = pidx(g, c[0], c[1], c[2]);
    int m[3];
    bool image = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      m[a] = c[a];
      if (c[a] < 0 || c[a] >= g.n[a]) {
        if (g.nf[a] == g.n[a])
          m[a] = c[a] < 0 ? c[a] + g.n[a] : c[a] - g.n[a];
        else
          image = false;
      }
    }
    if (image) {
      const int q = pidx(g, m[0], m[1], m[2]);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if (c[a] < 0) continue;  // no A-face at index -1
#pragma unroll
        for (int k = 0; k < 7; ++k) f.f[a][k][p] = f.f[a][k][q];
        f.sg[a][p] = f.sg[a][q];
      }
    } else {
      flux_point<T, RS, FO>(g, ph, c[0], c[1], c[2], p, w, bx, by, bz, f, mu, cx, cy, cz);
    }
  }
  count_codes(cnt, cx, cy, cz);
}

// ------------------------------------------------------------------------
// Fused flux sweep and conservative update of a stage (Eq. 7 with the
// cell-centred source).  A block of kSwX x kSwY threads owns a tile of
// kSwX x kSwY cell columns and walks kSwZ planes of them in z.  At each
// plane a thread computes the three lower faces of its cell; the upper x
// face comes from the next lane (a wave is one x-row of the tile), the
// upper y face from the next row through LDS, the upper z face from the
// next plane's step, whose z-stencil the thread keeps in registers.  Each
// flux is therefore computed once and its hydrodynamic components never
// go to memory, except on the seams of the tiles: the upper faces of a
// tile's last column, row and plane belong to the neighbouring tile (or,
// at index n, to the outer layer), which stores them to f; the stage
// update adds them.  The field components and mass-flux signs of every
// face go to f for the EMFs.
// ------------------------------------------------------------------------

// The sweep addresses its ~45 arrays as a 64-bit scalar base plus a 32-bit
// byte offset per lane (global loads and stores in their scalar-base form):
// two SGPRs an array, where a buffer resource takes four and the kernel's
// resources would no longer fit the scalar register file (spilled to
// vector-register lanes, a read and a write lane instruction per use).
template <class T>
__device__ __forceinline__ T gld(const T* base, unsigned off) {
  return *(const T*)((const char*)base + off);
}
template <class T>
__device__ __forceinline__ void gst(T* base, unsigned off, T v) {
  *(T*)((char*)base + off) = v;
}

// The 7 variables of one point of the A-face stencil (the order of
// load_stencil): rho, v_n, v_t1, v_t2, P, B_t1, B_t2.
template <class T, int A>
__device__ __forceinline__ void load_point(const Prim<T>& w, unsigned o, T v[7]) {
  constexpr int A1 = (A + 1) % 3, A2 = (A + 2) % 3;
  const T* src[7] = {w.w[0], w.w[1 + A], w.w[1 + A1], w.w[1 + A2], w.w[4], w.w[5 + A1], w.w[5 + A2]};
#pragma unroll
  for (int q = 0; q < 7; ++q) v[q] = gld(src[q], o);
}

// The A-face stencil of the cell at byte offset o and its face-normal
// field, as load_stencil; the points two below, one below and one above the
// cell lie at o + dm2, o + dm1, o + dp1 (modulo 2^32).
template <class T, int A, bool FO>
__device__ __forceinline__ Stencil<T> sweep_stencil(unsigned dm2, unsigned dm1, unsigned dp1,
                                                    const Prim<T>& w, const T* __restrict__ bn,
                                                    unsigned o) {
  Stencil<T> st;
  T v[7];
  if constexpr (!FO) {
    load_point<T, A>(w, o + dm2, v);
#pragma unroll
    for (int c = 0; c < 7; ++c) st.v[c][0] = v[c];
    load_point<T, A>(w, o + dp1, v);
#pragma unroll
    for (int c = 0; c < 7; ++c) st.v[c][3] = v[c];
  } else {
#pragma unroll
    for (int c = 0; c < 7; ++c) st.v[c][0] = st.v[c][3] = T(0);
  }
  load_point<T, A>(w, o + dm1, v);
#pragma unroll
  for (int c = 0; c < 7; ++c) st.v[c][1] = v[c];
  load_point<T, A>(w, o, v);
#pragma unroll
  for (int c = 0; c < 7; ++c) st.v[c][2] = v[c];
  st.bn = gld(bn, o);
  return st;
}

// Stores of a face solved by the sweep: field components and sign always;
// mass flux (store >= 1) or every component (store 2); the hydrodynamic
// components also if seam (another tile's cell needs them).
template <class T, int A>
__device__ __forceinline__ void store_face(const Flux<T>& f, const T F[7], unsigned o, int p,
                                           int store, bool seam) {
  gst(f.f[A][5], o, F[5]);
  gst(f.f[A][6], o, F[6]);
  f.sg[A][p] = F[0] > T(0) ? 1 : (F[0] < T(0) ? -1 : 0);
  const int cn = (seam || store >= 2) ? 5 : (store >= 1 ? 1 : 0);
  for (int c = 0; c < cn; ++c) gst(f.f[A][c], o, F[c]);
}

struct SweepGrid {
  int ntx, nty, nch, nblk;
};

// FP32: compiled for at least 4 waves per SIMD (at most 128 VGPRs).  The
// MUSCL variant then spills a few registers to scratch, which costs less
// than the fourth wave gains; the FP64 variants would spill heavily and keep
// the compiler's choice.
//
// INC (compensated FP32): s0's cells are not read; s1's cells receive the
// stage increment (the update without s0's value).
template <class T, int RS, bool FO, bool INC>
__global__ void __launch_bounds__(kSwX* kSwY)
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1, 8)))
    k_sweep(Geo g, Physics ph, SweepGrid sgd, Prim<T> w, Cons<T> s0, Cons<T> s1, Flux<T> f,
            Muscl<T> mu, Grav<T> gr, DtRef dtr, Counters cnt, int store) {
  static_assert(kSwX == 64, "a wave is one x-row of the tile");
  __shared__ T fy_up[2][5][kSwY][kSwX];
  // blocks -> (tile x, tile y, z-chunk), each XCD a contiguous range (the
  // hardware deals block b to XCD b mod 8): neighbouring tiles of the same
  // planes share that XCD's L2
  const unsigned nb = (unsigned)sgd.nblk, b0 = blockIdx.x;
  const unsigned q = nb >> 3, r = nb & 7u, x8 = b0 & 7u;
  const int b = (int)(x8 * q + (x8 < r ? x8 : r) + (b0 >> 3));
  const int tx = b % sgd.ntx, rest = b / sgd.ntx;
  const int ty = rest % sgd.nty, ch = rest / sgd.nty;
  const int lx = (int)threadIdx.x % kSwX, ly = (int)threadIdx.x / kSwX;
  const int i = tx * kSwX + lx, j = ty * kSwY + ly;
  const int k0 = ch * kSwZ, k1 = min(k0 + kSwZ, g.n[2]);
  const bool act = i < g.n[0] && j < g.n[1];
  const bool x_up = lx < kSwX - 1 && i + 1 < g.n[0];
  const bool y_up = ly < kSwY - 1 && j + 1 < g.n[1];
  const unsigned es = (unsigned)sizeof(T);
  // byte offsets of the x- and y-stencils' points from the cell: on a
  // periodic axis they wrap onto the interior images, so the ghost layers of
  // the primitives are never read there (the z-stencil's planes likewise)
  const unsigned xm2 = axis_step(g, 0, i, -2) * es, xm1 = axis_step(g, 0, i, -1) * es,
                 xp1 = axis_step(g, 0, i, 1) * es;
  const unsigned sy = (unsigned)g.sy * es, sz = (unsigned)g.sz * es;
  const unsigned ym2 = axis_step(g, 1, j, -2) * sy, ym1 = axis_step(g, 1, j, -1) * sy,
                 yp1 = axis_step(g, 1, j, 1) * sy;
  const double dt = (dtr.ptr ? *dtr.ptr : dtr.value) * dtr.factor;
  const T rx = (T)(dt / g.d[0]), ry = (T)(dt / g.d[1]), rz = (T)(dt / g.d[2]), dtT = (T)dt;
  // z-stencil of the z-face at plane k: planes k-2..k+1 in zs.v[.][0..3]
  // (first order: k-1, k in [1], [2])
  Stencil<T> zs;
#pragma unroll
  for (int c = 0; c < 7; ++c) zs.v[c][0] = zs.v[c][1] = zs.v[c][2] = zs.v[c][3] = T(0);
  if (act) {
    const unsigned o = (unsigned)pidx(g, i, j, k0) * es;
    T v[7];
    if constexpr (!FO) {
      load_point<T, 2>(w, o + axis_step(g, 2, k0, -2) * sz, v);
#pragma unroll
      for (int c = 0; c < 7; ++c) zs.v[c][0] = v[c];
      load_point<T, 2>(w, o, v);
#pragma unroll
      for (int c = 0; c < 7; ++c) zs.v[c][2] = v[c];
    }
    load_point<T, 2>(w, o + axis_step(g, 2, k0, -1) * sz, v);
#pragma unroll
    for (int c = 0; c < 7; ++c) zs.v[c][1] = v[c];
  }
  T up[5] = {T(0), T(0), T(0), T(0), T(0)};  // cell k-1 without its upper z flux
  int hll = 0, deg = 0;
  for (int k = k0; k < k1; ++k) {
    const int p = pidx(g, i, j, k);
    const unsigned o = (unsigned)p * es;
    T Fx[7], Fy[7], Fz[7];
    T un[5], S[5];
    if (!act) {  // lanes outside the box still feed the exchanges
#pragma unroll
      for (int c = 0; c < 5; ++c) Fx[c] = Fy[c] = T(0);
    } else {
      {  // the plane the z-stencil gains: k+1 (first order: k)
        T v[7];
        load_point<T, 2>(w, FO ? o : o + axis_step(g, 2, k, 1) * sz, v);
#pragma unroll
        for (int c = 0; c < 7; ++c) zs.v[c][FO ? 2 : 3] = v[c];
      }
      zs.bn = gld(s0.b[2], o);
      // one face family at a time, each stored as soon as it is solved (the
      // scheduling barriers keep a family's stencil loads next to its solve:
      // hoisting every load ahead of the first solve costs waves per SIMD).
      // To f: the field components and the sign of every face, the mass
      // flux if asked, the hydrodynamic components of the faces that other
      // tiles need (first column, row and plane of the tile).
      {
        const Stencil<T> sx = sweep_stencil<T, 0, FO>(xm2, xm1, xp1, w, s0.b[0], o);
        const int cx = face_solve<T, RS, FO>(ph, sx, mu, Fx);
        const int cc[3] = {i, j, k};
        if (cx) {
          const int mult = face_copies(g, cc, 0);
          hll += (cx & 1) * mult;
          deg += ((cx >> 1) & 1) * mult;
        }
        store_face<T, 0>(f, Fx, o, p, store, lx == 0);
      }
      __builtin_amdgcn_sched_barrier(0);
      {
        const Stencil<T> sy_st = sweep_stencil<T, 1, FO>(ym2, ym1, yp1, w, s0.b[1], o);
        const int cy = face_solve<T, RS, FO>(ph, sy_st, mu, Fy);
        const int cc[3] = {i, j, k};
        if (cy) {
          const int mult = face_copies(g, cc, 1);
          hll += (cy & 1) * mult;
          deg += ((cy >> 1) & 1) * mult;
        }
        store_face<T, 1>(f, Fy, o, p, store, ly == 0);
      }
      __builtin_amdgcn_sched_barrier(0);
      {
        const int cz = face_solve<T, RS, FO>(ph, zs, mu, Fz);
        const int cc[3] = {i, j, k};
        if (cz) {
          const int mult = face_copies(g, cc, 2);
          hll += (cz & 1) * mult;
          deg += ((cz >> 1) & 1) * mult;
        }
        store_face<T, 2>(f, Fz, o, p, store, k == k0);
      }
      // the stage's base value (INC: none, s1 gets the increment)
#pragma unroll
      for (int m = 0; m < 5; ++m) un[m] = INC ? T(0) : gld(s0.u[m], o);
      // source from the stage's primitives at the cell (z-frame order of
      // the z-stencil: rho, vz, vx, vy, ...)
      cell_source<T>(g, ph, gr, i, j, k, p, zs.v[0][2], zs.v[2][2], zs.v[3][2], zs.v[1][2], S);
    }
    // upper y faces through LDS (double buffered: one barrier a plane),
    // upper x faces from the next lane
    const int buf = (k - k0) & 1;
#pragma unroll
    for (int c = 0; c < 5; ++c) fy_up[buf][c][ly][lx] = Fy[c];
    __syncthreads();
    T fyu[5], fxu[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      fyu[c] = y_up ? fy_up[buf][c][ly + 1][lx] : T(0);
      fxu[c] = __shfl_down(Fx[c], 1, 64);
      if (!x_up) fxu[c] = T(0);
    }
    if (act) {
      if (k > k0) {  // the z-face at k is the upper face of cell k-1
        const unsigned om = o - (unsigned)g.sz * es;
#pragma unroll
        for (int m = 0; m < 5; ++m) gst(s1.u[m], om, up[m] - rz * Fz[frame_comp(2, m)]);
      }
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const int ax = frame_comp(0, m), ay = frame_comp(1, m), az = frame_comp(2, m);
        T v = un[m];
        v -= rx * (fxu[ax] - Fx[ax]);
        v -= ry * (fyu[ay] - Fy[ay]);
        v += rz * Fz[az];
        v += dtT * S[m];
        up[m] = v;
      }
      // slide the z-stencil one plane up
#pragma unroll
      for (int c = 0; c < 7; ++c) {
        zs.v[c][0] = zs.v[c][1];
        zs.v[c][1] = zs.v[c][2];
        if constexpr (!FO) zs.v[c][2] = zs.v[c][3];
      }
    }
  }
  if (act && k1 > k0) {  // the chunk's last plane: its upper z-face is a seam
    const unsigned o = (unsigned)pidx(g, i, j, k1 - 1) * es;
#pragma unroll
    for (int m = 0; m < 5; ++m) gst(s1.u[m], o, up[m]);
  }
  wave_add(hll, cnt.hll);
  wave_add(deg, cnt.deg);
}

template <class T, int RS, bool FO>
static void launch_sweep_rs(const Geo& g, const Physics& ph, Prim<T> w, Cons<T> s0, Cons<T> s1,
                            Flux<T> f, Muscl<T> m, Grav<T> gr, DtRef dt, Counters c,
                            int store, bool inc, hipStream_t st) {
  SweepGrid sg;
  sg.ntx = (g.n[0] + kSwX - 1) / kSwX;
  sg.nty = (g.n[1] + kSwY - 1) / kSwY;
  sg.nch = (g.n[2] + kSwZ - 1) / kSwZ;
  sg.nblk = sg.ntx * sg.nty * sg.nch;
  if constexpr (sizeof(T) == 4) {
    if (inc) {
      hipLaunchKernelGGL((k_sweep<T, RS, FO, true>), dim3((unsigned)sg.nblk),
                         dim3(kSwX * kSwY), 0, st, g, ph, sg, w, s0, s1, f, m, gr, dt, c, store);
      return;
    }
  }
  hipLaunchKernelGGL((k_sweep<T, RS, FO, false>), dim3((unsigned)sg.nblk), dim3(kSwX * kSwY), 0,
                     st, g, ph, sg, w, s0, s1, f, m, gr, dt, c, store);
}

template <class T, int RS>
static void launch_outer_rs(const Geo& g, const Physics& ph, Prim<T> w, Cons<T> s, Flux<T> f,
                            Muscl<T> m, Counters c, int store, hipStream_t st) {
  // the x-layer (the last 2 n_y n_z points) of a periodic x axis is left out
  // unless every flux is kept: its readers take the images at x-index n-1
  // and 0 instead, which lie in the cache lines they already read (the
  // layer itself costs a line per row and array at both ends of the rows)
  int npt = flux_shell_points(g);
  if (g.nf[0] == g.n[0] && store < 2) npt -= 2 * g.n[1] * g.n[2];
  const dim3 gr((unsigned)((npt + 255) / 256)), bl(256);
  if (m.first_order)
    hipLaunchKernelGGL((k_flux_shell<T, RS, true>), gr, bl, 0, st, g, ph, w, s.b[0], s.b[1],
                       s.b[2], f, m, c);
  else
    hipLaunchKernelGGL((k_flux_shell<T, RS, false>), gr, bl, 0, st, g, ph, w, s.b[0], s.b[1],
                       s.b[2], f, m, c);
}

template <class T>
void launch_flux_outer(const Geo& g, const Physics& ph, Prim<T> w, Cons<T> s, Flux<T> f,
                       Muscl<T> m, Counters c, int store, hipStream_t st) {
  if (ph.riemann == kRiemannHLL)
    launch_outer_rs<T, kRiemannHLL>(g, ph, w, s, f, m, c, store, st);
  else if (ph.riemann == kRiemannHLLC)
    launch_outer_rs<T, kRiemannHLLC>(g, ph, w, s, f, m, c, store, st);
  else
    launch_outer_rs<T, kRiemannHLLD>(g, ph, w, s, f, m, c, store, st);
}

template <class T, int RS>
static void launch_sweep_fo(const Geo& g, const Physics& ph, Prim<T> w, Cons<T> s0, Cons<T> s1,
                            Flux<T> f, Muscl<T> m, Grav<T> gr, DtRef dt, Counters c,
                            int store, bool inc, hipStream_t st) {
  if (m.first_order)
    launch_sweep_rs<T, RS, true>(g, ph, w, s0, s1, f, m, gr, dt, c, store, inc, st);
  else
    launch_sweep_rs<T, RS, false>(g, ph, w, s0, s1, f, m, gr, dt, c, store, inc, st);
}

template <class T>
void launch_sweep(const Geo& g, const Physics& ph, Prim<T> w, Cons<T> s0, Cons<T> s1,
                  Flux<T> f, Muscl<T> m, Grav<T> gr, DtRef dt, Counters c, int store, bool inc,
                  hipStream_t st) {
  const int sm = store;
  if (ph.riemann == kRiemannHLL)
    launch_sweep_fo<T, kRiemannHLL>(g, ph, w, s0, s1, f, m, gr, dt, c, sm, inc, st);
  else if (ph.riemann == kRiemannHLLC)
    launch_sweep_fo<T, kRiemannHLLC>(g, ph, w, s0, s1, f, m, gr, dt, c, sm, inc, st);
  else
    launch_sweep_fo<T, kRiemannHLLD>(g, ph, w, s0, s1, f, m, gr, dt, c, sm, inc, st);
}

template <class T, int RS>
static void launch_flux_rs(const Geo& g, const Span& sp, const Physics& ph, Prim<T> w, Cons<T> s,
                           Flux<T> f, Muscl<T> m, Counters c, hipStream_t st) {
  const dim3 gr = span_grid(sp), bl(kSpanThreads);
  if (m.first_order)
    hipLaunchKernelGGL((k_flux<T, RS, true>), gr, bl, 0, st, g, ph, sp, w, s.b[0], s.b[1], s.b[2],
                       f, m, c);
  else
    hipLaunchKernelGGL((k_flux<T, RS, false>), gr, bl, 0, st, g, ph, sp, w, s.b[0], s.b[1],
                       s.b[2], f, m, c);
}

template <class T>
void launch_flux(const Geo& g, const Physics& ph, Prim<T> w, Cons<T> s, Flux<T> f, Muscl<T> m,
                 Counters c, hipStream_t st) {
  const Span sp = make_span(g, -1, g.n[0], -1, g.n[1], -1, g.n[2]);
  if (ph.riemann == kRiemannHLL)
    launch_flux_rs<T, kRiemannHLL>(g, sp, ph, w, s, f, m, c, st);
  else if (ph.riemann == kRiemannHLLC)
    launch_flux_rs<T, kRiemannHLLC>(g, sp, ph, w, s, f, m, c, st);
  else
    launch_flux_rs<T, kRiemannHLLD>(g, sp, ph, w, s, f, m, c, st);
}

template void launch_flux<double>(const Geo&, const Physics&, Prim<double>, Cons<double>,
                                  Flux<double>, Muscl<double>, Counters, hipStream_t);
template void launch_flux<float>(const Geo&, const Physics&, Prim<float>, Cons<float>,
                                 Flux<float>, Muscl<float>, Counters, hipStream_t);
template void launch_flux_outer<double>(const Geo&, const Physics&, Prim<double>, Cons<double>,
                                        Flux<double>, Muscl<double>, Counters, int, hipStream_t);
template void launch_flux_outer<float>(const Geo&, const Physics&, Prim<float>, Cons<float>,
                                       Flux<float>, Muscl<float>, Counters, int, hipStream_t);
template void launch_sweep<double>(const Geo&, const Physics&, Prim<double>, Cons<double>,
                                   Cons<double>, Flux<double>, Muscl<double>, Grav<double>,
                                   DtRef, Counters, int, bool, hipStream_t);
template void launch_sweep<float>(const Geo&, const Physics&, Prim<float>, Cons<float>,
                                  Cons<float>, Flux<float>, Muscl<float>, Grav<float>, DtRef,
                                  Counters, int, bool, hipStream_t);

}  // namespace mhd
