// mhd_flux.hip -- the flux sweep of the step (section 2.1 of the paper):
// limited MUSCL reconstruction (Eq. 12-14) of the face states and the
// Riemann solver (HLLD, or HLL / HLLC) on all three face families of the
// padded grid in one launch.
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
    st.v[v][0] = FO ? T(0) : bld(T(), q, o - 2 * s);
    st.v[v][1] = bld(T(), q, o - s);
    st.v[v][2] = bld(T(), q, o);
    st.v[v][3] = FO ? T(0) : bld(T(), q, o + s);
  }
  st.bn = bld(T(), rsrc(bn, bytes), o);
  return st;
}

// Flux of the A-face at point p from its stencil: limited reconstruction
// (Eq. 12-14; FO: first order), the Riemann solver, the sign of the mass
// flux.  Returns the HLLD branch code (bit 0 HLL fallback, bit 1
// degenerate; 0 for the other solvers).
template <class T, int A, int RS, bool FO>
__device__ __forceinline__ int face_flux(const Physics& ph, unsigned bytes, const Stencil<T>& st,
                                         const Flux<T>& f, const Muscl<T>& mu, int p) {
  const unsigned o = (unsigned)p * (unsigned)sizeof(T);
  T l[7], r[7];
#pragma unroll
  for (int v = 0; v < 7; ++v) {
    if constexpr (FO) {
      l[v] = st.v[v][1];
      r[v] = st.v[v][2];
    } else {
      muscl_lr(mu, st.v[v][0], st.v[v][1], st.v[v][2], st.v[v][3], l[v], r[v]);
    }
  }
  const Face<T> L{l[0], l[1], l[2], l[3], l[4], l[5], l[6]};
  const Face<T> R{r[0], r[1], r[2], r[3], r[4], r[5], r[6]};
  T F[7];
  const int code = riemann_flux<T, RS>(ph, L, R, st.bn, F);
#pragma unroll
  for (int m = 0; m < 7; ++m) bst(F[m], rsrc(f.f[A][m], bytes), o);
  const int sg = F[0] > T(0) ? 1 : (F[0] < T(0) ? -1 : 0);
  __builtin_amdgcn_raw_buffer_store_b8((unsigned char)sg, rsrc(f.sg[A], bytes / sizeof(T)),
                                       (unsigned)p, 0, 0);
  return code;
}

// FP32: the loads of all three stencils are issued before the first
// Riemann solve, so each wave keeps 84 loads in flight instead of 28 (the
// sweep waits on memory latency more than on either roof; fewer waves fit,
// 4-5 per SIMD instead of 7, and the launch is still about 10 % faster).
// FP64 holds half as many values per register file and goes face by face.
template <class T, int RS, bool FO>
__global__ void __launch_bounds__(kSpanThreads) k_flux(Geo g, Physics ph, Span sp, Prim<T> w,
                                                       const T* __restrict__ bx,
                                                       const T* __restrict__ by,
                                                       const T* __restrict__ bz, Flux<T> f,
                                                       Muscl<T> mu, Counters cnt) {
  const Pt pt = span_point(g, sp);
  int cx = 0, cy = 0, cz = 0;
  if (pt.valid) {
    const unsigned bytes = (unsigned)g.np * (unsigned)sizeof(T);
    if constexpr (sizeof(T) == 4) {
      const Stencil<T> sx = load_stencil<T, 0, FO>(1, bytes, w, bx, pt.p);
      const Stencil<T> sy = load_stencil<T, 1, FO>(g.sy, bytes, w, by, pt.p);
      const Stencil<T> sz = load_stencil<T, 2, FO>(g.sz, bytes, w, bz, pt.p);
      if (pt.i >= 0) cx = face_flux<T, 0, RS, FO>(ph, bytes, sx, f, mu, pt.p);
      if (pt.j >= 0) cy = face_flux<T, 1, RS, FO>(ph, bytes, sy, f, mu, pt.p);
      if (pt.k >= 0) cz = face_flux<T, 2, RS, FO>(ph, bytes, sz, f, mu, pt.p);
    } else {
      if (pt.i >= 0)
        cx = face_flux<T, 0, RS, FO>(ph, bytes, load_stencil<T, 0, FO>(1, bytes, w, bx, pt.p), f,
                                     mu, pt.p);
      if (pt.j >= 0)
        cy = face_flux<T, 1, RS, FO>(ph, bytes, load_stencil<T, 1, FO>(g.sy, bytes, w, by, pt.p),
                                     f, mu, pt.p);
      if (pt.k >= 0)
        cz = face_flux<T, 2, RS, FO>(ph, bytes, load_stencil<T, 2, FO>(g.sz, bytes, w, bz, pt.p),
                                     f, mu, pt.p);
    }
  }
  wave_count((cx & 1) != 0, cnt.hll);
  wave_count((cy & 1) != 0, cnt.hll);
  wave_count((cz & 1) != 0, cnt.hll);
  wave_count((cx & 2) != 0, cnt.deg);
  wave_count((cy & 2) != 0, cnt.deg);
  wave_count((cz & 2) != 0, cnt.deg);
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

}  // namespace mhd
