// mhd_kernels.hip -- HIP kernels (gfx950, wave64) of the ideal-MHD
// TVD-MUSCL step with constrained transport (section 2.1 of the paper).
//
// Structure-of-arrays padded grid (see Geo).  Each kernel maps x to the 64
// lanes of a wave so every global access of a wave is a contiguous x-run.
#include <float.h>
#include <math.h>

#include "mhd_kernels.hpp"
#include "mhd_mlp.hpp"
#include "mhd_source.hpp"
#include "mhd_span.hpp"

namespace mhd {

// ------------------------------------------------------------------------
// Ghost fill.  Every ghost point takes the value of the interior point found
// by mapping each coordinate on its own (periodic wrap / outflow clamp), or
// the inflow state if any coordinate lies in an inflow ghost zone.  This is
// the result of filling x, then y, then z over the full extended ranges.
// ------------------------------------------------------------------------

__device__ __forceinline__ int map_axis(int c, int m, int n, int bclo, int bchi, bool& inflow) {
  if (c >= 0 && c < m) return c;
  const int bc = c < 0 ? bclo : bchi;
  if (bc == 0) {
    int r = c % n;
    return r < 0 ? r + n : r;
  }
  if (bc == 1) return c < 0 ? 0 : m - 1;
  inflow = true;
  return c;
}

// Thread t -> ghost point c (the 5 ghost layers of x, then of y, then of z,
// over the full extent of the other two axes); false past the last one.
// nl = 1 keeps of each axis' layers only the points at index n, whose only
// value filled is that axis' face n (*face_only = the axis, else -1): on a
// fully periodic box the fused stage path reads every other ghost at its
// interior image, and the faces n give the last cells their cell-centred B
// in the kernels outside the step (diagnostics, time step).
__device__ __forceinline__ bool ghost_point(const Geo& g, long long t, int nl, int c[3],
                                           int& face_only) {
  const long long E0 = g.ext[0], E1 = g.ext[1], E2 = g.ext[2];
  const long long nx = nl * E1 * E2, ny = nl * E0 * E2, nz = nl * E0 * E1;
  long long r;
  face_only = -1;
  if (t < nx) {
    const int l = nl == 5 ? (int)(t % 5) : 2;
    r = t / nl;
    c[0] = l < 2 ? l - 2 : g.n[0] + (l - 2);
    c[1] = (int)(r % E1) - NG;
    c[2] = (int)(r / E1) - NG;
    if (nl != 5) face_only = 0;
  } else if (t < nx + ny) {  // x fastest: a wave covers a run of one row
    r = t - nx;
    c[0] = (int)(r % E0) - NG;
    r /= E0;
    const int l = nl == 5 ? (int)(r % 5) : 2;
    c[1] = l < 2 ? l - 2 : g.n[1] + (l - 2);
    c[2] = (int)(r / nl) - NG;
    if (nl != 5) face_only = 1;
  } else if (t < nx + ny + nz) {
    r = t - nx - ny;
    c[0] = (int)(r % E0) - NG;
    r /= E0;
    c[1] = (int)(r % E1) - NG;
    const int l = nl == 5 ? (int)(r / E1) : 2;
    c[2] = l < 2 ? l - 2 : g.n[2] + (l - 2);
    if (nl != 5) face_only = 2;
  } else {
    return false;
  }
  return true;
}

static unsigned ghost_blocks(const Geo& g, int bs, int nl) {
  const long long tot =
      (long long)nl * ((long long)g.ext[1] * g.ext[2] + (long long)g.ext[0] * g.ext[2] +
                       (long long)g.ext[0] * g.ext[1]);
  return (unsigned)((tot + bs - 1) / bs);
}

template <class T>
__global__ void k_ghosts(Geo g, Physics ph, Cons<T> s, int nl) {
  int c[3];
  int face_only;
  if (!ghost_point(g, (long long)blockIdx.x * blockDim.x + threadIdx.x, nl, c, face_only)) return;
  const int p = pidx(g, c[0], c[1], c[2]);
  // every source value is loaded before the first store (a store through
  // one array pointer would otherwise order the next array's load after it)
  T v[8];
  float vl[5];  // compensated FP32: the low parts of the cell pairs
  bool put[8];
  const bool comp = s.lo[0] != nullptr;
  // cell arrays
  {
    bool inflow = false;
    int m[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      m[a] = map_axis(c[a], g.n[a], g.n[a], g.bc[2 * a], g.bc[2 * a + 1], inflow);
    const bool moved = m[0] != c[0] || m[1] != c[1] || m[2] != c[2];
    const int q0 = pidx(g, m[0], m[1], m[2]);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      put[q] = face_only < 0 && (inflow || moved);
      v[q] = !put[q] ? T(0) : (inflow ? (T)ph.inflow_u[q] : s.u[q][q0]);
      vl[q] = 0.f;
      if (comp && put[q]) {
        if (inflow) {
          float h;
          pair_split(ph.inflow_u[q], h, vl[q]);
          v[q] = (T)h;
        } else {
          vl[q] = s.lo[q][q0];
        }
      }
    }
  }
  // face arrays: the normal axis has nf interior entries
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    bool inflow = false;
    int m[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      m[a] = map_axis(c[a], a == f ? g.nf[a] : g.n[a], g.n[a], g.bc[2 * a], g.bc[2 * a + 1],
                      inflow);
    const bool moved = m[0] != c[0] || m[1] != c[1] || m[2] != c[2];
    put[5 + f] = (face_only < 0 || f == face_only) && (inflow || moved);
    v[5 + f] = !put[5 + f] ? T(0)
                           : (inflow ? (T)ph.inflow_b[f] : s.b[f][pidx(g, m[0], m[1], m[2])]);
  }
#pragma unroll
  for (int q = 0; q < 5; ++q)
    if (put[q]) {
      s.u[q][p] = v[q];
      if (comp) s.lo[q][p] = vl[q];
    }
#pragma unroll
  for (int f = 0; f < 3; ++f)
    if (put[5 + f]) s.b[f][p] = v[5 + f];
}

template <class T>
void launch_ghosts(const Geo& g, const Physics& ph, Cons<T> s, bool lite, hipStream_t st) {
  const int nl = lite ? 1 : 5;
  hipLaunchKernelGGL(k_ghosts<T>, dim3(ghost_blocks(g, 256, nl)), dim3(256), 0, st, g, ph, s,
                     nl);
}

// ------------------------------------------------------------------------
// Primitive recovery (Eq. 6 cell-centred B, P from Eq. 3) and cell EMF
// E = -v x B (Eq. 9) on all cells that have both faces: [-NG, n+NG-1]^3.
// FP32: cells that lose more than 6 bits in E - KE - ME (E/(E-KE-ME) > 64)
// redo KE, ME and P in FP64 from the stored FP32 values.
//
// The primitives, the CT face update and the CFL candidates are computed in
// more than one kernel (the primitive pass, the ghost-shell pass, the fused
// stage update) and must agree bitwise there: their functions contract a*b+c
// into an FMA only within one expression (fp contract(on)), so the result
// does not depend on which subexpressions a kernel happens to share.
// ------------------------------------------------------------------------

template <class T>
__device__ __forceinline__ T pressure(T gam, T rho, T mx, T my, T mz, T E, T b0x, T b1x, T b0y,
                                      T b1y, T b0z, T b1z, T& bcx, T& bcy, T& bcz, bool& rec,
                                      bool recover) {
#pragma clang fp contract(on)
  bcx = T(0.5) * (b0x + b1x);
  bcy = T(0.5) * (b0y + b1y);
  bcz = T(0.5) * (b0z + b1z);
  const T ke = T(0.5) * (mx * mx + my * my + mz * mz) * rcp(rho);
  const T me = T(0.5) * (bcx * bcx + bcy * bcy + bcz * bcz);
  const T eint = E - ke - me;
  rec = false;
  if constexpr (sizeof(T) == 4) {
    if (recover && !(T(64) * eint > E)) {
      const double bx = 0.5 * ((double)b0x + (double)b1x);
      const double by = 0.5 * ((double)b0y + (double)b1y);
      const double bz = 0.5 * ((double)b0z + (double)b1z);
      const double ked = 0.5 * ((double)mx * mx + (double)my * my + (double)mz * mz) / (double)rho;
      const double med = 0.5 * (bx * bx + by * by + bz * bz);
      rec = true;
      return (T)(((double)gam - 1.0) * ((double)E - ked - med));
    }
  }
  return (gam - T(1)) * eint;
}

// ------------------------------------------------------------------------
// Block reductions (256 threads = 4 waves of 64): wave shuffles, then the
// four wave results in fixed order.  Deterministic for a fixed launch.
// ------------------------------------------------------------------------

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Time-step candidate of one interior cell from its conserved state: the
// smallest dx_a / (|v_a| + c_f,a) over the three axes, in FP64 (the
// start-of-step state of a step that computes its own dt), formed as the
// inverse of the largest (|v_a| + c_f,a) / dx_a with one reciprocal of the
// density (two divisions a cell, where one per quotient took eight).  A
// non-finite value, rho <= 0 or P <= 0 sets the sticky status bit and
// gives +inf.
template <class T>
__device__ __forceinline__ double cfl_cell(const Geo& g, const Physics& ph, T rho_, T mx_, T my_,
                                           T mz_, T E_, T b0x, T b1x, T b0y, T b1y, T b0z, T b1z,
                                           unsigned* status) {
#pragma clang fp contract(on)
  const double rho = rho_, mx = mx_, my = my_, mz = mz_, E = E_;
  const double bc[3] = {0.5 * ((double)b0x + (double)b1x), 0.5 * ((double)b0y + (double)b1y),
                        0.5 * ((double)b0z + (double)b1z)};
  const double ir = 1.0 / rho;
  const double ke = 0.5 * (mx * mx + my * my + mz * mz) * ir;
  const double me = 0.5 * (bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
  const double P = (ph.gamma - 1.0) * (E - ke - me);
  const double v[3] = {mx * ir, my * ir, mz * ir};
  const bool ok = rho > 0.0 && P > 0.0 && isfinite(E) && isfinite(mx) && isfinite(my) &&
                  isfinite(mz) && isfinite(bc[0]) && isfinite(bc[1]) && isfinite(bc[2]);
  if (!ok) {
    atomicOr(status, 1u);
    return INFINITY;
  }
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double cf = fast_speed_id<double>(ir, P, bc[a], bc[(a + 1) % 3], bc[(a + 2) % 3],
                                            ph.gamma);
    const double w = (fabs(v[a]) + cf) * g.id[a];
    s = w > s ? w : s;
  }
  return 1.0 / s;
}

// Block minimum of r (kSpanThreads threads) into part[blockIdx.x].
__device__ __forceinline__ void block_min_to(double r, double* part) {
  __shared__ double red[kSpanThreads / 64];
  r = wave_min(r);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = red[0];
    for (int q = 1; q < kSpanThreads / 64; ++q) m = fmin(m, red[q]);
    part[blockIdx.x] = m;
  }
}

// Primitives and cell EMF of the cell at p from its conserved values and
// its lower (b0*) and upper (b1*) faces.  One function for every pass that
// writes primitives, so that they agree bitwise for the same inputs.  The
// primitive density is the state's own density array (w.w[0] is the cell
// array of the conserved set the primitives belong to), not written here.
template <class T>
__device__ __forceinline__ void store_prim(T gam, const Prim<T>& w, int p, T rho, T mx, T my,
                                           T mz, T E, T b0x, T b1x, T b0y, T b1y, T b0z, T b1z,
                                           bool& rec, bool recover) {
#pragma clang fp contract(on)
  T bcx, bcy, bcz;
  const T P = pressure(gam, rho, mx, my, mz, E, b0x, b1x, b0y, b1y, b0z, b1z, bcx, bcy, bcz, rec,
                       recover);
  const T ir = rcp(rho);
  const T vx = mx * ir, vy = my * ir, vz = mz * ir;
  w.w[1][p] = vx;
  w.w[2][p] = vy;
  w.w[3][p] = vz;
  w.w[4][p] = P;
  w.w[5][p] = bcx;
  w.w[6][p] = bcy;
  w.w[7][p] = bcz;
  w.ec[0][p] = vz * bcy - vy * bcz;
  w.ec[1][p] = vx * bcz - vz * bcx;
  w.ec[2][p] = vy * bcx - vx * bcy;
}

// Compensated FP32: primitives and cell EMF of a cell from the FP64 values
// of its pairs and its FP32 faces, every quantity in FP64 and rounded once
// to FP32 (every pass that writes primitives uses this function).
__device__ __forceinline__ void store_prim_comp(double gam, const Prim<float>& w, int p,
                                                const double u[5], float b0x, float b1x,
                                                float b0y, float b1y, float b0z, float b1z) {
  const double bcx = 0.5 * ((double)b0x + (double)b1x);
  const double bcy = 0.5 * ((double)b0y + (double)b1y);
  const double bcz = 0.5 * ((double)b0z + (double)b1z);
  const double ir = 1.0 / u[0];
  const double vx = u[1] * ir, vy = u[2] * ir, vz = u[3] * ir;
  const double ke = 0.5 * (u[1] * vx + u[2] * vy + u[3] * vz);
  const double me = 0.5 * (bcx * bcx + bcy * bcy + bcz * bcz);
  w.w[1][p] = (float)vx;
  w.w[2][p] = (float)vy;
  w.w[3][p] = (float)vz;
  w.w[4][p] = (float)((gam - 1.0) * (u[4] - ke - me));
  w.w[5][p] = (float)bcx;
  w.w[6][p] = (float)bcy;
  w.w[7][p] = (float)bcz;
  w.ec[0][p] = (float)(vz * bcy - vy * bcz);
  w.ec[1][p] = (float)(vx * bcz - vz * bcx);
  w.ec[2][p] = (float)(vy * bcx - vx * bcy);
}

// The FP64 values of the five cell pairs of s at p.
__device__ __forceinline__ void load_pairs(const Cons<float>& s, int p, double u[5]) {
#pragma unroll
  for (int m = 0; m < 5; ++m) u[m] = pair_value(s.u[m][p], s.lo[m][p]);
}

// CFL = true: the interior cells also give their time-step candidates,
// folded per block into part[] (the step's own dt, from the same loads).
template <class T, bool CFL>
__global__ void __launch_bounds__(kSpanThreads) k_prim(Geo g, Physics ph, Span sp, Cons<T> s,
                                                       Prim<T> w, Counters cnt, double* part) {
  const Pt pt = span_point(g, sp);
  bool rec = false;
  double r = INFINITY;
  if (pt.valid) {
    const int p = pt.p;
    const T rho = s.u[0][p], mx = s.u[1][p], my = s.u[2][p], mz = s.u[3][p], E = s.u[4][p];
    const T b0x = s.b[0][p], b1x = s.b[0][p + 1], b0y = s.b[1][p], b1y = s.b[1][p + g.sy];
    const T b0z = s.b[2][p], b1z = s.b[2][p + g.sz];
    const bool inside =
        pt.i >= 0 && pt.i < g.n[0] && pt.j >= 0 && pt.j < g.n[1] && pt.k >= 0 && pt.k < g.n[2];
    bool done = false;
    if constexpr (sizeof(T) == 4) {
      if (s.lo[0]) {  // compensated FP32
        double u[5];
        load_pairs(s, p, u);
        store_prim_comp(ph.gamma, w, p, u, b0x, b1x, b0y, b1y, b0z, b1z);
        if (CFL && inside)
          r = cfl_cell<double>(g, ph, u[0], u[1], u[2], u[3], u[4], b0x, b1x, b0y, b1y, b0z,
                               b1z, cnt.status);
        done = true;
      }
    }
    if (!done) {
      store_prim((T)ph.gamma, w, p, rho, mx, my, mz, E, b0x, b1x, b0y, b1y, b0z, b1z, rec,
                 ph.recover);
      if (CFL && inside)
        r = cfl_cell<T>(g, ph, rho, mx, my, mz, E, b0x, b1x, b0y, b1y, b0z, b1z, cnt.status);
    }
  }
  if constexpr (sizeof(T) == 4) wave_count(rec, cnt.fp64_rec);
  if constexpr (CFL) block_min_to(r, part);
}

// Thread t -> cell c of the ghost shell, [-NG, n+NG-1]^3 without the
// interior [0, n-1]^3: the 2 NG z-layers as whole planes, then the 2 NG
// y-layers of the interior planes as whole rows, then the 2 NG x-cells at
// the ends of each interior row; false past the last one.
__device__ __forceinline__ bool shell_cell(const Geo& g, int t, int c[3]) {
  const int w0 = g.n[0] + 2 * NG, w1 = g.n[1] + 2 * NG;
  const int nzl = 2 * NG * w0 * w1, nyl = 2 * NG * w0 * g.n[2];
  const int nxl = 2 * NG * g.n[1] * g.n[2];
  int l;
  if (t < nzl) {
    l = t / (w0 * w1);
    const int r = t - l * w0 * w1;
    c[2] = l < NG ? l - NG : g.n[2] + (l - NG);
    c[1] = r / w0 - NG;
    c[0] = r % w0 - NG;
  } else if (t < nzl + nyl) {
    t -= nzl;
    const int k = t / (2 * NG * w0);
    const int r = t - k * (2 * NG * w0);
    l = r / w0;
    c[2] = k;
    c[1] = l < NG ? l - NG : g.n[1] + (l - NG);
    c[0] = r - l * w0 - NG;
  } else if (t < nzl + nyl + nxl) {
    t -= nzl + nyl;
    l = t % (2 * NG);
    const int r = t / (2 * NG);
    c[2] = r / g.n[1];
    c[1] = r - c[2] * g.n[1];
    c[0] = l < NG ? l - NG : g.n[0] + (l - NG);
  } else {
    return false;
  }
  return true;
}

static int shell_cells(const Geo& g) {
  const int w0 = g.n[0] + 2 * NG, w1 = g.n[1] + 2 * NG;
  return 2 * NG * (w0 * w1 + w0 * g.n[2] + g.n[1] * g.n[2]);
}

// Primitives of the ghost shell (after a full ghost fill; the interior
// cells' come from the stage update).
template <class T>
__global__ void __launch_bounds__(256) k_prim_shell(Geo g, Physics ph, Cons<T> s, Prim<T> w,
                                                    Counters cnt) {
  int c[3];
  bool rec = false;
  if (shell_cell(g, (int)(blockIdx.x * 256u + threadIdx.x), c)) {
    const int p = pidx(g, c[0], c[1], c[2]);
    bool done = false;
    if constexpr (sizeof(T) == 4) {
      if (s.lo[0]) {  // compensated FP32
        double u[5];
        load_pairs(s, p, u);
        store_prim_comp(ph.gamma, w, p, u, s.b[0][p], s.b[0][p + 1], s.b[1][p],
                        s.b[1][p + g.sy], s.b[2][p], s.b[2][p + g.sz]);
        done = true;
      }
    }
    if (!done)
      store_prim((T)ph.gamma, w, p, s.u[0][p], s.u[1][p], s.u[2][p], s.u[3][p], s.u[4][p],
                 s.b[0][p], s.b[0][p + 1], s.b[1][p], s.b[1][p + g.sy], s.b[2][p],
                 s.b[2][p + g.sz], rec, ph.recover);
  }
  if constexpr (sizeof(T) == 4) wave_count(rec, cnt.fp64_rec);
}

template <class T>
void launch_prim_shell(const Geo& g, const Physics& ph, Cons<T> s, Prim<T> w, Counters c,
                       hipStream_t st) {
  const int n = shell_cells(g);
  hipLaunchKernelGGL(k_prim_shell<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, g, ph,
                     s, w, c);
}

static Span prim_span(const Geo& g) {
  return make_span(g, -NG, g.n[0] + NG - 1, -NG, g.n[1] + NG - 1, -NG, g.n[2] + NG - 1);
}

template <class T>
void launch_prim(const Geo& g, const Physics& ph, Cons<T> s, Prim<T> w, Counters c,
                 hipStream_t st) {
  const Span sp = prim_span(g);
  hipLaunchKernelGGL((k_prim<T, false>), span_grid(sp), dim3(kSpanThreads), 0, st, g, ph, sp, s,
                     w, c, nullptr);
}

// ------------------------------------------------------------------------
// Corrector flux sweep with the learned correction (coarse runs).  Same
// faces and HLLD flux as k_flux; then per face the 32 features of the
// 4-cell stencil go through the MLP on the matrix cores (one 64-face batch
// per wave), and outside shock cells the correction, clipped per component
// to tau (|F| + a_max |U_R - U_L|), is added before the fluxes are stored
// (so constrained transport sees the corrected B fluxes).
// ------------------------------------------------------------------------

struct MlpWaveLds {
  unsigned short X[64 * kXs];
  float Y[64 * 8];
};

// Offset, in points, from the face's upper cell (index c along A) to the
// cell d away along A: wrapped onto the interior images along a periodic A
// where the ghost layers are not filled (LITE).
template <bool LITE, int A>
__device__ __forceinline__ int face_step(const Geo& g, int c, int d) {
  return (LITE ? (int)axis_step(g, A, c, d) : d) * stride_of(g, A);
}

// Three phases, so that only the face scales stay live across the network
// (the reconstruction, the Riemann solve and their states would otherwise
// hold some 40 registers through it): the features from the four cells,
// the wave's inference, then the stencil read again (from the caches), the
// reconstruction, HLLD and the clipped correction.  FP32: at least 4 waves
// per SIMD (at most 128 VGPRs).  LITE (a fully periodic step): only the
// interior faces are solved, their stencils and the shock flag below the
// face wrapped onto the interior images (the ghost layers are not filled),
// each event counted as many times as the full range holds copies of the
// face.
// Blocks of 256 faces (the learned coarse step's three launches: 166 us
// each, against 167 with 128, 175 with 512 and 211 with 1024: the barriers
// around the network wait on every wave of the block).
constexpr int kMlpThreads = 256;

template <class T, int A, bool LITE>
__global__ void __launch_bounds__(kMlpThreads)
    __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1, 8)))
    k_flux_mlp(Geo g, Physics ph, Span sp, Prim<T> w, const T* __restrict__ bn, Flux<T> f,
               Muscl<T> mu, Counters cnt, MlpRef mlp) {
  __shared__ MlpWaveLds lds[kMlpThreads / 64];
  __shared__ PhiLds phi;
  MlpWaveLds& L = lds[threadIdx.x >> 6];
  for (int e = (int)threadIdx.x; e < kPhiN; e += kMlpThreads) {
    const float4 c = mlp.phi[e];
    phi.c0[e] = c.x;
    phi.c1[e] = c.y;
    phi.c2[e] = c.z;
  }
  constexpr int A1 = (A + 1) % 3, A2 = (A + 2) % 3;
  const int lane = threadIdx.x & 63;
  const Pt pt = span_point(g, sp);
  const bool valid = pt.valid;
  const int p = valid ? pt.p : 0;
  const int ci[3] = {pt.i, pt.j, pt.k};
  // the face-normal frame's 8 variables of cells 2 below .. 1 above the
  // face's upper cell along A
  const T* __restrict__ src[8] = {w.w[0], w.w[1 + A], w.w[1 + A1], w.w[1 + A2],
                                  w.w[4], w.w[5 + A], w.w[5 + A1], w.w[5 + A2]};
  FaceScale sc{};
  bool means_ok = false;
  if (valid) {
    const int so[4] = {face_step<LITE, A>(g, ci[A], -2), face_step<LITE, A>(g, ci[A], -1), 0,
                       face_step<LITE, A>(g, ci[A], 1)};
    float w8[32];
#pragma unroll
    for (int v = 0; v < 8; ++v)
#pragma unroll
      for (int c = 0; c < 4; ++c) w8[8 * c + v] = (float)src[v][p + so[c]];
    float x[32];
    means_ok = (w8[8] + w8[16] > 0.f) && (w8[12] + w8[20] > 0.f);
    sc = face_scale(w8, (float)ph.gamma);
    face_features(w8, sc, x);
#pragma unroll
    for (int c = 0; c < 32; c += 4)  // 8-byte stores (the row stride is 72 bytes)
      *(u32x2*)(L.X + lane * kXs + c) =
          u32x2{bf16_pair(x[c], x[c + 1]), bf16_pair(x[c + 2], x[c + 3])};
  } else {
#pragma unroll
    for (int c = 0; c < 32; ++c) L.X[lane * kXs + c] = 0;
  }
  __syncthreads();
  wave_mlp_infer((const u32x2*)mlp.frags, mlp.params, L.X, L.Y, phi);
  __syncthreads();
  int code = 0;
  bool corrected = false, gated = false;
  if (valid) {
    // formed again: nothing but the face scales lives across the network
    const int so[4] = {face_step<LITE, A>(g, ci[A], -2), face_step<LITE, A>(g, ci[A], -1), 0,
                       face_step<LITE, A>(g, ci[A], 1)};
    const int map[7] = {0, 1, 2, 3, 4, 6, 7};  // skip the cell-centred normal B
    T l[7], r[7];
#pragma unroll
    for (int v = 0; v < 7; ++v) {
      const T* __restrict__ a = src[map[v]];
      muscl_lr(mu, a[p + so[0]], a[p + so[1]], a[p], a[p + so[3]], l[v], r[v]);
    }
    const Face<T> Lf{l[0], l[1], l[2], l[3], l[4], l[5], l[6]};
    const Face<T> Rf{r[0], r[1], r[2], r[3], r[4], r[5], r[6]};
    const T b = bn[p];
    T F[7];
    code = hlld(Lf, Rf, b, (T)ph.gamma, (T)ph.igm1, F);
    if (mlp.shock[p + so[1]] || mlp.shock[p] || !means_ok) {
      gated = true;
    } else {
      float y[8], df[7];
#pragma unroll
      for (int o = 0; o < 8; ++o) y[o] = L.Y[lane * 8 + o];
      out_to_flux(sc, y, df);
      const T igm1 = (T)ph.igm1;
      T ul[7], fl[7], ur[7], fr[7];
      cons_flux(Lf, b, igm1, ul, fl);
      cons_flux(Rf, b, igm1, ur, fr);
      const T cfl = fast_speed(Lf.d, Lf.p, b, Lf.bt1, Lf.bt2, (T)ph.gamma);
      const T cfr = fast_speed(Rf.d, Rf.p, b, Rf.bt1, Rf.bt2, (T)ph.gamma);
      const T cmax = cfl > cfr ? cfl : cfr;
      const T sl = fabs((Lf.vn < Rf.vn ? Lf.vn : Rf.vn) - cmax);
      const T sr = fabs((Lf.vn > Rf.vn ? Lf.vn : Rf.vn) + cmax);
      const T amax = sl > sr ? sl : sr;
      const T tau = (T)mlp.tau, tauf = (T)mlp.tau_flux;
#pragma unroll
      for (int m = 0; m < 7; ++m) {
        const T lim = tauf * fabs(F[m]) + tau * amax * fabs(ur[m] - ul[m]);
        T d = (T)df[m];
        d = d > lim ? lim : (d < -lim ? -lim : d);
        F[m] += d;
      }
      corrected = true;
    }
#pragma unroll
    for (int m = 0; m < 7; ++m) f.f[A][m][p] = F[m];
    f.sg[A][p] = (int8_t)(F[0] > T(0) ? 1 : (F[0] < T(0) ? -1 : 0));
  }
  wave_count((code & 1) != 0, cnt.hll);
  wave_count((code & 2) != 0, cnt.deg);
  wave_count(corrected, cnt.mlp_faces);
  wave_count(gated, cnt.mlp_gated);
  if constexpr (LITE) {
    // the copies of the faces on the box's sides (a wave-uniform branch)
    const int extra = valid ? face_copies(g, ci, A) - 1 : 0;
    if (__ballot(extra != 0) != 0ull) {
      wave_add((code & 1) ? extra : 0, cnt.hll);
      wave_add((code & 2) ? extra : 0, cnt.deg);
      wave_add(corrected ? extra : 0, cnt.mlp_faces);
      wave_add(gated ? extra : 0, cnt.mlp_gated);
    }
  }
}

template <class T>
void launch_flux_mlp(const Geo& g, const Physics& ph, int axis, Prim<T> w, T* bn, Flux<T> f,
                     Muscl<T> m, Counters c, MlpRef mlp, bool lite, hipStream_t st) {
  // faces 0..n along the axis, rows -1..n across it (lite: the interior
  // faces 0..n-1, rows 0..n-1)
  const int lo = lite ? 0 : -1, e = lite ? -1 : 0;
  const Span sp = make_span(g, axis == 0 ? 0 : lo, g.n[0] + e, axis == 1 ? 0 : lo, g.n[1] + e,
                            axis == 2 ? 0 : lo, g.n[2] + e, kMlpThreads);
  const dim3 gr = span_grid(sp), bl(kMlpThreads);
  if (lite) {
    if (axis == 0)
      hipLaunchKernelGGL((k_flux_mlp<T, 0, true>), gr, bl, 0, st, g, ph, sp, w, bn, f, m, c, mlp);
    else if (axis == 1)
      hipLaunchKernelGGL((k_flux_mlp<T, 1, true>), gr, bl, 0, st, g, ph, sp, w, bn, f, m, c, mlp);
    else
      hipLaunchKernelGGL((k_flux_mlp<T, 2, true>), gr, bl, 0, st, g, ph, sp, w, bn, f, m, c, mlp);
  } else {
    if (axis == 0)
      hipLaunchKernelGGL((k_flux_mlp<T, 0, false>), gr, bl, 0, st, g, ph, sp, w, bn, f, m, c, mlp);
    else if (axis == 1)
      hipLaunchKernelGGL((k_flux_mlp<T, 1, false>), gr, bl, 0, st, g, ph, sp, w, bn, f, m, c, mlp);
    else
      hipLaunchKernelGGL((k_flux_mlp<T, 2, false>), gr, bl, 0, st, g, ph, sp, w, bn, f, m, c, mlp);
  }
}

// Shock cells of the stage state on cells [-1, n]^3 (lite: the interior
// cells, the others read at their images): some neighbour's pressure
// differs by more than `jump` times the cell's and the central divergence
// of v is negative.  Neighbours along a periodic axis wrap onto the
// interior images.
template <class T>
__global__ void __launch_bounds__(kSpanThreads) k_shock(Geo g, Span sp, Prim<T> w, uint8_t* shock,
                                                        double jump) {
  const Pt pt = span_point(g, sp);
  if (!pt.valid) return;
  const int p = pt.p;
  const int ci[3] = {pt.i, pt.j, pt.k};
  const T P = w.w[4][p];
  T jmax = T(0), div = T(0);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int s = stride_of(g, a);
    const int dn = (int)axis_step(g, a, ci[a], -1) * s, up = (int)axis_step(g, a, ci[a], 1) * s;
    const T jl = fabs(w.w[4][p + dn] - P) / P, jh = fabs(w.w[4][p + up] - P) / P;
    jmax = jl > jmax ? jl : jmax;
    jmax = jh > jmax ? jh : jmax;
    div += (w.w[1 + a][p + up] - w.w[1 + a][p + dn]) / (T(2) * (T)g.d[a]);
  }
  shock[p] = (jmax > (T)jump && div < T(0)) ? 1 : 0;
}

template <class T>
void launch_shock(const Geo& g, Prim<T> w, uint8_t* shock, double jump, bool lite,
                  hipStream_t st) {
  const int lo = lite ? 0 : -1, e = lite ? -1 : 0;
  const Span sp = make_span(g, lo, g.n[0] + e, lo, g.n[1] + e, lo, g.n[2] + e);
  hipLaunchKernelGGL(k_shock<T>, span_grid(sp), dim3(kSpanThreads), 0, st, g, sp, w, shock, jump);
}

// ------------------------------------------------------------------------
// Corner EMF (Eq. 10 with the derivative correction taken as the 3/4-point
// minus the 1/4-point value, the four faces touching the edge, and Eq. 11
// upwinding by the sign of the Riemann mass flux).  Edge component c is
// staggered along a = c+1 and b = c+2 (cyclic); edge index p sits at
// p - e_a/2 - e_b/2.  Face EMFs: at an a-face E_c = -F_a[B_b], at a b-face
// E_c = +F_b[B_a].
// ------------------------------------------------------------------------

template <class T>
__device__ __forceinline__ T upwind(int8_t sgn, T from_low, T from_high) {
  return sgn > 0 ? from_low : (sgn < 0 ? from_high : T(0.5) * (from_low + from_high));
}

// Faces and cells at index -1 and n of a periodic axis are read at their
// images n-1 and 0 (the fused flux sweep and the outer flux layer do not
// store those faces on a fully periodic box, and the stage's ghost fill
// leaves those cells out there; where both are filled they hold the same
// values): c is the point's (i, j, k).
template <class T, int C>
__device__ __forceinline__ T corner(const Geo& g, const Prim<T>& w, const Flux<T>& f, int p,
                                    const int c[3]) {
  constexpr int A = (C + 1) % 3, B = (C + 2) % 3;
  const int sa = stride_of(g, A), sb = stride_of(g, B);
  // the point itself (index n of a periodic axis at its image 0), then one
  // step down a and one down b from it (index 0 of a periodic axis wraps to
  // n-1); only the edge's two transverse axes a and b are stepped
  int pw = p;
  if (g.nf[A] == g.n[A] && c[A] == g.n[A]) pw -= g.n[A] * sa;
  if (g.nf[B] == g.n[B] && c[B] == g.n[B]) pw -= g.n[B] * sb;
  const int ca = c[A] == g.n[A] ? 0 : c[A], cb = c[B] == g.n[B] ? 0 : c[B];
  const int da = g.nf[A] == g.n[A] && ca == 0 ? (g.n[A] - 1) * sa : -sa;
  const int db = g.nf[B] == g.n[B] && cb == 0 ? (g.n[B] - 1) * sb : -sb;
  const int pa = pw + da, pb = pw + db;
  const T* __restrict__ fa = f.f[A][5];  // B_b flux at a-faces (t1 of the a-frame)
  const T* __restrict__ fb = f.f[B][6];  // B_a flux at b-faces (t2 of the b-frame)
  const int8_t* __restrict__ ga = f.sg[A];
  const int8_t* __restrict__ gb = f.sg[B];
  const T* __restrict__ cc = w.ec[C];
  const T X0 = -fa[pw], X1 = -fa[pb];
  const T Y0 = fb[pw], Y1 = fb[pa];
  // the four cells around the edge: pw, pw - e_a (pa), pw - e_b (pb), and
  // one step down both
  const int pab = pw + da + db;
  const T c00 = cc[pab], c10 = cc[pb], c01 = cc[pa], c11 = cc[pw];
  const T db1 = upwind(ga[pw], c01 - Y1, c11 - Y0);
  const T db3 = upwind(ga[pb], Y1 - c00, Y0 - c10);
  const T da1 = upwind(gb[pw], c10 - X1, c11 - X0);
  const T da3 = upwind(gb[pa], X1 - c00, X0 - c01);
  return T(0.25) * (X0 + X1 + Y0 + Y1) + T(0.25) * (db3 - db1) + T(0.25) * (da3 - da1);
}

// All three edges' loads are issued before any store (each edge of a point
// at the span's upper end is still inside the padded arrays; it is just not
// stored), so a wave makes one memory round trip instead of three.  Blocks
// of 512 points (the stage update keeps 256: 222 -> 214 us here, 470 -> 478
// us there).
constexpr int kEmfThreads = 512;

template <class T>
__global__ void __launch_bounds__(kEmfThreads) k_emf(Geo g, Span sp, Prim<T> w, Flux<T> f,
                                                     Edge<T> e) {
  const Pt pt = span_point(g, sp);
  if (!pt.valid) return;
  const int p = pt.p;
  const int c[3] = {pt.i, pt.j, pt.k};
  const T ex = corner<T, 0>(g, w, f, p, c);
  const T ey = corner<T, 1>(g, w, f, p, c);
  const T ez = corner<T, 2>(g, w, f, p, c);
  if (pt.i < g.n[0]) e.e[0][p] = ex;
  if (pt.j < g.n[1]) e.e[1][p] = ey;
  if (pt.k < g.n[2]) e.e[2][p] = ez;
}

template <class T>
void launch_emf(const Geo& g, Prim<T> w, Flux<T> f, Edge<T> e, hipStream_t st) {
  const Span sp = make_span(g, 0, g.n[0], 0, g.n[1], 0, g.n[2], kEmfThreads);
  hipLaunchKernelGGL(k_emf<T>, span_grid(sp), dim3(kEmfThreads), 0, st, g, sp, w, f, e);
}

// ------------------------------------------------------------------------
// Conservative update (Eq. 7, plus dt S at cell centres) and CT induction
// update (Eq. 8: dB_a/dt = -(dE_c/db - dE_b/dc), (a,b,c) cyclic).
// ------------------------------------------------------------------------

// CT update of the A-face at index q: B_A - dt (dE_C/db - dE_B/dc) with
// (A, B, C) cyclic, rb = dt/d_B, rc = dt/d_C.
// From values: the face's old field b, the C-edges at its lower and upper B
// side, the B-edges at its lower and upper C side (every kernel that forms a
// face uses this expression, so a face gets bitwise one value).
template <class T>
__device__ __forceinline__ T ct_value(T b, T rb, T ec_up, T ec, T rc, T eb_up, T eb) {
#pragma clang fp contract(on)
  return b - rb * (ec_up - ec) + rc * (eb_up - eb);
}

template <class T, int A>
__device__ __forceinline__ T ct_face(const Geo& g, const Cons<T>& s0, const Edge<T>& e, int q,
                                     T rb, T rc) {
  constexpr int B = (A + 1) % 3, C = (A + 2) % 3;
  const T* Ec = e.e[C];
  const T* Eb = e.e[B];
  return ct_value(s0.b[A][q], rb, Ec[q + stride_of(g, B)], Ec[q], rc, Eb[q + stride_of(g, C)],
                  Eb[q]);
}

// Index of the upper a-face of the cell at index c (point p) along a: face
// n of a periodic axis is read at its image, face 0 (a fully periodic step
// does not store face n; where it does, the two hold the same values).
__device__ __forceinline__ int upper_face(const Geo& g, int a, int c, int p) {
  const int s = stride_of(g, a);
  return g.nf[a] == g.n[a] && c == g.n[a] - 1 ? p + s - g.n[a] * s : p + s;
}

// The swept stage values of the interior cell (i, j, k) at p: u holds what
// the sweep left (its update, or the compensated increment); the fluxes of
// the cell's upper faces on the sweep's tile seams (the last column, row or
// plane of a tile), which the sweep left to f, are subtracted.  Returns
// whether the cell lies on a seam.
template <class T>
__device__ __forceinline__ bool add_seams(const Geo& g, const Flux<T>& f, int i, int j, int k,
                                          int p, T rx, T ry, T rz, T u[5]) {
  const bool sx = i % kSwX == kSwX - 1 || i == g.n[0] - 1;
  const bool sy = j % kSwY == kSwY - 1 || j == g.n[1] - 1;
  const bool sz = k % kSwZ == kSwZ - 1 || k == g.n[2] - 1;
  if (sx) {
    const int q = upper_face(g, 0, i, p);
#pragma unroll
    for (int m = 0; m < 5; ++m) u[m] -= rx * f.f[0][frame_comp(0, m)][q];
  }
  if (sy) {
    const int q = upper_face(g, 1, j, p);
#pragma unroll
    for (int m = 0; m < 5; ++m) u[m] -= ry * f.f[1][frame_comp(1, m)][q];
  }
  if (sz) {
    const int q = upper_face(g, 2, k, p);
#pragma unroll
    for (int m = 0; m < 5; ++m) u[m] -= rz * f.f[2][frame_comp(2, m)][q];
  }
  return sx || sy || sz;
}

// Compensated FP32: the rest of an interior cell's stage update from its
// new FP64 value v (s0's pair plus the increment): floors, the new pairs,
// then the primitives and cell EMF into wo and, CFL, the time-step
// candidate folded into the minimum r, both from the value the pairs hold
// (as every kernel that reads the pairs back computes them).
template <bool CFL>
__device__ __forceinline__ void finish_comp(const Geo& g, const Physics& ph, const Cons<float>& s1,
                                            const Prim<float>& wo, int p, double v[5],
                                            const float bnew[3], const float bup[3],
                                            const Counters& cnt, bool& hit, double& r) {
  if (ph.rho_floor > 0.0 || ph.p_floor > 0.0) {
    if (v[0] < ph.rho_floor) {
      v[0] = ph.rho_floor;
      hit = true;
    }
    const double bcx = 0.5 * ((double)bnew[0] + (double)bup[0]);
    const double bcy = 0.5 * ((double)bnew[1] + (double)bup[1]);
    const double bcz = 0.5 * ((double)bnew[2] + (double)bup[2]);
    const double P = (ph.gamma - 1.0) *
                     (v[4] - 0.5 * (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / v[0] -
                      0.5 * (bcx * bcx + bcy * bcy + bcz * bcz));
    if (P < ph.p_floor) {
      v[4] += (ph.p_floor - P) / (ph.gamma - 1.0);
      hit = true;
    }
  }
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    float h, l;
    pair_split(v[m], h, l);
    s1.u[m][p] = h;
    s1.lo[m][p] = l;
    v[m] = pair_value(h, l);
  }
  store_prim_comp(ph.gamma, wo, p, v, bnew[0], bup[0], bnew[1], bup[1], bnew[2], bup[2]);
  if constexpr (CFL)
    r = fmin(r, cfl_cell<double>(g, ph, v[0], v[1], v[2], v[3], v[4], bnew[0], bup[0], bnew[1],
                                 bup[1], bnew[2], bup[2], cnt.status));
}

// The rest of an interior cell's stage update, from its stage values u (or,
// compensated, its increment) and its new faces (lower bnew, upper bup):
// floors, the conserved values (stored where store_u, where a floor acts,
// and always in compensated FP32), the primitives and cell EMF into wo and,
// CFL, the cell's FP64 time-step candidate folded into the minimum r.  hit
// and rec are set (never cleared) where a floor acts and where the FP32
// pressure is recovered in FP64.
template <class T, bool CFL>
__device__ __forceinline__ void finish_cell(const Geo& g, const Physics& ph, const Cons<T>& s0,
                                            const Cons<T>& s1, const Prim<T>& wo, int p, T u[5],
                                            const T bnew[3], const T bup[3], bool store_u,
                                            bool comp, const Counters& cnt, bool& hit, bool& rec,
                                            double& r) {
  if constexpr (sizeof(T) == 4) {
    if (comp) {
      // the new pairs: s0's value plus the increment
      double v[5];
      load_pairs(s0, p, v);
#pragma unroll
      for (int m = 0; m < 5; ++m) v[m] += (double)u[m];
      finish_comp<CFL>(g, ph, s1, wo, p, v, bnew, bup, cnt, hit, r);
      return;
    }
  }
  const T gam = (T)ph.gamma;
  T rho = u[0], E = u[4];
  if (ph.rho_floor > 0.0 || ph.p_floor > 0.0) {
    // floors: rho raised to rho_floor, then E so that P >= p_floor
    if (rho < (T)ph.rho_floor) {
      rho = (T)ph.rho_floor;
      hit = true;
    }
    T bcx, bcy, bcz;
    bool rq;
    const T P = pressure(gam, rho, u[1], u[2], u[3], E, bnew[0], bup[0], bnew[1], bup[1],
                         bnew[2], bup[2], bcx, bcy, bcz, rq, ph.recover);
    if (P < (T)ph.p_floor) {
      E = E + ((T)ph.p_floor - P) / (gam - T(1));
      hit = true;
    }
  }
  if (store_u || hit) {
    s1.u[0][p] = rho;
    s1.u[1][p] = u[1];
    s1.u[2][p] = u[2];
    s1.u[3][p] = u[3];
    s1.u[4][p] = E;
  }
  store_prim(gam, wo, p, rho, u[1], u[2], u[3], E, bnew[0], bup[0], bnew[1], bup[1], bnew[2],
             bup[2], rec, ph.recover);
  if constexpr (CFL)
    r = fmin(r, cfl_cell<T>(g, ph, rho, u[1], u[2], u[3], E, bnew[0], bup[0], bnew[1], bup[1],
                            bnew[2], bup[2], cnt.status));
}

// One stage's update, fused with what follows it on every cell: the
// density and pressure floors, then the primitive recovery of the updated
// state into wo (and, CFL = true, the cell's FP64 time-step candidate for
// the next step, folded per block into part[]).  The cell-centred B of the
// updated faces needs the upper face of each axis, which another point
// owns: it is recomputed here with the same arithmetic (ct_face), so it is
// bitwise the value that point stores.  On a periodic axis (nf = n) the
// last cell's upper face n is the ghost copy of face 0: its old value and
// the EMFs of its edges (from fluxes whose stencils are ghost copies of
// face 0's) equal face 0's, so the recomputed value is face 0's new value
// and no wrap is needed.  s1's faces must not be s0's (the upper-face
// recomputation reads s0's faces while other points write s1's); s1's
// cells may be s0's.  w (the stage's primitives, read for the source) must
// not be wo.
//
// Every load of a point is issued whether or not the point's cell or faces
// are updated (the padded arrays hold every index the span reaches, and
// values of points that are not updated are discarded): guarding the loads
// per face family would split a wave's memory traffic into dependent round
// trips.
template <class T, bool CFL, bool SWEPT>
__global__ void __launch_bounds__(kSpanThreads) k_update(Geo g, Physics ph, Span sp, Cons<T> s0,
                                                         Cons<T> s1, Prim<T> w, Prim<T> wo,
                                                         Flux<T> f, Edge<T> e, Grav<T> gr,
                                                         DtRef dtr, Counters cnt, double* part,
                                                         Inc inc) {
  const Pt pt = span_point(g, sp);
  bool hit = false, rec = false;
  // compensated FP32: u below is the stage increment, added to s0's pairs
  const bool comp = sizeof(T) == 4 && s0.lo[0] != nullptr;
  double r = INFINITY;
  if (pt.valid) {
    const int i = pt.i, j = pt.j, k = pt.k;
    const double dt = (dtr.ptr ? *dtr.ptr : dtr.value) * dtr.factor;
    const int p = pt.p;
    const int cc[3] = {i, j, k};
    const T rx = (T)(dt / g.d[0]), ry = (T)(dt / g.d[1]), rz = (T)(dt / g.d[2]);
    const int up[3] = {p + 1, p + g.sy, p + g.sz};
    const T bnew[3] = {ct_face<T, 0>(g, s0, e, p, ry, rz), ct_face<T, 1>(g, s0, e, p, rz, rx),
                       ct_face<T, 2>(g, s0, e, p, rx, ry)};
    const T bup[3] = {ct_face<T, 0>(g, s0, e, up[0], ry, rz),
                      ct_face<T, 1>(g, s0, e, up[1], rz, rx),
                      ct_face<T, 2>(g, s0, e, up[2], rx, ry)};
    T u[5];
    bool store_u = !SWEPT;  // the sweep's value stands unless a seam or a floor changes it
    const bool interior = i < g.n[0] && j < g.n[1] && k < g.n[2];
    if constexpr (SWEPT) {
      // the sweep left the update of every cell, without the fluxes of the
      // upper faces on its tile seams (last column, row or plane of a tile)
#pragma unroll
      for (int m = 0; m < 5; ++m) u[m] = comp ? (T)inc.du[m][p] : s1.u[m][p];
      if (interior) store_u = add_seams(g, f, i, j, k, p, rx, ry, rz, u);
    } else {
      T S[5];
      cell_source<T>(g, ph, gr, i, j, k, p, w.w[0][p], w.w[1][p], w.w[2][p], w.w[3][p], S);
      const T dtT = (T)dt;
      const int qx = upper_face(g, 0, i, p), qy = upper_face(g, 1, j, p),
                qz = upper_face(g, 2, k, p);
#pragma unroll
      for (int m = 0; m < 5; ++m) {
        const T* fx = f.f[0][frame_comp(0, m)];
        const T* fy = f.f[1][frame_comp(1, m)];
        const T* fz = f.f[2][frame_comp(2, m)];
        T v = comp ? T(0) : s0.u[m][p];
        v -= rx * (fx[qx] - fx[p]);
        v -= ry * (fy[qy] - fy[p]);
        v -= rz * (fz[qz] - fz[p]);
        v += dtT * S[m];
        u[m] = v;
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int b = (a + 1) % 3, c = (a + 2) % 3;
      if (cc[a] < g.nf[a] && cc[b] < g.n[b] && cc[c] < g.n[c]) s1.b[a][p] = bnew[a];
    }
    if (interior)
      finish_cell<T, CFL>(g, ph, s0, s1, wo, p, u, bnew, bup, store_u, comp, cnt, hit, rec, r);
  }
  wave_count(hit, cnt.floor_hits);
  if constexpr (sizeof(T) == 4) wave_count(rec, cnt.fp64_rec);
  if constexpr (CFL) block_min_to(r, part);
}

static Span update_span(const Geo& g) {
  return make_span(g, 0, g.n[0], 0, g.n[1], 0, g.n[2]);
}

int update_cfl_blocks(const Geo& g) { return update_span(g).nblk; }

template <class T, bool SWEPT>
static void launch_update_sw(const Geo& g, const Physics& ph, Cons<T> s0, Cons<T> s1, Prim<T> w,
                             Prim<T> wo, Flux<T> f, Edge<T> e, Grav<T> gr, DtRef dt, Counters c,
                             double* cfl_part, Inc inc, hipStream_t st) {
  const Span sp = update_span(g);
  if (cfl_part)
    hipLaunchKernelGGL((k_update<T, true, SWEPT>), span_grid(sp), dim3(kSpanThreads), 0, st, g,
                       ph, sp, s0, s1, w, wo, f, e, gr, dt, c, cfl_part, inc);
  else
    hipLaunchKernelGGL((k_update<T, false, SWEPT>), span_grid(sp), dim3(kSpanThreads), 0, st, g,
                       ph, sp, s0, s1, w, wo, f, e, gr, dt, c, nullptr, inc);
}

template <class T>
void launch_update(const Geo& g, const Physics& ph, Cons<T> s0, Cons<T> s1, Prim<T> w,
                   Prim<T> wo, Flux<T> f, Edge<T> e, Grav<T> gr, DtRef dt, Counters c,
                   double* cfl_part, bool swept, Inc inc, hipStream_t st) {
  if (swept)
    launch_update_sw<T, true>(g, ph, s0, s1, w, wo, f, e, gr, dt, c, cfl_part, inc, st);
  else
    launch_update_sw<T, false>(g, ph, s0, s1, w, wo, f, e, gr, dt, c, cfl_part, inc, st);
}

// ------------------------------------------------------------------------
// CFL time step in FP64 (per-direction fast speed of the start-of-step
// state) and the sticky state check of interior cells.
// ------------------------------------------------------------------------

template <class T>
__global__ void __launch_bounds__(kSpanThreads) k_cfl(Geo g, Physics ph, Span sp, Cons<T> s,
                                                      double* part, Counters cnt) {
  const Pt pt = span_point(g, sp);
  double r = INFINITY;
  if (pt.valid) {
    const int p = pt.p;
    bool done = false;
    if constexpr (sizeof(T) == 4) {
      if (s.lo[0]) {  // compensated FP32: the pairs' values
        double u[5];
        load_pairs(s, p, u);
        r = cfl_cell<double>(g, ph, u[0], u[1], u[2], u[3], u[4], s.b[0][p], s.b[0][p + 1],
                             s.b[1][p], s.b[1][p + g.sy], s.b[2][p], s.b[2][p + g.sz],
                             cnt.status);
        done = true;
      }
    }
    if (!done)
      r = cfl_cell<T>(g, ph, s.u[0][p], s.u[1][p], s.u[2][p], s.u[3][p], s.u[4][p], s.b[0][p],
                      s.b[0][p + 1], s.b[1][p], s.b[1][p + g.sy], s.b[2][p], s.b[2][p + g.sz],
                      cnt.status);
  }
  block_min_to(r, part);
}

// Minimum of the per-block partials in two passes: kCflReduce blocks each
// fold a contiguous share into out[block]; then one block folds those and
// scales by the Courant number.  (One block walking every partial is
// latency bound: ~90 us for the 65k partials of a 256^3 box.)
constexpr int kCflReduce = 64;

__global__ void __launch_bounds__(256) k_cfl_reduce(const double* part, int nb, double* out) {
  __shared__ double red[4];
  const int share = (nb + kCflReduce - 1) / kCflReduce;
  const int lo = blockIdx.x * share, hi = min(nb, lo + share);
  double m = INFINITY;
  for (int q = lo + (int)threadIdx.x; q < hi; q += 256) m = fmin(m, part[q]);
  m = wave_min(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
}

__global__ void __launch_bounds__(64) k_cfl_final(const double* part, double cfl, double* dt_out) {
  double m = part[threadIdx.x];
  m = wave_min(m);
  if (threadIdx.x == 0) *dt_out = cfl * m;
}

static Span cfl_span(const Geo& g) {
  return make_span(g, 0, g.n[0] - 1, 0, g.n[1] - 1, 0, g.n[2] - 1);
}

int cfl_blocks(const Geo& g) {
  int nb = cfl_span(g).nblk;
  nb = nb > prim_span(g).nblk ? nb : prim_span(g).nblk;
  nb = nb > update_span(g).nblk ? nb : update_span(g).nblk;
  return nb + kPartCflBlocks + kCflReduce;
}

// dt_out = cfl x the minimum of the nb cell partials in part[] and (if
// pp.n) the particles' partials, which are written after them.
template <class T>
void launch_cfl_reduce(const Geo& g, const Physics& ph, double* part, int nb, double* dt_out,
                       Parts<T> pp, hipStream_t st) {
  static_assert(kCflReduce == 64, "k_cfl_final folds one wave");
  if (pp.n > 0) {
    launch_particle_cfl<T>(g, pp, part + nb, st);
    nb += kPartCflBlocks;
  }
  hipLaunchKernelGGL(k_cfl_reduce, dim3(kCflReduce), dim3(256), 0, st, part, nb, part + nb);
  hipLaunchKernelGGL(k_cfl_final, dim3(1), dim3(64), 0, st, part + nb, ph.cfl, dt_out);
}

template <class T>
void launch_prim_cfl(const Geo& g, const Physics& ph, Cons<T> s, Prim<T> w, double* part,
                     double* dt_out, Counters c, Parts<T> pp, hipStream_t st) {
  const Span sp = prim_span(g);
  hipLaunchKernelGGL((k_prim<T, true>), span_grid(sp), dim3(kSpanThreads), 0, st, g, ph, sp, s, w,
                     c, part);
  launch_cfl_reduce<T>(g, ph, part, sp.nblk, dt_out, pp, st);
}

template <class T>
void launch_cfl(const Geo& g, const Physics& ph, Cons<T> s, double* part, double* dt_out,
                Counters c, Parts<T> pp, hipStream_t st) {
  const Span sp = cfl_span(g);
  hipLaunchKernelGGL(k_cfl<T>, span_grid(sp), dim3(kSpanThreads), 0, st, g, ph, sp, s, part, c);
  launch_cfl_reduce<T>(g, ph, part, sp.nblk, dt_out, pp, st);
}

__global__ void k_advance_time(double* t, long long* step, DtRef dtr) {
  const double dt = (dtr.ptr ? *dtr.ptr : dtr.value) * dtr.factor;
  *t += dt;
  *step += 1;
}

void launch_advance_time(double* t, long long* step, DtRef dt, hipStream_t st) {
  hipLaunchKernelGGL(k_advance_time, dim3(1), dim3(1), 0, st, t, step, dt);
}

// ------------------------------------------------------------------------
// Diagnostics: FP64 sums of the conserved cell fields and of each face-B
// component, min rho, min P, max |div_h B| and max |B_face|.  Per-block
// partials (fixed shuffle order), then one block sums them in fixed order.
// ------------------------------------------------------------------------

constexpr int kDiagCols = 16;

template <class T>
__global__ void __launch_bounds__(BX* BY) k_diag(Geo g, Physics ph, Cons<T> s, double* part) {
  __shared__ double red[kDiagCols][BY];
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  double v[kDiagCols];
#pragma unroll
  for (int q = 0; q < kDiagCols; ++q) v[q] = 0.0;
  v[9] = INFINITY;   // rho min
  v[10] = INFINITY;  // P min
  if (i <= g.n[0] && j <= g.n[1]) {
    const int p = pidx(g, i, j, k);
    const int cc[3] = {i, j, k};
    if (i < g.n[0] && j < g.n[1] && k < g.n[2]) {
#pragma unroll
      for (int m = 0; m < 5; ++m) v[m] = (double)s.u[m][p];
      if constexpr (sizeof(T) == 4) {
        if (s.lo[0]) {  // compensated FP32: the pairs' values
#pragma unroll
          for (int m = 0; m < 5; ++m) v[m] += (double)s.lo[m][p];
        }
      }
      const double b0[3] = {(double)s.b[0][p], (double)s.b[1][p], (double)s.b[2][p]};
      const double b1[3] = {(double)s.b[0][p + 1], (double)s.b[1][p + g.sy],
                            (double)s.b[2][p + g.sz]};
      double bc[3], div = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        bc[a] = 0.5 * (b0[a] + b1[a]);
        div += (b1[a] - b0[a]) * g.id[a];
      }
      const double rho = v[0];
      const double ke = 0.5 * (v[1] * v[1] + v[2] * v[2] + v[3] * v[3]) / rho;
      const double me = 0.5 * (bc[0] * bc[0] + bc[1] * bc[1] + bc[2] * bc[2]);
      v[8] = fabs(div);
      v[9] = rho;
      v[10] = (ph.gamma - 1.0) * (v[4] - ke - me);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int b = (a + 1) % 3, c = (a + 2) % 3;
      if (cc[a] < g.nf[a] && cc[b] < g.n[b] && cc[c] < g.n[c]) {
        const double x = (double)s.b[a][p];
        v[5 + a] = x;
        v[11] = fmax(v[11], fabs(x));
      }
    }
  }
#pragma unroll
  for (int q = 0; q < kDiagCols; ++q) {
    double x = v[q];
    if (q == 9 || q == 10)
      x = wave_min(x);
    else if (q == 8 || q == 11)
      x = wave_max(x);
    else
      x = wave_sum(x);
    if (threadIdx.x == 0) red[q][threadIdx.y] = x;
  }
  __syncthreads();
  if (threadIdx.y == 0 && threadIdx.x < kDiagCols) {
    const int q = threadIdx.x;
    double x = red[q][0];
    for (int w = 1; w < BY; ++w) {
      const double y = red[q][w];
      if (q == 9 || q == 10)
        x = fmin(x, y);
      else if (q == 8 || q == 11)
        x = fmax(x, y);
      else
        x += y;
    }
    part[(size_t)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)) * kDiagCols +
         q] = x;
  }
}

// The per-block partials folded in two passes (one block walking every
// partial is latency bound: ~670 us for the 84k blocks of a 256^3 box):
// kDiagReduce blocks each fold a contiguous share of the rows, column by
// column (one wave a column), in a fixed order; then one block folds those.
constexpr int kDiagReduce = 64;

__global__ void k_diag_reduce(const double* part, int nb, double* out) {
  const int q = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const bool is_min = q == 9 || q == 10;
  const bool is_max = q == 8 || q == 11;
  const int share = (nb + kDiagReduce - 1) / kDiagReduce;
  const int lo = (int)blockIdx.x * share, hi = min(nb, lo + share);
  double x = is_min ? INFINITY : 0.0;
  for (int b = lo + lane; b < hi; b += 64) {
    const double y = part[(size_t)b * kDiagCols + q];
    x = is_min ? fmin(x, y) : (is_max ? fmax(x, y) : x + y);
  }
  x = is_min ? wave_min(x) : (is_max ? wave_max(x) : wave_sum(x));
  if (lane == 0) out[(size_t)blockIdx.x * kDiagCols + q] = x;
}

__global__ void k_diag_final(const double* part, int nb, double dv, double* out) {
  // one wave per column, 16 waves
  const int q = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const bool is_min = q == 9 || q == 10;
  const bool is_max = q == 8 || q == 11;
  double x = is_min ? INFINITY : 0.0;
  for (int b = lane; b < nb; b += 64) {
    const double y = part[(size_t)b * kDiagCols + q];
    x = is_min ? fmin(x, y) : (is_max ? fmax(x, y) : x + y);
  }
  x = is_min ? wave_min(x) : (is_max ? wave_max(x) : wave_sum(x));
  if (lane == 0) out[q] = (q < 8) ? x * dv : x;
}

static int diag_partials(const Geo& g) {
  const dim3 gr = grid_for(g.n[0] + 1, g.n[1] + 1, g.n[2] + 1);
  return (int)(gr.x * gr.y * gr.z);
}

int diag_blocks(const Geo& g) { return diag_partials(g) + kDiagReduce; }

template <class T>
void launch_diag(const Geo& g, const Physics& ph, Cons<T> s, double* part, double* out,
                 hipStream_t st) {
  const int nb = diag_partials(g);
  double* folded = part + (size_t)nb * kDiagCols;
  hipLaunchKernelGGL(k_diag<T>, grid_for(g.n[0] + 1, g.n[1] + 1, g.n[2] + 1), dim3(BX, BY), 0, st,
                     g, ph, s, part);
  hipLaunchKernelGGL(k_diag_reduce, dim3(kDiagReduce), dim3(64 * kDiagCols), 0, st, part, nb,
                     folded);
  hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(64 * kDiagCols), 0, st, folded, kDiagReduce,
                     g.d[0] * g.d[1] * g.d[2], out);
}

// ------------------------------------------------------------------------
// Interior <-> padded copies.
// ------------------------------------------------------------------------

template <class T, bool IN>
__global__ void __launch_bounds__(BX* BY) k_copy(Geo g, T* cell5, T* bx, T* by, T* bz,
                                                 Cons<T> s) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (i > g.n[0] || j > g.n[1]) return;
  const int p = pidx(g, i, j, k);
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  if (i < nx && j < ny && k < nz) {
    const size_t ncell = (size_t)nx * ny * nz;
    const size_t q = ((size_t)k * ny + j) * nx + i;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      if (IN)
        s.u[m][p] = cell5[m * ncell + q];
      else
        cell5[m * ncell + q] = s.u[m][p];
    }
  }
  T* arr[3] = {bx, by, bz};
  const int cc[3] = {i, j, k};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int e[3] = {nx, ny, nz};
    e[a] = g.nf[a];
    if (cc[0] < e[0] && cc[1] < e[1] && cc[2] < e[2]) {
      const size_t q = ((size_t)k * e[1] + j) * e[0] + i;
      if (IN)
        s.b[a][p] = arr[a][q];
      else
        arr[a][q] = s.b[a][p];
    }
  }
}

// Compensated FP32: FP64 interior arrays <-> the cell pairs and FP32 faces.
// A pair written out is its exact FP64 value, and splitting that value again
// gives the same pair (a checkpoint resumes bit for bit).
template <bool IN>
__global__ void __launch_bounds__(BX* BY) k_copy_comp(Geo g, double* cell5, double* bx,
                                                      double* by, double* bz, Cons<float> s) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (i > g.n[0] || j > g.n[1]) return;
  const int p = pidx(g, i, j, k);
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  if (i < nx && j < ny && k < nz) {
    const size_t ncell = (size_t)nx * ny * nz;
    const size_t q = ((size_t)k * ny + j) * nx + i;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      if (IN) {
        float h, l;
        pair_split(cell5[m * ncell + q], h, l);
        s.u[m][p] = h;
        s.lo[m][p] = l;
      } else {
        cell5[m * ncell + q] = pair_value(s.u[m][p], s.lo[m][p]);
      }
    }
  }
  double* arr[3] = {bx, by, bz};
  const int cc[3] = {i, j, k};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    int e[3] = {nx, ny, nz};
    e[a] = g.nf[a];
    if (cc[0] < e[0] && cc[1] < e[1] && cc[2] < e[2]) {
      const size_t q = ((size_t)k * e[1] + j) * e[0] + i;
      if (IN)
        s.b[a][p] = (float)arr[a][q];
      else
        arr[a][q] = (double)s.b[a][p];
    }
  }
}

void launch_scatter_comp(const Geo& g, const double* cell5, const double* bx, const double* by,
                         const double* bz, Cons<float> s, hipStream_t st) {
  hipLaunchKernelGGL((k_copy_comp<true>), grid_for(g.n[0] + 1, g.n[1] + 1, g.n[2] + 1),
                     dim3(BX, BY), 0, st, g, const_cast<double*>(cell5), const_cast<double*>(bx),
                     const_cast<double*>(by), const_cast<double*>(bz), s);
}

void launch_gather_comp(const Geo& g, Cons<float> s, double* cell5, double* bx, double* by,
                        double* bz, hipStream_t st) {
  hipLaunchKernelGGL((k_copy_comp<false>), grid_for(g.n[0] + 1, g.n[1] + 1, g.n[2] + 1),
                     dim3(BX, BY), 0, st, g, cell5, bx, by, bz, s);
}

template <class T>
void launch_scatter(const Geo& g, const T* cell5, const T* bx, const T* by, const T* bz,
                    Cons<T> s, hipStream_t st) {
  hipLaunchKernelGGL((k_copy<T, true>), grid_for(g.n[0] + 1, g.n[1] + 1, g.n[2] + 1),
                     dim3(BX, BY), 0, st, g, const_cast<T*>(cell5), const_cast<T*>(bx),
                     const_cast<T*>(by), const_cast<T*>(bz), s);
}

template <class T>
void launch_gather(const Geo& g, Cons<T> s, T* cell5, T* bx, T* by, T* bz, hipStream_t st) {
  hipLaunchKernelGGL((k_copy<T, false>), grid_for(g.n[0] + 1, g.n[1] + 1, g.n[2] + 1),
                     dim3(BX, BY), 0, st, g, cell5, bx, by, bz, s);
}

// ------------------------------------------------------------------------
// Passive scalars (mass fractions X_s, conserved as rho X_s).  The face flux
// is the face's mass flux times X reconstructed on the side the mass comes
// from.  One kernel per stage: each interior cell rebuilds the two faces of
// each axis it needs from X = (rho X) / rho on its 13-point stencil and
// applies the update, so no scalar flux array is written or read back (each
// face is computed by its two cells; the arithmetic is cheap next to the
// traffic an extra array pair per scalar and axis would cost).
// ------------------------------------------------------------------------

template <class T>
__device__ __forceinline__ T scalar_flux(T F, T xl, T xr) {
  return F > T(0) ? F * xl : (F < T(0) ? F * xr : T(0));
}

// NS (the scalar count) is a template parameter so that every load of a
// point -- 13 stencil values per scalar, the stage density and mass fluxes
// -- is issued before the first store (with a run-time count the stores of
// one scalar could alias the next one's loads and would order them).
template <class T, int NS>
__global__ void __launch_bounds__(kSpanThreads) k_scalar_update(Geo g, Span sp,
                                                                const T* __restrict__ rho,
                                                                Flux<T> f, Scal<T> x0, Scal<T> xs,
                                                                Scal<T> x1, Muscl<T> mu,
                                                                DtRef dtr) {
  const Pt pt = span_point(g, sp);
  if (!pt.valid) return;
  const int p = pt.p;
  const double dt = (dtr.ptr ? *dtr.ptr : dtr.value) * dtr.factor;
  const int st[3] = {1, g.sy, g.sz};
  // stencil point o of axis a: p + (o - 2) s_a (o = 2: the cell itself)
  T xv[NS][3][5], v0[NS];
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    const T* q = xs.x[m];
    const T c = q[p];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int o = 0; o < 5; ++o) xv[m][a][o] = o == 2 ? c : q[p + (o - 2) * st[a]];
    v0[m] = x0.x[m][p];
  }
  // 1 / rho on the stencil; mass fluxes of the low and high face
  T ir[3][5], flo[3], fhi[3], r[3];
  const T ic = rcp(rho[p]);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
#pragma unroll
    for (int o = 0; o < 5; ++o) ir[a][o] = o == 2 ? ic : rcp(rho[p + (o - 2) * st[a]]);
    flo[a] = f.f[a][0][p];
    // face n of a periodic x axis is read at its image, face 0
    const int up = a == 0 && g.nf[0] == g.n[0] && pt.i == g.n[0] - 1 ? p + 1 - g.n[0] : p + st[a];
    fhi[a] = f.f[a][0][up];
    r[a] = (T)(dt / g.d[a]);
  }
  T out[NS];
#pragma unroll
  for (int m = 0; m < NS; ++m) {
    T v = v0[m];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      T X[5];
#pragma unroll
      for (int o = 0; o < 5; ++o) X[o] = xv[m][a][o] * ir[a][o];
      T l0, r0, l1, r1;
      muscl_lr(mu, X[0], X[1], X[2], X[3], l0, r0);
      muscl_lr(mu, X[1], X[2], X[3], X[4], l1, r1);
      v -= r[a] * (scalar_flux(fhi[a], l1, r1) - scalar_flux(flo[a], l0, r0));
    }
    out[m] = v;
  }
#pragma unroll
  for (int m = 0; m < NS; ++m) x1.x[m][p] = out[m];
}

template <class T, int NS>
static void scalar_update_ns(const Geo& g, const Span& sp, const T* rho, Flux<T> f, Scal<T> x0,
                             Scal<T> xs, Scal<T> x1, Muscl<T> m, DtRef dt, hipStream_t st) {
  hipLaunchKernelGGL((k_scalar_update<T, NS>), span_grid(sp), dim3(kSpanThreads), 0, st, g, sp,
                     rho, f, x0, xs, x1, m, dt);
}

template <class T>
void launch_scalar_update(const Geo& g, const T* rho, Flux<T> f, Scal<T> x0, Scal<T> xs,
                          Scal<T> x1, int ns, Muscl<T> m, DtRef dt, hipStream_t st) {
  if (ns <= 0) return;
  const Span sp = make_span(g, 0, g.n[0] - 1, 0, g.n[1] - 1, 0, g.n[2] - 1);
  switch (ns) {
    case 1: scalar_update_ns<T, 1>(g, sp, rho, f, x0, xs, x1, m, dt, st); break;
    case 2: scalar_update_ns<T, 2>(g, sp, rho, f, x0, xs, x1, m, dt, st); break;
    case 3: scalar_update_ns<T, 3>(g, sp, rho, f, x0, xs, x1, m, dt, st); break;
    case 4: scalar_update_ns<T, 4>(g, sp, rho, f, x0, xs, x1, m, dt, st); break;
    case 5: scalar_update_ns<T, 5>(g, sp, rho, f, x0, xs, x1, m, dt, st); break;
    case 6: scalar_update_ns<T, 6>(g, sp, rho, f, x0, xs, x1, m, dt, st); break;
    case 7: scalar_update_ns<T, 7>(g, sp, rho, f, x0, xs, x1, m, dt, st); break;
    default: scalar_update_ns<T, 8>(g, sp, rho, f, x0, xs, x1, m, dt, st); break;
  }
}

// Ghost points of the scalar arrays: periodic wrap / outflow copy as for the
// cell fields; inflow ghosts hold no scalar.
template <class T>
__global__ void k_scalar_ghosts(Geo g, Scal<T> x, int ns) {
  int c[3];
  int face_only;
  if (!ghost_point(g, (long long)blockIdx.x * blockDim.x + threadIdx.x, 5, c, face_only)) return;
  const int p = pidx(g, c[0], c[1], c[2]);
  bool inflow = false;
  int m[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
    m[a] = map_axis(c[a], g.n[a], g.n[a], g.bc[2 * a], g.bc[2 * a + 1], inflow);
  if (inflow) {
    for (int q = 0; q < ns; ++q) x.x[q][p] = T(0);
  } else if (m[0] != c[0] || m[1] != c[1] || m[2] != c[2]) {
    const int q0 = pidx(g, m[0], m[1], m[2]);
    for (int q = 0; q < ns; ++q) x.x[q][p] = x.x[q][q0];
  }
}

template <class T>
void launch_scalar_ghosts(const Geo& g, Scal<T> x, int ns, hipStream_t st) {
  if (ns <= 0) return;
  hipLaunchKernelGGL(k_scalar_ghosts<T>, dim3(ghost_blocks(g, 256, 5)), dim3(256), 0, st, g, x,
                     ns);
}

template <class T, bool IN>
__global__ void __launch_bounds__(BX* BY) k_scalar_copy(Geo g, Scal<T> x, int ns, T* interior) {
  const int i = blockIdx.x * BX + threadIdx.x;
  const int j = blockIdx.y * BY + threadIdx.y;
  const int k = blockIdx.z;
  if (i >= g.n[0] || j >= g.n[1]) return;
  const int p = pidx(g, i, j, k);
  const size_t ncell = (size_t)g.n[0] * g.n[1] * g.n[2];
  const size_t q = ((size_t)k * g.n[1] + j) * g.n[0] + i;
  for (int m = 0; m < ns; ++m) {
    if (IN)
      x.x[m][p] = interior[m * ncell + q];
    else
      interior[m * ncell + q] = x.x[m][p];
  }
}

template <class T>
void launch_scalar_copy(const Geo& g, Scal<T> x, int ns, T* interior, bool in, hipStream_t st) {
  if (ns <= 0) return;
  const dim3 gr = grid_for(g.n[0], g.n[1], g.n[2]);
  if (in)
    hipLaunchKernelGGL((k_scalar_copy<T, true>), gr, dim3(BX, BY), 0, st, g, x, ns, interior);
  else
    hipLaunchKernelGGL((k_scalar_copy<T, false>), gr, dim3(BX, BY), 0, st, g, x, ns, interior);
}

// ------------------------------------------------------------------------
// Batch entry points for kernel-level parity tests.
// ------------------------------------------------------------------------

template <class T>
__global__ void k_hlld_batch(int64_t n, const T* wl, const T* wr, const T* bn, T gam, T igm1,
                             T* flux, int8_t* code) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const T* a = wl + 7 * t;
  const T* b = wr + 7 * t;
  const Face<T> L{a[0], a[1], a[2], a[3], a[4], a[5], a[6]};
  const Face<T> R{b[0], b[1], b[2], b[3], b[4], b[5], b[6]};
  T F[7];
  const int c = hlld(L, R, bn[t], gam, igm1, F);
#pragma unroll
  for (int m = 0; m < 7; ++m) flux[7 * t + m] = F[m];
  if (code) code[t] = (int8_t)c;
}

template <class T>
void launch_hlld_batch(int64_t n, const T* wl, const T* wr, const T* bn, T gam, T* flux,
                       int8_t* code, hipStream_t st) {
  if (n <= 0) return;
  const T igm1 = (T)(1.0 / ((double)gam - 1.0));
  hipLaunchKernelGGL(k_hlld_batch<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, wl,
                     wr, bn, gam, igm1, flux, code);
}

template <class T>
__global__ void k_recon_batch(int64_t n, const T* w4, Muscl<T> m, T* wl, T* wr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const T* w = w4 + 4 * t;
  muscl_lr(m, w[0], w[1], w[2], w[3], wl[t], wr[t]);
}

template <class T>
void launch_recon_batch(int64_t n, const T* w4, Muscl<T> m, T* wl, T* wr, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_recon_batch<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                     w4, m, wl, wr);
}

// ------------------------------------------------------------------------
// Explicit instantiations.
// ------------------------------------------------------------------------

#define MHD_INST(T)                                                                              \
  template void launch_ghosts<T>(const Geo&, const Physics&, Cons<T>, bool, hipStream_t);        \
  template void launch_prim<T>(const Geo&, const Physics&, Cons<T>, Prim<T>, Counters,           \
                               hipStream_t);                                                     \
  template void launch_prim_cfl<T>(const Geo&, const Physics&, Cons<T>, Prim<T>, double*,        \
                                   double*, Counters, Parts<T>, hipStream_t);                    \
  template void launch_emf<T>(const Geo&, Prim<T>, Flux<T>, Edge<T>, hipStream_t);              \
  template void launch_flux_mlp<T>(const Geo&, const Physics&, int, Prim<T>, T*, Flux<T>,        \
                                   Muscl<T>, Counters, MlpRef, bool, hipStream_t);               \
  template void launch_shock<T>(const Geo&, Prim<T>, uint8_t*, double, bool, hipStream_t);     \
  template void launch_prim_shell<T>(const Geo&, const Physics&, Cons<T>, Prim<T>, Counters,     \
                                     hipStream_t);                                               \
  template void launch_update<T>(const Geo&, const Physics&, Cons<T>, Cons<T>, Prim<T>, Prim<T>, \
                                 Flux<T>, Edge<T>, Grav<T>, DtRef, Counters, double*, bool, Inc, \
                                 hipStream_t);                                                   \
  template void launch_cfl_reduce<T>(const Geo&, const Physics&, double*, int, double*, Parts<T>, \
                                     hipStream_t);                                               \
  template void launch_cfl<T>(const Geo&, const Physics&, Cons<T>, double*, double*, Counters,   \
                              Parts<T>, hipStream_t);                                            \
  template void launch_diag<T>(const Geo&, const Physics&, Cons<T>, double*, double*,           \
                               hipStream_t);                                                     \
  template void launch_scatter<T>(const Geo&, const T*, const T*, const T*, const T*, Cons<T>,  \
                                  hipStream_t);                                                  \
  template void launch_gather<T>(const Geo&, Cons<T>, T*, T*, T*, T*, hipStream_t);             \
  template void launch_hlld_batch<T>(int64_t, const T*, const T*, const T*, T, T*, int8_t*,     \
                                     hipStream_t);                                               \
  template void launch_recon_batch<T>(int64_t, const T*, Muscl<T>, T*, T*, hipStream_t);       \
  template void launch_scalar_update<T>(const Geo&, const T*, Flux<T>, Scal<T>, Scal<T>,        \
                                        Scal<T>, int, Muscl<T>, DtRef, hipStream_t);            \
  template void launch_scalar_ghosts<T>(const Geo&, Scal<T>, int, hipStream_t);                 \
  template void launch_scalar_copy<T>(const Geo&, Scal<T>, int, T*, bool, hipStream_t);

MHD_INST(double)
MHD_INST(float)

}  // namespace mhd
