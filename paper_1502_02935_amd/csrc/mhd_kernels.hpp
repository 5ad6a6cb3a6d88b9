// mhd_kernels.hpp -- grid description, array bundles and kernel launchers
// of the ideal-MHD step (section 2.1 of the paper).  The kernels themselves
// live in mhd_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mhd_physics.hpp"

namespace mhd {

constexpr int NG = 2;  // ghost layers: MUSCL needs cells i-2..i+1 of face i

// Padded grid: every array (cells, faces, edges) has extent n + 2 NG + 1 per
// axis, x fastest; interior cell (i,j,k) is at (i+NG) + sy (j+NG) + sz (k+NG).
// Face (i,j,k) of the x-face arrays sits at x_{i-1/2}; edge (i,j,k) of the
// z-edge arrays at (x_{i-1/2}, y_{j-1/2}, z_k) (cyclically for x and y).
struct Geo {
  int n[3];
  int ext[3];
  int sy, sz;
  int np;       // points per padded array
  int nf[3];    // interior faces along each axis' own normal (n or n+1)
  int bc[6];
  double d[3];
  double id[3];  // 1 / d
  double x0[3];
};

// Conserved state: 5 cell arrays + 3 face arrays.  Compensated FP32
// (MHD_FP32_COMP): lo[m] holds the rest of cell value m, the value being
// the pair u[m] + lo[m] evaluated in FP64 (u[m] is its FP32 rounding, lo[m]
// the rounding of what remains: about 48 significant bits); lo[0] is null
// in the other modes.
template <class T>
struct Cons {
  T* u[5];
  T* b[3];
  float* lo[5];
};

// Compensated FP32: the stage increments of the cells the fused sweep
// leaves for the stage update to add to the pairs (null otherwise).
struct Inc {
  float* du[5];
};

// Value of a compensated pair.
__device__ __forceinline__ double pair_value(float hi, float lo) {
  return (double)hi + (double)lo;
}
// Split x into a pair: hi its FP32 rounding, lo the FP32 rounding of the
// rest; then renormalised so that hi is the FP32 rounding of hi + lo (a pair
// written out in FP64 and split again is the same pair).
__device__ __forceinline__ void pair_split(double x, float& hi, float& lo) {
  float h = (float)x;
  float l = (float)(x - (double)h);
  const double s = (double)h + (double)l;
  hi = (float)s;
  lo = (float)(s - (double)hi);
}

// Primitives rho, vx, vy, vz, P, Bcx, Bcy, Bcz and cell EMF.  w[0] is the
// density array of the conserved state the primitives belong to: the
// primitive passes read it there and never write it.
template <class T>
struct Prim {
  T* w[8];
  T* ec[3];
};

template <class T>
struct Flux {  // per axis, face frame rho, Mn, Mt1, Mt2, E, Bt1, Bt2
  T* f[3][7];
  int8_t* sg[3];  // sign of the mass flux
};

template <class T>
struct Edge {
  T* e[3];
};

// Event counters.  Each counter is spread over kCounterSlots slots, one
// 64-byte line apart, and a block adds into slot (block id mod kCounterSlots):
// a single shared address would serialise every wave's atomic in L2.
constexpr int kCounterSlots = 256;
constexpr int kCounterStride = 8;  // unsigned long longs per slot (64 bytes)
constexpr int kNumCounters = 6;  // hll, degenerate, floors, FP64 recoveries, MLP faces, gated

struct Counters {
  unsigned long long* hll;
  unsigned long long* deg;
  unsigned long long* floor_hits;
  unsigned long long* fp64_rec;
  unsigned long long* mlp_faces;
  unsigned long long* mlp_gated;
  unsigned int* status;
};

// Learned correction of the corrector fluxes (null params = off).
struct MlpRef {
  const float* params;    // FP32 master weights, 6792 (biases read from here)
  const unsigned* frags;  // the weights packed as bf16 MFMA fragments (launch_mlp_pack)
  const float4* phi;      // normal CDF table (kPhiN entries)
  double tau;           // clip factor of the dissipation-scale term
  double jump;          // relative pressure jump of a shock cell
  double tau_flux;      // clip factor of the flux-scale term
  uint8_t* shock;       // per padded cell
};

// Riemann solver of the flux sweeps: HLLD, or the paper's two gas-dynamic
// solvers HLL and HLLC (HLLC: pure gas dynamics, the field taken as zero).
enum { kRiemannHLLD = 0, kRiemannHLL = 1, kRiemannHLLC = 2 };

struct Physics {
  double gamma;
  double igm1;  // 1 / (gamma - 1)
  int riemann;  // kRiemann*
  double cfl;
  int source;
  double src[4];
  double rho_floor, p_floor;
  bool recover;        // FP32: redo cancelling pressures in FP64
  double inflow_u[5];  // conserved ghost state of inflow sides
  double inflow_b[3];
};

// Self-gravity: potential and its central gradient at the cells (padded
// arrays; null when the source is off).
template <class T>
struct Grav {
  T* psi;
  T* g[3];
};

// Workspace of the periodic Poisson solve: complex [nz][ny][nx] array (T
// pairs), per axis n/2 twiddles exp(-2 pi i q / n) (T pairs) and n
// eigenvalues of the 3-point Laplacian.
template <class T>
struct GravFFT {
  T* c;
  const T* tw[3];
  const T* lam[3];
};

// Passive scalars rho X_s (padded arrays, the first ns entries used).
constexpr int kMaxScalars = 8;
template <class T>
struct Scal {
  T* x[kMaxScalars];
};

// N-body particles (context precision, structure of arrays): positions and
// velocities [3][n] (x, y, z rows), masses [n], and each particle's index in
// the caller's order; n = 0: none.  The library keeps them sorted by tile
// (kTile^3 cells, the tile holding the particle's cell): toff[t] .. toff[t+1]
// are tile t's particles.
constexpr int kTile = 8;
constexpr int kChunk = 2048;  // particles per block of the deposit and the kick
template <class T>
struct Parts {
  T* x;
  T* v;
  T* m;
  int* id;
  long long n;
  const int* toff;   // [ntiles + 1]
  const int* chunk;  // [1 + 3 max_chunks]: count, then (tile, first, end) per chunk
  int nt[3];         // tiles per axis
  int ntiles;
  int max_chunks;    // n / kChunk + ntiles
};
// Scratch of the sort: the other buffer and the per-tile counters.
template <class T>
struct PartSort {
  T* x;
  T* v;
  T* m;
  int* id;
  int* cnt;    // [ntiles]
  int* off;    // [ntiles + 1]
  int* cur;    // [ntiles]
  int* coff;   // [ntiles + 1] chunk offsets
  int* chunk;  // [1 + 3 max_chunks]
};
constexpr int kPartCflBlocks = 1024;  // per-block CFL partials of the particles

// Time-step source: a value, or (if ptr != nullptr) a device scalar.
struct DtRef {
  double value;
  const double* ptr;
  double factor;  // 0.5 for the predictor, 1 for the corrector
};

// lite: of each axis' ghost layers only that axis' face at index n (for a
// fully periodic box whose stage path reads every other ghost at its
// interior image; the faces n give the last cells their cell-centred B in
// the kernels outside the step).
template <class T>
void launch_ghosts(const Geo& g, const Physics& ph, Cons<T> s, bool lite, hipStream_t st);
template <class T>
void launch_prim(const Geo& g, const Physics& ph, Cons<T> s, Prim<T> w, Counters c,
                 hipStream_t st);
// Primitives plus the per-block CFL candidates of the interior cells,
// reduced to dt_out (= cfl x min): the start of a step with its own dt.
template <class T>
void launch_prim_cfl(const Geo& g, const Physics& ph, Cons<T> s, Prim<T> w, double* part,
                     double* dt_out, Counters c, Parts<T> pp, hipStream_t st);
// Fluxes of all three face families (normal B from the face arrays of s).
template <class T>
void launch_flux(const Geo& g, const Physics& ph, Prim<T> w, Cons<T> s, Flux<T> f, Muscl<T> m,
                 Counters c, hipStream_t st);
// Fluxes of the A-faces with the learned correction (shock flags from
// launch_shock); lite: only the interior faces (a fully periodic step whose
// readers take the periodic images at the interior faces).
template <class T>
void launch_flux_mlp(const Geo& g, const Physics& ph, int axis, Prim<T> w, T* bn, Flux<T> f,
                     Muscl<T> m, Counters c, MlpRef mlp, bool lite, hipStream_t st);
// Shock flags of cells [-1, n]^3 (lite: the interior cells).
template <class T>
void launch_shock(const Geo& g, Prim<T> w, uint8_t* shock, double jump, bool lite,
                  hipStream_t st);
template <class T>
void launch_emf(const Geo& g, Prim<T> w, Flux<T> f, Edge<T> e, hipStream_t st);
// One stage's update of s0 into s1 (s1's faces must be other arrays than
// s0's; its cells may be s0's) with the floors and the primitives of the
// updated interior cells into wo (w: the stage's primitives, for the
// source; wo must be other arrays).  cfl_part != nullptr: the cells' FP64
// time-step candidates as update_cfl_blocks(g) per-block minima.  swept:
// s1's cells already hold the update of launch_sweep (seam fluxes still to
// add) instead of f holding every face's flux.
// Compensated FP32 (s0.lo non-null): the cells' new pairs are s0's pairs
// plus the stage increment in FP64 (swept: the increments the sweep left in
// inc, plus the seam fluxes; else the flux differences and dt S), always
// stored; the floors, pressure, primitives and time-step candidates come
// from the FP64 value.
template <class T>
void launch_update(const Geo& g, const Physics& ph, Cons<T> s0, Cons<T> s1, Prim<T> w,
                   Prim<T> wo, Flux<T> f, Edge<T> e, Grav<T> gr, DtRef dt, Counters c,
                   double* cfl_part, bool swept, Inc inc, hipStream_t st);
// Tiles of the fused flux sweep: kSwX x kSwY cells a block (one wave per
// x-row), walking kSwZ planes in z.
constexpr int kSwX = 64, kSwY = 8, kSwZ = 16;
// Fused flux sweep and conservative update of one stage (mhd_flux.hip):
// the fluxes of every face of the interior cells with the Riemann solver
// of ph and the reconstruction of m; into s1's cells the update of s0's
// cells with those fluxes and dt S, except the fluxes of the upper faces of
// tile seams, which go to f for launch_update(swept); the field
// components of the fluxes and the mass-flux signs of every face to f for
// the EMFs; store 1: also the mass fluxes (passive scalars), 2: every
// component.  s1's cells may be s0's.  launch_flux_outer completes f.
// inc (compensated FP32): s0's cells are not read and s1's cells receive
// the stage increment (the update without s0's value).
template <class T>
void launch_sweep(const Geo& g, const Physics& ph, Prim<T> w, Cons<T> s0, Cons<T> s1,
                  Flux<T> f, Muscl<T> m, Grav<T> gr, DtRef dt, Counters c, int store, bool inc,
                  hipStream_t st);
// After launch_sweep: every component of the faces of the points in the
// outer layer of the flux range, [-1, n]^3 without [0, n-1]^3 (the faces
// at index n and the ghost rows the EMFs need), copied from their periodic
// images (which the sweep solved) or, on outflow and inflow sides, solved
// with normal B from s's faces.  On a periodic x axis the points at x-index
// -1 and n are left out unless store is 2 (their readers -- the EMFs, the
// swept update's seams, the passive scalars -- wrap the x-index).
template <class T>
void launch_flux_outer(const Geo& g, const Physics& ph, Prim<T> w, Cons<T> s, Flux<T> f,
                       Muscl<T> m, Counters c, int store, hipStream_t st);
int update_cfl_blocks(const Geo& g);
// Primitives of the ghost shell [-NG, n+NG-1]^3 minus the interior (after
// a full ghost fill).
template <class T>
void launch_prim_shell(const Geo& g, const Physics& ph, Cons<T> s, Prim<T> w, Counters c,
                       hipStream_t st);
// Passive scalars of one stage: x1 = x0 - dt div F_X, with F_X the mass flux
// of f times X = xs / rho (rho: the stage's primitive density) reconstructed
// by m on the upwind side; interior cells.  x1 may be x0.
template <class T>
void launch_scalar_update(const Geo& g, const T* rho, Flux<T> f, Scal<T> x0, Scal<T> xs,
                          Scal<T> x1, int ns, Muscl<T> m, DtRef dt, hipStream_t st);
template <class T>
void launch_scalar_ghosts(const Geo& g, Scal<T> x, int ns, hipStream_t st);
// Interior [ns][nz][ny][nx] <-> padded scalar arrays.
template <class T>
void launch_scalar_copy(const Geo& g, Scal<T> x, int ns, T* interior, bool in, hipStream_t st);
// Psi of the stage density rho (padded primitive array) and its gradient
// into gr (mhd_gravity.hip).
template <class T>
void launch_self_gravity(const Geo& g, const Physics& ph, const T* rho, GravFFT<T> f, Grav<T> gr,
                         Parts<T> pp, DtRef h, hipStream_t st);
// CFL: per-block minima into part (size cfl_blocks(g), which also fits the
// partials of launch_prim_cfl and of the particles), then dt_out = cfl min
// over cells and (if pp.n) particles.
int cfl_blocks(const Geo& g);
template <class T>
void launch_cfl(const Geo& g, const Physics& ph, Cons<T> s, double* part, double* dt_out,
                Counters c, Parts<T> pp, hipStream_t st);
// dt_out from nb cell partials already in part (and the particles').
template <class T>
void launch_cfl_reduce(const Geo& g, const Physics& ph, double* part, int nb, double* dt_out,
                       Parts<T> pp, hipStream_t st);
// Particles (mhd_nbody.hip).  Per-block minima over the particles of
// d_a / |v_a| into part[0 .. kPartCflBlocks).
template <class T>
void launch_particle_cfl(const Geo& g, Parts<T> pp, double* part, hipStream_t st);
// Adds the cloud-in-cell density of the particles at x + h v (h = dt x
// dt.factor, positions wrapped) to the real parts of the complex array c
// ([nz][ny][nx] pairs).
template <class T>
void launch_deposit(const Geo& g, Parts<T> pp, DtRef h, T* c, hipStream_t st);
// Leapfrog with the potential gradient of gr (cell-centred, the corrector's):
// x_h = x + dt/2 v, v -= dt grad Psi(x_h), x = x_h + dt/2 v, positions wrapped.
template <class T>
void launch_kick_drift(const Geo& g, Parts<T> pp, Grav<T> gr, DtRef dt, hipStream_t st);
// Positions wrapped into the box and ids set to 0..n-1 (after the caller
// sets the particles).
template <class T>
void launch_particles_init(const Geo& g, Parts<T> pp, hipStream_t st);
// Counting sort of pp by tile into the buffers of s (which then hold the
// current order, with s.off the tile offsets).
template <class T>
void launch_particle_sort(const Geo& g, Parts<T> pp, PartSort<T> s, hipStream_t st);
// Positions and velocities in the caller's order (x_out, v_out may be null).
template <class T>
void launch_particles_out(Parts<T> pp, T* x_out, T* v_out, hipStream_t st);
void launch_advance_time(double* t, long long* step, DtRef dt, hipStream_t st);

// Diagnostics: writes 14 doubles to out: mass, M(3), E, bsum(3), divb_max,
// rho_min, p_min, bmax, (2 spare).  part holds diag_blocks(g) rows of 16
// doubles (the per-block partials and the first folding pass).
int diag_blocks(const Geo& g);
template <class T>
void launch_diag(const Geo& g, const Physics& ph, Cons<T> s, double* part, double* out,
                 hipStream_t st);

// Interior layout <-> padded layout.
template <class T>
void launch_scatter(const Geo& g, const T* cell5, const T* bx, const T* by, const T* bz,
                    Cons<T> s, hipStream_t st);
template <class T>
void launch_gather(const Geo& g, Cons<T> s, T* cell5, T* bx, T* by, T* bz, hipStream_t st);
// Compensated FP32: FP64 interior arrays <-> the pairs of s (cells) and
// its FP32 faces.
void launch_scatter_comp(const Geo& g, const double* cell5, const double* bx, const double* by,
                         const double* bz, Cons<float> s, hipStream_t st);
void launch_gather_comp(const Geo& g, Cons<float> s, double* cell5, double* bx, double* by,
                        double* bz, hipStream_t st);

// learned correction: training and data pipeline (mhd_mlp.hip)
void launch_mlp_forward(int64_t n, const float* x, const float* P, float* y, hipStream_t st);
size_t mlp_grad_workspace(int64_t n);
void launch_mlp_grad(int64_t n, const float* x, const float* t, const float* P, float* grad,
                     float* loss, float* part, hipStream_t st);
// Packs the weights of P into the bf16 fragments read by the fused sweep
// (frags: kMlpFragBytes bytes).
constexpr int kMlpFragBytes = 28 * 64 * 8;
// Normal CDF table of the in-step GELU: kPhiN intervals of 1 / kPhiScale on
// [-kPhiHalf, kPhiHalf), per interval the quadratic c0 + f (c1 + f c2) (f
// the position in the interval, 0..1) through Phi at its ends and midpoint,
// as 4 floats (c0, c1, c2, 0); written by the host at initialisation.
constexpr int kPhiScale = 32;
constexpr int kPhiHalf = 8;
constexpr int kPhiN = 2 * kPhiHalf * kPhiScale;
constexpr int kPhiBytes = kPhiN * 16;
void launch_mlp_pack(const float* P, unsigned* frags, hipStream_t st);
void launch_mlp_adam(float* P, float* m, float* v, const float* g, int64_t step, double lr,
                     double b1, double b2, double eps, hipStream_t st);
template <class T>
void launch_fluxacc(const Geo& g, Flux<T> f, T* acc, DtRef dt, hipStream_t st);
template <class T>
void launch_coarsen(const Geo& g, Cons<T> s, T* c5, T* bx, T* by, T* bz, hipStream_t st);
template <class T>
void launch_mlp_samples(const Geo& g, Prim<T> w, Flux<T> f, const uint8_t* shock, const T* acc,
                        double dt_c, double gam, int64_t n, const int32_t* faces, float* x,
                        float* t, uint8_t* mask, hipStream_t st);

template <class T>
void launch_hlld_batch(int64_t n, const T* wl, const T* wr, const T* bn, T gam, T* flux,
                       int8_t* code, hipStream_t st);
template <class T>
void launch_recon_batch(int64_t n, const T* w4, Muscl<T> m, T* wl, T* wr, hipStream_t st);

}  // namespace mhd
