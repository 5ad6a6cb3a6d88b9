// mhd_abi.hip -- C ABI of libmhd.so (declared in include/mhd.h): context,
// workspace carving and the step sequence.  One step is the
// predictor-corrector pair that gives the time-centred fluxes of Eq. 7:
//   predictor: primitives of U^n, first-order HLLD fluxes, corner EMFs,
//              U* = U^n - dt/2 div F + dt/2 S(W^n), B* = B^n - dt/2 curl E
//   corrector: primitives of U*, MUSCL (Eq. 12-14) + HLLD fluxes, corner EMFs,
//              U^{n+1} = U^n - dt div F + dt S(W*),  B^{n+1} = B^n - dt curl E
// with the ghost zones refilled after each stage.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "mhd.h"
#include "mhd_kernels.hpp"

using namespace mhd;

namespace {

constexpr size_t kAlign = 256;
// T arrays: two state sets (5 cells + 3 faces each), the primitives and cell
// EMF of the current state (7 + 3: the primitive density is the state's own
// density array), fluxes 21, edges 3, the primitives and cell EMF of the
// half step (7 + 3).
constexpr int kNumT = 60;
// Compensated FP32 adds 15 FP32 arrays after those: the low parts of the 5
// cell values of each state set (10), the stage increments of the cells (5).
constexpr int kCompT = 15;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Layout {
  size_t arr;       // bytes per padded T array
  size_t arr8;      // bytes per padded int8 array
  size_t off_t;     // T arrays
  size_t off_sg;    // sign arrays
  size_t off_misc;  // dt, t, step, status, diag_out
  size_t off_cnt;   // event counter slots
  size_t off_cfl;   // cfl partials
  size_t off_diag;  // diag partials
  size_t off_frag;  // learned correction: weights packed as bf16 MFMA fragments
  size_t off_phi;   // learned correction: the normal CDF table of its GELU
  size_t off_grav;  // self-gravity: 4 padded T arrays (Psi, grad Psi), the complex
                    // [nz][ny][nx] array, twiddle and eigenvalue tables (0 bytes if off)
  size_t off_scal;  // passive scalars: nscalar padded T arrays at t^n, then nscalar at
                    // t^{n+1/2}
  size_t off_part;  // particles: two buffers of x [3][npart], v [3][npart], m [npart];
                    // two id arrays [npart]; tile counters, offsets, cursors
  size_t total;
};

bool geo_of(const mhd_config* c, Geo* g) {
  const int n[3] = {c->nx, c->ny, c->nz};
  long long np = 1;
  for (int a = 0; a < 3; ++a) {
    if (n[a] < 1 || n[a] > (1 << 20)) return false;
    g->n[a] = n[a];
    g->ext[a] = n[a] + 2 * NG + 1;
    np *= g->ext[a];
    const bool plo = c->bc[2 * a] == MHD_BC_PERIODIC, phi = c->bc[2 * a + 1] == MHD_BC_PERIODIC;
    if (plo != phi) return false;
    g->nf[a] = n[a] + (plo ? 0 : 1);
    g->bc[2 * a] = c->bc[2 * a];
    g->bc[2 * a + 1] = c->bc[2 * a + 1];
  }
  if (np >= (1ll << 31) - 16) return false;
  g->sy = g->ext[0];
  g->sz = g->ext[0] * g->ext[1];
  g->np = (int)np;
  g->d[0] = c->dx;
  g->d[1] = c->dy;
  g->d[2] = c->dz;
  for (int a = 0; a < 3; ++a) g->id[a] = 1.0 / g->d[a];
  g->x0[0] = c->x0;
  g->x0[1] = c->y0;
  g->x0[2] = c->z0;
  return true;
}

bool config_ok(const mhd_config* c) {
  if (!c) return false;
  if (c->precision != MHD_FP64 && c->precision != MHD_FP32 && c->precision != MHD_FP32_COMP)
    return false;
  for (int q = 0; q < 6; ++q)
    if (c->bc[q] < MHD_BC_PERIODIC || c->bc[q] > MHD_BC_INFLOW) return false;
  if (!(c->dx > 0) || !(c->dy > 0) || !(c->dz > 0)) return false;
  if (!isfinite(c->x0) || !isfinite(c->y0) || !isfinite(c->z0)) return false;
  if (!(c->gamma > 1.0) || !isfinite(c->gamma)) return false;
  if (!(c->cfl > 0.0) || !(c->cfl <= 1.0)) return false;
  if (c->recon < MHD_RECON_PAPER || c->recon > MHD_RECON_FIRST) return false;
  if (!(c->kappa >= -1.0) || !(c->kappa < 1.0)) return false;
  if (c->source < MHD_SRC_NONE || c->source > MHD_SRC_SELF_GRAVITY) return false;
  if (c->source == MHD_SRC_SELF_GRAVITY) {
    // periodic box, extents powers of two up to 1024 (radix-2 FFT lines in LDS)
    const int n[3] = {c->nx, c->ny, c->nz};
    for (int a = 0; a < 3; ++a) {
      if (c->bc[2 * a] != MHD_BC_PERIODIC || c->bc[2 * a + 1] != MHD_BC_PERIODIC) return false;
      if (n[a] < 1 || n[a] > 1024 || (n[a] & (n[a] - 1)) != 0) return false;
    }
    if (!(c->src[0] >= 0.0) || !isfinite(c->src[0])) return false;
  }
  if (!(c->rho_floor >= 0.0) || !(c->p_floor >= 0.0)) return false;
  if (c->riemann < MHD_RIEMANN_HLLD || c->riemann > MHD_RIEMANN_HLLC) return false;
  if (c->nscalar < 0 || c->nscalar > MHD_MAX_SCALARS) return false;
  if (c->npart < 0 || c->npart > 0x7fffffffll) return false;
  if (c->npart > 0 && c->source != MHD_SRC_SELF_GRAVITY) return false;
  if (c->reserved != 0) return false;
  if (c->recovery != MHD_RECOVERY_FP64 && c->recovery != MHD_RECOVERY_OFF) return false;
  if (c->precision != MHD_FP32 && c->recovery != MHD_RECOVERY_FP64) return false;
  Geo g;
  if (!geo_of(c, &g)) return false;
  // the flux kernel addresses every padded array with 32-bit byte offsets
  const unsigned long long es = c->precision == MHD_FP64 ? 8ull : 4ull;
  return (unsigned long long)g.np * es <= 0xFFFFFFFFull;
}

int ntiles_of(const Geo& g) {
  return ((g.n[0] + kTile - 1) / kTile) * ((g.n[1] + kTile - 1) / kTile) *
         ((g.n[2] + kTile - 1) / kTile);
}

Layout layout_of(const mhd_config* c) {
  Geo g;
  geo_of(c, &g);
  const size_t es = c->precision == MHD_FP64 ? sizeof(double) : sizeof(float);
  Layout L;
  L.arr = align_up((size_t)g.np * es);
  L.arr8 = align_up((size_t)g.np);
  L.off_t = 0;
  L.off_sg = L.off_t + (kNumT + (c->precision == MHD_FP32_COMP ? kCompT : 0)) * L.arr;
  L.off_misc = L.off_sg + 4 * L.arr8;  // 3 sign arrays + shock flags
  L.off_cnt = L.off_misc + align_up(64 * sizeof(double));
  L.off_cfl = L.off_cnt + align_up((size_t)kNumCounters * kCounterSlots * kCounterStride *
                                   sizeof(unsigned long long));
  L.off_diag = L.off_cfl + align_up((size_t)cfl_blocks(g) * sizeof(double));
  L.off_frag = L.off_diag + align_up((size_t)diag_blocks(g) * 16 * sizeof(double));
  L.off_phi = L.off_frag + align_up((size_t)kMlpFragBytes);
  L.off_grav = L.off_phi + align_up((size_t)kPhiBytes);
  size_t grav = 0;
  if (c->source == MHD_SRC_SELF_GRAVITY) {
    const size_t ncell = (size_t)g.n[0] * g.n[1] * g.n[2];
    grav = 4 * L.arr + align_up(ncell * 2 * es);
    for (int a = 0; a < 3; ++a) grav += align_up((size_t)g.n[a] * 2 * es);  // twiddles, eigenvalues
  }
  L.off_scal = L.off_grav + grav;
  L.off_part = L.off_scal + 2 * (size_t)c->nscalar * L.arr;
  size_t part = 0;
  if (c->npart > 0) {
    const size_t np = (size_t)c->npart, nt = (size_t)ntiles_of(g);
    const size_t mc = np / kChunk + nt;  // chunks of at most kChunk particles per tile
    part = 2 * align_up(7 * np * es) + 2 * align_up(np * sizeof(int)) +
           align_up((4 * nt + 2 + 1 + 3 * mc) * sizeof(int));
  }
  L.total = L.off_part + part;
  return L;
}

// misc block (doubles): [0] dt, [1] t, [2] step (int64), [7] status
// (uint32), [16..31] diag output
enum { M_DT = 0, M_T = 1, M_STEP = 2, M_STATUS = 7, M_DIAG = 16 };

}  // namespace

struct mhd_ctx {
  mhd_config cfg;
  Geo g;
  Physics ph;
  hipStream_t st;
  char* ws;
  Layout L;
  bool sticky;
  // profiling: event i opens the interval of a kernel of class kind[i]; the
  // interval closes at event i + 1
  bool prof_on = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<int> ev_kind;
  size_t ev_used = 0;
  double prof_ms[16] = {0};
  int64_t prof_n[16] = {0};
  void mark(int kind) {
    if (!prof_on) return;
    if (ev_used == ev_pool.size()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        prof_on = false;
        return;
      }
      ev_pool.push_back(e);
      ev_kind.push_back(0);
    }
    ev_kind[ev_used] = kind;
    (void)hipEventRecord(ev_pool[ev_used], st);
    ++ev_used;
  }
  // fold the recorded intervals into the per-class sums (after a sync)
  void fold() {
    for (size_t i = 0; i + 1 < ev_used; ++i) {
      if (ev_kind[i] < 0) continue;
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev_pool[i], ev_pool[i + 1]) == hipSuccess) {
        prof_ms[ev_kind[i]] += ms;
        prof_n[ev_kind[i]] += 1;
      }
    }
    ev_used = 0;
  }
  ~mhd_ctx() {
    for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  }
  void* arr(int q) const { return ws + L.off_t + (size_t)q * L.arr; }
  int8_t* sg(int a) const { return (int8_t*)(ws + L.off_sg + (size_t)a * L.arr8); }
  uint8_t* shock() const { return (uint8_t*)(ws + L.off_sg + 3 * L.arr8); }
  // learned correction and fine-flux accumulation
  const float* mlp_params = nullptr;
  double mlp_tau = 0.5, mlp_jump = 0.5, mlp_tau_flux = 0.0;
  void* flux_acc = nullptr;
  MlpRef mlp_ref() const {
    MlpRef m;
    m.params = mlp_params;
    m.tau = mlp_tau;
    m.jump = mlp_jump;
    m.tau_flux = mlp_tau_flux;
    m.shock = shock();
    m.frags = frags();
    m.phi = (const float4*)(ws + L.off_phi);
    return m;
  }
  double* misc() const { return (double*)(ws + L.off_misc); }
  double* cfl_part() const { return (double*)(ws + L.off_cfl); }
  double* diag_part() const { return (double*)(ws + L.off_diag); }
  unsigned* frags() const { return (unsigned*)(ws + L.off_frag); }
  unsigned long long* counter_slots() const { return (unsigned long long*)(ws + L.off_cnt); }
  Counters counters() const {
    Counters c;
    unsigned long long* base = counter_slots();
    const size_t span = (size_t)kCounterSlots * kCounterStride;
    c.hll = base;
    c.deg = base + span;
    c.floor_hits = base + 2 * span;
    c.fp64_rec = base + 3 * span;
    c.mlp_faces = base + 4 * span;
    c.mlp_gated = base + 5 * span;
    c.status = (unsigned int*)(misc() + M_STATUS);
    return c;
  }
  // The corrector writes the new faces into the half step's face arrays
  // (the cells in place): fcur names the face set that holds U's faces.
  int fcur = 0;
  // w_valid: prim<T>(0) holds the primitives of U (interior and ghost
  // shell), as the last step left them; cfl_valid: cfl_part() holds that
  // step's update_cfl_blocks() partials of U's time-step candidates.
  bool w_valid = false, cfl_valid = false;
  // xg_stale: the last step ran lite (on a fully periodic box the fused path
  // reads every ghost at its interior image, so its stages fill only the
  // faces at index n, and neither the primitives' ghost shell nor the outer
  // flux layer); any other path refills the ghosts of U and its primitives
  // first.
  bool xg_stale = false;
  // keep every component of every face's flux in memory (mhd_set_full_fluxes)
  bool full_fluxes = false;
  // the last step kept every component of its corrector fluxes (full
  // fluxes, the learned correction or the flux accumulation was on):
  // mhd_mlp_samples reads them
  bool fluxes_kept = false;
  template <class T>
  Cons<T> cons(int set) const {  // set 0: U (t^n), 1: U* (half step)
    Cons<T> s;
    for (int m = 0; m < 5; ++m) s.u[m] = (T*)arr(8 * set + m);
    for (int a = 0; a < 3; ++a) s.b[a] = (T*)arr(8 * (set ^ fcur) + 5 + a);
    for (int m = 0; m < 5; ++m) s.lo[m] = comp() ? (float*)arr(kNumT + 5 * set + m) : nullptr;
    return s;
  }
  bool comp() const { return cfg.precision == MHD_FP32_COMP; }
  // compensated FP32: the sweep's stage increments of the cells
  Inc inc() const {
    Inc d;
    for (int m = 0; m < 5; ++m) d.du[m] = comp() ? (float*)arr(kNumT + 10 + m) : nullptr;
    return d;
  }
  template <class T>
  Cons<T> inc_cells() const {  // the increments as the cells of a destination set
    Cons<T> s = cons<T>(0);
    const Inc d = inc();
    for (int m = 0; m < 5; ++m) {
      s.u[m] = (T*)d.du[m];
      s.lo[m] = nullptr;
    }
    return s;
  }
  template <class T>
  Prim<T> prim(int set) const {  // set 0: of U, 1: of U* (the corrector's input)
    const int q = set ? 50 : 16;
    Prim<T> w;
    w.w[0] = (T*)arr(8 * set);  // rho of the primitives: the set's own cell density
    for (int m = 1; m < 8; ++m) w.w[m] = (T*)arr(q + m - 1);
    for (int a = 0; a < 3; ++a) w.ec[a] = (T*)arr(q + 7 + a);
    return w;
  }
  template <class T>
  Flux<T> flux() const {
    Flux<T> f;
    for (int a = 0; a < 3; ++a) {
      for (int m = 0; m < 7; ++m) f.f[a][m] = (T*)arr(26 + 7 * a + m);
      f.sg[a] = sg(a);
    }
    return f;
  }
  template <class T>
  Edge<T> edge() const {
    Edge<T> e;
    for (int a = 0; a < 3; ++a) e.e[a] = (T*)arr(47 + a);
    return e;
  }
  int nscalar() const { return cfg.nscalar; }
  template <class T>
  Scal<T> scal(int set) const {  // set 0: rho X at t^n, 1: at t^{n+1/2}
    Scal<T> s{};
    for (int m = 0; m < cfg.nscalar; ++m)
      s.x[m] = (T*)(ws + L.off_scal + ((size_t)set * cfg.nscalar + m) * L.arr);
    return s;
  }
  // particles: buffer `part_cur` holds the current order
  int part_cur = 0;
  template <class T>
  char* part_base(int which) const {
    const size_t np = (size_t)cfg.npart;
    return ws + L.off_part + (size_t)which * align_up(7 * np * sizeof(T));
  }
  template <class T>
  int* part_ids(int which) const {
    const size_t np = (size_t)cfg.npart;
    return (int*)(ws + L.off_part + 2 * align_up(7 * np * sizeof(T)) +
                  (size_t)which * align_up(np * sizeof(int)));
  }
  int* tile_ints() const {
    const size_t np = (size_t)cfg.npart;
    const size_t es = cfg.precision == MHD_FP64 ? sizeof(double) : sizeof(float);
    return (int*)(ws + L.off_part + 2 * align_up(7 * np * es) + 2 * align_up(np * sizeof(int)));
  }
  template <class T>
  Parts<T> parts(int which) const {
    Parts<T> p{};
    p.n = cfg.npart;
    if (p.n > 0) {
      T* b = (T*)part_base<T>(which);
      p.x = b;
      p.v = b + 3 * p.n;
      p.m = b + 6 * p.n;
      p.id = part_ids<T>(which);
      const int nt = ntiles_of(g);
      // tile ints: counters [nt], offsets [nt + 1], cursors [nt], chunk
      // offsets [nt + 1], chunk list [1 + 3 max_chunks]
      p.toff = tile_ints() + nt;
      p.chunk = tile_ints() + 4 * nt + 2;
      for (int a = 0; a < 3; ++a) p.nt[a] = (g.n[a] + kTile - 1) / kTile;
      p.ntiles = nt;
      p.max_chunks = (int)(cfg.npart / kChunk + nt);
    }
    return p;
  }
  template <class T>
  Parts<T> parts() const {
    return parts<T>(part_cur);
  }
  template <class T>
  PartSort<T> part_sort(int which) const {
    PartSort<T> s{};
    if (cfg.npart > 0) {
      const Parts<T> p = parts<T>(which);
      s.x = p.x;
      s.v = p.v;
      s.m = p.m;
      s.id = p.id;
      const int nt = ntiles_of(g);
      s.cnt = tile_ints();
      s.off = s.cnt + nt;
      s.cur = s.off + nt + 1;
      s.coff = s.cur + nt;
      s.chunk = s.coff + nt + 1;
    }
    return s;
  }
  bool gravity() const { return cfg.source == MHD_SRC_SELF_GRAVITY; }
  template <class T>
  Grav<T> grav() const {
    Grav<T> r{};
    if (!gravity()) return r;
    char* b = ws + L.off_grav;
    r.psi = (T*)b;
    for (int a = 0; a < 3; ++a) r.g[a] = (T*)(b + (1 + a) * L.arr);
    return r;
  }
  // tables: per axis n/2 twiddle pairs then n eigenvalues, each block aligned
  template <class T>
  GravFFT<T> grav_fft() const {
    GravFFT<T> f{};
    char* b = ws + L.off_grav + 4 * L.arr;
    f.c = (T*)b;
    b += align_up((size_t)g.n[0] * g.n[1] * g.n[2] * 2 * sizeof(T));
    for (int a = 0; a < 3; ++a) {
      f.tw[a] = (const T*)b;
      f.lam[a] = (const T*)(b + (size_t)g.n[a] * sizeof(T));  // after n/2 pairs
      b += align_up((size_t)g.n[a] * 2 * sizeof(T));
    }
    return f;
  }
};

namespace {

template <class T>
Muscl<T> muscl_of(int recon, double kappa) {
  Muscl<T> m;
  const double K1 = (1.0 - kappa) / 4.0, K2 = (1.0 + kappa) / 4.0;
  const double b = (3.0 - kappa) / (1.0 - kappa);
  m.first_order = recon == MHD_RECON_FIRST;
  if (recon == MHD_RECON_KAPPA) {
    m.cA = (T)K1;
    m.bA = (T)b;
    m.cB = (T)K2;
    m.bB = (T)b;
  } else {  // the paper's Eq. 13-14 as printed
    m.cA = (T)K2;
    m.bA = (T)1.0;
    m.cB = (T)K1;
    m.bB = (T)b;
  }
  return m;
}

Physics physics_of(const mhd_config* c) {
  Physics ph;
  ph.gamma = c->gamma;
  ph.igm1 = 1.0 / (c->gamma - 1.0);
  ph.riemann = c->riemann;
  ph.cfl = c->cfl;
  ph.source = c->source;
  for (int q = 0; q < 4; ++q) ph.src[q] = c->src[q];
  ph.rho_floor = c->rho_floor;
  ph.p_floor = c->p_floor;
  ph.recover = c->recovery == MHD_RECOVERY_FP64;
  const double* q = c->inflow;
  ph.inflow_u[0] = q[0];
  ph.inflow_u[1] = q[0] * q[1];
  ph.inflow_u[2] = q[0] * q[2];
  ph.inflow_u[3] = q[0] * q[3];
  ph.inflow_u[4] = q[4] / (c->gamma - 1.0) + 0.5 * q[0] * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) +
                   0.5 * (q[5] * q[5] + q[6] * q[6] + q[7] * q[7]);
  for (int a = 0; a < 3; ++a) ph.inflow_b[a] = q[5 + a];
  return ph;
}

int hip_status() {
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? MHD_OK : MHD_E_HIP;
}

}  // namespace

// Partial gradients of mhd_mlp_grad_noalloc: one row of MHD_MLP_NPARAM + 1
// floats per 64-sample block, for at most MHD_MLP_NOALLOC_MAX samples.  In
// host code this name is only a stand-in for the symbol: kernels get the
// device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) float scratch[(size_t)(MHD_MLP_NOALLOC_MAX / 64) *
                                               (MHD_MLP_NPARAM + 1)];

namespace {

constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch_addr[kScratchDevices];  // device address of `scratch`, per device

// Device address of `scratch` on device dev, which must be the current
// device; looked up on the first call on each device.
int scratch_address(int dev, float** out) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return MHD_E_HIP;
    g_scratch_addr[dev] = (float*)p;
  }
  *out = g_scratch_addr[dev];
  return MHD_OK;
}

template <class T>
void enqueue_step(mhd_ctx* c, DtRef dt) {
  // host-side ranges of the enqueueing (rocprofv3 --marker-trace): the
  // step, its predictor and its corrector
  roctxRangePushA("mhd_step");
  const Geo& g = c->g;
  const Counters cnt = c->counters();
  const Cons<T> U = c->cons<T>(0), Us = c->cons<T>(1);
  // the corrector's result: U's cells in place, the new faces in the half
  // step's face arrays (which become U's at the end of the step)
  Cons<T> Un = U;
  for (int a = 0; a < 3; ++a) Un.b[a] = Us.b[a];
  // compensated FP32: the sweeps leave the stage increments, which the
  // stage updates add to the pairs
  const bool comp = c->comp();
  const Cons<T> Dn = comp ? c->inc_cells<T>() : Us, Dc = comp ? c->inc_cells<T>() : Un;
  const Inc inc = c->inc();
  const Prim<T> W = c->prim<T>(0), Ws = c->prim<T>(1);
  const Flux<T> F = c->flux<T>();
  const Edge<T> E = c->edge<T>();
  const Muscl<T> first = muscl_of<T>(MHD_RECON_FIRST, c->cfg.kappa);
  const Muscl<T> second = muscl_of<T>(c->cfg.recon, c->cfg.kappa);
  const int ns = c->nscalar();
  const Scal<T> Xn = c->scal<T>(0), Xh = c->scal<T>(1);
  if (c->cfg.npart > 0) {  // particles sorted by tile at the start of every step
    c->mark(MHD_K_NBODY);
    launch_particle_sort<T>(g, c->parts<T>(), c->part_sort<T>(1 - c->part_cur), c->st);
    c->part_cur = 1 - c->part_cur;
  }
  const Parts<T> Pp = c->parts<T>();
  DtRef at_n = dt, at_half = dt;  // particle positions of the two potentials
  at_n.factor = 0.0;
  at_half.factor = 0.5;
  // the fused flux sweep: always in the predictor; in the corrector unless
  // the learned correction or the flux accumulation needs every face's full
  // flux in memory
  const bool swept = !c->mlp_params && !c->flux_acc;
  const int store = c->full_fluxes ? 2 : (ns > 0 ? 1 : 0);
  c->fluxes_kept = !swept || c->full_fluxes;
  // ghost layers, the primitives' ghost shell and the outer flux layer left
  // out of the stages: only where nothing of this step reads them (fully
  // periodic box, no flux accumulation, no passive scalar, no full fluxes
  // kept for samples): every reader takes the interior images
  bool per = true;
  for (int a = 0; a < 6; ++a) per = per && g.bc[a] == 0;
  const bool lite = per && !c->flux_acc && ns == 0 && !c->full_fluxes;
  if (c->xg_stale && !lite) {
    c->mark(MHD_K_GHOSTS);
    launch_ghosts<T>(g, c->ph, U, false, c->st);
    if (c->w_valid) {
      c->mark(MHD_K_PRIM);
      launch_prim_shell<T>(g, c->ph, U, W, cnt, c->st);
    }
  }
  c->xg_stale = lite;
  // primitives of U^n (and the step's own dt): left by the previous step's
  // corrector, else one pass over U
  c->mark(MHD_K_PRIM);
  if (!c->w_valid) {
    if (dt.ptr)
      launch_prim_cfl<T>(g, c->ph, U, W, c->cfl_part(), c->misc() + M_DT, cnt, Pp, c->st);
    else
      launch_prim<T>(g, c->ph, U, W, cnt, c->st);
  } else if (dt.ptr) {
    if (c->cfl_valid)
      launch_cfl_reduce<T>(g, c->ph, c->cfl_part(), update_cfl_blocks(g), c->misc() + M_DT, Pp,
                           c->st);
    else
      launch_cfl<T>(g, c->ph, U, c->cfl_part(), c->misc() + M_DT, cnt, Pp, c->st);
  }
  if (c->gravity()) {
    c->mark(MHD_K_GRAVITY);
    launch_self_gravity<T>(g, c->ph, W.w[0], c->grav_fft<T>(), c->grav<T>(), Pp, at_n, c->st);
  }
  DtRef half = dt;
  half.factor = 0.5;
  // predictor: first-order fluxes of U^n, half step into U* and its
  // primitives
  roctxRangePushA("mhd_predictor");
  c->mark(MHD_K_FLUX);
  launch_sweep<T>(g, c->ph, W, U, Dn, F, first, c->grav<T>(), half, cnt, store, comp, c->st);
  if (!lite) {
    c->mark(MHD_K_FLUX_OUTER);
    launch_flux_outer<T>(g, c->ph, W, U, F, first, cnt, store, c->st);
  }
  c->mark(MHD_K_EMF);
  launch_emf<T>(g, W, F, E, c->st);
  c->mark(MHD_K_UPDATE);
  launch_update<T>(g, c->ph, U, Us, W, Ws, F, E, c->grav<T>(), half, cnt, nullptr, true, inc,
                   c->st);
  if (ns) {
    c->mark(MHD_K_SCALARS);
    launch_scalar_update<T>(g, W.w[0], F, Xn, Xn, Xh, ns, first, half, c->st);
    launch_scalar_ghosts<T>(g, Xh, ns, c->st);
  }
  c->mark(MHD_K_GHOSTS);
  launch_ghosts<T>(g, c->ph, Us, lite, c->st);
  if (!lite) {
    c->mark(MHD_K_PRIM);
    launch_prim_shell<T>(g, c->ph, Us, Ws, cnt, c->st);
  }
  roctxRangePop();
  // corrector: MUSCL fluxes of U*, full step from U^n, the primitives of
  // U^{n+1} and the candidates of the next step's dt
  roctxRangePushA("mhd_corrector");
  if (c->gravity()) {
    c->mark(MHD_K_GRAVITY);
    launch_self_gravity<T>(g, c->ph, Ws.w[0], c->grav_fft<T>(), c->grav<T>(), Pp, at_half,
                           c->st);
  }
  if (c->mlp_params) {
    c->mark(MHD_K_SHOCK);
    launch_shock<T>(g, Ws, c->shock(), c->mlp_jump, lite, c->st);
    // the caller may change the weights between steps: repack every step
    launch_mlp_pack(c->mlp_params, c->frags(), c->st);
    for (int a = 0; a < 3; ++a) {
      c->mark(MHD_K_FLUX_MLP);
      launch_flux_mlp<T>(g, c->ph, a, Ws, Us.b[a], F, second, cnt, c->mlp_ref(), lite, c->st);
    }
  } else if (swept) {
    c->mark(MHD_K_FLUX);
    launch_sweep<T>(g, c->ph, Ws, Un, Dc, F, second, c->grav<T>(), dt, cnt, store, comp, c->st);
    if (!lite) {
      c->mark(MHD_K_FLUX_OUTER);
      launch_flux_outer<T>(g, c->ph, Ws, Us, F, second, cnt, store, c->st);
    }
  } else {
    c->mark(MHD_K_FLUX);
    launch_flux<T>(g, c->ph, Ws, Us, F, second, cnt, c->st);
  }
  if (c->flux_acc) {
    c->mark(MHD_K_OTHER);
    launch_fluxacc<T>(g, F, (T*)c->flux_acc, dt, c->st);
  }
  c->mark(MHD_K_EMF);
  launch_emf<T>(g, Ws, F, E, c->st);
  c->mark(MHD_K_UPDATE);
  launch_update<T>(g, c->ph, U, Un, Ws, W, F, E, c->grav<T>(), dt, cnt, c->cfl_part(), swept,
                   inc, c->st);
  if (ns) {
    c->mark(MHD_K_SCALARS);
    launch_scalar_update<T>(g, Ws.w[0], F, Xn, Xh, Xn, ns, second, dt, c->st);
    launch_scalar_ghosts<T>(g, Xn, ns, c->st);
  }
  c->mark(MHD_K_GHOSTS);
  launch_ghosts<T>(g, c->ph, Un, lite, c->st);
  if (!lite) {
    c->mark(MHD_K_PRIM);
    launch_prim_shell<T>(g, c->ph, Un, W, cnt, c->st);
  }
  if (Pp.n > 0) {
    c->mark(MHD_K_NBODY);
    launch_kick_drift<T>(g, Pp, c->grav<T>(), dt, c->st);
  }
  roctxRangePop();
  c->mark(MHD_K_OTHER);
  launch_advance_time(c->misc() + M_T, (long long*)(c->misc() + M_STEP), dt, c->st);
  c->mark(-1);
  c->fcur ^= 1;
  c->w_valid = true;
  c->cfl_valid = true;
  roctxRangePop();
}

template <class T>
void enqueue_cfl(mhd_ctx* c) {
  c->cfl_valid = false;  // the partials are this pass's now
  c->mark(MHD_K_CFL);
  launch_cfl<T>(c->g, c->ph, c->cons<T>(0), c->cfl_part(), c->misc() + M_DT, c->counters(),
                c->parts<T>(), c->st);
  c->mark(-1);
}

// The normal CDF table of the learned correction's GELU (layout in
// mhd_kernels.hpp), from Phi(x) = erfc(-x / sqrt 2) / 2 in FP64.
int upload_phi_table(mhd_ctx* c) {
  std::vector<float> h((size_t)kPhiN * 4);
  const auto Phi = [](double x) { return 0.5 * erfc(-x * 0.70710678118654752440); };
  for (int i = 0; i < kPhiN; ++i) {
    const double x0 = -kPhiHalf + (double)i / kPhiScale, dx = 1.0 / kPhiScale;
    const double p0 = Phi(x0), pm = Phi(x0 + 0.5 * dx), p1 = Phi(x0 + dx);
    h[4 * i] = (float)p0;
    h[4 * i + 1] = (float)(-3.0 * p0 + 4.0 * pm - p1);
    h[4 * i + 2] = (float)(2.0 * p0 - 4.0 * pm + 2.0 * p1);
    h[4 * i + 3] = 0.0f;
  }
  if (hipMemcpyAsync(c->ws + c->L.off_phi, h.data(), h.size() * sizeof(float),
                     hipMemcpyHostToDevice, c->st) != hipSuccess ||
      hipStreamSynchronize(c->st) != hipSuccess)
    return MHD_E_HIP;
  return MHD_OK;
}

// Twiddles exp(-2 pi i q / n) (q < n/2) and the 3-point Laplacian's
// eigenvalues (2 cos(2 pi m / n) - 2) / d^2 of each axis, computed in FP64
// and stored in the context precision, in the layout grav_fft() reads.
template <class T>
int upload_gravity_tables(mhd_ctx* c) {
  const GravFFT<T> f = c->grav_fft<T>();
  for (int a = 0; a < 3; ++a) {
    const int n = c->g.n[a];
    std::vector<T> h((size_t)n * 2, T(0));
    for (int q = 0; q < n / 2; ++q) {
      const double ang = 2.0 * 3.14159265358979323846 * q / n;
      h[2 * q] = (T)cos(ang);
      h[2 * q + 1] = (T)(-sin(ang));
    }
    for (int m = 0; m < n; ++m)
      h[(size_t)n + m] =
          (T)((2.0 * cos(2.0 * 3.14159265358979323846 * m / n) - 2.0) / (c->g.d[a] * c->g.d[a]));
    if (hipMemcpyAsync((void*)f.tw[a], h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice,
                       c->st) != hipSuccess ||
        hipStreamSynchronize(c->st) != hipSuccess)
      return MHD_E_HIP;
  }
  return MHD_OK;
}

int sync_status(mhd_ctx* c) {
  unsigned int st = 0;
  if (hipMemcpyAsync(&st, c->misc() + M_STATUS, sizeof(st), hipMemcpyDeviceToHost, c->st) !=
      hipSuccess)
    return MHD_E_HIP;
  if (hipStreamSynchronize(c->st) != hipSuccess) return MHD_E_HIP;
  if (st & MHD_ST_BAD_STATE) c->sticky = true;
  return c->sticky ? MHD_E_STATE : MHD_OK;
}

}  // namespace

extern "C" {

int mhd_abi_version(void) { return MHD_ABI_VERSION; }

const char* mhd_strerror(int code) {
  switch (code) {
    case MHD_OK: return "ok";
    case MHD_E_ARG: return "invalid argument or configuration";
    case MHD_E_HIP: return "HIP runtime error";
    case MHD_E_STATE: return "invalid state: non-finite value, rho <= 0 or P <= 0";
    case MHD_E_UNSUPPORTED: return "unsupported configuration";
    case MHD_E_WS: return "workspace too small or misaligned";
    default: return "unknown status";
  }
}

int mhd_workspace_bytes(const mhd_config* cfg, size_t* out) {
  if (!out || !config_ok(cfg)) return MHD_E_ARG;
  *out = layout_of(cfg).total;
  return MHD_OK;
}

int mhd_init(const mhd_config* cfg, void* d_ws, size_t ws_bytes, const void* d_cell5,
             const void* d_bx, const void* d_by, const void* d_bz, void* hip_stream,
             mhd_ctx** out) {
  if (!out || !config_ok(cfg) || !d_cell5 || !d_bx || !d_by || !d_bz) return MHD_E_ARG;
  *out = nullptr;
  const Layout L = layout_of(cfg);
  if (!d_ws || ws_bytes < L.total || ((uintptr_t)d_ws % kAlign) != 0) return MHD_E_WS;
  mhd_ctx* c = new (std::nothrow) mhd_ctx();
  if (!c) return MHD_E_HIP;
  c->cfg = *cfg;
  geo_of(cfg, &c->g);
  c->ph = physics_of(cfg);
  c->st = (hipStream_t)hip_stream;
  c->ws = (char*)d_ws;
  c->L = L;
  c->sticky = false;
  if (hipMemsetAsync(c->misc(), 0, 64 * sizeof(double), c->st) != hipSuccess ||
      hipMemsetAsync(c->counter_slots(), 0, L.off_cfl - L.off_cnt, c->st) != hipSuccess ||
      (L.total > L.off_scal &&
       hipMemsetAsync(c->ws + L.off_scal, 0, L.total - L.off_scal, c->st) != hipSuccess)) {
    delete c;
    return MHD_E_HIP;
  }
  if (cfg->npart > 0) {
    if (cfg->precision == MHD_FP64)
      launch_particles_init<double>(c->g, c->parts<double>(), c->st);
    else
      launch_particles_init<float>(c->g, c->parts<float>(), c->st);
  }
  if (c->gravity()) {
    const int rc = cfg->precision == MHD_FP64 ? upload_gravity_tables<double>(c)
                                              : upload_gravity_tables<float>(c);
    if (rc != MHD_OK) {
      delete c;
      return rc;
    }
  }
  if (upload_phi_table(c) != MHD_OK) {
    delete c;
    return MHD_E_HIP;
  }
  if (cfg->precision == MHD_FP64) {
    launch_scatter<double>(c->g, (const double*)d_cell5, (const double*)d_bx,
                           (const double*)d_by, (const double*)d_bz, c->cons<double>(0), c->st);
    launch_ghosts<double>(c->g, c->ph, c->cons<double>(0), false, c->st);
    enqueue_cfl<double>(c);
  } else if (c->comp()) {
    launch_scatter_comp(c->g, (const double*)d_cell5, (const double*)d_bx, (const double*)d_by,
                        (const double*)d_bz, c->cons<float>(0), c->st);
    launch_ghosts<float>(c->g, c->ph, c->cons<float>(0), false, c->st);
    enqueue_cfl<float>(c);
  } else {
    launch_scatter<float>(c->g, (const float*)d_cell5, (const float*)d_bx, (const float*)d_by,
                          (const float*)d_bz, c->cons<float>(0), c->st);
    launch_ghosts<float>(c->g, c->ph, c->cons<float>(0), false, c->st);
    enqueue_cfl<float>(c);
  }
  int rc = hip_status();
  if (rc == MHD_OK) rc = sync_status(c);
  if (rc != MHD_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return MHD_OK;
}

int mhd_step(mhd_ctx* c, const double* dt_host, int nsteps) {
  if (!c || nsteps < 0) return MHD_E_ARG;
  if (c->sticky) return MHD_E_STATE;
  if (dt_host)
    for (int s = 0; s < nsteps; ++s)
      if (!(dt_host[s] > 0.0) || !isfinite(dt_host[s])) return MHD_E_ARG;
  for (int s = 0; s < nsteps; ++s) {
    DtRef dt;
    dt.factor = 1.0;
    if (dt_host) {
      dt.value = dt_host[s];
      dt.ptr = nullptr;
    } else {
      dt.value = 0.0;
      dt.ptr = c->misc() + M_DT;
    }
    if (c->cfg.precision == MHD_FP64)
      enqueue_step<double>(c, dt);
    else
      enqueue_step<float>(c, dt);
  }
  return hip_status();
}

int mhd_dt(mhd_ctx* c, double* out) {
  if (!c || !out) return MHD_E_ARG;
  if (c->cfg.precision == MHD_FP64)
    enqueue_cfl<double>(c);
  else
    enqueue_cfl<float>(c);
  if (hip_status() != MHD_OK) return MHD_E_HIP;
  if (hipMemcpyAsync(out, c->misc() + M_DT, sizeof(double), hipMemcpyDeviceToHost, c->st) !=
      hipSuccess)
    return MHD_E_HIP;
  return sync_status(c);
}

int mhd_diag(mhd_ctx* c, mhd_diag_t* out) {
  if (!c || !out) return MHD_E_ARG;
  memset(out, 0, sizeof(*out));
  if (c->cfg.precision == MHD_FP64) {
    enqueue_cfl<double>(c);
    launch_diag<double>(c->g, c->ph, c->cons<double>(0), c->diag_part(), c->misc() + M_DIAG,
                        c->st);
  } else {
    enqueue_cfl<float>(c);
    launch_diag<float>(c->g, c->ph, c->cons<float>(0), c->diag_part(), c->misc() + M_DIAG, c->st);
  }
  if (hip_status() != MHD_OK) return MHD_E_HIP;
  double m[32];
  std::vector<unsigned long long> slots((size_t)kNumCounters * kCounterSlots * kCounterStride);
  if (hipMemcpyAsync(m, c->misc(), sizeof(m), hipMemcpyDeviceToHost, c->st) != hipSuccess ||
      hipMemcpyAsync(slots.data(), c->counter_slots(), slots.size() * sizeof(unsigned long long),
                     hipMemcpyDeviceToHost, c->st) != hipSuccess)
    return MHD_E_HIP;
  if (hipStreamSynchronize(c->st) != hipSuccess) return MHD_E_HIP;
  const double* d = m + M_DIAG;
  unsigned long long cn[kNumCounters] = {0, 0, 0, 0, 0, 0};
  for (int q = 0; q < kNumCounters; ++q)
    for (int sl = 0; sl < kCounterSlots; ++sl)
      cn[q] += slots[((size_t)q * kCounterSlots + sl) * kCounterStride];
  out->dt = m[M_DT];
  out->t = m[M_T];
  memcpy(&out->step, &m[M_STEP], sizeof(int64_t));
  out->mass = d[0];
  for (int a = 0; a < 3; ++a) out->mom[a] = d[1 + a];
  out->energy = d[4];
  for (int a = 0; a < 3; ++a) out->bsum[a] = d[5 + a];
  const double h = fmin(c->g.d[0], fmin(c->g.d[1], c->g.d[2]));
  out->divb_max = d[11] > 0.0 ? d[8] * h / d[11] : d[8] * h;
  out->rho_min = d[9];
  out->p_min = d[10];
  out->n_hll_fallback = (int64_t)cn[0];
  out->n_degenerate = (int64_t)cn[1];
  out->n_floor = (int64_t)cn[2];
  out->n_fp64_recovery = (int64_t)cn[3];
  out->n_mlp_faces = (int64_t)cn[4];
  out->n_mlp_gated = (int64_t)cn[5];
  unsigned int st;
  memcpy(&st, &m[M_STATUS], sizeof(st));
  out->status = st;
  if (st & MHD_ST_BAD_STATE) c->sticky = true;
  return c->sticky ? MHD_E_STATE : MHD_OK;
}

int mhd_get_state(mhd_ctx* c, void* d_cell5, void* d_bx, void* d_by, void* d_bz) {
  if (!c || !d_cell5 || !d_bx || !d_by || !d_bz) return MHD_E_ARG;
  if (c->cfg.precision == MHD_FP64)
    launch_gather<double>(c->g, c->cons<double>(0), (double*)d_cell5, (double*)d_bx,
                          (double*)d_by, (double*)d_bz, c->st);
  else if (c->comp())
    launch_gather_comp(c->g, c->cons<float>(0), (double*)d_cell5, (double*)d_bx, (double*)d_by,
                       (double*)d_bz, c->st);
  else
    launch_gather<float>(c->g, c->cons<float>(0), (float*)d_cell5, (float*)d_bx, (float*)d_by,
                         (float*)d_bz, c->st);
  if (hip_status() != MHD_OK) return MHD_E_HIP;
  if (hipStreamSynchronize(c->st) != hipSuccess) return MHD_E_HIP;
  return MHD_OK;
}

static int scalar_copy(mhd_ctx* c, void* d, bool in) {
  if (!c || !d || c->nscalar() == 0) return MHD_E_ARG;
  if (c->cfg.precision == MHD_FP64) {
    launch_scalar_copy<double>(c->g, c->scal<double>(0), c->nscalar(), (double*)d, in, c->st);
    if (in) launch_scalar_ghosts<double>(c->g, c->scal<double>(0), c->nscalar(), c->st);
  } else {
    launch_scalar_copy<float>(c->g, c->scal<float>(0), c->nscalar(), (float*)d, in, c->st);
    if (in) launch_scalar_ghosts<float>(c->g, c->scal<float>(0), c->nscalar(), c->st);
  }
  if (hip_status() != MHD_OK) return MHD_E_HIP;
  if (hipStreamSynchronize(c->st) != hipSuccess) return MHD_E_HIP;
  return MHD_OK;
}

int mhd_set_particles(mhd_ctx* c, const void* d_x, const void* d_v, const void* d_m) {
  if (!c || !d_x || !d_v || !d_m || c->cfg.npart <= 0) return MHD_E_ARG;
  const size_t es = c->cfg.precision == MHD_FP64 ? sizeof(double) : sizeof(float);
  const size_t n = (size_t)c->cfg.npart;
  char* b = es == sizeof(double) ? c->part_base<double>(c->part_cur)
                                 : c->part_base<float>(c->part_cur);
  if (hipMemcpyAsync(b, d_x, 3 * n * es, hipMemcpyDeviceToDevice, c->st) != hipSuccess ||
      hipMemcpyAsync(b + 3 * n * es, d_v, 3 * n * es, hipMemcpyDeviceToDevice, c->st) !=
          hipSuccess ||
      hipMemcpyAsync(b + 6 * n * es, d_m, n * es, hipMemcpyDeviceToDevice, c->st) != hipSuccess)
    return MHD_E_HIP;
  if (c->cfg.precision == MHD_FP64)
    launch_particles_init<double>(c->g, c->parts<double>(), c->st);
  else
    launch_particles_init<float>(c->g, c->parts<float>(), c->st);
  if (hip_status() != MHD_OK) return MHD_E_HIP;
  return hipStreamSynchronize(c->st) == hipSuccess ? MHD_OK : MHD_E_HIP;
}

int mhd_get_particles(mhd_ctx* c, void* d_x, void* d_v) {
  if (!c || c->cfg.npart <= 0 || (!d_x && !d_v)) return MHD_E_ARG;
  if (c->cfg.precision == MHD_FP64)
    launch_particles_out<double>(c->parts<double>(), (double*)d_x, (double*)d_v, c->st);
  else
    launch_particles_out<float>(c->parts<float>(), (float*)d_x, (float*)d_v, c->st);
  if (hip_status() != MHD_OK) return MHD_E_HIP;
  return hipStreamSynchronize(c->st) == hipSuccess ? MHD_OK : MHD_E_HIP;
}

int mhd_set_scalars(mhd_ctx* c, const void* d_rho_x) {
  return scalar_copy(c, const_cast<void*>(d_rho_x), true);
}

int mhd_get_scalars(mhd_ctx* c, void* d_rho_x) { return scalar_copy(c, d_rho_x, false); }

int mhd_debug_array(mhd_ctx* c, int what, void* d_out, size_t* n_out) {
  if (!c || !d_out || what < 0 || what > 38) return MHD_E_ARG;
  const size_t es = c->cfg.precision == MHD_FP64 ? sizeof(double) : sizeof(float);
  if (what >= 35) {
    if (!c->gravity()) return MHD_E_ARG;
    const char* src = c->ws + c->L.off_grav + (size_t)(what - 35) * c->L.arr;
    if (hipMemcpyAsync(d_out, src, (size_t)c->g.np * es, hipMemcpyDeviceToDevice, c->st) !=
        hipSuccess)
      return MHD_E_HIP;
    if (hipStreamSynchronize(c->st) != hipSuccess) return MHD_E_HIP;
    if (n_out) *n_out = (size_t)c->g.np;
    return MHD_OK;
  }
  int q;
  if (what < 21)
    q = 26 + what;  // fluxes
  else if (what < 24)
    q = 47 + (what - 21);  // edges
  else if (what < 27)
    q = 57 + (what - 24);  // cell EMF of the corrector's input
  else if (what == 27)
    q = 8;  // primitive density of the corrector's input: U*'s own density
  else
    q = 50 + (what - 28);  // other primitives of the corrector's input
  if (hipMemcpyAsync(d_out, c->arr(q), (size_t)c->g.np * es, hipMemcpyDeviceToDevice, c->st) !=
      hipSuccess)
    return MHD_E_HIP;
  if (hipStreamSynchronize(c->st) != hipSuccess) return MHD_E_HIP;
  if (n_out) *n_out = (size_t)c->g.np;
  return MHD_OK;
}

int mhd_profile(mhd_ctx* c, int enable) {
  if (!c) return MHD_E_ARG;
  if (c->prof_on && hipStreamSynchronize(c->st) != hipSuccess) return MHD_E_HIP;
  c->ev_used = 0;
  for (int q = 0; q < 16; ++q) {
    c->prof_ms[q] = 0.0;
    c->prof_n[q] = 0;
  }
  c->prof_on = enable != 0;
  return MHD_OK;
}

int mhd_profile_get(mhd_ctx* c, mhd_profile_t* out) {
  if (!c || !out) return MHD_E_ARG;
  if (hipStreamSynchronize(c->st) != hipSuccess) return MHD_E_HIP;
  c->fold();
  memset(out, 0, sizeof(*out));
  for (int q = 0; q < 16; ++q) {
    out->ms[q] = c->prof_ms[q];
    out->launches[q] = c->prof_n[q];
  }
  out->n_kinds = MHD_K_COUNT;
  return MHD_OK;
}

int mhd_destroy(mhd_ctx* c) {
  if (!c) return MHD_E_ARG;
  delete c;
  return MHD_OK;
}

// 2x coarse-graining needs even extents and, per axis, both sides periodic
// or both not.
static bool coarsenable(const mhd_ctx* c) {
  for (int a = 0; a < 3; ++a) {
    if (c->g.n[a] % 2 != 0) return false;
    if ((c->g.bc[2 * a] == MHD_BC_PERIODIC) != (c->g.bc[2 * a + 1] == MHD_BC_PERIODIC))
      return false;
  }
  return true;
}

int mhd_set_mlp(mhd_ctx* c, const float* d_params, const mhd_gate* gate) {
  if (!c) return MHD_E_ARG;
  if (!d_params) {
    c->mlp_params = nullptr;
    return MHD_OK;
  }
  if (c->cfg.riemann != MHD_RIEMANN_HLLD) return MHD_E_UNSUPPORTED;
  if (!gate || !(gate->tau >= 0.0) || !(gate->jump > 0.0) || !(gate->tau_flux >= 0.0))
    return MHD_E_ARG;
  c->mlp_params = d_params;
  c->mlp_tau = gate->tau;
  c->mlp_jump = gate->jump;
  c->mlp_tau_flux = gate->tau_flux;
  return MHD_OK;
}

int mhd_flux_accumulate(mhd_ctx* c, void* d_acc) {
  if (!c) return MHD_E_ARG;
  if (d_acc && c->comp()) return MHD_E_UNSUPPORTED;
  if (d_acc && !coarsenable(c)) return MHD_E_UNSUPPORTED;
  c->flux_acc = d_acc;
  return MHD_OK;
}

int mhd_coarsen(mhd_ctx* c, void* d_cell5, void* d_bx, void* d_by, void* d_bz) {
  if (!c || !d_cell5 || !d_bx || !d_by || !d_bz) return MHD_E_ARG;
  if (c->comp()) return MHD_E_UNSUPPORTED;
  if (!coarsenable(c)) return MHD_E_UNSUPPORTED;
  if (c->cfg.precision == MHD_FP64)
    launch_coarsen<double>(c->g, c->cons<double>(0), (double*)d_cell5, (double*)d_bx,
                           (double*)d_by, (double*)d_bz, c->st);
  else
    launch_coarsen<float>(c->g, c->cons<float>(0), (float*)d_cell5, (float*)d_bx, (float*)d_by,
                          (float*)d_bz, c->st);
  if (hip_status() != MHD_OK) return MHD_E_HIP;
  return hipStreamSynchronize(c->st) == hipSuccess ? MHD_OK : MHD_E_HIP;
}

int mhd_set_full_fluxes(mhd_ctx* c, int enable) {
  if (!c) return MHD_E_ARG;
  c->full_fluxes = enable != 0;
  return MHD_OK;
}

int mhd_mlp_samples(mhd_ctx* c, const void* d_acc, double dt_coarse, int64_t n,
                    const int32_t* d_faces, float* d_x, float* d_t, uint8_t* d_mask) {
  if (!c || n < 0 || !(dt_coarse > 0.0)) return MHD_E_ARG;
  if (n > 0 && (!d_acc || !d_faces || !d_x || !d_t || !d_mask)) return MHD_E_ARG;
  // the last step must have left every component of its corrector fluxes
  if (!c->fluxes_kept) return MHD_E_ARG;
  if (c->comp()) return MHD_E_UNSUPPORTED;

  if (n == 0) return MHD_OK;
  if (c->cfg.precision == MHD_FP64) {
    launch_shock<double>(c->g, c->prim<double>(1), c->shock(), c->mlp_jump, c->xg_stale, c->st);
    launch_mlp_samples<double>(c->g, c->prim<double>(1), c->flux<double>(), c->shock(),
                               (const double*)d_acc, dt_coarse, c->ph.gamma, n, d_faces, d_x, d_t,
                               d_mask, c->st);
  } else {
    launch_shock<float>(c->g, c->prim<float>(1), c->shock(), c->mlp_jump, c->xg_stale, c->st);
    launch_mlp_samples<float>(c->g, c->prim<float>(1), c->flux<float>(), c->shock(),
                              (const float*)d_acc, dt_coarse, c->ph.gamma, n, d_faces, d_x, d_t,
                              d_mask, c->st);
  }
  return hip_status();
}

int mhd_mlp_forward(int64_t n, const float* d_x, const float* d_params, float* d_y,
                    void* hip_stream) {
  if (n < 0 || (n > 0 && (!d_x || !d_params || !d_y))) return MHD_E_ARG;
  if (n == 0) return MHD_OK;
  launch_mlp_forward(n, d_x, d_params, d_y, (hipStream_t)hip_stream);
  return hip_status();
}

int mhd_mlp_grad_workspace_bytes(int64_t n, size_t* out) {
  if (n <= 0 || !out) return MHD_E_ARG;
  *out = mlp_grad_workspace(n);
  return MHD_OK;
}

int mhd_mlp_grad(int64_t n, const float* d_x, const float* d_t, const float* d_params,
                 float* d_grad, float* d_loss, void* d_ws, size_t ws_bytes, void* hip_stream) {
  if (n <= 0 || !d_x || !d_t || !d_params || !d_grad || !d_ws) return MHD_E_ARG;
  if (ws_bytes < mlp_grad_workspace(n)) return MHD_E_WS;
  launch_mlp_grad(n, d_x, d_t, d_params, d_grad, d_loss, (float*)d_ws, (hipStream_t)hip_stream);
  return hip_status();
}

int mhd_mlp_grad_noalloc(int64_t n, const float* d_x, const float* d_t, const float* d_params,
                         float* d_grad, float* d_loss, void* hip_stream) {
  if (n <= 0 || !d_x || !d_t || !d_params || !d_grad) return MHD_E_ARG;
  if (n > MHD_MLP_NOALLOC_MAX) return MHD_E_WS;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return MHD_E_HIP;
  if (dev < 0 || dev >= kScratchDevices) return MHD_E_UNSUPPORTED;
  if (hip_stream) {
    hipDevice_t sdev = -1;
    if (hipStreamGetDevice((hipStream_t)hip_stream, &sdev) != hipSuccess) return MHD_E_HIP;
    if (sdev != dev) return MHD_E_ARG;
  }
  float* part = nullptr;
  const int rc = scratch_address(dev, &part);
  if (rc != MHD_OK) return rc;
  launch_mlp_grad(n, d_x, d_t, d_params, d_grad, d_loss, part, (hipStream_t)hip_stream);
  return hip_status();
}

int mhd_mlp_adam(float* d_params, float* d_m, float* d_v, const float* d_grad, int64_t step,
                 double lr, double beta1, double beta2, double eps, void* hip_stream) {
  if (!d_params || !d_m || !d_v || !d_grad || step < 1 || !(lr >= 0.0) || !(beta1 >= 0.0) ||
      !(beta1 < 1.0) || !(beta2 >= 0.0) || !(beta2 < 1.0) || !(eps > 0.0))
    return MHD_E_ARG;
  launch_mlp_adam(d_params, d_m, d_v, d_grad, step, lr, beta1, beta2, eps,
                  (hipStream_t)hip_stream);
  return hip_status();
}

int mhd_hlld_batch(int precision, int64_t n, const void* d_wl, const void* d_wr, const void* d_bn,
                   double gamma, void* d_flux, int8_t* d_code, void* hip_stream) {
  if (n < 0 || (n > 0 && (!d_wl || !d_wr || !d_bn || !d_flux)) || !(gamma > 1.0))
    return MHD_E_ARG;
  if (n > (1ll << 31) * 256ll) return MHD_E_ARG;
  if (precision != MHD_FP64 && precision != MHD_FP32) return MHD_E_ARG;
  if (n == 0) return MHD_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  if (precision == MHD_FP64)
    launch_hlld_batch<double>(n, (const double*)d_wl, (const double*)d_wr, (const double*)d_bn,
                              gamma, (double*)d_flux, d_code, st);
  else if (precision == MHD_FP32)
    launch_hlld_batch<float>(n, (const float*)d_wl, (const float*)d_wr, (const float*)d_bn,
                             (float)gamma, (float*)d_flux, d_code, st);
  else
    return MHD_E_ARG;
  return hip_status();
}

int mhd_recon_batch(int precision, int64_t n, const void* d_w4, int recon, double kappa,
                    void* d_wl, void* d_wr, void* hip_stream) {
  if (n < 0 || (n > 0 && (!d_w4 || !d_wl || !d_wr))) return MHD_E_ARG;
  if (recon < MHD_RECON_PAPER || recon > MHD_RECON_FIRST || !(kappa >= -1.0) || !(kappa < 1.0))
    return MHD_E_ARG;
  if (n > (1ll << 31) * 256ll) return MHD_E_ARG;
  if (precision != MHD_FP64 && precision != MHD_FP32) return MHD_E_ARG;
  if (n == 0) return MHD_OK;
  hipStream_t st = (hipStream_t)hip_stream;
  if (precision == MHD_FP64)
    launch_recon_batch<double>(n, (const double*)d_w4, muscl_of<double>(recon, kappa),
                               (double*)d_wl, (double*)d_wr, st);
  else if (precision == MHD_FP32)
    launch_recon_batch<float>(n, (const float*)d_w4, muscl_of<float>(recon, kappa),
                              (float*)d_wl, (float*)d_wr, st);
  else
    return MHD_E_ARG;
  return hip_status();
}

}  // extern "C"
