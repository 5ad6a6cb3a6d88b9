/*
 * mhd.h -- C ABI of the MI355X (gfx950) ideal-MHD TVD-MUSCL step library
 * (libmhd.so).
 *
 * The library advances the conservation law of ideal magneto-gas dynamics
 * (Khoperskov et al., "Numerical code for multi-component galaxies",
 * section 2.1):
 *     dU/dt + dF/dx + dG/dy + dH/dz = S,    U = [rho, rho v, E, B]   (Eq. 1-2)
 * with the fluxes of Eq. 3 (P* = P + B^2/2, E = P/(gamma-1) + rho v^2/2 + B^2/2,
 * rationalised units), cell-centred rho, rho v, E and face-centred B
 * (Eq. 4-5), the finite-volume update of Eq. 7 and the constrained-transport
 * induction update of Eq. 8-11, HLLD fluxes and the kappa-MUSCL/minmod
 * reconstruction of Eq. 12-14.  One step is a predictor-corrector pair that
 * yields the time-centred fluxes F^{n+1/2} of Eq. 7: first-order fluxes of U^n
 * advance U and B by dt/2, then MUSCL fluxes of that half-step state advance
 * U^n and B^n by dt.
 *
 * Memory layout of every state array handed across this ABI (device memory,
 * x fastest, interior cells only, element type double for MHD_FP64 and
 * MHD_FP32_COMP, float for MHD_FP32):
 *     cell5 : [5][nz][ny][nx]     rho, Mx, My, Mz, E
 *     bx    : [nz][ny][nx + ox]   face (i,j,k) at x0 + i dx
 *     by    : [nz][ny + oy][nx]
 *     bz    : [nz + oz][ny][nx]
 * with o = 0 on a periodic axis and 1 otherwise (the last face is then a
 * boundary face that the induction update also advances).
 *
 * Ownership: the caller owns every device buffer and the HIP stream; the
 * library owns only the host-side context (freed by mhd_destroy).  The library
 * never allocates device memory: all scratch lives in the caller's workspace
 * (size from mhd_workspace_bytes), except for mhd_mlp_grad_noalloc, whose
 * scratch is a static device array of the library.  Work is enqueued on the caller's stream;
 * only mhd_init, mhd_dt, mhd_diag, mhd_get_state and mhd_debug_array wait for
 * it.  A context is bound to one stream and is not thread-safe.
 *
 * Errors: every call returns MHD_OK (0) or a negative mhd_status.  No C++
 * exception crosses the ABI.  MHD_E_STATE is sticky: once a kernel has seen a
 * non-finite value, rho <= 0 or P <= 0 in an interior cell, mhd_step refuses
 * to run and mhd_dt / mhd_diag report it.
 */
#ifndef MHD_H
#define MHD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MHD_ABI_VERSION 1

typedef enum mhd_status {
  MHD_OK = 0,
  MHD_E_ARG = -1,          /* bad argument or configuration */
  MHD_E_HIP = -2,          /* a HIP runtime call failed */
  MHD_E_STATE = -3,        /* non-finite, rho <= 0 or P <= 0 seen (sticky) */
  MHD_E_UNSUPPORTED = -4,  /* valid but not implemented combination */
  MHD_E_WS = -5            /* workspace too small or misaligned */
} mhd_status;

/* Precision of a context.  MHD_FP32: FP32 bulk; pressure redone in FP64
   where it cancels (see recovery), FP64 time step and sums.  MHD_FP32_COMP:
   compensated FP32 -- the 5 cell values rho, M, E kept as pairs of FP32
   numbers (hi = the value rounded to FP32, lo = the rounding of the rest:
   about 48 significant bits), each stage's increment (FP32 fluxes and
   reconstruction, as in MHD_FP32) added to the pairs in FP64, every
   pressure, primitive, time step and sum computed from the pairs' FP64
   values; face B in FP32.  Its state arrays across this ABI are double (the
   pairs' exact values; mhd_init rounds the faces to FP32 and splits the
   cells into pairs, so a state copied out and back in is the same state);
   its other arrays (passive scalars, particles, mhd_debug_array) are float.
   The training entry points (mhd_flux_accumulate, mhd_coarsen,
   mhd_mlp_samples) return MHD_E_UNSUPPORTED for it; n_fp64_recovery stays
   0. */
enum { MHD_FP64 = 0, MHD_FP32 = 1, MHD_FP32_COMP = 2 };
enum { MHD_RECOVERY_FP64 = 0, MHD_RECOVERY_OFF = 1 };
enum { MHD_BC_PERIODIC = 0, MHD_BC_OUTFLOW = 1, MHD_BC_INFLOW = 2 };
enum { MHD_RECON_PAPER = 0, MHD_RECON_KAPPA = 1, MHD_RECON_FIRST = 2 };
enum {
  MHD_SRC_NONE = 0,
  MHD_SRC_LOGPOT = 1,   /* Phi = v0^2/2 ln(Rc^2 + x^2 + y^2 + z^2/q^2); src = v0, Rc, q */
  MHD_SRC_UNIFORM = 2,  /* grad Phi = (gx, gy, gz);                      src = gx, gy, gz */
  MHD_SRC_GAUSS_X = 3,  /* Phi = -A exp(-(x/w)^2);                        src = A, w */
  MHD_SRC_SELF_GRAVITY = 4 /* self-gravity, Lap Psi = 4 pi G (rho - <rho>) on a
                              periodic box (section 2.1, FFT solver): src = G.
                              Needs periodic boundaries and power-of-two
                              extents up to 1024; Psi comes from each stage's
                              density, S from its central gradient */
};

/* Status bits (mhd_diag_t.status). */
enum { MHD_ST_BAD_STATE = 1u };

/* Riemann solver of both stages (section 2.1: HLLD for magneto-gas
   dynamics; HLL and HLLC for pure gas dynamics).  HLL uses the outer wave
   speeds of HLLD and is valid with a field; HLLC is the gas-dynamic
   three-wave solver and takes the field to be zero (the magnetic flux
   components are zero): use it only for B = 0.  The learned correction
   (mhd_set_mlp) requires HLLD. */
enum { MHD_RIEMANN_HLLD = 0, MHD_RIEMANN_HLL = 1, MHD_RIEMANN_HLLC = 2 };

typedef struct mhd_config {
  int32_t nx, ny, nz;     /* interior cells, each >= 1; a padded array,
                             (nx+5)(ny+5)(nz+5) elements, must stay below
                             2^31 elements and 4 GiB */
  int32_t precision;      /* MHD_FP64, MHD_FP32 or MHD_FP32_COMP (see above) */
  int32_t bc[6];          /* -x, +x, -y, +y, -z, +z; periodic must be set on both sides */
  double x0, y0, z0;      /* lower corner of the domain */
  double dx, dy, dz;      /* cell sizes, > 0 */
  double gamma;           /* ratio of specific heats, > 1 */
  double cfl;             /* Courant number of the global time step, in (0, 1) */
  int32_t recon;          /* MHD_RECON_*: reconstruction of the corrector stage */
  int32_t source;         /* MHD_SRC_* */
  double kappa;           /* kappa of Eq. 12-14, in [-1, 1); 1/3 in the paper */
  double src[4];          /* parameters of the source model */
  double rho_floor;       /* 0 = off; else rho is raised to it after each update */
  double p_floor;         /* 0 = off; else E is raised so that P >= p_floor */
  double inflow[8];       /* ghost primitive state of MHD_BC_INFLOW sides:
                             rho, vx, vy, vz, P, Bx, By, Bz */
  int32_t riemann;        /* MHD_RIEMANN_*: HLLD (0, default), or the gas-dynamic HLL or HLLC */
  int32_t nscalar;        /* passive scalars, 0..MHD_MAX_SCALARS (see mhd_set_scalars) */
  int32_t recovery;       /* MHD_FP32: MHD_RECOVERY_FP64 (0, default) redoes the pressure
                             in FP64 in cells where E / (E - rho v^2/2 - B^2/2) > 64;
                             MHD_RECOVERY_OFF (1) keeps every pressure in FP32 (to
                             measure what the recovery gives).  Must be 0 in the other
                             precisions */
  int32_t reserved;       /* must be 0 */
  int64_t npart;          /* N-body particles, >= 0; > 0 needs MHD_SRC_SELF_GRAVITY (see
                             mhd_set_particles) */
} mhd_config;

/* Most passive scalars per context. */
#define MHD_MAX_SCALARS 8

typedef struct mhd_diag_t {
  double t;               /* simulated time */
  int64_t step;           /* completed steps */
  double dt;              /* CFL step of the current state */
  double mass;            /* sum over interior cells of rho dV (FP64) */
  double mom[3];          /* sum of rho v dV */
  double energy;          /* sum of E dV */
  double bsum[3];         /* sum over interior faces of B_d dV */
  double divb_max;        /* max over interior cells |div_h B| min(dx,dy,dz) / max|B_face| */
  double rho_min, p_min;  /* over interior cells */
  int64_t n_floor;        /* floor activations */
  int64_t n_hll_fallback; /* faces where HLLD fell back to HLL */
  int64_t n_degenerate;   /* faces with a degenerate HLLD star state */
  int64_t n_fp64_recovery;/* FP32 mode: cell evaluations whose pressure was redone in FP64 */
  int64_t n_mlp_faces;    /* corrector faces that received the learned correction */
  int64_t n_mlp_gated;    /* corrector faces kept plain because they touch a shock cell */
  uint32_t status;        /* MHD_ST_* bits */
  uint32_t pad;
} mhd_diag_t;

typedef struct mhd_ctx mhd_ctx;

/* ABI version (MHD_ABI_VERSION). */
int mhd_abi_version(void);

/* Static description of an mhd_status code; never NULL. */
const char *mhd_strerror(int code);

/* Device workspace bytes needed for cfg (padded state, half-step state,
   primitives, fluxes, edge EMFs, reduction scratch, passive scalars at the
   two time levels, particles).  Returns MHD_E_ARG for
   an invalid configuration. */
int mhd_workspace_bytes(const mhd_config *cfg, size_t *out);

/* Creates a context on the caller's stream (hip_stream: a hipStream_t, NULL =
   the null stream).  d_ws: device workspace of ws_bytes >= the value from
   mhd_workspace_bytes, 256-byte aligned; it must outlive the context.
   d_cell5, d_bx, d_by, d_bz: the initial state U at t = 0 in the layout of
   this header, copied into the workspace (the caller may free them after the
   call).  Fills the ghost zones, checks the state (MHD_E_STATE if any
   interior cell is non-finite or has rho <= 0 or P <= 0) and computes the
   first CFL dt.  Synchronises the stream. */
int mhd_init(const mhd_config *cfg, void *d_ws, size_t ws_bytes, const void *d_cell5,
             const void *d_bx, const void *d_by, const void *d_bz, void *hip_stream,
             mhd_ctx **out);

/* Advances nsteps >= 0 steps (Eq. 7-8 via the predictor-corrector pair).
   dt_host NULL: each step uses the CFL dt of its own initial state, computed
   and kept on the device (no host synchronisation).  Otherwise dt_host[s]
   (host memory, > 0) is the size of step s.  Asynchronous; returns
   MHD_E_STATE without enqueuing anything once the sticky state error is set
   (that is checked at the last synchronising call). */
int mhd_step(mhd_ctx *ctx, const double *dt_host, int nsteps);

/* CFL step dt = cfl min over interior cells and axes d of
   dx_d / (|v_d| + c_f,d) of the current state, in FP64.  Synchronises. */
int mhd_dt(mhd_ctx *ctx, double *out);

/* FP64 diagnostics of the current state (see mhd_diag_t).  Synchronises.
   Returns MHD_E_STATE (with *out filled) if the sticky status is set. */
int mhd_diag(mhd_ctx *ctx, mhd_diag_t *out);

/* Copies the interior state out, same layout and precision as mhd_init
   (a checkpoint: mhd_init on it resumes bit-for-bit).  Synchronises. */
int mhd_get_state(mhd_ctx *ctx, void *d_cell5, void *d_bx, void *d_by, void *d_bz);

/* Passive scalars (the multi-species advection of section 2.1): nscalar
   mass fractions X_s, each carried by the flow as the conserved density
   rho X_s with no source.  On every face the scalar flux is the mass flux
   F_rho of that face (the final one, after any learned correction) times X_s
   reconstructed like the other variables of the stage (first order in the
   predictor, the configured MUSCL in the corrector) on the side the mass
   comes from: F_rho X_L if F_rho > 0, F_rho X_R if F_rho < 0, 0 otherwise,
   with X = (rho X) / rho of the stage's primitives.  The floors leave rho X
   unchanged; inflow ghosts hold X = 0.  Sums of rho X over a periodic box
   are conserved to rounding, and a uniform X stays uniform.
   d_rho_x: device array [nscalar][nz][ny][nx] of the context precision
   (interior cells, x fastest).  mhd_init sets every scalar to zero;
   mhd_set_scalars replaces them (ghost zones refilled), mhd_get_scalars
   copies them out.  Both synchronise; MHD_E_ARG if the context has no
   scalars or the pointer is NULL. */
int mhd_set_scalars(mhd_ctx *ctx, const void *d_rho_x);
int mhd_get_scalars(mhd_ctx *ctx, void *d_rho_x);

/* N-body particles (section 2.1: particle-in-cell dynamics with the
   "flip-flop" integrator and a mass-conserving second-order mass
   assignment), moving in the periodic self-gravity potential together with
   the gas.  Mass assignment is cloud in cell: a particle is a cube of one
   cell's size, and each cell receives the particle's mass times the
   fraction of the cube inside it, divided by the cell volume.  The force is
   minus the cell-centred central gradient of Psi interpolated with the
   same weights (so the total momentum of gas and particles is kept).  The
   leapfrog of each step, with the gas stages: the predictor's potential
   uses the particles at x; the corrector's uses them at x_h = x + dt/2 v;
   then v += dt (-grad Psi)(x_h) and x = x_h + dt/2 v.  Positions wrap
   into the box.  With src[1] = 1 the gas is decoupled: it neither sources
   nor feels the potential (particles only).  The CFL step also obeys
   dt <= cfl min over particles and axes of d_a / |v_a|.  The deposit adds
   with atomics, so runs with particles are not bitwise reproducible.
   d_x, d_v: device arrays [3][npart] (rows x, y, z), d_m: [npart], of the
   context precision.  mhd_init sets every particle to rest at the box
   corner with zero mass; mhd_set_particles replaces them (positions
   wrapped), mhd_get_particles copies positions and velocities out (either
   pointer may be NULL).  Both synchronise; MHD_E_ARG if the context has no
   particles or a required pointer is NULL. */
int mhd_set_particles(mhd_ctx *ctx, const void *d_x, const void *d_v, const void *d_m);
int mhd_get_particles(mhd_ctx *ctx, void *d_x, void *d_v);

/* enable != 0: the steps from now on keep every component of every face's
   flux of each stage in the workspace, as mhd_mlp_samples and the flux
   entries of mhd_debug_array read them (the learned correction's sampling,
   checks); enable == 0 (the default): the fused flux sweep keeps only what
   the EMFs, passive scalars and tile seams need, and those entries read
   stale values.  Takes effect at the next mhd_step.  Steps with a learned
   correction or a flux accumulator keep every flux either way. */
int mhd_set_full_fluxes(mhd_ctx *ctx, int enable);

/* Copies one internal padded array of the last corrector stage to d_out
   (element type of the context precision, [nz+5][ny+5][nx+5], x fastest,
   interior cell (i,j,k) at ((k+2)(ny+5) + j+2)(nx+5) + i+2):
   what 0..6 x-face flux (rho, Mn, Mt1, Mt2, E, Bt1, Bt2 in the face frame
   (x,y,z)), 7..13 y-face flux (frame (y,z,x)), 14..20 z-face flux (frame
   (z,x,y)), 21..23 edge EMF Ex, Ey, Ez, 24..26 cell EMF, 27..34 primitives
   rho, vx, vy, vz, P, Bcx, Bcy, Bcz, and with self-gravity 35 Psi and
   36..38 its gradient at the cells.  *n_out gets the element count.  On a
   box periodic on all sides, steps without full fluxes, passive scalars,
   learned correction or flux accumulation leave the ghost layers of the
   cell arrays, the primitives' ghost shell and the fluxes outside the
   interior faces unrefreshed (their readers take the interior images):
   read the interior entries.  Synchronises. */
int mhd_debug_array(mhd_ctx *ctx, int what, void *d_out, size_t *n_out);

/* Kernel classes timed by the profiling hook. */
enum {
  MHD_K_GHOSTS = 0,
  MHD_K_PRIM = 1,     /* primitives; in a step that computes its own dt also the
                         CFL candidates of the start-of-step state and their
                         reduction to dt */
  MHD_K_FLUX = 2,     /* fluxes of all three face families, one launch: the fused
                         flux sweep with the stage's conservative update, or (with
                         a flux accumulator) the plain flux kernel */
  MHD_K_FLUX_MLP = 3, /* corrector flux sweeps with the learned correction,
                         one launch per axis */
  MHD_K_SHOCK = 4,    /* shock cells of the corrector state (learned runs) */
  MHD_K_EMF = 5,
  MHD_K_UPDATE = 6,
  MHD_K_CFL = 7,
  MHD_K_OTHER = 8,
  MHD_K_GRAVITY = 9,  /* self-gravity Poisson solve (FFTs, k-space division, gradient) */
  MHD_K_SCALARS = 10, /* passive-scalar face fluxes and update, and their ghost fill */
  MHD_K_NBODY = 11,   /* particle kick and drift (their deposit is part of MHD_K_GRAVITY) */
  MHD_K_FLUX_OUTER = 12, /* fluxes of the outer layer of the flux range after the fused
                            sweep (copied from periodic images or solved) */
  MHD_K_COUNT = 13
};

typedef struct mhd_profile_t {
  double ms[16];        /* summed device time per kernel class (MHD_K_*) */
  int64_t launches[16]; /* launches per class */
  int32_t n_kinds;      /* MHD_K_COUNT */
  int32_t pad;
} mhd_profile_t;

/* enable != 0: from now on every kernel mhd_step enqueues is bracketed by HIP
   events on the context's stream (host-side event objects only, no device
   memory); enable == 0 stops.  Enabling clears earlier records. */
int mhd_profile(mhd_ctx *ctx, int enable);

/* Sums the recorded event intervals per kernel class.  Synchronises. */
int mhd_profile_get(mhd_ctx *ctx, mhd_profile_t *out);

/* Releases the host context (not the caller's device memory). */
int mhd_destroy(mhd_ctx *ctx);

/* ---- learned flux correction (2x-coarsened runs) ------------------------
   A 32-64-64-8 MLP with GELU hidden layers (parameter vector of
   MHD_MLP_NPARAM FP32 values: W1[64][32], b1[64], W2[64][64], b2[64],
   W3[8][64], b3[8]; weights used in bfloat16, FP32 accumulation on the
   matrix cores) maps the 32 normalised primitives of a face's 4-cell stencil
   (rho, vn, vt1, vt2, P, Bn, Bt1, Bt2 per cell, divided by the two-cell face
   means: rho/rho_m, (v - v_m)/c_m, P/(rho_m c_m^2), B/(sqrt(rho_m) c_m)) to a
   correction of the face's corrector flux (scales rho_m c_m, rho_m c_m^2,
   rho_m c_m^3, sqrt(rho_m) c_m^2, Galilean shift by v_m; output 5, the normal
   B, unused).  It is added to the HLLD flux before constrained transport,
   except on faces touching a shock cell (a neighbour's pressure differs by
   more than `jump` times the cell's and div v < 0) or whose two-cell means of
   rho or P are not positive, and clipped per component to
   tau_flux |F| + tau a_max |U_R - U_L|. */
#define MHD_MLP_NPARAM 6792

typedef struct mhd_gate {
  double tau;       /* clip factor of the dissipation-scale term a_max |U_R - U_L|, >= 0 */
  double jump;      /* relative pressure jump marking a shock cell, > 0 */
  double tau_flux;  /* clip factor of the flux-scale term |F|, >= 0 */
} mhd_gate;

/* Enables the fused correction in the corrector sweeps (d_params: device
   FP32 [MHD_MLP_NPARAM], caller-owned, read at every step while enabled) or
   disables it (d_params NULL). */
int mhd_set_mlp(mhd_ctx *ctx, const float *d_params, const mhd_gate *gate);

/* While d_acc is non-NULL, every step adds dt times the mean corrector flux
   over the 2x2 fine faces tiling each face at the lower side of a cell of
   the 2x-coarsened grid: d_acc [3][7][nz/2][ny/2][nx/2] (context precision;
   components in the face frame rho, Mn, Mt1, Mt2, E, Bt1, Bt2; the last
   boundary face of a non-periodic axis is not accumulated).  The caller
   zeroes it.  Needs even extents and, per axis, both sides periodic or both
   not (else MHD_E_UNSUPPORTED). */
int mhd_flux_accumulate(mhd_ctx *ctx, void *d_acc);

/* Writes the 2x-coarsened state (2^3 volume means, 2^2 face means) in the
   interior layout of this header for the half-size grid with the same
   boundary kinds (n/2 + 1 faces along a non-periodic axis, the last one
   tiled by the fine boundary faces).  Same requirements as
   mhd_flux_accumulate.  Synchronises. */
int mhd_coarsen(mhd_ctx *ctx, void *d_cell5, void *d_bx, void *d_by, void *d_bz);

/* Training samples from the last step of a (coarse) context, which must
   have been taken with mhd_set_full_fluxes on (or with the learned
   correction or a flux accumulator active); MHD_E_ARG otherwise, also
   before the first step:
   for n faces d_faces [n][4] = (axis, i, j, k) with 0 <= i,j,k < n_axis,
   d_x [n][32] = features of the corrector state, d_t [n][8] = the MLP
   output that would turn its corrector flux into d_acc/dt_coarse (d_acc
   from mhd_flux_accumulate on the fine run over the same interval),
   d_mask [n] = 1 if the face touches a shock cell, 2 if the face index is
   invalid (then x, t are zero).  Asynchronous. */
int mhd_mlp_samples(mhd_ctx *ctx, const void *d_acc, double dt_coarse, int64_t n,
                    const int32_t *d_faces, float *d_x, float *d_t, uint8_t *d_mask);

/* y [n][8] = MLP(x [n][32]) with the parameters d_params.  Asynchronous. */
int mhd_mlp_forward(int64_t n, const float *d_x, const float *d_params, float *d_y,
                    void *hip_stream);

/* Scratch bytes for mhd_mlp_grad on n samples. */
int mhd_mlp_grad_workspace_bytes(int64_t n, size_t *out);

/* d_grad [MHD_MLP_NPARAM] = gradient of L = mean over samples and outputs
   of (MLP(x) - t)^2; *d_loss = L (device float).  Deterministic (fixed
   reduction order).  d_ws: scratch of mhd_mlp_grad_workspace_bytes(n).
   Asynchronous. */
int mhd_mlp_grad(int64_t n, const float *d_x, const float *d_t, const float *d_params,
                 float *d_grad, float *d_loss, void *d_ws, size_t ws_bytes, void *hip_stream);

/* Gradient without allocation.  For callers that cannot allocate device
   memory or hand over a workspace: code under HIP graph capture, tight
   training loops, harnesses that forbid hipMalloc.  Same result as
   mhd_mlp_grad (same kernels, same fixed reduction order: bitwise equal),
   with the per-block partial gradients in a static device array of the
   library instead of the caller's workspace; it calls no hipMalloc, hipFree
   or other allocating routine.  n: 1 .. MHD_MLP_NOALLOC_MAX samples
   (MHD_E_WS above it).  The array holds MHD_MLP_NOALLOC_MAX / 64 rows of
   MHD_MLP_NPARAM + 1 floats (13.9 MB); every GPU the library runs on keeps
   its own copy until the process ends.  All calls on one GPU share that
   copy, so calls that overlap on one GPU (two streams, two threads) race
   and must be serialised by the caller; each call writes every value it
   reads from the array before reading it, so nothing carries over between
   calls.  hip_stream must belong to the current device (MHD_E_ARG
   otherwise).  d_loss may be NULL.  Asynchronous. */
#define MHD_MLP_NOALLOC_MAX 32768
int mhd_mlp_grad_noalloc(int64_t n, const float *d_x, const float *d_t, const float *d_params,
                         float *d_grad, float *d_loss, void *hip_stream);

/* One Adam update (bias-corrected, step >= 1) of d_params with moments
   d_m, d_v (zero-initialised by the caller).  Asynchronous. */
int mhd_mlp_adam(float *d_params, float *d_m, float *d_v, const float *d_grad, int64_t step,
                 double lr, double beta1, double beta2, double eps, void *hip_stream);

/* ---- kernel-level entry points used by the parity tests ---------------- */

/* HLLD flux (Miyoshi & Kusano 2005, the solver section 2.1 names) of n
   faces in the face-normal frame on the device: d_wl, d_wr [n][7] =
   rho, vn, vt1, vt2, P, Bt1, Bt2; d_bn [n]; d_flux [n][7] = rho, Mn, Mt1,
   Mt2, E, Bt1, Bt2; d_code [n] (int8: bit0 HLL fallback, bit1 degenerate
   star state; may be NULL).  precision selects double or float arrays.
   Asynchronous on hip_stream. */
int mhd_hlld_batch(int precision, int64_t n, const void *d_wl, const void *d_wr,
                   const void *d_bn, double gamma, void *d_flux, int8_t *d_code,
                   void *hip_stream);

/* Eq. 12-14 interface values of n 4-cell stencils d_w4 [n][4] (face between
   cells 1 and 2) into d_wl, d_wr [n].  Asynchronous on hip_stream. */
int mhd_recon_batch(int precision, int64_t n, const void *d_w4, int recon, double kappa,
                    void *d_wl, void *d_wr, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
