/*
 * orc.c -- plain, slow, FP64 CPU oracle for one explicit TVD-MUSCL ideal-MHD
 * step with constrained transport.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  It shares no
 * source with the GPU library.  Every loop is a plain scalar triple loop over
 * a padded grid; the only parallelism is an OpenMP split over z-planes.
 *
 * Paper: Khoperskov, Vasiliev, Khoperskov, Lubimov, "Numerical code for
 * multi-component galaxies: from N-body to chemistry and magnetic fields",
 * section 2.1 (gas dynamics).  Readings used where the paper is silent or
 * misprinted (each restated where it is implemented):
 *   R1  time integrator: predictor-corrector reaching t^{n+1/2}: first-order
 *       half step, then a MUSCL full step from U^n (the paper only names
 *       fluxes at n+1/2 in Eq. 7).
 *   R2  Eq. 13-14 are used as printed (K2 on minmod(dw_{i-1},dw_i), K1 on
 *       minmod(dw_i, b dw_{i-1})); the textbook kappa-scheme is a flag.
 *   R3  Eq. 10: the derivative correction is (3/4-point) minus (1/4-point);
 *       the printed order fails the one-dimensional reduction.
 *   R4  Eq. 10 uses the four faces that touch the edge.
 *   R5  Eq. 8: the second bracket is E_y (the curl), not E_z.
 *   R6  Eq. 11 upwinds by the sign of the Riemann mass flux at the face.
 *   R7  only the two transverse B components are reconstructed; the normal
 *       one is the face value.
 *   R8  HLLD: Miyoshi & Kusano wave-speed estimate; star states whose
 *       denominator rho (S-u)(S-S_M) - Bn^2 is within 1e-3 p_T* of zero (the
 *       outer fast-speed estimate meets the star Alfven speed) keep their
 *       transverse v and B; HLL flux if S_M is not strictly inside (S_L, S_R).
 *       The star formulas carry v*.B* ~ 1/den^2, so the energy flux of the
 *       regular branch grows like 1/den near the degenerate case: with a
 *       threshold of 1e-8 p_T* it is off by up to 100x for |den| ~ 1e-8..1e-6
 *       p_T*; at 1e-3 p_T* the switch moves the flux by about 0.1 %.
 *   R9  CFL: dt = C min_cells min_d dx_d / (|v_d| + c_f,d) at step start.
 *   R10 source S = (0, -rho grad Phi, -rho v.grad Phi, 0) at cell centres,
 *       dt/2 S(W^n) in the predictor, dt S(W*) in the corrector.
 */
#include "orc.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NG 2
#ifndef DEG_EPS
#define DEG_EPS 1.0e-3
#endif

#define M_PI_ORC 3.14159265358979323846

struct orc_grid {
  orc_config c;
  int n[3];
  int ext[3];
  long st[3];     /* strides of the padded layout */
  long np;        /* points per padded array */
  double d[3];
  int per[3];
  double *u[5], *b[3];    /* state at t^n */
  double *us[5], *bs[3];  /* predictor state at t^{n+1/2} */
  double *w[8];           /* primitives rho, vx, vy, vz, P, Bcx, Bcy, Bcz */
  double *ec[3];          /* cell-centred EMF */
  double *fl[3][8];       /* face fluxes per axis, global components */
  signed char *sg[3];     /* sign of the mass flux per face */
  double *e[3];           /* edge EMFs */
  double t;
  int64_t step;
  int64_t n_floor, n_hll, n_deg;
  /* learned correction of the corrector fluxes */
  double *mlp;            /* NULL = off; else ORC_MLP_NPARAM values */
  double mlp_tau, mlp_jump, mlp_tau_flux;
  unsigned char *shock;   /* per cell: 1 = shock cell (no correction on its faces) */
  int64_t n_mlp, n_gated;
  /* self-gravity: potential and its central gradient at the cells (padded) */
  double *psi, *gpsi[3];
  /* particles: positions, velocities ([3][npart]), masses; half-step
     positions of the current step */
  double *xp, *vp, *mp, *xh;
  /* passive scalars: rho X at t^n and t^{n+1/2}, X of the stage, fluxes */
  double *xs[ORC_MAX_SCALAR], *xss[ORC_MAX_SCALAR], *xw[ORC_MAX_SCALAR];
  double *xf[3][ORC_MAX_SCALAR];
};

static long at(const orc_grid *g, int i, int j, int k) {
  return (long)(i + NG) + g->st[1] * (long)(j + NG) + g->st[2] * (long)(k + NG);
}

int orc_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Single-face physics in the face-normal frame (n, t1, t2).               */
/* A frame state is w = rho, vn, vt1, vt2, P, Bt1, Bt2 plus the normal Bn. */
/* ------------------------------------------------------------------------ */

/* Eq. 3 conserved vector: E = P/(gamma-1) + rho v^2/2 + B^2/2. */
void orc_prim_to_cons(const double w[7], double bn, double gam, double u[7]) {
  double v2 = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
  double b2 = bn * bn + w[5] * w[5] + w[6] * w[6];
  u[0] = w[0];
  u[1] = w[0] * w[1];
  u[2] = w[0] * w[2];
  u[3] = w[0] * w[3];
  u[4] = w[4] / (gam - 1.0) + 0.5 * w[0] * v2 + 0.5 * b2;
  u[5] = w[5];
  u[6] = w[6];
}

/* Eq. 3 physical flux F along the normal, P* = P + B^2/2. */
void orc_phys_flux(const double w[7], double bn, double gam, double f[7]) {
  double u[7];
  orc_prim_to_cons(w, bn, gam, u);
  double b2 = bn * bn + w[5] * w[5] + w[6] * w[6];
  double pt = w[4] + 0.5 * b2;
  double vb = w[1] * bn + w[2] * w[5] + w[3] * w[6];
  f[0] = w[0] * w[1];
  f[1] = w[0] * w[1] * w[1] + pt - bn * bn;
  f[2] = w[0] * w[1] * w[2] - bn * w[5];
  f[3] = w[0] * w[1] * w[3] - bn * w[6];
  f[4] = (u[4] + pt) * w[1] - vb * bn;
  f[5] = w[5] * w[1] - bn * w[2];
  f[6] = w[6] * w[1] - bn * w[3];
}

/* Fast magnetosonic speed along the normal.  The textbook discriminant
   (a^2+b^2)^2 - 4 a^2 bn^2 is rewritten as (a^2-b^2)^2 + 4 a^2 bt^2, a sum of
   non-negative terms. */
double orc_fast_speed(const double w[7], double bn, double gam) {
  double a2 = gam * w[4] / w[0];
  double bt2 = (w[5] * w[5] + w[6] * w[6]) / w[0];
  double b2 = (bn * bn + w[5] * w[5] + w[6] * w[6]) / w[0];
  double dd = a2 - b2;
  double cf2 = 0.5 * ((a2 + b2) + sqrt(dd * dd + 4.0 * a2 * bt2));
  return sqrt(cf2);
}

/* One side of the HLLD star region (Miyoshi & Kusano 2005, section 3).
   S is the outer wave speed of this side, SM the contact speed, pts the star
   total pressure.  Outputs the star conserved vector and v*.B*. */
static int hlld_star(const double w[7], const double u[7], double bn,
                     double S, double SM, double pts, double us[7],
                     double *vbs, double *dens) {
  double rho = w[0], vn = w[1], vt1 = w[2], vt2 = w[3];
  double bt1 = w[5], bt2 = w[6];
  double pt = w[4] + 0.5 * (bn * bn + bt1 * bt1 + bt2 * bt2);
  double ds = rho * (S - vn) / (S - SM);
  double den = rho * (S - vn) * (S - SM) - bn * bn;
  double vs1, vs2, bs1, bs2;
  int degenerate = 0;
  if (fabs(den) > DEG_EPS * pts) {
    vs1 = vt1 - bn * bt1 * (SM - vn) / den;
    vs2 = vt2 - bn * bt2 * (SM - vn) / den;
    bs1 = bt1 * (rho * (S - vn) * (S - vn) - bn * bn) / den;
    bs2 = bt2 * (rho * (S - vn) * (S - vn) - bn * bn) / den;
  } else {
    /* S*_alpha -> S_alpha: the transverse field and velocity do not jump. */
    vs1 = vt1;
    vs2 = vt2;
    bs1 = bt1;
    bs2 = bt2;
    degenerate = 1;
  }
  double vb = vn * bn + vt1 * bt1 + vt2 * bt2;
  double vbstar = SM * bn + vs1 * bs1 + vs2 * bs2;
  double es = ((S - vn) * u[4] - pt * vn + pts * SM + bn * (vb - vbstar)) / (S - SM);
  us[0] = ds;
  us[1] = ds * SM;
  us[2] = ds * vs1;
  us[3] = ds * vs2;
  us[4] = es;
  us[5] = bs1;
  us[6] = bs2;
  *vbs = vbstar;
  *dens = ds;
  return degenerate;
}

int orc_hlld(const double wl[7], const double wr[7], double bn, double gam,
             double flux[7]) {
  double ul[7], ur[7], fl[7], fr[7];
  orc_prim_to_cons(wl, bn, gam, ul);
  orc_prim_to_cons(wr, bn, gam, ur);
  orc_phys_flux(wl, bn, gam, fl);
  orc_phys_flux(wr, bn, gam, fr);

  /* Outer wave speeds: min/max of the normal velocities -/+ the larger fast
     speed. */
  double cfl = orc_fast_speed(wl, bn, gam);
  double cfr = orc_fast_speed(wr, bn, gam);
  double cmax = cfl > cfr ? cfl : cfr;
  double SL = (wl[1] < wr[1] ? wl[1] : wr[1]) - cmax;
  double SR = (wl[1] > wr[1] ? wl[1] : wr[1]) + cmax;
  int m;
  if (SL > 0.0) {
    for (m = 0; m < 7; ++m) flux[m] = fl[m];
    return 0;
  }
  if (SR < 0.0) {
    for (m = 0; m < 7; ++m) flux[m] = fr[m];
    return 0;
  }

  /* Contact speed and star total pressure. */
  double ptl = wl[4] + 0.5 * (bn * bn + wl[5] * wl[5] + wl[6] * wl[6]);
  double ptr = wr[4] + 0.5 * (bn * bn + wr[5] * wr[5] + wr[6] * wr[6]);
  double al = wl[0] * (SL - wl[1]);
  double ar = wr[0] * (SR - wr[1]);
  double SM = (ar * wr[1] - al * wl[1] - ptr + ptl) / (ar - al);
  double pts = (ar * ptl - al * ptr + al * ar * (wr[1] - wl[1])) / (ar - al);

  if (!(SL < SM && SM < SR)) {
    /* HLL flux: two-wave average between SL and SR. */
    for (m = 0; m < 7; ++m)
      flux[m] = (SR * fl[m] - SL * fr[m] + SL * SR * (ur[m] - ul[m])) / (SR - SL);
    return 1;
  }

  double usl[7], usr[7], vbsl, vbsr, dsl, dsr;
  int deg = hlld_star(wl, ul, bn, SL, SM, pts, usl, &vbsl, &dsl);
  deg |= hlld_star(wr, ur, bn, SR, SM, pts, usr, &vbsr, &dsr);

  /* Double-star states across the rotational discontinuities. */
  double sl = sqrt(dsl), sr = sqrt(dsr);
  double SsL = SM - fabs(bn) / sl;
  double SsR = SM + fabs(bn) / sr;
  double sgn = bn > 0.0 ? 1.0 : (bn < 0.0 ? -1.0 : 0.0);
  double vl1 = usl[2] / dsl, vl2 = usl[3] / dsl;
  double vr1 = usr[2] / dsr, vr2 = usr[3] / dsr;
  double vss1 = (sl * vl1 + sr * vr1 + sgn * (usr[5] - usl[5])) / (sl + sr);
  double vss2 = (sl * vl2 + sr * vr2 + sgn * (usr[6] - usl[6])) / (sl + sr);
  double bss1 = (sr * usl[5] + sl * usr[5] + sgn * sl * sr * (vr1 - vl1)) / (sl + sr);
  double bss2 = (sr * usl[6] + sl * usr[6] + sgn * sl * sr * (vr2 - vl2)) / (sl + sr);
  double vbss = SM * bn + vss1 * bss1 + vss2 * bss2;

  double fs[7];
  if (SsL >= 0.0) {
    /* F*_L = F_L + S_L (U*_L - U_L) */
    for (m = 0; m < 7; ++m) flux[m] = fl[m] + SL * (usl[m] - ul[m]);
  } else if (SM >= 0.0) {
    /* F**_L = F*_L + S*_L (U**_L - U*_L) */
    double uss[7] = {dsl, dsl * SM, dsl * vss1, dsl * vss2,
                     usl[4] - sl * sgn * (vbsl - vbss), bss1, bss2};
    for (m = 0; m < 7; ++m) fs[m] = fl[m] + SL * (usl[m] - ul[m]);
    for (m = 0; m < 7; ++m) flux[m] = fs[m] + SsL * (uss[m] - usl[m]);
  } else if (SsR >= 0.0) {
    double uss[7] = {dsr, dsr * SM, dsr * vss1, dsr * vss2,
                     usr[4] + sr * sgn * (vbsr - vbss), bss1, bss2};
    for (m = 0; m < 7; ++m) fs[m] = fr[m] + SR * (usr[m] - ur[m]);
    for (m = 0; m < 7; ++m) flux[m] = fs[m] + SsR * (uss[m] - usr[m]);
  } else {
    for (m = 0; m < 7; ++m) flux[m] = fr[m] + SR * (usr[m] - ur[m]);
  }
  return deg ? 2 : 0;
}

/* HLL (Harten, Lax & van Leer): one intermediate state between the outer
   waves, with the outer speeds of orc_hlld. */
int orc_hll(const double wl[7], const double wr[7], double bn, double gam,
            double flux[7]) {
  double ul[7], ur[7], fl[7], fr[7];
  int m;
  orc_prim_to_cons(wl, bn, gam, ul);
  orc_prim_to_cons(wr, bn, gam, ur);
  orc_phys_flux(wl, bn, gam, fl);
  orc_phys_flux(wr, bn, gam, fr);
  double cfl = orc_fast_speed(wl, bn, gam);
  double cfr = orc_fast_speed(wr, bn, gam);
  double cmax = cfl > cfr ? cfl : cfr;
  double SL = (wl[1] < wr[1] ? wl[1] : wr[1]) - cmax;
  double SR = (wl[1] > wr[1] ? wl[1] : wr[1]) + cmax;
  if (SL > 0.0) {
    for (m = 0; m < 7; ++m) flux[m] = fl[m];
  } else if (SR < 0.0) {
    for (m = 0; m < 7; ++m) flux[m] = fr[m];
  } else {
    for (m = 0; m < 7; ++m)
      flux[m] = (SR * fl[m] - SL * fr[m] + SL * SR * (ur[m] - ul[m])) / (SR - SL);
  }
  return 0;
}

/* HLLC (Toro, Spruce & Speares) for gas dynamics: the HLL fan split at the
   contact S* into two star states of equal pressure and normal velocity. */
int orc_hllc(const double wl[7], const double wr[7], double bn, double gam,
             double flux[7]) {
  double gl[7], gr[7], ul[7], ur[7], fl[7], fr[7];
  int m;
  (void)bn;
  for (m = 0; m < 7; ++m) {
    gl[m] = m < 5 ? wl[m] : 0.0;
    gr[m] = m < 5 ? wr[m] : 0.0;
  }
  orc_prim_to_cons(gl, 0.0, gam, ul);
  orc_prim_to_cons(gr, 0.0, gam, ur);
  orc_phys_flux(gl, 0.0, gam, fl);
  orc_phys_flux(gr, 0.0, gam, fr);
  double cl = sqrt(gam * gl[4] / gl[0]), cr = sqrt(gam * gr[4] / gr[0]);
  double cmax = cl > cr ? cl : cr;
  double SL = (gl[1] < gr[1] ? gl[1] : gr[1]) - cmax;
  double SR = (gl[1] > gr[1] ? gl[1] : gr[1]) + cmax;
  if (SL > 0.0) {
    for (m = 0; m < 7; ++m) flux[m] = fl[m];
    return 0;
  }
  if (SR < 0.0) {
    for (m = 0; m < 7; ++m) flux[m] = fr[m];
    return 0;
  }
  double ml = gl[0] * (SL - gl[1]), mr = gr[0] * (SR - gr[1]);
  double Ss = (gr[4] - gl[4] + ml * gl[1] - mr * gr[1]) / (ml - mr);
  const double *w = Ss >= 0.0 ? gl : gr;
  const double *u = Ss >= 0.0 ? ul : ur;
  const double *f = Ss >= 0.0 ? fl : fr;
  double S = Ss >= 0.0 ? SL : SR;
  double fac = w[0] * (S - w[1]) / (S - Ss);
  double us[7];
  us[0] = fac;
  us[1] = fac * Ss;
  us[2] = fac * w[2];
  us[3] = fac * w[3];
  us[4] = fac * (u[4] / w[0] + (Ss - w[1]) * (Ss + w[4] / (w[0] * (S - w[1]))));
  us[5] = 0.0;
  us[6] = 0.0;
  for (m = 0; m < 7; ++m) flux[m] = f[m] + S * (us[m] - u[m]);
  return 0;
}

/* minmod limiter: the argument of smaller magnitude when both have the same
   strict sign, else 0.  The sign test is by comparison, never by a*b. */
double orc_minmod(double a, double b) {
  if (a > 0.0 && b > 0.0) return a <= b ? a : b;
  if (a < 0.0 && b < 0.0) return a >= b ? a : b;
  return 0.0;
}

/* Eq. 12-14.  The paper's form is dW_i = K2 mm(dw_{i-1}, dw_i)
   + K1 mm(dw_i, b dw_{i-1}); the textbook kappa-scheme is
   dW_i = K1 mm(dw_{i-1}, b dw_i) + K2 mm(dw_i, b dw_{i-1}).  Both are
   cA mm(dw_{i-1}, bA dw_i) + cB mm(dw_i, bB dw_{i-1}). */
static void recon_coef(int recon, double kappa, double *cA, double *bA,
                       double *cB, double *bB) {
  double K1 = (1.0 - kappa) / 4.0;
  double K2 = (1.0 + kappa) / 4.0;
  double b = (3.0 - kappa) / (1.0 - kappa);
  if (recon == ORC_RECON_KAPPA) {
    *cA = K1; *bA = b; *cB = K2; *bB = b;
  } else {
    *cA = K2; *bA = 1.0; *cB = K1; *bB = b;
  }
}

void orc_recon(const double w[4], int recon, double kappa, double *wl,
               double *wr) {
  if (recon == ORC_RECON_FIRST) {
    *wl = w[1];
    *wr = w[2];
    return;
  }
  double cA, bA, cB, bB;
  recon_coef(recon, kappa, &cA, &bA, &cB, &bB);
  double dm = w[1] - w[0]; /* dw_{i-1} */
  double d0 = w[2] - w[1]; /* dw_i     */
  double dp = w[3] - w[2]; /* dw_{i+1} */
  double dWi = cA * orc_minmod(dm, bA * d0) + cB * orc_minmod(d0, bB * dm);
  double dWi1 = cA * orc_minmod(dp, bA * d0) + cB * orc_minmod(d0, bB * dp);
  *wl = w[1] + dWi;
  *wr = w[2] - dWi1;
}

/* ------------------------------------------------------------------------ */
/* Learned flux correction: 32-64-64-8 MLP, GELU hidden layers.             */
/* ------------------------------------------------------------------------ */

double orc_bf16(double x) {
  float f = (float)x;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf / nan */
  u += 0x7fffu + ((u >> 16) & 1u);                         /* ties to even */
  u &= 0xffff0000u;
  memcpy(&f, &u, 4);
  return (double)f;
}

static double gelu(double x) { return 0.5 * x * (1.0 + erf(x / sqrt(2.0))); }
static double gelu_d(double x) {
  return 0.5 * (1.0 + erf(x / sqrt(2.0))) + x * exp(-0.5 * x * x) / sqrt(2.0 * 3.14159265358979323846);
}

/* parameter offsets */
#define P_W1 0
#define P_B1 (P_W1 + 64 * 32)
#define P_W2 (P_B1 + 64)
#define P_B2 (P_W2 + 64 * 64)
#define P_W3 (P_B2 + 64)
#define P_B3 (P_W3 + 8 * 64)

static double rnd(int bf16, double v) { return bf16 ? orc_bf16(v) : v; }

/* One sample: activations a1, h1, a2, h2 (h rounded when bf16) and y. */
static void mlp_one(const double *P, int bf16, const double *x, double *a1, double *h1,
                    double *a2, double *h2, double *y) {
  double xr[32];
  int i, j;
  for (j = 0; j < 32; ++j) xr[j] = rnd(bf16, x[j]);
  for (i = 0; i < 64; ++i) {
    double acc = P[P_B1 + i];
    for (j = 0; j < 32; ++j) acc += rnd(bf16, P[P_W1 + i * 32 + j]) * xr[j];
    a1[i] = acc;
    h1[i] = rnd(bf16, gelu(acc));
  }
  for (i = 0; i < 64; ++i) {
    double acc = P[P_B2 + i];
    for (j = 0; j < 64; ++j) acc += rnd(bf16, P[P_W2 + i * 64 + j]) * h1[j];
    a2[i] = acc;
    h2[i] = rnd(bf16, gelu(acc));
  }
  for (i = 0; i < 8; ++i) {
    double acc = P[P_B3 + i];
    for (j = 0; j < 64; ++j) acc += rnd(bf16, P[P_W3 + i * 64 + j]) * h2[j];
    y[i] = acc;
  }
}

void orc_mlp_forward(const double *params, int bf16, long n, const double *x, double *y) {
  long b;
#pragma omp parallel for schedule(static)
  for (b = 0; b < n; ++b) {
    double a1[64], h1[64], a2[64], h2[64];
    mlp_one(params, bf16, x + 32 * b, a1, h1, a2, h2, y + 8 * b);
  }
}

void orc_mlp_backward(const double *params, int bf16, long n, const double *x,
                      const double *dy, double *grad) {
  const double *P = params;
  long b;
  int i, j;
  memset(grad, 0, sizeof(double) * ORC_MLP_NPARAM);
  for (b = 0; b < n; ++b) {
    double a1[64], h1[64], a2[64], h2[64], y[8], xr[32];
    double dz3[8], dh2[64], dz2[64], dh1[64], dz1[64];
    mlp_one(P, bf16, x + 32 * b, a1, h1, a2, h2, y);
    for (j = 0; j < 32; ++j) xr[j] = rnd(bf16, x[32 * b + j]);
    /* output layer: y = W3 h2 + b3 */
    for (i = 0; i < 8; ++i) {
      grad[P_B3 + i] += dy[8 * b + i];
      dz3[i] = rnd(bf16, dy[8 * b + i]);
      for (j = 0; j < 64; ++j) grad[P_W3 + i * 64 + j] += dz3[i] * h2[j];
    }
    for (j = 0; j < 64; ++j) {
      double acc = 0.0;
      for (i = 0; i < 8; ++i) acc += rnd(bf16, P[P_W3 + i * 64 + j]) * dz3[i];
      dh2[j] = acc;
    }
    /* second hidden layer */
    for (i = 0; i < 64; ++i) {
      double dz = dh2[i] * gelu_d(a2[i]);
      grad[P_B2 + i] += dz;
      dz2[i] = rnd(bf16, dz);
      for (j = 0; j < 64; ++j) grad[P_W2 + i * 64 + j] += dz2[i] * h1[j];
    }
    for (j = 0; j < 64; ++j) {
      double acc = 0.0;
      for (i = 0; i < 64; ++i) acc += rnd(bf16, P[P_W2 + i * 64 + j]) * dz2[i];
      dh1[j] = acc;
    }
    /* first hidden layer */
    for (i = 0; i < 64; ++i) {
      double dz = dh1[i] * gelu_d(a1[i]);
      grad[P_B1 + i] += dz;
      dz1[i] = rnd(bf16, dz);
      for (j = 0; j < 32; ++j) grad[P_W1 + i * 32 + j] += dz1[i] * xr[j];
    }
  }
}

/* Face means of cells 1 and 2 of the stencil: rho_m, v_m[3], c_m. */
static void face_means(const double w8[32], double gamma, double *rm, double vm[3], double *cm) {
  const double *c1 = w8 + 8, *c2 = w8 + 16;
  int d;
  *rm = 0.5 * (c1[0] + c2[0]);
  for (d = 0; d < 3; ++d) vm[d] = 0.5 * (c1[1 + d] + c2[1 + d]);
  *cm = sqrt(gamma * 0.5 * (c1[4] + c2[4]) / *rm);
}

void orc_mlp_features(const double w8[32], double gamma, double x[32]) {
  double rm, vm[3], cm;
  int c, d;
  face_means(w8, gamma, &rm, vm, &cm);
  for (c = 0; c < 4; ++c) {
    const double *w = w8 + 8 * c;
    double *o = x + 8 * c;
    o[0] = w[0] / rm;
    for (d = 0; d < 3; ++d) o[1 + d] = (w[1 + d] - vm[d]) / cm;
    o[4] = w[4] / (rm * cm * cm);
    for (d = 0; d < 3; ++d) o[5 + d] = w[5 + d] / (sqrt(rm) * cm);
  }
}

void orc_mlp_out_to_flux(const double w8[32], double gamma, const double y[8], double df[7]) {
  double rm, vm[3], cm;
  int d;
  face_means(w8, gamma, &rm, vm, &cm);
  double fr = rm * cm * y[0];              /* mass flux correction */
  double fm[3];                            /* momentum, mean-flow frame */
  for (d = 0; d < 3; ++d) fm[d] = rm * cm * cm * y[1 + d];
  double fe = rm * cm * cm * cm * y[4];    /* energy, mean-flow frame */
  double v2 = vm[0] * vm[0] + vm[1] * vm[1] + vm[2] * vm[2];
  df[0] = fr;
  for (d = 0; d < 3; ++d) df[1 + d] = fm[d] + vm[d] * fr;
  df[4] = fe + (vm[0] * fm[0] + vm[1] * fm[1] + vm[2] * fm[2]) + 0.5 * v2 * fr;
  df[5] = sqrt(rm) * cm * cm * y[6];
  df[6] = sqrt(rm) * cm * cm * y[7];
}

void orc_mlp_flux_to_out(const double w8[32], double gamma, const double df[7], double y[8]) {
  double rm, vm[3], cm;
  int d;
  face_means(w8, gamma, &rm, vm, &cm);
  double fr = df[0];
  double fm[3];
  for (d = 0; d < 3; ++d) fm[d] = df[1 + d] - vm[d] * fr;
  double v2 = vm[0] * vm[0] + vm[1] * vm[1] + vm[2] * vm[2];
  double fe = df[4] - (vm[0] * fm[0] + vm[1] * fm[1] + vm[2] * fm[2]) - 0.5 * v2 * fr;
  y[0] = fr / (rm * cm);
  for (d = 0; d < 3; ++d) y[1 + d] = fm[d] / (rm * cm * cm);
  y[4] = fe / (rm * cm * cm * cm);
  y[5] = 0.0;
  y[6] = df[5] / (sqrt(rm) * cm * cm);
  y[7] = df[6] / (sqrt(rm) * cm * cm);
}

void orc_hlld_batch(long n, const double *wl, const double *wr, const double *bn,
                    double gamma, double *flux, int32_t *code) {
  long t;
#pragma omp parallel for schedule(static)
  for (t = 0; t < n; ++t) {
    int c = orc_hlld(wl + 7 * t, wr + 7 * t, bn[t], gamma, flux + 7 * t);
    if (code) code[t] = c;
  }
}

void orc_recon_batch(long n, const double *w4, int recon, double kappa, double *wl,
                     double *wr) {
  long t;
#pragma omp parallel for schedule(static)
  for (t = 0; t < n; ++t) orc_recon(w4 + 4 * t, recon, kappa, wl + t, wr + t);
}

/* ------------------------------------------------------------------------ */
/* Grid set-up                                                              */
/* ------------------------------------------------------------------------ */

static double *alloc_arr(long n) { return (double *)calloc((size_t)n, sizeof(double)); }

void orc_destroy(orc_grid *g);

orc_grid *orc_create(const orc_config *cfg) {
  orc_grid *g = (orc_grid *)calloc(1, sizeof(orc_grid));
  int a, m;
  if (!g) return NULL;
  g->c = *cfg;
  if (cfg->riemann < ORC_RIEMANN_HLLD || cfg->riemann > ORC_RIEMANN_HLLC) { free(g); return NULL; }
  g->n[0] = cfg->nx; g->n[1] = cfg->ny; g->n[2] = cfg->nz;
  g->d[0] = cfg->dx; g->d[1] = cfg->dy; g->d[2] = cfg->dz;
  for (a = 0; a < 3; ++a) {
    if (g->n[a] < 1) { free(g); return NULL; }
    g->ext[a] = g->n[a] + 2 * NG + 1;
    g->per[a] = cfg->bc[2 * a] == ORC_BC_PERIODIC;
    if ((cfg->bc[2 * a] == ORC_BC_PERIODIC) != (cfg->bc[2 * a + 1] == ORC_BC_PERIODIC)) {
      free(g);
      return NULL;
    }
  }
  g->st[0] = 1;
  g->st[1] = g->ext[0];
  g->st[2] = (long)g->ext[0] * g->ext[1];
  g->np = g->st[2] * g->ext[2];
  for (m = 0; m < 5; ++m) { g->u[m] = alloc_arr(g->np); g->us[m] = alloc_arr(g->np); }
  for (a = 0; a < 3; ++a) {
    g->b[a] = alloc_arr(g->np); g->bs[a] = alloc_arr(g->np);
    g->ec[a] = alloc_arr(g->np); g->e[a] = alloc_arr(g->np);
    g->sg[a] = (signed char *)calloc((size_t)g->np, 1);
    for (m = 0; m < 8; ++m) g->fl[a][m] = alloc_arr(g->np);
  }
  for (m = 0; m < 8; ++m) g->w[m] = alloc_arr(g->np);
  g->shock = (unsigned char *)calloc((size_t)g->np, 1);
  if (cfg->nscalar < 0 || cfg->nscalar > ORC_MAX_SCALAR) { orc_destroy(g); return NULL; }
  if (cfg->npart < 0 || (cfg->npart > 0 && cfg->source != ORC_SRC_SELF_GRAVITY)) {
    orc_destroy(g);
    return NULL;
  }
  if (cfg->npart > 0) {
    g->xp = alloc_arr(3 * cfg->npart);
    g->vp = alloc_arr(3 * cfg->npart);
    g->mp = alloc_arr(cfg->npart);
    g->xh = alloc_arr(3 * cfg->npart);
  }
  for (m = 0; m < cfg->nscalar; ++m) {
    g->xs[m] = alloc_arr(g->np);
    g->xss[m] = alloc_arr(g->np);
    g->xw[m] = alloc_arr(g->np);
    for (a = 0; a < 3; ++a) g->xf[a][m] = alloc_arr(g->np);
  }
  if (cfg->source == ORC_SRC_SELF_GRAVITY) {
    /* the potential of a periodic box only */
    for (a = 0; a < 3; ++a)
      if (!g->per[a]) { orc_destroy(g); return NULL; }
    g->psi = alloc_arr(g->np);
    for (a = 0; a < 3; ++a) g->gpsi[a] = alloc_arr(g->np);
  }
  return g;
}

int orc_set_mlp(orc_grid *g, const double *params, double tau, double jump, double tau_flux) {
  free(g->mlp);
  g->mlp = NULL;
  if (!params) return 0;
  g->mlp = (double *)malloc(sizeof(double) * ORC_MLP_NPARAM);
  memcpy(g->mlp, params, sizeof(double) * ORC_MLP_NPARAM);
  g->mlp_tau = tau;
  g->mlp_jump = jump;
  g->mlp_tau_flux = tau_flux;
  return 0;
}

void orc_destroy(orc_grid *g) {
  int a, m;
  if (!g) return;
  for (m = 0; m < 5; ++m) { free(g->u[m]); free(g->us[m]); }
  for (a = 0; a < 3; ++a) {
    free(g->b[a]); free(g->bs[a]); free(g->ec[a]); free(g->e[a]); free(g->sg[a]);
    for (m = 0; m < 8; ++m) free(g->fl[a][m]);
  }
  for (m = 0; m < 8; ++m) free(g->w[m]);
  free(g->shock);
  free(g->mlp);
  free(g->psi);
  for (a = 0; a < 3; ++a) free(g->gpsi[a]);
  free(g->xp); free(g->vp); free(g->mp); free(g->xh);
  for (m = 0; m < ORC_MAX_SCALAR; ++m) {
    free(g->xs[m]); free(g->xss[m]); free(g->xw[m]);
    for (a = 0; a < 3; ++a) free(g->xf[a][m]);
  }
  free(g);
}

long orc_padded_size(const orc_grid *g) { return g->np; }

void orc_set_time(orc_grid *g, double t, int64_t step) { g->t = t; g->step = step; }

/* Number of faces along axis a of the face array normal to a. */
static int nface(const orc_grid *g, int a) { return g->n[a] + (g->per[a] ? 0 : 1); }

/* ------------------------------------------------------------------------ */
/* O1: ghost fill, ng = 2, x then y then z over the full padded ranges.     */
/* ------------------------------------------------------------------------ */

/* Source coordinate of a ghost coordinate c along axis a, or -1000 for an
   inflow ghost.  interior = number of interior entries along a. */
static int ghost_src(const orc_grid *g, int a, int c, int interior) {
  int side = c < 0 ? 0 : 1;
  int bc = g->c.bc[2 * a + side];
  if (bc == ORC_BC_PERIODIC) {
    int n = g->n[a];
    return ((c % n) + n) % n;
  }
  if (bc == ORC_BC_OUTFLOW) return c < 0 ? 0 : interior - 1;
  return -1000;
}

/* Inflow value of field m (0..4 cell conserved, 5..7 face B). */
static double inflow_value(const orc_grid *g, int m) {
  const double *q = g->c.inflow;
  double gam = g->c.gamma;
  switch (m) {
    case 0: return q[0];
    case 1: return q[0] * q[1];
    case 2: return q[0] * q[2];
    case 3: return q[0] * q[3];
    case 4:
      return q[4] / (gam - 1.0) + 0.5 * q[0] * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) +
             0.5 * (q[5] * q[5] + q[6] * q[6] + q[7] * q[7]);
    default: return m < 8 ? q[m] : 0.0;  /* passive scalars: none flows in */
  }
}

/* normal = axis along which this array is face-centred, or -1 for cells. */
static void fill_ghosts_one(orc_grid *g, double *arr, int normal, int m) {
  int a;
  double vin = inflow_value(g, m);
  for (a = 0; a < 3; ++a) {
    int interior = (a == normal) ? nface(g, a) : g->n[a];
    int ax1 = (a + 1) % 3, ax2 = (a + 2) % 3;
    int c1, c2, c;
    for (c2 = -NG; c2 <= g->n[ax2] + NG; ++c2)
      for (c1 = -NG; c1 <= g->n[ax1] + NG; ++c1)
        for (c = -NG; c <= g->n[a] + NG; ++c) {
          if (c >= 0 && c < interior) continue;
          int src = ghost_src(g, a, c, interior);
          int dst[3], s[3];
          dst[a] = c; dst[ax1] = c1; dst[ax2] = c2;
          long pd = at(g, dst[0], dst[1], dst[2]);
          if (src == -1000) {
            arr[pd] = vin;
          } else {
            s[a] = src; s[ax1] = c1; s[ax2] = c2;
            arr[pd] = arr[at(g, s[0], s[1], s[2])];
          }
        }
  }
}

static void fill_ghosts(orc_grid *g, double *const u[5], double *const b[3]) {
  int m;
  for (m = 0; m < 5; ++m) fill_ghosts_one(g, u[m], -1, m);
  for (m = 0; m < 3; ++m) fill_ghosts_one(g, b[m], m, 5 + m);
}

static void fill_ghosts_scalars(orc_grid *g, double *const x[ORC_MAX_SCALAR]) {
  int m;
  for (m = 0; m < g->c.nscalar; ++m) fill_ghosts_one(g, x[m], -1, 100);
}

/* X_s = (rho X_s) / rho of the stage, on every padded cell the sweeps read. */
static void scalar_prims(orc_grid *g, double *const x[ORC_MAX_SCALAR]) {
  int m;
  long p;
  for (m = 0; m < g->c.nscalar; ++m)
    for (p = 0; p < g->np; ++p) g->xw[m][p] = g->w[0][p] != 0.0 ? x[m][p] / g->w[0][p] : 0.0;
}

/* ------------------------------------------------------------------------ */
/* O2: primitives and cell EMF (Eq. 6, Eq. 9).                              */
/* ------------------------------------------------------------------------ */

/* Primitives of one cell: rho, vx, vy, vz, P, Bcx, Bcy, Bcz. */
static void cell_prim(const orc_grid *g, double *const u[5], double *const b[3],
                      long p, double w[8]) {
  double gam = g->c.gamma;
  double rho = u[0][p];
  double bcx = 0.5 * (b[0][p] + b[0][p + g->st[0]]);
  double bcy = 0.5 * (b[1][p] + b[1][p + g->st[1]]);
  double bcz = 0.5 * (b[2][p] + b[2][p + g->st[2]]);
  double ke = 0.5 * (u[1][p] * u[1][p] + u[2][p] * u[2][p] + u[3][p] * u[3][p]) / rho;
  double me = 0.5 * (bcx * bcx + bcy * bcy + bcz * bcz);
  w[0] = rho;
  w[1] = u[1][p] / rho;
  w[2] = u[2][p] / rho;
  w[3] = u[3][p] / rho;
  w[4] = (gam - 1.0) * (u[4][p] - ke - me);
  w[5] = bcx;
  w[6] = bcy;
  w[7] = bcz;
}

static void primitives(orc_grid *g, double *const u[5], double *const b[3]) {
  int k;
#pragma omp parallel for schedule(static)
  for (k = -NG; k <= g->n[2] + NG - 1; ++k) {
    int i, j, m;
    for (j = -NG; j <= g->n[1] + NG - 1; ++j)
      for (i = -NG; i <= g->n[0] + NG - 1; ++i) {
        long p = at(g, i, j, k);
        double w[8];
        cell_prim(g, u, b, p, w);
        for (m = 0; m < 8; ++m) g->w[m][p] = w[m];
        /* E = -v x B */
        g->ec[0][p] = w[3] * w[6] - w[2] * w[7];
        g->ec[1][p] = w[1] * w[7] - w[3] * w[5];
        g->ec[2][p] = w[2] * w[5] - w[1] * w[6];
      }
  }
}

/* ------------------------------------------------------------------------ */
/* Shock cells of the stage state: some neighbour's pressure differs by     */
/* more than `jump` times the cell's, and the flow converges (central       */
/* div v < 0).  The learned correction is not applied on their faces.       */
/* ------------------------------------------------------------------------ */

static void shock_cells(orc_grid *g) {
  int k;
#pragma omp parallel for schedule(static)
  for (k = -1; k <= g->n[2]; ++k) {
    int i, j, a;
    for (j = -1; j <= g->n[1]; ++j)
      for (i = -1; i <= g->n[0]; ++i) {
        long p = at(g, i, j, k);
        double P = g->w[4][p], jmax = 0.0, div = 0.0;
        for (a = 0; a < 3; ++a) {
          long s = g->st[a];
          double jl = fabs(g->w[4][p - s] - P) / P, jh = fabs(g->w[4][p + s] - P) / P;
          if (jl > jmax) jmax = jl;
          if (jh > jmax) jmax = jh;
          div += (g->w[1 + a][p + s] - g->w[1 + a][p - s]) / (2.0 * g->d[a]);
        }
        g->shock[p] = (jmax > g->mlp_jump && div < 0.0) ? 1 : 0;
      }
  }
}

/* Learned correction of one corrector face flux f (frame order).  Faces
   touching a shock cell keep the plain flux (caller); a face whose two-cell
   means of rho or P are not positive keeps it too (returns 0); elsewhere each
   component of the correction is clipped to
   tau_flux |F| + tau a_max |U_R - U_L|. */
static int mlp_correct(const orc_grid *g, const double w8[32], const double wl[7],
                       const double wr[7], double bn, double f[7]) {
  double x[32], y[8], df[7], ul[7], ur[7];
  double gam = g->c.gamma;
  int m;
  if (!(w8[8] + w8[16] > 0.0) || !(w8[12] + w8[20] > 0.0)) return 0;
  orc_mlp_features(w8, gam, x);
  orc_mlp_forward(g->mlp, 1, 1, x, y);
  orc_mlp_out_to_flux(w8, gam, y, df);
  orc_prim_to_cons(wl, bn, gam, ul);
  orc_prim_to_cons(wr, bn, gam, ur);
  double cfl = orc_fast_speed(wl, bn, gam), cfr = orc_fast_speed(wr, bn, gam);
  double cmax = cfl > cfr ? cfl : cfr;
  double sl = fabs((wl[1] < wr[1] ? wl[1] : wr[1]) - cmax);
  double sr = fabs((wl[1] > wr[1] ? wl[1] : wr[1]) + cmax);
  double amax = sl > sr ? sl : sr;
  for (m = 0; m < 7; ++m) {
    double lim = g->mlp_tau_flux * fabs(f[m]) + g->mlp_tau * amax * fabs(ur[m] - ul[m]);
    double d = df[m];
    if (d > lim) d = lim;
    if (d < -lim) d = -lim;
    f[m] += d;
  }
  return 1;
}

/* ------------------------------------------------------------------------ */
/* O4 / O9: flux sweep along axis a.                                        */
/* ------------------------------------------------------------------------ */

static void sweep(orc_grid *g, int a, double *const bf[3], int recon) {
  int t1 = (a + 1) % 3, t2 = (a + 2) % 3;
  long s = g->st[a];
  /* frame variable -> primitive array: rho, vn, vt1, vt2, P, Bt1, Bt2 */
  double *src[7] = {g->w[0], g->w[1 + a], g->w[1 + t1], g->w[1 + t2], g->w[4],
                    g->w[5 + t1], g->w[5 + t2]};
  int lo[3], hi[3], k;
  int64_t nhll = 0, ndeg = 0, nmlp = 0, ngate = 0;
  int learned = g->mlp != NULL && recon != ORC_RECON_FIRST;
  /* normal: faces 0..n; transverse: rows -1..n, which the corner EMFs of
     the boundary edges need */
  for (k = 0; k < 3; ++k) { lo[k] = -1; hi[k] = g->n[k]; }
  lo[a] = 0; hi[a] = g->n[a];
#pragma omp parallel for schedule(static) reduction(+ : nhll, ndeg, nmlp, ngate)
  for (k = lo[2]; k <= hi[2]; ++k) {
    int i, j, v, c;
    for (j = lo[1]; j <= hi[1]; ++j)
      for (i = lo[0]; i <= hi[0]; ++i) {
        long p = at(g, i, j, k); /* face between cells p - s and p */
        double wl[7], wr[7], f[7];
        for (v = 0; v < 7; ++v) {
          double st4[4] = {src[v][p - 2 * s], src[v][p - s], src[v][p], src[v][p + s]};
          orc_recon(st4, recon, g->c.kappa, &wl[v], &wr[v]);
        }
        int code = g->c.riemann == ORC_RIEMANN_HLL
                       ? orc_hll(wl, wr, bf[a][p], g->c.gamma, f)
                       : g->c.riemann == ORC_RIEMANN_HLLC
                             ? orc_hllc(wl, wr, bf[a][p], g->c.gamma, f)
                             : orc_hlld(wl, wr, bf[a][p], g->c.gamma, f);
        if (code & 1) nhll++;
        if (code & 2) ndeg++;
        if (learned) {
          if (g->shock[p - s] || g->shock[p]) {
            ngate++;
          } else {
            /* stencil of 8 frame primitives: rho, vn, vt1, vt2, P, Bn, Bt1, Bt2 */
            double w8[32];
            for (c = 0; c < 4; ++c) {
              long q = p + (c - 2) * s;
              w8[8 * c + 0] = g->w[0][q];
              w8[8 * c + 1] = g->w[1 + a][q];
              w8[8 * c + 2] = g->w[1 + t1][q];
              w8[8 * c + 3] = g->w[1 + t2][q];
              w8[8 * c + 4] = g->w[4][q];
              w8[8 * c + 5] = g->w[5 + a][q];
              w8[8 * c + 6] = g->w[5 + t1][q];
              w8[8 * c + 7] = g->w[5 + t2][q];
            }
            if (mlp_correct(g, w8, wl, wr, bf[a][p], f))
              nmlp++;
            else
              ngate++;
          }
        }
        g->fl[a][0][p] = f[0];
        g->fl[a][1 + a][p] = f[1];
        g->fl[a][1 + t1][p] = f[2];
        g->fl[a][1 + t2][p] = f[3];
        g->fl[a][4][p] = f[4];
        g->fl[a][5 + a][p] = 0.0;
        g->fl[a][5 + t1][p] = f[5];
        g->fl[a][5 + t2][p] = f[6];
        g->sg[a][p] = f[0] > 0.0 ? 1 : (f[0] < 0.0 ? -1 : 0);
        /* passive scalars ride on the (final) mass flux, upwinded */
        for (c = 0; c < g->c.nscalar; ++c) {
          double xl, xr;
          double st4[4] = {g->xw[c][p - 2 * s], g->xw[c][p - s], g->xw[c][p], g->xw[c][p + s]};
          orc_recon(st4, recon, g->c.kappa, &xl, &xr);
          g->xf[a][c][p] = f[0] > 0.0 ? f[0] * xl : (f[0] < 0.0 ? f[0] * xr : 0.0);
        }
      }
  }
  g->n_hll += nhll;
  g->n_deg += ndeg;
  g->n_mlp += nmlp;
  g->n_gated += ngate;
}

/* ------------------------------------------------------------------------ */
/* O5 / O6: corner EMF, Eq. 10 with R3/R4, Eq. 11 with R6.                  */
/* ------------------------------------------------------------------------ */

/* Upwind choice of Eq. 11: the value on the side the mass flux comes from. */
static double upwind(int sign, double from_low, double from_high) {
  if (sign > 0) return from_low;
  if (sign < 0) return from_high;
  return 0.5 * (from_low + from_high);
}

/* Edge EMF component c, staggered along a = c+1 and b = c+2 (cyclic).
   Edge index p sits at p - ea/2 - eb/2. */
static void corner_emf(orc_grid *g, int c) {
  int a = (c + 1) % 3, b = (c + 2) % 3;
  long sa = g->st[a], sb = g->st[b];
  const double *fa = g->fl[a][5 + b]; /* a-face flux of B_b */
  const double *fb = g->fl[b][5 + a]; /* b-face flux of B_a */
  const signed char *ga = g->sg[a], *gb = g->sg[b];
  const double *cc = g->ec[c];
  double *out = g->e[c];
  int lo[3] = {0, 0, 0}, hi[3], k;
  hi[a] = g->n[a];
  hi[b] = g->n[b];
  hi[c] = g->n[c] - 1;
#pragma omp parallel for schedule(static)
  for (k = lo[2]; k <= hi[2]; ++k) {
    int i, j;
    for (j = lo[1]; j <= hi[1]; ++j)
      for (i = lo[0]; i <= hi[0]; ++i) {
        long p = at(g, i, j, k);
        /* face EMFs: at an a-face E_c = -Fa[B_b]; at a b-face E_c = +Fb[B_a] */
        double X0 = -fa[p], X1 = -fa[p - sb];      /* (a-1/2, b), (a-1/2, b-1) */
        double Y0 = fb[p], Y1 = fb[p - sa];        /* (a, b-1/2), (a-1, b-1/2) */
        double c00 = cc[p - sa - sb], c10 = cc[p - sb]; /* (a-1,b-1), (a,b-1) */
        double c01 = cc[p - sa], c11 = cc[p];           /* (a-1,b),   (a,b)   */
        /* derivatives along b, upwinded by the a-face mass flux */
        double db_q1 = upwind(ga[p], c01 - Y1, c11 - Y0);          /* b - 1/4 */
        double db_q3 = upwind(ga[p - sb], Y1 - c00, Y0 - c10);     /* b - 3/4 */
        /* derivatives along a, upwinded by the b-face mass flux */
        double da_q1 = upwind(gb[p], c10 - X1, c11 - X0);          /* a - 1/4 */
        double da_q3 = upwind(gb[p - sa], X1 - c00, X0 - c01);     /* a - 3/4 */
        out[p] = 0.25 * (X0 + X1 + Y0 + Y1) + 0.25 * (db_q3 - db_q1) +
                 0.25 * (da_q3 - da_q1);
      }
  }
}

/* ------------------------------------------------------------------------ */
/* O12: source vector S = (0, -rho grad Phi, -rho v.grad Phi, 0).          */
/* ------------------------------------------------------------------------ */

static void grad_phi(const orc_grid *g, double x, double y, double z, double gp[3]) {
  const double *s = g->c.src;
  gp[0] = gp[1] = gp[2] = 0.0;
  switch (g->c.source) {
    case ORC_SRC_LOGPOT: {
      double v0 = s[0], rc = s[1], q = s[2];
      double den = rc * rc + x * x + y * y + z * z / (q * q);
      gp[0] = v0 * v0 * x / den;
      gp[1] = v0 * v0 * y / den;
      gp[2] = v0 * v0 * (z / (q * q)) / den;
      break;
    }
    case ORC_SRC_UNIFORM:
      gp[0] = s[0]; gp[1] = s[1]; gp[2] = s[2];
      break;
    case ORC_SRC_GAUSS_X: {
      double A = s[0], wd = s[1];
      /* Phi = -A exp(-(x/w)^2) -> dPhi/dx = 2 A x / w^2 exp(-(x/w)^2) */
      gp[0] = 2.0 * A * x / (wd * wd) * exp(-(x / wd) * (x / wd));
      break;
    }
    default:
      break;
  }
}

/* ------------------------------------------------------------------------ */
/* Self-gravity (the paper's Poisson equation), periodic box.               */
/* ------------------------------------------------------------------------ */

/* One-dimensional DFT along a line of n values (stride st) of re/im, from
   the definition: X_k = sum_j x_j exp(sign 2 pi i j k / n). */
static void dft_line(double *re, double *im, int n, long st, int sign, double *tr, double *ti) {
  int j, k;
  for (k = 0; k < n; ++k) {
    double sr = 0.0, si = 0.0;
    for (j = 0; j < n; ++j) {
      double a = sign * 2.0 * M_PI_ORC * (double)(((long)j * k) % n) / (double)n;
      double c = cos(a), s = sin(a);
      sr += re[j * st] * c - im[j * st] * s;
      si += re[j * st] * s + im[j * st] * c;
    }
    tr[k] = sr;
    ti[k] = si;
  }
  for (k = 0; k < n; ++k) {
    re[k * st] = tr[k];
    im[k * st] = ti[k];
  }
}

static void dft3(double *re, double *im, int nx, int ny, int nz, int sign) {
  int n[3] = {nx, ny, nz};
  long st[3] = {1, nx, (long)nx * ny};
  int a;
  for (a = 0; a < 3; ++a) {
    if (n[a] == 1) continue;
    int b = (a + 1) % 3, c = (a + 2) % 3;
    int ib;
#pragma omp parallel for schedule(static)
    for (ib = 0; ib < n[b]; ++ib) {
      double *tr = (double *)malloc(sizeof(double) * (size_t)n[a]);
      double *ti = (double *)malloc(sizeof(double) * (size_t)n[a]);
      int ic;
      for (ic = 0; ic < n[c]; ++ic) {
        long o = ib * st[b] + ic * st[c];
        dft_line(re + o, im + o, n[a], st[a], sign, tr, ti);
      }
      free(tr);
      free(ti);
    }
  }
}

void orc_poisson_periodic(int nx, int ny, int nz, double dx, double dy, double dz, double G,
                          const double *rho, double *psi) {
  long N = (long)nx * ny * nz, q;
  double *re = (double *)malloc(sizeof(double) * (size_t)N);
  double *im = (double *)calloc((size_t)N, sizeof(double));
  for (q = 0; q < N; ++q) re[q] = rho[q];
  dft3(re, im, nx, ny, nz, -1);
  int i, j, k;
  for (k = 0; k < nz; ++k)
    for (j = 0; j < ny; ++j)
      for (i = 0; i < nx; ++i) {
        /* eigenvalue of the 7-point Laplacian for mode (i, j, k) */
        double lam = (2.0 * cos(2.0 * M_PI_ORC * i / nx) - 2.0) / (dx * dx) +
                     (2.0 * cos(2.0 * M_PI_ORC * j / ny) - 2.0) / (dy * dy) +
                     (2.0 * cos(2.0 * M_PI_ORC * k / nz) - 2.0) / (dz * dz);
        long p = ((long)k * ny + j) * nx + i;
        if (i == 0 && j == 0 && k == 0) {
          re[p] = 0.0;
          im[p] = 0.0;
        } else {
          re[p] *= 4.0 * M_PI_ORC * G / lam;
          im[p] *= 4.0 * M_PI_ORC * G / lam;
        }
      }
  dft3(re, im, nx, ny, nz, +1);
  for (q = 0; q < N; ++q) psi[q] = re[q] / (double)N;
  free(re);
  free(im);
}

/* Psi of the stage density (primitives w[0]) and its central gradient at
   every interior cell, with periodic wrap. */
/* ------------------------------------------------------------------------ */
/* N-body particles: cloud-in-cell weights, deposit, interpolation.         */
/* ------------------------------------------------------------------------ */

static int gas_decoupled(const orc_grid *g) {
  return g->c.source == ORC_SRC_SELF_GRAVITY && g->c.src[1] == 1.0;
}

/* Along axis a: the particle's cube [x - d/2, x + d/2] overlaps cells c0
   and c0 + 1 (wrapped) with fractions w0 = 1 - f, w1 = f; in cell-centre
   units s = (x - x0)/d - 1/2, c0 = floor(s), f = s - c0. */
static void cic_axis(const orc_grid *g, int a, double x, int c[2], double w[2]) {
  double x0 = a == 0 ? g->c.x0 : (a == 1 ? g->c.y0 : g->c.z0);
  double s = (x - x0) / g->d[a] - 0.5;
  double fl = floor(s);
  int n = g->n[a];
  long c0 = (long)fl;
  c[0] = (int)(((c0 % n) + n) % n);
  c[1] = (c[0] + 1) % n;
  w[1] = s - fl;
  w[0] = 1.0 - w[1];
}

void orc_particle_deposit(const orc_grid *g, const double *x, double *rho) {
  int nx = g->n[0], ny = g->n[1], nz = g->n[2];
  long N = (long)nx * ny * nz, n = g->c.npart, q;
  double idv = 1.0 / (g->d[0] * g->d[1] * g->d[2]);
  for (q = 0; q < N; ++q) rho[q] = 0.0;
  for (q = 0; q < n; ++q) {
    int ci[2], cj[2], ck[2], a, b, e;
    double wi[2], wj[2], wk[2];
    cic_axis(g, 0, x[q], ci, wi);
    cic_axis(g, 1, x[n + q], cj, wj);
    cic_axis(g, 2, x[2 * n + q], ck, wk);
    for (e = 0; e < 2; ++e)
      for (b = 0; b < 2; ++b)
        for (a = 0; a < 2; ++a)
          rho[((long)ck[e] * ny + cj[b]) * nx + ci[a]] += g->mp[q] * wi[a] * wj[b] * wk[e] * idv;
  }
}

void orc_particle_interp(const orc_grid *g, const double *f, const double *x, long n,
                         double *out) {
  int nx = g->n[0], ny = g->n[1];
  long q;
  for (q = 0; q < n; ++q) {
    int ci[2], cj[2], ck[2], a, b, e;
    double wi[2], wj[2], wk[2], s = 0.0;
    cic_axis(g, 0, x[q], ci, wi);
    cic_axis(g, 1, x[n + q], cj, wj);
    cic_axis(g, 2, x[2 * n + q], ck, wk);
    for (e = 0; e < 2; ++e)
      for (b = 0; b < 2; ++b)
        for (a = 0; a < 2; ++a) s += wi[a] * wj[b] * wk[e] * f[((long)ck[e] * ny + cj[b]) * nx + ci[a]];
    out[q] = s;
  }
}

/* x mapped into [lo, lo + L) */
static double wrap_coord(double x, double lo, double L) {
  return x - L * floor((x - lo) / L);
}

static void wrap_positions(const orc_grid *g, double *x) {
  long n = g->c.npart, q;
  double lo[3] = {g->c.x0, g->c.y0, g->c.z0};
  int a;
  for (a = 0; a < 3; ++a)
    for (q = 0; q < n; ++q) x[a * n + q] = wrap_coord(x[a * n + q], lo[a], g->n[a] * g->d[a]);
}

/* Potential of the gas density of the stage (unless decoupled) plus the
   particles deposited at xpart (if any), and its central gradient. */
static void self_gravity(orc_grid *g, const double *xpart) {
  int nx = g->n[0], ny = g->n[1], nz = g->n[2];
  long N = (long)nx * ny * nz;
  double *rho = (double *)calloc((size_t)N, sizeof(double));
  double *psi = (double *)calloc((size_t)N, sizeof(double));
  int i, j, k;
  if (xpart) orc_particle_deposit(g, xpart, rho);
  if (!gas_decoupled(g))
    for (k = 0; k < nz; ++k)
      for (j = 0; j < ny; ++j)
        for (i = 0; i < nx; ++i) rho[((long)k * ny + j) * nx + i] += g->w[0][at(g, i, j, k)];
  orc_poisson_periodic(nx, ny, nz, g->d[0], g->d[1], g->d[2], g->c.src[0], rho, psi);
  for (k = 0; k < nz; ++k)
    for (j = 0; j < ny; ++j)
      for (i = 0; i < nx; ++i) {
        long p = at(g, i, j, k);
#define PSI(ii, jj, kk) psi[((long)(((kk) + nz) % nz) * ny + (((jj) + ny) % ny)) * nx + (((ii) + nx) % nx)]
        g->psi[p] = PSI(i, j, k);
        g->gpsi[0][p] = (PSI(i + 1, j, k) - PSI(i - 1, j, k)) / (2.0 * g->d[0]);
        g->gpsi[1][p] = (PSI(i, j + 1, k) - PSI(i, j - 1, k)) / (2.0 * g->d[1]);
        g->gpsi[2][p] = (PSI(i, j, k + 1) - PSI(i, j, k - 1)) / (2.0 * g->d[2]);
#undef PSI
      }
  free(rho);
  free(psi);
}

/* ------------------------------------------------------------------------ */
/* O7 / O11: conservative update (Eq. 7) and CT induction update (Eq. 8).  */
/* ------------------------------------------------------------------------ */

static void update(orc_grid *g, double dt, double *const u0[5], double *const b0[3],
                   double *const u1[5], double *const b1[3], double *const x0[ORC_MAX_SCALAR],
                   double *const x1[ORC_MAX_SCALAR]) {
  int a, k;
  /* passive scalars: conservative update, no source */
  {
    double rx = dt / g->d[0], ry = dt / g->d[1], rz = dt / g->d[2];
    int m;
    for (m = 0; m < g->c.nscalar; ++m) {
#pragma omp parallel for schedule(static)
      for (k = 0; k < g->n[2]; ++k) {
        int i, j;
        for (j = 0; j < g->n[1]; ++j)
          for (i = 0; i < g->n[0]; ++i) {
            long p = at(g, i, j, k);
            double v = x0[m][p];
            v -= rx * (g->xf[0][m][p + g->st[0]] - g->xf[0][m][p]);
            v -= ry * (g->xf[1][m][p + g->st[1]] - g->xf[1][m][p]);
            v -= rz * (g->xf[2][m][p + g->st[2]] - g->xf[2][m][p]);
            x1[m][p] = v;
          }
      }
    }
  }
  /* faces first (the floors below need the new cell-centred B) */
  for (a = 0; a < 3; ++a) {
    int b = (a + 1) % 3, c = (a + 2) % 3;
    long sb = g->st[b], sc = g->st[c];
    const double *Ec = g->e[c], *Eb = g->e[b];
    double rb = dt / g->d[b], rc = dt / g->d[c];
    int hi[3];
    hi[0] = g->n[0] - 1; hi[1] = g->n[1] - 1; hi[2] = g->n[2] - 1;
    hi[a] = nface(g, a) - 1;
#pragma omp parallel for schedule(static)
    for (k = 0; k <= hi[2]; ++k) {
      int i, j;
      for (j = 0; j <= hi[1]; ++j)
        for (i = 0; i <= hi[0]; ++i) {
          long p = at(g, i, j, k);
          /* dB_a/dt = -(curl E)_a = -(dE_c/db - dE_b/dc) */
          b1[a][p] = b0[a][p] - rb * (Ec[p + sb] - Ec[p]) + rc * (Eb[p + sc] - Eb[p]);
        }
    }
  }
  double rx = dt / g->d[0], ry = dt / g->d[1], rz = dt / g->d[2];
  double gam = g->c.gamma;
  int64_t nfl = 0;
#pragma omp parallel for schedule(static) reduction(+ : nfl)
  for (k = 0; k < g->n[2]; ++k) {
    int i, j, m;
    for (j = 0; j < g->n[1]; ++j)
      for (i = 0; i < g->n[0]; ++i) {
        long p = at(g, i, j, k);
        double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (g->c.source != ORC_SRC_NONE) {
          double gp[3];
          double x = g->c.x0 + (i + 0.5) * g->d[0];
          double y = g->c.y0 + (j + 0.5) * g->d[1];
          double z = g->c.z0 + (k + 0.5) * g->d[2];
          if (gas_decoupled(g)) {
            gp[0] = gp[1] = gp[2] = 0.0;
          } else if (g->c.source == ORC_SRC_SELF_GRAVITY) {
            gp[0] = g->gpsi[0][p];
            gp[1] = g->gpsi[1][p];
            gp[2] = g->gpsi[2][p];
          } else {
            grad_phi(g, x, y, z, gp);
          }
          double rho = g->w[0][p];
          s[1] = -rho * gp[0];
          s[2] = -rho * gp[1];
          s[3] = -rho * gp[2];
          s[4] = -rho * (g->w[1][p] * gp[0] + g->w[2][p] * gp[1] + g->w[3][p] * gp[2]);
        }
        for (m = 0; m < 5; ++m) {
          double v = u0[m][p];
          v -= rx * (g->fl[0][m][p + g->st[0]] - g->fl[0][m][p]);
          v -= ry * (g->fl[1][m][p + g->st[1]] - g->fl[1][m][p]);
          v -= rz * (g->fl[2][m][p + g->st[2]] - g->fl[2][m][p]);
          v += dt * s[m];
          u1[m][p] = v;
        }
        if (g->c.rho_floor > 0.0 || g->c.p_floor > 0.0) {
          int hit = 0;
          if (u1[0][p] < g->c.rho_floor) { u1[0][p] = g->c.rho_floor; hit = 1; }
          /* cell-centred B of the updated faces; on a periodic axis the
             upper face of the last cell is the first face (its ghost copy
             is not written until the next ghost fill) */
          int idx[3];
          double bcn[3];
          idx[0] = i; idx[1] = j; idx[2] = k;
          for (m = 0; m < 3; ++m) {
            long up = p + g->st[m];
            if (g->per[m] && idx[m] == g->n[m] - 1) up = p - (long)(g->n[m] - 1) * g->st[m];
            bcn[m] = 0.5 * (b1[m][p] + b1[m][up]);
          }
          double bcx = bcn[0], bcy = bcn[1], bcz = bcn[2];
          double rho = u1[0][p];
          double ke = 0.5 * (u1[1][p] * u1[1][p] + u1[2][p] * u1[2][p] + u1[3][p] * u1[3][p]) / rho;
          double me = 0.5 * (bcx * bcx + bcy * bcy + bcz * bcz);
          double P = (gam - 1.0) * (u1[4][p] - ke - me);
          if (P < g->c.p_floor) { u1[4][p] += (g->c.p_floor - P) / (gam - 1.0); hit = 1; }
          nfl += hit;
        }
      }
  }
  g->n_floor += nfl;
}

/* ------------------------------------------------------------------------ */
/* O3: CFL time step (R9).                                                  */
/* ------------------------------------------------------------------------ */

double orc_dt(orc_grid *g) {
  double gam = g->c.gamma;
  double best = INFINITY;
  int k;
#pragma omp parallel for schedule(static) reduction(min : best)
  for (k = 0; k < g->n[2]; ++k) {
    int i, j, a;
    for (j = 0; j < g->n[1]; ++j)
      for (i = 0; i < g->n[0]; ++i) {
        double w[8];
        cell_prim(g, g->u, g->b, at(g, i, j, k), w);
        for (a = 0; a < 3; ++a) {
          int t1 = (a + 1) % 3, t2 = (a + 2) % 3;
          double w7[7] = {w[0], w[1 + a], w[1 + t1], w[1 + t2], w[4], w[5 + t1], w[5 + t2]};
          double cf = orc_fast_speed(w7, w[5 + a], gam);
          double v = fabs(w[1 + a]);
          double r = g->d[a] / (v + cf);
          if (r < best) best = r;
        }
      }
  }
  /* particles: no particle crosses more than cfl cells along an axis */
  {
    long n = g->c.npart, q;
    int a;
    for (a = 0; a < 3; ++a)
      for (q = 0; q < n; ++q) {
        double v = fabs(g->vp[a * n + q]);
        if (v > 0.0 && g->d[a] / v < best) best = g->d[a] / v;
      }
  }
  return g->c.cfl * best;
}

/* Kick with the corrector's potential at the half-step positions, then
   the second half drift. */
static void particles_kick_drift(orc_grid *g, double dt) {
  long n = g->c.npart, q;
  int nx = g->n[0], ny = g->n[1], nz = g->n[2], a, i, j, k;
  long N = (long)nx * ny * nz;
  double *f = (double *)malloc((size_t)N * sizeof(double));
  double *acc = (double *)malloc((size_t)n * sizeof(double));
  for (a = 0; a < 3; ++a) {
    for (k = 0; k < nz; ++k)
      for (j = 0; j < ny; ++j)
        for (i = 0; i < nx; ++i) f[((long)k * ny + j) * nx + i] = g->gpsi[a][at(g, i, j, k)];
    orc_particle_interp(g, f, g->xh, n, acc);
    for (q = 0; q < n; ++q) g->vp[a * n + q] -= dt * acc[q];
  }
  for (a = 0; a < 3; ++a)
    for (q = 0; q < n; ++q) g->xp[a * n + q] = g->xh[a * n + q] + 0.5 * dt * g->vp[a * n + q];
  wrap_positions(g, g->xp);
  free(f);
  free(acc);
}

/* ------------------------------------------------------------------------ */
/* One step (R1): predictor to t^{n+1/2}, corrector to t^{n+1}.            */
/* ------------------------------------------------------------------------ */

double orc_step(orc_grid *g, double dt) {
  int a;
  if (!(dt > 0.0)) dt = orc_dt(g);
  /* predictor: first-order fluxes of U^n, half step */
  primitives(g, g->u, g->b);
  scalar_prims(g, g->xs);
  if (g->c.source == ORC_SRC_SELF_GRAVITY) self_gravity(g, g->c.npart ? g->xp : NULL);
  for (a = 0; a < 3; ++a) sweep(g, a, g->b, ORC_RECON_FIRST);
  for (a = 0; a < 3; ++a) corner_emf(g, a);
  update(g, 0.5 * dt, g->u, g->b, g->us, g->bs, g->xs, g->xss);
  fill_ghosts(g, g->us, g->bs);
  fill_ghosts_scalars(g, g->xss);
  /* corrector: MUSCL fluxes of U*, full step from U^n */
  primitives(g, g->us, g->bs);
  scalar_prims(g, g->xss);
  if (g->c.npart) {
    long n = g->c.npart, q;
    for (q = 0; q < 3 * n; ++q) g->xh[q] = g->xp[q] + 0.5 * dt * g->vp[q];
    wrap_positions(g, g->xh);
  }
  if (g->c.source == ORC_SRC_SELF_GRAVITY) self_gravity(g, g->c.npart ? g->xh : NULL);
  if (g->mlp) shock_cells(g);
  for (a = 0; a < 3; ++a) sweep(g, a, g->bs, g->c.recon);
  for (a = 0; a < 3; ++a) corner_emf(g, a);
  update(g, dt, g->u, g->b, g->u, g->b, g->xs, g->xs);
  fill_ghosts(g, g->u, g->b);
  fill_ghosts_scalars(g, g->xs);
  if (g->c.npart) particles_kick_drift(g, dt);
  g->t += dt;
  g->step += 1;
  return dt;
}

/* ------------------------------------------------------------------------ */
/* State in / out                                                           */
/* ------------------------------------------------------------------------ */

void orc_set_particles(orc_grid *g, const double *x, const double *v, const double *m) {
  long n = g->c.npart, q;
  for (q = 0; q < 3 * n; ++q) {
    g->xp[q] = x[q];
    g->vp[q] = v[q];
  }
  for (q = 0; q < n; ++q) g->mp[q] = m[q];
  wrap_positions(g, g->xp);
}

void orc_get_particles(const orc_grid *g, double *x, double *v) {
  long n = g->c.npart, q;
  for (q = 0; q < 3 * n; ++q) {
    x[q] = g->xp[q];
    v[q] = g->vp[q];
  }
}

void orc_set_scalars(orc_grid *g, const double *rho_x) {
  int nx = g->n[0], ny = g->n[1], nz = g->n[2], i, j, k, m;
  long ncell = (long)nx * ny * nz;
  for (m = 0; m < g->c.nscalar; ++m)
    for (k = 0; k < nz; ++k)
      for (j = 0; j < ny; ++j)
        for (i = 0; i < nx; ++i)
          g->xs[m][at(g, i, j, k)] = rho_x[m * ncell + ((long)k * ny + j) * nx + i];
  fill_ghosts_scalars(g, g->xs);
}

void orc_get_scalars(const orc_grid *g, double *rho_x) {
  int nx = g->n[0], ny = g->n[1], nz = g->n[2], i, j, k, m;
  long ncell = (long)nx * ny * nz;
  for (m = 0; m < g->c.nscalar; ++m)
    for (k = 0; k < nz; ++k)
      for (j = 0; j < ny; ++j)
        for (i = 0; i < nx; ++i)
          rho_x[m * ncell + ((long)k * ny + j) * nx + i] = g->xs[m][at(g, i, j, k)];
}

int orc_set_state(orc_grid *g, const double *cell5, const double *bx,
                  const double *by, const double *bz) {
  int nx = g->n[0], ny = g->n[1], nz = g->n[2];
  int fx = nface(g, 0), fy = nface(g, 1), fz = nface(g, 2);
  int i, j, k, m;
  long ncell = (long)nx * ny * nz;
  for (m = 0; m < 5; ++m)
    for (k = 0; k < nz; ++k)
      for (j = 0; j < ny; ++j)
        for (i = 0; i < nx; ++i)
          g->u[m][at(g, i, j, k)] = cell5[m * ncell + ((long)k * ny + j) * nx + i];
  for (k = 0; k < nz; ++k)
    for (j = 0; j < ny; ++j)
      for (i = 0; i < fx; ++i) g->b[0][at(g, i, j, k)] = bx[((long)k * ny + j) * fx + i];
  for (k = 0; k < nz; ++k)
    for (j = 0; j < fy; ++j)
      for (i = 0; i < nx; ++i) g->b[1][at(g, i, j, k)] = by[((long)k * fy + j) * nx + i];
  for (k = 0; k < fz; ++k)
    for (j = 0; j < ny; ++j)
      for (i = 0; i < nx; ++i) g->b[2][at(g, i, j, k)] = bz[((long)k * ny + j) * nx + i];
  fill_ghosts(g, g->u, g->b);
  for (k = 0; k < nz; ++k)
    for (j = 0; j < ny; ++j)
      for (i = 0; i < nx; ++i) {
        double w[8];
        cell_prim(g, g->u, g->b, at(g, i, j, k), w);
        for (m = 0; m < 8; ++m)
          if (!isfinite(w[m])) return -3;
        if (!(w[0] > 0.0) || !(w[4] > 0.0)) return -3;
      }
  return 0;
}

void orc_get_state(const orc_grid *g, double *cell5, double *bx, double *by,
                   double *bz) {
  int nx = g->n[0], ny = g->n[1], nz = g->n[2];
  int fx = nface(g, 0), fy = nface(g, 1), fz = nface(g, 2);
  int i, j, k, m;
  long ncell = (long)nx * ny * nz;
  if (cell5)
    for (m = 0; m < 5; ++m)
      for (k = 0; k < nz; ++k)
        for (j = 0; j < ny; ++j)
          for (i = 0; i < nx; ++i)
            cell5[m * ncell + ((long)k * ny + j) * nx + i] = g->u[m][at(g, i, j, k)];
  if (bx)
    for (k = 0; k < nz; ++k)
      for (j = 0; j < ny; ++j)
        for (i = 0; i < fx; ++i) bx[((long)k * ny + j) * fx + i] = g->b[0][at(g, i, j, k)];
  if (by)
    for (k = 0; k < nz; ++k)
      for (j = 0; j < fy; ++j)
        for (i = 0; i < nx; ++i) by[((long)k * fy + j) * nx + i] = g->b[1][at(g, i, j, k)];
  if (bz)
    for (k = 0; k < fz; ++k)
      for (j = 0; j < ny; ++j)
        for (i = 0; i < nx; ++i) bz[((long)k * ny + j) * nx + i] = g->b[2][at(g, i, j, k)];
}

/* ------------------------------------------------------------------------ */
/* Diagnostics: Neumaier-compensated FP64 sums.                             */
/* ------------------------------------------------------------------------ */

typedef struct { double s, c; } ksum;
static void kadd(ksum *k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
  else k->c += (x - t) + k->s;
  k->s = t;
}
static double kval(const ksum *k) { return k->s + k->c; }

void orc_diag_get(orc_grid *g, orc_diag *out) {
  int nx = g->n[0], ny = g->n[1], nz = g->n[2];
  double dv = g->d[0] * g->d[1] * g->d[2];
  ksum s[5], bs[3];
  int i, j, k, m, a;
  memset(s, 0, sizeof s);
  memset(bs, 0, sizeof bs);
  double rmin = INFINITY, pmin = INFINITY, bmax = 0.0, dmax = 0.0;
  for (k = 0; k < nz; ++k)
    for (j = 0; j < ny; ++j)
      for (i = 0; i < nx; ++i) {
        long p = at(g, i, j, k);
        double w[8];
        cell_prim(g, g->u, g->b, p, w);
        for (m = 0; m < 5; ++m) kadd(&s[m], g->u[m][p]);
        if (w[0] < rmin) rmin = w[0];
        if (w[4] < pmin) pmin = w[4];
        double dvb = (g->b[0][p + g->st[0]] - g->b[0][p]) / g->d[0] +
                     (g->b[1][p + g->st[1]] - g->b[1][p]) / g->d[1] +
                     (g->b[2][p + g->st[2]] - g->b[2][p]) / g->d[2];
        if (fabs(dvb) > dmax) dmax = fabs(dvb);
      }
  for (a = 0; a < 3; ++a) {
    int hi[3] = {nx, ny, nz};
    hi[a] = nface(g, a);
    for (k = 0; k < hi[2]; ++k)
      for (j = 0; j < hi[1]; ++j)
        for (i = 0; i < hi[0]; ++i) {
          double v = g->b[a][at(g, i, j, k)];
          kadd(&bs[a], v);
          if (fabs(v) > bmax) bmax = fabs(v);
        }
  }
  double h = g->d[0];
  if (g->d[1] < h) h = g->d[1];
  if (g->d[2] < h) h = g->d[2];
  out->t = g->t;
  out->step = g->step;
  out->mass = kval(&s[0]) * dv;
  out->mom[0] = kval(&s[1]) * dv;
  out->mom[1] = kval(&s[2]) * dv;
  out->mom[2] = kval(&s[3]) * dv;
  out->energy = kval(&s[4]) * dv;
  for (a = 0; a < 3; ++a) out->bsum[a] = kval(&bs[a]) * dv;
  out->divb_max = bmax > 0.0 ? dmax * h / bmax : dmax * h;
  out->rho_min = rmin;
  out->p_min = pmin;
  out->n_floor = g->n_floor;
  out->n_hll_fallback = g->n_hll;
  out->n_degenerate = g->n_deg;
  out->n_mlp_faces = g->n_mlp;
  out->n_mlp_gated = g->n_gated;
}

/* ------------------------------------------------------------------------ */
/* Debug access to the last corrector stage.                                */
/* ------------------------------------------------------------------------ */

long orc_debug_array(const orc_grid *g, int what, double *out) {
  long p;
  const double *src = NULL;
  if (what >= 0 && what < 24) src = g->fl[what / 8][what % 8];
  else if (what >= 24 && what < 27) src = g->e[what - 24];
  else if (what >= 27 && what < 30) src = g->ec[what - 27];
  else if (what >= 33 && what < 41) src = g->w[what - 33];
  else if (what >= 41 && what < 45 && g->psi) src = what == 41 ? g->psi : g->gpsi[what - 42];
  else if (what >= 30 && what < 33) {
    for (p = 0; p < g->np; ++p) out[p] = (double)g->sg[what - 30][p];
    return g->np;
  } else {
    return -1;
  }
  memcpy(out, src, (size_t)g->np * sizeof(double));
  return g->np;
}
