/*
 * orc_driver.c -- runs the FP64 oracle through its paths under the address
 * and undefined-behaviour sanitizers (built and run by
 * tests/test_sanitizers.py): a ragged 3-D box with mixed boundaries, the
 * disc potential and floors; the other fixed potentials, inflow sides,
 * passive scalars and the learned correction; the gas-dynamic solvers;
 * self-gravity with particles; the single-face entry points.  Prints one
 * checksum line; any sanitizer report makes the run fail.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "orc.h"

static unsigned long long lcg = 88172645463325252ull;
static double urand(void) {
  lcg = lcg * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(lcg >> 11) * (1.0 / 9007199254740992.0);
}

/* Smooth-ish random state with a divergence-free field from edge vector
   potentials (so the oracle accepts it under any boundary kinds). */
static void make_state(const orc_config *c, double *cell5, double *bx, double *by, double *bz) {
  const int nx = c->nx, ny = c->ny, nz = c->nz;
  const int ox = c->bc[0] != ORC_BC_PERIODIC, oy = c->bc[2] != ORC_BC_PERIODIC,
            oz = c->bc[4] != ORC_BC_PERIODIC;
  const long nc = (long)nx * ny * nz;
  double *az = calloc((size_t)(nx + 2) * (ny + 2) * (nz + 2), sizeof(double));
  int i, j, k;
  for (k = 0; k < nz + 2; ++k)
    for (j = 0; j < ny + 2; ++j)
      for (i = 0; i < nx + 2; ++i)
        az[((long)k * (ny + 2) + j) * (nx + 2) + i] =
            0.05 * sin(0.7 * i + 0.3 * j) * cos(0.5 * k) * c->dx;
#define AZ(i, j, k) az[((long)(k) * (ny + 2) + (j)) * (nx + 2) + (i)]
  for (k = 0; k < nz; ++k)
    for (j = 0; j < ny; ++j)
      for (i = 0; i < nx + ox; ++i)
        bx[((long)k * ny + j) * (nx + ox) + i] = 0.6 + (AZ(i, j + 1, k) - AZ(i, j, k)) / c->dy;
  for (k = 0; k < nz; ++k)
    for (j = 0; j < ny + oy; ++j)
      for (i = 0; i < nx; ++i)
        by[((long)k * (ny + oy) + j) * nx + i] = 0.3 - (AZ(i + 1, j, k) - AZ(i, j, k)) / c->dx;
  for (k = 0; k < nz + oz; ++k)
    for (j = 0; j < ny; ++j)
      for (i = 0; i < nx; ++i) bz[((long)k * ny + j) * nx + i] = -0.2;
#undef AZ
  free(az);
  for (k = 0; k < nz; ++k)
    for (j = 0; j < ny; ++j)
      for (i = 0; i < nx; ++i) {
        const long q = ((long)k * ny + j) * nx + i;
        const double rho = 1.0 + 0.3 * urand(), p = 0.5 + 0.2 * urand();
        const double v[3] = {0.3 * (urand() - 0.5), 0.3 * (urand() - 0.5), 0.3 * (urand() - 0.5)};
        /* a generous energy: P stays positive whatever the cell-centred B */
        cell5[q] = rho;
        cell5[nc + q] = rho * v[0];
        cell5[2 * nc + q] = rho * v[1];
        cell5[3 * nc + q] = rho * v[2];
        cell5[4 * nc + q] = p / (c->gamma - 1.0) + 0.5 * rho * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) + 0.5;
      }
}

static double run(orc_config c, int nsteps, int mlp, int scal) {
  const long nc = (long)c.nx * c.ny * c.nz;
  const int ox = c.bc[0] != ORC_BC_PERIODIC, oy = c.bc[2] != ORC_BC_PERIODIC,
            oz = c.bc[4] != ORC_BC_PERIODIC;
  const long nbx = (long)c.nz * c.ny * (c.nx + ox), nby = (long)c.nz * (c.ny + oy) * c.nx,
             nbz = (long)(c.nz + oz) * c.ny * c.nx;
  double *cell5 = malloc(sizeof(double) * 5 * nc), *bx = malloc(sizeof(double) * nbx),
         *by = malloc(sizeof(double) * nby), *bz = malloc(sizeof(double) * nbz);
  double sum = 0.0;
  orc_grid *g;
  int s;
  make_state(&c, cell5, bx, by, bz);
  g = orc_create(&c);
  if (!g || orc_set_state(g, cell5, bx, by, bz) != 0) {
    fprintf(stderr, "oracle rejected the state\n");
    exit(2);
  }
  if (mlp) {
    double *par = malloc(sizeof(double) * 6792);
    for (s = 0; s < 6792; ++s) par[s] = 0.05 * (urand() - 0.5);
    orc_set_mlp(g, par, 0.5, 0.5, 0.1);
    free(par);
  }
  if (scal) {
    double *x = malloc(sizeof(double) * c.nscalar * nc);
    for (s = 0; s < c.nscalar * nc; ++s) x[s] = urand();
    orc_set_scalars(g, x);
    orc_get_scalars(g, x);
    sum += x[0];
    free(x);
  }
  if (c.npart > 0) {
    const long n = c.npart;
    double *x = malloc(sizeof(double) * 3 * n), *v = malloc(sizeof(double) * 3 * n),
           *m = malloc(sizeof(double) * n), *rho = malloc(sizeof(double) * nc);
    long q;
    for (q = 0; q < n; ++q) {
      x[q] = c.x0 + urand() * c.nx * c.dx;
      x[n + q] = c.y0 + urand() * c.ny * c.dy;
      x[2 * n + q] = c.z0 + urand() * c.nz * c.dz;
      v[q] = v[n + q] = v[2 * n + q] = 0.1 * (urand() - 0.5);
      m[q] = 1.0 / n;
    }
    orc_set_particles(g, x, v, m);
    orc_particle_deposit(g, x, rho);
    orc_particle_interp(g, rho, x, n, m);
    sum += rho[0] + m[0];
    free(x);
    free(v);
    free(m);
    free(rho);
  }
  for (s = 0; s < nsteps; ++s) sum += orc_step(g, 0.0);
  {
    orc_diag d;
    orc_diag_get(g, &d);
    sum += d.mass + d.energy + d.divb_max;
    orc_get_state(g, cell5, bx, by, bz);
    sum += cell5[0] + bx[0] + by[0] + bz[0];
  }
  {
    const long np = orc_padded_size(g);
    double *a = malloc(sizeof(double) * np);
    int w;
    for (w = 0; w < 35; ++w)
      if (orc_debug_array(g, w, a) > 0) sum += a[np / 2];
    free(a);
  }
  orc_destroy(g);
  free(cell5);
  free(bx);
  free(by);
  free(bz);
  return sum;
}

int main(void) {
  double sum = 0.0;
  orc_config c;
  int a, q;
  memset(&c, 0, sizeof c);
  c.nx = 13;
  c.ny = 9;
  c.nz = 7;
  c.dx = c.dy = c.dz = 0.1;
  c.gamma = 5.0 / 3.0;
  c.cfl = 0.4;
  c.kappa = 1.0 / 3.0;
  /* disc potential, floors, x periodic, y outflow, z inflow */
  c.bc[0] = c.bc[1] = ORC_BC_PERIODIC;
  c.bc[2] = c.bc[3] = ORC_BC_OUTFLOW;
  c.bc[4] = c.bc[5] = ORC_BC_INFLOW;
  c.inflow[0] = 1.0; c.inflow[1] = 0.1; c.inflow[2] = -0.05; c.inflow[3] = 0.02;
  c.inflow[4] = 0.6; c.inflow[5] = 0.6; c.inflow[6] = 0.3; c.inflow[7] = -0.2;
  c.x0 = -0.6; c.y0 = -0.4; c.z0 = -0.3;
  c.source = ORC_SRC_LOGPOT;
  c.src[0] = 1.0; c.src[1] = 0.5; c.src[2] = 0.8;
  c.rho_floor = 0.9; c.p_floor = 0.55;
  sum += run(c, 3, 0, 0);
  /* the other potentials, both MUSCL forms, first order, scalars, learned correction */
  c.rho_floor = c.p_floor = 0.0;
  c.source = ORC_SRC_GAUSS_X; c.src[0] = 0.5; c.src[1] = 0.3;
  c.recon = ORC_RECON_KAPPA;
  c.nscalar = 3;
  sum += run(c, 2, 1, 1);
  c.nscalar = 0;
  c.source = ORC_SRC_UNIFORM; c.src[0] = 0.1; c.src[1] = -0.2; c.src[2] = 0.05;
  c.recon = ORC_RECON_FIRST;
  sum += run(c, 2, 0, 0);
  /* gas-dynamic solvers, all outflow */
  c.source = ORC_SRC_NONE;
  c.recon = ORC_RECON_PAPER;
  for (a = 0; a < 6; ++a) c.bc[a] = ORC_BC_OUTFLOW;
  for (q = ORC_RIEMANN_HLL; q <= ORC_RIEMANN_HLLC; ++q) {
    c.riemann = q;
    sum += run(c, 2, 0, 0);
  }
  c.riemann = ORC_RIEMANN_HLLD;
  /* self-gravity with particles on a periodic power-of-two box */
  for (a = 0; a < 6; ++a) c.bc[a] = ORC_BC_PERIODIC;
  c.nx = 16; c.ny = 8; c.nz = 4;
  c.source = ORC_SRC_SELF_GRAVITY; c.src[0] = 1.0; c.src[1] = 0.0;
  c.npart = 50;
  sum += run(c, 2, 0, 0);
  /* single-face entry points */
  for (q = 0; q < 1000; ++q) {
    double wl[7], wr[7], f[7], w4[4], l, r;
    for (a = 0; a < 7; ++a) {
      wl[a] = a == 0 || a == 4 ? 0.1 + urand() : urand() - 0.5;
      wr[a] = a == 0 || a == 4 ? 0.1 + urand() : urand() - 0.5;
    }
    orc_hlld(wl, wr, urand() - 0.5, 5.0 / 3.0, f);
    sum += f[q % 7];
    orc_hll(wl, wr, urand() - 0.5, 5.0 / 3.0, f);
    sum += f[q % 7];
    orc_hllc(wl, wr, 0.0, 1.4, f);
    sum += f[q % 7];
    for (a = 0; a < 4; ++a) w4[a] = urand();
    orc_recon(w4, q % 3, 1.0 / 3.0, &l, &r);
    sum += l + r;
  }
  printf("checksum %.17g\n", sum);
  return isfinite(sum) ? 0 : 1;
}
