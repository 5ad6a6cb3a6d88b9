// abi_driver.cpp -- drives the host side of the C ABI (include/mhd.h) under
// the address and undefined-behaviour sanitizers (host code only; built and
// run by tests/test_sanitizers.py, no GPU needed): the configuration
// checks of mhd_workspace_bytes for valid and invalid configurations of
// every kind, the workspace arithmetic, the error strings and the argument
// checks that every entry point makes before it touches the device.
#include <stdio.h>
#include <string.h>

#include "mhd.h"

static int failures = 0;
#define EXPECT(cond)                                                 \
  do {                                                               \
    if (!(cond)) {                                                   \
      fprintf(stderr, "line %d: expectation failed: %s\n", __LINE__, #cond); \
      ++failures;                                                    \
    }                                                                \
  } while (0)

static mhd_config base() {
  mhd_config c;
  memset(&c, 0, sizeof c);
  c.nx = 16;
  c.ny = 8;
  c.nz = 4;
  c.dx = c.dy = c.dz = 0.1;
  c.gamma = 5.0 / 3.0;
  c.cfl = 0.4;
  c.kappa = 1.0 / 3.0;
  return c;
}

int main() {
  EXPECT(mhd_abi_version() == MHD_ABI_VERSION);
  for (int code = -8; code <= 2; ++code) EXPECT(mhd_strerror(code) && mhd_strerror(code)[0]);
  size_t n = 0, n64 = 0, n32 = 0;
  mhd_config c = base();
  EXPECT(mhd_workspace_bytes(&c, &n64) == MHD_OK && n64 > 0 && n64 % 256 == 0);
  c.precision = MHD_FP32;
  EXPECT(mhd_workspace_bytes(&c, &n32) == MHD_OK && n32 < n64);
  c.recovery = MHD_RECOVERY_OFF;
  EXPECT(mhd_workspace_bytes(&c, &n) == MHD_OK);
  // every boundary kind, solver, reconstruction and source
  for (int bc = MHD_BC_PERIODIC; bc <= MHD_BC_INFLOW; ++bc)
    for (int rs = MHD_RIEMANN_HLLD; rs <= MHD_RIEMANN_HLLC; ++rs)
      for (int rc = MHD_RECON_PAPER; rc <= MHD_RECON_FIRST; ++rc)
        for (int src = MHD_SRC_NONE; src <= MHD_SRC_GAUSS_X; ++src) {
          mhd_config d = base();
          for (int a = 0; a < 6; ++a) d.bc[a] = bc;
          d.riemann = rs;
          d.recon = rc;
          d.source = src;
          d.nscalar = (bc + rs + rc) % (MHD_MAX_SCALARS + 1);
          EXPECT(mhd_workspace_bytes(&d, &n) == MHD_OK && n >= n64);
        }
  {  // self-gravity with particles on a periodic power-of-two box
    mhd_config d = base();
    d.source = MHD_SRC_SELF_GRAVITY;
    d.src[0] = 1.0;
    d.npart = 12345;
    EXPECT(mhd_workspace_bytes(&d, &n) == MHD_OK && n > n64);
  }
  // invalid configurations
  {
    mhd_config bad[24];
    int k = 0;
    for (int q = 0; q < 24; ++q) bad[q] = base();
    bad[k++].nx = 0;
    bad[k++].ny = -3;
    bad[k++].dx = 0.0;
    bad[k++].gamma = 1.0;
    bad[k++].cfl = 0.0;
    bad[k++].cfl = 1.5;
    bad[k++].precision = 7;
    bad[k++].recon = 9;
    bad[k++].kappa = 1.0;
    bad[k++].source = 11;
    bad[k++].rho_floor = -1.0;
    bad[k].bc[0] = MHD_BC_PERIODIC, bad[k++].bc[1] = MHD_BC_OUTFLOW;
    bad[k++].bc[2] = 9;
    bad[k++].nscalar = MHD_MAX_SCALARS + 1;
    bad[k++].npart = 10;  // particles need self-gravity
    bad[k++].reserved = 1;
    bad[k++].recovery = 5;
    bad[k++].recovery = MHD_RECOVERY_OFF;  // FP64 has no recovery to switch off
    bad[k].nx = 2048, bad[k].ny = 2048, bad[k++].nz = 1024;
    bad[k].source = MHD_SRC_SELF_GRAVITY, bad[k++].nx = 24;  // not a power of two
    for (int q = 0; q < k; ++q) EXPECT(mhd_workspace_bytes(&bad[q], &n) == MHD_E_ARG);
  }
  EXPECT(mhd_workspace_bytes(&c, nullptr) == MHD_E_ARG);
  EXPECT(mhd_workspace_bytes(nullptr, &n) == MHD_E_ARG);
  // entry points with a null context or null buffers
  mhd_ctx* ctx = nullptr;
  mhd_diag_t dg;
  double dt = 0.0;
  EXPECT(mhd_init(&c, nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, &ctx) == MHD_E_ARG);
  EXPECT(mhd_step(nullptr, nullptr, 1) == MHD_E_ARG);
  EXPECT(mhd_dt(nullptr, &dt) == MHD_E_ARG);
  EXPECT(mhd_diag(nullptr, &dg) == MHD_E_ARG);
  EXPECT(mhd_get_state(nullptr, nullptr, nullptr, nullptr, nullptr) == MHD_E_ARG);
  EXPECT(mhd_set_scalars(nullptr, nullptr) == MHD_E_ARG);
  EXPECT(mhd_get_scalars(nullptr, nullptr) == MHD_E_ARG);
  EXPECT(mhd_set_particles(nullptr, nullptr, nullptr, nullptr) == MHD_E_ARG);
  EXPECT(mhd_get_particles(nullptr, nullptr, nullptr) == MHD_E_ARG);
  EXPECT(mhd_set_full_fluxes(nullptr, 1) == MHD_E_ARG);
  EXPECT(mhd_debug_array(nullptr, 0, nullptr, &n) == MHD_E_ARG);
  EXPECT(mhd_profile(nullptr, 1) == MHD_E_ARG);
  EXPECT(mhd_profile_get(nullptr, nullptr) == MHD_E_ARG);
  EXPECT(mhd_set_mlp(nullptr, nullptr, nullptr) == MHD_E_ARG);
  EXPECT(mhd_flux_accumulate(nullptr, nullptr) == MHD_E_ARG);
  EXPECT(mhd_coarsen(nullptr, nullptr, nullptr, nullptr, nullptr) == MHD_E_ARG);
  EXPECT(mhd_mlp_samples(nullptr, nullptr, 1.0, 0, nullptr, nullptr, nullptr, nullptr) ==
         MHD_E_ARG);
  EXPECT(mhd_destroy(nullptr) == MHD_E_ARG);
  EXPECT(mhd_mlp_grad_workspace_bytes(0, &n) == MHD_E_ARG);
  EXPECT(mhd_mlp_grad_workspace_bytes(1000, &n) == MHD_OK && n > 0);
  EXPECT(mhd_mlp_forward(-1, nullptr, nullptr, nullptr, nullptr) == MHD_E_ARG);
  EXPECT(mhd_mlp_forward(0, nullptr, nullptr, nullptr, nullptr) == MHD_OK);
  EXPECT(mhd_mlp_grad(0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr) ==
         MHD_E_ARG);
  EXPECT(mhd_mlp_adam(nullptr, nullptr, nullptr, nullptr, 1, 1e-3, 0.9, 0.999, 1e-8, nullptr) ==
         MHD_E_ARG);
  EXPECT(mhd_hlld_batch(MHD_FP64, -1, nullptr, nullptr, nullptr, 1.4, nullptr, nullptr,
                        nullptr) == MHD_E_ARG);
  EXPECT(mhd_hlld_batch(5, 1, nullptr, nullptr, nullptr, 1.4, nullptr, nullptr, nullptr) ==
         MHD_E_ARG);
  EXPECT(mhd_hlld_batch(MHD_FP32, 0, nullptr, nullptr, nullptr, 1.4, nullptr, nullptr,
                        nullptr) == MHD_OK);
  EXPECT(mhd_recon_batch(MHD_FP64, 1, nullptr, 0, 0.3, nullptr, nullptr, nullptr) == MHD_E_ARG);
  EXPECT(mhd_recon_batch(MHD_FP32, 0, nullptr, 0, 0.3, nullptr, nullptr, nullptr) == MHD_OK);
  printf("abi host checks: %d failures\n", failures);
  return failures ? 1 : 0;
}
