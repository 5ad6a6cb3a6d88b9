// mhd_source.hpp -- the source S of the conservation law at a cell centre
// (section 2.1: the gravity of a fixed potential or of the self-gravity
// solve): momentum -rho grad Phi, energy -rho v . grad Phi.
#pragma once

#include "mhd_kernels.hpp"

namespace mhd {

// grad Phi of the fixed potentials at (x, y, z): 1 logarithmic (v0, rc, q),
// 2 uniform field, 3 Gaussian well along x (depth A, width wd).
__device__ __forceinline__ void grad_phi(const Physics& ph, double x, double y, double z,
                                         double gp[3]) {
  gp[0] = gp[1] = gp[2] = 0.0;
  if (ph.source == 1) {
    const double v0 = ph.src[0], rc = ph.src[1], q = ph.src[2];
    const double den = rc * rc + x * x + y * y + z * z / (q * q);
    gp[0] = v0 * v0 * x / den;
    gp[1] = v0 * v0 * y / den;
    gp[2] = v0 * v0 * (z / (q * q)) / den;
  } else if (ph.source == 2) {
    gp[0] = ph.src[0];
    gp[1] = ph.src[1];
    gp[2] = ph.src[2];
  } else if (ph.source == 3) {
    const double A = ph.src[0], wd = ph.src[1];
    gp[0] = 2.0 * A * x / (wd * wd) * exp(-(x / wd) * (x / wd));
  }
}

// S (global components rho, Mx, My, Mz, E) of cell (i, j, k) at point p from
// the stage's density and velocity there; zero without a source.
template <class T>
__device__ __forceinline__ void cell_source(const Geo& g, const Physics& ph, const Grav<T>& gr,
                                            int i, int j, int k, int p, T rho, T vx, T vy, T vz,
                                            T S[5]) {
  S[0] = S[1] = S[2] = S[3] = S[4] = T(0);
  if (ph.source == 0) return;
  double gp[3];
  if (ph.source == 4 && ph.src[1] == 1.0) {  // gas decoupled from gravity
    gp[0] = gp[1] = gp[2] = 0.0;
  } else if (ph.source == 4) {
    gp[0] = gr.g[0][p];
    gp[1] = gr.g[1][p];
    gp[2] = gr.g[2][p];
  } else {
    grad_phi(ph, g.x0[0] + (i + 0.5) * g.d[0], g.x0[1] + (j + 0.5) * g.d[1],
             g.x0[2] + (k + 0.5) * g.d[2], gp);
  }
  const T gx = (T)gp[0], gy = (T)gp[1], gz = (T)gp[2];
  S[1] = -rho * gx;
  S[2] = -rho * gy;
  S[3] = -rho * gz;
  S[4] = -rho * (vx * gx + vy * gy + vz * gz);
}

}  // namespace mhd
