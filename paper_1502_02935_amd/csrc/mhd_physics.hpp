// mhd_physics.hpp -- device functions of one face: minmod-limited MUSCL
// reconstruction (Eq. 12-14) and the HLLD approximate Riemann solver
// (Miyoshi & Kusano 2005, the MHD solver of section 2.1), templated on the
// arithmetic type (double, or float for the FP32 bulk path).
//
// A face state is given in the face-normal frame (n, t1, t2) with
// (n, t1, t2) a cyclic permutation of (x, y, z):
//   w = rho, vn, vt1, vt2, P, Bt1, Bt2   plus the face-normal field Bn.
// The flux is returned in the same frame: rho, Mn, Mt1, Mt2, E, Bt1, Bt2
// (the Bn flux is identically zero, Eq. 3).
//
// Divisions are grouped so that each denominator is inverted once.  In FP32
// the reciprocal and the square root are the hardware v_rcp_f32 and
// v_sqrt_f32 (1 ulp each); in FP64 both are correctly rounded.  a*b+c is
// contracted to an FMA only within one expression (fp contract(on)), so a
// face gives bitwise the same flux in every kernel that computes it (the
// faces at index n of a periodic axis, computed by the outer-layer pass,
// must equal the faces at 0 from the sweep).
#pragma once

#include <hip/hip_runtime.h>

namespace mhd {

// Relative size (to the star total pressure) below which an HLLD star-state
// denominator rho (S - u)(S - S_M) - Bn^2 is treated as zero: the outer
// fast-speed estimate meets the star-region Alfven speed and the star
// transverse v and B formulas diverge (their v*.B* term like 1/den^2, the
// energy flux like 1/den).  Same constant in both precisions; it sits far
// above the FP32 rounding level of den.
constexpr double kDegenerate = 1.0e-3;

__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float root(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double root(double x) { return sqrt(x); }
// q = sqrt(x) and iq = 1/sqrt(x): in FP32 from the hardware v_rsq_f32.
__device__ __forceinline__ void root_pair(float x, float& q, float& iq) {
  iq = __builtin_amdgcn_rsqf(x);
  q = x * iq;
}
__device__ __forceinline__ void root_pair(double x, double& q, double& iq) {
  q = sqrt(x);
  iq = 1.0 / q;
}

template <class T>
struct Face {
  T d, vn, vt1, vt2, p, bt1, bt2;
};

// minmod(a, b): the argument of smaller magnitude when both share a strict
// sign, else zero -- which is the median of (a, b, 0).
__device__ __forceinline__ float minmod(float a, float b) {
  return __builtin_amdgcn_fmed3f(a, b, 0.0f);
}
__device__ __forceinline__ double minmod(double a, double b) {
  return fmax(fmin(a, b), fmin(fmax(a, b), 0.0));
}

// Coefficients of dW = cA mm(dw_back, bA dw_mid) + cB mm(dw_mid, bB dw_back).
template <class T>
struct Muscl {
  T cA, bA, cB, bB;
  int first_order;
};

// Left/right interface values at the face between cells 1 and 2 of the
// stencil w0..w3 (Eq. 12-14), limited (the caller knows the stage is not
// first order).
template <class T>
__device__ __forceinline__ void muscl_lr_limited(const Muscl<T>& m, T w0, T w1, T w2, T w3,
                                                 T& wl, T& wr) {
#pragma clang fp contract(on)
  const T back = w1 - w0, mid = w2 - w1, fwd = w3 - w2;
  const T dl = m.cA * minmod(back, m.bA * mid) + m.cB * minmod(mid, m.bB * back);
  const T dr = m.cA * minmod(fwd, m.bA * mid) + m.cB * minmod(mid, m.bB * fwd);
  wl = w1 + dl;
  wr = w2 - dr;
}

// The same with the run-time choice of first order (m.first_order: the
// interface values are the two cell values).
template <class T>
__device__ __forceinline__ void muscl_lr(const Muscl<T>& m, T w0, T w1, T w2, T w3, T& wl,
                                         T& wr) {
#pragma clang fp contract(on)
  if (m.first_order) {
    wl = w1;
    wr = w2;
    return;
  }
  const T back = w1 - w0, mid = w2 - w1, fwd = w3 - w2;
  const T dl = m.cA * minmod(back, m.bA * mid) + m.cB * minmod(mid, m.bB * back);
  const T dr = m.cA * minmod(fwd, m.bA * mid) + m.cB * minmod(mid, m.bB * fwd);
  wl = w1 + dl;
  wr = w2 - dr;
}

// Fast magnetosonic speed along n; the discriminant is written as
// (a^2 - b^2)^2 + 4 a^2 bt^2 so it never goes negative by cancellation.
template <class T>
__device__ __forceinline__ T fast_speed_id(T id, T p, T bn, T bt1, T bt2, T gam) {
#pragma clang fp contract(on)
  const T a2 = gam * p * id;
  const T bt2s = (bt1 * bt1 + bt2 * bt2) * id;
  const T b2 = bt2s + bn * bn * id;
  const T q = a2 - b2;
  return root(T(0.5) * ((a2 + b2) + root(q * q + T(4) * a2 * bt2s)));
}
// The same from the density d itself (id = 1/d).
template <class T>
__device__ __forceinline__ T fast_speed(T d, T p, T bn, T bt1, T bt2, T gam) {
  return fast_speed_id(rcp(d), p, bn, bt1, bt2, gam);
}

// Conserved vector and physical flux (Eq. 3) of a face state; igm1 =
// 1/(gamma - 1).
template <class T>
__device__ __forceinline__ void cons_flux(const Face<T>& s, T bn, T igm1, T u[7], T f[7]) {
#pragma clang fp contract(on)
  const T v2 = s.vn * s.vn + s.vt1 * s.vt1 + s.vt2 * s.vt2;
  const T b2 = bn * bn + s.bt1 * s.bt1 + s.bt2 * s.bt2;
  const T pt = s.p + T(0.5) * b2;
  const T vb = s.vn * bn + s.vt1 * s.bt1 + s.vt2 * s.bt2;
  u[0] = s.d;
  u[1] = s.d * s.vn;
  u[2] = s.d * s.vt1;
  u[3] = s.d * s.vt2;
  u[4] = s.p * igm1 + T(0.5) * s.d * v2 + T(0.5) * b2;
  u[5] = s.bt1;
  u[6] = s.bt2;
  f[0] = u[1];
  f[1] = u[1] * s.vn + pt - bn * bn;
  f[2] = u[1] * s.vt1 - bn * s.bt1;
  f[3] = u[1] * s.vt2 - bn * s.bt2;
  f[4] = (u[4] + pt) * s.vn - vb * bn;
  f[5] = s.bt1 * s.vn - bn * s.vt1;
  f[6] = s.bt2 * s.vn - bn * s.vt2;
}

// Star state of one side: density, transverse v and B, energy, v.B.
template <class T>
struct Star {
  T d, v1, v2, b1, b2, e, vb;
};

// HLL flux (Harten, Lax & van Leer): one intermediate state between the
// outer waves, with the outer speeds of the HLLD solver.
template <class T>
__device__ __forceinline__ int hll(const Face<T>& L, const Face<T>& R, T bn, T gam, T igm1,
                                   T f[7]) {
#pragma clang fp contract(on)
  T ul[7], fl[7], ur[7], fr[7];
  cons_flux(L, bn, igm1, ul, fl);
  cons_flux(R, bn, igm1, ur, fr);
  const T cfl = fast_speed(L.d, L.p, bn, L.bt1, L.bt2, gam);
  const T cfr = fast_speed(R.d, R.p, bn, R.bt1, R.bt2, gam);
  const T cmax = cfl > cfr ? cfl : cfr;
  const T SL = (L.vn < R.vn ? L.vn : R.vn) - cmax;
  const T SR = (L.vn > R.vn ? L.vn : R.vn) + cmax;
  if (SL > T(0)) {
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] = fl[m];
  } else if (SR < T(0)) {
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] = fr[m];
  } else {
    const T inv = rcp(SR - SL);
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] = (SR * fl[m] - SL * fr[m] + SL * SR * (ur[m] - ul[m])) * inv;
  }
  return 0;
}

// HLLC flux of pure gas dynamics (Toro, Spruce & Speares): the field is
// taken to be zero, so the B components of the flux are zero; outer speeds
// from the sound speeds, the contact speed S* from the two outer jump
// conditions, star states of equal pressure and normal velocity.
template <class T>
__device__ __forceinline__ int hllc(const Face<T>& L0, const Face<T>& R0, T gam, T igm1, T f[7]) {
#pragma clang fp contract(on)
  const Face<T> L{L0.d, L0.vn, L0.vt1, L0.vt2, L0.p, T(0), T(0)};
  const Face<T> R{R0.d, R0.vn, R0.vt1, R0.vt2, R0.p, T(0), T(0)};
  T ul[7], fl[7], ur[7], fr[7];
  cons_flux(L, T(0), igm1, ul, fl);
  cons_flux(R, T(0), igm1, ur, fr);
  const T cl = root(gam * L.p * rcp(L.d)), cr = root(gam * R.p * rcp(R.d));
  const T cmax = cl > cr ? cl : cr;
  const T SL = (L.vn < R.vn ? L.vn : R.vn) - cmax;
  const T SR = (L.vn > R.vn ? L.vn : R.vn) + cmax;
  if (SL > T(0)) {
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] = fl[m];
    return 0;
  }
  if (SR < T(0)) {
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] = fr[m];
    return 0;
  }
  const T ml = L.d * (SL - L.vn), mr = R.d * (SR - R.vn);
  const T Ss = (R.p - L.p + ml * L.vn - mr * R.vn) * rcp(ml - mr);
  const bool left = Ss >= T(0);
  const Face<T>& w = left ? L : R;
  const T S = left ? SL : SR;
  const T e = left ? ul[4] : ur[4];
  const T sv = S - w.vn;
  const T fac = w.d * sv * rcp(S - Ss);
  const T us[5] = {fac, fac * Ss, fac * w.vt1, fac * w.vt2,
                   fac * (e * rcp(w.d) + (Ss - w.vn) * (Ss + w.p * rcp(w.d * sv)))};
#pragma unroll
  for (int m = 0; m < 5; ++m) f[m] = (left ? fl[m] : fr[m]) + S * (us[m] - (left ? ul[m] : ur[m]));
  f[5] = T(0);
  f[6] = T(0);
  return 0;
}

// Star state of one side without its energy: density, transverse v and B
// (the energy is needed for the side whose flux is returned only).
template <class T>
__device__ __forceinline__ Star<T> star_base(const Face<T>& s, T bn, T S, T SM, T pts,
                                             int& degenerate) {
#pragma clang fp contract(on)
  Star<T> r;
  const T sv = S - s.vn;
  const T ism = rcp(S - SM);
  const T dsv = s.d * sv;
  r.d = dsv * ism;
  const T den = dsv * (S - SM) - bn * bn;
  if (fabs(den) > T(kDegenerate) * pts) {
    const T iden = rcp(den);
    const T kv = bn * (SM - s.vn) * iden;
    const T kb = (dsv * sv - bn * bn) * iden;
    r.v1 = s.vt1 - s.bt1 * kv;
    r.v2 = s.vt2 - s.bt2 * kv;
    r.b1 = s.bt1 * kb;
    r.b2 = s.bt2 * kb;
  } else {
    r.v1 = s.vt1;
    r.v2 = s.vt2;
    r.b1 = s.bt1;
    r.b2 = s.bt2;
    degenerate = 1;
  }
  r.e = T(0);
  r.vb = T(0);
  return r;
}

// HLLD flux (igm1 = 1/(gamma - 1)).  Returns bit0 if the HLL flux was used
// (S_M outside (S_L, S_R)), bit1 if a star state was degenerate.  The side
// whose conserved state and flux enter the result -- the upwind side of a
// supersonic face, else the side of the contact the face lies on -- is
// picked before any flux is formed, so each face forms one physical flux
// (both only when it falls back to HLL).
template <class T>
__device__ __forceinline__ int hlld(const Face<T>& L, const Face<T>& R, T bn, T gam, T igm1,
                                    T f[7]) {
#pragma clang fp contract(on)
  const T cfl = fast_speed(L.d, L.p, bn, L.bt1, L.bt2, gam);
  const T cfr = fast_speed(R.d, R.p, bn, R.bt1, R.bt2, gam);
  const T cmax = cfl > cfr ? cfl : cfr;
  const T SL = (L.vn < R.vn ? L.vn : R.vn) - cmax;
  const T SR = (L.vn > R.vn ? L.vn : R.vn) + cmax;
  const T ptl = L.p + T(0.5) * (bn * bn + L.bt1 * L.bt1 + L.bt2 * L.bt2);
  const T ptr = R.p + T(0.5) * (bn * bn + R.bt1 * R.bt1 + R.bt2 * R.bt2);
  const T al = L.d * (SL - L.vn);
  const T ar = R.d * (SR - R.vn);
  const T ia = rcp(ar - al);
  const T SM = (ar * R.vn - al * L.vn - ptr + ptl) * ia;
  const T pts = (ar * ptl - al * ptr + al * ar * (R.vn - L.vn)) * ia;
  const bool sup = SL > T(0) || SR < T(0);
  const bool left = sup ? SL > T(0) : SM >= T(0);
  const Face<T> w = left ? L : R;
  T u0[7], f0[7];
  cons_flux(w, bn, igm1, u0, f0);
  if (sup) {
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] = f0[m];
    return 0;
  }
  if (!(SL < SM && SM < SR)) {
    T uo[7], fo[7];
    cons_flux(left ? R : L, bn, igm1, uo, fo);
    const T inv = rcp(SR - SL);
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      const T ul = left ? u0[m] : uo[m], ur = left ? uo[m] : u0[m];
      const T fl = left ? f0[m] : fo[m], fr = left ? fo[m] : f0[m];
      f[m] = (SR * fl - SL * fr + SL * SR * (ur - ul)) * inv;
    }
    return 1;
  }
  int deg = 0;
  const Star<T> sl = star_base(L, bn, SL, SM, pts, deg);
  const Star<T> sr = star_base(R, bn, SR, SM, pts, deg);
  T ql, qr, iql, iqr;
  root_pair(sl.d, ql, iql);
  root_pair(sr.d, qr, iqr);
  const T abn = fabs(bn);
  const T SsL = SM - abn * iql;
  const T SsR = SM + abn * iqr;
  const T S = left ? SL : SR;
  Star<T> s = left ? sl : sr;
  {  // the chosen side's star energy and v*.B*
    const T sv = S - w.vn;
    const T ism = rcp(S - SM);
    const T pt = w.p + T(0.5) * (bn * bn + w.bt1 * w.bt1 + w.bt2 * w.bt2);
    const T vb = w.vn * bn + w.vt1 * w.bt1 + w.vt2 * w.bt2;
    s.vb = SM * bn + s.v1 * s.b1 + s.v2 * s.b2;
    s.e = (sv * u0[4] - pt * w.vn + pts * SM + bn * (vb - s.vb)) * ism;
  }
  // F*_a = F_a + S_a (U*_a - U_a)
  const T us[7] = {s.d, s.d * SM, s.d * s.v1, s.d * s.v2, s.e, s.b1, s.b2};
#pragma unroll
  for (int m = 0; m < 7; ++m) f[m] = f0[m] + S * (us[m] - u0[m]);
  const bool inner = left ? (SsL < T(0)) : (SsR < T(0) ? false : true);
  if (inner) {
    // double-star state across the rotational discontinuity on this side
    const T sg = bn > T(0) ? T(1) : (bn < T(0) ? T(-1) : T(0));
    const T inv = rcp(ql + qr);
    const T v1 = (ql * sl.v1 + qr * sr.v1 + sg * (sr.b1 - sl.b1)) * inv;
    const T v2 = (ql * sl.v2 + qr * sr.v2 + sg * (sr.b2 - sl.b2)) * inv;
    const T b1 = (qr * sl.b1 + ql * sr.b1 + sg * ql * qr * (sr.v1 - sl.v1)) * inv;
    const T b2 = (qr * sl.b2 + ql * sr.b2 + sg * ql * qr * (sr.v2 - sl.v2)) * inv;
    const T vb = SM * bn + v1 * b1 + v2 * b2;
    const T ess = left ? (s.e - ql * sg * (s.vb - vb)) : (s.e + qr * sg * (s.vb - vb));
    const T Ss = left ? SsL : SsR;
    const T uss[7] = {s.d, s.d * SM, s.d * v1, s.d * v2, ess, b1, b2};
#pragma unroll
    for (int m = 0; m < 7; ++m) f[m] += Ss * (uss[m] - us[m]);
  }
  return deg ? 2 : 0;
}

}  // namespace mhd
