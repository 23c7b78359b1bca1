// hydro_device.hpp -- device-side arithmetic shared by the forward and the
// adjoint kernels of libhydro: ghost-cell maps, conserved->primitive recovery,
// flux splitting, the WENO7 reconstruction, jet helpers.
#pragma once

#include <hip/hip_runtime.h>

#include "hydro_internal.hpp"

namespace hydro {

// ---------------------------------------------------------------------------
// Ghost-cell index map: outflow = copy of the edge cell, periodic = wrap.
__device__ __forceinline__ int map_idx(int p, int n, int bc) {
  if (bc) {
    int r = p % n;
    return r < 0 ? r + n : r;
  }
  return min(max(p, 0), n - 1);
}

template <class R>
__device__ __forceinline__ void load5(const R* __restrict__ W, long long nc, long long cell, R u[5]) {
#pragma unroll
  for (int c = 0; c < 5; ++c) u[c] = W[c * nc + cell];
}

// ---------------------------------------------------------------------------
// Reciprocal for FP64: hardware estimate, two Newton steps (quadratic
// convergence from the estimate's ~23 bits to full precision).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

// num / den from one reciprocal plus a residual correction: the estimate
// (~23 bits) after one Newton step (~46 bits) gives q = num r to ~2^-46, and
// q + (num - den q) r squares that error away (below the rounding of q).
__device__ __forceinline__ double div_nr(double num, double den) {
  double r = __builtin_amdgcn_rcp(den);
  r = fma(fma(-den, r, 1.0), r, r);
  const double q = num * r;
  return fma(fma(-den, q, num), r, q);
}

// sqrt(x) for normal x > 0: reciprocal square root estimate, two coupled
// Newton iterations for sqrt(x) and 1/(2 sqrt(x)), one residual correction.
__device__ __forceinline__ double sqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  return fma(fma(-g, g, x), h, g);
}

// Conserved -> primitive for p = e/3 (FP64): e = 3(E^2 - M^2)/(E + sqrt(4E^2
// - 3M^2)), v = M/(E + e/3).  Non-admissible cells are fixed up for the
// primitive calculation only (E <= 1e-12: vacuum at rest; |M| >= (1-1e-10) E:
// M rescaled to that speed) and counted.
struct PrimV {
  double e;
  double v[3];
};

__device__ __forceinline__ PrimV c2p(double E, double Mx, double My, double Mz, unsigned& fix) {
  PrimV r;
  if (E <= kEFloor) {
    ++fix;
    r.e = kEFloor;
    r.v[0] = r.v[1] = r.v[2] = 0.0;
    return r;
  }
  double M2 = Mx * Mx + My * My + Mz * Mz;
  if (M2 >= kVCap * kVCap * E * E) {
    ++fix;
    const double sc = kVCap * E / sqrt(M2);
    Mx = Mx * sc;
    My = My * sc;
    Mz = Mz * sc;
    M2 = Mx * Mx + My * My + Mz * Mz;
  }
  const double e = div_nr(3.0 * (E * E - M2), E + sqrt_nr(4.0 * E * E - 3.0 * M2));
  const double iW = rcp_nr(E + e * (1.0 / 3.0));
  r.e = e;
  r.v[0] = Mx * iW;
  r.v[1] = My * iW;
  r.v[2] = Mz * iW;
  return r;
}

template <class R>
__device__ __forceinline__ PrimV c2p(const R u[5], unsigned& fix) {
  return c2p((double)u[0], (double)u[1], (double)u[2], (double)u[3], fix);
}

// Physical flux along axis AX and its Lax-Friedrichs split (alpha = 1):
// f = (M_AX, M_x v_AX + p d_{x,AX}, M_y v_AX + p d_{y,AX}, M_z v_AX + p d_{z,AX}, N v_AX).
template <class R, int AX>
__device__ __forceinline__ void split_flux(const R u[5], const PrimV& p, R Fp[5], R Fm[5]) {
  const R vd = (R)p.v[AX];
  const R pr = (R)(p.e * (1.0 / 3.0));
  R f[5];
  f[0] = u[1 + AX];
  f[1] = (AX == 0) ? u[1] * vd + pr : u[1] * vd;
  f[2] = (AX == 1) ? u[2] * vd + pr : u[2] * vd;
  f[3] = (AX == 2) ? u[3] * vd + pr : u[3] * vd;
  f[4] = u[4] * vd;
#pragma unroll
  for (int c = 0; c < 5; ++c) {  // (f +- u)/2 with one rounding: u/2 is exact
    const R hu = R(0.5) * u[c];
    Fp[c] = fma(R(0.5), f[c], hu);
    Fm[c] = fma(R(0.5), f[c], -hu);
  }
}

// ---------------------------------------------------------------------------
// WENO7 value at x_{i+1/2} from the left, a0..a6 = a_{i-3}..a_{i+3}.
// The candidates q_k of the 4-point stencils enter as 35 d_k (q_k - a_{i}),
// d = (1, 12, 18, 4)/35, written with the first differences, and the result
// is a_i + sum w_k 35 d_k (q_k - a_i) / sum w_k 35 d_k.  Smoothness indicators (Jiang-Shu: the
// integral over cell i of the squared derivatives of stencil k's cubic) are
// evaluated from the nested differences D1, D2, D3 of the stencil values:
//   b_k = s_k^2 + 13/12 c_k^2 + 781/720 D3_k^2 + eps,
//   s_k = D1_k + h_k D2_k + m_k D3_k   (h = 5/2, 3/2, 1/2, -1/2;
//                                        m = 11/6, 1/3, -1/6, 1/3),
//   c_k = D2_k + g_k D3_k             (g = 2, 1, 0, -1),
// so they vanish exactly on flat stencils.  WENO-Z (p = 2):
// w_k = 1 + (tau/b_k)^2, tau = |b0 - b3 + 3(b1 - b2)|; Jiang-Shu: w_k = 1/b_k^2;
// the result is sum w_k d_k q_k / sum w_k d_k.
template <class R>
__device__ __forceinline__ R rcp_approx(R x);
template <>
__device__ __forceinline__ float rcp_approx<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}
template <>
__device__ __forceinline__ double rcp_approx<double>(double x) {
  return 1.0 / x;
}

template <class R>
__device__ __forceinline__ R smoothness(R D1, R D2, R D3, R h, R m, R g, R eps) {
  const R sk = fma(m, D3, fma(h, D2, D1));
  const R ck = (g == R(0)) ? D2 : fma(g, D3, D2);  // g is a literal: no select survives
  return fma(sk, sk, fma(R(13.0 / 12.0) * ck, ck, fma(R(781.0 / 720.0) * D3, D3, eps)));
}

// WENO5 value at x_{i+1/2} from the left, b0..b4 = a_{i-2}..a_{i+2}, in the
// same form as weno7: candidates d_k (q_k - a_i) from first differences
// (d = (1, 6, 3)/10), Jiang-Shu indicators b_k = c1^2 + 13/12 D2^2 + eps with
// c1 = D1 + h_k D2 (h = 3/2, 1/2, -1/2), WENO-Z tau = |b0 - b2|.
template <class R, int S>
__device__ __forceinline__ R weno5(R b0, R b1, R b2, R b3, R b4, R eps) {
  const R e0 = b1 - b0, e1 = b2 - b1, e2 = b3 - b2, e3 = b4 - b3;
  // candidates as 10 d_k (q_k - b2) (the 10 cancels against sum 10 w_k d_k)
  const R r0 = fma(R(5.0 / 6.0), e1, R(-1.0 / 3.0) * e0);
  const R r1 = fma(R(2.0), e2, e1);
  const R r2 = fma(R(-0.5), e3, R(2.0) * e2);
  if (S == kWeno5Linear) return fma((r0 + r1) + r2, R(0.1), b2);
  const R f0 = e1 - e0, f1 = e2 - e1, f2 = e3 - e2;
  const R s0 = fma(R(1.5), f0, e0), s1 = fma(R(0.5), f1, e1), s2 = fma(R(-0.5), f2, e2);
  const R be0 = fma(s0, s0, fma(R(13.0 / 12.0) * f0, f0, eps));
  const R be1 = fma(s1, s1, fma(R(13.0 / 12.0) * f1, f1, eps));
  const R be2 = fma(s2, s2, fma(R(13.0 / 12.0) * f2, f2, eps));
  if (sizeof(R) == 8) {
    // common denominator: with B_k = b_k^2, WENO-Z d_k (B_k + tau^2) prod_{j!=k} B_j,
    // Jiang-Shu d_k prod_{j!=k} B_j
    // (WENO-Z: (B_0 + tau^2) B_1 = B_0 B_1 + tau^2 B_1, and so on.)
    const R B0 = be0 * be0, B1 = be1 * be1, B2 = be2 * be2;
    const R P01 = B0 * B1;
    R A0, A1, A2;
    if (S == kWeno5Z) {
      const R tau = fabs(be0 - be2);
      const R t2 = tau * tau;
      A0 = fma(t2, B1, P01) * B2;
      A1 = fma(t2, B0, P01) * B2;
      A2 = (B2 + t2) * P01;
    } else {
      A0 = B1 * B2;
      A1 = B0 * B2;
      A2 = P01;
    }
    const R num = fma(A2, r2, fma(A1, r1, A0 * r0));
    const R den = fma(A2, R(3.0), fma(A1, R(6.0), A0));
    return b2 + (R)div_nr((double)num, (double)den);
  } else {
    const R i0 = rcp_approx<R>(be0), i1 = rcp_approx<R>(be1), i2 = rcp_approx<R>(be2);
    R w0, w1, w2;
    if (S == kWeno5Z) {
      const R tau = fabs(be0 - be2);
      const R s0z = tau * i0, s1z = tau * i1, s2z = tau * i2;
      w0 = fma(s0z, s0z, R(1));
      w1 = fma(s1z, s1z, R(1));
      w2 = fma(s2z, s2z, R(1));
    } else {
      w0 = i0 * i0;
      w1 = i1 * i1;
      w2 = i2 * i2;
    }
    const R num = fma(w2, r2, fma(w1, r1, w0 * r0));
    const R den = fma(w2, R(3.0), fma(w1, R(6.0), w0));
    return fma(num, rcp_approx<R>(den), b2);
  }
}

// Schemes kWeno5*: the 5th-order reconstruction from the middle five values
// (a_{i-2}..a_{i+2}) of the same 7-point window.
// The WENO7 value in two parts: the front (candidates and smoothness
// indicators) and the back (weights and the normalised combination).
template <class R>
struct W7Front {
  R a3, r0, r1, r2, r3, b0, b1, b2, b3;
};

template <class R, int S>
__device__ __forceinline__ W7Front<R> weno7_front(R a0, R a1, R a2, R a3, R a4, R a5, R a6, R eps) {
  W7Front<R> w;
  w.a3 = a3;
  // nested differences of the seven values
  const R e0 = a1 - a0, e1 = a2 - a1, e2 = a3 - a2, e3 = a4 - a3, e4 = a5 - a4, e5 = a6 - a5;
  // candidates as 35 d_k (q_k - a3), from the differences (the factor 35
  // cancels against the weights' denominator sum 35 w_k d_k)
  w.r0 = fma(R(13.0 / 12.0), e2, fma(R(-10.0 / 12.0), e1, R(3.0 / 12.0) * e0));
  w.r1 = fma(R(3.0), e3, fma(R(4.0), e2, -e1));
  w.r2 = fma(R(-1.5), e4, fma(R(9.0), e3, R(1.5) * e2));
  w.r3 = fma(R(1.0 / 3.0), e5, fma(R(-4.0 / 3.0), e4, R(3.0) * e3));
  if (S == kWenoLinear) return w;

  const R f0 = e1 - e0, f1 = e2 - e1, f2 = e3 - e2, f3 = e4 - e3, f4 = e5 - e4;
  const R g0 = f1 - f0, g1 = f2 - f1, g2 = f3 - f2, g3 = f4 - f3;
  w.b0 = smoothness<R>(e0, f0, g0, R(2.5), R(11.0 / 6.0), R(2), eps);
  w.b1 = smoothness<R>(e1, f1, g1, R(1.5), R(1.0 / 3.0), R(1), eps);
  w.b2 = smoothness<R>(e2, f2, g2, R(0.5), R(-1.0 / 6.0), R(0), eps);
  w.b3 = smoothness<R>(e3, f3, g3, R(-0.5), R(1.0 / 3.0), R(-1), eps);
  return w;
}

template <class R, int S>
__device__ __forceinline__ R weno7_back(const W7Front<R>& w) {
  const R a3 = w.a3, r0 = w.r0, r1 = w.r1, r2 = w.r2, r3 = w.r3;
  if (S == kWenoLinear) return fma((r0 + r1) + (r2 + r3), R(1.0 / 35.0), a3);
  const R b0 = w.b0, b1 = w.b1, b2 = w.b2, b3 = w.b3;
  if (sizeof(R) == 8) {
    // Weights over a common denominator: with B_k = b_k^2 the WENO-Z weight
    // d_k (1 + tau^2/B_k) is proportional to d_k (B_k + tau^2) prod_{j!=k} B_j,
    // the Jiang-Shu weight d_k/B_k to d_k prod_{j!=k} B_j.  One division.
    // (WENO-Z: (B_0 + tau^2) B_1 = B_0 B_1 + tau^2 B_1, and so on, one fma each.)
    const R B0 = b0 * b0, B1 = b1 * b1, B2 = b2 * b2, B3 = b3 * b3;
    const R P01 = B0 * B1, P23 = B2 * B3;
    R A0, A1, A2, A3;
    if (S == kWenoZ) {
      const R tau = fabs(fma(R(3), b1 - b2, b0 - b3));
      const R t2 = tau * tau;
      A0 = fma(t2, B1, P01) * P23;
      A1 = fma(t2, B0, P01) * P23;
      A2 = fma(t2, B3, P23) * P01;
      A3 = fma(t2, B2, P23) * P01;
    } else {
      A0 = B1 * P23;
      A1 = B0 * P23;
      A2 = P01 * B3;
      A3 = P01 * B2;
    }
    const R num = fma(A3, r3, fma(A2, r2, fma(A1, r1, A0 * r0)));
    const R den = fma(A3, R(4.0), fma(A2, R(18.0), fma(A1, R(12.0), A0)));
    return a3 + (R)div_nr((double)num, (double)den);
  } else {
    const R i0 = rcp_approx<R>(b0), i1 = rcp_approx<R>(b1), i2 = rcp_approx<R>(b2), i3 = rcp_approx<R>(b3);
    R w0, w1, w2, w3;
    if (S == kWenoZ) {
      const R tau = fabs(fma(R(3), b1 - b2, b0 - b3));
      const R s0 = tau * i0, s1 = tau * i1, s2 = tau * i2, s3 = tau * i3;
      w0 = fma(s0, s0, R(1));
      w1 = fma(s1, s1, R(1));
      w2 = fma(s2, s2, R(1));
      w3 = fma(s3, s3, R(1));
    } else {
      w0 = i0 * i0;
      w1 = i1 * i1;
      w2 = i2 * i2;
      w3 = i3 * i3;
    }
    const R num = fma(w3, r3, fma(w2, r2, fma(w1, r1, w0 * r0)));
    const R den = fma(w3, R(4.0), fma(w2, R(18.0), fma(w1, R(12.0), w0)));
    return fma(num, rcp_approx<R>(den), a3);
  }
}

template <class R, int S>
__device__ __forceinline__ R weno7(R a0, R a1, R a2, R a3, R a4, R a5, R a6, R eps) {
  if (S >= kWeno5Z) return weno5<R, S>(a1, a2, a3, a4, a5, eps);
  return weno7_back<R, S>(weno7_front<R, S>(a0, a1, a2, a3, a4, a5, a6, eps));
}

// Two neighbouring reconstructions from the eight values v0..v7: lo from
// v0..v6, hi from v1..v7, each by exactly the arithmetic of weno7.  Their
// shared differences are formed once; the fronts of both come first and the
// backs one after the other, which keeps fewer values live than interleaving
// the two.
template <class R, int S>
__device__ __forceinline__ void weno7_pair(R v0, R v1, R v2, R v3, R v4, R v5, R v6, R v7, R eps, R& lo,
                                           R& hi) {
  if (S >= kWeno5Z) {
    lo = weno5<R, S>(v1, v2, v3, v4, v5, eps);
    hi = weno5<R, S>(v2, v3, v4, v5, v6, eps);
    return;
  }
  const W7Front<R> wl = weno7_front<R, S>(v0, v1, v2, v3, v4, v5, v6, eps);
  const W7Front<R> wh = weno7_front<R, S>(v1, v2, v3, v4, v5, v6, v7, eps);
  __builtin_amdgcn_sched_barrier(0);
  lo = weno7_back<R, S>(wl);
  __builtin_amdgcn_sched_barrier(0);
  hi = weno7_back<R, S>(wh);
}

// Face flux from the 8-point window Fp/Fm[m] = split fluxes at i-3+m:
// F(i+1/2) = R_L(F+_{i-3..i+3}) + R_L(F-_{i+4..i-2}).
template <class R, int S>
__device__ __forceinline__ R face_flux(const R* fp, const R* fm, R eps) {
  return weno7<R, S>(fp[0], fp[1], fp[2], fp[3], fp[4], fp[5], fp[6], eps) +
         weno7<R, S>(fm[7], fm[6], fm[5], fm[4], fm[3], fm[2], fm[1], eps);
}

// ---------------------------------------------------------------------------
// MUSTA-FORCE flux (Toro's multi-stage centred flux), the alternative solver:
// kernels take it as the flag kMusta on the scheme template argument and then
// keep the conserved values (not the split fluxes) in their LDS tiles.  The
// face states uL, uR come from the WENO reconstruction of those values; on a
// local two-cell mesh with dt/dx = 0.9 (S_max = 1) each stage forms the FORCE
// flux, the mean of the Lax-Friedrichs flux (fL + fR)/2 - (uR - uL)/(2 * 0.9)
// and the flux of the Richtmyer state (uL + uR)/2 - 0.45 (fR - fL); the last
// stage's FORCE flux is the face flux, the stages before it move the local
// states: uL -= 0.9 (F - fL), uR -= 0.9 (fR - F).  Recovery in FP64 as
// everywhere; fixed-up recoveries are counted.
template <class R, int AX>
__device__ __forceinline__ void phys_flux(const R u[5], R f[5], unsigned& fix) {
  const PrimV p = c2p(u, fix);
  const R vd = (R)p.v[AX];
  const R pr = (R)(p.e * (1.0 / 3.0));
  f[0] = u[1 + AX];
  f[1] = (AX == 0) ? u[1] * vd + pr : u[1] * vd;
  f[2] = (AX == 1) ? u[2] * vd + pr : u[2] * vd;
  f[3] = (AX == 2) ? u[3] * vd + pr : u[3] * vd;
  f[4] = u[4] * vd;
}

template <class R, int AX>
__device__ __forceinline__ void musta_force(R uL[5], R uR[5], int k, R F[5], unsigned& fix) {
  for (int l = 1;; ++l) {
    R fL[5], fR[5], uM[5], fM[5];
    phys_flux<R, AX>(uL, fL, fix);
    phys_flux<R, AX>(uR, fR, fix);
#pragma unroll
    for (int c = 0; c < 5; ++c) uM[c] = R(0.5) * (uL[c] + uR[c]) - R(0.45) * (fR[c] - fL[c]);
    phys_flux<R, AX>(uM, fM, fix);
#pragma unroll
    for (int c = 0; c < 5; ++c) F[c] = R(0.5) * ((R(0.5) * (fL[c] + fR[c]) - R(0.5 / 0.9) * (uR[c] - uL[c])) + fM[c]);
    if (l >= k) return;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      uL[c] = uL[c] - R(0.9) * (F[c] - fL[c]);
      uR[c] = uR[c] - R(0.9) * (fR[c] - F[c]);
    }
  }
}

// One face with the MUSTA-FORCE flux: at(c, m) is component c of the
// conserved value at window point m = 0..7 (points i-3..i+4 for face i+1/2);
// uL from points 0..6, uR from the mirrored stencil 7..1 (WENO5: the middle
// five of each).
template <class R, int SC, int AX, class At>
__device__ __forceinline__ void musta_face(At at, R eps, int k, R F[5], unsigned& fix) {
  R uL[5], uR[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    uL[c] = weno7<R, SC>(at(c, 0), at(c, 1), at(c, 2), at(c, 3), at(c, 4), at(c, 5), at(c, 6), eps);
    uR[c] = weno7<R, SC>(at(c, 7), at(c, 6), at(c, 5), at(c, 4), at(c, 3), at(c, 2), at(c, 1), eps);
  }
  musta_force<R, AX>(uL, uR, k, F, fix);
}

// ---------------------------------------------------------------------------
// Positivity-preserving flux limiter (after Zhang and Shu).  Kernels take it
// as the flag kPP on the scheme template argument.
//
// A forward-Euler update u_i - sum_d (dt/dx_d)(F_{d,i+1/2} - F_{d,i-1/2}) is
// the mean over the axes, with weights (dt/dx_d) / sum(dt/dx), of the two
// half states of each axis
//   R = u_i - mu (F_{i+1/2} - f_i/2),   L = u_i + mu (F_{i-1/2} - f_i/2),
// mu = 2 dt sum_d 1/dx_d.  For the first-order flux F+(u_i) + F-(u_{i+1})
// they are (1 - mu/2) u_i + mu/2 (u_{i+1} - f_{i+1}) and (1 - mu/2) u_i +
// mu/2 (u_{i-1} + f_{i-1}): admissible for mu/2 <= 1, since u +- f(u) is for
// alpha = 1.  Each face flux F becomes theta F + (1 - theta) F_LF with the
// largest theta of the chord rule (below) that keeps E - |M| >= kPPEps and
// N >= kPPEps in the half state on each side of the face.  The split fluxes
// of the two cells give u = F+ - F-, f = F+ + F- and F_LF = F+_i + F-_{i+1}.
// FP64 in every form; a face that needs no limiting keeps its flux bit for bit.
constexpr double kPPEps = 1e-13;

// Largest theta in [0, 1] with h(theta) >= 0 for h concave: 1 if h(1) >= 0,
// 0 if h(0) <= 0, else the root of the chord from (0, h0) to (1, h1), below
// which h stays above the chord and so non-negative.
__device__ __forceinline__ double pp_chord(double h0, double h1) {
  if (h1 >= 0.0) return 1.0;
  if (h0 <= 0.0) return 0.0;
  return h0 / (h0 - h1);
}

// E - |M| >= eps and N >= eps for E, |M|^2, N, without the square root.
__device__ __forceinline__ bool pp_inside(double E, double m2, double N) {
  const double a = E - kPPEps;
  return a >= 0.0 && a * a >= m2 && N >= kPPEps;
}

// E, |M|^2 and N of a half state next to a face (side 0: the low cell's
// u - mu (F - f/2), side 1: the high cell's u + mu (F - f/2)) for the face flux
// F_c = H_c, or (lf) the first-order flux F+_low + F-_high.
struct PPHalf {
  double e, m2, n;
};

template <class R, class Get>
__device__ __forceinline__ PPHalf pp_half(const R H[5], Get get, double mu, int side, bool lf) {
  PPHalf r = {0.0, 0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double p = (double)get(c, 2 * side), m = (double)get(c, 2 * side + 1);
    const double F = lf ? (double)get(c, 0) + (double)get(c, 3) : (double)H[c];
    const double hs = side ? fma(mu, fma(-0.5, p + m, F), p - m) : fma(-mu, fma(-0.5, p + m, F), p - m);
    if (c == 0) r.e = hs;
    else if (c == 4) r.n = hs;
    else r.m2 = fma(hs, hs, r.m2);
  }
  return r;
}

// theta of one side from its half states with the first-order flux (s0) and
// with H (s1).
__device__ __forceinline__ double pp_side(const PPHalf& s0, const PPHalf& s1) {
  const double tq = pp_chord(s0.e - sqrt(s0.m2) - kPPEps, s1.e - sqrt(s1.m2) - kPPEps);
  const double tn = pp_chord(s0.n - kPPEps, s1.n - kPPEps);
  return fmin(tq, tn);
}

// H: the face's five fluxes (in/out).  get(c, k) returns component c of the
// split fluxes of the two cells next to the face: k = 0 F+ and 1 F- of the
// cell on the low side, 2 F+ and 3 F- of the cell on the high side.  Half
// states are folded into E, |M|^2 and N component by component and one side
// at a time, so that few values stay live.
template <class R, class Get>
__device__ __forceinline__ void pp_limit(R H[5], Get get, double mu) {
  bool inside;
  __asm__ __volatile__("" ::: "memory");
  {
    const PPHalf a1 = pp_half<R>(H, get, mu, 0, false);
    inside = pp_inside(a1.e, a1.m2, a1.n);
  }
  __asm__ __volatile__("" ::: "memory");
  if (inside) {
    const PPHalf b1 = pp_half<R>(H, get, mu, 1, false);
    inside = pp_inside(b1.e, b1.m2, b1.n);
  }
  if (inside) return;
  // rarely taken: each side again, with the first-order flux beside it.  The
  // empty asm with a memory clobber makes the compiler read the split fluxes
  // again here instead of keeping them in registers across the common path.
  __asm__ __volatile__("" ::: "memory");
  const double ta = pp_side(pp_half<R>(H, get, mu, 0, true), pp_half<R>(H, get, mu, 0, false));
  __asm__ __volatile__("" ::: "memory");
  const double tb = pp_side(pp_half<R>(H, get, mu, 1, true), pp_half<R>(H, get, mu, 1, false));
  const double th = fmin(ta, tb);
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double fl = (double)get(c, 0) + (double)get(c, 3);
    H[c] = (R)fma(th, (double)H[c], (1.0 - th) * fl);
  }
}

__device__ __forceinline__ void add_fixups(unsigned long long* ctr, unsigned fix) {
  if (fix) atomicAdd(ctr, (unsigned long long)fix);
}

// ---------------------------------------------------------------------------
// Jet helpers (Eq. 3, nearest grid point, cell centres, T(e)).
__device__ __forceinline__ int ngp_index(double x, int n, double dx) {
  const double x_lo = -0.5 * n * dx;
  const double u = (x - x_lo) / dx + 1e-9;
  const double f = floor(u);
  if (f < 0.0 || f >= (double)n) return -1;
  return (int)f;
}

__device__ __forceinline__ double temperature(double e, double g, double hc) {
  return pow(30.0 * e * (hc * hc * hc) / (g * 3.14159265358979323846 * 3.14159265358979323846), 0.25);
}

__device__ __forceinline__ double energy_loss(const JetDev& jt, double T, double ell, double hc) {
  return jt.kappa_coll * jt.crcf * T * T / hc + jt.kappa_rad * jt.crcf * T * T * T * ell / (hc * hc);
}

__device__ __forceinline__ double cell_centre(int i, int n, double dx) { return (i - 0.5 * (n - 1)) * dx; }

}  // namespace hydro
