// hydro_adjoint.hip -- reverse mode (vector-Jacobian products) of one SSP-RK3
// stage, of the jet source, of the anisotropy observable eps2 and of the
// primitive->conserved map of the initial state.
//
// For a stage  Y = a U^n + b (W + dt L(W)),  L = D + S, the reverse sweep
// needs G = (dL/dW)^T lambda_Y.  D's part goes face by face:
//   phi(face i+1/2) = (lambda_{i+1} - lambda_i)/dx       (face adjoint)
//   -> reverse of F(i+1/2) = R_L(F+_{i-3..i+3}) + R_L(F-_{i+4..i-2})
//   -> adjoints of the split fluxes at each point
//   -> (F+- = (f +- W)/2, f through the FP64 conserved->primitive recovery)
//   -> adjoint of W at the point; ghost points pass theirs to the cell they copy.
// A workgroup owns a whole line along the axis, so every face that touches a
// cell of the line is handled in the same workgroup: each lane reverses its
// face, writes the seven partials to LDS, and each lane gathers the partials
// of its own point in a fixed order (deterministic, no atomics).

#include <hip/hip_runtime.h>

#include "hydro_device.hpp"
#include "hydro_internal.hpp"

namespace hydro {

// ---------------------------------------------------------------------------
// Conserved -> primitive with its derivatives (FP64).  Without fix-up:
// s = sqrt(4E^2 - 3M^2), e = s - E (evaluated as 3(E^2 - M^2)/(E + s)),
// de/dE = 4E/s - 1, de/dM_j = -3 M_j/s, v = M/(E + e/3).
struct PrimJ {
  double E;
  double e, v[3], iW;  // values; iW = 1/(E + p) = 1/(E + e/3)
  double eE, eM[3];    // de/dE, de/dM_j (at the possibly rescaled M)
  double Mc[3];        // M used in the recovery (rescaled when capped)
  double Mh[3];        // M/|M| (cap)
  double capf;         // (1 - 1e-10) E / |M| (cap)
  bool vac, cap;
};

__device__ __forceinline__ PrimJ c2p_jac(double E, double Mx, double My, double Mz) {
  PrimJ J;
  J.E = E;
  J.vac = false;
  J.cap = false;
  J.capf = 1.0;
  double M[3] = {Mx, My, Mz};
  if (E <= kEFloor) {
    J.vac = true;
    J.e = kEFloor;
    J.iW = 1.0 / (kEFloor + kEFloor / 3.0);
    for (int k = 0; k < 3; ++k) {
      J.v[k] = 0.0;
      J.eM[k] = 0.0;
      J.Mc[k] = 0.0;
      J.Mh[k] = 0.0;
    }
    J.eE = 0.0;
    return J;
  }
  double M2 = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  if (M2 >= kVCap * kVCap * E * E) {
    J.cap = true;
    const double inrm = 1.0 / sqrt(M2);
    const double sc = kVCap * E * inrm;
    J.capf = sc;
    for (int k = 0; k < 3; ++k) {
      J.Mh[k] = M[k] * inrm;
      M[k] = M[k] * sc;
    }
    M2 = M[0] * M[0] + M[1] * M[1] + M[2] * M[2];
  }
  const double s = sqrt(4.0 * E * E - 3.0 * M2);
  const double is = 1.0 / s;
  const double e = 3.0 * (E * E - M2) / (E + s);
  J.e = e;
  J.iW = 1.0 / (E + e * (1.0 / 3.0));
  for (int k = 0; k < 3; ++k) {
    J.Mc[k] = M[k];
    J.v[k] = M[k] * J.iW;
    J.eM[k] = -3.0 * M[k] * is;
  }
  J.eE = 4.0 * E * is - 1.0;
  return J;
}

// The same Jacobian for an admissible cell (no fix-up) whose e is known from
// the recovery: sqrt(4E^2 - 3M^2) = E + e, one division.
__device__ __forceinline__ PrimJ c2p_jac_known(double E, double Mx, double My, double Mz, double e) {
  PrimJ J;
  J.E = E;
  J.vac = false;
  J.cap = false;
  J.capf = 1.0;
  const double M[3] = {Mx, My, Mz};
  const double s = E + e;
  const double W = E + e * (1.0 / 3.0);
  const double inv = rcp_nr(s * W);
  const double is = W * inv;
  J.e = e;
  J.iW = s * inv;
  for (int k = 0; k < 3; ++k) {
    J.Mc[k] = M[k];
    J.Mh[k] = 0.0;
    J.v[k] = M[k] * J.iW;
    J.eM[k] = -3.0 * M[k] * is;
  }
  J.eE = 4.0 * E * is - 1.0;
  return J;
}

// Given adjoints eb of e and vb of v, the adjoints of (E, M):
// with Q = (vb . v)/(E + p) and kappa = eb - Q/3:
//   Eb = kappa de/dE - Q,  Mb_k = kappa de/dM_k + vb_k/(E + p),
// then through the velocity cap M' = c M, c = (1 - 1e-10) E/|M|.
__device__ __forceinline__ void c2p_vjp(const PrimJ& J, double eb, const double vb[3], double& Eb, double Mb[3]) {
  if (J.vac) {
    Eb = 0.0;
    Mb[0] = Mb[1] = Mb[2] = 0.0;
    return;
  }
  const double Q = (vb[0] * J.v[0] + vb[1] * J.v[1] + vb[2] * J.v[2]) * J.iW;
  const double kap = eb - Q * (1.0 / 3.0);
  double Ebp = kap * J.eE - Q;
  double Mbp[3];
  for (int k = 0; k < 3; ++k) Mbp[k] = kap * J.eM[k] + vb[k] * J.iW;
  if (!J.cap) {
    Eb = Ebp;
    for (int k = 0; k < 3; ++k) Mb[k] = Mbp[k];
    return;
  }
  const double dM = Mbp[0] * J.Mc[0] + Mbp[1] * J.Mc[1] + Mbp[2] * J.Mc[2];
  const double dh = Mbp[0] * J.Mh[0] + Mbp[1] * J.Mh[1] + Mbp[2] * J.Mh[2];
  Eb = Ebp + dM / J.E;
  for (int k = 0; k < 3; ++k) Mb[k] = J.capf * (Mbp[k] - J.Mh[k] * dh);
}

// Adjoint of the split fluxes at one point (axis AX): ap, am are the adjoints
// of F+ and F-; returns the adjoint of the conserved W of that point.
template <class R, int AX>
__device__ __forceinline__ void split_flux_vjp(const R u[5], const PrimJ& J, const double ap[5], const double am[5],
                                               double ub[5]) {
  double fb[5];
  for (int c = 0; c < 5; ++c) {
    fb[c] = 0.5 * (ap[c] + am[c]);
    ub[c] = 0.5 * (ap[c] - am[c]);
  }
  const double vd = (double)(R)J.v[AX];
  ub[1 + AX] += fb[0];
  double vbd = 0.0;
  for (int j = 0; j < 3; ++j) {
    ub[1 + j] += fb[1 + j] * vd;
    vbd += fb[1 + j] * (double)u[1 + j];
  }
  ub[4] += fb[4] * vd;
  vbd += fb[4] * (double)u[4];
  const double pb = fb[1 + AX];
  double vb[3] = {0.0, 0.0, 0.0};
  vb[AX] = vbd;
  double Eb, Mb[3];
  c2p_vjp(J, pb * (1.0 / 3.0), vb, Eb, Mb);
  ub[0] += Eb;
  for (int k = 0; k < 3; ++k) ub[1 + k] += Mb[k];
}

// ---------------------------------------------------------------------------
// Reverse mode of weno7: ab[m] = phi * dR/da_m for the reconstruction of
// a0..a6 (same forward arithmetic: differences, candidates d_k (q_k - a3),
// smoothness from differences, Z or JS weights, R = a3 + sum w r / sum w d),
// then the chain back through weights, smoothness indicators, candidates and
// differences.  Every multiply-add is an explicit fma.
template <class R, int S>
__device__ __forceinline__ void weno7_vjp(const R* a, R phi, R eps, R* ab) {
  const R e0 = a[1] - a[0], e1 = a[2] - a[1], e2 = a[3] - a[2], e3 = a[4] - a[3], e4 = a[5] - a[4],
          e5 = a[6] - a[5];
  R eb[6], fb[5], gb[4];
  R rb0, rb1, rb2, rb3;
  if (S == kWenoLinear) {
    rb0 = rb1 = rb2 = rb3 = phi;
#pragma unroll
    for (int k = 0; k < 6; ++k) eb[k] = R(0);
#pragma unroll
    for (int k = 0; k < 5; ++k) fb[k] = R(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) gb[k] = R(0);
  } else {
    const R r0 = fma(R(13.0 / 420.0), e2, fma(R(-10.0 / 420.0), e1, R(3.0 / 420.0) * e0));
    const R r1 = fma(R(3.0 / 35.0), e3, fma(R(4.0 / 35.0), e2, R(-1.0 / 35.0) * e1));
    const R r2 = fma(R(-3.0 / 70.0), e4, fma(R(18.0 / 70.0), e3, R(3.0 / 70.0) * e2));
    const R r3 = fma(R(1.0 / 105.0), e5, fma(R(-4.0 / 105.0), e4, R(9.0 / 105.0) * e3));
    const R f[5] = {e1 - e0, e2 - e1, e3 - e2, e4 - e3, e5 - e4};
    const R g[4] = {f[1] - f[0], f[2] - f[1], f[3] - f[2], f[4] - f[3]};
    const R e[4] = {e0, e1, e2, e3};
    const R hk[4] = {R(2.5), R(1.5), R(0.5), R(-0.5)};
    const R mk[4] = {R(11.0 / 6.0), R(1.0 / 3.0), R(-1.0 / 6.0), R(1.0 / 3.0)};
    const R gk[4] = {R(2), R(1), R(0), R(-1)};
    // X_k = 13/12 c_k and Y_k = 781/720 D3_k are kept: half the indicator's
    // partials in c_k and D3_k
    R b[4], sk[4], ck[4], X[4], Y[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      sk[k] = fma(mk[k], g[k], fma(hk[k], f[k], e[k]));
      ck[k] = fma(gk[k], g[k], f[k]);
      X[k] = R(13.0 / 12.0) * ck[k];
      Y[k] = R(781.0 / 720.0) * g[k];
      b[k] = fma(sk[k], sk[k], fma(X[k], ck[k], fma(Y[k], g[k], eps)));
    }
    R iv[4];
    if (sizeof(R) == 8) {
      const R p01 = b[0] * b[1], p23 = b[2] * b[3];
      const R inv = (R)rcp_nr((double)(p01 * p23));
      const R u23 = inv * p23, u01 = inv * p01;
      iv[0] = u23 * b[1];
      iv[1] = u23 * b[0];
      iv[2] = u01 * b[3];
      iv[3] = u01 * b[2];
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) iv[k] = rcp_approx<R>(b[k]);
    }
    R w[4], s[4];
    R traw = R(0);
    if (S == kWenoZ) {
      traw = fma(R(3), b[1] - b[2], b[0] - b[3]);
      const R tau = fabs(traw);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        s[k] = tau * iv[k];
        w[k] = fma(s[k], s[k], R(1));
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k) w[k] = iv[k] * iv[k];
    }
    const R dk[4] = {R(1.0 / 35.0), R(12.0 / 35.0), R(18.0 / 35.0), R(4.0 / 35.0)};
    const R den = fma(w[3], dk[3], fma(w[2], dk[2], fma(w[1], dk[1], w[0] * dk[0])));
    const R num = fma(w[3], r3, fma(w[2], r2, fma(w[1], r1, w[0] * r0)));
    const R invd = sizeof(R) == 8 ? (R)rcp_nr((double)den) : rcp_approx<R>(den);
    const R corr = num * invd;
    const R pin = phi * invd;
    rb0 = pin * w[0];
    rb1 = pin * w[1];
    rb2 = pin * w[2];
    rb3 = pin * w[3];
    const R rr[4] = {r0, r1, r2, r3};
    // bb2[k] = 2 dR/db_k, formed directly (4 dR/dw_k below): the factor 2 of
    // every partial of b_k = s_k^2 + X_k c_k + Y_k D3_k + eps then needs no
    // multiply (powers of two scale exactly, so this is bit-identical to
    // forming dR/db_k and doubling it)
    const R pin4 = R(4) * pin;
    R bb2[4];
    R taub2 = R(0);  // 2 dR/dtau
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const R wb4 = pin4 * fma(-dk[k], corr, rr[k]);  // 4 dR/dw_k
      if (S == kWenoZ) {
        const R t2 = wb4 * (s[k] * iv[k]);  // 2 dR/dtau through w_k
        bb2[k] = -t2 * s[k];
        taub2 = taub2 + t2;
      } else {
        bb2[k] = -wb4 * (w[k] * iv[k]);
      }
    }
    if (S == kWenoZ) {
      const R t = traw < R(0) ? -taub2 : taub2;  // tau = |traw|
      bb2[0] = bb2[0] + t;
      bb2[1] = fma(R(3), t, bb2[1]);
      bb2[2] = fma(R(-3), t, bb2[2]);
      bb2[3] = bb2[3] - t;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const R sb = sk[k] * bb2[k];  // s_k partial
      const R cb = X[k] * bb2[k];   // c_k partial
      const R gd = Y[k] * bb2[k];   // D3_k partial (direct term)
      eb[k] = sb;
      fb[k] = fma(hk[k], sb, cb);
      gb[k] = (k == 2) ? fma(mk[k], sb, gd) : fma(mk[k], sb, fma(gk[k], cb, gd));  // g_2 = 0
    }
    eb[4] = R(0);
    eb[5] = R(0);
    fb[4] = R(0);
  }
  // candidates r_k(e)
  eb[0] = fma(R(3.0 / 420.0), rb0, eb[0]);
  eb[1] = fma(R(-1.0 / 35.0), rb1, fma(R(-10.0 / 420.0), rb0, eb[1]));
  eb[2] = fma(R(3.0 / 70.0), rb2, fma(R(4.0 / 35.0), rb1, fma(R(13.0 / 420.0), rb0, eb[2])));
  eb[3] = fma(R(9.0 / 105.0), rb3, fma(R(18.0 / 70.0), rb2, fma(R(3.0 / 35.0), rb1, eb[3])));
  eb[4] = fma(R(-4.0 / 105.0), rb3, fma(R(-3.0 / 70.0), rb2, eb[4]));
  eb[5] = fma(R(1.0 / 105.0), rb3, eb[5]);
  // second differences g_j = f_{j+1} - f_j, first f_j = e_{j+1} - e_j, e_j = a_{j+1} - a_j
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    fb[j + 1] = fb[j + 1] + gb[j];
    fb[j] = fb[j] - gb[j];
  }
#pragma unroll
  for (int j = 0; j < 5; ++j) {
    eb[j + 1] = eb[j + 1] + fb[j];
    eb[j] = eb[j] - fb[j];
  }
  ab[0] = -eb[0];
#pragma unroll
  for (int j = 1; j < 6; ++j) ab[j] = eb[j - 1] - eb[j];
  ab[6] = eb[5];
  ab[3] = ab[3] + phi;
}

// ---------------------------------------------------------------------------
// Line adjoint along axis AX: one workgroup per line (blockDim >= n, <= 1024).
// G (first: =, else +=) receives (dD_AX/dW)^T mu for the faces -1/2..n-3/2
// of the line (periodic: face -1/2 is also the right face of cell n-1); the
// outflow face n-1/2 is added by k_bound_adj.
__device__ __forceinline__ long long line_base(int AX, long long L, const Grid& g, long long& stride) {
  const int nx = g.n[0], ny = g.n[1];
  if (AX == 0) {
    stride = 1;
    return L * nx;
  }
  if (AX == 1) {
    stride = nx;
    const long long x = L % nx, z = L / nx;
    return z * (long long)nx * ny + x;
  }
  stride = (long long)nx * ny;
  const long long x = L % nx, y = L / nx;
  return y * nx + x;
}

__device__ __forceinline__ long long n_lines(int AX, const Grid& g) {
  return AX == 0 ? (long long)g.n[1] * g.n[2] : (AX == 1 ? (long long)g.n[0] * g.n[2] : (long long)g.n[0] * g.n[1]);
}

// Block order: consecutive lines (neighbours in memory for the y/z axes) go
// to the same XCD (blocks are dealt round-robin over the 8 XCDs).
__device__ __forceinline__ long long xcd_line(long long nlines) {
  const long long per = (nlines + 7) / 8;
  return (long long)(blockIdx.x % 8) * per + blockIdx.x / 8;
}

template <class R, int S, int AX, int TBMAX, int NL>
__global__ void __launch_bounds__(TBMAX) k_line_adj(AdjArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const long long nlines = n_lines(AX, a.g);
  // NL neighbouring lines (consecutive x) per workgroup, lanes interleaved
  // line-fastest, so that the strided loads and stores of y and z lines
  // fetch NL neighbouring values per cache line; each line has its own LDS
  // area (pitch chosen so that the lines' copies fall in different banks)
  const long long ngroups = nlines / NL;
  const long long grp = xcd_line(ngroups);
  if (grp >= ngroups) return;  // whole workgroup
  const int xi = threadIdx.x % NL;
  const long long L = grp * NL + xi;
  const int n = a.g.n[AX];
  const int bc = a.g.bc[AX];
  const int P = n + 8;
  const int Q = n + 16;
  const long long nc = a.g.nc;
  long long stride;
  const long long base = line_base(AX, L, a.g, stride);
  R* s = reinterpret_cast<R*>(smem_raw) + (long long)xi * line_adj_pitch(n, NL);
  R* sFp = s;               // [5][P]
  R* sFm = s + 5 * P;       // [5][P]
  R* sX = s + 10 * P;       // [2][7][Q]; first used to stage mu [5][n]
  const int tid = threadIdx.x / NL;  // point / face of the lane in its line
  const int TB = blockDim.x / NL;    // lanes per line
  unsigned fix = 0;

  // Points: lane tid < n recomputes the split fluxes of its own cell (slot
  // tid + 4).  A ghost point (slots 0..3, n+4..n+7) is a copy of the cell it
  // maps to, so its split fluxes are copied in LDS, and in the reverse its
  // split-flux adjoints are added to that cell's before the one split-flux
  // VJP (the same Jacobian, so this equals reversing the ghost on its own).
  R uo[5];
  double eo = 0.0;     // recovered e of the own cell
  bool fixed = false;  // the recovery fixed the own cell up
  if (tid < n) {
    load5(a.W, nc, base + (long long)tid * stride, uo);
    const unsigned f0 = fix;
    const PrimV pv = c2p(uo, fix);
    eo = pv.e;
    fixed = fix != f0;
    R Fp[5], Fm[5];
    split_flux<R, AX>(uo, pv, Fp, Fm);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      sFp[c * P + tid + 4] = Fp[c];
      sFm[c * P + tid + 4] = Fm[c];
    }
  }
  R my[5];  // mu of the lane's own cell (used by the fused combine)
  if (tid < n) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      my[c] = (c == 4 && a.skip_n) ? R(0) : a.mu[c * nc + base + (long long)tid * stride];
      sX[c * n + tid] = my[c];
    }
  }
  __syncthreads();
  // ghost slot of lane tid < 8: slot jg, copy of cell map_idx(jg - 4)
  const int jg = tid < 4 ? tid : n + tid;
  if (tid < 8) {
    const int src = map_idx(jg - 4, n, bc) + 4;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      sFp[c * P + jg] = sFp[c * P + src];
      sFm[c * P + jg] = sFm[c * P + src];
    }
  }
  // face adjoints phi(x - 1/2) = (mu(x) - mu(x-1)) / dx
  R phi[5];
  if (tid < n) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const R left = tid > 0 ? sX[c * n + tid - 1] : (bc ? sX[c * n + n - 1] : R(0));
      phi[c] = (sX[c * n + tid] - left) * a.inv_d;
    }
  }
  __syncthreads();
  for (int z = tid; z < 14 * 16; z += TB) {  // pads: 8 below and 8 above each row
    const int row = z >> 4, k = z & 15;
    sX[row * Q + (k < 8 ? k : n + k)] = R(0);
  }

  // slot j is argument m of face j - m (F+) and of face j - 7 + m (F-)
  auto gather = [&](int j, R& sp, R& sm) {
    sp = R(0);
    sm = R(0);
#pragma unroll
    for (int m = 0; m < 7; ++m) {
      sp = sp + sX[m * Q + j - m + 8];
      sm = sm + sX[(7 + m) * Q + j - 7 + m + 8];
    }
  };
  R acc[2][5];  // [split][field] of the own cell
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    if (c == 4 && a.skip_n) {  // uniform over the workgroup
      acc[0][c] = acc[1][c] = R(0);
      continue;
    }
    if (tid < n) {
      R args[7], ab[7];
#pragma unroll
      for (int m = 0; m < 7; ++m) args[m] = sFp[c * P + tid + m];
      weno7_vjp<R, S>(args, phi[c], a.eps, ab);
#pragma unroll
      for (int m = 0; m < 7; ++m) sX[m * Q + tid + 8] = ab[m];
#pragma unroll
      for (int m = 0; m < 7; ++m) args[m] = sFm[c * P + tid + 7 - m];
      weno7_vjp<R, S>(args, phi[c], a.eps, ab);
#pragma unroll
      for (int m = 0; m < 7; ++m) sX[(7 + m) * Q + tid + 8] = ab[m];
    }
    __syncthreads();
    if (tid < n) gather(tid + 4, acc[0][c], acc[1][c]);
    if (tid < 8) {
      // the ghost's sums go to slots 0..7 of field c's rows, which no lane
      // reads again (field c's reconstructions are done)
      R gp, gm;
      gather(jg, gp, gm);
      sFp[c * P + tid] = gp;
      sFm[c * P + tid] = gm;
    }
    __syncthreads();
  }

  if (tid < n) {
    // ghosts in slot order onto the cells they copy
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const int j = g < 4 ? g : n + g;
      if (map_idx(j - 4, n, bc) == tid) {
#pragma unroll
        for (int c = 0; c < 5; ++c) {
          if (c == 4 && a.skip_n) continue;  // slots still hold field 4's split fluxes
          acc[0][c] = acc[0][c] + sFp[c * P + g];
          acc[1][c] = acc[1][c] + sFm[c * P + g];
        }
      }
    }
    // split-flux adjoint -> adjoint of W at the cell
    const double E = (double)uo[0], Mx = (double)uo[1], My = (double)uo[2], Mz = (double)uo[3];
    const PrimJ J = fixed ? c2p_jac(E, Mx, My, Mz) : c2p_jac_known(E, Mx, My, Mz, eo);
    double ap[5], am[5], ub[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      ap[c] = (double)acc[0][c];
      am[c] = (double)acc[1][c];
    }
    split_flux_vjp<R, AX>(uo, J, ap, am, ub);
    const long long cell = base + (long long)tid * stride;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const long long q = c * nc + cell;
      const R gv = a.first ? (R)ub[c] : a.G[q] + (R)ub[c];
      if (a.stage == 0) {
        a.G[q] = gv;
      } else {
        const R t = fma(a.dt, gv, my[c]);
        if (a.stage == 3) {
          a.lW[q] = R(2.0 / 3.0) * t;
          a.acc[q] = R(1.0 / 3.0) * my[c];
        } else if (a.stage == 2) {
          a.lW[q] = R(0.25) * t;
          a.acc[q] = fma(R(0.75), my[c], a.acc[q]);
        } else {
          a.lW[q] = a.acc[q] + t;
        }
      }
    }
  }
  add_fixups(a.fixups, fix);
}

// Outflow face n-1/2 of every line along AX: phi = -mu(n-1)/dx.  Its
// stencil points n-4..n+3 are the cells clamp(n-4+m) (the ghosts copy cell
// n-1), so they fall into runs of equal cells; the first point of a run
// stands for it.  A workgroup takes 32 lines: (1) one lane per run recovers
// its cell and forms the split fluxes; (2) one lane per (line, field, split)
// reverses that reconstruction; (3) the lane of each run adds the run's
// reconstruction adjoints in point order, reverses the split through the
// cell's Jacobian and adds the result to G (distinct cells, so no two lanes
// touch the same element).
constexpr int kBoundLines = 32;

__device__ __forceinline__ int bound_cell(int n, int m) { return min(max(n - 4 + m, 0), n - 1); }
// first point of m's run of equal cells
__device__ __forceinline__ int bound_rep(int n, int m) {
  const int k = bound_cell(n, m);
  return k == 0 ? 0 : k - (n - 4);
}

template <class R, int S, int AX>
__global__ void __launch_bounds__(kBoundLines * 10) k_bound_adj(AdjArgs<R> a) {
  __shared__ R sF[kBoundLines][4][10];        // split fluxes of the runs' cells (F+ 0..4, F- 5..9)
  __shared__ double sA[kBoundLines][8][10];   // reconstruction adjoints per point
  const long long nlines = n_lines(AX, a.g);
  const int n = a.g.n[AX];
  const long long nc = a.g.nc;
  const int tid = threadIdx.x;
  unsigned fix = 0;
  // (1) lane = (line, point m < 4); point m starts a run when its cell
  // differs from point m-1's (points 4..7 are in point 3's run)
  const int l1 = tid >> 2, m1 = tid & 3;
  const long long L1 = (long long)blockIdx.x * kBoundLines + l1;
  const bool act1 = tid < kBoundLines * 4 && L1 < nlines && (m1 == 0 || bound_cell(n, m1) != bound_cell(n, m1 - 1));
  // the face adjoint of lane (line, field, split) of step (2) and the G of
  // the run's cell, loaded first so that their latency overlaps step (1)
  const int l2 = tid / 10, r2 = tid % 10, c2 = r2 >> 1, sp2 = r2 & 1;
  const long long L2 = (long long)blockIdx.x * kBoundLines + l2;
  R phi = R(0);
  if (L2 < nlines && !(c2 == 4 && a.skip_n)) {
    long long stride;
    const long long base = line_base(AX, L2, a.g, stride);
    phi = -a.mu[c2 * nc + base + (long long)(n - 1) * stride] * a.inv_d;
  }
  R u[5], gpre[5];
  double eo = 0.0;
  bool fixed = false;
  long long cell1 = 0;
  if (act1) {
    long long stride;
    cell1 = line_base(AX, L1, a.g, stride) + (long long)bound_cell(n, m1) * stride;
#pragma unroll
    for (int c = 0; c < 5; ++c) gpre[c] = a.G[c * nc + cell1];
    load5(a.W, nc, cell1, u);
    const unsigned f0 = fix;
    const PrimV pv = c2p(u, fix);
    eo = pv.e;
    fixed = fix != f0;
    R Fp[5], Fm[5];
    split_flux<R, AX>(u, pv, Fp, Fm);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      sF[l1][m1][c] = Fp[c];
      sF[l1][m1][5 + c] = Fm[c];
    }
  }
  __syncthreads();
  // (2) reconstruction adjoints, lane = (line, field, split)
  {
    const int l = l2, c = c2, sp = sp2;
    if (L2 < nlines) {
      R args[7], ab[7];
      if (sp == 0) {
#pragma unroll
        for (int m = 0; m < 7; ++m) args[m] = sF[l][bound_rep(n, m)][c];
        weno7_vjp<R, S>(args, phi, a.eps, ab);
#pragma unroll
        for (int m = 0; m < 7; ++m) sA[l][m][c] = (double)ab[m];
        sA[l][7][c] = 0.0;
      } else {
#pragma unroll
        for (int m = 0; m < 7; ++m) args[m] = sF[l][bound_rep(n, 7 - m)][5 + c];
        weno7_vjp<R, S>(args, phi, a.eps, ab);
#pragma unroll
        for (int m = 0; m < 7; ++m) sA[l][7 - m][5 + c] = (double)ab[m];
        sA[l][0][5 + c] = 0.0;
      }
    }
  }
  __syncthreads();
  // (3) the run's adjoints in point order, the split-flux adjoint, G
  if (act1) {
    double ap[5], am[5], ub[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) ap[c] = am[c] = 0.0;
    const int k = bound_cell(n, m1);
    for (int m = m1; m < 8 && bound_cell(n, m) == k; ++m) {
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        ap[c] = ap[c] + sA[l1][m][c];
        am[c] = am[c] + sA[l1][m][5 + c];
      }
    }
    const double E = (double)u[0], Mx = (double)u[1], My = (double)u[2], Mz = (double)u[3];
    const PrimJ J = fixed ? c2p_jac(E, Mx, My, Mz) : c2p_jac_known(E, Mx, My, Mz, eo);
    split_flux_vjp<R, AX>(u, J, ap, am, ub);
#pragma unroll
    for (int c = 0; c < 5; ++c) a.G[c * nc + cell1] = gpre[c] + (R)ub[c];
  }
  add_fixups(a.fixups, fix);
}

// ---------------------------------------------------------------------------
// Jet source adjoint: G += (dS/dW)^T mu at the deposit cells, and
// grad[j] += bdt * (dS/dtheta)^T mu for theta = (kappa_rad, kappa_coll, x0, y0, z0).
template <class R>
__global__ void __launch_bounds__(512) k_jet_adj(JetAdjArgs a) {
  const R* W = static_cast<const R*>(a.W);
  const R* mu = static_cast<const R*>(a.mu);
  R* G = static_cast<R*>(a.G);
  const long long nc = a.g.nc;
  const double dV = a.g.dx[0] * a.g.dx[1] * a.g.dx[2];
  const double hc = a.hbarc;
  __shared__ double red[8][12];  // per-wave sums
  __shared__ double tot[12];     // the workgroup's sums
  __shared__ double wraw[3][7], wax[3][7], dwax[3][7];
  __shared__ int ctr_s[3];
  __shared__ int inside_s;
  const int t = threadIdx.x;
  for (int j = 0; j < a.njet; ++j) {
    const JetDev jt = a.s->jets[j];
    const bool chi = a.Ehist[j] > 0.0;
    const double ell = a.t - jt.t_start;
    // footprint weights: lane t < 21 takes axis t / 7, offset t % 7 (the
    // sums over the seven offsets in offset order, as one lane would)
    const int wd = t / 7, wm = t % 7;
    // the lane's axis by selects (an index by wd would put the structs in
    // scratch memory)
    auto pick = [wd](double v0, double v1, double v2) { return wd == 0 ? v0 : (wd == 1 ? v1 : v2); };
    const int wn = wd == 0 ? a.g.n[0] : (wd == 1 ? a.g.n[1] : a.g.n[2]);
    const double wdx = pick(a.g.dx[0], a.g.dx[1], a.g.dx[2]);
    double wx = 0.0, wdel = 0.0, wsig2 = 1.0;
    if (t < 21) {
      wx = pick(jt.x0[0], jt.x0[1], jt.x0[2]) + pick(jt.dir[0], jt.dir[1], jt.dir[2]) * ell;
      const int c = ngp_index(wx, wn, wdx);
      if (wm == 0) ctr_s[wd] = c;
      wsig2 = wdx * wdx;
      wdel = cell_centre(c - 3 + wm, wn, wdx) - wx;
      if (a.deposit == 1) wraw[wd][wm] = exp(-(wdel * wdel) / (2.0 * wsig2));
    }
    __syncthreads();
    if (t == 0) inside_s = (chi && ell >= 0.0 && ctr_s[0] >= 0 && ctr_s[1] >= 0 && ctr_s[2] >= 0) ? 1 : 0;
    if (a.deposit == 1) {
      if (t < 21) {
        double sum = 0.0;
        for (int m = 0; m < 7; ++m) sum = sum + wraw[wd][m];
        wax[wd][wm] = wraw[wd][wm] / sum;
      }
      __syncthreads();
      if (t < 21) {
        double dsum = 0.0;
        for (int m = 0; m < 7; ++m) {
          const double del = cell_centre(ctr_s[wd] - 3 + m, wn, wdx) - wx;
          dsum += wax[wd][m] * del / wsig2;
        }
        dwax[wd][wm] = wax[wd][wm] * (wdel / wsig2 - dsum);  // d w_m / d x
      }
    }
    __syncthreads();
    if (inside_s) {
      if (a.deposit == 0) {
        if (t == 0) {
          const long long cell = ((long long)ctr_s[2] * a.g.n[1] + ctr_s[1]) * a.g.n[0] + ctr_s[0];
          R gv[4];  // the cell's G, read with its state
          for (int k = 0; k < 4; ++k) gv[k] = G[k * nc + cell];
          const PrimJ J = c2p_jac((double)W[cell], (double)W[nc + cell], (double)W[2 * nc + cell],
                                  (double)W[3 * nc + cell]);
          const double T = temperature(J.e, a.eos_dof, hc);
          const double sig = ((double)mu[cell] + jt.dir[0] * (double)mu[nc + cell] +
                              jt.dir[1] * (double)mu[2 * nc + cell] + jt.dir[2] * (double)mu[3 * nc + cell]) / dV;
          const double dPdT = 2.0 * jt.kappa_coll * jt.crcf * T / hc + 3.0 * jt.kappa_rad * jt.crcf * T * T * ell / (hc * hc);
          const double eb = sig * dPdT * T / (4.0 * J.e);
          const double vb[3] = {0.0, 0.0, 0.0};
          double Eb, Mb[3];
          c2p_vjp(J, eb, vb, Eb, Mb);
          G[cell] = gv[0] + (R)Eb;
          for (int k = 0; k < 3; ++k) G[(1 + k) * nc + cell] = gv[1 + k] + (R)Mb[k];
          double* gr = a.grad + 5 * j;
          gr[0] += a.bdt * sig * jt.crcf * T * T * T * ell / (hc * hc);
          gr[1] += a.bdt * sig * jt.crcf * T * T / hc;
        }
      } else {
        // 7^3 footprint, thread t < 343
        double w = 0.0, T = 0.0, sig = 0.0, dw[3] = {0.0, 0.0, 0.0};
        long long cell = -1;
        PrimJ J;
        R gv[4];  // the cell's G, read with its state
        if (t < 343) {
          const int mi = t % 7, mj = (t / 7) % 7, mk = t / 49;
          const int i = ctr_s[0] - 3 + mi, jj = ctr_s[1] - 3 + mj, k = ctr_s[2] - 3 + mk;
          if (i >= 0 && i < a.g.n[0] && jj >= 0 && jj < a.g.n[1] && k >= 0 && k < a.g.n[2]) {
            cell = ((long long)k * a.g.n[1] + jj) * a.g.n[0] + i;
            w = wax[0][mi] * wax[1][mj] * wax[2][mk];
            dw[0] = dwax[0][mi] * wax[1][mj] * wax[2][mk];
            dw[1] = wax[0][mi] * dwax[1][mj] * wax[2][mk];
            dw[2] = wax[0][mi] * wax[1][mj] * dwax[2][mk];
            for (int q = 0; q < 4; ++q) gv[q] = G[q * nc + cell];
            J = c2p_jac((double)W[cell], (double)W[nc + cell], (double)W[2 * nc + cell], (double)W[3 * nc + cell]);
            T = temperature(J.e, a.eos_dof, hc);
            sig = ((double)mu[cell] + jt.dir[0] * (double)mu[nc + cell] + jt.dir[1] * (double)mu[2 * nc + cell] +
                   jt.dir[2] * (double)mu[3 * nc + cell]) / dV;
          }
        }
        // reductions: 0 wsum, 1 sum wT, 2 sum sig w, 3-5 sum sig dw, 6-8 sum dw T, 9-11 sum dw;
        // butterfly within each wave, then lane r < 12 adds the eight waves in order
#pragma unroll
        for (int r = 0; r < 12; ++r) {
          double v = r == 0 ? w : r == 1 ? w * T : r == 2 ? sig * w : r < 6 ? sig * dw[r - 3] : r < 9 ? dw[r - 6] * T : dw[r - 9];
#pragma unroll
          for (int off = 32; off > 0; off >>= 1) v = v + __shfl_xor(v, off, 64);
          if ((t & 63) == 0) red[t >> 6][r] = v;
        }
        __syncthreads();
        if (t < 12) {
          double v = red[0][t];
          for (int wv = 1; wv < 8; ++wv) v = v + red[wv][t];
          tot[t] = v;
        }
        __syncthreads();
        const double wsum = tot[0];
        const double Tj = tot[1] / wsum;
        const double Pj = energy_loss(jt, Tj, ell, hc);
        const double dJdP = tot[2];
        const double dPdT = 2.0 * jt.kappa_coll * jt.crcf * Tj / hc + 3.0 * jt.kappa_rad * jt.crcf * Tj * Tj * ell / (hc * hc);
        const double dJdT = dJdP * dPdT;
        if (cell >= 0) {
          const double eb = dJdT * (w / wsum) * T / (4.0 * J.e);
          const double vb[3] = {0.0, 0.0, 0.0};
          double Eb, Mb[3];
          c2p_vjp(J, eb, vb, Eb, Mb);
          G[cell] = gv[0] + (R)Eb;
          for (int k = 0; k < 3; ++k) G[(1 + k) * nc + cell] = gv[1 + k] + (R)Mb[k];
        }
        if (t == 0) {
          double* gr = a.grad + 5 * j;
          gr[0] += a.bdt * dJdP * jt.crcf * Tj * Tj * Tj * ell / (hc * hc);
          gr[1] += a.bdt * dJdP * jt.crcf * Tj * Tj / hc;
          for (int d = 0; d < 3; ++d) {
            const double dTj = (tot[6 + d] - Tj * tot[9 + d]) / wsum;
            gr[2 + d] += a.bdt * (Pj * tot[3 + d] + dJdT * dTj);
          }
        }
      }
    }
    __syncthreads();
  }
}

template <class R>
__global__ void __launch_bounds__(256) k_copy(const R* __restrict__ src, R* __restrict__ dst, long long n) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) dst[q] = src[q];
}

__global__ void k_copy_f64(const double* __restrict__ src, double* __restrict__ dst, int n) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) dst[q] = src[q];
}

template <class R>
__global__ void __launch_bounds__(256) k_fill(R* dst, long long n, R v) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) dst[q] = v;
}

// ---------------------------------------------------------------------------
// eps2 = sum (y^2 - x^2) e / sum (y^2 + x^2) e on the z = 0 plane (mean of
// the two middle planes for even nz).  Partial sums per block, then one block;
// the seed kernel writes d eps2 / dU on those planes (other cells: 0).
__device__ __forceinline__ void z0_planes(int nz, int& k0, int& k1) {
  if (nz % 2 == 0) {
    k0 = nz / 2 - 1;
    k1 = nz / 2;
  } else {
    k0 = k1 = (nz - 1) / 2;
  }
}

template <class R>
__global__ void __launch_bounds__(256) k_eps2_partial(const R* __restrict__ U, Grid g, double* part) {
  const int nx = g.n[0], ny = g.n[1];
  int k0, k1;
  z0_planes(g.n[2], k0, k1);
  const long long nc = g.nc;
  double num = 0.0, den = 0.0;
  unsigned fix = 0;
  for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < (long long)nx * ny;
       q += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(q % nx), j = (int)(q / nx);
    const double x = cell_centre(i, nx, g.dx[0]), y = cell_centre(j, ny, g.dx[1]);
    const long long ca = ((long long)k0 * ny + j) * nx + i, cb = ((long long)k1 * ny + j) * nx + i;
    const PrimV pa = c2p((double)U[ca], (double)U[nc + ca], (double)U[2 * nc + ca], (double)U[3 * nc + ca], fix);
    const PrimV pb = c2p((double)U[cb], (double)U[nc + cb], (double)U[2 * nc + cb], (double)U[3 * nc + cb], fix);
    const double e = 0.5 * (pa.e + pb.e);
    num += (y * y - x * x) * e;
    den += (y * y + x * x) * e;
  }
  __shared__ double rn[256], rd[256];
  rn[threadIdx.x] = num;
  rd[threadIdx.x] = den;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      rn[threadIdx.x] += rn[threadIdx.x + h];
      rd[threadIdx.x] += rd[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = rn[0];
    part[2 * blockIdx.x + 1] = rd[0];
  }
}

__global__ void __launch_bounds__(256) k_eps2_final(const double* part, int nb, double* out3) {
  __shared__ double rn[256], rd[256];
  double num = 0.0, den = 0.0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) {
    num += part[2 * b];
    den += part[2 * b + 1];
  }
  rn[threadIdx.x] = num;
  rd[threadIdx.x] = den;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      rn[threadIdx.x] += rn[threadIdx.x + h];
      rd[threadIdx.x] += rd[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out3[0] = rn[0] / rd[0];
    out3[1] = rn[0];
    out3[2] = rd[0];
  }
}

template <class R>
__global__ void __launch_bounds__(256) k_eps2_seed(const R* __restrict__ U, Grid g, const double* eps3, R* lam,
                                                   double scale) {
  const int nx = g.n[0], ny = g.n[1];
  int k0, k1;
  z0_planes(g.n[2], k0, k1);
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)nx * ny) return;
  const long long nc = g.nc;
  const int i = (int)(q % nx), j = (int)(q / nx);
  const double x = cell_centre(i, nx, g.dx[0]), y = cell_centre(j, ny, g.dx[1]);
  const double eps2 = eps3[0], den = eps3[2];
  const double de = scale * 0.5 * ((y * y - x * x) - eps2 * (y * y + x * x)) / den;  // d eps2 / d e_plane
  const int planes[2] = {k0, k1};
  for (int p = 0; p < 2; ++p) {
    const long long cell = ((long long)planes[p] * ny + j) * nx + i;
    const PrimJ J = c2p_jac((double)U[cell], (double)U[nc + cell], (double)U[2 * nc + cell], (double)U[3 * nc + cell]);
    const double vb[3] = {0.0, 0.0, 0.0};
    double Eb, Mb[3];
    c2p_vjp(J, de, vb, Eb, Mb);
    if (k0 == k1 && p == 1) break;  // odd nz: the single plane takes both halves
    const double f = (k0 == k1) ? 2.0 : 1.0;
    lam[cell] = lam[cell] + (R)(f * Eb);
    for (int k = 0; k < 3; ++k) lam[(1 + k) * nc + cell] = lam[(1 + k) * nc + cell] + (R)(f * Mb[k]);
  }
}

// Adjoint of primitive (e, v, n) -> conserved (FP64 out [5][nc]):
// E = (4/3 g2 - 1/3) e, M = 4/3 e g2 v, N = n g, g2 = 1/(1 - v^2).
template <class R>
__global__ void __launch_bounds__(256) k_prim_vjp(const double* __restrict__ prim, const R* __restrict__ lam,
                                                  double* __restrict__ out, long long nc) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  const double e = prim[q], n = prim[4 * nc + q];
  const double v[3] = {prim[nc + q], prim[2 * nc + q], prim[3 * nc + q]};
  const double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
  const double g2 = 1.0 / (1.0 - v2);
  const double gm = sqrt(g2);
  const double lE = (double)lam[q], lN = (double)lam[4 * nc + q];
  const double lM[3] = {(double)lam[nc + q], (double)lam[2 * nc + q], (double)lam[3 * nc + q]};
  const double lMv = lM[0] * v[0] + lM[1] * v[1] + lM[2] * v[2];
  out[q] = lE * (4.0 * g2 - 1.0) / 3.0 + 4.0 / 3.0 * g2 * lMv;
  for (int k = 0; k < 3; ++k) {
    // d g2 / d v_k = 2 v_k g2^2
    const double dg2 = 2.0 * v[k] * g2 * g2;
    out[(1 + k) * nc + q] = lE * 4.0 / 3.0 * e * dg2 + 4.0 / 3.0 * e * (g2 * lM[k] + dg2 * lMv) + lN * n * v[k] * g2 * gm;
  }
  out[4 * nc + q] = lN * gm;
}

// ---------------------------------------------------------------------------
// Host-side launchers.
template <class R, int S>
void launch_bound_adj(int AX, const AdjArgs<R>& a, long long nl, hipStream_t st) {
  const unsigned nbb = (unsigned)((nl + kBoundLines - 1) / kBoundLines);
  const dim3 tb(kBoundLines * 10);
  if (AX == 0) hipLaunchKernelGGL((k_bound_adj<R, S, 0>), dim3(nbb), tb, 0, st, a);
  if (AX == 1) hipLaunchKernelGGL((k_bound_adj<R, S, 1>), dim3(nbb), tb, 0, st, a);
  if (AX == 2) hipLaunchKernelGGL((k_bound_adj<R, S, 2>), dim3(nbb), tb, 0, st, a);
}

// Lines per workgroup of a line adjoint along AX: 1 for x lines (contiguous);
// for y and z lines the request or fewer, so that n_x is a multiple, the
// workgroup has at most 1024 lanes and its LDS stays within 64 KiB.
// Automatic: 2 in FP32 (at n = 128 five such workgroups fit a CU's LDS, the
// occupancy of one line per workgroup, and the strided loads fetch half the
// cache lines: 128^3 backward 170 -> 150 ms; 4 lines: 156 ms), 1 in FP64
// (twice the LDS per line: two lines cost a workgroup per CU, 3 % slower).
template <class R>
int line_adj_lines(int AX, const AdjArgs<R>& a) {
  if (AX == 0) return 1;
  const int n = a.g.n[AX];
  int nl = a.lines > 0 ? a.lines : (sizeof(R) == 4 ? 2 : 1);
  while (nl > 1 && (a.g.n[0] % nl != 0 || n * nl > 1024 ||
                    (size_t)line_adj_pitch(n, nl) * nl * sizeof(R) > 65536))
    nl /= 2;
  return nl;
}

template <class R, int S, int AX, int NL>
void launch_line_adj(const AdjArgs<R>& a, hipStream_t st) {
  const int n = a.g.n[AX];
  const long long nlines = AX == 0 ? (long long)a.g.n[1] * a.g.n[2]
                                   : (AX == 1 ? (long long)a.g.n[0] * a.g.n[2] : (long long)a.g.n[0] * a.g.n[1]);
  const long long ng = nlines / NL;
  const int tb = ((n * NL + 63) / 64) * 64;
  const size_t lds = (size_t)line_adj_pitch(n, NL) * NL * sizeof(R);
  const unsigned nb = (unsigned)(((ng + 7) / 8) * 8);
  if (tb <= 256)
    hipLaunchKernelGGL((k_line_adj<R, S, AX, 256, NL>), dim3(nb), dim3(tb), lds, st, a);
  else
    hipLaunchKernelGGL((k_line_adj<R, S, AX, 1024, NL>), dim3(nb), dim3(tb), lds, st, a);
}

template <class R, int S>
void launch_adj_axis_t(int AX, const AdjArgs<R>& a0, hipStream_t st) {
  AdjArgs<R> a = a0;
  a.inv_d = R(1.0 / a.g.dx[AX]);
  const long long nl = AX == 0 ? (long long)a.g.n[1] * a.g.n[2]
                               : (AX == 1 ? (long long)a.g.n[0] * a.g.n[2] : (long long)a.g.n[0] * a.g.n[1]);
  // The outflow face n-1/2 adds to G: before the line kernel when that one
  // finishes G (fused combine), after it when that one starts G (first).
  const bool bound = a.g.bc[AX] == 0;
  if (bound && a.stage != 0) launch_bound_adj<R, S>(AX, a, nl, st);
  const int lines = line_adj_lines<R>(AX, a);
  if (AX == 0) launch_line_adj<R, S, 0, 1>(a, st);
  if (AX == 1) {
    if (lines == 4) launch_line_adj<R, S, 1, 4>(a, st);
    else if (lines == 2) launch_line_adj<R, S, 1, 2>(a, st);
    else launch_line_adj<R, S, 1, 1>(a, st);
  }
  if (AX == 2) {
    if (lines == 4) launch_line_adj<R, S, 2, 4>(a, st);
    else if (lines == 2) launch_line_adj<R, S, 2, 2>(a, st);
    else launch_line_adj<R, S, 2, 1>(a, st);
  }
  if (bound && a.stage == 0) launch_bound_adj<R, S>(AX, a, nl, st);
}

template <class R>
hipError_t launch_adj_axis(int AX, const AdjArgs<R>& a, int scheme, hipStream_t st) {
  if (scheme == kWenoJS)
    launch_adj_axis_t<R, kWenoJS>(AX, a, st);
  else if (scheme == kWenoLinear)
    launch_adj_axis_t<R, kWenoLinear>(AX, a, st);
  else
    launch_adj_axis_t<R, kWenoZ>(AX, a, st);
  return hipGetLastError();
}

template <class R>
hipError_t launch_jet_adj(const JetAdjArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((k_jet_adj<R>), dim3(1), dim3(512), 0, st, a);
  return hipGetLastError();
}

template <class R>
hipError_t launch_copy(const R* src, R* dst, long long n, hipStream_t st) {
  hipLaunchKernelGGL((k_copy<R>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_copy_f64(const double* src, double* dst, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

template <class R>
hipError_t launch_fill(R* dst, long long n, R v, hipStream_t st) {
  hipLaunchKernelGGL((k_fill<R>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, dst, n, v);
  return hipGetLastError();
}

template <class R>
hipError_t launch_eps2(const R* U, const Grid& g, double* part, double* out3, hipStream_t st) {
  hipLaunchKernelGGL((k_eps2_partial<R>), dim3(256), dim3(256), 0, st, U, g, part);
  hipLaunchKernelGGL(k_eps2_final, dim3(1), dim3(256), 0, st, part, 256, out3);
  return hipGetLastError();
}

template <class R>
hipError_t launch_eps2_seed(const R* U, const Grid& g, const double* out3, R* lam, double scale, hipStream_t st) {
  const long long np = (long long)g.n[0] * g.n[1];
  hipLaunchKernelGGL((k_eps2_seed<R>), dim3((unsigned)((np + 255) / 256)), dim3(256), 0, st, U, g, out3, lam, scale);
  return hipGetLastError();
}

template <class R>
hipError_t launch_prim_vjp(const double* prim, const R* lam, double* out, long long nc, hipStream_t st) {
  hipLaunchKernelGGL((k_prim_vjp<R>), dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, st, prim, lam, out, nc);
  return hipGetLastError();
}

#define HYDRO_ADJ_INSTANTIATE(R)                                                                               \
  template hipError_t launch_adj_axis<R>(int, const AdjArgs<R>&, int, hipStream_t);                           \
  template hipError_t launch_jet_adj<R>(const JetAdjArgs&, hipStream_t);                                     \
  template hipError_t launch_copy<R>(const R*, R*, long long, hipStream_t);                                   \
  template hipError_t launch_fill<R>(R*, long long, R, hipStream_t);                                          \
  template hipError_t launch_eps2<R>(const R*, const Grid&, double*, double*, hipStream_t);                    \
  template hipError_t launch_eps2_seed<R>(const R*, const Grid&, const double*, R*, double, hipStream_t);       \
  template hipError_t launch_prim_vjp<R>(const double*, const R*, double*, long long, hipStream_t);

HYDRO_ADJ_INSTANTIATE(double)
HYDRO_ADJ_INSTANTIATE(float)

}  // namespace hydro
