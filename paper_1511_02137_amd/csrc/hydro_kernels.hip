// hydro_kernels.hip -- HIP kernels of one SSP-RK3 stage for gfx950.
//
// The stage computes L(W) = D(W) + S(W) and the Runge-Kutta combine:
//   D: flux divergence of 7th-order WENO reconstructions of the
//      Lax-Friedrichs split fluxes F+- = (f +- W)/2 (alpha = 1), one axis at
//      a time, component by component (Eq. 1 with the paper's WENO7);
//   S: jet source, Eq. (2) and Eq. (3);
//   combine: Shu-Osher SSP-RK3.
//
// Work split (all kernels of a stage run on one stream):
//   k_xface   one workgroup per x-row.  Each lane recovers primitives for its
//             cell, stores the split x-fluxes of the row plus 4+4 ghost cells
//             in LDS, reconstructs its left face and writes the x-divergence.
//   k_xbound  the right boundary face of every row (outflow x only).
//   k_march   lanes along x (coalesced), each lane marches along y or z over
//             a segment, keeping the split fluxes of the 8-point stencil in
//             registers: one new cell and one face per step, no halo recompute.
//             The y-march adds its divergence to D; the z-march adds its own,
//             then does the RK combine and writes the stage output.
//   k_jet     the source at the jet cells (between the y- and z-march).
// All recovery of primitives is FP64; the flux and WENO arithmetic is in the
// field type R (double or float).  FP contraction is off: every fma is
// explicit, so every face is computed by the same sequence of roundings.

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
  const double e = 3.0 * (E * E - M2) / (E + sqrt(4.0 * E * E - 3.0 * M2));
  const double W = E + e / 3.0;
  r.e = e;
  r.v[0] = Mx / W;
  r.v[1] = My / W;
  r.v[2] = Mz / W;
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
  const R pr = (R)(p.e / 3.0);
  R f[5];
  f[0] = u[1 + AX];
  f[1] = (AX == 0) ? u[1] * vd + pr : u[1] * vd;
  f[2] = (AX == 1) ? u[2] * vd + pr : u[2] * vd;
  f[3] = (AX == 2) ? u[3] * vd + pr : u[3] * vd;
  f[4] = u[4] * vd;
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    Fp[c] = R(0.5) * (f[c] + u[c]);
    Fm[c] = R(0.5) * (f[c] - u[c]);
  }
}

// ---------------------------------------------------------------------------
// WENO7 value at x_{i+1/2} from the left, a0..a6 = a_{i-3}..a_{i+3}.
// The candidates q_k of the 4-point stencils enter as d_k (q_k - a_{i}),
// d = (1, 12, 18, 4)/35, written with the first differences, and the result
// is a_i + sum w_k d_k (q_k - a_i) / sum w_k d_k.  Smoothness indicators (Jiang-Shu: the
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
  const R ck = fma(g, D3, D2);
  return fma(sk, sk, fma(R(13.0 / 12.0) * ck, ck, fma(R(781.0 / 720.0) * D3, D3, eps)));
}

// Reciprocal for FP64: hardware estimate, two Newton steps (quadratic
// convergence from the estimate's ~23 bits to full precision).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}

// num / den from one reciprocal plus a residual correction.
__device__ __forceinline__ double div_nr(double num, double den) {
  const double r = rcp_nr(den);
  const double q = num * r;
  return fma(fma(-den, q, num), r, q);
}

template <class R, int S>
__device__ __forceinline__ R weno7(R a0, R a1, R a2, R a3, R a4, R a5, R a6, R eps) {
  // nested differences of the seven values
  const R e0 = a1 - a0, e1 = a2 - a1, e2 = a3 - a2, e3 = a4 - a3, e4 = a5 - a4, e5 = a6 - a5;
  // candidates as d_k (q_k - a3), from the differences
  const R r0 = fma(R(13.0 / 420.0), e2, fma(R(-10.0 / 420.0), e1, R(3.0 / 420.0) * e0));
  const R r1 = fma(R(3.0 / 35.0), e3, fma(R(4.0 / 35.0), e2, R(-1.0 / 35.0) * e1));
  const R r2 = fma(R(-3.0 / 70.0), e4, fma(R(18.0 / 70.0), e3, R(3.0 / 70.0) * e2));
  const R r3 = fma(R(1.0 / 105.0), e5, fma(R(-4.0 / 105.0), e4, R(9.0 / 105.0) * e3));
  if (S == kWenoLinear) return a3 + ((r0 + r1) + (r2 + r3));

  const R f0 = e1 - e0, f1 = e2 - e1, f2 = e3 - e2, f3 = e4 - e3, f4 = e5 - e4;
  const R g0 = f1 - f0, g1 = f2 - f1, g2 = f3 - f2, g3 = f4 - f3;
  const R b0 = smoothness<R>(e0, f0, g0, R(2.5), R(11.0 / 6.0), R(2), eps);
  const R b1 = smoothness<R>(e1, f1, g1, R(1.5), R(1.0 / 3.0), R(1), eps);
  const R b2 = smoothness<R>(e2, f2, g2, R(0.5), R(-1.0 / 6.0), R(0), eps);
  const R b3 = smoothness<R>(e3, f3, g3, R(-0.5), R(1.0 / 3.0), R(-1), eps);

  if (sizeof(R) == 8) {
    // Weights over a common denominator: with B_k = b_k^2 the WENO-Z weight
    // d_k (1 + tau^2/B_k) is proportional to d_k (B_k + tau^2) prod_{j!=k} B_j,
    // the Jiang-Shu weight d_k/B_k to d_k prod_{j!=k} B_j.  One division.
    const R B0 = b0 * b0, B1 = b1 * b1, B2 = b2 * b2, B3 = b3 * b3;
    const R P01 = B0 * B1, P23 = B2 * B3;
    R A0 = B1 * P23, A1 = B0 * P23, A2 = P01 * B3, A3 = P01 * B2;
    if (S == kWenoZ) {
      const R tau = fabs(fma(R(3), b1 - b2, b0 - b3));
      const R t2 = tau * tau;
      A0 = (B0 + t2) * A0;
      A1 = (B1 + t2) * A1;
      A2 = (B2 + t2) * A2;
      A3 = (B3 + t2) * A3;
    }
    const R num = fma(A3, r3, fma(A2, r2, fma(A1, r1, A0 * r0)));
    const R den = fma(A3, R(4.0 / 35.0), fma(A2, R(18.0 / 35.0), fma(A1, R(12.0 / 35.0), A0 * R(1.0 / 35.0))));
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
    const R den = fma(w3, R(4.0 / 35.0), fma(w2, R(18.0 / 35.0), fma(w1, R(12.0 / 35.0), w0 * R(1.0 / 35.0))));
    return fma(num, rcp_approx<R>(den), a3);
  }
}

// Face flux from the 8-point window Fp/Fm[m] = split fluxes at i-3+m:
// F(i+1/2) = R_L(F+_{i-3..i+3}) + R_L(F-_{i+4..i-2}).
template <class R, int S>
__device__ __forceinline__ R face_flux(const R* fp, const R* fm, R eps) {
  return weno7<R, S>(fp[0], fp[1], fp[2], fp[3], fp[4], fp[5], fp[6], eps) +
         weno7<R, S>(fm[7], fm[6], fm[5], fm[4], fm[3], fm[2], fm[1], eps);
}

__device__ __forceinline__ void add_fixups(unsigned long long* ctr, unsigned fix) {
  if (fix) atomicAdd(ctr, (unsigned long long)fix);
}

// ---------------------------------------------------------------------------
// x-faces: one workgroup per row (blockDim = nx rounded up to 64).
// LDS slot j holds the split fluxes of padded position p = j - 4.
template <class R, int S, int TB>
__global__ void __launch_bounds__(TB) k_xface(StageArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* s = reinterpret_cast<R*>(smem_raw);
  const int nx = a.g.n[0];
  const int P = nx + 8;
  R* sFp = s;
  R* sFm = s + 5 * P;
  const long long nc = a.g.nc;
  const long long rowbase = (long long)blockIdx.x * nx;
  unsigned fix = 0;

  for (int t = threadIdx.x; t < nx + 8; t += TB) {
    const int j = (t < nx) ? t + 4 : (t < nx + 4 ? t - nx : t);
    const int src = map_idx(j - 4, nx, a.g.bc[0]);
    R u[5];
    load5(a.W, nc, rowbase + src, u);
    const PrimV pv = c2p(u, fix);
    R Fp[5], Fm[5];
    split_flux<R, 0>(u, pv, Fp, Fm);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      sFp[c * P + j] = Fp[c];
      sFm[c * P + j] = Fm[c];
    }
  }
  __syncthreads();

  const int x = threadIdx.x;
  R Fh[5];
  if (x < nx) {
    // face x - 1/2: F+ at x-4..x+2 (slots x..x+6), F- at x-3..x+3 (slots x+1..x+7)
#pragma unroll
    for (int c = 0; c < 5; ++c) Fh[c] = face_flux<R, S>(sFp + c * P + x, sFm + c * P + x, a.eps);
  }
  __syncthreads();
  R* sF = s;  // [5][nx]
  if (x < nx) {
#pragma unroll
    for (int c = 0; c < 5; ++c) sF[c * nx + x] = Fh[c];
  }
  __syncthreads();
  if (x < nx) {
    const bool last = (x + 1 == nx);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const R l = sF[c * nx + x];
      R* d = a.D + c * nc + rowbase + x;
      if (!last) {
        *d = (l - sF[c * nx + x + 1]) * a.inv_d;
      } else if (a.g.bc[0]) {
        *d = (l - sF[c * nx]) * a.inv_d;  // periodic: the right face is face -1/2
      } else {
        *d = l;  // finished by k_xbound
      }
    }
  }
  add_fixups(a.fixups, fix);
}

// Right boundary face of every row (outflow x): points nx-4..nx+3.
template <class R, int S>
__global__ void __launch_bounds__(256) k_xbound(StageArgs<R> a) {
  const int nx = a.g.n[0];
  const long long rows = (long long)a.g.n[1] * a.g.n[2];
  const long long row = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rows) return;
  const long long nc = a.g.nc;
  const long long rowbase = row * nx;
  unsigned fix = 0;
  R fp[5][8], fm[5][8];
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    const int src = map_idx(nx - 4 + m, nx, 0);
    R u[5];
    load5(a.W, nc, rowbase + src, u);
    const PrimV pv = c2p(u, fix);
    R Fp[5], Fm[5];
    split_flux<R, 0>(u, pv, Fp, Fm);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      fp[c][m] = Fp[c];
      fm[c][m] = Fm[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const R r = face_flux<R, S>(fp[c], fm[c], a.eps);
    R* d = a.D + c * nc + rowbase + nx - 1;
    *d = (*d - r) * a.inv_d;
  }
  add_fixups(a.fixups, fix);
}

// ---------------------------------------------------------------------------
// March along axis AX (1 = y, 2 = z).  blockDim = (64, BY): lanes along x,
// threadIdx.y over the other transverse axis; blockIdx.z = segment of `seg`
// cells along AX.  LAST: z-march, which finishes L and does the RK combine.
template <class R, int S, int AX, bool LAST>
__global__ void __launch_bounds__(256) k_march(StageArgs<R> a) {
  const int nx = a.g.n[0], ny = a.g.n[1], nz = a.g.n[2];
  const int x = blockIdx.x * 64 + threadIdx.x;
  const int o = blockIdx.y * blockDim.y + threadIdx.y;
  const int n = (AX == 1) ? ny : nz;
  const int no = (AX == 1) ? nz : ny;
  if (x >= nx || o >= no) return;
  const long long nc = a.g.nc;
  const long long stride = (AX == 1) ? (long long)nx : (long long)nx * ny;
  const long long base = (AX == 1) ? (long long)o * nx * ny + x : (long long)o * nx + x;
  const int bc = a.g.bc[AX];
  const int i0 = blockIdx.z * a.seg;
  const int i1 = min(i0 + a.seg, n);
  unsigned fix = 0;

  R fp[5][8], fm[5][8];  // split fluxes at points i-3..i+4 for face i+1/2
#pragma unroll
  for (int m = 0; m < 8; ++m) {
    R u[5];
    load5(a.W, nc, base + (long long)map_idx(i0 - 4 + m, n, bc) * stride, u);
    const PrimV pv = c2p(u, fix);
    R Fp[5], Fm[5];
    split_flux<R, AX>(u, pv, Fp, Fm);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      fp[c][m] = Fp[c];
      fm[c][m] = Fm[c];
    }
  }
  R prev[5];
#pragma unroll
  for (int c = 0; c < 5; ++c) prev[c] = face_flux<R, S>(fp[c], fm[c], a.eps);

  for (int i = i0; i < i1; ++i) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
#pragma unroll
      for (int m = 0; m < 7; ++m) {
        fp[c][m] = fp[c][m + 1];
        fm[c][m] = fm[c][m + 1];
      }
    }
    {
      R u[5];
      load5(a.W, nc, base + (long long)map_idx(i + 4, n, bc) * stride, u);
      const PrimV pv = c2p(u, fix);
      R Fp[5], Fm[5];
      split_flux<R, AX>(u, pv, Fp, Fm);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        fp[c][7] = Fp[c];
        fm[c][7] = Fm[c];
      }
    }
    const long long cell = base + (long long)i * stride;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const R fh = face_flux<R, S>(fp[c], fm[c], a.eps);
      const R div = (prev[c] - fh) * a.inv_d;
      prev[c] = fh;
      R* d = a.D + c * nc + cell;
      if (!LAST) {
        *d = *d + div;
      } else {
        const R L = *d + div;
        const R w = a.W[c * nc + cell];
        R outv;
        if (a.stage == 0) {
          outv = L;  // right-hand side only
        } else if (a.stage == 1) {
          outv = w + a.dt * L;
        } else if (a.stage == 2) {
          outv = R(0.75) * a.Un[c * nc + cell] + R(0.25) * (w + a.dt * L);
        } else {
          outv = R(1.0 / 3.0) * a.Un[c * nc + cell] + R(2.0 / 3.0) * (w + a.dt * L);
        }
        a.out[c * nc + cell] = outv;
      }
    }
  }
  add_fixups(a.fixups, fix);
}

// ---------------------------------------------------------------------------
// y- or z-faces from an LDS tile (AX = 1 or 2).  A workgroup of 512 lanes
// owns 16 cells along x (coalesced 128-byte rows) by 32 cells along AX at one
// value of the remaining axis.  It stores the split AX-fluxes of its 16 x 40
// points (4 ghost rows on each side) in LDS, reconstructs the 33 face rows
// (one face per lane, one extra row for 16 lanes) and forms the divergence.
// LAST (z): adds D, does the RK combine with the cell's own stage input kept
// in registers from the load, and writes the stage output.
constexpr int kTileX = 16;
constexpr int kTileA = 32;
constexpr int kTileP = kTileA + 8;   // points along AX
constexpr int kTileXP = kTileX;      // x pitch of the LDS arrays (128-byte rows)

template <class R, int S, int AX, bool LAST>
__global__ void __launch_bounds__(512) k_tile(StageArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* s = reinterpret_cast<R*>(smem_raw);
  R* sFp = s;                              // [5][kTileP][kTileXP]
  R* sFm = s + 5 * kTileP * kTileXP;       // [5][kTileP][kTileXP]
  const int nx = a.g.n[0], ny = a.g.n[1];
  const int n = a.g.n[AX];
  const int bc = a.g.bc[AX];
  const long long nc = a.g.nc;
  const int tx = threadIdx.x & (kTileX - 1);
  const int ta = threadIdx.x >> 4;  // 0..31
  const int x = blockIdx.x * kTileX + tx;
  const int a0 = blockIdx.y * kTileA;
  const int o = blockIdx.z;
  const long long stride = (AX == 1) ? (long long)nx : (long long)nx * ny;
  const long long base = (AX == 1) ? (long long)o * nx * ny + x : (long long)o * nx + x;
  const bool xin = x < nx;
  unsigned fix = 0;

  R own[5];
  // pass 1: own cell (slot ta + 4)
  {
    const int p = a0 + ta;
    if (xin) {
      load5(a.W, nc, base + (long long)map_idx(p, n, bc) * stride, own);
      const PrimV pv = c2p(own, fix);
      R Fp[5], Fm[5];
      split_flux<R, AX>(own, pv, Fp, Fm);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        sFp[(c * kTileP + ta + 4) * kTileXP + tx] = Fp[c];
        sFm[(c * kTileP + ta + 4) * kTileXP + tx] = Fm[c];
      }
    }
  }
  // pass 2: 4 ghost rows on each side (128 lanes)
  if (threadIdx.x < 8 * kTileX) {
    const int h = ta;  // 0..7
    const int j = (h < 4) ? h : h + kTileA;
    const int p = a0 - 4 + j;
    if (xin) {
      R u[5];
      load5(a.W, nc, base + (long long)map_idx(p, n, bc) * stride, u);
      const PrimV pv = c2p(u, fix);
      R Fp[5], Fm[5];
      split_flux<R, AX>(u, pv, Fp, Fm);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        sFp[(c * kTileP + j) * kTileXP + tx] = Fp[c];
        sFm[(c * kTileP + j) * kTileXP + tx] = Fm[c];
      }
    }
  }
  __syncthreads();

  // faces f = 0..32: face (a0 - 1 + f) + 1/2; F+ at slots f..f+6, F- at f+1..f+7
  const int nf = min(kTileA, n - a0) + 1;  // face rows this tile needs
  R Fh[5], Fh2[5];
  const bool has1 = xin && ta < nf;
  const bool has2 = xin && threadIdx.x < kTileX && kTileA < nf;
  if (has1) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const R* fp = sFp + (c * kTileP + ta) * kTileXP + tx;
      const R* fm = sFm + (c * kTileP + ta) * kTileXP + tx;
      Fh[c] = weno7<R, S>(fp[0], fp[kTileXP], fp[2 * kTileXP], fp[3 * kTileXP], fp[4 * kTileXP], fp[5 * kTileXP],
                          fp[6 * kTileXP], a.eps) +
              weno7<R, S>(fm[7 * kTileXP], fm[6 * kTileXP], fm[5 * kTileXP], fm[4 * kTileXP], fm[3 * kTileXP],
                          fm[2 * kTileXP], fm[kTileXP], a.eps);
    }
  }
  if (has2) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const R* fp = sFp + (c * kTileP + kTileA) * kTileXP + tx;
      const R* fm = sFm + (c * kTileP + kTileA) * kTileXP + tx;
      Fh2[c] = weno7<R, S>(fp[0], fp[kTileXP], fp[2 * kTileXP], fp[3 * kTileXP], fp[4 * kTileXP], fp[5 * kTileXP],
                           fp[6 * kTileXP], a.eps) +
               weno7<R, S>(fm[7 * kTileXP], fm[6 * kTileXP], fm[5 * kTileXP], fm[4 * kTileXP], fm[3 * kTileXP],
                           fm[2 * kTileXP], fm[kTileXP], a.eps);
    }
  }
  __syncthreads();
  R* sF = s;  // [5][kTileA + 1][kTileXP]
  if (has1) {
#pragma unroll
    for (int c = 0; c < 5; ++c) sF[(c * (kTileA + 1) + ta) * kTileXP + tx] = Fh[c];
  }
  if (has2) {
#pragma unroll
    for (int c = 0; c < 5; ++c) sF[(c * (kTileA + 1) + kTileA) * kTileXP + tx] = Fh2[c];
  }
  __syncthreads();

  const int ac = a0 + ta;
  if (xin && ac < n) {
    const long long cell = base + (long long)ac * stride;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const R div = (sF[(c * (kTileA + 1) + ta) * kTileXP + tx] - sF[(c * (kTileA + 1) + ta + 1) * kTileXP + tx]) * a.inv_d;
      R* d = a.D + c * nc + cell;
      if (!LAST) {
        *d = *d + div;
      } else {
        const R L = *d + div;
        const R w = own[c];
        R outv;
        if (a.stage == 0) {
          outv = L;
        } else if (a.stage == 1) {
          outv = w + a.dt * L;
        } else if (a.stage == 2) {
          outv = R(0.75) * a.Un[c * nc + cell] + R(0.25) * (w + a.dt * L);
        } else {
          outv = R(1.0 / 3.0) * a.Un[c * nc + cell] + R(2.0 / 3.0) * (w + a.dt * L);
        }
        a.out[c * nc + cell] = outv;
      }
    }
  }
  add_fixups(a.fixups, fix);
}

// ---------------------------------------------------------------------------
// Jet source (Eq. 2 and 3).  One workgroup of 512 threads; jets in order.
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

template <class R>
__global__ void __launch_bounds__(512) k_jet(JetArgs a) {
  const R* W = static_cast<const R*>(a.W);
  R* D = static_cast<R*>(a.D);
  const long long nc = a.g.nc;
  const double dV = a.g.dx[0] * a.g.dx[1] * a.g.dx[2];
  __shared__ double red_w[512], red_t[512];
  __shared__ double wax[3][7];
  __shared__ int ctr_s[3];
  __shared__ int inside_s;
  unsigned fix = 0;
  for (int j = 0; j < a.njet; ++j) {
    const JetDev jt = a.s->jets[j];
    const bool chi = a.s->E_jet[j] > 0.0;
    const double ell = a.t - jt.t_start;
    double P = 0.0;
    if (threadIdx.x == 0) {
      int in = (chi && ell >= 0.0) ? 1 : 0;
      for (int d = 0; d < 3; ++d) {
        const double x = jt.x0[d] + jt.dir[d] * ell;
        const int c = ngp_index(x, a.g.n[d], a.g.dx[d]);
        ctr_s[d] = c;
        if (c < 0) in = 0;
        if (a.deposit == 1) {
          double sum = 0.0;
          for (int m = 0; m < 7; ++m) {
            const double del = cell_centre(c - 3 + m, a.g.n[d], a.g.dx[d]) - x;
            wax[d][m] = exp(-(del * del) / (2.0 * a.g.dx[d] * a.g.dx[d]));
            sum = sum + wax[d][m];
          }
          for (int m = 0; m < 7; ++m) wax[d][m] = wax[d][m] / sum;
        }
      }
      inside_s = in;
    }
    __syncthreads();
    if (inside_s) {
      if (a.deposit == 0) {
        if (threadIdx.x == 0) {
          const long long cell = ((long long)ctr_s[2] * a.g.n[1] + ctr_s[1]) * a.g.n[0] + ctr_s[0];
          R u[5];
          load5(W, nc, cell, u);
          const PrimV pv = c2p(u, fix);
          const double T = temperature(pv.e, a.eos_dof, a.hbarc);
          P = energy_loss(jt, T, ell, a.hbarc);
          const double s0 = P / dV;
          D[cell] = D[cell] + (R)s0;
          for (int d = 0; d < 3; ++d) D[(1 + d) * nc + cell] = D[(1 + d) * nc + cell] + (R)(jt.dir[d] * s0);
        }
      } else {
        // 7^3 footprint, thread t < 343 owns cell (mi, mj, mk)
        const int t = threadIdx.x;
        double w = 0.0, wT = 0.0;
        long long cell = -1;
        if (t < 343) {
          const int mi = t % 7, mj = (t / 7) % 7, mk = t / 49;
          const int i = ctr_s[0] - 3 + mi, jj = ctr_s[1] - 3 + mj, k = ctr_s[2] - 3 + mk;
          if (i >= 0 && i < a.g.n[0] && jj >= 0 && jj < a.g.n[1] && k >= 0 && k < a.g.n[2]) {
            cell = ((long long)k * a.g.n[1] + jj) * a.g.n[0] + i;
            w = wax[0][mi] * wax[1][mj] * wax[2][mk];
            R u[5];
            load5(W, nc, cell, u);
            const PrimV pv = c2p(u, fix);
            wT = w * temperature(pv.e, a.eos_dof, a.hbarc);
          }
        }
        red_w[t] = w;
        red_t[t] = wT;
        __syncthreads();
        for (int h = 256; h > 0; h >>= 1) {
          if (t < h) {
            red_w[t] = red_w[t] + red_w[t + h];
            red_t[t] = red_t[t] + red_t[t + h];
          }
          __syncthreads();
        }
        const double wsum = red_w[0];
        const double T = red_t[0] / wsum;
        const double Pj = energy_loss(jt, T, ell, a.hbarc);
        P = Pj * wsum;
        if (cell >= 0) {
          const double s0 = Pj * w / dV;
          D[cell] = D[cell] + (R)s0;
          for (int d = 0; d < 3; ++d) D[(1 + d) * nc + cell] = D[(1 + d) * nc + cell] + (R)(jt.dir[d] * s0);
        }
      }
    }
    if (threadIdx.x == 0 && a.stage > 0) {
      a.s->P[a.stage - 1][j] = P;
      if (a.stage == 3 && chi) {
        const double dep =
            a.dt * ((1.0 / 6.0) * a.s->P[0][j] + (1.0 / 6.0) * a.s->P[1][j] + (2.0 / 3.0) * a.s->P[2][j]);
        a.s->ledger = a.s->ledger + dep;
        const double rest = a.s->E_jet[j] - dep;
        a.s->E_jet[j] = rest > 0.0 ? rest : 0.0;
      }
    }
    __syncthreads();
  }
  add_fixups(&a.s->fixups, fix);
}

// ---------------------------------------------------------------------------
// FP64 sums of the five fields, fixed order: per-block partials, then one block.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

template <class R>
__global__ void __launch_bounds__(256) k_sums_partial(const R* __restrict__ U, long long nc, double* part) {
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 5; ++c) acc[c] += (double)U[c * nc + i];
  }
  __shared__ double red[5][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < 5; ++c) {
    const double v = wave_sum(acc[c]);
    if (lane == 0) red[c][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    const int c = threadIdx.x;
    part[(long long)blockIdx.x * 5 + c] = (red[c][0] + red[c][1]) + (red[c][2] + red[c][3]);
  }
}

__global__ void __launch_bounds__(256) k_sums_final(const double* part, int nblocks, double dV, DevScalars* s) {
  __shared__ double red[5][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int c = 0; c < 5; ++c) {
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) acc += part[(long long)b * 5 + c];
    const double v = wave_sum(acc);
    if (lane == 0) red[c][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < 5) {
    const int c = threadIdx.x;
    s->sums[c] = ((red[c][0] + red[c][1]) + (red[c][2] + red[c][3])) * dV;
  }
}

// ---------------------------------------------------------------------------
// Primitive (e, vx, vy, vz, n; FP64) -> conserved: E = (e+p) g^2 - p,
// M = (e+p) g^2 v, N = n g, p = e/3.
template <class R>
__global__ void __launch_bounds__(256) k_prim_to_cons(const double* __restrict__ prim, R* __restrict__ U, long long nc) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nc) return;
  const double e = prim[q], v0 = prim[nc + q], v1 = prim[2 * nc + q], v2 = prim[3 * nc + q], n = prim[4 * nc + q];
  const double v2s = v0 * v0 + v1 * v1 + v2 * v2;
  const double g2 = 1.0 / (1.0 - v2s);
  const double p = e / 3.0;
  const double w = (e + p) * g2;
  U[q] = (R)(w - p);
  U[nc + q] = (R)(w * v0);
  U[2 * nc + q] = (R)(w * v1);
  U[3 * nc + q] = (R)(w * v2);
  U[4 * nc + q] = (R)(n * sqrt(g2));
}

// Conserved -> (e, vx, vy, vz, n, T) in the field type.
template <class R>
__global__ void __launch_bounds__(256) k_primitives(const R* __restrict__ U, R* __restrict__ prim, long long nc,
                                                    double g, double hc, unsigned long long* fixups) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned fix = 0;
  if (q < nc) {
    R u[5];
    load5(U, nc, q, u);
    const PrimV pv = c2p(u, fix);
    const double v2 = pv.v[0] * pv.v[0] + pv.v[1] * pv.v[1] + pv.v[2] * pv.v[2];
    prim[q] = (R)pv.e;
    prim[nc + q] = (R)pv.v[0];
    prim[2 * nc + q] = (R)pv.v[1];
    prim[3 * nc + q] = (R)pv.v[2];
    prim[4 * nc + q] = (R)((double)u[4] * sqrt(1.0 - v2));
    prim[5 * nc + q] = (R)temperature(pv.e, g, hc);
  }
  add_fixups(fixups, fix);
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from hydro_api.hip).
template <class R, int S>
void launch_xface_t(const StageArgs<R>& base, hipStream_t st) {
  StageArgs<R> a = base;
  const int nx = a.g.n[0];
  a.inv_d = R(1.0 / a.g.dx[0]);
  const size_t lds = (size_t)max(10 * (nx + 8), 5 * nx) * sizeof(R);
  const unsigned rows = (unsigned)((long long)a.g.n[1] * a.g.n[2]);
  if (nx <= 256) {
    hipLaunchKernelGGL((k_xface<R, S, 256>), dim3(rows), dim3(256), lds, st, a);
  } else {
    hipLaunchKernelGGL((k_xface<R, S, 1024>), dim3(rows), dim3(1024), lds, st, a);
  }
}

template <class R, int S>
void launch_xbound_t(const StageArgs<R>& base, hipStream_t st) {
  StageArgs<R> a = base;
  a.inv_d = R(1.0 / a.g.dx[0]);
  const long long rows = (long long)a.g.n[1] * a.g.n[2];
  const unsigned nb = (unsigned)((rows + 255) / 256);
  hipLaunchKernelGGL((k_xbound<R, S>), dim3(nb), dim3(256), 0, st, a);
}

template <class R, int S, int AX>
void launch_march_t(const StageArgs<R>& base, int seg, hipStream_t st) {
  StageArgs<R> a = base;
  const int nx = a.g.n[0], ny = a.g.n[1], nz = a.g.n[2];
  a.seg = seg;
  a.inv_d = R(1.0 / a.g.dx[AX]);
  const int n = (AX == 1) ? ny : nz;
  const int no = (AX == 1) ? nz : ny;
  dim3 grid((nx + 63) / 64, (no + 3) / 4, (n + seg - 1) / seg);
  hipLaunchKernelGGL((k_march<R, S, AX, AX == 2>), grid, dim3(64, 4), 0, st, a);
}

template <class R, int S, int AX>
void launch_tile_t(const StageArgs<R>& base, hipStream_t st) {
  StageArgs<R> a = base;
  const int nx = a.g.n[0];
  a.inv_d = R(1.0 / a.g.dx[AX]);
  const int n = a.g.n[AX];
  const int no = (AX == 1) ? a.g.n[2] : a.g.n[1];
  const size_t lds = (size_t)2 * 5 * kTileP * kTileXP * sizeof(R);
  dim3 grid((nx + kTileX - 1) / kTileX, (n + kTileA - 1) / kTileA, no);
  hipLaunchKernelGGL((k_tile<R, S, AX, AX == 2>), grid, dim3(512), lds, st, a);
}

// kernel: 0 x-faces, 1 x boundary faces, 2 y-march, 3 z-march (+ combine),
// 4 y-tile, 5 z-tile (+ combine)
template <class R>
hipError_t launch_face_kernel(int kernel, const StageArgs<R>& a, int scheme, int seg, hipStream_t st) {
#define HYDRO_DISPATCH(S)                                  \
  switch (kernel) {                                        \
    case 0: launch_xface_t<R, S>(a, st); break;            \
    case 1: launch_xbound_t<R, S>(a, st); break;           \
    case 2: launch_march_t<R, S, 1>(a, seg, st); break;    \
    case 3: launch_march_t<R, S, 2>(a, seg, st); break;    \
    case 4: launch_tile_t<R, S, 1>(a, st); break;          \
    default: launch_tile_t<R, S, 2>(a, st); break;         \
  }
  if (scheme == kWenoJS) {
    HYDRO_DISPATCH(kWenoJS)
  } else if (scheme == kWenoLinear) {
    HYDRO_DISPATCH(kWenoLinear)
  } else {
    HYDRO_DISPATCH(kWenoZ)
  }
#undef HYDRO_DISPATCH
  return hipGetLastError();
}

template <class R>
hipError_t launch_jet(const JetArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((k_jet<R>), dim3(1), dim3(512), 0, st, a);
  return hipGetLastError();
}

template <class R>
hipError_t launch_sums(const R* U, long long nc, double dV, double* part, DevScalars* s, hipStream_t st) {
  hipLaunchKernelGGL((k_sums_partial<R>), dim3(kSumBlocks), dim3(256), 0, st, U, nc, part);
  hipLaunchKernelGGL(k_sums_final, dim3(1), dim3(256), 0, st, part, kSumBlocks, dV, s);
  return hipGetLastError();
}

template <class R>
hipError_t launch_prim_to_cons(const double* prim, R* U, long long nc, hipStream_t st) {
  const unsigned nb = (unsigned)((nc + 255) / 256);
  hipLaunchKernelGGL((k_prim_to_cons<R>), dim3(nb), dim3(256), 0, st, prim, U, nc);
  return hipGetLastError();
}

template <class R>
hipError_t launch_primitives(const R* U, R* prim, long long nc, double g, double hc, unsigned long long* fixups,
                             hipStream_t st) {
  const unsigned nb = (unsigned)((nc + 255) / 256);
  hipLaunchKernelGGL((k_primitives<R>), dim3(nb), dim3(256), 0, st, U, prim, nc, g, hc, fixups);
  return hipGetLastError();
}

#define HYDRO_INSTANTIATE(R)                                                                          \
  template hipError_t launch_face_kernel<R>(int, const StageArgs<R>&, int, int, hipStream_t);          \
  template hipError_t launch_jet<R>(const JetArgs&, hipStream_t);                                     \
  template hipError_t launch_sums<R>(const R*, long long, double, double*, DevScalars*, hipStream_t); \
  template hipError_t launch_prim_to_cons<R>(const double*, R*, long long, hipStream_t);              \
  template hipError_t launch_primitives<R>(const R*, R*, long long, double, double, unsigned long long*, hipStream_t);

HYDRO_INSTANTIATE(double)
HYDRO_INSTANTIATE(float)

}  // namespace hydro
