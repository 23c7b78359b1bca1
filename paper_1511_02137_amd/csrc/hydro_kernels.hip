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
//   k_xface   one workgroup per group of whole x-rows.  Each lane recovers
//             primitives for its cell, stores the split x-fluxes of the row
//             plus 4+4 ghost cells in LDS, reconstructs one split of two
//             neighbouring faces (or both splits of its left face) and
//             writes the x-divergence.
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

#include "hydro_device.hpp"
#include "hydro_internal.hpp"

namespace hydro {

// ---------------------------------------------------------------------------
// x-faces: a workgroup owns rpi = blockDim / nx whole rows (row0, row0 + 1,
// ...; fewer at the end of the grid).  LDS per row: the split fluxes of its nx
// cells and 8 ghost slots (slot j holds padded position j - 4), then the face
// values.  One lane per cell: it recovers its cell, stores the split fluxes
// (also into every ghost slot that copies the cell), reconstructs faces
// (rows of even length: lane 2q + h the split h of faces 2q - 1/2 and
// 2q + 1/2; otherwise the cell's left face) and forms the divergence; the
// outflow right face of the last cell is added by k_xbound.
// What the face kernels keep per point: the Lax-Friedrichs split fluxes
// (F+, F-), or with MUSTA-FORCE the conserved values themselves (in the F+
// slots; no recovery needed).
template <class R, int S, int AX>
__device__ __forceinline__ void point_values(const R u[5], R Fp[5], R Fm[5], unsigned& fix) {
  if constexpr ((S & kMusta) != 0) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      Fp[c] = u[c];
      Fm[c] = R(0);
    }
  } else {
    const PrimV pv = c2p(u, fix);
    split_flux<R, AX>(u, pv, Fp, Fm);
  }
}

// SSP-RK3 combine of the last face kernel of a stage (z).  With L = Dxy + Dz
// (Dxy: the x and y divergences and the source, already in D; Dz: the z
// divergence), the stage value w + dt L enters as p = w + dt Dxy, then
// p + dt Dz (two fmas), so that a kernel can fold w into p before its
// reconstructions and keep one value per field instead of two.  Stage 0
// returns L itself.
template <class R>
__device__ __forceinline__ R rk_pre(int stage, R w, R dxy, R dt) {
  return stage == 0 ? dxy : fma(dt, dxy, w);
}
template <class R>
__device__ __forceinline__ R rk_out(int stage, R p, R dz, R dt, const R* Un, long long i) {
  if (stage == 0) return p + dz;
  const R v = fma(dt, dz, p);
  if (stage == 1) return v;
  if (stage == 2) return R(0.75) * Un[i] + R(0.25) * v;
  return R(1.0 / 3.0) * Un[i] + R(2.0 / 3.0) * v;
}
// the same with U^n already read (un; used in stages 2 and 3 only)
template <class R>
__device__ __forceinline__ R rk_out_v(int stage, R p, R dz, R dt, R un) {
  if (stage == 0) return p + dz;
  const R v = fma(dt, dz, p);
  if (stage == 1) return v;
  if (stage == 2) return R(0.75) * un + R(0.25) * v;
  return R(1.0 / 3.0) * un + R(2.0 / 3.0) * v;
}

template <class R, int S, bool PAIRS>
__device__ __forceinline__ void xrows_body(const StageArgs<R>& a, long long row0, int rpi, R* s) {
  const int nx = a.g.n[0];
  const int P = nx + 8;
  const long long rows = (long long)a.g.n[1] * a.g.n[2];
  const long long nc = a.g.nc;
  const int r = threadIdx.x / nx;
  const int x = threadIdx.x - r * nx;
  const long long row = row0 + r;
  const bool act = r < rpi && row < rows;
  const long long rowbase = row * nx;
  R* sFp = s + (size_t)r * 10 * P;
  R* sFm = sFp + 5 * P;
  unsigned fix = 0;
  // Plain WENO faces of rows with an even number of cells are taken in
  // pairs (as in the y/z tiles); the F- points are then stored in reverse
  // slot order.
  const bool pair = PAIRS && (S & (kPP | kMusta)) == 0 && (nx & 1) == 0;
  const int mrev = pair ? P - 1 : 0, msgn = pair ? -1 : 1;  // F- slot j at mrev + msgn j

  if (act) {
    R u[5];
    load5(a.W, nc, rowbase + x, u);
    R Fp[5], Fm[5];
    point_values<R, S, 0>(u, Fp, Fm, fix);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      sFp[c * P + x + 4] = Fp[c];
      sFm[c * P + mrev + msgn * (x + 4)] = Fm[c];
    }
    // ghost slots 0..3 and nx+4..nx+7, each filled by the lane whose cell it
    // copies: outflow, the edge lanes; periodic, the lanes four from the far
    // end (rows of at least 8 cells; shorter rows take the general map)
    auto put = [&](int j) {
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        sFp[c * P + j] = Fp[c];
        sFm[c * P + mrev + msgn * j] = Fm[c];
      }
    };
    if (nx >= 8) {
      if (a.g.bc[0]) {
        if (x >= nx - 4) put(x - nx + 4);
        if (x < 4) put(nx + 4 + x);
      } else if (x == 0 || x == nx - 1) {
        const int j0 = x == 0 ? 0 : nx + 4;
        for (int k = 0; k < 4; ++k) put(j0 + k);
      }
    } else {
      for (int g = 0; g < 8; ++g) {
        const int j = g < 4 ? g : nx + g;
        if (map_idx(j - 4, nx, a.g.bc[0]) == x) put(j);
      }
    }
  }
  __syncthreads();

  if (pair) {
    // lane (q, h) = (x >> 1, x & 1): split h of the faces x' - 1/2, x' = 2q,
    // 2q + 1, one field at a time; the two split values go into the field's
    // own F+ and F- areas once every lane of the workgroup is past it
    const int q = x >> 1, h = x & 1;
    const R* b = h ? sFm + (P - 9 - 2 * q) : sFp + 2 * q;
    R* dst = h ? sFm : sFp;
    const int fa = 2 * q + h, fb = 2 * q + 1 - h;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      R lo, hi;
      if (act) {
        const R* v = b + c * P;
        weno7_pair<R, (S & 7)>(v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7], a.eps, lo, hi);
      }
      __syncthreads();
      if (act) {
        dst[c * P + fa] = lo;
        dst[c * P + fb] = hi;
      }
    }
    __syncthreads();
    if (act) {
      const int xr = (x + 1 == nx) ? 0 : x + 1;  // periodic: the right face of cell nx-1 is face -1/2
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        const R l = sFp[c * P + x] + sFm[c * P + x];
        R* d = a.D + c * nc + rowbase + x;
        if (x + 1 < nx || a.g.bc[0]) {
          *d = (l - (sFp[c * P + xr] + sFm[c * P + xr])) * a.inv_d;
        } else {
          *d = l;  // finished by k_xbound
        }
      }
    }
    add_fixups(a.fixups, fix);
    return;
  }
  R Fh[5];
  if (act) {
    // face x - 1/2: F+ at x-4..x+2 (slots x..x+6), F- at x-3..x+3 (slots x+1..x+7)
#pragma unroll
    for (int c = 0; c < 5 && (S & kMusta) == 0; ++c)
      Fh[c] = face_flux<R, (S & 7)>(sFp + c * P + x, sFm + c * P + x, a.eps);
    if constexpr ((S & kMusta) != 0)
      musta_face<R, (S & 7), 0>([&](int c, int m) { return sFp[c * P + x + m]; }, a.eps, a.musta_k, Fh, fix);
    if constexpr ((S & kPP) != 0) {  // cells x - 1 and x: slots x + 3 and x + 4
      pp_limit<R>(
          Fh, [&](int c, int k) { return ((k & 1) ? sFm : sFp)[c * P + x + 3 + (k >> 1)]; }, a.pp_mu);
    }
  }
  __syncthreads();
  R* sF = s + (size_t)r * 5 * nx;  // [5][nx] per row
  if (act) {
#pragma unroll
    for (int c = 0; c < 5; ++c) sF[c * nx + x] = Fh[c];
  }
  __syncthreads();
  if (act) {
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

template <class R, int S, int TB>
__global__ void __launch_bounds__(TB) k_xface(StageArgs<R> a, int rpi) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  xrows_body<R, S, true>(a, (long long)blockIdx.x * rpi, rpi, reinterpret_cast<R*>(smem_raw));
}

// Right boundary face of every row (outflow x): points nx-4..nx+3 (the last
// four copies of cell nx-1).  A workgroup takes 32 rows: one lane per (row,
// point) forms the split fluxes, one lane per (row, field, split) does one
// reconstruction, one lane per (row, field) adds R+ + R- to finish D.
constexpr int kXBoundRows = 32;

template <class R, int S>
__device__ __forceinline__ void xbound_body(const StageArgs<R>& a, long long group) {
  __shared__ R sF[kXBoundRows][8][10];
  __shared__ R sR[kXBoundRows][10];
  const int nx = a.g.n[0];
  const long long rows = (long long)a.g.n[1] * a.g.n[2];
  const long long nc = a.g.nc;
  const int t = threadIdx.x;
  unsigned fix = 0;
  if (t < kXBoundRows * 8) {
    const int l = t >> 3, m = t & 7;
    const long long row = group * kXBoundRows + l;
    if (row < rows) {
      R u[5];
      load5(a.W, nc, row * nx + map_idx(nx - 4 + m, nx, 0), u);
      R Fp[5], Fm[5];
      point_values<R, S, 0>(u, Fp, Fm, fix);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        sF[l][m][c] = Fp[c];
        sF[l][m][5 + c] = Fm[c];
      }
    }
  }
  __syncthreads();
  {
    const int l = t / 10, r = t % 10, c = r >> 1;
    const long long row = group * kXBoundRows + l;
    if (row < rows) {
      const int cm = ((S & kMusta) != 0) ? c : 5 + c;  // MUSTA: both states from the conserved values
      sR[l][r] = (r & 1) == 0
                     ? weno7<R, (S & 7)>(sF[l][0][c], sF[l][1][c], sF[l][2][c], sF[l][3][c], sF[l][4][c], sF[l][5][c],
                                   sF[l][6][c], a.eps)
                     : weno7<R, (S & 7)>(sF[l][7][cm], sF[l][6][cm], sF[l][5][cm], sF[l][4][cm],
                                   sF[l][3][cm], sF[l][2][cm], sF[l][1][cm], a.eps);
    }
  }
  __syncthreads();
  if constexpr ((S & kMusta) != 0) {  // one lane per row: the MUSTA-FORCE flux of (uL, uR)
    if (t < kXBoundRows && group * kXBoundRows + t < rows) {
      const int l = t;
      R uL[5], uR[5], F[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        uL[c] = sR[l][2 * c];
        uR[c] = sR[l][2 * c + 1];
      }
      musta_force<R, 0>(uL, uR, a.musta_k, F, fix);
#pragma unroll
      for (int c = 0; c < 5; ++c) sF[l][0][c] = F[c];  // point 0 is no longer read
    }
    __syncthreads();
  }
  if constexpr ((S & kPP) != 0) {  // one lane per row: cell nx-1 (point 3) and its copy (point 4)
    if (t < kXBoundRows && group * kXBoundRows + t < rows) {
      const int l = t;
      R H[5];
#pragma unroll
      for (int c = 0; c < 5; ++c) H[c] = sR[l][2 * c] + sR[l][2 * c + 1];
      pp_limit<R>(H, [&](int c, int k) { return sF[l][3 + (k >> 1)][(k & 1) * 5 + c]; }, a.pp_mu);
#pragma unroll
      for (int c = 0; c < 5; ++c) sF[l][0][c] = H[c];  // point 0 is no longer read
    }
    __syncthreads();
  }
  if (t < kXBoundRows * 5) {
    const int l = t / 5, c = t % 5;
    const long long row = group * kXBoundRows + l;
    if (row < rows) {
      const R r = ((S & (kPP | kMusta)) != 0) ? sF[l][0][c] : sR[l][2 * c] + sR[l][2 * c + 1];
      R* d = a.D + c * nc + row * nx + nx - 1;
      *d = (*d - r) * a.inv_d;
    }
  }
  add_fixups(a.fixups, fix);
}

template <class R, int S>
__global__ void __launch_bounds__(kXBoundRows * 10) k_xbound(StageArgs<R> a) {
  xbound_body<R, S>(a, blockIdx.x);
}

// ---------------------------------------------------------------------------
// March along axis AX (1 = y, 2 = z).  blockDim = (64, BY): lanes along x,
// threadIdx.y over the other transverse axis; blockIdx.z = segment of `seg`
// cells along AX.  LAST: z-march, which finishes L and does the RK combine.
// The limiter on the march's window: the face between window points 3 and 4.
template <class R>
__device__ __forceinline__ void march_limit(R H[5], const R (&fp)[5][8], const R (&fm)[5][8], double mu) {
  pp_limit<R>(H, [&](int c, int k) { return (k & 1) ? fm[c][3 + (k >> 1)] : fp[c][3 + (k >> 1)]; }, mu);
}

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
    R Fp[5], Fm[5];
    point_values<R, S, AX>(u, Fp, Fm, fix);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      fp[c][m] = Fp[c];
      fm[c][m] = Fm[c];
    }
  }
  auto face = [&](R fh[5]) {
    if constexpr ((S & kMusta) != 0) {
      musta_face<R, (S & 7), AX>([&](int c, int m) { return fp[c][m]; }, a.eps, a.musta_k, fh, fix);
    } else {
#pragma unroll
      for (int c = 0; c < 5; ++c) fh[c] = face_flux<R, (S & 7)>(fp[c], fm[c], a.eps);
      if constexpr ((S & kPP) != 0) march_limit<R>(fh, fp, fm, a.pp_mu);
    }
  };
  R prev[5];
  face(prev);

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
      R Fp[5], Fm[5];
      point_values<R, S, AX>(u, Fp, Fm, fix);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        fp[c][7] = Fp[c];
        fm[c][7] = Fm[c];
      }
    }
    const long long cell = base + (long long)i * stride;
    R fh[5];
    face(fh);
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const R div = (prev[c] - fh[c]) * a.inv_d;
      prev[c] = fh[c];
      R* d = a.D + c * nc + cell;
      if (!LAST) {
        *d = *d + div;
      } else {
        const R p = rk_pre(a.stage, a.W[c * nc + cell], *d, a.dt);
        a.out[c * nc + cell] = rk_out(a.stage, p, div, a.dt, a.Un, c * nc + cell);
      }
    }
  }
  add_fixups(a.fixups, fix);
}

// ---------------------------------------------------------------------------
// y- or z-faces from an LDS tile (AX = 1 or 2).  A workgroup of 512 lanes
// owns 16 cells along x (coalesced 128-byte rows) by 31 cells along AX at one
// value of the remaining axis, so that its 32 face rows are exactly one face
// per lane (or, in pairs, one split of two faces per lane).  It stores the
// split AX-fluxes of its 16 x 39 points (4 ghost rows on each side) in LDS,
// reconstructs the face rows and forms the divergence; each lane's D is
// loaded before the reconstructions to hide its latency.
// LAST (z): adds D, does the RK combine (rk_pre, rk_out) and writes the
// stage output.
constexpr int kTileX = 16;
constexpr int kTileXP = kTileX;      // x pitch of the LDS arrays (128-byte rows)

// Tile length along the axis: 31 cells (32 face rows, one face per lane)
// or 32 cells (33 face rows, the last one by 16 lanes); the launchers pick
// the one that wastes less for the axis length (tile_len).
// The limiter on an LDS tile laid out [c][slot][pitch]: face row f lies
// between the points in slots f + 3 and f + 4, column col.
template <class R, int kP, int kPitch>
__device__ __forceinline__ void tile_limit(R H[5], const R* sFp, const R* sFm, int f, int col, double mu) {
  pp_limit<R>(
      H, [&](int c, int k) { return ((k & 1) ? sFm : sFp)[(c * kP + f + 3 + (k >> 1)) * kPitch + col]; }, mu);
}

template <class R, int S, int AX, bool LAST, int kTileA, bool PAIRS>
__device__ __forceinline__ void tile_body(const StageArgs<R>& a, int bx, int by, int bz, R* s) {
  constexpr int kTileP = kTileA + 8;  // points along AX
  // Plain WENO faces are taken in pairs (see below); then the F- points are
  // stored in reverse slot order, so that both splits read increasing slots.
  // FP64 32-cell y tiles keep one face per lane: their 33rd face row on top
  // of a pair takes them to 84 VGPRs, one workgroup per CU fewer (slower).
  constexpr bool kPair = PAIRS && (S & (kPP | kMusta)) == 0 && (sizeof(R) == 4 || kTileA == 31 || LAST);
  auto ms = [](int j) { return kPair ? kTileP - 1 - j : j; };
  R* sFp = s;                              // [5][kTileP][kTileXP]
  R* sFm = s + 5 * kTileP * kTileXP;       // [5][kTileP][kTileXP]
  const int nx = a.g.n[0], ny = a.g.n[1];
  const int n = a.g.n[AX];
  const int bc = a.g.bc[AX];
  const long long nc = a.g.nc;
  const int tx = threadIdx.x & (kTileX - 1);
  const int ta = threadIdx.x >> 4;  // 0..31: own cell a0 + ta (ta < kTileA), face row ta
  const int x = bx * kTileX + tx;
  const int a0 = by * kTileA;
  const int o = bz;
  const long long stride = (AX == 1) ? (long long)nx : (long long)nx * ny;
  const long long base = (AX == 1) ? (long long)o * nx * ny + x : (long long)o * nx + x;
  const bool xin = x < nx;
  unsigned fix = 0;

  const int ac = a0 + ta;
  const bool own_ok = xin && ta < kTileA && ac < n;
  const long long cell = base + (long long)ac * stride;
  // dpre: the own cell's D, loaded early so that its latency overlaps the
  // ghost rows and the reconstructions; LAST: loaded with the cell's W and
  // folded into the combine's p = w + dt D at once (rk_pre), so W need not
  // stay in registers
  R dpre[5];
  // pass 1: own cell (slot ta + 4)
  {
    const int p = a0 + ta;
    if (xin && ta < kTileA) {
      R own[5];
      load5(a.W, nc, base + (long long)map_idx(p, n, bc) * stride, own);
      if (LAST && own_ok) {
#pragma unroll
        for (int c = 0; c < 5; ++c) dpre[c] = a.D[c * nc + cell];
      }
      R Fp[5], Fm[5];
      point_values<R, S, AX>(own, Fp, Fm, fix);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        sFp[(c * kTileP + ta + 4) * kTileXP + tx] = Fp[c];
        sFm[(c * kTileP + ms(ta + 4)) * kTileXP + tx] = Fm[c];
      }
      if (LAST && own_ok) {
#pragma unroll
        for (int c = 0; c < 5; ++c) dpre[c] = rk_pre(a.stage, own[c], dpre[c], a.dt);
      }
    }
  }
  if (!LAST && own_ok) {
#pragma unroll
    for (int c = 0; c < 5; ++c) dpre[c] = a.D[c * nc + cell];
  }
  // pass 2: 4 ghost rows on each side (128 lanes)
  if (threadIdx.x < 8 * kTileX) {
    const int h = ta;  // 0..7
    const int j = (h < 4) ? h : h + kTileA;
    const int p = a0 - 4 + j;
    if (xin) {
      R u[5];
      load5(a.W, nc, base + (long long)map_idx(p, n, bc) * stride, u);
      R Fp[5], Fm[5];
      point_values<R, S, AX>(u, Fp, Fm, fix);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        sFp[(c * kTileP + j) * kTileXP + tx] = Fp[c];
        sFm[(c * kTileP + ms(j)) * kTileXP + tx] = Fm[c];
      }
    }
  }
  __syncthreads();

  // face rows f = 0..kTileA: face (a0 - 1 + f) + 1/2; F+ at slots f..f+6, F- at f+1..f+7
  const int nf = min(kTileA, n - a0) + 1;  // face rows this tile needs
  R Fh[5], Fh2[5];
  const bool has1 = xin && ta < nf;
  const bool has2 = (kTileA + 1) * kTileX > 512 && xin && threadIdx.x < kTileX && kTileA < nf;
  // Pairs: lane (q, h) = (ta >> 1, ta & 1) reconstructs split h (0: F+, 1: F-)
  // of the face rows 2q and 2q + 1 from the 8 points they span, read in
  // increasing slot order v0..v7: windows v0..v6 and v1..v7 share their
  // differences and third-difference terms.  F+: v_j = slot 2q + j, the
  // windows give rows 2q, 2q + 1; F- (mirrored stencils, reversed storage):
  // v_j = F- at slot 2q + 8 - j, the windows give rows 2q + 1, 2q.  One field
  // at a time: once every lane is past field c, its two split values per face
  // row go into field c's own F+ and F- areas (rows in natural order), so a
  // lane holds two results, not ten.
  const int pq = ta >> 1, ph = ta & 1;
  const bool hasp = kPair && xin && 2 * pq < nf;
  if constexpr (kPair) {
    const R* b = (ph ? sFm + (kTileP - 9 - 2 * pq) * kTileXP : sFp + 2 * pq * kTileXP) + tx;
    R* dst = (ph ? sFm : sFp) + tx;
    const int fa = 2 * pq + ph, fb = 2 * pq + 1 - ph;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      R lo, hi, f2p, f2m;
      if (hasp) {
        const R* v = b + c * kTileP * kTileXP;
        const R v0 = v[0], v1 = v[kTileXP], v2 = v[2 * kTileXP], v3 = v[3 * kTileXP], v4 = v[4 * kTileXP],
                v5 = v[5 * kTileXP], v6 = v[6 * kTileXP], v7 = v[7 * kTileXP];
        weno7_pair<R, (S & 7)>(v0, v1, v2, v3, v4, v5, v6, v7, a.eps, lo, hi);
      }
      if (has2) {  // row kTileA: F+ at slots kTileA..kTileA+6, F- at kTileA+7..kTileA+1 (reversed: 0..6)
        const R* fp = sFp + (c * kTileP + kTileA) * kTileXP + tx;
        const R* fm = sFm + c * kTileP * kTileXP + tx;
        f2p = weno7<R, (S & 7)>(fp[0], fp[kTileXP], fp[2 * kTileXP], fp[3 * kTileXP], fp[4 * kTileXP],
                                fp[5 * kTileXP], fp[6 * kTileXP], a.eps);
        f2m = weno7<R, (S & 7)>(fm[0], fm[kTileXP], fm[2 * kTileXP], fm[3 * kTileXP], fm[4 * kTileXP],
                                fm[5 * kTileXP], fm[6 * kTileXP], a.eps);
      }
      __syncthreads();
      if (hasp) {
        dst[(c * kTileP + fa) * kTileXP] = lo;
        dst[(c * kTileP + fb) * kTileXP] = hi;
      }
      if (has2) {
        sFp[(c * kTileP + kTileA) * kTileXP + tx] = f2p;
        sFm[(c * kTileP + kTileA) * kTileXP + tx] = f2m;
      }
    }
  } else if constexpr ((S & kMusta) != 0) {  // face row f: points in slots f..f+7
    auto at = [&](int f) {
      return [=](int c, int m) { return sFp[(c * kTileP + f + m) * kTileXP + tx]; };
    };
    if (has1) musta_face<R, (S & 7), AX>(at(ta), a.eps, a.musta_k, Fh, fix);
    if (has2) musta_face<R, (S & 7), AX>(at(kTileA), a.eps, a.musta_k, Fh2, fix);
  } else if (has1) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const R* fp = sFp + (c * kTileP + ta) * kTileXP + tx;
      const R* fm = sFm + (c * kTileP + ta) * kTileXP + tx;
      Fh[c] = weno7<R, (S & 7)>(fp[0], fp[kTileXP], fp[2 * kTileXP], fp[3 * kTileXP], fp[4 * kTileXP], fp[5 * kTileXP],
                          fp[6 * kTileXP], a.eps) +
              weno7<R, (S & 7)>(fm[7 * kTileXP], fm[6 * kTileXP], fm[5 * kTileXP], fm[4 * kTileXP], fm[3 * kTileXP],
                          fm[2 * kTileXP], fm[kTileXP], a.eps);
    }
  }
  if ((S & kMusta) == 0 && !kPair && has2) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const R* fp = sFp + (c * kTileP + kTileA) * kTileXP + tx;
      const R* fm = sFm + (c * kTileP + kTileA) * kTileXP + tx;
      Fh2[c] = weno7<R, (S & 7)>(fp[0], fp[kTileXP], fp[2 * kTileXP], fp[3 * kTileXP], fp[4 * kTileXP], fp[5 * kTileXP],
                           fp[6 * kTileXP], a.eps) +
               weno7<R, (S & 7)>(fm[7 * kTileXP], fm[6 * kTileXP], fm[5 * kTileXP], fm[4 * kTileXP], fm[3 * kTileXP],
                           fm[2 * kTileXP], fm[kTileXP], a.eps);
    }
  }
  if constexpr ((S & kPP) != 0) {  // face row f: cells at slots f + 3 and f + 4
    if (has1) tile_limit<R, kTileP, kTileXP>(Fh, sFp, sFm, ta, tx, a.pp_mu);
    if (has2) tile_limit<R, kTileP, kTileXP>(Fh2, sFp, sFm, kTileA, tx, a.pp_mu);
  }
  __syncthreads();
  // face values: pairs keep the two splits apart in the F+ and F- areas
  // ([5][kTileP][kTileXP], rows 0..kTileA) and form the face flux F+ + F-
  // where it is used; otherwise sF [5][kTileA + 1][kTileXP] holds it
  constexpr int kFP = kPair ? kTileP : kTileA + 1;
  R* sF = s;
  R* sG = sFm;
  if (!kPair) {
    if (has1) {
#pragma unroll
      for (int c = 0; c < 5; ++c) sF[(c * kFP + ta) * kTileXP + tx] = Fh[c];
    }
    if (has2) {
#pragma unroll
      for (int c = 0; c < 5; ++c) sF[(c * kFP + kTileA) * kTileXP + tx] = Fh2[c];
    }
    __syncthreads();
  }

  if (own_ok) {
    // LAST, stages 2 and 3: the five U^n values are read before any output
    // is stored (out may be U^n itself, so the compiler would otherwise keep
    // each read behind the previous field's store: five round trips)
    R unv[5];
    if (LAST && a.stage >= 2) {
#pragma unroll
      for (int c = 0; c < 5; ++c) unv[c] = a.Un[c * nc + cell];
    }
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const int i0 = (c * kFP + ta) * kTileXP + tx, i1 = i0 + kTileXP;
      const R fl = kPair ? sF[i0] + sG[i0] : sF[i0];
      const R fr = kPair ? sF[i1] + sG[i1] : sF[i1];
      const R div = (fl - fr) * a.inv_d;
      if (!LAST) {
        a.D[c * nc + cell] = dpre[c] + div;
      } else {
        a.out[c * nc + cell] = rk_out_v(a.stage, dpre[c], div, a.dt, unv[c]);
      }
    }
  }
  add_fixups(a.fixups, fix);
}


template <class R, int S, int AX, bool LAST, int A>
__global__ void __launch_bounds__(512) k_tile(StageArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  const int by = a.order ? blockIdx.z : blockIdx.y;  // tile along AX
  const int bz = a.order ? blockIdx.y : blockIdx.z;  // transverse index
  tile_body<R, S, AX, LAST, A, true>(a, blockIdx.x, by, bz, reinterpret_cast<R*>(smem_raw));
}

// ---------------------------------------------------------------------------
// x-faces from an LDS tile: a workgroup of 512 lanes owns 31 or 32 cells
// along x (tile_len) by 16 rows along y at one z.  The (A + 8) x 16 points
// (4 ghosts on each side) are loaded x-fastest (coalesced) and their split
// x-fluxes stored [c][x][y], so a face lane (y fastest) reads them without
// bank conflicts; the A + 1 face rows are reconstructed (one face per lane;
// for A = 32 one extra row by 16 lanes) and the divergence is formed with
// lanes x-fastest again and assigned to D (x is the first axis).  Same
// per-face arithmetic as k_xface + k_xbound.
constexpr int kXTileY = 16;
constexpr int kXFacePitch = kXTileY + 1;

template <class R, int S, int kXTileX>
__device__ __forceinline__ void xtile_body(const StageArgs<R>& a, int bx, int by, int bz, R* s) {
  constexpr int kXTileP = kXTileX + 8;
  R* sFp = s;                                // [5][kXTileP][kXTileY]
  R* sFm = s + 5 * kXTileP * kXTileY;        // [5][kXTileP][kXTileY]
  const int nx = a.g.n[0], ny = a.g.n[1];
  const int bc = a.g.bc[0];
  const long long nc = a.g.nc;
  const int x0 = bx * kXTileX, y0 = by * kXTileY;
  const long long zbase = (long long)bz * nx * ny;
  unsigned fix = 0;
  for (int t = threadIdx.x; t < kXTileP * kXTileY; t += 512) {
    const int j = t % kXTileP, r = t / kXTileP;
    const int y = y0 + r;
    if (y < ny) {
      R u[5];
      load5(a.W, nc, zbase + (long long)y * nx + map_idx(x0 - 4 + j, nx, bc), u);
      R Fp[5], Fm[5];
      point_values<R, S, 0>(u, Fp, Fm, fix);
#pragma unroll
      for (int c = 0; c < 5; ++c) {
        sFp[(c * kXTileP + j) * kXTileY + r] = Fp[c];
        sFm[(c * kXTileP + j) * kXTileY + r] = Fm[c];
      }
    }
  }
  __syncthreads();

  // faces f = 0..32: face (x0 - 1 + f) + 1/2; F+ at slots f..f+6, F- at f+1..f+7
  const int r = threadIdx.x & (kXTileY - 1);
  const int f = threadIdx.x >> 4;  // 0..31: face row f
  const int nf = min(kXTileX, nx - x0) + 1;
  const bool yin = y0 + r < ny;
  const bool has1 = yin && f < nf;
  const bool has2 = (kXTileX + 1) * kXTileY > 512 && yin && threadIdx.x < kXTileY && kXTileX < nf;
  R Fh[5], Fh2[5];
  if constexpr ((S & kMusta) != 0) {  // face row f: points in slots f..f+7
    auto at = [&](int fr) {
      return [=](int c, int m) { return sFp[(c * kXTileP + fr + m) * kXTileY + r]; };
    };
    if (has1) musta_face<R, (S & 7), 0>(at(f), a.eps, a.musta_k, Fh, fix);
    if (has2) musta_face<R, (S & 7), 0>(at(kXTileX), a.eps, a.musta_k, Fh2, fix);
  } else if (has1) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const R* fp = sFp + (c * kXTileP + f) * kXTileY + r;
      const R* fm = sFm + (c * kXTileP + f) * kXTileY + r;
      Fh[c] = weno7<R, (S & 7)>(fp[0], fp[kXTileY], fp[2 * kXTileY], fp[3 * kXTileY], fp[4 * kXTileY], fp[5 * kXTileY],
                          fp[6 * kXTileY], a.eps) +
              weno7<R, (S & 7)>(fm[7 * kXTileY], fm[6 * kXTileY], fm[5 * kXTileY], fm[4 * kXTileY], fm[3 * kXTileY],
                          fm[2 * kXTileY], fm[kXTileY], a.eps);
    }
  }
  if ((S & kMusta) == 0 && has2) {
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const R* fp = sFp + (c * kXTileP + kXTileX) * kXTileY + r;
      const R* fm = sFm + (c * kXTileP + kXTileX) * kXTileY + r;
      Fh2[c] = weno7<R, (S & 7)>(fp[0], fp[kXTileY], fp[2 * kXTileY], fp[3 * kXTileY], fp[4 * kXTileY], fp[5 * kXTileY],
                           fp[6 * kXTileY], a.eps) +
               weno7<R, (S & 7)>(fm[7 * kXTileY], fm[6 * kXTileY], fm[5 * kXTileY], fm[4 * kXTileY], fm[3 * kXTileY],
                           fm[2 * kXTileY], fm[kXTileY], a.eps);
    }
  }
  if constexpr ((S & kPP) != 0) {  // face row f: cells at slots f + 3 and f + 4
    if (has1) tile_limit<R, kXTileP, kXTileY>(Fh, sFp, sFm, f, r, a.pp_mu);
    if (has2) tile_limit<R, kXTileP, kXTileY>(Fh2, sFp, sFm, kXTileX, r, a.pp_mu);
  }
  __syncthreads();
  R* sF = s;  // [5][kXTileX + 1][kXFacePitch]
  if (has1) {
#pragma unroll
    for (int c = 0; c < 5; ++c) sF[(c * (kXTileX + 1) + f) * kXFacePitch + r] = Fh[c];
  }
  if (has2) {
#pragma unroll
    for (int c = 0; c < 5; ++c) sF[(c * (kXTileX + 1) + kXTileX) * kXFacePitch + r] = Fh2[c];
  }
  __syncthreads();

  const int xa = threadIdx.x & 31, ra = threadIdx.x >> 5;
  if (xa < kXTileX && x0 + xa < nx && y0 + ra < ny) {
    const long long cell = zbase + (long long)(y0 + ra) * nx + x0 + xa;
#pragma unroll
    for (int c = 0; c < 5; ++c) {
      const R l = sF[(c * (kXTileX + 1) + xa) * kXFacePitch + ra];
      const R rr = sF[(c * (kXTileX + 1) + xa + 1) * kXFacePitch + ra];
      a.D[c * nc + cell] = (l - rr) * a.inv_d;
    }
  }
  add_fixups(a.fixups, fix);
}

template <class R, int S, int A>
__global__ void __launch_bounds__(512) k_xtile(StageArgs<R> a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  xtile_body<R, S, A>(a, blockIdx.x, blockIdx.y, blockIdx.z, reinterpret_cast<R*>(smem_raw));
}

// ---------------------------------------------------------------------------
// Jet source (Eq. 2 and 3).  One workgroup of 512 threads; jets in order.
template <class R>
__device__ __forceinline__ void jet_body(const JetArgs& a) {
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
          R u[5], dv[4];  // the cell's state and its D, read together
          load5(W, nc, cell, u);
          for (int d = 0; d < 4; ++d) dv[d] = D[d * nc + cell];
          const PrimV pv = c2p(u, fix);
          const double T = temperature(pv.e, a.eos_dof, a.hbarc);
          P = energy_loss(jt, T, ell, a.hbarc);
          const double s0 = P / dV;
          D[cell] = dv[0] + (R)s0;
          for (int d = 0; d < 3; ++d) D[(1 + d) * nc + cell] = dv[1 + d] + (R)(jt.dir[d] * s0);
        }
      } else {
        // 7^3 footprint, thread t < 343 owns cell (mi, mj, mk)
        const int t = threadIdx.x;
        double w = 0.0, wT = 0.0;
        long long cell = -1;
        R dv[4];  // the cell's D, read with its state
        if (t < 343) {
          const int mi = t % 7, mj = (t / 7) % 7, mk = t / 49;
          const int i = ctr_s[0] - 3 + mi, jj = ctr_s[1] - 3 + mj, k = ctr_s[2] - 3 + mk;
          if (i >= 0 && i < a.g.n[0] && jj >= 0 && jj < a.g.n[1] && k >= 0 && k < a.g.n[2]) {
            cell = ((long long)k * a.g.n[1] + jj) * a.g.n[0] + i;
            w = wax[0][mi] * wax[1][mj] * wax[2][mk];
            R u[5];
            load5(W, nc, cell, u);
            for (int d = 0; d < 4; ++d) dv[d] = D[d * nc + cell];
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
          D[cell] = dv[0] + (R)s0;
          for (int d = 0; d < 3; ++d) D[(1 + d) * nc + cell] = dv[1 + d] + (R)(jt.dir[d] * s0);
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

template <class R>
__global__ void __launch_bounds__(512) k_jet(JetArgs a) {
  jet_body<R>(a);
}

// ---------------------------------------------------------------------------
// FP64 sums of the five fields, fixed order: per-block partials, then one block.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

template <class R>
__device__ __forceinline__ void sums_partial_body(const R* __restrict__ U, long long nc, double* part, int b, int nb) {
  double acc[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (long long i = (long long)b * blockDim.x + threadIdx.x; i < nc; i += (long long)nb * blockDim.x) {
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
    part[(long long)b * 5 + c] = (red[c][0] + red[c][1]) + (red[c][2] + red[c][3]);
  }
}

template <class R>
__global__ void __launch_bounds__(256) k_sums_partial(const R* __restrict__ U, long long nc, double* part) {
  sums_partial_body<R>(U, nc, part, blockIdx.x, gridDim.x);
}

__device__ __forceinline__ void sums_final_body(const double* part, int nblocks, double dV, double* sums) {
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
    sums[c] = ((red[c][0] + red[c][1]) + (red[c][2] + red[c][3])) * dV;
  }
}

__global__ void __launch_bounds__(256) k_sums_final(const double* part, int nblocks, double dV, double* sums) {
  sums_final_body(part, nblocks, dV, sums);
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
// Batched stage kernels.  Each workgroup walks the work items blockIdx.x,
// blockIdx.x + gridDim.x, ... (persistent when the grid is smaller than the
// item count); an item is one tile of one event and runs the same body as the
// single-event kernel, so every face has the same arithmetic.
__device__ __forceinline__ int batch_event_of(const long long* off, int n, long long item) {
  int lo = 0, hi = n;  // off[lo] <= item < off[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= item) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <class R>
__device__ __forceinline__ StageArgs<R> batch_stage_args(const BatchEvent& ev, int stage, R eps, int AX) {
  StageArgs<R> a;
  R* U = static_cast<R*>(ev.U);
  R* U1 = static_cast<R*>(ev.U1);
  R* U2 = static_cast<R*>(ev.U2);
  a.W = (stage <= 1) ? U : (stage == 2 ? U1 : U2);
  a.Un = U;
  a.out = (stage <= 1) ? U1 : (stage == 2 ? U2 : U);
  a.D = static_cast<R*>(ev.D);
  a.g = ev.g;
  a.order = 0;
  a.inv_d = (R)ev.inv_d[AX];
  a.dt = (R)ev.dt;
  a.eps = eps;
  a.stage = stage;
  a.seg = 0;
  a.fixups = &ev.dev->fixups;
  a.pp_mu = ev.pp_mu;
  a.musta_k = ev.musta_k;
  return a;
}

__device__ __forceinline__ double batch_stage_time(const BatchEvent& ev, long long step, int stage) {
  const double tn = ev.t0 + (double)step * ev.dt;
  const double c = stage == 2 ? 1.0 : (stage == 3 ? 0.5 : 0.0);
  return tn + c * ev.dt;
}

// x, y or z tiles of every event (xtile_body, tile_body).
template <class R, int S, int AX>
__global__ void __launch_bounds__(512) k_btile(BatchArgs<R> b) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* s = reinterpret_cast<R*>(smem_raw);
  for (long long it = blockIdx.x; it < b.items; it += gridDim.x) {
    const int e = batch_event_of(b.off, b.n_events, it);
    const BatchEvent& ev = b.ev[e];
    const long long local = it - b.off[e];
    const StageArgs<R> a = batch_stage_args<R>(ev, b.stage, b.eps, AX);
    const int A = tile_len(ev.g.n[AX]);
    if (AX == 0) {
      const int gx = (ev.g.n[0] + A - 1) / A, gy = (ev.g.n[1] + kXTileY - 1) / kXTileY;
      const int bx = (int)(local % gx), by = (int)((local / gx) % gy), bz = (int)(local / ((long long)gx * gy));
      if (A == 31) xtile_body<R, S, 31>(a, bx, by, bz, s);
      else xtile_body<R, S, 32>(a, bx, by, bz, s);
    } else {
      const int gx = (ev.g.n[0] + kTileX - 1) / kTileX, ga = (ev.g.n[AX] + A - 1) / A;
      const int bx = (int)(local % gx), by = (int)((local / gx) % ga), bz = (int)(local / ((long long)gx * ga));
      if (A == 31) tile_body<R, S, AX, AX == 2, 31, false>(a, bx, by, bz, s);
      else tile_body<R, S, AX, AX == 2, 32, false>(a, bx, by, bz, s);
    }
    __syncthreads();  // the next item overwrites the LDS tile
  }
}

// The same when every event has the tile length A along the axis (the
// launcher checks): one tile body instead of two, so the y/z faces are taken
// in pairs as in the single-event kernels (same bits either way).  PERSIST:
// workgroups walk items blockIdx.x, blockIdx.x + gridDim.x, ...; otherwise
// one item per workgroup (the loop's live state costs ~20 VGPRs, a
// workgroup per CU).
template <class R, int S, int AX, int A>
__device__ __forceinline__ void btile_item(const BatchArgs<R>& b, long long it, R* s) {
  const int e = batch_event_of(b.off, b.n_events, it);
  const BatchEvent& ev = b.ev[e];
  const long long local = it - b.off[e];
  const StageArgs<R> a = batch_stage_args<R>(ev, b.stage, b.eps, AX);
  if (AX == 0) {
    const int gx = (ev.g.n[0] + A - 1) / A, gy = (ev.g.n[1] + kXTileY - 1) / kXTileY;
    const int bx = (int)(local % gx), by = (int)((local / gx) % gy), bz = (int)(local / ((long long)gx * gy));
    xtile_body<R, S, A>(a, bx, by, bz, s);
  } else {
    const int gx = (ev.g.n[0] + kTileX - 1) / kTileX, ga = (ev.g.n[AX] + A - 1) / A;
    const int bx = (int)(local % gx), by = (int)((local / gx) % ga), bz = (int)(local / ((long long)gx * ga));
    tile_body<R, S, AX, AX == 2, A, true>(a, bx, by, bz, s);
  }
}

template <class R, int S, int AX, int A, bool PERSIST>
__global__ void __launch_bounds__(512) k_btile_u(BatchArgs<R> b) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* s = reinterpret_cast<R*>(smem_raw);
  if constexpr (PERSIST) {
    for (long long it = blockIdx.x; it < b.items; it += gridDim.x) {
      btile_item<R, S, AX, A>(b, it, s);
      __syncthreads();  // the next item overwrites the LDS tile
    }
  } else {
    if ((long long)blockIdx.x < b.items) btile_item<R, S, AX, A>(b, blockIdx.x, s);  // uniform
  }
}

// x rows of every event: items are groups of TB / nx rows (xrows_body).
template <class R, int S, int TB>
__global__ void __launch_bounds__(TB) k_bxrows(BatchArgs<R> b) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* s = reinterpret_cast<R*>(smem_raw);
  for (long long it = blockIdx.x; it < b.items; it += gridDim.x) {
    const int e = batch_event_of(b.off, b.n_events, it);
    const BatchEvent& ev = b.ev[e];
    const int rpi = xrow_rows(ev.g.n[0], TB, (int)sizeof(R));
    const StageArgs<R> a = batch_stage_args<R>(ev, b.stage, b.eps, 0);
    xrows_body<R, S, sizeof(R) == 4>(a, (it - b.off[e]) * rpi, rpi, s);  // FP64 pairs cost 18 VGPRs here
    __syncthreads();  // the next item overwrites the LDS rows
  }
}

// Outflow right x-face of every event with outflow x: items are groups of
// kXBoundRows rows (xbound_body).
template <class R, int S>
__global__ void __launch_bounds__(kXBoundRows * 10) k_bxbound(BatchArgs<R> b) {
  for (long long it = blockIdx.x; it < b.items; it += gridDim.x) {
    const int e = batch_event_of(b.off, b.n_events, it);
    const BatchEvent& ev = b.ev[e];
    const StageArgs<R> a = batch_stage_args<R>(ev, b.stage, b.eps, 0);
    xbound_body<R, S>(a, it - b.off[e]);
    __syncthreads();
  }
}

// Jets of every event: one workgroup per event.
template <class R>
__global__ void __launch_bounds__(512) k_bjet(BatchArgs<R> b) {
  const BatchEvent& ev = b.ev[blockIdx.x];
  if (ev.njet == 0) return;  // whole workgroup
  const int stage = b.stage;
  JetArgs j;
  j.W = (stage <= 1) ? ev.U : (stage == 2 ? ev.U1 : ev.U2);
  j.D = ev.D;
  j.s = ev.dev;
  j.g = ev.g;
  j.njet = ev.njet;
  j.stage = stage;
  j.deposit = ev.deposit;
  j.t = batch_stage_time(ev, *b.step, stage);
  j.dt = ev.dt;
  j.eos_dof = ev.eos_dof;
  j.hbarc = ev.hbarc;
  jet_body<R>(j);
}

// FP64 conservation sums of every event (grid kSumBlocks x n_events, then n_events).
template <class R>
__global__ void __launch_bounds__(256) k_bsums_partial(BatchArgs<R> b) {
  const BatchEvent& ev = b.ev[blockIdx.y];
  sums_partial_body<R>(static_cast<const R*>(ev.U), ev.g.nc, ev.part, blockIdx.x, gridDim.x);
}

template <class R>
__global__ void __launch_bounds__(256) k_bsums_final(BatchArgs<R> b) {
  const BatchEvent& ev = b.ev[blockIdx.x];
  sums_final_body(ev.part, kSumBlocks, ev.dV, ev.dev->sums);
}

__global__ void k_bstep(long long* step) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *step = *step + 1;
}

// ---------------------------------------------------------------------------
// Host-side launchers (called from hydro_api.hip).
template <class R, int S>
void launch_xface_t(const StageArgs<R>& base, hipStream_t st) {
  StageArgs<R> a = base;
  const int nx = a.g.n[0];
  a.inv_d = R(1.0 / a.g.dx[0]);
  const int n1 = nx;
  const int TB = xrow_block(&n1, 1, (int)sizeof(R));
  const int rpi = xrow_rows(nx, TB, (int)sizeof(R));
  const size_t lds = xrow_lds_bytes(nx, rpi, (int)sizeof(R));
  const long long rows = (long long)a.g.n[1] * a.g.n[2];
  const unsigned nb = (unsigned)((rows + rpi - 1) / rpi);
  switch (TB) {
    case 256: hipLaunchKernelGGL((k_xface<R, S, 256>), dim3(nb), dim3(256), lds, st, a, rpi); break;
    case 384: hipLaunchKernelGGL((k_xface<R, S, 384>), dim3(nb), dim3(384), lds, st, a, rpi); break;
    case 512: hipLaunchKernelGGL((k_xface<R, S, 512>), dim3(nb), dim3(512), lds, st, a, rpi); break;
    default: hipLaunchKernelGGL((k_xface<R, S, 1024>), dim3(nb), dim3(1024), lds, st, a, rpi); break;
  }
}

template <class R, int S>
void launch_xbound_t(const StageArgs<R>& base, hipStream_t st) {
  StageArgs<R> a = base;
  a.inv_d = R(1.0 / a.g.dx[0]);
  const long long rows = (long long)a.g.n[1] * a.g.n[2];
  const unsigned nb = (unsigned)((rows + kXBoundRows - 1) / kXBoundRows);
  hipLaunchKernelGGL((k_xbound<R, S>), dim3(nb), dim3(kXBoundRows * 10), 0, st, a);
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
  const int A = tile_len(n);
  const size_t lds = (size_t)2 * 5 * (A + 8) * kTileXP * sizeof(R);
  a.order = (base.order >> (AX - 1)) & 1;
  dim3 grid((nx + kTileX - 1) / kTileX, (n + A - 1) / A, no);
  if (a.order) grid = dim3(grid.x, no, grid.y);
  if (A == 31) hipLaunchKernelGGL((k_tile<R, S, AX, AX == 2, 31>), grid, dim3(512), lds, st, a);
  else hipLaunchKernelGGL((k_tile<R, S, AX, AX == 2, 32>), grid, dim3(512), lds, st, a);
}

template <class R, int S>
void launch_xtile_t(const StageArgs<R>& base, hipStream_t st) {
  StageArgs<R> a = base;
  a.inv_d = R(1.0 / a.g.dx[0]);
  const int A = tile_len(a.g.n[0]);
  const size_t lds = (size_t)2 * 5 * (A + 8) * kXTileY * sizeof(R);
  dim3 grid((a.g.n[0] + A - 1) / A, (a.g.n[1] + kXTileY - 1) / kXTileY, a.g.n[2]);
  if (A == 31) hipLaunchKernelGGL((k_xtile<R, S, 31>), grid, dim3(512), lds, st, a);
  else hipLaunchKernelGGL((k_xtile<R, S, 32>), grid, dim3(512), lds, st, a);
}

// kernel: 0 x-faces, 1 x boundary faces, 2 y-march, 3 z-march (+ combine),
// 4 y-tile, 5 z-tile (+ combine), 6 x-tile (all x faces, boundary included)
template <class R>
hipError_t launch_face_kernel(int kernel, const StageArgs<R>& a, int scheme, int seg, hipStream_t st) {
#define HYDRO_DISPATCH(S)                                  \
  switch (kernel) {                                        \
    case 0: launch_xface_t<R, S>(a, st); break;            \
    case 1: launch_xbound_t<R, S>(a, st); break;           \
    case 2: launch_march_t<R, S, 1>(a, seg, st); break;    \
    case 3: launch_march_t<R, S, 2>(a, seg, st); break;    \
    case 4: launch_tile_t<R, S, 1>(a, st); break;          \
    case 5: launch_tile_t<R, S, 2>(a, st); break;          \
    default: launch_xtile_t<R, S>(a, st); break;           \
  }
  switch (scheme) {
    case kWenoJS: HYDRO_DISPATCH(kWenoJS) break;
    case kWenoLinear: HYDRO_DISPATCH(kWenoLinear) break;
    case kWeno5Z: HYDRO_DISPATCH(kWeno5Z) break;
    case kWeno5JS: HYDRO_DISPATCH(kWeno5JS) break;
    case kWeno5Linear: HYDRO_DISPATCH(kWeno5Linear) break;
    case kWenoZ | kPP: HYDRO_DISPATCH(kWenoZ | kPP) break;
    case kWenoJS | kPP: HYDRO_DISPATCH(kWenoJS | kPP) break;
    case kWenoLinear | kPP: HYDRO_DISPATCH(kWenoLinear | kPP) break;
    case kWeno5Z | kPP: HYDRO_DISPATCH(kWeno5Z | kPP) break;
    case kWeno5JS | kPP: HYDRO_DISPATCH(kWeno5JS | kPP) break;
    case kWeno5Linear | kPP: HYDRO_DISPATCH(kWeno5Linear | kPP) break;
    case kWenoZ | kMusta: HYDRO_DISPATCH(kWenoZ | kMusta) break;
    case kWeno5Z | kMusta: HYDRO_DISPATCH(kWeno5Z | kMusta) break;
    default: HYDRO_DISPATCH(kWenoZ) break;
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
hipError_t launch_sums(const R* U, long long nc, double dV, double* part, double* sums, hipStream_t st) {
  hipLaunchKernelGGL((k_sums_partial<R>), dim3(kSumBlocks), dim3(256), 0, st, U, nc, part);
  hipLaunchKernelGGL(k_sums_final, dim3(1), dim3(256), 0, st, part, kSumBlocks, dV, sums);
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

// Work items of one event for the batched launches: 0 x tiles, 1 and 2 y/z
// tiles, 3 x-row groups of xrow_rows(nx, xtb) rows, 4 groups of kXBoundRows
// rows for the outflow x face (none for periodic x).  An x pass is either 0
// or 3 + 4.
long long batch_items(int AX, const Grid& g, int xtb, int elem) {
  const long long rows = (long long)g.n[1] * g.n[2];
  if (AX == 3) {
    const int rpi = xrow_rows(g.n[0], xtb, elem);
    return (rows + rpi - 1) / rpi;
  }
  if (AX == 4) return g.bc[0] ? 0 : (rows + kXBoundRows - 1) / kXBoundRows;
  const int A = tile_len(g.n[AX]);
  if (AX == 0) return (long long)((g.n[0] + A - 1) / A) * ((g.n[1] + kXTileY - 1) / kXTileY) * g.n[2];
  const int no = AX == 1 ? g.n[2] : g.n[1];
  return (long long)((g.n[0] + kTileX - 1) / kTileX) * ((g.n[AX] + A - 1) / A) * no;
}

// blocks: workgroups of the launch (0: one per item).
template <class R, int S>
void launch_btile_u(int AX, int A, bool persist, dim3 grid, const BatchArgs<R>& b, hipStream_t st) {
  const size_t lds = (size_t)2 * 5 * (A + 8) * 16 * sizeof(R);
  const dim3 tb(512);
#define HYDRO_BTU(AXV, AV)                                                                 \
  if (AX == AXV && A == AV) {                                                              \
    if (persist) hipLaunchKernelGGL((k_btile_u<R, S, AXV, AV, true>), grid, tb, lds, st, b);  \
    else hipLaunchKernelGGL((k_btile_u<R, S, AXV, AV, false>), grid, tb, lds, st, b);          \
  }
  HYDRO_BTU(0, 31) HYDRO_BTU(1, 31) HYDRO_BTU(2, 31) HYDRO_BTU(0, 32) HYDRO_BTU(1, 32) HYDRO_BTU(2, 32)
#undef HYDRO_BTU
}

template <class R>
hipError_t launch_batch_axis(int AX, const BatchArgs<R>& b, int scheme, long long blocks, hipStream_t st) {
  const long long nb = (blocks <= 0 || blocks > b.items) ? b.items : blocks;
  if (nb <= 0) return hipSuccess;
  const size_t lds = (size_t)2 * 5 * (32 + 8) * 16 * sizeof(R);  // the largest y/z tile (A = 32)
  const dim3 grid((unsigned)nb), tb(512);
  const size_t xl = (size_t)b.xlds;
  // the uniform-tile-length kernels for plain WENO faces and WENO7-Z with the
  // limiter (the other limited schemes and MUSTA-FORCE keep the general one)
  const bool uni = (scheme & (kPP | kMusta)) == 0 || scheme == (kWenoZ | kPP);
#define HYDRO_BAXIS(S)                                                                                      \
  if (AX == 3) {                                                                                            \
    switch (b.xtb) {                                                                                        \
      case 256: hipLaunchKernelGGL((k_bxrows<R, S, 256>), grid, dim3(256), xl, st, b); break;                 \
      case 384: hipLaunchKernelGGL((k_bxrows<R, S, 384>), grid, dim3(384), xl, st, b); break;                 \
      case 512: hipLaunchKernelGGL((k_bxrows<R, S, 512>), grid, dim3(512), xl, st, b); break;                 \
      default: hipLaunchKernelGGL((k_bxrows<R, S, 1024>), grid, dim3(1024), xl, st, b); break;                \
    }                                                                                                       \
  } else if (AX == 4) {                                                                                     \
    hipLaunchKernelGGL((k_bxbound<R, S>), grid, dim3(kXBoundRows * 10), 0, st, b);                          \
  } else if (uni && (b.tile_a == 31 || b.tile_a == 32)) {                                                  \
    if ((S & kPP) != 0) launch_btile_u<R, (kWenoZ | kPP)>(AX, b.tile_a, nb < b.items, grid, b, st);         \
    else launch_btile_u<R, (S & 7)>(AX, b.tile_a, nb < b.items, grid, b, st);                                \
  } else if (AX == 0) {                                                                                     \
    hipLaunchKernelGGL((k_btile<R, S, 0>), grid, tb, lds, st, b);                                          \
  } else if (AX == 1) {                                                                                     \
    hipLaunchKernelGGL((k_btile<R, S, 1>), grid, tb, lds, st, b);                                          \
  } else {                                                                                                  \
    hipLaunchKernelGGL((k_btile<R, S, 2>), grid, tb, lds, st, b);                                          \
  }
  switch (scheme) {
    case kWenoJS: HYDRO_BAXIS(kWenoJS) break;
    case kWenoLinear: HYDRO_BAXIS(kWenoLinear) break;
    case kWeno5Z: HYDRO_BAXIS(kWeno5Z) break;
    case kWeno5JS: HYDRO_BAXIS(kWeno5JS) break;
    case kWeno5Linear: HYDRO_BAXIS(kWeno5Linear) break;
    case kWenoZ | kPP: HYDRO_BAXIS(kWenoZ | kPP) break;
    case kWenoJS | kPP: HYDRO_BAXIS(kWenoJS | kPP) break;
    case kWenoLinear | kPP: HYDRO_BAXIS(kWenoLinear | kPP) break;
    case kWeno5Z | kPP: HYDRO_BAXIS(kWeno5Z | kPP) break;
    case kWeno5JS | kPP: HYDRO_BAXIS(kWeno5JS | kPP) break;
    case kWeno5Linear | kPP: HYDRO_BAXIS(kWeno5Linear | kPP) break;
    case kWenoZ | kMusta: HYDRO_BAXIS(kWenoZ | kMusta) break;
    case kWeno5Z | kMusta: HYDRO_BAXIS(kWeno5Z | kMusta) break;
    default: HYDRO_BAXIS(kWenoZ) break;
  }
#undef HYDRO_BAXIS
  return hipGetLastError();
}

template <class R>
hipError_t launch_batch_jet(const BatchArgs<R>& b, hipStream_t st) {
  hipLaunchKernelGGL((k_bjet<R>), dim3(b.n_events), dim3(512), 0, st, b);
  return hipGetLastError();
}

template <class R>
hipError_t launch_batch_sums(const BatchArgs<R>& b, long long* step, hipStream_t st) {
  hipLaunchKernelGGL((k_bsums_partial<R>), dim3(kSumBlocks, b.n_events), dim3(256), 0, st, b);
  hipLaunchKernelGGL((k_bsums_final<R>), dim3(b.n_events), dim3(256), 0, st, b);
  if (step) hipLaunchKernelGGL(k_bstep, dim3(1), dim3(64), 0, st, step);
  return hipGetLastError();
}

#define HYDRO_INSTANTIATE(R)                                                                          \
  template hipError_t launch_batch_axis<R>(int, const BatchArgs<R>&, int, long long, hipStream_t);      \
  template hipError_t launch_batch_jet<R>(const BatchArgs<R>&, hipStream_t);                          \
  template hipError_t launch_batch_sums<R>(const BatchArgs<R>&, long long*, hipStream_t);              \
  template hipError_t launch_face_kernel<R>(int, const StageArgs<R>&, int, int, hipStream_t);          \
  template hipError_t launch_jet<R>(const JetArgs&, hipStream_t);                                     \
  template hipError_t launch_sums<R>(const R*, long long, double, double*, double*, hipStream_t);     \
  template hipError_t launch_prim_to_cons<R>(const double*, R*, long long, hipStream_t);              \
  template hipError_t launch_primitives<R>(const R*, R*, long long, double, double, unsigned long long*, hipStream_t);

HYDRO_INSTANTIATE(double)
HYDRO_INSTANTIATE(float)

}  // namespace hydro
