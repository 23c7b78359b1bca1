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

#include "hydro_device.hpp"
#include "hydro_internal.hpp"

namespace hydro {

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
