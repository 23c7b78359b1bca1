// hydro_freezeout.hip -- freeze-out of an evolved state into particles and
// their azimuthal distribution: the step the paper plans after its jet runs
// (section "Results", closing paragraph: freeze-out, elliptic flow and higher
// flow harmonics).
//
// Cooper-Frye on the fixed-time hypersurface of U (d sigma_mu = (dV, 0, 0,
// 0)) for a massless Boltzmann species of degeneracy g at zero chemical
// potential, the quanta of the p = e/3 fluid, T = T(e) of its equation of
// state.  At rapidity 0 along z a particle of transverse momentum p_T and
// azimuth phi has p.u = gamma p_T D, D = 1 - vx cos phi - vy sin phi, so
//   dN/(p_T dp_T dy dphi) = g/(2 pi hbar c)^3 sum_cells dV p_T exp(-gamma p_T D/T),
//   dN/(dy dphi)          = g/(2 pi hbar c)^3 sum_cells dV 2 T^3/(gamma D)^3
// (the p_T integral of the first, int p^2 exp(-a p) dp = 2/a^3).
//
// Work: every cell contributes to every output (row, phi_k), a few flops
// each, so the pass is arithmetic, not traffic: each workgroup recovers the
// primitives of 256 cells at a time (FP64, coalesced loads of the five
// fields), keeps per cell (w = g dV 2 T^3/gamma^3 / (2 pi hbar c)^3, vx, vy,
// gamma/T, g dV/(2 pi hbar c)^3) in LDS, and each lane then adds those cells
// to the outputs it owns, reading the cell values as LDS broadcasts.  With
// fewer outputs than lanes the lanes form groups that take every
// groups-th cell of the chunk.  Partial sums are per workgroup and fixed
// cell order; a second pass adds the workgroups in order, a third forms the
// harmonics.  No atomics: results are run-to-run identical.

#include <hip/hip_runtime.h>

#include "hydro_internal.hpp"

#include "hydro_device.hpp"

namespace hydro {

namespace {

// OPL: outputs per lane, ceil(n_out / 256) rounded up to 1, 2 or 4 (its
// arrays live in registers: fewer outputs, more waves).
template <class R, int OPL>
__global__ void __launch_bounds__(kFoThreads) k_fo_partial(FreezeArgs<R> a) {
  __shared__ double s_w[kFoThreads], s_vx[kFoThreads], s_vy[kFoThreads], s_gt[kFoThreads], s_wp[kFoThreads];
  __shared__ double s_red[kFoThreads];
  const int tid = threadIdx.x;
  // Outputs of this lane.  groups > 1 (n_out <= 128): lane tid is in group
  // tid / n_out and owns output tid % n_out; the groups split the chunk's
  // cells.  groups == 1: lane tid owns outputs tid + 256 m, m < OPL.
  const int per = (a.groups > 1) ? a.n_out : kFoThreads;  // stride between a lane's outputs
  const int grp = (a.groups > 1) ? tid / a.n_out : 0;
  const int o0 = (a.groups > 1) ? tid % a.n_out : tid;
  const bool active = grp < a.groups;
  double acc[OPL], cph[OPL], sph[OPL], ptv[OPL];
  int row[OPL];
  bool own[OPL];
#pragma unroll
  for (int m = 0; m < OPL; ++m) {
    const int o = o0 + m * per;
    own[m] = active && (a.groups > 1 ? m == 0 : o < a.n_out);
    const int k = own[m] ? o % a.n_phi : 0;
    row[m] = own[m] ? o / a.n_phi : 0;
    double sv, cv;
    sincospi(2.0 * (double)k / (double)a.n_phi, &sv, &cv);
    cph[m] = cv;
    sph[m] = sv;
    ptv[m] = row[m] > 0 ? a.pt[row[m] - 1] : 0.0;
    acc[m] = 0.0;
  }
  unsigned fix = 0;
  const long long nchunk = (a.nc + kFoThreads - 1) / kFoThreads;
  for (long long ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const long long cell = ch * kFoThreads + tid;
    double w = 0.0, wp = 0.0, vx = 0.0, vy = 0.0, gt = 0.0;
    if (cell < a.nc) {
      R u[5];
      load5(a.U, a.nc, cell, u);
      const PrimV pv = c2p(u, fix);
      const double T = temperature(pv.e, a.eos_dof, a.hbarc);
      if (T >= a.T_min) {
        const double v2 = pv.v[0] * pv.v[0] + pv.v[1] * pv.v[1] + pv.v[2] * pv.v[2];
        const double ig = sqrt_nr(1.0 - v2);  // 1/gamma
        w = a.pref_dV * 2.0 * (T * ig) * (T * ig) * (T * ig);
        wp = a.pref_dV;
        gt = div_nr(1.0, ig * T);
        vx = pv.v[0];
        vy = pv.v[1];
      }
    }
    __syncthreads();  // the previous chunk is no longer read
    s_w[tid] = w;
    s_wp[tid] = wp;
    s_vx[tid] = vx;
    s_vy[tid] = vy;
    s_gt[tid] = gt;
    __syncthreads();
    const int ncell = (int)min((long long)kFoThreads, a.nc - ch * kFoThreads);
    if (active) {
      for (int c = grp; c < ncell; c += a.groups) {
        const double cwp = s_wp[c];
        if (cwp == 0.0) continue;  // below T_min (or past the grid): contributes nothing
        const double cw = s_w[c], cvx = s_vx[c], cvy = s_vy[c], cgt = s_gt[c];
#pragma unroll
        for (int m = 0; m < OPL; ++m) {
          if (!own[m]) continue;
          const double D = fma(-cvy, sph[m], fma(-cvx, cph[m], 1.0));
          if (row[m] == 0) {
            const double q = rcp_nr(D);
            acc[m] = fma(cw, q * q * q, acc[m]);
          } else {
            acc[m] = fma(cwp * ptv[m], exp(-ptv[m] * cgt * D), acc[m]);
          }
        }
      }
    }
  }
  add_fixups(a.fixups, fix);
  double* out = a.part + (long long)blockIdx.x * a.n_out;
  if (a.groups > 1) {
    // groups in order: lane (g, o) holds group g's sum for output o
    s_red[tid] = acc[0];
    __syncthreads();
    if (tid < a.n_out) {
      double t = s_red[tid];
      for (int g = 1; g < a.groups; ++g) t += s_red[g * a.n_out + tid];
      out[tid] = t;
    }
  } else {
#pragma unroll
    for (int m = 0; m < OPL; ++m)
      if (own[m]) out[o0 + m * per] = acc[m];
  }
}

// spectra[o] = sum over workgroups b in order of part[b][o].
__global__ void __launch_bounds__(256) k_fo_final(const double* part, int nblocks, int n_out, double* spectra) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_out) return;
  double t = 0.0;
  for (int b = 0; b < nblocks; ++b) t += part[(long long)b * n_out + o];
  spectra[o] = t;
}

// Harmonics of row blockIdx.x: lane n (0..n_harm) forms harm[row][n] =
// (sum cos(n phi_k) s_k, sum sin(n phi_k) s_k) / sum s_k, lane 0 gives
// (dN/dy, 0) with dN/dy = (2 pi / n_phi) sum s_k.
__global__ void __launch_bounds__(64) k_fo_harm(const double* spectra, int n_phi, int n_harm, double* harm) {
  const int r = blockIdx.x, n = threadIdx.x;
  if (n > n_harm) return;
  const double* s = spectra + (long long)r * n_phi;
  double tot = 0.0;
  for (int k = 0; k < n_phi; ++k) tot += s[k];
  double* h = harm + ((long long)r * (n_harm + 1) + n) * 2;
  if (n == 0) {
    h[0] = 2.0 * 3.14159265358979323846 / n_phi * tot;
    h[1] = 0.0;
    return;
  }
  double cs = 0.0, sn = 0.0;
  for (int k = 0; k < n_phi; ++k) {
    double sv, cv;
    sincospi(2.0 * (double)(((long long)n * k) % n_phi) / (double)n_phi, &sv, &cv);
    cs = fma(cv, s[k], cs);
    sn = fma(sv, s[k], sn);
  }
  h[0] = cs / tot;
  h[1] = sn / tot;
}

}  // namespace

template <class R>
hipError_t launch_freezeout(const FreezeArgs<R>& a, double* spectra, double* harm, int n_harm, hipStream_t st) {
  static_assert(kFoOutPerLane == 4, "outputs per lane: 1, 2 or 4");
  const int opl = (a.n_out + kFoThreads - 1) / kFoThreads;
  if (opl <= 1) hipLaunchKernelGGL((k_fo_partial<R, 1>), dim3(kFoBlocks), dim3(kFoThreads), 0, st, a);
  else if (opl == 2) hipLaunchKernelGGL((k_fo_partial<R, 2>), dim3(kFoBlocks), dim3(kFoThreads), 0, st, a);
  else hipLaunchKernelGGL((k_fo_partial<R, 4>), dim3(kFoBlocks), dim3(kFoThreads), 0, st, a);
  hipLaunchKernelGGL(k_fo_final, dim3((a.n_out + 255) / 256), dim3(256), 0, st, a.part, kFoBlocks, a.n_out, spectra);
  if (harm) hipLaunchKernelGGL(k_fo_harm, dim3(a.rows), dim3(64), 0, st, spectra, a.n_phi, n_harm, harm);
  return hipGetLastError();
}

template hipError_t launch_freezeout<double>(const FreezeArgs<double>&, double*, double*, int, hipStream_t);
template hipError_t launch_freezeout<float>(const FreezeArgs<float>&, double*, double*, int, hipStream_t);

}  // namespace hydro
