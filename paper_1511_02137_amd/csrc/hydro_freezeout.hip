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
// to the outputs it owns, reading the cell values as LDS broadcasts.  Up to
// 256 azimuths a lane owns one azimuth in every row (D and gamma D/T once per
// cell and azimuth; the p_T rows' exponentials by a table-driven exp), and
// 256 / n_phi lane groups take every groups-th cell of the chunk; beyond 256
// azimuths a lane owns up to four (row, azimuth) outputs.  Partial sums are
// per workgroup and fixed cell order; a second pass adds the workgroups' sums
// in a fixed order, a third forms the harmonics.  No atomics: results are
// run-to-run identical.

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

// e^x for x <= 0 in FP64 by a table-driven reduction (Tang's method):
// x = (32 k + j) ln2/32 + r with |r| <= ln2/64, e^x = 2^k 2^(j/32) e^r, e^r
// from its Taylor polynomial of degree 6 (remainder below r^7/7! < 2e-18),
// 2^(j/32) from the table `tab` (32 entries), ln2/32 split in a 32-bit high
// part (exact products t * hi) and a low part.  Within 2 ulp of e^x (checked
// against extended-precision exp on 2e7 points of [-745, 0]); 0 below -745.2,
// where e^x rounds to zero.
__device__ __forceinline__ double exp_neg(double x, const double* tab) {
  const double xc = fmax(x, -746.0);  // keeps t within int (below -745.2 the result is 0 anyway)
  const double t = rint(xc * 46.16624130844683);  // x 32/ln2
  const int n = (int)t;
  const int j = n & 31, k = n >> 5;
  const double r = fma(-t, -0x1.718432a1b0e26p-40, fma(-t, 0x1.62e42ff000000p-6, xc));
  double p = fma(r, 1.0 / 720.0, 1.0 / 120.0);
  p = fma(r, p, 1.0 / 24.0);
  p = fma(r, p, 1.0 / 6.0);
  p = fma(r, p, 0.5);
  p = fma(r, p, 1.0);
  p = fma(r, p, 1.0);
  const double v = ldexp(tab[j] * p, k);
  return x < -745.2 ? 0.0 : v;
}

// The spectra with lanes owning azimuths (n_phi <= 256): lane tid is in group
// tid / n_phi (groups = 256 / n_phi split the chunk's cells) and owns azimuth
// tid % n_phi in every row, so D = 1 - vx cos phi - vy sin phi and gamma D / T
// are formed once per cell and azimuth for all rows.  Row r > 0 adds
// g dV/(2 pi hbar c)^3 p_T exp(-p_T gamma D / T) with exp_neg; the rows' sums
// are reduced over the groups one row at a time, in group order.  MP >= n_pt
// bounds the rows at compile time (the accumulators stay in registers).
template <class R, int MP>
__global__ void __launch_bounds__(kFoThreads) k_fo_phi(FreezeArgs<R> a) {
  __shared__ double s_w[kFoThreads], s_vx[kFoThreads], s_vy[kFoThreads], s_gt[kFoThreads], s_wp[kFoThreads];
  __shared__ double s_red[kFoThreads];
  __shared__ double s_tab[32];
  const int tid = threadIdx.x;
  if (tid < 32) s_tab[tid] = exp2((double)tid / 32.0);
  const int grp = tid / a.n_phi;
  const int k = tid % a.n_phi;
  const bool active = grp < a.groups;
  const int npt = a.rows - 1;
  double sph, cph;
  sincospi(2.0 * (double)k / (double)a.n_phi, &sph, &cph);
  double acc[1 + MP];
#pragma unroll
  for (int r = 0; r <= MP; ++r) acc[r] = 0.0;
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
        const double D = fma(-cvy, sph, fma(-cvx, cph, 1.0));
        const double q = rcp_nr(D);
        acc[0] = fma(cw, q * q * q, acc[0]);
        const double aD = cgt * D;
#pragma unroll
        for (int r = 1; r <= MP; ++r) {
          if (r <= npt) {  // uniform
            const double ptv = a.pt[r - 1];
            acc[r] = fma(cwp * ptv, exp_neg(-ptv * aD, s_tab), acc[r]);
          }
        }
      }
    }
  }
  add_fixups(a.fixups, fix);
  double* out = a.part + (long long)blockIdx.x * a.n_out;
#pragma unroll
  for (int r = 0; r <= MP; ++r) {
    if (r <= npt) {  // uniform
      __syncthreads();
      s_red[tid] = acc[r];
      __syncthreads();
      if (tid < a.n_phi) {
        double t = s_red[tid];
        for (int g = 1; g < a.groups; ++g) t += s_red[g * a.n_phi + tid];
        out[r * a.n_phi + tid] = t;
      }
    }
  }
}

// spectra[o] = sum of part[b][o] over the workgroups b: a workgroup takes 64
// outputs (lane = output, coalesced rows of part); wave w of 16 adds the
// blocks w, w + 16, ... in order, then the 16 wave sums are added in order.
constexpr int kFoFinalWaves = 16;
__global__ void __launch_bounds__(64 * kFoFinalWaves) k_fo_final(const double* part, int nblocks, int n_out,
                                                                double* spectra) {
  __shared__ double s_sum[kFoFinalWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int o = blockIdx.x * 64 + lane;
  double t = 0.0;
  if (o < n_out)
    for (int b = w; b < nblocks; b += kFoFinalWaves) t += part[(long long)b * n_out + o];
  s_sum[w][lane] = t;
  __syncthreads();
  if (w == 0 && o < n_out) {
    double v = s_sum[0][lane];
    for (int k = 1; k < kFoFinalWaves; ++k) v += s_sum[k][lane];
    spectra[o] = v;
  }
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
  h[0] = tot != 0.0 ? cs / tot : 0.0;  // no particles (every cell below T_min): no flow
  h[1] = tot != 0.0 ? sn / tot : 0.0;
}

}  // namespace

template <class R>
hipError_t launch_freezeout(const FreezeArgs<R>& a, double* spectra, double* harm, int n_harm, hipStream_t st) {
  static_assert(kFoOutPerLane == 4, "outputs per lane: 1, 2 or 4");
  if (a.n_phi <= kFoThreads) {
    // lanes own azimuths: groups of n_phi lanes split the cells
    FreezeArgs<R> b = a;
    b.groups = kFoThreads / a.n_phi;
    const int npt = a.rows - 1;
    static_assert(kFoMaxPt == 15, "row bounds 0, 2, 5, 10, 15");
    if (npt == 0) hipLaunchKernelGGL((k_fo_phi<R, 0>), dim3(kFoBlocks), dim3(kFoThreads), 0, st, b);
    else if (npt <= 2) hipLaunchKernelGGL((k_fo_phi<R, 2>), dim3(kFoBlocks), dim3(kFoThreads), 0, st, b);
    else if (npt <= 5) hipLaunchKernelGGL((k_fo_phi<R, 5>), dim3(kFoBlocks), dim3(kFoThreads), 0, st, b);
    else if (npt <= 10) hipLaunchKernelGGL((k_fo_phi<R, 10>), dim3(kFoBlocks), dim3(kFoThreads), 0, st, b);
    else hipLaunchKernelGGL((k_fo_phi<R, 15>), dim3(kFoBlocks), dim3(kFoThreads), 0, st, b);
  } else {
    const int opl = (a.n_out + kFoThreads - 1) / kFoThreads;
    if (opl <= 1) hipLaunchKernelGGL((k_fo_partial<R, 1>), dim3(kFoBlocks), dim3(kFoThreads), 0, st, a);
    else if (opl == 2) hipLaunchKernelGGL((k_fo_partial<R, 2>), dim3(kFoBlocks), dim3(kFoThreads), 0, st, a);
    else hipLaunchKernelGGL((k_fo_partial<R, 4>), dim3(kFoBlocks), dim3(kFoThreads), 0, st, a);
  }
  hipLaunchKernelGGL(k_fo_final, dim3((a.n_out + 63) / 64), dim3(64 * kFoFinalWaves), 0, st, a.part, kFoBlocks,
                     a.n_out, spectra);
  if (harm) hipLaunchKernelGGL(k_fo_harm, dim3(a.rows), dim3(64), 0, st, spectra, a.n_phi, n_harm, harm);
  return hipGetLastError();
}

template hipError_t launch_freezeout<double>(const FreezeArgs<double>&, double*, double*, int, hipStream_t);
template hipError_t launch_freezeout<float>(const FreezeArgs<float>&, double*, double*, int, hipStream_t);

}  // namespace hydro
