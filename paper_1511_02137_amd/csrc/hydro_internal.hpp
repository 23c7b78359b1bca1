// hydro_internal.hpp -- structures shared by the host part of libhydro and
// its HIP kernels.  Not part of the public ABI (see include/hydro.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace hydro {

constexpr int kMaxJets = 64;       // jets per context
constexpr double kEFloor = 1e-12;  // E at or below: vacuum fix-up
constexpr double kVCap = 1.0 - 1e-10;  // |v| cap of the fix-up
constexpr int kSumBlocks = 1024;   // fixed number of reduction blocks (fixed order)

// WENO7 with Z, Jiang-Shu or linear weights; 3..5: the same for WENO5.
enum Scheme { kWenoZ = 0, kWenoJS = 1, kWenoLinear = 2, kWeno5Z = 3, kWeno5JS = 4, kWeno5Linear = 5 };
// Flag on the face kernels' scheme template argument: positivity-preserving
// flux limiter on.
constexpr int kPP = 8;
// Flag on the same argument: MUSTA-FORCE face fluxes of WENO-reconstructed
// conserved states instead of WENO of the Lax-Friedrichs split fluxes.
constexpr int kMusta = 16;

// Grid of one event.
struct Grid {
  int n[3];        // nx, ny, nz
  int bc[3];       // 0 outflow, 1 periodic
  double dx[3];    // cell widths
  long long nc;    // nx*ny*nz
};

// Static description of a jet on the device (FP64).
struct JetDev {
  double x0[3];
  double dir[3];
  double t_start;
  double kappa_rad, kappa_coll, crcf;
};

// Per-context device scalars (library-owned, a few KB).
struct DevScalars {
  JetDev jets[kMaxJets];
  double E_jet[kMaxJets];     // remaining energy
  double P[3][kMaxJets];      // deposited rate of each stage of the current step
  double ledger;              // deposited energy so far
  double sums[5];             // conservation sums (x dV) of the last hydro_sums call
  double step_sums[5];        // conservation sums (x dV) taken by the last RK3 step
  unsigned long long fixups;  // conserved->primitive fix-ups
  unsigned long long fixups_save;  // fixups on entry to an adjoint sweep (restored on exit)
};

// Arguments of the stage kernels (device pointers).
template <class R>
struct StageArgs {
  const R* W;   // stage input [5][nc]
  const R* Un;  // U^n (stages 2 and 3)
  R* out;       // stage output (may alias Un in stage 3)
  R* D;         // flux divergence accumulator [5][nc]
  Grid g;
  R inv_d;      // 1/dx of the kernel's axis
  R dt;
  R eps;        // epsilon of the WENO weights
  int stage;    // 1, 2, 3 (RK stage); 0: write L = D + S instead of combining
  int seg;      // march segment length (y/z kernels)
  int order;    // LDS tiles: bit AX-1 set = blockIdx.y runs over the transverse axis, blockIdx.z over the tiles
  unsigned long long* fixups;
  double pp_mu;  // 2 dt sum_d 1/dx_d, the half-state factor of the positivity limiter
  int musta_k;   // MUSTA-FORCE stages
};

// Arguments of the jet kernel.
struct JetArgs {
  const void* W;   // stage input
  void* D;         // divergence accumulator (source is added)
  DevScalars* s;
  Grid g;
  int njet;
  int stage;       // 1, 2, 3 (stage 3 also advances E_jet and the ledger); 0: RHS only
  int deposit;     // 0 NGP, 1 Gauss
  double t;        // stage time
  double dt;
  double eos_dof, hbarc;
};

// Cells per LDS tile along the reconstructed axis: 31 (32 face rows, one per
// lane of a 512-lane workgroup) unless 32-cell tiles (33 face rows, the last
// row by 16 lanes, measured ~12 % slower per tile) cover n with less waste.
__host__ __device__ constexpr int tile_len(int n) {
  return ((n + 30) / 31) * 31 * 100 < 112 * (((n + 31) / 32) * 32) ? 31 : 32;
}

// x-row kernels: workgroup of TB lanes holding TB / nx whole rows.  LDS per
// row: max(10 (nx + 8), 5 nx) words.  xrow_block picks TB in {256, 384, 512,
// 1024} for a set of row lengths: every nx <= TB, the LDS of TB / nx rows
// <= 64 KiB, and the fewest lane slots for the cells (ties: the smaller TB).
__host__ __device__ inline size_t xrow_lds_bytes(int nx, int rpi, int elem) {
  const int per_row = 10 * (nx + 8) > 5 * nx ? 10 * (nx + 8) : 5 * nx;
  return (size_t)rpi * per_row * elem;
}

// Rows per workgroup of TB lanes: TB / nx, fewer if their LDS exceeds 64 KiB.
__host__ __device__ inline int xrow_rows(int nx, int TB, int elem) {
  int rpi = TB / nx;
  while (rpi > 1 && xrow_lds_bytes(nx, rpi, elem) > 65536) --rpi;
  return rpi;
}

inline int xrow_block(const int* nxs, int count, int elem) {
  const int cand[4] = {256, 384, 512, 1024};
  int best = 1024;
  double best_cost = 1e300;
  for (int k = 0; k < 4; ++k) {
    const int TB = cand[k];
    bool ok = true;
    double cost = 0.0;
    for (int e = 0; e < count && ok; ++e) {
      const int nx = nxs[e];
      if (nx > TB) ok = false;
      else cost += (double)TB / (double)(xrow_rows(nx, TB, elem) * nx);  // lane slots per cell
    }
    if (ok && cost < best_cost * (1.0 - 1e-12)) {
      best_cost = cost;
      best = TB;
    }
  }
  return best;
}

// One event of a batch (device table, see hydro_batch.hip).
struct BatchEvent {
  Grid g;
  void* U;            // caller's state [5][nc]
  void* U1;           // stage states and divergence (workspace)
  void* U2;
  void* D;
  double* part;       // reduction partials [kSumBlocks][5]
  DevScalars* dev;    // jets, E_jet, ledger, sums, fix-ups
  double t0, dt;
  double inv_d[3];    // 1/dx per axis
  double dV;
  double eos_dof, hbarc;
  double pp_mu;       // 2 dt sum_d 1/dx_d (positivity limiter)
  int musta_k;        // MUSTA-FORCE stages
  int njet;
  int deposit;
};

// Arguments of the batched kernels: the work items of one axis are the tiles
// of every event in event order; off[e] is the first item of event e.
template <class R>
struct BatchArgs {
  const BatchEvent* ev;
  const long long* off;   // [n_events + 1] for the launched axis
  long long items;        // off[n_events]
  const long long* step;  // device step counter (stage times)
  int n_events;
  int stage;              // 1..3; 0: L written to U1 (no state change)
  R eps;
  int xtb;                // workgroup size of the x-row launch (rows per item: xtb / nx)
  int tile_a;             // 31 or 32: every event's tile length along the launched axis (0: they differ)
  long long xlds;         // its dynamic LDS bytes (the largest event)
};

// Arguments of the line adjoint kernels (device pointers).
template <class R>
struct AdjArgs {
  const R* W;   // stage input
  const R* mu;  // adjoint of the stage output (lambda_Y)
  R* G;         // (dL/dW)^T mu accumulator [5][nc]
  Grid g;
  R inv_d;      // 1/dx of the kernel's axis (set by the launcher)
  R eps;        // epsilon of the WENO weights
  int first;    // 1: G = contribution, 0: G += contribution
  unsigned long long* fixups;
  // RK combine in reverse, fused into the last axis (stage 0: none, G is
  // stored).  With b_k the stage weight of W and a_k that of U^n:
  //   lW = b_k (mu + dt G), acc (adjoint of U^n) += a_k mu; stage 1: lW = acc + mu + dt G.
  int stage;
  R dt;
  R* acc;
  R* lW;
  // 1: the N component of mu is taken as zero; N's reverse reconstructions are
  // skipped and its outputs (G, lW, acc) are zero.  N enters no other field's
  // flux and no source, so with a zero N adjoint on entry this is exact.
  int skip_n;
  // lines per workgroup of the y and z line adjoints requested by the caller
  // (0: automatic; 1, 2 or 4); the launcher takes fewer where they do not fit
  int lines;
};

// LDS of the line adjoint kernel, in elements of the field type: split fluxes
// [2][5][n+8] and the face partials of both splits [2][7][n+16] (face x at
// x+8, zero pads so the gather needs no bounds tests).
constexpr long long line_adj_lds_elems(int n) { return 10LL * (n + 8) + 14LL * (n + 16); }
// Elements between the LDS areas of the nl lines of one line-adjoint
// workgroup: padded so that neighbouring lines' copies of a slot are 32/nl
// four-byte banks apart.
constexpr long long line_adj_pitch(int n, int nl) {
  return nl == 1 ? line_adj_lds_elems(n)
                 : line_adj_lds_elems(n) + ((32 / nl - line_adj_lds_elems(n) % 32) % 32 + 32) % 32;
}

// Arguments of the jet-source adjoint kernel.
struct JetAdjArgs {
  const void* W;        // stage input
  const void* mu;       // adjoint of the stage output
  void* G;              // accumulator
  DevScalars* s;
  const double* Ehist;  // jet energies at the start of the step [kMaxJets]
  double* grad;         // parameter gradients [njet][5] (+=)
  Grid g;
  int njet;
  int deposit;
  double t;             // stage time
  double bdt;           // b_k * dt of the stage
  double eos_dof, hbarc;
};

// Freeze-out spectra (hydro_freezeout): limits and arguments.
constexpr int kFoThreads = 256;           // lanes per workgroup
constexpr int kFoMaxOut = 1024;           // (1 + n_pt) * n_phi outputs
constexpr int kFoOutPerLane = kFoMaxOut / kFoThreads;
constexpr int kFoMaxPt = 15;              // p_T values of the differential rows
constexpr int kFoMaxHarm = 32;            // harmonics n = 1..n_harm
constexpr int kFoBlocks = 1024;           // workgroups of the partial-sum pass (fixed order)

template <class R>
struct FreezeArgs {
  const R* U;
  long long nc;
  int n_phi;             // azimuths phi_k = 2 pi k / n_phi
  int rows;              // 1 + n_pt
  int n_out;             // rows * n_phi
  int groups;            // lane groups sharing one set of outputs (n_out <= kFoThreads / groups)
  double pt[kFoMaxPt];   // p_T of rows 1..
  double T_min;          // cells with T < T_min are left out
  double pref_dV;        // g dV / (2 pi hbar c)^3
  double eos_dof, hbarc; // T(e) of the fluid
  double* part;          // [kFoBlocks][n_out] partial sums
  unsigned long long* fixups;
};

}  // namespace hydro
