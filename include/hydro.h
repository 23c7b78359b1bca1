/* hydro.h -- C ABI of libhydro: the per-stage update of (3+1)D ideal
 * relativistic hydrodynamics with a jet source on a Cartesian grid, for
 * AMD MI355X (gfx950).
 *
 * The problem is the one of Marcinkowski et al., "Jet-induced modifications
 * of the characteristic of the bulk nuclear matter" (arXiv:1511.02137),
 * section "Simulation setup":
 *   Eq. (1)  d_mu T^{mu nu} = d_mu((e+p) u^mu u^nu - p g^{mu nu}) = S^nu, with
 *            the conserved variables energy, momentum and charge density;
 *   Eq. (2)  S^nu(x) = sum_i (-dE/dt, -dM/dt) delta^3(x - x_i(t));
 *   Eq. (3)  -dE/dx = kappa_rad (C_R/C_F) T^3 x + kappa_coll (C_R/C_F) T^2;
 *   7th-order WENO in space, third-order Runge-Kutta in time;
 *   EOS p = e/3 (Fig. 3 caption); dx = 0.1 fm, dt = 0.02 fm/c, 256^3 grid.
 *
 * Units: lengths fm, times fm/c, e / E / M GeV fm^-3, n / N fm^-3, T GeV,
 * jet energies GeV.  T follows from e = g pi^2/30 T^4/(hbar c)^3.
 *
 * Conventions for every entry point:
 *   - The state U is caller-owned device memory laid out as five fields
 *     [E, Mx, My, Mz, N][nz][ny][nx], x fastest (structure of arrays), with
 *     E = T^00, M_i = T^0i, N = n u^0; element type double (HYDRO_F64) or
 *     float (HYDRO_F32).  Cells are centred: x_i = (i - (nx-1)/2) dx.
 *   - Large buffers (U, primitives, adjoint fields, workspace) belong to the
 *     caller.  The library owns only the opaque context: configuration, jet
 *     table and a few small device scalars (jet energies, ledger, sums).
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the default
 *     stream) unless stated otherwise.  The calls on one context share its
 *     workspace (the divergence buffer, reduction partials) and its device
 *     scalars, so they are ordered by the caller: one stream, or a
 *     synchronisation between streams.  Calls on one context that overlap
 *     race; different contexts are independent (but for the static array
 *     of hydro_sums_noalloc, below).
 *   - Every function returns a hydro_status.  Argument errors return
 *     HYDRO_EINVAL before any side effect; HIP errors return HYDRO_EDEVICE
 *     and hydro_last_error() gives the HIP error text.  Nothing aborts or
 *     throws across the ABI.
 */
#ifndef HYDRO_H
#define HYDRO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HYDRO_OK = 0,
  HYDRO_EINVAL = -1,    /* bad argument or configuration */
  HYDRO_ENOMEM = -2,    /* a device allocation of the library failed (the
                           environment variable HYDRO_ALLOC_LIMIT_BYTES, a byte
                           count, makes larger allocations fail, for tests) */
  HYDRO_EDEVICE = -3,   /* a HIP call failed */
  HYDRO_ENONPHYS = -4,  /* strict mode: a non-admissible cell was met */
  HYDRO_ESTATE = -5     /* call not valid in the context's current state */
} hydro_status;

typedef enum {
  HYDRO_F64 = 0,  /* all arithmetic in FP64 */
  HYDRO_F32 = 1   /* fields and flux arithmetic FP32; conserved->primitive
                     recovery, conservation sums, jet source and parameter
                     gradients in FP64 */
} hydro_precision;

typedef enum { HYDRO_BC_OUTFLOW = 0, HYDRO_BC_PERIODIC = 1 } hydro_bc;

/* Discretisation of the delta function of Eq. (2). */
typedef enum {
  HYDRO_DEP_NGP = 0,   /* the cell that holds the jet; ties to the upper cell */
  HYDRO_DEP_GAUSS = 1  /* separable Gaussian, sigma = dx, over 7^3 cells */
} hydro_deposit;

/* Nonlinear weights of the 7th-order WENO reconstruction. */
/* Reconstruction: 7th-order WENO (the paper's scheme) with WENO-Z, Jiang-Shu
 * or linear weights; or the 5th-order WENO the paper names as its
 * alternative (section "Simulation setup"), same weight variants, stencil
 * a_{i-2}..a_{i+2}, ideal weights (1, 6, 3)/10, WENO-Z tau = |b0 - b2|.
 * hydro_adjoint_step supports the WENO7 schemes only. */
typedef enum {
  HYDRO_WENO_Z = 0,
  HYDRO_WENO_JS = 1,
  HYDRO_WENO_LINEAR = 2,
  HYDRO_WENO5_Z = 3,
  HYDRO_WENO5_JS = 4,
  HYDRO_WENO5_LINEAR = 5
} hydro_weno;

/* Face-flux limiter.  HYDRO_LIMITER_PP: the positivity-preserving flux
 * limiter after Zhang and Shu (the WENO reference of the paper): each face
 * flux F becomes theta F + (1 - theta) F_LF, F_LF = F+(u_i) + F-(u_{i+1})
 * the first-order Lax-Friedrichs flux, theta in [0, 1] the largest value of
 * a chord rule that keeps the half states u_i - mu (F - f(u_i)/2) and
 * u_{i+1} + mu (F - f(u_{i+1})/2), mu = 2 dt sum_d 1/dx_d, inside
 * { E - |M| >= 1e-13, N >= 1e-13 }.  For admissible input states and
 * dt sum_d 1/dx_d <= 1 every stage output is then admissible (E > |M|,
 * N > 0) up to rounding, with no recovery fix-ups.  Faces that need no
 * limiting keep their WENO flux exactly.  FP64 arithmetic in both forms.
 * hydro_adjoint_step does not support it (HYDRO_EINVAL). */
typedef enum { HYDRO_LIMITER_NONE = 0, HYDRO_LIMITER_PP = 1 } hydro_limiter;

/* Face flux.  HYDRO_FLUX_WENO_LF (default): WENO reconstruction of the
 * Lax-Friedrichs split fluxes (section "Simulation setup").
 * HYDRO_FLUX_MUSTA: the MUSTA-FORCE flux the paper names as its other solver
 * (Toro's multi-stage FORCE flux): the face states are the WENO
 * reconstructions (cfg.weno, WENO7-Z or WENO5-Z) of the conserved values from
 * the left (cells i-3..i+3) and from the right (the mirrored stencil), and
 * cfg.musta_k stages of the FORCE flux on a local two-cell mesh with
 * dt/dx = 0.9 (wave speeds bounded by 1) give the face flux.  Second order on
 * point values.  Not with the limiter; hydro_adjoint_step refuses it. */
typedef enum { HYDRO_FLUX_WENO_LF = 0, HYDRO_FLUX_MUSTA = 1 } hydro_flux;

typedef struct {
  int32_t n[3];        /* cells along x, y, z >= 1; n[0] <= 811 (FP64) or 1024 (FP32),
                          n[1], n[2] <= 65535 */
  double dx[3];        /* cell widths [fm], > 0 */
  double t0;           /* initial time [fm/c] */
  double dt;           /* time step [fm/c], > 0 */
  int32_t bc[3];       /* hydro_bc per axis; outflow = zero-gradient ghost cells */
  int32_t precision;   /* hydro_precision */
  int32_t weno;        /* hydro_weno (default HYDRO_WENO_Z) */
  int32_t deposit;     /* hydro_deposit */
  double weno_eps;     /* epsilon of the weights, (GeV/fm^3)^2 scale; 1e-6.
                          At least 1e-30 in FP64 and 1e-12 in FP32 (the
                          weights' products and squares stay in range);
                          smaller values return HYDRO_EINVAL */
  int32_t weno_p;      /* exponent of the WENO-Z weights; 2 (only 2 is built) */
  int32_t strict;      /* 1: hydro_sums reports HYDRO_ENONPHYS after fix-ups */
  double eos_dof;      /* g of e = g pi^2/30 T^4/(hbar c)^3; 47.5 */
  double hbarc;        /* hbar c [GeV fm]; 0.1973269804 */
  int32_t limiter;     /* hydro_limiter (default HYDRO_LIMITER_NONE) */
  int32_t flux;        /* hydro_flux (default HYDRO_FLUX_WENO_LF) */
  int32_t musta_k;     /* MUSTA-FORCE stages, 1..8 (default 2) */
} hydro_config;

/* One jet (Eq. 2, 3): a straight line at the speed of light from x0 in
 * direction dir (unit vector), created at t_start.  It deposits energy and
 * momentum dir * energy at the rate P = kappa_coll (C_R/C_F) T^2/(hbar c) +
 * kappa_rad (C_R/C_F) T^3 l/(hbar c)^2 [GeV/fm], l = t - t_start the path
 * length, T the local temperature of the stage input.  It deposits while its
 * energy (initially E0, decreased by what it deposits) is positive. */
typedef struct {
  double x0[3];
  double dir[3];
  double E0;
  double t_start;
  double kappa_rad;
  double kappa_coll;
  double cr_over_cf;
} hydro_jet;

typedef struct hydro_ctx hydro_ctx;

/* Fill *cfg with the defaults: the paper's 256^3 shape, dx = 0.1 fm,
 * dt = 0.02 fm/c, t0 = 1 fm/c, outflow, FP64, WENO-Z, NGP deposit, no
 * limiter, WENO-LF face fluxes (musta_k = 2). */
void hydro_default_config(hydro_config* cfg);

/* Bytes of caller-provided device workspace that hydro_init needs for cfg:
 * two stage states and one flux-divergence field (15 words per cell) plus
 * reduction partials (conservation sums, eps2, freeze-out: 8 MiB).
 * adjoint_k > 0 adds room for the 3*adjoint_k stage
 * states one hydro_adjoint_step of adjoint_k steps recomputes (or
 * hydro_rk3_step_record of adjoint_k steps keeps) and for the adjoint
 * fields.  Returns 0 for an invalid cfg. */
size_t hydro_workspace_bytes(const hydro_config* cfg, int adjoint_k);

/* Create a context and set U from primitive fields: the conserved variables
 * of Eq. (1) -- energy and momentum densities T^{0 nu} and the charge density
 * (section "Simulation setup") -- of an initial state given at t0 (the paper
 * starts at t0 = 1 fm/c, section "Results"), with p = e/3 (Fig. 3 caption).
 *   prim0     [5][nz][ny][nx] double: e, vx, vy, vz, n; host or device
 *             memory (detected); |v| < 1, e > 0.  May be NULL: U is then
 *             taken as already initialised by the caller.
 *   U         device, [5][nz][ny][nx] of the precision's type; written.
 *   workspace device, >= hydro_workspace_bytes(cfg, adjoint_k) bytes,
 *             256-byte aligned; owned by the caller, used until destroy.
 *   ws_bytes  its size.
 * The conversion is E = (e+p) gamma^2 - p, M = (e+p) gamma^2 v, N = n gamma
 * with p = e/3.  The context starts at step 0, t = t0, with no jets. */
int hydro_init(const hydro_config* cfg, const double* prim0, void* U, void* workspace,
               size_t ws_bytes, void* stream, hydro_ctx** out);

/* Append a jet; *jet_id (may be NULL) receives its index.  Synchronous. */
int hydro_add_jet(hydro_ctx* ctx, const hydro_jet* jet, int* jet_id);

/* Eq. (1) with the source of Eq. (2)-(3), integrated as the paper states
 * (section "Simulation setup": 7th-order WENO in space, third-order
 * Runge-Kutta in time; dx, dt of the Fig. 3 caption).
 * Advance U (in place) by nsteps Shu-Osher SSP-RK3 steps:
 *   U1 = U + dt L(U);  U2 = 3/4 U + 1/4 (U1 + dt L(U1));
 *   U  = 1/3 U + 2/3 (U2 + dt L(U2)),
 * stage times t_n, t_n + dt, t_n + dt/2, with t_n = t0 + n dt.  L = D + S is
 * the flux divergence of the component-wise WENO7 reconstruction of the
 * Lax-Friedrichs split fluxes F+- = (f +- U)/2 (alpha = 1) plus the jet
 * source.  After each step the jet energies and the deposited-energy ledger
 * advance by dt (P1/6 + P2/6 + 2 P3/3) and the FP64 sums of U dV are taken
 * (hydro_step_sums). */
int hydro_rk3_step(hydro_ctx* ctx, void* U, int nsteps, void* stream);

/* Right-hand side of one stage, L(U) = D(U) + S(U) at time t, into L
 * (device, same layout and type as U, not aliasing U).  Jets deposit with
 * their current energies; E_jet and the ledger are not advanced.  With
 * HYDRO_LIMITER_PP the face fluxes are those limited for a forward-Euler
 * step of length cfg.dt (the limiter depends on dt). */
int hydro_rhs(hydro_ctx* ctx, const void* U, double t, void* L, void* stream);

/* Primitive fields of U: prim [6][nz][ny][nx] of U's type: e, vx, vy, vz,
 * n, T (device).  Recovery in FP64 with p = e/3 (Fig. 3 caption) from the
 * definition T^{0 nu} = (e+p) u^0 u^nu - p g^{0 nu} of Eq. (1); T is the
 * local temperature that Eq. (3) uses (section "Simulation setup"). */
int hydro_primitives(hydro_ctx* ctx, const void* U, void* prim, void* stream);

/* The totals that Eq. (1) conserves without a source and the energy the
 * jets deposit through Eq. (2)-(3) (section "Simulation setup").
 * Synchronous: out[0..4] = sum over cells of E, Mx, My, Mz, N times dV
 * (FP64, fixed reduction order), out[5] = deposited-energy ledger.
 * Returns HYDRO_ENONPHYS when a sum is not finite (a NaN or infinity in U,
 * out still written) and, in strict mode, after a fix-up. */
int hydro_sums(hydro_ctx* ctx, const void* U, double out[6], void* stream);

/* The same totals as taken by the last hydro_rk3_step on ctx (section
 * "Simulation setup"; zero before the first step and after hydro_reset or
 * hydro_set_state).
 * Synchronous: out[0..4] = sums of E, Mx, My, Mz, N times dV of U after that
 * step (the kernels and order of hydro_sums, so bit for bit its values for
 * that U), out[5] = deposited-energy ledger.  HYDRO_ENONPHYS when a sum is
 * not finite. */
int hydro_step_sums(hydro_ctx* ctx, double out[6]);

/* Freeze-out: particles from the evolved fluid and their flow harmonics,
 * the step the paper plans next (section "Results", closing paragraph: add
 * freeze-out to study elliptic flow and higher flow harmonics).  Reading:
 * Cooper-Frye on the fixed-time hypersurface of U (d sigma_mu = (dV, 0, 0,
 * 0)) for a massless Boltzmann species of degeneracy dof at zero chemical
 * potential (the quanta of the p = e/3 fluid), T = T(e) of the fluid's
 * equation of state (cfg.eos_dof), at rapidity 0 along z.  With
 * D = 1 - vx cos phi - vy sin phi and gamma the cell's Lorentz factor:
 *   spectra[0][k]     = dN/(dy dphi)         = dof/(2 pi hbar c)^3 sum dV 2 T^3/(gamma D)^3,
 *   spectra[1 + j][k] = dN/(p_T dp_T dy dphi) = dof/(2 pi hbar c)^3 sum dV p_T exp(-gamma p_T D/T)
 * at phi_k = 2 pi k / n_phi (GeV^-2 for the differential rows, p_T = pt[j]),
 * summed over the cells with T >= T_min.  harm (may be NULL) [1 + n_pt]
 * [n_harm + 1][2]: harm[r][0] = (dN/dy of row r by the trapezoid rule
 * (2 pi/n_phi) sum_k, 0), harm[r][n] = (sum_k cos(n phi_k) s_k, sum_k
 * sin(n phi_k) s_k) / sum_k s_k of row r (0 when the row is empty: no
 * cell at or above T_min): v_n is the modulus of that pair, its angle / n
 * the n-th event-plane angle (x = the reaction plane of the initial
 * ellipsoid).  Both outputs are device FP64, written asynchronously;
 * primitives are recovered in FP64 (fix-ups counted as in hydro_primitives).
 * Fixed reduction order (run-to-run identical).  Limits: 0 <= n_pt <= 15,
 * (1 + n_pt) n_phi <= 1024, 0 <= n_harm <= 32 with 2 n_harm < n_phi,
 * pt[j] > 0, dof > 0, T_min >= 0; else HYDRO_EINVAL.  Reduction partials use
 * the context's workspace. */
typedef struct {
  int32_t n_phi;    /* azimuths */
  int32_t n_pt;     /* p_T-differential rows */
  int32_t n_harm;   /* harmonics */
  int32_t reserved; /* 0 */
  double pt[15];    /* GeV */
  double T_min;     /* GeV; 0 keeps every cell */
  double dof;       /* degeneracy of the emitted species */
} hydro_freezeout_params;

int hydro_freezeout(hydro_ctx* ctx, const void* U, const hydro_freezeout_params* fp, double* spectra,
                    double* harm, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the sums
 * of hydro_sums, asynchronous on `stream` and without any allocation.
 *   out  device FP64 [6], written: out[0..4] = sum of E, Mx, My, Mz, N times
 *        dV, out[5] = deposited-energy ledger; the context's last sums are
 *        updated as by hydro_sums.  Host memory returns HYDRO_EINVAL.
 * The same kernels and fixed reduction order as hydro_sums, so the values
 * are bit for bit those of hydro_sums.  The reduction partials live in a
 * static device array of the library (kSumBlocks x 5 FP64 = 40 KiB per
 * device, held until the process ends) instead of the workspace; every call
 * overwrites all of them, so any grid that hydro_init accepts fits and no
 * size is refused.  Calls that overlap on one device (other streams, other
 * contexts) share that array and race: serialise them.  Strict mode is not
 * checked here (no synchronisation); hydro_diag reports fix-ups. */
int hydro_sums_noalloc(hydro_ctx* ctx, const void* U, double* out, void* stream);

/* Synchronous: time, step index and the jets' remaining energies.
 * hydro_set_state restores them with the ledger (a restart; the step sums
 * read by hydro_step_sums become zero until the next step). */
int hydro_get_state(hydro_ctx* ctx, double* t, int64_t* step, double* E_jet, int n_jet);
int hydro_set_state(hydro_ctx* ctx, int64_t step, const double* E_jet, int n_jet, double ledger);

/* Synchronous: number of conserved->primitive fix-ups so far. */
int hydro_diag(hydro_ctx* ctx, int64_t* fixups);

/* Synchronous: set U from primitive fields prim0 (device FP64, as in
 * hydro_init) and restart the context: step 0, jet energies E0, ledger 0. */
int hydro_reset(hydro_ctx* ctx, const double* prim0, void* U, void* stream);

/* Replace the parameters of jet `id` (synchronous; same checks as
 * hydro_add_jet; E0 resets the jet's remaining energy). */
int hydro_set_jet(hydro_ctx* ctx, int id, const hydro_jet* jet);

/* The energy-weighted anisotropy on the z = 0 plane,
 *   eps2 = sum (y^2 - x^2) e / sum (y^2 + x^2) e,
 * e the rest-frame energy density (mean of the two middle planes for even
 * nz, the middle plane for odd nz), x and y cell centres from the grid
 * origin.  eps2_out: device double (may be NULL).  If seed is not NULL it
 * receives scale * d eps2 / dU (device, layout and type of U, zero off the
 * z = 0 planes). */
int hydro_loss_eps2(hydro_ctx* ctx, const void* U, double* eps2_out, void* seed, double scale, void* stream);

/* Reverse sweep (hand-written adjoint) over the nsteps SSP-RK3 steps that
 * start from the checkpoint U_ckpt taken at step index step0 with jet
 * energies E_jet0 (host [n_jet]; may be NULL without jets).  On entry
 * lambda (device, layout and type of U) holds dJ/dU at step step0 + nsteps,
 * on exit dJ/dU at step0.  grad_jets (device FP64 [n_jet][5]: d/dkappa_rad,
 * d/dkappa_coll, d/dx0, d/dy0, d/dz0; origin derivatives are zero for the
 * NGP deposit) is incremented in FP64.  The stage states of the segment are
 * recomputed into the workspace, which must have been sized with
 * hydro_workspace_bytes(cfg, adjoint_k >= nsteps); each axis must fit the
 * line adjoint's LDS tile ((24 n + 304) words <= 64 KiB: n <= 328 in FP64,
 * n <= 670 in FP32), else HYDRO_EINVAL.  The
 * context's U, step, jet energies and ledger are left unchanged. */
int hydro_adjoint_step(hydro_ctx* ctx, const void* U_ckpt, int64_t step0, const double* E_jet0, int nsteps,
                       void* lambda, double* grad_jets, void* stream);

/* The same reverse sweep without the recompute, for runs whose stage states
 * fit in HBM.  hydro_rk3_step_record advances U by nsteps steps exactly as
 * hydro_rk3_step does (Eq. (1)-(3), SSP-RK3; the same values bit for bit,
 * step sums, jet energies and ledger included) and keeps every step's three
 * stage states and its jet energies in the workspace's adjoint region (sized
 * with hydro_workspace_bytes(cfg, adjoint_k >= nsteps); 3 nsteps states of U's
 * size), replacing an earlier record.  hydro_adjoint_recorded then runs
 * hydro_adjoint_step's sweep over the recorded steps: lambda (device, layout
 * and type of U) in: dJ/dU after them, out: dJ/dU before them; grad_jets
 * (device FP64 [n_jet][5]) is incremented; the result is bit for bit that of
 * hydro_adjoint_step from the record's first state.  The record stays valid
 * for further sweeps (other seeds) until hydro_adjoint_step, hydro_reset,
 * hydro_set_state, hydro_add_jet or hydro_set_jet, after which
 * hydro_adjoint_recorded returns HYDRO_ESTATE.  The same schemes and grid
 * limits as hydro_adjoint_step (HYDRO_EINVAL otherwise); the context's U,
 * step, jet energies and ledger are left unchanged by the sweep. */
int hydro_rk3_step_record(hydro_ctx* ctx, void* U, int nsteps, void* stream);
int hydro_adjoint_recorded(hydro_ctx* ctx, void* lambda, double* grad_jets, void* stream);

/* Adjoint of the primitive->conserved map of hydro_init at prim0 (device
 * FP64 [5][nz][ny][nx]): grad_prim (device FP64, same layout) =
 * (dU/dprim)^T lambda, i.e. d/de, d/dvx, d/dvy, d/dvz, d/dn. */
int hydro_init_vjp(hydro_ctx* ctx, const double* prim0, const void* lambda, double* grad_prim, void* stream);

/* Options of a context.  The launch shapes (0-2) do not change results: every
 * variant computes each face with the same arithmetic.  HYDRO_OPT_ADJ_SKIP_N
 * = 1 makes hydro_adjoint_step take the N component of lambda as zero on
 * entry, skip N's reverse reconstructions and return a zero N component: N
 * enters no other field's flux and no source, so for a loss that does not
 * depend on N (eps2 depends on e and v only) the result is the same as with
 * 0 (the default) and the line adjoints do 4/5 of the reconstruction work. */
typedef enum {
  HYDRO_OPT_YZ_KERNEL = 0,  /* y/z faces: 0 = LDS tiles (default), 1 = register marches */
  HYDRO_OPT_MARCH_SEG = 1,  /* cells per march segment (default 32) */
  HYDRO_OPT_X_KERNEL = 2,   /* x faces: 0 = one row per workgroup (default), 1 = 32 x 16 LDS tiles */
  HYDRO_OPT_ADJ_SKIP_N = 3, /* 0 (default) or 1, see above */
  HYDRO_OPT_TILE_ORDER = 4, /* order of the y/z LDS tiles' workgroups, 0..3: bit 0 (y tiles), bit 1 (z
                               tiles) set = neighbouring workgroups share the tile index and step the
                               transverse axis, clear = they step along the axis; default 2 */
  HYDRO_OPT_ADJ_LINES = 5   /* lines per workgroup of the y and z line adjoints: 0 = automatic
                               (default: 2 in FP32, 1 in FP64), 1, 2 or 4; fewer where n_x is not a
                               multiple or the workgroup would exceed 1024 lanes or 64 KiB of LDS.
                               Neighbouring x lines share the workgroup, so their strided loads
                               share cache lines; every line is computed by the same arithmetic
                               (same results) */
} hydro_option;

/* Set / read an option; HYDRO_EINVAL for an unknown option or bad value. */
int hydro_set_option(hydro_ctx* ctx, int option, int value);
int hydro_get_option(hydro_ctx* ctx, int option, int* value);

/* Kernel classes of a step, for hydro_profile_read. */
typedef enum {
  HYDRO_K_XFACE = 0,   /* x-faces of every row */
  HYDRO_K_XBOUND = 1,  /* right boundary x-face of every row (outflow) */
  HYDRO_K_YMARCH = 2,  /* y-faces (LDS tiles or marches along y) */
  HYDRO_K_JET = 3,     /* jet source */
  HYDRO_K_ZMARCH = 4,  /* z-faces (LDS tiles or marches along z) and the RK combine */
  HYDRO_K_SUMS = 5,    /* FP64 conservation sums */
  HYDRO_K_ADJ = 6,     /* line adjoint kernels of one axis (hydro_adjoint_step) */
  HYDRO_NK = 7
} hydro_kernel_class;

/* Diagnostics: with enable != 0, every later launch of hydro_rk3_step is
 * bracketed by HIP events recorded on its stream.  Not for use under graph
 * capture. */
int hydro_profile(hydro_ctx* ctx, int enable);

/* Synchronous: total milliseconds and launch counts per kernel class since
 * the last read (arrays of nk entries, nk <= HYDRO_NK); then clears. */
int hydro_profile_read(hydro_ctx* ctx, double* ms, int64_t* launches, int nk);

/* Text of the last error on ctx (or of the last failed hydro_init if ctx is
 * NULL).  Valid until the next call on ctx. */
const char* hydro_last_error(const hydro_ctx* ctx);

void hydro_destroy(hydro_ctx* ctx);

/* ------------------------------------------------------------------------
 * Batches: many independent events (each its own grid, spacing, times,
 * boundaries, deposit and jets) advanced together, as an ensemble of the
 * paper's problem.  The events must share precision, weno, weno_eps and
 * weno_p.  Per RK stage there is one launch per axis whose workgroups walk
 * the work items of every event (x: 31/32 x 16-cell tiles or groups of whole
 * rows, y and z: 16 x 31/32-cell tiles), one launch for the jets of every
 * event, and per step one FP64 reduction launch; each
 * face is computed with the same arithmetic as hydro_rk3_step, so every
 * event evolves exactly as it would alone.  Stage times come from a device
 * step counter; the launches of one step are captured once into a HIP graph
 * that hydro_batch_run replays.
 * ------------------------------------------------------------------------ */
typedef struct hydro_batch hydro_batch;

/* Device workspace for a batch: per event two stage states and one
 * divergence field (15 words per cell), each block 256-byte aligned.
 * Returns 0 for an invalid or incompatible list. */
size_t hydro_batch_workspace_bytes(const hydro_config* cfgs, int n_events);

/* Create a batch.
 *   cfgs[n_events]   per-event configurations (host).
 *   prim0            NULL, or [n_events] pointers (each NULL or FP64
 *                    primitives [5][nz][ny][nx] in host or device memory,
 *                    as in hydro_init); NULL entries leave U[e] as is.
 *   U[n_events]      caller-owned device states, written from prim0.
 *   workspace        device, >= hydro_batch_workspace_bytes, 256-aligned,
 *                    caller-owned, used until destroy.
 * All events start at step 0 with no jets.  Errors: hydro_batch_last_error(NULL). */
int hydro_batch_create(const hydro_config* cfgs, int n_events, const double* const* prim0, void* const* U,
                       void* workspace, size_t ws_bytes, void* stream, hydro_batch** out);

/* Append a jet to event `event` (synchronous; checks as hydro_add_jet). */
int hydro_batch_add_jet(hydro_batch* b, int event, const hydro_jet* jet, int* jet_id);

/* Advance every event by nsteps SSP-RK3 steps (as hydro_rk3_step, including
 * the jet energies, ledgers and FP64 sums of each event). */
int hydro_batch_run(hydro_batch* b, int nsteps, void* stream);

/* Right-hand side L = D + S of every event at its current time into its
 * first stage buffer (workspace); no state changes.  For timing/tuning. */
int hydro_batch_rhs(hydro_batch* b, void* stream);

/* Launch-shape options of a batch (results do not depend on them). */
typedef enum {
  HYDRO_BOPT_BLOCKS_X = 0,  /* workgroups of the x launch: 0 = one per tile, else a persistent grid */
  HYDRO_BOPT_BLOCKS_Y = 1,
  HYDRO_BOPT_BLOCKS_Z = 2,
  HYDRO_BOPT_GRAPH = 3,     /* 1 (default): replay a captured graph per step; 0: direct launches */
  HYDRO_BOPT_X_ROWS = 4     /* x faces: 0 (default) = 31/32 x 16 LDS tiles; 1 = groups of whole rows
                               plus a launch for the outflow x faces */
} hydro_batch_option;

int hydro_batch_set_option(hydro_batch* b, int option, long long value);
int hydro_batch_get_option(hydro_batch* b, int option, long long* value);

/* Pick the x-face form (tiles or whole rows) and the workgroup count of each
 * axis launch: the candidates 0 (one per work item) and c * (number of CUs),
 * c in {1, 2, 3, 4, 6, 8}, are timed on this batch (median of 5 launches of
 * the right-hand-side form, no state change) and the fastest kept.
 * cache_path (may be NULL) is a text file of "key bx by bz xrows" lines, the
 * key a hash of the GPU, precision, scheme and the sorted event shapes: a hit
 * skips the timing (*from_cache = 1), a miss appends the picks.
 * Synchronous. */
int hydro_batch_autotune(hydro_batch* b, const char* cache_path, void* stream, int* from_cache);

/* Synchronous: sums of event `event` taken by the last batch step, as
 * hydro_sums (ledger in out[5]; HYDRO_ENONPHYS, out still written, when a
 * sum is not finite or, in strict mode, after a fix-up of that event). */
int hydro_batch_sums(hydro_batch* b, int event, double out[6]);

/* Synchronous: time, step and the remaining jet energies of one event. */
int hydro_batch_get_state(hydro_batch* b, int event, double* t, int64_t* step, double* E_jet, int n_jet);

/* Synchronous: conserved->primitive fix-ups of all events. */
int hydro_batch_diag(hydro_batch* b, int64_t* fixups);

const char* hydro_batch_last_error(const hydro_batch* b);
void hydro_batch_destroy(hydro_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* HYDRO_H */
