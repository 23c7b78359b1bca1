// hydro_api.hip -- host side of libhydro: the C ABI of include/hydro.h.
//
// The context keeps the configuration, the jet table and a small block of
// device scalars; all large buffers are the caller's.  A step is a fixed
// sequence of launches on the caller's stream with no host synchronisation,
// so a caller may capture it in a HIP graph.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "hydro.h"
#include "hydro_internal.hpp"

#include "hydro_host.hpp"

using namespace hydro;

struct hydro_ctx {
  hydro_config cfg;
  Grid g;
  int device = 0;    // HIP device current at hydro_init
  int njet = 0;
  hydro_jet jets[kMaxJets];
  DevScalars* dev = nullptr;
  unsigned char* ws = nullptr;
  size_t ws_bytes = 0;
  void* U1 = nullptr;
  void* U2 = nullptr;
  void* D = nullptr;
  double* part = nullptr;
  double* eps_part = nullptr;  // 256 x 2 partial sums of eps2
  double* eps_out = nullptr;   // eps2, numerator, denominator
  double* fo_part = nullptr;   // freeze-out partial sums [kFoBlocks][kFoMaxOut]
  // adjoint region (capacity adj_k steps)
  int adj_k = 0;
  unsigned char* states = nullptr;  // 3 adj_k stage states
  void* lamA = nullptr;
  void* lamB = nullptr;
  void* lacc = nullptr;
  void* G = nullptr;
  double* Ehist = nullptr;  // [adj_k][kMaxJets]
  double* Esave = nullptr;  // [kMaxJets + 1]
  // steps whose stage states and jet energies hydro_rk3_step_record left in
  // the adjoint region (rec_n = 0: none, or overwritten since)
  int64_t rec_step0 = 0;
  int rec_n = 0;
  size_t field_bytes = 0;
  int64_t step = 0;
  int seg = 32;      // march segment length
  int yz_tile = 1;   // 1: y/z faces from LDS tiles, 0: register-window marches
  int x_tile = 0;    // 1: x faces from 32 x 16 LDS tiles, 0: one row per workgroup
  int adj_skip_n = 0;  // 1: the adjoint sweep takes lambda_N as zero and skips N
  int adj_lines = 0;   // lines per workgroup of the y/z line adjoints (0: automatic)
  int tile_order = 2;  // HYDRO_OPT_TILE_ORDER: z tiles step the transverse axis (measured 6 % faster)
  std::string err;
  // per-kernel timing (hydro_profile): event pairs recorded around launches
  bool prof = false;
  struct Mark {
    int kernel;
    hipEvent_t b, e;
  };
  std::vector<Mark> marks;
  std::vector<hipEvent_t> pool;
};

namespace {

thread_local std::string g_init_error;

// Reduction partials of hydro_sums_noalloc: the kSumBlocks x 5 FP64 partial
// sums (40 KiB) of the conservation-sum reduction, one copy per device, held
// until the process ends.  The reduction always runs kSumBlocks blocks and
// each block overwrites its own five partials, so the array needs no
// clearing and any grid fits.  Host code never passes the symbol itself: the
// per-device address comes from hipGetSymbolAddress, taken once per device in
// hydro_init with that device current.
constexpr int kMaxDevices = 64;
constexpr int kScratchDoubles = kSumBlocks * 5;

}  // namespace

static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {

std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
hipError_t g_scratch_err[kMaxDevices] = {};

// Takes the address of `scratch` on device `dev` (current) once.
void scratch_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev]) return;
  double* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(reinterpret_cast<void**>(&ptr), HIP_SYMBOL(scratch));
  if (e == hipSuccess && ptr) {
    g_scratch_ptr[dev] = ptr;
  } else {
    g_scratch_err[dev] = e == hipSuccess ? hipErrorInvalidSymbol : e;
  }
}

double* scratch_for(int dev, hipError_t* why) {
  if (dev < 0 || dev >= kMaxDevices) {
    *why = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  *why = g_scratch_err[dev];
  return g_scratch_ptr[dev];
}

struct WsLayout {
  size_t U1, U2, D, part, eps_part, eps_out, fo_part, fwd_total;
  size_t states, lamA, lamB, lacc, G, Ehist, Esave, total;
  size_t field;
};

WsLayout layout(const hydro_config* c, int adjoint_k) {
  WsLayout L;
  const size_t field = align256((size_t)5 * ncells(c) * elem_size(c));
  L.field = field;
  L.U1 = 0;
  L.U2 = L.U1 + field;
  L.D = L.U2 + field;
  L.part = L.D + field;
  L.eps_part = L.part + align256((size_t)kSumBlocks * 5 * sizeof(double));
  L.eps_out = L.eps_part + align256(512 * sizeof(double));
  L.fo_part = L.eps_out + align256(8 * sizeof(double));
  L.fwd_total = L.fo_part + align256((size_t)kFoBlocks * kFoMaxOut * sizeof(double));
  L.states = L.lamA = L.lamB = L.lacc = L.G = L.Ehist = L.Esave = L.fwd_total;
  L.total = L.fwd_total;
  if (adjoint_k > 0) {
    L.states = L.fwd_total;
    L.lamA = L.states + (size_t)3 * adjoint_k * field;
    L.lamB = L.lamA + field;
    L.lacc = L.lamB + field;
    L.G = L.lacc + field;
    L.Ehist = L.G + field;
    L.Esave = L.Ehist + align256((size_t)adjoint_k * kMaxJets * sizeof(double));
    L.total = L.Esave + align256((kMaxJets + 1) * sizeof(double));
  }
  return L;
}

int fail(hydro_ctx* ctx, int code, const std::string& m) {
  if (ctx) ctx->err = m;
  return code;
}

int hip_fail(hydro_ctx* ctx, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  if (ctx) ctx->err = m;
  return HYDRO_EDEVICE;
}

hipEvent_t take_event(hydro_ctx* ctx) {
  if (!ctx->pool.empty()) {
    hipEvent_t ev = ctx->pool.back();
    ctx->pool.pop_back();
    return ev;
  }
  hipEvent_t ev = nullptr;
  if (hipEventCreate(&ev) != hipSuccess) return nullptr;
  return ev;
}

// Brackets one launch with events when profiling is on.
struct ProfScope {
  hydro_ctx* ctx;
  int kernel;
  hipStream_t st;
  hipEvent_t b = nullptr;
  ProfScope(hydro_ctx* c, int k, hipStream_t s) : ctx(c), kernel(k), st(s) {
    if (ctx->prof) {
      b = take_event(ctx);
      if (b) (void)hipEventRecord(b, st);
    }
  }
  ~ProfScope() {
    if (b) {
      hipEvent_t e = take_event(ctx);
      if (e) {
        (void)hipEventRecord(e, st);
        ctx->marks.push_back({kernel, b, e});
      } else {
        ctx->pool.push_back(b);
      }
    }
  }
};

// One stage: L(W) at time t, then (stage 1..3) the RK combine into out, or
// (stage 0) L itself into out.
template <class R>
hipError_t stage_impl(hydro_ctx* ctx, const R* W, const R* Un, R* out, int stage, double t, hipStream_t st) {
  const hydro_config& c = ctx->cfg;
  StageArgs<R> a;
  a.g = ctx->g;
  a.dt = (R)c.dt;
  a.eps = (R)c.weno_eps;
  a.fixups = &ctx->dev->fixups;
  a.seg = ctx->seg;
  a.order = ctx->tile_order;
  a.stage = stage;
  a.W = W;
  a.Un = Un;
  a.out = out;
  a.D = static_cast<R*>(ctx->D);
  a.pp_mu = pp_mu(c);
  a.musta_k = c.musta_k;
  const int scheme = face_scheme(c);
  hipError_t e;
  {
    ProfScope p(ctx, HYDRO_K_XFACE, st);
    e = launch_face_kernel<R>(ctx->x_tile ? 6 : 0, a, scheme, ctx->seg, st);
  }
  if (e == hipSuccess && c.bc[0] == HYDRO_BC_OUTFLOW && !ctx->x_tile) {
    ProfScope p(ctx, HYDRO_K_XBOUND, st);
    e = launch_face_kernel<R>(1, a, scheme, ctx->seg, st);
  }
  if (e == hipSuccess) {
    ProfScope p(ctx, HYDRO_K_YMARCH, st);
    e = launch_face_kernel<R>(ctx->yz_tile ? 4 : 2, a, scheme, ctx->seg, st);
  }
  if (e == hipSuccess && ctx->njet > 0) {
    JetArgs j;
    j.W = W;
    j.D = a.D;
    j.s = ctx->dev;
    j.g = ctx->g;
    j.njet = ctx->njet;
    j.stage = stage;
    j.deposit = c.deposit;
    j.t = t;
    j.dt = c.dt;
    j.eos_dof = c.eos_dof;
    j.hbarc = c.hbarc;
    ProfScope p(ctx, HYDRO_K_JET, st);
    e = launch_jet<R>(j, st);
  }
  if (e == hipSuccess) {
    ProfScope p(ctx, HYDRO_K_ZMARCH, st);
    e = launch_face_kernel<R>(ctx->yz_tile ? 5 : 3, a, scheme, ctx->seg, st);
  }
  return e;
}

template <class R>
int step_impl(hydro_ctx* ctx, R* U, int nsteps, hipStream_t st) {
  const hydro_config& c = ctx->cfg;
  const double dt = c.dt;
  R* U1 = static_cast<R*>(ctx->U1);
  R* U2 = static_cast<R*>(ctx->U2);
  const double cstage[3] = {0.0, 1.0, 0.5};
  const double dV = c.dx[0] * c.dx[1] * c.dx[2];
  for (int s = 0; s < nsteps; ++s) {
    const double tn = c.t0 + (double)ctx->step * dt;
    for (int k = 1; k <= 3; ++k) {
      const R* W = (k == 1) ? U : (k == 2 ? U1 : U2);
      R* out = (k == 1) ? U1 : (k == 2 ? U2 : U);
      hipError_t e = stage_impl<R>(ctx, W, U, out, k, tn + cstage[k - 1] * dt, st);
      if (e != hipSuccess) return hip_fail(ctx, e, "stage launch");
    }
    hipError_t e;
    {
      ProfScope p(ctx, HYDRO_K_SUMS, st);
      e = launch_sums<R>(U, ctx->g.nc, dV, ctx->part, ctx->dev->step_sums, st);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "sums launch");
    ctx->step += 1;
  }
  return HYDRO_OK;
}

bool adjoint_fits(const hydro_config* c, std::string* why) {
  if (c->weno > 2) {
    if (why) *why = "the adjoint is built for the WENO7 schemes only";
    return false;
  }
  if (c->limiter != HYDRO_LIMITER_NONE || c->flux != HYDRO_FLUX_WENO_LF) {
    if (why) *why = "the adjoint is built for WENO-LF fluxes without the limiter";
    return false;
  }
  for (int d = 0; d < 3; ++d) {
    const size_t lds = (size_t)line_adj_lds_elems(c->n[d]) * elem_size(c);
    if (lds > 65536 || c->n[d] > 1024) {
      if (why) *why = "grid too large along an axis for the line adjoint (LDS line tile)";
      return false;
    }
  }
  return true;
}

#define HYDRO_TRY(x)                        \
  do {                                      \
    e = (x);                                \
    if (e != hipSuccess) return hip_fail(ctx, e, #x); \
  } while (0)

// Stage state k (0: U^n, 1, 2: the inputs of stages 2 and 3) of step i of the
// adjoint region.
template <class R>
R* state_ptr(hydro_ctx* ctx, int i, int k) {
  return reinterpret_cast<R*>(ctx->states) + (size_t)(3 * i + k) * (ctx->field_bytes / sizeof(R));
}

// Keeps the context's jet energies, ledger and fix-up count: the recomputed
// stages and the reverse kernels recover primitives again, which must not
// count as new fix-ups of the run (8-byte moves, bit for bit).
int adjoint_save(hydro_ctx* ctx, hipStream_t st) {
  hipError_t e = hipSuccess;
  HYDRO_TRY(launch_copy_f64(ctx->dev->E_jet, ctx->Esave, kMaxJets, st));
  HYDRO_TRY(launch_copy_f64(&ctx->dev->ledger, ctx->Esave + kMaxJets, 1, st));
  HYDRO_TRY(launch_copy_f64(reinterpret_cast<const double*>(&ctx->dev->fixups),
                            reinterpret_cast<double*>(&ctx->dev->fixups_save), 1, st));
  return HYDRO_OK;
}

int adjoint_restore(hydro_ctx* ctx, hipStream_t st) {
  hipError_t e = hipSuccess;
  HYDRO_TRY(launch_copy_f64(ctx->Esave, ctx->dev->E_jet, kMaxJets, st));
  HYDRO_TRY(launch_copy_f64(ctx->Esave + kMaxJets, &ctx->dev->ledger, 1, st));
  HYDRO_TRY(launch_copy_f64(reinterpret_cast<const double*>(&ctx->dev->fixups_save),
                            reinterpret_cast<double*>(&ctx->dev->fixups), 1, st));
  return HYDRO_OK;
}

// Reverse sweep over the K steps from step0 whose stage states and jet
// energies are in the adjoint region.
template <class R>
int sweep_impl(hydro_ctx* ctx, int64_t step0, int K, R* lam, double* grad, hipStream_t st);

template <class R>
int adjoint_impl(hydro_ctx* ctx, const R* Uc, int64_t step0, const double* E0, int K, R* lam, double* grad,
                 hipStream_t st) {
  const hydro_config& c = ctx->cfg;
  const double dt = c.dt;
  const long long n5 = 5 * ctx->g.nc;
  auto st_ptr = [&](int i, int k) { return state_ptr<R>(ctx, i, k); };
  hipError_t e = hipSuccess;
  ctx->rec_n = 0;  // the recompute overwrites any recorded steps
  int rc = adjoint_save(ctx, st);
  if (rc != HYDRO_OK) return rc;
  // the checkpoint's jet energies (host memory): ordered after the saves above
  HYDRO_TRY(hipStreamSynchronize(st));
  if (ctx->njet > 0) HYDRO_TRY(hipMemcpy(ctx->dev->E_jet, E0, (size_t)ctx->njet * sizeof(double), hipMemcpyHostToDevice));
  // recompute the stage states of the segment
  HYDRO_TRY(launch_copy<R>(Uc, st_ptr(0, 0), n5, st));
  for (int i = 0; i < K; ++i) {
    const double tn = c.t0 + (double)(step0 + i) * dt;
    HYDRO_TRY(launch_copy_f64(ctx->dev->E_jet, ctx->Ehist + (size_t)i * kMaxJets, kMaxJets, st));
    HYDRO_TRY(stage_impl<R>(ctx, st_ptr(i, 0), st_ptr(i, 0), st_ptr(i, 1), 1, tn, st));
    HYDRO_TRY(stage_impl<R>(ctx, st_ptr(i, 1), st_ptr(i, 0), st_ptr(i, 2), 2, tn + dt, st));
    // the segment's last output is the next checkpoint, which the reverse
    // sweep does not read (the jet energies are restored below)
    if (i + 1 < K) HYDRO_TRY(stage_impl<R>(ctx, st_ptr(i, 2), st_ptr(i, 0), st_ptr(i + 1, 0), 3, tn + 0.5 * dt, st));
  }
  rc = sweep_impl<R>(ctx, step0, K, lam, grad, st);
  if (rc != HYDRO_OK) return rc;
  return adjoint_restore(ctx, st);
}

// Forward steps as step_impl, with the stage states of every step and the jet
// energies at its start kept in the adjoint region (stage 3 writes the next
// step's U^n there, the last one U), so that a reverse sweep needs no
// recompute.  Bit for bit the values of step_impl.
template <class R>
int record_impl(hydro_ctx* ctx, R* U, int nsteps, hipStream_t st) {
  const hydro_config& c = ctx->cfg;
  const double dt = c.dt;
  const long long n5 = 5 * ctx->g.nc;
  const double cstage[3] = {0.0, 1.0, 0.5};
  const double dV = c.dx[0] * c.dx[1] * c.dx[2];
  auto st_ptr = [&](int i, int k) { return state_ptr<R>(ctx, i, k); };
  hipError_t e = hipSuccess;
  ctx->rec_n = 0;
  const int64_t step0 = ctx->step;
  HYDRO_TRY(launch_copy<R>(U, st_ptr(0, 0), n5, st));
  for (int i = 0; i < nsteps; ++i) {
    const double tn = c.t0 + (double)ctx->step * dt;
    HYDRO_TRY(launch_copy_f64(ctx->dev->E_jet, ctx->Ehist + (size_t)i * kMaxJets, kMaxJets, st));
    R* out3 = (i + 1 < nsteps) ? st_ptr(i + 1, 0) : U;
    for (int k = 1; k <= 3; ++k) {
      R* out = (k < 3) ? st_ptr(i, k) : out3;
      HYDRO_TRY(stage_impl<R>(ctx, st_ptr(i, k - 1), st_ptr(i, 0), out, k, tn + cstage[k - 1] * dt, st));
    }
    {
      ProfScope p(ctx, HYDRO_K_SUMS, st);
      HYDRO_TRY(launch_sums<R>(out3, ctx->g.nc, dV, ctx->part, ctx->dev->step_sums, st));
    }
    ctx->step += 1;
  }
  ctx->rec_step0 = step0;
  ctx->rec_n = nsteps;
  return HYDRO_OK;
}

template <class R>
int sweep_impl(hydro_ctx* ctx, int64_t step0, int K, R* lam, double* grad, hipStream_t st) {
  const hydro_config& c = ctx->cfg;
  const double dt = c.dt;
  auto st_ptr = [&](int i, int k) { return state_ptr<R>(ctx, i, k); };
  R* lamA = static_cast<R*>(ctx->lamA);
  R* lamB = static_cast<R*>(ctx->lamB);
  R* acc = static_cast<R*>(ctx->lacc);
  R* G = static_cast<R*>(ctx->G);
  hipError_t e = hipSuccess;
  AdjArgs<R> a;
  a.g = ctx->g;
  a.eps = (R)c.weno_eps;
  a.fixups = &ctx->dev->fixups;
  a.G = G;
  a.dt = (R)dt;
  a.acc = acc;
  a.stage = 0;
  a.skip_n = ctx->adj_skip_n;
  a.lines = ctx->adj_lines;
  const double cst[3] = {0.0, 1.0, 0.5};
  const double bst[3] = {1.0, 0.25, 2.0 / 3.0};
  for (int i = K - 1; i >= 0; --i) {
    const double tn = c.t0 + (double)(step0 + i) * dt;
    for (int k = 3; k >= 1; --k) {
      const R* lY = (k == 3) ? lam : (k == 2 ? lamA : lamB);
      a.lW = (k == 3) ? lamA : (k == 2 ? lamB : lam);
      a.W = st_ptr(i, k - 1);
      a.mu = lY;
      // y starts G, z adds, the jet source adds at its cells, x adds and
      // applies the reverse RK combine (x lines are contiguous in memory, so
      // the combine's five extra fields are read and written coalesced)
      const int order[3] = {1, 2, 0};
      for (int step_ax = 0; step_ax < 3; ++step_ax) {
        const int ax = order[step_ax];
        if (step_ax == 2 && ctx->njet > 0) {
          JetAdjArgs j;
          j.W = a.W;
          j.mu = lY;
          j.G = G;
          j.s = ctx->dev;
          j.Ehist = ctx->Ehist + (size_t)i * kMaxJets;
          j.grad = grad;
          j.g = ctx->g;
          j.njet = ctx->njet;
          j.deposit = c.deposit;
          j.t = tn + cst[k - 1] * dt;
          j.bdt = bst[k - 1] * dt;
          j.eos_dof = c.eos_dof;
          j.hbarc = c.hbarc;
          HYDRO_TRY(launch_jet_adj<R>(j, st));
        }
        a.first = step_ax == 0 ? 1 : 0;
        a.stage = step_ax == 2 ? k : 0;
        ProfScope p(ctx, HYDRO_K_ADJ, st);
        HYDRO_TRY(launch_adj_axis<R>(ax, a, c.weno, st));
      }
    }
  }
  return HYDRO_OK;
}

template <class R>
int recorded_impl(hydro_ctx* ctx, R* lam, double* grad, hipStream_t st) {
  int rc = adjoint_save(ctx, st);
  if (rc != HYDRO_OK) return rc;
  rc = sweep_impl<R>(ctx, ctx->rec_step0, ctx->rec_n, lam, grad, st);
  if (rc != HYDRO_OK) return rc;
  return adjoint_restore(ctx, st);
}
#undef HYDRO_TRY

}  // namespace

extern "C" {

void hydro_default_config(hydro_config* c) {
  if (!c) return;
  std::memset(c, 0, sizeof(*c));
  for (int d = 0; d < 3; ++d) {
    c->n[d] = 256;
    c->dx[d] = 0.1;
    c->bc[d] = HYDRO_BC_OUTFLOW;
  }
  c->t0 = 1.0;
  c->dt = 0.02;
  c->precision = HYDRO_F64;
  c->weno = HYDRO_WENO_Z;
  c->deposit = HYDRO_DEP_NGP;
  c->weno_eps = 1e-6;
  c->weno_p = 2;
  c->strict = 0;
  c->eos_dof = 47.5;
  c->hbarc = 0.1973269804;
  c->limiter = HYDRO_LIMITER_NONE;
  c->flux = HYDRO_FLUX_WENO_LF;
  c->musta_k = 2;
}

size_t hydro_workspace_bytes(const hydro_config* cfg, int adjoint_k) {
  if (!config_ok(cfg, nullptr) || adjoint_k < 0) return 0;
  if (adjoint_k > 0 && !adjoint_fits(cfg, nullptr)) return 0;
  return layout(cfg, adjoint_k).total;
}

int hydro_init(const hydro_config* cfg, const double* prim0, void* U, void* workspace, size_t ws_bytes,
               void* stream, hydro_ctx** out) {
  std::string why;
  if (!out) {
    g_init_error = "out is NULL";
    return HYDRO_EINVAL;
  }
  *out = nullptr;
  if (!config_ok(cfg, &why)) {
    g_init_error = why;
    return HYDRO_EINVAL;
  }
  const WsLayout L = layout(cfg, 0);
  if (!U || !workspace) {
    g_init_error = "U and workspace must be device pointers";
    return HYDRO_EINVAL;
  }
  if (((uintptr_t)workspace & 255) != 0) {
    g_init_error = "workspace must be 256-byte aligned";
    return HYDRO_EINVAL;
  }
  if (ws_bytes < L.total) {
    g_init_error = "workspace too small";
    return HYDRO_EINVAL;
  }
  hydro_ctx* ctx = new (std::nothrow) hydro_ctx();
  if (!ctx) {
    g_init_error = "out of host memory";
    return HYDRO_ENOMEM;
  }
  ctx->cfg = *cfg;
  ctx->g = make_grid(cfg);
  ctx->ws = static_cast<unsigned char*>(workspace);
  ctx->ws_bytes = ws_bytes;
  ctx->U1 = ctx->ws + L.U1;
  ctx->U2 = ctx->ws + L.U2;
  ctx->D = ctx->ws + L.D;
  ctx->part = reinterpret_cast<double*>(ctx->ws + L.part);
  ctx->eps_part = reinterpret_cast<double*>(ctx->ws + L.eps_part);
  ctx->eps_out = reinterpret_cast<double*>(ctx->ws + L.eps_out);
  ctx->fo_part = reinterpret_cast<double*>(ctx->ws + L.fo_part);
  ctx->field_bytes = L.field;
  {
    int k = 0;
    while (k < 100000 && layout(cfg, k + 1).total <= ws_bytes) ++k;
    ctx->adj_k = k;
    if (k > 0) {
      const WsLayout A = layout(cfg, k);
      ctx->states = ctx->ws + A.states;
      ctx->lamA = ctx->ws + A.lamA;
      ctx->lamB = ctx->ws + A.lamB;
      ctx->lacc = ctx->ws + A.lacc;
      ctx->G = ctx->ws + A.G;
      ctx->Ehist = reinterpret_cast<double*>(ctx->ws + A.Ehist);
      ctx->Esave = reinterpret_cast<double*>(ctx->ws + A.Esave);
    }
  }
  // march segment: full short axes, 32 cells otherwise
  ctx->seg = 32;
  hipStream_t st = static_cast<hipStream_t>(stream);

  hipError_t e = hipGetDevice(&ctx->device);
  if (e != hipSuccess) {
    g_init_error = std::string("hipGetDevice: ") + hipGetErrorString(e);
    delete ctx;
    return HYDRO_EDEVICE;
  }
  scratch_setup(ctx->device);
  e = lib_malloc(&ctx->dev, sizeof(DevScalars));
  if (e != hipSuccess) {
    g_init_error = std::string("hipMalloc: ") + hipGetErrorString(e);
    delete ctx;
    return HYDRO_ENOMEM;
  }
  DevScalars zero;
  std::memset(&zero, 0, sizeof(zero));
  e = hipMemcpy(ctx->dev, &zero, sizeof(zero), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    g_init_error = std::string("hipMemcpy: ") + hipGetErrorString(e);
    (void)hipFree(ctx->dev);
    delete ctx;
    return HYDRO_EDEVICE;
  }

  if (prim0) {
    const long long nc = ctx->g.nc;
    const double* dprim = prim0;
    double* tmp = nullptr;
    if (!is_device_pointer(prim0)) {
      e = lib_malloc(&tmp, (size_t)5 * nc * sizeof(double));
      if (e != hipSuccess) {
        g_init_error = std::string("hipMalloc(prim0 staging): ") + hipGetErrorString(e);
        (void)hipFree(ctx->dev);
        delete ctx;
        return HYDRO_ENOMEM;
      }
      e = hipMemcpyAsync(tmp, prim0, (size_t)5 * nc * sizeof(double), hipMemcpyHostToDevice, st);
      dprim = tmp;
    }
    if (e == hipSuccess) {
      e = cfg->precision == HYDRO_F32 ? launch_prim_to_cons<float>(dprim, static_cast<float*>(U), nc, st)
                                      : launch_prim_to_cons<double>(dprim, static_cast<double*>(U), nc, st);
    }
    if (tmp) {
      hipError_t e2 = hipStreamSynchronize(st);
      if (e == hipSuccess) e = e2;
      e2 = hipFree(tmp);
      if (e == hipSuccess) e = e2;
    }
    if (e != hipSuccess) {
      g_init_error = std::string("prim->cons: ") + hipGetErrorString(e);
      (void)hipFree(ctx->dev);
      delete ctx;
      return HYDRO_EDEVICE;
    }
  }
  *out = ctx;
  return HYDRO_OK;
}

int hydro_add_jet(hydro_ctx* ctx, const hydro_jet* jet, int* jet_id) {
  if (!ctx || !jet) return HYDRO_EINVAL;
  if (ctx->njet >= kMaxJets) return fail(ctx, HYDRO_EINVAL, "too many jets");
  if (const char* why = jet_error(jet)) return fail(ctx, HYDRO_EINVAL, why);
  const int id = ctx->njet;
  JetDev jd;
  for (int d = 0; d < 3; ++d) {
    jd.x0[d] = jet->x0[d];
    jd.dir[d] = jet->dir[d];
  }
  jd.t_start = jet->t_start;
  jd.kappa_rad = jet->kappa_rad;
  jd.kappa_coll = jet->kappa_coll;
  jd.crcf = jet->cr_over_cf;
  hipError_t e = hipMemcpy(&ctx->dev->jets[id], &jd, sizeof(jd), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(&ctx->dev->E_jet[id], &jet->E0, sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_add_jet");
  ctx->jets[id] = *jet;
  ctx->njet = id + 1;
  ctx->rec_n = 0;
  if (jet_id) *jet_id = id;
  return HYDRO_OK;
}

int hydro_rk3_step(hydro_ctx* ctx, void* U, int nsteps, void* stream) {
  if (!ctx || !U || nsteps < 0) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_rk3_step");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ctx->cfg.precision == HYDRO_F32) return step_impl<float>(ctx, static_cast<float*>(U), nsteps, st);
  return step_impl<double>(ctx, static_cast<double*>(U), nsteps, st);
}

int hydro_rhs(hydro_ctx* ctx, const void* U, double t, void* L, void* stream) {
  if (!ctx || !U || !L || U == L || !std::isfinite(t)) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_rhs");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = ctx->cfg.precision == HYDRO_F32
                     ? stage_impl<float>(ctx, static_cast<const float*>(U), nullptr, static_cast<float*>(L), 0, t, st)
                     : stage_impl<double>(ctx, static_cast<const double*>(U), nullptr, static_cast<double*>(L), 0, t, st);
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_rhs");
  return HYDRO_OK;
}

int hydro_primitives(hydro_ctx* ctx, const void* U, void* prim, void* stream) {
  if (!ctx || !U || !prim) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_primitives");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (ctx->cfg.precision == HYDRO_F32)
    e = launch_primitives<float>(static_cast<const float*>(U), static_cast<float*>(prim), ctx->g.nc,
                                 ctx->cfg.eos_dof, ctx->cfg.hbarc, &ctx->dev->fixups, st);
  else
    e = launch_primitives<double>(static_cast<const double*>(U), static_cast<double*>(prim), ctx->g.nc,
                                  ctx->cfg.eos_dof, ctx->cfg.hbarc, &ctx->dev->fixups, st);
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_primitives");
  return HYDRO_OK;
}

int hydro_sums(hydro_ctx* ctx, const void* U, double out[6], void* stream) {
  if (!ctx || !U || !out) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_sums");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double dV = ctx->cfg.dx[0] * ctx->cfg.dx[1] * ctx->cfg.dx[2];
  hipError_t e = ctx->cfg.precision == HYDRO_F32
                     ? launch_sums<float>(static_cast<const float*>(U), ctx->g.nc, dV, ctx->part, ctx->dev->sums, st)
                     : launch_sums<double>(static_cast<const double*>(U), ctx->g.nc, dV, ctx->part, ctx->dev->sums, st);
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_sums launch");
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_sums sync");
  DevScalars h;
  e = hipMemcpy(&h, ctx->dev, sizeof(DevScalars), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_sums copy");
  for (int c = 0; c < 5; ++c) out[c] = h.sums[c];
  out[5] = h.ledger;
  for (int c = 0; c < 6; ++c)
    if (!std::isfinite(out[c])) return fail(ctx, HYDRO_ENONPHYS, "non-finite sums (NaN or infinity in the state)");
  if (ctx->cfg.strict && h.fixups > 0) return fail(ctx, HYDRO_ENONPHYS, "non-admissible cells were fixed up");
  return HYDRO_OK;
}

int hydro_sums_noalloc(hydro_ctx* ctx, const void* U, double* out, void* stream) {
  if (!ctx || !U || !out) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_sums_noalloc");
  if (!is_device_pointer(out)) return fail(ctx, HYDRO_EINVAL, "hydro_sums_noalloc: out must be device memory");
  static_assert(kScratchDoubles >= kSumBlocks * 5, "scratch holds the reduction partials");
  hipError_t why = hipSuccess;
  double* part = scratch_for(ctx->device, &why);
  if (!part) return hip_fail(ctx, why, "hydro_sums_noalloc: address of the static scratch array");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double dV = ctx->cfg.dx[0] * ctx->cfg.dx[1] * ctx->cfg.dx[2];
  hipError_t e = ctx->cfg.precision == HYDRO_F32
                     ? launch_sums<float>(static_cast<const float*>(U), ctx->g.nc, dV, part, ctx->dev->sums, st)
                     : launch_sums<double>(static_cast<const double*>(U), ctx->g.nc, dV, part, ctx->dev->sums, st);
  if (e == hipSuccess) e = launch_copy_f64(ctx->dev->sums, out, 5, st);
  if (e == hipSuccess) e = launch_copy_f64(&ctx->dev->ledger, out + 5, 1, st);
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_sums_noalloc launch");
  return HYDRO_OK;
}

int hydro_step_sums(hydro_ctx* ctx, double out[6]) {
  if (!ctx || !out) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_step_sums");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_step_sums sync");
  DevScalars h;
  e = hipMemcpy(&h, ctx->dev, sizeof(DevScalars), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_step_sums copy");
  for (int c = 0; c < 5; ++c) out[c] = h.step_sums[c];
  out[5] = h.ledger;
  for (int c = 0; c < 6; ++c)
    if (!std::isfinite(out[c])) return fail(ctx, HYDRO_ENONPHYS, "non-finite sums (NaN or infinity in the state)");
  return HYDRO_OK;
}

int hydro_freezeout(hydro_ctx* ctx, const void* U, const hydro_freezeout_params* fp, double* spectra,
                    double* harm, void* stream) {
  if (!ctx || !U || !fp || !spectra) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_freezeout");
  const int rows = 1 + fp->n_pt;
  if (fp->n_pt < 0 || fp->n_pt > kFoMaxPt || fp->n_phi < 1 || (long long)rows * fp->n_phi > kFoMaxOut)
    return fail(ctx, HYDRO_EINVAL, "hydro_freezeout: need 0 <= n_pt <= 15, n_phi >= 1, (1 + n_pt) n_phi <= 1024");
  if (fp->n_harm < 0 || fp->n_harm > kFoMaxHarm || 2 * fp->n_harm >= fp->n_phi)
    return fail(ctx, HYDRO_EINVAL, "hydro_freezeout: need 0 <= n_harm <= 32 and 2 n_harm < n_phi");
  if (!(fp->dof > 0.0) || !std::isfinite(fp->dof) || !(fp->T_min >= 0.0) || !std::isfinite(fp->T_min))
    return fail(ctx, HYDRO_EINVAL, "hydro_freezeout: need dof > 0 and T_min >= 0, finite");
  for (int j = 0; j < fp->n_pt; ++j)
    if (!(fp->pt[j] > 0.0) || !std::isfinite(fp->pt[j]))
      return fail(ctx, HYDRO_EINVAL, "hydro_freezeout: p_T values must be positive and finite");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const double pi = 3.14159265358979323846;
  const double dV = ctx->cfg.dx[0] * ctx->cfg.dx[1] * ctx->cfg.dx[2];
  const double l = 2.0 * pi * ctx->cfg.hbarc;
  hipError_t e;
  auto fill = [&](auto& a) {
    a.nc = ctx->g.nc;
    a.n_phi = fp->n_phi;
    a.rows = rows;
    a.n_out = rows * fp->n_phi;
    a.groups = a.n_out < kFoThreads ? kFoThreads / a.n_out : 1;
    for (int j = 0; j < kFoMaxPt; ++j) a.pt[j] = j < fp->n_pt ? fp->pt[j] : 0.0;
    a.T_min = fp->T_min;
    a.pref_dV = fp->dof * dV / (l * l * l);
    a.eos_dof = ctx->cfg.eos_dof;
    a.hbarc = ctx->cfg.hbarc;
    a.part = ctx->fo_part;
    a.fixups = &ctx->dev->fixups;
  };
  if (ctx->cfg.precision == HYDRO_F32) {
    FreezeArgs<float> a;
    fill(a);
    a.U = static_cast<const float*>(U);
    e = launch_freezeout<float>(a, spectra, harm, fp->n_harm, st);
  } else {
    FreezeArgs<double> a;
    fill(a);
    a.U = static_cast<const double*>(U);
    e = launch_freezeout<double>(a, spectra, harm, fp->n_harm, st);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_freezeout launch");
  return HYDRO_OK;
}

int hydro_get_state(hydro_ctx* ctx, double* t, int64_t* step, double* E_jet, int n_jet) {
  if (!ctx || n_jet < 0 || (n_jet > 0 && !E_jet)) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_get_state");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_get_state sync");
  if (t) *t = ctx->cfg.t0 + (double)ctx->step * ctx->cfg.dt;
  if (step) *step = ctx->step;
  const int m = n_jet < ctx->njet ? n_jet : ctx->njet;
  if (m > 0) {
    e = hipMemcpy(E_jet, ctx->dev->E_jet, (size_t)m * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return hip_fail(ctx, e, "hydro_get_state copy");
  }
  return HYDRO_OK;
}

int hydro_set_state(hydro_ctx* ctx, int64_t step, const double* E_jet, int n_jet, double ledger) {
  if (!ctx || step < 0 || n_jet != ctx->njet || (n_jet > 0 && !E_jet))
    return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_set_state");
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess && n_jet > 0)
    e = hipMemcpy(ctx->dev->E_jet, E_jet, (size_t)n_jet * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(&ctx->dev->ledger, &ledger, sizeof(double), hipMemcpyHostToDevice);
  // the step sums belonged to the state before the restart
  const double zeros[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (e == hipSuccess) e = hipMemcpy(ctx->dev->step_sums, zeros, sizeof(zeros), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_set_state");
  ctx->step = step;
  ctx->rec_n = 0;
  return HYDRO_OK;
}

int hydro_diag(hydro_ctx* ctx, int64_t* fixups) {
  if (!ctx || !fixups) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_diag");
  unsigned long long f = 0;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(&f, &ctx->dev->fixups, sizeof(f), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_diag");
  *fixups = (int64_t)f;
  return HYDRO_OK;
}

int hydro_reset(hydro_ctx* ctx, const double* prim0, void* U, void* stream) {
  if (!ctx || !prim0 || !U) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_reset");
  if (!is_device_pointer(prim0)) return fail(ctx, HYDRO_EINVAL, "hydro_reset needs prim0 in device memory");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = ctx->cfg.precision == HYDRO_F32
                     ? launch_prim_to_cons<float>(prim0, static_cast<float*>(U), ctx->g.nc, st)
                     : launch_prim_to_cons<double>(prim0, static_cast<double*>(U), ctx->g.nc, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  double E0[kMaxJets];
  for (int j = 0; j < ctx->njet; ++j) E0[j] = ctx->jets[j].E0;
  const double zero = 0.0;
  if (e == hipSuccess && ctx->njet > 0)
    e = hipMemcpy(ctx->dev->E_jet, E0, (size_t)ctx->njet * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(&ctx->dev->ledger, &zero, sizeof(double), hipMemcpyHostToDevice);
  const double zeros[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (e == hipSuccess) e = hipMemcpy(ctx->dev->step_sums, zeros, sizeof(zeros), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_reset");
  ctx->step = 0;
  ctx->rec_n = 0;
  return HYDRO_OK;
}

int hydro_set_jet(hydro_ctx* ctx, int id, const hydro_jet* jet) {
  if (!ctx || !jet || id < 0 || id >= ctx->njet) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_set_jet");
  if (const char* why = jet_error(jet)) return fail(ctx, HYDRO_EINVAL, why);
  JetDev jd;
  for (int d = 0; d < 3; ++d) {
    jd.x0[d] = jet->x0[d];
    jd.dir[d] = jet->dir[d];
  }
  jd.t_start = jet->t_start;
  jd.kappa_rad = jet->kappa_rad;
  jd.kappa_coll = jet->kappa_coll;
  jd.crcf = jet->cr_over_cf;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(&ctx->dev->jets[id], &jd, sizeof(jd), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(&ctx->dev->E_jet[id], &jet->E0, sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_set_jet");
  ctx->jets[id] = *jet;
  ctx->rec_n = 0;
  return HYDRO_OK;
}

int hydro_loss_eps2(hydro_ctx* ctx, const void* U, double* eps2_out, void* seed, double scale, void* stream) {
  if (!ctx || !U) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_loss_eps2");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const long long n5 = 5 * ctx->g.nc;
  hipError_t e;
  if (ctx->cfg.precision == HYDRO_F32) {
    e = launch_eps2<float>(static_cast<const float*>(U), ctx->g, ctx->eps_part, ctx->eps_out, st);
    if (e == hipSuccess && seed) e = launch_fill<float>(static_cast<float*>(seed), n5, 0.0f, st);
    if (e == hipSuccess && seed)
      e = launch_eps2_seed<float>(static_cast<const float*>(U), ctx->g, ctx->eps_out, static_cast<float*>(seed), scale, st);
  } else {
    e = launch_eps2<double>(static_cast<const double*>(U), ctx->g, ctx->eps_part, ctx->eps_out, st);
    if (e == hipSuccess && seed) e = launch_fill<double>(static_cast<double*>(seed), n5, 0.0, st);
    if (e == hipSuccess && seed)
      e = launch_eps2_seed<double>(static_cast<const double*>(U), ctx->g, ctx->eps_out, static_cast<double*>(seed), scale, st);
  }
  if (e == hipSuccess && eps2_out) e = launch_copy_f64(ctx->eps_out, eps2_out, 1, st);
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_loss_eps2");
  return HYDRO_OK;
}

int hydro_adjoint_step(hydro_ctx* ctx, const void* U_ckpt, int64_t step0, const double* E_jet0, int nsteps,
                       void* lambda, double* grad_jets, void* stream) {
  if (!ctx || !U_ckpt || !lambda || nsteps < 0 || step0 < 0) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_adjoint_step");
  if (ctx->njet > 0 && (!E_jet0 || !grad_jets)) return fail(ctx, HYDRO_EINVAL, "jets need E_jet0 and grad_jets");
  if (nsteps > ctx->adj_k) return fail(ctx, HYDRO_EINVAL, "workspace holds fewer adjoint steps than nsteps");
  std::string why;
  if (!adjoint_fits(&ctx->cfg, &why)) return fail(ctx, HYDRO_EINVAL, why);
  if (nsteps == 0) return HYDRO_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ctx->cfg.precision == HYDRO_F32)
    return adjoint_impl<float>(ctx, static_cast<const float*>(U_ckpt), step0, E_jet0, nsteps, static_cast<float*>(lambda),
                               grad_jets, st);
  return adjoint_impl<double>(ctx, static_cast<const double*>(U_ckpt), step0, E_jet0, nsteps,
                              static_cast<double*>(lambda), grad_jets, st);
}

int hydro_rk3_step_record(hydro_ctx* ctx, void* U, int nsteps, void* stream) {
  if (!ctx || !U || nsteps < 1) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_rk3_step_record");
  if (nsteps > ctx->adj_k) return fail(ctx, HYDRO_EINVAL, "workspace holds fewer adjoint steps than nsteps");
  std::string why;
  if (!adjoint_fits(&ctx->cfg, &why)) return fail(ctx, HYDRO_EINVAL, why);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ctx->cfg.precision == HYDRO_F32) return record_impl<float>(ctx, static_cast<float*>(U), nsteps, st);
  return record_impl<double>(ctx, static_cast<double*>(U), nsteps, st);
}

int hydro_adjoint_recorded(hydro_ctx* ctx, void* lambda, double* grad_jets, void* stream) {
  if (!ctx || !lambda) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_adjoint_recorded");
  if (ctx->njet > 0 && !grad_jets) return fail(ctx, HYDRO_EINVAL, "jets need grad_jets");
  if (ctx->rec_n == 0)
    return fail(ctx, HYDRO_ESTATE, "no recorded steps: hydro_rk3_step_record first (hydro_adjoint_step, "
                                   "hydro_reset, hydro_set_state, hydro_add_jet and hydro_set_jet discard the record)");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ctx->cfg.precision == HYDRO_F32)
    return recorded_impl<float>(ctx, static_cast<float*>(lambda), grad_jets, st);
  return recorded_impl<double>(ctx, static_cast<double*>(lambda), grad_jets, st);
}

int hydro_init_vjp(hydro_ctx* ctx, const double* prim0, const void* lambda, double* grad_prim, void* stream) {
  if (!ctx || !prim0 || !lambda || !grad_prim) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_init_vjp");
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = ctx->cfg.precision == HYDRO_F32
                     ? launch_prim_vjp<float>(prim0, static_cast<const float*>(lambda), grad_prim, ctx->g.nc, st)
                     : launch_prim_vjp<double>(prim0, static_cast<const double*>(lambda), grad_prim, ctx->g.nc, st);
  if (e != hipSuccess) return hip_fail(ctx, e, "hydro_init_vjp");
  return HYDRO_OK;
}

int hydro_set_option(hydro_ctx* ctx, int option, int value) {
  if (!ctx) return HYDRO_EINVAL;
  switch (option) {
    case HYDRO_OPT_YZ_KERNEL:
      if (value != 0 && value != 1) return fail(ctx, HYDRO_EINVAL, "HYDRO_OPT_YZ_KERNEL takes 0 or 1");
      ctx->yz_tile = value == 0 ? 1 : 0;
      return HYDRO_OK;
    case HYDRO_OPT_MARCH_SEG:
      if (value < 1 || value > 4096) return fail(ctx, HYDRO_EINVAL, "HYDRO_OPT_MARCH_SEG must be in [1, 4096]");
      ctx->seg = value;
      return HYDRO_OK;
    case HYDRO_OPT_X_KERNEL:
      if (value != 0 && value != 1) return fail(ctx, HYDRO_EINVAL, "HYDRO_OPT_X_KERNEL takes 0 or 1");
      ctx->x_tile = value;
      return HYDRO_OK;
    case HYDRO_OPT_ADJ_SKIP_N:
      if (value != 0 && value != 1) return fail(ctx, HYDRO_EINVAL, "HYDRO_OPT_ADJ_SKIP_N takes 0 or 1");
      ctx->adj_skip_n = value;
      return HYDRO_OK;
    case HYDRO_OPT_TILE_ORDER:
      if (value < 0 || value > 3) return fail(ctx, HYDRO_EINVAL, "HYDRO_OPT_TILE_ORDER takes 0..3");
      ctx->tile_order = value;
      return HYDRO_OK;
    case HYDRO_OPT_ADJ_LINES:
      if (value != 0 && value != 1 && value != 2 && value != 4)
        return fail(ctx, HYDRO_EINVAL, "HYDRO_OPT_ADJ_LINES takes 0, 1, 2 or 4");
      ctx->adj_lines = value;
      return HYDRO_OK;
    default:
      return fail(ctx, HYDRO_EINVAL, "unknown option");
  }
}

int hydro_get_option(hydro_ctx* ctx, int option, int* value) {
  if (!ctx || !value) return HYDRO_EINVAL;
  switch (option) {
    case HYDRO_OPT_YZ_KERNEL: *value = ctx->yz_tile ? 0 : 1; return HYDRO_OK;
    case HYDRO_OPT_MARCH_SEG: *value = ctx->seg; return HYDRO_OK;
    case HYDRO_OPT_X_KERNEL: *value = ctx->x_tile; return HYDRO_OK;
    case HYDRO_OPT_ADJ_SKIP_N: *value = ctx->adj_skip_n; return HYDRO_OK;
    case HYDRO_OPT_TILE_ORDER: *value = ctx->tile_order; return HYDRO_OK;
    case HYDRO_OPT_ADJ_LINES: *value = ctx->adj_lines; return HYDRO_OK;
    default: return fail(ctx, HYDRO_EINVAL, "unknown option");
  }
}

int hydro_profile(hydro_ctx* ctx, int enable) {
  if (!ctx) return HYDRO_EINVAL;
  ctx->prof = enable != 0;
  return HYDRO_OK;
}

int hydro_profile_read(hydro_ctx* ctx, double* ms, int64_t* launches, int nk) {
  if (!ctx || nk < 0 || (nk > 0 && (!ms || !launches))) return fail(ctx, HYDRO_EINVAL, "bad arguments to hydro_profile_read");
  for (int k = 0; k < nk; ++k) {
    ms[k] = 0.0;
    launches[k] = 0;
  }
  hipError_t err = hipSuccess;
  for (auto& m : ctx->marks) {
    if (err == hipSuccess) err = hipEventSynchronize(m.e);
    float t = 0.0f;
    if (err == hipSuccess) err = hipEventElapsedTime(&t, m.b, m.e);
    if (err == hipSuccess && m.kernel < nk) {
      ms[m.kernel] += t;
      launches[m.kernel] += 1;
    }
    ctx->pool.push_back(m.b);
    ctx->pool.push_back(m.e);
  }
  ctx->marks.clear();
  if (err != hipSuccess) return hip_fail(ctx, err, "hydro_profile_read");
  return HYDRO_OK;
}

const char* hydro_last_error(const hydro_ctx* ctx) {
  if (!ctx) return g_init_error.c_str();
  return ctx->err.c_str();
}

void hydro_destroy(hydro_ctx* ctx) {
  if (!ctx) return;
  if (ctx->dev) (void)hipFree(ctx->dev);
  for (auto& m : ctx->marks) {
    (void)hipEventDestroy(m.b);
    (void)hipEventDestroy(m.e);
  }
  for (auto ev : ctx->pool) (void)hipEventDestroy(ev);
  delete ctx;
}

}  // extern "C"
