// hydro_batch.hip -- host side of the batch API of include/hydro.h: many
// independent events (uneven grids, their own jets) advanced together.
//
// Per stage there is one launch per axis whose workgroups walk the work items
// of every event (x: groups of whole rows, y/z: LDS tiles; a persistent grid
// of a few workgroups per CU, or one workgroup per item), one launch for the
// outflow x faces and one for the jets of every event, and per step one FP64
// reduction launch and a device step counter (stage times are computed on the
// device from it).  The launches of one step are captured once into a HIP
// graph and the graph is replayed for every step.  The grid size of each axis
// is picked by a small autotuner that times the candidates on the batch
// itself (right-hand-side form of a stage, which changes no state) and keeps
// its picks in a text cache keyed by the batch's shape classes.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "hydro.h"
#include "hydro_host.hpp"
#include "hydro_internal.hpp"

using namespace hydro;

struct hydro_batch {
  int n = 0;
  std::vector<hydro_config> cfg;
  std::vector<std::vector<hydro_jet>> jets;
  std::vector<BatchEvent> ev;      // host copy of the device table
  BatchEvent* d_ev = nullptr;      // device table [n]
  long long* d_off = nullptr;      // device item offsets [5][n + 1] (x tiles, y, z, x rows, x boundary)
  std::vector<long long> off;      // host copy
  DevScalars* d_dev = nullptr;     // per-event device scalars [n]
  double* d_part = nullptr;        // reduction partials [n][kSumBlocks][5]
  long long* d_step = nullptr;     // device step counter
  int64_t step = 0;
  int cus = 256;
  long long blocks[3] = {0, 0, 0}; // workgroups per axis launch (0: one per item)
  int xrows = 0;                   // x pass: 0 LDS tiles, 1 groups of whole rows (+ boundary faces)
  int tile_a[3] = {0, 0, 0};       // per axis: the tile length every event shares (31, 32), else 0
  int xtb = 256;                   // x-row workgroup size
  long long xlds = 0;              // its dynamic LDS
  int use_graph = 1;
  hipStream_t cap = nullptr;       // capture stream (never runs work)
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  std::string err;
};

namespace {

thread_local std::string g_batch_error;

int bfail(hydro_batch* b, int code, const std::string& m) {
  if (b) b->err = m;
  else g_batch_error = m;
  return code;
}

int bhip(hydro_batch* b, hipError_t e, const char* where) {
  return bfail(b, HYDRO_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

void drop_graph(hydro_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

bool compatible(const hydro_config& a, const hydro_config& c) {
  return a.precision == c.precision && a.weno == c.weno && a.weno_eps == c.weno_eps && a.weno_p == c.weno_p &&
         a.limiter == c.limiter && a.flux == c.flux && a.musta_k == c.musta_k;
}

size_t field_bytes(const hydro_config& c) { return align256((size_t)5 * ncells(&c) * elem_size(&c)); }

template <class R>
BatchArgs<R> batch_args(const hydro_batch* b, int AX, int stage) {
  BatchArgs<R> a;
  a.ev = b->d_ev;
  a.off = b->d_off + (size_t)AX * (b->n + 1);
  a.items = b->off[(size_t)AX * (b->n + 1) + b->n];
  a.step = b->d_step;
  a.n_events = b->n;
  a.stage = stage;
  a.eps = (R)b->cfg[0].weno_eps;
  a.xtb = b->xtb;
  a.xlds = b->xlds;
  a.tile_a = AX <= 2 ? b->tile_a[AX] : 0;
  return a;
}

// One stage of every event: x tiles (or x rows and the outflow x faces),
// y tiles, jets, z tiles (+ RK combine).
template <class R>
hipError_t stage_launches(hydro_batch* b, int stage, hipStream_t st) {
  const int scheme = face_scheme(b->cfg[0]);
  hipError_t e;
  if (b->xrows) {
    e = launch_batch_axis<R>(3, batch_args<R>(b, 3, stage), scheme, b->blocks[0], st);
    if (e == hipSuccess) e = launch_batch_axis<R>(4, batch_args<R>(b, 4, stage), scheme, 0, st);
  } else {
    e = launch_batch_axis<R>(0, batch_args<R>(b, 0, stage), scheme, b->blocks[0], st);
  }
  if (e == hipSuccess) e = launch_batch_axis<R>(1, batch_args<R>(b, 1, stage), scheme, b->blocks[1], st);
  if (e == hipSuccess) e = launch_batch_jet<R>(batch_args<R>(b, 0, stage), st);
  if (e == hipSuccess) e = launch_batch_axis<R>(2, batch_args<R>(b, 2, stage), scheme, b->blocks[2], st);
  return e;
}

template <class R>
hipError_t step_launches(hydro_batch* b, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (int k = 1; k <= 3 && e == hipSuccess; ++k) e = stage_launches<R>(b, k, st);
  if (e == hipSuccess) e = launch_batch_sums<R>(batch_args<R>(b, 0, 3), b->d_step, st);
  return e;
}

hipError_t step_any(hydro_batch* b, hipStream_t st) {
  return b->cfg[0].precision == HYDRO_F32 ? step_launches<float>(b, st) : step_launches<double>(b, st);
}

hipError_t capture(hydro_batch* b) {
  drop_graph(b);
  hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return e;
  hipError_t el = step_any(b, b->cap);
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(b->cap, &g);
  if (el != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return el;
  }
  if (e != hipSuccess) return e;
  b->graph = g;
  e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    (void)hipGraphDestroy(g);
    b->graph = nullptr;
    b->exec = nullptr;
  }
  return e;
}

// 64-bit FNV-1a of the batch's tuning key.
std::string tune_key(const hydro_batch* b) {
  std::vector<std::string> shapes;
  for (const auto& c : b->cfg) {
    char s[64];
    std::snprintf(s, sizeof(s), "%dx%dx%d", c.n[0], c.n[1], c.n[2]);
    shapes.push_back(s);
  }
  std::sort(shapes.begin(), shapes.end());
  std::ostringstream k;
  hipDeviceProp_t p;
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (hipGetDeviceProperties(&p, dev) == hipSuccess) k << p.gcnArchName << ":" << p.multiProcessorCount;
  k << ":p" << b->cfg[0].precision << ":w" << b->cfg[0].weno << ":l" << b->cfg[0].limiter << ":f" << b->cfg[0].flux
    << ":" << b->cfg[0].musta_k;
  for (const auto& s : shapes) k << ":" << s;
  unsigned long long h = 1469598103934665603ULL;
  for (unsigned char ch : k.str()) {
    h ^= ch;
    h *= 1099511628211ULL;
  }
  char out[32];
  std::snprintf(out, sizeof(out), "%016llx", h);
  return out;
}

// Cache lines: "key bx by bz xrows".
bool cache_lookup(const char* path, const std::string& key, long long blocks[3], int* xrows) {
  if (!path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {  // the last entry for a key wins
    std::istringstream ls(line);
    std::string k;
    long long v[4];
    if (ls >> k >> v[0] >> v[1] >> v[2] >> v[3] && k == key) {
      for (int a = 0; a < 3; ++a) blocks[a] = v[a];
      *xrows = v[3] ? 1 : 0;
      found = true;
    }
  }
  return found;
}

void cache_store(const char* path, const std::string& key, const long long blocks[3], int xrows) {
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << key << " " << blocks[0] << " " << blocks[1] << " " << blocks[2] << " " << xrows << "\n";
}

// Median time (ms) of `reps` launches of one axis kernel in right-hand-side
// form (stage 0: writes only the workspace).
template <class R>
hipError_t time_axis(hydro_batch* b, int AX, long long blocks, int reps, hipStream_t st, float* ms) {
  hipEvent_t e0, e1;
  hipError_t e = hipEventCreate(&e0);
  if (e != hipSuccess) return e;
  e = hipEventCreate(&e1);
  if (e != hipSuccess) {
    (void)hipEventDestroy(e0);
    return e;
  }
  std::vector<float> t;
  const BatchArgs<R> a = batch_args<R>(b, AX, 0);
  const int scheme = face_scheme(b->cfg[0]);
  // each timed launch follows a launch of the axis that precedes it in a
  // stage (z before x, x before y, y before z), so that the caches hold
  // what they hold in a step, not the timed launch's own inputs
  const int prev = (AX == 1) ? 0 : (AX == 2 ? 1 : 2);
  const BatchArgs<R> ap = batch_args<R>(b, prev, 0);
  for (int r = 0; r <= reps && e == hipSuccess; ++r) {
    e = launch_batch_axis<R>(prev, ap, scheme, prev == 0 ? 0 : b->blocks[prev], st);
    if (e == hipSuccess) e = hipEventRecord(e0, st);
    if (e == hipSuccess) e = launch_batch_axis<R>(AX, a, scheme, blocks, st);
    if (e == hipSuccess) e = hipEventRecord(e1, st);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float x = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&x, e0, e1);
    if (r > 0) t.push_back(x);  // first launch is a warm-up
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e == hipSuccess) {
    std::sort(t.begin(), t.end());
    *ms = t[t.size() / 2];
  }
  return e;
}

template <class R>
int autotune_impl(hydro_batch* b, const char* cache, hipStream_t st, int* from_cache) {
  const std::string key = tune_key(b);
  long long best[3];
  int xr = 0;
  if (cache_lookup(cache, key, best, &xr)) {
    for (int a = 0; a < 3; ++a) b->blocks[a] = best[a];
    b->xrows = xr;
    if (from_cache) *from_cache = 1;
    drop_graph(b);
    return HYDRO_OK;
  }
  const long long cand[] = {0, 1, 2, 3, 4, 6, 8};
  // x: LDS tiles (item list 0) or groups of whole rows (3) plus the outflow
  // faces (4, one workgroup per item, timed once); y and z: tiles (1, 2)
  const int lists[4] = {0, 3, 1, 2};
  float xbound = 0.f;
  {
    hipError_t e = time_axis<R>(b, 4, 0, 5, st, &xbound);
    if (e != hipSuccess) return bhip(b, e, "autotune launch");
  }
  float tx[2] = {1e30f, 1e30f};
  long long bx[2] = {0, 0};
  for (int li = 0; li < 4; ++li) {
    const int AX = lists[li];
    float tbest = 1e30f;
    long long pick = 0;
    for (long long c : cand) {
      const long long blocks = c * b->cus;
      float ms = 0.f;
      hipError_t e = time_axis<R>(b, AX, blocks, 5, st, &ms);
      if (e != hipSuccess) return bhip(b, e, "autotune launch");
      if (AX == 3) ms += xbound;
      if (ms < tbest) {
        tbest = ms;
        pick = blocks;
      }
    }
    if (AX == 0 || AX == 3) {
      tx[AX == 3] = tbest;
      bx[AX == 3] = pick;
    } else {
      b->blocks[AX] = pick;
    }
  }
  b->xrows = tx[1] < tx[0] ? 1 : 0;
  b->blocks[0] = bx[b->xrows];
  cache_store(cache, key, b->blocks, b->xrows);
  if (from_cache) *from_cache = 0;
  drop_graph(b);
  return HYDRO_OK;
}

}  // namespace

extern "C" {

size_t hydro_batch_workspace_bytes(const hydro_config* cfgs, int n_events) {
  if (!cfgs || n_events < 1) return 0;
  size_t total = 0;
  for (int e = 0; e < n_events; ++e) {
    if (!config_ok(&cfgs[e], nullptr) || !compatible(cfgs[0], cfgs[e])) return 0;
    total += 3 * field_bytes(cfgs[e]);
  }
  return total;
}

int hydro_batch_create(const hydro_config* cfgs, int n_events, const double* const* prim0, void* const* U,
                       void* workspace, size_t ws_bytes, void* stream, hydro_batch** out) {
  if (!out) return bfail(nullptr, HYDRO_EINVAL, "out is NULL");
  *out = nullptr;
  if (!cfgs || n_events < 1 || !U || !workspace) return bfail(nullptr, HYDRO_EINVAL, "bad arguments to hydro_batch_create");
  std::string why;
  for (int e = 0; e < n_events; ++e) {
    if (!config_ok(&cfgs[e], &why)) return bfail(nullptr, HYDRO_EINVAL, "event " + std::to_string(e) + ": " + why);
    if (!compatible(cfgs[0], cfgs[e]))
      return bfail(nullptr, HYDRO_EINVAL, "events must share precision, weno, weno_eps and weno_p");
    if (!U[e]) return bfail(nullptr, HYDRO_EINVAL, "U[e] is NULL");
  }
  if (((uintptr_t)workspace & 255) != 0) return bfail(nullptr, HYDRO_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < hydro_batch_workspace_bytes(cfgs, n_events)) return bfail(nullptr, HYDRO_EINVAL, "workspace too small");

  hydro_batch* b = new (std::nothrow) hydro_batch();
  if (!b) return bfail(nullptr, HYDRO_ENOMEM, "out of host memory");
  b->n = n_events;
  b->cfg.assign(cfgs, cfgs + n_events);
  b->jets.resize(n_events);
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || b->cus < 1) b->cus = 256;
  hipStream_t st = static_cast<hipStream_t>(stream);

  auto cleanup = [&](int code, const std::string& m) {
    g_batch_error = m;
    if (b->d_ev) (void)hipFree(b->d_ev);
    if (b->d_off) (void)hipFree(b->d_off);
    if (b->d_dev) (void)hipFree(b->d_dev);
    if (b->d_part) (void)hipFree(b->d_part);
    if (b->d_step) (void)hipFree(b->d_step);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return code;
  };
  hipError_t e = lib_malloc(&b->d_ev, sizeof(BatchEvent) * n_events);
  if (e == hipSuccess) e = lib_malloc(&b->d_off, sizeof(long long) * 5 * (n_events + 1));
  if (e == hipSuccess) e = lib_malloc(&b->d_dev, sizeof(DevScalars) * n_events);
  if (e == hipSuccess) e = lib_malloc(&b->d_part, sizeof(double) * (size_t)n_events * kSumBlocks * 5);
  if (e == hipSuccess) e = lib_malloc(&b->d_step, sizeof(long long));
  if (e != hipSuccess) return cleanup(HYDRO_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
  if (e != hipSuccess) return cleanup(HYDRO_EDEVICE, std::string("hipStreamCreate: ") + hipGetErrorString(e));

  unsigned char* ws = static_cast<unsigned char*>(workspace);
  b->ev.resize(n_events);
  b->off.assign((size_t)5 * (n_events + 1), 0);
  {
    std::vector<int> nxs(n_events);
    for (int i = 0; i < n_events; ++i) nxs[i] = cfgs[i].n[0];
    const int elem = (int)elem_size(&cfgs[0]);
    b->xtb = xrow_block(nxs.data(), n_events, elem);
    for (int AX = 0; AX < 3; ++AX) {
      int A = tile_len(cfgs[0].n[AX]);
      for (int i = 1; i < n_events; ++i)
        if (tile_len(cfgs[i].n[AX]) != A) A = 0;
      b->tile_a[AX] = A;
    }
    b->xlds = 0;
    for (int i = 0; i < n_events; ++i)
      b->xlds = std::max<long long>(b->xlds, (long long)xrow_lds_bytes(nxs[i], xrow_rows(nxs[i], b->xtb, elem), elem));
  }
  for (int i = 0; i < n_events; ++i) {
    const hydro_config& c = cfgs[i];
    BatchEvent& v = b->ev[i];
    std::memset(&v, 0, sizeof(v));
    v.g = make_grid(&c);
    v.U = U[i];
    const size_t fb = field_bytes(c);
    v.U1 = ws;
    v.U2 = ws + fb;
    v.D = ws + 2 * fb;
    ws += 3 * fb;
    v.part = b->d_part + (size_t)i * kSumBlocks * 5;
    v.dev = b->d_dev + i;
    v.t0 = c.t0;
    v.dt = c.dt;
    for (int d = 0; d < 3; ++d) v.inv_d[d] = 1.0 / c.dx[d];
    v.dV = c.dx[0] * c.dx[1] * c.dx[2];
    v.pp_mu = pp_mu(c);
    v.musta_k = c.musta_k;
    v.eos_dof = c.eos_dof;
    v.hbarc = c.hbarc;
    v.njet = 0;
    v.deposit = c.deposit;
    for (int a = 0; a < 5; ++a)
      b->off[(size_t)a * (n_events + 1) + i + 1] =
          b->off[(size_t)a * (n_events + 1) + i] + batch_items(a, v.g, b->xtb, (int)elem_size(&c));
  }
  std::vector<DevScalars> zero(n_events);
  std::memset(zero.data(), 0, sizeof(DevScalars) * n_events);
  const long long step0 = 0;
  e = hipMemcpy(b->d_ev, b->ev.data(), sizeof(BatchEvent) * n_events, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_off, b->off.data(), sizeof(long long) * b->off.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_dev, zero.data(), sizeof(DevScalars) * n_events, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->d_step, &step0, sizeof(step0), hipMemcpyHostToDevice);
  if (e != hipSuccess) return cleanup(HYDRO_EDEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));

  // initial states from primitives (host or device FP64), per event
  if (prim0) {
    for (int i = 0; i < n_events && e == hipSuccess; ++i) {
      if (!prim0[i]) continue;
      const long long nc = b->ev[i].g.nc;
      const double* dprim = prim0[i];
      double* tmp = nullptr;
      if (!is_device_pointer(prim0[i])) {
        e = lib_malloc(&tmp, (size_t)5 * nc * sizeof(double));
        if (e == hipSuccess) e = hipMemcpy(tmp, prim0[i], (size_t)5 * nc * sizeof(double), hipMemcpyHostToDevice);
        dprim = tmp;
      }
      if (e == hipSuccess)
        e = cfgs[0].precision == HYDRO_F32 ? launch_prim_to_cons<float>(dprim, static_cast<float*>(U[i]), nc, st)
                                           : launch_prim_to_cons<double>(dprim, static_cast<double*>(U[i]), nc, st);
      if (tmp) {
        hipError_t e2 = hipStreamSynchronize(st);
        if (e == hipSuccess) e = e2;
        e2 = hipFree(tmp);
        if (e == hipSuccess) e = e2;
      }
    }
    if (e != hipSuccess) return cleanup(HYDRO_EDEVICE, std::string("prim->cons: ") + hipGetErrorString(e));
  }
  // default launch shape: two workgroups per CU on every axis
  for (int a = 0; a < 3; ++a) b->blocks[a] = 2LL * b->cus;
  *out = b;
  return HYDRO_OK;
}

int hydro_batch_add_jet(hydro_batch* b, int event, const hydro_jet* jet, int* jet_id) {
  if (!b || !jet || event < 0 || event >= b->n) return bfail(b, HYDRO_EINVAL, "bad arguments to hydro_batch_add_jet");
  BatchEvent& v = b->ev[event];
  if (v.njet >= kMaxJets) return bfail(b, HYDRO_EINVAL, "too many jets");
  if (const char* why = jet_error(jet)) return bfail(b, HYDRO_EINVAL, why);
  const int id = v.njet;
  JetDev jd;
  for (int d = 0; d < 3; ++d) {
    jd.x0[d] = jet->x0[d];
    jd.dir[d] = jet->dir[d];
  }
  jd.t_start = jet->t_start;
  jd.kappa_rad = jet->kappa_rad;
  jd.kappa_coll = jet->kappa_coll;
  jd.crcf = jet->cr_over_cf;
  DevScalars* s = b->d_dev + event;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(&s->jets[id], &jd, sizeof(jd), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(&s->E_jet[id], &jet->E0, sizeof(double), hipMemcpyHostToDevice);
  v.njet = id + 1;
  if (e == hipSuccess) e = hipMemcpy(&b->d_ev[event].njet, &v.njet, sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    v.njet = id;
    return bhip(b, e, "hydro_batch_add_jet");
  }
  b->jets[event].push_back(*jet);
  if (jet_id) *jet_id = id;
  return HYDRO_OK;
}

int hydro_batch_run(hydro_batch* b, int nsteps, void* stream) {
  if (!b || nsteps < 0) return bfail(b, HYDRO_EINVAL, "bad arguments to hydro_batch_run");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (nsteps == 0) return HYDRO_OK;
  if (b->use_graph) {
    if (!b->exec) {
      hipError_t e = capture(b);
      if (e != hipSuccess) return bhip(b, e, "graph capture");
    }
    for (int s = 0; s < nsteps; ++s) {
      hipError_t e = hipGraphLaunch(b->exec, st);
      if (e != hipSuccess) return bhip(b, e, "hipGraphLaunch");
    }
  } else {
    for (int s = 0; s < nsteps; ++s) {
      hipError_t e = step_any(b, st);
      if (e != hipSuccess) return bhip(b, e, "batch step launch");
    }
  }
  b->step += nsteps;
  return HYDRO_OK;
}

int hydro_batch_rhs(hydro_batch* b, void* stream) {
  if (!b) return HYDRO_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = b->cfg[0].precision == HYDRO_F32 ? stage_launches<float>(b, 0, st) : stage_launches<double>(b, 0, st);
  if (e != hipSuccess) return bhip(b, e, "hydro_batch_rhs");
  return HYDRO_OK;
}

int hydro_batch_autotune(hydro_batch* b, const char* cache_path, void* stream, int* from_cache) {
  if (!b) return HYDRO_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  return b->cfg[0].precision == HYDRO_F32 ? autotune_impl<float>(b, cache_path, st, from_cache)
                                          : autotune_impl<double>(b, cache_path, st, from_cache);
}

int hydro_batch_set_option(hydro_batch* b, int option, long long value) {
  if (!b) return HYDRO_EINVAL;
  switch (option) {
    case HYDRO_BOPT_BLOCKS_X:
    case HYDRO_BOPT_BLOCKS_Y:
    case HYDRO_BOPT_BLOCKS_Z:
      if (value < 0) return bfail(b, HYDRO_EINVAL, "workgroup count must be >= 0");
      b->blocks[option - HYDRO_BOPT_BLOCKS_X] = value;
      drop_graph(b);
      return HYDRO_OK;
    case HYDRO_BOPT_GRAPH:
      if (value != 0 && value != 1) return bfail(b, HYDRO_EINVAL, "HYDRO_BOPT_GRAPH takes 0 or 1");
      b->use_graph = (int)value;
      return HYDRO_OK;
    case HYDRO_BOPT_X_ROWS:
      if (value != 0 && value != 1) return bfail(b, HYDRO_EINVAL, "HYDRO_BOPT_X_ROWS takes 0 or 1");
      b->xrows = (int)value;
      drop_graph(b);
      return HYDRO_OK;
    default:
      return bfail(b, HYDRO_EINVAL, "unknown batch option");
  }
}

int hydro_batch_get_option(hydro_batch* b, int option, long long* value) {
  if (!b || !value) return HYDRO_EINVAL;
  switch (option) {
    case HYDRO_BOPT_BLOCKS_X:
    case HYDRO_BOPT_BLOCKS_Y:
    case HYDRO_BOPT_BLOCKS_Z: *value = b->blocks[option - HYDRO_BOPT_BLOCKS_X]; return HYDRO_OK;
    case HYDRO_BOPT_GRAPH: *value = b->use_graph; return HYDRO_OK;
    case HYDRO_BOPT_X_ROWS: *value = b->xrows; return HYDRO_OK;
    default: return bfail(b, HYDRO_EINVAL, "unknown batch option");
  }
}

int hydro_batch_sums(hydro_batch* b, int event, double out[6]) {
  if (!b || !out || event < 0 || event >= b->n) return bfail(b, HYDRO_EINVAL, "bad arguments to hydro_batch_sums");
  hipError_t e = hipDeviceSynchronize();
  DevScalars* s = b->d_dev + event;
  unsigned long long fix = 0;
  if (e == hipSuccess) e = hipMemcpy(out, s->sums, 5 * sizeof(double), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(out + 5, &s->ledger, sizeof(double), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(&fix, &s->fixups, sizeof(fix), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bhip(b, e, "hydro_batch_sums");
  // as hydro_sums: non-finite sums, and fix-ups in strict mode, are reported
  for (int c = 0; c < 6; ++c)
    if (!std::isfinite(out[c])) return bfail(b, HYDRO_ENONPHYS, "non-finite sums (NaN or infinity in the event's state)");
  if (b->cfg[event].strict && fix > 0) return bfail(b, HYDRO_ENONPHYS, "non-admissible cells of the event were fixed up");
  return HYDRO_OK;
}

int hydro_batch_get_state(hydro_batch* b, int event, double* t, int64_t* step, double* E_jet, int n_jet) {
  if (!b || event < 0 || event >= b->n || n_jet < 0 || (n_jet > 0 && !E_jet))
    return bfail(b, HYDRO_EINVAL, "bad arguments to hydro_batch_get_state");
  hipError_t e = hipDeviceSynchronize();
  long long st = 0;
  if (e == hipSuccess) e = hipMemcpy(&st, b->d_step, sizeof(st), hipMemcpyDeviceToHost);
  const int nj = std::min(n_jet, b->ev[event].njet);
  if (e == hipSuccess && nj > 0) e = hipMemcpy(E_jet, b->d_dev[event].E_jet, nj * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return bhip(b, e, "hydro_batch_get_state");
  if (step) *step = st;
  if (t) *t = b->cfg[event].t0 + (double)st * b->cfg[event].dt;
  return HYDRO_OK;
}

int hydro_batch_diag(hydro_batch* b, int64_t* fixups) {
  if (!b || !fixups) return HYDRO_EINVAL;
  hipError_t e = hipDeviceSynchronize();
  unsigned long long tot = 0;
  for (int i = 0; i < b->n && e == hipSuccess; ++i) {
    unsigned long long f = 0;
    e = hipMemcpy(&f, &b->d_dev[i].fixups, sizeof(f), hipMemcpyDeviceToHost);
    tot += f;
  }
  if (e != hipSuccess) return bhip(b, e, "hydro_batch_diag");
  *fixups = (int64_t)tot;
  return HYDRO_OK;
}

const char* hydro_batch_last_error(const hydro_batch* b) { return b ? b->err.c_str() : g_batch_error.c_str(); }

void hydro_batch_destroy(hydro_batch* b) {
  if (!b) return;
  (void)hipDeviceSynchronize();
  drop_graph(b);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  (void)hipFree(b->d_ev);
  (void)hipFree(b->d_off);
  (void)hipFree(b->d_dev);
  (void)hipFree(b->d_part);
  (void)hipFree(b->d_step);
  delete b;
}

}  // extern "C"
