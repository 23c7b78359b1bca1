// hydro_host.hpp -- host-side helpers shared by the single-event API
// (hydro_api.hip) and the batch API (hydro_batch.hip): configuration checks,
// grid set-up, and the declarations of the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <string>

#include "hydro.h"
#include "hydro_internal.hpp"

namespace hydro {

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Every device allocation of the library goes through here.  With the
// environment variable HYDRO_ALLOC_LIMIT_BYTES set (a decimal byte count),
// larger allocations fail as if the device were out of memory, so that the
// HYDRO_ENOMEM paths can be exercised from the host; unset, it is hipMalloc.
template <class T>
inline hipError_t lib_malloc(T** p, size_t bytes) {
  const char* lim = std::getenv("HYDRO_ALLOC_LIMIT_BYTES");
  if (lim && *lim) {
    char* end = nullptr;
    const unsigned long long v = std::strtoull(lim, &end, 10);
    if (end != lim && bytes > v) {
      *p = nullptr;
      return hipErrorOutOfMemory;
    }
  }
  return hipMalloc(reinterpret_cast<void**>(p), bytes);
}

inline size_t elem_size(const hydro_config* c) { return c->precision == HYDRO_F32 ? sizeof(float) : sizeof(double); }

inline long long ncells(const hydro_config* c) { return (long long)c->n[0] * c->n[1] * c->n[2]; }

inline bool config_ok(const hydro_config* c, std::string* why) {
  auto fail = [&](const char* m) {
    if (why) *why = m;
    return false;
  };
  if (!c) return fail("config is NULL");
  for (int d = 0; d < 3; ++d) {
    if (c->n[d] < 1) return fail("n[d] must be >= 1");
    if (!(c->dx[d] > 0.0) || !std::isfinite(c->dx[d])) return fail("dx[d] must be > 0");
    if (c->bc[d] != HYDRO_BC_OUTFLOW && c->bc[d] != HYDRO_BC_PERIODIC) return fail("bad bc");
  }
  if (c->n[0] > 1024) return fail("n[0] must be <= 1024");
  // the x-face kernel keeps the split fluxes of one row (+8 ghosts) in LDS
  if ((size_t)10 * (c->n[0] + 8) * elem_size(c) > 65536) return fail("n[0] too large for the x-row LDS tile");
  if ((long long)c->n[1] * c->n[2] > 2147483647LL) return fail("too many rows");
  if (c->n[1] > 65535 || c->n[2] > 65535) return fail("n[1], n[2] must be <= 65535");
  if (!(c->dt > 0.0) || !std::isfinite(c->dt) || !std::isfinite(c->t0)) return fail("dt must be > 0");
  if (c->precision != HYDRO_F64 && c->precision != HYDRO_F32) return fail("bad precision");
  if (c->weno < 0 || c->weno > 5) return fail("bad weno");
  if (c->limiter != HYDRO_LIMITER_NONE && c->limiter != HYDRO_LIMITER_PP) return fail("bad limiter");
  if (c->flux != HYDRO_FLUX_WENO_LF && c->flux != HYDRO_FLUX_MUSTA) return fail("bad flux");
  if (c->flux == HYDRO_FLUX_MUSTA) {
    if (c->musta_k < 1 || c->musta_k > 8) return fail("musta_k must be in [1, 8]");
    if (c->weno != HYDRO_WENO_Z && c->weno != HYDRO_WENO5_Z) return fail("MUSTA-FORCE is built with WENO7-Z or WENO5-Z states");
    if (c->limiter != HYDRO_LIMITER_NONE) return fail("MUSTA-FORCE is built without the limiter");
  }
  if (c->deposit != HYDRO_DEP_NGP && c->deposit != HYDRO_DEP_GAUSS) return fail("bad deposit");
  if (!(c->weno_eps > 0.0) || !std::isfinite(c->weno_eps)) return fail("weno_eps must be > 0");
  // FP64 weights take products of four squared indicators (each >= eps), which
  // stay normal for eps >= 1e-30; FP32 weights square tau / b_k (b_k >= eps),
  // which stays below the FP32 maximum for tau up to 1e7 when eps >= 1e-12
  if (c->weno_eps < (c->precision == HYDRO_F32 ? 1e-12 : 1e-30))
    return fail("weno_eps too small for the weights' arithmetic (FP64 needs >= 1e-30, FP32 >= 1e-12)");
  if (c->weno_p != 2) return fail("only weno_p = 2 is built");
  if (!(c->eos_dof > 0.0) || !(c->hbarc > 0.0)) return fail("eos_dof and hbarc must be > 0");
  return true;
}

// Checks of a jet's parameters (hydro_add_jet, hydro_set_jet,
// hydro_batch_add_jet): nullptr when they are usable, else the reason.
inline const char* jet_error(const hydro_jet* jet) {
  const double n2 = jet->dir[0] * jet->dir[0] + jet->dir[1] * jet->dir[1] + jet->dir[2] * jet->dir[2];
  if (!(std::fabs(n2 - 1.0) < 1e-9)) return "jet direction must be a unit vector";
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(jet->x0[d])) return "jet origin must be finite";
  if (!(jet->E0 >= 0.0) || !std::isfinite(jet->t_start) || !std::isfinite(jet->kappa_rad) ||
      !std::isfinite(jet->kappa_coll) || !std::isfinite(jet->cr_over_cf))
    return "bad jet parameters";
  return nullptr;
}

// Template scheme argument of the face kernels: the WENO scheme, plus kPP
// with the positivity-preserving limiter, plus kMusta with MUSTA-FORCE fluxes.
inline int face_scheme(const hydro_config& c) {
  return c.weno | (c.limiter == HYDRO_LIMITER_PP ? kPP : 0) | (c.flux == HYDRO_FLUX_MUSTA ? kMusta : 0);
}

// Half-state factor of the positivity-preserving limiter: 2 dt sum_d 1/dx_d.
inline double pp_mu(const hydro_config& c) { return 2.0 * c.dt * ((1.0 / c.dx[0] + 1.0 / c.dx[1]) + 1.0 / c.dx[2]); }

inline Grid make_grid(const hydro_config* c) {
  Grid g;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = c->n[d];
    g.bc[d] = c->bc[d];
    g.dx[d] = c->dx[d];
  }
  g.nc = ncells(c);
  return g;
}

inline bool is_device_pointer(const void* p) {
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return attr.type == hipMemoryTypeDevice;
}

// Launchers (hydro_kernels.hip, hydro_adjoint.hip).
template <class R>
hipError_t launch_face_kernel(int kernel, const StageArgs<R>& a, int scheme, int seg, hipStream_t st);
template <class R>
hipError_t launch_jet(const JetArgs& a, hipStream_t st);
template <class R>
hipError_t launch_sums(const R* U, long long nc, double dV, double* part, double* sums, hipStream_t st);
template <class R>
hipError_t launch_prim_to_cons(const double* prim, R* U, long long nc, hipStream_t st);
template <class R>
hipError_t launch_primitives(const R* U, R* prim, long long nc, double g, double hc, unsigned long long* fixups,
                             hipStream_t st);
template <class R>
hipError_t launch_adj_axis(int AX, const AdjArgs<R>& a, int scheme, hipStream_t st);
template <class R>
hipError_t launch_jet_adj(const JetAdjArgs& a, hipStream_t st);
template <class R>
hipError_t launch_copy(const R* src, R* dst, long long n, hipStream_t st);
hipError_t launch_copy_f64(const double* src, double* dst, int n, hipStream_t st);
template <class R>
hipError_t launch_fill(R* dst, long long n, R v, hipStream_t st);
template <class R>
hipError_t launch_eps2(const R* U, const Grid& g, double* part, double* out3, hipStream_t st);
template <class R>
hipError_t launch_eps2_seed(const R* U, const Grid& g, const double* out3, R* lam, double scale, hipStream_t st);
template <class R>
hipError_t launch_prim_vjp(const double* prim, const R* lam, double* out, long long nc, hipStream_t st);
template <class R>
hipError_t launch_batch_axis(int AX, const BatchArgs<R>& b, int scheme, long long blocks, hipStream_t st);
template <class R>
hipError_t launch_batch_jet(const BatchArgs<R>& b, hipStream_t st);
template <class R>
hipError_t launch_batch_sums(const BatchArgs<R>& b, long long* step, hipStream_t st);
long long batch_items(int AX, const Grid& g, int xtb, int elem);
template <class R>
hipError_t launch_freezeout(const FreezeArgs<R>& a, double* spectra, double* harm, int n_harm, hipStream_t st);

}  // namespace hydro
