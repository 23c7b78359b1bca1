// hydro_oracle.cpp -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
//
// A plain, slow CPU implementation in FP64 of one SSP-RK3 step of the ideal
// relativistic hydrodynamics with a jet source that the paper describes:
//   * Eq. (1): d_mu T^{mu nu} = S^nu for T^{mu nu} = (e+p) u^mu u^nu - p g^{mu nu},
//     plus the charge current d_mu (n u^mu) = 0 (the paper lists the charge
//     density among the conserved variables; section "Simulation setup").
//   * Eq. (2): a point source S^nu = sum_i (-dE/dt, -dM/dt) delta^3(x - x_i(t)).
//   * Eq. (3): -dE/dx = kappa_rad (C_R/C_F) T^3 x + kappa_coll (C_R/C_F) T^2.
//   * 7th-order WENO in space and third-order Runge-Kutta in time
//     (section "Simulation setup"), EOS p = e/3 (Fig. 3 caption).
// Where the paper is silent the readings used are the ones listed in the
// design notes of this repository (units with hbar*c, WENO-Z weights,
// Lax-Friedrichs splitting with alpha = 1, Shu-Osher SSP-RK3, NGP or Gaussian
// deposition, outflow = zero-gradient ghost cells, ...).
//
// Only tests/, __graft_entry__.smoke() and the cpu_baseline leg of bench.py
// may load this file's library.  It shares no code, header, table or helper
// with the HIP library: the two are independent implementations.
//
// Everything is written in the order the method defines it: explicit ghost
// cells, conserved->primitive recovery on every cell, per-axis face fluxes,
// flux divergence, source, RK combine.  No tiling, no fusion.  The scalar type
// is a template parameter so that the same code runs in double and in
// std::complex<double> (complex-step derivatives).  All branches look at real
// parts only, so the complex run is the analytic continuation of the real one.
//
// Build: g++ -O2 -std=c++17 -fopenmp -ffp-contract=off -fPIC -shared
//        (oracle/build_oracle.py does this).

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cplx = std::complex<double>;

inline double re(double x) { return x; }
inline double re(const cplx& z) { return z.real(); }

// |x| continued analytically: x * sign(Re x).
inline double aabs(double x) { return std::fabs(x); }
inline cplx aabs(const cplx& z) { return z.real() < 0.0 ? -z : z; }

inline double csqrt(double x) { return std::sqrt(x); }
inline cplx csqrt(const cplx& z) { return std::sqrt(z); }
inline double cexp(double x) { return std::exp(x); }
inline cplx cexp(const cplx& z) { return std::exp(z); }
inline double cquarter(double x) { return std::pow(x, 0.25); }
inline cplx cquarter(const cplx& z) { return std::pow(z, 0.25); }

// A double that counts its arithmetic (adds and subtracts, multiplies,
// divides, square roots; negation and |x| are free), for counting the work of
// the plain formulation.  Counters are per thread.
struct Counted {
  double v;
  Counted() : v(0.0) {}
  Counted(double x) : v(x) {}  // NOLINT: implicit, so that literals mix in
};
thread_local long long g_flops[4];  // add, mul, div, sqrt
inline Counted operator+(Counted a, Counted b) { ++g_flops[0]; return Counted(a.v + b.v); }
inline Counted operator-(Counted a, Counted b) { ++g_flops[0]; return Counted(a.v - b.v); }
inline Counted operator*(Counted a, Counted b) { ++g_flops[1]; return Counted(a.v * b.v); }
inline Counted operator/(Counted a, Counted b) { ++g_flops[2]; return Counted(a.v / b.v); }
inline Counted operator-(Counted a) { return Counted(-a.v); }
inline double re(const Counted& x) { return x.v; }
inline Counted aabs(const Counted& x) { return Counted(std::fabs(x.v)); }
inline Counted csqrt(const Counted& x) { ++g_flops[3]; return Counted(std::sqrt(x.v)); }

}  // namespace

extern "C" {

// Problem description (the oracle's own struct; it is laid out independently
// of the library's configuration struct).
typedef struct {
  int32_t n[3];       // cells along x, y, z
  double dx[3];       // cell widths [fm]
  double t0, dt;      // start time and step [fm/c]
  int32_t bc[3];      // 0 = outflow (zero-gradient), 1 = periodic
  int32_t weno;       // 0 = WENO-Z, 1 = Jiang-Shu, 2 = linear weights
  int32_t deposit;    // 0 = nearest grid point, 1 = Gaussian (sigma = dx, +-3 cells)
  int32_t weno_p;     // exponent p of the WENO-Z weights (2)
  double weno_eps;    // epsilon of the weights (1e-6)
  double eos_dof;     // g in e = g pi^2/30 T^4 / (hbar c)^3   (47.5)
  double hbarc;       // hbar c [GeV fm]                           (0.1973269804)
  int32_t limiter;    // 0 = none, 1 = positivity-preserving flux limiter
  int32_t flux;       // 0 = WENO of the Lax-Friedrichs split fluxes, 1 = MUSTA-FORCE
  int32_t musta_k;    // MUSTA stages (flux = 1), >= 1
} ocfg;

typedef struct {
  double x0[3];        // position at t_start [fm]
  double dir[3];       // unit direction (the jet moves at c)
  double E0;           // initial energy [GeV]
  double t_start;      // creation time [fm/c]
  double kappa_rad;    // Eq. (3)
  double kappa_coll;   // Eq. (3)
  double cr_over_cf;   // C_R / C_F
} ojet;

}  // extern "C"

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEFloor = 1e-12;       // E below this: vacuum fix-up
constexpr double kVCap = 1.0 - 1e-10;   // |v| cap of the fix-up

template <class S>
struct Jet {
  S x0[3];
  double dir[3];
  double t_start;
  S krad, kcoll;
  double crcf;
};

struct Grid {
  int n[3];
  int p[3];  // padded extents (n + 8)
  size_t ncell() const { return (size_t)n[0] * n[1] * n[2]; }
  size_t npad() const { return (size_t)p[0] * p[1] * p[2]; }
  size_t at(int i, int j, int k) const { return ((size_t)k * n[1] + j) * n[0] + i; }
  size_t atp(int I, int J, int K) const { return ((size_t)K * p[1] + J) * p[0] + I; }
};

Grid make_grid(const ocfg& c) {
  Grid g;
  for (int d = 0; d < 3; ++d) {
    g.n[d] = c.n[d];
    g.p[d] = c.n[d] + 8;
  }
  return g;
}

// Ghost index map: padded index I in [0, n+8) -> interior index.
int map_index(int I, int n, int bc) {
  int i = I - 4;
  if (bc == 1) return ((i % n) + n) % n;
  return std::min(std::max(i, 0), n - 1);
}

// ---------------------------------------------------------------------------
// Conserved -> primitive for p = e/3 (closed form).  With W = E + p the
// definitions E = (e+p) gamma^2 - p, M = (e+p) gamma^2 v give
// 3 W^2 - 4 E W + M^2 = 0, hence e = -E + sqrt(4E^2 - 3M^2), written here in
// the cancellation-free form 3(E^2 - M^2)/(E + sqrt(4E^2 - 3M^2)).
// Non-admissible states are fixed up for the primitive calculation only.
template <class S>
struct Prim {
  S e, v[3], n;
};

template <class S>
Prim<S> cons_to_prim(S E, S Mx, S My, S Mz, S N, long long* fixups) {
  Prim<S> r;
  if (re(E) <= kEFloor) {
    ++*fixups;
    r.e = S(kEFloor);
    r.v[0] = r.v[1] = r.v[2] = S(0.0);
    r.n = N;
    return r;
  }
  S M2 = Mx * Mx + My * My + Mz * Mz;
  if (re(M2) >= kVCap * kVCap * re(E) * re(E)) {
    ++*fixups;
    S scale = kVCap * E / csqrt(M2);
    Mx = Mx * scale;
    My = My * scale;
    Mz = Mz * scale;
    M2 = Mx * Mx + My * My + Mz * Mz;
  }
  S e = 3.0 * (E * E - M2) / (E + csqrt(4.0 * E * E - 3.0 * M2));
  S p = e / 3.0;
  S W = E + p;
  r.e = e;
  r.v[0] = Mx / W;
  r.v[1] = My / W;
  r.v[2] = Mz / W;
  S v2 = r.v[0] * r.v[0] + r.v[1] * r.v[1] + r.v[2] * r.v[2];
  r.n = N * csqrt(1.0 - v2);
  return r;
}

// Temperature from e = g pi^2 / 30 * T^4 / (hbar c)^3, T in GeV.
template <class S>
S temperature(const S& e, const ocfg& c) {
  return cquarter(30.0 * e * (c.hbarc * c.hbarc * c.hbarc) / (c.eos_dof * kPi * kPi));
}

// ---------------------------------------------------------------------------
// WENO7 reconstruction of the value at x_{i+1/2} from the left, given
// a[0..6] = a_{i-3}..a_{i+3} (point values treated as cell averages).
// Candidate values q_k on the four 4-point stencils, ideal weights
// (1, 12, 18, 4)/35, smoothness indicators from the Jiang-Shu integral
// definition, and WENO-Z (tau = |b0 + 3b1 - 3b2 - b3|), Jiang-Shu or linear
// weights.
template <class S>
S weno7_left(const S* a, int scheme, double eps, int pz) {
  const S& m3 = a[0];
  const S& m2 = a[1];
  const S& m1 = a[2];
  const S& z0 = a[3];
  const S& p1 = a[4];
  const S& p2 = a[5];
  const S& p3 = a[6];

  S q[4];
  q[0] = (-3.0 * m3 + 13.0 * m2 - 23.0 * m1 + 25.0 * z0) / 12.0;
  q[1] = (1.0 * m2 - 5.0 * m1 + 13.0 * z0 + 3.0 * p1) / 12.0;
  q[2] = (-1.0 * m1 + 7.0 * z0 + 7.0 * p1 - 1.0 * p2) / 12.0;
  q[3] = (3.0 * z0 + 13.0 * p1 - 5.0 * p2 + 1.0 * p3) / 12.0;

  const double d[4] = {1.0 / 35.0, 12.0 / 35.0, 18.0 / 35.0, 4.0 / 35.0};

  if (scheme == 2) {
    return d[0] * q[0] + d[1] * q[1] + d[2] * q[2] + d[3] * q[3];
  }

  // Smoothness indicators, Jiang-Shu definition: beta_k = sum_{l=1..3}
  // int_{cell i} (d^l p_k / dx^l)^2 dx (unit cell width), p_k the cubic whose
  // cell averages are the four stencil values.  With p_k = c0 + c1 x + c2 x^2
  // + c3 x^3 about the centre of cell i the integral is
  //   (c1 + c3/4)^2 + 13/3 c2^2 + 781/20 c3^2,
  // and c1..c3 follow from the differences D1, D2, D3 of the stencil values:
  //   c3 = D3/6,  c2 = D2/2 + g_k D3,  c1 = D1 + h_k D2 + m_k D3.
  // Written with differences, beta vanishes exactly on flat stencils.
  const double gk[4] = {1.0, 0.5, 0.0, -0.5};
  const double hk[4] = {2.5, 1.5, 0.5, -0.5};
  const double mk[4] = {43.0 / 24.0, 7.0 / 24.0, -5.0 / 24.0, 7.0 / 24.0};
  S b[4];
  for (int k = 0; k < 4; ++k) {
    const S* f = a + k;  // a_{i-3+k} .. a_{i+k}
    S d1a = f[1] - f[0], d1b = f[2] - f[1], d1c = f[3] - f[2];
    S d2a = d1b - d1a, d2b = d1c - d1b;
    S D1 = d1a, D2 = d2a, D3 = d2b - d2a;
    S c3 = D3 / 6.0;
    S c2 = D2 / 2.0 + gk[k] * D3;
    S c1 = D1 + hk[k] * D2 + mk[k] * D3;
    S t = c1 + c3 / 4.0;
    b[k] = t * t + (13.0 / 3.0) * c2 * c2 + (781.0 / 20.0) * c3 * c3;
  }

  S alpha[4];
  if (scheme == 1) {
    for (int k = 0; k < 4; ++k) alpha[k] = d[k] / ((eps + b[k]) * (eps + b[k]));
  } else {
    S tau = aabs(b[0] + 3.0 * b[1] - 3.0 * b[2] - b[3]);
    for (int k = 0; k < 4; ++k) {
      S r = tau / (b[k] + eps);
      S rp = S(1.0);
      for (int m = 0; m < pz; ++m) rp = rp * r;
      alpha[k] = d[k] * (1.0 + rp);
    }
  }
  S sum = alpha[0] + alpha[1] + alpha[2] + alpha[3];
  S out = S(0.0);
  for (int k = 0; k < 4; ++k) out = out + (alpha[k] / sum) * q[k];
  return out;
}

// ---------------------------------------------------------------------------
// WENO5 reconstruction of the value at x_{i+1/2} from the left, given
// a[0..4] = a_{i-2}..a_{i+2}: candidate values q_k of the three quadratics
// with the stencil values as cell averages, ideal weights (1, 6, 3)/10,
// Jiang-Shu smoothness indicators beta_k = sum_{l=1,2} int_{cell i}
// (d^l p_k/dx^l)^2 dx, and WENO-Z (tau = |b0 - b2|), Jiang-Shu or linear
// weights, with the same eps and exponent conventions as weno7_left.
template <class S>
S weno5_left(const S* a, int scheme, double eps, int pz) {
  S q[3];
  q[0] = (2.0 * a[0] - 7.0 * a[1] + 11.0 * a[2]) / 6.0;
  q[1] = (-1.0 * a[1] + 5.0 * a[2] + 2.0 * a[3]) / 6.0;
  q[2] = (2.0 * a[2] + 5.0 * a[3] - 1.0 * a[4]) / 6.0;
  const double d[3] = {0.1, 0.6, 0.3};
  if (scheme == 2) return d[0] * q[0] + d[1] * q[1] + d[2] * q[2];
  // With p_k = c0 + c1 x + c2 x^2 about the centre of cell i the integral is
  // c1^2 + 13/3 c2^2; from the stencil differences D1, D2:
  //   c2 = D2/2,  c1 = D1 + h_k D2,  h = 3/2, 1/2, -1/2.
  const double hk[3] = {1.5, 0.5, -0.5};
  S b[3];
  for (int k = 0; k < 3; ++k) {
    const S* f = a + k;  // a_{i-2+k} .. a_{i+k}
    S D1 = f[1] - f[0];
    S D2 = (f[2] - f[1]) - D1;
    S c2 = D2 / 2.0;
    S c1 = D1 + hk[k] * D2;
    b[k] = c1 * c1 + (13.0 / 3.0) * c2 * c2;
  }
  S alpha[3];
  if (scheme == 1) {
    for (int k = 0; k < 3; ++k) alpha[k] = d[k] / ((eps + b[k]) * (eps + b[k]));
  } else {
    S tau = aabs(b[0] - b[2]);
    for (int k = 0; k < 3; ++k) {
      S r = tau / (b[k] + eps);
      S rp = S(1.0);
      for (int m = 0; m < pz; ++m) rp = rp * r;
      alpha[k] = d[k] * (1.0 + rp);
    }
  }
  S sum = alpha[0] + alpha[1] + alpha[2];
  S out = S(0.0);
  for (int k = 0; k < 3; ++k) out = out + (alpha[k] / sum) * q[k];
  return out;
}

// ---------------------------------------------------------------------------
// Cell-centre coordinate of index i along an axis with n cells.
inline double centre(int i, int n, double dx) { return (i - 0.5 * (n - 1)) * dx; }

// Nearest-grid-point cell along one axis; -1 when outside the box.
// u = (x - x_lo)/dx + 1e-9 with x_lo = -n dx / 2; ties go to the upper cell.
int ngp_index(double x, int n, double dx) {
  double x_lo = -0.5 * n * dx;
  double u = (x - x_lo) / dx + 1e-9;
  double f = std::floor(u);
  if (f < 0.0 || f >= (double)n) return -1;
  return (int)f;
}

// ---------------------------------------------------------------------------
template <class S>
struct Solver {
  ocfg c;
  Grid g;
  std::vector<Jet<S>> jets;
  long long fixups = 0;

  // scratch
  std::vector<S> Wp;               // padded conserved [5][npad]
  std::vector<S> pe, pv0, pv1, pv2;  // padded primitives e, v
  std::vector<S> face;             // face fluxes of one line

  explicit Solver(const ocfg& cfg) : c(cfg), g(make_grid(cfg)) {
    Wp.resize(5 * g.npad());
    pe.resize(g.npad());
    pv0.resize(g.npad());
    pv1.resize(g.npad());
    pv2.resize(g.npad());
  }

  // RHS L(W) = D(W) + S(W) at time t.  chi[j] = 1 if jet j still has energy.
  // P_eff[j] receives the energy-loss rate actually deposited [GeV/fm].
  void rhs(const S* W, double t, const int* chi, S* L, S* P_eff) {
    const size_t nc = g.ncell();
    const size_t np = g.npad();
    // 1. ghost cells (each padded cell copies its mapped interior cell)
    for (int K = 0; K < g.p[2]; ++K) {
      int k = map_index(K, g.n[2], c.bc[2]);
      for (int J = 0; J < g.p[1]; ++J) {
        int j = map_index(J, g.n[1], c.bc[1]);
        for (int I = 0; I < g.p[0]; ++I) {
          int i = map_index(I, g.n[0], c.bc[0]);
          for (int f = 0; f < 5; ++f) Wp[f * np + g.atp(I, J, K)] = W[f * nc + g.at(i, j, k)];
        }
      }
    }
    // 2. conserved -> primitive on every padded cell
    long long fx = 0;
#pragma omp parallel for reduction(+ : fx) schedule(static)
    for (long long q = 0; q < (long long)np; ++q) {
      Prim<S> pr = cons_to_prim(Wp[0 * np + q], Wp[1 * np + q], Wp[2 * np + q], Wp[3 * np + q],
                                Wp[4 * np + q], &fx);
      pe[q] = pr.e;
      pv0[q] = pr.v[0];
      pv1[q] = pr.v[1];
      pv2[q] = pr.v[2];
    }
    fixups += fx;

    for (size_t q = 0; q < 5 * nc; ++q) L[q] = S(0.0);

    // 3.-5. per-axis face fluxes and flux divergence
    for (int d = 0; d < 3; ++d) axis_divergence(d, L);

    // 6. jet source
    source(W, t, chi, L, P_eff);
  }

  // Physical flux f_d of component comp at padded cell q.
  S flux(int d, int comp, size_t q) const {
    const size_t np = g.npad();
    const S* v[3] = {&pv0[q], &pv1[q], &pv2[q]};
    S vd = *v[d];
    S p = pe[q] / 3.0;
    switch (comp) {
      case 0: return Wp[(1 + d) * np + q];                            // T^{0d} = M_d
      case 1: return Wp[1 * np + q] * vd + (d == 0 ? p : S(0.0));     // T^{xd}
      case 2: return Wp[2 * np + q] * vd + (d == 1 ? p : S(0.0));     // T^{yd}
      case 3: return Wp[3 * np + q] * vd + (d == 2 ? p : S(0.0));     // T^{zd}
      default: return Wp[4 * np + q] * vd;                            // N v_d
    }
  }

  void axis_divergence(int d, S* L) {
    const size_t nc = g.ncell();
    const size_t np = g.npad();
    const int n = g.n[d];
    const double dx = c.dx[d];
    const int e1 = (d + 1) % 3, e2 = (d + 2) % 3;  // the two other axes
    const int n1 = g.n[e1], n2 = g.n[e2];
#pragma omp parallel for collapse(2) schedule(static)
    for (int b = 0; b < n2; ++b) {
      for (int a = 0; a < n1; ++a) {
        std::vector<S> Fp(n + 8), Fm(n + 8), Fh(5 * (n + 1));
        long long line_fx = 0;
        auto padded = [&](int P) {
          int idx[3];
          idx[d] = P;
          idx[e1] = a + 4;
          idx[e2] = b + 4;
          return g.atp(idx[0], idx[1], idx[2]);
        };
        if (c.flux == 1) {
          musta_faces(d, padded, n, Fh.data(), &line_fx);
        }
        for (int comp = 0; comp < 5 && c.flux == 0; ++comp) {
          // split fluxes along the line, padded index P in [0, n+8)
          for (int P = 0; P < n + 8; ++P) {
            size_t q = padded(P);
            S f = flux(d, comp, q);
            S u = Wp[comp * np + q];
            Fp[P] = 0.5 * (f + u);  // Lax-Friedrichs splitting, alpha = 1
            Fm[P] = 0.5 * (f - u);
          }
          // faces i+1/2 for i = -1..n-1 (Fh[comp][i+1])
          S* Fc = &Fh[comp * (n + 1)];
          for (int i = -1; i < n; ++i) {
            int P = i + 4;  // padded index of cell i
            if (c.weno >= 3) {  // 5th order: three ghost cells are used
              S left[5], right[5];
              for (int m = 0; m < 5; ++m) {
                left[m] = Fp[P - 2 + m];    // F+ at i-2..i+2
                right[m] = Fm[P + 3 - m];   // F- at i+3..i-1 (mirrored stencil)
              }
              Fc[i + 1] = weno5_left(left, c.weno - 3, c.weno_eps, c.weno_p) +
                          weno5_left(right, c.weno - 3, c.weno_eps, c.weno_p);
              continue;
            }
            S left[7], right[7];
            for (int m = 0; m < 7; ++m) {
              left[m] = Fp[P - 3 + m];    // F+ at i-3..i+3
              right[m] = Fm[P + 4 - m];   // F- at i+4..i-2 (mirrored stencil)
            }
            Fc[i + 1] = weno7_left(left, c.weno, c.weno_eps, c.weno_p) +
                        weno7_left(right, c.weno, c.weno_eps, c.weno_p);
          }
        }
        if (c.limiter == 1) {
          for (int i = -1; i < n; ++i) {
            size_t qa = padded(i + 4), qb = padded(i + 5);
            S uA[5], fA[5], uB[5], fB[5], H[5];
            for (int comp = 0; comp < 5; ++comp) {
              uA[comp] = Wp[comp * np + qa];
              fA[comp] = flux(d, comp, qa);
              uB[comp] = Wp[comp * np + qb];
              fB[comp] = flux(d, comp, qb);
              H[comp] = Fh[comp * (n + 1) + i + 1];
            }
            limit_face(uA, fA, uB, fB, H);
            for (int comp = 0; comp < 5; ++comp) Fh[comp * (n + 1) + i + 1] = H[comp];
          }
        }
        if (line_fx) {
#pragma omp atomic
          fixups += line_fx;
        }
        for (int comp = 0; comp < 5; ++comp) {
          const S* Fc = &Fh[comp * (n + 1)];
          for (int i = 0; i < n; ++i) {
            int idx[3];
            idx[d] = i;
            idx[e1] = a;
            idx[e2] = b;
            size_t cell = g.at(idx[0], idx[1], idx[2]);
            L[comp * nc + cell] = L[comp * nc + cell] + (-(Fc[i + 1] - Fc[i]) / dx);
          }
        }
      }
    }
  }

  // Physical flux along d of an arbitrary conserved state (recovered with the
  // same fix-ups as the grid cells; fixed-up recoveries are counted in *fx).
  static void state_flux(int d, const S u[5], S f[5], long long* fx) {
    Prim<S> p = cons_to_prim(u[0], u[1], u[2], u[3], u[4], fx);
    S pr = p.e / 3.0;
    f[0] = u[1 + d];
    for (int m = 0; m < 3; ++m) f[1 + m] = u[1 + m] * p.v[d] + (m == d ? pr : S(0.0));
    f[4] = u[4] * p.v[d];
  }

  // MUSTA-FORCE flux (Toro's multi-stage centred flux) of the states uL, uR
  // at one face, on a local two-cell mesh with dt_loc/dx_loc = C/S_max,
  // C = 0.9, S_max = 1 (the speed of light).  Each stage forms the FORCE
  // flux, the mean of the Lax-Friedrichs flux
  //   (f(uL) + f(uR))/2 - (uR - uL)/(2 lam)
  // and the flux of the Richtmyer state (uL + uR)/2 - lam (f(uR) - f(uL))/2;
  // the last stage's FORCE flux is the result, the stages before it advance
  // the local states: uL -= lam (F - f(uL)), uR -= lam (f(uR) - F).
  static constexpr double kMustaCfl = 0.9;

  static void musta_force(int d, S uL[5], S uR[5], int k, S F[5], long long* fx) {
    const double lam = kMustaCfl;
    for (int l = 1; l <= k; ++l) {
      S fL[5], fR[5], uM[5], fM[5];
      state_flux(d, uL, fL, fx);
      state_flux(d, uR, fR, fx);
      for (int m = 0; m < 5; ++m) uM[m] = 0.5 * (uL[m] + uR[m]) - 0.5 * lam * (fR[m] - fL[m]);
      state_flux(d, uM, fM, fx);
      for (int m = 0; m < 5; ++m) {
        S flf = 0.5 * (fL[m] + fR[m]) - (0.5 / lam) * (uR[m] - uL[m]);
        F[m] = 0.5 * (flf + fM[m]);
      }
      if (l == k) return;
      for (int m = 0; m < 5; ++m) {
        uL[m] = uL[m] - lam * (F[m] - fL[m]);
        uR[m] = uR[m] - lam * (fR[m] - F[m]);
      }
    }
  }

  // Faces of one line with the MUSTA-FORCE flux of the left and right states
  // reconstructed component-wise from the conserved point values by the
  // configured WENO scheme (the left state from cells i-3..i+3, the right
  // one from the mirrored stencil i+4..i-2; WENO5: i-2..i+2 and i+3..i-1).
  template <class Padded>
  void musta_faces(int d, Padded padded, int n, S* Fh, long long* fx) const {
    const size_t np = g.npad();
    for (int i = -1; i < n; ++i) {
      int P = i + 4;
      S uL[5], uR[5], F[5];
      for (int comp = 0; comp < 5; ++comp) {
        if (c.weno >= 3) {
          S left[5], right[5];
          for (int m = 0; m < 5; ++m) {
            left[m] = Wp[comp * np + padded(P - 2 + m)];
            right[m] = Wp[comp * np + padded(P + 3 - m)];
          }
          uL[comp] = weno5_left(left, c.weno - 3, c.weno_eps, c.weno_p);
          uR[comp] = weno5_left(right, c.weno - 3, c.weno_eps, c.weno_p);
        } else {
          S left[7], right[7];
          for (int m = 0; m < 7; ++m) {
            left[m] = Wp[comp * np + padded(P - 3 + m)];
            right[m] = Wp[comp * np + padded(P + 4 - m)];
          }
          uL[comp] = weno7_left(left, c.weno, c.weno_eps, c.weno_p);
          uR[comp] = weno7_left(right, c.weno, c.weno_eps, c.weno_p);
        }
      }
      musta_force(d, uL, uR, c.musta_k, F, fx);
      for (int comp = 0; comp < 5; ++comp) Fh[comp * (n + 1) + i + 1] = F[comp];
    }
  }

  // Positivity-preserving flux limiter (after Zhang and Shu, the WENO
  // reference of the paper).  A forward-Euler update of a cell,
  //   u_i - sum_d lam_d (F_{d,i+1/2} - F_{d,i-1/2}),   lam_d = dt/dx_d,
  // equals sum_d w_d (R_d + L_d)/2 with w_d = lam_d / sum lam and the two
  // half states
  //   R_d = u_i - mu (F_{d,i+1/2} - f_d(u_i)/2),  L_d = u_i + mu (F_{d,i-1/2} - f_d(u_i)/2),
  // mu = 2 dt sum_d 1/dx_d.  With the first-order Lax-Friedrichs flux
  // F = (f(u_i) + u_i)/2 + (f(u_{i+1}) - u_{i+1})/2 they are
  //   R = (1 - mu/2) u_i + mu/2 (u_{i+1} - f(u_{i+1})),
  //   L = (1 - mu/2) u_i + mu/2 (u_{i-1} + f(u_{i-1})),
  // admissible for mu/2 <= 1 because u +- f(u) is (alpha = 1).  The face flux
  // becomes theta F_high + (1 - theta) F_LF with the largest theta of the
  // chord rule below that keeps both half states next to the face in
  //   { E - |M| >= eps, N >= eps }  (convex: the first function is concave).
  // The source adds (P, P dir) with |dir| = 1 and the RK3 stages are convex
  // combinations, so whole steps stay in the set.
  static constexpr double kPPEps = 1e-13;

  // Largest theta in [0, 1] with h(theta) >= 0 given h concave on [0, 1]:
  // 1 if h(1) >= 0, 0 if h(0) <= 0, else the chord's root h(0)/(h(0) - h(1))
  // (concavity puts h above the chord).
  static S chord_theta(const S& h0, const S& h1) {
    if (re(h1) >= 0.0) return S(1.0);
    if (re(h0) <= 0.0) return S(0.0);
    return h0 / (h0 - h1);
  }

  // theta for one half state s(theta) = s0 + theta (s1 - s0).
  static S side_theta(const S s0[5], const S s1[5]) {
    S m0 = csqrt(s0[1] * s0[1] + s0[2] * s0[2] + s0[3] * s0[3]);
    S m1 = csqrt(s1[1] * s1[1] + s1[2] * s1[2] + s1[3] * s1[3]);
    S tq = chord_theta(s0[0] - m0 - kPPEps, s1[0] - m1 - kPPEps);
    S tn = chord_theta(s0[4] - kPPEps, s1[4] - kPPEps);
    return re(tn) < re(tq) ? tn : tq;
  }

  void limit_face(const S uA[5], const S fA[5], const S uB[5], const S fB[5], S H[5]) const {
    const double mu = 2.0 * c.dt * (1.0 / c.dx[0] + 1.0 / c.dx[1] + 1.0 / c.dx[2]);
    limit_face_mu(mu, uA, fA, uB, fB, H);
  }

  // Returns theta; H becomes theta H + (1 - theta) F_LF.
  static S limit_face_mu(double mu, const S uA[5], const S fA[5], const S uB[5], const S fB[5], S H[5]) {
    S FL[5], RA0[5], RA1[5], LB0[5], LB1[5];
    for (int comp = 0; comp < 5; ++comp) {
      FL[comp] = 0.5 * (fA[comp] + uA[comp]) + 0.5 * (fB[comp] - uB[comp]);
      RA0[comp] = uA[comp] - mu * (FL[comp] - 0.5 * fA[comp]);
      RA1[comp] = uA[comp] - mu * (H[comp] - 0.5 * fA[comp]);
      LB0[comp] = uB[comp] + mu * (FL[comp] - 0.5 * fB[comp]);
      LB1[comp] = uB[comp] + mu * (H[comp] - 0.5 * fB[comp]);
    }
    S ta = side_theta(RA0, RA1);
    S tb = side_theta(LB0, LB1);
    S th = re(tb) < re(ta) ? tb : ta;
    for (int comp = 0; comp < 5; ++comp) H[comp] = th * H[comp] + (1.0 - th) * FL[comp];
    return th;
  }

  S cell_temperature(int i, int j, int k) const {
    size_t q = g.atp(i + 4, j + 4, k + 4);
    return temperature(pe[q], c);
  }

  // Energy-loss rate, Eq. (3), in GeV/fm for path length ell [fm].
  S eloss(const Jet<S>& jt, const S& T, double ell) const {
    const double hc = c.hbarc;
    return jt.kcoll * jt.crcf * T * T / hc + jt.krad * jt.crcf * T * T * T * ell / (hc * hc);
  }

  void source(const S* W, double t, const int* chi, S* L, S* P_eff) {
    (void)W;
    const size_t nc = g.ncell();
    const double dV = c.dx[0] * c.dx[1] * c.dx[2];
    for (size_t j = 0; j < jets.size(); ++j) {
      P_eff[j] = S(0.0);
      const Jet<S>& jt = jets[j];
      if (!chi[j]) continue;
      double ell = t - jt.t_start;
      if (ell < 0.0) continue;  // not created yet
      S x[3];
      for (int d = 0; d < 3; ++d) x[d] = jt.x0[d] + jt.dir[d] * ell;
      int ctr[3];
      bool inside = true;
      for (int d = 0; d < 3; ++d) {
        ctr[d] = ngp_index(re(x[d]), g.n[d], c.dx[d]);
        if (ctr[d] < 0) inside = false;
      }
      if (!inside) continue;
      if (c.deposit == 0) {
        S T = cell_temperature(ctr[0], ctr[1], ctr[2]);
        S P = eloss(jt, T, ell);
        S s0 = P / dV;
        size_t cell = g.at(ctr[0], ctr[1], ctr[2]);
        L[0 * nc + cell] = L[0 * nc + cell] + s0;
        for (int d = 0; d < 3; ++d) L[(1 + d) * nc + cell] = L[(1 + d) * nc + cell] + jt.dir[d] * s0;
        P_eff[j] = P;
      } else {
        // separable Gaussian weights, sigma = dx, over the 7 cells around the
        // nearest cell, each 1-D vector normalised to unit sum
        S w[3][7];
        for (int d = 0; d < 3; ++d) {
          S sum = S(0.0);
          for (int m = 0; m < 7; ++m) {
            int idx = ctr[d] - 3 + m;
            S del = centre(idx, g.n[d], c.dx[d]) - x[d];
            w[d][m] = cexp(-(del * del) / (2.0 * c.dx[d] * c.dx[d]));
            sum = sum + w[d][m];
          }
          for (int m = 0; m < 7; ++m) w[d][m] = w[d][m] / sum;
        }
        S wsum = S(0.0), Tsum = S(0.0);
        for (int mk = 0; mk < 7; ++mk)
          for (int mj = 0; mj < 7; ++mj)
            for (int mi = 0; mi < 7; ++mi) {
              int i = ctr[0] - 3 + mi, jj = ctr[1] - 3 + mj, k = ctr[2] - 3 + mk;
              if (i < 0 || i >= g.n[0] || jj < 0 || jj >= g.n[1] || k < 0 || k >= g.n[2]) continue;
              S ww = w[0][mi] * w[1][mj] * w[2][mk];
              wsum = wsum + ww;
              Tsum = Tsum + ww * cell_temperature(i, jj, k);
            }
        S T = Tsum / wsum;
        S P = eloss(jt, T, ell);
        for (int mk = 0; mk < 7; ++mk)
          for (int mj = 0; mj < 7; ++mj)
            for (int mi = 0; mi < 7; ++mi) {
              int i = ctr[0] - 3 + mi, jj = ctr[1] - 3 + mj, k = ctr[2] - 3 + mk;
              if (i < 0 || i >= g.n[0] || jj < 0 || jj >= g.n[1] || k < 0 || k >= g.n[2]) continue;
              S ww = w[0][mi] * w[1][mj] * w[2][mk];
              S s0 = P * ww / dV;
              size_t cell = g.at(i, jj, k);
              L[0 * nc + cell] = L[0 * nc + cell] + s0;
              for (int d = 0; d < 3; ++d)
                L[(1 + d) * nc + cell] = L[(1 + d) * nc + cell] + jt.dir[d] * s0;
            }
        P_eff[j] = P * wsum;
      }
    }
  }

  // One Shu-Osher SSP-RK3 step:
  //   U1 = Un + dt L(Un)                 at t_n
  //   U2 = 3/4 Un + 1/4 (U1 + dt L(U1))  at t_n + dt
  //   U  = 1/3 Un + 2/3 (U2 + dt L(U2))  at t_n + dt/2
  // E_jet and the deposited-energy ledger advance by dt * sum_k b_k P_k with
  // b = (1/6, 1/6, 2/3), the weights of the three stage evaluations.
  void step(S* U, long long step_index, S* Ejet, S* ledger) {
    const size_t m = 5 * g.ncell();
    const double dt = c.dt;
    const double tn = c.t0 + (double)step_index * dt;
    const size_t nj = jets.size();
    std::vector<int> chi(nj);
    for (size_t j = 0; j < nj; ++j) chi[j] = re(Ejet[j]) > 0.0 ? 1 : 0;
    std::vector<S> Un(U, U + m), U1(m), U2(m), L(m);
    std::vector<S> P1(nj), P2(nj), P3(nj);

    rhs(Un.data(), tn + 0.0 * dt, chi.data(), L.data(), P1.data());
    for (size_t q = 0; q < m; ++q) U1[q] = Un[q] + dt * L[q];

    rhs(U1.data(), tn + 1.0 * dt, chi.data(), L.data(), P2.data());
    for (size_t q = 0; q < m; ++q) U2[q] = 0.75 * Un[q] + 0.25 * (U1[q] + dt * L[q]);

    rhs(U2.data(), tn + 0.5 * dt, chi.data(), L.data(), P3.data());
    for (size_t q = 0; q < m; ++q) U[q] = (1.0 / 3.0) * Un[q] + (2.0 / 3.0) * (U2[q] + dt * L[q]);

    for (size_t j = 0; j < nj; ++j) {
      if (!chi[j]) continue;
      S dep = dt * ((1.0 / 6.0) * P1[j] + (1.0 / 6.0) * P2[j] + (2.0 / 3.0) * P3[j]);
      *ledger = *ledger + dep;
      S rest = Ejet[j] - dep;
      Ejet[j] = re(rest) > 0.0 ? rest : S(0.0);
    }
  }
};

template <class S>
Jet<S> to_jet(const ojet& j) {
  Jet<S> r;
  for (int d = 0; d < 3; ++d) {
    r.x0[d] = S(j.x0[d]);
    r.dir[d] = j.dir[d];
  }
  r.t_start = j.t_start;
  r.krad = S(j.kappa_rad);
  r.kcoll = S(j.kappa_coll);
  r.crcf = j.cr_over_cf;
  return r;
}

// Primitive (e, vx, vy, vz, n) -> conserved (E, Mx, My, Mz, N), p = e/3.
template <class S>
void prim_to_cons(size_t nc, const S* e, const double* v0, const double* v1, const double* v2,
                  const double* n, S* U) {
  for (size_t q = 0; q < nc; ++q) {
    double v2s = v0[q] * v0[q] + v1[q] * v1[q] + v2[q] * v2[q];
    double g2 = 1.0 / (1.0 - v2s);
    S p = e[q] / 3.0;
    S w = (e[q] + p) * g2;
    U[0 * nc + q] = w - p;
    U[1 * nc + q] = w * v0[q];
    U[2 * nc + q] = w * v1[q];
    U[3 * nc + q] = w * v2[q];
    U[4 * nc + q] = S(n[q] * std::sqrt(g2));
  }
}

// Energy-weighted anisotropy on the z = 0 plane:
// eps2 = sum (y^2 - x^2) e / sum (y^2 + x^2) e, x and y from the grid origin,
// e on z = 0 as the mean of the two middle planes (even nz) or the middle plane.
template <class S>
S eps2_of(const ocfg& c, const S* U, long long* fixups) {
  Grid g = make_grid(c);
  const size_t nc = g.ncell();
  int k0, k1;
  if (g.n[2] % 2 == 0) {
    k0 = g.n[2] / 2 - 1;
    k1 = g.n[2] / 2;
  } else {
    k0 = k1 = (g.n[2] - 1) / 2;
  }
  S num = S(0.0), den = S(0.0);
  for (int j = 0; j < g.n[1]; ++j) {
    double y = centre(j, g.n[1], c.dx[1]);
    for (int i = 0; i < g.n[0]; ++i) {
      double x = centre(i, g.n[0], c.dx[0]);
      size_t a = g.at(i, j, k0), b = g.at(i, j, k1);
      Prim<S> pa = cons_to_prim(U[a], U[nc + a], U[2 * nc + a], U[3 * nc + a], U[4 * nc + a], fixups);
      Prim<S> pb = cons_to_prim(U[b], U[nc + b], U[2 * nc + b], U[3 * nc + b], U[4 * nc + b], fixups);
      S e = 0.5 * (pa.e + pb.e);
      num = num + (y * y - x * x) * e;
      den = den + (y * y + x * x) * e;
    }
  }
  return num / den;
}

// ---------------------------------------------------------------------------
// Freeze-out, the step the paper plans next (section "Results", closing
// paragraph: add freeze-out and study elliptic flow and higher harmonics).
// Cooper-Frye on the fixed-time hypersurface of the state U, d sigma_mu =
// (dV, 0, 0, 0), emitting a massless Boltzmann species of degeneracy g at
// zero chemical potential (the quanta of the p = e/3 fluid), T = T(e) of the
// fluid's equation of state.  At rapidity 0 along z (p_z = 0, p^0 = p_T) a
// particle of azimuth phi has p.u = gamma p_T (1 - vx cos phi - vy sin phi), so
//   E dN/d^3p = g / ((2 pi hbar c)^3) sum_cells dV p_T exp(-gamma p_T D / T),
//   D = 1 - vx cos phi - vy sin phi,
// and over all p_T (int_0^inf p^2 exp(-a p) dp = 2 / a^3)
//   dN/(dy dphi) = g / ((2 pi hbar c)^3) sum_cells dV 2 T^3 / (gamma D)^3.
// Units: p_T and T in GeV, dV in fm^3, hbar c in GeV fm.  Cells with T < T_min
// are left out (T_min = 0 keeps every cell).  Rows of out ([1 + n_pt][n_phi]):
// row 0 dN/(dy dphi), row 1 + j dN/(p_T dp_T dy dphi) at p_T = pt[j], each at
// phi_k = 2 pi k / n_phi.  Per z-plane partial sums, then the planes in order.
void freezeout_spectra(const ocfg& c, const double* U, int n_phi, int n_pt, const double* pt, double T_min,
                       double dof, double* out, long long* fixups) {
  Grid g = make_grid(c);
  const size_t nc = g.ncell();
  const double dV = c.dx[0] * c.dx[1] * c.dx[2];
  const double pref = dof / std::pow(2.0 * kPi * c.hbarc, 3);
  const int rows = 1 + n_pt;
  std::vector<double> cphi(n_phi), sphi(n_phi);
  for (int k = 0; k < n_phi; ++k) {
    cphi[k] = std::cos(2.0 * kPi * k / n_phi);
    sphi[k] = std::sin(2.0 * kPi * k / n_phi);
  }
  std::vector<double> plane((size_t)g.n[2] * rows * n_phi, 0.0);
  std::vector<long long> pfx(g.n[2], 0);
#pragma omp parallel for schedule(static)
  for (int kz = 0; kz < g.n[2]; ++kz) {
    double* acc = &plane[(size_t)kz * rows * n_phi];
    for (int j = 0; j < g.n[1]; ++j) {
      for (int i = 0; i < g.n[0]; ++i) {
        const size_t q = g.at(i, j, kz);
        Prim<double> p = cons_to_prim(U[q], U[nc + q], U[2 * nc + q], U[3 * nc + q], U[4 * nc + q], &pfx[kz]);
        const double T = temperature(p.e, c);
        if (T < T_min) continue;
        const double gam = 1.0 / std::sqrt(1.0 - (p.v[0] * p.v[0] + p.v[1] * p.v[1] + p.v[2] * p.v[2]));
        for (int k = 0; k < n_phi; ++k) {
          const double D = 1.0 - p.v[0] * cphi[k] - p.v[1] * sphi[k];
          const double a = gam * D;
          acc[k] += pref * dV * 2.0 * T * T * T / (a * a * a);
          for (int r = 0; r < n_pt; ++r) acc[(size_t)(1 + r) * n_phi + k] += pref * dV * pt[r] * std::exp(-pt[r] * a / T);
        }
      }
    }
  }
  for (int o = 0; o < rows * n_phi; ++o) out[o] = 0.0;
  for (int kz = 0; kz < g.n[2]; ++kz) {
    for (int o = 0; o < rows * n_phi; ++o) out[o] += plane[(size_t)kz * rows * n_phi + o];
    if (fixups) *fixups += pfx[kz];
  }
}

// Flow harmonics of an azimuthal distribution sampled at phi_k = 2 pi k/n_phi:
// out[0] = (dN/dy, 0) with dN/dy = (2 pi / n_phi) sum_k s_k (the trapezoid rule
// of a periodic function), out[n] = (sum_k cos(n phi_k) s_k, sum_k sin(n phi_k)
// s_k) / sum_k s_k for n = 1..n_harm: v_n is the modulus of that pair and
// atan2(sin, cos)/n the n-th event-plane angle.
void flow_harmonics(const double* s, int n_phi, int n_harm, double* out) {
  double tot = 0.0;
  for (int k = 0; k < n_phi; ++k) tot += s[k];
  out[0] = 2.0 * kPi / n_phi * tot;
  out[1] = 0.0;
  for (int n = 1; n <= n_harm; ++n) {
    double cs = 0.0, sn = 0.0;
    for (int k = 0; k < n_phi; ++k) {
      const double ang = 2.0 * kPi * (double)(((long long)n * k) % n_phi) / n_phi;
      cs += std::cos(ang) * s[k];
      sn += std::sin(ang) * s[k];
    }
    // a row with no particles (every cell below T_min) has no flow: 0, not 0/0
    out[2 * n] = tot != 0.0 ? cs / tot : 0.0;
    out[2 * n + 1] = tot != 0.0 ? sn / tot : 0.0;
  }
}

template <class S>
int run_impl(const ocfg* cfg, const ojet* jets, int njet, S* U, int nsteps, long long step0,
             S* Ejet, S* ledger, long long* fixups, const std::vector<Jet<S>>* cjets) {
  Solver<S> s(*cfg);
  if (cjets) {
    s.jets = *cjets;
  } else {
    for (int j = 0; j < njet; ++j) s.jets.push_back(to_jet<S>(jets[j]));
  }
  for (int st = 0; st < nsteps; ++st) s.step(U, step0 + st, Ejet, ledger);
  if (fixups) *fixups += s.fixups;
  return 0;
}

bool valid(const ocfg* c) {
  if (!c) return false;
  for (int d = 0; d < 3; ++d) {
    if (c->n[d] < 1 || c->dx[d] <= 0.0) return false;
    if (c->bc[d] != 0 && c->bc[d] != 1) return false;
  }
  if (c->weno < 0 || c->weno > 5 || c->deposit < 0 || c->deposit > 1 || c->weno_p < 1) return false;
  if (c->limiter < 0 || c->limiter > 1) return false;
  if (c->flux < 0 || c->flux > 1 || (c->flux == 1 && (c->musta_k < 1 || c->limiter != 0))) return false;
  return c->dt > 0.0;
}

}  // namespace

extern "C" {

// Number of OpenMP threads the oracle's loops use.
int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Set the OpenMP thread count of later calls (timing on one core or all).
void oracle_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

// WENO5 left-biased reconstruction of five values (unit tests).
double oracle_weno5(const double* a, int scheme, double eps, int p) {
  return weno5_left<double>(a, scheme, eps, p);
}

// WENO7 left-biased reconstruction of seven values (unit tests).
double oracle_weno7(const double* a, int scheme, double eps, int p) {
  return weno7_left<double>(a, scheme, eps, p);
}

// Primitive [e,vx,vy,vz,n] -> conserved [E,Mx,My,Mz,N], arrays [5][ncell].
int oracle_prim_to_cons(const ocfg* c, const double* prim, double* U) {
  if (!valid(c)) return -1;
  size_t nc = (size_t)c->n[0] * c->n[1] * c->n[2];
  prim_to_cons<double>(nc, prim, prim + nc, prim + 2 * nc, prim + 3 * nc, prim + 4 * nc, U);
  return 0;
}

// Conserved -> primitive [e,vx,vy,vz,n,T], arrays [6][ncell].
int oracle_cons_to_prim(const ocfg* c, const double* U, double* prim, long long* fixups) {
  if (!valid(c)) return -1;
  size_t nc = (size_t)c->n[0] * c->n[1] * c->n[2];
  long long fx = 0;
  for (size_t q = 0; q < nc; ++q) {
    Prim<double> p = cons_to_prim(U[q], U[nc + q], U[2 * nc + q], U[3 * nc + q], U[4 * nc + q], &fx);
    prim[q] = p.e;
    prim[nc + q] = p.v[0];
    prim[2 * nc + q] = p.v[1];
    prim[3 * nc + q] = p.v[2];
    prim[4 * nc + q] = p.n;
    prim[5 * nc + q] = temperature(p.e, *c);
  }
  if (fixups) *fixups = fx;
  return 0;
}

// L(U) = D(U) + S(U) at time t (one stage's right-hand side).
int oracle_rhs(const ocfg* c, const ojet* jets, int njet, const int* chi, const double* U, double t,
               double* L, double* P_eff, long long* fixups) {
  if (!valid(c) || njet < 0) return -1;
  Solver<double> s(*c);
  for (int j = 0; j < njet; ++j) s.jets.push_back(to_jet<double>(jets[j]));
  std::vector<int> ch(njet, 1);
  if (chi)
    for (int j = 0; j < njet; ++j) ch[j] = chi[j];
  std::vector<double> P(njet + 1);
  s.rhs(U, t, ch.data(), L, P.data());
  if (P_eff)
    for (int j = 0; j < njet; ++j) P_eff[j] = P[j];
  if (fixups) *fixups = s.fixups;
  return 0;
}

// nsteps SSP-RK3 steps starting at step index step0 (t_n = t0 + n dt).
// U [5][ncell] in/out; Ejet [njet] in/out; ledger in/out.
int oracle_run(const ocfg* c, const ojet* jets, int njet, double* U, int nsteps, long long step0,
               double* Ejet, double* ledger, long long* fixups) {
  if (!valid(c) || njet < 0 || nsteps < 0) return -1;
  long long fx = 0;
  run_impl<double>(c, jets, njet, U, nsteps, step0, Ejet, ledger, &fx, nullptr);
  if (fixups) *fixups = fx;
  return 0;
}

// sum_cells U_f dV for the five fields, accumulated in long double.
int oracle_sums(const ocfg* c, const double* U, double* out5) {
  if (!valid(c)) return -1;
  size_t nc = (size_t)c->n[0] * c->n[1] * c->n[2];
  double dV = c->dx[0] * c->dx[1] * c->dx[2];
  for (int f = 0; f < 5; ++f) {
    long double acc = 0.0L;
    for (size_t q = 0; q < nc; ++q) acc += (long double)U[f * nc + q];
    out5[f] = (double)(acc * (long double)dV);
  }
  return 0;
}

int oracle_eps2(const ocfg* c, const double* U, double* out) {
  if (!valid(c)) return -1;
  long long fx = 0;
  *out = eps2_of<double>(*c, U, &fx);
  return 0;
}

// Freeze-out spectra and flow harmonics of U (see freezeout_spectra and
// flow_harmonics): spectra [1 + n_pt][n_phi], harm [1 + n_pt][n_harm + 1][2].
int oracle_freezeout(const ocfg* c, const double* U, int n_phi, int n_pt, const double* pt, double T_min,
                     double dof, int n_harm, double* spectra, double* harm, long long* fixups) {
  if (!valid(c) || n_phi < 1 || n_pt < 0 || (n_pt > 0 && !pt) || n_harm < 0 || !(dof > 0.0)) return -1;
  long long fx = 0;
  freezeout_spectra(*c, U, n_phi, n_pt, pt, T_min, dof, spectra, &fx);
  for (int r = 0; r <= n_pt; ++r)
    flow_harmonics(spectra + (size_t)r * n_phi, n_phi, n_harm, harm + (size_t)r * (n_harm + 1) * 2);
  if (fixups) *fixups = fx;
  return 0;
}

// Complex-step derivative of eps2(after nsteps) with respect to one input:
//   which = 0: kappa_rad of jet `jet`, 1: kappa_coll, 2: x0, 3: y0, 4: z0,
//           5: the initial energy density along direction de[ncell].
// Returns d eps2 = Im(eps2(input + i h)) / h in *deriv and Re in *value.
int oracle_eps2_complex_step(const ocfg* c, const ojet* jets, int njet, const double* prim0,
                             int nsteps, int which, int jet, double h, const double* de,
                             double* value, double* deriv) {
  if (!valid(c) || njet < 0 || nsteps < 0 || which < 0 || which > 5) return -1;
  if (which < 5 && (jet < 0 || jet >= njet)) return -1;
  if (which == 5 && !de) return -1;
  size_t nc = (size_t)c->n[0] * c->n[1] * c->n[2];
  std::vector<cplx> e(nc);
  for (size_t q = 0; q < nc; ++q) e[q] = cplx(prim0[q], which == 5 ? h * de[q] : 0.0);
  std::vector<cplx> U(5 * nc);
  prim_to_cons<cplx>(nc, e.data(), prim0 + nc, prim0 + 2 * nc, prim0 + 3 * nc, prim0 + 4 * nc, U.data());
  std::vector<Jet<cplx>> cj;
  for (int j = 0; j < njet; ++j) cj.push_back(to_jet<cplx>(jets[j]));
  if (which < 5) {
    Jet<cplx>& t = cj[jet];
    cplx ih(0.0, h);
    if (which == 0) t.krad += ih;
    if (which == 1) t.kcoll += ih;
    if (which >= 2) t.x0[which - 2] += ih;
  }
  std::vector<cplx> Ej(njet);
  for (int j = 0; j < njet; ++j) Ej[j] = cplx(jets[j].E0, 0.0);
  cplx ledger(0.0, 0.0);
  long long fx = 0;
  run_impl<cplx>(c, nullptr, njet, U.data(), nsteps, 0, Ej.data(), &ledger, &fx, &cj);
  cplx r = eps2_of<cplx>(*c, U.data(), &fx);
  *value = r.real();
  *deriv = r.imag() / h;
  return 0;
}

// Directional derivative of nsteps steps from step 0 by the complex-step
// method: the run from U0 + i h V (jets at their E0) gives U(nsteps) as the
// real part and J V = Im / h, with J the Jacobian of the state after nsteps
// with respect to the initial conserved state.  Arrays [5][ncell].
int oracle_jvp(const ocfg* c, const ojet* jets, int njet, const double* U0, const double* V,
               int nsteps, double h, double* Uout, double* JV) {
  if (!valid(c) || njet < 0 || nsteps < 0 || !(h > 0.0)) return -1;
  size_t m = 5 * (size_t)c->n[0] * c->n[1] * c->n[2];
  std::vector<cplx> U(m);
  for (size_t q = 0; q < m; ++q) U[q] = cplx(U0[q], h * V[q]);
  std::vector<Jet<cplx>> cj;
  for (int j = 0; j < njet; ++j) cj.push_back(to_jet<cplx>(jets[j]));
  std::vector<cplx> Ej(njet);
  for (int j = 0; j < njet; ++j) Ej[j] = cplx(jets[j].E0, 0.0);
  cplx ledger(0.0, 0.0);
  long long fx = 0;
  run_impl<cplx>(c, nullptr, njet, U.data(), nsteps, 0, Ej.data(), &ledger, &fx, &cj);
  for (size_t q = 0; q < m; ++q) {
    Uout[q] = U[q].real();
    JV[q] = U[q].imag() / h;
  }
  return 0;
}

// The flux limiter on one face along axis d between the cells with conserved
// states uA (low side) and uB (high side): H (five face fluxes) in/out,
// *theta the limiter's weight of the high-order flux.
int oracle_limit_face(const ocfg* c, int d, const double* uA, const double* uB, double* H, double* theta) {
  if (!valid(c) || d < 0 || d > 2) return -1;
  long long fx = 0;
  double fA[5], fB[5];
  const double* us[2] = {uA, uB};
  double* fs[2] = {fA, fB};
  for (int k = 0; k < 2; ++k) {
    const double* u = us[k];
    Prim<double> p = cons_to_prim(u[0], u[1], u[2], u[3], u[4], &fx);
    const double pr = p.e / 3.0;
    fs[k][0] = u[1 + d];
    for (int m = 0; m < 3; ++m) fs[k][1 + m] = u[1 + m] * p.v[d] + (m == d ? pr : 0.0);
    fs[k][4] = u[4] * p.v[d];
  }
  const double mu = 2.0 * c->dt * (1.0 / c->dx[0] + 1.0 / c->dx[1] + 1.0 / c->dx[2]);
  *theta = Solver<double>::limit_face_mu(mu, uA, fA, uB, fB, H);
  return 0;
}

// MUSTA-FORCE flux along axis d of the face states uL, uR with k stages;
// uLk, uRk (may be NULL) receive the local states the last stage started from.
int oracle_musta_flux(int d, const double* uL, const double* uR, int k, double* F, double* uLk, double* uRk) {
  if (d < 0 || d > 2 || k < 1) return -1;
  double a[5], b[5];
  for (int m = 0; m < 5; ++m) {
    a[m] = uL[m];
    b[m] = uR[m];
  }
  long long fx = 0;
  Solver<double>::musta_force(d, a, b, k, F, &fx);
  for (int m = 0; m < 5; ++m) {
    if (uLk) uLk[m] = a[m];
    if (uRk) uRk[m] = b[m];
  }
  return 0;
}

// Operation counts {adds, multiplies, divides, square roots} of one call of
// the plain formulation: what = 0 a WENO7 reconstruction, 1 a WENO5
// reconstruction (scheme 0 Z, 1 JS, 2 linear), 2 a conserved->primitive
// recovery of an admissible state.
int oracle_count_flops(int what, int scheme, long long* out4) {
  if (what < 0 || what > 2 || scheme < 0 || scheme > 2 || !out4) return -1;
  for (int k = 0; k < 4; ++k) g_flops[k] = 0;
  if (what == 0) {
    Counted a[7] = {1.0, 1.3, 0.7, 2.1, 1.9, 2.6, 2.2};
    (void)weno7_left<Counted>(a, scheme, 1e-6, 2);
  } else if (what == 1) {
    Counted a[5] = {1.0, 1.3, 0.7, 2.1, 1.9};
    (void)weno5_left<Counted>(a, scheme, 1e-6, 2);
  } else {
    long long fx = 0;
    (void)cons_to_prim<Counted>(Counted(5.0), Counted(1.0), Counted(-0.5), Counted(0.3), Counted(0.8), &fx);
  }
  for (int k = 0; k < 4; ++k) out4[k] = g_flops[k];
  return 0;
}

}  // extern "C"
