// C entry points of the FP64 oracle (test infrastructure only; see scheme.hpp).
//
// Exchange layout ("interior layout") used by every entry point that takes
// whole fields: C-order arrays with x fastest,
//   cells  : (nz, ny, nx)
//   Bx face: (nz, ny, nx+1)   By face: (nz, ny+1, nx)   Bz face: (nz+1, ny, nx)
// In 2D nz = 1 and Bz is a cell array (1, ny, nx).
#include <algorithm>
#include <chrono>
#include <cstring>
#include <exception>
#include <string>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "scheme.hpp"

using namespace orc;

namespace {

thread_local std::string g_err;

int fail(const std::string& m) {
  g_err = m;
  return -1;
}

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1 };

// Interior-layout extent of field slot s along axis a.
int iext(const Layout& L, int s, int a) {
  int n = L.n[a];
  if (L.is_face(s) && s - 5 == a) n += 1;
  return n;
}

size_t iindex(const Layout& L, int s, int i, int j, int k) {
  return ((size_t)k * iext(L, s, 1) + j) * iext(L, s, 0) + i;
}


// Physical boundary fill (reading: periodic wrap, or zero-gradient outflow
// with the normal face copied from the last domain face).  Every band element
// takes the value of the element it maps to inside the domain.
template <class T> void fill_physical(State<T>& S, const int* bc) {
  const Layout& L = S.L;
  for (int s = 0; s < NVAR; ++s) {
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = -L.gd(a);
      hi[a] = L.n[a] + L.gd(a) + ((L.is_face(s) && s - 5 == a) ? 1 : 0);
    }
    for (int k = lo[2]; k < hi[2]; ++k)
      for (int j = lo[1]; j < hi[1]; ++j)
        for (int i = lo[0]; i < hi[0]; ++i) {
          int c[3] = {i, j, k};
          int m[3] = {i, j, k};
          bool inside = true;
          for (int a = 0; a < L.ndim; ++a) {
            bool normal = L.is_face(s) && s - 5 == a;
            int n = L.n[a];
            if (bc[a] == BC_PERIODIC) {
              if (c[a] < 0 || c[a] >= n) {
                inside = false;
                m[a] = ((c[a] % n) + n) % n;
              }
            } else {
              int top = normal ? n : n - 1;
              if (c[a] < 0) { inside = false; m[a] = 0; }
              if (c[a] > top) { inside = false; m[a] = top; }
            }
          }
          if (!inside) S.at(s, i, j, k) = S.at(s, m[0], m[1], m[2]);
        }
  }
}

// CFL time step: dt = C / max over interior cells of sum_d (|v_d| + c_f,d)/dx_d,
// with c_f,d the fast speed for the cell-centred field component B_d.
template <class T> double cfl_dt(const State<T>& S, const StepParams& P, double cfl) {
  const Layout& L = S.L;
  double mx = 0.0;
  for (int k = 0; k < L.n[2]; ++k)
    for (int j = 0; j < L.n[1]; ++j)
      for (int i = 0; i < L.n[0]; ++i) {
        double U[NVAR], W[NVAR];
        for (int s = 0; s < 5; ++s) U[s] = value(S.at(s, i, j, k));
        for (int a = 0; a < 3; ++a) U[5 + a] = value(bcell(S, a, i, j, k));
        cons_to_prim(U, W, P.gamma);
        double B2 = W[5] * W[5] + W[6] * W[6] + W[7] * W[7];
        double acc = 0.0;
        for (int d = 0; d < L.ndim; ++d) {
          double cf = fast_speed(W[0], W[4], B2, W[5 + d], P.gamma);
          acc += (std::fabs(W[1 + d]) + cf) / P.dx[d];
        }
        mx = std::max(mx, acc);
      }
  return cfl / mx;
}

Layout make_layout(int ndim, const int* n, int g) {
  if (ndim != 2 && ndim != 3) throw std::runtime_error("ndim must be 2 or 3");
  Layout L;
  L.ndim = ndim;
  for (int a = 0; a < 3; ++a) L.n[a] = a < ndim ? n[a] : 1;
  L.g = g;
  return L;
}

// Load interior-layout primitive data (rho, vx, vy, vz, p cells; B faces)
// into a banded conserved state, then fill the band.
State<double> load_primitive(const Layout& L, const double* const* prim, const double* const* bf, const int* bc,
                             double gamma) {
  State<double> S(L);
  for (int s = 5; s < 8; ++s)
    for (int k = 0; k < iext(L, s, 2); ++k)
      for (int j = 0; j < iext(L, s, 1); ++j)
        for (int i = 0; i < iext(L, s, 0); ++i) S.at(s, i, j, k) = bf[s - 5][iindex(L, s, i, j, k)];
  fill_physical(S, bc);
  for (int k = 0; k < L.n[2]; ++k)
    for (int j = 0; j < L.n[1]; ++j)
      for (int i = 0; i < L.n[0]; ++i) {
        size_t ii = iindex(L, 0, i, j, k);
        double W[NVAR], U[NVAR];
        for (int q = 0; q < 5; ++q) W[q] = prim[q][ii];
        for (int a = 0; a < 3; ++a) W[5 + a] = bcell(S, a, i, j, k);
        prim_to_cons(W, U, gamma);
        for (int s = 0; s < 5; ++s) S.at(s, i, j, k) = U[s];
      }
  fill_physical(S, bc);
  return S;
}

void store_interior(const State<double>& S, double* const* out) {
  const Layout& L = S.L;
  for (int s = 0; s < NVAR; ++s)
    for (int k = 0; k < iext(L, s, 2); ++k)
      for (int j = 0; j < iext(L, s, 1); ++j)
        for (int i = 0; i < iext(L, s, 0); ++i) out[s][iindex(L, s, i, j, k)] = S.at(s, i, j, k);
}

}  // namespace

extern "C" {

// Edge EMF of every later step: 0 arithmetic mean (Balsara & Spicer), 1
// upwinded (Gardiner & Stone); 2 is 1 with the upwind side swapped, a
// planted mistake that only the sensitivity tests use.  Returns the previous
// choice, or -1 for a bad value (unchanged).
int orc_set_emf(int mode) {
  if (mode < 0 || mode > 2) return -1;
  const int old = emf_mode();
  emf_mode() = mode;
  return old;
}

const char* orc_last_error() { return g_err.c_str(); }

int orc_max_threads() {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

double orc_minmod(double a, double b) { return minmod(a, b); }

void orc_prim_to_cons(const double* W, double* U, double gamma) { prim_to_cons(W, U, gamma); }
void orc_cons_to_prim(const double* U, double* W, double gamma) { cons_to_prim(U, W, gamma); }
void orc_phys_flux(const double* W, int d, double gamma, double* F) { phys_flux(W, d, gamma, F); }
double orc_fast_speed(double rho, double p, double B2, double Bn, double gamma) {
  return fast_speed(rho, p, B2, Bn, gamma);
}

// One HLLD flux on rotated primitive states L, R (8 values each; L[5] is B_n).
// info (may be NULL) receives {region, degen_star_L, degen_star_R, degen_dstar}.
void orc_hlld(const double* L, const double* R, double gamma, double* F, int* info) {
  HlldInfo inf;
  hlld(L, R, gamma, F, &inf);
  if (info) {
    info[0] = inf.region;
    info[1] = inf.degen_star_L;
    info[2] = inf.degen_star_R;
    info[3] = inf.degen_dstar;
  }
}

// HLLD path counts since the last call (see HlldStats: evaluations, outer
// star degenerate, inner states evaluated, inner states degenerate) into
// out[4]; the counters restart from zero, counting only while `enable`.
void orc_hlld_stats(int enable, long long* out) {
  for (int k = 0; k < 4; ++k) {
    if (out) out[k] = HlldStats::counts()[k].load();
    HlldStats::counts()[k].store(0);
  }
  HlldStats::on() = enable != 0;
}

// Uniform single-grid run.  Band g; the band is refilled from the physical
// boundary every `fill_every` steps (2*fill_every <= g).  dt of each step is
// dts_in[s] if dts_in is given, else the CFL step of the current interior.
// out: 8 interior-layout arrays (rho, mx, my, mz, E, Bx, By, Bz).
// dts_out (may be NULL) receives the dt of every step.  Returns 0 or -1.
int orc_uniform_run(int ndim, const int* n, const int* bc, double gamma, double cfl, const double* dx, int g,
                    int fill_every, int nsteps, const double* dts_in, const double* const* prim,
                    const double* const* bface, double* const* out, double* dts_out) {
  try {
    if (fill_every < 1 || 2 * fill_every > g) return fail("need 1 <= fill_every and 2*fill_every <= g");
    Layout L = make_layout(ndim, n, g);
    StepParams P{gamma, {dx[0], dx[1], ndim > 2 ? dx[2] : 1.0}, emf_mode()};
    State<double> S = load_primitive(L, prim, bface, bc, gamma);
    State<double> T2(L);
    int gv = g;
    for (int s = 0; s < nsteps; ++s) {
      if (s % fill_every == 0) {
        fill_physical(S, bc);
        gv = g;
      }
      double dt = dts_in ? dts_in[s] : cfl_dt(S, P, cfl);
      if (dts_out) dts_out[s] = dt;
      step(S, T2, gv, dt, P);
      std::swap(S, T2);
      gv -= 2;
    }
    store_interior(S, out);
    return 0;
  } catch (const std::exception& e) {
    return fail(e.what());
  }
}

// Time `nsteps` steps of the uniform run above (state set-up excluded);
// returns seconds, or -1 on error.
double orc_uniform_time(int ndim, const int* n, const int* bc, double gamma, double cfl, const double* dx, int g,
                        int fill_every, int nsteps, const double* const* prim, const double* const* bface) {
  try {
    Layout L = make_layout(ndim, n, g);
    StepParams P{gamma, {dx[0], dx[1], ndim > 2 ? dx[2] : 1.0}, emf_mode()};
    State<double> S = load_primitive(L, prim, bface, bc, gamma);
    State<double> T2(L);
    int gv = g;
    auto t0 = std::chrono::steady_clock::now();
    for (int s = 0; s < nsteps; ++s) {
      if (s % fill_every == 0) {
        fill_physical(S, bc);
        gv = g;
      }
      double dt = cfl_dt(S, P, cfl);
      step(S, T2, gv, dt, P);
      std::swap(S, T2);
      gv -= 2;
    }
    auto t1 = std::chrono::steady_clock::now();
    return std::chrono::duration<double>(t1 - t0).count();
  } catch (const std::exception& e) {
    fail(e.what());
    return -1.0;
  }
}

// One step on banded arrays in the oracle's own banded layout (cells
// (n+2g) per active axis, faces one longer along their normal, x fastest).
// Input valid on band gv; output valid on band gv-2.
int orc_step_banded(int ndim, const int* n, int g, int gv, double gamma, const double* dx, double dt,
                    const double* const* in, double* const* out) {
  try {
    Layout L = make_layout(ndim, n, g);
    StepParams P{gamma, {dx[0], dx[1], ndim > 2 ? dx[2] : 1.0}, emf_mode()};
    State<double> S(L), O(L);
    for (int s = 0; s < NVAR; ++s) std::memcpy(S.f[s].data(), in[s], L.fsize(s) * sizeof(double));
    step(S, O, gv, dt, P);
    for (int s = 0; s < NVAR; ++s) std::memcpy(out[s], O.f[s].data(), L.fsize(s) * sizeof(double));
    return 0;
  } catch (const std::exception& e) {
    return fail(e.what());
  }
}

// Fill the band of banded arrays from the physical boundary conditions.
int orc_fill_banded(int ndim, const int* n, int g, const int* bc, double* const* f) {
  try {
    Layout L = make_layout(ndim, n, g);
    State<double> S(L);
    for (int s = 0; s < NVAR; ++s) std::memcpy(S.f[s].data(), f[s], L.fsize(s) * sizeof(double));
    fill_physical(S, bc);
    for (int s = 0; s < NVAR; ++s) std::memcpy(f[s], S.f[s].data(), L.fsize(s) * sizeof(double));
    return 0;
  } catch (const std::exception& e) {
    return fail(e.what());
  }
}

// CFL dt of banded arrays (interior cells only).
double orc_dt_banded(int ndim, const int* n, int g, double gamma, double cfl, const double* dx,
                     const double* const* f) {
  Layout L = make_layout(ndim, n, g);
  StepParams P{gamma, {dx[0], dx[1], ndim > 2 ? dx[2] : 1.0}, emf_mode()};
  State<double> S(L);
  for (int s = 0; s < NVAR; ++s) std::memcpy(S.f[s].data(), f[s], L.fsize(s) * sizeof(double));
  return cfl_dt(S, P, cfl);
}

}  // extern "C"

// ------------------------------------------------------------ flop counts
// A scalar that counts its arithmetic (+, -, *, /, sqrt each one flop) so the
// algorithmic work of the scheme's pieces can be read off the oracle itself.
namespace {
struct Cnt {
  double v;
  static long long n;
  Cnt(double x = 0.0) : v(x) {}
};
long long Cnt::n = 0;
inline Cnt operator+(const Cnt& a, const Cnt& b) { ++Cnt::n; return Cnt(a.v + b.v); }
inline Cnt operator-(const Cnt& a, const Cnt& b) { ++Cnt::n; return Cnt(a.v - b.v); }
inline Cnt operator*(const Cnt& a, const Cnt& b) { ++Cnt::n; return Cnt(a.v * b.v); }
inline Cnt operator/(const Cnt& a, const Cnt& b) { ++Cnt::n; return Cnt(a.v / b.v); }
inline Cnt operator-(const Cnt& a) { return Cnt(-a.v); }
inline Cnt operator*(double a, const Cnt& b) { ++Cnt::n; return Cnt(a * b.v); }
inline Cnt operator*(const Cnt& a, double b) { ++Cnt::n; return Cnt(a.v * b); }
inline Cnt operator/(const Cnt& a, double b) { ++Cnt::n; return Cnt(a.v / b); }
inline Cnt operator/(double a, const Cnt& b) { ++Cnt::n; return Cnt(a / b.v); }
inline Cnt operator+(const Cnt& a, double b) { ++Cnt::n; return Cnt(a.v + b); }
inline Cnt operator-(const Cnt& a, double b) { ++Cnt::n; return Cnt(a.v - b); }
inline Cnt operator-(double a, const Cnt& b) { ++Cnt::n; return Cnt(a - b.v); }
// found by argument-dependent lookup from the templated scheme
inline double value(const Cnt& x) { return x.v; }
inline Cnt Sqrt(const Cnt& x) { ++Cnt::n; return Cnt(std::sqrt(x.v)); }
}  // namespace
long long g_marks[4];
namespace orc {
template <> struct OmpSafe<Cnt> { static constexpr bool value = false; };
template <> struct StepMark<Cnt> {
  static void mark(int k) { g_marks[k] = Cnt::n; }
};
}  // namespace orc

extern "C" {

// Flop counts of one step on an n^ndim periodic patch with band 2 of a
// smooth state (every HLLD face takes the double-star path in practice).
// out[0] = total flops of the step, out[1] = cells updated, out[2] = cells
// whose predicted states were formed, out[3] = HLLD faces evaluated,
// out[4..7] = flops of the phases: primitives + slopes + predictor, HLLD
// fluxes, EMFs, update.
int orc_count_step_flops(int ndim, int n, double* out) {
  try {
    int nn[3] = {n, n, n};
    Layout L = make_layout(ndim, nn, 2);
    State<Cnt> S(L), O(L);
    // smooth state: rho ~ 1, small v, p = 1, B ~ 0.3 with a gentle variation
    for (int s = 0; s < NVAR; ++s)
      for (size_t e = 0; e < L.fsize(s); ++e) {
        double x = 0.37 * (double)e;
        double v = 0.0;
        switch (s) {
          case 0: v = 1.0 + 0.05 * std::sin(x); break;
          case 1: v = 0.05 * std::sin(1.3 * x); break;
          case 2: v = 0.05 * std::cos(0.7 * x); break;
          case 3: v = 0.04 * std::sin(0.9 * x); break;
          case 4: v = 2.0 + 0.02 * std::cos(x); break;
          case 5: v = 0.3; break;
          case 6: v = 0.2 + 0.01 * std::sin(0.5 * x); break;
          default: v = -0.1; break;
        }
        S.f[s][e] = Cnt(v);
      }
    StepParams P{5.0 / 3.0, {1.0 / n, 1.0 / n, 1.0 / n}};
    Cnt::n = 0;
    step(S, O, 2, Cnt(1e-4), P);
    long long m = n + 2;  // cells with predicted states per axis: [-1, n+1)
    out[0] = (double)Cnt::n;
    out[1] = std::pow((double)n, ndim);
    out[2] = std::pow((double)m, ndim);
    out[3] = (double)ndim * (double)(n + 1) * std::pow((double)m, ndim - 1);
    out[4] = (double)g_marks[1];
    out[5] = (double)(g_marks[2] - g_marks[1]);
    out[6] = (double)(g_marks[3] - g_marks[2]);
    out[7] = (double)(Cnt::n - g_marks[3]);
    return 0;
  } catch (const std::exception& e) {
    return fail(e.what());
  }
}

// Flops of one HLLD evaluation on a generic state (double-star path).
long long orc_count_hlld_flops() {
  Cnt L[8] = {1.0, 0.05, 0.02, -0.01, 1.0, 0.3, 0.2, -0.1};
  Cnt R[8] = {0.9, 0.04, 0.01, 0.0, 0.95, 0.3, 0.25, -0.05};
  Cnt F[7];
  Cnt::n = 0;
  hlld(L, R, 5.0 / 3.0, F);
  return Cnt::n;
}

}  // extern "C"
