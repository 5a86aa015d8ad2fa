// FP64 oracle of the tangent-linear model and the discrete adjoint of the
// single-grid advance (test infrastructure only).
//
// Both derivatives are taken of the oracle's own templated step by operator
// overloading, so they are the exact derivatives of the implemented map with
// every branch (minmod choice, min/max of wave speeds, HLLD region and
// degeneracy tests) frozen at the primal values:
//   * forward mode: a dual number carries one tangent direction;
//   * reverse mode: each step is recorded on a tape (one node per arithmetic
//     operation, its operands and local partials) and swept backwards.
// Problem: periodic grid, band 2 refilled every step, dt frozen; controls
// are the initial cell density and velocity (pressure and face B fixed); the
// loss is the kinetic energy sum over cells c in a box S of |m_c|^2/(2 rho_c)
// times the cell volume after the last step.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "scheme.hpp"

namespace {

thread_local std::string j_err;

// ------------------------------------------------------------------ dual
struct Dual {
  double v, d;
  Dual(double x = 0.0) : v(x), d(0.0) {}
  Dual(double x, double dx) : v(x), d(dx) {}
};
inline Dual operator+(const Dual& a, const Dual& b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(const Dual& a, const Dual& b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator*(const Dual& a, const Dual& b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(const Dual& a, const Dual& b) {
  const double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual operator-(const Dual& a) { return Dual(-a.v, -a.d); }
inline Dual operator+(const Dual& a, double b) { return Dual(a.v + b, a.d); }
inline Dual operator-(const Dual& a, double b) { return Dual(a.v - b, a.d); }
inline Dual operator-(double a, const Dual& b) { return Dual(a - b.v, -b.d); }
inline Dual operator*(double a, const Dual& b) { return Dual(a * b.v, a * b.d); }
inline Dual operator*(const Dual& a, double b) { return Dual(a.v * b, a.d * b); }
inline Dual operator/(const Dual& a, double b) { return Dual(a.v / b, a.d / b); }
inline Dual operator/(double a, const Dual& b) {
  const double q = a / b.v;
  return Dual(q, -q * b.d / b.v);
}
inline double value(const Dual& x) { return x.v; }
inline Dual Sqrt(const Dual& x) {
  const double s = std::sqrt(x.v);
  return Dual(s, x.d / (2.0 * s));
}

// ------------------------------------------------------------------ tape
struct Tape {
  std::vector<int32_t> a, b;
  std::vector<double> da, db;
  int32_t push(int32_t x, double dx, int32_t y, double dy) {
    a.push_back(x);
    da.push_back(dx);
    b.push_back(y);
    db.push_back(dy);
    return (int32_t)a.size() - 1;
  }
  void clear() {
    a.clear();
    b.clear();
    da.clear();
    db.clear();
  }
};
Tape g_tape;

// A taped value: index of its node (-1 for a constant) and its primal value.
struct Adj {
  int32_t i;
  double v;
  Adj(double x = 0.0) : i(-1), v(x) {}
  Adj(int32_t idx, double x) : i(idx), v(x) {}
};
inline Adj mk(double v, int32_t x, double dx, int32_t y, double dy) {
  if (x < 0 && y < 0) return Adj(v);
  return Adj(g_tape.push(x, dx, y, dy), v);
}
inline Adj operator+(const Adj& a, const Adj& b) { return mk(a.v + b.v, a.i, 1.0, b.i, 1.0); }
inline Adj operator-(const Adj& a, const Adj& b) { return mk(a.v - b.v, a.i, 1.0, b.i, -1.0); }
inline Adj operator*(const Adj& a, const Adj& b) { return mk(a.v * b.v, a.i, b.v, b.i, a.v); }
inline Adj operator/(const Adj& a, const Adj& b) {
  const double q = a.v / b.v;
  return mk(q, a.i, 1.0 / b.v, b.i, -q / b.v);
}
inline Adj operator-(const Adj& a) { return mk(-a.v, a.i, -1.0, -1, 0.0); }
inline Adj operator+(const Adj& a, double b) { return mk(a.v + b, a.i, 1.0, -1, 0.0); }
inline Adj operator-(const Adj& a, double b) { return mk(a.v - b, a.i, 1.0, -1, 0.0); }
inline Adj operator-(double a, const Adj& b) { return mk(a - b.v, b.i, -1.0, -1, 0.0); }
inline Adj operator*(double a, const Adj& b) { return mk(a * b.v, b.i, a, -1, 0.0); }
inline Adj operator*(const Adj& a, double b) { return mk(a.v * b, a.i, b, -1, 0.0); }
inline Adj operator/(const Adj& a, double b) { return mk(a.v / b, a.i, 1.0 / b, -1, 0.0); }
inline Adj operator/(double a, const Adj& b) {
  const double q = a / b.v;
  return mk(q, b.i, -q / b.v, -1, 0.0);
}
inline double value(const Adj& x) { return x.v; }
inline Adj Sqrt(const Adj& x) {
  const double s = std::sqrt(x.v);
  return mk(s, x.i, 0.5 / s, -1, 0.0);
}

}  // namespace

namespace orc {
template <> struct OmpSafe<Adj> { static constexpr bool value = false; };
}  // namespace orc

using namespace orc;

namespace {

Layout lay(int ndim, const int* n, int g) {
  Layout L;
  L.ndim = ndim;
  for (int a = 0; a < 3; ++a) L.n[a] = a < ndim ? n[a] : 1;
  L.g = g;
  return L;
}

int iext(const Layout& L, int s, int a) { return L.n[a] + ((L.is_face(s) && s - 5 == a) ? 1 : 0); }
size_t iidx(const Layout& L, int s, int i, int j, int k) {
  return ((size_t)k * iext(L, s, 1) + j) * iext(L, s, 0) + i;
}

// periodic band fill of any scalar type (copies; on a tape the band element
// becomes the same variable as its source)
template <class T> void fill_periodic(State<T>& S) {
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
          int c[3] = {i, j, k}, m[3] = {i, j, k};
          bool in = true;
          for (int a = 0; a < L.ndim; ++a) {
            const int n = L.n[a];
            if (c[a] < 0 || c[a] >= n) {
              in = false;
              m[a] = ((c[a] % n) + n) % n;
            }
          }
          if (!in) S.at(s, i, j, k) = S.at(s, m[0], m[1], m[2]);
        }
  }
}

// Initial conserved state from controls (rho, v) and fixed (p, face B).
template <class T>
State<T> initial_state(const Layout& L, const T* rho, const T* vx, const T* vy, const T* vz, const double* p,
                       const double* const* bf, double gamma) {
  State<T> S(L);
  for (int s = 5; s < 8; ++s)
    for (int k = 0; k < iext(L, s, 2); ++k)
      for (int j = 0; j < iext(L, s, 1); ++j)
        for (int i = 0; i < iext(L, s, 0); ++i) S.at(s, i, j, k) = T(bf[s - 5][iidx(L, s, i, j, k)]);
  fill_periodic(S);
  for (int k = 0; k < L.n[2]; ++k)
    for (int j = 0; j < L.n[1]; ++j)
      for (int i = 0; i < L.n[0]; ++i) {
        const size_t c = iidx(L, 0, i, j, k);
        T W[NVAR], U[NVAR];
        W[0] = rho[c];
        W[1] = vx[c];
        W[2] = vy[c];
        W[3] = vz[c];
        W[4] = T(p[c]);
        for (int a = 0; a < 3; ++a) W[5 + a] = bcell(S, a, i, j, k);
        prim_to_cons(W, U, gamma);
        for (int s = 0; s < 5; ++s) S.at(s, i, j, k) = U[s];
      }
  return S;
}

// Kinetic energy of the cells of box S (lo[a] .. lo[a]+len[a]-1, periodic).
template <class T> T loss(const State<T>& S, const int* lo, const int* len, double dv) {
  const Layout& L = S.L;
  T J = T(0.0);
  for (int k = 0; k < (L.ndim == 3 ? len[2] : 1); ++k)
    for (int j = 0; j < len[1]; ++j)
      for (int i = 0; i < len[0]; ++i) {
        const int x = (lo[0] + i) % L.n[0], y = (lo[1] + j) % L.n[1], z = L.ndim == 3 ? (lo[2] + k) % L.n[2] : 0;
        const T& r = S.at(0, x, y, z);
        const T& mx = S.at(1, x, y, z);
        const T& my = S.at(2, x, y, z);
        const T& mz = S.at(3, x, y, z);
        J = J + (mx * mx + my * my + mz * mz) / (2.0 * r) * dv;
      }
  return J;
}

template <class T>
State<T> run(State<T> S, int nsteps, const double* dts, const StepParams& P) {
  State<T> O(S.L);
  for (int s = 0; s < nsteps; ++s) {
    fill_periodic(S);
    step(S, O, 2, T(dts[s]), P);
    std::swap(S, O);
  }
  return S;
}

StepParams params(int ndim, const int* n, double gamma) {
  return StepParams{gamma, {1.0 / n[0], 1.0 / n[1], ndim == 3 ? 1.0 / n[2] : 1.0}, 0};
}

double cell_volume(int ndim, const int* n) {
  double dv = 1.0;
  for (int a = 0; a < ndim; ++a) dv /= n[a];
  return dv;
}

}  // namespace

extern "C" {

const char* orc_adj_last_error() { return j_err.c_str(); }

// Loss after nsteps (plain double).  prim: rho, vx, vy, vz, p (interior
// layout); b: 3 face arrays.
int orc_ke_loss(int ndim, const int* n, double gamma, int nsteps, const double* dts, const double* const* prim,
                const double* const* b, const int* lo, const int* len, double* J) {
  try {
    Layout L = lay(ndim, n, 2);
    State<double> S = initial_state<double>(L, prim[0], prim[1], prim[2], prim[3], prim[4], b, gamma);
    S = run(S, nsteps, dts, params(ndim, n, gamma));
    *J = loss(S, lo, len, cell_volume(ndim, n));
    return 0;
  } catch (const std::exception& e) {
    j_err = e.what();
    return -1;
  }
}

// Branch signature of the plain forward run behind orc_ke_loss (see
// BranchLog in scheme.hpp).
int orc_ke_branch_signature(int ndim, const int* n, double gamma, int nsteps, const double* dts,
                            const double* const* prim, const double* const* b, uint64_t* sig) {
  try {
    Layout L = lay(ndim, n, 2);
    BranchLog::on() = true;
    BranchLog::hash() = 1469598103934665603ull;
    State<double> S = initial_state<double>(L, prim[0], prim[1], prim[2], prim[3], prim[4], b, gamma);
    S = run(S, nsteps, dts, params(ndim, n, gamma));
    *sig = BranchLog::hash();
    BranchLog::on() = false;
    return 0;
  } catch (const std::exception& e) {
    BranchLog::on() = false;
    j_err = e.what();
    return -1;
  }
}

// Tangent-linear model: dJ along the control direction (drho, dvx, dvy, dvz)
// (interior layout), by forward-mode dual numbers.
int orc_ke_tlm(int ndim, const int* n, double gamma, int nsteps, const double* dts, const double* const* prim,
               const double* const* b, const int* lo, const int* len, const double* const* dir, double* J,
               double* dJ) {
  try {
    Layout L = lay(ndim, n, 2);
    const size_t nc = (size_t)L.n[0] * L.n[1] * L.n[2];
    std::vector<Dual> r(nc), vx(nc), vy(nc), vz(nc);
    for (size_t c = 0; c < nc; ++c) {
      r[c] = Dual(prim[0][c], dir[0][c]);
      vx[c] = Dual(prim[1][c], dir[1][c]);
      vy[c] = Dual(prim[2][c], dir[2][c]);
      vz[c] = Dual(prim[3][c], dir[3][c]);
    }
    State<Dual> S = initial_state<Dual>(L, r.data(), vx.data(), vy.data(), vz.data(), prim[4], b, gamma);
    S = run(S, nsteps, dts, params(ndim, n, gamma));
    Dual Jd = loss(S, lo, len, cell_volume(ndim, n));
    *J = Jd.v;
    *dJ = Jd.d;
    return 0;
  } catch (const std::exception& e) {
    j_err = e.what();
    return -1;
  }
}

// Gradient of J with respect to the controls (rho, vx, vy, vz), written to
// grad[0..3] (interior layout), by reverse mode: the forward states are
// kept in double, then each step is taped and swept backwards from the last.
int orc_ke_grad(int ndim, const int* n, double gamma, int nsteps, const double* dts, const double* const* prim,
                const double* const* b, const int* lo, const int* len, double* const* grad, double* J) {
  try {
    Layout L = lay(ndim, n, 2);
    StepParams P = params(ndim, n, gamma);
    const double dv = cell_volume(ndim, n);
    // forward in double, keeping every state
    std::vector<State<double>> states;
    states.push_back(initial_state<double>(L, prim[0], prim[1], prim[2], prim[3], prim[4], b, gamma));
    {
      State<double> O(L);
      for (int s = 0; s < nsteps; ++s) {
        State<double> S = states.back();
        fill_periodic(S);
        step(S, O, 2, dts[s], P);
        states.push_back(O);
      }
    }
    // adjoint of the loss
    std::vector<std::vector<double>> lam(NVAR);
    {
      g_tape.clear();
      State<Adj> S(L);
      for (int s = 0; s < NVAR; ++s)
        for (size_t e = 0; e < L.fsize(s); ++e) S.f[s][e] = Adj(g_tape.push(-1, 0.0, -1, 0.0), states.back().f[s][e]);
      Adj Ja = loss(S, lo, len, dv);
      *J = Ja.v;
      std::vector<double> adj(g_tape.a.size(), 0.0);
      if (Ja.i >= 0) adj[Ja.i] = 1.0;
      for (int32_t t = (int32_t)g_tape.a.size() - 1; t >= 0; --t) {
        if (adj[t] == 0.0) continue;
        if (g_tape.a[t] >= 0) adj[g_tape.a[t]] += adj[t] * g_tape.da[t];
        if (g_tape.b[t] >= 0) adj[g_tape.b[t]] += adj[t] * g_tape.db[t];
      }
      for (int s = 0; s < NVAR; ++s) {
        lam[s].assign(L.fsize(s), 0.0);
        for (size_t e = 0; e < L.fsize(s); ++e) lam[s][e] = adj[S.f[s][e].i];
      }
    }
    // steps, last to first
    for (int st = nsteps - 1; st >= 0; --st) {
      g_tape.clear();
      State<Adj> S(L), O(L);
      std::vector<int32_t> in_idx[NVAR];
      for (int s = 0; s < NVAR; ++s) {
        in_idx[s].resize(L.fsize(s));
        for (size_t e = 0; e < L.fsize(s); ++e) {
          int32_t id = g_tape.push(-1, 0.0, -1, 0.0);
          in_idx[s][e] = id;
          S.f[s][e] = Adj(id, states[st].f[s][e]);
        }
      }
      fill_periodic(S);
      step(S, O, 2, Adj(dts[st]), P);
      std::vector<double> adj(g_tape.a.size(), 0.0);
      // seed with the adjoint of the outputs that the step owns (interior
      // cells and faces [0, n] along the normal); band outputs are not state
      for (int s = 0; s < NVAR; ++s)
        for (int k = 0; k < iext(L, s, 2); ++k)
          for (int j = 0; j < iext(L, s, 1); ++j)
            for (int i = 0; i < iext(L, s, 0); ++i) {
              const size_t e = L.idx(s, i, j, k);
              const Adj& v = O.f[s][e];
              if (v.i >= 0) adj[v.i] += lam[s][e];
            }
      for (int32_t t = (int32_t)g_tape.a.size() - 1; t >= 0; --t) {
        const double at = adj[t];
        if (at == 0.0) continue;
        if (g_tape.a[t] >= 0) adj[g_tape.a[t]] += at * g_tape.da[t];
        if (g_tape.b[t] >= 0) adj[g_tape.b[t]] += at * g_tape.db[t];
      }
      for (int s = 0; s < NVAR; ++s)
        for (size_t e = 0; e < L.fsize(s); ++e) lam[s][e] = adj[in_idx[s][e]];
    }
    // chain to the controls through the initial state
    {
      g_tape.clear();
      const size_t nc = (size_t)L.n[0] * L.n[1] * L.n[2];
      std::vector<Adj> r(nc), vx(nc), vy(nc), vz(nc);
      for (size_t c = 0; c < nc; ++c) {
        r[c] = Adj(g_tape.push(-1, 0.0, -1, 0.0), prim[0][c]);
        vx[c] = Adj(g_tape.push(-1, 0.0, -1, 0.0), prim[1][c]);
        vy[c] = Adj(g_tape.push(-1, 0.0, -1, 0.0), prim[2][c]);
        vz[c] = Adj(g_tape.push(-1, 0.0, -1, 0.0), prim[3][c]);
      }
      State<Adj> S = initial_state<Adj>(L, r.data(), vx.data(), vy.data(), vz.data(), prim[4], b, gamma);
      std::vector<double> adj(g_tape.a.size(), 0.0);
      for (int s = 0; s < 5; ++s)
        for (int k = 0; k < L.n[2]; ++k)
          for (int j = 0; j < L.n[1]; ++j)
            for (int i = 0; i < L.n[0]; ++i) {
              const size_t e = L.idx(s, i, j, k);
              if (S.f[s][e].i >= 0) adj[S.f[s][e].i] += lam[s][e];
            }
      for (int32_t t = (int32_t)g_tape.a.size() - 1; t >= 0; --t) {
        const double at = adj[t];
        if (at == 0.0) continue;
        if (g_tape.a[t] >= 0) adj[g_tape.a[t]] += at * g_tape.da[t];
        if (g_tape.b[t] >= 0) adj[g_tape.b[t]] += at * g_tape.db[t];
      }
      for (size_t c = 0; c < nc; ++c) {
        grad[0][c] = adj[r[c].i];
        grad[1][c] = adj[vx[c].i];
        grad[2][c] = adj[vy[c].i];
        grad[3][c] = adj[vz[c].i];
      }
    }
    g_tape.clear();
    g_tape.a.shrink_to_fit();
    g_tape.b.shrink_to_fit();
    g_tape.da.shrink_to_fit();
    g_tape.db.shrink_to_fit();
    return 0;
  } catch (const std::exception& e) {
    j_err = e.what();
    g_tape.clear();
    return -1;
  }
}

// Vector-Jacobian product of one step of the single periodic grid (band 2
// refilled first, dt given): lam_in = (dU'/dU)^T lam_out.  U and the
// adjoints are the eight interior arrays (cells; faces with n+1 entries
// along their normal).  The periodic fill makes the input face n a copy of
// face 0, so lam_in of face n is 0 and face 0 carries both.
int orc_step_vjp(int ndim, const int* n, double gamma, double dt, const double* const* U,
                 const double* const* lam_out, double* const* lam_in) {
  try {
    Layout L = lay(ndim, n, 2);
    StepParams P = params(ndim, n, gamma);
    g_tape.clear();
    State<Adj> S(L), O(L);
    std::vector<std::vector<int32_t>> ids(NVAR);
    for (int s = 0; s < NVAR; ++s) {
      ids[s].assign(L.fsize(s), -1);
      for (int k = 0; k < iext(L, s, 2); ++k)
        for (int j = 0; j < iext(L, s, 1); ++j)
          for (int i = 0; i < iext(L, s, 0); ++i) {
            const size_t e = L.idx(s, i, j, k);
            const int32_t id = g_tape.push(-1, 0.0, -1, 0.0);
            ids[s][e] = id;
            S.f[s][e] = Adj(id, U[s][iidx(L, s, i, j, k)]);
          }
    }
    fill_periodic(S);
    step(S, O, 2, Adj(dt), P);
    std::vector<double> adj(g_tape.a.size(), 0.0);
    for (int s = 0; s < NVAR; ++s)
      for (int k = 0; k < iext(L, s, 2); ++k)
        for (int j = 0; j < iext(L, s, 1); ++j)
          for (int i = 0; i < iext(L, s, 0); ++i) {
            const Adj& v = O.at(s, i, j, k);
            if (v.i >= 0) adj[v.i] += lam_out[s][iidx(L, s, i, j, k)];
          }
    for (int32_t t = (int32_t)g_tape.a.size() - 1; t >= 0; --t) {
      const double at = adj[t];
      if (at == 0.0) continue;
      if (g_tape.a[t] >= 0) adj[g_tape.a[t]] += at * g_tape.da[t];
      if (g_tape.b[t] >= 0) adj[g_tape.b[t]] += at * g_tape.db[t];
    }
    for (int s = 0; s < NVAR; ++s)
      for (int k = 0; k < iext(L, s, 2); ++k)
        for (int j = 0; j < iext(L, s, 1); ++j)
          for (int i = 0; i < iext(L, s, 0); ++i)
            lam_in[s][iidx(L, s, i, j, k)] = adj[ids[s][L.idx(s, i, j, k)]];
    g_tape.clear();
    return 0;
  } catch (const std::exception& e) {
    j_err = e.what();
    g_tape.clear();
    return -1;
  }
}


// Vector-Jacobian product of one substep of every grid of one level, the
// batched level map of the adjoint: each grid's band is first refreshed by
// the same-level copy -- a band cell lying in a grid's interior, or a band
// face lying in or on the boundary of one (periodic images included), takes
// that element of the lowest-index such grid -- and every other band
// element (the prolonged part) is a constant of the map; then every grid
// takes one band-2 step of size dt (Sec. 1 and the abstract: the grid's
// advance reads nothing but its own band).  The own elements of a grid are
// its cells [0, n) and its faces [0, n] along their normal ([0, n) across);
// a face shared by two grids is an own element of both.
//   Nl: the level's cells per axis (periodic); boxes: ngrids x (lo[3],
//   hi[3]) in level cells; banded: ngrids*8 pointers, each grid's state in
//   the oracle's banded layout with band g (constant band values and own
//   values are read here); sel[0..nsel): the grids whose output adjoint is
//   given (lam_out: nsel*8 interior-layout pointers; zero on other grids);
//   lam_in: ngrids*8 interior-layout pointers, the adjoint of the input on
//   every grid's own elements (written in full).
int orc_level_vjp(int ndim, const int* Nl, int g, double gamma, const double* dx, double dt, int ngrids,
                  const int* boxes, const double* const* banded, int nsel, const int* sel,
                  const double* const* lam_out, double* const* lam_in) {
  try {
    if (g < 2) throw std::runtime_error("band too narrow");
    std::vector<Layout> Ls(ngrids);
    for (int G = 0; G < ngrids; ++G) {
      int n[3];
      for (int a = 0; a < 3; ++a) n[a] = a < ndim ? boxes[6 * G + 3 + a] - boxes[6 * G + a] : 1;
      Ls[G] = lay(ndim, n, g);
      for (int s = 0; s < NVAR; ++s) {
        size_t m = (size_t)iext(Ls[G], s, 0) * iext(Ls[G], s, 1) * iext(Ls[G], s, 2);
        std::fill(lam_in[8 * G + s], lam_in[8 * G + s] + m, 0.0);
      }
    }
    auto lo = [&](int G, int a) { return a < ndim ? boxes[6 * G + a] : 0; };
    auto hi = [&](int G, int a) { return a < ndim ? boxes[6 * G + 3 + a] : 1; };
    auto wrap = [&](int (&p)[3]) {
      for (int a = 0; a < ndim; ++a) p[a] = ((p[a] % Nl[a]) + Nl[a]) % Nl[a];
    };
    // grid whose interior holds the (wrapped) level cell p, or -1
    auto owner = [&](const int (&p)[3]) {
      for (int H = 0; H < ngrids; ++H) {
        bool in = true;
        for (int a = 0; a < 3; ++a) in = in && p[a] >= lo(H, a) && p[a] < hi(H, a);
        if (in) return H;
      }
      return -1;
    };
    // source (grid, local index) of element (s, level position p) under the
    // same-level copy, or false
    auto source = [&](int s, const int (&p)[3], int& H, int (&loc)[3]) {
      const bool face = Ls[0].is_face(s);
      const int d = s - 5;
      H = -1;
      for (int side = 0; side < (face ? 2 : 1); ++side) {
        int c[3] = {p[0], p[1], p[2]};
        if (side == 1) c[d] -= 1;
        wrap(c);
        const int w = owner(c);
        if (w < 0 || (H >= 0 && w >= H)) continue;
        H = w;
        for (int a = 0; a < 3; ++a) loc[a] = c[a] - lo(w, a);
        if (side == 1) loc[d] += 1;
      }
      return H >= 0;
    };
    StepParams P{gamma, {dx[0], dx[1], ndim == 3 ? dx[2] : 1.0}, 0};
    for (int t = 0; t < nsel; ++t) {
      const int G = sel[t];
      if (G < 0 || G >= ngrids) throw std::runtime_error("selected grid out of range");
      const Layout& L = Ls[G];
      g_tape.clear();
      // tape variables of this pass: (grid, slot, interior index) -> node
      std::vector<std::vector<int32_t>> ids((size_t)ngrids * NVAR);
      auto var = [&](int H, int s, const int (&q)[3]) {
        std::vector<int32_t>& v = ids[(size_t)H * NVAR + s];
        if (v.empty()) v.assign((size_t)iext(Ls[H], s, 0) * iext(Ls[H], s, 1) * iext(Ls[H], s, 2), -1);
        const size_t e = iidx(Ls[H], s, q[0], q[1], q[2]);
        if (v[e] < 0) v[e] = g_tape.push(-1, 0.0, -1, 0.0);
        const double val = banded[8 * H + s][Ls[H].idx(s, q[0], q[1], q[2])];
        return Adj(v[e], val);
      };
      State<Adj> S(L), O(L);
      for (int s = 0; s < NVAR; ++s) {
        const bool face = L.is_face(s);
        for (int k = -L.gd(2); k < L.n[2] + L.gd(2) + ((face && s == 7) ? 1 : 0); ++k)
          for (int j = -L.gd(1); j < L.n[1] + L.gd(1) + ((face && s == 6) ? 1 : 0); ++j)
            for (int i = -L.gd(0); i < L.n[0] + L.gd(0) + ((face && s == 5) ? 1 : 0); ++i) {
              const int x[3] = {i, j, k};
              bool own = true;
              for (int a = 0; a < ndim; ++a) {
                const int top = (face && s - 5 == a) ? L.n[a] : L.n[a] - 1;
                own = own && x[a] >= 0 && x[a] <= top;
              }
              if (own) {
                S.at(s, i, j, k) = var(G, s, x);
                continue;
              }
              int p[3] = {lo(G, 0) + i, lo(G, 1) + j, lo(G, 2) + k}, H, loc[3];
              if (source(s, p, H, loc))
                S.at(s, i, j, k) = var(H, s, loc);
              else
                S.at(s, i, j, k) = Adj(banded[8 * G + s][L.idx(s, i, j, k)]);
            }
      }
      step(S, O, 2, Adj(dt), P);
      std::vector<double> adj(g_tape.a.size(), 0.0);
      for (int s = 0; s < NVAR; ++s)
        for (int k = 0; k < iext(L, s, 2); ++k)
          for (int j = 0; j < iext(L, s, 1); ++j)
            for (int i = 0; i < iext(L, s, 0); ++i) {
              const Adj& v = O.at(s, i, j, k);
              if (v.i >= 0) adj[v.i] += lam_out[8 * t + s][iidx(L, s, i, j, k)];
            }
      for (int32_t q = (int32_t)g_tape.a.size() - 1; q >= 0; --q) {
        const double aq = adj[q];
        if (aq == 0.0) continue;
        if (g_tape.a[q] >= 0) adj[g_tape.a[q]] += aq * g_tape.da[q];
        if (g_tape.b[q] >= 0) adj[g_tape.b[q]] += aq * g_tape.db[q];
      }
      for (int H = 0; H < ngrids; ++H)
        for (int s = 0; s < NVAR; ++s) {
          const std::vector<int32_t>& v = ids[(size_t)H * NVAR + s];
          for (size_t e = 0; e < v.size(); ++e)
            if (v[e] >= 0) lam_in[8 * H + s][e] += adj[v[e]];
        }
    }
    g_tape.clear();
    g_tape.a.shrink_to_fit();
    g_tape.b.shrink_to_fit();
    g_tape.da.shrink_to_fit();
    g_tape.db.shrink_to_fit();
    return 0;
  } catch (const std::exception& e) {
    j_err = e.what();
    g_tape.clear();
    return -1;
  }
}

}  // extern "C"
