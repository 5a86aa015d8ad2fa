// Oracle for the ideal-MHD patch advance: plain, slow, FP64 reference.
//
// TEST INFRASTRUCTURE ONLY. Nothing in the product library includes, links or
// calls this code; only tests, the smoke check and the CPU-baseline leg of the
// benchmark load it. It shares no source with the HIP path.
//
// The paper (Carroll-Nellenback et al., "Efficient Parallelization for AMR MHD
// Multiphysics Calculations", Sec. 1 and the abstract) relies on a hyperbolic
// advance of each grid that is decoupled from its neighbours by ghost cells,
// and defers the scheme itself to the AstroBEAR code paper.  The scheme used
// here is fixed as: unsplit MUSCL-Hancock on primitive variables with minmod
// slopes, HLLD Riemann fluxes (Miyoshi & Kusano 2005, J. Comput. Phys. 208,
// 315) and constrained transport of face-centred B with the arithmetic edge
// average of Balsara & Spicer (1999).  Each function below names the step it
// implements; the numbered readings (R1..) are listed in the design notes.
//
// Every routine is templated on the scalar type so the same arithmetic can be
// evaluated in double, in forward-mode dual numbers (tangent-linear model) and
// on a reverse-mode tape (adjoint).  Branches compare primal values only, which
// is exactly "branches frozen from the forward pass".
#pragma once
#include <atomic>
#include <cmath>
#include <utility>
#include <cstddef>
#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace orc {

// OpenMP is used only over independent cells/faces of one pass; scalar types
// that record a global tape set this to false.
template <class T> struct OmpSafe { static constexpr bool value = true; };

// Phase marks of one step (used only by the flop-counting scalar to split
// the step's work into its parts; a no-op for every other type).
template <class T> struct StepMark {
  static void mark(int) {}
};

// Branch log: when enabled, every data-dependent decision of the scheme
// (minmod choice, min/max, sign, clamp, HLLD region and degeneracy) is folded
// into a running FNV-1a hash in evaluation order, so two runs that took the
// same branches everywhere have the same signature.  Used to tell apart
// finite-difference directions that cross a kink of the piecewise-smooth map.
struct BranchLog {
  static bool& on() {
    static bool v = false;
    return v;
  }
  static uint64_t& hash() {
    static uint64_t h = 1469598103934665603ull;
    return h;
  }
  static void note(int choice) {
    if (!on()) return;
    uint64_t& h = hash();
    h ^= (uint64_t)(choice + 1);
    h *= 1099511628211ull;
  }
};

// ---------------------------------------------------------------- scalar glue
inline double value(double x) { return x; }
inline double Sqrt(double x) { return std::sqrt(x); }

template <class T> inline T Abs(const T& x) {
  BranchLog::note(value(x) < 0.0);
  return value(x) < 0.0 ? -x : x;
}
template <class T> inline T Min(const T& a, const T& b) {
  BranchLog::note(value(b) < value(a));
  return value(b) < value(a) ? b : a;
}
template <class T> inline T Max(const T& a, const T& b) {
  BranchLog::note(value(b) > value(a));
  return value(b) > value(a) ? b : a;
}

// Path counts of the HLLD evaluations, for tests that must show which
// branches a run reached (off unless enabled): [0] evaluations, [1] one side's
// outer star state degenerate, [2] inner (double-star) states evaluated,
// [3] inner states degenerate.
struct HlldStats {
  static bool& on() {
    static bool v = false;
    return v;
  }
  static std::atomic<long long>* counts() {
    static std::atomic<long long> c[4];
    return c;
  }
  static void add(int k) {
    if (on()) counts()[k].fetch_add(1, std::memory_order_relaxed);
  }
};

// Primitive slots (lab frame) and conserved slots share indices 0..7:
//   W = (rho, vx, vy, vz, p, Bx, By, Bz),  U = (rho, mx, my, mz, E, Bx, By, Bz).
enum { RHO = 0, VX = 1, PRS = 4, BXS = 5 };
enum { NVAR = 8 };

// minmod(a, b): zero if a*b <= 0, else the argument of smaller magnitude
// (slope limiter of the MUSCL reconstruction).  On |a| == |b| it returns a.
template <class T> inline T minmod(const T& a, const T& b) {
  if (value(a) * value(b) <= 0.0) {
    BranchLog::note(0);
    return T(0.0);
  }
  const bool pick_b = std::fabs(value(b)) < std::fabs(value(a));
  BranchLog::note(pick_b ? 2 : 1);
  return pick_b ? b : a;
}

// Conserved from primitive: m = rho v, E = p/(gamma-1) + rho|v|^2/2 + |B|^2/2
// (magnetic pressure |B|^2/2, i.e. units with the 4 pi absorbed in B).
template <class T> inline void prim_to_cons(const T* W, T* U, double gamma) {
  U[0] = W[0];
  U[1] = W[0] * W[1];
  U[2] = W[0] * W[2];
  U[3] = W[0] * W[3];
  T ke = 0.5 * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
  T me = 0.5 * (W[5] * W[5] + W[6] * W[6] + W[7] * W[7]);
  U[4] = W[4] / (gamma - 1.0) + ke + me;
  U[5] = W[5];
  U[6] = W[6];
  U[7] = W[7];
}

// Primitive from conserved: v = m/rho, p = (gamma-1)(E - rho|v|^2/2 - |B|^2/2).
template <class T> inline void cons_to_prim(const T* U, T* W, double gamma) {
  W[0] = U[0];
  W[1] = U[1] / U[0];
  W[2] = U[2] / U[0];
  W[3] = U[3] / U[0];
  T ke = 0.5 * U[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
  T me = 0.5 * (U[5] * U[5] + U[6] * U[6] + U[7] * U[7]);
  W[4] = (gamma - 1.0) * (U[4] - ke - me);
  W[5] = U[5];
  W[6] = U[6];
  W[7] = U[7];
}

// Ideal-MHD physical flux in lab direction d of the primitive state W.
// F(rho) = rho v_d; F(m_a) = rho v_d v_a + delta_ad pT - B_d B_a;
// F(E) = (E + pT) v_d - B_d (v.B); F(B_a) = B_a v_d - B_d v_a (zero for a = d).
template <class T> inline void phys_flux(const T* W, int d, double gamma, T* F) {
  T U[NVAR];
  prim_to_cons(W, U, gamma);
  const T& r = W[0];
  const T* v = W + 1;
  const T* B = W + 5;
  T pT = W[4] + 0.5 * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
  T vB = v[0] * B[0] + v[1] * B[1] + v[2] * B[2];
  F[0] = r * v[d];
  for (int a = 0; a < 3; ++a) F[1 + a] = r * v[d] * v[a] - B[d] * B[a];
  F[1 + d] = F[1 + d] + pT;
  F[4] = (U[4] + pT) * v[d] - B[d] * vB;
  for (int a = 0; a < 3; ++a) F[5 + a] = B[a] * v[d] - B[d] * v[a];
  F[5 + d] = T(0.0);
}

// Fast magnetosonic speed along direction with normal field Bn:
// c_f^2 = ( (gamma p + |B|^2)/rho + sqrt( ((gamma p + |B|^2)/rho)^2 - 4 gamma p Bn^2 / rho^2 ) ) / 2.
template <class T> inline T fast_speed(const T& rho, const T& p, const T& B2, const T& Bn, double gamma) {
  T a = (gamma * p + B2) / rho;
  T disc = a * a - 4.0 * gamma * p * Bn * Bn / (rho * rho);
  BranchLog::note(value(disc) < 0.0);
  if (value(disc) < 0.0) disc = T(0.0);
  return Sqrt(0.5 * (a + Sqrt(disc)));
}

// Cyclic frame of direction d: (n, t1, t2) = (d, d+1, d+2) mod 3.
inline int tdir(int d, int k) { return (d + k) % 3; }

// Branch record of one HLLD evaluation (used by tests to report which
// region / degeneracy path a face took).
struct HlldInfo {
  int region = 0;  // 0: F_L, 1: F*_L, 2: F**_L, 3: F**_R, 4: F*_R, 5: F_R
  bool degen_star_L = false, degen_star_R = false, degen_dstar = false;
};

// HLLD approximate Riemann solver of Miyoshi & Kusano (2005), written from
// their equations.  Inputs are rotated primitive states
//   (rho, u_n, u_t1, u_t2, p, B_n, B_t1, B_t2)
// with the same B_n on both sides.  Output: 7 flux components
//   (rho, m_n, m_t1, m_t2, E, B_t1, B_t2).
// Wave speeds: S_L = min(u_L,u_R) - max(cf_L,cf_R), S_R = max(u_L,u_R) + max(cf_L,cf_R).
// Degenerate single-star (|D| <= 1e-12 pT*) keeps tangential v, B; degenerate
// double-star (Bn^2/2 <= 1e-12 pT*) sets U** = U*.
template <class T>
inline void hlld(const T* L, const T* R, double gamma, T* F, HlldInfo* info = nullptr) {
  const T& Bn = L[5];
  T rL = L[0], uL = L[1], vL = L[2], wL = L[3], pL = L[4], byL = L[6], bzL = L[7];
  T rR = R[0], uR = R[1], vR = R[2], wR = R[3], pR = R[4], byR = R[6], bzR = R[7];

  T B2L = Bn * Bn + byL * byL + bzL * bzL;
  T B2R = Bn * Bn + byR * byR + bzR * bzR;
  T ptL = pL + 0.5 * B2L;
  T ptR = pR + 0.5 * B2R;
  T EL = pL / (gamma - 1.0) + 0.5 * rL * (uL * uL + vL * vL + wL * wL) + 0.5 * B2L;
  T ER = pR / (gamma - 1.0) + 0.5 * rR * (uR * uR + vR * vR + wR * wR) + 0.5 * B2R;

  T cfL = fast_speed(rL, pL, B2L, Bn, gamma);
  T cfR = fast_speed(rR, pR, B2R, Bn, gamma);
  T cmax = Max(cfL, cfR);
  T SL = Min(uL, uR) - cmax;
  T SR = Max(uL, uR) + cmax;

  // Physical fluxes of the two states (rotated, 7 components).
  auto pflux = [&](const T& r, const T& u, const T& v, const T& w, const T& pt, const T& E,
                   const T& by, const T& bz, T* f) {
    T vB = u * Bn + v * by + w * bz;
    f[0] = r * u;
    f[1] = r * u * u + pt - Bn * Bn;
    f[2] = r * u * v - Bn * by;
    f[3] = r * u * w - Bn * bz;
    f[4] = (E + pt) * u - Bn * vB;
    f[5] = by * u - Bn * v;
    f[6] = bz * u - Bn * w;
  };
  T FL[7], FR[7];
  pflux(rL, uL, vL, wL, ptL, EL, byL, bzL, FL);
  pflux(rR, uR, vR, wR, ptR, ER, byR, bzR, FR);

  HlldInfo inf;
  HlldStats::add(0);
  BranchLog::note(10 + (value(SL) > 0.0));
  if (value(SL) > 0.0) {  // whole fan moves right: upwind flux is F_L
    for (int c = 0; c < 7; ++c) F[c] = FL[c];
    inf.region = 0;
    if (info) *info = inf;
    return;
  }

  // Contact speed and star total pressure.
  T dL = SL - uL, dR = SR - uR;
  T SM = (dR * rR * uR - dL * rL * uL - ptR + ptL) / (dR * rR - dL * rL);
  T pts = ptL + rL * dL * (SM - uL);

  // Outer star states (one side at a time).
  struct Star { T r, v, w, by, bz, E; };
  auto star = [&](const T& r, const T& u, const T& v, const T& w, const T& pt, const T& E,
                  const T& by, const T& bz, const T& S, bool& degen) {
    Star s;
    T dS = S - u;
    T dSM = S - SM;
    s.r = r * dS / dSM;
    T D = r * dS * dSM - Bn * Bn;
    degen = std::fabs(value(D)) <= 1e-12 * value(pts);
    BranchLog::note(20 + degen);
    if (degen) {
      s.v = v; s.w = w; s.by = by; s.bz = bz;
    } else {
      T fv = Bn * (SM - u) / D;
      s.v = v - by * fv;
      s.w = w - bz * fv;
      T fb = (r * dS * dS - Bn * Bn) / D;
      s.by = by * fb;
      s.bz = bz * fb;
    }
    T vB = u * Bn + v * by + w * bz;
    T vBs = SM * Bn + s.v * s.by + s.w * s.bz;
    s.E = (dS * E - pt * u + pts * SM + Bn * (vB - vBs)) / dSM;
    return s;
  };
  bool dgL = false, dgR = false;
  Star sL = star(rL, uL, vL, wL, ptL, EL, byL, bzL, SL, dgL);
  Star sR = star(rR, uR, vR, wR, ptR, ER, byR, bzR, SR, dgR);
  inf.degen_star_L = dgL;
  inf.degen_star_R = dgR;
  if (dgL || dgR) HlldStats::add(1);

  T sqL = Sqrt(sL.r), sqR = Sqrt(sR.r);
  T SLs = SM - Abs(Bn) / sqL;
  T SRs = SM + Abs(Bn) / sqR;

  // Conserved 7-vectors.
  auto consv = [&](const T& r, const T& u, const T& v, const T& w, const T& E, const T& by,
                   const T& bz, T* q) {
    q[0] = r; q[1] = r * u; q[2] = r * v; q[3] = r * w; q[4] = E; q[5] = by; q[6] = bz;
  };
  T UL[7], UR[7], UsL[7], UsR[7];
  consv(rL, uL, vL, wL, EL, byL, bzL, UL);
  consv(rR, uR, vR, wR, ER, byR, bzR, UR);
  consv(sL.r, SM, sL.v, sL.w, sL.E, sL.by, sL.bz, UsL);
  consv(sR.r, SM, sR.v, sR.w, sR.E, sR.by, sR.bz, UsR);

  // F*_a = F_a + S_a (U*_a - U_a).
  T FsL[7], FsR[7];
  for (int c = 0; c < 7; ++c) {
    FsL[c] = FL[c] + SL * (UsL[c] - UL[c]);
    FsR[c] = FR[c] + SR * (UsR[c] - UR[c]);
  }

  // Region cascade (first true test wins): S*_L >= 0 -> F*_L; S_M >= 0 -> F**_L;
  // S*_R >= 0 -> F**_R; S_R >= 0 -> F*_R; otherwise F_R.
  BranchLog::note(30 + (value(SLs) >= 0.0) + 2 * (value(SM) >= 0.0) + 4 * (value(SRs) >= 0.0) +
                  8 * (value(SR) >= 0.0));
  if (value(SLs) >= 0.0) {
    for (int c = 0; c < 7; ++c) F[c] = FsL[c];
    inf.region = 1;
    if (info) *info = inf;
    return;
  }
  if (!(value(SM) >= 0.0) && !(value(SRs) >= 0.0)) {
    if (value(SR) >= 0.0) {
      for (int c = 0; c < 7; ++c) F[c] = FsR[c];
      inf.region = 4;
    } else {
      for (int c = 0; c < 7; ++c) F[c] = FR[c];
      inf.region = 5;
    }
    if (info) *info = inf;
    return;
  }

  // Inner (double-star) states.
  T UssL[7], UssR[7];
  bool dd = 0.5 * value(Bn) * value(Bn) <= 1e-12 * value(pts);
  BranchLog::note(50 + dd);
  inf.degen_dstar = dd;
  HlldStats::add(2);
  if (dd) HlldStats::add(3);
  if (dd) {
    for (int c = 0; c < 7; ++c) { UssL[c] = UsL[c]; UssR[c] = UsR[c]; }
  } else {
    double sg = value(Bn) > 0.0 ? 1.0 : -1.0;
    T inv = 1.0 / (sqL + sqR);
    T vss = (sqL * sL.v + sqR * sR.v + (sR.by - sL.by) * sg) * inv;
    T wss = (sqL * sL.w + sqR * sR.w + (sR.bz - sL.bz) * sg) * inv;
    T byss = (sqL * sR.by + sqR * sL.by + sqL * sqR * (sR.v - sL.v) * sg) * inv;
    T bzss = (sqL * sR.bz + sqR * sL.bz + sqL * sqR * (sR.w - sL.w) * sg) * inv;
    T vBss = SM * Bn + vss * byss + wss * bzss;
    T vBsL = SM * Bn + sL.v * sL.by + sL.w * sL.bz;
    T vBsR = SM * Bn + sR.v * sR.by + sR.w * sR.bz;
    T EssL = sL.E - sqL * (vBsL - vBss) * sg;
    T EssR = sR.E + sqR * (vBsR - vBss) * sg;
    consv(sL.r, SM, vss, wss, EssL, byss, bzss, UssL);
    consv(sR.r, SM, vss, wss, EssR, byss, bzss, UssR);
  }
  if (value(SM) >= 0.0) {
    for (int c = 0; c < 7; ++c) F[c] = FsL[c] + SLs * (UssL[c] - UsL[c]);
    inf.region = 2;
  } else {
    for (int c = 0; c < 7; ++c) F[c] = FsR[c] + SRs * (UssR[c] - UsR[c]);
    inf.region = 3;
  }
  if (info) *info = inf;
}

// ------------------------------------------------------------ grid storage
// A patch: interior n[d] cells per axis, band g (ghost width) on the active
// axes.  Cells are indexed c in [-g, n+g); the face with index f along axis d
// sits between cells f-1 and f, f in [-g, n+g].  Inactive axes (z in 2D) have
// n = 1 and no band.  In 2D the third field Bz is cell-centred.
struct Layout {
  int ndim = 3;
  int n[3] = {1, 1, 1};
  int g = 0;
  int gd(int d) const { return d < ndim ? g : 0; }
  int ext(int d) const { return n[d] + 2 * gd(d); }
  // extents of the array of field slot s (0..7): cells, or faces along s-5
  int fext(int s, int d) const {
    bool face = s >= 5 && (s - 5) < ndim && (s - 5) == d;
    return ext(d) + (face ? 1 : 0);
  }
  size_t fsize(int s) const { return (size_t)fext(s, 0) * fext(s, 1) * fext(s, 2); }
  size_t idx(int s, int i, int j, int k) const {
    return ((size_t)(k + gd(2)) * fext(s, 1) + (size_t)(j + gd(1))) * fext(s, 0) + (size_t)(i + gd(0));
  }
  bool is_face(int s) const { return s >= 5 && (s - 5) < ndim; }
};

template <class T> struct State {
  Layout L;
  std::vector<T> f[NVAR];  // rho, mx, my, mz, E (cells); Bx, By, Bz (faces; Bz cells in 2D)
  State() {}
  explicit State(const Layout& l) : L(l) {
    for (int s = 0; s < NVAR; ++s) f[s].assign(L.fsize(s), T(0.0));
  }
  T& at(int s, int i, int j, int k) { return f[s][L.idx(s, i, j, k)]; }
  const T& at(int s, int i, int j, int k) const { return f[s][L.idx(s, i, j, k)]; }
};

// Index box [lo, hi) in the patch's index space (per axis).
struct Range {
  int lo[3], hi[3];
};

// Cell-centred B: the mean of the two bounding faces on active axes; in 2D
// Bz is already cell-centred.
template <class T> inline T bcell(const State<T>& S, int a, int i, int j, int k) {
  if (a < S.L.ndim) {
    int ii = i + (a == 0), jj = j + (a == 1), kk = k + (a == 2);
    return 0.5 * (S.at(5 + a, i, j, k) + S.at(5 + a, ii, jj, kk));
  }
  return S.at(5 + a, i, j, k);
}

// Edge EMF of the constrained-transport update: 0 the arithmetic mean of the
// four adjacent face values (Balsara & Spicer 1999); 1 the upwinded form of
// Gardiner & Stone (2005, J. Comput. Phys. 205, 509), which adds to that mean
// the differences between face values and a cell-centred reference EMF,
// each taken on the upwind side of the mass flux through the face it starts
// from.
struct StepParams {
  double gamma;
  double dx[3];
  int emf;
};

// Process-wide EMF choice of the oracle's drivers (set from the C API).
inline int& emf_mode() {
  static int m = 0;
  return m;
}

// Error raised when a cell reaches non-positive density or pressure.
struct NonPhysical : std::runtime_error {
  using std::runtime_error::runtime_error;
};

// Face fluxes (lab-frame slots, stored at the high-side cell of each face,
// one array per direction) and edge EMFs (one array per edge axis, stored at
// the high-side cell in the two other axes) of one step, for the
// synchronisation of AMR levels.  Same cell indexing as the patch.
template <class T> struct StepCapture {
  std::vector<T> flux;  // [d][cell][slot]
  std::vector<T> emf;   // [a][cell]
  size_t ncell = 0;
  int ex[3] = {1, 1, 1}, g[3] = {0, 0, 0};
  size_t cid(int i, int j, int k) const {
    return ((size_t)(k + g[2]) * ex[1] + (size_t)(j + g[1])) * ex[0] + (size_t)(i + g[0]);
  }
  const T& F(int d, int slot, int i, int j, int k) const { return flux[((size_t)d * ncell + cid(i, j, k)) * NVAR + slot]; }
  const T& E(int a, int i, int j, int k) const { return emf[(size_t)a * ncell + cid(i, j, k)]; }
};

// ---------------------------------------------------------------- one step
// One unsplit MUSCL-Hancock / HLLD / CT step on a patch whose input is valid
// on cells [-gv, n+gv) and faces [-gv, n+gv].  Output is written on cells
// [-gv+2, n+gv-2) and on faces with normal index in [-gv+2, n+gv-2] (transverse
// cells in [-gv+2, n+gv-2)); everything else in `out` is copied from `in`.
// The steps follow the scheme in order:
//   (1) primitives and cell-centred B, (2) minmod slopes of the 7 primitives
//   other than the normal field, (3) face states W +- dW/2 with the normal B
//   taken from the face, (4) Hancock increment dU = -dt/2 sum_d
//   [F_d(W_{d+}) - F_d(W_{d-})]/dx_d added to U(W_{d+-}), (5) HLLD on every
//   face with B_n the time-n face value, (6) edge EMFs as the arithmetic mean
//   of the four adjacent face values, (7) conservative update of cells and CT
//   update of faces.
template <class T>
void step(const State<T>& in, State<T>& out, int gv, T dt, const StepParams& P, StepCapture<T>* cap = nullptr) {
  const Layout& L = in.L;
  const int nd = L.ndim;
  const double gamma = P.gamma;
  if (gv < 2 || gv > L.g) throw std::runtime_error("step: band too narrow");
  const bool OMP_OK = OmpSafe<T>::value && !BranchLog::on();
  (void)OMP_OK;
  out = in;

  auto lo = [&](int d, int w) { return d < nd ? -gv + w : 0; };
  auto hi = [&](int d, int w) { return d < nd ? L.n[d] + gv - w : L.n[d]; };
  const int ex[3] = {L.ext(0), L.ext(1), L.ext(2)};
  const int g0 = L.gd(0), g1 = L.gd(1), g2 = L.gd(2);
  auto cid = [&](int i, int j, int k) {
    return ((size_t)(k + g2) * ex[1] + (size_t)(j + g1)) * ex[0] + (size_t)(i + g0);
  };
  const size_t ncell = (size_t)ex[0] * ex[1] * ex[2];

  int bad = 0;  // set when a cell has non-positive density or pressure

  // (1) primitives on [-gv, n+gv).
  std::vector<T> W((size_t)NVAR * ncell, T(0.0));
#pragma omp parallel for collapse(2) reduction(| : bad) if (OMP_OK)
  for (int k = lo(2, 0); k < hi(2, 0); ++k)
    for (int j = lo(1, 0); j < hi(1, 0); ++j)
      for (int i = lo(0, 0); i < hi(0, 0); ++i) {
        T U[NVAR];
        for (int s = 0; s < 5; ++s) U[s] = in.at(s, i, j, k);
        for (int a = 0; a < 3; ++a) U[5 + a] = bcell(in, a, i, j, k);
        T* w = &W[NVAR * cid(i, j, k)];
        cons_to_prim(U, w, gamma);
        if (value(w[0]) <= 0.0 || value(w[4]) <= 0.0) bad = 1;
      }

  // (2)-(4) slopes, face states, Hancock predictor on [-gv+1, n+gv-1).
  // Pred[(d*2+side)*ncell + c] holds the predicted primitive face state.
  std::vector<T> Pred((size_t)nd * 2 * NVAR * ncell, T(0.0));
  // upwinded EMF only: reference EMF -v x B with v of the half-step cell
  // state U + dU (dU the Hancock increment) and the cell-centred B at time n,
  // one array per component
  const bool gs = P.emf == 1 || P.emf == 2;  // 2: the same with the upwind side swapped (planted mistake, tests only)
  std::vector<T> Ecc(gs ? (size_t)3 * ncell : 0, T(0.0));
#pragma omp parallel for collapse(2) reduction(| : bad) if (OMP_OK)
  for (int k = lo(2, 1); k < hi(2, 1); ++k)
    for (int j = lo(1, 1); j < hi(1, 1); ++j)
      for (int i = lo(0, 1); i < hi(0, 1); ++i) {
        const T* w = &W[NVAR * cid(i, j, k)];
        T face[3][2][NVAR];
        for (int d = 0; d < nd; ++d) {
          int di = d == 0, dj = d == 1, dk = d == 2;
          const T* wm = &W[NVAR * cid(i - di, j - dj, k - dk)];
          const T* wp = &W[NVAR * cid(i + di, j + dj, k + dk)];
          for (int q = 0; q < NVAR; ++q) {
            T dq = (q == 5 + d) ? T(0.0) : minmod(w[q] - wm[q], wp[q] - w[q]);
            face[d][0][q] = w[q] - 0.5 * dq;
            face[d][1][q] = w[q] + 0.5 * dq;
          }
          face[d][0][5 + d] = in.at(5 + d, i, j, k);
          face[d][1][5 + d] = in.at(5 + d, i + di, j + dj, k + dk);
        }
        T dU[NVAR];
        for (int q = 0; q < NVAR; ++q) dU[q] = T(0.0);
        for (int d = 0; d < nd; ++d) {
          T Fm[NVAR], Fp[NVAR];
          phys_flux(face[d][0], d, gamma, Fm);
          phys_flux(face[d][1], d, gamma, Fp);
          for (int q = 0; q < NVAR; ++q) dU[q] = dU[q] - (0.5 * dt) * (Fp[q] - Fm[q]) / P.dx[d];
        }
        if (gs) {
          T Uc[NVAR];
          prim_to_cons(w, Uc, gamma);
          for (int q = 0; q < NVAR; ++q) Uc[q] = Uc[q] + dU[q];
          const T ir = 1.0 / Uc[0];
          const T vx = Uc[1] * ir, vy = Uc[2] * ir, vz = Uc[3] * ir;
          // B at time n: the face Riemann problems take their normal field at
          // time n, so for grid-aligned flow this is the EMF they return
          const T bx = w[5], by = w[6], bz = w[7];
          Ecc[0 * ncell + cid(i, j, k)] = vz * by - vy * bz;
          Ecc[1 * ncell + cid(i, j, k)] = vx * bz - vz * bx;
          Ecc[2 * ncell + cid(i, j, k)] = vy * bx - vx * by;
        }
        for (int d = 0; d < nd; ++d)
          for (int side = 0; side < 2; ++side) {
            T U[NVAR];
            prim_to_cons(face[d][side], U, gamma);
            for (int q = 0; q < NVAR; ++q) U[q] = U[q] + dU[q];
            T* wb = &Pred[((size_t)(d * 2 + side) * ncell + cid(i, j, k)) * NVAR];
            cons_to_prim(U, wb, gamma);
            if (value(wb[0]) <= 0.0 || value(wb[4]) <= 0.0) bad = 1;
          }
      }

  if (bad) throw NonPhysical("non-positive density or pressure");
  StepMark<T>::mark(1);

  // (5) HLLD fluxes.  Flux[d] at face index f (between cells f-1 and f along
  // d) is stored at the cell index of its high-side cell.  Lab-frame slots.
  std::vector<T> Flux((size_t)nd * NVAR * ncell, T(0.0));
  for (int d = 0; d < nd; ++d) {
    int di = d == 0, dj = d == 1, dk = d == 2;
    int flo[3], fhi[3];
    for (int a = 0; a < 3; ++a) {
      flo[a] = lo(a, 1);
      fhi[a] = hi(a, 1);
    }
    flo[d] = -gv + 2;
    fhi[d] = L.n[d] + gv - 1;  // face index <= n+gv-2
#pragma omp parallel for collapse(2) if (OMP_OK)
    for (int k = flo[2]; k < fhi[2]; ++k)
      for (int j = flo[1]; j < fhi[1]; ++j)
        for (int i = flo[0]; i < fhi[0]; ++i) {
          const T* wl = &Pred[((size_t)(d * 2 + 1) * ncell + cid(i - di, j - dj, k - dk)) * NVAR];
          const T* wr = &Pred[((size_t)(d * 2 + 0) * ncell + cid(i, j, k)) * NVAR];
          T Bn = in.at(5 + d, i, j, k);
          T rl[NVAR], rr[NVAR];
          for (int c = 0; c < 3; ++c) {
            int a = tdir(d, c);
            rl[1 + c] = wl[1 + a];
            rr[1 + c] = wr[1 + a];
            rl[5 + c] = wl[5 + a];
            rr[5 + c] = wr[5 + a];
          }
          rl[0] = wl[0]; rr[0] = wr[0];
          rl[4] = wl[4]; rr[4] = wr[4];
          rl[5] = Bn; rr[5] = Bn;
          T fr[7];
          hlld(rl, rr, gamma, fr);
          T* F = &Flux[((size_t)d * ncell + cid(i, j, k)) * NVAR];
          F[0] = fr[0];
          F[4] = fr[4];
          for (int c = 0; c < 3; ++c) F[1 + tdir(d, c)] = fr[1 + c];
          F[5 + d] = T(0.0);
          F[5 + tdir(d, 1)] = fr[5];
          F[5 + tdir(d, 2)] = fr[6];
        }
  }
  StepMark<T>::mark(2);
  auto FX = [&](int d, int s, int i, int j, int k) -> const T& {
    return Flux[((size_t)d * ncell + cid(i, j, k)) * NVAR + s];
  };

  // (6) EMFs.  The face EMF of a flux through an x-face is E_z = -F_x(By),
  // E_y = +F_x(Bz); y-face: E_x = -F_y(Bz), E_z = +F_y(Bx); z-face: E_y = -F_z(Bx),
  // E_x = +F_z(By).  Edge a at (high-side cell index) averages four faces.
  std::vector<T> Emf((size_t)3 * ncell, T(0.0));
  auto EM = [&](int a, int i, int j, int k) -> T& { return Emf[(size_t)a * ncell + cid(i, j, k)]; };
  // 3D edge E_a lies along axis a; it touches faces normal to b and c (the
  // two other axes).  Its index is the high-side cell in b and c.
  for (int a = 0; a < 3; ++a) {
    if (nd == 2 && a != 2) continue;
    int b = (a + 1) % 3, c = (a + 2) % 3;
    int elo[3], ehi[3];
    for (int x = 0; x < 3; ++x) {
      elo[x] = lo(x, 1);
      ehi[x] = hi(x, 1);
    }
    elo[b] = b < nd ? -gv + 2 : 0;
    ehi[b] = b < nd ? L.n[b] + gv - 1 : L.n[b];
    elo[c] = c < nd ? -gv + 2 : 0;
    ehi[c] = c < nd ? L.n[c] + gv - 1 : L.n[c];
#pragma omp parallel for collapse(2) if (OMP_OK)
    for (int k = elo[2]; k < ehi[2]; ++k)
      for (int j = elo[1]; j < ehi[1]; ++j)
        for (int i = elo[0]; i < ehi[0]; ++i) {
          int e[3] = {i, j, k};
          // faces normal to b: at b-index e[b], c-index e[c]-1 and e[c]
          // E_a from a b-face flux: rotated frame of b is (b, c, a) so E_a = -F_b(B_c).
          // E_a from a c-face flux: rotated frame of c is (c, a, b) so E_a = +F_c(B_b).
          int m1[3] = {i, j, k};
          m1[c] -= 1;
          int m2[3] = {i, j, k};
          m2[b] -= 1;
          T s1 = -FX(b, 5 + c, m1[0], m1[1], m1[2]) - FX(b, 5 + c, e[0], e[1], e[2]);
          T s2 = FX(c, 5 + b, m2[0], m2[1], m2[2]) + FX(c, 5 + b, e[0], e[1], e[2]);
          if (!gs) {
            EM(a, i, j, k) = 0.25 * (s1 + s2);
            continue;
          }
          // Gardiner & Stone: with b the first and c the second transverse
          // axis, face values bS, bN (b-faces below / above the edge in c),
          // cW, cE (c-faces below / above in b), reference EMFs of the four
          // cells around the edge, and four half-cell differences along b or
          // c, each taken on the upwind side of the mass flux through the face
          // it starts from (their mean when that flux is zero).
          const T bS = -FX(b, 5 + c, m1[0], m1[1], m1[2]), bN = -FX(b, 5 + c, e[0], e[1], e[2]);
          const T cW = FX(c, 5 + b, m2[0], m2[1], m2[2]), cE = FX(c, 5 + b, e[0], e[1], e[2]);
          int sw[3] = {i, j, k};
          sw[b] -= 1;
          sw[c] -= 1;
          auto ER = [&](const int (&q)[3]) -> T { return Ecc[(size_t)a * ncell + cid(q[0], q[1], q[2])]; };
          const T eSW = ER(sw), eSE = ER(m1), eNW = ER(m2), eNE = ER(e);
          const bool swap = P.emf == 2;
          auto upw = [swap](T flux, T up_low, T up_high) -> T {
            if (swap) std::swap(up_low, up_high);
            if (value(flux) > 0.0) return up_low;
            if (value(flux) < 0.0) return up_high;
            return 0.5 * (up_low + up_high);
          };
          // along c, between the edge and the b-face above it (mass flux of
          // that face along b picks the low or high side in b), and below
          const T dc_hi = upw(FX(b, 0, e[0], e[1], e[2]), eNW - cW, eNE - cE);
          const T dc_lo = upw(FX(b, 0, m1[0], m1[1], m1[2]), cW - eSW, cE - eSE);
          // along b, between the edge and the c-face to its high side, and low
          const T db_hi = upw(FX(c, 0, e[0], e[1], e[2]), eSE - bS, eNE - bN);
          const T db_lo = upw(FX(c, 0, m2[0], m2[1], m2[2]), bS - eSW, bN - eNW);
          EM(a, i, j, k) = 0.25 * (s1 + s2) + 0.25 * ((dc_lo - dc_hi) + (db_lo - db_hi));
        }
  }

  StepMark<T>::mark(3);
  // (7) update cells [-gv+2, n+gv-2).
  const int ncons = nd == 2 ? 6 : 5;  // in 2D Bz (slot 7) is a cell quantity
#pragma omp parallel for collapse(2) if (OMP_OK)
  for (int k = lo(2, 2); k < hi(2, 2); ++k)
    for (int j = lo(1, 2); j < hi(1, 2); ++j)
      for (int i = lo(0, 2); i < hi(0, 2); ++i) {
        for (int q = 0; q < ncons; ++q) {
          int s = q < 5 ? q : 7;
          T acc = T(0.0);
          for (int d = 0; d < nd; ++d) {
            int di = d == 0, dj = d == 1, dk = d == 2;
            acc = acc + (FX(d, s, i + di, j + dj, k + dk) - FX(d, s, i, j, k)) / P.dx[d];
          }
          out.at(s, i, j, k) = in.at(s, i, j, k) - dt * acc;
        }
      }
  // Faces: dB/dt = -curl E.
  for (int d = 0; d < nd; ++d) {
    int b = (d + 1) % 3, c = (d + 2) % 3;
    int flo[3], fhi[3];
    for (int x = 0; x < 3; ++x) {
      flo[x] = lo(x, 2);
      fhi[x] = hi(x, 2);
    }
    flo[d] = -gv + 2;
    fhi[d] = L.n[d] + gv - 1;
#pragma omp parallel for collapse(2) if (OMP_OK)
    for (int k = flo[2]; k < fhi[2]; ++k)
      for (int j = flo[1]; j < fhi[1]; ++j)
        for (int i = flo[0]; i < fhi[0]; ++i) {
          // (curl E)_d = d_b E_c - d_c E_b.  E_c is indexed by its high-side
          // cell in d and b; E_b by its high-side cell in c and d.
          T curl = T(0.0);
          if (b < nd) {
            int p[3] = {i, j, k};
            p[b] += 1;
            curl = curl + (EM(c, p[0], p[1], p[2]) - EM(c, i, j, k)) / P.dx[b];
          }
          if (c < nd) {
            int p[3] = {i, j, k};
            p[c] += 1;
            curl = curl - (EM(b, p[0], p[1], p[2]) - EM(b, i, j, k)) / P.dx[c];
          }
          out.at(5 + d, i, j, k) = in.at(5 + d, i, j, k) - dt * curl;
        }
  }
  if (cap) {
    cap->flux = std::move(Flux);
    cap->emf = std::move(Emf);
    cap->ncell = ncell;
    for (int a = 0; a < 3; ++a) {
      cap->ex[a] = ex[a];
      cap->g[a] = L.gd(a);
    }
  }
}

}  // namespace orc
