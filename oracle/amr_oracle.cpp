// FP64 oracle of the multilevel cycle with extended ghost zones (test
// infrastructure only; the product library never uses it).
//
// The paper's level cycle (Sec. 4, Threaded Multilevel Advance) visits the
// levels in the order 0, 1, 2, 2, 1, 2, 2 for three levels and applies
// (P)rolongation, (A)dvance, (S)ynchronisation and (R)estriction; grids are
// regular arrays of cells nested in coarser grids with dx_{l-1} = R dx_l
// (Sec. 2); extended ghost zones let each level advance on its own (Sec. 1,
// abstract).  This file runs that cycle serially, one grid at a time:
//   cycle(l): FULL fill of level l+1 from level l; advance level l; then R
//             times { SAME_LEVEL refill of level l+1 if k > 0; cycle(l+1) };
//             synchronise level l+1 into level l.
// Ghost fill: a band element that lies in (cells) or on the boundary of
// (faces) a same-level interior takes that value (lowest grid id), periodic
// images included; otherwise (FULL fill above level 0) it is prolonged from
// level l-1: cells by minmod-limited linear reconstruction of the conserved
// variables, faces by the divergence-free reconstruction of Balsara (2001).
// Synchronisation: reflux of uncovered coarse cells on coarse/fine faces,
// EMF correction of uncovered coarse faces on coarse/fine edges, then
// restriction (mean) of fine cells and faces into covered coarse data.
// Coarse data are read through level-wide lookups (owner grid of each
// position), never through another grid's band.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>
#include <unordered_map>
#include <vector>

#include "scheme.hpp"

namespace orc {
namespace {

thread_local std::string a_err;
int g_skip = 0;  // planted omissions for sensitivity tests: 1 reflux, 2 EMF fix, 4 restriction

int ipow(int b, int e) {
  int r = 1;
  while (e-- > 0) r *= b;
  return r;
}
int fdiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
int pmod(int a, int b) { return ((a % b) + b) % b; }

struct Grid {
  int level;
  int lo[3], hi[3];
  State<double> S;
  StepCapture<double> coarse_cap;             // last step (as the coarse side of a sync)
  std::vector<StepCapture<double>> fine_caps;  // substeps since the last sync (fine side)
};

struct Amr {
  int nd = 3, L = 1, R = 2, g = 4;
  int N0[3] = {1, 1, 1};
  double dx0[3] = {1, 1, 1};
  double gamma = 5.0 / 3.0, cfl = 0.4;
  std::vector<Grid> G;
  std::vector<std::vector<int>> lev;
  // cell -> grid lookup per level: grids listed under every 8^3-cell block
  // they touch (levels are sparse: a deep level spans far more cells than
  // its grids hold)
  std::vector<std::unordered_map<int64_t, std::vector<int>>> owner;
  double dt0 = 0.0;
  bool dry = false;        // record the level order only
  std::vector<int> trace;  // levels in the order they advance

  int N(int l, int a) const { return a < nd ? N0[a] * ipow(R, l) : 1; }
  double dx(int l, int a) const { return a < nd ? dx0[a] / ipow(R, l) : 1.0; }

  void wrap(int l, int (&p)[3]) const {
    for (int a = 0; a < nd; ++a) p[a] = pmod(p[a], N(l, a));
  }
  static int64_t bkey(int bx, int by, int bz) { return ((int64_t)bz << 42) | ((int64_t)by << 21) | (int64_t)bx; }
  // grid of level l whose interior holds the (already wrapped) cell p, or -1
  int owner_at(int l, const int (&p)[3]) const {
    auto it = owner[l].find(bkey(p[0] >> 3, p[1] >> 3, p[2] >> 3));
    if (it == owner[l].end()) return -1;
    for (int gi : it->second) {
      const Grid& q = G[gi];
      if (p[0] >= q.lo[0] && p[0] < q.hi[0] && p[1] >= q.lo[1] && p[1] < q.hi[1] && p[2] >= q.lo[2] &&
          p[2] < q.hi[2])
        return gi;
    }
    return -1;
  }
  // grid whose interior holds cell p of level l (periodic), or -1
  int own_cell(int l, const int (&p0)[3]) const {
    int p[3] = {p0[0], p0[1], p0[2]};
    wrap(l, p);
    return owner_at(l, p);
  }

  void build_owner() {
    owner.assign(L, {});
    for (int l = 0; l < L; ++l) {
      for (int gi : lev[l]) {
        const Grid& g0 = G[gi];
        for (int bz = g0.lo[2] >> 3; bz <= (g0.hi[2] - 1) >> 3; ++bz)
          for (int by = g0.lo[1] >> 3; by <= (g0.hi[1] - 1) >> 3; ++by)
            for (int bx = g0.lo[0] >> 3; bx <= (g0.hi[0] - 1) >> 3; ++bx) {
              std::vector<int>& v = owner[l][bkey(bx, by, bz)];
              for (int o : v) {
                const Grid& q = G[o];
                bool meet = true;
                for (int a = 0; a < 3; ++a) meet = meet && g0.lo[a] < q.hi[a] && q.lo[a] < g0.hi[a];
                if (meet) throw std::runtime_error("grids of one level overlap");
              }
              v.push_back(gi);
            }
      }
    }
  }

  // ---- level-wide accessors (owners' interiors only) ----
  double cell_value(int l, int slot, const int (&p0)[3]) const {
    int p[3] = {p0[0], p0[1], p0[2]};
    wrap(l, p);
    int o = owner_at(l, p);
    if (o < 0) throw std::runtime_error("cell lookup outside the level");
    const Grid& q = G[o];
    return q.S.at(slot, p[0] - q.lo[0], p[1] - q.lo[1], p[2] - q.lo[2]);
  }
  // face with normal d at index p (face p sits below cell p along d): value
  // from the lowest-id grid having it in its interior or on its boundary
  bool face_owner(int l, int d, const int (&p0)[3], int& o, int (&loc)[3]) const {
    int best = -1;
    int bl[3] = {0, 0, 0};
    for (int side = 0; side < 2; ++side) {
      int c[3] = {p0[0], p0[1], p0[2]};
      if (side == 1) c[d] -= 1;
      wrap(l, c);
      int w = owner_at(l, c);
      if (w < 0) continue;
      if (best < 0 || w < best) {
        best = w;
        for (int a = 0; a < 3; ++a) bl[a] = c[a] - G[w].lo[a];
        if (side == 1) bl[d] += 1;
      }
    }
    if (best < 0) return false;
    o = best;
    for (int a = 0; a < 3; ++a) loc[a] = bl[a];
    return true;
  }
  double face_value(int l, int d, const int (&p)[3]) const {
    int o, loc[3];
    if (!face_owner(l, d, p, o, loc)) throw std::runtime_error("face lookup outside the level");
    return G[o].S.at(5 + d, loc[0], loc[1], loc[2]);
  }

  bool is_face_slot(int s) const { return s >= 5 && s - 5 < nd; }

  // ---- prolongation (R = 2) ----
  double prolong_cell(int l, int slot, const int (&pf)[3]) const {
    int pc[3];
    for (int a = 0; a < 3; ++a) pc[a] = a < nd ? fdiv(pf[a], 2) : 0;
    double c = cell_value(l - 1, slot, pc);
    double v = c;
    for (int a = 0; a < nd; ++a) {
      int m[3] = {pc[0], pc[1], pc[2]}, p[3] = {pc[0], pc[1], pc[2]};
      m[a] -= 1;
      p[a] += 1;
      double sl = minmod(c - cell_value(l - 1, slot, m), cell_value(l - 1, slot, p) - c);
      v += (pmod(pf[a], 2) ? 0.25 : -0.25) * sl;
    }
    return v;
  }
  // minmod slope along axis t of the face field d at coarse face index p
  double face_slope(int l, int d, const int (&p)[3], int t) const {
    int m[3] = {p[0], p[1], p[2]}, q[3] = {p[0], p[1], p[2]};
    m[t] -= 1;
    q[t] += 1;
    double c = face_value(l, d, p);
    return minmod(c - face_value(l, d, m), face_value(l, d, q) - c);
  }
  double prolong_face(int l, int d, const int (&pf)[3]) const {
    const int cl = l - 1;
    int pc[3];
    for (int a = 0; a < 3; ++a) pc[a] = a < nd ? fdiv(pf[a], 2) : 0;
    if (pmod(pf[d], 2) == 0) {
      // fine face on a coarse face: B + sum_t (+-1/4) slope_t(B)
      int f[3] = {pc[0], pc[1], pc[2]};
      f[d] = pf[d] / 2;
      double v = face_value(cl, d, f);
      for (int t = 0; t < nd; ++t) {
        if (t == d) continue;
        v += (pmod(pf[t], 2) ? 0.25 : -0.25) * face_slope(cl, d, f, t);
      }
      return v;
    }
    // fine face inside the coarse cell pc, on its mid-plane normal to d:
    // B_d(0, eta, zeta) = a0 + sum_t a_t (+-1/2), a0 = (B+ + B-)/2 - a_dd,
    // a_t = (slope_t B+ + slope_t B-)/4,
    // a_dd = -(dx_d/2) sum_t (slope_d B_t+ - slope_d B_t-) / (4 dx_t)
    int fm[3] = {pc[0], pc[1], pc[2]}, fp[3] = {pc[0], pc[1], pc[2]};
    fp[d] += 1;
    double bm = face_value(cl, d, fm), bp = face_value(cl, d, fp);
    double add = 0.0;
    double v = 0.0;
    for (int t = 0; t < nd; ++t) {
      if (t == d) continue;
      double at = 0.25 * (face_slope(cl, d, fp, t) + face_slope(cl, d, fm, t));
      v += (pmod(pf[t], 2) ? 0.5 : -0.5) * at;
      int tm[3] = {pc[0], pc[1], pc[2]}, tp[3] = {pc[0], pc[1], pc[2]};
      tp[t] += 1;
      add += (face_slope(cl, t, tp, d) - face_slope(cl, t, tm, d)) / (4.0 * dx(cl, t));
    }
    add *= -0.5 * dx(cl, d);
    return 0.5 * (bp + bm) - add + v;
  }

  // Run body(gi) for every grid of level l, grids on separate threads (each
  // call writes only its own grid; an exception is rethrown afterwards).
  template <class Body> void per_grid(int l, Body&& body) {
    const std::vector<int>& gl = lev[l];
    std::string err;
#pragma omp parallel for schedule(dynamic, 1)
    for (int t = 0; t < (int)gl.size(); ++t) {
      try {
        body(gl[t]);
      } catch (const std::exception& e) {
#pragma omp critical
        if (err.empty()) err = e.what();
      }
    }
    if (!err.empty()) throw std::runtime_error(err);
  }

  // ---- ghost fill of level l ----
  void fill(int l, bool full) {
    if (dry) return;
    const int ncls = nd == 3 ? 4 : 3;
    per_grid(l, [&](int gi) {
      Grid& q = G[gi];
      const Layout& Lq = q.S.L;
      for (int cls = 0; cls < ncls; ++cls) {
        const int d = cls - 1;  // face normal for cls >= 1
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
          lo[a] = -Lq.gd(a);
          hi[a] = Lq.n[a] + Lq.gd(a) + ((cls >= 1 && a == d) ? 1 : 0);
        }
        for (int k = lo[2]; k < hi[2]; ++k)
          for (int j = lo[1]; j < hi[1]; ++j)
            for (int i = lo[0]; i < hi[0]; ++i) {
              int x[3] = {i, j, k};
              bool own = true;
              for (int a = 0; a < nd; ++a) {
                int top = (cls >= 1 && a == d) ? Lq.n[a] : Lq.n[a] - 1;
                if (x[a] < 0 || x[a] > top) own = false;
              }
              if (own) continue;
              int p[3] = {q.lo[0] + i, q.lo[1] + j, q.lo[2] + k};
              if (cls == 0) {
                int o = own_cell(l, p);
                int slots[6] = {0, 1, 2, 3, 4, 7};
                int ns = nd == 2 ? 6 : 5;
                if (o >= 0) {
                  for (int t = 0; t < ns; ++t) q.S.at(slots[t], i, j, k) = cell_value(l, slots[t], p);
                } else if (full && l > 0) {
                  for (int t = 0; t < ns; ++t) q.S.at(slots[t], i, j, k) = prolong_cell(l, slots[t], p);
                } else if (l == 0) {
                  throw std::runtime_error("level 0 does not cover the domain");
                }
              } else {
                int o, loc[3];
                if (face_owner(l, d, p, o, loc)) {
                  q.S.at(5 + d, i, j, k) = G[o].S.at(5 + d, loc[0], loc[1], loc[2]);
                } else if (full && l > 0) {
                  q.S.at(5 + d, i, j, k) = prolong_face(l, d, p);
                } else if (l == 0) {
                  throw std::runtime_error("level 0 does not cover the domain");
                }
              }
            }
      }
    });
  }

  // ---- time step ----
  double compute_dt() const {
    double mx = 0.0;
    for (const Grid& q : G) {
      const Layout& Lq = q.S.L;
      for (int k = 0; k < Lq.n[2]; ++k)
        for (int j = 0; j < Lq.n[1]; ++j)
          for (int i = 0; i < Lq.n[0]; ++i) {
            double U[NVAR], W[NVAR];
            for (int s = 0; s < 5; ++s) U[s] = q.S.at(s, i, j, k);
            for (int a = 0; a < 3; ++a) U[5 + a] = bcell(q.S, a, i, j, k);
            cons_to_prim(U, W, gamma);
            double B2 = W[5] * W[5] + W[6] * W[6] + W[7] * W[7];
            double acc = 0.0;
            for (int d = 0; d < nd; ++d)
              acc += (std::fabs(W[1 + d]) + fast_speed(W[0], W[4], B2, W[5 + d], gamma)) / dx0[d];
            mx = std::max(mx, acc);
          }
    }
    return cfl / mx;
  }

  // ---- advance every grid of level l at its k-th substep ----
  void advance(int l, int k) {
    trace.push_back(l);
    if (dry) return;
    const int gv = l == 0 ? g : g - 2 * (k % R);
    const double dt = dt0 / ipow(R, l);
    StepParams P{gamma, {dx(l, 0), dx(l, 1), dx(l, 2)}, emf_mode()};
    per_grid(l, [&](int gi) {
      Grid& q = G[gi];
      State<double> out(q.S.L);
      StepCapture<double> cap;
      step(q.S, out, gv, dt, P, &cap);
      q.S = std::move(out);
      if (l + 1 < L) q.coarse_cap = cap;
      if (l > 0) q.fine_caps.push_back(std::move(cap));
    });
  }

  bool covered(int c, const int (&pc)[3]) const {
    int pf[3];
    for (int a = 0; a < 3; ++a) pf[a] = a < nd ? R * pc[a] : 0;
    return own_cell(c + 1, pf) >= 0;
  }

  // mean over the R^(nd-1) fine faces on coarse face pc (normal d) of the
  // captured flux slot of fine substep k, times dt_f
  double fine_flux_sum(int f, int d, int slot, const int (&pcf)[3], int fine_grid) const {
    const Grid& q = G[fine_grid];
    const double dtf = dt0 / ipow(R, f);
    double tot = 0.0;
    for (size_t k = 0; k < q.fine_caps.size(); ++k) {
      double m = 0.0;
      int cnt = 0;
      int o1 = (d + 1) % 3, o2 = (d + 2) % 3;
      int n1 = o1 < nd ? R : 1, n2 = o2 < nd ? R : 1;
      for (int a1 = 0; a1 < n1; ++a1)
        for (int a2 = 0; a2 < n2; ++a2) {
          int p[3];
          p[d] = R * pcf[d];
          p[o1] = o1 < nd ? R * pcf[o1] + a1 : 0;
          p[o2] = o2 < nd ? R * pcf[o2] + a2 : 0;
          m += q.fine_caps[k].F(d, slot, p[0] - q.lo[0], p[1] - q.lo[1], p[2] - q.lo[2]);
          ++cnt;
        }
      tot += dtf * (m / cnt);
    }
    return tot;
  }

  // Is the coarse edge along axis a (index e: high-side cells in the two
  // other axes) a coarse/fine edge?  If so, fine_grid is the lowest-id fine
  // grid owning a covered fine cell next to it and ew the edge index in that
  // grid's periodic frame.
  bool cf_edge(int c, int a, const int (&e)[3], int& fine_grid, int (&ew)[3]) const {
    int b = (a + 1) % 3, cc = (a + 2) % 3;
    int ncov = 0, nall = 0;
    fine_grid = -1;
    for (int db = 0; db < 2; ++db)
      for (int dc = 0; dc < 2; ++dc) {
        if ((b >= nd && db) || (cc >= nd && dc)) continue;
        int p[3] = {e[0], e[1], e[2]};
        if (b < nd) p[b] -= db;
        if (cc < nd) p[cc] -= dc;
        ++nall;
        if (covered(c, p)) {
          ++ncov;
          int pf[3];
          for (int x = 0; x < 3; ++x) pf[x] = x < nd ? R * p[x] : 0;
          int pw[3] = {pf[0], pf[1], pf[2]};
          wrap(c + 1, pw);
          int o = owner_at(c + 1, pw);
          if (o >= 0 && (fine_grid < 0 || o < fine_grid)) {
            fine_grid = o;
            for (int x = 0; x < 3; ++x) ew[x] = e[x] + (pw[x] - pf[x]) / R;
          }
        }
      }
    return ncov > 0 && ncov < nall;
  }

  double fine_emf_sum(int f, int a, const int (&ec)[3], int fine_grid) const {
    const Grid& q = G[fine_grid];
    const double dtf = dt0 / ipow(R, f);
    double tot = 0.0;
    const int na = a < nd ? R : 1;
    for (size_t k = 0; k < q.fine_caps.size(); ++k) {
      double m = 0.0;
      for (int s = 0; s < na; ++s) {
        int p[3];
        for (int x = 0; x < 3; ++x) p[x] = x < nd ? R * ec[x] : 0;
        if (a < nd) p[a] += s;
        m += q.fine_caps[k].E(a, p[0] - q.lo[0], p[1] - q.lo[1], p[2] - q.lo[2]);
      }
      tot += dtf * (m / na);
    }
    return tot;
  }

  // ---- synchronisation of level f into level c = f-1 ----
  void sync(int f) {
    if (dry) return;
    const int c = f - 1;
    const double dtc = dt0 / ipow(R, c);
    const int ncs = nd == 2 ? 6 : 5;
    const int cslots[6] = {0, 1, 2, 3, 4, 7};
    // each phase writes only the coarse grid it visits: grids run on threads
    // (1) reflux of uncovered coarse cells
    if (!(g_skip & 1)) per_grid(c, [&](int gi) {
      Grid& q = G[gi];
      for (int k = 0; k < q.S.L.n[2]; ++k)
        for (int j = 0; j < q.S.L.n[1]; ++j)
          for (int i = 0; i < q.S.L.n[0]; ++i) {
            int pu[3] = {q.lo[0] + i, q.lo[1] + j, q.lo[2] + k};
            if (covered(c, pu)) continue;
            for (int d = 0; d < nd; ++d)
              for (int side = -1; side <= 1; side += 2) {
                int pv[3] = {pu[0], pu[1], pu[2]};
                pv[d] += side;
                if (!covered(c, pv)) continue;
                // face between u and v: global index pf (face below cell pf)
                int pf[3] = {pu[0], pu[1], pu[2]};
                if (side > 0) pf[d] += 1;
                int lf[3] = {pf[0] - q.lo[0], pf[1] - q.lo[1], pf[2] - q.lo[2]};
                // fine grid owning the fine cells of v next to the face
                int fc[3];
                for (int a = 0; a < 3; ++a) fc[a] = a < nd ? R * pv[a] : 0;
                if (side < 0) fc[d] += R - 1;
                int fg = own_cell(f, fc);
                // the fine faces in the frame of that fine grid (undo wrap)
                int pfw[3] = {pf[0], pf[1], pf[2]};
                {
                  int fcw[3] = {fc[0], fc[1], fc[2]};
                  wrap(f, fcw);
                  for (int a = 0; a < nd; ++a) {
                    int shift = fcw[a] - fc[a];  // multiple of N_f
                    pfw[a] = pf[a] + shift / R;
                  }
                }
                for (int t = 0; t < ncs; ++t) {
                  int s = cslots[t];
                  double delta = dtc * q.coarse_cap.F(d, s, lf[0], lf[1], lf[2]) - fine_flux_sum(f, d, s, pfw, fg);
                  q.S.at(s, i, j, k) += (side > 0 ? 1.0 : -1.0) * delta / dx(c, d);
                }
              }
          }
    });
    // (2) EMF correction of coarse faces with no covered neighbour
    if (!(g_skip & 2)) per_grid(c, [&](int gi) {
      Grid& q = G[gi];
      for (int d = 0; d < nd; ++d) {
        int lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
          lo[a] = 0;
          hi[a] = q.S.L.n[a] + ((a == d) ? 1 : 0);
        }
        for (int k = lo[2]; k < hi[2]; ++k)
          for (int j = lo[1]; j < hi[1]; ++j)
            for (int i = lo[0]; i < hi[0]; ++i) {
              int pf[3] = {q.lo[0] + i, q.lo[1] + j, q.lo[2] + k};
              int pm[3] = {pf[0], pf[1], pf[2]};
              pm[d] -= 1;
              if (covered(c, pf) || covered(c, pm)) continue;
              // (curl dE)_d = d_b dE_c - d_c dE_b, b = d+1, c = d+2
              const int b = (d + 1) % 3, cx = (d + 2) % 3;
              double corr = 0.0;
              for (int term = 0; term < 2; ++term) {
                int ea = term == 0 ? cx : b;  // edge axis
                int da = term == 0 ? b : cx;  // derivative axis
                if (da >= nd) continue;
                if (nd == 2 && ea != 2) continue;
                double sgn = term == 0 ? 1.0 : -1.0;
                for (int up = 0; up < 2; ++up) {
                  int e[3] = {pf[0], pf[1], pf[2]};
                  e[da] += up;
                  int fg = -1, ew[3] = {0, 0, 0};
                  if (!cf_edge(c, ea, e, fg, ew)) continue;
                  int le[3] = {e[0] - q.lo[0], e[1] - q.lo[1], e[2] - q.lo[2]};
                  double dE = fine_emf_sum(f, ea, ew, fg) - dtc * q.coarse_cap.E(ea, le[0], le[1], le[2]);
                  corr += sgn * (up ? 1.0 : -1.0) * dE / dx(c, da);
                }
              }
              q.S.at(5 + d, i, j, k) -= corr;
            }
      }
    });
    // (3) restriction of covered cells and of faces with a covered neighbour
    if (!(g_skip & 4)) per_grid(c, [&](int gi) {
      Grid& q = G[gi];
      for (int k = 0; k < q.S.L.n[2]; ++k)
        for (int j = 0; j < q.S.L.n[1]; ++j)
          for (int i = 0; i < q.S.L.n[0]; ++i) {
            int pc[3] = {q.lo[0] + i, q.lo[1] + j, q.lo[2] + k};
            if (!covered(c, pc)) continue;
            int pf[3];
            for (int a = 0; a < 3; ++a) pf[a] = a < nd ? R * pc[a] : 0;
            for (int t = 0; t < ncs; ++t) {
              double m = 0.0;
              int cnt = 0;
              for (int dz = 0; dz < (nd == 3 ? R : 1); ++dz)
                for (int dy = 0; dy < R; ++dy)
                  for (int dxx = 0; dxx < R; ++dxx) {
                    int p[3] = {pf[0] + dxx, pf[1] + dy, pf[2] + dz};
                    m += cell_value(f, cslots[t], p);
                    ++cnt;
                  }
              q.S.at(cslots[t], i, j, k) = m / cnt;
            }
          }
      for (int d = 0; d < nd; ++d) {
        for (int k = 0; k < q.S.L.n[2] + (d == 2 ? 1 : 0); ++k)
          for (int j = 0; j < q.S.L.n[1] + (d == 1 ? 1 : 0); ++j)
            for (int i = 0; i < q.S.L.n[0] + (d == 0 ? 1 : 0); ++i) {
              int pfc[3] = {q.lo[0] + i, q.lo[1] + j, q.lo[2] + k};
              int pm[3] = {pfc[0], pfc[1], pfc[2]};
              pm[d] -= 1;
              if (!covered(c, pfc) && !covered(c, pm)) continue;
              int o1 = (d + 1) % 3, o2 = (d + 2) % 3;
              double m = 0.0;
              int cnt = 0;
              for (int a1 = 0; a1 < (o1 < nd ? R : 1); ++a1)
                for (int a2 = 0; a2 < (o2 < nd ? R : 1); ++a2) {
                  int p[3];
                  p[d] = R * pfc[d];
                  p[o1] = o1 < nd ? R * pfc[o1] + a1 : 0;
                  p[o2] = o2 < nd ? R * pfc[o2] + a2 : 0;
                  m += face_value(f, d, p);
                  ++cnt;
                }
              q.S.at(5 + d, i, j, k) = m / cnt;
            }
      }
    });
    for (int gi : lev[f]) G[gi].fine_caps.clear();
  }

  void cycle(int l, int k) {
    if (l + 1 < L) fill(l + 1, true);
    advance(l, k);
    if (l + 1 < L) {
      for (int kk = 0; kk < R; ++kk) {
        if (kk > 0) fill(l + 1, false);
        cycle(l + 1, kk);
      }
      sync(l + 1);
    }
  }

  void coarse_step(double dt_fixed) {
    dt0 = dt_fixed > 0 ? dt_fixed : compute_dt();
    fill(0, false);
    cycle(0, 0);
  }
};

Amr* make_amr(int ndim, const int* N0, int nlev, int g, double gamma, double cfl, const double* dx0, int ngrids,
              const int* desc) {
  Amr* A = new Amr();
  A->nd = ndim;
  A->L = nlev;
  A->R = 2;
  A->g = g;
  for (int a = 0; a < 3; ++a) {
    A->N0[a] = a < ndim ? N0[a] : 1;
    A->dx0[a] = a < ndim ? dx0[a] : 1.0;
  }
  A->gamma = gamma;
  A->cfl = cfl;
  A->lev.assign(nlev, {});
  for (int i = 0; i < ngrids; ++i) {
    Grid q;
    q.level = desc[7 * i];
    for (int a = 0; a < 3; ++a) {
      q.lo[a] = desc[7 * i + 1 + a];
      q.hi[a] = desc[7 * i + 4 + a];
    }
    Layout Lq;
    Lq.ndim = ndim;
    for (int a = 0; a < 3; ++a) Lq.n[a] = a < ndim ? q.hi[a] - q.lo[a] : 1;
    Lq.g = g;
    q.S = State<double>(Lq);
    A->lev[q.level].push_back(i);
    A->G.push_back(std::move(q));
  }
  A->build_owner();
  return A;
}

// interior-layout helpers (cells (nz,ny,nx); faces one longer on their normal)
int iext(const Layout& L, int s, int a) { return L.n[a] + ((L.is_face(s) && s - 5 == a) ? 1 : 0); }
size_t iidx(const Layout& L, int s, int i, int j, int k) {
  return ((size_t)k * iext(L, s, 1) + j) * iext(L, s, 0) + i;
}

void load_grid(Amr& A, int gi, const double* const* prim, const double* const* bf) {
  Grid& q = A.G[gi];
  const Layout& L = q.S.L;
  for (int s = 5; s < 8; ++s)
    for (int k = 0; k < iext(L, s, 2); ++k)
      for (int j = 0; j < iext(L, s, 1); ++j)
        for (int i = 0; i < iext(L, s, 0); ++i) q.S.at(s, i, j, k) = bf[s - 5][iidx(L, s, i, j, k)];
  for (int k = 0; k < L.n[2]; ++k)
    for (int j = 0; j < L.n[1]; ++j)
      for (int i = 0; i < L.n[0]; ++i) {
        size_t ii = iidx(L, 0, i, j, k);
        double W[NVAR], U[NVAR];
        for (int t = 0; t < 5; ++t) W[t] = prim[t][ii];
        for (int a = 0; a < 3; ++a) W[5 + a] = bcell(q.S, a, i, j, k);
        prim_to_cons(W, U, A.gamma);
        for (int t = 0; t < 5; ++t) q.S.at(t, i, j, k) = U[t];
      }
}

void store_grid(const Amr& A, int gi, double* const* out) {
  const Grid& q = A.G[gi];
  const Layout& L = q.S.L;
  for (int s = 0; s < NVAR; ++s)
    for (int k = 0; k < iext(L, s, 2); ++k)
      for (int j = 0; j < iext(L, s, 1); ++j)
        for (int i = 0; i < iext(L, s, 0); ++i) out[s][iidx(L, s, i, j, k)] = q.S.at(s, i, j, k);
}

// ---- (O)verlap: a new iteration of grids from the previous one ----
// The paper's successive iterations of grids on a level and the transfer of
// the fluid variables from the previous iteration (Sec. 2; the O of the level
// cycle, Sec. 4).  Levels are taken coarse to fine.  A new cell lying in an
// old same-level interior takes that value, otherwise it is prolonged from
// the new level l-1 (minmod-linear, as in the band fill).  A new face lying
// in or on an old same-level interior takes that value (lowest old grid id);
// otherwise a face on a coarse face is reconstructed on that face (as in the
// band fill) and the faces inside an uncovered coarse cell are the mean of
// the two opposite boundary faces corrected by the smallest change that makes
// every fine cell divergence-free: with r(c) the divergence of fine cell c
// under those means, p solves the cell-graph Laplacian L p = r (edge weights
// 1/dx_d^2, solved in its eigenbasis, the 2^nd sign patterns
// chi_s(c) = (-1)^(s.c), eigenvalue 2 sum_{d in s} 1/dx_d^2), and the face
// between cells c (low side) and c + e_d loses (p(c) - p(c + e_d)) / dx_d.
void project_cell_faces(Amr& A, int l, Grid& q, const int (&pc)[3]) {
  const int nd = A.nd;
  const int nc = 1 << nd;
  double dx[3];
  for (int d = 0; d < 3; ++d) dx[d] = A.dx(l, d);
  // local index of fine cell c (bits along x, y, z) and its face along d
  auto face = [&](int d, int c, int up) -> double& {
    int x[3] = {0, 0, 0};
    for (int a = 0; a < nd; ++a) x[a] = 2 * pc[a] + ((c >> a) & 1) - q.lo[a];
    x[d] += up;
    return q.S.at(5 + d, x[0], x[1], x[2]);
  };
  // interior faces: mean of the boundary faces in line with them
  for (int d = 0; d < nd; ++d)
    for (int c = 0; c < nc; ++c) {
      if ((c >> d) & 1) continue;  // the face above cell c (bit d = 0) is interior
      const int c1 = c | (1 << d);
      face(d, c, 1) = 0.5 * (face(d, c, 0) + face(d, c1, 1));
    }
  double r[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int c = 0; c < nc; ++c)
    for (int d = 0; d < nd; ++d) r[c] += (face(d, c, 1) - face(d, c, 0)) / dx[d];
  double pot[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int sgn = 1; sgn < nc; ++sgn) {
    double lam = 0.0, dot = 0.0;
    for (int d = 0; d < nd; ++d)
      if ((sgn >> d) & 1) lam += 2.0 / (dx[d] * dx[d]);
    for (int c = 0; c < nc; ++c) dot += (__builtin_popcount(sgn & c) & 1 ? -1.0 : 1.0) * r[c];
    for (int c = 0; c < nc; ++c) pot[c] += (__builtin_popcount(sgn & c) & 1 ? -1.0 : 1.0) * dot / (nc * lam);
  }
  for (int d = 0; d < nd; ++d)
    for (int c = 0; c < nc; ++c) {
      if ((c >> d) & 1) continue;
      const int c1 = c | (1 << d);
      face(d, c, 1) -= (pot[c] - pot[c1]) / dx[d];
    }
}

void overlap(const Amr& Ao, Amr& An) {
  const int nd = An.nd;
  const int ns = nd == 2 ? 6 : 5;
  const int slots[6] = {0, 1, 2, 3, 4, 7};
  for (int l = 0; l < An.L; ++l) {
    for (int gi : An.lev[l]) {
      Grid& q = An.G[gi];
      const Layout& Lq = q.S.L;
      for (int k = 0; k < Lq.n[2]; ++k)
        for (int j = 0; j < Lq.n[1]; ++j)
          for (int i = 0; i < Lq.n[0]; ++i) {
            int p[3] = {q.lo[0] + i, q.lo[1] + j, q.lo[2] + k};
            const bool old = Ao.own_cell(l, p) >= 0;
            if (!old && l == 0) throw std::runtime_error("overlap: level-0 cell not covered by the old level 0");
            for (int t = 0; t < ns; ++t)
              q.S.at(slots[t], i, j, k) = old ? Ao.cell_value(l, slots[t], p) : An.prolong_cell(l, slots[t], p);
          }
      for (int d = 0; d < nd; ++d)
        for (int k = 0; k < Lq.n[2] + (d == 2 ? 1 : 0); ++k)
          for (int j = 0; j < Lq.n[1] + (d == 1 ? 1 : 0); ++j)
            for (int i = 0; i < Lq.n[0] + (d == 0 ? 1 : 0); ++i) {
              int p[3] = {q.lo[0] + i, q.lo[1] + j, q.lo[2] + k};
              int o, loc[3];
              if (Ao.face_owner(l, d, p, o, loc)) {
                q.S.at(5 + d, i, j, k) = Ao.G[o].S.at(5 + d, loc[0], loc[1], loc[2]);
              } else if (l == 0) {
                throw std::runtime_error("overlap: level-0 face not covered by the old level 0");
              } else if (pmod(p[d], 2) == 0) {
                q.S.at(5 + d, i, j, k) = An.prolong_face(l, d, p);
              }
              // faces inside an uncovered coarse cell: projected below
            }
      if (l == 0) continue;
      // uncovered coarse cells under the grid (new grids are R-aligned)
      for (int ck = q.lo[2] / 2; ck < (nd == 3 ? q.hi[2] / 2 : 1); ++ck)
        for (int cj = q.lo[1] / 2; cj < q.hi[1] / 2; ++cj)
          for (int ci = q.lo[0] / 2; ci < q.hi[0] / 2; ++ci) {
            int f[3] = {2 * ci, 2 * cj, nd == 3 ? 2 * ck : 0};
            if (Ao.own_cell(l, f) >= 0) continue;
            int pc[3] = {ci, cj, ck};
            project_cell_faces(An, l, q, pc);
          }
    }
  }
}

}  // namespace
}  // namespace orc

using namespace orc;

extern "C" {

const char* orc_amr_last_error() { return a_err.c_str(); }

// Omit parts of the synchronisation (bit 1 reflux, 2 EMF fix, 4
// restriction); only the tests that show the invariants catch each
// omission use this.
void orc_amr_set_skip(int bits) { g_skip = bits; }

// Level visited by each advance of one coarse step of an nlev-level
// hierarchy with ratio 2, in the serial cycle order.  Returns the count.
int orc_amr_level_order(int nlev, int* out, int cap) {
  Amr A;
  A.L = nlev;
  A.R = 2;
  A.dry = true;
  A.cycle(0, 0);
  int n = (int)A.trace.size();
  for (int i = 0; i < n && i < cap; ++i) out[i] = A.trace[i];
  return n;
}

// Run `ncoarse` coarse steps of a hierarchy in the serial level order.
// desc: ngrids x (level, lo[3], hi[3]).  prim: ngrids*5 pointers, b:
// ngrids*3 pointers (interior layout per grid), out: ngrids*8 pointers.
// dts_in (may be NULL) fixes dt0 of each coarse step; dts_out (may be NULL)
// receives them.  Returns 0 or -1 (orc_amr_last_error()).
int orc_amr_run(int ndim, const int* N0, int nlev, int g, double gamma, double cfl, const double* dx0, int ngrids,
                const int* desc, const double* const* prim, const double* const* b, int ncoarse,
                const double* dts_in, double* const* out, double* dts_out) {
  Amr* A = nullptr;
  try {
    A = make_amr(ndim, N0, nlev, g, gamma, cfl, dx0, ngrids, desc);
    for (int i = 0; i < ngrids; ++i) load_grid(*A, i, prim + 5 * i, b + 3 * i);
    for (int s = 0; s < ncoarse; ++s) {
      A->coarse_step(dts_in ? dts_in[s] : -1.0);
      if (dts_out) dts_out[s] = A->dt0;
    }
    for (int i = 0; i < ngrids; ++i) store_grid(*A, i, out + 8 * i);
    delete A;
    return 0;
  } catch (const std::exception& e) {
    a_err = e.what();
    delete A;
    return -1;
  }
}

// Seconds of `ncoarse` coarse steps (set-up excluded), or -1.
double orc_amr_time(int ndim, const int* N0, int nlev, int g, double gamma, double cfl, const double* dx0,
                    int ngrids, const int* desc, const double* const* prim, const double* const* b, int ncoarse) {
  Amr* A = nullptr;
  try {
    A = make_amr(ndim, N0, nlev, g, gamma, cfl, dx0, ngrids, desc);
    for (int i = 0; i < ngrids; ++i) load_grid(*A, i, prim + 5 * i, b + 3 * i);
    auto t0 = std::chrono::steady_clock::now();
    for (int s = 0; s < ncoarse; ++s) A->coarse_step(-1.0);
    auto t1 = std::chrono::steady_clock::now();
    delete A;
    return std::chrono::duration<double>(t1 - t0).count();
  } catch (const std::exception& e) {
    a_err = e.what();
    delete A;
    return -1.0;
  }
}

// Fill the band of every grid of `level` (full = 1: copy then prolong; 0:
// copy only) after loading conserved interiors given directly (cons: ngrids*8
// interior-layout pointers), and return every grid's banded arrays in the
// oracle's own banded layout (banded: ngrids*8 pointers).
int orc_amr_fill(int ndim, const int* N0, int nlev, int g, const double* dx0, int ngrids, const int* desc,
                 const double* const* cons, int level, int full, double* const* banded) {
  Amr* A = nullptr;
  try {
    A = make_amr(ndim, N0, nlev, g, 5.0 / 3.0, 0.4, dx0, ngrids, desc);
    for (int i = 0; i < ngrids; ++i) {
      Grid& q = A->G[i];
      const Layout& L = q.S.L;
      for (int s = 0; s < NVAR; ++s)
        for (int k = 0; k < iext(L, s, 2); ++k)
          for (int j = 0; j < iext(L, s, 1); ++j)
            for (int ii = 0; ii < iext(L, s, 0); ++ii) q.S.at(s, ii, j, k) = cons[8 * i + s][iidx(L, s, ii, j, k)];
    }
    A->fill(level, full != 0);
    for (int i = 0; i < ngrids; ++i)
      for (int s = 0; s < NVAR; ++s)
        std::memcpy(banded[8 * i + s], A->G[i].S.f[s].data(), A->G[i].S.f[s].size() * sizeof(double));
    delete A;
    return 0;
  } catch (const std::exception& e) {
    a_err = e.what();
    delete A;
    return -1;
  }
}


// (O)verlap from the previous iteration of grids (old_desc, conserved
// interiors old_cons: nold*8 interior-layout pointers) into a new iteration
// (new_desc; new_cons receives nnew*8 interior-layout arrays).  Both
// hierarchies share the domain, ratio and level count; new boxes are aligned
// to multiples of R.  Returns 0 or -1 (orc_amr_last_error()).
int orc_amr_overlap(int ndim, const int* N0, int nlev, int g, const double* dx0, int nold, const int* old_desc,
                    const double* const* old_cons, int nnew, const int* new_desc, double* const* new_cons) {
  Amr* Ao = nullptr;
  Amr* An = nullptr;
  try {
    Ao = make_amr(ndim, N0, nlev, g, 5.0 / 3.0, 0.4, dx0, nold, old_desc);
    An = make_amr(ndim, N0, nlev, g, 5.0 / 3.0, 0.4, dx0, nnew, new_desc);
    for (int i = 0; i < nnew; ++i)
      for (int a = 0; a < ndim; ++a)
        if (An->G[i].level > 0 && (pmod(An->G[i].lo[a], 2) || pmod(An->G[i].hi[a], 2)))
          throw std::runtime_error("overlap: new box not aligned to the refinement ratio");
    for (int i = 0; i < nold; ++i) {
      Grid& q = Ao->G[i];
      const Layout& L = q.S.L;
      for (int s = 0; s < NVAR; ++s)
        for (int k = 0; k < iext(L, s, 2); ++k)
          for (int j = 0; j < iext(L, s, 1); ++j)
            for (int ii = 0; ii < iext(L, s, 0); ++ii) q.S.at(s, ii, j, k) = old_cons[8 * i + s][iidx(L, s, ii, j, k)];
    }
    overlap(*Ao, *An);
    for (int i = 0; i < nnew; ++i) store_grid(*An, i, new_cons + 8 * i);
    delete Ao;
    delete An;
    return 0;
  } catch (const std::exception& e) {
    a_err = e.what();
    delete Ao;
    delete An;
    return -1;
  }
}

// Like orc_amr_run, with conserved interiors given directly (cons: ngrids*8
// interior-layout pointers) instead of primitives.
int orc_amr_run_cons(int ndim, const int* N0, int nlev, int g, double gamma, double cfl, const double* dx0,
                     int ngrids, const int* desc, const double* const* cons, int ncoarse, const double* dts_in,
                     double* const* out, double* dts_out) {
  Amr* A = nullptr;
  try {
    A = make_amr(ndim, N0, nlev, g, gamma, cfl, dx0, ngrids, desc);
    for (int i = 0; i < ngrids; ++i) {
      Grid& q = A->G[i];
      const Layout& L = q.S.L;
      for (int s = 0; s < NVAR; ++s)
        for (int k = 0; k < iext(L, s, 2); ++k)
          for (int j = 0; j < iext(L, s, 1); ++j)
            for (int ii = 0; ii < iext(L, s, 0); ++ii) q.S.at(s, ii, j, k) = cons[8 * i + s][iidx(L, s, ii, j, k)];
    }
    for (int s = 0; s < ncoarse; ++s) {
      A->coarse_step(dts_in ? dts_in[s] : -1.0);
      if (dts_out) dts_out[s] = A->dt0;
    }
    for (int i = 0; i < ngrids; ++i) store_grid(*A, i, out + 8 * i);
    delete A;
    return 0;
  } catch (const std::exception& e) {
    a_err = e.what();
    delete A;
    return -1;
  }
}

}  // extern "C"
