// Host-side table builders of libamrmhd.so: validation of a hierarchy, the
// batched and per-grid work lists (and the predictive schedule), the ghost
// fill maps, the proper-nesting check and the synchronisation tables.  Run
// once by amr_create() (or on the host only by amr_validate()).
#include "runtime_internal.hpp"

namespace amrrt {

// ------------------------------------------------------------ validation
void validate(const amr_params* p, const amr_grid* grids, int ngrids) {
  if (!p || !grids || ngrids <= 0) throw Error(AMR_EINVAL, "null params/grids or ngrids <= 0");
  if (p->ndim != 2 && p->ndim != 3) throw Error(AMR_EINVAL, "ndim must be 2 or 3");
  if (p->nlevels < 1 || p->nlevels > 12) throw Error(AMR_EINVAL, "nlevels must be in [1, 12]");
  if (p->nlevels > 1 && p->ratio != 2) throw Error(AMR_EUNSUPPORTED, "only refinement ratio 2 is implemented");
  if (p->ratio < 2) throw Error(AMR_EINVAL, "ratio must be >= 2");
  if (p->emf != AMR_EMF_MEAN && p->emf != AMR_EMF_UPWIND) throw Error(AMR_EINVAL, "emf must be 0 or 1");
  if (p->dtype != AMR_F32 && p->dtype != AMR_F64) throw Error(AMR_EINVAL, "dtype must be AMR_F32 or AMR_F64");
  if (p->ghost < 2) throw Error(AMR_EINVAL, "ghost width must be >= 2");
  if (p->nlevels > 1 && p->ghost < 2 * p->ratio)
    throw Error(AMR_EINVAL, "ghost width must be >= 2R so fine grids run R substeps per fill");
  if (p->nlevels > 1 && p->ghost % p->ratio != 0) throw Error(AMR_EINVAL, "ghost width must be a multiple of R");
  if (!(p->gamma > 1.0)) throw Error(AMR_EINVAL, "gamma must be > 1");
  if (!(p->cfl > 0.0)) throw Error(AMR_EINVAL, "cfl must be > 0");
  for (int d = 0; d < p->ndim; ++d) {
    if (p->domain[d] < 1) throw Error(AMR_EINVAL, "domain extents must be >= 1");
    if (!(p->dx0[d] > 0.0)) throw Error(AMR_EINVAL, "dx0 must be > 0");
    if (p->bc[d] != AMR_BC_PERIODIC && p->bc[d] != AMR_BC_OUTFLOW) throw Error(AMR_EINVAL, "bad boundary code");
    if (p->nlevels > 1 && p->bc[d] != AMR_BC_PERIODIC)
      throw Error(AMR_EUNSUPPORTED, "multi-level hierarchies require periodic boundaries");
  }
  for (int i = 0; i < ngrids; ++i) {
    const amr_grid& G = grids[i];
    if (G.level < 0 || G.level >= p->nlevels) throw Error(AMR_EINVAL, "grid " + std::to_string(i) + ": bad level");
    for (int d = 0; d < 3; ++d) {
      if (d >= p->ndim) {
        if (G.lo[d] != 0 || G.hi[d] != 1) throw Error(AMR_EINVAL, "grid " + std::to_string(i) + ": unused axis must be [0,1)");
        continue;
      }
      if (G.hi[d] <= G.lo[d]) throw Error(AMR_EINVAL, "grid " + std::to_string(i) + ": empty box");
      const int N = p->domain[d] * ipow(p->ratio, G.level);
      if (G.lo[d] < 0 || G.hi[d] > N) throw Error(AMR_EINVAL, "grid " + std::to_string(i) + ": box outside the domain");
      if (G.level > 0 && (G.lo[d] % p->ratio || G.hi[d] % p->ratio))
        throw Error(AMR_EINVAL, "grid " + std::to_string(i) + ": fine box not aligned to the refinement ratio");
      if (G.hi[d] - G.lo[d] < p->ghost / 2 && p->nlevels > 1)
        throw Error(AMR_EINVAL, "grid " + std::to_string(i) + ": grid narrower than half the band");
    }
  }
}

// ------------------------------------------------------------ work lists
// Tile width for a W x H region covered by 256-thread tiles of tw x (256/tw)
// threads that overlap their neighbours by `ov` cells: policy 0 takes 16 x 16;
// policy 1 the width that launches the fewest tiles (wider on ties, for
// longer coalesced rows).
int pick_tile(int W, int H, int ov, int policy) {
  if (policy == 0) return 16;
  int best = 16;
  int64_t bc = INT64_MAX;
  for (int tw = kMaxTile; tw >= kMinTile; --tw) {
    const int th = 256 / tw;
    if (th - ov < 1 || tw - ov < 1) continue;
    const int64_t c = (int64_t)((W + tw - ov - 1) / (tw - ov)) * ((H + th - ov - 1) / (th - ov));
    if (c < bc) {
      bc = c;
      best = tw;
    }
  }
  return best;
}

void check_tile(int tw) {
  if (tw < kMinTile || tw > kMaxTile) throw Error(AMR_EINVAL, "internal: tile width out of range");
  if ((tw + 2) * (256 / tw + 2) > 396) throw Error(AMR_EINVAL, "internal: tile plane exceeds the LDS plane");
}

void add_grid_items(amr_hierarchy* h, int gi, int gv, std::vector<FluxItem>& fl, std::vector<UpdItem>& ul) {
  const GridDesc& G = h->desc[gi];
  const int cl = -gv + 1;
  int ch[3], uh[3];
  for (int d = 0; d < 3; ++d) {
    ch[d] = d < h->ndim ? G.n[d] + gv - 1 : 1;
    uh[d] = d < h->ndim ? G.n[d] + gv - 2 : 0;
  }
  const int zc = h->zchunk;
  const int zlo = h->ndim == 3 ? cl : 0;
  const int ftw = pick_tile(ch[0] - cl, ch[1] - cl, 1, h->tile_policy), fth = 256 / ftw;
  check_tile(ftw);
  // a column's planes in ceil(D / zc) chunks of near-equal length (each
  // chunk recomputes a plane or two at its ends, so a short remainder chunk
  // costs more per plane than an even split)
  const int FD = ch[2] - zlo, fnz = h->ndim == 3 ? (FD + zc - 1) / zc : 1;
  for (int zi = 0; zi < fnz; ++zi)
    for (int y0 = cl; y0 < ch[1]; y0 += fth - 1)
      for (int x0 = cl; x0 < ch[0]; x0 += ftw - 1) {
        FluxItem it{};
        it.tw = ftw;
        it.grid = gi;
        it.gv = gv;
        it.x0 = x0;
        it.y0 = y0;
        it.z0 = h->ndim == 3 ? zlo + (int)((int64_t)FD * zi / fnz) : 0;
        it.z1 = h->ndim == 3 ? zlo + (int)((int64_t)FD * (zi + 1) / fnz) : 1;
        fl.push_back(it);
      }
  const int ul0 = -gv + 2;
  const int uzlo = h->ndim == 3 ? ul0 : 0;
  const int uzhi = h->ndim == 3 ? uh[2] + 1 : 1;
  const int utw = pick_tile(uh[0] - ul0 + 1, uh[1] - ul0 + 1, 0, h->tile_policy), uth = 256 / utw;
  check_tile(utw);
  const int uzc = h->upd_zchunk;
  for (int z0 = uzlo; z0 < uzhi; z0 += (h->ndim == 3 ? uzc : 1))
    for (int y0 = ul0; y0 <= uh[1]; y0 += uth)
      for (int x0 = ul0; x0 <= uh[0]; x0 += utw) {
        UpdItem it{};
        it.tw = utw;
        it.grid = gi;
        it.gv = gv;
        it.x0 = x0;
        it.y0 = y0;
        it.z0 = z0;
        it.z1 = h->ndim == 3 ? std::min(z0 + uzc, uzhi) : 1;
        ul.push_back(it);
      }
  // fused flux-update tiles: each owns (tw - 2) x (th - 2) cells of the
  // update region (tiles overlap by two) and the z-planes [z0, z1) of the
  // update's planes [ul, uh_z] (the top plane holds z-faces only)
  if (!h->upwind_emf) {
    const int xtw = pick_tile(uh[0] - ul0, uh[1] - ul0, 2, h->tile_policy), xth = 256 / xtw;
    check_tile(xtw);
    // the column's planes in near-equal chunks, as for the flux items
    const int xzhi = h->ndim == 3 ? uh[2] + 1 : 1;
    const int D = xzhi - uzlo, nzc = h->ndim == 3 ? (D + zc - 1) / zc : 1;
    for (int zi = 0; zi < nzc; ++zi)
      for (int y0 = ul0; y0 < uh[1]; y0 += xth - 2)
        for (int x0 = ul0; x0 < uh[0]; x0 += xtw - 2) {
          FluxItem it{};
          it.tw = xtw;
          it.grid = gi;
          it.gv = gv;
          it.x0 = x0;
          it.y0 = y0;
          it.z0 = uzlo + (int)((int64_t)D * zi / nzc);
          it.z1 = uzlo + (int)((int64_t)D * (zi + 1) / nzc);
          h->h_xitems.push_back(it);
        }
  }
  if (!h->upwind_emf) return;
  // upwinded edge EMFs: the update's planes, one more column and row (the
  // update reads the edges at e and e + 1 along both transverse axes)
  const int etw = pick_tile(uh[0] - ul0 + 2, uh[1] - ul0 + 2, 0, h->tile_policy), eth = 256 / etw;
  check_tile(etw);
  for (int z0 = uzlo; z0 < uzhi; z0 += (h->ndim == 3 ? uzc : 1))
    for (int y0 = ul0; y0 <= uh[1] + 1; y0 += eth)
      for (int x0 = ul0; x0 <= uh[0] + 1; x0 += etw) {
        UpdItem it{};
        it.tw = etw;
        it.grid = gi;
        it.gv = gv;
        it.x0 = x0;
        it.y0 = y0;
        it.z0 = z0;
        it.z1 = h->ndim == 3 ? std::min(z0 + uzc, uzhi) : 1;
        h->h_eitems.push_back(it);
      }
}

LaunchList make_list(amr_hierarchy* h, const std::vector<std::pair<int, int>>& grid_bands) {
  LaunchList L;
  L.flux.off = (int)h->h_fitems.size();
  L.upd.off = (int)h->h_uitems.size();
  L.emf.off = (int)h->h_eitems.size();
  L.fused.off = (int)h->h_xitems.size();
  for (auto& gb : grid_bands) add_grid_items(h, gb.first, gb.second, h->h_fitems, h->h_uitems);
  L.emf.n = (int)h->h_eitems.size() - L.emf.off;
  L.fused.n = (int)h->h_xitems.size() - L.fused.off;
  L.flux.n = (int)h->h_fitems.size() - L.flux.off;
  L.upd.n = (int)h->h_uitems.size() - L.upd.off;
  // longest items first (most z-planes): blocks take items in list order,
  // so the short ones fill the end of the launch instead of starting late.
  // With XCD chunking the order holds inside each eighth of the list (the
  // chunks of the launch), so items stay in their chunk, next to the tiles
  // they share halos with; without it, over the whole list.
  auto longest_first = [&](std::vector<FluxItem>& v, int off, int n) {
    const int parts = h->xcd_chunks ? 8 : 1;
    const int C = (n + parts - 1) / parts;
    for (int c = 0; c < parts && c * C < n; ++c) {
      auto b = v.begin() + off + c * C;
      auto e = v.begin() + off + std::min(n, (c + 1) * C);
      std::stable_sort(b, e, [](const FluxItem& x, const FluxItem& y) { return x.z1 - x.z0 > y.z1 - y.z0; });
    }
  };
  longest_first(h->h_fitems, L.flux.off, L.flux.n);
  // The last fused items of the list (the shortest, about the last 8% of
  // the work, counting each item's planes plus the three a chunk adds) are
  // cut into chunks of at most 8 planes: when the queue runs dry each block
  // is left with a short item, so the launch's tail shrinks.  Each piece
  // recomputes its chunk's end planes, as any z-chunk does, so results do
  // not change.  Only lists without XCD chunks: there every eighth of the
  // list drains on its own.
  if (!h->xcd_chunks && h->ndim == 3 && L.fused.n > 0) {
    std::vector<FluxItem> v(h->h_xitems.begin() + L.fused.off, h->h_xitems.end());
    std::stable_sort(v.begin(), v.end(), [](const FluxItem& x, const FluxItem& y) { return x.z1 - x.z0 > y.z1 - y.z0; });
    int64_t total = 0;
    for (const FluxItem& it : v) total += it.z1 - it.z0 + 3;
    std::vector<FluxItem> out;
    out.reserve(v.size() + v.size() / 4);
    int64_t acc = 0;
    for (const FluxItem& it : v) {
      const int D = it.z1 - it.z0;
      acc += D + 3;
      if (acc * 100 > total * 92 && D > 8) {
        const int n = (D + 7) / 8;
        for (int i = 0; i < n; ++i) {
          FluxItem piece = it;
          piece.z0 = it.z0 + D * i / n;
          piece.z1 = it.z0 + D * (i + 1) / n;
          out.push_back(piece);
        }
      } else {
        out.push_back(it);
      }
    }
    std::stable_sort(out.begin(), out.end(), [](const FluxItem& x, const FluxItem& y) { return x.z1 - x.z0 > y.z1 - y.z0; });
    h->h_xitems.resize(L.fused.off);
    h->h_xitems.insert(h->h_xitems.end(), out.begin(), out.end());
    L.fused.n = (int)out.size();
  } else {
    longest_first(h->h_xitems, L.fused.off, L.fused.n);
  }
  return L;
}

int64_t cells_of(const amr_grid& G) {
  return (int64_t)(G.hi[0] - G.lo[0]) * (G.hi[1] - G.lo[1]) * (G.hi[2] - G.lo[2]);
}

// Valid band a level-l grid steps from at its k-th step of a coarse step.
// Levels above 0 are filled once per parent step with the full band g = 2R
// and consume 2 cells per substep.  Level 0 is refilled before each of its
// steps and nothing reads its band after the step, so it steps from band 2
// (a step needs 2 band cells; its interior is the same for any band >= 2,
// since a cell depends only on data within 2 cells).
int step_band(const amr_hierarchy* h, int l, int k) { return l == 0 ? 2 : h->g - 2 * (k % h->R); }

// Predicted cost of one step of grid gi from band gv: the cells of the
// flux kernel's computed region.
double step_work(const amr_hierarchy* h, int gi, int gv) {
  double w = 1.0;
  for (int a = 0; a < h->ndim; ++a) w *= (double)(h->grids[gi].hi[a] - h->grids[gi].lo[a] + 2 * gv - 2);
  return w;
}

// Cycle of every step of every grid in one coarse step: cyc[gi][k] for the
// k-th step of grid gi (k < R^level).  The step k of a level-l grid may run
// in any launch cycle of its window [k W, (k+1) W), W = R^(L-1-l): its band
// is filled at the window's start and its result is first needed (registers,
// synchronisation, the next step) at the window's end.  Schedule 0 runs it
// at the window's start.  Schedule 1 spreads each window's grids over the
// window's cycles with the paper's predictive balancing (Sec. 5), launch
// cycles standing in for processors: with eta(c) the work already placed in
// cycle c by the finer levels (placed first: the finest level cannot move),
// the level's share of cycle c is g(c) = gbar - (eta(c) - etabar) (gbar its
// mean work per cycle of the window, etabar the window's mean eta), which
// makes eta(c) + g(c) equal over the window; grids are dealt largest first
// to the cycle with the largest unfilled share (lowest cycle on ties).
void plan_eta(const amr_hierarchy* h, int schedule, std::vector<std::vector<int>>& cyc, std::vector<double>& load) {
  const int L = h->nlev, R = h->R;
  const int ncyc = ipow(R, L - 1);
  cyc.assign(h->grids.size(), {});
  load.assign(ncyc, 0.0);
  for (int l = L - 1; l >= 0; --l) {
    const int span = ipow(R, L - 1 - l), nsteps = ipow(R, l);
    for (int gi : h->level_grids[l]) cyc[gi].assign(nsteps, 0);
    for (int k = 0; k < nsteps; ++k) {
      const int c0 = k * span;
      const int gv = step_band(h, l, k);
      std::vector<std::pair<double, int>> w;
      double tot = 0.0;
      for (int gi : h->level_grids[l]) {
        w.push_back({step_work(h, gi, gv), gi});
        tot += w.back().first;
      }
      std::vector<double> share(span, 0.0), got(span, 0.0);
      if (schedule == 1 && span > 1) {
        double etabar = 0.0;
        for (int c = 0; c < span; ++c) etabar += load[c0 + c];
        etabar /= span;
        const double gbar = tot / span;
        for (int c = 0; c < span; ++c) share[c] = gbar - (load[c0 + c] - etabar);
        std::stable_sort(w.begin(), w.end(), [](const std::pair<double, int>& a, const std::pair<double, int>& b) {
          return a.first > b.first || (a.first == b.first && a.second < b.second);
        });
      }
      for (auto& wg : w) {
        int best = 0;
        if (schedule == 1)
          for (int c = 1; c < span; ++c)
            if (share[c] - got[c] > share[best] - got[best]) best = c;
        got[best] += wg.first;
        cyc[wg.second][k] = c0 + best;
      }
      for (int c = 0; c < span; ++c) load[c0 + c] += got[c];
    }
  }
}

void build_lists(amr_hierarchy* h) {
  const int L = h->nlev;
  const int ncyc = ipow(h->R, L - 1);
  // batched lists: grids of every level stepping in cycle c, finest level
  // first, larger grids first within a level
  for (int c = 0; c < ncyc; ++c) {
    std::vector<std::pair<int, int>> gb;
    for (int l = L - 1; l >= 0; --l) {
      const int span = ipow(h->R, L - 1 - l);
      if (c % span) continue;
      const int k = c / span;  // substep index of level l in this coarse step
      const int gv = step_band(h, l, k);
      std::vector<int> gl = h->level_grids[l];
      std::stable_sort(gl.begin(), gl.end(),
                       [&](int a, int b) { return cells_of(h->grids[a]) > cells_of(h->grids[b]); });
      for (int gi : gl) gb.push_back({gi, gv});
    }
    h->cycle_lists.push_back(make_list(h, gb));
  }
  // eta-balanced lists: same items, each (grid, step) in the cycle plan_eta
  // gives it; finest level first, larger grids first within a level
  {
    std::vector<std::vector<int>> cyc;
    plan_eta(h, 1, cyc, h->cycle_work[1]);
    std::vector<std::vector<int>> cyc0;
    plan_eta(h, 0, cyc0, h->cycle_work[0]);
    for (int c = 0; c < ncyc; ++c) {
      std::vector<std::pair<int, int>> gb;
      for (int l = L - 1; l >= 0; --l) {
        const int span = ipow(h->R, L - 1 - l);
        const int k = c / span;
        const int gv = step_band(h, l, k);
        std::vector<int> gl;
        for (int gi : h->level_grids[l])
          if (cyc[gi][k] == c) gl.push_back(gi);
        std::stable_sort(gl.begin(), gl.end(),
                         [&](int a, int b) { return cells_of(h->grids[a]) > cells_of(h->grids[b]); });
        for (int gi : gl) gb.push_back({gi, gv});
      }
      h->eta_lists.push_back(make_list(h, gb));
    }
  }
  // per-grid lists for every band the per-grid path may use
  for (int gi = 0; gi < (int)h->grids.size(); ++gi)
    for (int b = 2; b <= h->g; ++b) h->grid_lists[{gi, b}] = make_list(h, {{gi, b}});
  // single-level hierarchies: all grids with an explicit band
  if (L == 1)
    for (int b = 2; b <= h->g; ++b) {
      std::vector<std::pair<int, int>> gb;
      for (int gi : h->level_grids[0]) gb.push_back({gi, b});
      h->level0_band_lists[b] = make_list(h, gb);
    }
  // every level's grids with band 2: the forward pass the adjoint recomputes
  for (int l = 0; l < L; ++l) {
    std::vector<std::pair<int, int>> gb;
    for (int gi : h->level_grids[l]) gb.push_back({gi, 2});
    h->band2_lists.push_back(make_list(h, gb));
  }
  h->d_fitems = dev_upload(h->h_fitems);
  h->d_uitems = dev_upload(h->h_uitems);
  h->d_eitems = dev_upload(h->h_eitems);
  h->d_xitems = dev_upload(h->h_xitems);
  // CFL items: (grid, interior plane, first row, rows), about 1k cells each
  std::vector<int4> cf;
  for (int gi = 0; gi < (int)h->grids.size(); ++gi) {
    const GridDesc& G = h->desc[gi];
    const int nz = h->ndim == 3 ? G.n[2] : 1;
    const int rows = std::max(1, std::min(G.n[1], 1024 / std::max(1, G.n[0])));
    for (int k = 0; k < nz; ++k)
      for (int j0 = 0; j0 < G.n[1]; j0 += rows) cf.push_back(make_int4(gi, k, j0, std::min(rows, G.n[1] - j0)));
  }
  h->n_cfl = (int)cf.size();
  h->d_cfl = dev_upload(cf);
}

// ------------------------------------------------------------ fill maps
// Field classes: 0 cells, 1 + d faces along d.
bool own_elem(const GridDesc& G, int ndim, int cls, const int (&x)[3]) {
  for (int a = 0; a < ndim; ++a) {
    const int top = (cls == 1 + a) ? G.n[a] : G.n[a] - 1;
    if (x[a] < 0 || x[a] > top) return false;
  }
  return true;
}

void class_extent(const GridDesc& G, int ndim, int cls, int (&lo)[3], int (&hi)[3]) {
  for (int a = 0; a < 3; ++a) {
    if (a >= ndim) {
      lo[a] = 0;
      hi[a] = 1;
      continue;
    }
    lo[a] = -G.g;
    hi[a] = G.n[a] + G.g + ((cls == 1 + a) ? 1 : 0);
  }
}


void build_fill_maps(amr_hierarchy* h) {
  const int nd = h->ndim;
  const int ncls = nd == 3 ? 4 : 3;  // 2D: Bz is a cell field, copied with the cells
  std::vector<LevelIndex> idx(h->nlev);
  for (int l = 0; l < h->nlev; ++l) idx[l].build(h, l);
  h->d_copy.assign(h->nlev, nullptr);
  h->n_copy.assign(h->nlev, 0);
  h->d_copy2.assign(h->nlev, nullptr);
  h->n_copy2.assign(h->nlev, 0);
  h->copy2_cls.assign(h->nlev, make_int4(0, 0, 0, 0));
  h->copy_cls.assign(h->nlev, make_int4(0, 0, 0, 0));
  h->h_copy.assign(h->nlev, {});
  h->d_pcell.assign(h->nlev, nullptr);
  h->d_pface.assign(h->nlev, nullptr);
  h->n_pcell.assign(h->nlev, 0);
  h->n_pface.assign(h->nlev, 0);

  for (int l = 0; l < h->nlev; ++l) {
    const LevelIndex& LI = idx[l];
    // grids are independent: worker threads build each grid's entries into
    // its own lists, concatenated in grid order afterwards
    struct GridMaps {
      std::vector<CopyEntry> cp[4];
      std::vector<CopyEntry> cp2[4];  // the entries within 2 cells of the interior
      std::vector<ProlongEntry> pc, pf;
    };
    const std::vector<int>& lg = h->level_grids[l];
    std::vector<GridMaps> per(lg.size());
    auto one_grid = [&](size_t slot) {
    const int gi = lg[slot];
    LevelIndex::Memo par;  // lookups of this grid's band on the parent level
    std::vector<int> qa[3], qb[3], owna, ownb;
    PaintScratch ps;
    std::vector<CopyEntry>(&cp)[4] = per[slot].cp;
    std::vector<CopyEntry>(&cp2)[4] = per[slot].cp2;
    std::vector<ProlongEntry>& pc = per[slot].pc;
    std::vector<ProlongEntry>& pf = per[slot].pf;
    {
      const GridDesc& G = h->desc[gi];
      const amr_grid& GG = h->grids[gi];
      for (int cls = 0; cls < ncls; ++cls) {
        int lo[3], hi[3];
        class_extent(G, nd, cls, lo, hi);
        const int fa = cls - 1;  // normal axis of a face class, -1 for cells
        int ext[3];
        for (int a = 0; a < 3; ++a) ext[a] = hi[a] - lo[a];
        // Per axis and band index x: the wrapped position of the cell holding
        // the element (qa; positions clamped into the domain first on outflow
        // axes) and, along a face class's normal, of the cell below it (qb);
        // -1 where that cell lies outside an outflow domain.
        for (int a = 0; a < 3; ++a) {
          qa[a].resize(ext[a]);
          qb[a].resize(ext[a]);
          for (int x = 0; x < ext[a]; ++x) {
            int v = GG.lo[a] + lo[a] + x;
            if (a < nd && h->p.bc[a] != AMR_BC_PERIODIC) {
              const int top = (cls == 1 + a) ? LI.N[a] : LI.N[a] - 1;
              v = std::min(std::max(v, 0), top);
            }
            qa[a][x] = LI.wrap1(a, v);
            qb[a][x] = a == fa ? LI.wrap1(a, v - 1) : qa[a][x];
          }
        }
        // owner maps: the grid of this level holding cell qa (ownb: cell qb)
        paint_owners(h, lg, qa, owna, ps);
        if (fa >= 0) paint_owners(h, lg, qb, ownb, ps);
        for (int k = lo[2]; k < hi[2]; ++k)
          for (int j = lo[1]; j < hi[1]; ++j)
            for (int i = lo[0]; i < hi[0]; ++i) {
              const int x[3] = {i, j, k};
              if (own_elem(G, nd, cls, x)) continue;
              const int xi[3] = {i - lo[0], j - lo[1], k - lo[2]};
              const size_t o = ((size_t)xi[2] * ext[1] + xi[1]) * ext[0] + xi[0];
              // a same-level source: the lowest-id grid of this level whose
              // interior holds the element as a cell, or as a face on its
              // boundary (the cell above or below the face along its normal)
              int src_grid = -1;
              int sp[3] = {0, 0, 0};
              const int band_pos[3] = {GG.lo[0] + i, GG.lo[1] + j, GG.lo[2] + k};
              auto take = [&](int sg, std::vector<int>(&q)[3], int up) {
                int e[3] = {q[0][xi[0]], q[1][xi[1]], q[2][xi[2]]};
                if (up >= 0) e[up] += 1;
                // the own grid through a periodic image only at another position
                if (sg == gi && e[0] == band_pos[0] && e[1] == band_pos[1] && e[2] == band_pos[2]) return false;
                src_grid = sg;
                for (int a = 0; a < 3; ++a) sp[a] = e[a];
                return true;
              };
              bool found = false;
              const int sa = owna[o], sb = fa >= 0 ? ownb[o] : -1;
              if (sa >= 0) found = (sb >= 0 && sb < sa) ? take(sb, qb, fa) : take(sa, qa, -1);
              if (!found && sb >= 0) found = take(sb, qb, fa);
              const int64_t dst = elem(G, nd, i, j, k);
              if (src_grid >= 0) {
                const GridDesc& S = h->desc[src_grid];
                const amr_grid& SG = h->grids[src_grid];
                const int64_t src = elem(S, nd, sp[0] - SG.lo[0], sp[1] - SG.lo[1], sp[2] - SG.lo[2]);
                cp[cls].push_back(CopyEntry{(int32_t)dst, (int32_t)src});
                const int x2[3] = {i, j, k};
                bool near2 = true;
                for (int a = 0; a < nd; ++a) {
                  const int top = G.n[a] + ((cls == 1 + a) ? 2 : 1);
                  near2 = near2 && x2[a] >= -2 && x2[a] <= top;
                }
                if (near2) cp2[cls].push_back(CopyEntry{(int32_t)dst, (int32_t)src});
                continue;
              }
              if (l == 0) throw Error(AMR_EINVAL, "level 0 does not tile the domain (uncovered band element)");
              // prolongation from level l-1
              const LevelIndex& PI = idx[l - 1];
              const int gpos[3] = {GG.lo[0] + i, GG.lo[1] + j, GG.lo[2] + k};
              if (cls == 0) {
                int cc[3] = {floordiv(gpos[0], 2), floordiv(gpos[1], 2), nd == 3 ? floordiv(gpos[2], 2) : 0};
                if (!PI.wrap(cc)) throw Error(AMR_EINVAL, "prolongation source outside the domain");
                int pg = PI.find_cell(cc, par);
                if (pg < 0) throw Error(AMR_EINVAL, "proper nesting violated: band cell has no parent");
                const GridDesc& P = h->desc[pg];
                const amr_grid& PG = h->grids[pg];
                int code = 0;
                for (int a = 0; a < nd; ++a) code |= (posmod(gpos[a], 2) << a);
                for (int a = 0; a < nd; ++a)
                  if (cc[a] - PG.lo[a] < -P.g + 1 || cc[a] - PG.lo[a] > P.n[a] + P.g - 2)
                    throw Error(AMR_EINVAL, "internal: prolongation stencil leaves the parent box");
                pc.push_back(ProlongEntry{(int32_t)dst,
                                          (int32_t)elem(P, nd, cc[0] - PG.lo[0], cc[1] - PG.lo[1], cc[2] - PG.lo[2]),
                                          pg, code});
              } else {
                const int d = cls - 1;
                const bool mid = posmod(gpos[d], 2) == 1;
                int cc[3];
                for (int a = 0; a < 3; ++a) cc[a] = a < nd ? floordiv(gpos[a], 2) : 0;
                // on-face: coarse face index gpos[d]/2 (stored at that cell);
                // pick the coarse cell on its high side if covered, else low
                int w[3] = {cc[0], cc[1], cc[2]};
                int pg = -1;
                if (PI.wrap(w)) pg = PI.find_cell(w, par);
                if (!mid && pg < 0) {
                  int w2[3] = {cc[0], cc[1], cc[2]};
                  w2[d] -= 1;
                  if (PI.wrap(w2)) {
                    pg = PI.find_cell(w2, par);
                    if (pg >= 0) {
                      w[0] = w2[0];
                      w[1] = w2[1];
                      w[2] = w2[2];
                      w[d] += 1;
                    }
                  }
                }
                if (pg < 0) throw Error(AMR_EINVAL, "proper nesting violated: band face has no parent");
                const GridDesc& P = h->desc[pg];
                const amr_grid& PG = h->grids[pg];
                const int a1 = (d + 1) % 3, a2 = (d + 2) % 3;
                for (int a = 0; a < nd; ++a)
                  if (w[a] - PG.lo[a] < -P.g + 1 || w[a] - PG.lo[a] > P.n[a] + P.g - 2)
                    throw Error(AMR_EINVAL, "internal: prolongation stencil leaves the parent box");
                int code = d | (mid ? 4 : 0);
                if (a1 < nd && posmod(gpos[a1], 2)) code |= 8;
                if (a2 < nd && posmod(gpos[a2], 2)) code |= 16;
                pf.push_back(ProlongEntry{(int32_t)dst,
                                          (int32_t)elem(P, nd, w[0] - PG.lo[0], w[1] - PG.lo[1], w[2] - PG.lo[2]), pg,
                                          code});
              }
            }
      }
    }
    };
    parallel_for(lg.size(), one_grid);
    // concatenate: copies class by class (cells, x-, y-, z-faces), each in
    // grid order; prolongations in grid order.  Every grid's lists go to
    // offsets known in advance, copied (and freed) by the worker threads.
    const size_t ng = per.size();
    std::vector<size_t> o1(4 * ng + 1, 0), o2(4 * ng + 1, 0), opc(ng + 1, 0), opf(ng + 1, 0);
    for (int c = 0; c < 4; ++c)
      for (size_t g = 0; g < ng; ++g) {
        o1[c * ng + g + 1] = o1[c * ng + g] + per[g].cp[c].size();
        o2[c * ng + g + 1] = o2[c * ng + g] + per[g].cp2[c].size();
      }
    for (size_t g = 0; g < ng; ++g) {
      opc[g + 1] = opc[g] + per[g].pc.size();
      opf[g + 1] = opf[g] + per[g].pf.size();
    }
    RawVec<CopyEntry> all(o1[4 * ng]), all2(o2[4 * ng]);
    RawVec<ProlongEntry> pc(opc[ng]), pf(opf[ng]);
    parallel_for(ng, [&](size_t g) {
      GridMaps& m = per[g];
      for (int c = 0; c < 4; ++c) {
        std::copy(m.cp[c].begin(), m.cp[c].end(), all.begin() + o1[c * ng + g]);
        std::copy(m.cp2[c].begin(), m.cp2[c].end(), all2.begin() + o2[c * ng + g]);
      }
      std::copy(m.pc.begin(), m.pc.end(), pc.begin() + opc[g]);
      std::copy(m.pf.begin(), m.pf.end(), pf.begin() + opf[g]);
      m = GridMaps();
    });
    const int4 cls = make_int4((int)o1[ng], (int)o1[2 * ng], (int)o1[3 * ng], (int)o1[4 * ng]);
    const int4 cls2 = make_int4((int)o2[ng], (int)o2[2 * ng], (int)o2[3 * ng], (int)o2[4 * ng]);
    h->copy2_cls[l] = cls2;
    h->n_copy2[l] = (int)all2.size();
    h->d_copy2[l] = dev_upload(all2);
    h->copy_cls[l] = cls;
    h->n_copy[l] = (int)all.size();
    h->d_copy[l] = dev_upload(all);
    h->h_copy[l] = std::move(all);
    h->n_pcell[l] = (int)pc.size();
    h->n_pface[l] = (int)pf.size();
    h->d_pcell[l] = dev_upload(pc);
    h->d_pface[l] = dev_upload(pf);
  }
}

void check_nesting(amr_hierarchy* h) {
  const int nd = h->ndim;
  for (int l = 1; l < h->nlev; ++l) {
    LevelIndex PI;
    PI.build(h, l - 1);
    const int buf = h->g / h->R + 1;
    // grids checked on worker threads; the lowest failing grid is reported
    const std::vector<int>& lg = h->level_grids[l];
    std::vector<char> bad(lg.size(), 0);
    parallel_for(lg.size(), [&](size_t t) {
      const amr_grid& G = h->grids[lg[t]];
      int lo[3], hi[3];
      for (int a = 0; a < 3; ++a) {
        lo[a] = a < nd ? G.lo[a] / h->R - buf : 0;
        hi[a] = a < nd ? G.hi[a] / h->R + buf : 1;
      }
      LevelIndex::Memo memo;
      for (int k = lo[2]; k < hi[2]; ++k)
        for (int j = lo[1]; j < hi[1]; ++j)
          for (int i = lo[0]; i < hi[0]; ++i) {
            int c[3] = {i, j, k};
            if (!PI.wrap(c) || PI.find_cell(c, memo) < 0) {
              bad[t] = 1;
              return;
            }
          }
    });
    for (size_t t = 0; t < lg.size(); ++t)
      if (bad[t]) throw Error(AMR_EINVAL, "grid " + std::to_string(lg[t]) + " violates proper nesting");
  }
  // no overlap within a level
  for (int l = 0; l < h->nlev; ++l) {
    const auto& gl = h->level_grids[l];
    for (size_t a = 0; a < gl.size(); ++a)
      for (size_t b = a + 1; b < gl.size(); ++b) {
        const amr_grid &A = h->grids[gl[a]], &B = h->grids[gl[b]];
        bool ov = true;
        for (int d = 0; d < 3; ++d) ov = ov && A.lo[d] < B.hi[d] && B.lo[d] < A.hi[d];
        if (ov) throw Error(AMR_EINVAL, "grids " + std::to_string(gl[a]) + " and " + std::to_string(gl[b]) + " overlap");
      }
  }
}


// ------------------------------------------------------------ sync tables
// Coarse/fine registers, reflux, EMF-fix and restriction entries of fine
// level f (see sync_internal.hpp).  Positions on periodic levels are taken in
// the frame of the grid that stores them.
void build_sync_tables(amr_hierarchy* h, int f) {
  const int nd = h->ndim, R = h->R, c = f - 1;
  LevelIndex CI, FI;
  CI.build(h, c);
  FI.build(h, f);
  for (int a = 0; a < nd; ++a)
    if (CI.N[a] >= (1 << 20)) throw Error(AMR_EUNSUPPORTED, "level exceeds 2^20 cells along an axis");
  const double dxc[3] = {h->p.dx0[0] / ipow(R, c), h->p.dx0[1] / ipow(R, c), nd == 3 ? h->p.dx0[2] / ipow(R, c) : 1.0};
  SyncTables& T = h->sync[f];
  // edge registers deduplicated by (axis, wrapped edge index): the key packs
  // the axis and three coordinates below 2^20 each
  auto edge_key = [](int a, const int (&w)[3]) {
    return (((int64_t)a << 60) | ((int64_t)w[2] << 40) | ((int64_t)w[1] << 20) | (int64_t)w[0]);
  };
  // Coarse grids are independent: worker threads build each grid's entries
  // with grid-local register numbers (edge registers deduplicated within the
  // grid); a pass in grid order then numbers the face registers one after
  // another and each edge register where it first appears, which gives the
  // tables of a single pass over the grids in order.
  struct LocalEdge {
    int64_t key;
    EdgeRegEntry c, f;
  };
  struct GridSync {
    std::vector<FaceRegEntry> frc, frf;
    std::vector<RefluxEntry> rfx;
    std::vector<EmfFixEntry> efx;  // reg[]: indices into edges
    std::vector<RestrictEntry> rst;
    std::vector<LocalEdge> edges;
    int nfreg = 0;
  };
  const std::vector<int>& cgrids = h->level_grids[c];
  std::vector<GridSync> per(cgrids.size());
  parallel_for(cgrids.size(), [&](size_t slot) {
    const int gi = cgrids[slot];
    GridSync& out = per[slot];
    std::vector<FaceRegEntry>&frc = out.frc, &frf = out.frf;
    std::vector<RefluxEntry>& rfx = out.rfx;
    std::vector<EmfFixEntry>& efx = out.efx;
    std::vector<RestrictEntry>& rst = out.rst;
    int& nfreg = out.nfreg;
    std::unordered_map<int64_t, int> edge_id;  // key -> index in out.edges
    // covered(p) for coarse cells p of the current coarse grid's box grown by
    // one cell: a mask filled from the fine grids' boxes (and their periodic
    // images) before the grid's elements are visited
    std::vector<uint8_t> mask, near;  // near: a covered cell within one cell (any direction)
    int mlo[3] = {0, 0, 0}, mext[3] = {1, 1, 1};
    auto near_covered = [&](const int (&pc)[3]) {
      int64_t o = 0;
      for (int a = 2; a >= 0; --a) o = o * mext[a] + (pc[a] - mlo[a]);
      return near[o] != 0;
    };
    auto covered = [&](const int (&pc)[3]) {
      int64_t o = 0;
      for (int a = 2; a >= 0; --a) {
        const int x = pc[a] - mlo[a];
        if (x < 0 || x >= mext[a]) throw Error(AMR_EINVAL, "internal: covered() outside the grid's mask");
        o = o * mext[a] + x;
      }
      return mask[o] != 0;
    };
    auto build_mask = [&](const amr_grid& CG) {
      for (int a = 0; a < 3; ++a) {
        mlo[a] = a < nd ? CG.lo[a] - 1 : 0;
        mext[a] = a < nd ? CG.hi[a] - CG.lo[a] + 2 : 1;
      }
      mask.assign((size_t)mext[0] * mext[1] * mext[2], 0);
      for (int fgi : h->level_grids[f]) {
        const amr_grid& FG = h->grids[fgi];
        // coarse box of the fine grid (boxes are aligned to R), then every
        // periodic image that meets the mask box
        int flo[3], fhi[3];
        for (int a = 0; a < 3; ++a) {
          flo[a] = a < nd ? FG.lo[a] / R : 0;
          fhi[a] = a < nd ? FG.hi[a] / R : 1;
        }
        for (int sz = -1; sz <= 1; ++sz)
          for (int sy = -1; sy <= 1; ++sy)
            for (int sx = -1; sx <= 1; ++sx) {
              const int sh[3] = {sx, sy, sz};
              int lo[3], hi[3];
              bool ok = true;
              for (int a = 0; a < 3; ++a) {
                if (a >= nd || h->p.bc[a] != AMR_BC_PERIODIC) {
                  if (sh[a] != 0) ok = false;
                  lo[a] = std::max(flo[a], mlo[a]);
                  hi[a] = std::min(fhi[a], mlo[a] + mext[a]);
                } else {
                  const int off = sh[a] * CI.N[a];
                  lo[a] = std::max(flo[a] + off, mlo[a]);
                  hi[a] = std::min(fhi[a] + off, mlo[a] + mext[a]);
                }
                ok = ok && lo[a] < hi[a];
              }
              if (!ok) continue;
              for (int z = lo[2]; z < hi[2]; ++z)
                for (int y = lo[1]; y < hi[1]; ++y)
                  for (int x = lo[0]; x < hi[0]; ++x)
                    mask[((size_t)(z - mlo[2]) * mext[1] + (y - mlo[1])) * mext[0] + (x - mlo[0])] = 1;
            }
      }
      near.assign(mask.size(), 0);
      for (int z = 0; z < mext[2]; ++z)
        for (int y = 0; y < mext[1]; ++y)
          for (int x = 0; x < mext[0]; ++x) {
            if (!mask[((size_t)z * mext[1] + y) * mext[0] + x]) continue;
            for (int dz = (nd == 3 ? -1 : 0); dz <= (nd == 3 ? 1 : 0); ++dz)
              for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                  const int X = x + dx, Y = y + dy, Z = z + dz;
                  if (X < 0 || Y < 0 || Z < 0 || X >= mext[0] || Y >= mext[1] || Z >= mext[2]) continue;
                  near[((size_t)Z * mext[1] + Y) * mext[0] + X] = 1;
                }
          }
    };
    // fine grid owning fine cell p (unwrapped); shift = wrap(p) - p
    LevelIndex::Memo fmemo;
    auto fine_owner = [&](const int (&p)[3], int (&shift)[3]) {
      int w[3] = {p[0], p[1], p[2]};
      if (!FI.wrap(w)) return -1;
      for (int a = 0; a < 3; ++a) shift[a] = w[a] - p[a];
      return FI.find_cell(w, fmemo);
    };
    const GridDesc& C = h->desc[gi];
    const amr_grid& CG = h->grids[gi];
    build_mask(CG);
    // cells: restriction or reflux
    for (int k = 0; k < C.n[2]; ++k)
      for (int j = 0; j < C.n[1]; ++j)
        for (int i = 0; i < C.n[0]; ++i) {
          int pu[3] = {CG.lo[0] + i, CG.lo[1] + j, CG.lo[2] + k};
          if (covered(pu)) {
            int pf[3], sh[3];
            for (int a = 0; a < 3; ++a) pf[a] = a < nd ? R * pu[a] : 0;
            int fg = fine_owner(pf, sh);
            const amr_grid& FG = h->grids[fg];
            rst.push_back(RestrictEntry{(int32_t)elem(C, nd, i, j, k),
                                        (int32_t)elem(h->desc[fg], nd, pf[0] + sh[0] - FG.lo[0],
                                                      pf[1] + sh[1] - FG.lo[1], pf[2] + sh[2] - FG.lo[2]),
                                        fg, -1});
            continue;
          }
          RefluxEntry re{};
          re.cell = (int32_t)elem(C, nd, i, j, k);
          for (int d = 0; d < nd; ++d)
            for (int side = -1; side <= 1; side += 2) {
              int pv[3] = {pu[0], pu[1], pu[2]};
              pv[d] += side;
              if (!covered(pv)) continue;
              int lf[3] = {i, j, k};
              if (side > 0) lf[d] += 1;
              const int r = nfreg++;
              FaceRegEntry ec{};
              ec.reg = r;
              ec.d = d;
              ec.grid = gi;
              ec.n = 1;
              ec.e[0] = (int32_t)elem(C, nd, lf[0], lf[1], lf[2]);
              frc.push_back(ec);
              // fine faces on the coarse face, in the frame of their grid
              int fc[3];
              for (int a = 0; a < 3; ++a) fc[a] = a < nd ? R * pv[a] : 0;
              if (side < 0) fc[d] += R - 1;
              int sh[3];
              int fg = fine_owner(fc, sh);
              if (fg < 0) throw Error(AMR_EINVAL, "internal: covered cell without fine owner");
              const amr_grid& FG = h->grids[fg];
              FaceRegEntry ef{};
              ef.reg = r;
              ef.d = d;
              ef.grid = fg;
              int gf[3];
              for (int a = 0; a < 3; ++a) gf[a] = a < nd ? R * (CG.lo[a] + lf[a]) + sh[a] : 0;
              const int o1 = (d + 1) % 3, o2 = (d + 2) % 3;
              for (int a1 = 0; a1 < (o1 < nd ? R : 1); ++a1)
                for (int a2 = 0; a2 < (o2 < nd ? R : 1); ++a2) {
                  int p[3] = {gf[0], gf[1], gf[2]};
                  p[o1] += a1;
                  p[o2] += a2;
                  ef.e[ef.n++] = (int32_t)elem(h->desc[fg], nd, p[0] - FG.lo[0], p[1] - FG.lo[1], p[2] - FG.lo[2]);
                }
              frf.push_back(ef);
              re.reg[re.n] = r;
              re.coef[re.n] = (side > 0 ? 1.0 : -1.0) / dxc[d];
              ++re.n;
            }
          if (re.n > 0) rfx.push_back(re);
        }
    // faces: restriction (a covered neighbour) or EMF fix (C/F edges)
    for (int d = 0; d < nd; ++d) {
      for (int k = 0; k < C.n[2] + (d == 2 ? 1 : 0); ++k)
        for (int j = 0; j < C.n[1] + (d == 1 ? 1 : 0); ++j)
          for (int i = 0; i < C.n[0] + (d == 0 ? 1 : 0); ++i) {
            int pf[3] = {CG.lo[0] + i, CG.lo[1] + j, CG.lo[2] + k};
            int pm[3] = {pf[0], pf[1], pf[2]};
            pm[d] -= 1;
            // faces with no covered cell within one cell of either side have
            // nothing to restrict or correct
            if (!near_covered(pf) && !near_covered(pm)) continue;
            const bool cu = covered(pf), cm = covered(pm);
            if (cu || cm) {
              // fine faces from the lowest-id fine grid owning a neighbour
              int best = -1, bsh[3] = {0, 0, 0};
              for (int side = 0; side < 2; ++side) {
                if ((side == 0 && !cu) || (side == 1 && !cm)) continue;
                int fc[3];
                for (int a = 0; a < 3; ++a) fc[a] = a < nd ? R * pf[a] : 0;
                if (side == 1) fc[d] -= 1;
                int sh[3];
                int fg = fine_owner(fc, sh);
                if (fg >= 0 && (best < 0 || fg < best)) {
                  best = fg;
                  for (int a = 0; a < 3; ++a) bsh[a] = sh[a];
                }
              }
              const amr_grid& FG = h->grids[best];
              int q[3];
              for (int a = 0; a < 3; ++a) q[a] = a < nd ? R * pf[a] + bsh[a] - FG.lo[a] : 0;
              rst.push_back(RestrictEntry{(int32_t)elem(C, nd, i, j, k),
                                          (int32_t)elem(h->desc[best], nd, q[0], q[1], q[2]), best, d});
              continue;
            }
            // (curl dE)_d = d_b dE_cc - d_cc dE_b with b = d+1, cc = d+2
            EmfFixEntry fx{};
            fx.face = (int32_t)elem(C, nd, i, j, k);
            fx.d = d;
            const int b = (d + 1) % 3, cc = (d + 2) % 3;
            for (int term = 0; term < 2; ++term) {
              const int ea = term == 0 ? cc : b;
              const int da = term == 0 ? b : cc;
              if (da >= nd) continue;
              if (nd == 2 && ea != 2) continue;
              const double sgn = term == 0 ? 1.0 : -1.0;
              for (int up = 0; up < 2; ++up) {
                int e[3] = {pf[0], pf[1], pf[2]};
                e[da] += up;
                // neighbouring coarse cells of the edge (offsets -1/0 in the
                // two axes other than ea)
                const int b2 = (ea + 1) % 3, c2 = (ea + 2) % 3;
                int ncov = 0, nall = 0, fg = -1, fsh[3] = {0, 0, 0}, fcell[3] = {0, 0, 0};
                for (int db = 0; db < 2; ++db)
                  for (int dc = 0; dc < 2; ++dc) {
                    if ((b2 >= nd && db) || (c2 >= nd && dc)) continue;
                    int p[3] = {e[0], e[1], e[2]};
                    if (b2 < nd) p[b2] -= db;
                    if (c2 < nd) p[c2] -= dc;
                    ++nall;
                    if (!covered(p)) continue;
                    ++ncov;
                    int fc[3];
                    for (int a = 0; a < 3; ++a) fc[a] = a < nd ? R * p[a] : 0;
                    int sh[3];
                    int o = fine_owner(fc, sh);
                    if (o >= 0 && (fg < 0 || o < fg)) {
                      fg = o;
                      for (int a = 0; a < 3; ++a) {
                        fsh[a] = sh[a];
                        fcell[a] = fc[a];
                      }
                    }
                  }
                (void)fcell;
                if (!(ncov > 0 && ncov < nall)) continue;
                // dedupe registers by (axis, wrapped edge index)
                int w[3] = {e[0], e[1], e[2]};
                for (int a = 0; a < nd; ++a) w[a] = posmod(w[a], CI.N[a]);
                const int64_t key = edge_key(ea, w);
                int re;
                auto it = edge_id.find(key);
                if (it == edge_id.end()) {
                  re = (int)out.edges.size();
                  edge_id[key] = re;
                  EdgeRegEntry ec{};
                  ec.reg = re;
                  ec.a = ea;
                  ec.grid = gi;
                  ec.n = 1;
                  ec.e[0] = (int32_t)elem(C, nd, e[0] - CG.lo[0], e[1] - CG.lo[1], e[2] - CG.lo[2]);
                  const amr_grid& FG = h->grids[fg];
                  EdgeRegEntry ef{};
                  ef.reg = re;
                  ef.a = ea;
                  ef.grid = fg;
                  const int na = ea < nd ? R : 1;
                  for (int s2 = 0; s2 < na; ++s2) {
                    int p[3];
                    for (int a = 0; a < 3; ++a) p[a] = a < nd ? R * e[a] + fsh[a] - FG.lo[a] : 0;
                    if (ea < nd) p[ea] += s2;
                    ef.e[ef.n++] = (int32_t)elem(h->desc[fg], nd, p[0], p[1], p[2]);
                  }
                  out.edges.push_back(LocalEdge{key, ec, ef});
                } else {
                  re = it->second;
                }
                if (fx.n >= 4) throw Error(AMR_EINVAL, "internal: more than 4 edges on a face");
                fx.reg[fx.n] = re;
                fx.coef[fx.n] = sgn * (up ? 1.0 : -1.0) / dxc[da];
                ++fx.n;
              }
            }
            if (fx.n > 0) efx.push_back(fx);
          }
    }
  });
  // grid order: face registers numbered consecutively, edge registers at
  // their first appearance
  std::vector<FaceRegEntry> frc, frf;
  std::vector<EdgeRegEntry> erc, erf;
  std::vector<RefluxEntry> rfx;
  std::vector<EmfFixEntry> efx;
  std::vector<RestrictEntry> rst;
  std::unordered_map<int64_t, int> edge_id;
  int nfreg = 0;
  std::vector<int> gid;
  for (GridSync& g : per) {
    for (FaceRegEntry e : g.frc) {
      e.reg += nfreg;
      frc.push_back(e);
    }
    for (FaceRegEntry e : g.frf) {
      e.reg += nfreg;
      frf.push_back(e);
    }
    for (RefluxEntry e : g.rfx) {
      for (int i = 0; i < e.n; ++i) e.reg[i] += nfreg;
      rfx.push_back(e);
    }
    nfreg += g.nfreg;
    gid.resize(g.edges.size());
    for (size_t k = 0; k < g.edges.size(); ++k) {
      LocalEdge& le = g.edges[k];
      auto it = edge_id.find(le.key);
      if (it != edge_id.end()) {
        gid[k] = it->second;
        continue;
      }
      const int id = (int)edge_id.size();
      edge_id[le.key] = id;
      gid[k] = id;
      le.c.reg = id;
      le.f.reg = id;
      erc.push_back(le.c);
      erf.push_back(le.f);
    }
    for (EmfFixEntry e : g.efx) {
      for (int i = 0; i < e.n; ++i) e.reg[i] = gid[e.reg[i]];
      efx.push_back(e);
    }
    rst.insert(rst.end(), g.rst.begin(), g.rst.end());
    g = GridSync();
  }
  T.nfreg = nfreg;
  T.nereg = (int)edge_id.size();
  // face fluxes the registers read (the fused kernel stores only these)
  {
    if (h->h_fmask.empty()) h->h_fmask.assign(h->total_elems, 0);
    auto mark = [&](int64_t e, int d) {
      if (e < 0 || e >= h->total_elems) throw Error(AMR_EINVAL, "internal: register face outside the pools");
      h->h_fmask[e] |= (uint8_t)(1u << d);
    };
    for (const auto* v : {&frc, &frf})
      for (const FaceRegEntry& r : *v)
        for (int i = 0; i < r.n; ++i) mark(r.e[i], r.d);
    for (const auto* v : {&erc, &erf})
      for (const EdgeRegEntry& r : *v) {
        const GridDesc& G = h->desc[r.grid];
        const int64_t st[3] = {1, G.P[0], h->ndim == 3 ? (int64_t)G.P[0] * G.P[1] : 0};
        const int B = (r.a + 1) % 3, C = (r.a + 2) % 3;
        for (int i = 0; i < r.n; ++i) {
          mark(r.e[i] - st[C], B);
          mark(r.e[i], B);
          mark(r.e[i] - st[B], C);
          mark(r.e[i], C);
        }
      }
  }
  T.d_freg_c = dev_upload(frc);
  T.n_freg_c = (int)frc.size();
  T.d_freg_f = dev_upload(frf);
  T.n_freg_f = (int)frf.size();
  T.d_ereg_c = dev_upload(erc);
  T.n_ereg_c = (int)erc.size();
  T.d_ereg_f = dev_upload(erf);
  T.n_ereg_f = (int)erf.size();
  T.d_reflux = dev_upload(rfx);
  T.n_reflux = (int)rfx.size();
  T.d_emffix = dev_upload(efx);
  T.n_emffix = (int)efx.size();
  T.d_restrict = dev_upload(rst);
  T.n_restrict = (int)rst.size();
  const int64_t fbytes = (int64_t)(1 + R) * nfreg * 6 * (int64_t)h->esize;
  const int64_t ebytes = (int64_t)(1 + R) * T.nereg * (int64_t)h->esize;
  T.reg_bytes = (fbytes + 255) / 256 * 256 + ebytes;
}

// Validate and build every table of a hierarchy (device uploads skipped in
// host-only mode).
amr_hierarchy* build_hierarchy(const amr_params* p, const amr_grid* grids, int32_t ngrids) {
  validate(p, grids, ngrids);
  amr_hierarchy* h = new amr_hierarchy();
  try {
    h->p = *p;
    h->ndim = p->ndim;
    h->nlev = p->nlevels;
    h->R = p->ratio;
    h->g = p->ghost;
    h->esize = p->dtype == AMR_F64 ? 8 : 4;
    h->grids.assign(grids, grids + ngrids);
    h->level_grids.assign(h->nlev, {});
    for (int i = 0; i < ngrids; ++i) h->level_grids[grids[i].level].push_back(i);
    for (int l = 0; l < h->nlev; ++l)
      if (h->level_grids[l].empty()) throw Error(AMR_EINVAL, "level " + std::to_string(l) + " has no grids");
    // layout: padded boxes, offsets aligned to 64 elements
    int64_t off = 0;
    for (int i = 0; i < ngrids; ++i) {
      GridDesc G{};
      for (int d = 0; d < 3; ++d) {
        G.n[d] = grids[i].hi[d] - grids[i].lo[d];
        G.lo[d] = grids[i].lo[d];
        G.P[d] = d < h->ndim ? G.n[d] + 2 * h->g + 1 : 1;
      }
      G.g = h->g;
      G.level = grids[i].level;
      G.off = off;
      off += (int64_t)G.P[0] * G.P[1] * G.P[2];
      off = (off + 63) / 64 * 64;
      h->desc.push_back(G);
    }
    h->total_elems = off;
    if (off >= ((int64_t)1 << 31)) throw Error(AMR_EUNSUPPORTED, "hierarchy exceeds 2^31 elements per pool");
    // the advance kernels address the level arrays by 32-bit byte offsets
    if (off * h->esize >= ((int64_t)1 << 32)) throw Error(AMR_EUNSUPPORTED, "hierarchy exceeds 4 GiB per field");
    h->upwind_emf = p->emf == AMR_EMF_UPWIND;
    h->flux_bytes = (h->upwind_emf ? 27 : 21) * off * (int64_t)h->esize;
    h->reg_offset = (h->flux_bytes + 255) / 256 * 256;
    check_nesting(h);
    h->d_desc = dev_upload(h->desc);
    build_fill_maps(h);
    build_lists(h);
    h->sync.resize(h->nlev);
    int64_t reg_bytes = 0;
    for (int l = 1; l < h->nlev; ++l) {
      build_sync_tables(h, l);
      h->sync[l].reg_off = h->reg_offset + reg_bytes;
      reg_bytes += (h->sync[l].reg_bytes + 255) / 256 * 256;
    }
    h->workspace_bytes = h->reg_offset + reg_bytes;
    h->d_fmask = dev_upload(h->h_fmask);
    if (!g_host_only) {  // host-only builds keep it for amr_selfcheck_addressing
      h->h_fmask.clear();
      h->h_fmask.shrink_to_fit();
    }
    h->adj.resize(h->nlev);
    return h;
  } catch (...) {
    delete h;
    throw;
  }
}

// Rebuild every work list for the current tile policy / z-chunk.
void rebuild_lists(amr_hierarchy* h) {
  for (auto g : h->graph_exec)
    if (g) (void)hipGraphExecDestroy(g);
  h->graph_exec[0] = h->graph_exec[1] = nullptr;
  HIPCHK(hipFree(h->d_fitems));
  HIPCHK(hipFree(h->d_uitems));
  HIPCHK(hipFree(h->d_eitems));
  h->d_eitems = nullptr;
  h->h_eitems.clear();
  HIPCHK(hipFree(h->d_xitems));
  h->d_xitems = nullptr;
  h->h_xitems.clear();
  HIPCHK(hipFree(h->d_cfl));
  h->d_fitems = nullptr;
  h->d_uitems = nullptr;
  h->d_cfl = nullptr;
  h->h_fitems.clear();
  h->h_uitems.clear();
  h->cycle_lists.clear();
  h->eta_lists.clear();
  h->grid_lists.clear();
  h->level0_band_lists.clear();
  h->band2_lists.clear();
  build_lists(h);
}

void set_update_zchunk(amr_hierarchy* h, int zchunk) {
  if (zchunk < 1 || zchunk > 4096) throw Error(AMR_EINVAL, "update z-chunk must be in [1, 4096]");
  if (zchunk != h->upd_zchunk) {
    h->upd_zchunk = zchunk;
    rebuild_lists(h);
  }
}

void set_launch_config(amr_hierarchy* h, int policy, int zchunk, int mode) {
  if (policy != 0 && policy != 1) throw Error(AMR_EINVAL, "tile policy must be 0 or 1");
  if (zchunk < 1 || zchunk > 4096) throw Error(AMR_EINVAL, "z-chunk must be in [1, 4096]");
  if (mode < 0 || mode > 63) throw Error(AMR_EINVAL, "launch mode must be in [0, 63]");
  h->persistent = (mode & 1) != 0;
  h->claim = 1 << ((mode >> 4) & 3);
  h->persistent_flux = (mode & 5) != 0;
  const bool xcd = (mode & 2) != 0;
  h->fused = (mode & 8) != 0;
  // the item order depends on the XCD chunking (see make_list)
  if (policy != h->tile_policy || zchunk != h->zchunk || xcd != h->xcd_chunks) {
    h->tile_policy = policy;
    h->zchunk = zchunk;
    h->xcd_chunks = xcd;
    rebuild_lists(h);
  }
}

}  // namespace amrrt
