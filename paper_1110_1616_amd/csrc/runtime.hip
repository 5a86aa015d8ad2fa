// Host runtime and C ABI of libamrmhd.so (see include/amr.h).
//
// amr_create() validates the hierarchy and builds, once, every device table
// the hot path needs: grid descriptors, ghost-fill gather maps, batched work
// lists of each launch cycle (finest level first) and per-grid lists for
// the per-grid path.  The calls after that only enqueue kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/amr.h"
#include "amr_internal.hpp"
#include "fill_internal.hpp"
#include "sync_internal.hpp"

using namespace amr;

namespace {

thread_local std::string g_last_error;

struct Error : std::runtime_error {
  amr_status code;
  Error(amr_status c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define HIPCHK(x)                                                                                         \
  do {                                                                                                    \
    hipError_t e_ = (x);                                                                                  \
    if (e_ != hipSuccess) throw Error(AMR_EHIP, std::string(#x) + ": " + hipGetErrorString(e_));          \
  } while (0)

#define HIPCHK_NOTHROW(x) (void)(x)

template <class T> T* dev_upload(const std::vector<T>& v) {
  if (v.empty()) return nullptr;
  T* p = nullptr;
  HIPCHK(hipMalloc((void**)&p, v.size() * sizeof(T)));
  HIPCHK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return p;
}

struct Box {
  int lo[3], hi[3];
};

struct ListRef {
  int off = 0, n = 0;
};

struct LaunchList {
  ListRef flux, upd;
};

}  // namespace

struct amr_hierarchy {
  amr_params p{};
  int ndim = 3;
  int nlev = 1;
  int R = 2;
  int g = 2;
  size_t esize = 8;
  std::vector<amr_grid> grids;
  std::vector<GridDesc> desc;
  std::vector<std::vector<int>> level_grids;
  int64_t total_elems = 0;
  int64_t flux_bytes = 0;
  int64_t reg_offset = 0;
  int64_t workspace_bytes = 0;

  // device tables
  GridDesc* d_desc = nullptr;
  FluxItem* d_fitems = nullptr;
  UpdItem* d_uitems = nullptr;
  std::vector<FluxItem> h_fitems;
  std::vector<UpdItem> h_uitems;
  int4* d_cfl = nullptr;
  int n_cfl = 0;
  ErrBlock* d_err = nullptr;  // error block + CFL accumulator (handle-owned)

  // fill maps per level
  std::vector<CopyEntry*> d_copy;
  std::vector<int> n_copy;
  std::vector<int4> copy_cls;
  std::vector<ProlongEntry*> d_pcell, d_pface;
  std::vector<int> n_pcell, n_pface;

  // synchronisation tables per fine level
  std::vector<SyncTables> sync;

  // launch lists
  std::vector<LaunchList> cycle_lists;                 // per launch cycle (batched)
  std::map<std::pair<int, int>, LaunchList> grid_lists;  // (grid, band) -> per-grid list
  std::map<int, LaunchList> level0_band_lists;          // band -> all level-0 grids
  int zchunk = 16;

  // optional per-kernel timing with HIP events on the launch stream
  bool timing = false;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, int>> ev_pairs[2];  // [0] flux, [1] update: (start, stop) pool indices
  int ev_used = 0;
  int take_event() {
    if (ev_used == (int)ev_pool.size()) {
      hipEvent_t e;
      HIPCHK_NOTHROW(hipEventCreate(&e));
      ev_pool.push_back(e);
    }
    return ev_used++;
  }

  ~amr_hierarchy() {
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    (void)hipFree(d_desc);
    (void)hipFree(d_fitems);
    (void)hipFree(d_uitems);
    (void)hipFree(d_cfl);
    (void)hipFree(d_err);
    for (auto p : d_copy) (void)hipFree(p);
    for (auto p : d_pcell) (void)hipFree(p);
    for (auto p : d_pface) (void)hipFree(p);
    for (auto& s : sync) s.release();
  }
};

namespace {

int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
int posmod(int a, int b) { return ((a % b) + b) % b; }

// Spatial lookup of grids of one level by 16-cell buckets.
struct LevelIndex {
  const amr_hierarchy* h = nullptr;
  int level = 0;
  int N[3] = {1, 1, 1};
  std::unordered_map<int64_t, std::vector<int>> buckets;
  static constexpr int B = 16;
  int64_t key(int bx, int by, int bz) const { return ((int64_t)bz * 1000003 + by) * 1000003 + bx; }
  void build(const amr_hierarchy* hh, int l) {
    h = hh;
    level = l;
    for (int d = 0; d < 3; ++d) N[d] = d < h->ndim ? h->p.domain[d] * ipow(h->R, l) : 1;
    for (int gi : h->level_grids[l]) {
      const amr_grid& G = h->grids[gi];
      for (int bz = floordiv(G.lo[2], B); bz <= floordiv(G.hi[2] - 1, B); ++bz)
        for (int by = floordiv(G.lo[1], B); by <= floordiv(G.hi[1] - 1, B); ++by)
          for (int bx = floordiv(G.lo[0], B); bx <= floordiv(G.hi[0] - 1, B); ++bx)
            buckets[key(bx, by, bz)].push_back(gi);
    }
  }
  // Wrap a cell position on periodic axes; returns false if outside a
  // non-periodic domain.
  bool wrap(int (&c)[3]) const {
    for (int d = 0; d < h->ndim; ++d) {
      if (h->p.bc[d] == AMR_BC_PERIODIC) c[d] = posmod(c[d], N[d]);
      else if (c[d] < 0 || c[d] >= N[d]) return false;
    }
    return true;
  }
  // Grid whose interior holds cell c (already wrapped), or -1.
  int find_cell(const int (&c)[3]) const {
    auto it = buckets.find(key(floordiv(c[0], B), floordiv(c[1], B), floordiv(c[2], B)));
    if (it == buckets.end()) return -1;
    for (int gi : it->second) {
      const amr_grid& G = h->grids[gi];
      bool in = true;
      for (int d = 0; d < 3; ++d) in = in && c[d] >= G.lo[d] && c[d] < G.hi[d];
      if (in) return gi;
    }
    return -1;
  }
};

int64_t elem(const GridDesc& G, int ndim, int i, int j, int k) {
  const int gz = ndim == 3 ? G.g : 0;
  return G.off + (int64_t)(i + G.g) + (int64_t)(j + G.g) * G.P[0] + (int64_t)(k + gz) * G.P[0] * G.P[1];
}

// ------------------------------------------------------------ validation
void validate(const amr_params* p, const amr_grid* grids, int ngrids) {
  if (!p || !grids || ngrids <= 0) throw Error(AMR_EINVAL, "null params/grids or ngrids <= 0");
  if (p->ndim != 2 && p->ndim != 3) throw Error(AMR_EINVAL, "ndim must be 2 or 3");
  if (p->nlevels < 1 || p->nlevels > 12) throw Error(AMR_EINVAL, "nlevels must be in [1, 12]");
  if (p->nlevels > 1 && p->ratio != 2) throw Error(AMR_EUNSUPPORTED, "only refinement ratio 2 is implemented");
  if (p->ratio < 2) throw Error(AMR_EINVAL, "ratio must be >= 2");
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
  for (int z0 = zlo; z0 < ch[2]; z0 += (h->ndim == 3 ? zc : 1))
    for (int y0 = cl; y0 < ch[1]; y0 += kFluxTile)
      for (int x0 = cl; x0 < ch[0]; x0 += kFluxTile) {
        FluxItem it{};
        it.grid = gi;
        it.gv = gv;
        it.x0 = x0;
        it.y0 = y0;
        it.z0 = z0;
        it.z1 = h->ndim == 3 ? std::min(z0 + zc, ch[2]) : 1;
        fl.push_back(it);
      }
  const int ul0 = -gv + 2;
  const int uzlo = h->ndim == 3 ? ul0 : 0;
  const int uzhi = h->ndim == 3 ? uh[2] + 1 : 1;
  for (int z0 = uzlo; z0 < uzhi; z0 += (h->ndim == 3 ? zc : 1))
    for (int y0 = ul0; y0 <= uh[1]; y0 += kUpdTile)
      for (int x0 = ul0; x0 <= uh[0]; x0 += kUpdTile) {
        UpdItem it{};
        it.grid = gi;
        it.gv = gv;
        it.x0 = x0;
        it.y0 = y0;
        it.z0 = z0;
        it.z1 = h->ndim == 3 ? std::min(z0 + zc, uzhi) : 1;
        ul.push_back(it);
      }
}

LaunchList make_list(amr_hierarchy* h, const std::vector<std::pair<int, int>>& grid_bands) {
  LaunchList L;
  L.flux.off = (int)h->h_fitems.size();
  L.upd.off = (int)h->h_uitems.size();
  for (auto& gb : grid_bands) add_grid_items(h, gb.first, gb.second, h->h_fitems, h->h_uitems);
  L.flux.n = (int)h->h_fitems.size() - L.flux.off;
  L.upd.n = (int)h->h_uitems.size() - L.upd.off;
  return L;
}

int64_t cells_of(const amr_grid& G) {
  return (int64_t)(G.hi[0] - G.lo[0]) * (G.hi[1] - G.lo[1]) * (G.hi[2] - G.lo[2]);
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
      const int gv = l == 0 ? h->g : h->g - 2 * (k % h->R);
      std::vector<int> gl = h->level_grids[l];
      std::stable_sort(gl.begin(), gl.end(),
                       [&](int a, int b) { return cells_of(h->grids[a]) > cells_of(h->grids[b]); });
      for (int gi : gl) gb.push_back({gi, gv});
    }
    h->cycle_lists.push_back(make_list(h, gb));
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
  h->d_fitems = dev_upload(h->h_fitems);
  h->d_uitems = dev_upload(h->h_uitems);
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
  h->copy_cls.assign(h->nlev, make_int4(0, 0, 0, 0));
  h->d_pcell.assign(h->nlev, nullptr);
  h->d_pface.assign(h->nlev, nullptr);
  h->n_pcell.assign(h->nlev, 0);
  h->n_pface.assign(h->nlev, 0);

  for (int l = 0; l < h->nlev; ++l) {
    const LevelIndex& LI = idx[l];
    std::vector<CopyEntry> cp[4];
    std::vector<ProlongEntry> pc, pf;
    for (int gi : h->level_grids[l]) {
      const GridDesc& G = h->desc[gi];
      const amr_grid& GG = h->grids[gi];
      for (int cls = 0; cls < ncls; ++cls) {
        int lo[3], hi[3];
        class_extent(G, nd, cls, lo, hi);
        for (int k = lo[2]; k < hi[2]; ++k)
          for (int j = lo[1]; j < hi[1]; ++j)
            for (int i = lo[0]; i < hi[0]; ++i) {
              const int x[3] = {i, j, k};
              if (own_elem(G, nd, cls, x)) continue;
              // global position, then (for level 0 outflow) clamp into the domain
              int p[3] = {GG.lo[0] + i, GG.lo[1] + j, GG.lo[2] + k};
              bool outside = false;
              for (int a = 0; a < nd; ++a) {
                if (h->p.bc[a] == AMR_BC_PERIODIC) continue;
                const int top = (cls == 1 + a) ? LI.N[a] : LI.N[a] - 1;
                if (p[a] < 0) { p[a] = 0; outside = true; }
                if (p[a] > top) { p[a] = top; outside = true; }
              }
              (void)outside;
              // find a same-level source: the element must be a cell of, or a
              // face on the boundary of, another grid's interior (lowest id)
              int src_grid = -1;
              int sp[3] = {0, 0, 0};
              // candidates: the cell itself and, for faces, the cell below
              // along the normal (faces on a grid's high boundary)
              for (int cand = 0; cand < 2 && src_grid < 0; ++cand) {
                if (cand == 1 && cls == 0) break;
                int c[3] = {p[0], p[1], p[2]};
                if (cand == 1) c[cls - 1] -= 1;
                int w[3] = {c[0], c[1], c[2]};
                if (!LI.wrap(w)) continue;
                int s = LI.find_cell(w);
                if (s < 0) continue;
                // the element itself, in the wrapped frame of grid s
                int e[3] = {w[0], w[1], w[2]};
                if (cand == 1) e[cls - 1] += 1;
                // prefer the lowest grid id among grids sharing a face
                if (cand == 0 && cls > 0) {
                  int c2[3] = {w[0], w[1], w[2]};
                  c2[cls - 1] -= 1;
                  int w2[3] = {c2[0], c2[1], c2[2]};
                  if (LI.wrap(w2)) {
                    int s2 = LI.find_cell(w2);
                    if (s2 >= 0 && s2 < s) {
                      s = s2;
                      e[0] = w2[0];
                      e[1] = w2[1];
                      e[2] = w2[2];
                      e[cls - 1] += 1;
                    }
                  }
                }
                if (s == gi) {
                  // own grid through a periodic image: allowed only if the
                  // element differs from this band position
                  bool same = e[0] == GG.lo[0] + i && e[1] == GG.lo[1] + j && e[2] == GG.lo[2] + k;
                  if (same) continue;
                }
                src_grid = s;
                sp[0] = e[0];
                sp[1] = e[1];
                sp[2] = e[2];
              }
              const int64_t dst = elem(G, nd, i, j, k);
              if (src_grid >= 0) {
                const GridDesc& S = h->desc[src_grid];
                const amr_grid& SG = h->grids[src_grid];
                const int64_t src = elem(S, nd, sp[0] - SG.lo[0], sp[1] - SG.lo[1], sp[2] - SG.lo[2]);
                cp[cls].push_back(CopyEntry{(int32_t)dst, (int32_t)src});
                continue;
              }
              if (l == 0) throw Error(AMR_EINVAL, "level 0 does not tile the domain (uncovered band element)");
              // prolongation from level l-1
              const LevelIndex& PI = idx[l - 1];
              const int gpos[3] = {GG.lo[0] + i, GG.lo[1] + j, GG.lo[2] + k};
              if (cls == 0) {
                int cc[3] = {floordiv(gpos[0], 2), floordiv(gpos[1], 2), nd == 3 ? floordiv(gpos[2], 2) : 0};
                if (!PI.wrap(cc)) throw Error(AMR_EINVAL, "prolongation source outside the domain");
                int pg = PI.find_cell(cc);
                if (pg < 0) throw Error(AMR_EINVAL, "proper nesting violated: band cell has no parent");
                const GridDesc& P = h->desc[pg];
                const amr_grid& PG = h->grids[pg];
                int code = 0;
                for (int a = 0; a < nd; ++a) code |= (posmod(gpos[a], 2) << a);
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
                if (PI.wrap(w)) pg = PI.find_cell(w);
                if (!mid && pg < 0) {
                  int w2[3] = {cc[0], cc[1], cc[2]};
                  w2[d] -= 1;
                  if (PI.wrap(w2)) {
                    pg = PI.find_cell(w2);
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
    std::vector<CopyEntry> all;
    int4 cls = make_int4(0, 0, 0, 0);
    for (int c = 0; c < 4; ++c) {
      all.insert(all.end(), cp[c].begin(), cp[c].end());
      int v = (int)all.size();
      if (c == 0) cls.x = v;
      if (c == 1) cls.y = v;
      if (c == 2) cls.z = v;
      if (c == 3) cls.w = v;
    }
    h->copy_cls[l] = cls;
    h->n_copy[l] = (int)all.size();
    h->d_copy[l] = dev_upload(all);
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
    for (int gi : h->level_grids[l]) {
      const amr_grid& G = h->grids[gi];
      int lo[3], hi[3];
      for (int a = 0; a < 3; ++a) {
        lo[a] = a < nd ? G.lo[a] / h->R - buf : 0;
        hi[a] = a < nd ? G.hi[a] / h->R + buf : 1;
      }
      for (int k = lo[2]; k < hi[2]; ++k)
        for (int j = lo[1]; j < hi[1]; ++j)
          for (int i = lo[0]; i < hi[0]; ++i) {
            int c[3] = {i, j, k};
            if (!PI.wrap(c) || PI.find_cell(c) < 0)
              throw Error(AMR_EINVAL, "grid " + std::to_string(gi) + " violates proper nesting");
          }
    }
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

template <class T> DevState<T> dstate(const amr_state* s) {
  DevState<T> d;
  for (int i = 0; i < 8; ++i) d.f[i] = (T*)s->f[i];
  return d;
}

template <class T> DevFlux<T> dflux(const amr_hierarchy* h, void* ws) {
  DevFlux<T> F;
  char* base = (char*)ws;
  const int64_t stride = h->total_elems * (int64_t)sizeof(T);
  for (int d = 0; d < 3; ++d)
    for (int q = 0; q < 7; ++q) F.f[d][q] = (T*)(base + (int64_t)(d * 7 + q) * stride);
  return F;
}

Phys phys(const amr_hierarchy* h) {
  Phys ph;
  ph.gamma = h->p.gamma;
  for (int d = 0; d < 3; ++d) ph.dx0[d] = h->p.dx0[d];
  ph.ndim = h->ndim;
  ph.ratio = h->R;
  return ph;
}

amr_status fail(const std::exception& e) {
  g_last_error = e.what();
  if (auto* er = dynamic_cast<const Error*>(&e)) return er->code;
  return AMR_ENOMEM;
}

template <class T>
void run_list(amr_hierarchy* h, const LaunchList& L, const amr_state* Uin, amr_state* Uout, const double* dt0,
              void* ws, hipStream_t s) {
  DevState<T> ui = dstate<T>(Uin), uo = dstate<T>(Uout);
  DevFlux<T> F = dflux<T>(h, ws);
  Phys ph = phys(h);
  int e0 = 0, e1 = 0, e2 = 0;
  if (h->timing) {
    e0 = h->take_event();
    e1 = h->take_event();
    e2 = h->take_event();
    HIPCHK(hipEventRecord(h->ev_pool[e0], s));
  }
  launch_flux<T>(h->ndim, h->d_desc, h->d_fitems + L.flux.off, L.flux.n, ui, F, dt0, ph, h->d_err, s);
  HIPCHK(hipGetLastError());
  if (h->timing) HIPCHK(hipEventRecord(h->ev_pool[e1], s));
  launch_update<T>(h->ndim, h->d_desc, h->d_uitems + L.upd.off, L.upd.n, ui, uo, F, dt0, ph, s);
  HIPCHK(hipGetLastError());
  if (h->timing) {
    HIPCHK(hipEventRecord(h->ev_pool[e2], s));
    h->ev_pairs[0].push_back({e0, e1});
    h->ev_pairs[1].push_back({e1, e2});
  }
}

}  // namespace

extern "C" {

const char* amr_last_error(void) { return g_last_error.c_str(); }

const char* amr_strerror(amr_status s) {
  switch (s) {
    case AMR_OK: return "ok";
    case AMR_EINVAL: return "invalid argument or hierarchy";
    case AMR_EHIP: return "HIP runtime error";
    case AMR_ENOMEM: return "out of memory";
    case AMR_ESTATE: return "non-physical state on the device";
    case AMR_EUNSUPPORTED: return "unsupported request";
  }
  return "unknown status";
}

amr_status amr_create(const amr_params* p, const amr_grid* grids, int32_t ngrids, amr_hierarchy** out) {
  if (out) *out = nullptr;
  amr_hierarchy* h = nullptr;
  try {
    if (!out) throw Error(AMR_EINVAL, "out is NULL");
    validate(p, grids, ngrids);
    h = new amr_hierarchy();
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
    h->flux_bytes = 21 * off * (int64_t)h->esize;
    h->reg_offset = (h->flux_bytes + 255) / 256 * 256;
    check_nesting(h);
    h->d_desc = dev_upload(h->desc);
    build_fill_maps(h);
    build_lists(h);
    h->sync.resize(h->nlev);
    int64_t reg_bytes = 0;
    for (int l = 1; l < h->nlev; ++l) reg_bytes += build_sync_tables(h->ndim, h->R, h->desc, h->grids, h->level_grids,
                                                                     h->p, l, h->sync[l], h->reg_offset + reg_bytes,
                                                                     h->esize);
    h->workspace_bytes = h->reg_offset + reg_bytes;
    HIPCHK(hipMalloc((void**)&h->d_err, 256));
    HIPCHK(hipMemset(h->d_err, 0, 256));
    HIPCHK(hipDeviceSynchronize());
    *out = h;
    return AMR_OK;
  } catch (const std::exception& e) {
    delete h;
    return fail(e);
  }
}

amr_status amr_destroy(amr_hierarchy* h) {
  if (!h) return AMR_EINVAL;
  (void)hipDeviceSynchronize();
  delete h;
  return AMR_OK;
}

amr_status amr_layout(const amr_hierarchy* h, int64_t* state_elems, int64_t* workspace_bytes,
                      int64_t* grid_offsets) {
  if (!h) return AMR_EINVAL;
  if (state_elems) *state_elems = h->total_elems;
  if (workspace_bytes) *workspace_bytes = h->workspace_bytes;
  if (grid_offsets)
    for (size_t i = 0; i < h->desc.size(); ++i) grid_offsets[i] = h->desc[i].off;
  return AMR_OK;
}

amr_status amr_load_primitive(amr_hierarchy* h, int32_t grid, const double* const* prim, const double* const* b,
                              amr_state* U, void* stream) {
  try {
    if (!h || !prim || !b || !U) throw Error(AMR_EINVAL, "null argument");
    if (grid < 0 || grid >= (int)h->desc.size()) throw Error(AMR_EINVAL, "grid index out of range");
    hipStream_t s = (hipStream_t)stream;
    if (h->esize == 8)
      launch_load_prim<double>(h->ndim, h->desc[grid], prim, b, dstate<double>(U), h->p.gamma, s);
    else
      launch_load_prim<float>(h->ndim, h->desc[grid], prim, b, dstate<float>(U), h->p.gamma, s);
    HIPCHK(hipGetLastError());
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_store_interior(amr_hierarchy* h, int32_t grid, const amr_state* U, double* const* out,
                              void* stream) {
  try {
    if (!h || !U || !out) throw Error(AMR_EINVAL, "null argument");
    if (grid < 0 || grid >= (int)h->desc.size()) throw Error(AMR_EINVAL, "grid index out of range");
    hipStream_t s = (hipStream_t)stream;
    if (h->esize == 8)
      launch_store<double>(h->ndim, h->desc[grid], dstate<double>(U), out, s);
    else
      launch_store<float>(h->ndim, h->desc[grid], dstate<float>(U), out, s);
    HIPCHK(hipGetLastError());
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_compute_dt(amr_hierarchy* h, const amr_state* U, double* dt0, void* workspace, void* stream) {
  try {
    if (!h || !U || !dt0) throw Error(AMR_EINVAL, "null argument");
    (void)workspace;
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* acc = (unsigned long long*)((char*)h->d_err + 64);
    if (h->esize == 8)
      launch_cfl<double>(h->ndim, h->d_desc, h->d_cfl, h->n_cfl, dstate<double>(U), phys(h), acc, h->d_err, h->p.cfl,
                         dt0, s);
    else
      launch_cfl<float>(h->ndim, h->d_desc, h->d_cfl, h->n_cfl, dstate<float>(U), phys(h), acc, h->d_err, h->p.cfl,
                        dt0, s);
    HIPCHK(hipGetLastError());
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_fill_ghosts_prolong(amr_hierarchy* h, int32_t level, int32_t mode, amr_state* U, void* stream) {
  try {
    if (!h || !U) throw Error(AMR_EINVAL, "null argument");
    if (level < 0 || level >= h->nlev) throw Error(AMR_EINVAL, "level out of range");
    if (mode != AMR_FILL_FULL && mode != AMR_FILL_SAME_LEVEL) throw Error(AMR_EINVAL, "bad fill mode");
    hipStream_t s = (hipStream_t)stream;
    // copies first, then prolongation (prolongation reads only the parent level)
    if (h->esize == 8) {
      launch_copy<double>(h->ndim, h->d_copy[level], h->n_copy[level], h->copy_cls[level], dstate<double>(U), s);
      if (mode == AMR_FILL_FULL && level > 0)
        launch_prolong<double>(h->ndim, h->d_pcell[level], h->n_pcell[level], h->d_pface[level], h->n_pface[level],
                               h->d_desc, dstate<double>(U), phys(h), s);
    } else {
      launch_copy<float>(h->ndim, h->d_copy[level], h->n_copy[level], h->copy_cls[level], dstate<float>(U), s);
      if (mode == AMR_FILL_FULL && level > 0)
        launch_prolong<float>(h->ndim, h->d_pcell[level], h->n_pcell[level], h->d_pface[level], h->n_pface[level],
                              h->d_desc, dstate<float>(U), phys(h), s);
    }
    HIPCHK(hipGetLastError());
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_advance_patches(amr_hierarchy* h, int32_t cycle, const int32_t* grid_subset, int32_t nsubset,
                               int32_t band, const amr_state* U_in, amr_state* U_out, const double* dt0,
                               void* workspace, void* stream) {
  try {
    if (!h || !U_in || !U_out || !dt0 || !workspace) throw Error(AMR_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    std::vector<const LaunchList*> lists;
    if (cycle >= 0) {
      if (band > 0) {
        if (h->nlev != 1) throw Error(AMR_EINVAL, "an explicit band with a batched cycle needs a single level");
        auto it = h->level0_band_lists.find(band);
        if (it == h->level0_band_lists.end()) throw Error(AMR_EINVAL, "band must be in [2, ghost]");
        lists.push_back(&it->second);
      } else {
        if (cycle >= (int)h->cycle_lists.size()) throw Error(AMR_EINVAL, "cycle out of range");
        lists.push_back(&h->cycle_lists[cycle]);
      }
    } else {
      if (!grid_subset || nsubset <= 0) throw Error(AMR_EINVAL, "per-grid path needs a grid list");
      for (int i = 0; i < nsubset; ++i) {
        auto it = h->grid_lists.find({grid_subset[i], band});
        if (it == h->grid_lists.end()) throw Error(AMR_EINVAL, "bad grid id or band for the per-grid path");
        lists.push_back(&it->second);
      }
    }
    for (const LaunchList* L : lists) {
      if (h->esize == 8)
        run_list<double>(h, *L, U_in, U_out, dt0, workspace, s);
      else
        run_list<float>(h, *L, U_in, U_out, dt0, workspace, s);
    }
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_restrict_fluxfix(amr_hierarchy* h, int32_t fine_level, const amr_state* U_fine, amr_state* U_coarse,
                                void* workspace, void* stream) {
  (void)h; (void)fine_level; (void)U_fine; (void)U_coarse; (void)workspace; (void)stream;
  g_last_error = "amr_restrict_fluxfix: not built yet";
  return AMR_EUNSUPPORTED;
}

amr_status amr_advance_adjoint(amr_hierarchy* h, int32_t grid_or_level, int32_t nsteps, const double* dts,
                               const amr_state* U_checkpoint, amr_state* lambda_inout, void* workspace,
                               void* stream) {
  (void)h; (void)grid_or_level; (void)nsteps; (void)dts; (void)U_checkpoint; (void)lambda_inout; (void)workspace;
  (void)stream;
  g_last_error = "amr_advance_adjoint: not built yet";
  return AMR_EUNSUPPORTED;
}

amr_status amr_set_kernel_timing(amr_hierarchy* h, int32_t enable) {
  if (!h) return AMR_EINVAL;
  h->timing = enable != 0;
  h->ev_pairs[0].clear();
  h->ev_pairs[1].clear();
  h->ev_used = 0;
  return AMR_OK;
}

amr_status amr_kernel_times(amr_hierarchy* h, double* flux_ms, double* update_ms, int64_t* nlaunch) {
  try {
    if (!h) throw Error(AMR_EINVAL, "null handle");
    double acc[2] = {0.0, 0.0};
    for (int k = 0; k < 2; ++k)
      for (auto& pr : h->ev_pairs[k]) {
        HIPCHK(hipEventSynchronize(h->ev_pool[pr.second]));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->ev_pool[pr.first], h->ev_pool[pr.second]));
        acc[k] += ms;
      }
    if (flux_ms) *flux_ms = acc[0];
    if (update_ms) *update_ms = acc[1];
    if (nlaunch) *nlaunch = (int64_t)h->ev_pairs[0].size();
    h->ev_pairs[0].clear();
    h->ev_pairs[1].clear();
    h->ev_used = 0;
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_get_error_flags(amr_hierarchy* h, uint32_t* flags, int64_t* first_bad_cell) {
  try {
    if (!h) throw Error(AMR_EINVAL, "null handle");
    ErrBlock e{};
    HIPCHK(hipDeviceSynchronize());
    HIPCHK(hipMemcpy(&e, h->d_err, sizeof(e), hipMemcpyDeviceToHost));
    if (flags) *flags = e.flags;
    if (first_bad_cell) *first_bad_cell = e.flags ? e.first_bad : -1;
    ErrBlock z{};
    HIPCHK(hipMemcpy(h->d_err, &z, sizeof(z), hipMemcpyHostToDevice));
    return e.flags ? AMR_ESTATE : AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

}  // extern "C"
