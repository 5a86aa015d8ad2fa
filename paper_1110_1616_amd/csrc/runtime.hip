// Host runtime and C ABI of libamrmhd.so (see include/amr.h).
//
// amr_create() validates the hierarchy and builds, once, every device table
// the hot path needs: grid descriptors, ghost-fill gather maps, batched work
// lists of each launch cycle (finest level first) and per-grid lists for
// the per-grid path.  The calls after that only enqueue kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <exception>
#include <mutex>
#include <thread>
#include <type_traits>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/amr.h"
#include "adjoint_internal.hpp"
#include "amr_internal.hpp"
#include "fill_internal.hpp"
#include "frozen_internal.hpp"
#include "regrid_internal.hpp"
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

// When set, table builders run on the host only (amr_validate).
thread_local bool g_host_only = false;

template <class T> T* dev_upload(const std::vector<T>& v) {
  if (v.empty() || g_host_only) return nullptr;
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
  ListRef flux, upd, emf;
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
  UpdItem* d_eitems = nullptr;  // upwinded EMF only: edge-EMF tiles
  std::vector<UpdItem> h_eitems;
  std::vector<FluxItem> h_fitems;
  std::vector<UpdItem> h_uitems;
  int4* d_cfl = nullptr;
  int n_cfl = 0;
  ErrBlock* d_err = nullptr;  // error block + CFL accumulator (handle-owned)

  // fill maps per level (host copies of the same-level copy maps are kept
  // for the adjoint's transpose)
  std::vector<std::vector<CopyEntry>> h_copy;
  std::vector<CopyEntry*> d_copy;
  std::vector<int> n_copy;
  std::vector<int4> copy_cls;
  // the copy entries within 2 cells of each interior: the same-level fills
  // before a step from band 2 (level 0, and the refresh before substeps k >= 1)
  std::vector<CopyEntry*> d_copy2;
  std::vector<int> n_copy2;
  std::vector<int4> copy2_cls;
  std::vector<ProlongEntry*> d_pcell, d_pface;
  std::vector<int> n_pcell, n_pface;

  // synchronisation tables per fine level
  std::vector<SyncTables> sync;

  // launch lists
  std::vector<LaunchList> cycle_lists;                 // per launch cycle (batched)
  // eta-balanced schedule: the grids of a level step anywhere inside the
  // cycles of their step's window (see plan_eta); predicted work per cycle
  int schedule = 0;  // 0: every level at the start of its window; 1: eta-balanced
  bool upwind_emf = false;  // edge EMF of CT: arithmetic mean or upwinded
  std::vector<LaunchList> eta_lists;
  std::vector<double> cycle_work[2];
  std::map<std::pair<int, int>, LaunchList> grid_lists;  // (grid, band) -> per-grid list
  std::map<int, LaunchList> level0_band_lists;          // band -> all level-0 grids
  std::vector<LaunchList> band2_lists;                  // per level: all its grids, band 2

  // adjoint tables per level, built on first use
  struct AdjTables {
    bool built = false;
    int2* d_items = nullptr;  // (grid, first local element) of 256-element chunks
    int nitems = 0;
    InvCopy* d_inv = nullptr;  // band copy transposed: source -> its band images
    int ninv = 0;
    int32_t* d_dsts = nullptr;
    int64_t e0 = 0, e1 = 0;  // element range of the level's grids
  };
  std::vector<AdjTables> adj;
  // refinement-flag work items per level, built on first use
  std::vector<FlagItem*> d_flag_items;
  std::vector<int> n_flag_items;
  int zchunk = 16;
  int upd_zchunk = 2;  // planes per update / edge-EMF work item (the update prefers short ones)
  int tile_policy = 1;  // 0: 16 x 16 tiles; 1: per-grid width with the fewest tiles
  bool persistent = false;     // persistent launches popping d_queue, or one block per item
  bool persistent_flux = false;  // the flux kernel persistent (implied by `persistent`)
  bool xcd_chunks = false;     // item lists cut into one contiguous chunk per XCD
  WorkQueue* d_queue = nullptr;
  int flux_pblocks = 0, upd_pblocks = 0;  // persistent grid sizes (resident blocks on the device)

  // captured coarse steps: graph[p] starts from level-0 parity bit p
  hipGraphExec_t graph_exec[2] = {nullptr, nullptr};
  uint32_t graph_parity[2] = {0, 0};
  bool capturing = false;

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
    for (auto g : graph_exec)
      if (g) (void)hipGraphExecDestroy(g);
    for (auto e : ev_pool) (void)hipEventDestroy(e);
    (void)hipFree(d_desc);
    (void)hipFree(d_fitems);
    (void)hipFree(d_uitems);
    (void)hipFree(d_eitems);
    (void)hipFree(d_cfl);
    (void)hipFree(d_err);
    (void)hipFree(d_queue);
    for (auto p : d_copy) (void)hipFree(p);
    for (auto p : d_copy2) (void)hipFree(p);
    for (auto p : d_pcell) (void)hipFree(p);
    for (auto p : d_pface) (void)hipFree(p);
    for (auto& s : sync) s.release();
    for (auto p : d_flag_items) (void)hipFree(p);
    for (auto& a : adj) {
      (void)hipFree(a.d_items);
      (void)hipFree(a.d_inv);
      (void)hipFree(a.d_dsts);
    }
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
  bool holds(int gi, const int (&c)[3]) const {
    if (gi < 0 || gi >= (int)h->grids.size()) return false;
    const amr_grid& G = h->grids[gi];
    if (G.level != level) return false;
    for (int d = 0; d < 3; ++d)
      if (c[d] < G.lo[d] || c[d] >= G.hi[d]) return false;
    return true;
  }
  // Grid whose interior holds cell c (already wrapped), or -1.  Lookups come
  // in runs from one grid, so each thread first tries its last two hits (the
  // grids of a level are disjoint: a grid of this level holding c is the
  // answer, whatever lookup produced it).
  int find_cell(const int (&c)[3]) const {
    thread_local int memo[2] = {-1, -1};
    thread_local unsigned turn = 0;
    for (int m = 0; m < 2; ++m)
      if (holds(memo[m], c)) return memo[m];
    auto it = buckets.find(key(floordiv(c[0], B), floordiv(c[1], B), floordiv(c[2], B)));
    if (it == buckets.end()) return -1;
    for (int gi : it->second) {
      if (holds(gi, c)) {
        memo[turn++ & 1] = gi;
        return gi;
      }
    }
    return -1;
  }
};

// Pool element of (i, j, k) in grid G; every table entry goes through here,
// so an index outside the grid's padded box is caught on the host.
int64_t elem(const GridDesc& G, int ndim, int i, int j, int k) {
  const int gz = ndim == 3 ? G.g : 0;
  const int x[3] = {i, j, k};
  for (int a = 0; a < 3; ++a) {
    const int lo = a < ndim ? -G.g : 0, hi = a < ndim ? G.n[a] + G.g : 0;
    if (x[a] < lo || x[a] > hi) throw Error(AMR_EINVAL, "internal: table element outside its grid's box");
  }
  return G.off + (int64_t)(i + G.g) + (int64_t)(j + G.g) * G.P[0] + (int64_t)(k + gz) * G.P[0] * G.P[1];
}

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
  for (int z0 = zlo; z0 < ch[2]; z0 += (h->ndim == 3 ? zc : 1))
    for (int y0 = cl; y0 < ch[1]; y0 += fth - 1)
      for (int x0 = cl; x0 < ch[0]; x0 += ftw - 1) {
        FluxItem it{};
        it.tw = ftw;
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
  for (auto& gb : grid_bands) add_grid_items(h, gb.first, gb.second, h->h_fitems, h->h_uitems);
  L.emf.n = (int)h->h_eitems.size() - L.emf.off;
  L.flux.n = (int)h->h_fitems.size() - L.flux.off;
  L.upd.n = (int)h->h_uitems.size() - L.upd.off;
  // longest flux items first inside each eighth of the list (the XCD chunks
  // of the launch): blocks take items in list order, so the short ones
  // (a grid's last z-chunk) fill the end of the launch instead of starting
  // late; items stay in their chunk, next to the tiles they share halos with
  const int C = (L.flux.n + 7) / 8;
  for (int c = 0; c < 8 && c * C < L.flux.n; ++c) {
    auto b = h->h_fitems.begin() + L.flux.off + c * C;
    auto e = h->h_fitems.begin() + L.flux.off + std::min(L.flux.n, (c + 1) * C);
    std::stable_sort(b, e, [](const FluxItem& x, const FluxItem& y) { return x.z1 - x.z0 > y.z1 - y.z0; });
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

// Run fn(i) for i in [0, n) on up to hardware_concurrency() threads; the
// first exception thrown by any call is rethrown here.
template <class Fn> void parallel_for(size_t n, Fn&& fn) {
  const unsigned hw = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
  const unsigned nt = (unsigned)std::min<size_t>(hw, n);
  if (nt <= 1) {
    for (size_t i = 0; i < n; ++i) fn(i);
    return;
  }
  std::atomic<size_t> next{0};
  std::exception_ptr err;
  std::mutex mu;
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < nt; ++t)
    pool.emplace_back([&]() {
      for (;;) {
        const size_t i = next.fetch_add(1);
        if (i >= n) return;
        try {
          fn(i);
        } catch (...) {
          std::lock_guard<std::mutex> g(mu);
          if (!err) err = std::current_exception();
          next.store(n);
          return;
        }
      }
    });
  for (auto& th : pool) th.join();
  if (err) std::rethrow_exception(err);
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
                int pg = PI.find_cell(cc);
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
    // grid order; prolongations in grid order
    size_t ncp[4] = {0, 0, 0, 0}, npc = 0, npf = 0;
    for (const GridMaps& m : per) {
      for (int c = 0; c < 4; ++c) ncp[c] += m.cp[c].size();
      npc += m.pc.size();
      npf += m.pf.size();
    }
    std::vector<CopyEntry> all;
    all.reserve(ncp[0] + ncp[1] + ncp[2] + ncp[3]);
    int4 cls = make_int4(0, 0, 0, 0);
    for (int c = 0; c < 4; ++c) {
      for (const GridMaps& m : per) all.insert(all.end(), m.cp[c].begin(), m.cp[c].end());
      int v = (int)all.size();
      if (c == 0) cls.x = v;
      if (c == 1) cls.y = v;
      if (c == 2) cls.z = v;
      if (c == 3) cls.w = v;
    }
    std::vector<CopyEntry> all2;
    int4 cls2 = make_int4(0, 0, 0, 0);
    for (int c = 0; c < 4; ++c) {
      for (const GridMaps& m : per) all2.insert(all2.end(), m.cp2[c].begin(), m.cp2[c].end());
      int v = (int)all2.size();
      if (c == 0) cls2.x = v;
      if (c == 1) cls2.y = v;
      if (c == 2) cls2.z = v;
      if (c == 3) cls2.w = v;
    }
    h->copy2_cls[l] = cls2;
    h->n_copy2[l] = (int)all2.size();
    h->d_copy2[l] = dev_upload(all2);
    std::vector<ProlongEntry> pc, pf;
    pc.reserve(npc);
    pf.reserve(npf);
    for (GridMaps& m : per) {
      pc.insert(pc.end(), m.pc.begin(), m.pc.end());
      pf.insert(pf.end(), m.pf.begin(), m.pf.end());
      m = GridMaps();
    }
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


// ------------------------------------------------------------ sync tables
// Coarse/fine registers, reflux, EMF-fix and restriction entries of fine
// level f (see sync_internal.hpp).  Positions on periodic levels are taken in
// the frame of the grid that stores them.
void build_sync_tables(amr_hierarchy* h, int f) {
  const int nd = h->ndim, R = h->R, c = f - 1;
  LevelIndex CI, FI;
  CI.build(h, c);
  FI.build(h, f);
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
  auto fine_owner = [&](const int (&p)[3], int (&shift)[3]) {
    int w[3] = {p[0], p[1], p[2]};
    if (!FI.wrap(w)) return -1;
    for (int a = 0; a < 3; ++a) shift[a] = w[a] - p[a];
    return FI.find_cell(w);
  };
  const double dxc[3] = {h->p.dx0[0] / ipow(R, c), h->p.dx0[1] / ipow(R, c), nd == 3 ? h->p.dx0[2] / ipow(R, c) : 1.0};
  SyncTables& T = h->sync[f];
  std::vector<FaceRegEntry> frc, frf;
  std::vector<EdgeRegEntry> erc, erf;
  std::vector<RefluxEntry> rfx;
  std::vector<EmfFixEntry> efx;
  std::vector<RestrictEntry> rst;
  std::map<std::vector<int>, int> edge_id;
  int nfreg = 0;

  for (int gi : h->level_grids[c]) {
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
                std::vector<int> key = {ea, w[0], w[1], w[2]};
                int re;
                auto it = edge_id.find(key);
                if (it == edge_id.end()) {
                  re = (int)edge_id.size();
                  edge_id[key] = re;
                  EdgeRegEntry ec{};
                  ec.reg = re;
                  ec.a = ea;
                  ec.grid = gi;
                  ec.n = 1;
                  ec.e[0] = (int32_t)elem(C, nd, e[0] - CG.lo[0], e[1] - CG.lo[1], e[2] - CG.lo[2]);
                  erc.push_back(ec);
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
                  erf.push_back(ef);
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
  }
  T.nfreg = nfreg;
  T.nereg = (int)edge_id.size();
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
  for (int a = 0; a < 3; ++a) {
    F.e[a] = h->upwind_emf ? (T*)(base + (int64_t)(21 + a) * stride) : nullptr;
    F.edge[a] = h->upwind_emf ? (T*)(base + (int64_t)(24 + a) * stride) : nullptr;
  }
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
void run_list(amr_hierarchy* h, const LaunchList& L, const amr_state* Ua, const amr_state* Ub, uint32_t parity,
              const double* dt0, void* ws, hipStream_t s) {
  DevState<T> s0 = dstate<T>(Ua), s1 = dstate<T>(Ub);
  DevFlux<T> F = dflux<T>(h, ws);
  Phys ph = phys(h);
  int e0 = 0, e1 = 0, e2 = 0;
  const bool timing = h->timing && !h->capturing;
  if (timing) {
    e0 = h->take_event();
    e1 = h->take_event();
    e2 = h->take_event();
    HIPCHK(hipEventRecord(h->ev_pool[e0], s));
  }
  launch_flux<T>(h->ndim, h->d_desc, h->d_fitems + L.flux.off, L.flux.n, s0, s1, parity, F, dt0, ph, h->d_err,
                 h->d_queue, h->persistent_flux ? h->flux_pblocks : 0, h->xcd_chunks, h->upwind_emf, s);
  HIPCHK(hipGetLastError());
  if (timing) HIPCHK(hipEventRecord(h->ev_pool[e1], s));
  if constexpr (std::is_same<T, float>::value || std::is_same<T, double>::value) {
    if (h->upwind_emf) {
      launch_emf<T>(h->ndim, h->d_desc, h->d_eitems + L.emf.off, L.emf.n, F, s);
      HIPCHK(hipGetLastError());
    }
  }
  launch_update<T>(h->ndim, h->d_desc, h->d_uitems + L.upd.off, L.upd.n, s0, s1, parity, F, dt0, ph, h->d_queue,
                   h->persistent ? h->upd_pblocks : 0, h->xcd_chunks, h->upwind_emf, s);
  HIPCHK(hipGetLastError());
  if (timing) {
    HIPCHK(hipEventRecord(h->ev_pool[e2], s));
    h->ev_pairs[0].push_back({e0, e1});
    h->ev_pairs[1].push_back({e1, e2});
  }
}

// Registers written after level l stepped at its substep k: the coarse side
// of the sync with level l+1 and the fine side (slot 1 + k mod R) of the sync
// with level l-1.
template <class T>
void write_registers(amr_hierarchy* h, int l, int k, const double* dt0, void* ws, hipStream_t s) {
  DevFlux<T> F = dflux<T>(h, ws);
  const double div = (double)ipow(h->R, l);
  if (l + 1 < h->nlev) {
    const SyncTables& t = h->sync[l + 1];
    T* freg = (T*)((char*)ws + t.reg_off);
    T* ereg = (T*)((char*)ws + t.reg_off + ((int64_t)(1 + h->R) * t.nfreg * 6 * (int64_t)sizeof(T) + 255) / 256 * 256);
    launch_registers<T>(h->ndim, h->d_desc, t.d_freg_c, t.n_freg_c, t.d_ereg_c, t.n_ereg_c, F, freg, ereg, t.nfreg,
                        t.nereg, 0, dt0, div, h->upwind_emf, s);
    HIPCHK(hipGetLastError());
  }
  if (l >= 1) {
    const SyncTables& t = h->sync[l];
    T* freg = (T*)((char*)ws + t.reg_off);
    T* ereg = (T*)((char*)ws + t.reg_off + ((int64_t)(1 + h->R) * t.nfreg * 6 * (int64_t)sizeof(T) + 255) / 256 * 256);
    launch_registers<T>(h->ndim, h->d_desc, t.d_freg_f, t.n_freg_f, t.d_ereg_f, t.n_ereg_f, F, freg, ereg, t.nfreg,
                        t.nereg, 1 + k % h->R, dt0, div, h->upwind_emf, s);
    HIPCHK(hipGetLastError());
  }
}

template <class T>
void do_sync(amr_hierarchy* h, int f, const amr_state* Uf, amr_state* Uc, void* ws, hipStream_t s) {
  // the synchronisation kernels are unrolled over ratio 2, the only one a
  // multi-level hierarchy accepts
  if (h->R != 2) throw Error(AMR_EUNSUPPORTED, "synchronisation needs refinement ratio 2");
  const SyncTables& t = h->sync[f];
  const T* freg = (const T*)((char*)ws + t.reg_off);
  const T* ereg =
      (const T*)((char*)ws + t.reg_off + ((int64_t)(1 + h->R) * t.nfreg * 6 * (int64_t)sizeof(T) + 255) / 256 * 256);
  launch_sync<T>(h->ndim, h->R, h->d_desc, t, freg, ereg, dstate<T>(Uf), dstate<T>(Uc), s);
  HIPCHK(hipGetLastError());
}

template <class T>
void do_fill(amr_hierarchy* h, int level, int mode, amr_state* Ul, const amr_state* Up, hipStream_t s,
             bool band2_only = false) {
  if (band2_only)
    launch_copy<T>(h->ndim, h->d_copy2[level], h->n_copy2[level], h->copy2_cls[level], dstate<T>(Ul), s);
  else
    launch_copy<T>(h->ndim, h->d_copy[level], h->n_copy[level], h->copy_cls[level], dstate<T>(Ul), s);
  if (mode == AMR_FILL_FULL && level > 0)
    launch_prolong<T>(h->ndim, h->d_pcell[level], h->n_pcell[level], h->d_pface[level], h->n_pface[level], h->d_desc,
                      dstate<T>(Up), dstate<T>(Ul), phys(h), s);
  HIPCHK(hipGetLastError());
}

template <class T>
void do_dt(amr_hierarchy* h, const amr_state* Ua, const amr_state* Ub, uint32_t parity, double* dt0, hipStream_t s) {
  unsigned long long* acc = (unsigned long long*)((char*)h->d_err + 64);
  launch_cfl<T>(h->ndim, h->d_desc, h->d_cfl, h->n_cfl, dstate<T>(Ua), dstate<T>(Ub), parity, phys(h), acc, h->d_err,
                h->p.cfl, dt0, s);
  HIPCHK(hipGetLastError());
}

// One coarse step of the whole hierarchy.  mode 0: batched launch cycles
// (every level stepping in a cycle in one launch, finest level first); mode
// 1: the serial level order with one launch per grid (the per-grid path).
template <class T>
void coarse_step(amr_hierarchy* h, amr_state* Ua, amr_state* Ub, uint32_t& par, double* dt0, void* ws, int mode,
                 hipStream_t s) {
  const int L = h->nlev, R = h->R;
  auto cur = [&](int l) { return ((par >> l) & 1u) ? Ub : Ua; };
  do_dt<T>(h, Ua, Ub, par, dt0, s);
  // level 0 steps from band 2 (step_band): its same-level fill copies that much
  do_fill<T>(h, 0, AMR_FILL_SAME_LEVEL, cur(0), cur(0), s, true);
  if (mode == 0) {
    const int ncyc = ipow(R, L - 1);
    const std::vector<LaunchList>& lists = h->schedule == 1 ? h->eta_lists : h->cycle_lists;
    for (int c = 0; c < ncyc; ++c) {
      // band fills of the levels whose step window starts here
      for (int l = 1; l < L; ++l) {
        const int span = ipow(R, L - 1 - l);
        if (c % span) continue;
        const int k = c / span;
        // the refresh before substeps k >= 1 feeds a step from band 2
        if (k % R == 0) do_fill<T>(h, l, AMR_FILL_FULL, cur(l), cur(l - 1), s);
        else do_fill<T>(h, l, AMR_FILL_SAME_LEVEL, cur(l), cur(l - 1), s, step_band(h, l, k) == 2);
      }
      run_list<T>(h, lists[c], Ua, Ub, par, dt0, ws, s);
      // levels whose window ends here: every grid has stepped; registers,
      // then the level's buffers swap, then the synchronisations it closes
      uint32_t ending = 0;
      for (int l = 0; l < L; ++l) {
        const int span = ipow(R, L - 1 - l);
        if ((c + 1) % span) continue;
        ending |= 1u << l;
        write_registers<T>(h, l, c / span, dt0, ws, s);
      }
      par ^= ending;
      for (int f = L - 1; f >= 1; --f)
        if ((c + 1) % ipow(R, L - f) == 0) do_sync<T>(h, f, cur(f), cur(f - 1), ws, s);
    }
  } else {
    std::function<void(int, int)> cyc = [&](int l, int k) {
      if (l + 1 < L) do_fill<T>(h, l + 1, AMR_FILL_FULL, cur(l + 1), cur(l), s);
      const int band = step_band(h, l, k);
      for (int gi : h->level_grids[l]) run_list<T>(h, h->grid_lists.at({gi, band}), Ua, Ub, par, dt0, ws, s);
      write_registers<T>(h, l, k, dt0, ws, s);
      par ^= 1u << l;
      if (l + 1 < L) {
        for (int kk = 0; kk < R; ++kk) {
          if (kk > 0) do_fill<T>(h, l + 1, AMR_FILL_SAME_LEVEL, cur(l + 1), cur(l), s, step_band(h, l + 1, kk) == 2);
          cyc(l + 1, kk);
        }
        do_sync<T>(h, l + 1, cur(l + 1), cur(l), ws, s);
      }
    };
    cyc(0, 0);
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

namespace {
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
    h->adj.resize(h->nlev);
    return h;
  } catch (...) {
    delete h;
    throw;
  }
}
}  // namespace

amr_status amr_create(const amr_params* p, const amr_grid* grids, int32_t ngrids, amr_hierarchy** out) {
  if (out) *out = nullptr;
  amr_hierarchy* h = nullptr;
  try {
    if (!out) throw Error(AMR_EINVAL, "out is NULL");
    g_host_only = false;
    h = build_hierarchy(p, grids, ngrids);
    HIPCHK(hipMalloc((void**)&h->d_err, 256));
    HIPCHK(hipMemset(h->d_err, 0, 256));
    HIPCHK(hipMalloc((void**)&h->d_queue, sizeof(WorkQueue)));
    HIPCHK(hipMemset(h->d_queue, 0, sizeof(WorkQueue)));
    {
      int dev = 0, fb = 1, ub = 1;
      HIPCHK(hipGetDevice(&dev));
      hipDeviceProp_t prop;
      HIPCHK(hipGetDeviceProperties(&prop, dev));
      if (h->esize == 8)
        kernel_occupancy<double>(h->ndim, &fb, &ub);
      else
        kernel_occupancy<float>(h->ndim, &fb, &ub);
      h->flux_pblocks = prop.multiProcessorCount * fb;
      h->upd_pblocks = prop.multiProcessorCount * ub;
    }
    HIPCHK(hipDeviceSynchronize());
    *out = h;
    return AMR_OK;
  } catch (const std::exception& e) {
    delete h;
    return fail(e);
  }
}

amr_status amr_validate(const amr_params* p, const amr_grid* grids, int32_t ngrids, int64_t* stats) {
  amr_hierarchy* h = nullptr;
  try {
    g_host_only = true;
    h = build_hierarchy(p, grids, ngrids);
    g_host_only = false;
    if (stats) {
      int64_t ncopy = 0, npro = 0, nsync = 0;
      for (int l = 0; l < h->nlev; ++l) {
        ncopy += h->n_copy[l];
        npro += h->n_pcell[l] + h->n_pface[l];
      }
      for (int l = 1; l < h->nlev; ++l) {
        const SyncTables& t = h->sync[l];
        nsync += t.n_freg_c + t.n_freg_f + t.n_ereg_c + t.n_ereg_f + t.n_reflux + t.n_emffix + t.n_restrict;
      }
      stats[0] = (int64_t)h->grids.size();
      stats[1] = h->total_elems;
      stats[2] = h->workspace_bytes;
      stats[3] = ncopy;
      stats[4] = npro;
      stats[5] = nsync;
      stats[6] = (int64_t)h->h_fitems.size();
      stats[7] = (int64_t)h->h_uitems.size();
    }
    delete h;
    return AMR_OK;
  } catch (const std::exception& e) {
    g_host_only = false;
    delete h;
    return fail(e);
  }
}

amr_status amr_plan_schedule(const amr_params* p, const amr_grid* grids, int32_t ngrids, int32_t schedule,
                             double* cycle_work, int32_t* step_cycle) {
  try {
    if (schedule != 0 && schedule != 1) throw Error(AMR_EINVAL, "schedule must be 0 or 1");
    validate(p, grids, ngrids);
    amr_hierarchy h;
    h.p = *p;
    h.ndim = p->ndim;
    h.nlev = p->nlevels;
    h.R = p->ratio;
    h.g = p->ghost;
    h.grids.assign(grids, grids + ngrids);
    h.level_grids.assign(h.nlev, {});
    for (int i = 0; i < ngrids; ++i) h.level_grids[grids[i].level].push_back(i);
    std::vector<std::vector<int>> cyc;
    std::vector<double> load;
    plan_eta(&h, schedule, cyc, load);
    if (cycle_work) std::copy(load.begin(), load.end(), cycle_work);
    if (step_cycle) {
      size_t q = 0;
      for (int i = 0; i < ngrids; ++i)
        for (int c : cyc[i]) step_cycle[q++] = c;
    }
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_set_schedule(amr_hierarchy* h, int32_t schedule) {
  try {
    if (!h) throw Error(AMR_EINVAL, "null argument");
    if (schedule != 0 && schedule != 1) throw Error(AMR_EINVAL, "schedule must be 0 or 1");
    if (schedule != h->schedule) {
      for (auto& g : h->graph_exec)
        if (g) {
          (void)hipGraphExecDestroy(g);
          g = nullptr;
        }
      h->schedule = schedule;
    }
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_get_schedule(const amr_hierarchy* h, int32_t* schedule, double* cycle_work) {
  if (!h || !schedule) return AMR_EINVAL;
  *schedule = h->schedule;
  if (cycle_work) std::copy(h->cycle_work[h->schedule].begin(), h->cycle_work[h->schedule].end(), cycle_work);
  return AMR_OK;
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

amr_status amr_compute_dt(amr_hierarchy* h, const amr_state* U_a, const amr_state* U_b, uint32_t parity,
                          double* dt0, void* stream) {
  try {
    if (!h || !U_a || !U_b || !dt0) throw Error(AMR_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    if (h->esize == 8)
      do_dt<double>(h, U_a, U_b, parity, dt0, s);
    else
      do_dt<float>(h, U_a, U_b, parity, dt0, s);
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_fill_ghosts_prolong(amr_hierarchy* h, int32_t level, int32_t mode, amr_state* U_level,
                                   const amr_state* U_parent, void* stream) {
  try {
    if (!h || !U_level) throw Error(AMR_EINVAL, "null argument");
    if (level < 0 || level >= h->nlev) throw Error(AMR_EINVAL, "level out of range");
    if (mode != AMR_FILL_FULL && mode != AMR_FILL_SAME_LEVEL) throw Error(AMR_EINVAL, "bad fill mode");
    if (mode == AMR_FILL_FULL && level > 0 && !U_parent) throw Error(AMR_EINVAL, "FULL fill needs the parent state");
    hipStream_t s = (hipStream_t)stream;
    if (h->esize == 8)
      do_fill<double>(h, level, mode, U_level, U_parent, s);
    else
      do_fill<float>(h, level, mode, U_level, U_parent, s);
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_advance_patches(amr_hierarchy* h, int32_t cycle, const int32_t* grid_subset, int32_t nsubset,
                               int32_t band, const amr_state* U_a, const amr_state* U_b, uint32_t parity,
                               const double* dt0, void* workspace, void* stream) {
  try {
    if (!h || !U_a || !U_b || !dt0 || !workspace) throw Error(AMR_EINVAL, "null argument");
    hipStream_t s = (hipStream_t)stream;
    const bool f64 = h->esize == 8;
    auto run = [&](const LaunchList& L) {
      if (f64)
        run_list<double>(h, L, U_a, U_b, parity, dt0, workspace, s);
      else
        run_list<float>(h, L, U_a, U_b, parity, dt0, workspace, s);
    };
    auto regs = [&](int l, int k) {
      if (f64)
        write_registers<double>(h, l, k, dt0, workspace, s);
      else
        write_registers<float>(h, l, k, dt0, workspace, s);
    };
    if (cycle >= 0) {
      if (band > 0) {
        if (h->nlev != 1) throw Error(AMR_EINVAL, "an explicit band with a batched cycle needs a single level");
        auto it = h->level0_band_lists.find(band);
        if (it == h->level0_band_lists.end()) throw Error(AMR_EINVAL, "band must be in [2, ghost]");
        run(it->second);
      } else {
        if (cycle >= (int)h->cycle_lists.size()) throw Error(AMR_EINVAL, "cycle out of range");
        run(h->cycle_lists[cycle]);
        const int L = h->nlev;
        for (int l = 0; l < L; ++l) {
          const int span = ipow(h->R, L - 1 - l);
          if (cycle % span == 0) regs(l, cycle / span);
        }
      }
    } else {
      if (!grid_subset || nsubset <= 0) throw Error(AMR_EINVAL, "per-grid path needs a grid list");
      std::vector<int> levels;
      for (int i = 0; i < nsubset; ++i) {
        auto it = h->grid_lists.find({grid_subset[i], band});
        if (it == h->grid_lists.end()) throw Error(AMR_EINVAL, "bad grid id or band for the per-grid path");
        run(it->second);
        const int l = h->desc[grid_subset[i]].level;
        if (std::find(levels.begin(), levels.end(), l) == levels.end()) levels.push_back(l);
      }
      for (int l : levels) regs(l, l == 0 ? 0 : (h->g - band) / 2);
    }
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_restrict_fluxfix(amr_hierarchy* h, int32_t fine_level, const amr_state* U_fine, amr_state* U_coarse,
                                void* workspace, void* stream) {
  try {
    if (!h || !U_fine || !U_coarse || !workspace) throw Error(AMR_EINVAL, "null argument");
    if (fine_level < 1 || fine_level >= h->nlev) throw Error(AMR_EINVAL, "fine_level must be in [1, nlevels)");
    hipStream_t s = (hipStream_t)stream;
    if (h->esize == 8)
      do_sync<double>(h, fine_level, U_fine, U_coarse, workspace, s);
    else
      do_sync<float>(h, fine_level, U_fine, U_coarse, workspace, s);
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_coarse_step(amr_hierarchy* h, amr_state* U_a, amr_state* U_b, uint32_t* parity, double* dt0,
                           void* workspace, int32_t mode, void* stream) {
  try {
    if (!h || !U_a || !U_b || !parity || !dt0 || !workspace) throw Error(AMR_EINVAL, "null argument");
    if (mode != 0 && mode != 1) throw Error(AMR_EINVAL, "mode must be 0 (batched) or 1 (per-grid)");
    hipStream_t s = (hipStream_t)stream;
    uint32_t par = *parity;
    if (h->esize == 8)
      coarse_step<double>(h, U_a, U_b, par, dt0, workspace, mode, s);
    else
      coarse_step<float>(h, U_a, U_b, par, dt0, workspace, mode, s);
    *parity = par;
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_graph_capture(amr_hierarchy* h, amr_state* U_a, amr_state* U_b, uint32_t parity, double* dt0,
                             void* workspace, int32_t mode, void* stream) {
  try {
    if (!h || !U_a || !U_b || !dt0 || !workspace) throw Error(AMR_EINVAL, "null argument");
    if (!stream) throw Error(AMR_EINVAL, "graph capture needs a non-default stream");
    if (mode != 0 && mode != 1) throw Error(AMR_EINVAL, "mode must be 0 (batched) or 1 (per-grid)");
    hipStream_t s = (hipStream_t)stream;
    for (auto& g : h->graph_exec)
      if (g) {
        HIPCHK(hipGraphExecDestroy(g));
        g = nullptr;
      }
    uint32_t par = parity;
    for (int k = 0; k < 2; ++k) {
      const uint32_t start = par;
      h->capturing = true;
      HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
      try {
        if (h->esize == 8)
          coarse_step<double>(h, U_a, U_b, par, dt0, workspace, mode, s);
        else
          coarse_step<float>(h, U_a, U_b, par, dt0, workspace, mode, s);
      } catch (...) {
        hipGraph_t gdrop;
        (void)hipStreamEndCapture(s, &gdrop);
        if (gdrop) (void)hipGraphDestroy(gdrop);
        h->capturing = false;
        throw;
      }
      hipGraph_t graph = nullptr;
      HIPCHK(hipStreamEndCapture(s, &graph));
      h->capturing = false;
      hipGraphExec_t ex = nullptr;
      hipError_t ie = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      HIPCHK(ie);
      const int slot = start & 1u;
      h->graph_exec[slot] = ex;
      h->graph_parity[slot] = start;
      if (par == start) break;  // every level returns to its buffer: one graph suffices
    }
    return AMR_OK;
  } catch (const std::exception& e) {
    h->capturing = false;
    return fail(e);
  }
}

amr_status amr_graph_launch(amr_hierarchy* h, uint32_t* parity, void* stream) {
  try {
    if (!h || !parity) throw Error(AMR_EINVAL, "null argument");
    const int slot = *parity & 1u;
    if (!h->graph_exec[slot] || h->graph_parity[slot] != *parity)
      throw Error(AMR_EINVAL, "no captured coarse step starts from this parity");
    HIPCHK(hipGraphLaunch(h->graph_exec[slot], (hipStream_t)stream));
    // level 0 steps once per coarse step; level l > 0 steps R^l (even) times
    *parity ^= (h->R % 2 == 0) ? 1u : ((1u << h->nlev) - 1u);
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

}  // extern "C"

namespace {

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
  if (mode < 0 || mode > 7) throw Error(AMR_EINVAL, "launch mode must be in [0, 7]");
  h->persistent = (mode & 1) != 0;
  h->persistent_flux = (mode & 5) != 0;
  h->xcd_chunks = (mode & 2) != 0;
  if (policy != h->tile_policy || zchunk != h->zchunk) {
    h->tile_policy = policy;
    h->zchunk = zchunk;
    rebuild_lists(h);
  }
}

// Milliseconds of `reps` passes over every launch cycle's batched advance,
// reading the current buffers and writing the other ones.
template <class T>
double time_cycles(amr_hierarchy* h, const amr_state* Ua, const amr_state* Ub, uint32_t parity, const double* dt0,
                   void* ws, int reps, hipStream_t s) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const bool timing = h->timing;
  h->timing = false;
  for (const LaunchList& L : h->cycle_lists) run_list<T>(h, L, Ua, Ub, parity, dt0, ws, s);  // warm-up
  HIPCHK(hipEventRecord(e0, s));
  for (int r = 0; r < reps; ++r)
    for (const LaunchList& L : h->cycle_lists) run_list<T>(h, L, Ua, Ub, parity, dt0, ws, s);
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipEventSynchronize(e1));
  h->timing = timing;
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return (double)ms;
}

template <class T>
int autotune(amr_hierarchy* h, amr_state* Ua, amr_state* Ub, uint32_t parity, double* dt0, void* ws, int reps,
             amr_tune_entry* out, hipStream_t s) {
  // valid bands on every level and a current dt0 (the next coarse step
  // refills the bands and recomputes dt0 itself)
  for (int l = 0; l < h->nlev; ++l) {
    amr_state* cur = ((parity >> l) & 1u) ? Ub : Ua;
    amr_state* par = l > 0 ? (((parity >> (l - 1)) & 1u) ? Ub : Ua) : nullptr;
    do_fill<T>(h, l, l > 0 ? AMR_FILL_FULL : AMR_FILL_SAME_LEVEL, cur, par, s);
  }
  do_dt<T>(h, Ua, Ub, parity, dt0, s);
  const int zc[4] = {8, 12, 16, 32};
  const int modes[6] = {0, 1, 2, 3, 4, 6};
  int best = -1, n = 0, bpol = 1, bzc = 8, bmode = 0;
  double best_ms = 0.0;
  for (int pol = 0; pol < 2; ++pol)
    for (int zi = 0; zi < 4; ++zi)
      for (int mi = 0; mi < 6; ++mi, ++n) {
        set_launch_config(h, pol, zc[zi], modes[mi]);
        const double ms = time_cycles<T>(h, Ua, Ub, parity, dt0, ws, reps, s);
        if (out) out[n] = amr_tune_entry{pol, zc[zi], modes[mi], h->upd_zchunk, ms};
        if (best < 0 || ms < best_ms) {
          best = n;
          best_ms = ms;
          bpol = pol;
          bzc = zc[zi];
          bmode = modes[mi];
        }
      }
  set_launch_config(h, bpol, bzc, bmode);
  // then the update's planes per item, under the kept configuration
  const int uzc[4] = {1, 2, 4, 8};
  int ubest = h->upd_zchunk;
  for (int ui = 0; ui < 4; ++ui, ++n) {
    set_update_zchunk(h, uzc[ui]);
    const double ms = time_cycles<T>(h, Ua, Ub, parity, dt0, ws, reps, s);
    if (out) out[n] = amr_tune_entry{bpol, bzc, bmode, uzc[ui], ms};
    if (ms < best_ms) {
      best = n;
      best_ms = ms;
      ubest = uzc[ui];
    }
  }
  set_update_zchunk(h, ubest);
  return best;
}

int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

// Level of an adjoint selection: a whole level (v < 0: level -(v+1)) or a
// grid that is the only one on its level.
int adjoint_level(const amr_hierarchy* h, int32_t grid_or_level) {
  if (grid_or_level >= 0) {
    if (grid_or_level >= (int)h->desc.size()) throw Error(AMR_EINVAL, "grid index out of range");
    const int l = h->desc[grid_or_level].level;
    if (h->level_grids[l].size() != 1)
      throw Error(AMR_EUNSUPPORTED, "the adjoint of one grid needs it to be alone on its level; pass its level");
    return l;
  }
  const int l = -(grid_or_level + 1);
  if (l < 0 || l >= h->nlev) throw Error(AMR_EINVAL, "level out of range");
  return l;
}

struct AdjLayout {
  int64_t stride, region0, off_states, state_bytes, off_lam, off_dts, total;
};

AdjLayout adjoint_layout(const amr_hierarchy* h, int level, int nsteps) {
  const amr_hierarchy::AdjTables& t = h->adj[level];
  AdjLayout a;
  int64_t e0 = INT64_MAX, e1 = 0;
  if (t.built) {
    e0 = t.e0;
    e1 = t.e1;
  } else {
    for (int gi : h->level_grids[level]) {
      const GridDesc& G = h->desc[gi];
      e0 = std::min<int64_t>(e0, G.off);
      e1 = std::max<int64_t>(e1, G.off + (int64_t)G.P[0] * G.P[1] * G.P[2]);
    }
  }
  const int64_t es = (int64_t)h->esize;
  a.stride = (e1 - e0 + 63) / 64 * 64;
  a.region0 = align256(std::max<int64_t>(h->flux_bytes, (int64_t)kAdjArrays * a.stride * es));
  a.state_bytes = 8 * h->total_elems * es;
  a.off_states = a.region0;
  a.off_lam = a.off_states + align256((int64_t)nsteps * a.state_bytes);
  a.off_dts = a.off_lam + align256(a.state_bytes);
  a.total = a.off_dts + align256(8 * (int64_t)nsteps);
  return a;
}

void build_adjoint_tables(amr_hierarchy* h, int level) {
  amr_hierarchy::AdjTables& t = h->adj[level];
  if (t.built) return;
  std::vector<int2> items;
  t.e0 = INT64_MAX;
  t.e1 = 0;
  for (int gi : h->level_grids[level]) {
    const GridDesc& G = h->desc[gi];
    const int box = G.P[0] * G.P[1] * G.P[2];
    for (int s = 0; s < box; s += 256) items.push_back(make_int2(gi, s));
    t.e0 = std::min<int64_t>(t.e0, G.off);
    t.e1 = std::max<int64_t>(t.e1, G.off + box);
  }
  // transpose of the same-level band copy: group (class, source) -> dsts
  const std::vector<CopyEntry>& cp = h->h_copy[level];
  const int4 cb = h->copy_cls[level];
  const int bounds[4] = {cb.x, cb.y, cb.z, cb.w};
  std::vector<std::pair<int64_t, int32_t>> keyed;  // (class * 2^32 + src, dst)
  keyed.reserve(cp.size());
  for (int i = 0; i < (int)cp.size(); ++i) {
    int cls = 0;
    while (cls < 3 && i >= bounds[cls]) ++cls;
    const CopyEntry& c = cp[i];
    if (c.src < t.e0 || c.src >= t.e1 || c.dst < t.e0 || c.dst >= t.e1)
      throw Error(AMR_EINVAL, "internal: band copy leaves the level's element range");
    keyed.push_back({((int64_t)cls << 32) | (int64_t)(uint32_t)c.src, c.dst});
  }
  std::sort(keyed.begin(), keyed.end());
  std::vector<InvCopy> inv;
  std::vector<int32_t> dsts;
  for (size_t i = 0; i < keyed.size();) {
    size_t j = i;
    InvCopy e{};
    e.src = (int32_t)(keyed[i].first & 0xffffffffLL);
    e.cls = (int32_t)(keyed[i].first >> 32);
    e.begin = (int32_t)dsts.size();
    while (j < keyed.size() && keyed[j].first == keyed[i].first) dsts.push_back(keyed[j++].second);
    e.end = (int32_t)dsts.size();
    inv.push_back(e);
    i = j;
  }
  t.nitems = (int)items.size();
  t.ninv = (int)inv.size();
  t.d_items = dev_upload(items);
  t.d_inv = dev_upload(inv);
  t.d_dsts = dev_upload(dsts);
  t.built = true;
}

template <class T>
void adjoint_run(amr_hierarchy* h, int level, int nsteps, const double* dts, const amr_state* Uc, amr_state* lam,
                 void* ws, hipStream_t s) {
  build_adjoint_tables(h, level);
  const amr_hierarchy::AdjTables& t = h->adj[level];
  const AdjLayout a = adjoint_layout(h, level, nsteps);
  char* base = (char*)ws;
  const int64_t arr = h->total_elems * (int64_t)sizeof(T);
  auto state_at = [&](int k) {
    amr_state st;
    for (int q = 0; q < 8; ++q) st.f[q] = base + a.off_states + (int64_t)k * a.state_bytes + q * arr;
    return st;
  };
  double* d_dts = (double*)(base + a.off_dts);
  launch_put_values(d_dts, dts, nsteps, s);
  HIPCHK(hipGetLastError());
  // forward recompute of the segment's step inputs; band elements that the
  // same-level copy does not fill keep the checkpoint's values
  for (int k = 0; k < nsteps; ++k) {
    amr_state sk = state_at(k);
    for (int q = 0; q < 8; ++q) HIPCHK(hipMemcpyAsync(sk.f[q], Uc->f[q], arr, hipMemcpyDeviceToDevice, s));
  }
  const bool timing = h->timing;
  h->timing = false;
  for (int k = 0; k < nsteps; ++k) {
    amr_state sk = state_at(k);
    launch_copy<T>(h->ndim, h->d_copy[level], h->n_copy[level], h->copy_cls[level], dstate<T>(&sk), s);
    HIPCHK(hipGetLastError());
    if (k + 1 < nsteps) {
      amr_state sn = state_at(k + 1);
      run_list<T>(h, h->band2_lists[level], &sk, &sn, 0u, d_dts + k, ws, s);
    }
  }
  h->timing = timing;
  // reverse sweep
  AdjBuffers buf;
  const int64_t ab = a.stride * (int64_t)sizeof(T);
  buf.ps = base;
  buf.af = base + 42 * ab;
  buf.ac = base + (42 + 45) * ab;
  buf.au = base + (42 + 45 + 38) * ab;
  buf.tmp = base + (42 + 45 + 38 + 9) * ab;
  buf.stride = a.stride;
  buf.e0 = t.e0;
  amr_state other;
  for (int q = 0; q < 8; ++q) other.f[q] = base + a.off_lam + q * arr;
  // ping-pong so that the last reverse step writes lam itself (its kernels
  // write only the level's grid boxes, so other levels' entries stay): with
  // an odd step count the seed is first copied into the workspace buffer
  const amr_state* Lp = lam;
  const amr_state* Lo = &other;
  if (nsteps % 2 == 1) {
    const int64_t es = (int64_t)sizeof(T);
    for (int q = 0; q < 8; ++q)
      HIPCHK(hipMemcpyAsync((char*)other.f[q] + t.e0 * es, (const char*)lam->f[q] + t.e0 * es, (t.e1 - t.e0) * es,
                            hipMemcpyDeviceToDevice, s));
    Lp = &other;
    Lo = lam;
  }
  const Phys ph = phys(h);
  for (int k = nsteps - 1; k >= 0; --k) {
    amr_state sk = state_at(k);
    launch_adjoint_step<T>(h->ndim, h->d_desc, t.d_items, t.nitems, t.d_inv, t.ninv, t.d_dsts, dstate<T>(&sk),
                           dstate<T>(Lp), dstate<T>(Lo), buf, dts[k], ph, s);
    HIPCHK(hipGetLastError());
    std::swap(Lp, Lo);
  }
}

// Frozen-branch advance: pairs (base, perturbed) in workspace, the same
// fill + band-2 step sequence as the adjoint's forward map.
int64_t frozen_workspace(const amr_hierarchy* h) {
  const int64_t es2 = 2 * (int64_t)h->esize;
  return align256(21 * h->total_elems * es2) + 2 * align256(8 * h->total_elems * es2) + 256;
}

template <class S>
void frozen_run(amr_hierarchy* h, int level, int nsteps, const double* dts, const amr_state* Ub, amr_state* Up,
                void* ws, hipStream_t s) {
  using P = Frozen<S>;
  char* base = (char*)ws;
  const int64_t arr = h->total_elems * (int64_t)sizeof(P);
  const int64_t off_s0 = align256(21 * arr);
  const int64_t off_s1 = off_s0 + align256(8 * arr);
  double* d_dt = (double*)(off_s1 + align256(8 * arr) + base);
  amr_state st[2];
  for (int q = 0; q < 8; ++q) {
    st[0].f[q] = base + off_s0 + q * arr;
    st[1].f[q] = base + off_s1 + q * arr;
  }
  launch_pack<S>(dstate<S>(Ub), dstate<S>(Up), dstate<P>(&st[0]), h->total_elems, s);
  launch_pack<S>(dstate<S>(Ub), dstate<S>(Up), dstate<P>(&st[1]), h->total_elems, s);
  HIPCHK(hipGetLastError());
  const bool timing = h->timing;
  h->timing = false;
  int cur = 0;
  for (int k = 0; k < nsteps; ++k) {
    launch_put_values(d_dt, dts + k, 1, s);
    launch_copy<P>(h->ndim, h->d_copy[level], h->n_copy[level], h->copy_cls[level], dstate<P>(&st[cur]), s);
    HIPCHK(hipGetLastError());
    run_list<P>(h, h->band2_lists[level], &st[cur], &st[1 - cur], 0u, d_dt, ws, s);
    cur = 1 - cur;
  }
  h->timing = timing;
  int64_t e0 = INT64_MAX, e1 = 0;
  for (int gi : h->level_grids[level]) {
    const GridDesc& G = h->desc[gi];
    e0 = std::min<int64_t>(e0, G.off);
    e1 = std::max<int64_t>(e1, G.off + (int64_t)G.P[0] * G.P[1] * G.P[2]);
  }
  launch_unpack<S>(dstate<P>(&st[cur]), dstate<S>(Up), e0, e1, s);
  HIPCHK(hipGetLastError());
}

}  // namespace

extern "C" {

amr_status amr_frozen_workspace(const amr_hierarchy* h, int64_t* bytes) {
  if (!h || !bytes) return AMR_EINVAL;
  if (h->upwind_emf) {
    g_last_error = "the frozen-branch forward supports the arithmetic-mean EMF only";
    return AMR_EUNSUPPORTED;
  }
  *bytes = frozen_workspace(h);
  return AMR_OK;
}

amr_status amr_advance_frozen(amr_hierarchy* h, int32_t level, int32_t nsteps, const double* dts,
                              const amr_state* U_base, amr_state* U_pert, void* workspace, void* stream) {
  try {
    if (!h || !dts || !U_base || !U_pert || !workspace) throw Error(AMR_EINVAL, "null argument");
    if (h->upwind_emf) throw Error(AMR_EUNSUPPORTED, "the frozen-branch forward supports the arithmetic-mean EMF only");
    if (level < 0 || level >= h->nlev) throw Error(AMR_EINVAL, "level out of range");
    if (nsteps < 1) throw Error(AMR_EINVAL, "nsteps must be >= 1");
    for (int k = 0; k < nsteps; ++k)
      if (!(dts[k] > 0.0)) throw Error(AMR_EINVAL, "step sizes must be > 0");
    hipStream_t s = (hipStream_t)stream;
    if (h->esize == 8)
      frozen_run<double>(h, level, nsteps, dts, U_base, U_pert, workspace, s);
    else
      frozen_run<float>(h, level, nsteps, dts, U_base, U_pert, workspace, s);
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_adjoint_workspace(const amr_hierarchy* h, int32_t grid_or_level, int32_t nsteps, int64_t* bytes) {
  try {
    if (!h || !bytes) throw Error(AMR_EINVAL, "null argument");
    if (h->upwind_emf) throw Error(AMR_EUNSUPPORTED, "the adjoint supports the arithmetic-mean EMF only");
    if (nsteps < 1) throw Error(AMR_EINVAL, "nsteps must be >= 1");
    const int level = adjoint_level(h, grid_or_level);
    *bytes = adjoint_layout(h, level, nsteps).total;
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_advance_adjoint(amr_hierarchy* h, int32_t grid_or_level, int32_t nsteps, const double* dts,
                               const amr_state* U_checkpoint, amr_state* lambda_inout, void* workspace,
                               void* stream) {
  try {
    if (!h || !dts || !U_checkpoint || !lambda_inout || !workspace) throw Error(AMR_EINVAL, "null argument");
    if (h->upwind_emf) throw Error(AMR_EUNSUPPORTED, "the adjoint supports the arithmetic-mean EMF only");
    if (nsteps < 1) throw Error(AMR_EINVAL, "nsteps must be >= 1");
    for (int k = 0; k < nsteps; ++k)
      if (!(dts[k] > 0.0)) throw Error(AMR_EINVAL, "step sizes must be > 0");
    const int level = adjoint_level(h, grid_or_level);
    hipStream_t s = (hipStream_t)stream;
    if (h->esize == 8)
      adjoint_run<double>(h, level, nsteps, dts, U_checkpoint, lambda_inout, workspace, s);
    else
      adjoint_run<float>(h, level, nsteps, dts, U_checkpoint, lambda_inout, workspace, s);
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_store_interior_adjoint(amr_hierarchy* h, int32_t grid, const double* const* g, amr_state* lambda,
                                      void* stream) {
  try {
    if (!h || !g || !lambda) throw Error(AMR_EINVAL, "null argument");
    if (grid < 0 || grid >= (int)h->desc.size()) throw Error(AMR_EINVAL, "grid index out of range");
    Ptr8 gp;
    for (int q = 0; q < 8; ++q) gp.p[q] = g[q];
    hipStream_t s = (hipStream_t)stream;
    if (h->esize == 8)
      launch_store_adj<double>(h->ndim, h->desc[grid], gp, dstate<double>(lambda), s);
    else
      launch_store_adj<float>(h->ndim, h->desc[grid], gp, dstate<float>(lambda), s);
    HIPCHK(hipGetLastError());
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_load_primitive_adjoint(amr_hierarchy* h, int32_t grid, const double* const* prim,
                                      const amr_state* lambda, double* const* grad, void* stream) {
  try {
    if (!h || !prim || !lambda || !grad) throw Error(AMR_EINVAL, "null argument");
    if (grid < 0 || grid >= (int)h->desc.size()) throw Error(AMR_EINVAL, "grid index out of range");
    Ptr8 pp{};
    MutPtr8 gp{};
    for (int q = 0; q < 4; ++q) {
      pp.p[q] = prim[q];
      gp.p[q] = grad[q];
    }
    hipStream_t s = (hipStream_t)stream;
    if (h->esize == 8)
      launch_load_prim_adj<double>(h->ndim, h->desc[grid], pp, dstate<double>(lambda), gp, s);
    else
      launch_load_prim_adj<float>(h->ndim, h->desc[grid], pp, dstate<float>(lambda), gp, s);
    HIPCHK(hipGetLastError());
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
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

amr_status amr_set_launch_config(amr_hierarchy* h, int32_t tile_policy, int32_t zchunk, int32_t launch_mode) {
  try {
    if (!h) throw Error(AMR_EINVAL, "null argument");
    set_launch_config(h, tile_policy, zchunk, launch_mode);
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_set_update_zchunk(amr_hierarchy* h, int32_t zchunk) {
  try {
    if (!h) throw Error(AMR_EINVAL, "null argument");
    set_update_zchunk(h, zchunk);
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_get_update_zchunk(const amr_hierarchy* h, int32_t* zchunk) {
  if (!h || !zchunk) return AMR_EINVAL;
  *zchunk = h->upd_zchunk;
  return AMR_OK;
}

amr_status amr_get_launch_config(const amr_hierarchy* h, int32_t* tile_policy, int32_t* zchunk, int32_t* launch_mode) {
  if (!h) return AMR_EINVAL;
  if (tile_policy) *tile_policy = h->tile_policy;
  if (zchunk) *zchunk = h->zchunk;
  if (launch_mode)
    *launch_mode = (h->persistent ? 1 : 0) | (h->xcd_chunks ? 2 : 0) | (h->persistent_flux && !h->persistent ? 4 : 0);
  return AMR_OK;
}

amr_status amr_autotune(amr_hierarchy* h, amr_state* U_a, amr_state* U_b, uint32_t parity, double* dt0,
                        void* workspace, int32_t reps, amr_tune_entry* results, int32_t* chosen, void* stream) {
  try {
    if (!h || !U_a || !U_b || !dt0 || !workspace) throw Error(AMR_EINVAL, "null argument");
    if (reps < 1) throw Error(AMR_EINVAL, "reps must be >= 1");
    hipStream_t s = (hipStream_t)stream;
    const int b = h->esize == 8 ? autotune<double>(h, U_a, U_b, parity, dt0, workspace, reps, results, s)
                                : autotune<float>(h, U_a, U_b, parity, dt0, workspace, reps, results, s);
    if (chosen) *chosen = b;
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

}  // extern "C"

// ============================================================ regridding
namespace {

// Interior cells of the grids of `level`, grids in increasing index: the
// flag layout (each grid x fastest, then y, then z).
int64_t level_cells(const amr_hierarchy* h, int level) {
  int64_t n = 0;
  for (int gi : h->level_grids[level]) {
    const amr_grid& G = h->grids[gi];
    int64_t c = 1;
    for (int a = 0; a < h->ndim; ++a) c *= G.hi[a] - G.lo[a];
    n += c;
  }
  return n;
}

void ensure_flag_items(amr_hierarchy* h, int level) {
  if ((int)h->d_flag_items.size() < h->nlev) {
    h->d_flag_items.resize(h->nlev, nullptr);
    h->n_flag_items.resize(h->nlev, 0);
  }
  if (h->d_flag_items[level]) return;
  std::vector<FlagItem> items;
  int64_t out = 0;
  for (int gi : h->level_grids[level]) {
    const amr_grid& G = h->grids[gi];
    int64_t c = 1;
    for (int a = 0; a < h->ndim; ++a) c *= G.hi[a] - G.lo[a];
    if (c > INT32_MAX) throw Error(AMR_EUNSUPPORTED, "grid too large to flag");
    for (int64_t f = 0; f < c; f += 256) items.push_back(FlagItem{gi, (int32_t)f, (int32_t)std::min<int64_t>(c, f + 256), 0, out});
    out += c;
  }
  if (items.size() > (size_t)INT32_MAX) throw Error(AMR_EUNSUPPORTED, "too many flag items");
  h->n_flag_items[level] = (int)items.size();
  h->d_flag_items[level] = dev_upload(items);
}

template <class T>
void do_flags(amr_hierarchy* h, int level, amr_state* Ul, amr_state* Up, double theta, uint8_t* flags, hipStream_t s) {
  // the band of the level from the current data: at level > 0 the parent's
  // same-level band parts first (prolongation stencils reach into them)
  if (level > 0) {
    do_fill<T>(h, level - 1, AMR_FILL_SAME_LEVEL, Up, Up, s);
    do_fill<T>(h, level, AMR_FILL_FULL, Ul, Up, s);
  } else {
    do_fill<T>(h, 0, AMR_FILL_SAME_LEVEL, Ul, Ul, s);
  }
  ensure_flag_items(h, level);
  launch_flag<T>(h->ndim, h->d_desc, h->d_flag_items[level], h->n_flag_items[level], dstate<T>(Ul), theta, flags, s);
  HIPCHK(hipGetLastError());
}

// Nestable cells of one level: c is nestable when the cube c + [-buf, buf]^d
// lies in the union of the level's interiors (periodic images on periodic
// axes).  Held as a byte map over a region: the bounding box of the level's
// grids grown by `margin`, or the whole axis on a periodic axis the grown
// box reaches across.
struct NestMap {
  int nd = 3;
  int N[3] = {1, 1, 1};
  int lo[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
  bool full[3] = {false, false, false};  // region spans the whole periodic axis
  bool periodic[3] = {false, false, false};
  std::vector<uint8_t> cov, nest;

  int64_t at(const int (&x)[3]) const {
    return ((int64_t)(x[2] - lo[2]) * ext[1] + (x[1] - lo[1])) * ext[0] + (x[0] - lo[0]);
  }
  // Cell (already wrapped on periodic axes) inside the map region?
  bool inside(int (&x)[3]) const {
    for (int a = 0; a < 3; ++a) {
      if (x[a] < lo[a] || x[a] >= lo[a] + ext[a]) return false;
    }
    return true;
  }
  bool wrap(int (&x)[3]) const {
    for (int a = 0; a < nd; ++a) {
      if (periodic[a]) x[a] = posmod(x[a], N[a]);
      else if (x[a] < 0 || x[a] >= N[a]) return false;
    }
    return true;
  }
  bool nestable(int (&x)[3]) const {
    if (!wrap(x) || !inside(x)) return false;
    return nest[at(x)] != 0;
  }

  void build(const amr_hierarchy* h, int level, int buf, int margin) {
    nd = h->ndim;
    for (int a = 0; a < 3; ++a) {
      N[a] = a < nd ? h->p.domain[a] * ipow(h->R, level) : 1;
      periodic[a] = a < nd && h->p.bc[a] == AMR_BC_PERIODIC;
    }
    int blo[3] = {INT32_MAX, INT32_MAX, INT32_MAX}, bhi[3] = {INT32_MIN, INT32_MIN, INT32_MIN};
    for (int gi : h->level_grids[level])
      for (int a = 0; a < 3; ++a) {
        blo[a] = std::min(blo[a], h->grids[gi].lo[a]);
        bhi[a] = std::max(bhi[a], h->grids[gi].hi[a]);
      }
    int64_t cells = 1;
    for (int a = 0; a < 3; ++a) {
      if (a >= nd) {
        lo[a] = 0;
        ext[a] = 1;
        full[a] = false;
      } else {
        int l0 = blo[a] - margin, l1 = bhi[a] + margin;
        if (periodic[a] && (l0 < 0 || l1 > N[a])) {
          lo[a] = 0;
          ext[a] = N[a];
          full[a] = true;
        } else {
          lo[a] = std::max(l0, 0);
          ext[a] = std::min(l1, N[a]) - lo[a];
          full[a] = false;
        }
      }
      cells *= ext[a];
    }
    if (cells > ((int64_t)1 << 28)) throw Error(AMR_EUNSUPPORTED, "level region too large to regrid");
    cov.assign(cells, 0);
    for (int gi : h->level_grids[level]) {
      const amr_grid& G = h->grids[gi];
      for (int k = G.lo[2]; k < G.hi[2]; ++k)
        for (int j = G.lo[1]; j < G.hi[1]; ++j)
          for (int i = G.lo[0]; i < G.hi[0]; ++i) {
            int x[3] = {i, j, k};
            if (inside(x)) cov[at(x)] = 1;
          }
    }
    // erode by the cube, one axis at a time (a window count of uncovered
    // cells along each line; outside the region counts as uncovered unless
    // the region spans the periodic axis)
    nest = cov;
    std::vector<uint8_t> tmp;
    std::vector<int> pre;
    for (int a = 0; a < nd; ++a) {
      tmp = nest;
      const int n = ext[a];
      const int64_t stride = a == 0 ? 1 : (a == 1 ? (int64_t)ext[0] : (int64_t)ext[0] * ext[1]);
      int o1 = (a + 1) % 3, o2 = (a + 2) % 3;
      pre.assign(n + 2 * buf + 1, 0);
      for (int v = 0; v < ext[o2]; ++v)
        for (int u = 0; u < ext[o1]; ++u) {
          int x[3];
          x[a] = lo[a];
          x[o1] = lo[o1] + u;
          x[o2] = lo[o2] + v;
          const int64_t base = at(x);
          // prefix counts of uncovered cells over the line extended by buf
          // on both sides (wrapped on a full periodic axis, else uncovered)
          for (int j = 0; j < n + 2 * buf; ++j) {
            int q = j - buf;
            int unc;
            if (full[a]) unc = tmp[base + (int64_t)posmod(q, n) * stride] ? 0 : 1;
            else unc = (q < 0 || q >= n) ? 1 : (tmp[base + (int64_t)q * stride] ? 0 : 1);
            pre[j + 1] = pre[j] + unc;
          }
          for (int i = 0; i < n; ++i) nest[base + (int64_t)i * stride] = (pre[i + 2 * buf + 1] - pre[i]) == 0 ? 1 : 0;
        }
    }
  }
  // every cell of box B (level cells inside [0, N)) nestable
  bool box(const IBox& B) const {
    for (int k = B.lo[2]; k < B.hi[2]; ++k)
      for (int j = B.lo[1]; j < B.hi[1]; ++j)
        for (int i = B.lo[0]; i < B.hi[0]; ++i) {
          int x[3] = {i, j, k};
          if (!nestable(x)) return false;
        }
    return true;
  }
};

template <class T>
std::vector<amr_grid> do_regrid(amr_hierarchy* h, int level, amr_state* Ul, amr_state* Up,
                                const amr_regrid_params* rp, hipStream_t s) {
  const int nd = h->ndim, R = h->R;
  const int64_t ncell = level_cells(h, level);
  std::vector<uint8_t> fl(ncell);
  if (ncell > 0) {
    uint8_t* d_fl = nullptr;
    HIPCHK(hipMalloc((void**)&d_fl, ncell));
    try {
      do_flags<T>(h, level, Ul, Up, rp->theta, d_fl, s);
      HIPCHK(hipStreamSynchronize(s));
      HIPCHK(hipMemcpy(fl.data(), d_fl, ncell, hipMemcpyDeviceToHost));
    } catch (...) {
      (void)hipFree(d_fl);
      throw;
    }
    HIPCHK(hipFree(d_fl));
  }
  const int buf = h->g / R + 1;
  NestMap nm;
  nm.build(h, level, buf, buf + rp->buffer + 1);
  std::vector<uint8_t> mark(nm.cov.size(), 0);  // cells to cover, over the map region
  int64_t f = 0;
  for (int gi : h->level_grids[level]) {
    const amr_grid& G = h->grids[gi];
    int n[3] = {1, 1, 1};
    for (int a = 0; a < nd; ++a) n[a] = G.hi[a] - G.lo[a];
    for (int k = 0; k < n[2]; ++k)
      for (int j = 0; j < n[1]; ++j)
        for (int i = 0; i < n[0]; ++i, ++f) {
          if (!fl[f]) continue;
          const int b = rp->buffer;
          const int bz = nd == 3 ? b : 0;
          for (int dz = -bz; dz <= bz; ++dz)
            for (int dy = -b; dy <= b; ++dy)
              for (int dx = -b; dx <= b; ++dx) {
                int x[3] = {G.lo[0] + i + dx, G.lo[1] + j + dy, G.lo[2] + k + dz};
                if (!nm.nestable(x)) continue;  // also wraps x
                mark[nm.at(x)] = 1;
              }
        }
  }
  // the grids of level + 2 stay: the new level + 1 must hold each of them
  // grown by buf level-(l+1) cells
  if (level + 2 < h->nlev)
    for (int gi : h->level_grids[level + 2]) {
      const amr_grid& G = h->grids[gi];
      int c0[3] = {0, 0, 0}, c1[3] = {1, 1, 1};
      for (int a = 0; a < nd; ++a) {
        c0[a] = floordiv(floordiv(G.lo[a], R) - buf, R);
        c1[a] = -floordiv(-(floordiv(G.hi[a], R) + buf), R);
      }
      for (int k = c0[2]; k < c1[2]; ++k)
        for (int j = c0[1]; j < c1[1]; ++j)
          for (int i = c0[0]; i < c1[0]; ++i) {
            int x[3] = {i, j, k};
            if (!nm.nestable(x))
              throw Error(AMR_EINVAL, "grid " + std::to_string(gi) + " of level " + std::to_string(level + 2) +
                                          " cannot nest in level " + std::to_string(level));
            mark[nm.at(x)] = 1;
          }
    }
  std::vector<std::array<int, 3>> pv;
  for (int k = 0; k < nm.ext[2]; ++k)
    for (int j = 0; j < nm.ext[1]; ++j)
      for (int i = 0; i < nm.ext[0]; ++i) {
        const int x[3] = {nm.lo[0] + i, nm.lo[1] + j, nm.lo[2] + k};
        if (mark[nm.at(x)]) pv.push_back(std::array<int, 3>{x[0], x[1], x[2]});
      }
  const int Nl[3] = {nm.N[0], nm.N[1], nm.N[2]};
  std::vector<IBox> boxes =
      cluster_boxes(nd, Nl, pv, rp->efficiency, rp->max_box, [&](const IBox& B) { return nm.box(B); });
  std::vector<amr_grid> out;
  for (const amr_grid& G : h->grids)
    if (G.level <= level) out.push_back(G);
  for (const IBox& B : boxes) {
    amr_grid G{};
    G.level = level + 1;
    for (int a = 0; a < 3; ++a) {
      G.lo[a] = a < nd ? R * B.lo[a] : 0;
      G.hi[a] = a < nd ? R * B.hi[a] : 1;
    }
    out.push_back(G);
  }
  for (const amr_grid& G : h->grids)
    if (G.level >= level + 2) out.push_back(G);
  return out;
}

// (O)verlap maps of one level of hn from the previous iteration ho.
struct OverlapMaps {
  std::vector<CopyEntry> cp;  // cells, then x-, y-, z-faces
  int4 cls = make_int4(0, 0, 0, 0);
  std::vector<ProlongEntry> pc, pf;
  std::vector<ProjEntry> pj;
};

OverlapMaps build_overlap(const amr_hierarchy* hn, const amr_hierarchy* ho, int l) {
  const int nd = hn->ndim;
  LevelIndex OI;
  OI.build(ho, l);
  LevelIndex PI;
  if (l > 0) PI.build(hn, l - 1);
  const auto& lg = hn->level_grids[l];
  struct Per {
    std::vector<CopyEntry> cp[4];
    std::vector<ProlongEntry> pc, pf;
    std::vector<ProjEntry> pj;
  };
  std::vector<Per> per(lg.size());
  auto one = [&](size_t t) {
    const int gi = lg[t];
    Per& m = per[t];
    const amr_grid& GG = hn->grids[gi];
    const GridDesc& G = hn->desc[gi];
    int n[3] = {1, 1, 1};
    for (int a = 0; a < nd; ++a) n[a] = GG.hi[a] - GG.lo[a];
    // old owner of the element; for faces the lower old grid id of the two
    // cells that share it
    auto old_src = [&](int cls, const int (&p)[3], int64_t& src) -> bool {
      int best = -1;
      int be[3] = {0, 0, 0};
      for (int cand = 0; cand < (cls == 0 ? 1 : 2); ++cand) {
        int w[3] = {p[0], p[1], p[2]};
        if (cand == 1) w[cls - 1] -= 1;
        if (!OI.wrap(w)) continue;
        const int og = OI.find_cell(w);
        if (og < 0) continue;
        if (best < 0 || og < best) {
          best = og;
          be[0] = w[0];
          be[1] = w[1];
          be[2] = w[2];
          if (cand == 1) be[cls - 1] += 1;
        }
      }
      if (best < 0) return false;
      const amr_grid& SG = ho->grids[best];
      src = elem(ho->desc[best], nd, be[0] - SG.lo[0], be[1] - SG.lo[1], be[2] - SG.lo[2]);
      return true;
    };
    for (int cls = 0; cls < (nd == 3 ? 4 : 3); ++cls) {
      const int d = cls - 1;
      int top[3];
      for (int a = 0; a < 3; ++a) top[a] = a < nd ? n[a] + ((cls > 0 && a == d) ? 1 : 0) : 1;
      for (int k = 0; k < top[2]; ++k)
        for (int j = 0; j < top[1]; ++j)
          for (int i = 0; i < top[0]; ++i) {
            const int p[3] = {GG.lo[0] + i, GG.lo[1] + j, GG.lo[2] + k};
            const int64_t dst = elem(G, nd, i, j, k);
            int64_t src = 0;
            if (old_src(cls, p, src)) {
              m.cp[cls].push_back(CopyEntry{(int32_t)dst, (int32_t)src});
              continue;
            }
            if (l == 0) throw Error(AMR_EINVAL, "overlap: level-0 element not covered by the old level 0");
            if (cls == 0) {
              int cc[3] = {floordiv(p[0], 2), floordiv(p[1], 2), nd == 3 ? floordiv(p[2], 2) : 0};
              if (!PI.wrap(cc)) throw Error(AMR_EINVAL, "overlap: prolongation source outside the domain");
              const int pg = PI.find_cell(cc);
              if (pg < 0) throw Error(AMR_EINVAL, "overlap: new cell has no parent");
              const GridDesc& P = hn->desc[pg];
              const amr_grid& PG = hn->grids[pg];
              int code = 0;
              for (int a = 0; a < nd; ++a) code |= (posmod(p[a], 2) << a);
              for (int a = 0; a < nd; ++a)
                if (cc[a] - PG.lo[a] < -P.g + 1 || cc[a] - PG.lo[a] > P.n[a] + P.g - 2)
                  throw Error(AMR_EINVAL, "internal: prolongation stencil leaves the parent box");
              m.pc.push_back(ProlongEntry{(int32_t)dst,
                                          (int32_t)elem(P, nd, cc[0] - PG.lo[0], cc[1] - PG.lo[1], cc[2] - PG.lo[2]),
                                          pg, code});
              continue;
            }
            if (posmod(p[d], 2) == 1) continue;  // inside a coarse cell: projected
            int cc[3];
            for (int a = 0; a < 3; ++a) cc[a] = a < nd ? floordiv(p[a], 2) : 0;
            int w[3] = {cc[0], cc[1], cc[2]};
            int pg = -1;
            if (PI.wrap(w)) pg = PI.find_cell(w);
            if (pg < 0) {
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
            if (pg < 0) throw Error(AMR_EINVAL, "overlap: new face has no parent");
            const GridDesc& P = hn->desc[pg];
            const amr_grid& PG = hn->grids[pg];
            const int a1 = (d + 1) % 3, a2 = (d + 2) % 3;
            for (int a = 0; a < nd; ++a)
              if (w[a] - PG.lo[a] < -P.g + 1 || w[a] - PG.lo[a] > P.n[a] + P.g - 2)
                throw Error(AMR_EINVAL, "internal: prolongation stencil leaves the parent box");
            int code = d;
            if (a1 < nd && posmod(p[a1], 2)) code |= 8;
            if (a2 < nd && posmod(p[a2], 2)) code |= 16;
            m.pf.push_back(ProlongEntry{(int32_t)dst,
                                        (int32_t)elem(P, nd, w[0] - PG.lo[0], w[1] - PG.lo[1], w[2] - PG.lo[2]), pg,
                                        code});
          }
    }
    if (l == 0) return;
    for (int a = 0; a < nd; ++a)
      if (posmod(GG.lo[a], 2) || posmod(GG.hi[a], 2))
        throw Error(AMR_EINVAL, "overlap: new box not aligned to the refinement ratio");
    const int cz = nd == 3 ? n[2] / 2 : 1;
    for (int k = 0; k < cz; ++k)
      for (int j = 0; j < n[1] / 2; ++j)
        for (int i = 0; i < n[0] / 2; ++i) {
          const int loc[3] = {2 * i, 2 * j, nd == 3 ? 2 * k : 0};
          int w[3] = {GG.lo[0] + loc[0], GG.lo[1] + loc[1], GG.lo[2] + loc[2]};
          if (OI.wrap(w) && OI.find_cell(w) >= 0) continue;  // copied coarse cell
          m.pj.push_back(ProjEntry{gi, (int32_t)elem(G, nd, loc[0], loc[1], loc[2])});
        }
  };
  parallel_for(lg.size(), one);
  OverlapMaps M;
  for (int c = 0; c < 4; ++c) {
    for (Per& m : per) M.cp.insert(M.cp.end(), m.cp[c].begin(), m.cp[c].end());
    const int v = (int)M.cp.size();
    if (c == 0) M.cls.x = v;
    if (c == 1) M.cls.y = v;
    if (c == 2) M.cls.z = v;
    if (c == 3) M.cls.w = v;
  }
  for (Per& m : per) {
    M.pc.insert(M.pc.end(), m.pc.begin(), m.pc.end());
    M.pf.insert(M.pf.end(), m.pf.begin(), m.pf.end());
    M.pj.insert(M.pj.end(), m.pj.begin(), m.pj.end());
  }
  return M;
}

template <class T>
void do_overlap(amr_hierarchy* hn, int l, amr_state* Un, amr_state* Up, const amr_hierarchy* ho, const amr_state* Uo,
                hipStream_t s) {
  OverlapMaps M = build_overlap(hn, ho, l);
  CopyEntry* d_cp = nullptr;
  ProlongEntry *d_pc = nullptr, *d_pf = nullptr;
  ProjEntry* d_pj = nullptr;
  try {
    d_cp = dev_upload(M.cp);
    d_pc = dev_upload(M.pc);
    d_pf = dev_upload(M.pf);
    d_pj = dev_upload(M.pj);
    launch_copy2<T>(hn->ndim, d_cp, (int)M.cp.size(), M.cls, dstate<T>(Uo), dstate<T>(Un), s);
    if (l > 0) {
      launch_prolong<T>(hn->ndim, d_pc, (int)M.pc.size(), d_pf, (int)M.pf.size(), hn->d_desc, dstate<T>(Up),
                        dstate<T>(Un), phys(hn), s);
      launch_project<T>(hn->ndim, d_pj, (int)M.pj.size(), hn->d_desc, dstate<T>(Un), phys(hn), s);
    }
    HIPCHK(hipGetLastError());
    // the level's own band, for flags and for the next level's prolongation
    if (l > 0) do_fill<T>(hn, l, AMR_FILL_FULL, Un, Up, s);
    else do_fill<T>(hn, 0, AMR_FILL_SAME_LEVEL, Un, Un, s);
    HIPCHK(hipStreamSynchronize(s));
  } catch (...) {
    (void)hipStreamSynchronize(s);
    (void)hipFree(d_cp);
    (void)hipFree(d_pc);
    (void)hipFree(d_pf);
    (void)hipFree(d_pj);
    throw;
  }
  HIPCHK(hipFree(d_cp));
  HIPCHK(hipFree(d_pc));
  HIPCHK(hipFree(d_pf));
  HIPCHK(hipFree(d_pj));
}

}  // namespace

extern "C" {

amr_status amr_level_cells(const amr_hierarchy* h, int32_t level, int64_t* ncells) {
  try {
    if (!h || !ncells) throw Error(AMR_EINVAL, "null argument");
    if (level < 0 || level >= h->nlev) throw Error(AMR_EINVAL, "level out of range");
    *ncells = level_cells(h, level);
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_cluster_boxes(int32_t ndim, const int32_t* extent, const uint8_t* mask, const uint8_t* admissible,
                             double efficiency, int32_t max_box, int32_t* boxes, int32_t capacity, int32_t* nout) {
  try {
    if (!extent || !mask || !nout) throw Error(AMR_EINVAL, "null argument");
    if (ndim != 2 && ndim != 3) throw Error(AMR_EINVAL, "ndim must be 2 or 3");
    if (!(efficiency > 0.0 && efficiency <= 1.0) || max_box < 1) throw Error(AMR_EINVAL, "bad clustering parameters");
    int N[3] = {1, 1, 1};
    int64_t cells = 1;
    for (int a = 0; a < ndim; ++a) {
      if (extent[a] < 1) throw Error(AMR_EINVAL, "extent must be >= 1");
      N[a] = extent[a];
      cells *= N[a];
    }
    if (cells > ((int64_t)1 << 31)) throw Error(AMR_EUNSUPPORTED, "index space too large");
    std::vector<std::array<int, 3>> pts;
    for (int k = 0; k < N[2]; ++k)
      for (int j = 0; j < N[1]; ++j)
        for (int i = 0; i < N[0]; ++i)
          if (mask[((int64_t)k * N[1] + j) * N[0] + i]) pts.push_back(std::array<int, 3>{i, j, k});
    auto adm = [&](const IBox& B) {
      if (!admissible) return true;
      for (int k = B.lo[2]; k < B.hi[2]; ++k)
        for (int j = B.lo[1]; j < B.hi[1]; ++j)
          for (int i = B.lo[0]; i < B.hi[0]; ++i)
            if (!admissible[((int64_t)k * N[1] + j) * N[0] + i]) return false;
      return true;
    };
    std::vector<IBox> b = cluster_boxes(ndim, N, pts, efficiency, max_box, adm);
    *nout = (int32_t)b.size();
    if ((int32_t)b.size() > capacity || (!boxes && !b.empty()))
      throw Error(AMR_EINVAL, "output capacity too small (needed in *nout)");
    for (size_t q = 0; q < b.size(); ++q)
      for (int a = 0; a < 3; ++a) {
        boxes[6 * q + a] = b[q].lo[a];
        boxes[6 * q + 3 + a] = b[q].hi[a];
      }
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_flag_cells(amr_hierarchy* h, int32_t level, amr_state* U_level, amr_state* U_parent, double theta,
                          uint8_t* flags, void* stream) {
  try {
    if (!h || !U_level || !flags) throw Error(AMR_EINVAL, "null argument");
    if (level < 0 || level >= h->nlev) throw Error(AMR_EINVAL, "level out of range");
    if (level > 0 && !U_parent) throw Error(AMR_EINVAL, "flags above level 0 need the parent state");
    if (!(theta >= 0.0)) throw Error(AMR_EINVAL, "theta must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    if (h->esize == 8)
      do_flags<double>(h, level, U_level, U_parent, theta, flags, s);
    else
      do_flags<float>(h, level, U_level, U_parent, theta, flags, s);
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_regrid(amr_hierarchy* h, int32_t level, amr_state* U_level, amr_state* U_parent,
                      const amr_regrid_params* params, amr_grid* out, int32_t capacity, int32_t* nout, void* stream) {
  try {
    if (!h || !U_level || !params || !nout) throw Error(AMR_EINVAL, "null argument");
    if (level < 0 || level > h->nlev - 2) throw Error(AMR_EINVAL, "level must be in [0, nlevels - 2]");
    if (level > 0 && !U_parent) throw Error(AMR_EINVAL, "regrid above level 0 needs the parent state");
    if (!(params->theta >= 0.0) || !(params->efficiency > 0.0 && params->efficiency <= 1.0) || params->buffer < 0 ||
        params->max_box < 1)
      throw Error(AMR_EINVAL, "bad regrid parameters");
    hipStream_t s = (hipStream_t)stream;
    std::vector<amr_grid> g = h->esize == 8 ? do_regrid<double>(h, level, U_level, U_parent, params, s)
                                            : do_regrid<float>(h, level, U_level, U_parent, params, s);
    *nout = (int32_t)g.size();
    if ((int32_t)g.size() > capacity || !out) throw Error(AMR_EINVAL, "output capacity too small (needed in *nout)");
    std::copy(g.begin(), g.end(), out);
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

amr_status amr_overlap(amr_hierarchy* h_new, int32_t level, amr_state* U_new, amr_state* U_new_parent,
                       const amr_hierarchy* h_old, const amr_state* U_old, void* stream) {
  try {
    if (!h_new || !h_old || !U_new || !U_old) throw Error(AMR_EINVAL, "null argument");
    if (level < 0 || level >= h_new->nlev) throw Error(AMR_EINVAL, "level out of range");
    if (level > 0 && !U_new_parent) throw Error(AMR_EINVAL, "overlap above level 0 needs the new parent state");
    if (h_new->ndim != h_old->ndim || h_new->nlev != h_old->nlev || h_new->R != h_old->R ||
        h_new->esize != h_old->esize)
      throw Error(AMR_EINVAL, "the two hierarchies differ in ndim, levels, ratio or dtype");
    for (int a = 0; a < 3; ++a)
      if (h_new->p.domain[a] != h_old->p.domain[a] || h_new->p.bc[a] != h_old->p.bc[a] ||
          h_new->p.dx0[a] != h_old->p.dx0[a])
        throw Error(AMR_EINVAL, "the two hierarchies differ in domain, spacing or boundaries");
    hipStream_t s = (hipStream_t)stream;
    if (h_new->esize == 8)
      do_overlap<double>(h_new, level, U_new, U_new_parent, h_old, U_old, s);
    else
      do_overlap<float>(h_new, level, U_new, U_new_parent, h_old, U_old, s);
    return AMR_OK;
  } catch (const std::exception& e) {
    return fail(e);
  }
}

}  // extern "C"
