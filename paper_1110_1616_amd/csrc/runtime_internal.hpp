// Host runtime internals of libamrmhd.so shared by its translation units:
// the hierarchy handle (the opaque amr_hierarchy of include/amr.h), error
// handling, the table builders (tables.hip) and the launch drivers
// (runtime.hip).  Not part of the public ABI.
#pragma once
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

namespace amrrt {

using namespace amr;

extern thread_local std::string g_last_error;
// When set, table builders run on the host only (amr_validate).
extern thread_local bool g_host_only;

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

// Allocator whose value-less construct leaves trivially constructible
// elements uninitialised: large host tables sized first and then filled by
// worker threads are not zeroed (and paged in) by one thread beforehand.
template <class T> struct DefaultInitAlloc : std::allocator<T> {
  template <class U> struct rebind {
    using other = DefaultInitAlloc<U>;
  };
  DefaultInitAlloc() = default;
  template <class U> DefaultInitAlloc(const DefaultInitAlloc<U>&) {}
  template <class U> void construct(U* p) { ::new ((void*)p) U; }
  template <class U, class... A> void construct(U* p, A&&... a) { ::new ((void*)p) U(std::forward<A>(a)...); }
};
template <class T> using RawVec = std::vector<T, DefaultInitAlloc<T>>;

template <class T, class A> T* dev_upload(const std::vector<T, A>& v) {
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
  ListRef fused;  // the same grid steps as fused flux-update items
};

}  // namespace amrrt

using namespace amr;
using amrrt::LaunchList;

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
  FluxItem* d_xitems = nullptr;  // fused flux-update items
  std::vector<FluxItem> h_xitems;
  // per element: bit d where a coarse/fine register reads the face flux
  // normal to d (the fused kernel stores only those)
  std::vector<uint8_t> h_fmask;
  uint8_t* d_fmask = nullptr;
  bool fused = false;  // launch mode bit 3: one fused flux-update kernel per launch
  int fused_pblocks = 0;
  int4* d_cfl = nullptr;
  int n_cfl = 0;
  ErrBlock* d_err = nullptr;  // error block + CFL accumulator (handle-owned)

  // fill maps per level (host copies of the same-level copy maps are kept
  // for the adjoint's transpose)
  std::vector<amrrt::RawVec<CopyEntry>> h_copy;
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
  int claim = 1;               // work items a block takes at a time (launch mode bits 4-5)
  WorkQueue* d_queue = nullptr;
  int flux_pblocks = 0, upd_pblocks = 0;  // persistent grid sizes (resident blocks on the device)
  int device = 0;  // the device the tables live on (current at amr_create)

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
    (void)hipFree(d_xitems);
    (void)hipFree(d_fmask);
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

namespace amrrt {

inline int ipow(int b, int e) {
  int r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

inline int floordiv(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }
inline int posmod(int a, int b) { return ((a % b) + b) % b; }

// Spatial lookup of the grids of one level by cubic buckets of cells.
struct LevelIndex {
  const amr_hierarchy* h = nullptr;
  int level = 0;
  int N[3] = {1, 1, 1};
  // buckets of B^3 cells (sparse: fine levels cover little of their domain)
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
      if (h->p.bc[d] == AMR_BC_PERIODIC) {
        // positions come within one period of the domain: no division then
        if (c[d] < 0) c[d] += N[d];
        else if (c[d] >= N[d]) c[d] -= N[d];
        if (c[d] < 0 || c[d] >= N[d]) c[d] = posmod(c[d], N[d]);
      } else if (c[d] < 0 || c[d] >= N[d]) {
        return false;
      }
    }
    return true;
  }
  // One axis of wrap(): the wrapped position, or -1 outside a non-periodic
  // domain.
  int wrap1(int a, int v) const {
    if (a >= h->ndim) return v;
    if (h->p.bc[a] == AMR_BC_PERIODIC) {
      if (v < 0) v += N[a];
      else if (v >= N[a]) v -= N[a];
      if (v < 0 || v >= N[a]) v = posmod(v, N[a]);
      return v;
    }
    return (v < 0 || v >= N[a]) ? -1 : v;
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
  // in runs from a few grids, so the caller's memo keeps the last eight hits,
  // tried first (the grids of a level are disjoint: a grid of this level
  // holding c is the answer, whatever lookup produced it).
  struct Memo {
    int g[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
    unsigned turn = 0;
  };
  int find_cell(const int (&c)[3], Memo& memo) const {
    for (int m = 0; m < 8; ++m)
      if (holds(memo.g[m], c)) return memo.g[m];
    auto it = buckets.find(key(floordiv(c[0], B), floordiv(c[1], B), floordiv(c[2], B)));
    if (it == buckets.end()) return -1;
    for (int gi : it->second) {
      if (holds(gi, c)) {
        memo.g[memo.turn++ & 7] = gi;
        return gi;
      }
    }
    return -1;
  }
  int find_cell(const int (&c)[3]) const {
    Memo m;
    return find_cell(c, m);
  }
};

// Owner map of a box of positions: own[(z * ny + y) * nx + x] is the grid
// among `grids` (disjoint boxes) whose interior holds the cell
// (q[0][x], q[1][y], q[2][z]), or -1; a negative q (a position outside the
// domain) has no owner.  Each grid is tested against the runs of consecutive
// positions on each axis (a few comparisons) and painted only where it holds
// them, so the cost is the number of grids plus the painted elements, not
// their product.
struct PaintScratch {
  std::vector<std::pair<int, int>> runs[3];
  std::vector<int> vals, sel[3];
};
inline void paint_owners(const amr_hierarchy* h, const std::vector<int>& grids, const std::vector<int> (&q)[3],
                         std::vector<int>& own, PaintScratch& ps) {
  const size_t nx = q[0].size(), ny = q[1].size(), nz = q[2].size();
  own.assign(nx * ny * nz, -1);
  for (int a = 0; a < 3; ++a) {
    ps.vals.clear();
    for (int v : q[a])
      if (v >= 0) ps.vals.push_back(v);
    std::sort(ps.vals.begin(), ps.vals.end());
    ps.runs[a].clear();
    for (int v : ps.vals) {
      if (!ps.runs[a].empty() && v <= ps.runs[a].back().second) {
        ps.runs[a].back().second = std::max(ps.runs[a].back().second, v + 1);
        continue;
      }
      ps.runs[a].push_back({v, v + 1});
    }
  }
  for (int g : grids) {
    const amr_grid& S = h->grids[g];
    bool hit = true;
    for (int a = 0; a < 3 && hit; ++a) {
      bool any = false;
      for (const auto& r : ps.runs[a]) any = any || (r.first < S.hi[a] && S.lo[a] < r.second);
      hit = any;
    }
    if (!hit) continue;
    for (int a = 0; a < 3; ++a) {
      ps.sel[a].clear();
      for (int x = 0; x < (int)q[a].size(); ++x)
        if (q[a][x] >= S.lo[a] && q[a][x] < S.hi[a]) ps.sel[a].push_back(x);
    }
    for (int z : ps.sel[2])
      for (int y : ps.sel[1])
        for (int x : ps.sel[0]) own[((size_t)z * ny + y) * nx + x] = g;
  }
}

// Pool element of (i, j, k) in grid G; every table entry goes through here,
// so an index outside the grid's padded box is caught on the host.
inline int64_t elem(const GridDesc& G, int ndim, int i, int j, int k) {
  const int gz = ndim == 3 ? G.g : 0;
  const int x[3] = {i, j, k};
  for (int a = 0; a < 3; ++a) {
    const int lo = a < ndim ? -G.g : 0, hi = a < ndim ? G.n[a] + G.g : 0;
    if (x[a] < lo || x[a] > hi) throw Error(AMR_EINVAL, "internal: table element outside its grid's box");
  }
  return G.off + (int64_t)(i + G.g) + (int64_t)(j + G.g) * G.P[0] + (int64_t)(k + gz) * G.P[0] * G.P[1];
}

// Run fn(i) for i in [0, n) on up to hardware_concurrency() threads; the
// first exception thrown by any call is rethrown here.
template <class Fn> inline void parallel_for(size_t n, Fn&& fn) {
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

inline int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

template <class T> DevState<T> dstate(const amr_state* s) {
  DevState<T> d;
  for (int i = 0; i < 8; ++i) d.f[i] = (T*)s->f[i];
  return d;
}

template <class T> DevFlux<T> dflux(const amr_hierarchy* h, void* ws) {
  DevFlux<T> F;
  char* base = (char*)ws;
  const int64_t stride = h->total_elems * (int64_t)sizeof(T);
  F.base = base;
  F.stride = (uint64_t)stride;
  for (int d = 0; d < 3; ++d)
    for (int q = 0; q < 7; ++q) F.f[d][q] = (T*)(base + (int64_t)(d * 7 + q) * stride);
  for (int a = 0; a < 3; ++a) {
    F.e[a] = h->upwind_emf ? (T*)(base + (int64_t)(21 + a) * stride) : nullptr;
    F.edge[a] = h->upwind_emf ? (T*)(base + (int64_t)(24 + a) * stride) : nullptr;
  }
  return F;
}

Phys phys(const amr_hierarchy* h);
amr_status fail(const std::exception& e);

// ---- table builders (tables.hip)
void validate(const amr_params* p, const amr_grid* grids, int ngrids);
int pick_tile(int W, int H, int ov, int policy);
int64_t cells_of(const amr_grid& G);
int step_band(const amr_hierarchy* h, int l, int k);
double step_work(const amr_hierarchy* h, int gi, int gv);
void plan_eta(const amr_hierarchy* h, int schedule, std::vector<std::vector<int>>& cyc, std::vector<double>& load);
void build_lists(amr_hierarchy* h);
bool own_elem(const GridDesc& G, int ndim, int cls, const int (&x)[3]);
void class_extent(const GridDesc& G, int ndim, int cls, int (&lo)[3], int (&hi)[3]);
void build_fill_maps(amr_hierarchy* h);
void check_nesting(amr_hierarchy* h);
void build_sync_tables(amr_hierarchy* h, int f);
amr_hierarchy* build_hierarchy(const amr_params* p, const amr_grid* grids, int32_t ngrids);
void rebuild_lists(amr_hierarchy* h);
void set_update_zchunk(amr_hierarchy* h, int zchunk);
void set_launch_config(amr_hierarchy* h, int policy, int zchunk, int mode);

// ---- launch drivers (runtime.hip; instantiated for float and double, and
// run_list also for the frozen-branch pair types)
template <class T>
void run_list(amr_hierarchy* h, const LaunchList& L, const amr_state* Ua, const amr_state* Ub, uint32_t parity,
              const double* dt0, void* ws, hipStream_t s);
template <class T> void write_registers(amr_hierarchy* h, int l, int k, const double* dt0, void* ws, hipStream_t s);
template <class T> void do_sync(amr_hierarchy* h, int f, const amr_state* Uf, amr_state* Uc, void* ws, hipStream_t s);
template <class T>
void do_fill(amr_hierarchy* h, int level, int mode, amr_state* Ul, const amr_state* Up, hipStream_t s,
             bool band2_only = false);
template <class T>
void do_dt(amr_hierarchy* h, const amr_state* Ua, const amr_state* Ub, uint32_t parity, double* dt0, hipStream_t s);
template <class T>
void coarse_step(amr_hierarchy* h, amr_state* Ua, amr_state* Ub, uint32_t& par, double* dt0, void* ws, int mode,
                 hipStream_t s);
// The body of amr_advance_patches with the workspace given (runtime.hip).
void advance_patches(amr_hierarchy* h, int32_t cycle, const int32_t* grid_subset, int32_t nsubset, int32_t band,
                     const amr_state* U_a, const amr_state* U_b, uint32_t parity, const double* dt0, void* workspace,
                     hipStream_t s);
// Resolve, once per device, the device address of the allocation-free
// entry point's static scratch array on the current device (noalloc.hip).
void scratch_init_device(int device);

}  // namespace amrrt
