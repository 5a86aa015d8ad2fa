// Host check of the advance kernels' addressing (no GPU needed).
//
// The flux kernel addresses the level arrays by 32-bit byte offsets from
// uniform base pointers (IdxB); the update kernel and the tables by 64-bit
// element indices (Idx).  For every work list of a hierarchy and an element
// size of 4, 8 or 16 bytes this walks the work items exactly as the two
// kernels do (same tile geometry, same per-lane predicates) and checks that
//   - every 32-bit byte offset the flux kernel loads from or stores to is
//     the 64-bit element offset times the element size (no wrap error);
//   - every element it touches lies in its grid's padded box;
//   - no face flux (or reference EMF) has two writers within one launch;
//   - every face flux the update kernel reads (directly, or through the
//     edge EMFs) was written by the flux kernel of the same launch.
#include "advance_common.hpp"
#include "runtime_internal.hpp"

using namespace amr;
using namespace amrrt;

namespace {

struct alignas(8) Pair16 {
  double a, b;
};

struct Counts {
  int64_t loads = 0, stores = 0, reads = 0;
};

// ring entry r of the tile's LDS plane without its corners (as the flux
// kernel maps its first 2 (tw + th) lanes)
void ring_entry_host(int r, int tw, int th, int& ex, int& ey) {
  if (r < tw) { ex = r + 1; ey = 0; }
  else if (r < 2 * tw) { ex = r - tw + 1; ey = th + 1; }
  else if (r < 2 * tw + th) { ex = 0; ey = r - 2 * tw + 1; }
  else { ex = tw + 1; ey = r - 2 * tw - th + 1; }
}

[[noreturn]] void bad(const std::string& what, const FluxItem* fi, int64_t e) {
  std::string s = "addressing check: " + what + " at element " + std::to_string(e);
  if (fi)
    s += " (flux item grid " + std::to_string(fi->grid) + " band " + std::to_string(fi->gv) + " x0 " +
         std::to_string(fi->x0) + " y0 " + std::to_string(fi->y0) + " z " + std::to_string(fi->z0) + ".." +
         std::to_string(fi->z1) + " tw " + std::to_string(fi->tw) + ")";
  throw Error(AMR_EINVAL, s);
}

template <int NDIM, class T> struct Walker {
  const amr_hierarchy* h;
  Counts* cnt;
  // writers per element of the face-flux arrays (3 directions) and of the
  // reference EMF (index 3); reset after each list via `touched`
  std::vector<uint8_t>* wr;
  std::vector<int64_t>* touched;

  void access(const GridDesc& G, const IdxB<NDIM, T>& bx, const Idx<NDIM>& ix, int i, int j, int k, int di, int dj,
              int dk, const FluxItem& it) {
    const int64_t e = ix(i, j, k) + di + (int64_t)dj * ix.sy + (NDIM == 3 ? (int64_t)dk * ix.sz : 0);
    const int64_t box0 = G.off, box1 = G.off + (int64_t)G.P[0] * G.P[1] * G.P[2];
    if (e < box0 || e >= box1) bad("access outside the grid's padded box", &it, e);
    // the kernel's own offset arithmetic: base offset plus byte strides
    auto b = bx(i, j, k);
    b = b + (decltype(b))(di * (int32_t)sizeof(T) + dj * bx.sy + (NDIM == 3 ? dk * bx.sz : 0));
    if ((uint64_t)b != (uint64_t)e * sizeof(T)) bad("byte offset differs from the element offset", &it, e);
    ++cnt->loads;
  }
  void load_cell(const GridDesc& G, const IdxB<NDIM, T>& bx, const Idx<NDIM>& ix, int i, int j, int k,
                 const FluxItem& it) {
    access(G, bx, ix, i, j, k, 0, 0, 0, it);  // cell fields and low faces
    access(G, bx, ix, i, j, k, 1, 0, 0, it);  // high x-face
    access(G, bx, ix, i, j, k, 0, 1, 0, it);  // high y-face
    if (NDIM == 3) access(G, bx, ix, i, j, k, 0, 0, 1, it);  // high z-face
  }
  void store(int d, const GridDesc& G, const IdxB<NDIM, T>& bx, const Idx<NDIM>& ix, int i, int j, int k,
             const FluxItem& it) {
    const int64_t e = ix(i, j, k);
    if (e < G.off || e >= G.off + (int64_t)G.P[0] * G.P[1] * G.P[2]) bad("store outside the grid's padded box", &it, e);
    if ((uint64_t)bx(i, j, k) != (uint64_t)e * sizeof(T)) bad("store byte offset differs from the element offset", &it, e);
    uint8_t& w = wr[d][e];
    if (w) bad("face flux with two writers in one launch", &it, e);
    w = 1;
    touched[d].push_back(e);
    ++cnt->stores;
  }

  void flux_item(const FluxItem& it) {
    const GridDesc& G = h->desc[it.grid];
    const Idx<NDIM> ix(G);
    const IdxB<NDIM, T> bx(G);
    const int gv = it.gv, cl = -gv + 1;
    const int chx = G.n[0] + gv - 1, chy = G.n[1] + gv - 1;
    const int wlo = -gv, whix = G.n[0] + gv, whiy = G.n[1] + gv;
    const int tw = it.tw, th = 256 / tw;
    const int kstart = NDIM == 3 ? std::max(it.z0 - 1, cl) : 0;
    const int kend = NDIM == 3 ? it.z1 : 1;
    const bool upwind = h->upwind_emf;
    for (int tid = 0; tid < 256; ++tid) {
      const int tx = tid % tw, ty = tid / tw;
      const bool live = ty < th;
      const int cx = it.x0 - 1 + tx, cy = it.y0 - 1 + ty;
      const bool act = live && cx >= cl && cx < chx && cy >= cl && cy < chy;
      const bool own = act && tx >= 1 && ty >= 1;
      const int nring = 2 * (tw + th);
      int rex = 0, rey = 0;
      if (tid < nring) ring_entry_host(tid, tw, th, rex, rey);
      const int rcx = it.x0 - 2 + rex, rcy = it.y0 - 2 + rey;
      const bool rok = tid < nring && rcx >= wlo && rcx < whix && rcy >= wlo && rcy < whiy;
      const bool ook = live && cx >= wlo && cx < whix && cy >= wlo && cy < whiy;
      // prologue
      if (NDIM == 3 && ook) load_cell(G, bx, ix, cx, cy, kstart - 1, it);
      if (ook) load_cell(G, bx, ix, cx, cy, kstart, it);
      if (NDIM == 3 && ook) load_cell(G, bx, ix, cx, cy, kstart + 1, it);
      if (rok) load_cell(G, bx, ix, rcx, rcy, kstart, it);
      for (int k = kstart; k < kend; ++k) {
        if (NDIM == 3) {
          if (ook && k + 2 <= kend) load_cell(G, bx, ix, cx, cy, k + 2, it);
          if (rok) load_cell(G, bx, ix, rcx, rcy, k + 1, it);
        }
        if (upwind && act && k >= it.z0 && (tx >= 1 || cx == cl) && (ty >= 1 || cy == cl))
          store(3, G, bx, ix, cx, cy, k, it);
        if (own && k >= it.z0) {
          if (cx > cl) store(0, G, bx, ix, cx, cy, k, it);
          if (cy > cl) store(1, G, bx, ix, cx, cy, k, it);
          if (NDIM == 3 && k > cl) store(2, G, bx, ix, cx, cy, k, it);
        }
      }
    }
  }

  void read(int d, int64_t e, const UpdItem& u) {
    if (e < 0 || e >= h->total_elems || !wr[d][e]) {
      FluxItem f{};
      f.grid = u.grid;
      f.gv = u.gv;
      f.x0 = u.x0;
      f.y0 = u.y0;
      f.z0 = u.z0;
      f.z1 = u.z1;
      f.tw = u.tw;
      bad("update reads a face flux (direction " + std::to_string(d) + ") no flux tile wrote", &f, e);
    }
    ++cnt->reads;
  }
  // edge EMF along axis A at the edge whose high-side element is e (mean
  // of the four face fluxes around it)
  void edge(int A, int64_t e, const int64_t (&st)[3], const UpdItem& u) {
    const int B = (A + 1) % 3, C = (A + 2) % 3;
    read(B, e - st[C], u);
    read(B, e, u);
    read(C, e - st[B], u);
    read(C, e, u);
  }

  void update_item(const UpdItem& u) {
    const GridDesc& G = h->desc[u.grid];
    const Idx<NDIM> ix(G);
    const int gv = u.gv;
    const int uhx = G.n[0] + gv - 2, uhy = G.n[1] + gv - 2, uhz = NDIM == 3 ? G.n[2] + gv - 2 : 0;
    const int tw = u.tw, th = 256 / tw;
    const int64_t st[3] = {1, ix.sy, NDIM == 3 ? (int64_t)ix.sz : 0};
    for (int tid = 0; tid < 256; ++tid) {
      const int tx = tid % tw, ty = tid / tw;
      if (ty >= th) continue;
      const int cx = u.x0 + tx, cy = u.y0 + ty;
      if (cx > uhx || cy > uhy) continue;
      for (int k = u.z0; k < u.z1; ++k) {
        const int64_t e = ix(cx, cy, k);
        const bool cell = cx < uhx && cy < uhy && (NDIM == 2 || k < uhz);
        if (cell)
          for (int d = 0; d < NDIM; ++d) {
            read(d, e, u);
            read(d, e + st[d], u);
          }
        if (h->upwind_emf) continue;  // edges come from the edge-EMF kernel
        if (NDIM == 3) {
          if (cy < uhy && k < uhz) {
            edge(2, e, st, u);
            edge(2, e + st[1], st, u);
            edge(1, e, st, u);
            edge(1, e + st[2], st, u);
          }
          if (cx < uhx && k < uhz) {
            edge(0, e, st, u);
            edge(0, e + st[2], st, u);
            edge(2, e, st, u);
            edge(2, e + st[0], st, u);
          }
          if (cx < uhx && cy < uhy) {
            edge(1, e, st, u);
            edge(1, e + st[0], st, u);
            edge(0, e, st, u);
            edge(0, e + st[1], st, u);
          }
        } else {
          if (cy < uhy) {
            edge(2, e, st, u);
            edge(2, e + st[1], st, u);
          }
          if (cx < uhx) {
            edge(2, e, st, u);
            edge(2, e + st[0], st, u);
          }
        }
      }
    }
  }

  // ---- the fused flux-update kernel (see fused.hip), same predicates ----
  // counts of updates per element (cells, B_x, B_y, B_z) and of flux stores
  std::vector<uint8_t>* up;      // [4]
  std::vector<int64_t>* utouch;  // [4]
  static bool owns(int t, int tdim, int c, int clo, int chi) {
    return (t >= 1 && t <= tdim - 2) || (t == 0 && c == clo) || (t == tdim - 1 && c == chi);
  }
  void upd(int which, int64_t e, const FluxItem& it) {
    uint8_t& w = up[which][e];
    if (w) bad("fused: element updated twice in one launch (field class " + std::to_string(which) + ")", &it, e);
    w = 1;
    utouch[which].push_back(e);
    ++cnt->reads;
  }
  void fused_item(const FluxItem& it) {
    const GridDesc& G = h->desc[it.grid];
    const Idx<NDIM> ix(G);
    const IdxB<NDIM, T> bx(G);
    const int gv = it.gv, cl = -gv + 1;
    const int chx = G.n[0] + gv - 1, chy = G.n[1] + gv - 1;
    const int wlo = -gv, whix = G.n[0] + gv, whiy = G.n[1] + gv;
    const int ul = -gv + 2;
    const int uhx = G.n[0] + gv - 2, uhy = G.n[1] + gv - 2, uhz = NDIM == 3 ? G.n[2] + gv - 2 : 1;
    const int tw = it.tw, th = 256 / tw;
    const int z0 = NDIM == 3 ? it.z0 : 0, z1 = NDIM == 3 ? it.z1 : 1;
    const int kstart = NDIM == 3 ? z0 - 1 : 0, kend = NDIM == 3 ? std::min(z1, uhz) : 0;
    const uint8_t* mask = h->h_fmask.empty() ? nullptr : h->h_fmask.data();
    auto lane = [&](int t, int& cx, int& cy, bool& live, bool& act, bool& xf, bool& yf) {
      const int tx = t % tw, ty = t / tw;
      live = ty < th;
      cx = it.x0 - 1 + tx;
      cy = it.y0 - 1 + ty;
      act = live && cx >= cl && cx < chx && cy >= cl && cy < chy;
      xf = act && tx >= 1 && cx > cl;
      yf = act && ty >= 1 && cy > cl;
    };
    auto need = [&](bool c, const char* what, int64_t e) {
      if (!c) bad(std::string("fused: ") + what, &it, e);
    };
    for (int tid = 0; tid < 256; ++tid) {
      const int tx = tid % tw, ty = tid / tw;
      int cx, cy;
      bool live, act, xf, yf;
      lane(tid, cx, cy, live, act, xf, yf);
      const bool ucol = tx >= 1 && tx <= tw - 2 && cx >= ul && cx < uhx;
      const bool urow = ty >= 1 && ty <= th - 2 && cy >= ul && cy < uhy;
      const bool ucell = live && ucol && urow;
      const bool ubx = live && urow && (ucol || (tx >= 1 && cx == uhx));
      const bool uby = live && ucol && (urow || (ty >= 1 && cy == uhy));
      const bool sx = owns(tx, tw, cx, cl, chx - 1), sy = owns(ty, th, cy, cl, chy - 1);
      const bool rok_dummy = false;
      (void)rok_dummy;
      // neighbour lanes
      auto nb = [&](int t, bool& nact, bool& nxf, bool& nyf) {
        int a, b;
        bool l;
        lane(t, a, b, l, nact, nxf, nyf);
      };
      bool l_act, l_xf, l_yf, d_act, d_xf, d_yf, r_act, r_xf, r_yf, u_act, u_xf, u_yf;
      l_act = l_xf = l_yf = d_act = d_xf = d_yf = r_act = r_xf = r_yf = u_act = u_xf = u_yf = false;
      if (tx >= 1) nb(tid - 1, l_act, l_xf, l_yf);
      if (ty >= 1) nb(tid - tw, d_act, d_xf, d_yf);
      if (tx + 1 < tw) nb(tid + 1, r_act, r_xf, r_yf);
      if (ty + 1 < th && tid + tw < 256) nb(tid + tw, u_act, u_xf, u_yf);
      const bool ook = live && cx >= wlo && cx < whix && cy >= wlo && cy < whiy;
      if (ook) {
        if (NDIM == 3) load_cell(G, bx, ix, cx, cy, kstart - 1, it);
        for (int k = kstart; k <= kend + (NDIM == 3 ? 1 : 0); ++k) load_cell(G, bx, ix, cx, cy, k, it);
      }
      const bool ez = xf && yf;
      if (ez) need(d_xf && l_yf, "E_z reads a face its neighbour lane did not solve", ix(cx, cy, 0));
      for (int k = kstart; k <= kend; ++k) {
        const int64_t e = ix(cx, cy, k);
        const bool zf = NDIM == 3 && act && k >= z0;
        if (act && mask && (mask[e] & 7u)) {
          const bool plane_ok = NDIM == 2 || (k >= z0 && k < z1) || (k == kstart && z0 == ul);
          if (xf && (mask[e] & 1u) && sx && sy && plane_ok) store(0, G, bx, ix, cx, cy, k, it);
          if (yf && (mask[e] & 2u) && sx && sy && plane_ok) store(1, G, bx, ix, cx, cy, k, it);
          if (zf && (mask[e] & 4u) && sx && sy && k < z1) store(2, G, bx, ix, cx, cy, k, it);
        }
        const bool exv = NDIM == 3 && k >= z0 && yf, eyv = NDIM == 3 && k >= z0 && xf;
        if (exv) need(d_act, "E_x reads a z-face its neighbour lane did not solve", e);
        if (eyv) need(l_act, "E_y reads a z-face its neighbour lane did not solve", e);
        if (NDIM == 3) {
          if (ucell && k >= z0 && k < z1) {
            need(eyv && exv && r_xf && u_yf, "B_z face update reads an EMF that was not formed", e);
            upd(3, e, it);
          }
          const int kk = k - 1;
          if (kk >= z0 && kk < z1 && kk < uhz) {
            const int64_t ec = ix(cx, cy, kk);
            if (ucell) {
              need(xf && r_xf && yf && u_yf && zf, "cell update reads a flux that was not formed", ec);
              upd(0, ec, it);
            }
            if (ubx) {
              need(ez && u_xf && u_yf && eyv && kk >= z0, "B_x update reads an EMF that was not formed", ec);
              upd(1, ec, it);
            }
            if (uby) {
              need(ez && r_xf && r_yf && exv && kk >= z0, "B_y update reads an EMF that was not formed", ec);
              upd(2, ec, it);
            }
          }
        } else {
          if (ucell) {
            need(xf && r_xf && yf && u_yf, "cell update reads a flux that was not formed", e);
            upd(0, e, it);
          }
          if (ubx) {
            need(ez && u_xf && u_yf, "B_x update reads an EMF that was not formed", e);
            upd(1, e, it);
          }
          if (uby) {
            need(ez && r_xf && r_yf, "B_y update reads an EMF that was not formed", e);
            upd(2, e, it);
          }
        }
      }
    }
  }
  // every update-region element of every grid step in the list updated once
  // and every face flux a register reads stored once
  void fused_coverage(const LaunchList& L) {
    std::vector<std::pair<int, int>> steps;
    for (int i = 0; i < L.fused.n; ++i) {
      const FluxItem& it = h->h_xitems[L.fused.off + i];
      if (steps.empty() || steps.back() != std::make_pair(it.grid, it.gv)) steps.push_back({it.grid, it.gv});
    }
    const uint8_t* mask = h->h_fmask.empty() ? nullptr : h->h_fmask.data();
    for (auto gs : steps) {
      const GridDesc& G = h->desc[gs.first];
      const Idx<NDIM> ix(G);
      const int gv = gs.second, ul = -gv + 2, cl = -gv + 1;
      const int uh[3] = {G.n[0] + gv - 2, G.n[1] + gv - 2, NDIM == 3 ? G.n[2] + gv - 2 : 1};
      const int zl = NDIM == 3 ? ul : 0;
      FluxItem f{};
      f.grid = gs.first;
      f.gv = gv;
      for (int k = zl; k <= uh[2]; ++k)
        for (int j = ul; j <= uh[1]; ++j)
          for (int i = ul; i <= uh[0]; ++i) {
            const int64_t e = ix(i, j, k);
            const bool ci = i < uh[0], cj = j < uh[1], ck = NDIM == 2 || k < uh[2];
            if (ci && cj && ck && !up[0][e]) bad("fused: cell not updated", &f, e);
            if (cj && ck && !up[1][e]) bad("fused: B_x face not updated", &f, e);
            if (ci && ck && !up[2][e]) bad("fused: B_y face not updated", &f, e);
            if (NDIM == 3 && ci && cj && !up[3][e]) bad("fused: B_z face not updated", &f, e);
          }
      if (!mask) continue;
      // register faces of this grid's step: within the computed face region
      const int ch[3] = {G.n[0] + gv - 1, G.n[1] + gv - 1, NDIM == 3 ? G.n[2] + gv - 1 : 1};
      const int zc0 = NDIM == 3 ? cl : 0;
      for (int k = zc0; k < ch[2]; ++k)
        for (int j = cl; j < ch[1]; ++j)
          for (int i = cl; i < ch[0]; ++i) {
            const int64_t e = ix(i, j, k);
            for (int d = 0; d < NDIM; ++d)
              if ((mask[e] >> d) & 1u) {
                const int c[3] = {i, j, k};
                if (c[d] == cl) continue;  // no face below the computed region
                if (!wr[d][e]) bad("fused: a register's face flux was not stored (direction " + std::to_string(d) + ")", &f, e);
              }
          }
    }
  }

  void list(const LaunchList& L) {
    if (!h->upwind_emf && L.fused.n > 0) {
      for (int i = 0; i < L.fused.n; ++i) fused_item(h->h_xitems[L.fused.off + i]);
      fused_coverage(L);
      for (int d = 0; d < 4; ++d) {
        for (int64_t e : touched[d]) wr[d][e] = 0;
        touched[d].clear();
        for (int64_t e : utouch[d]) up[d][e] = 0;
        utouch[d].clear();
      }
    }
    for (int i = 0; i < L.flux.n; ++i) flux_item(h->h_fitems[L.flux.off + i]);
    for (int i = 0; i < L.upd.n; ++i) update_item(h->h_uitems[L.upd.off + i]);
    for (int d = 0; d < 4; ++d) {
      for (int64_t e : touched[d]) wr[d][e] = 0;
      touched[d].clear();
    }
  }
};

template <int NDIM, class T> void check_all(const amr_hierarchy* h, Counts& cnt) {
  std::vector<uint8_t> wr[4], up[4];
  std::vector<int64_t> touched[4], utouch[4];
  for (auto& w : wr) w.assign(h->total_elems, 0);
  for (auto& w : up) w.assign(h->total_elems, 0);
  Walker<NDIM, T> W{h, &cnt, wr, touched, up, utouch};
  for (const LaunchList& L : h->cycle_lists) W.list(L);
  for (const LaunchList& L : h->eta_lists) W.list(L);
  for (const LaunchList& L : h->band2_lists) W.list(L);
  for (const auto& kv : h->level0_band_lists) W.list(kv.second);
  for (const auto& kv : h->grid_lists) W.list(kv.second);
}

template <class T> void check_dim(const amr_hierarchy* h, Counts& cnt) {
  if (h->ndim == 3)
    check_all<3, T>(h, cnt);
  else
    check_all<2, T>(h, cnt);
}

}  // namespace

extern "C" {

// See the file comment.  elem_bytes: 4, 8 or 16.  stats (may be NULL, else
// 3 entries): flux-kernel loads and stores and update-kernel reads checked.
// AMR_OK when every check passes, AMR_EINVAL with the first failure in
// amr_last_error() otherwise.  Needs no GPU.
amr_status amr_selfcheck_addressing(const amr_params* p, const amr_grid* grids, int32_t ngrids, int32_t elem_bytes,
                                    int64_t* stats) {
  amr_hierarchy* h = nullptr;
  try {
    if (elem_bytes != 4 && elem_bytes != 8 && elem_bytes != 16) throw Error(AMR_EINVAL, "elem_bytes must be 4, 8 or 16");
    g_host_only = true;
    h = build_hierarchy(p, grids, ngrids);
    g_host_only = false;
    if (h->total_elems * (int64_t)elem_bytes >= ((int64_t)1 << 32))
      throw Error(AMR_EUNSUPPORTED, "field arrays of this element size exceed 4 GiB");
    Counts cnt;
    if (elem_bytes == 4)
      check_dim<float>(h, cnt);
    else if (elem_bytes == 8)
      check_dim<double>(h, cnt);
    else
      check_dim<Pair16>(h, cnt);
    if (stats) {
      stats[0] = cnt.loads;
      stats[1] = cnt.stores;
      stats[2] = cnt.reads;
    }
    delete h;
    return AMR_OK;
  } catch (const std::exception& e) {
    g_host_only = false;
    delete h;
    return fail(e);
  }
}

}  // extern "C"
