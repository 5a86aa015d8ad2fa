// Host drivers of regridding and the (O)verlap transfer: refinement flags,
// Berger-Rigoutsos clustering under proper nesting, the new iteration's
// grid list and the transfer of the fluid variables into it.
#include "runtime_internal.hpp"

using namespace amr;
using namespace amrrt;

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
  RawVec<CopyEntry> cp;  // cells, then x-, y-, z-faces
  int4 cls = make_int4(0, 0, 0, 0);
  RawVec<ProlongEntry> pc, pf;
  RawVec<ProjEntry> pj;
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
    LevelIndex::Memo omemo, pmemo;  // lookups on the old level and the new parent level
    const amr_grid& GG = hn->grids[gi];
    const GridDesc& G = hn->desc[gi];
    int n[3] = {1, 1, 1};
    for (int a = 0; a < nd; ++a) n[a] = GG.hi[a] - GG.lo[a];
    // old owner of the element: the old grid of this level holding the cell
    // (qa), or for faces the lower old grid id of the two cells that share it
    // (qb: the cell below along the normal), from owner maps painted per
    // class from the old grids that hold any of those cells
    std::vector<int> qa[3], qb[3], owna, ownb;
    PaintScratch ps;
    int top[3] = {1, 1, 1};
    auto old_src = [&](int cls, int i, int j, int k, int64_t& src) -> bool {
      const size_t o = ((size_t)k * top[1] + j) * top[0] + i;
      const int sa = owna[o], sb = cls > 0 ? ownb[o] : -1;
      int best = sa, be[3];
      const int xi[3] = {i, j, k};
      for (int a = 0; a < 3; ++a) be[a] = qa[a][xi[a]];
      if (sb >= 0 && (best < 0 || sb < best)) {
        best = sb;
        for (int a = 0; a < 3; ++a) be[a] = qb[a][xi[a]];
        be[cls - 1] += 1;
      }
      if (best < 0) return false;
      const amr_grid& SG = ho->grids[best];
      src = elem(ho->desc[best], nd, be[0] - SG.lo[0], be[1] - SG.lo[1], be[2] - SG.lo[2]);
      return true;
    };
    for (int cls = 0; cls < (nd == 3 ? 4 : 3); ++cls) {
      const int d = cls - 1;
      for (int a = 0; a < 3; ++a) {
        top[a] = a < nd ? n[a] + ((cls > 0 && a == d) ? 1 : 0) : 1;
        qa[a].resize(top[a]);
        qb[a].resize(top[a]);
        for (int x = 0; x < top[a]; ++x) {
          qa[a][x] = OI.wrap1(a, GG.lo[a] + x);
          qb[a][x] = a == d ? OI.wrap1(a, GG.lo[a] + x - 1) : qa[a][x];
        }
      }
      paint_owners(ho, ho->level_grids[l], qa, owna, ps);
      if (cls > 0) paint_owners(ho, ho->level_grids[l], qb, ownb, ps);
      for (int k = 0; k < top[2]; ++k)
        for (int j = 0; j < top[1]; ++j)
          for (int i = 0; i < top[0]; ++i) {
            const int p[3] = {GG.lo[0] + i, GG.lo[1] + j, GG.lo[2] + k};
            const int64_t dst = elem(G, nd, i, j, k);
            int64_t src = 0;
            if (old_src(cls, i, j, k, src)) {
              m.cp[cls].push_back(CopyEntry{(int32_t)dst, (int32_t)src});
              continue;
            }
            if (l == 0) throw Error(AMR_EINVAL, "overlap: level-0 element not covered by the old level 0");
            if (cls == 0) {
              int cc[3] = {floordiv(p[0], 2), floordiv(p[1], 2), nd == 3 ? floordiv(p[2], 2) : 0};
              if (!PI.wrap(cc)) throw Error(AMR_EINVAL, "overlap: prolongation source outside the domain");
              const int pg = PI.find_cell(cc, pmemo);
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
            if (PI.wrap(w)) pg = PI.find_cell(w, pmemo);
            if (pg < 0) {
              int w2[3] = {cc[0], cc[1], cc[2]};
              w2[d] -= 1;
              if (PI.wrap(w2)) {
                pg = PI.find_cell(w2, pmemo);
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
          if (OI.wrap(w) && OI.find_cell(w, omemo) >= 0) continue;  // copied coarse cell
          m.pj.push_back(ProjEntry{gi, (int32_t)elem(G, nd, loc[0], loc[1], loc[2])});
        }
  };
  parallel_for(lg.size(), one);
  // concatenation: copies class by class, each in grid order; the rest in
  // grid order; every grid's lists go to offsets known in advance, copied
  // by the worker threads
  const size_t ng = per.size();
  std::vector<size_t> oc(4 * ng + 1, 0), opc(ng + 1, 0), opf(ng + 1, 0), opj(ng + 1, 0);
  for (int c = 0; c < 4; ++c)
    for (size_t g = 0; g < ng; ++g) oc[c * ng + g + 1] = oc[c * ng + g] + per[g].cp[c].size();
  for (size_t g = 0; g < ng; ++g) {
    opc[g + 1] = opc[g] + per[g].pc.size();
    opf[g + 1] = opf[g] + per[g].pf.size();
    opj[g + 1] = opj[g] + per[g].pj.size();
  }
  OverlapMaps M;
  M.cp.resize(oc[4 * ng]);
  M.pc.resize(opc[ng]);
  M.pf.resize(opf[ng]);
  M.pj.resize(opj[ng]);
  M.cls = make_int4((int)oc[ng], (int)oc[2 * ng], (int)oc[3 * ng], (int)oc[4 * ng]);
  parallel_for(ng, [&](size_t g) {
    Per& m = per[g];
    for (int c = 0; c < 4; ++c) std::copy(m.cp[c].begin(), m.cp[c].end(), M.cp.begin() + oc[c * ng + g]);
    std::copy(m.pc.begin(), m.pc.end(), M.pc.begin() + opc[g]);
    std::copy(m.pf.begin(), m.pf.end(), M.pf.begin() + opf[g]);
    std::copy(m.pj.begin(), m.pj.end(), M.pj.begin() + opj[g]);
    m = Per();
  });
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
