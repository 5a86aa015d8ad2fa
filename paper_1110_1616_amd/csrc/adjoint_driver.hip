// Host drivers of the discrete adjoint (checkpointed recompute, then the
// reverse steps) and of the frozen-branch forward used to check it.
#include "runtime_internal.hpp"

using namespace amr;
using namespace amrrt;

namespace {

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
  const RawVec<CopyEntry>& cp = h->h_copy[level];
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

}  // extern "C"
