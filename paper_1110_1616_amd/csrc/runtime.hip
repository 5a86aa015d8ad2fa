// Host runtime and C ABI of libamrmhd.so (see include/amr.h).
//
// amr_create() validates the hierarchy and builds, once, every device table
// the hot path needs: grid descriptors, ghost-fill gather maps, batched work
// lists of each launch cycle (finest level first) and per-grid lists for
// the per-grid path.  The calls after that only enqueue kernels.
#include "runtime_internal.hpp"

using namespace amr;
using namespace amrrt;

namespace amrrt {

thread_local std::string g_last_error;
thread_local bool g_host_only = false;

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
  if constexpr (std::is_same<T, float>::value || std::is_same<T, double>::value) {
    if (h->fused && !h->upwind_emf) {
      // one fused flux-update launch; the update's event pair measures zero
      launch_fused<T>(h->ndim, h->d_desc, h->d_xitems + L.fused.off, L.fused.n, s0, s1, parity, F, h->d_fmask, dt0, ph,
                      h->d_err, h->d_queue, h->persistent_flux ? h->fused_pblocks : 0, h->xcd_chunks, h->claim, s);
      HIPCHK(hipGetLastError());
      if (timing) {
        HIPCHK(hipEventRecord(h->ev_pool[e1], s));
        HIPCHK(hipEventRecord(h->ev_pool[e2], s));
        h->ev_pairs[0].push_back({e0, e1});
        h->ev_pairs[1].push_back({e1, e2});
      }
      return;
    }
  }
  launch_flux<T>(h->ndim, h->d_desc, h->d_fitems + L.flux.off, L.flux.n, s0, s1, parity, F, dt0, ph, h->d_err,
                 h->d_queue, h->persistent_flux ? h->flux_pblocks : 0, h->xcd_chunks, h->claim, h->upwind_emf,
                 s);
  HIPCHK(hipGetLastError());
  if (timing) HIPCHK(hipEventRecord(h->ev_pool[e1], s));
  if constexpr (std::is_same<T, float>::value || std::is_same<T, double>::value) {
    if (h->upwind_emf) {
      launch_emf<T>(h->ndim, h->d_desc, h->d_eitems + L.emf.off, L.emf.n, F, s);
      HIPCHK(hipGetLastError());
    }
  }
  launch_update<T>(h->ndim, h->d_desc, h->d_uitems + L.upd.off, L.upd.n, s0, s1, parity, F, dt0, ph, h->d_queue,
                   h->persistent ? h->upd_pblocks : 0, h->xcd_chunks, h->claim, h->upwind_emf, s);
  HIPCHK(hipGetLastError());
  if (timing) {
    HIPCHK(hipEventRecord(h->ev_pool[e2], s));
    h->ev_pairs[0].push_back({e0, e1});
    h->ev_pairs[1].push_back({e1, e2});
  }
}

// Registers written after level l stepped at its substep k: the coarse side
// of the sync with level l+1 and the fine side (slot 1 + k mod R) of the sync
// with level l-1, queued as jobs of one batched register launch.
template <class T>
void flush_registers(amr_hierarchy* h, RegJobs<T>& jobs, const double* dt0, void* ws, hipStream_t s) {
  launch_register_jobs<T>(h->ndim, h->d_desc, jobs, dflux<T>(h, ws), dt0, h->upwind_emf, s);
  HIPCHK(hipGetLastError());
  jobs.n = 0;
  jobs.total = 0;
}

template <class T>
void add_registers(amr_hierarchy* h, int l, int k, const double* dt0, void* ws, RegJobs<T>& jobs, hipStream_t s) {
  const double div = (double)ipow(h->R, l);
  auto add = [&](const SyncTables& t, const FaceRegEntry* fe, int nf, const EdgeRegEntry* ee, int ne, int slot) {
    if (nf + ne <= 0) return;
    if (jobs.n == kMaxRegJobs) flush_registers<T>(h, jobs, dt0, ws, s);
    T* freg = (T*)((char*)ws + t.reg_off);
    T* ereg = (T*)((char*)ws + t.reg_off + ((int64_t)(1 + h->R) * t.nfreg * 6 * (int64_t)sizeof(T) + 255) / 256 * 256);
    jobs.j[jobs.n++] = RegJob<T>{fe, ee, freg, ereg, nf, ne, t.nfreg, t.nereg, slot, jobs.total, div};
    jobs.total += nf + ne;
  };
  if (l + 1 < h->nlev) {
    const SyncTables& t = h->sync[l + 1];
    add(t, t.d_freg_c, t.n_freg_c, t.d_ereg_c, t.n_ereg_c, 0);
  }
  if (l >= 1) {
    const SyncTables& t = h->sync[l];
    add(t, t.d_freg_f, t.n_freg_f, t.d_ereg_f, t.n_ereg_f, 1 + k % h->R);
  }
}

template <class T>
void write_registers(amr_hierarchy* h, int l, int k, const double* dt0, void* ws, hipStream_t s) {
  RegJobs<T> jobs;
  add_registers<T>(h, l, k, dt0, ws, jobs, s);
  flush_registers<T>(h, jobs, dt0, ws, s);
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
             bool band2_only) {
  if (mode == AMR_FILL_FULL && level > 0 && !band2_only)
    launch_fill_full<T>(h->ndim, h->d_copy[level], h->n_copy[level], h->copy_cls[level], h->d_pcell[level],
                        h->n_pcell[level], h->d_pface[level], h->n_pface[level], h->d_desc, dstate<T>(Up),
                        dstate<T>(Ul), phys(h), s);
  else if (band2_only)
    launch_copy<T>(h->ndim, h->d_copy2[level], h->n_copy2[level], h->copy2_cls[level], dstate<T>(Ul), s);
  else
    launch_copy<T>(h->ndim, h->d_copy[level], h->n_copy[level], h->copy_cls[level], dstate<T>(Ul), s);
  if (mode == AMR_FILL_FULL && level > 0 && band2_only)
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

// Whether level l > 0 needs its same-level band refresh before substeps
// k >= 1.  A substep from band 4 also advances the band cells within 2 of
// the interior, from the same inputs and with the same arithmetic as the
// neighbours that own them (the decoupling by extended ghost zones), so
// those cells already equal the neighbours' interiors bit for bit; only a
// synchronisation with a finer level (restriction, reflux, EMF fix) can
// change a level's interiors between its substeps.  The finest level has
// none, and its refresh would copy equal values.
static bool refresh_needed(const amr_hierarchy* h, int l) { return l + 1 < h->nlev; }

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
        // the refresh before substeps k >= 1 feeds a step from band 2; on
        // the finest level it is skipped (see refresh_needed)
        if (k % R == 0) do_fill<T>(h, l, AMR_FILL_FULL, cur(l), cur(l - 1), s);
        else if (refresh_needed(h, l))
          do_fill<T>(h, l, AMR_FILL_SAME_LEVEL, cur(l), cur(l - 1), s, step_band(h, l, k) == 2);
      }
      run_list<T>(h, lists[c], Ua, Ub, par, dt0, ws, s);
      // levels whose window ends here: every grid has stepped; registers
      // (one launch for all of them), then the level's buffers swap, then
      // the synchronisations it closes
      uint32_t ending = 0;
      RegJobs<T> jobs;
      for (int l = 0; l < L; ++l) {
        const int span = ipow(R, L - 1 - l);
        if ((c + 1) % span) continue;
        ending |= 1u << l;
        add_registers<T>(h, l, c / span, dt0, ws, jobs, s);
      }
      flush_registers<T>(h, jobs, dt0, ws, s);
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
          if (kk > 0 && refresh_needed(h, l + 1))
            do_fill<T>(h, l + 1, AMR_FILL_SAME_LEVEL, cur(l + 1), cur(l), s, step_band(h, l + 1, kk) == 2);
          cyc(l + 1, kk);
        }
        do_sync<T>(h, l + 1, cur(l + 1), cur(l), ws, s);
      }
    };
    cyc(0, 0);
  }
}


#define AMR_RT_INST(T)                                                                                          \
  template void run_list<T>(amr_hierarchy*, const LaunchList&, const amr_state*, const amr_state*, uint32_t,     \
                            const double*, void*, hipStream_t);                                                  \
  template void write_registers<T>(amr_hierarchy*, int, int, const double*, void*, hipStream_t);                \
  template void do_sync<T>(amr_hierarchy*, int, const amr_state*, amr_state*, void*, hipStream_t);              \
  template void do_fill<T>(amr_hierarchy*, int, int, amr_state*, const amr_state*, hipStream_t, bool);           \
  template void do_dt<T>(amr_hierarchy*, const amr_state*, const amr_state*, uint32_t, double*, hipStream_t);    \
  template void coarse_step<T>(amr_hierarchy*, amr_state*, amr_state*, uint32_t&, double*, void*, int, hipStream_t);
AMR_RT_INST(float)
AMR_RT_INST(double)
#undef AMR_RT_INST
template void run_list<FrozenD>(amr_hierarchy*, const LaunchList&, const amr_state*, const amr_state*, uint32_t,
                                const double*, void*, hipStream_t);
template void run_list<FrozenF>(amr_hierarchy*, const LaunchList&, const amr_state*, const amr_state*, uint32_t,
                                const double*, void*, hipStream_t);

void advance_patches(amr_hierarchy* h, int32_t cycle, const int32_t* grid_subset, int32_t nsubset, int32_t band,
                     const amr_state* U_a, const amr_state* U_b, uint32_t parity, const double* dt0, void* workspace,
                     hipStream_t s) {
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
    // levels in order of first appearance (a fixed array: the allocation-free
    // entry point runs this too)
    int levels[32], nl = 0;
    for (int i = 0; i < nsubset; ++i) {
      auto it = h->grid_lists.find({grid_subset[i], band});
      if (it == h->grid_lists.end()) throw Error(AMR_EINVAL, "bad grid id or band for the per-grid path");
      run(it->second);
      const int l = h->desc[grid_subset[i]].level;
      if (std::find(levels, levels + nl, l) == levels + nl) levels[nl++] = l;
    }
    for (int i = 0; i < nl; ++i) regs(levels[i], levels[i] == 0 ? 0 : (h->g - band) / 2);
  }
}

}  // namespace amrrt

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
      h->fused_pblocks = prop.multiProcessorCount *
                         (h->esize == 8 ? fused_occupancy<double>(h->ndim) : fused_occupancy<float>(h->ndim));
      h->device = dev;
      scratch_init_device(dev);
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
    advance_patches(h, cycle, grid_subset, nsubset, band, U_a, U_b, parity, dt0, workspace, (hipStream_t)stream);
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
    *launch_mode = (h->persistent ? 1 : 0) | (h->xcd_chunks ? 2 : 0) | (h->persistent_flux && !h->persistent ? 4 : 0) |
                 (h->fused ? 8 : 0) | ((h->claim == 8 ? 3 : h->claim / 2) << 4);
  return AMR_OK;
}

}  // extern "C"
