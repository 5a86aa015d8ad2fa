// Autotuner of the batched advance: times launch configurations on the
// hierarchy itself and keeps the fastest (amr_autotune).
#include "runtime_internal.hpp"

using namespace amr;
using namespace amrrt;

namespace {

// Milliseconds of the batched advance launches of `reps` passes over every
// launch cycle, reading the current buffers and writing the other ones.
// Before each cycle the band fills that open level windows there run as in a
// coarse step (untimed; they rewrite the values the bands already hold), so
// each advance starts from the cache state it meets in a coarse step: timed
// back to back instead, configurations rank differently from the coarse step.
template <class T>
double time_cycles(amr_hierarchy* h, amr_state* Ua, amr_state* Ub, uint32_t parity, const double* dt0, void* ws,
                   int reps, hipStream_t s) {
  const int L = h->nlev, R = h->R, ncyc = (int)h->cycle_lists.size();
  auto cur = [&](int l) { return ((parity >> l) & 1u) ? Ub : Ua; };
  auto fills = [&](int c) {
    if (c == 0) do_fill<T>(h, 0, AMR_FILL_SAME_LEVEL, cur(0), cur(0), s, true);
    for (int l = 1; l < L; ++l) {
      const int span = ipow(R, L - 1 - l);
      if (c % span == 0 && (c / span) % R == 0) do_fill<T>(h, l, AMR_FILL_FULL, cur(l), cur(l - 1), s);
    }
  };
  // events and the per-kernel timing switch are restored on every exit
  struct Events {
    std::vector<hipEvent_t> v;
    ~Events() {
      for (hipEvent_t e : v)
        if (e) (void)hipEventDestroy(e);
    }
  } ev;
  ev.v.assign(2 * (size_t)ncyc * reps, nullptr);
  for (hipEvent_t& e : ev.v) HIPCHK(hipEventCreate(&e));
  struct KeepTiming {
    amr_hierarchy* h;
    bool on;
    ~KeepTiming() { h->timing = on; }
  } keep{h, h->timing};
  h->timing = false;
  for (int c = 0; c < ncyc; ++c) run_list<T>(h, h->cycle_lists[c], Ua, Ub, parity, dt0, ws, s);  // warm-up
  size_t n = 0;
  for (int r = 0; r < reps; ++r)
    for (int c = 0; c < ncyc; ++c, n += 2) {
      fills(c);
      HIPCHK(hipEventRecord(ev.v[n], s));
      run_list<T>(h, h->cycle_lists[c], Ua, Ub, parity, dt0, ws, s);
      HIPCHK(hipEventRecord(ev.v[n + 1], s));
    }
  HIPCHK(hipEventSynchronize(ev.v.back()));
  double ms = 0.0;
  for (size_t i = 0; i < n; i += 2) {
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, ev.v[i], ev.v[i + 1]));
    ms += t;
  }
  return ms;
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
  const int zc[5] = {8, 12, 16, 24, 32};
  const int modes[10] = {0, 1, 2, 3, 4, 6, 8, 10, 12, 14};
  int best = -1, n = 0, bpol = 1, bzc = 8, bmode = 0;
  double best_ms = 0.0;
  for (int pol = 0; pol < 2; ++pol)
    for (int zi = 0; zi < 5; ++zi)
      for (int mi = 0; mi < 10; ++mi, ++n) {
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
  // then the work items a block takes at a time (launch mode bits 4-5)
  int cbest = bmode;
  for (int ci = 1; ci <= 3; ++ci, ++n) {
    const int mode = bmode | (ci << 4);
    set_launch_config(h, bpol, bzc, mode);
    const double ms = time_cycles<T>(h, Ua, Ub, parity, dt0, ws, reps, s);
    if (out) out[n] = amr_tune_entry{bpol, bzc, mode, ubest, ms};
    if (ms < best_ms) {
      best = n;
      best_ms = ms;
      cbest = mode;
    }
  }
  set_launch_config(h, bpol, bzc, cbest);
  return best;
}

}  // namespace

extern "C" {

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
