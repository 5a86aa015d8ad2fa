// Autotuner of the batched advance: times launch configurations on the
// hierarchy itself and keeps the fastest (amr_autotune).
#include "runtime_internal.hpp"

using namespace amr;
using namespace amrrt;

namespace {

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
