// Synchronisation tables and launchers of libamrmhd.so (internal).
//
// For each fine level f (coarse level c = f-1), built once by amr_create():
//   face registers: one per coarse/fine face (a coarse face with exactly one
//     covered neighbour); slot 0 holds dt_c F_c of the coarse step, slots
//     1..R hold dt_f <F_f> (mean over the fine faces) of each fine substep;
//   edge registers: one per coarse/fine edge (its neighbouring coarse cells
//     are partly covered); slot 0 holds dt_c E_c, slots 1..R dt_f <E_f>;
//   reflux entries (one per uncovered coarse cell with coarse/fine faces),
//   EMF-fix entries (one per copy of a coarse face with no covered
//     neighbour that touches a coarse/fine edge),
//   restriction entries for covered coarse cells and for every copy of a
//     coarse face with a covered neighbour.
// Registers are written, never accumulated, so the result does not depend
// on launch order.
#pragma once
#include <vector>

#include "amr_internal.hpp"

namespace amr {

struct FaceRegEntry {  // register <- dt * mean of flux d at n elements of grid
  int32_t reg, d, grid, n;
  int32_t e[4];
};
struct EdgeRegEntry {  // register <- dt * mean of EMF along axis a at n edges of grid
  int32_t reg, a, grid, n;
  int32_t e[2];
  int32_t pad[2];
};
struct RefluxEntry {  // cell += sum_i coef_i (reg_c - sum_k reg_f[k])
  int32_t cell, n;
  int32_t reg[6];
  double coef[6];
};
struct EmfFixEntry {  // face (normal d) -= sum_i coef_i (sum_k regE_f[k] - regE_c)
  int32_t face, d, n, pad;
  int32_t reg[4];
  double coef[4];
};
struct RestrictEntry {  // coarse element <- mean of fine elements of grid fgrid
  int32_t dst, src, fgrid, d;  // d = -1: cell (R^ndim cells); else face normal d
};

struct SyncTables {
  int nfreg = 0, nereg = 0;
  int64_t reg_off = 0;  // byte offset of this level's registers in the workspace
  int64_t reg_bytes = 0;
  FaceRegEntry *d_freg_c = nullptr, *d_freg_f = nullptr;
  EdgeRegEntry *d_ereg_c = nullptr, *d_ereg_f = nullptr;
  int n_freg_c = 0, n_freg_f = 0, n_ereg_c = 0, n_ereg_f = 0;
  RefluxEntry* d_reflux = nullptr;
  int n_reflux = 0;
  EmfFixEntry* d_emffix = nullptr;
  int n_emffix = 0;
  RestrictEntry* d_restrict = nullptr;
  int n_restrict = 0;
  void release() {
    (void)hipFree(d_freg_c);
    (void)hipFree(d_freg_f);
    (void)hipFree(d_ereg_c);
    (void)hipFree(d_ereg_f);
    (void)hipFree(d_reflux);
    (void)hipFree(d_emffix);
    (void)hipFree(d_restrict);
  }
};

// Register writes of one side of one sync (slot 0: coarse, slot 1..R: fine
// substep) from the face fluxes of the launch that just ran; the table of
// entries [begin, begin + nf + ne) of a batched launch.
template <class T> struct RegJob {
  const FaceRegEntry* fe;
  const EdgeRegEntry* ee;
  T* freg;
  T* ereg;
  int nf, ne, nfreg, nereg, slot, begin;
  double dt_div;  // level l steps dt0 / R^l
};
// Every register write that follows one launch cycle (the levels whose step
// window ends there, both sides of each of their syncs): one kernel launch.
constexpr int kMaxRegJobs = 16;
template <class T> struct RegJobs {
  RegJob<T> j[kMaxRegJobs];
  int n = 0, total = 0;
};
template <class T>
void launch_register_jobs(int ndim, const GridDesc* grids, const RegJobs<T>& jobs, DevFlux<T> F, const double* dt0,
                          bool upwind_emf, hipStream_t s);

// Reflux, EMF fix (coarse level state Uc) and restriction (fine Uf -> Uc).
template <class T>
void launch_sync(int ndim, int R, const GridDesc* grids, const SyncTables& t, const T* freg, const T* ereg,
                 DevState<T> Uf, DevState<T> Uc, hipStream_t s);

}  // namespace amr
