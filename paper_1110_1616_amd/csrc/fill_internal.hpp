// Internal fill / CFL / marshalling types and launchers of libamrmhd.so.
#pragma once
#include "amr_internal.hpp"

namespace amr {

// Band element copy: pool element dst takes the value of element src.  The
// map of one fill lists cells first, then x-, y- and z-faces; int4 class
// bounds give the end of each group.
struct CopyEntry {
  int32_t dst;
  int32_t src;
};

// Band element prolongation from the parent level (see the kernels for the
// meaning of `code`).  src is the coarse element, pgrid its grid.
struct ProlongEntry {
  int32_t dst;
  int32_t src;
  int32_t pgrid;
  int32_t code;
};

template <class T>
void launch_copy(int ndim, const CopyEntry* ent, int n, int4 cls, DevState<T> U, hipStream_t s);
// A full band fill (the copies and both prolongations) in one launch.
template <class T>
void launch_fill_full(int ndim, const CopyEntry* cp, int nc, int4 cls, const ProlongEntry* cells, int ncells,
                      const ProlongEntry* faces, int nfaces, const GridDesc* grids, DevState<T> Us, DevState<T> Ud,
                      Phys ph, hipStream_t s);
// Prolongation reads the parent level from Us and writes the band into Ud.
template <class T>
void launch_prolong(int ndim, const ProlongEntry* cells, int ncells, const ProlongEntry* faces, int nfaces,
                    const GridDesc* grids, DevState<T> Us, DevState<T> Ud, Phys ph, hipStream_t s);
template <class T>
void launch_cfl(int ndim, const GridDesc* grids, const int4* items, int nitems, DevState<T> S0, DevState<T> S1,
                uint32_t parity, Phys ph, unsigned long long* acc, ErrBlock* err, double cfl, double* dt0,
                hipStream_t s);
template <class T>
void launch_load_prim(int ndim, const GridDesc& G, const double* const* prim, const double* const* b,
                      DevState<T> U, double gamma, hipStream_t s);
template <class T>
void launch_store(int ndim, const GridDesc& G, DevState<T> U, double* const* out, hipStream_t s);

}  // namespace amr
