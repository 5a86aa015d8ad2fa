/*
 * amr.h -- C ABI of libamrmhd.so: batched ideal-MHD advance of AMR patches
 * carrying extended ghost zones, on one AMD Instinct MI355X (gfx950).
 *
 * The problem statement follows Carroll-Nellenback, Shroyer, Frank & Ding,
 * "Efficient Parallelization for AMR MHD Multiphysics Calculations;
 * Implementation in AstroBEAR":
 *   - grids ("patches") are regular arrays of cells; grids of level l have cell
 *     width dx_l, with dx_{l-1} = R dx_l, and every grid above level 0 is
 *     nested in the grids of level l-1 (Sec. 2, AMR Algorithm);
 *   - ghost cells decouple the advances of grids of one level, and extended
 *     ghost zones decouple the levels, so each grid on each level advances
 *     on its own for several substeps (abstract; Sec. 1);
 *   - the operations of a level step are prolongation, advance,
 *     synchronisation and restriction, visited finest-level-preferred
 *     (Sec. 4, Threaded Multilevel Advance; Fig. 2).
 * The hyperbolic advance itself is an unsplit second-order MUSCL-Hancock
 * update on primitives with minmod limiting, HLLD fluxes and constrained
 * transport of face-centred B.
 *
 * Memory and ownership.  All field and workspace memory is owned by the
 * caller (device memory, e.g. torch tensors); sizes come from amr_layout().
 * A state is eight pools (rho, mx, my, mz, E cell-centred; Bx, By, Bz
 * face-centred; in 2D Bz is cell-centred) of the hierarchy's dtype.  Each
 * grid occupies a padded box of (n_d + 2g + 1) elements per active axis at
 * its own element offset; element (i, j, k) of grid G, with i in [-g, n_x+g],
 * sits at offset_G + ((k+g_z) P_y + (j+g)) P_x + (i+g) where P_d = n_d + 2g + 1
 * (g_z = 0, P_z = 1 in 2D).  Cells use i < n_x + g; a face with index f along
 * its normal lies between cells f-1 and f.  The handle owns only small device
 * tables built by amr_create().
 *
 * Streams and errors.  Every call that takes a `stream` (a hipStream_t, NULL
 * for the default stream) only enqueues work and returns; nothing
 * synchronises the host except amr_get_error_flags(), amr_store_interior()'s
 * caller-side copies and amr_destroy().  Calls return an amr_status; no C++
 * exception crosses the ABI.  Argument and hierarchy errors are reported
 * synchronously.  Non-physical states met on the device (rho <= 0 or p <= 0)
 * raise a sticky device flag read by amr_get_error_flags().  A handle must not
 * be used from two host threads at once.
 */
#ifndef AMRMHD_AMR_H
#define AMRMHD_AMR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  AMR_OK = 0,
  AMR_EINVAL = -1,       /* bad argument or hierarchy */
  AMR_EHIP = -2,         /* a HIP runtime call failed */
  AMR_ENOMEM = -3,       /* host allocation or a device table allocation failed */
  AMR_ESTATE = -4,       /* non-physical state flagged on the device */
  AMR_EUNSUPPORTED = -5  /* valid request this build does not implement */
} amr_status;

typedef enum { AMR_F32 = 0, AMR_F64 = 1 } amr_dtype;
typedef enum { AMR_BC_PERIODIC = 0, AMR_BC_OUTFLOW = 1 } amr_bc;
typedef enum { AMR_FILL_FULL = 0, AMR_FILL_SAME_LEVEL = 1 } amr_fill_mode;

/* One grid: level and interior cell box [lo, hi) in level-l cell indices
 * (Sec. 2: a regular array of cells on level l).  Unused axes: lo 0, hi 1. */
typedef struct {
  int32_t level;
  int32_t lo[3], hi[3];
} amr_grid;

/* Problem parameters.  ghost = g, the band width in cells of the grid's own
 * level; g >= 2 on a single level and g >= 2R when nlevels > 1 so that a fine
 * grid runs its R substeps from one fill (each step consumes 2 band cells).
 * domain = level-0 cells per axis; dx0 = level-0 cell widths; R = ratio. */
typedef struct {
  int32_t ndim;      /* 2 or 3 */
  int32_t nlevels;   /* >= 1 */
  int32_t ratio;     /* R, refinement ratio (2) */
  int32_t ghost;     /* g */
  int32_t dtype;     /* amr_dtype */
  int32_t bc[3];     /* amr_bc per axis */
  int32_t domain[3]; /* level-0 cells per axis */
  double dx0[3];
  double gamma;      /* ratio of specific heats */
  double cfl;        /* Courant number C of the time step */
} amr_params;

/* Eight device pools (see Memory above). */
typedef struct {
  void* f[8];
} amr_state;

typedef struct amr_hierarchy amr_hierarchy;

/* Build a hierarchy from `ngrids` host grid records.  Validates the problem
 * (ndim, ratio, ghost width, dtype), each box, alignment of level-l boxes to
 * multiples of R, non-overlap within a level and proper nesting (each
 * level-l>0 interior grown by g/R + 1 level-(l-1) cells lies in the union of
 * level-(l-1) interiors, periodic images included).  Builds the device
 * tables: grid descriptors, ghost fill maps (same-level copy before
 * prolongation), synchronisation registers and the finest-level-first work
 * lists of every launch cycle.  On failure *out is NULL and the status says
 * why (amr_last_error() has the text). */
amr_status amr_create(const amr_params* p, const amr_grid* grids, int32_t ngrids, amr_hierarchy** out);

/* Release the handle and its device tables (synchronises the device). */
amr_status amr_destroy(amr_hierarchy* h);

/* Sizes the caller allocates: elements per state pool (each of the 8),
 * bytes of workspace for the advance, and (if grid_offsets is not NULL) each
 * grid's element offset (host array of ngrids). */
amr_status amr_layout(const amr_hierarchy* h, int64_t* state_elems, int64_t* workspace_bytes,
                      int64_t* grid_offsets);

/* Convert host-generated primitive data of one grid into its conserved
 * interior in U (a HIP kernel; data rounded once to the hierarchy dtype).
 * prim: 5 device pointers (rho, vx, vy, vz, p) to float64 arrays in the
 * grid's interior layout (nz, ny, nx), x fastest; b: 3 device pointers to
 * float64 face arrays (nz, ny, nx+1), (nz, ny+1, nx), (nz+1, ny, nx) (2D:
 * Bz is a (1, ny, nx) cell array).  Interior faces on both boundaries are
 * taken as given; cell-centred B is the mean of the two faces. */
amr_status amr_load_primitive(amr_hierarchy* h, int32_t grid, const double* const* prim, const double* const* b,
                              amr_state* U, void* stream);

/* Copy one grid's interior (cells [0, n), faces [0, n] along their normal)
 * from U into 8 float64 device arrays in the interior layout above. */
amr_status amr_store_interior(amr_hierarchy* h, int32_t grid, const amr_state* U, double* const* out,
                              void* stream);

/* Time step of the coarse level: dt0 = C / max over all interior cells of
 * all levels of sum_d (|v_d| + c_f,d) / dx0_d, c_f,d the fast speed along d.
 * Written to the device scalar *dt0 (no host synchronisation); level l then
 * steps dt0 / R^l.  The maximum is a wavefront reduction plus an
 * order-independent atomic maximum, so dt0 is deterministic.  workspace:
 * the advance workspace (its first 256 bytes hold the reduction scratch). */
amr_status amr_compute_dt(amr_hierarchy* h, const amr_state* U, double* dt0, void* workspace, void* stream);

/* Ghost fill of every grid of `level` in U (paper: (P)rolongation plus the
 * same-level exchange that ghost cells need; Sec. 4).  Band elements that
 * lie in (cells) or on the boundary of (faces) another grid's interior of the
 * same level, periodic images included, are copied from it.  With
 * AMR_FILL_FULL the remaining band elements are prolonged from level-1 data
 * in the same U: cells by minmod-limited linear reconstruction of the
 * conserved variables, faces by the divergence-free reconstruction of
 * Balsara (2001, J. Comput. Phys. 174, 614); at level 0 they take the
 * outflow boundary (zero gradient; normal face copied from the last domain
 * face).  AMR_FILL_SAME_LEVEL copies only (the refresh before substeps k >=
 * 1 of a parent step). */
amr_status amr_fill_ghosts_prolong(amr_hierarchy* h, int32_t level, int32_t mode, amr_state* U, void* stream);

/* One substep of a set of grids from U_in to U_out (the (A)dvance of Sec. 4).
 * Each grid g advances by dt0 / R^level(g) on the region its valid band
 * allows: input valid on band `band` (cells [-band, n+band)), output valid on
 * band-2.  cycle >= 0 selects the prebuilt batched work list of launch cycle
 * `cycle` (0 <= cycle < R^(nlevels-1)): every grid of every level whose step
 * falls in that cycle, in one batched launch ordered finest level first, with
 * each level's band taken from its substep index (band argument ignored).
 * cycle < 0 advances exactly the grids in grid_subset[0..nsubset) (host
 * array) with the given band, one grid per launch, in list order: the
 * per-grid path.  Boundary fluxes and EMFs of each stepped grid are
 * accumulated into the synchronisation registers in workspace. */
amr_status amr_advance_patches(amr_hierarchy* h, int32_t cycle, const int32_t* grid_subset, int32_t nsubset,
                               int32_t band, const amr_state* U_in, amr_state* U_out, const double* dt0,
                               void* workspace, void* stream);

/* Synchronise level fine_level-1 with fine_level after the fine level's R
 * substeps (the (S)ynchronise and (R)estrict of Sec. 4): reflux of the
 * uncovered coarse cells at coarse/fine faces with the time-integrated fine
 * fluxes, correction of uncovered coarse faces at coarse/fine edges with the
 * time-integrated fine EMFs, and restriction (mean) of fine cells and faces
 * into covered coarse cells and faces.  U_fine and U_coarse may be the same
 * state; registers are read from workspace and cleared. */
amr_status amr_restrict_fluxfix(amr_hierarchy* h, int32_t fine_level, const amr_state* U_fine,
                                amr_state* U_coarse, void* workspace, void* stream);

/* Discrete adjoint of nsteps single-level steps of one grid or all grids of
 * one level (limiter and Riemann branches frozen from the recomputed forward
 * pass; constrained transport and the periodic ghost fill included).
 * grid_or_level >= 0: that grid; < 0: every grid of level -(v+1).  dts: host
 * array of the nsteps frozen step sizes.  U_checkpoint: state at the first
 * step.  lambda_inout: on entry the adjoint at the last step, on exit at the
 * first.  Forward states of the segment are recomputed into workspace. */
amr_status amr_advance_adjoint(amr_hierarchy* h, int32_t grid_or_level, int32_t nsteps, const double* dts,
                               const amr_state* U_checkpoint, amr_state* lambda_inout, void* workspace,
                               void* stream);

/* Measurement hooks.  With timing enabled, every batched or per-grid
 * advance records HIP events on its stream around its flux and update
 * kernels; amr_kernel_times() waits for them and returns the summed kernel
 * durations (ms) and the number of advance launches since timing was
 * enabled or last read, then resets the counters. */
amr_status amr_set_kernel_timing(amr_hierarchy* h, int32_t enable);
amr_status amr_kernel_times(amr_hierarchy* h, double* flux_ms, double* update_ms, int64_t* nlaunch);

/* Read the sticky device error flags (synchronises the stream).  flags bit 0:
 * non-physical state met.  first_bad_cell: element index of one such cell or
 * -1.  Clears the flags. */
amr_status amr_get_error_flags(amr_hierarchy* h, uint32_t* flags, int64_t* first_bad_cell);

/* Text of the last error on this host thread. */
const char* amr_last_error(void);
const char* amr_strerror(amr_status s);

#ifdef __cplusplus
}
#endif

#endif /* AMRMHD_AMR_H */
