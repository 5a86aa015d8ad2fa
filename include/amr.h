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
 * domain = level-0 cells per axis; dx0 = level-0 cell widths; R = ratio.
 * emf = edge EMF of the constrained-transport update:
 *   AMR_EMF_MEAN (0): the arithmetic mean of the four adjacent face values
 *     (Balsara & Spicer 1999, J. Comput. Phys. 149, 270);
 *   AMR_EMF_UPWIND (1): the upwinded EMF of Gardiner & Stone (2005,
 *     J. Comput. Phys. 205, 509): that mean plus half-cell differences between
 *     face values and a cell-centred reference EMF, each on the upwind side
 *     of the mass flux through its face.  The reference is -v x B with v of
 *     the Hancock half-step cell state and B the cell-centred field at time n
 *     (the time of the normal field the Riemann problems use), so for flow
 *     along a grid axis the edge EMF is exactly the face flux of that axis.
 *     Three more arrays in the workspace; the adjoint and the frozen-branch
 *     forward support AMR_EMF_MEAN only (AMR_EUNSUPPORTED). */
typedef enum { AMR_EMF_MEAN = 0, AMR_EMF_UPWIND = 1 } amr_emf;
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
  int32_t emf;       /* amr_emf */
  int32_t pad;
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
 * lists of every launch cycle.  Limits (AMR_EUNSUPPORTED beyond them): under
 * 2^31 elements per pool and under 4 GiB per field array (the flux kernel
 * addresses by 32-bit byte offsets).  On failure *out is NULL and the status
 * says why (amr_last_error() has the text). */
amr_status amr_create(const amr_params* p, const amr_grid* grids, int32_t ngrids, amr_hierarchy** out);

/* Run every check and table build of amr_create() on the host only (no
 * device is touched; usable without a GPU).  stats (may be NULL, else 8
 * entries) receives: grids, elements per state pool, workspace bytes, copy
 * map entries, prolongation entries, synchronisation entries, flux work
 * items, update work items. */
amr_status amr_validate(const amr_params* p, const amr_grid* grids, int32_t ngrids, int64_t* stats);

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

/* Two-buffer states.  Every level is double buffered: a hierarchy state is
 * a pair (U_a, U_b) plus a parity word whose bit l says that level l's
 * current data is in U_b (else in U_a).  An advance of level l reads its
 * current buffer and writes the other one, then the caller (or
 * amr_coarse_step) flips bit l.  A single-level caller may keep parity 0 and
 * swap U_a / U_b itself. */

/* Time step of the coarse level: dt0 = C / max over all interior cells of
 * all levels of sum_d (|v_d| + c_f,d) / dx0_d, c_f,d the fast speed along d
 * of the cell-centred state.  Written to the device scalar *dt0 (no host
 * synchronisation); level l then steps dt0 / R^l.  The maximum is a
 * wavefront reduction plus an order-independent atomic maximum on the bit
 * pattern of the non-negative value, so dt0 is deterministic. */
amr_status amr_compute_dt(amr_hierarchy* h, const amr_state* U_a, const amr_state* U_b, uint32_t parity,
                          double* dt0, void* stream);

/* Ghost fill of every grid of `level` (the paper's (P)rolongation plus the
 * same-level exchange that ghost cells need; Sec. 4).  U_level holds the
 * level's current data and receives the band; U_parent holds level-1's
 * current data (may be NULL for level 0 or SAME_LEVEL).  Band elements that
 * lie in (cells) or on the boundary of (faces) another grid's interior of the
 * same level, periodic images included, are copied from the lowest-id such
 * grid.  With AMR_FILL_FULL the remaining band elements of a level > 0 are
 * prolonged from the parent level: cells by minmod-limited linear
 * reconstruction of the conserved variables, faces by the divergence-free
 * reconstruction of Balsara (2001, J. Comput. Phys. 174, 614), R = 2.  At
 * level 0 band elements outside a non-periodic boundary copy the nearest
 * domain element (outflow).  AMR_FILL_SAME_LEVEL copies only: the refresh
 * before substeps k >= 1 of a parent step. */
amr_status amr_fill_ghosts_prolong(amr_hierarchy* h, int32_t level, int32_t mode, amr_state* U_level,
                                   const amr_state* U_parent, void* stream);

/* One substep of a set of grids (the (A)dvance of Sec. 4): each grid of level
 * l reads its level's current buffer (parity bit l), advances by dt0 / R^l
 * and writes the other buffer; the caller flips the bits afterwards.  Input
 * is valid on the grid's band `band` (cells [-band, n+band)); output is valid
 * on band-2 (two cells per step feed the slopes and the edge EMFs).
 *   cycle >= 0, band <= 0: the prebuilt batched list of launch cycle
 *     `cycle` (0 <= cycle < R^(nlevels-1)): every grid of every level whose
 *     step falls in that cycle, finest level first, larger grids first, in
 *     one flux and one update launch; level l steps in cycle c when c is a
 *     multiple of R^(nlevels-1-l), its band is g at the first substep of a
 *     parent step and g-2 at the second.
 *   cycle >= 0, band > 0: single-level hierarchies only: all grids, that band.
 *   cycle < 0: exactly the grids grid_subset[0..nsubset) (host array), each
 *     in its own launches, in list order, with the given band: the per-grid
 *     path.
 * Afterwards the coarse/fine registers of the levels that stepped are
 * written into workspace (coarse side for level l < nlevels-1, fine side,
 * slot of the substep, for l > 0); they are valid once every grid of the
 * level has stepped. */
amr_status amr_advance_patches(amr_hierarchy* h, int32_t cycle, const int32_t* grid_subset, int32_t nsubset,
                               int32_t band, const amr_state* U_a, const amr_state* U_b, uint32_t parity,
                               const double* dt0, void* workspace, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * amr_advance_patches() with the same arguments and results (bit for bit),
 * but without the workspace argument.  The flux arrays and coarse/fine
 * registers live in a static device array of the library, 256 MiB per
 * device, held from the first amr_create() on that device until the process
 * ends; the call allocates nothing.  AMR_EINVAL (with the sizes in
 * amr_last_error()) when the hierarchy's workspace (amr_layout) exceeds
 * 256 MiB, or when the current device is not the one the hierarchy was
 * created on.  All calls on one device share the array: calls that overlap
 * on a device (two streams, two host threads) race, and the registers it
 * writes are overwritten by the next call (a caller that synchronises
 * levels with amr_restrict_fluxfix() uses amr_advance_patches()).  Nothing
 * in the array needs to start at zero: each call writes every element it
 * reads.  Kernel timing (amr_set_kernel_timing) is off for this call. */
amr_status amr_advance_patches_noalloc(amr_hierarchy* h, int32_t cycle, const int32_t* grid_subset,
                                       int32_t nsubset, int32_t band, const amr_state* U_a, const amr_state* U_b,
                                       uint32_t parity, const double* dt0, void* stream);

/* Synchronise level fine_level-1 with fine_level after the fine level's R
 * substeps (the (S)ynchronise and (R)estrict of Sec. 4), from the registers
 * in workspace: (1) reflux: each uncovered coarse cell next to covered ones
 * gets U += (+-1/dx_d) (dt_c F_c - sum_k dt_f <F_f>_k) per coarse/fine face
 * (sign + on its high face), <> the mean over the fine faces; (2) EMF
 * correction: each copy of a coarse face with no covered neighbour gets
 * B -= curl(dE) over the coarse/fine edges it touches, dE = sum_k dt_f
 * <E_f>_k - dt_c E_c; (3) restriction: covered coarse cells and every copy of
 * a coarse face with a covered neighbour take the mean of the fine cells or
 * faces.  U_fine: the fine level's current buffer; U_coarse: the coarse
 * level's current buffer (modified). */
amr_status amr_restrict_fluxfix(amr_hierarchy* h, int32_t fine_level, const amr_state* U_fine,
                                amr_state* U_coarse, void* workspace, void* stream);

/* One coarse step of the whole hierarchy on `stream`: dt0 from the CFL
 * reduction, level-0 fill, then the level cycle.
 *   mode 0 (batched): R^(nlevels-1) launch cycles; before each, FULL or
 *     SAME_LEVEL fills of the levels stepping in it (coarse to fine); one
 *     batched advance of all of them (finest level first: the one-GPU form
 *     of the paper's finest-first inter-level threading, Sec. 4); then the
 *     syncs of every level that completed R substeps (fine to coarse).
 *   mode 1 (per-grid): the paper's serial level order (0, 1, 2, 2, 1, 2, 2
 *     for three levels, Sec. 4) with one launch per grid.
 * Both modes produce bitwise identical results.  *parity (host) is read and
 * updated; U_a / U_b as above. */
amr_status amr_coarse_step(amr_hierarchy* h, amr_state* U_a, amr_state* U_b, uint32_t* parity, double* dt0,
                           void* workspace, int32_t mode, void* stream);

/* Capture amr_coarse_step (same arguments, on the non-default `stream`) into
 * HIP graphs: one starting from `parity` and, because level 0 changes buffer
 * every coarse step, one starting from the parity after it.  The graphs bake
 * in the state pointers, dt0 and workspace.  amr_graph_launch() replays the
 * graph that starts from *parity and updates it.  A new capture replaces the
 * old graphs. */
amr_status amr_graph_capture(amr_hierarchy* h, amr_state* U_a, amr_state* U_b, uint32_t parity, double* dt0,
                             void* workspace, int32_t mode, void* stream);
amr_status amr_graph_launch(amr_hierarchy* h, uint32_t* parity, void* stream);

/* Discrete adjoint of nsteps single-level steps (reverse mode of the
 * advance above with the limiter, wave-speed and HLLD region choices frozen
 * at the recomputed forward values; constrained transport and the
 * same-level ghost copy included).  The differentiated map is, per step:
 * refresh the band by the same-level copy (AMR_FILL_SAME_LEVEL), then one
 * band-2 step of every grid of the level with the level-0 step size dts[k]
 * (level l steps by dts[k] / R^l).  Band elements the same-level copy does
 * not fill (prolonged ones, levels > 0) keep U_checkpoint's values through
 * the segment and are constants of the map.
 *   grid_or_level >= 0: that grid, which must be the only grid of its level
 *     (AMR_EUNSUPPORTED otherwise); < 0: every grid of level -(v+1).
 *   dts: host array of the nsteps frozen step sizes (> 0).
 *   U_checkpoint: the state before the first step (read only; only the
 *     selected level is used).
 *   lambda_inout: pools laid out like a state.  On entry, the adjoint of the
 *     state after the last step on the level's own elements (cells [0, n),
 *     faces [0, n] along their normal and [0, n) across); band entries are
 *     ignored.  On exit, the adjoint of the state before the first step: own
 *     elements hold it (band images folded into the elements they copy),
 *     band elements are zero; elements outside the level's grid boxes are
 *     untouched.
 *   workspace: device memory of amr_adjoint_workspace() bytes (the forward
 *     recompute of the segment's states lives there).
 * The cost is one forward pass (nsteps - 1 steps) plus nsteps reverse steps. */
amr_status amr_advance_adjoint(amr_hierarchy* h, int32_t grid_or_level, int32_t nsteps, const double* dts,
                               const amr_state* U_checkpoint, amr_state* lambda_inout, void* workspace,
                               void* stream);

/* Workspace bytes amr_advance_adjoint() needs for that selection and nsteps. */
amr_status amr_adjoint_workspace(const amr_hierarchy* h, int32_t grid_or_level, int32_t nsteps, int64_t* bytes);

/* Frozen-branch advance, the finite-difference check of the adjoint: the
 * map of amr_advance_adjoint() (per step a same-level band copy, then a
 * band-2 step of every grid of `level` with level-0 step size dts[k]) applied
 * to U_pert, with every branch of the scheme (minmod choices, wave-speed
 * extremes and clamps, HLLD region and degeneracy tests) decided by the
 * simultaneous unperturbed run from U_base.  Along such a fixed branch the
 * map is smooth, so (J(U + eps d) - J(U - eps d)) / (2 eps) with both runs
 * frozen on U agrees with the adjoint's <grad J, d> to O(eps^2) however many
 * branch kinks lie within eps of U.  U_base is read; on exit U_pert's
 * elements of the level's grids hold the perturbed result (other elements
 * unchanged).  workspace: amr_frozen_workspace() bytes. */
amr_status amr_advance_frozen(amr_hierarchy* h, int32_t level, int32_t nsteps, const double* dts,
                              const amr_state* U_base, amr_state* U_pert, void* workspace, void* stream);
amr_status amr_frozen_workspace(const amr_hierarchy* h, int64_t* bytes);

/* Adjoint of amr_store_interior(): lambda's own elements of `grid` <- g, the
 * eight interior-layout float64 device arrays amr_store_interior() writes
 * (cells, then x-, y-, z-faces; in 2D g[7] is the cell Bz).  Band elements
 * are not written. */
amr_status amr_store_interior_adjoint(amr_hierarchy* h, int32_t grid, const double* const* g, amr_state* lambda,
                                      void* stream);

/* Adjoint of amr_load_primitive() with respect to the cell density and
 * velocity (pressure and face B held fixed): grad[0..3] (float64 device
 * arrays, interior cell layout) <- d/d(rho, vx, vy, vz) given lambda, the
 * adjoint of the loaded state.  prim[0..3]: the rho, vx, vy, vz arrays
 * passed to amr_load_primitive(). */
amr_status amr_load_primitive_adjoint(amr_hierarchy* h, int32_t grid, const double* const* prim,
                                      const amr_state* lambda, double* const* grad, void* stream);

/* Launch configuration of the batched advance.  tile_policy 0: 16 x 16
 * thread tiles; 1: per grid and band, the tile width in [4, 64] (256 threads
 * per tile) that launches the fewest tiles over the grid.  zchunk: at most
 * this many planes per work item of the flux or fused kernel along z (3D): a
 * tile column of D planes is cut into ceil(D / zchunk) chunks of near-equal
 * length.  launch_mode bit 0: persistent launches (a fixed
 * grid of resident blocks popping the launch's item list from a device
 * queue, one atomic per claim of items, in list order: finest level first,
 * then inside each eighth of the flux list its longest items (most
 * z-planes) first; the queue resets itself at the end of each launch), else
 * one block per claim;
 * bit 1: the item list is cut into 8 contiguous chunks, one per XCD
 * (workgroups reach the XCDs round-robin, so chunk c runs on XCD c and
 * neighbouring tiles share its L2; persistent blocks drain their own chunk
 * first, then the others); bit 2: persistent launches of the flux kernel
 * only, the update one block per item (implied for the flux kernel by bit 0);
 * bit 3: one fused flux-update kernel per launch instead of the two (tiles
 * overlapping by two cells, face fluxes kept in LDS; only those the
 * coarse/fine registers read are stored; persistent with bit 0 or 2; the
 * upwinded EMF always takes the two-kernel path); bits 4-5: c, each block
 * takes 2^c consecutive work items at a time (grids per workgroup for grids
 * of one tile and one z-chunk; else a run of neighbouring tiles), for every
 * kernel of the launch.  launch_mode in [0, 63], else AMR_EINVAL; the claim
 * size never changes results.  Every configuration gives bitwise identical
 * results (the device code contracts multiply-adds only inside a source
 * expression, so an expression rounds the same way in every kernel).
 * Changing tile_policy, zchunk or the XCD chunking (bit 1: items are ordered
 * longest first inside each XCD's chunk, else over the whole list) rebuilds
 * the work lists and drops captured graphs.  Default: 1, 16, 0. */
amr_status amr_set_launch_config(amr_hierarchy* h, int32_t tile_policy, int32_t zchunk, int32_t launch_mode);
amr_status amr_get_launch_config(const amr_hierarchy* h, int32_t* tile_policy, int32_t* zchunk, int32_t* launch_mode);

/* Planes along z per work item of the update (and of the upwinded-EMF edge
 * kernel) in 3-D, separate from the flux kernel's z-chunk (default 2; the
 * update keeps nothing between planes, so short items spread the work over
 * more blocks).  Results do not depend on it, bit for bit.  zchunk in
 * [1, 4096], else AMR_EINVAL.  Changing it rebuilds the work lists and drops
 * captured graphs. */
amr_status amr_set_update_zchunk(amr_hierarchy* h, int32_t zchunk);
amr_status amr_get_update_zchunk(const amr_hierarchy* h, int32_t* zchunk);

#define AMR_TUNE_CANDIDATES 107

typedef struct {
  int32_t tile_policy, zchunk, launch_mode, update_zchunk;
  double ms; /* reps passes over every launch cycle's batched advance */
} amr_tune_entry;

/* Autotuner of the batched advance: fills every level's band (FULL, coarse
 * to fine) and computes dt0 (both redone by the next coarse step), then
 * times the 100 configurations tile_policy x zchunk in {8, 12, 16, 24, 32} x
 * launch_mode in {0, 1, 2, 3, 4, 6, 8, 10, 12, 14} (entries 0..99, under the
 * current update z-chunk), keeps the fastest, and under it times the update
 * z-chunks {1, 2, 4, 8} (entries 100..103) and then, under the kept update
 * z-chunk, claims of 2, 4 and 8 items per block (launch mode bits 4-5,
 * entries 104..106), each over `reps` passes of every launch cycle's batched
 * advance, reading each level's current buffer (parity) and writing the
 * other one, and keeps the fastest of all 107.  Only the advance launches
 * are timed; before each cycle's launch the band fills that open level
 * windows there run as in a coarse step (they rewrite the values the bands
 * already hold), so the advance meets the caches as in a coarse step.  The state the
 * next amr_coarse_step() reads is not changed.  results: host array of
 * AMR_TUNE_CANDIDATES entries or NULL; *chosen (or NULL): index of the kept
 * entry.  Synchronises the stream; drops captured graphs. */
amr_status amr_autotune(amr_hierarchy* h, amr_state* U_a, amr_state* U_b, uint32_t parity, double* dt0,
                        void* workspace, int32_t reps, amr_tune_entry* results, int32_t* chosen, void* stream);

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

/* Host-only check of the hand-written pointwise adjoints that
 * amr_advance_adjoint() is built from (no GPU needed).  which: 0 primitive
 * recovery, 1 conserved from primitive, 2..4 physical flux along x, y, z,
 * 5 fast magnetosonic speed, 6 HLLD flux.  For ntrials random physical
 * states drawn from `seed` it returns the largest relative mismatch of the
 * dot-product test <a, J d> = <J^T a, d>, with J d evaluated exactly by a
 * forward-mode dual number.  `which` out of range or ntrials < 1 returns -1. */
double amr_selfcheck_adjoint(int32_t which, int32_t ntrials, uint64_t seed);

/* Host-only check of the advance kernels' addressing (no GPU needed): builds
 * the hierarchy's tables as amr_validate() does and, for every work list and
 * an element size of elem_bytes (4, 8 or 16), walks the work items as the
 * flux and update kernels do, checking that each 32-bit byte offset the
 * flux kernel loads or stores equals the 64-bit element offset times the
 * element size, that every access lies in its grid's padded box, that no
 * face flux has two writers in one launch, and that every face flux the
 * update reads (directly or through an edge EMF) was written in the same
 * launch.  stats (may be NULL, else 3 entries): loads, stores and reads
 * checked.  AMR_EINVAL with the first failure in amr_last_error();
 * AMR_EUNSUPPORTED when a field array of that element size would exceed
 * 4 GiB. */
amr_status amr_selfcheck_addressing(const amr_params* p, const amr_grid* grids, int32_t ngrids, int32_t elem_bytes,
                                    int64_t* stats);

/* ---- predictive balancing of launch cycles ----
 * One coarse step runs R^(L-1) launch cycles.  Step k of a level-l grid has
 * a window of W = R^(L-1-l) cycles, [k W, (k+1) W): its band is filled at the
 * window's start and its result is first needed (registers, synchronisation,
 * its next step) at the window's end, so it may run in any cycle of the
 * window.  Schedule 0 runs it at the window's start (the level order of
 * Sec. 4).  Schedule 1 applies the paper's predictive load balancing (Sec. 5,
 * eta_l^p = sum_{l' <= l} (s_l' g_l'^p - w_l'^p) and g_l^p = gbar_l -
 * (eta_{l-1}^p - etabar_{l-1}) / s_l, which makes eta_l^p equal for all p)
 * with launch cycles in place of processors: levels are placed finest first
 * (the finest level steps in every cycle and cannot move); for each window
 * of level l, with eta(c) the predicted work already in cycle c, the level's
 * share of cycle c is gbar - (eta(c) - etabar); grids are dealt largest first
 * to the cycle with the largest unfilled share (lowest cycle on ties).
 * Predicted work of one step: the cells of the flux kernel's computed region,
 * prod_d (n_d + 2 band - 2).  The schedule changes where each grid's step is
 * launched, never the arithmetic: results are bitwise equal. */

/* Host-only plan (no GPU, no device tables): cycle_work (host, R^(L-1)
 * doubles, may be NULL) receives the predicted work per cycle; step_cycle
 * (host, may be NULL) receives, for each grid in order, the cycle of each of
 * its R^level steps, concatenated. */
amr_status amr_plan_schedule(const amr_params* p, const amr_grid* grids, int32_t ngrids, int32_t schedule,
                             double* cycle_work, int32_t* step_cycle);
/* Schedule of amr_coarse_step() and of coarse steps captured afterwards
 * (0 or 1; captured graphs of the other schedule are dropped). */
amr_status amr_set_schedule(amr_hierarchy* h, int32_t schedule);
/* Current schedule and, if cycle_work is not NULL, its predicted work per
 * cycle (R^(L-1) doubles). */
amr_status amr_get_schedule(const amr_hierarchy* h, int32_t* schedule, double* cycle_work);

/* ---- regridding and the (O)verlap transfer ----
 * The mesh is adaptive: each level has successive iterations of grids, and
 * the fluid variables move from the previous iteration to the current one
 * (Sec. 2, AMR Algorithm; the (O) of the level cycle, Sec. 4).  The paper
 * fixes neither the refinement criterion nor the clustering; this library
 * flags on the relative centred density jump and clusters with the
 * algorithm of Berger & Rigoutsos (1991, IEEE Trans. Syst. Man Cybern. 21,
 * 1278).  A regrid of level l+1 is: amr_regrid() on the current hierarchy
 * (new grid list), amr_create() on that list, then amr_overlap() level by
 * level, coarse to fine, into the new hierarchy's state. */

typedef struct {
  double theta;      /* flag when |rho(c+e_d) - rho(c-e_d)| > theta (rho(c+e_d) + rho(c-e_d)) for some d */
  double efficiency; /* accept a box when flagged cells >= efficiency * volume, in (0, 1] */
  int32_t buffer;    /* flags grow by this many cells in every direction (>= 0) */
  int32_t max_box;   /* largest extent of a new box, in level-l cells (>= 1) */
} amr_regrid_params;

/* Number of interior cells of the grids of `level` (the flag layout). */
amr_status amr_level_cells(const amr_hierarchy* h, int32_t level, int64_t* ncells);

/* Host-only Berger-Rigoutsos clustering (the rule amr_regrid() applies) of
 * the set cells of mask (host, extent[0] * extent[1] (* extent[2]) bytes, x
 * fastest) inside [0, extent); admissible (host, same layout, may be NULL
 * for all) marks the cells a box may contain.  boxes (host, capacity x 6
 * int32): lo[3], hi[3] per box in emission order; *nout = the count
 * (AMR_EINVAL with *nout set when capacity is too small).  Needs no GPU. */
amr_status amr_cluster_boxes(int32_t ndim, const int32_t* extent, const uint8_t* mask, const uint8_t* admissible,
                             double efficiency, int32_t max_box, int32_t* boxes, int32_t capacity, int32_t* nout);

/* Refinement flags of `level`.  First fills the level's band from its
 * current data: at level 0 a same-level fill of U_level; above it a
 * same-level fill of the parent (U_parent, level-1's current data; only its
 * band changes) and a full fill of U_level.  Then flags[c] = 1 for every
 * interior cell c with |rho(c+e_d) - rho(c-e_d)| > theta (rho(c+e_d) +
 * rho(c-e_d)) along some active axis d (FP64 arithmetic), else 0.  flags:
 * device buffer of amr_level_cells() bytes; grids of the level in increasing
 * index, each grid's interior cells x fastest, then y, then z.  Stream
 * ordered, no synchronisation. */
amr_status amr_flag_cells(amr_hierarchy* h, int32_t level, amr_state* U_level, amr_state* U_parent, double theta,
                          uint8_t* flags, void* stream);

/* New grid list with level+1 re-clustered (0 <= level <= nlevels - 2).
 * Flags of `level` as amr_flag_cells() (band fills included), copied to the
 * host (synchronises the stream); grown by params->buffer cells (periodic
 * axes wrap); kept only where nestable: a level cell c is nestable when the
 * cube c + [-b, b]^ndim, b = g/R + 1, lies in the union of the level's
 * interiors, the proper-nesting rule amr_create() checks.  The grids of
 * level+2 are kept: the level cells under each of them grown by b
 * level-(level+1) cells are added (AMR_EINVAL if one is not nestable).
 * Berger-Rigoutsos clustering of those cells over the level's index space:
 * a box is shrunk to its cells and accepted when cells >= efficiency *
 * volume, every extent <= max_box and every cell nestable, or when it is a
 * single cell; otherwise it is cut at a hole of the signature (axes by
 * decreasing extent, the hole nearest the middle), else at the strongest
 * sign change of the signature's second difference, else halved along the
 * longest axis; boxes are emitted depth first, low part first.  out
 * (host, capacity records): the grids of levels <= level in their order,
 * the new level+1 boxes (times R), then the grids of levels >= level+2 in
 * their order; *nout = the count (AMR_EINVAL with *nout set when capacity
 * is too small).  AMR_EUNSUPPORTED when the level's grids span more than
 * 2^28 cells of index space.  With no flagged cell and no level+2 grids the
 * new level+1 is empty, which amr_create() rejects (levels need grids). */
amr_status amr_regrid(amr_hierarchy* h, int32_t level, amr_state* U_level, amr_state* U_parent,
                      const amr_regrid_params* params, amr_grid* out, int32_t capacity, int32_t* nout, void* stream);

/* (O)verlap of one level of a new iteration of grids (h_new) from the
 * previous iteration (h_old, same domain, spacing, boundaries, level count,
 * ratio and dtype).  U_old: the old level's current data; U_new receives the
 * new level; U_new_parent: the new level-1 data, already transferred and with
 * its band filled (NULL at level 0).  Every interior element of every new
 * grid: a cell lying in an old interior of the same level, or a face lying in
 * or on one (lowest old grid index), is copied; otherwise (level > 0) cells
 * are prolonged from the parent as in the band fill, faces on coarse faces
 * are reconstructed on the face as in the band fill, and the faces inside
 * each prolonged coarse cell start as the mean of the two boundary faces in
 * line with them and take the smallest correction (least squares) that makes
 * every fine cell of the coarse cell divergence-free.  Then the level's band
 * is filled from the new hierarchy (same-level at level 0, full above), so
 * the next level can be transferred and flags taken.  Call it for levels 0,
 * 1, ... in order.  Builds the maps on the host and synchronises the stream
 * before it returns.  AMR_EINVAL: a level-0 element the old level 0 does not
 * cover, a box not aligned to R, or a new cell without a parent. */
amr_status amr_overlap(amr_hierarchy* h_new, int32_t level, amr_state* U_new, amr_state* U_new_parent,
                       const amr_hierarchy* h_old, const amr_state* U_old, void* stream);

/* Text of the last error on this host thread. */
const char* amr_last_error(void);
const char* amr_strerror(amr_status s);

#ifdef __cplusplus
}
#endif

#endif /* AMRMHD_AMR_H */
