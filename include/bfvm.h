/*
 * bfvm.h -- C ABI of the MI355X (gfx950) diffusion-decay library.
 *
 * The library advances S substrate densities on an nx x ny x nz voxel grid by
 * the locally-one-dimensional (LOD) backward-Euler step of BioFVM-B: a bulk
 * source/sink term, then Dirichlet overwrites interleaved with three implicit
 * 1-D sweeps along x, y and z, each sweep solving one constant-coefficient
 * tridiagonal system per grid line with the Thomas algorithm (paper Sec. 2,
 * the 7-stage solver and Algorithm 1; Thomas constants of App. A), under
 * zero-flux boundaries.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Field layout: a dense array of nz*ny*nx*nsub elements, element
 *    ((z*ny + y)*nx + x)*nsub + s; substrate innermost, x the contiguous
 *    spatial axis.  Element type double (BFVM_F64) or float (BFVM_F32,
 *    BFVM_F32_FAST).
 *  - Field pointers passed to bfvm_step / bfvm_sweep / bfvm_step_adjoint are
 *    DEVICE pointers owned by the caller (for example a contiguous torch
 *    tensor).  The library never frees or reallocates them.  Work is enqueued
 *    asynchronously on the grid's HIP stream; the caller keeps the buffers
 *    alive until that stream has finished the work.
 *  - Arrays passed to bfvm_set_* are HOST pointers; they are copied before
 *    the call returns and may be freed afterwards.
 *  - Voxel indices are flat: (z*ny + y)*nx + x, in [0, nx*ny*nz).
 *  - Units follow the paper: um, min, um^2/min, 1/min.
 *  - Every call returns a status code and never throws.  Arguments are
 *    validated before any device work; a call that fails validation leaves
 *    the grid unchanged.  bfvm_last_error() gives a thread-local detail text
 *    for the last failing call of the calling thread.
 *  - Library-owned device memory (coefficient tables, source and Dirichlet
 *    lists, adjoint workspace) is allocated by bfvm_set_* / the first adjoint
 *    call and freed by bfvm_destroy.  bfvm_step and bfvm_sweep allocate
 *    nothing.
 */
#ifndef BFVM_H
#define BFVM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define BFVM_OK        0
#define BFVM_EINVAL  (-1)   /* bad size, parameter, NULL pointer, unknown dtype, non-finite value */
#define BFVM_ERANGE  (-2)   /* voxel index outside [0, nx*ny*nz) */
#define BFVM_ESTATE  (-3)   /* call out of order (e.g. step before set_params) */
#define BFVM_EDEVICE (-4)   /* HIP runtime error; bfvm_last_error() has hipGetErrorString text */
#define BFVM_ENOMEM  (-5)   /* host or device allocation failed */
#define BFVM_EOFF    (-6)   /* the requested feature is switched off in this library version */
#define BFVM_EIO     (-7)   /* a file could not be opened, read or written */

/* ---- storage / arithmetic types ---------------------------------------- */
#define BFVM_F64       0    /* double storage, double arithmetic, double coefficients */
#define BFVM_F32       1    /* float storage, double in-register arithmetic, double coefficients */
#define BFVM_F32_FAST  2    /* float storage, float arithmetic, coefficients rounded to float */

typedef struct bfvm_grid_s* bfvm_grid;

/* Create a grid of nx*ny*nz voxels with nsub substrates and spacings
 * hx, hy, hz (um).  dtype is one of BFVM_F64 / BFVM_F32 / BFVM_F32_FAST.
 * stream is a hipStream_t (NULL = the null stream) on the current device.
 * Grid size follows the microenvironment resize of Sec. 5.3; the per-axis
 * spacing generalises the single dx of App. A.
 * Errors: EINVAL (n < 1, nsub < 1, h <= 0 or non-finite, bad dtype, out NULL),
 * ENOMEM. */
int bfvm_create(bfvm_grid* out, int64_t nx, int64_t ny, int64_t nz, int32_t nsub,
                double hx, double hy, double hz, int32_t dtype, void* stream);

/* Release all library-owned memory of g.  Synchronises g's stream first.
 * NULL is accepted and ignored. */
int bfvm_destroy(bfvm_grid g);

/* Use another hipStream_t for subsequent work (NULL = the null stream). */
int bfvm_set_stream(bfvm_grid g, void* stream);

/* Diffusion coefficients D[nsub] (um^2/min, >= 0), decay rates
 * lambda[nsub] (1/min, >= 0) and the time step dt (min, > 0).  Builds, in
 * FP64 on the host, the Thomas constants of every (axis, substrate): with
 * r = dt*D/h^2 and beta = dt*lambda/3, the diagonal 1+r+beta at the line
 * ends and 1+2r+beta inside (1+beta for a one-voxel line), off-diagonals -r,
 * denom_i and c'_i as in App. A (eqs. for denom and constant_c).  The decay
 * is split into thirds over the three sweeps.
 * Errors: EINVAL (NULL, negative or non-finite value, dt <= 0), ENOMEM, EDEVICE. */
int bfvm_set_params(bfvm_grid g, const double* D, const double* lambda, double dt);

/* Bulk source/sink cells (production and uptake by cells, Sec. 5.3).
 * count entries; voxel[count]; secretion, saturation, uptake: [count*nsub]
 * (entry k, substrate s at k*nsub + s).  Each step first applies, per voxel
 * and substrate,  u <- (u + dt*sum_k S_k*rho_k) / (1 + dt*sum_k (S_k + U_k)),
 * the implicit bulk update of BioFVM, with entries of the same voxel merged
 * additively.  count = 0 removes all sources.  Replaces any previous list.
 * Requires set_params (the merged terms depend on dt).
 * Errors: EINVAL (count < 0, NULL with count > 0, negative or non-finite
 * rates), ERANGE (voxel index), ESTATE (no params yet), ENOMEM, EDEVICE. */
int bfvm_set_sources(bfvm_grid g, int64_t count, const int64_t* voxel,
                     const double* secretion, const double* saturation, const double* uptake);

/* Dirichlet voxels (Sec. 2: four Dirichlet applications per step, before the
 * x, y and z sweeps and after the z sweep).  value, active: [count*nsub];
 * entry (k, s) with active != 0 overwrites u[voxel[k], s] with value at each
 * application; inactive entries have no effect; for repeated (voxel, s) the
 * last active entry wins.  count = 0 removes all.  Replaces any previous list.
 * Errors: EINVAL, ERANGE, ENOMEM, EDEVICE. */
int bfvm_set_dirichlet(bfvm_grid g, int64_t count, const int64_t* voxel,
                       const double* value, const uint8_t* active);

/* Advance the device field by nsteps LOD steps, in place:
 *   Src, Dir, X, Dir, Y, Dir, Z, Dir   (per step).
 * This is the diffusion-decay solver of Sec. 2: the seven stages (four
 * Dirichlet applications interleaved with the x, y and z Thomas solves of
 * Algorithm 1), preceded by the cells' bulk source/sink update of Sec. 5.3.
 * Asynchronous on the grid's stream; allocates nothing.
 * Errors: EINVAL (field NULL, nsteps < 0), ESTATE (no params), EDEVICE. */
int bfvm_step(bfvm_grid g, void* field, int64_t nsteps);

/* One Thomas sweep along axis (0 = x, 1 = y, 2 = z) of every line and
 * substrate, in place, with no source or Dirichlet stage (Algorithm 1).
 * Errors: EINVAL, ESTATE, EDEVICE. */
int bfvm_sweep(bfvm_grid g, void* field, int32_t axis);

/* One x-slab's share of the x sweep in the distributed solver of Sec. 3.2
 * (the domain split along x into slabs, one per process; the forward
 * elimination runs slab after slab and hands each slab's last x-plane of
 * eliminated values to the next; the backward substitution runs back and
 * hands each slab's first x-plane of solution values to the previous; the
 * lines are processed in blocks, k * processes of them by Eq. 5, so that
 * the slabs overlap).  Chained forward over slabs 0..P-1 and backward over
 * P-1..0 for every block of lines, the two calls give bfvm_sweep's x sweep
 * up to rounding order.
 *   g:      the grid of the WHOLE domain (global nx, ny, nz, S; params set):
 *           its Thomas constants at global x positions are used;
 *   slab:   device array of the slab, [nz][ny][x1 - x0][S] of the grid's
 *           storage type (x fastest, then substrate innermost), updated in
 *           place: the forward call replaces the field values by the
 *           eliminated values d', the backward call d' by the solution;
 *   x0, x1: the slab's x range, 0 <= x0 < x1 <= nx, x1 - x0 <= 2048;
 *   l0, l1: the block of lines, 0 <= l0 < l1 <= ny * nz * S; line
 *           L = (z * ny + y) * S + s;
 *   carry_in:  device array of l1 - l0 values of the compute type (double;
 *           float for BFVM_F32_FAST), entry L - l0 for line L: forward,
 *           d' at x0 - 1 (NULL exactly when x0 == 0); backward, the
 *           solution at x1 (NULL exactly when x1 == nx);
 *   carry_out: device array of l1 - l0 compute-type values: forward, d' at
 *           x1 - 1; backward, the solution at x0.
 * Asynchronous on the grid's stream; allocates nothing; the arrays are the
 * caller's.  Each call reads and writes every slab element of its lines
 * once.  Errors: EINVAL (ranges, NULL slab or carry_out, carry_in given or
 * missing against the rule above, a slab longer than 2048 or whose
 * constants do not fit the LDS), ESTATE (no params), EDEVICE. */
int bfvm_xslab_forward(bfvm_grid g, void* slab, int64_t x0, int64_t x1, int64_t l0, int64_t l1, const void* carry_in,
                       void* carry_out);
int bfvm_xslab_backward(bfvm_grid g, void* slab, int64_t x0, int64_t x1, int64_t l0, int64_t l1,
                        const void* carry_in, void* carry_out);

/* Reverse of one step (not in the paper; the transpose of the step above).
 * field_in: device field at the START of the forward step (not modified).
 * grad: device field, on entry dL/du after the step, on exit dL/du before it.
 * grad_D, grad_lambda: HOST [nsub], INCREMENTED by this step's dL/dD and
 * dL/dlambda.  Recomputes the forward sweeps from field_in into a
 * library-owned workspace of three fields (allocated on the first call),
 * then runs Dir^T, Z^T, Dir^T, Y^T, Dir^T, X^T, Dir^T, Src^T, where each
 * sweep transpose is a transposed Thomas solve (A = L U, solve U^T then L^T),
 * and accumulates per substrate -y^T (L_N x) (w.r.t. r) and -y^T x (w.r.t.
 * beta) with L_N the zero-flux Laplacian: each transposed sweep forms the
 * sums of its lines from the y it holds and the recomputed x, then two
 * launches add the lines of each substrate in a fixed order (chunks of
 * lines, then the chunks: deterministic).  Lines of up to 512 voxels whose
 * tile rows are whole, 16-byte aligned chunks (z; y on plan kinds 1 and 5;
 * x on kind 3 with nsub a multiple of the values per chunk) run a fixed
 * tile shape, 16 values per thread in 512-thread tiles, whatever the axis's
 * plan: z recomputed and transposed in one pass, y and x with the
 * recomputed x fetched into LDS during the solve.
 * Synchronises the stream before returning.
 * Errors: EINVAL, ESTATE, ENOMEM, EDEVICE. */
int bfvm_step_adjoint(bfvm_grid g, const void* field_in, void* grad,
                      double* grad_D, double* grad_lambda);

/* bfvm_step_adjoint for callers that cannot allocate device memory: code
 * under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and synchronisation as
 * bfvm_step_adjoint, and the same kernels; the workspace (three sweep
 * outputs, per-line sums, results) comes from a device array of 98 MiB
 * that the library's code object carries (each GPU the library runs on
 * holds one copy until the process ends) instead of allocations.  The call
 * allocates no device memory, and no host memory except to format an error
 * message.  Limit: 3 * (field bytes, rounded up to 256) + 16 bytes per line
 * of each axis (nelem/nx + nelem/ny + nelem/nz lines) + 48 bytes per
 * substrate must fit in 98 MiB; the 128^3 x 2 FP64 grid does (96 MiB of
 * sweep outputs, 1.5 MiB of sums).  Every call on one GPU shares that GPU's
 * array: calls that overlap on one GPU (several threads or streams) race.
 * Errors: EINVAL (NULL pointers, grid too large: nothing is enqueued),
 * ESTATE, EDEVICE. */
int bfvm_step_adjoint_noalloc(bfvm_grid g, const void* field_in, void* grad, double* grad_D,
                              double* grad_lambda);

/* Device memory the library holds for this grid (coefficient tables, source
 * and Dirichlet lists, adjoint workspace once allocated), in bytes, as the
 * HIP runtime sizes the allocations; the caller-owned fields are not
 * included.  Errors: EINVAL. */
int bfvm_device_bytes(bfvm_grid g, int64_t* bytes);

/* ---- device-side field set-up ----------------------------------------- */
/* Fill a device field of this grid with seeded uniform values in [lo, hi):
 * element i (layout index) = lo + (hi - lo) * U_i, where U_i = (key_i >> 11)
 * * 2^-53, key_i = mix(k ^ i), k = mix(seed ^ (stream << 56)) and mix is the
 * SplitMix64 finaliser (Steele, Lea and Flood, OOPSLA 2014).  FP32 fields
 * get the double value rounded to nearest.  Enqueued on the grid's stream;
 * nothing is copied through host memory (grids beyond host RAM).
 * Errors: EINVAL (NULL field, non-finite or reversed bounds). */
int bfvm_fill_uniform(bfvm_grid g, void* field, uint64_t seed, uint32_t stream, double lo, double hi);

/* The Gaussian initial profile of the end-to-end run (Sec. 5.3), plus seeded
 * noise: element (z, y, x, s) = peak * exp(-d^2 / (2 sigma^2)) + noise * U_i,
 * d = distance of the voxel centre (x + 1/2, y + 1/2, z + 1/2) from (cx, cy,
 * cz), in voxel units; U_i as in bfvm_fill_uniform.  Enqueued on the grid's
 * stream.  Errors: EINVAL (NULL field, sigma <= 0, non-finite values). */
int bfvm_fill_gaussian(bfvm_grid g, void* field, double cx, double cy, double cz, double sigma, double peak,
                       double noise, uint64_t seed, uint32_t stream);

/* Copy a device field of this grid to host memory (host_dst holds
 * nx*ny*nz*nsub elements of the grid's storage type), the read-back behind
 * the end-to-end run's saving of the concentrations (Sec. 5.3).  host_dst
 * is caller-owned (pageable or pinned).  Synchronising: returns after the
 * work enqueued on the grid's stream and the copy have finished.
 * Errors: EINVAL, EDEVICE. */
int bfvm_read_field(bfvm_grid g, const void* field, void* host_dst);

/* Field files.  The paper's end-to-end run writes its initial and final
 * concentrations to files (Sec. 5.3, MATLAB format); these write and read
 * NumPy .npy files instead: C order, shape (nz, ny, nx, nsub), element type
 * '<f8' (BFVM_F64) or '<f4' (BFVM_F32, BFVM_F32_FAST), no conversion.
 * The data moves in 32 MB chunks through two pinned host buffers that the
 * grid allocates on first use (64 MB, freed by bfvm_destroy), so that the
 * device copies on the grid's stream overlap the file I/O.
 *
 * bfvm_save_npy writes format version 1.0 after the work already enqueued on
 * the grid's stream; it returns when the file is complete and closed.
 * bfvm_load_npy reads format versions 1.0-3.0 into a device field of the
 * grid; a file holding shape (nz, ny, nx) is accepted when nsub == 1.  It
 * returns when the data is on the device (the grid's stream is synchronised).
 * Errors: EINVAL (NULL pointers; not a .npy file; element type, order, shape
 * or size that does not match the grid), EIO (open, read, write or close
 * failed), ENOMEM, EDEVICE.  After an error the file or field contents are
 * unspecified. */
int bfvm_save_npy(bfvm_grid g, const void* field, const char* path);
int bfvm_load_npy(bfvm_grid g, void* field, const char* path);

/* Stage timing for measurement.  While enabled, every kernel launch of the
 * grid is bracketed by HIP events on the grid's stream.  Stages: 0 source,
 * 1 Dirichlet, 2 x sweep, 3 y sweep, 4 z sweep.  bfvm_timing_read
 * synchronises, returns the summed milliseconds and launch count of a stage
 * since the last reset, and bfvm_timing_reset clears them. */
int bfvm_timing_enable(bfvm_grid g, int32_t enable);
int bfvm_timing_read(bfvm_grid g, int32_t stage, double* total_ms, int64_t* launches);
int bfvm_timing_reset(bfvm_grid g);

/* Elements swept by a stage since the last reset (sum over its launches),
 * for per-launch byte counts: stages 2..4 only. */
int bfvm_timing_elements(bfvm_grid g, int32_t stage, int64_t* elements);

/* Step schedule.  0: the three sweeps each run over the whole field.
 * 1: the x sweep runs over the whole field, then the y and z sweeps run back
 * to back on x-slabs of slab_width columns, each slab's Dirichlet entries
 * being overwritten between its y and z sweeps.  2: the x and y sweeps run
 * back to back on z-slabs of slab_width planes, then the z sweep runs over
 * the whole field.  The lines of both sweeps of a pair lie inside the slab,
 * so every schedule is the same composition (bitwise the same results); the
 * fused ones let the second sweep of a pair find the first one's output in
 * the GPU's memory-side cache.  -1 (default) is 0, the fastest measured;
 * slab_width 0 picks a slab of about 128 MB.  bfvm_get_schedule returns the
 * schedule and width steps will use.  Errors: EINVAL. */
int bfvm_set_schedule(bfvm_grid g, int32_t schedule, int64_t slab_width);
int bfvm_get_schedule(bfvm_grid g, int32_t* schedule, int64_t* slab_width);

/* Launch plan of a sweep axis, as chosen by the library or set by the
 * tuner.  kind: 0 one-thread-per-line two-pass kernel, 1 register-segmented
 * kernel with strided loads (y/z), 2 register-segmented kernel staged
 * through LDS (x), 3 the kind-1 kernel with every (row, substrate) of the x
 * axis as one line (x), 4 the kind-2 layout in a persistent loop that
 * prefetches the next rows during each solve (x; m 8 or 16, rows of whole
 * 16-byte chunks; runs as kind 2 on a field that is not 16-byte aligned),
 * 5 the kind-1 layout (y/z) or the kind-3 layout (x) with each line taken
 * in two parts by one block of at most 512 threads, the first part kept in
 * LDS between its passes (lines of K*m < n <= 2*K*m, K = 64*w/lpw; runs as
 * the kind-1 / kind-3 plan with as few segments as cover the line for the
 * transposed sweeps, or where the coefficient rows and the LDS copy would
 * take more than half of the CU's LDS).
 * m: elements per thread; w: waves per workgroup; lpw: lines per wave
 * (strided kernels) or rows per workgroup (LDS kernels).  bfvm_set_plan
 * validates the plan against the grid and the device's LDS per workgroup
 * and returns EINVAL for one that does not fit (too few segments, LDS too
 * large, rows that do not split into 16-byte chunks). */
int bfvm_get_plan(bfvm_grid g, int32_t axis, int32_t* kind, int32_t* m, int32_t* w, int32_t* lpw);
int bfvm_set_plan(bfvm_grid g, int32_t axis, int32_t kind, int32_t m, int32_t w, int32_t lpw);

/* Pick each axis's plan by measurement (a utility around the method, not
 * part of it).  For every axis, the current plan and a candidate set are
 * tried, and the fastest is kept:
 *   - x: LDS row tiles and pipelined row tiles of 1-16 rows, and row lines
 *     of 16 or 32 per tile;
 *   - y, z: strided tiles of 16, 32 or 64 lines;
 *   - each with 8, 16 or 32 elements per thread.
 * A candidate is timed over `reps` sweeps (1..100) after one warm-up
 * sweep, with HIP events on the grid's stream.  The sweeps run in place
 * on `field`, a device field of the grid: its contents are overwritten
 * (each sweep is a contraction, so values stay bounded).  best_ms (host
 * [3], may be NULL) receives each axis's time per sweep.  Synchronising.
 * Errors: EINVAL (NULL pointers, reps), ESTATE (before set_params),
 * EDEVICE. */
int bfvm_autotune(bfvm_grid g, void* field, int32_t reps, float* best_ms);

/* Device memory for a field of this grid, with its placement chosen by
 * measurement (a utility around the method, like bfvm_autotune).  The rate
 * of the sweeps on a field depends on where its allocation lands in device
 * memory; so `candidates` allocations of the field's size are made side by
 * side (fewer if they would leave less than max(1/16 of the device, 4 GB)
 * free), each is filled with bounded values and timed on one x, y and z
 * sweep set (after one untimed set) with HIP events on the grid's stream,
 * and the fastest is kept; the others are freed before the call returns.
 * *field receives the kept allocation (nx*ny*nz*nsub elements of the grid's
 * storage type, 256-byte aligned), owned by the caller and released with
 * bfvm_field_free; its contents are unspecified.  cand_ms (host
 * [candidates], may be NULL) receives the timed sweep set of each
 * candidate in ms, -1 for candidates not allocated.  With one candidate
 * the call is a plain device allocation.  Synchronising.
 * Errors: EINVAL (NULL grid or field, candidates outside [1, 16]), ESTATE
 * (before set_params), ENOMEM, EDEVICE. */
int bfvm_field_alloc(bfvm_grid g, int32_t candidates, void** field, float* cand_ms);
/* Release a field allocated by bfvm_field_alloc (NULL is ignored).  The
 * caller makes sure no enqueued work still uses it.  Errors: EDEVICE. */
int bfvm_field_free(void* field);

/* ---- batched domains -------------------------------------------------- */
/*
 * Many independent grids (uneven sizes and substrate counts, any mix of
 * storage types) advanced together.  Each domain's step is cut into work
 * items per stage; in the default grouped mode one kernel launch per stage
 * (a sweep stage: one launch per (storage type, elements per thread) class)
 * covers that stage of every domain, and the launches of one step are
 * captured once in a hipGraph and replayed.  Results are those of bfvm_step
 * on each grid (the same Thomas constants, sources and Dirichlet lists; the
 * x, y and z sweeps use the register-segmented solver with coefficients read
 * from the global tables), up to the rounding of the reciprocal-based
 * solver.  Not in the paper; the paper's closest knob is the block count of
 * its pipelined x sweep (Sec. 3.2, Eq. 5).
 *
 * The member grids are borrowed: they must stay alive while the batch
 * exists.  Their params, sources and Dirichlet lists may change between
 * batch calls (bfvm_set_params / set_sources / set_dirichlet on a member
 * grid): every batch call that runs work first re-reads any grid changed
 * since the batch last read it and rebuilds its programs, so the next
 * bfvm_batch_step / step_adjoint captures its graph again.  A setter must
 * not run while batch work is in flight (the batch calls below return only
 * after their work has finished).
 * The grouped kernels take lines of up to 256 voxels, with line length x
 * substrates at most 2048 on every axis (e.g. 256 voxels x 8 substrates),
 * at most 256 substrates and fewer than 2^31 elements.  A member beyond
 * these limits joins the same graph through its own grid's kernels (as
 * bfvm_step with the plain schedule and the grid's plans; its reverse step
 * as bfvm_step_adjoint, in the grid's own workspace), on a stream of its
 * own beside the grouped launches; such a grid may hold one member only.
 * The batch's calls are not thread-safe; calls on one batch from several
 * threads must be serialised, and a member grid beyond the limits must not
 * run its own reverse step while the batch's is in flight.
 */
typedef struct bfvm_batch_s* bfvm_batch;

#define BFVM_BATCH_GROUPED    0   /* one launch per stage over all domains (default) */
#define BFVM_BATCH_PERSISTENT 1   /* one persistent launch per step: switched off (BFVM_EOFF) */

/* grids[ndomains] (each with set_params done) and fields[ndomains] (device
 * pointers, each holding its grid's field).  stream = hipStream_t; NULL makes
 * the batch create its own non-blocking stream (graphs cannot capture the
 * null stream).  Errors: EINVAL (sizes, NULLs, a grid beyond the grouped
 * limits given for two members), ESTATE (a grid without params), ENOMEM,
 * EDEVICE. */
int bfvm_batch_create(bfvm_batch* out, int32_t ndomains, const bfvm_grid* grids, void* const* fields,
                      void* stream);
int bfvm_batch_destroy(bfvm_batch b);

/* Select the execution mode.  BFVM_BATCH_PERSISTENT returns BFVM_EOFF: its
 * cross-block dependency waits did not complete on gfx950.  Changing the
 * mode resets the tile plans to the defaults.  Errors: EINVAL, EOFF. */
int bfvm_batch_set_mode(bfvm_batch b, int32_t mode);

/* Re-point the per-domain buffers (which = 0: fields, 1: gradients).  The
 * grouped kernels read the pointers from device descriptors at run time, so
 * the graphs stay; a member beyond the grouped limits carries its pointers
 * in its launches, and a change of one makes the next step or reverse step
 * capture its graph again. */
int bfvm_batch_set_fields(bfvm_batch b, int32_t which, void* const* ptrs);

/* nsteps steps of every domain by replaying the captured graph, then waits
 * for the batch stream.  There is no separate capture call: the graph is
 * captured on the first call (and again after a plan, mode or member-grid
 * change).  Errors: EINVAL, EDEVICE. */
int bfvm_batch_step(bfvm_batch b, int64_t nsteps);
/* The same with the launches enqueued directly (no graph). */
int bfvm_batch_step_eager(bfvm_batch b, int64_t nsteps);

/* One reverse step for the distinct domains subset[count] (fields = the
 * state at the start of the step, gradients set with
 * bfvm_batch_set_fields(b, 1, ...)): the adjoint of bfvm_step_adjoint for
 * every domain of the subset, as one captured graph (rebuilt when the subset
 * changes).  grad_D, grad_lambda: HOST arrays of sum_{i} nsub(subset[i])
 * values, in subset order, INCREMENTED (per-item partial sums added on the
 * host in a fixed order: deterministic).  Allocates the subset's workspace
 * (three fields per domain) when the subset changes; a member beyond the
 * grouped limits uses (and on first use allocates) its grid's own.
 * Errors: EINVAL (incl. a repeated domain), ERANGE, ESTATE (no gradient
 * buffers), ENOMEM, EDEVICE. */
int bfvm_batch_step_adjoint(bfvm_batch b, int32_t count, const int32_t* subset, double* grad_D,
                            double* grad_lambda);

/* Autotuner: picks per (axis, line length, substrates, storage type) class
 * the lines per tile (16, 32, 64) and elements per thread (4, 8, 12, 16), and
 * the work per item, by timing the batch step; reuses / writes a JSON cache
 * at cache_path (NULL: no cache), keyed by the GPU architecture and mode.
 * best_ms: the tuned step time.  Runs steps on the fields (their contents
 * change). */
int bfvm_batch_autotune(bfvm_batch b, const char* cache_path, double* best_ms);

/* Elements per thread (m) and lines per tile (lpw) of a domain's axis.
 * ESTATE for a member beyond the grouped limits (its grid's own plan,
 * bfvm_get_plan, applies). */
int bfvm_batch_get_plan(bfvm_batch b, int32_t domain, int32_t axis, int32_t* m, int32_t* lpw);

/* Set a domain axis's plan by hand (the autotuner's choice otherwise):
 * m in {4, 8, 12, 16} (8 at most in persistent mode), lpw in {16, 32, 64},
 * and the 512 / lpw segments of m elements must cover the line.  Rebuilds
 * the forward program; the next reverse step rebuilds its own.  The
 * transposed sweeps of an M = 16 axis run as M = 8 with half the lines per
 * tile (at least 16) where those still cover the line.  Errors: EINVAL
 * (NULL batch, unsupported or too small plan), ERANGE (domain or axis),
 * ESTATE (a member beyond the grouped limits: use bfvm_set_plan on its
 * grid), EDEVICE. */
int bfvm_batch_set_plan(bfvm_batch b, int32_t domain, int32_t axis, int32_t m, int32_t lpw);
/* Work items of one forward step, kernel launches per step, work per item. */
int bfvm_batch_info(bfvm_batch b, int64_t* items, int32_t* launches, int64_t* chunk_elems);

/* Text of a status code, and the calling thread's last error detail. */
const char* bfvm_status_string(int status);
const char* bfvm_last_error(void);

/* Library version string. */
const char* bfvm_version(void);

#ifdef __cplusplus
}
#endif

#endif /* BFVM_H */
