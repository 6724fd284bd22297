/*
 * mpdata.h -- C ABI of libmpdata, an MI355X (gfx950) implementation of the
 * MPDATA advection time step.
 *
 * The operation.  One MPDATA time step advances a cell-centred scalar psi
 * through a chain of dependent stencil stages that read five input matrices
 * (psi, the three face Courant numbers u1, u2, u3, and the density h) and
 * produce one output matrix, psi at the next time level (paper, section 5.2,
 * "Introduction to MPDATA"; the 7-point neighbourhood maximum of Listing 1
 * is one of the stages).  The stages are the donor-cell (upwind) pass, the
 * antidiffusive pseudo-velocities, the non-oscillatory limiter (bounds,
 * factors, limited velocities) and the corrective donor-cell pass, as
 * defined in the MPDATA literature the paper cites (Smolarkiewicz 1984;
 * Smolarkiewicz & Grabowski 1990; the density-weighted form of Smolarkiewicz
 * & Margolin 1998).  The library fuses all stages of a step into one
 * kernel, so intermediates never leave the chip (the paper's (3+1)D
 * decomposition idea, section 5.3, recast for LDS and registers).
 *
 * Conventions shared by every entry point.
 *  - All functions are thread-compatible, never abort and never throw;
 *    they return MPDATA_OK (0) or a negative error code.  The text of the
 *    last error of a context is returned by mpdata_last_error().
 *  - Grid: nx * ny * nz cells, C order [k][j][i] with i (x) fastest.
 *  - Face Courant arrays hold n+1 faces along their own axis:
 *      u1[nz][ny][nx+1]   face i' lies between cells i'-1 and i'
 *      u2[nz][ny+1][nx]
 *      u3[nz+1][ny][nx]
 *    A positive value carries mass toward +axis.  With periodic boundaries
 *    face n along an axis is the same face as face 0 and must hold the
 *    same value (checked by mpdata_create).
 *  - Element type: double for MPDATA_FP64; float for MPDATA_FP32, which
 *    stores fields and runs the bulk stencil in FP32 while the limiter's
 *    inflow/outflow sums and its divides run in FP64; each factor, capped
 *    at 1, is rounded once to FP32 and the minimum of two factors is taken
 *    on the rounded values, which equals the rounded FP64 minimum bit for
 *    bit (rounding is monotone).  Mass sums are compensated (double-double).
 *  - Range of psi: FP64 steps stay finite for |psi| below about 1e100 (the
 *    pseudo-velocity divides once per face by a product of three ratio
 *    denominators); FP32 steps take the three ratios separately and stay
 *    finite for |psi| below about 1e37, at any small magnitude.
 *  - Pointers named "device" are device memory of the current HIP device;
 *    the caller owns them and keeps them alive until mpdata_destroy().  The
 *    library allocates no device memory: everything it needs beyond the
 *    caller's arrays lives in the caller's workspace.
 *  - Work is enqueued on the caller's HIP stream (hipStream_t passed as
 *    void*, NULL = the legacy default stream) and is asynchronous unless
 *    stated otherwise.
 */
#ifndef MPDATA_H
#define MPDATA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MPDATA_ABI_VERSION 1

enum {
    MPDATA_OK = 0,
    MPDATA_EINVAL = -1,     /* invalid argument (message says which) */
    MPDATA_ENOMEM = -2,     /* workspace too small / host allocation failed */
    MPDATA_EDEVICE = -3,    /* a HIP call failed (message holds its text) */
    MPDATA_ENOTSUP = -4,    /* valid but unsupported combination */
    MPDATA_ENONFINITE = -5  /* a mass sum found NaN or Inf in psi */
};

enum { MPDATA_FP64 = 0, MPDATA_FP32 = 1 };
/* flags: NO_GRAPH -- launch every step on its own instead of replaying a
 * captured graph of step launches (a graph is otherwise built at creation).
 * VSIGN -- fields of variable sign: the
 * ratios of the antidiffusive pseudo-velocity take |psi1| in place of psi1
 * (the variable-sign option of the MPDATA literature the paper cites,
 * Smolarkiewicz & Margolin 1998).  DIV -- flows that are not divergence-free:
 * the pseudo-velocity gains the divergent-flow term -(1/4)(U/G) dv, dv the
 * centred divergence of the pass's velocity field across the face
 * (Smolarkiewicz 1984); on a discretely divergence-free flow it adds exact
 * zeros.  VSIGN and DIV are built for the default launch shapes (tile 0, 2
 * or 5).  TVEL -- Courant numbers that change in time (single-grid contexts,
 * iord 2, default launch shape, not with VSIGN): mpdata_step_tv advances the
 * state with the Courant numbers given at both ends of every step; see
 * there. */
enum { MPDATA_FLAG_NO_GRAPH = 1, MPDATA_FLAG_VSIGN = 2, MPDATA_FLAG_DIV = 4, MPDATA_FLAG_TVEL = 8 };
enum { MPDATA_BC_PERIODIC = 0, MPDATA_BC_OPEN = 1 }; /* OPEN = zero gradient */

typedef struct {
    int32_t nx, ny, nz;   /* cells, each >= 1; every array < 2^31 elements
                             and (nx+1)*(ny+1)*word < 2 GiB (one x-y plane
                             is addressed with 32-bit byte offsets, and an
                             offset of 2^31 masks a lane) */
    int32_t dtype;        /* MPDATA_FP64 or MPDATA_FP32 */
    int32_t bc;           /* MPDATA_BC_PERIODIC or MPDATA_BC_OPEN (all axes) */
    int32_t iord;         /* 1: donor cell only; k = 2 .. 16: k - 1 corrective
                             passes (Smolarkiewicz 1984: pass j > 1 corrects
                             the result of pass j - 1 with the limited
                             velocity of pass j - 1 as its Courant numbers;
                             its limiter bounds run over psi^n and every
                             iterate of the step).  iord > 2 needs the
                             default launch shape (tile 0) and runs on
                             single-grid contexts only */
    int32_t nonos;        /* 1: non-oscillatory limiter on (needs iord >= 2) */
    int32_t tile;         /* launch shape: 0 = library default, else an id
                             from mpdata_tile_count()/mpdata_tile_info();
                             tile 7 (24x32 regions) is built for FP32 only */
    int32_t flags;        /* MPDATA_FLAG_* bits, 0 = defaults */
    int32_t reserved;     /* must be 0 */
    double eps;           /* >= 1e-30 and finite (MPDATA_EINVAL otherwise),
                             regularises the ratio denominators of the
                             pseudo-velocity and of the limiter; 1e-15 is the
                             usual value.  The floor keeps the common
                             denominators the kernels divide by (about
                             h eps^3 in FP64 on a zero background, and
                             (IN + eps)(OUT + eps) in the limiter) normal */
} mpdata_params;

typedef struct mpdata_ctx mpdata_ctx; /* opaque */

/* Bytes of workspace mpdata_create() needs for these parameters (0 if they
 * are invalid).  The workspace holds the second psi buffer of the time loop
 * and the mass-reduction partials; with iord > 2 also the intermediate
 * iterates, the limited velocities (face arrays) and, with the limiter, psi1
 * of the first pass and the running bounds of the middle passes (one set;
 * two from iord 4 on). */
size_t mpdata_workspace_bytes(const mpdata_params *p);

/* Validates the parameters and arrays and binds them to a new context.
 *   psi        device, read-write, nx*ny*nz elements: the state, updated in
 *              place by mpdata_step()
 *   u1,u2,u3,h device, read-only for the lifetime of the context
 *   workspace  device, >= mpdata_workspace_bytes(p) bytes, 256-byte aligned
 *   stream     hipStream_t of the caller (NULL = default stream)
 * Checks: dims >= 1, enum ranges, eps >= 1e-30, non-NULL 16-byte-aligned
 * pointers, h > 0 everywhere, and (periodic) face n == face 0 bit for bit
 * on every axis.  These checks read the arrays and synchronise the stream.
 * On success *out receives the context; on failure *out is set to NULL. */
int mpdata_create(const mpdata_params *p, void *psi, const void *u1, const void *u2,
                  const void *u3, const void *h, void *workspace, size_t ws_bytes,
                  void *stream, mpdata_ctx **out);

/* Enqueues nsteps >= 0 time steps.  On return of the enqueued work psi holds
 * the state after the steps (an odd step count ends with one device copy
 * from the workspace into psi).  Each step is one launch of the persistent
 * fused kernel over a plan of (tile, z-range) segments balanced across the
 * GPU (iord 2), or a chain of iord - 1 launches of it over the same plan
 * (iord > 2: the fused step, then one launch per further corrective pass).
 * Runs of 8 steps are replayed from a hipGraph built by mpdata_create
 * (unless MPDATA_FLAG_NO_GRAPH). */
int mpdata_step(mpdata_ctx *ctx, int32_t nsteps);

/* Time steps with Courant numbers that change in time (a context created
 * with MPDATA_FLAG_TVEL; MPDATA_ENOTSUP otherwise).  The velocity bound to
 * the context (u1, u2, u3 of mpdata_create, or the last level of the
 * previous call) is the level at the start of the first step; u1[s], u2[s],
 * u3[s] (host arrays of nsteps device pointers, each array laid out as at
 * mpdata_create) are the levels at the end of step s, so step s runs from
 * level s to level s + 1.  Every stage of a step uses the Courant numbers
 * of its start; holding them over the step leaves a first-order error, the
 * flux (1/2) dt (dU/dt) psi, which the first corrective pass takes back by
 * adding (U(end) - U(start)) / 2 to the antidiffusive pseudo-velocity of
 * every face (zero on the boundary-normal faces of an open domain).  This
 * is the time-dependent-flow correction of the generalised MPDATA of the
 * literature the paper cites (section 5.2 defers the scheme to it); with
 * equal levels it adds exact zeros.  Ownership: the caller keeps every level
 * alive until the steps that read it have run; afterwards the last level is
 * bound to the context (read by later steps, mpdata_step included, which
 * holds it over each step) until the next call.  Each level's periodic face
 * pairs are checked on the stream: a mismatch is reported by the next
 * mpdata_sync or mpdata_mass as MPDATA_EINVAL (the steps that used the level
 * have run).  An odd step count ends with one device copy into psi, as in
 * mpdata_step; the steps are launched one by one (no graph). */
int mpdata_step_tv(mpdata_ctx *ctx, int32_t nsteps, const void *const *u1, const void *const *u2,
                   const void *const *u3);

/* Mass M = sum over cells of h*psi with a compensated (double-double)
 * reduction: wave-level and block-level partials, then one deterministic
 * final pass.  Synchronises the stream; MPDATA_ENONFINITE if psi holds a
 * NaN or Inf. */
int mpdata_mass(mpdata_ctx *ctx, double *out);

/* The mass of mpdata_mass without a context and without any allocation,
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid it).  M = sum of
 * h[i]*psi[i] over n cells of the caller's device arrays psi and h (element
 * type by dtype: MPDATA_FP64 double, MPDATA_FP32 float), reduced by the same
 * kernels and block count as mpdata_mass (so the same bits for the same
 * arrays), asynchronously on stream; the result, one double, is written to
 * out_device (device memory of the caller) and may be NaN or Inf (no check:
 * nothing is synchronised).  The partials live in a fixed 16 KiB device
 * array of the library (one per GPU, held until the process ends), not in
 * a workspace: calls that overlap on one GPU (other streams, other threads)
 * share it and race; serialise them.  n from 0 to 2^31 - 1 (a grid's cell
 * limit); MPDATA_EINVAL for a bad dtype, a NULL pointer or n outside that
 * range, MPDATA_EDEVICE if a launch fails.  Calls no hipMalloc, hipFree or
 * allocating routine. */
int mpdata_mass_noalloc(int32_t dtype, const void *psi, const void *h, int64_t n,
                        double *out_device, void *stream);

/* Device-to-device copies of the state (asynchronous on the stream). */
int mpdata_get_psi(mpdata_ctx *ctx, void *dst_device);
int mpdata_set_psi(mpdata_ctx *ctx, const void *src_device);

/* Waits for all work enqueued by this context (MPDATA_EINVAL if a time level
 * given to mpdata_step_tv broke periodicity). */
int mpdata_sync(mpdata_ctx *ctx);

/* Number of time steps executed since creation (or the last set_psi). */
int64_t mpdata_steps_done(const mpdata_ctx *ctx);

/* Waits for the work enqueued by the context, then releases it (NULL-safe);
 * afterwards the caller may free the workspace and the arrays.  Never frees
 * caller memory. */
void mpdata_destroy(mpdata_ctx *ctx);

/* Message of the last failed call on ctx ("" if none); with ctx == NULL the
 * message of the last failed mpdata_create() on this thread. */
const char *mpdata_last_error(const mpdata_ctx *ctx);

/* Launch shapes of the fused step kernel.  Shape id 1..count; for each the
 * x-y output tile (tx, ty) and the threads per workgroup. */
int mpdata_tile_count(void);
int mpdata_tile_info(int32_t id, int32_t *tx, int32_t *ty, int32_t *threads);

/* The shape id that params.tile = 0 selects for (dtype, bc), or 0 if dtype
 * or bc is not one of the enum values. */
int32_t mpdata_default_tile(int32_t dtype, int32_t bc);

/* Resident workgroups of the step kernel for (dtype, tile, bc, nonos) on the
 * current device: *per_cu per compute unit, *cus compute units.
 * MPDATA_EINVAL for an unknown dtype or tile id, MPDATA_ENOTSUP when no step
 * kernel is built for that combination (tile 7 with FP64). */
int mpdata_occupancy(int32_t dtype, int32_t tile, int32_t bc, int32_t nonos, int32_t *per_cu,
                     int32_t *cus);

/* ------------------------------------------------------------------ batches
 * Many independent grids of uneven sizes advanced together: every step is
 * ONE launch of the persistent kernel whose workgroups walk a plan of
 * segments (grid, tile_x, tile_y, z0, z1) -- the x-y output tile
 * (tile_x, tile_y) of that grid over planes [z0, z1).  All grids of a batch
 * share dtype, bc, iord (must be 2), nonos and eps; their sizes differ.  The
 * plan decides which workgroup runs which segment (the per-CU assignment of
 * uneven blocks); it can come from the library (plan == NULL: an even split
 * of the work in planes) or from a caller-side tuner. */
typedef struct mpdata_batch mpdata_batch; /* opaque */

typedef struct {
    int32_t tile;            /* launch shape id, 1..mpdata_tile_count() */
    int32_t nwg;             /* workgroups of the persistent launch, >= 1 */
    int32_t nseg;            /* number of segments */
    int32_t seg_cols;        /* 0 or 5: seg rows are grid, tile_x, tile_y, z0, z1
                                (every grid in shape `tile`); 6: a sixth column
                                names the segment's shape, so that each grid
                                takes its own (per-size-class shapes in one
                                launch): tile 5 or 7 (32x24 and 24x32 regions,
                                768 threads each), the same for all segments of
                                a grid, FP32 periodic grids without VSIGN, DIV
                                or TVEL; `tile` is then 5 or 7 as well */
    const int32_t *seg;      /* host, nseg x seg_cols int32 */
    const int32_t *wg_begin; /* host, nwg + 1 int32: workgroup w runs segments
                                [wg_begin[w], wg_begin[w+1]) in order */
} mpdata_plan;

/* Workspace bytes for a batch of n grids whose plans hold at most
 * max_segments segments and max_wg workgroups (0 if the params are invalid
 * or not batchable). */
size_t mpdata_batch_workspace_bytes(int32_t n, const mpdata_params *params, int32_t max_segments,
                                    int32_t max_wg);

/* Segments and workgroups of the library's default plan for these grids and
 * launch shape (tile 0 = default shape) on the current device. */
int mpdata_batch_default_plan_size(int32_t n, const mpdata_params *params, int32_t tile,
                                   int32_t *nseg, int32_t *nwg);

/* Binds n >= 1 grids (params[i] and the device arrays psi[i], u1[i], u2[i],
 * u3[i], h[i], as for mpdata_create) and a plan (NULL = default).  A plan is
 * checked: every output tile of every grid covered exactly once over all
 * planes.  Synchronises the stream. */
int mpdata_batch_create(int32_t n, const mpdata_params *params, void *const *psi,
                        const void *const *u1, const void *const *u2, const void *const *u3,
                        const void *const *h, void *workspace, size_t ws_bytes, void *stream,
                        const mpdata_plan *plan, mpdata_batch **out);

/* nsteps >= 0 steps of every grid (asynchronous). */
int mpdata_batch_step(mpdata_batch *b, int32_t nsteps);

/* One step of every grid with the duration of each segment recorded:
 * cycles_out[s] receives the wall-clock ticks (100 MHz) segment s of the plan
 * took while all workgroups ran together.  Synchronises the stream. */
int mpdata_batch_profile_step(mpdata_batch *b, int64_t *cycles_out, int32_t nseg);

/* Mass of grid i (as mpdata_mass); synchronises the stream. */
int mpdata_batch_mass(mpdata_batch *b, int32_t i, double *out);

int mpdata_batch_sync(mpdata_batch *b);

/* -------------------------------------------------------------------- pools
 * A pool is a batch whose membership changes between calls: the serving
 * engine of continuous batching.  Grids join (mpdata_pool_add, validated
 * once) and leave (mpdata_pool_remove) at any time between steps; every
 * mpdata_pool_step advances all current members by the same number of
 * steps with one persistent launch per step over a plan rebuilt on the host
 * for the current members and uploaded asynchronously.  All members share
 * dtype, bc, nonos, eps and the launch shape given at creation (iord 2).
 * Each member brings its own second psi buffer (psi_scratch, same size as
 * psi); after every mpdata_pool_step a member's state is in its psi. */
typedef struct mpdata_pool mpdata_pool; /* opaque */

/* Workspace bytes of a pool with at most max_grids members whose plans hold
 * at most max_segments segments. */
size_t mpdata_pool_workspace_bytes(int32_t max_grids, int32_t max_segments);

/* shared: dtype, bc, nonos, eps, tile and flags of every member (its nx, ny,
 * nz, iord are ignored). */
int mpdata_pool_create(const mpdata_params *shared, int32_t max_grids, int32_t max_segments,
                       void *workspace, size_t ws_bytes, void *stream, mpdata_pool **out);

/* Adds a grid; the checks of mpdata_create run on validate_stream (the
 * stream the arrays were written on; NULL = the pool's stream), which is
 * synchronised.  *slot receives its id (>= 0). */
int mpdata_pool_add(mpdata_pool *pool, int32_t nx, int32_t ny, int32_t nz, void *psi,
                    void *psi_scratch, const void *u1, const void *u2, const void *u3,
                    const void *h, void *validate_stream, int32_t *slot);

/* Removes a member (its arrays are no longer referenced after the work
 * already enqueued on the pool's stream). */
int mpdata_pool_remove(mpdata_pool *pool, int32_t slot);

/* nsteps >= 0 steps of every member (asynchronous on the pool's stream). */
int mpdata_pool_step(mpdata_pool *pool, int32_t nsteps);

int32_t mpdata_pool_size(const mpdata_pool *pool);             /* current members */
int mpdata_pool_sync(mpdata_pool *pool);
void mpdata_pool_destroy(mpdata_pool *pool);                   /* NULL-safe */
const char *mpdata_pool_last_error(const mpdata_pool *pool);   /* NULL: last create */
void mpdata_batch_destroy(mpdata_batch *b);                 /* NULL-safe; waits for
                                                               the batch's work first */
const char *mpdata_batch_last_error(const mpdata_batch *b); /* NULL: last create */

/* -------------------------------------- model-based load imbalancing (host)
 * The paper's functional performance model (section 3) and its partitioning
 * algorithm (section 4, Algorithm 1) for p identical processors -- here the
 * XCDs of one GPU, each running a slab of planes of one grid.  speed[k] is
 * s(k*dx), the speed of one processor on a workload of k granules measured
 * while all processors run together (k = 0..nspeed-1; speed[0] unused; any
 * positive unit).  Host-only: no device is touched. */

/* Theorem 1's condition s(x)/x >= s(y)/y for all x < y over the table.
 * Returns the number of violating pairs (>= 0; 0 = the balanced split is
 * optimal), the first one in (*x_bad, *y_bad) as workloads (may be NULL),
 * or MPDATA_EINVAL for a bad table (nspeed < 2, dx < 1, a speed <= 0). */
int mpdata_fpm_check(const double *speed, int32_t nspeed, int32_t dx, int32_t *x_bad,
                     int32_t *y_bad);

/* Algorithm 1: workload n (multiple of p*dx), p even.  Starting from the even
 * share n/p, moves dx at a time from half of the processors to the other
 * half while the smaller share keeps at least dx, timing each split as
 * max(x_hi/s(x_hi), x_lo/s(x_lo)), and returns the first split of least
 * time: *x_lo for the odd-numbered processors, *x_hi for the even-numbered
 * ones, *t_min the predicted time (x unit / s unit).  The table must cover
 * every workload the moves reach (2n/p - dx); MPDATA_EINVAL otherwise. */
int mpdata_fpm_partition(const double *speed, int32_t nspeed, int32_t n, int32_t p, int32_t dx,
                         int32_t *x_lo, int32_t *x_hi, double *t_min);

/* Version of this ABI (MPDATA_ABI_VERSION). */
int mpdata_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* MPDATA_H */
