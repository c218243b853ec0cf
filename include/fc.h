/*
 * fc.h -- C ABI of the MI355X (gfx950) patch-based quadtree AMR library.
 *
 * The method is that of Calhoun & Burstedde, "ForestClaw: a parallel
 * algorithm for patch-based adaptive mesh refinement on a forest of
 * quadtrees" (arXiv:1703.03116): fixed mx x mx patches with m ghost layers
 * on the leaves of a 2:1 balanced quadtree (Sec. 2), ghost regions filled by
 * copying from same-size neighbours, averaging fine neighbours (eq.
 * ghost_coarse) and limited interpolation from coarse neighbours (eq.
 * ghost_fine) in the order of Algorithm 1 (Sec. 2.2), a single-grid
 * wave-propagation update per patch (Sec. 5), tagging and regridding
 * (Sec. 4.1) and multirate time stepping (the paper's time-stepping
 * section).
 *
 * Conventions for every entry point:
 *   - Return FC_OK (0) or a negative fc_status; no exception crosses the
 *     ABI.  fc_last_error() returns a message for the calling thread's last
 *     failure.
 *   - Errors detectable on the host (bad arguments, unbalanced mesh, ghost
 *     width, capacity, wrong state) are returned before anything is queued.
 *     Device faults surface as FC_ERR_HIP from the call that observes them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is queued on it and is asynchronous unless stated.
 *   - Pointers marked "device" must be device memory owned by the caller;
 *     the library never frees them.  Pointers marked "host" are read during
 *     the call only.
 *   - A store is not thread-safe; distinct stores are independent.
 *
 * Patch data layout in device memory (the "patch store"): two buffers of
 * nfields x capacity x N x N doubles, N = mx + 2 mbc, field-major (SoA),
 * x fastest; slot p holds the patch whose store index is p.  Stores are
 * ordered by level, then by Morton (Z-order) index inside a level (Sec. 2).
 * Which buffer holds the current state of a level alternates with each
 * advance of that level; fc_set_interior / fc_get_interior hide this.
 */
#ifndef FC_H
#define FC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fc_status;
enum {
    FC_OK = 0,
    FC_ERR_ARG = -1,          /* invalid argument                                   */
    FC_ERR_UNBALANCED = -2,   /* leaves not 2:1 balanced over faces and corners      */
    FC_ERR_GHOST_WIDTH = -3,  /* m > mx/4 or mx odd: Prop. 2.1 condition violated     */
    FC_ERR_HIP = -4,          /* a HIP runtime call failed                            */
    FC_ERR_CFL = -5,          /* a step's Courant number exceeded cfl_max             */
    FC_ERR_STATE = -6,        /* call out of order (e.g. not bound)                   */
    FC_ERR_CAPACITY = -7,     /* more leaves than the store's capacity                */
    FC_ERR_COVER = -8,        /* leaves overlap or do not tile the unit square        */
    FC_ERR_NONFINITE = -9     /* a patch holds a NaN (found by the tagging reduction) */
};

enum { FC_EQ_ADVECTION = 0, FC_EQ_SWE = 1 };
enum { FC_BC_PERIODIC = 0, FC_BC_REFLECT = 1 };
enum { FC_VEL_NONE = 0, FC_VEL_CONSTANT = 1, FC_VEL_SWIRL = 2 };
enum { FC_LIM_MC = 0, FC_LIM_LW = 1, FC_LIM_FIRST = 2, FC_LIM_MINMOD = 3 };
enum { FC_STEP_MULTIRATE = 0, FC_STEP_GLOBAL = 1 };
enum {
    FC_MODE_PER_LEVEL = 0,       /* fill launch + advance launch per level-step                    */
    FC_MODE_FUSED = 1,           /* one persistent kernel, device-wide barriers between level-steps */
    FC_MODE_FUSED_GRAPH = 2,     /* one ghost-gathering kernel per level-step, replayed as a graph  */
    FC_MODE_FUSED_LEVELS = 3,    /* the same kernels launched one by one from the host             */
    FC_MODE_PERSISTENT_GRAPH = 4 /* the persistent kernel replayed as a graph                      */
};

/* A quadrant: on one unit-square block 0 <= ix, iy < 2^level.  On a brick of
 * nbx x nby blocks (fc_patchstore_create_brick) 0 <= ix < nbx 2^level,
 * 0 <= iy < nby 2^level: block (ix >> level, iy >> level), the low bits the
 * quadrant's coordinates in that block's own indices. */
typedef struct { int32_t level, ix, iy; } fc_leaf;

typedef struct {
    int32_t mx;            /* interior cells per patch edge: 8, 16 or 32            */
    int32_t mbc;           /* ghost layers m; the scheme needs 2; Prop. 2.1: m<=mx/4 */
    int32_t equation;      /* FC_EQ_ADVECTION (1 field) or FC_EQ_SWE (h, hu, hv)     */
    int32_t limiter;       /* FC_LIM_*                                               */
    int32_t bc[4];         /* x-lo, x-hi, y-lo, y-hi: FC_BC_PERIODIC | FC_BC_REFLECT */
    int32_t velocity;      /* advection: FC_VEL_CONSTANT (u,v) | FC_VEL_SWIRL (T)    */
    double vel_params[3];  /* constant: (u, v, -); swirl: (T, -, -)                  */
    double gravity;        /* shallow water g                                        */
    int32_t min_level;     /* coarsest level of the multirate recursion              */
    int32_t max_level;     /* finest level allowed (regridding caps refinement here) */
    int32_t time_stepping; /* FC_STEP_MULTIRATE | FC_STEP_GLOBAL                     */
    int32_t reserved;
    int64_t capacity;      /* patch slots; >= number of leaves; regrid up to this    */
    double cfl_max;        /* > 0: largest Courant number a step may reach (a
                              larger one is an error, or a rejected step in
                              fc_advance_adaptive); 0: not checked              */
    double map_alpha;      /* mapped grid (Sec. 1 metric terms, Sec. 5.2 runs
                              one): the physical cell of computational point
                              (xi, eta) is the image of
                              X = (xi, eta) + alpha sin(2 pi xi) sin(2 pi eta) (1, 1),
                              |alpha| < 1/(2 pi); 0: Cartesian.  Non-zero needs
                              one periodic block and scalar advection; steps
                              then take the capacity form (cell areas kappa h^2)
                              in every execution form, and averages from fine
                              to coarse cells are area-weighted              */
} fc_config;

typedef struct fc_patchstore fc_patchstore;

/* Last error message of the calling thread ("" if none).  Static storage. */
const char *fc_last_error(void);

/* Create a store for a leaf set (host array, any order).  Validates: leaves
 * in range, tiling of the unit square, 2:1 balance over faces and corners
 * with periodic wrap where periodic (Sec. 2), mbc >= 2 and 4 mbc <= mx (Prop.
 * 2.1), nleaves <= capacity.  perm_out (host, may be NULL) receives, for
 * each input leaf k, its store index.  Host memory only is allocated. */
fc_status fc_patchstore_create(const fc_config *cfg, int64_t nleaves, const fc_leaf *leaves,
                               fc_patchstore **out, int64_t *perm_out);

/* The same on a multiblock brick (Sec. 2.3): an nbx x nby arrangement of
 * unit blocks, each a quadtree with its own index orientation.  orient
 * (host, nbx * nby codes, block (bx, by) at bx + nbx by; NULL: all 0) gives
 * each block's index directions against the brick's: bit 0 exchanges the
 * two, then bit 1 reverses the brick's first direction and bit 2 its second
 * (the eight index transforms of eq. transform, A diagonal or anti-diagonal
 * with entries +-1).  Leaves are in the blocks' own coordinates (fc_leaf);
 * patch data is stored and exchanged in each block's own index directions,
 * and every ghost copy, eq. ghost_coarse average and eq. ghost_fine
 * interpolation across a block boundary goes through the index transform
 * between the two patches.  Tiling and 2:1 balance are checked in the
 * brick's geometry, across block boundaries.  A brick other than one block
 * of code 0 needs periodic sides and scalar advection at a constant
 * velocity (vel_params in the brick's directions); fc_adapt_device,
 * fc_step_uniform and fc_adjoint_step take one block of code 0 only
 * (FC_ERR_ARG).  Errors: FC_ERR_ARG for nbx or nby < 1, nbx nby > 65536, a
 * code outside 0..7 or the above; the rest as fc_patchstore_create. */
fc_status fc_patchstore_create_brick(const fc_config *cfg, int32_t nbx, int32_t nby, const int32_t *orient,
                                     int64_t nleaves, const fc_leaf *leaves, fc_patchstore **out,
                                     int64_t *perm_out);
fc_status fc_patchstore_destroy(fc_patchstore *ps);

/* Sizes of the caller-owned device memory: q_doubles = doubles per patch
 * buffer (nfields * capacity * N * N; two such buffers are needed) and
 * ws_bytes = workspace bytes (metadata, velocity tables, schedule, state;
 * with cfl_max > 0 also room to keep one copy of the interiors, for
 * rejected steps). */
fc_status fc_patchstore_sizes(const fc_patchstore *ps, int64_t *q_doubles, int64_t *ws_bytes);

/* Bind caller-owned device memory (q0, q1: q_doubles each; workspace:
 * ws_bytes, 256-byte aligned) and upload the metadata on `stream`.  The
 * memory is borrowed until destroy or the next bind. */
fc_status fc_patchstore_bind(fc_patchstore *ps, double *q0, double *q1, void *workspace, void *stream);

/* Number of leaves, the store's leaves in store order (host array of
 * nleaves), and the levels' current times. */
fc_status fc_patchstore_info(const fc_patchstore *ps, int64_t *nleaves, int32_t *min_level,
                             int32_t *max_level);
fc_status fc_patchstore_leaves(const fc_patchstore *ps, fc_leaf *out);

/* The neighbour records the ghost-gathering kernels read (host copy, for
 * checks on the host): out[nleaves][12][4] int32 in store order, per patch
 * the face halves W, W, E, E, S, S, N, N (lower half first) and the corners
 * SW, SE, NW, NE, each (type, slot, fx, fy).  type bits 0-3: 0 none (a
 * wall), 1 same size, 2 coarse, 3 fine; bits 4-7 the reflecting walls of
 * the neighbour; bits 8-10 the orientation code of the index transform A
 * (bit 0 exchanges i and j, bit 1 negates the first result, bit 2 the
 * second).  A ghost cell (i, j) of the patch maps into neighbour `slot`'s
 * own indices as A (i, j) + F (same size: its cell; coarse: the level-l
 * index inside it, halved for the coarse cell, the parity giving d_k), or
 * 2 A (i, j) + F (fine: the first of four cells at +{0,1}^2), F = (fx, fy)
 * (Sec. 2.3, eq. transform). */
fc_status fc_patchstore_records(const fc_patchstore *ps, int32_t *out);

/* Interior data in input-leaf order, device arrays [nleaves][nfields][mx][mx]
 * (the order of the leaves passed to create or to the last regrid). */
fc_status fc_set_interior(fc_patchstore *ps, const double *src, void *stream);
fc_status fc_get_interior(fc_patchstore *ps, double *dst, void *stream);
/* Whole current patch arrays including ghosts, [nleaves][nfields][N][N]. */
fc_status fc_get_patches(fc_patchstore *ps, double *dst, void *stream);

/* Ghost filling (Algorithm 1): fill every ghost cell of the patches with
 * level in [level_lo, level_hi] in the current buffers.  Levels >= level_lo
 * are synchronised; level_lo - 1 is read at time fraction `alpha` of its
 * last step: alpha == 1 reads its current state, otherwise
 * q_old + alpha (q - q_old) (multirate time interpolation).  Copy from
 * same-size neighbours and eq. ghost_coarse averaging from finer ones read
 * interiors only; eq. ghost_fine interpolation from a coarser neighbour
 * uses a minmod-limited one-sided gradient over the coarse 5-point stencil,
 * whose ghost values are themselves evaluated by copy/averaging; reflecting
 * walls mirror the data (negating the normal momentum), periodic sides
 * wrap.  Exact parity with the four phases of Algorithm 1. */
fc_status fc_ghost_fill(fc_patchstore *ps, int32_t level_lo, int32_t level_hi, double alpha,
                        void *stream);

/* One step of the unsplit wave-propagation scheme (Riemann fluctuations,
 * limited second-order correction, transverse propagation, conservative
 * update) on every patch of `level`, from time t by dt.  The ghosts of that
 * level must be valid (fc_ghost_fill).  The level's current buffer flips;
 * the previous state stays readable as q_old.  cfl_dev (device double, may
 * be NULL) is max-accumulated with the step's Courant number. */
fc_status fc_advance_level(fc_patchstore *ps, int32_t level, double t, double dt, double *cfl_dev,
                           void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * step as fc_advance_level, bitwise, whose per-patch Courant maxima (the
 * partial results reduced into *cfl_dev) live in a fixed device array of the
 * library instead of the store's workspace.  The call allocates nothing and
 * issues kernel launches only.  Limit: stores of at most 65536 slots
 * (capacity; FC_ERR_CAPACITY otherwise, before anything is queued); the
 * array holds 512 KiB on every GPU the library runs on, until the process
 * ends.  All calls on one GPU share that GPU's array: calls that overlap on
 * one GPU (other streams, other threads) race; each call clears the slots it
 * reduces over.  Other errors as fc_advance_level. */
fc_status fc_advance_level_noalloc(fc_patchstore *ps, int32_t level, double t, double dt, double *cfl_dev,
                                   void *stream);

/* As above; with cfl_max > 0 in the configuration and cfl_dev given, a
 * Courant number above cfl_max is recorded on the device and reported as
 * FC_ERR_CFL by fc_check_device.
 *
 * One coarse step of the configured time stepping, from the store's time t
 * by dt_coarse (multirate: level l takes 2^(l-min_level) steps of
 * dt_coarse / 2^(l-min_level); global: every level one step of dt_coarse).
 * mode FC_MODE_PER_LEVEL: a fill launch and an advance launch per
 * level-step; FC_MODE_FUSED: one persistent kernel per chunk of up to 50
 * coarse steps that evaluates ghosts on the fly and walks all level-steps
 * with device-wide barriers; FC_MODE_PERSISTENT_GRAPH: that kernel replayed
 * from a captured hipGraph; FC_MODE_FUSED_GRAPH: one ghost-gathering advance
 * kernel per level-step (no fill launch), a chunk of up to 50 coarse steps
 * captured once as a hipGraph and replayed (time, step and buffer parities
 * live in device memory); FC_MODE_FUSED_LEVELS: those kernels launched one
 * by one from the host.  All modes compute bitwise the same result.
 * nsteps coarse steps are taken.  cfl_dev as above.  The store's time
 * advances by nsteps * dt_coarse. */
fc_status fc_advance_coarse_steps(fc_patchstore *ps, double dt_coarse, int32_t nsteps, int32_t mode,
                                  double *cfl_dev, void *stream);
/* Advance the store to time t_end with a coarse step chosen from the
 * measured Courant number, as Clawpack does (the time step the paper's
 * solver library takes; Sec. 5 runs Clawpack): each coarse step is tried
 * with dt = *dt_inout (the last one shortened to land on t_end); if its
 * Courant number (the maximum over every level-step of the coarse step, the
 * same value cfl_dev receives above) exceeds cfl_max the step is rejected:
 * the interiors are restored from a copy taken before it, and it is tried
 * again with dt * cfl_target / CFL (dt / 2 if the Courant number is not a
 * finite number: the try blew up).  After an accepted step the next try is
 * dt * cfl_target / CFL.  The store's time ends at exactly t_end.
 * *dt_inout receives the next proposed coarse step; steps_out / rejected_out
 * (may be NULL) the accepted and rejected coarse steps.  Synchronises
 * `stream` once per coarse step (the Courant number decides on the host).
 * Needs cfl_max > 0 at create (FC_ERR_STATE otherwise); FC_ERR_ARG for
 * dt <= 0, cfl_target outside (0, cfl_max] or max_steps < 1; FC_ERR_CFL when
 * one step is rejected eight times in a row; stops after max_steps accepted
 * steps (check the time). */
fc_status fc_advance_adaptive(fc_patchstore *ps, double t_end, double cfl_target, int32_t mode,
                              double *dt_inout, int32_t max_steps, int32_t *steps_out,
                              int32_t *rejected_out, void *stream);

/* Set-up for the graph modes: capture and instantiate, without running them,
 * the graphs that a call fc_advance_coarse_steps(ps, dt_coarse, nsteps,
 * mode) made next (from the store's current parities) replays, so that the
 * one-time capture cost stays out of that call.  The schedule captured is
 * the multirate recursion of the time-stepping section.  A no-op for the
 * other modes.  FC_ERR_ARG for dt_coarse <= 0, nsteps < 0 or an unknown
 * mode.  Allocates nothing on the device beyond the graphs themselves. */
fc_status fc_prepare_steps(fc_patchstore *ps, double dt_coarse, int32_t nsteps, int32_t mode, void *stream);
/* Store time (host value of the time all levels are synchronised at). */
fc_status fc_get_time(const fc_patchstore *ps, double *t);
fc_status fc_set_time(fc_patchstore *ps, double t);

/* Tagging (Sec. 4.1): per patch, in input-leaf order, g = max over interior
 * cells of |grad q| (central differences of field 0 divided by 2h; ghosts
 * must be valid).  tags_dev[k] = +1 if g > tau_refine and level < max_level,
 * -1 if g <= tau_coarsen and level > min_level, else 0.  gmax2_dev (may be
 * NULL) receives g^2.  Device arrays of nleaves entries.  The reduction
 * carries NaN through: a patch whose gradient is NaN gets g^2 = NaN and tag
 * 0, and fc_check_device then reports FC_ERR_NONFINITE. */
fc_status fc_tag_refine(fc_patchstore *ps, double tau_refine, double tau_coarsen, int8_t *tags_dev,
                        double *gmax2_dev, void *stream);

/* Adaptation on the host (Sec. 4.1): from tags in input-leaf order (host
 * array; +1 refine, -1 coarsen, 0 keep) every leaf gets a target level, its
 * level plus its tag within [min_level, max_level].  With smooth != 0 that
 * target is raised to the largest target of the leaves touching it across a
 * face or a corner (smooth refinement, Sec. 4.2: a buffer of refined patches
 * around the finest ones).  A leaf whose target is above its level is
 * refined once; a family of four sibling leaves whose targets are all below
 * their level is replaced by its parent; then leaves are refined until 2:1
 * balanced.  Writes the new leaves sorted by (level, iy, ix) into out (host,
 * room for cap leaves; FC_ERR_CAPACITY otherwise) and their count into n_out. */
fc_status fc_adapt(const fc_patchstore *ps, const int8_t *tags, int32_t smooth, fc_leaf *out, int64_t cap,
                   int64_t *n_out);
/* The same adaptation on the device, from tags_dev (device array in
 * input-leaf order, as fc_tag_refine writes it): the leaves are painted on a
 * map of the finest level (4^max_level cells, in the workspace), targets,
 * their neighbourhood maxima, refinement, coarsening and 2:1 balance passes
 * run there, and only the new leaf list comes back to the host (out, sorted
 * as fc_adapt sorts it; the same leaves bit for bit).  Synchronises `stream`
 * once per balance pass.  Needs max_level <= 10 (FC_ERR_ARG otherwise);
 * FC_ERR_CAPACITY if the new set exceeds the store's capacity or cap. */
fc_status fc_adapt_device(fc_patchstore *ps, const int8_t *tags_dev, int32_t smooth, fc_leaf *out,
                          int64_t cap, int64_t *n_out, void *stream);

/* Regrid (Sec. 4.1): replace the leaf set by new_leaves (host) and transfer
 * the solution: unchanged leaves are copied, children are interpolated from
 * their parent with the ghost-fill interpolation (fill ghosts first),
 * parents are the mean of their four children.  All levels must be
 * synchronised.  Afterwards "input-leaf order" is the order of new_leaves.
 * A leaf set that is not a valid 2:1 tiling, or has a leaf that is neither
 * an old leaf, a child of one nor the parent of four, is rejected before
 * anything changes (the store stays as it was). */
fc_status fc_regrid(fc_patchstore *ps, int64_t nleaves, const fc_leaf *new_leaves, void *stream);

/* One step of the unsplit scheme (the same step as fc_advance_level after
 * a same-size fill, bitwise) on a uniform periodic level of scalar
 * advection, from q_in to q_out: device arrays [nleaves][1][mx][mx] in
 * input-leaf order, 16-byte aligned, q_out != q_in (FC_ERR_ARG otherwise,
 * also for a non-uniform mesh, other equations or non-periodic sides).  The
 * store's solution and time are left as they were; the step starts at t.
 * This is the form the adjoint's recomputation walks through. */
fc_status fc_step_uniform(fc_patchstore *ps, int32_t level, double t, double dt, const double *q_in,
                          double *q_out, void *stream);

/* Adjoint of one uniform-level scalar step (fill by same-size copy, then
 * advance): lambda_out = (J_adv J_fill)^T lambda_in with the limiter
 * branches frozen at the step's input state q_in.  q_in, lambda_in,
 * lambda_out: device arrays [nleaves][1][mx][mx] in input-leaf order,
 * 16-byte aligned.  Needs a uniform level and periodic boundaries
 * (FC_ERR_ARG otherwise).  lambda_out must not be lambda_in or q_in
 * (FC_ERR_ARG).  The store's solution is left as it was. */
fc_status fc_adjoint_step(fc_patchstore *ps, int32_t level, double t, double dt, const double *q_in,
                          const double *lambda_in, double *lambda_out, void *stream);

/* Synchronise `stream` and report device-side errors raised since bind:
 * a device-wide barrier that timed out (FC_ERR_HIP), an interpolation
 * stencil that needed a third level (FC_ERR_HIP; excluded by Prop. 2.1), a
 * Courant number above cfl_max (FC_ERR_CFL), a NaN met by the tagging
 * reduction (FC_ERR_NONFINITE).  The flags stay raised until the next bind. */
fc_status fc_check_device(fc_patchstore *ps, void *stream);

/* Choose the launch configuration of the advance kernels by timing every
 * variant on the bound store (results are bitwise equal): threads (waves) per
 * patch and, for scalar advection on a Cartesian grid, the tile shape of the
 * edge sweeps (fc_set_tile).  A variant other than the default (scalar
 * advection, also on a mapped grid: 64 threads at mx = 8, else 256, shortest
 * segments; shallow water: 192 at mx = 8, 512 at mx = 16) is taken only if it
 * is at least 5% faster (best of three interleaved timing rounds).  Returns
 * the chosen threads per patch (fc_get_launch gives both). */
fc_status fc_autotune(fc_patchstore *ps, int32_t *threads_out, void *stream);
/* Set the threads per patch directly.  Scalar advection: 64 or 128 at
 * mx = 8; 64, 128 or 256 at mx = 16; 128, 256 or 512 at mx = 32.  Shallow
 * water: 64, 128 or 192 at mx = 8; 256, 384, 512 or 640 at mx = 16 (a
 * mapped grid: those of scalar advection).  FC_ERR_ARG otherwise.  Resets the
 * tile shape to the default.  Drops captured graphs.  Whatever the variant,
 * FC_MODE_FUSED_GRAPH steps a level of scalar advection on 32x32 Cartesian
 * patches that is not complete and holds at most four patches per CU with
 * 512 threads per patch (one round of workgroups, so one workgroup's latency
 * decides; the same bits). */
fc_status fc_set_variant(fc_patchstore *ps, int32_t threads_per_patch);
/* Tile shape of the scalar edge sweeps (Cartesian grid): every interior
 * line is cut into segments of seg_cells cells, one per work item.  0 (or
 * the default) = the shortest that gives every segment its own thread,
 * max(4, min(mx, 2 mx^2 / threads)); the other choice is twice that, where a
 * line still splits into an even number of segments (mx = 16 at 128 or 256
 * threads: 8; mx = 32 at 256: 16, at 512: 8).  FC_ERR_ARG otherwise (and for
 * shallow water and mapped grids, which have one tile shape).  Drops
 * captured graphs. */
fc_status fc_set_tile(fc_patchstore *ps, int32_t seg_cells);
/* The current launch configuration: threads per patch and cells per sweep
 * segment (either may be NULL). */
fc_status fc_get_launch(const fc_patchstore *ps, int32_t *threads_per_patch, int32_t *seg_cells);
/* Workgroups of the persistent kernel: 0 = as many as can be co-resident
 * (occupancy x compute units), else min(grid, that).  max_grid (may be
 * NULL) receives the co-resident maximum. */
fc_status fc_set_persistent_grid(fc_patchstore *ps, int32_t grid, int32_t *max_grid);

#ifdef __cplusplus
}
#endif
#endif /* FC_H */
