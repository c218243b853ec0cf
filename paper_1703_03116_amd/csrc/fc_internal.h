// fc_internal.h -- structures shared by the host runtime and the gfx950
// kernels of the AMR library.  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define FC_MAXLEV 24
#define FC_NREC 12   // neighbour records per patch: 4 faces x 2 halves + 4 corners

// Neighbour record types: what covers one ghost region of a patch.
enum { NB_NONE = 0, NB_SAME = 1, NB_COARSE = 2, NB_FINE = 3 };

// One ghost region (a face half or a corner) of a patch P at level l.
// type: bits 0-3 the NB_* kind, bits 4-7 the reflecting walls of the covering
// leaf (PatchInfo::walls of slot `id`; a coarse stencil folds at them), bits
// 8-10 the orientation code of the index transform A below (Sec. 2.3, eq.
// transform: bit 0 exchanges the two indices, bit 1 negates the first
// result, bit 2 the second; 0 between patches of one block).  A P-local
// index (i, j) (level-l cells, periodic images already unwrapped) maps into
// the covering leaf `id` (a store slot), in that leaf's own indices, as
//   SAME:   neighbour cell = A (i, j) + F
//   COARSE: level-l index inside the coarse leaf = A (i, j) + F; the coarse
//           cell is that >> 1, its parity selects d_k (in the coarse leaf's
//           indices)
//   FINE:   first of the four fine cells = 2 A (i, j) + F, the four at
//           + {0, 1} in each index (eq. ghost_coarse averages all four)
// with F = (fx, fy).
struct NbrRec {
    int32_t type, id, fx, fy;
};

// Per-patch geometry.  level, (ix, iy) in brick coordinates.  walls: bit 0
// x-lo, 1 x-hi, 2 y-lo, 3 y-hi are reflecting walls touching this patch (in
// its own indices); bits 8-10 the orientation code of the patch's block (its
// own index directions against the brick's, as in NbrRec).
struct PatchInfo {
    int32_t level, ix, iy, walls;
};

// Regrid transfer plan for one new slot.
enum { TR_COPY = 0, TR_REFINE = 1, TR_COARSEN = 2 };
struct TransferRec {
    int32_t kind, src[4], cx, cy, pad;
};

// One level-step of a coarse step: advance `level` (-1: every level, global
// stepping) from t_base + off * dt_coarse by scale * dt_coarse, its coarser
// neighbour level read at time fraction alpha.
struct SchedEntry {
    int32_t level, pad;
    double off, scale, alpha;
};

// Device-resident state used by the persistent kernel (graph replays read
// and update it, so replays need no host involvement).
// coarse steps per graph replay / persistent launch (at most)
constexpr int FC_TCHUNK = 50;

struct DevState {
    double t;                  // time all levels are synchronised at
    double dt_coarse;
    unsigned long long cfl_bits;  // max Courant number (bits of a non-negative double)
    uint32_t curmask;          // bit l: current buffer of level l
    uint32_t bar_count, bar_gen;
    int32_t err;               // bit 0: barrier spin limit hit; bit 1: stencil out of range;
                               // bit 2: graph did not cover a level; bit 3: NaN met by tagging;
                               // bit 4: Courant number above cfl_max
    int32_t pad;
    // ts[k]: the time after k further coarse steps, accumulated as the host
    // accumulates it (t += dt_coarse), k = 0 .. FC_TCHUNK
    double ts[FC_TCHUNK + 1];
};

// Everything a kernel needs to read or evaluate patch data.
struct Ctx {
    double *q0, *q1;           // the two patch buffers [F][cap][N][N]
    const PatchInfo *info;     // [cap]
    const NbrRec *nbr;         // [cap][FC_NREC]
    int32_t cap;               // slot stride inside a field plane
    int32_t F, eq, lim;
    uint32_t curmask;          // bit l: current buffer of level l
    int32_t clevel;            // level read time-interpolated (-1: none)
    double alpha;              // its time fraction (1: current state)
    // per level, velocity factor tables (see vt_* below), NULL if unused
    const double *vt[FC_MAXLEV];
    int32_t velocity;
    double vel_u, vel_v, vel_T, g;
    double vel_invT;           // 1 / T of the swirl field
    int32_t *err;              // device error flags
    // bit l: level l holds all 4^l quadrants (slots lstart[l] + Morton index)
    // and wraps periodically, so neighbour slots follow from the index
    uint32_t complete;
    int32_t lstart[FC_MAXLEV];
    unsigned long long *cflp;  // per-slot max Courant number (bits of a non-negative double) [cap];
                               // NULL: not recorded
    int32_t stream_out;        // advance output by streaming (nontemporal) stores
    // mapped grid (Sec. 1 metric terms): per level the capacity table K[k],
    // k = (I + J + 1) mod n, of cell (I, J) (n entries); all NULL on a
    // Cartesian grid
    const double *mk[FC_MAXLEV];
    int32_t mapped;
};

// Velocity factor tables of one level with n = mx 2^l cells per axis and m
// ghost layers, stored back to back (each indexed from -m):
//   ex[I] = sin^2(pi x_I),        x edges  I in [-m, n+m]      (n+2m+1)
//   cx[I] = sin(2 pi x_I) sigma,  x centres I in [-m, n+m)      (n+2m)
//   ey, cy the same along y.  sigma = sin(pi h)/(pi h).  Indices wrap where
// the axis is periodic.  Swirl: u(edge I, row J) = ex[I] cy[J] c(t),
// v(col I, edge J) = -ey[J] cx[I] c(t), c(t) = cos(pi t / T).
__host__ __device__ inline int64_t vt_size(int n, int m) { return 2 * (n + 2 * m + 1) + 2 * (n + 2 * m); }
__host__ __device__ inline int64_t vt_ex(int n, int m) { return m; }
__host__ __device__ inline int64_t vt_cx(int n, int m) { return (n + 2 * m + 1) + m; }
__host__ __device__ inline int64_t vt_ey(int n, int m) { return (n + 2 * m + 1) + (n + 2 * m) + m; }
__host__ __device__ inline int64_t vt_cy(int n, int m) { return 2 * (n + 2 * m + 1) + (n + 2 * m) + m; }

// Level ranges of the store (slots are grouped by level).
struct LevelRange {
    int32_t start[FC_MAXLEV], count[FC_MAXLEV];
};

// ---- kernel launchers (fc_kernels.hip) --------------------------------
struct LaunchCfg {
    int mx, nt;                // patch edge, threads per patch
    int seg;                   // scalar sweeps: cells per segment (0: the shortest that fits)
};

// Tile shapes of the scalar advance: the shortest segment that lets every
// interior line segment have its own thread, max(4, min(mx, 2 mx^2 / nt)),
// and, where the segments of a line still split into two halves, twice that
// (fewer, longer items: fewer edges computed twice, more threads left for
// the outer lines).  0 where there is no long variant.
inline int tile_default(int mx, int nt) {
    int sg = 2 * mx * mx / nt;
    if (sg < 4) sg = 4;
    if (sg > mx) sg = mx;
    return sg;
}
inline int tile_long(int mx, int nt) {
    const int sg = 2 * tile_default(mx, nt);
    return (mx / sg >= 2 && (mx / sg) % 2 == 0) ? sg : 0;
}

hipError_t launch_init_tables(int level, int mx, int periodic_x, int periodic_y, double *vt, hipStream_t s);
// capacity table of a mapped level with n cells per axis (alpha: the mapping's amplitude)
hipError_t launch_init_capacity(int n, double alpha, double *K, hipStream_t s);
// reset_cfl: also zero the n per-slot Courant maxima
hipError_t launch_set_state(DevState *st, double t, double dt, uint32_t curmask, int reset_cfl, unsigned long long *cflp, int n,
                            hipStream_t s);
hipError_t launch_zero_cfl(unsigned long long *cflp, int n, hipStream_t s);
hipError_t launch_fill(const Ctx &c, int mx, int first, int count, hipStream_t s);
hipError_t launch_advance(const Ctx &c, LaunchCfg lc, int level, int first, int count, double t, double dt,
                          int fused, hipStream_t s);
// ncoarse coarse steps in one launch (device-wide barrier between level-steps)
hipError_t launch_persistent(const Ctx &c, LaunchCfg lc, const SchedEntry *sched, int nsched,
                             const LevelRange *ranges_dev, int ncoarse, DevState *state, int grid,
                             hipStream_t s);
// eq: the kernel kind (0 scalar advection, 1 shallow water, 2 scalar
// advection on a mapped grid)
int persistent_max_grid(LaunchCfg lc, int eq);
// one level-step (schedule entry e over slots [first, first+count), coarse
// step cidx of a chunk of steps dt_coarse, buffer parities mask), ghosts
// gathered on the fly, one workgroup per patch
hipError_t launch_level_step(const Ctx &c, LaunchCfg lc, const SchedEntry &e, int first, int count, int cidx,
                             uint32_t mask, double dt_coarse, DevState *st, hipStream_t s);
// advance the device time by ncoarse coarse steps and flip the parities
hipError_t launch_finish_chunk(DevState *st, int ncoarse, uint32_t flip, hipStream_t s);
hipError_t launch_set_interior(const Ctx &c, int mx, const int32_t *slot_of_leaf, int n, const double *src,
                               hipStream_t s);
hipError_t launch_get_interior(const Ctx &c, int mx, const int32_t *slot_of_leaf, int n, double *dst,
                               int full, hipStream_t s);
hipError_t launch_tag(const Ctx &c, int mx, const int32_t *slot_of_leaf, int n, int lmin, int lmax,
                      double tau_r, double tau_c, int8_t *tags, double *g2, hipStream_t s);
hipError_t launch_consolidate(const Ctx &c, int mx, int n, hipStream_t s);
hipError_t launch_transfer(const Ctx &c, int mx, const TransferRec *plan, int n, hipStream_t s);
// *cfl_dev = max(*cfl_dev, device state's maximum, max of the n slots); with
// cfl_max > 0 a maximum above it raises bit 16 of *err
hipError_t launch_export_cfl(DevState *state, const unsigned long long *cflp, int n, double *cfl_dev, double cfl_max,
                             int32_t *err, hipStream_t s);
// restore == 0: save[leaf k in store order][F][mx][mx] <- the current
// interiors of slot k; restore == 1: the reverse
hipError_t launch_copy_interiors(const Ctx &c, int mx, int n, double *save, int restore, hipStream_t s);
hipError_t launch_step_leaf(const Ctx &c, int mx, int level, int first, int count, double t, double dt,
                            const int32_t *leaf_of_slot, const double *q_in, double *q_out, hipStream_t s);
// Adaptation on the device over a map of the finest level L (2^L x 2^L
// cells): owner map, per-slot target and neighbour maximum, the new levels
// painted into lev_a (launch_adapt_device); 2:1 balance passes from one map
// into the other (b starts as a copy of a; *changed raised when a leaf was
// refined); the leaves of a map as (level, ix, iy) triples (*count may
// exceed cap: only cap are written).
hipError_t launch_adapt_device(const Ctx &c, const int32_t *slot_of_leaf, const int8_t *tags, int nleaf, int L,
                               int periodic_x, int periodic_y, int lmin, int lmax, int smooth, int32_t *owner,
                               int32_t *target, int32_t *T, int8_t *lev_a, int8_t *lev_b, int32_t *flags,
                               hipStream_t s);
hipError_t launch_balance_pass(const int8_t *a, int8_t *b, int L, int periodic_x, int periodic_y, int lmin, int lmax,
                               int32_t *changed, hipStream_t s);
hipError_t launch_extract_leaves(const int8_t *a, int L, int cap, int32_t *count, int32_t *out, hipStream_t s);
hipError_t launch_adjoint(const Ctx &c, int mx, int level, int first, int count, double t, double dt, const int32_t *leaf_of_slot,
                          const double *q_in, const double *lam_in, double *lam_out, hipStream_t s);
