/*
 * fc_oracle.c -- plain, slow, FP64 CPU oracle for the quadtree-AMR
 * advance + ghost-fill path of Calhoun & Burstedde, "ForestClaw: a parallel
 * algorithm for patch-based adaptive mesh refinement on a forest of
 * quadtrees" (arXiv:1703.03116).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * code, header, table or helper with the GPU library; it is built with
 * -O2 -ffp-contract=off (no fused multiply-add, no fast-math).
 *
 * What it computes, and where each rule comes from:
 *   - leaves on one unit-square block, or on a brick of unit blocks each
 *     with its own index orientation (Sec. 2.3, multiblock), 2:1 balance
 *     over faces and corners across block boundaries too (Sec. 2, quadtree
 *     layout), fixed mx x mx patches with m ghost layers stored as one
 *     contiguous array per patch in the block's own indices (Sec. 2);
 *   - ghost filling in the four phases of Algorithm 1 (Sec. 2.2): copy from
 *     same-size neighbours and averaging of fine interiors (eq. ghost_coarse,
 *     Sec. 2.3), physical boundary conditions, coarse->fine interpolation
 *     with a limited one-sided gradient (eq. ghost_fine, Sec. 2.3), boundary
 *     conditions again.  Neighbours are found by GEOMETRIC POINT LOCATION of
 *     each ghost-cell centre in a hash map of leaves -- no neighbour tables;
 *     on a brick every index goes through the brick's indices into the
 *     neighbour's own (the index transforms of Sec. 2.3).
 *   - the single-grid update: the unsplit wave-propagation scheme the paper
 *     runs through Clawpack (Sec. 5, cited, not written out in the paper):
 *     Riemann fluctuations, MC-limited second-order correction, transverse
 *     propagation of the corrected fluctuations, conservative update.
 *     Scalar advection with edge velocities from a stream function (Sec. 5.1
 *     defines the velocity through a stream function) and the shallow-water
 *     system with a Roe solver and Harten-Hyman entropy fix.
 *   - multirate subcycling (coarse-first recursion, time-interpolated coarse
 *     data) and global stepping (the commented-out time-stepping section of
 *     the paper describes both; only global stepping is demonstrated).
 *   - tagging, adaptation with 2:1 balance, and solution transfer
 *     (Sec. 4.1: children interpolated with the ghost-fill interpolation,
 *     parents averaged from four siblings).
 *   - the tangent step (limiter branches frozen) and its hand-written
 *     transpose for the scalar scheme, plus the ghost-copy transpose.
 *
 * Readings of points the paper leaves open are listed next to the code that
 * takes them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { EQ_ADV = 0, EQ_SWE = 1 };
enum { BC_PERIODIC = 0, BC_REFLECT = 1 };
enum { VEL_NONE = 0, VEL_CONST = 1, VEL_SWIRL = 2 };
enum { LIM_MC = 0, LIM_LW = 1, LIM_FIRST = 2, LIM_MINMOD = 3 };
enum { ERR_STENCIL = 1, ERR_UNBALANCED = 2, ERR_COVER = 4, ERR_WIDTH = 8, ERR_ARG = 16 };

typedef struct { int level, ix, iy; } OLeaf;

typedef struct Orc {
    int mx, m, N, F, eq, lim, bc[4], vel;
    double vp[3], g;
    int lmin, lmax;
    int n;
    OLeaf *lv;      /* leaves as given: block from the high bits, own indices of the block below */
    /* multiblock brick (Sec. 2.3): nbx x nby unit blocks, ori[bx + nbx by]
     * the index orientation of each block; ph[k] is leaf k in brick
     * coordinates (the point-location key) */
    int nbx, nby;
    int *ori;
    OLeaf *ph;
    double *q, *qold, *qhat;
    int hcap;
    int *hidx;
    int err;
    /* mapped grid (0: Cartesian): the computational square mapped by
     * X(xi, eta) = (xi, eta) + alpha sin(2 pi xi) sin(2 pi eta) (1, 1) */
    double map_alpha;
    /* tangent/adjoint support (scalar only): frozen forward state */
} Orc;

/* ------------------------------------------------------------------ */
/* leaf hash map: (level, ix, iy) -> leaf index                         */
/* ------------------------------------------------------------------ */
static uint64_t hkey(int l, int ix, int iy) {
    uint64_t k = ((uint64_t)(uint32_t)l << 48) ^ ((uint64_t)(uint32_t)iy << 24) ^ (uint64_t)(uint32_t)ix;
    k ^= k >> 33; k *= 0xff51afd7ed558ccdULL; k ^= k >> 33; k *= 0xc4ceb9fe1a85ec53ULL; k ^= k >> 33;
    return k;
}

/* ------------------------------------------------------------------ */
/* multiblock brick: index orientations (Sec. 2.3)                      */
/* ------------------------------------------------------------------ */
/* A block's own indices (a, b), n cells (or quadrants) per block side,
 * against the brick's indices inside that block: code bit 0 exchanges the
 * two directions, then bit 1 reverses the brick's first direction and bit 2
 * its second.  Each map has the form of eq. transform, A diagonal or
 * anti-diagonal with entries +-1, and is used unchanged for indices outside
 * [0, n) (ghost cells). */
static void own_to_brick(int code, int n, int a, int b, int *x, int *y) {
    int p = (code & 1) ? b : a, q = (code & 1) ? a : b;
    *x = (code & 2) ? n - 1 - p : p;
    *y = (code & 4) ? n - 1 - q : q;
}
static void brick_to_own(int code, int n, int x, int y, int *a, int *b) {
    int p = (code & 2) ? n - 1 - x : x, q = (code & 4) ? n - 1 - y : y;
    *a = (code & 1) ? q : p;
    *b = (code & 1) ? p : q;
}
static int block_code(const Orc *o, int bx, int by) {
    if (!o->ori || bx < 0 || by < 0 || bx >= o->nbx || by >= o->nby) return 0;
    return o->ori[bx + o->nbx * by];
}
static int leaf_code(const Orc *o, int k) {
    const OLeaf *L = &o->lv[k];
    return block_code(o, L->ix >> L->level, L->iy >> L->level);
}
static int is_brick(const Orc *o) {
    if (o->nbx != 1 || o->nby != 1) return 1;
    return o->ori && o->ori[0] != 0;
}

/* brick coordinates of the level-l quadrant with block-own coordinates (ix, iy) */
static OLeaf quad_to_brick(const Orc *o, int l, int ix, int iy) {
    int bx = ix >> l, by = iy >> l, n = 1 << l, x, y;
    own_to_brick(block_code(o, bx, by), n, ix - bx * n, iy - by * n, &x, &y);
    OLeaf r = {l, bx * n + x, by * n + y};
    return r;
}

/* Brick index (X, Y) of the level-r cell (i, j) of leaf k, counted from the
 * leaf's first cell in the leaf's own indices (r >= the leaf's level; (i, j)
 * may lie outside the leaf).  No periodic wrap. */
static void cell_to_brick(const Orc *o, int k, int r, int i, int j, int *X, int *Y) {
    const OLeaf *L = &o->lv[k];
    int l = L->level, sc = o->mx << (r - l), n = o->mx << r;
    int bx = L->ix >> l, by = L->iy >> l, x, y;
    own_to_brick(block_code(o, bx, by), n, (L->ix - (bx << l)) * sc + i, (L->iy - (by << l)) * sc + j, &x, &y);
    *X = bx * n + x;
    *Y = by * n + y;
}
/* The inverse: leaf k's own index of the level-r cell at brick index (X, Y)
 * (a cell of k's block). */
static void brick_to_cell(const Orc *o, int k, int r, int X, int Y, int *i, int *j) {
    const OLeaf *L = &o->lv[k];
    int l = L->level, sc = o->mx << (r - l), n = o->mx << r;
    int bx = L->ix >> l, by = L->iy >> l, a, b;
    brick_to_own(block_code(o, bx, by), n, X - bx * n, Y - by * n, &a, &b);
    *i = a - (L->ix - (bx << l)) * sc;
    *j = b - (L->iy - (by << l)) * sc;
}

/* the hash map is keyed by brick coordinates */
static void hash_build(Orc *o) {
    int cap = 16;
    while (cap < 4 * o->n) cap <<= 1;
    o->hcap = cap;
    free(o->hidx);
    o->hidx = (int *)malloc(sizeof(int) * cap);
    for (int i = 0; i < cap; i++) o->hidx[i] = -1;
    for (int k = 0; k < o->n; k++) {
        uint64_t h = hkey(o->ph[k].level, o->ph[k].ix, o->ph[k].iy) & (uint64_t)(cap - 1);
        while (o->hidx[h] >= 0) h = (h + 1) & (uint64_t)(cap - 1);
        o->hidx[h] = k;
    }
}

/* brick coordinates of every leaf, then the hash map */
static void index_leaves(Orc *o) {
    free(o->ph);
    o->ph = (OLeaf *)malloc(sizeof(OLeaf) * (o->n > 0 ? o->n : 1));
    for (int k = 0; k < o->n; k++) o->ph[k] = quad_to_brick(o, o->lv[k].level, o->lv[k].ix, o->lv[k].iy);
    hash_build(o);
}

/* leaf at brick coordinates (l, ix, iy), -1 if none */
static int find_leaf(const Orc *o, int l, int ix, int iy) {
    if (l < 0) return -1;
    if (ix < 0 || iy < 0 || ix >= (o->nbx << l) || iy >= (o->nby << l)) return -1;
    uint64_t h = hkey(l, ix, iy) & (uint64_t)(o->hcap - 1);
    while (o->hidx[h] >= 0) {
        const OLeaf *L = &o->ph[o->hidx[h]];
        if (L->level == l && L->ix == ix && L->iy == iy) return o->hidx[h];
        h = (h + 1) & (uint64_t)(o->hcap - 1);
    }
    return -1;
}

/* leaf at block-own coordinates (l, ix, iy) (parents, children and siblings
 * share their block and so their indices), -1 if none */
static int find_local(const Orc *o, int l, int ix, int iy) {
    if (l < 0 || ix < 0 || iy < 0 || ix >= (o->nbx << l) || iy >= (o->nby << l)) return -1;
    OLeaf b = quad_to_brick(o, l, ix, iy);
    return find_leaf(o, b.level, b.ix, b.iy);
}

/* Leaf containing the centre of level-l cell (I, J), I, J inside [0, mx 2^l).
 * 2:1 balance means it is the level-l quadrant itself, its parent, or one of
 * its children.  Returns the leaf index, -1 if none. */
static int locate(const Orc *o, int l, int I, int J) {
    int qx = I / o->mx, qy = J / o->mx;
    int k = find_leaf(o, l, qx, qy);
    if (k >= 0) return k;
    k = find_leaf(o, l - 1, qx >> 1, qy >> 1);
    if (k >= 0) return k;
    return find_leaf(o, l + 1, (2 * I) / o->mx, (2 * J) / o->mx);
}

/* ------------------------------------------------------------------ */
/* patch storage                                                        */
/* ------------------------------------------------------------------ */
static inline double *pat(const Orc *o, double *base, int k) {
    return base + (size_t)k * o->F * o->N * o->N;
}
/* field f, local cell (i, j) with -m <= i, j < mx + m */
static inline double *cell(const Orc *o, double *p, int f, int i, int j) {
    return p + ((size_t)f * o->N + (j + o->m)) * o->N + (i + o->m);
}

static int is_ghost(const Orc *o, int i, int j) {
    return i < 0 || j < 0 || i >= o->mx || j >= o->mx;
}

/* ------------------------------------------------------------------ */
/* create / destroy / data movement                                     */
/* ------------------------------------------------------------------ */
/* 1 if the level-lf quadrant (X, Y) lies inside a leaf of level <= lcap */
static int covered_by_le(const Orc *o, int lf, int X, int Y, int lcap) {
    for (int l2 = lcap; l2 >= 0; l2--)
        if (find_leaf(o, l2, X >> (lf - l2), Y >> (lf - l2)) >= 0) return 1;
    return 0;
}

/* 2:1 condition for one leaf against all face and corner neighbours */
static int balanced_at(const Orc *o, const OLeaf *L) {
    int l = L->level, lf = l + 2, nfx = o->nbx << lf, nfy = o->nby << lf;
    int x0 = L->ix * 4, y0 = L->iy * 4;
    for (int dy = -1; dy <= 1; dy++)
        for (int dx = -1; dx <= 1; dx++) {
            if (!dx && !dy) continue;
            int xs0 = dx < 0 ? x0 - 1 : dx > 0 ? x0 + 4 : x0;
            int xs1 = dx < 0 ? x0 - 1 : dx > 0 ? x0 + 4 : x0 + 3;
            int ys0 = dy < 0 ? y0 - 1 : dy > 0 ? y0 + 4 : y0;
            int ys1 = dy < 0 ? y0 - 1 : dy > 0 ? y0 + 4 : y0 + 3;
            for (int yy = ys0; yy <= ys1; yy++)
                for (int xx = xs0; xx <= xs1; xx++) {
                    int X = xx, Y = yy;
                    if (X < 0 || X >= nfx) {
                        if (o->bc[X < 0 ? 0 : 1] != BC_PERIODIC) continue;
                        X = (X + nfx) % nfx;
                    }
                    if (Y < 0 || Y >= nfy) {
                        if (o->bc[Y < 0 ? 2 : 3] != BC_PERIODIC) continue;
                        Y = (Y + nfy) % nfy;
                    }
                    if (!covered_by_le(o, lf, X, Y, l + 1)) return 0;
                }
        }
    return 1;
}

static int check_mesh(Orc *o) {
    /* leaves must tile the brick (the unit square for one block): areas sum
     * to the number of blocks and no two overlap */
    int err = 0;
    double area = 0.0;
    index_leaves(o);
    for (int k = 0; k < o->n; k++) {
        const OLeaf *L = &o->lv[k];
        if (L->level < 0 || L->level > 20 || L->ix < 0 || L->iy < 0 || L->ix >= (o->nbx << L->level) ||
            L->iy >= (o->nby << L->level))
            return ERR_ARG;
    }
    for (int k = 0; k < o->n; k++) {
        const OLeaf *L = &o->lv[k];
        area += ldexp(1.0, -2 * L->level);
        /* an ancestor that is also a leaf means overlap */
        for (int a = 1; a <= L->level; a++)
            if (find_local(o, L->level - a, L->ix >> a, L->iy >> a) >= 0) err |= ERR_COVER;
        if (find_local(o, L->level, L->ix, L->iy) != k) err |= ERR_COVER;
    }
    if (fabs(area - (double)o->nbx * o->nby) > 1e-12) err |= ERR_COVER;
    if (err) return err;
    /* 2:1 balance over faces and corners (Sec. 2): every quadrant two levels
     * finer that touches a leaf across a face or corner must lie inside a
     * leaf at most one level finer than that leaf; across block boundaries
     * too (brick coordinates). */
    for (int k = 0; k < o->n; k++)
        if (!balanced_at(o, &o->ph[k])) err |= ERR_UNBALANCED;
    return err;
}

/* A brick of nbx x nby unit blocks (Sec. 2.3); ori: nbx*nby orientation
 * codes (block (bx, by) at bx + nbx by), NULL for all zero.  Leaves (level,
 * ix, iy): block (ix >> level, iy >> level), the low bits the quadrant's
 * coordinates in the block's own indices.  A brick other than one block
 * of code 0 takes periodic sides and scalar advection at a constant
 * velocity (given in the brick's directions). */
Orc *orc_create_brick(int mx, int mbc, int eq, int lim, const int *bc, int vel, const double *vp, double g,
                      int lmin, int lmax, int nbx, int nby, const int *ori, int n, const int *leaves, int *status) {
    Orc *o = (Orc *)calloc(1, sizeof(Orc));
    o->nbx = nbx > 0 ? nbx : 1;
    o->nby = nby > 0 ? nby : 1;
    if (ori) {
        o->ori = (int *)malloc(sizeof(int) * o->nbx * o->nby);
        for (int b = 0; b < o->nbx * o->nby; b++) o->ori[b] = ori[b] & 7;
    }
    o->mx = mx; o->m = mbc; o->N = mx + 2 * mbc;
    o->eq = eq; o->F = eq == EQ_SWE ? 3 : 1; o->lim = lim;
    for (int s = 0; s < 4; s++) o->bc[s] = bc[s];
    o->vel = vel;
    for (int s = 0; s < 3; s++) o->vp[s] = vp[s];
    o->g = g; o->lmin = lmin; o->lmax = lmax;
    o->n = n;
    o->lv = (OLeaf *)malloc(sizeof(OLeaf) * (n > 0 ? n : 1));
    for (int k = 0; k < n; k++) {
        o->lv[k].level = leaves[3 * k];
        o->lv[k].ix = leaves[3 * k + 1];
        o->lv[k].iy = leaves[3 * k + 2];
    }
    *status = 0;
    /* Prop. 2.1: m <= M/4 (the interpolation stencil here is 3 wide) */
    if (mbc < 2 || 4 * mbc > mx || (mx & 1)) { *status = ERR_WIDTH; }
    if (nbx < 1 || nby < 1) *status |= ERR_ARG;
    if (ori)
        for (int b = 0; b < o->nbx * o->nby; b++)
            if (ori[b] < 0 || ori[b] > 7) *status |= ERR_ARG;
    if (is_brick(o) && (eq != EQ_ADV || vel == VEL_SWIRL || bc[0] != BC_PERIODIC || bc[1] != BC_PERIODIC ||
                        bc[2] != BC_PERIODIC || bc[3] != BC_PERIODIC))
        *status |= ERR_ARG;
    int e = check_mesh(o);
    if (e) *status |= e;
    size_t sz = (size_t)(n > 0 ? n : 1) * o->F * o->N * o->N;
    o->q = (double *)calloc(sz, sizeof(double));
    o->qold = (double *)calloc(sz, sizeof(double));
    o->qhat = (double *)calloc(sz, sizeof(double));
    return o;
}

Orc *orc_create(int mx, int mbc, int eq, int lim, const int *bc, int vel, const double *vp,
                double g, int lmin, int lmax, int n, const int *leaves, int *status) {
    return orc_create_brick(mx, mbc, eq, lim, bc, vel, vp, g, lmin, lmax, 1, 1, NULL, n, leaves, status);
}

/* Map the grid (Sec. 1 mapped grids): X(xi, eta) = (xi, eta) + alpha sin(2 pi
 * xi) sin(2 pi eta) (1, 1), invertible for |alpha| < 1/(2 pi).  One block,
 * periodic sides, scalar advection (velocities stay edge fluxes per unit
 * computational length).  Returns 0 or ERR_ARG. */
int orc_set_mapping(Orc *o, double alpha) {
    if (!(fabs(alpha) < 0.5 / M_PI)) return ERR_ARG;
    if (alpha != 0.0 && (is_brick(o) || o->eq != EQ_ADV || o->bc[0] != BC_PERIODIC || o->bc[2] != BC_PERIODIC))
        return ERR_ARG;
    o->map_alpha = alpha;
    return 0;
}

void orc_destroy(Orc *o) {
    if (!o) return;
    free(o->lv); free(o->q); free(o->qold); free(o->qhat); free(o->hidx); free(o->ph); free(o->ori);
    free(o);
}

int orc_nleaves(const Orc *o) { return o->n; }
void orc_leaves(const Orc *o, int *out) {
    for (int k = 0; k < o->n; k++) {
        out[3 * k] = o->lv[k].level; out[3 * k + 1] = o->lv[k].ix; out[3 * k + 2] = o->lv[k].iy;
    }
}
int orc_error(const Orc *o) { return o->err; }
void orc_clear_error(Orc *o) { o->err = 0; }

/* interior data in leaf order, [n][F][mx][mx] */
void orc_set_interior(Orc *o, const double *src) {
    for (int k = 0; k < o->n; k++)
        for (int f = 0; f < o->F; f++)
            for (int j = 0; j < o->mx; j++)
                for (int i = 0; i < o->mx; i++)
                    *cell(o, pat(o, o->q, k), f, i, j) =
                        src[(((size_t)k * o->F + f) * o->mx + j) * o->mx + i];
}
void orc_get_interior(const Orc *o, double *dst) {
    for (int k = 0; k < o->n; k++)
        for (int f = 0; f < o->F; f++)
            for (int j = 0; j < o->mx; j++)
                for (int i = 0; i < o->mx; i++)
                    dst[(((size_t)k * o->F + f) * o->mx + j) * o->mx + i] =
                        *cell(o, pat(o, o->q, k), f, i, j);
}
/* full arrays including ghosts, [n][F][N][N] */
void orc_get_full(const Orc *o, double *dst) {
    memcpy(dst, o->q, sizeof(double) * (size_t)o->n * o->F * o->N * o->N);
}
void orc_set_full(Orc *o, const double *src) {
    memcpy(o->q, src, sizeof(double) * (size_t)o->n * o->F * o->N * o->N);
}
void orc_get_old_interior(const Orc *o, double *dst) {
    for (int k = 0; k < o->n; k++)
        for (int f = 0; f < o->F; f++)
            for (int j = 0; j < o->mx; j++)
                for (int i = 0; i < o->mx; i++)
                    dst[(((size_t)k * o->F + f) * o->mx + j) * o->mx + i] =
                        *cell(o, pat(o, o->qold, k), f, i, j);
}
void orc_set_threads(int nt) {
#ifdef _OPENMP
    omp_set_num_threads(nt > 0 ? nt : 1);
#else
    (void)nt;
#endif
}
int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* ghost filling: Algorithm 1 by point location                         */
/* ------------------------------------------------------------------ */
static double minmod(double a, double b) {
    /* minmod of the two one-sided differences (limited gradient, Sec. 2.3
     * "one-sided differences" and Sec. 4.1 "monotone" interpolation) */
    if (a * b <= 0.0) return 0.0;
    return fabs(a) < fabs(b) ? a : b;
}

/* Fold a global index along one axis for a periodic side: returns the
 * wrapped index or -1 if the cell is exterior to a physical wall. */
static int wrap_axis(const Orc *o, int I, int nl, int side_lo, int side_hi) {
    if (I < 0) return o->bc[side_lo] == BC_PERIODIC ? I + nl : -1;
    if (I >= nl) return o->bc[side_hi] == BC_PERIODIC ? I - nl : -1;
    return I;
}

/* source array for reading leaf k during a fill: the time-interpolated copy
 * for the coarse level just below the filled range, the state otherwise */
static double *src_of(const Orc *o, int k, int clevel) {
    return o->lv[k].level == clevel ? pat(o, o->qhat, k) : pat(o, o->q, k);
}

static void poison_ghosts(const Orc *o, double *p) {
    for (int f = 0; f < o->F; f++)
        for (int j = -o->m; j < o->mx + o->m; j++)
            for (int i = -o->m; i < o->mx + o->m; i++)
                if (is_ghost(o, i, j)) *cell(o, p, f, i, j) = NAN;
}

/* Brick index of the level-r cell (i, j) of leaf k (own indices from its
 * first cell), wrapped on periodic sides of the brick; returns 0 if the cell
 * lies outside a physical wall. */
static int ghost_to_brick(const Orc *o, int k, int r, int i, int j, int *X, int *Y) {
    int nl = o->mx << r;
    cell_to_brick(o, k, r, i, j, X, Y);
    *X = wrap_axis(o, *X, o->nbx * nl, 0, 1);
    *Y = wrap_axis(o, *Y, o->nby * nl, 2, 3);
    return *X >= 0 && *Y >= 0;
}

/* ------------------------------------------------------------------ */
/* mapped grids: cell areas (the metric terms of a second-order finite   */
/* volume scheme on a mapped grid, Sec. 1; Sec. 5.2 runs one)            */
/* ------------------------------------------------------------------ */
/* Jacobian determinant of the mapping at (xi, eta): with w = alpha s(xi)
 * t(eta), s = sin(2 pi xi), t = sin(2 pi eta), X = (xi + w, eta + w), so
 * det = (1 + w_xi)(1 + w_eta) - w_eta w_xi = 1 + w_xi + w_eta. */
static double map_jacobian(const Orc *o, double xi, double eta) {
    double tp = 2.0 * M_PI;
    double w_xi = o->map_alpha * tp * cos(tp * xi) * sin(tp * eta);
    double w_eta = o->map_alpha * tp * sin(tp * xi) * cos(tp * eta);
    return 1.0 + w_xi + w_eta;
}

/* Area of the mapped image of level-l cell (I, J), the integral of the
 * Jacobian over the cell (4 x 4 Gauss-Legendre points: for this smooth
 * mapping on cells of at most 1/32 it is exact to rounding), over the
 * computational area h^2: the capacity.  Exact areas nest: a cell's area is
 * the sum of its four children's, so area-weighted averages conserve mass.
 * 1 on a Cartesian grid.  Indices wrap periodically. */
static double capacity(const Orc *o, int l, int I, int J) {
    if (o->map_alpha == 0.0) return 1.0;
    static const double gx[4] = {-0.8611363115940526, -0.3399810435848563, 0.3399810435848563, 0.8611363115940526};
    static const double gw[4] = {0.3478548451374538, 0.6521451548625461, 0.6521451548625461, 0.3478548451374538};
    int n = o->mx << l;
    double h = 1.0 / n;
    I = ((I % n) + n) % n;
    J = ((J % n) + n) % n;
    double xc = (I + 0.5) * h, yc = (J + 0.5) * h, sum = 0.0;
    for (int b = 0; b < 4; b++)
        for (int a = 0; a < 4; a++)
            sum += gw[a] * gw[b] * map_jacobian(o, xc + 0.5 * h * gx[a], yc + 0.5 * h * gx[b]);
    return 0.25 * sum; /* (h/2)^2 sum / h^2 */
}

/* capacity of local cell (i, j) of leaf k */
static double cell_capacity(const Orc *o, int k, int i, int j) {
    const OLeaf *L = &o->lv[k];
    return capacity(o, L->level, L->ix * o->mx + i, L->iy * o->mx + j);
}

double orc_capacity(const Orc *o, int l, int I, int J) { return capacity(o, l, I, J); }

/* Phase "copy and average": coarse ghost regions of leaf k (Alg. 1, first
 * loop).  Sec. 2.3: every index of this patch is carried into the
 * neighbour's own indices (through the brick's, which amounts to eq.
 * transform and, for a fine neighbour, the fine points I_f^k of the
 * direction vectors d_k taken in this patch's indices). */
static void fill_coarse_ghosts(Orc *o, int k, int clevel) {
    const OLeaf *P = &o->lv[k];
    int l = P->level, mx = o->mx;
    double *dst = src_of(o, k, clevel);
    for (int j = -o->m; j < mx + o->m; j++)
        for (int i = -o->m; i < mx + o->m; i++) {
            if (!is_ghost(o, i, j)) continue;
            int I, J;
            if (!ghost_to_brick(o, k, l, i, j, &I, &J)) continue; /* exterior: boundary conditions */
            int kk = locate(o, l, I, J);
            if (kk < 0) { o->err |= ERR_STENCIL; continue; }
            const OLeaf *L = &o->lv[kk];
            double *s = src_of(o, kk, clevel);
            if (L->level == l) {
                /* same size: q_c(I_c) = q_n(I_n) */
                int a, b;
                brick_to_cell(o, kk, l, I, J, &a, &b);
                for (int f = 0; f < o->F; f++) *cell(o, dst, f, i, j) = *cell(o, s, f, a, b);
            } else if (L->level == l + 1) {
                /* eq. ghost_coarse: mean of the four fine cells I_f^k,
                 * k = 0..3 in the order of the direction vectors d_k of
                 * this (coarse) patch: fine cell (2i, 2j) + (1 + d_k) / 2 */
                int fa[4], fb[4];
                for (int d = 0; d < 4; d++) {
                    int X, Y;
                    ghost_to_brick(o, k, l + 1, 2 * i + (d & 1), 2 * j + (d >> 1), &X, &Y);
                    brick_to_cell(o, kk, l + 1, X, Y, &fa[d], &fb[d]);
                }
                if (o->map_alpha == 0.0) {
                    for (int f = 0; f < o->F; f++)
                        *cell(o, dst, f, i, j) = 0.25 * (*cell(o, s, f, fa[0], fb[0]) + *cell(o, s, f, fa[1], fb[1]) +
                                                         *cell(o, s, f, fa[2], fb[2]) + *cell(o, s, f, fa[3], fb[3]));
                } else {
                    /* mapped grid: the area-weighted mean of the four fine
                     * cells (their areas, not the mean, carry the mass) */
                    double a[4], asum = 0.0;
                    for (int d = 0; d < 4; d++) {
                        a[d] = cell_capacity(o, kk, fa[d], fb[d]);
                        asum += a[d];
                    }
                    for (int f = 0; f < o->F; f++) {
                        double m = 0.0;
                        for (int d = 0; d < 4; d++) m += a[d] * *cell(o, s, f, fa[d], fb[d]);
                        *cell(o, dst, f, i, j) = m / asum;
                    }
                }
            }
            /* L coarser: a fine ghost region, filled by interpolation */
        }
}

/* Physical boundary conditions on the exterior ghost regions of leaf k:
 * x-walls over all rows, then y-walls over all columns, so exterior corners
 * are covered (Sec. 2.2: both edge and corner exterior regions). */
static void apply_bc(Orc *o, int k, int clevel) {
    const OLeaf *P = &o->lv[k];
    int mx = o->mx, m = o->m, nq = 1 << P->level;
    double *p = src_of(o, k, clevel);
    if (P->ix == 0 && o->bc[0] == BC_REFLECT)
        for (int f = 0; f < o->F; f++) {
            double sg = (o->eq == EQ_SWE && f == 1) ? -1.0 : 1.0;
            for (int j = -m; j < mx + m; j++)
                for (int i = -m; i < 0; i++) *cell(o, p, f, i, j) = sg * *cell(o, p, f, -1 - i, j);
        }
    if (P->ix == nq - 1 && o->bc[1] == BC_REFLECT)
        for (int f = 0; f < o->F; f++) {
            double sg = (o->eq == EQ_SWE && f == 1) ? -1.0 : 1.0;
            for (int j = -m; j < mx + m; j++)
                for (int i = mx; i < mx + m; i++) *cell(o, p, f, i, j) = sg * *cell(o, p, f, 2 * mx - 1 - i, j);
        }
    if (P->iy == 0 && o->bc[2] == BC_REFLECT)
        for (int f = 0; f < o->F; f++) {
            double sg = (o->eq == EQ_SWE && f == 2) ? -1.0 : 1.0;
            for (int j = -m; j < 0; j++)
                for (int i = -m; i < mx + m; i++) *cell(o, p, f, i, j) = sg * *cell(o, p, f, i, -1 - j);
        }
    if (P->iy == nq - 1 && o->bc[3] == BC_REFLECT)
        for (int f = 0; f < o->F; f++) {
            double sg = (o->eq == EQ_SWE && f == 2) ? -1.0 : 1.0;
            for (int j = mx; j < mx + m; j++)
                for (int i = -m; i < mx + m; i++) *cell(o, p, f, i, j) = sg * *cell(o, p, f, i, 2 * mx - 1 - j);
        }
}

/* Fine ghost regions of leaf k (level l+1) from coarse level l (Alg. 1, third
 * loop), eq. ghost_fine: q_f = q_c + (h/4) grad~ q_c . d_k, the gradient from
 * limited one-sided differences on the coarse grid, which may read the coarse
 * grid's own ghost cells (filled in the earlier phases). */
static void fill_fine_ghosts(Orc *o, int k, int clevel) {
    const OLeaf *P = &o->lv[k];
    int l = P->level, mx = o->mx;
    double *dst = pat(o, o->q, k);
    for (int j = -o->m; j < mx + o->m; j++)
        for (int i = -o->m; i < mx + o->m; i++) {
            if (!is_ghost(o, i, j)) continue;
            int I, J;
            if (!ghost_to_brick(o, k, l, i, j, &I, &J)) continue;
            int kk = locate(o, l, I, J);
            if (kk < 0 || o->lv[kk].level != l - 1) continue;
            double *s = src_of(o, kk, clevel);
            /* the fine cell in the coarse leaf's own indices, at the fine
             * resolution (Sec. 2.3: the stencil and d_k live in the coarse
             * grid's index space) */
            int a, b;
            brick_to_cell(o, kk, l, I, J, &a, &b);
            int ic = a >> 1, jc = b >> 1;
            /* d_k: +1 when the fine cell is the upper half of the coarse cell */
            double dx = (a & 1) ? 1.0 : -1.0, dy = (b & 1) ? 1.0 : -1.0;
            for (int f = 0; f < o->F; f++) {
                double c = *cell(o, s, f, ic, jc);
                double xm = *cell(o, s, f, ic - 1, jc), xp = *cell(o, s, f, ic + 1, jc);
                double ym = *cell(o, s, f, ic, jc - 1), yp = *cell(o, s, f, ic, jc + 1);
                if (isnan(c) || isnan(xm) || isnan(xp) || isnan(ym) || isnan(yp)) o->err |= ERR_STENCIL;
                double sx = minmod(xp - c, c - xm);
                double sy = minmod(yp - c, c - ym);
                *cell(o, dst, f, i, j) = c + 0.25 * (dx * sx + dy * sy);
            }
        }
}

/* Fill every ghost cell of the leaves with level in [lo, hi].  Levels >= lo
 * are synchronised; level lo-1 is read at time fraction alpha of its last
 * step: alpha == 1 means synchronised (use the state itself), otherwise
 * q_old + alpha (q - q_old) on its interior, whose coarse ghost regions are
 * then filled from that interpolated level and from level lo. */
void orc_ghost_fill(Orc *o, int lo, int hi, double alpha) {
    int cl = lo - 1;
    int n = o->n;
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < n; k++) {
        int l = o->lv[k].level;
        if (l == cl) {
            double *d = pat(o, o->qhat, k), *q = pat(o, o->q, k), *qo = pat(o, o->qold, k);
            for (int f = 0; f < o->F; f++)
                for (int j = 0; j < o->mx; j++)
                    for (int i = 0; i < o->mx; i++) {
                        double a = *cell(o, q, f, i, j), b = *cell(o, qo, f, i, j);
                        *cell(o, d, f, i, j) = alpha == 1.0 ? a : b + alpha * (a - b);
                    }
            poison_ghosts(o, d);
        } else if (l >= lo && l <= hi) {
            poison_ghosts(o, pat(o, o->q, k));
        }
    }
    /* 1: copy and average, all levels */
#pragma omp parallel for schedule(dynamic, 4)
    for (k = 0; k < n; k++) {
        int l = o->lv[k].level;
        if (l >= cl && l <= hi) fill_coarse_ghosts(o, k, cl);
    }
    /* 2: boundary conditions, levels lo-1 .. hi-1 */
#pragma omp parallel for schedule(static)
    for (k = 0; k < n; k++) {
        int l = o->lv[k].level;
        if (l >= cl && l <= hi - 1) apply_bc(o, k, cl);
    }
    /* 3: interpolation, in increasing level order */
    for (int l = cl; l <= hi - 1; l++) {
#pragma omp parallel for schedule(dynamic, 4)
        for (k = 0; k < n; k++)
            if (o->lv[k].level == l + 1 && l + 1 >= lo) fill_fine_ghosts(o, k, cl);
    }
    /* 4: boundary conditions, levels lo .. hi */
#pragma omp parallel for schedule(static)
    for (k = 0; k < n; k++) {
        int l = o->lv[k].level;
        if (l >= lo && l <= hi) apply_bc(o, k, cl);
    }
}

/* ------------------------------------------------------------------ */
/* velocities (scalar advection)                                        */
/* ------------------------------------------------------------------ */
/* Stream function psi; u = psi_y, v = -psi_x (Sec. 5.1).  Edge values are
 * exact edge averages, (psi(end) - psi(start)) / h, written in a
 * cancellation-free product form; the swirl field is evaluated at the step's
 * mid time. */
static int wrap_idx(int I, int nl) { I %= nl; return I < 0 ? I + nl : I; }

/* A constant velocity (u, v), given in the brick's directions, seen in the
 * own indices of a block with orientation code `code`: its component along
 * the block's first (dir 0) or second (dir 1) index direction.  A reversed
 * brick direction reverses the component; with the directions exchanged the
 * block's first index runs along the brick's second direction. */
static double const_own(const Orc *o, int code, int dir) {
    double u = (code & 2) ? -o->vp[0] : o->vp[0];
    double v = (code & 4) ? -o->vp[1] : o->vp[1];
    if (code & 1) return dir == 0 ? v : u;
    return dir == 0 ? u : v;
}

/* edge velocities of a leaf whose block has orientation code `code` (the
 * swirl field lives on one block of code 0) */
static double vel_u(const Orc *o, int code, int l, int Ie, int Jc, double tm) {
    if (o->vel == VEL_CONST) return const_own(o, code, 0);
    if (o->vel == VEL_NONE) return 0.0;
    int nl = o->mx << l;
    double h = 1.0 / nl;
    int I = (o->bc[0] == BC_PERIODIC) ? wrap_idx(Ie, nl) : Ie;
    int J = (o->bc[2] == BC_PERIODIC) ? wrap_idx(Jc, nl) : Jc;
    double x = I * h, y = (J + 0.5) * h;
    double sx = sin(M_PI * x);
    double sig = sin(M_PI * h) / (M_PI * h);
    double c = cos(M_PI * tm / o->vp[0]);
    return sx * sx * sin(2.0 * M_PI * y) * sig * c;
}
static double vel_v(const Orc *o, int code, int l, int Ic, int Je, double tm) {
    if (o->vel == VEL_CONST) return const_own(o, code, 1);
    if (o->vel == VEL_NONE) return 0.0;
    int nl = o->mx << l;
    double h = 1.0 / nl;
    int I = (o->bc[0] == BC_PERIODIC) ? wrap_idx(Ic, nl) : Ic;
    int J = (o->bc[2] == BC_PERIODIC) ? wrap_idx(Je, nl) : Je;
    double x = (I + 0.5) * h, y = J * h;
    double sy = sin(M_PI * y);
    double sig = sin(M_PI * h) / (M_PI * h);
    double c = cos(M_PI * tm / o->vp[0]);
    return -(sy * sy * sin(2.0 * M_PI * x) * sig * c);
}

/* Read-only accessor for the tests: the edge velocity the scalar step uses.
 * dir 0: u on x-edge I (between cells I-1 and I) of row J; dir 1: v on
 * y-edge J of column I; level-l indices, at time tm. */
double orc_edge_velocity(const Orc *o, int l, int dir, int I, int J, double tm) {
    return dir == 0 ? vel_u(o, 0, l, I, J, tm) : vel_v(o, 0, l, I, J, tm);
}

/* ------------------------------------------------------------------ */
/* scalar wave-propagation step on one patch                            */
/* ------------------------------------------------------------------ */
static double limited(int lim, double W, double Wu) {
    if (lim == LIM_LW) return W;
    if (lim == LIM_FIRST) return 0.0;
    if (W * Wu <= 0.0) return 0.0;
    double aw = fabs(W), au = fabs(Wu);
    if (lim == LIM_MINMOD) return W > 0 ? fmin(aw, au) : -fmin(aw, au);
    /* MC: phi(theta) W with phi = max(0, min((1+theta)/2, 2, 2 theta)),
     * theta = Wu / W, written without the division; ties resolve to the
     * first argument of the chain */
    double a = 0.5 * fabs(W + Wu), b = 2.0 * aw, c = 2.0 * au;
    double mn = a;
    if (b < mn) mn = b;
    if (c < mn) mn = c;
    return W > 0 ? mn : -mn;
}

/* branch code of the limiter for the tangent: 0 zero, 1 half-sum, 2 twice W,
 * 3 twice Wu, 4 identity (Lax-Wendroff) */
static int limiter_branch(int lim, double W, double Wu) {
    if (lim == LIM_LW) return 4;
    if (lim == LIM_FIRST) return 0;
    if (W * Wu <= 0.0) return 0;
    double aw = fabs(W), au = fabs(Wu);
    if (lim == LIM_MINMOD) return aw <= au ? 2 : 3; /* minmod: |W| or |Wu| (scaled below) */
    double a = 0.5 * fabs(W + Wu), b = 2.0 * aw, c = 2.0 * au;
    int br = 1;
    double mn = a;
    if (b < mn) { mn = b; br = 2; }
    if (c < mn) { mn = c; br = 3; }
    return br;
}
static double limited_lin(int lim, int br, double dW, double dWu) {
    if (br == 0) return 0.0;
    if (br == 4) return dW;
    if (lim == LIM_MINMOD) return br == 2 ? dW : dWu;
    if (br == 1) return 0.5 * (dW + dWu);
    if (br == 2) return 2.0 * dW;
    return 2.0 * dWu;
}

typedef struct {
    int N, m, mx;
    double *Ft, *Gt, *Apx, *Amx, *Bpy, *Bmy; /* (N+1) x (N+1), offset m */
} Work;

static void work_alloc(Work *w, int mx, int m) {
    w->mx = mx; w->m = m; w->N = mx + 2 * m;
    size_t s = (size_t)(w->N + 1) * (w->N + 1);
    w->Ft = (double *)calloc(s, sizeof(double)); w->Gt = (double *)calloc(s, sizeof(double));
    w->Apx = (double *)calloc(s, sizeof(double)); w->Amx = (double *)calloc(s, sizeof(double));
    w->Bpy = (double *)calloc(s, sizeof(double)); w->Bmy = (double *)calloc(s, sizeof(double));
}
static void work_free(Work *w) {
    free(w->Ft); free(w->Gt); free(w->Apx); free(w->Amx); free(w->Bpy); free(w->Bmy);
}
/* edge arrays: [row][col], row/col in [-m, mx+m] */
#define WE(w, a, r, c) ((a)[((size_t)((r) + (w)->m)) * ((w)->N + 1) + ((c) + (w)->m)])

/* One step of the unsplit scheme for scalar advection on leaf k.
 * Q: patch array with valid ghosts; out: new interior written into Qn
 * (another patch-sized array); returns the CFL number of the step.
 * If frozen != NULL the step is the tangent (Jacobian) applied to dQ with
 * the limiter branches taken from Q; Qn then receives J dQ. */
static double adv_step(const Orc *o, int k, const double *Q, double *Qn, double t, double dt,
                       Work *w, const double *dQ) {
    const OLeaf *P = &o->lv[k];
    int mx = o->mx, l = P->level;
    double h = 1.0 / (mx << l), lam = dt / h, tm = t + 0.5 * dt;
    int gx = P->ix * mx, gy = P->iy * mx, oc = leaf_code(o, k);
    size_t s = (size_t)(w->N + 1) * (w->N + 1);
    memset(w->Ft, 0, s * sizeof(double)); memset(w->Gt, 0, s * sizeof(double));
    const double *D = dQ ? dQ : Q; /* data the (linear in D) update acts on */
#define QQ(i, j) (*cell(o, (double *)Q, 0, (i), (j)))
#define DD(i, j) (*cell(o, (double *)D, 0, (i), (j)))
    /* Capacity form on a mapped grid (Clawpack's, as the mapped-grid schemes
     * the paper cites use it): a cell's fluctuations and flux differences are
     * scaled by lam / kappa of that cell, a transverse wave by lam / kappa of
     * the cell its fluctuation entered, the correction's (1 - lam |s|) by the
     * mean of lam / kappa of the edge's two cells; the Courant number is
     * lam / kappa of the cell a wave enters times its speed.  kappa = 1 on a
     * Cartesian grid gives back the plain scheme, bit for bit. */
#define LK(i, j) (lam / cell_capacity(o, k, (i), (j)))
    double cmax = 0.0;
    /* x-edges (i-1/2, j), i in [0, mx], j in [-1, mx] */
    for (int j = -1; j <= mx; j++)
        for (int i = 0; i <= mx; i++) {
            double s_ = vel_u(o, oc, l, gx + i, gy + j, tm);
            double W = DD(i, j) - DD(i - 1, j);
            double Ap = (s_ > 0 ? s_ : 0.0) * W, Am = (s_ < 0 ? s_ : 0.0) * W;
            WE(w, w->Apx, j, i) = Ap; WE(w, w->Amx, j, i) = Am;
            double Wl;
            if (dQ) {
                double W0 = QQ(i, j) - QQ(i - 1, j);
                double Wu0 = s_ > 0 ? QQ(i - 1, j) - QQ(i - 2, j) : QQ(i + 1, j) - QQ(i, j);
                double Wu = s_ > 0 ? DD(i - 1, j) - DD(i - 2, j) : DD(i + 1, j) - DD(i, j);
                Wl = limited_lin(o->lim, limiter_branch(o->lim, W0, Wu0), W, Wu);
            } else {
                double Wu = s_ > 0 ? DD(i - 1, j) - DD(i - 2, j) : DD(i + 1, j) - DD(i, j);
                Wl = limited(o->lim, W, Wu);
            }
            double lr = LK(i, j), ll = LK(i - 1, j);
            double C = fabs(s_) * (1.0 - 0.5 * (ll + lr) * fabs(s_)) * Wl;
            WE(w, w->Ft, j, i) += 0.5 * C;
            double Aps = Ap - C, Ams = Am + C;
            double vpu = vel_v(o, oc, l, gx + i, gy + j + 1, tm), vpd = vel_v(o, oc, l, gx + i, gy + j, tm);
            double vmu = vel_v(o, oc, l, gx + i - 1, gy + j + 1, tm), vmd = vel_v(o, oc, l, gx + i - 1, gy + j, tm);
            WE(w, w->Gt, j + 1, i) -= 0.5 * lr * (vpu > 0 ? vpu : 0.0) * Aps;
            WE(w, w->Gt, j, i) -= 0.5 * lr * (vpd < 0 ? vpd : 0.0) * Aps;
            WE(w, w->Gt, j + 1, i - 1) -= 0.5 * ll * (vmu > 0 ? vmu : 0.0) * Ams;
            WE(w, w->Gt, j, i - 1) -= 0.5 * ll * (vmd < 0 ? vmd : 0.0) * Ams;
            if (j >= 0 && j < mx) {
                double c_ = s_ > 0 ? lr * s_ : (s_ < 0 ? ll * -s_ : 0.0);
                if (c_ > cmax) cmax = c_;
            }
        }
    /* y-edges (i, j-1/2), j in [0, mx], i in [-1, mx] */
    for (int i = -1; i <= mx; i++)
        for (int j = 0; j <= mx; j++) {
            double s_ = vel_v(o, oc, l, gx + i, gy + j, tm);
            double V = DD(i, j) - DD(i, j - 1);
            double Bp = (s_ > 0 ? s_ : 0.0) * V, Bm = (s_ < 0 ? s_ : 0.0) * V;
            WE(w, w->Bpy, j, i) = Bp; WE(w, w->Bmy, j, i) = Bm;
            double Vl;
            if (dQ) {
                double V0 = QQ(i, j) - QQ(i, j - 1);
                double Vu0 = s_ > 0 ? QQ(i, j - 1) - QQ(i, j - 2) : QQ(i, j + 1) - QQ(i, j);
                double Vu = s_ > 0 ? DD(i, j - 1) - DD(i, j - 2) : DD(i, j + 1) - DD(i, j);
                Vl = limited_lin(o->lim, limiter_branch(o->lim, V0, Vu0), V, Vu);
            } else {
                double Vu = s_ > 0 ? DD(i, j - 1) - DD(i, j - 2) : DD(i, j + 1) - DD(i, j);
                Vl = limited(o->lim, V, Vu);
            }
            double lu = LK(i, j), ld = LK(i, j - 1);
            double C = fabs(s_) * (1.0 - 0.5 * (ld + lu) * fabs(s_)) * Vl;
            WE(w, w->Gt, j, i) += 0.5 * C;
            double Bps = Bp - C, Bms = Bm + C;
            double upr = vel_u(o, oc, l, gx + i + 1, gy + j, tm), upl = vel_u(o, oc, l, gx + i, gy + j, tm);
            double umr = vel_u(o, oc, l, gx + i + 1, gy + j - 1, tm), uml = vel_u(o, oc, l, gx + i, gy + j - 1, tm);
            WE(w, w->Ft, j, i + 1) -= 0.5 * lu * (upr > 0 ? upr : 0.0) * Bps;
            WE(w, w->Ft, j, i) -= 0.5 * lu * (upl < 0 ? upl : 0.0) * Bps;
            WE(w, w->Ft, j - 1, i + 1) -= 0.5 * ld * (umr > 0 ? umr : 0.0) * Bms;
            WE(w, w->Ft, j - 1, i) -= 0.5 * ld * (uml < 0 ? uml : 0.0) * Bms;
            if (i >= 0 && i < mx) {
                double c_ = s_ > 0 ? lu * s_ : (s_ < 0 ? ld * -s_ : 0.0);
                if (c_ > cmax) cmax = c_;
            }
        }
    /* conservative update of the interior */
    for (int j = 0; j < mx; j++)
        for (int i = 0; i < mx; i++) {
            double fl = WE(w, w->Apx, j, i) + WE(w, w->Amx, j, i + 1) + WE(w, w->Bpy, j, i) + WE(w, w->Bmy, j + 1, i);
            double df = WE(w, w->Ft, j, i + 1) - WE(w, w->Ft, j, i) + WE(w, w->Gt, j + 1, i) - WE(w, w->Gt, j, i);
            double lc = LK(i, j);
            *cell(o, Qn, 0, i, j) = DD(i, j) - lc * fl - lc * df;
        }
#undef QQ
#undef DD
#undef LK
    return cmax;
}

/* ------------------------------------------------------------------ */
/* shallow water: Roe solver with Harten-Hyman entropy fix              */
/* ------------------------------------------------------------------ */
/* Riemann problem normal to an edge, in the frame (h, hn, ht): n is the
 * normal momentum, t the tangential one.  Outputs waves wv[p][3], speeds
 * s[p], fluctuations am/ap and the Roe state (un, ut, c) for the transverse
 * solve. */
typedef struct { double wv[3][3], s[3], am[3], ap[3], un, ut, c; } Rie;

static void roe_normal(double g, const double *qL, const double *qR, Rie *r) {
    double hL = qL[0], hR = qR[0];
    double uL = qL[1] / hL, uR = qR[1] / hR, vL = qL[2] / hL, vR = qR[2] / hR;
    double sL = sqrt(hL), sR = sqrt(hR);
    double hb = 0.5 * (hL + hR);
    double uh = (sL * uL + sR * uR) / (sL + sR);
    double vh = (sL * vL + sR * vR) / (sL + sR);
    double ch = sqrt(g * hb);
    double d0 = qR[0] - qL[0], d1 = qR[1] - qL[1], d2 = qR[2] - qL[2];
    double a1 = ((uh + ch) * d0 - d1) / (2.0 * ch);
    double a2 = d2 - vh * d0;
    double a3 = (d1 - (uh - ch) * d0) / (2.0 * ch);
    r->wv[0][0] = a1; r->wv[0][1] = a1 * (uh - ch); r->wv[0][2] = a1 * vh;
    r->wv[1][0] = 0.0; r->wv[1][1] = 0.0; r->wv[1][2] = a2;
    r->wv[2][0] = a3; r->wv[2][1] = a3 * (uh + ch); r->wv[2][2] = a3 * vh;
    r->s[0] = uh - ch; r->s[1] = uh; r->s[2] = uh + ch;
    r->un = uh; r->ut = vh; r->c = ch;
    for (int e = 0; e < 3; e++) { r->am[e] = 0.0; r->ap[e] = 0.0; }
    /* family 2 and the default split of families 1 and 3 */
    /* Harten-Hyman entropy fix on transonic rarefactions, family 1 */
    double l1L = uL - sqrt(g * hL);
    double hm = hL + r->wv[0][0];
    double l1R = (qL[1] + r->wv[0][1]) / hm - sqrt(g * hm);
    int fix1 = (l1L < 0.0 && l1R > 0.0);
    double hm3 = hR - r->wv[2][0];
    double l3L = (qR[1] - r->wv[2][1]) / hm3 + sqrt(g * hm3);
    double l3R = uR + sqrt(g * hR);
    int fix3 = (l3L < 0.0 && l3R > 0.0);
    for (int p = 0; p < 3; p++) {
        double sm, sp;
        if (p == 0 && fix1) {
            double beta = (l1R - r->s[0]) / (l1R - l1L);
            sm = beta * l1L; sp = (1.0 - beta) * l1R;
        } else if (p == 2 && fix3) {
            double beta = (l3R - r->s[2]) / (l3R - l3L);
            sm = beta * l3L; sp = (1.0 - beta) * l3R;
        } else {
            sm = r->s[p] < 0 ? r->s[p] : 0.0;
            sp = r->s[p] > 0 ? r->s[p] : 0.0;
        }
        for (int e = 0; e < 3; e++) { r->am[e] += sm * r->wv[p][e]; r->ap[e] += sp * r->wv[p][e]; }
    }
}

/* transverse split of a fluctuation vector A (frame h, hn, ht) into the
 * parts moving in +t and -t, using the edge's Roe state */
static void roe_transverse(const Rie *r, const double *A, double *bp, double *bm) {
    double un = r->un, ut = r->ut, c = r->c;
    double b1 = ((ut + c) * A[0] - A[2]) / (2.0 * c);
    double b2 = A[1] - un * A[0];
    double b3 = (A[2] - (ut - c) * A[0]) / (2.0 * c);
    double mu[3] = {ut - c, ut, ut + c};
    double rv[3][3] = {{1.0, un, ut - c}, {0.0, 1.0, 0.0}, {1.0, un, ut + c}};
    double be[3] = {b1, b2, b3};
    for (int e = 0; e < 3; e++) { bp[e] = 0.0; bm[e] = 0.0; }
    for (int p = 0; p < 3; p++) {
        double mp = mu[p] > 0 ? mu[p] : 0.0, mm = mu[p] < 0 ? mu[p] : 0.0;
        for (int e = 0; e < 3; e++) { bp[e] += mp * be[p] * rv[p][e]; bm[e] += mm * be[p] * rv[p][e]; }
    }
}

static double phi_lim(int lim, double th) {
    if (lim == LIM_LW) return 1.0;
    if (lim == LIM_FIRST) return 0.0;
    if (lim == LIM_MINMOD) return th <= 0 ? 0.0 : (th < 1.0 ? th : 1.0);
    double a = 0.5 * (1.0 + th), b = 2.0, c = 2.0 * th;
    double mn = a;
    if (b < mn) mn = b;
    if (c < mn) mn = c;
    return mn > 0.0 ? mn : 0.0;
}

/* the system step: same structure as the scalar one with vector waves */
static double swe_step(const Orc *o, int k, const double *Q, double *Qn, double dt) {
    const OLeaf *P = &o->lv[k];
    int mx = o->mx, m = o->m, N = o->N, l = P->level;
    double h = 1.0 / (mx << l), lam = dt / h, g = o->g;
    int E = N + 1;
    /* per-edge storage over the full frame, offset m */
    size_t ne = (size_t)E * E;
    Rie *rx = (Rie *)malloc(sizeof(Rie) * ne);
    Rie *ry = (Rie *)malloc(sizeof(Rie) * ne);
    double *Ft = (double *)calloc(ne * 3, sizeof(double));
    double *Gt = (double *)calloc(ne * 3, sizeof(double));
#define IX(r, c) (((size_t)((r) + m)) * E + ((c) + m))
#define QV(f, i, j) (*cell(o, (double *)Q, (f), (i), (j)))
    double smax = 0.0;
    /* x-edges: Riemann problems on i in [-1, mx+1], j in [-1, mx] (the
     * extra columns provide upwind waves for the limiter) */
    for (int j = -1; j <= mx; j++)
        for (int i = -1; i <= mx + 1; i++) {
            double qL[3] = {QV(0, i - 1, j), QV(1, i - 1, j), QV(2, i - 1, j)};
            double qR[3] = {QV(0, i, j), QV(1, i, j), QV(2, i, j)};
            roe_normal(g, qL, qR, &rx[IX(j, i)]);
        }
    /* y-edges: frame (h, hv, hu) */
    for (int i = -1; i <= mx; i++)
        for (int j = -1; j <= mx + 1; j++) {
            double qL[3] = {QV(0, i, j - 1), QV(2, i, j - 1), QV(1, i, j - 1)};
            double qR[3] = {QV(0, i, j), QV(2, i, j), QV(1, i, j)};
            roe_normal(g, qL, qR, &ry[IX(j, i)]);
        }
    /* x sweep: correction and transverse on i in [0, mx], j in [-1, mx] */
    for (int j = -1; j <= mx; j++)
        for (int i = 0; i <= mx; i++) {
            Rie *r = &rx[IX(j, i)];
            double C[3] = {0, 0, 0};
            for (int p = 0; p < 3; p++) {
                const Rie *ru = r->s[p] > 0 ? &rx[IX(j, i - 1)] : &rx[IX(j, i + 1)];
                double ww = 0, wu = 0;
                for (int e = 0; e < 3; e++) { ww += r->wv[p][e] * r->wv[p][e]; wu += ru->wv[p][e] * r->wv[p][e]; }
                double ph = ww == 0.0 ? 0.0 : phi_lim(o->lim, wu / ww);
                double as = fabs(r->s[p]);
                for (int e = 0; e < 3; e++) C[e] += as * (1.0 - lam * as) * ph * r->wv[p][e];
                if (j >= 0 && j < mx && as > smax) smax = as;
            }
            double Aps[3], Ams[3];
            for (int e = 0; e < 3; e++) {
                Ft[IX(j, i) * 3 + e] += 0.5 * C[e];
                Aps[e] = r->ap[e] - C[e];
                Ams[e] = r->am[e] + C[e];
            }
            double bp[3], bm[3];
            roe_transverse(r, Aps, bp, bm);
            for (int e = 0; e < 3; e++) {
                Gt[IX(j + 1, i) * 3 + e] -= 0.5 * lam * bp[e];
                Gt[IX(j, i) * 3 + e] -= 0.5 * lam * bm[e];
            }
            roe_transverse(r, Ams, bp, bm);
            for (int e = 0; e < 3; e++) {
                Gt[IX(j + 1, i - 1) * 3 + e] -= 0.5 * lam * bp[e];
                Gt[IX(j, i - 1) * 3 + e] -= 0.5 * lam * bm[e];
            }
        }
    /* y sweep, frame (h, hv, hu): results mapped back to (h, hu, hv) */
    for (int i = -1; i <= mx; i++)
        for (int j = 0; j <= mx; j++) {
            Rie *r = &ry[IX(j, i)];
            double C[3] = {0, 0, 0};
            for (int p = 0; p < 3; p++) {
                const Rie *ru = r->s[p] > 0 ? &ry[IX(j - 1, i)] : &ry[IX(j + 1, i)];
                double ww = 0, wu = 0;
                for (int e = 0; e < 3; e++) { ww += r->wv[p][e] * r->wv[p][e]; wu += ru->wv[p][e] * r->wv[p][e]; }
                double ph = ww == 0.0 ? 0.0 : phi_lim(o->lim, wu / ww);
                double as = fabs(r->s[p]);
                for (int e = 0; e < 3; e++) C[e] += as * (1.0 - lam * as) * ph * r->wv[p][e];
                if (i >= 0 && i < mx && as > smax) smax = as;
            }
            double Bps[3], Bms[3];
            for (int e = 0; e < 3; e++) { Bps[e] = r->ap[e] - C[e]; Bms[e] = r->am[e] + C[e]; }
            /* G~ in (h, hu, hv) order */
            Gt[IX(j, i) * 3 + 0] += 0.5 * C[0];
            Gt[IX(j, i) * 3 + 1] += 0.5 * C[2];
            Gt[IX(j, i) * 3 + 2] += 0.5 * C[1];
            double ap_[3], am_[3];
            roe_transverse(r, Bps, ap_, am_);
            int sw[3] = {0, 2, 1};
            for (int e = 0; e < 3; e++) {
                Ft[IX(j, i + 1) * 3 + sw[e]] -= 0.5 * lam * ap_[e];
                Ft[IX(j, i) * 3 + sw[e]] -= 0.5 * lam * am_[e];
            }
            roe_transverse(r, Bms, ap_, am_);
            for (int e = 0; e < 3; e++) {
                Ft[IX(j - 1, i + 1) * 3 + sw[e]] -= 0.5 * lam * ap_[e];
                Ft[IX(j - 1, i) * 3 + sw[e]] -= 0.5 * lam * am_[e];
            }
        }
    for (int j = 0; j < mx; j++)
        for (int i = 0; i < mx; i++) {
            const Rie *xl = &rx[IX(j, i)], *xr = &rx[IX(j, i + 1)];
            const Rie *yd = &ry[IX(j, i)], *yu = &ry[IX(j + 1, i)];
            int sw[3] = {0, 2, 1};
            for (int f = 0; f < 3; f++) {
                double fl = xl->ap[f] + xr->am[f] + yd->ap[sw[f]] + yu->am[sw[f]];
                double df = Ft[IX(j, i + 1) * 3 + f] - Ft[IX(j, i) * 3 + f] + Gt[IX(j + 1, i) * 3 + f] -
                            Gt[IX(j, i) * 3 + f];
                *cell(o, Qn, f, i, j) = QV(f, i, j) - lam * fl - lam * df;
            }
        }
#undef IX
#undef QV
    free(rx); free(ry); free(Ft); free(Gt);
    return lam * smax;
}

/* ------------------------------------------------------------------ */
/* advancing levels                                                     */
/* ------------------------------------------------------------------ */
/* Advance every leaf of `level` by dt from time t (ghosts must be valid).
 * The state before the step is kept as q_old for time interpolation.
 * Returns the largest CFL number seen. */
double orc_advance_level(Orc *o, int level, double t, double dt) {
    double cfl = 0.0;
    int n = o->n;
#pragma omp parallel
    {
        Work w;
        work_alloc(&w, o->mx, o->m);
        size_t psz = (size_t)o->F * o->N * o->N;
        double *tmp = (double *)malloc(sizeof(double) * psz);
        double loc = 0.0;
        int k;
#pragma omp for schedule(dynamic, 2)
        for (k = 0; k < n; k++) {
            if (o->lv[k].level != level) continue;
            double *q = pat(o, o->q, k);
            double c = o->eq == EQ_SWE ? swe_step(o, k, q, tmp, dt) : adv_step(o, k, q, tmp, t, dt, &w, NULL);
            if (c > loc) loc = c;
            memcpy(pat(o, o->qold, k), q, sizeof(double) * psz);
            for (int f = 0; f < o->F; f++)
                for (int j = 0; j < o->mx; j++)
                    for (int i = 0; i < o->mx; i++) *cell(o, q, f, i, j) = *cell(o, tmp, f, i, j);
        }
#pragma omp critical
        if (loc > cfl) cfl = loc;
        free(tmp);
        work_free(&w);
    }
    return cfl;
}

/* Multirate coarse-first recursion: fill level l at t (coarser level
 * time-interpolated), advance level l, then take two half steps on l+1. */
static double mr_step(Orc *o, int l, double t, double dtl, double alpha) {
    orc_ghost_fill(o, l, l, alpha);
    double cfl = orc_advance_level(o, l, t, dtl);
    if (l < o->lmax) {
        double c1 = mr_step(o, l + 1, t, 0.5 * dtl, 0.0);
        double c2 = mr_step(o, l + 1, t + 0.5 * dtl, 0.5 * dtl, 0.5);
        if (c1 > cfl) cfl = c1;
        if (c2 > cfl) cfl = c2;
    }
    return cfl;
}

/* One coarse step.  mode 0: multirate (dt halves per level below lmin);
 * mode 1: global stepping, every level takes dt (the caller passes the
 * finest level's step).  Returns the largest CFL number. */
double orc_coarse_step(Orc *o, double t, double dt, int mode) {
    if (mode == 0) return mr_step(o, o->lmin, t, dt, 1.0);
    orc_ghost_fill(o, o->lmin, o->lmax, 1.0);
    double cfl = 0.0;
    for (int l = o->lmin; l <= o->lmax; l++) {
        double c = orc_advance_level(o, l, t, dt);
        if (c > cfl) cfl = c;
    }
    return cfl;
}

/* ------------------------------------------------------------------ */
/* tagging, adaptation, transfer (Sec. 4.1)                             */
/* ------------------------------------------------------------------ */
/* Per leaf: g = max over interior cells of |grad q| (central differences of
 * field 0 divided by 2h; ghosts must be valid).  +1 refine if g > tau_r and
 * level < lmax, -1 coarsen candidate if g <= tau_c and level > lmin.
 * The comparison is made on squares: g^2 > tau^2. */
void orc_tag(const Orc *o, double tau_r, double tau_c, signed char *tags, double *gmax) {
    int n = o->n;
    int k;
#pragma omp parallel for schedule(static)
    for (k = 0; k < n; k++) {
        const OLeaf *P = &o->lv[k];
        double h = 1.0 / (o->mx << P->level);
        double *q = pat(o, o->q, k);
        double g2 = 0.0;
        for (int j = 0; j < o->mx; j++)
            for (int i = 0; i < o->mx; i++) {
                double gx = (*cell(o, q, 0, i + 1, j) - *cell(o, q, 0, i - 1, j)) / (2.0 * h);
                double gy = (*cell(o, q, 0, i, j + 1) - *cell(o, q, 0, i, j - 1)) / (2.0 * h);
                double v = gx * gx + gy * gy;
                if (v > g2) g2 = v;
            }
        signed char tg = 0;
        if (g2 > tau_r * tau_r && P->level < o->lmax) tg = 1;
        else if (g2 <= tau_c * tau_c && P->level > o->lmin) tg = -1;
        tags[k] = tg;
        if (gmax) gmax[k] = g2;
    }
}

static int cmp_leaf(const void *a, const void *b) {
    const int *x = (const int *)a, *y = (const int *)b;
    if (x[0] != y[0]) return x[0] - y[0];
    if (x[2] != y[2]) return x[2] - y[2];
    return x[1] - y[1];
}

/* Leaf containing the level-lq quadrant (X, Y) (brick coordinates, inside the
 * brick), found by searching levels lq, lq-1, ..., 0; -1 if none. */
static int leaf_containing(const Orc *o, int lq, int X, int Y) {
    for (int l2 = lq; l2 >= 0; l2--) {
        int k = find_leaf(o, l2, X >> (lq - l2), Y >> (lq - l2));
        if (k >= 0) return k;
    }
    return -1;
}

/* Smooth refinement (Sec. 4.2): every leaf's target level is its level plus
 * its tag (kept within [lmin, lmax]); the level passed on to adaptation is the
 * maximum of the targets of the leaf and of every leaf touching it across a
 * face or a corner.  The neighbours are found by point location on the ring
 * of level-(l+1) quadrants around the leaf (each is covered by one leaf of
 * level l-1, l or l+1 on a 2:1 balanced mesh); periodic sides wrap, walls
 * have no neighbour. */
static void smooth_targets(const Orc *o, const int *target, int *T) {
    for (int k = 0; k < o->n; k++) {
        const OLeaf *L = &o->ph[k]; /* brick coordinates: the ring crosses blocks */
        int lq = L->level + 1, nqx = o->nbx << lq, nqy = o->nby << lq, m = target[k];
        for (int dy = -1; dy <= 2; dy++)
            for (int dx = -1; dx <= 2; dx++) {
                if (dx >= 0 && dx <= 1 && dy >= 0 && dy <= 1) continue; /* the leaf itself */
                int X = 2 * L->ix + dx, Y = 2 * L->iy + dy;
                if (X < 0 || X >= nqx) { if (o->bc[X < 0 ? 0 : 1] != BC_PERIODIC) continue; X = (X + nqx) % nqx; }
                if (Y < 0 || Y >= nqy) { if (o->bc[Y < 0 ? 2 : 3] != BC_PERIODIC) continue; Y = (Y + nqy) % nqy; }
                int kk = leaf_containing(o, lq, X, Y);
                if (kk >= 0 && target[kk] > m) m = target[kk];
            }
        T[k] = m;
    }
}

/* New leaf set from tags (+1 refine, -1 coarsen, 0 keep), Sec. 4.1: each
 * leaf's level target is its level plus its tag within [lmin, lmax]; with
 * `smooth` the target is first raised to the largest of its face and corner
 * neighbours' targets (Sec. 4.2).  A leaf whose target is above its level is
 * refined once; a family of four sibling leaves whose targets are all below
 * their level is replaced by its parent; then leaves are refined until the
 * set is 2:1 balanced over faces and corners (coarsening is not guaranteed).
 * Output sorted by (level, iy, ix).  Returns the count; out must hold 4*n
 * leaves (-1 on overflow). */
static int adapt_impl(const Orc *o, const signed char *tags, int smooth, int *out, int cap) {
    int cnt = 0;
    int *target = (int *)malloc(sizeof(int) * (o->n > 0 ? o->n : 1));
    int *T = (int *)malloc(sizeof(int) * (o->n > 0 ? o->n : 1));
    for (int k = 0; k < o->n; k++) {
        int t = o->lv[k].level + tags[k];
        if (t > o->lmax) t = o->lmax;
        if (t < o->lmin) t = o->lmin;
        target[k] = t;
        T[k] = t;
    }
    if (smooth) smooth_targets(o, target, T);
    char *done = (char *)calloc(o->n, 1);
    for (int k = 0; k < o->n; k++) {
        if (done[k]) continue;
        const OLeaf *L = &o->lv[k];
        if (T[k] < L->level && L->level > o->lmin) {
            int px = L->ix >> 1, py = L->iy >> 1, sib[4], ok = 1;
            for (int c = 0; c < 4; c++) {
                sib[c] = find_local(o, L->level, 2 * px + (c & 1), 2 * py + (c >> 1));
                if (sib[c] < 0 || !(T[sib[c]] < L->level)) ok = 0;
            }
            if (ok) {
                for (int c = 0; c < 4; c++) done[sib[c]] = 1;
                out[3 * cnt] = L->level - 1; out[3 * cnt + 1] = px; out[3 * cnt + 2] = py; cnt++;
                continue;
            }
        }
        done[k] = 1;
        if (T[k] > L->level && L->level < o->lmax) {
            for (int c = 0; c < 4; c++) {
                out[3 * cnt] = L->level + 1; out[3 * cnt + 1] = 2 * L->ix + (c & 1);
                out[3 * cnt + 2] = 2 * L->iy + (c >> 1); cnt++;
            }
        } else {
            out[3 * cnt] = L->level; out[3 * cnt + 1] = L->ix; out[3 * cnt + 2] = L->iy; cnt++;
        }
    }
    free(target);
    free(T);
    free(done);
    /* balance by refinement, using a temporary oracle for point queries */
    for (;;) {
        Orc tmp;
        memset(&tmp, 0, sizeof(tmp));
        tmp.mx = o->mx; tmp.n = cnt; tmp.lv = (OLeaf *)out;
        tmp.nbx = o->nbx; tmp.nby = o->nby; tmp.ori = o->ori;
        for (int s = 0; s < 4; s++) tmp.bc[s] = o->bc[s];
        index_leaves(&tmp);
        int nref = 0;
        int *ref = (int *)calloc(cnt, sizeof(int));
        for (int k = 0; k < cnt; k++) {
            ref[k] = !balanced_at(&tmp, &tmp.ph[k]);
            if (ref[k]) nref++;
        }
        free(tmp.hidx);
        free(tmp.ph);
        if (!nref) { free(ref); break; }
        int *nw = (int *)malloc(sizeof(int) * 3 * (cnt + 3 * nref));
        int c2 = 0;
        for (int k = 0; k < cnt; k++) {
            if (ref[k]) {
                for (int c = 0; c < 4; c++) {
                    nw[3 * c2] = out[3 * k] + 1; nw[3 * c2 + 1] = 2 * out[3 * k + 1] + (c & 1);
                    nw[3 * c2 + 2] = 2 * out[3 * k + 2] + (c >> 1); c2++;
                }
            } else {
                nw[3 * c2] = out[3 * k]; nw[3 * c2 + 1] = out[3 * k + 1]; nw[3 * c2 + 2] = out[3 * k + 2]; c2++;
            }
        }
        if (c2 > cap) { free(nw); free(ref); return -1; }
        memcpy(out, nw, sizeof(int) * 3 * c2);
        cnt = c2;
        free(nw); free(ref);
    }
    qsort(out, cnt, sizeof(int) * 3, cmp_leaf);
    return cnt;
}

int orc_adapt(const Orc *o, const signed char *tags, int *out, int cap) { return adapt_impl(o, tags, 0, out, cap); }
int orc_adapt_smooth(const Orc *o, const signed char *tags, int *out, int cap) {
    return adapt_impl(o, tags, 1, out, cap);
}

/* Replace the leaf set by new_leaves and transfer the solution: unchanged
 * leaves are copied, new children are interpolated from their parent with
 * the ghost-fill interpolation (parent ghosts must be valid), new parents are
 * the mean of their four children (Sec. 4.1).  Returns 0 or an error code. */
int orc_regrid(Orc *o, int n_new, const int *leaves_new) {
    int st = 0;
    Orc *nw = orc_create_brick(o->mx, o->m, o->eq, o->lim, o->bc, o->vel, o->vp, o->g, o->lmin, o->lmax, o->nbx,
                               o->nby, o->ori, n_new,
                         leaves_new, &st);
    if (st) { orc_destroy(nw); return st; }
    nw->map_alpha = o->map_alpha;
    int mx = o->mx;
    for (int k = 0; k < n_new; k++) {
        const OLeaf *L = &nw->lv[k];
        double *d = pat(nw, nw->q, k);
        int ko = find_local(o, L->level, L->ix, L->iy);
        if (ko >= 0) {
            memcpy(d, pat(o, o->q, ko), sizeof(double) * o->F * o->N * o->N);
            continue;
        }
        int kp = find_local(o, L->level - 1, L->ix >> 1, L->iy >> 1);
        if (kp >= 0) {
            double *s = pat(o, o->q, kp);
            int ox = (L->ix & 1) * (mx / 2), oy = (L->iy & 1) * (mx / 2);
            for (int f = 0; f < o->F; f++)
                for (int j = 0; j < mx; j++)
                    for (int i = 0; i < mx; i++) {
                        int ic = ox + i / 2, jc = oy + j / 2;
                        double dx = (i & 1) ? 1.0 : -1.0, dy = (j & 1) ? 1.0 : -1.0;
                        double c = *cell(o, s, f, ic, jc);
                        double sx = minmod(*cell(o, s, f, ic + 1, jc) - c, c - *cell(o, s, f, ic - 1, jc));
                        double sy = minmod(*cell(o, s, f, ic, jc + 1) - c, c - *cell(o, s, f, ic, jc - 1));
                        *cell(o, d, f, i, j) = c + 0.25 * (dx * sx + dy * sy);
                    }
            continue;
        }
        /* coarsened: all four children must be leaves of the old set */
        int kc[4];
        for (int c = 0; c < 4; c++) {
            kc[c] = find_local(o, L->level + 1, 2 * L->ix + (c & 1), 2 * L->iy + (c >> 1));
            if (kc[c] < 0) { orc_destroy(nw); return ERR_ARG; }
        }
        for (int f = 0; f < o->F; f++)
            for (int j = 0; j < mx; j++)
                for (int i = 0; i < mx; i++) {
                    int cx = i >= mx / 2, cy = j >= mx / 2;
                    int kf = kc[cx + 2 * cy];
                    double *s = pat(o, o->q, kf);
                    int fi = 2 * i - cx * mx, fj = 2 * j - cy * mx;
                    if (o->map_alpha == 0.0) {
                        *cell(o, d, f, i, j) = 0.25 * (*cell(o, s, f, fi, fj) + *cell(o, s, f, fi + 1, fj) +
                                                       *cell(o, s, f, fi, fj + 1) + *cell(o, s, f, fi + 1, fj + 1));
                    } else {
                        /* mapped grid: area-weighted mean of the four children's cells */
                        double a0 = cell_capacity(o, kf, fi, fj), a1 = cell_capacity(o, kf, fi + 1, fj);
                        double a2 = cell_capacity(o, kf, fi, fj + 1), a3 = cell_capacity(o, kf, fi + 1, fj + 1);
                        double m = a0 * *cell(o, s, f, fi, fj) + a1 * *cell(o, s, f, fi + 1, fj) +
                                   a2 * *cell(o, s, f, fi, fj + 1) + a3 * *cell(o, s, f, fi + 1, fj + 1);
                        *cell(o, d, f, i, j) = m / (a0 + a1 + a2 + a3);
                    }
                }
    }
    /* swap the new mesh in */
    free(o->lv); free(o->q); free(o->qold); free(o->qhat); free(o->hidx); free(o->ph);
    o->lv = nw->lv; o->q = nw->q; o->qold = nw->qold; o->qhat = nw->qhat; o->hidx = nw->hidx;
    o->ph = nw->ph; o->hcap = nw->hcap; o->n = nw->n;
    free(nw->ori);
    free(nw);
    return 0;
}

/* ------------------------------------------------------------------ */
/* tangent and adjoint of one uniform-level scalar step                 */
/* ------------------------------------------------------------------ */
/* Tangent: given the forward state q (interior, leaf order, ghosts filled
 * internally by copy) and a direction d (interior), return J d where J is the
 * Jacobian of  fill + advance  with the limiter branches frozen at q. */
void orc_tangent_step(Orc *o, int level, double t, double dt, const double *qin, const double *din,
                      double *dout) {
    int n = o->n, mx = o->mx;
    size_t psz = (size_t)o->N * o->N;
    /* forward state with ghosts */
    orc_set_interior(o, qin);
    orc_ghost_fill(o, level, level, 1.0);
    double *qf = (double *)malloc(sizeof(double) * n * psz);
    memcpy(qf, o->q, sizeof(double) * n * psz);
    /* direction with ghosts: the fill is linear when only copies occur */
    orc_set_interior(o, din);
    orc_ghost_fill(o, level, level, 1.0);
    int k;
#pragma omp parallel
    {
        Work w;
        work_alloc(&w, mx, o->m);
        double *tmp = (double *)malloc(sizeof(double) * psz);
#pragma omp for schedule(dynamic, 2)
        for (k = 0; k < n; k++) {
            adv_step(o, k, qf + k * psz, tmp, t, dt, &w, pat(o, o->q, k));
            for (int j = 0; j < mx; j++)
                for (int i = 0; i < mx; i++) dout[((size_t)k * mx + j) * mx + i] = *cell(o, tmp, 0, i, j);
        }
        free(tmp);
        work_free(&w);
    }
    free(qf);
}

/* Transpose of the tangent, written by hand: lam_out = (J_adv J_fill)^T lam_in.
 * The advance transpose scatters each interior cell's adjoint back through the
 * update, the edge fluxes, the limiter (frozen branch) and the differences
 * into a full patch-sized adjoint (interior + ghosts); the ghost-copy
 * transpose then adds every ghost cell's adjoint to the interior cell it was
 * copied from.  Only same-level copies are supported (uniform meshes). */
void orc_adjoint_step(Orc *o, int level, double t, double dt, const double *qin, const double *lin,
                      double *lout) {
    int n = o->n, mx = o->mx, m = o->m;
    size_t psz = (size_t)o->N * o->N;
    if (is_brick(o)) { o->err |= ERR_ARG; return; } /* one block of code 0 */
    orc_set_interior(o, qin);
    orc_ghost_fill(o, level, level, 1.0);
    double *abar = (double *)calloc(n * psz, sizeof(double)); /* adjoint of patch arrays */
    int k;
#pragma omp parallel
    {
        size_t E = (size_t)(o->N + 1);
        double *Ftb = (double *)malloc(sizeof(double) * E * E);
        double *Gtb = (double *)malloc(sizeof(double) * E * E);
#define EB(a, r, c) ((a)[((size_t)((r) + m)) * E + ((c) + m)])
#pragma omp for schedule(dynamic, 2)
        for (k = 0; k < n; k++) {
            const OLeaf *P = &o->lv[k];
            int l = P->level;
            double h = 1.0 / (mx << l), lam = dt / h, tm = t + 0.5 * dt;
            int gx = P->ix * mx, gy = P->iy * mx, oc = leaf_code(o, k);
            double *Q = pat(o, o->q, k);
            double *Ab = abar + k * psz;
            memset(Ftb, 0, sizeof(double) * E * E);
            memset(Gtb, 0, sizeof(double) * E * E);
#define QQ(i, j) (*cell(o, Q, 0, (i), (j)))
#define AB(i, j) (*cell(o, Ab, 0, (i), (j)))
            /* adjoint of the update: Qn = D - lam*fl - lam*df */
            double *Apxb = (double *)calloc(E * E, sizeof(double));
            double *Amxb = (double *)calloc(E * E, sizeof(double));
            double *Bpyb = (double *)calloc(E * E, sizeof(double));
            double *Bmyb = (double *)calloc(E * E, sizeof(double));
            for (int j = 0; j < mx; j++)
                for (int i = 0; i < mx; i++) {
                    double b = lin[((size_t)k * mx + j) * mx + i];
                    AB(i, j) += b;
                    EB(Apxb, j, i) -= lam * b; EB(Amxb, j, i + 1) -= lam * b;
                    EB(Bpyb, j, i) -= lam * b; EB(Bmyb, j + 1, i) -= lam * b;
                    EB(Ftb, j, i + 1) -= lam * b; EB(Ftb, j, i) += lam * b;
                    EB(Gtb, j + 1, i) -= lam * b; EB(Gtb, j, i) += lam * b;
                }
            /* adjoint of the y sweep (it ran second, so it is undone first) */
            for (int i = mx; i >= -1; i--)
                for (int j = mx; j >= 0; j--) {
                    double s_ = vel_v(o, oc, l, gx + i, gy + j, tm);
                    double upr = vel_u(o, oc, l, gx + i + 1, gy + j, tm), upl = vel_u(o, oc, l, gx + i, gy + j, tm);
                    double umr = vel_u(o, oc, l, gx + i + 1, gy + j - 1, tm), uml = vel_u(o, oc, l, gx + i, gy + j - 1, tm);
                    double Bpsb = -0.5 * lam * (upr > 0 ? upr : 0.0) * EB(Ftb, j, i + 1)
                                  - 0.5 * lam * (upl < 0 ? upl : 0.0) * EB(Ftb, j, i);
                    double Bmsb = -0.5 * lam * (umr > 0 ? umr : 0.0) * EB(Ftb, j - 1, i + 1)
                                  - 0.5 * lam * (uml < 0 ? uml : 0.0) * EB(Ftb, j - 1, i);
                    double Cb = 0.5 * EB(Gtb, j, i) - Bpsb + Bmsb;
                    double Bpb = EB(Bpyb, j, i) + Bpsb, Bmb = EB(Bmyb, j, i) + Bmsb;
                    double Vb = (s_ > 0 ? s_ : 0.0) * Bpb + (s_ < 0 ? s_ : 0.0) * Bmb;
                    double Vlb = fabs(s_) * (1.0 - lam * fabs(s_)) * Cb;
                    double V0 = QQ(i, j) - QQ(i, j - 1);
                    double Vu0 = s_ > 0 ? QQ(i, j - 1) - QQ(i, j - 2) : QQ(i, j + 1) - QQ(i, j);
                    int br = limiter_branch(o->lim, V0, Vu0);
                    double Vb2 = 0, Vub = 0;
                    if (br == 4) Vb2 = Vlb;
                    else if (br != 0) {
                        if (o->lim == LIM_MINMOD) { if (br == 2) Vb2 = Vlb; else Vub = Vlb; }
                        else if (br == 1) { Vb2 = 0.5 * Vlb; Vub = 0.5 * Vlb; }
                        else if (br == 2) Vb2 = 2.0 * Vlb;
                        else Vub = 2.0 * Vlb;
                    }
                    Vb += Vb2;
                    AB(i, j) += Vb; AB(i, j - 1) -= Vb;
                    if (s_ > 0) { AB(i, j - 1) += Vub; AB(i, j - 2) -= Vub; }
                    else { AB(i, j + 1) += Vub; AB(i, j) -= Vub; }
                }
            /* adjoint of the x sweep */
            for (int j = mx; j >= -1; j--)
                for (int i = mx; i >= 0; i--) {
                    double s_ = vel_u(o, oc, l, gx + i, gy + j, tm);
                    double vpu = vel_v(o, oc, l, gx + i, gy + j + 1, tm), vpd = vel_v(o, oc, l, gx + i, gy + j, tm);
                    double vmu = vel_v(o, oc, l, gx + i - 1, gy + j + 1, tm), vmd = vel_v(o, oc, l, gx + i - 1, gy + j, tm);
                    double Apsb = -0.5 * lam * (vpu > 0 ? vpu : 0.0) * EB(Gtb, j + 1, i)
                                  - 0.5 * lam * (vpd < 0 ? vpd : 0.0) * EB(Gtb, j, i);
                    double Amsb = -0.5 * lam * (vmu > 0 ? vmu : 0.0) * EB(Gtb, j + 1, i - 1)
                                  - 0.5 * lam * (vmd < 0 ? vmd : 0.0) * EB(Gtb, j, i - 1);
                    double Cb = 0.5 * EB(Ftb, j, i) - Apsb + Amsb;
                    double Apb = EB(Apxb, j, i) + Apsb, Amb = EB(Amxb, j, i) + Amsb;
                    double Wb = (s_ > 0 ? s_ : 0.0) * Apb + (s_ < 0 ? s_ : 0.0) * Amb;
                    double Wlb = fabs(s_) * (1.0 - lam * fabs(s_)) * Cb;
                    double W0 = QQ(i, j) - QQ(i - 1, j);
                    double Wu0 = s_ > 0 ? QQ(i - 1, j) - QQ(i - 2, j) : QQ(i + 1, j) - QQ(i, j);
                    int br = limiter_branch(o->lim, W0, Wu0);
                    double Wb2 = 0, Wub = 0;
                    if (br == 4) Wb2 = Wlb;
                    else if (br != 0) {
                        if (o->lim == LIM_MINMOD) { if (br == 2) Wb2 = Wlb; else Wub = Wlb; }
                        else if (br == 1) { Wb2 = 0.5 * Wlb; Wub = 0.5 * Wlb; }
                        else if (br == 2) Wb2 = 2.0 * Wlb;
                        else Wub = 2.0 * Wlb;
                    }
                    Wb += Wb2;
                    AB(i, j) += Wb; AB(i - 1, j) -= Wb;
                    if (s_ > 0) { AB(i - 1, j) += Wub; AB(i - 2, j) -= Wub; }
                    else { AB(i + 1, j) += Wub; AB(i, j) -= Wub; }
                }
            free(Apxb); free(Amxb); free(Bpyb); free(Bmyb);
#undef QQ
#undef AB
        }
        free(Ftb); free(Gtb);
#undef EB
    }
    /* transpose of the ghost copy: every ghost cell of leaf k was copied from
     * an interior cell of a same-level leaf; add its adjoint there */
    for (k = 0; k < n * mx * mx; k++) lout[k] = 0.0;
    for (k = 0; k < n; k++) {
        const OLeaf *P = &o->lv[k];
        int l = P->level, nl = mx << l;
        double *Ab = abar + k * psz;
        for (int j = -m; j < mx + m; j++)
            for (int i = -m; i < mx + m; i++) {
                double b = *cell(o, Ab, 0, i, j);
                if (!is_ghost(o, i, j)) {
                    lout[((size_t)k * mx + j) * mx + i] += b;
                    continue;
                }
                int I = wrap_axis(o, P->ix * mx + i, nl, 0, 1);
                int J = wrap_axis(o, P->iy * mx + j, nl, 2, 3);
                if (I < 0 || J < 0) continue;
                int kk = locate(o, l, I, J);
                if (kk < 0 || o->lv[kk].level != l) { o->err |= ERR_ARG; continue; }
                const OLeaf *L = &o->lv[kk];
                lout[((size_t)kk * mx + (J - L->iy * mx)) * mx + (I - L->ix * mx)] += b;
            }
    }
    free(abar);
}
