// fc_kernels.hip -- gfx950 kernels of the patch-based quadtree AMR path.
//
// Ghost filling.  Algorithm 1 of the paper (Sec. 2.2) materialises ghost
// data in four phases because its interpolation stencil reads the coarse
// grid's ghost cells, which must be copied/averaged first.  Here every ghost
// value is evaluated directly from patch *interiors*: copy (same size),
// eq. ghost_coarse averaging (finer neighbour), or eq. ghost_fine
// interpolation whose five coarse stencil values are themselves evaluated by
// copy/averaging.  Prop. 2.1 guarantees a stencil never needs a third level,
// so one gather pass reproduces the four phases, needs no ordering between
// patches and can run inside the advance kernel (the fused form).
//
// Advance.  One workgroup per patch stages the (mx+4)^2 tile in LDS and runs
// the unsplit wave-propagation step (Sec. 5 runs Clawpack's): x- and y-edge
// fluctuations, MC-limited second-order corrections, transverse propagation
// of the corrected fluctuations, conservative update; written in gather form
// so that no two threads accumulate into one location.
#include "fc_internal.h"

#include <math.h>

namespace {

constexpr int MB = 2;  // ghost layers used by the kernels

// element index of cell (i, j) (ghost-inclusive local indices) of field f of
// slot p; the store keeps a buffer below 2^32 doubles
__device__ __forceinline__ uint32_t qidx(int cap, int N, int f, int p, int i, int j) {
    return ((uint32_t)(f * cap + p) * N + (uint32_t)(j + MB)) * N + (uint32_t)(i + MB);
}

// The time-dependent part of a kernel's view of the store: which buffer holds
// each level's current state, and which level is read time-interpolated.
// Kept apart from the (read-only, kernel-argument) Ctx so that kernels that
// walk several level-steps never copy Ctx into private memory.
struct View {
    uint32_t curmask;
    int clevel;
    double alpha;
};

__device__ __forceinline__ View view_of(const Ctx &c) { return View{c.curmask, c.clevel, c.alpha}; }
__device__ __forceinline__ double *buf_of(const Ctx &c, const View &v, int l) {
    return ((v.curmask >> l) & 1u) ? c.q1 : c.q0;
}
__device__ __forceinline__ double *other_of(const Ctx &c, const View &v, int l) {
    return ((v.curmask >> l) & 1u) ? c.q0 : c.q1;
}

// State of level l at the fill time: current, or q_old + alpha (q - q_old)
// for the time-interpolated coarse level.
template <int MX>
__device__ __forceinline__ double read_state(const Ctx &c, const View &w, int p, int l, int i, int j, int f) {
    constexpr int N = MX + 2 * MB;
    const uint32_t k = qidx(c.cap, N, f, p, i, j);
    const bool b = (w.curmask >> l) & 1u;
    double v = (b ? c.q1 : c.q0)[k];
    if (l == w.clevel && w.alpha != 1.0) {
        const double vo = (b ? c.q0 : c.q1)[k];
        v = vo + w.alpha * (v - vo);
    }
    return v;
}

__device__ __forceinline__ double minmod(double a, double b) {
    return (a * b <= 0.0) ? 0.0 : (fabs(a) < fabs(b) ? a : b);
}

template <int MX>
__device__ __forceinline__ int region_rec(int i, int j) {
    const int rx = i < 0 ? 0 : (i >= MX ? 2 : 1);
    const int ry = j < 0 ? 0 : (j >= MX ? 2 : 1);
    if (ry == 1) return (rx == 0 ? 0 : 2) + (j >= MX / 2 ? 1 : 0);
    if (rx == 1) return (ry == 0 ? 4 : 6) + (i >= MX / 2 ? 1 : 0);
    return 8 + (rx == 2 ? 1 : 0) + (ry == 2 ? 2 : 0);
}

// Reflecting walls: mirror the index into the patch; the normal momentum of
// the shallow-water system changes sign.  Returns the sign factors.
template <int MX>
__device__ __forceinline__ void fold(int walls, int &i, int &j, double &su, double &sv) {
    su = 1.0; sv = 1.0;
    if (i < 0 && (walls & 1)) { i = -1 - i; su = -1.0; }
    else if (i >= MX && (walls & 2)) { i = 2 * MX - 1 - i; su = -1.0; }
    if (j < 0 && (walls & 4)) { j = -1 - j; sv = -1.0; }
    else if (j >= MX && (walls & 8)) { j = 2 * MX - 1 - j; sv = -1.0; }
}

template <int F>
__device__ __forceinline__ void apply_signs(double *v, double su, double sv) {
    if (F == 3) { v[1] *= su; v[2] *= sv; }
}

__device__ __forceinline__ int rec_kind(const NbrRec &r) { return r.type & 15; }
__device__ __forceinline__ int rec_walls(const NbrRec &r) { return (r.type >> 4) & 15; }

// The record's index transform (eq. transform): (I, J) = s A (i, j) + F,
// A from the orientation code in type bits 8-10 (bit 0 exchanges the two
// indices, bit 1 negates the first result, bit 2 the second), s = 1 for a
// same-size or coarse neighbour and 2 for the first of a fine neighbour's
// four cells.  Identity on one block: (i, j) + F.
__device__ __forceinline__ void rec_map(const NbrRec &r, int i, int j, int s, int &I, int &J) {
    const int o = r.type >> 8;
    int a = (o & 1) ? j : i, b = (o & 1) ? i : j;
    a = (o & 2) ? -a : a;
    b = (o & 4) ? -b : b;
    I = s * a + r.fx;
    J = s * b + r.fy;
}

// Capacity (cell area over h^2) of the level-l cell at global index (I, J)
// of a mapped grid, from the level's table (it depends on I + J only);
// indices wrap periodically.
__device__ __forceinline__ double capacity_at(const Ctx &c, int l, int n, int I, int J) {
    int k = (I + J + 1) % n;
    k = k < 0 ? k + n : k;
    return c.mk[l][k];
}

// eq. ghost_coarse on a mapped grid: the area-weighted mean of the four
// cells (i, j), (i+1, j), (i, j+1), (i+1, j+1) (values y0 .. y3) of the
// level-lf leaf in `slot` -- the areas, not the count, carry the mass.
template <int MX>
__device__ __forceinline__ double area_mean4(const Ctx &c, int slot, int lf, int i, int j, double y0, double y1,
                                             double y2, double y3) {
    const PatchInfo P = c.info[slot];
    const int n = MX << lf, I = P.ix * MX + i, J = P.iy * MX + j;
    const double a0 = capacity_at(c, lf, n, I, J), a1 = capacity_at(c, lf, n, I + 1, J);
    const double a2 = capacity_at(c, lf, n, I, J + 1), a3 = capacity_at(c, lf, n, I + 1, J + 1);
    return (a0 * y0 + a1 * y1 + a2 * y2 + a3 * y3) / (a0 + a1 + a2 + a3);
}

// eq. ghost_fine at local (i, j) of a level-l patch whose ghost region is
// covered by the coarse patch of `rec`: q_c + (1/4)(d_x s_x + d_y s_y), s the
// minmod of the one-sided differences on the coarse grid, d = +1 for the
// upper half.  The four stencil neighbours of the coarse cell are the coarse
// patch's interior or its ghost values (copy from its same-size neighbour,
// eq. ghost_coarse average of its fine neighbour, or its interior mirrored at
// a wall; Prop. 2.1 excludes a third level).  The coarse patch's walls come
// with the record, so the records of the regions the neighbours fall in are
// loaded at once, and then every value: two dependent rounds of loads, with
// no load behind a branch.
// PIPE: overlap the fields' loads (two fields' values live at once); off
// where the kernel's register budget is too small for that.  MAP: a mapped
// grid (fine neighbours averaged by area).
template <int MX, int F, bool PIPE = true, bool MAP = false>
__device__ __forceinline__ void coarse_interp(const Ctx &c, const View &w, int l, int i, int j, const NbrRec rec,
                                              double *v) {
    constexpr int N = MX + 2 * MB;
    int I, J;
    rec_map(rec, i, j, 1, I, J);  // fine-level index inside the coarse leaf, in its own indices
    const int ic = I >> 1, jc = J >> 1;
    const double dx = (I & 1) ? 1.0 : -1.0, dy = (J & 1) ? 1.0 : -1.0;
    const int C = rec.id, lc = l - 1, cw = rec_walls(rec);
    int ni[4] = {ic - 1, ic + 1, ic, ic}, nj[4] = {jc, jc, jc - 1, jc + 1};
    double su[4], sv[4];
    bool in[4];
    NbrRec nr[4];
#pragma unroll
    for (int n = 0; n < 4; n++) {
        fold<MX>(cw, ni[n], nj[n], su[n], sv[n]);
        in[n] = ni[n] >= 0 && ni[n] < MX && nj[n] >= 0 && nj[n] < MX;
        nr[n] = c.nbr[C * FC_NREC + (in[n] ? 0 : region_rec<MX>(ni[n], nj[n]))];
    }
    // the coarse level is read time-interpolated in a multirate fill
    const bool tint = lc == w.clevel && w.alpha != 1.0;
    const double *cur_c = buf_of(c, w, lc), *old_c = other_of(c, w, lc), *cur_f = buf_of(c, w, l);
    // per neighbour: one coarse cell (current, old) or four fine cells (at
    // +0, +1, +N, +N+1 from the first)
    uint32_t k[4];
    bool fine[4], bad[4];
    int fs[4], fi[4], fj[4];  // MAP: slot and first cell of a fine neighbour
#pragma unroll
    for (int n = 0; n < 4; n++) {
        const int kind = rec_kind(nr[n]);
        fine[n] = !in[n] && kind == NB_FINE;
        bad[n] = !in[n] && kind != NB_SAME && kind != NB_FINE;
        const int slot = (in[n] || bad[n]) ? C : nr[n].id;
        int ci, cj;
        rec_map(nr[n], ni[n], nj[n], fine[n] ? 2 : 1, ci, cj);
        ci = in[n] ? ni[n] : (bad[n] ? 0 : ci);
        cj = in[n] ? nj[n] : (bad[n] ? 0 : cj);
        fs[n] = slot;
        fi[n] = ci;
        fj[n] = cj;
        k[n] = qidx(c.cap, N, 0, slot, ci, cj);
        if (bad[n]) atomicOr(c.err, 2);
    }
    const uint32_t kc = qidx(c.cap, N, 0, C, ic, jc);
    const uint32_t plane = (uint32_t)c.cap * N * N;
    // the five stencil values of field f (centre, then xm, xp, ym, yp:
    // current and old value, or four fine cells)
    auto load = [&](int f, double (&x)[5][4]) {
        const uint32_t fo = f * plane;
        x[0][0] = cur_c[kc + fo];
        x[0][2] = old_c[kc + fo];
#pragma unroll
        for (int n = 0; n < 4; n++) {
            const double *b0 = (fine[n] ? cur_f : cur_c) + k[n] + fo, *b1 = (fine[n] ? cur_f : old_c) + k[n] + fo;
            const int d1 = fine[n] ? 1 : 0, dn = fine[n] ? N : 0;
            x[n + 1][0] = b0[0];
            x[n + 1][1] = b0[d1];
            x[n + 1][2] = b1[dn];
            x[n + 1][3] = b1[dn + d1];
        }
    };
    auto combine = [&](int f, const double (&x)[5][4]) {
        const double cc = tint ? x[0][2] + w.alpha * (x[0][0] - x[0][2]) : x[0][0];
        double nv[4];
#pragma unroll
        for (int n = 0; n < 4; n++) {
            const double *y = x[n + 1];
            double t;
            if constexpr (MAP)
                t = fine[n] ? area_mean4<MX>(c, fs[n], l, fi[n], fj[n], y[0], y[1], y[2], y[3])
                            : (tint ? y[2] + w.alpha * (y[0] - y[2]) : y[0]);
            else
                t = fine[n] ? 0.25 * (y[0] + y[1] + y[2] + y[3]) : (tint ? y[2] + w.alpha * (y[0] - y[2]) : y[0]);
            if (bad[n]) t = __builtin_nan("");
            if (F == 3 && f == 1) t *= su[n];
            if (F == 3 && f == 2) t *= sv[n];
            nv[n] = t;
        }
        const double sx = minmod(nv[1] - cc, cc - nv[0]);
        const double sy = minmod(nv[3] - cc, cc - nv[2]);
        return cc + 0.25 * (dx * sx + dy * sy);
    };
    double xa[5][4];
    if constexpr (F == 1) {
        load(0, xa);
        v[0] = combine(0, xa);
    } else if constexpr (!PIPE) {
#pragma unroll 1
        for (int f = 0; f < F; f++) {
            load(f, xa);
            v[f] = combine(f, xa);
        }
    } else {
        // software-pipelined over the fields: at most two fields' values are
        // live, so the three-field kernels keep their register budget, and
        // the next field's loads are in flight while one is combined
        double xb[5][4];
        load(0, xa);
        load(1, xb);
        v[0] = combine(0, xa);
        load(2, xa);
        v[1] = combine(1, xb);
        v[2] = combine(2, xa);
    }
}

// Ghost value at local (i, j) of patch p (level l) lying in region r of the
// frame (no wall folding): copy, eq. ghost_coarse average or eq. ghost_fine
// interpolation, as the region's neighbour record says.
template <int MX, int F, bool PIPE = true, bool MAP = false>
__device__ __forceinline__ void ghost_cell_rec(const Ctx &c, const View &w, int l, int i, int j, const NbrRec rec,
                                               double *v) {
    const int kind = rec_kind(rec);
    if (kind == NB_SAME) {
        int a, b;
        rec_map(rec, i, j, 1, a, b);
#pragma unroll
        for (int f = 0; f < F; f++) v[f] = read_state<MX>(c, w, rec.id, l, a, b, f);
    } else if (kind == NB_FINE) {
        int li, lj;
        rec_map(rec, i, j, 2, li, lj);
        if constexpr (MAP) {
#pragma unroll
            for (int f = 0; f < F; f++)
                v[f] = area_mean4<MX>(c, rec.id, l + 1, li, lj, read_state<MX>(c, w, rec.id, l + 1, li, lj, f),
                                      read_state<MX>(c, w, rec.id, l + 1, li + 1, lj, f),
                                      read_state<MX>(c, w, rec.id, l + 1, li, lj + 1, f),
                                      read_state<MX>(c, w, rec.id, l + 1, li + 1, lj + 1, f));
        } else {
#pragma unroll
            for (int f = 0; f < F; f++)
                v[f] = 0.25 * (read_state<MX>(c, w, rec.id, l + 1, li, lj, f) + read_state<MX>(c, w, rec.id, l + 1, li + 1, lj, f) +
                               read_state<MX>(c, w, rec.id, l + 1, li, lj + 1, f) +
                               read_state<MX>(c, w, rec.id, l + 1, li + 1, lj + 1, f));
        }
    } else if (kind == NB_COARSE) {
        coarse_interp<MX, F, PIPE, MAP>(c, w, l, i, j, rec, v);
    } else {
        atomicOr(c.err, 2);
#pragma unroll
        for (int f = 0; f < F; f++) v[f] = __builtin_nan("");
    }
}

template <int MX, int F, bool PIPE = true, bool MAP = false>
__device__ __forceinline__ void ghost_cell_r(const Ctx &c, const View &w, int p, int l, int i, int j, int r,
                                             double *v) {
    ghost_cell_rec<MX, F, PIPE, MAP>(c, w, l, i, j, c.nbr[p * FC_NREC + r], v);
}

// Ghost value of patch p (geometry P) at local (i, j): the result of
// Algorithm 1.
template <int MX, int F, bool PIPE = true, bool MAP = false>
__device__ __forceinline__ void ghost_cell_of(const Ctx &c, const View &w, int p, const PatchInfo &P, int i, int j,
                                              double *v) {
    const int l = P.level;
    double su, sv;
    fold<MX>(P.walls, i, j, su, sv);
    if (i >= 0 && i < MX && j >= 0 && j < MX) {
#pragma unroll
        for (int f = 0; f < F; f++) v[f] = read_state<MX>(c, w, p, l, i, j, f);
    } else {
        ghost_cell_r<MX, F, PIPE, MAP>(c, w, p, l, i, j, region_rec<MX>(i, j), v);
    }
    apply_signs<F>(v, su, sv);
}

template <int MX, int F, bool MAP = false>
__device__ void ghost_cell(const Ctx &c, const View &w, int p, int i, int j, double *v) {
    const PatchInfo P = c.info[p];
    ghost_cell_of<MX, F, true, MAP>(c, w, p, P, i, j, v);
}

// g-th cell of the ghost frame in region-major order: the eight face halves
// (MB x MX/2 cells each, numbered as region_rec numbers them), then the four
// MB x MB corners.  Consecutive g share a region and so a neighbour record.
// Branch-free: lanes of a wave fall in different regions, and a branch per
// region kind would run every kind on every wave.
template <int MX>
__device__ __forceinline__ void ghost_region_index(int g, int &i, int &j, int &r) {
    constexpr int H = MX / 2, HF = MB * H;
    // face halves: region rf, `across` cells from the patch edge, `along` it
    const int rf = g / HF, k = g % HF, along = (rf & 1) * H + k % H, across = k / H;
    const int ac = (rf & 2) ? MX + across : across - MB;  // upper (right) side for odd rf >> 1
    const bool xface = rf < 4;                            // left and right faces first
    // corners: MB x MB cells each, regions 8 .. 11
    const int kc = g - 8 * HF, rc = 8 + kc / (MB * MB), a = kc % MB, b = (kc / MB) % MB;
    const bool face = g < 8 * HF;
    i = face ? (xface ? ac : along) : ((rc & 1) ? MX + a : a - MB);
    j = face ? (xface ? along : ac) : ((rc & 2) ? MX + b : b - MB);
    r = face ? rf : rc;
}

// g-th ghost cell of the (MX+4)^2 frame: two bottom rows, two top rows, then
// the left/right pairs of every interior row.
template <int MX>
__device__ __forceinline__ void ghost_index(int g, int &i, int &j) {
    constexpr int N = MX + 2 * MB;
    if (g < MB * N) { j = g / N - MB; i = g % N - MB; return; }
    g -= MB * N;
    if (g < MB * N) { j = MX + g / N; i = g % N - MB; return; }
    g -= MB * N;
    j = g / (2 * MB);
    const int k = g % (2 * MB);
    i = k < MB ? k - MB : MX + k - MB;
}

// Morton index <-> quadrant coordinates (x on the even bits, y on the odd)
__device__ __forceinline__ uint32_t morton_spread(uint32_t x) {
    x &= 0xffffu;
    x = (x | (x << 8)) & 0x00ff00ffu;
    x = (x | (x << 4)) & 0x0f0f0f0fu;
    x = (x | (x << 2)) & 0x33333333u;
    return (x | (x << 1)) & 0x55555555u;
}
// Morton index of the neighbour (dx, dy) in {-1, 0, 1}^2 of quadrant m on a
// periodic level l < 16, by dilated-integer arithmetic on m's x bits (even)
// and y bits (odd) within the level's 2l bits: no interleaving per call.
// The six candidates are uniform over the workgroup; the caller selects.
__device__ __forceinline__ void morton_nbr(uint32_t m, int l, uint32_t &x0, uint32_t &xp, uint32_t &xm, uint32_t &y0,
                                           uint32_t &yp, uint32_t &ym) {
    const uint32_t win = (1u << (2 * l)) - 1u, ex = 0x55555555u & win, ey = 0xAAAAAAAAu & win;
    x0 = m & ex;
    y0 = m & ey;
    xp = ((x0 | ~ex) + 1u) & ex;  // carries pass the y bits; the top x bit wraps to 0
    xm = (x0 - 1u) & ex;          // borrows likewise; 0 wraps to the top
    yp = ((y0 | ~ey) + 2u) & ey;
    ym = (y0 - 2u) & ey;
}

__device__ __forceinline__ uint32_t morton_compact(uint32_t x) {
    x &= 0x55555555u;
    x = (x | (x >> 1)) & 0x33333333u;
    x = (x | (x >> 2)) & 0x0f0f0f0fu;
    x = (x | (x >> 4)) & 0x00ff00ffu;
    return (x | (x >> 8)) & 0x0000ffffu;
}

// XCD-aware block -> work item map: consecutive Morton patches go to one
// XCD (blocks are dispatched round-robin over the 8 XCDs), so neighbour
// reads hit that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int count) {
    const int x = b & 7, r = b >> 3;
    int base = 0;
    for (int k = 0; k < x; k++) base += (count - k + 7) >> 3;
    return base + r;
}

// ------------------------------------------------------------------------
// fill: materialise ghost values (per-level form)
// ------------------------------------------------------------------------
template <int MX, int F, bool MAP = false>
__global__ void __launch_bounds__(256) fill_kernel(Ctx c, int first) {
    constexpr int N = MX + 2 * MB, NG = N * N - MX * MX;
    const int p = first + blockIdx.x;
    const int l = c.info[p].level;
    const View w = view_of(c);
    double *out = buf_of(c, w, l);
    for (int g = threadIdx.x; g < NG; g += blockDim.x) {
        int i, j;
        ghost_index<MX>(g, i, j);
        double v[F];
        ghost_cell<MX, F, MAP>(c, w, p, i, j, v);
#pragma unroll
        for (int f = 0; f < F; f++) out[qidx(c.cap, N, f, p, i, j)] = v[f];
    }
}

// ------------------------------------------------------------------------
// scalar advection step
// ------------------------------------------------------------------------
template <int MX>
struct ScalarSmem {
    static constexpr int N = MX + 2 * MB;
    static constexpr int NP = N + 1;  // odd row strides: row- and column-wise lanes hit distinct banks
    static constexpr int S = MX + 1;
    double q[N * NP];                 // the tile; after the sweeps, the new interior (staged for the store)
    double tx[(MX + 2) * S];          // TX(i, j) = A+*_{i-1/2} + A-*_{i+1/2} at [(j+1) S + i], rows -1..MX
    double ty[(MX + 2) * S];          // TY(i, j) at [(i+1) S + j], columns -1..MX
    double ux[MX + 1], uy[MX + 2];    // u(e, j) = ux[e] * uy[j+1]
    double vy[MX + 1], vx[MX + 2];    // v(i, e) = vy[e] * vx[i+1]
    double red[16];
    unsigned long long cfl;           // the patch's Courant number (bits of a non-negative double)
};

// Cells per edge-sweep item: every interior line is split into MX/SEG
// segments and the x- and y-items of the interior lines fill at most NT
// threads; a segment of SEG cells computes its SEG+1 edges.
template <int MX, int NT>
constexpr int scalar_seg() {
    int sg = 2 * MX * MX / NT;
    if (sg < 4) sg = 4;
    if (sg > MX) sg = MX;
    return sg;
}

// A streaming store of two doubles (16-byte aligned): the step's output is
// not read again within the launch, so it need not stay dirty in the XCD's
// L2 until the end-of-kernel write-back (the host decides where it pays).
typedef double dpair __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store_stream2(double *p, double a, double b) {
    dpair v;
    v.x = a;
    v.y = b;
    __builtin_nontemporal_store(v, reinterpret_cast<dpair *>(p));
}

__device__ __forceinline__ double posp(double a) { return a > 0.0 ? a : 0.0; }
__device__ __forceinline__ double negp(double a) { return a < 0.0 ? a : 0.0; }

// Second-order correction C = |s| (1 - lam |s|) W~ of one wave W, with W~
// the limited wave and Wu its upwind neighbour.  Limiter codes: 0 MC,
// 1 Lax-Wendroff (no limiting), 2 first order, 3 minmod.  The MC value
// phi(theta) W, theta = Wu / W, is formed without the division: zero unless
// W Wu > 0, else sign(W) min((|W| + |Wu|) / 2, 2 |W|, 2 |Wu|).
template <int LIM>
__device__ __forceinline__ double correction(double W, double Wu, double as, double lam) {
    if constexpr (LIM == 2) return 0.0;
    const double k = as - (lam * as) * as;
    if constexpr (LIM == 1) return k * W;
    const double aw = fabs(W), au = fabs(Wu);
    double m;
    if constexpr (LIM == 3) m = fmin(aw, au);
    else m = fmin(0.5 * (aw + au), 2.0 * fmin(aw, au));
    return (W * Wu > 0.0) ? k * copysign(m, W) : 0.0;  // k < 0 where lam |s| > 1
}

// Maximum of a non-negative double over a wave64 with DPP row operations
// (no trip through LDS): shifts by 1, 2, 4 and 8 within each row of 16 lanes,
// then row broadcasts of lane 15 and lane 31.  Lanes whose source lies
// outside the row keep their own value.  Lane 63 ends with the maximum.
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_max_step(double v) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    const int lo2 = __builtin_amdgcn_update_dpp(lo, lo, CTRL, ROWS, 0xf, false);
    const int hi2 = __builtin_amdgcn_update_dpp(hi, hi, CTRL, ROWS, 0xf, false);
    return fmax(v, __hiloint2double(hi2, lo2));
}
__device__ __forceinline__ double wave_max_last_lane(double v) {
    v = dpp_max_step<0x111, 0xf>(v);  // row_shr:1
    v = dpp_max_step<0x112, 0xf>(v);  // row_shr:2
    v = dpp_max_step<0x114, 0xf>(v);  // row_shr:4
    v = dpp_max_step<0x118, 0xf>(v);  // row_shr:8
    v = dpp_max_step<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_max_step<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// Velocity factors of a patch into LDS, at the mid-step time t + dt/2 with
// t = *tdev + t when tdev is given (threads k0 .. k0+MX+1 do the work;
// blockDim >= k0 + MX + 2).  Two parts: fetch_velocity issues the loads (the
// device-resident start time first), put_velocity evaluates c(t) and writes
// LDS; a caller that issues its tile loads between the two lets the cosine
// run while they are in flight (a wave's loads retire in order, so a wait
// for a load issued after the tile would wait for the whole tile).
struct VelRegs {
    double tv, ex, ey, cy, cx;
};

template <int MX>
__device__ __forceinline__ void fetch_velocity(const Ctx &c, int l, int gx, int gy, const double *tdev, int k0,
                                               VelRegs &v) {
    const int k = (int)threadIdx.x - k0;
    v.tv = v.ex = v.ey = v.cy = v.cx = 0.0;
    if (c.velocity == 2 && k >= 0 && k < MX + 2) {
        if (tdev) {
            // a per-lane zero the compiler cannot see through keeps this a
            // vector load: a scalar one would be waited on together with
            // the kernel arguments, ahead of the first tile loads
            int zero;
            asm volatile("v_mov_b32 %0, 0" : "=v"(zero));
            v.tv = tdev[zero];
        }
        const int n = MX << l;
        const double *vt = c.vt[l];
        if (k <= MX) {
            v.ex = vt[vt_ex(n, MB) + gx + k];
            v.ey = vt[vt_ey(n, MB) + gy + k];
        }
        v.cy = vt[vt_cy(n, MB) + gy + k - 1];
        v.cx = vt[vt_cx(n, MB) + gx + k - 1];
    }
}

//
// The same wave also finds the patch's largest edge speed.  The velocity is
// a product of one factor per axis, u(e, j) = ux(e) uy(j), and rounding a
// product of non-negative numbers is monotone in each, so the largest |u|
// over the x-edges of the interior rows is max|ux| max|uy| exactly
// (likewise for v).  The factors are at hand here, while the tile's loads
// are still in flight; s.cfl receives the unscaled maximum.  (The lanes
// k0 .. k0+MX+1 lie in one wave for every launch variant.)  A constant
// velocity is given in the brick's directions; `orient` (the block's
// orientation code) turns it into the patch's own: a reversed brick
// direction negates its component, exchanged directions exchange them.
template <int MX>
__device__ __forceinline__ void put_velocity(const Ctx &c, ScalarSmem<MX> &s, double t, double dt,
                                             const double *tdev, int k0, const VelRegs &v, int orient = 0) {
    const int k = (int)threadIdx.x - k0;
    if ((int)threadIdx.x / 64 != k0 / 64) return;
    double ux = 0.0, uy = 0.0, vy = 0.0, vx = 0.0;
    if (k >= 0 && k < MX + 2) {
        if (c.velocity == 2) {
            if (tdev) t = v.tv + t;
            const double tm = t + 0.5 * dt;
            const double ct = cos(M_PI * (tm * c.vel_invT));
            ux = v.ex; vy = v.ey;
            uy = v.cy * ct;
            vx = -(v.cx * ct);
        } else {
            const double bu = (orient & 2) ? -c.vel_u : c.vel_u, bv = (orient & 4) ? -c.vel_v : c.vel_v;
            ux = (orient & 1) ? bv : bu;
            vy = (orient & 1) ? bu : bv;
            uy = 1.0;
            vx = 1.0;
        }
        if (k <= MX) { s.ux[k] = ux; s.vy[k] = vy; }
        s.uy[k] = uy;
        s.vx[k] = vx;
    }
    const bool in_e = k >= 0 && k <= MX, in_c = k >= 1 && k <= MX;
    const double ax = wave_max_last_lane(in_e ? fabs(ux) : 0.0), ay = wave_max_last_lane(in_e ? fabs(vy) : 0.0);
    const double bx = wave_max_last_lane(in_c ? fabs(uy) : 0.0), by = wave_max_last_lane(in_c ? fabs(vx) : 0.0);
    if ((threadIdx.x & 63) == 63) s.cfl = (unsigned long long)__double_as_longlong(fmax(ax * bx, ay * by));
}

template <int MX>
__device__ void load_velocity(const Ctx &c, ScalarSmem<MX> &s, int l, int gx, int gy, double t, double dt,
                              const double *tdev, int k0, int orient = 0) {
    VelRegs v;
    fetch_velocity<MX>(c, l, gx, gy, tdev, k0, v);
    put_velocity<MX>(c, s, t, dt, tdev, k0, v, orient);
}

// Upwind side of a line.  Every velocity this library advects with is a
// product of a factor along the line (ux for rows, vy for columns) and one
// across it, and the factor along the line has one sign over the line: the
// swirl's ex, ey = sin^2 >= 0, a constant velocity is constant.  So the sign
// of the across factor (swirl) or of the product at the first edge (constant
// velocity) gives every edge's: all s >= 0 (POS) or all s <= 0.  The sweeps
// below take that side as a template argument instead of selecting per edge;
// at s = 0 either side gives a zero correction and zero fluctuations, so the
// results agree with a per-edge choice up to the sign of zeros.
__device__ __forceinline__ bool line_pos(int velocity, double ve0, double vl) {
    return (velocity == 2 ? vl : ve0 * vl) >= 0.0;
}

// One segment of one interior line: edges e0 .. e0+SEG (edge e lies between
// cells e-1 and e of the line), cells e0 .. e0+SEG-1.  DIR 0: x-edges of row
// `line`; DIR 1: y-edges of column `line`.  Writes TX (TY) of the cells and
// returns the line's partial update of each cell in R:
//   rows     Rx = Q - lam TX + lam/2 (C_{i+1/2} - C_{i-1/2}),
//   columns  Ry = lam/2 (C_{j+1/2} - C_{j-1/2}) - lam TY.
// POS: every edge speed of the line is >= 0 (else <= 0): the upwind wave is
// the previous (next) edge's, A+ W = s W and A- W = 0 (A+ W = 0, A- W = s W).
template <int MX, int SEG, int LIM, int DIR, bool POS>
__device__ __forceinline__ void sweep_side(ScalarSmem<MX> &s, int line, int e0, double lam, double (&R)[SEG]) {
    constexpr int NP = ScalarSmem<MX>::NP, S = ScalarSmem<MX>::S;
    constexpr int STR = DIR == 0 ? 1 : NP;
    const double *qp = DIR == 0 ? &s.q[(line + MB) * NP + MB + e0 - 2] : &s.q[(MB + e0 - 2) * NP + line + MB];
    const double *ve = DIR == 0 ? &s.ux[e0] : &s.vy[e0];
    const double vl = DIR == 0 ? s.uy[line + 1] : s.vx[line + 1];
    double q[SEG + 4];
#pragma unroll
    for (int k = 0; k < SEG + 4; k++) q[k] = qp[k * STR];
    double aprev = 0.0, cprev = 0.0;
#pragma unroll
    for (int k = 0; k <= SEG; k++) {  // edge e0 + k, between q[k+1] and q[k+2]
        const double u = ve[k] * vl;
        const double W = q[k + 2] - q[k + 1];
        const double Wu = POS ? q[k + 1] - q[k] : q[k + 3] - q[k + 2];
        const double C = correction<LIM>(W, Wu, POS ? u : -u, lam);
        const double aps = POS ? u * W - C : -C;
        const double ams = POS ? C : u * W + C;
        if (k > 0) {  // cell e0 + k - 1
            const int cc = e0 + k - 1;
            const double T = aprev + ams;
            if (DIR == 0) {
                s.tx[(line + 1) * S + cc] = T;
                R[k - 1] = q[k + 1] - lam * T + (0.5 * lam) * (C - cprev);
            } else {
                s.ty[(line + 1) * S + cc] = T;
                R[k - 1] = (0.5 * lam) * (C - cprev) - lam * T;
            }
        }
        aprev = aps;
        cprev = C;
    }
}

template <int MX, int SEG, int LIM, int DIR>
__device__ __forceinline__ void sweep_segment(ScalarSmem<MX> &s, int line, int e0, double lam, bool pos,
                                              double (&R)[SEG]) {
    if (pos) sweep_side<MX, SEG, LIM, DIR, true>(s, line, e0, lam, R);
    else sweep_side<MX, SEG, LIM, DIR, false>(s, line, e0, lam, R);
}

// The same for a line outside the interior (row -1 or MX: DIR 0, column -1
// or MX: DIR 1), TX (TY) only.  Direction-generic (per-lane stride and base)
// so that a wave holding both kinds takes one path.
template <int MX, int SEG, int LIM, bool POS>
__device__ __forceinline__ void outer_side(ScalarSmem<MX> &s, int dir, int line, int e0, double lam) {
    constexpr int NP = ScalarSmem<MX>::NP, S = ScalarSmem<MX>::S;
    const int str = dir == 0 ? 1 : NP;
    const double *qp = dir == 0 ? &s.q[(line + MB) * NP + MB + e0 - 2] : &s.q[(MB + e0 - 2) * NP + line + MB];
    const double *ve = dir == 0 ? &s.ux[e0] : &s.vy[e0];
    const double vl = dir == 0 ? s.uy[line + 1] : s.vx[line + 1];
    double *to = (dir == 0 ? s.tx : s.ty) + (line + 1) * S + e0 - 1;
    double q[SEG + 4];
#pragma unroll
    for (int k = 0; k < SEG + 4; k++) q[k] = qp[k * str];
    double aprev = 0.0;
#pragma unroll
    for (int k = 0; k <= SEG; k++) {
        const double u = ve[k] * vl;
        const double W = q[k + 2] - q[k + 1];
        const double Wu = POS ? q[k + 1] - q[k] : q[k + 3] - q[k + 2];
        const double C = correction<LIM>(W, Wu, POS ? u : -u, lam);
        const double ams = POS ? C : u * W + C;
        if (k > 0) to[k] = aprev + ams;
        aprev = POS ? u * W - C : -C;
    }
}

template <int MX, int SEG, int LIM>
__device__ __forceinline__ void sweep_outer(ScalarSmem<MX> &s, int velocity, int dir, int line, int e0, double lam) {
    const double ve0 = dir == 0 ? s.ux[e0] : s.vy[e0];
    const double vl = dir == 0 ? s.uy[line + 1] : s.vx[line + 1];
    if (line_pos(velocity, ve0, vl)) outer_side<MX, SEG, LIM, true>(s, dir, line, e0, lam);
    else outer_side<MX, SEG, LIM, false>(s, dir, line, e0, lam);
}

// Final update of a cell, as two direction parts:
//   Q_new = [Rx + lam^2/2 (TF_{i+1/2} - TF_{i-1/2})] + [Ry + lam^2/2 (TG_{j+1/2} - TG_{j-1/2})]
// with TF(e) = u+ TY(e-1) + u- TY(e) on x-edges and TG(e) = v+ TX(e-1) +
// v- TX(e) on y-edges (one term, on the line's upwind side).  Each item adds
// the transverse term of its own line's edges, evaluated once per edge: the
// x-items form the first bracket for their row segment, the y-items the
// second for their column segment.
template <int MX, int SEG>
__device__ __forceinline__ void part_row(const ScalarSmem<MX> &s, int j, int e0, double lam, bool pos,
                                         double (&R)[SEG]) {
    constexpr int S = ScalarSmem<MX>::S;
    const double uyj = s.uy[j + 1];
    double ty[SEG + 2];
#pragma unroll
    for (int k = 0; k < SEG + 2; k++) ty[k] = s.ty[(e0 + k) * S + j];  // TY(e0 - 1 + k, j)
    double tf[SEG + 1];
#pragma unroll
    for (int k = 0; k <= SEG; k++) tf[k] = (s.ux[e0 + k] * uyj) * (pos ? ty[k] : ty[k + 1]);
    const double hl2 = 0.5 * lam * lam;
#pragma unroll
    for (int k = 0; k < SEG; k++) R[k] = R[k] + hl2 * (tf[k + 1] - tf[k]);
}

template <int MX, int SEG>
__device__ __forceinline__ void part_col(const ScalarSmem<MX> &s, int i, int e0, double lam, bool pos,
                                         double (&R)[SEG]) {
    constexpr int S = ScalarSmem<MX>::S;
    const double vxi = s.vx[i + 1];
    double tx[SEG + 2];
#pragma unroll
    for (int k = 0; k < SEG + 2; k++) tx[k] = s.tx[(e0 + k) * S + i];  // TX(i, e0 - 1 + k)
    double tg[SEG + 1];
#pragma unroll
    for (int k = 0; k <= SEG; k++) tg[k] = (s.vy[e0 + k] * vxi) * (pos ? tx[k] : tx[k + 1]);
    const double hl2 = 0.5 * lam * lam;
#pragma unroll
    for (int k = 0; k < SEG; k++) R[k] = R[k] + hl2 * (tg[k + 1] - tg[k]);
}

// One step on patch p of level l: stage its tile, compute, write the new
// interior into the level's other buffer.  FUSED: ghosts evaluated on the fly
// instead of read from the patch's own ghost cells.
//   Edge sweeps: one item per (line, segment); every item keeps its
//   direction's partial sums in registers and, after the barrier, adds its
//   transverse term to them.
// Arrays of a uniform periodic level in input-leaf order (the form the
// adjoint's recomputation steps through): [nleaves][mx][mx].
struct LeafIO {
    const double *qin;
    double *qout;
    const int32_t *leaf_of_slot;
};

// The sweeps of one limiter (work items as in advance_scalar_lim).
template <int MX, int NT, int LIM, int SEG>
__device__ __forceinline__ void scalar_sweeps(ScalarSmem<MX> &s, int tid, bool xs, bool ys, int line, int e0,
                                              double lam, bool pos, int velocity, double (&R)[SEG]) {
    constexpr int NI = MX * (MX / SEG);
    constexpr int SO = 2, NO = 4 * (MX / SO);
    constexpr int GT0 = (NT - 2 * NI >= NO) ? 2 * NI : NI;
    if (xs) sweep_segment<MX, SEG, LIM, 0>(s, line, e0, lam, pos, R);
    else if (ys) sweep_segment<MX, SEG, LIM, 1>(s, line, e0, lam, pos, R);
    if (tid >= GT0 && tid < GT0 + NO) {  // rows -1, MX and columns -1, MX: TX, TY only
        const int k = tid - GT0, g = k / (MX / SO);
        sweep_outer<MX, SO, LIM>(s, velocity, g >> 1, (g & 1) ? MX : -1, (k % (MX / SO)) * SO, lam);
    }
}

// LEAF: read the step's input from io->qin and write its result to io->qout
// instead of the store's buffers (uniform periodic level: every ghost value
// is a same-size copy); the arithmetic is the same code either way.
// The limiter (c.lim) selects the sweeps only: the load and gather before
// them and the transverse terms and the store after them are one code path,
// so that no value loaded ahead is held across four copies of the kernel.
// SEGC: cells per sweep segment (0: the shortest that fits, scalar_seg).
template <int MX, int NT, bool FUSED, bool LEAF = false, int SEGC = 0>
__device__ __forceinline__ void advance_scalar_lim(const Ctx &c, const View &w, ScalarSmem<MX> &s, int p, int lev,
                                                   double t, double dt, const double *tdev,
                                                   const unsigned long long *slot, double &cfl,
                                                   const LeafIO *io = nullptr) {
    constexpr int N = MX + 2 * MB, NP = ScalarSmem<MX>::NP;
    // Work split (items = line segments): threads [0, NI) sweep the interior
    // rows, [NI, 2 NI) the interior columns; each half of either set covers
    // one half of the patch.  After the sweeps every item adds its
    // direction's transverse term and parks its part in LDS; the store sums
    // the row and column parts of each cell.  The four
    // outer lines are cut into segments of two cells, one per thread of the
    // lower-half column items (or of idle threads), so that no wave carries a
    // long extra chain into the barrier; the odd ghost cells and c(t) go to
    // the same threads.
    constexpr int SEG = SEGC ? SEGC : scalar_seg<MX, NT>(), NSEG = MX / SEG, NI = MX * NSEG, HI = NI / 2;
    constexpr int SO = 2, NO = 4 * (MX / SO);  // outer-line segment length and item count
    constexpr int GT0 = (NT - 2 * NI >= NO) ? 2 * NI : NI;  // first thread of the outer-line items
    static_assert(2 * NI <= NT && NSEG % 2 == 0, "interior items must fit one pass, in two halves");
    static_assert(GT0 + NO <= NT, "outer-line items must fit one pass");
    static_assert(NI + MX + 2 <= NT, "velocity factors are loaded by threads NI .. NI+MX+1");
    const int tid = threadIdx.x;
    // The loads that depend only on the slot (interior, neighbour records)
    // are issued before the patch record arrives, so that the ghost values
    // wait on one memory round trip after them, not two.
    const int l = lev >= 0 ? lev : c.info[p].level;
    const double lam = dt * (double)(MX << l);  // dt / h, exact: h = 1 / (MX 2^l)
    const double *in = buf_of(c, w, l);
    double *out = other_of(c, w, l);
    const size_t base = (size_t)p * N * N;
    // rows are 16-byte aligned (N and MB even): two cells per load
    if constexpr (LEAF) {
        // A complete periodic level: every neighbour's slot follows from the
        // Morton index.  Each thread loads all its leaf indices, then all its
        // values (indices past the end clamped, so no load waits behind a
        // branch), then writes LDS: two dependent memory round trips.
        constexpr int NG = N * N - MX * MX;
        constexpr int NV = (MX * MX / 2 + NT - 1) / NT, NGH = (NG + NT - 1) / NT;
        const uint32_t m = (uint32_t)(p - c.lstart[l]);
        const int ix = (int)morton_compact(m), iy = (int)morton_compact(m >> 1), wrap = (1 << l) - 1;
        auto side = [](int i) { return i < 0 ? -1 : (i >= MX ? 1 : 0); };
        const int self = io->leaf_of_slot[p];
        int gi[NGH], gj[NGH], gl[NGH];
#pragma unroll
        for (int v = 0; v < NGH; v++) {
            int r;
            ghost_region_index<MX>(min(tid + v * NT, NG - 1), gi[v], gj[v], r);
            const int dx = side(gi[v]), dy = side(gj[v]);
            gl[v] = io->leaf_of_slot[c.lstart[l] + (int)(morton_spread((uint32_t)((ix + dx) & wrap)) |
                                                         (morton_spread((uint32_t)((iy + dy) & wrap)) << 1))];
        }
        const double *qi = io->qin + (size_t)self * MX * MX;
        double2 iv[NV];
#pragma unroll
        for (int v = 0; v < NV; v++)
            iv[v] = *reinterpret_cast<const double2 *>(qi + 2 * min(tid + v * NT, MX * MX / 2 - 1));
        double gv[NGH];
#pragma unroll
        for (int v = 0; v < NGH; v++) {
            const int dx = side(gi[v]), dy = side(gj[v]);
            gv[v] = io->qin[(size_t)gl[v] * MX * MX + (gj[v] - dy * MX) * MX + gi[v] - dx * MX];
        }
        load_velocity<MX>(c, s, l, ix * MX, iy * MX, t, dt, nullptr, NI);
#pragma unroll
        for (int v = 0; v < NV; v++) {
            const int k = tid + v * NT, i = 2 * (k % (MX / 2)), j = k / (MX / 2);
            if (k < MX * MX / 2) {
                s.q[(j + MB) * NP + i + MB] = iv[v].x;
                s.q[(j + MB) * NP + i + MB + 1] = iv[v].y;
            }
        }
#pragma unroll
        for (int v = 0; v < NGH; v++)
            if (tid + v * NT < NG) s.q[(gj[v] + MB) * NP + gi[v] + MB] = gv[v];
    } else if (!FUSED) {
        const PatchInfo P = c.info[p];
        load_velocity<MX>(c, s, l, P.ix * MX, P.iy * MX, t, dt, tdev, NI, P.walls >> 8);
        for (int k = tid; k < N * N / 2; k += NT) {
            const int i = 2 * (k % (N / 2)), j = k / (N / 2);
            const double2 v = *reinterpret_cast<const double2 *>(&in[base + j * N + i]);
            s.q[j * NP + i] = v.x;
            s.q[j * NP + i + 1] = v.y;
        }
        if (slot && tid == 0) s.red[15] = __longlong_as_double((long long)*slot);
    } else {
        constexpr int NG = N * N - MX * MX;
        constexpr int NV = (MX * MX / 2 + NT - 1) / NT, NGH = (NG + NT - 1) / NT;
        // A complete periodic level: every neighbour is a same-level patch
        // whose slot follows from the Morton index, so no record is read and
        // all loads of the step leave at once, the velocity's first.
        const bool complete = lev >= 0 && ((c.complete >> lev) & 1u);
        const uint32_t m = (uint32_t)(p - c.lstart[l]);
        const int ix = (int)morton_compact(m), iy = (int)morton_compact(m >> 1);
        VelRegs vr;
        double2 iv[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) {
            const int k = tid + v * NT, i = 2 * (k % (MX / 2)), j = k / (MX / 2);
            if (k < MX * MX / 2) iv[v] = *reinterpret_cast<const double2 *>(&in[base + (j + MB) * N + i + MB]);
        }
        const int g0 = (tid + NT - NI) % NT;  // the odd ghost cells go to a lightly loaded wave
        if (complete) {
            uint32_t mx0, mxp, mxm, my0, myp, mym;
            morton_nbr(m, l, mx0, mxp, mxm, my0, myp, mym);
            double gv[NGH];
            int gi[NGH], gj[NGH];
#pragma unroll
            for (int v = 0; v < NGH; v++) {
                int r;
                gi[v] = gj[v] = 0;
                if (g0 + v * NT < NG) {
                    ghost_region_index<MX>(g0 + v * NT, gi[v], gj[v], r);
                    const int dx = gi[v] < 0 ? -1 : (gi[v] >= MX ? 1 : 0), dy = gj[v] < 0 ? -1 : (gj[v] >= MX ? 1 : 0);
                    const uint32_t nx = dx > 0 ? mxp : (dx < 0 ? mxm : mx0);
                    const uint32_t ny = dy > 0 ? myp : (dy < 0 ? mym : my0);
                    const uint32_t q = (uint32_t)c.lstart[l] + (nx | ny);
                    gv[v] = in[(size_t)q * N * N + (size_t)((gj[v] - dy * MX + MB) * N + gi[v] - dx * MX + MB)];
                }
            }
            const double sold = (slot && tid == NT - 1) ? __longlong_as_double((long long)*slot) : 0.0;
            // the velocity factors last: held from the start, they would
            // outlast the ghost loads' registers and push the kernel past
            // the register budget of five workgroups per CU
            fetch_velocity<MX>(c, l, ix * MX, iy * MX, tdev, NI, vr);
            put_velocity<MX>(c, s, t, dt, tdev, NI, vr);
            if (slot && tid == NT - 1) s.red[15] = sold;
#pragma unroll
            for (int v = 0; v < NV; v++) {
                const int k = tid + v * NT, i = 2 * (k % (MX / 2)), j = k / (MX / 2);
                if (k < MX * MX / 2) {
                    s.q[(j + MB) * NP + i + MB] = iv[v].x;
                    s.q[(j + MB) * NP + i + MB + 1] = iv[v].y;
                }
            }
#pragma unroll
            for (int v = 0; v < NGH; v++)
                if (g0 + v * NT < NG) s.q[(gj[v] + MB) * NP + gi[v] + MB] = gv[v];
        } else {
            int gi[NGH], gj[NGH];
            NbrRec gr[NGH];
#pragma unroll
            for (int v = 0; v < NGH; v++) {
                int r = 0;
                gi[v] = gj[v] = 0;
                if (g0 + v * NT < NG) {
                    ghost_region_index<MX>(g0 + v * NT, gi[v], gj[v], r);
                    gr[v] = c.nbr[p * FC_NREC + r];
                }
            }
            // the CFL slot's old value (read by the workgroup's last thread, parked
            // in LDS so that no register holds it across the step)
            const double sold = (slot && tid == NT - 1) ? __longlong_as_double((long long)*slot) : 0.0;
            const PatchInfo P = c.info[p];
            load_velocity<MX>(c, s, l, P.ix * MX, P.iy * MX, t, dt, tdev, NI, P.walls >> 8);
            if (slot && tid == NT - 1) s.red[15] = sold;
#pragma unroll
            for (int v = 0; v < NV; v++) {
                const int k = tid + v * NT, i = 2 * (k % (MX / 2)), j = k / (MX / 2);
                if (k < MX * MX / 2) {
                    s.q[(j + MB) * NP + i + MB] = iv[v].x;
                    s.q[(j + MB) * NP + i + MB + 1] = iv[v].y;
                }
            }
            if ((P.walls & 15) == 0) {
#pragma unroll
                for (int v = 0; v < NGH; v++) {
                    if (g0 + v * NT < NG) {
                        double val[1];
                        ghost_cell_rec<MX, 1>(c, w, l, gi[v], gj[v], gr[v], val);
                        s.q[(gj[v] + MB) * NP + gi[v] + MB] = val[0];
                    }
                }
            } else {
                for (int g = g0; g < NG; g += NT) {
                    int i, j;
                    ghost_index<MX>(g, i, j);
                    double val[1];
                    ghost_cell<MX, 1>(c, w, p, i, j, val);
                    s.q[(j + MB) * NP + i + MB] = val[0];
                }
            }
        }
    }
    __syncthreads();
    double R[SEG];
    int line = 0, e0 = 0;
    const bool xs = tid < NI, ys = !xs && tid < 2 * NI;
    const int half = (xs ? tid : tid - NI) / HI, r = (xs ? tid : tid - NI) % HI;
    bool pos = true;
    if (xs) {
        line = half * (MX / 2) + r % (MX / 2);
        e0 = (r / (MX / 2)) * SEG;
        pos = line_pos(c.velocity, s.ux[e0], s.uy[line + 1]);
    } else if (ys) {
        line = r % MX;
        e0 = (half * (NSEG / 2) + r / MX) * SEG;
        pos = line_pos(c.velocity, s.vy[e0], s.vx[line + 1]);
    }
    switch (c.lim) {
        case 1: scalar_sweeps<MX, NT, 1, SEG>(s, tid, xs, ys, line, e0, lam, pos, c.velocity, R); break;
        case 2: scalar_sweeps<MX, NT, 2, SEG>(s, tid, xs, ys, line, e0, lam, pos, c.velocity, R); break;
        case 3: scalar_sweeps<MX, NT, 3, SEG>(s, tid, xs, ys, line, e0, lam, pos, c.velocity, R); break;
        default: scalar_sweeps<MX, NT, 0, SEG>(s, tid, xs, ys, line, e0, lam, pos, c.velocity, R); break;
    }
    __syncthreads();
    // direction parts: columns into the tile's interior (nothing reads the
    // staged interior after the sweeps); rows stay in registers and are
    // added to them after the barrier (one row item per cell, so no race)
    if (xs) {
        part_row<MX, SEG>(s, line, e0, lam, pos, R);
    } else if (ys) {
        part_col<MX, SEG>(s, line, e0, lam, pos, R);
#pragma unroll
        for (int k = 0; k < SEG; k++) s.q[(e0 + k + MB) * NP + line + MB] = R[k];
    }
    __syncthreads();
    if (xs) {
        double *qr = &s.q[(line + MB) * NP + e0 + MB];
#pragma unroll
        for (int k = 0; k < SEG; k++) qr[k] = qr[k] + R[k];
    }
    __syncthreads();
    // Whole rows go out, ghost columns included (they carry the values the
    // step gathered; nothing reads a patch's own ghost cells before the next
    // fill or gather overwrites them): rows MB .. MB+MX-1 are one contiguous
    // range, so L2 writes back full lines instead of partial ones at every
    // row end.
    if constexpr (LEAF) {
        double *qo = io->qout + (size_t)io->leaf_of_slot[p] * MX * MX;
        for (int k = threadIdx.x; k < MX * MX / 2; k += NT) {
            const int i = 2 * (k % (MX / 2)), j = k / (MX / 2);
            // plain stores: the next step reads this state right away
            *reinterpret_cast<double2 *>(qo + 2 * k) =
                make_double2(s.q[(j + MB) * NP + i + MB], s.q[(j + MB) * NP + i + MB + 1]);
        }
    } else {
        for (int k = threadIdx.x; k < MX * N / 2; k += NT) {
            const int i = 2 * (k % (N / 2)), j = k / (N / 2) + MB;
            const double a = s.q[j * NP + i], b = s.q[j * NP + i + 1];
            if (c.stream_out) store_stream2(&out[base + j * N + i], a, b);
            else *reinterpret_cast<double2 *>(&out[base + j * N + i]) = make_double2(a, b);
        }
    }
    cfl = fmax(cfl, lam * __longlong_as_double((long long)s.cfl));
}

// lev: the patch's level when the caller knows it (a level-step), else -1;
// tdev: if given, the step starts at *tdev + t;
// slot: if given, its old value is left in s.red[15] for reduce_cfl_slot
template <int MX, int NT, bool FUSED, int SEGC = 0>
__device__ __forceinline__ void advance_scalar_patch(const Ctx &c, const View &w, ScalarSmem<MX> &s, int p, int lev,
                                                     double t, double dt, double &cfl, const double *tdev = nullptr,
                                                     const unsigned long long *slot = nullptr) {
    advance_scalar_lim<MX, NT, FUSED, false, SEGC>(c, w, s, p, lev, t, dt, tdev, slot, cfl);
}

// block-wide max of a non-negative double, then one atomicMax on its bits
// (kernels that run one workgroup per patch record per slot instead: a
// thousand atomics on one address serialise in L2)
template <int NT>
__device__ void reduce_cfl(double v, double *red, unsigned long long *cfl_bits) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int k = 1; k < NT / 64; k++) m = fmax(m, red[k]);
        if (cfl_bits && m > 0.0) atomicMax(cfl_bits, (unsigned long long)__double_as_longlong(m));
    }
}

// The workgroup owns its patch's slot for the whole launch: thread 0 reads
// the slot when the workgroup starts (the latency hides behind the step) and
// stores max(old, block max) at the end -- a plain store, where a device-wide
// atomic would add a round trip to memory before the workgroup can retire.
__device__ __forceinline__ double cfl_slot_old(const unsigned long long *slot) {
    return (slot && threadIdx.x == 0) ? __longlong_as_double((long long)*slot) : 0.0;
}

// scalar kernels: every thread already holds the patch's Courant number
__device__ __forceinline__ void store_cfl_slot(unsigned long long *slot, double old, double cfl) {
    if (threadIdx.x == 0 && slot) *slot = (unsigned long long)__double_as_longlong(fmax(old, cfl));
}

template <int NT>
__device__ void reduce_cfl_slot(double v, double *red, unsigned long long *slot, double old) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    if (threadIdx.x == 0 && slot) {
        double m = red[0];
        for (int k = 1; k < NT / 64; k++) m = fmax(m, red[k]);
        *slot = (unsigned long long)__double_as_longlong(fmax(old, m));
    }
}

// Waves per SIMD the kernels are compiled for (the register budget).  Scalar
// mx = 32: the LDS tile (29.8 KB) admits five workgroups per CU, and the
// register budget is set so that all five are resident (at most eight waves
// per SIMD).  Shallow water at mx = 16: two workgroups per CU (the LDS tile
// and accumulators take 68 KB).
template <int MX, int NT, int EQ>
constexpr int min_waves() {
    if ((EQ == 0 || EQ == 2) && MX == 32) {  // 2: the mapped grid's capacity form (30.4 KB)
        const int w = (5 * NT / 64 + 3) / 4;
        return w < 8 ? w : 8;
    }
    return (EQ == 1 && MX == 16 && NT >= 256) ? NT / 128 : 1;
}

template <int MX, int NT, bool FUSED, int SEGC = 0>
__global__ void __launch_bounds__(NT, (min_waves<MX, NT, 0>())) advance_scalar_kernel(Ctx c, int first, int count, int level, double t,
                                                                                     double dt) {
    __shared__ ScalarSmem<MX> s;
    const int p = first + xcd_remap(blockIdx.x, count);
    unsigned long long *slot = c.cflp ? c.cflp + p : nullptr;
    double cfl = 0.0;
    advance_scalar_patch<MX, NT, FUSED, SEGC>(c, view_of(c), s, p, level, t, dt, cfl, nullptr, slot);
    store_cfl_slot(slot, s.red[15], cfl);
}

// ------------------------------------------------------------------------
// mapped grids: capacity-form step (scalar advection)
// ------------------------------------------------------------------------
// The computational square is mapped by X = (xi, eta) + alpha sin(2 pi xi)
// sin(2 pi eta) (1, 1); a cell's capacity is the exact area of its image
// over h^2.  The Jacobian is 1 + 2 pi alpha sin(2 pi (xi + eta)), whose
// integral over a cell of side h gives
//   kappa = 1 + 2 pi alpha sigma^2 sin(2 pi (xi_c + eta_c)), sigma = sin(pi h)/(pi h),
// a function of I + J alone: per level a table K[k], k = (I + J + 1) mod n.
__global__ void init_capacity_kernel(int n, double alpha, double *K) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double h = 1.0 / (double)n;
    const double sig = sin(M_PI * h) / (M_PI * h);
    K[k] = 1.0 + 2.0 * M_PI * alpha * (sig * sig) * sin(2.0 * M_PI * ((double)k * h));
}

// The mapped step has the Cartesian step's structure (line sweeps that keep
// partial sums in registers, transverse terms TX / TY staged in LDS) with
// dt / h replaced per cell by dt / (kappa h), which depends on I + J only:
// one value per diagonal of the tile.  Capacity form (Clawpack's, the form
// mapped-grid wave propagation takes): the fluctuations entering a cell and
// its flux differences are scaled by that cell's dt / (kappa h); a
// transverse wave by that of the cell its corrected fluctuation entered (so
// TX(i, j) = dt / (kappa h)_{ij} (A+* W_{i-1/2} + A-* W_{i+1/2})); the
// correction C = |s| (1 - nubar |s|) W~ takes nubar, the mean over the edge's
// two cells; the Courant number is dt / (kappa h) of the cell a wave enters
// times its speed.
template <int MX>
struct MappedSmem : ScalarSmem<MX> {
    double dk[2 * (MX + 2 * MB)];  // dt / (kappa h) of the cells (i, j) with i + j = d - 2 MB
    unsigned long long mcfl;       // the patch's Courant number (bits of a non-negative double)
};

// One segment of one interior line (as sweep_segment): edges e0 .. e0+SEG,
// cells e0 .. e0+SEG-1; TX (TY) of the cells into LDS and the line's partial
// update of each cell in R:
//   rows     Rx = Q - TX + L/2 (C_{i+1/2} - C_{i-1/2}),
//   columns  Ry = L/2 (C_{j+1/2} - C_{j-1/2}) - TY,
// L the cell's dt / (kappa h); cm: the largest Courant number of the edges.
// POS: the line's upwind side, as in sweep_side.
template <int MX, int SEG, int LIM, int DIR, bool POS>
__device__ __forceinline__ void msweep_side(MappedSmem<MX> &s, int line, int e0, double (&R)[SEG], double &cm) {
    constexpr int NP = ScalarSmem<MX>::NP, S = ScalarSmem<MX>::S;
    constexpr int STR = DIR == 0 ? 1 : NP;
    const double *qp = DIR == 0 ? &s.q[(line + MB) * NP + MB + e0 - 2] : &s.q[(MB + e0 - 2) * NP + line + MB];
    const double *ve = DIR == 0 ? &s.ux[e0] : &s.vy[e0];
    const double vl = DIR == 0 ? s.uy[line + 1] : s.vx[line + 1];
    const double *lk = &s.dk[line + e0 - 1 + 2 * MB];  // lk[k]: cell e0 - 1 + k of the line
    double q[SEG + 4];
#pragma unroll
    for (int k = 0; k < SEG + 4; k++) q[k] = qp[k * STR];
    const double *L = lk;  // read where used: held in registers they cost the fifth workgroup per CU
    double aprev = 0.0, cprev = 0.0;
#pragma unroll
    for (int k = 0; k <= SEG; k++) {  // edge e0 + k, between cells e0+k-1 (q[k+1], L[k]) and e0+k (q[k+2], L[k+1])
        const double u = ve[k] * vl;
        const double W = q[k + 2] - q[k + 1];
        const double Wu = POS ? q[k + 1] - q[k] : q[k + 3] - q[k + 2];
        const double C = correction<LIM>(W, Wu, POS ? u : -u, 0.5 * (L[k] + L[k + 1]));
        const double aps = POS ? u * W - C : -C;
        const double ams = POS ? C : u * W + C;
        cm = fmax(cm, POS ? L[k + 1] * u : L[k] * -u);
        if (k > 0) {  // cell e0 + k - 1
            const int cc = e0 + k - 1;
            const double T = L[k] * (aprev + ams);
            if (DIR == 0) {
                s.tx[(line + 1) * S + cc] = T;
                R[k - 1] = q[k + 1] - T + (0.5 * L[k]) * (C - cprev);
            } else {
                s.ty[(line + 1) * S + cc] = T;
                R[k - 1] = (0.5 * L[k]) * (C - cprev) - T;
            }
        }
        aprev = aps;
        cprev = C;
    }
}

template <int MX, int SEG, int LIM, int DIR>
__device__ __forceinline__ void msweep_segment(MappedSmem<MX> &s, int line, int e0, bool pos, double (&R)[SEG],
                                               double &cm) {
    if (pos) msweep_side<MX, SEG, LIM, DIR, true>(s, line, e0, R, cm);
    else msweep_side<MX, SEG, LIM, DIR, false>(s, line, e0, R, cm);
}

// The same for a line outside the interior (as sweep_outer): TX (TY) only.
template <int MX, int SEG, int LIM, bool POS>
__device__ __forceinline__ void mouter_side(MappedSmem<MX> &s, int dir, int line, int e0) {
    constexpr int NP = ScalarSmem<MX>::NP, S = ScalarSmem<MX>::S;
    const int str = dir == 0 ? 1 : NP;
    const double *qp = dir == 0 ? &s.q[(line + MB) * NP + MB + e0 - 2] : &s.q[(MB + e0 - 2) * NP + line + MB];
    const double *ve = dir == 0 ? &s.ux[e0] : &s.vy[e0];
    const double vl = dir == 0 ? s.uy[line + 1] : s.vx[line + 1];
    const double *lk = &s.dk[line + e0 - 1 + 2 * MB];
    double *to = (dir == 0 ? s.tx : s.ty) + (line + 1) * S + e0 - 1;
    double q[SEG + 4], L[SEG + 2];
#pragma unroll
    for (int k = 0; k < SEG + 4; k++) q[k] = qp[k * str];
#pragma unroll
    for (int k = 0; k < SEG + 2; k++) L[k] = lk[k];
    double aprev = 0.0;
#pragma unroll
    for (int k = 0; k <= SEG; k++) {
        const double u = ve[k] * vl;
        const double W = q[k + 2] - q[k + 1];
        const double Wu = POS ? q[k + 1] - q[k] : q[k + 3] - q[k + 2];
        const double C = correction<LIM>(W, Wu, POS ? u : -u, 0.5 * (L[k] + L[k + 1]));
        const double ams = POS ? C : u * W + C;
        if (k > 0) to[k] = L[k] * (aprev + ams);
        aprev = POS ? u * W - C : -C;
    }
}

template <int MX, int SEG, int LIM>
__device__ __forceinline__ void msweep_outer(MappedSmem<MX> &s, int velocity, int dir, int line, int e0) {
    const double ve0 = dir == 0 ? s.ux[e0] : s.vy[e0];
    const double vl = dir == 0 ? s.uy[line + 1] : s.vx[line + 1];
    if (line_pos(velocity, ve0, vl)) mouter_side<MX, SEG, LIM, true>(s, dir, line, e0);
    else mouter_side<MX, SEG, LIM, false>(s, dir, line, e0);
}

// Transverse terms of a row segment: R += L/2 (TF_{i+1/2} - TF_{i-1/2}),
// TF(e) = u+ TY(e-1) + u- TY(e) (the TY already scaled by their cells' L; one
// term, on the line's upwind side); columns likewise with TG and TX.
template <int MX, int SEG>
__device__ __forceinline__ void mpart_row(const MappedSmem<MX> &s, int j, int e0, bool pos, double (&R)[SEG]) {
    constexpr int S = ScalarSmem<MX>::S;
    const double uyj = s.uy[j + 1];
    double ty[SEG + 2];
#pragma unroll
    for (int k = 0; k < SEG + 2; k++) ty[k] = s.ty[(e0 + k) * S + j];  // TY(e0 - 1 + k, j)
    double tf[SEG + 1];
#pragma unroll
    for (int k = 0; k <= SEG; k++) tf[k] = (s.ux[e0 + k] * uyj) * (pos ? ty[k] : ty[k + 1]);
#pragma unroll
    for (int k = 0; k < SEG; k++) R[k] = R[k] + (0.5 * s.dk[e0 + k + j + 2 * MB]) * (tf[k + 1] - tf[k]);
}

template <int MX, int SEG>
__device__ __forceinline__ void mpart_col(const MappedSmem<MX> &s, int i, int e0, bool pos, double (&R)[SEG]) {
    constexpr int S = ScalarSmem<MX>::S;
    const double vxi = s.vx[i + 1];
    double tx[SEG + 2];
#pragma unroll
    for (int k = 0; k < SEG + 2; k++) tx[k] = s.tx[(e0 + k) * S + i];  // TX(i, e0 - 1 + k)
    double tg[SEG + 1];
#pragma unroll
    for (int k = 0; k <= SEG; k++) tg[k] = (s.vy[e0 + k] * vxi) * (pos ? tx[k] : tx[k + 1]);
#pragma unroll
    for (int k = 0; k < SEG; k++) R[k] = R[k] + (0.5 * s.dk[i + e0 + k + 2 * MB]) * (tg[k + 1] - tg[k]);
}

// The sweeps of one limiter (work items as in advance_mapped_patch).
template <int MX, int NT, int LIM>
__device__ __forceinline__ void mapped_sweeps(MappedSmem<MX> &s, int tid, bool xs, bool ys, int line, int e0,
                                              bool pos, int velocity, double (&R)[scalar_seg<MX, NT>()],
                                              double &cm) {
    constexpr int SEG = scalar_seg<MX, NT>(), NI = MX * (MX / SEG);
    constexpr int SO = 2, NO = 4 * (MX / SO);
    constexpr int GT0 = (NT - 2 * NI >= NO) ? 2 * NI : NI;
    if (xs) msweep_segment<MX, SEG, LIM, 0>(s, line, e0, pos, R, cm);
    else if (ys) msweep_segment<MX, SEG, LIM, 1>(s, line, e0, pos, R, cm);
    if (tid >= GT0 && tid < GT0 + NO) {  // rows -1, MX and columns -1, MX: TX, TY only
        const int k = tid - GT0, g = k / (MX / SO);
        msweep_outer<MX, SO, LIM>(s, velocity, g >> 1, (g & 1) ? MX : -1, (k % (MX / SO)) * SO);
    }
}

// One capacity-form step of patch p (level lev, or its own if lev < 0) on
// its filled tile, or (FUSED) with its ghost values gathered from the
// neighbours' interiors (area-weighted averages); the work split is the
// Cartesian step's.  tdev: if given, the step starts at *tdev + t.
template <int MX, int NT, bool FUSED = false>
__device__ void advance_mapped_patch(const Ctx &c, const View &w, MappedSmem<MX> &s, int p, int lev, double t,
                                     double dt, double &cfl, const double *tdev = nullptr) {
    constexpr int N = MX + 2 * MB, NP = ScalarSmem<MX>::NP;
    constexpr int SEG = scalar_seg<MX, NT>(), NSEG = MX / SEG, NI = MX * NSEG, HI = NI / 2;
    constexpr int SO = 2, NO = 4 * (MX / SO);
    constexpr int GT0 = (NT - 2 * NI >= NO) ? 2 * NI : NI;
    static_assert(2 * NI <= NT && NSEG % 2 == 0, "interior items must fit one pass, in two halves");
    static_assert(GT0 + NO <= NT, "outer-line items must fit one pass");
    static_assert(NI + MX + 2 <= NT, "velocity factors are loaded by threads NI .. NI+MX+1");
    const int tid = threadIdx.x;
    const PatchInfo P = c.info[p];
    const int l = lev >= 0 ? lev : P.level, n = MX << l;
    const double lam = dt * (double)n;  // dt / h, exact
    const double *in = buf_of(c, w, l);
    double *out = other_of(c, w, l);
    const size_t base = (size_t)p * N * N;
    load_velocity<MX>(c, s, l, P.ix * MX, P.iy * MX, t, dt, tdev, NI);
    if constexpr (FUSED) {
        constexpr int NG = N * N - MX * MX;
        for (int k = tid; k < MX * MX / 2; k += NT) {
            const int i = 2 * (k % (MX / 2)), j = k / (MX / 2);
            const double2 v = *reinterpret_cast<const double2 *>(&in[base + (j + MB) * N + i + MB]);
            s.q[(j + MB) * NP + i + MB] = v.x;
            s.q[(j + MB) * NP + i + MB + 1] = v.y;
        }
        for (int g = tid; g < NG; g += NT) {
            int i, j;
            ghost_index<MX>(g, i, j);
            double val[1];
            ghost_cell<MX, 1, true>(c, w, p, i, j, val);
            s.q[(j + MB) * NP + i + MB] = val[0];
        }
    } else {
        for (int k = tid; k < N * N / 2; k += NT) {
            const int i = 2 * (k % (N / 2)), j = k / (N / 2);
            const double2 v = *reinterpret_cast<const double2 *>(&in[base + j * N + i]);
            s.q[j * NP + i] = v.x;
            s.q[j * NP + i + 1] = v.y;
        }
    }
    for (int d = tid; d < 2 * N - 1; d += NT) {
        int k = (P.ix * MX + P.iy * MX + d - 2 * MB + 1) % n;
        k = k < 0 ? k + n : k;
        s.dk[d] = lam / c.mk[l][k];
    }
    if (tid == 0) s.mcfl = 0ull;
    __syncthreads();
    double R[SEG];
    double cm = 0.0;
    int line = 0, e0 = 0;
    const bool xs = tid < NI, ys = !xs && tid < 2 * NI;
    const int half = (xs ? tid : tid - NI) / HI, r = (xs ? tid : tid - NI) % HI;
    bool pos = true;
    if (xs) {
        line = half * (MX / 2) + r % (MX / 2);
        e0 = (r / (MX / 2)) * SEG;
        pos = line_pos(c.velocity, s.ux[e0], s.uy[line + 1]);
    } else if (ys) {
        line = r % MX;
        e0 = (half * (NSEG / 2) + r / MX) * SEG;
        pos = line_pos(c.velocity, s.vy[e0], s.vx[line + 1]);
    }
    switch (c.lim) {
        case 1: mapped_sweeps<MX, NT, 1>(s, tid, xs, ys, line, e0, pos, c.velocity, R, cm); break;
        case 2: mapped_sweeps<MX, NT, 2>(s, tid, xs, ys, line, e0, pos, c.velocity, R, cm); break;
        case 3: mapped_sweeps<MX, NT, 3>(s, tid, xs, ys, line, e0, pos, c.velocity, R, cm); break;
        default: mapped_sweeps<MX, NT, 0>(s, tid, xs, ys, line, e0, pos, c.velocity, R, cm); break;
    }
    cm = wave_max_last_lane(cm);
    if ((tid & 63) == 63) atomicMax(&s.mcfl, (unsigned long long)__double_as_longlong(cm));
    __syncthreads();
    if (xs) {
        mpart_row<MX, SEG>(s, line, e0, pos, R);
    } else if (ys) {
        mpart_col<MX, SEG>(s, line, e0, pos, R);
#pragma unroll
        for (int k = 0; k < SEG; k++) s.q[(e0 + k + MB) * NP + line + MB] = R[k];
    }
    __syncthreads();
    if (xs) {
        double *qr = &s.q[(line + MB) * NP + e0 + MB];
#pragma unroll
        for (int k = 0; k < SEG; k++) qr[k] = qr[k] + R[k];
    }
    __syncthreads();
    for (int k = threadIdx.x; k < MX * N / 2; k += NT) {
        const int i = 2 * (k % (N / 2)), j = k / (N / 2) + MB;
        const double a = s.q[j * NP + i], b = s.q[j * NP + i + 1];
        if (c.stream_out) store_stream2(&out[base + j * N + i], a, b);
        else *reinterpret_cast<double2 *>(&out[base + j * N + i]) = make_double2(a, b);
    }
    cfl = fmax(cfl, __longlong_as_double((long long)s.mcfl));
}

template <int MX, int NT, bool FUSED>
__global__ void __launch_bounds__(NT, (min_waves<MX, NT, 0>())) advance_mapped_kernel(Ctx c, int first, int count,
                                                                                      int level, double t, double dt) {
    __shared__ MappedSmem<MX> s;
    const int p = first + xcd_remap(blockIdx.x, count);
    unsigned long long *slot = c.cflp ? c.cflp + p : nullptr;
    const double old = cfl_slot_old(slot);
    double cfl = 0.0;
    const View w = view_of(c);
    advance_mapped_patch<MX, NT, FUSED>(c, w, s, p, level, t, dt, cfl);
    store_cfl_slot(slot, old, cfl);
}

// one step of a uniform periodic level from leaf-order q_in to q_out
template <int MX, int NT>
__global__ void __launch_bounds__(NT, (min_waves<MX, NT, 0>())) step_leaf_kernel(Ctx c, int first, int count, int level,
                                                                                double t, double dt, LeafIO io) {
    __shared__ ScalarSmem<MX> s;
    const int p = first + xcd_remap(blockIdx.x, count);
    const View w = view_of(c);
    double cfl = 0.0;
    advance_scalar_lim<MX, NT, false, true>(c, w, s, p, level, t, dt, nullptr, nullptr, cfl, &io);
}

// ------------------------------------------------------------------------
// shallow-water step: Roe solver, Harten-Hyman entropy fix, MC-limited
// waves, transverse splitting in the Roe eigenbasis (system form of the
// same unsplit scheme; the paper runs Clawpack's wave-propagation solvers)
// ------------------------------------------------------------------------
// Tile of one shallow-water patch and its per-cell accumulators.  The tile
// rows have an odd stride so that lanes walking a column hit distinct banks.
template <int MX>
struct SweSmem {
    static constexpr int N = MX + 2 * MB;
    static constexpr int NP = N + 1;                // tile row stride
    static constexpr int AP = MX + 1;               // accumulator line stride
    static constexpr int NA = (MX + 2) * AP;        // accumulator cells per direction: lines -1..MX
    double q[3][N * NP];   // h, hu, hv
    double u[N * NP];      // hu / h
    double v[N * NP];      // hv / h
    double sh[N * NP];     // sqrt(h)
    double cs[N * NP];     // sqrt(g h)
    // [direction][component][cell]: components 0..2 the normal part of the
    // cell's update (h, hu, hv), 3..5 the transverse waves it sends across
    // its upper (right) side, 6..8 across its lower (left) side, already
    // scaled by lam^2 / 2.  Each receives exactly two contributions, one per
    // edge of the cell, added to -0 (order-independent bits).
    double acc[2][9][NA];
    unsigned long long cfl;  // largest wave speed over interior edges (bits of a non-negative double)
    double red[16];
};

// Roe linearisation of one edge in the frame (h, h u_n, h u_t) from the two
// cells' staged values (un, ut: velocities; sh = sqrt(h)).  r: alpha_1..3,
// u_hat, v_hat, c_hat.
__device__ __forceinline__ void roe_edge(double g, double hL, double nL, double tL, double unL, double utL, double shL,
                                         double hR, double nR, double tR, double unR, double utR, double shR,
                                         double *r) {
    const double hb = 0.5 * (hL + hR);
    const double is = 1.0 / (shL + shR);
    const double uh = (shL * unL + shR * unR) * is;
    const double vh = (shL * utL + shR * utR) * is;
    const double ch = sqrt(g * hb);
    const double i2c = 0.5 / ch;
    const double d0 = hR - hL, d1 = nR - nL, d2 = tR - tL;
    r[0] = ((uh + ch) * d0 - d1) * i2c;
    r[1] = d2 - vh * d0;
    r[2] = (d1 - (uh - ch) * d0) * i2c;
    r[3] = uh; r[4] = vh; r[5] = ch;
}

__device__ __forceinline__ void waves_of(const double *r, double W[3][3], double sp[3]) {
    const double uh = r[3], vh = r[4], ch = r[5];
    W[0][0] = r[0]; W[0][1] = r[0] * (uh - ch); W[0][2] = r[0] * vh;
    W[1][0] = 0.0; W[1][1] = 0.0; W[1][2] = r[1];
    W[2][0] = r[2]; W[2][1] = r[2] * (uh + ch); W[2][2] = r[2] * vh;
    sp[0] = uh - ch; sp[1] = uh; sp[2] = uh + ch;
}

__device__ __forceinline__ double phi_limit(int lim, double th) {
    if (lim == 1) return 1.0;
    if (lim == 2) return 0.0;
    if (lim == 3) return th <= 0 ? 0.0 : (th < 1.0 ? th : 1.0);
    const double mn = fmin(0.5 * (1.0 + th), fmin(2.0, 2.0 * th));
    return mn > 0.0 ? mn : 0.0;
}

// split A (frame h, n, t) into its +t and -t moving parts with the Roe state r
// (i2c = 1 / (2 c), shared by the two splits of an edge)
__device__ __forceinline__ void roe_transverse(const double *r, double i2c, const double *A, double *bp, double *bm) {
    const double un = r[3], ut = r[4], c = r[5];
    const double be[3] = {((ut + c) * A[0] - A[2]) * i2c, A[1] - un * A[0], (A[2] - (ut - c) * A[0]) * i2c};
    const double mu[3] = {ut - c, ut, ut + c};
    const double rv[3][3] = {{1.0, un, ut - c}, {0.0, 1.0, 0.0}, {1.0, un, ut + c}};
#pragma unroll
    for (int e = 0; e < 3; e++) { bp[e] = 0.0; bm[e] = 0.0; }
#pragma unroll
    for (int p = 0; p < 3; p++) {
        const double mp = mu[p] > 0 ? mu[p] : 0.0, mm = mu[p] < 0 ? mu[p] : 0.0;
#pragma unroll
        for (int e = 0; e < 3; e++) { bp[e] += mp * be[p] * rv[p][e]; bm[e] += mm * be[p] * rv[p][e]; }
    }
}

// One edge, the whole of its update: the Roe solves of the edge and of its
// two neighbours along the line (their waves are the limiter's upwind waves),
// fluctuations with the Harten-Hyman fix on transonic rarefactions of
// families 1 and 3, MC-limited correction C, corrected fluctuations and
// their transverse splits.  Line `line` of direction `dir` (0: x-edges of a
// row, 1: y-edges of a column); edge e lies between cells e-1 and e.  Adds
// its parts to the accumulators of cells e-1 and e; returns the largest
// wave speed at the edge.
template <int MX>
__device__ __forceinline__ double swe_edge(SweSmem<MX> &s, double g, int lim, double lam, int dir, int line, int e) {
    constexpr int NP = SweSmem<MX>::NP, AP = SweSmem<MX>::AP;
    const int fn = dir == 0 ? 1 : 2, ft = 3 - fn;  // normal / tangential momentum fields
    const double *un = dir == 0 ? s.u : s.v, *ut = dir == 0 ? s.v : s.u;
    // cells e-2 .. e+1 of the line
    const int k0 = dir == 0 ? (line + MB) * NP + (e - 2 + MB) : (e - 2 + MB) * NP + (line + MB);
    const int st = dir == 0 ? 1 : NP;
    double h[4], n[4], t[4], a[4], b[4], r2[4];
#pragma unroll
    for (int m = 0; m < 4; m++) {
        const int k = k0 + m * st;
        h[m] = s.q[0][k]; n[m] = s.q[fn][k]; t[m] = s.q[ft][k];
        a[m] = un[k]; b[m] = ut[k]; r2[m] = s.sh[k];
    }
    double rl[6], r[6], rh[6];
    roe_edge(g, h[0], n[0], t[0], a[0], b[0], r2[0], h[1], n[1], t[1], a[1], b[1], r2[1], rl);
    roe_edge(g, h[1], n[1], t[1], a[1], b[1], r2[1], h[2], n[2], t[2], a[2], b[2], r2[2], r);
    roe_edge(g, h[2], n[2], t[2], a[2], b[2], r2[2], h[3], n[3], t[3], a[3], b[3], r2[3], rh);
    double W[3][3], sp[3];
    waves_of(r, W, sp);
    // Harten-Hyman fix (the middle states are needed only where the outer
    // speed has the sign that allows a transonic rarefaction)
    const double cL = s.cs[k0 + st], cR = s.cs[k0 + 2 * st];
    const double l1L = a[1] - cL;
    double l1R = 0.0;
    if (l1L < 0.0) {
        const double hm = h[1] + W[0][0];
        l1R = (n[1] + W[0][1]) / hm - sqrt(g * hm);
    }
    const bool fix1 = l1L < 0.0 && l1R > 0.0;
    const double l3R = a[2] + cR;
    double l3L = 0.0;
    if (l3R > 0.0) {
        const double hm3 = h[2] - W[2][0];
        l3L = (n[2] - W[2][1]) / hm3 + sqrt(g * hm3);
    }
    const bool fix3 = l3L < 0.0 && l3R > 0.0;
    double am[3] = {0, 0, 0}, ap[3] = {0, 0, 0};
#pragma unroll
    for (int p = 0; p < 3; p++) {
        double sm, spp;
        if (p == 0 && fix1) {
            const double beta = (l1R - sp[0]) / (l1R - l1L);
            sm = beta * l1L; spp = (1.0 - beta) * l1R;
        } else if (p == 2 && fix3) {
            const double beta = (l3R - sp[2]) / (l3R - l3L);
            sm = beta * l3L; spp = (1.0 - beta) * l3R;
        } else {
            sm = sp[p] < 0 ? sp[p] : 0.0;
            spp = sp[p] > 0 ? sp[p] : 0.0;
        }
#pragma unroll
        for (int f = 0; f < 3; f++) { am[f] += sm * W[p][f]; ap[f] += spp * W[p][f]; }
    }
    // MC limiter on each wave against the upwind wave of its family
    double Wl[3][3], spl[3], Wh[3][3], sph[3];
    waves_of(rl, Wl, spl);
    waves_of(rh, Wh, sph);
    double C[3] = {0, 0, 0}, smax = 0.0;
#pragma unroll
    for (int p = 0; p < 3; p++) {
        double ww = 0, wu = 0;
#pragma unroll
        for (int f = 0; f < 3; f++) {
            const double wup = sp[p] > 0 ? Wl[p][f] : Wh[p][f];
            ww += W[p][f] * W[p][f];
            wu += wup * W[p][f];
        }
        const double ph = ww == 0.0 ? 0.0 : phi_limit(lim, wu / ww);
        const double as = fabs(sp[p]);
#pragma unroll
        for (int f = 0; f < 3; f++) C[f] += as * (1.0 - lam * as) * ph * W[p][f];
        smax = fmax(smax, as);
    }
    double Aps[3], Ams[3], bpp[3], bmp[3], bpm[3], bmm[3];
#pragma unroll
    for (int f = 0; f < 3; f++) { Aps[f] = ap[f] - C[f]; Ams[f] = am[f] + C[f]; }
    const double i2c = 0.5 / r[5];
    roe_transverse(r, i2c, Aps, bpp, bmp);
    roe_transverse(r, i2c, Ams, bpm, bmm);
    // back to (h, hu, hv): frame component c goes to field 0, fn, ft
    const double hl = 0.5 * lam, hl2 = 0.5 * lam * lam;
    // cell e (right of the edge) and cell e-1 (left): accumulator index along
    // the line, line -1 .. MX
    const int ar = (line + 1) * AP + e, al = ar - 1;
    double *A = &s.acc[dir][0][0];
#pragma unroll
    for (int c = 0; c < 3; c++) {
        const int f = c == 0 ? 0 : (c == 1 ? fn : ft);
        if (e < MX) {
            atomicAdd(&A[(0 + f) * SweSmem<MX>::NA + ar], -lam * Aps[c] - hl * C[c]);
            atomicAdd(&A[(3 + f) * SweSmem<MX>::NA + ar], hl2 * bpp[c]);
            atomicAdd(&A[(6 + f) * SweSmem<MX>::NA + ar], hl2 * bmp[c]);
        }
        if (e > 0) {
            atomicAdd(&A[(0 + f) * SweSmem<MX>::NA + al], -lam * Ams[c] + hl * C[c]);
            atomicAdd(&A[(3 + f) * SweSmem<MX>::NA + al], hl2 * bpm[c]);
            atomicAdd(&A[(6 + f) * SweSmem<MX>::NA + al], hl2 * bmm[c]);
        }
    }
    return (line >= 0 && line < MX) ? smax : 0.0;
}

// One step on a shallow-water patch: stage the tile (with per-cell
// velocities, sqrt(h) and sqrt(g h)), one pass over every x- and y-edge
// (each a whole edge update, accumulated into the two cells it touches),
// one pass over the cells.  Two barriers after the staging.  cfl is
// max-accumulated with the patch's Courant number (in every thread).
template <int MX, int NT, bool FUSED>
__device__ void advance_swe_patch(const Ctx &c, const View &w, SweSmem<MX> &s, int p, double dt, double &cfl) {
    constexpr int N = MX + 2 * MB, NP = SweSmem<MX>::NP, NA = SweSmem<MX>::NA, AP = SweSmem<MX>::AP;
    constexpr int NE = (MX + 1) * (MX + 2);  // edges per direction: MX+1 along each of lines -1..MX
    const PatchInfo P = c.info[p];
    const int l = P.level;
    // h = 1 / (MX 2^l) is a power of two: dt / h is exact as a product
    const double lam = dt * (double)(MX << l), g = c.g;
    const double *in = buf_of(c, w, l);
    double *out = other_of(c, w, l);
    auto stage = [&](int i, int j, const double (&v)[3]) {
        const int k = (j + MB) * NP + i + MB;
#pragma unroll
        for (int f = 0; f < 3; f++) s.q[f][k] = v[f];
        s.u[k] = v[1] / v[0];
        s.v[k] = v[2] / v[0];
        s.sh[k] = sqrt(v[0]);
        s.cs[k] = sqrt(g * v[0]);
    };
    if (!FUSED) {
        for (int k = threadIdx.x; k < N * N; k += NT) {
            double v[3];
#pragma unroll
            for (int f = 0; f < 3; f++) v[f] = in[(size_t)(f * c.cap + p) * N * N + k];
            stage(k % N - MB, k / N - MB, v);
        }
    } else {
        // ghost cells (items below NG) and interior cells in one item space,
        // so that their loads go out together
        constexpr int NG = N * N - MX * MX;
        for (int k = threadIdx.x; k < N * N; k += NT) {
            int i, j;
            double v[3];
            if (k < NG) {
                ghost_index<MX>(k, i, j);
                // the 512- and 640-thread variants are held to 128 and 96
                // registers (two workgroups per CU)
                ghost_cell_of<MX, 3, (NT <= 384)>(c, w, p, P, i, j, v);
            } else {
                i = (k - NG) % MX;
                j = (k - NG) / MX;
#pragma unroll
                for (int f = 0; f < 3; f++) v[f] = in[(size_t)(f * c.cap + p) * N * N + (j + MB) * N + i + MB];
            }
            stage(i, j, v);
        }
    }
    {
        double *A = &s.acc[0][0][0];
        for (int k = threadIdx.x; k < 2 * 9 * NA; k += NT) A[k] = -0.0;
        if (threadIdx.x == 0) s.cfl = 0ull;
    }
    __syncthreads();
    double smax = 0.0;
    for (int k = threadIdx.x; k < 2 * NE; k += NT) {
        const int dir = k >= NE ? 1 : 0, kk = k - dir * NE;
        smax = fmax(smax, swe_edge<MX>(s, g, c.lim, lam, dir, kk / (MX + 1) - 1, kk % (MX + 1)));
    }
    smax = wave_max_last_lane(smax);
    if ((threadIdx.x & 63) == 63 && smax > 0.0) atomicMax(&s.cfl, (unsigned long long)__double_as_longlong(smax));
    __syncthreads();
    // the update of cell (i, j): Q + [x normal + x transverse] + [y normal + y transverse]
    for (int k = threadIdx.x; k < 3 * MX * MX; k += NT) {
        const int f = k / (MX * MX), i = k % MX, j = (k / MX) % MX;
        const double *X = &s.acc[0][0][0], *Y = &s.acc[1][0][0];
        const int xc = (j + 1) * AP + i, yc = (i + 1) * AP + j;
        const double tx = X[(3 + f) * NA + xc] + X[(6 + f) * NA + xc + AP] - X[(3 + f) * NA + xc - AP] - X[(6 + f) * NA + xc];
        const double ty = Y[(3 + f) * NA + yc] + Y[(6 + f) * NA + yc + AP] - Y[(3 + f) * NA + yc - AP] - Y[(6 + f) * NA + yc];
        const double q = s.q[f][(j + MB) * NP + i + MB];
        out[(size_t)(f * c.cap + p) * N * N + (j + MB) * N + i + MB] = q + (X[f * NA + xc] + ty) + (Y[f * NA + yc] + tx);
    }
    cfl = fmax(cfl, lam * __longlong_as_double((long long)s.cfl));
}

template <int MX, int NT, bool FUSED>
__global__ void __launch_bounds__(NT, (min_waves<MX, NT, 1>())) advance_swe_kernel(Ctx c, int first, int count, double dt) {
    __shared__ SweSmem<MX> s;
    const int p = first + xcd_remap(blockIdx.x, count);
    unsigned long long *slot = c.cflp ? c.cflp + p : nullptr;
    const double old = cfl_slot_old(slot);
    double cfl = 0.0;
    advance_swe_patch<MX, NT, FUSED>(c, view_of(c), s, p, dt, cfl);
    store_cfl_slot(slot, old, cfl);
}

// ------------------------------------------------------------------------
// adjoint of one uniform-level scalar step (fill by copy, then advance)
// ------------------------------------------------------------------------
// On a uniform periodic level every ghost value is a same-size copy, so the
// patch step is the global stencil of the unsplit scheme (Sec. 3) and the
// transpose of copy + advance is the global transposed stencil:
//   lambda_out(c) = sum over d of dQnew(d)/dQ(c) lambda_in(d),
// with d within two cells of c.  It is evaluated in gather form, one
// workgroup per patch: lambda_in with two ghost layers and q with three
// (along the axes only) come straight from the neighbours' interiors.
//
// The step is piecewise linear in Q; its Jacobian is the step with the
// limiter branches frozen at the forward state.  Per line (a row for the x
// sweep, a column for the y sweep; L = lambda_in, lam = dt/h):
//   Tbar(i) = -lam L(i) + lam^2/2 (s+_up (L(i) - L_up(i)) + s-_dn (L_dn(i) - L(i)))
//             adjoint of the cell's total fluctuation (TX or TY), the
//             transverse edges' speeds s_up, s_dn on either side of the line;
//   per edge e (between cells e-1 and e, speed u, W = Q(e) - Q(e-1), Wu its
//   upwind neighbour):
//   Cbar = lam/2 (L(e-1) - L(e)) - Tbar(e) + Tbar(e-1),  w = |u| (1 - lam |u|) Cbar,
//   g(e) = u+ Tbar(e) + u- Tbar(e-1) + dphi/dW w,  h(e) = dphi/dWu w,
//   D(e) = g(e) + [u(e+1) > 0] h(e+1) + [u(e-1) <= 0] h(e-1)
//             total adjoint of the difference W(e);
//   cell i receives D(i) - D(i+1).
// lambda_out(c) = L(c) + (row part) + (column part).

// Partial derivatives of the limited wave phi(W, Wu) (the correction's
// factor k excluded) on the forward branch.  Ties follow the forward
// limiter's order: the half sum, then 2|W|, then 2|Wu|; minmod takes W on a tie.
template <int LIM>
__device__ __forceinline__ void limiter_partials(double W, double Wu, double &dW, double &dWu) {
    if constexpr (LIM == 2) { dW = 0.0; dWu = 0.0; return; }
    if constexpr (LIM == 1) { dW = 1.0; dWu = 0.0; return; }
    const bool on = W * Wu > 0.0;
    const double aw = fabs(W), au = fabs(Wu);
    if constexpr (LIM == 3) {
        const bool tw = aw <= au;
        dW = (on && tw) ? 1.0 : 0.0;
        dWu = (on && !tw) ? 1.0 : 0.0;
        return;
    }
    const double a = 0.5 * (aw + au), b = 2.0 * aw, cc = 2.0 * au;
    const bool t1 = b < a;
    const bool t2 = cc < (t1 ? b : a);
    dW = (!on || t2) ? 0.0 : (t1 ? 2.0 : 0.5);
    dWu = !on ? 0.0 : (t2 ? 2.0 : (t1 ? 0.0 : 0.5));
}

template <int MX>
struct AdjSmem {
    static constexpr int NQ = MX + 6, QP = NQ + 1;  // q, three ghost layers (corners unused)
    static constexpr int NL = MX + 4, LP = NL + 1;  // lambda_in, two ghost layers
    double q[NQ * QP];
    double l[NL * LP];  // after the sweeps, the interior takes L + the row part of each cell
    // velocity factors (the forward step's): x-edge e -> ue[e + 1], row j ->
    // uc[j + 2]; y-edge e -> ve[e + 1], column i -> vc[i + 2]
    double ue[MX + 3], uc[MX + 4], ve[MX + 3], vc[MX + 4];
};

// One segment of one line: cells e0 .. e0+SEG-1 of row `line` (DIR 0) or
// column `line` (DIR 1).  Returns D(i) - D(i+1) of each cell.  The edges
// e0-1 .. e0+SEG+1 are walked in order with a window of three differences W,
// two cells (L, Tbar) and the last two edges' (g, h, upwind side), so that
// few values are live at once: D of an edge is complete once the edge after
// it has its h.
template <int MX, int SEG, int LIM, int DIR>
__device__ __forceinline__ void adjoint_line(const AdjSmem<MX> &s, int line, int e0, double lam, double (&R)[SEG]) {
    using A = AdjSmem<MX>;
    constexpr int SQ = DIR == 0 ? 1 : A::QP, SL = DIR == 0 ? 1 : A::LP, XL = DIR == 0 ? A::LP : 1;
    const double *qp = DIR == 0 ? &s.q[(line + 3) * A::QP + 3] : &s.q[3 * A::QP + line + 3];
    const double *lp = DIR == 0 ? &s.l[(line + 2) * A::LP + 2] : &s.l[2 * A::LP + line + 2];
    const double *ea = DIR == 0 ? &s.ue[1] : &s.ve[1];   // speed factor of the line's edges
    const double *ca = DIR == 0 ? &s.vc[2] : &s.uc[2];   // cell factor of the transverse edges
    const double lf = DIR == 0 ? s.uc[line + 2] : s.vc[line + 2];
    const double fup = DIR == 0 ? s.ve[line + 2] : s.ue[line + 2];  // transverse edge line + 1/2
    const double fdn = DIR == 0 ? s.ve[line + 1] : s.ue[line + 1];  // transverse edge line - 1/2
    const double hl = 0.5 * lam, hl2 = 0.5 * lam * lam;
    // window cell k is cell e0 - 2 + k: its L and Tbar
    auto cell = [&](int k, double &L, double &T) {
        const double *lc = lp + (e0 - 2 + k) * SL;
        const double Lc = lc[0], Lu = lc[XL], Ld = lc[-XL];
        const double cf = ca[e0 - 2 + k];
        L = Lc;
        T = hl2 * (posp(fup * cf) * (Lc - Lu) + negp(fdn * cf) * (Ld - Lc)) - lam * Lc;
    };
    // q at cell e0 - 3 + k; W(k) = q(k + 1) - q(k) is the difference at edge e0 - 2 + k
    auto qv = [&](int k) { return qp[(e0 - 3 + k) * SQ]; };
    const double q0 = qv(0), q1 = qv(1);
    double q2 = qv(2);
    double wm = q1 - q0, w0 = q2 - q1;  // W at edges m - 1 and m (window edge m is edge e0 - 1 + m)
    double L0, T0;
    cell(0, L0, T0);
    double g1 = 0.0, h1 = 0.0, h2 = 0.0, D1 = 0.0;  // the previous edge's g, h; the one before's h
    bool up1 = false, up2 = false;
#pragma unroll
    for (int m = 0; m < SEG + 3; m++) {
        const double q3 = qv(m + 3);
        const double wp = q3 - q2;  // W at edge m + 1
        double L1, T1;
        cell(m + 1, L1, T1);
        // edge m: between window cells m and m + 1
        const double u = ea[e0 - 1 + m] * lf;
        const bool up = u > 0.0;
        const double W = w0;
        const double Wu = up ? wm : wp;
        const double tr = T1, tl = T0;
        const double au = fabs(u);
        const double wb = (au * (1.0 - lam * au)) * (hl * (L0 - L1) - tr + tl);
        double dW, dWu;
        limiter_partials<LIM>(W, Wu, dW, dWu);
        const double g = posp(u) * tr + negp(u) * tl + dW * wb;
        const double h = dWu * wb;
        if (m >= 2) {  // D of edge m - 1 (cell boundary e0 + m - 2)
            const double D = g1 + (up ? h : 0.0) + (up2 ? 0.0 : h2);
            if (m >= 3) R[m - 3] = D1 - D;
            D1 = D;
        }
        h2 = h1; up2 = up1;
        g1 = g; h1 = h; up1 = up;
        wm = w0; w0 = wp; q2 = q3;
        L0 = L1; T0 = T1;
    }
}

template <int MX, int NT>
constexpr int adj_seg() { return (2 * MX * MX / NT) < 4 ? 4 : 2 * MX * MX / NT; }

// mx = 32: the tiles of q and lambda_in (23.1 KB) admit six workgroups per CU,
// and the register budget is set for all six (five for minmod, whose
// partials take a few more registers)
template <int MX, int NT, int LIM>
__global__ void __launch_bounds__(NT, (MX == 32 ? (LIM == 3 ? 5 : 6) : 1)) adjoint_kernel(Ctx c, int level, int first, int count,
                                                                         double t, double dt,
                                                                         const int32_t *leaf_of_slot,
                                                                         const double *q_in, const double *lam_in,
                                                                         double *lam_out) {
    using A = AdjSmem<MX>;
    constexpr int SEG = adj_seg<MX, NT>(), NI = MX * (MX / SEG);  // segments per direction
    static_assert(2 * NI <= NT && MX % SEG == 0, "one segment per thread");
    constexpr int NG2 = (MX + 4) * (MX + 4) - MX * MX;             // lambda ghost ring
    constexpr int NVI = (MX * MX / 2 + NT - 1) / NT, NVA = (12 * MX + NT - 1) / NT, NVR = (NG2 + NT - 1) / NT;
    __shared__ A s;
    const int tid = threadIdx.x;
    const int p = first + xcd_remap(blockIdx.x, count);
    const int l = level;
    const double lam = dt * (double)(MX << l);  // dt / h, exact: h = 1 / (MX 2^l)
    const size_t PS = (size_t)MX * MX;
    // A complete periodic level: the slot of every neighbour follows from the
    // Morton index.  All leaf indices are loaded first, then all values, so the
    // staging costs two memory round trips.
    const uint32_t m = (uint32_t)(p - c.lstart[l]);
    const int ix = (int)morton_compact(m), iy = (int)morton_compact(m >> 1), wrap = (1 << l) - 1;
    auto leaf_at = [&](int dx, int dy) {
        return leaf_of_slot[c.lstart[l] + (int)(morton_spread((uint32_t)((ix + dx) & wrap)) |
                                                  (morton_spread((uint32_t)((iy + dy) & wrap)) << 1))];
    };
    auto side = [](int i) { return i < 0 ? -1 : (i >= MX ? 1 : 0); };
    // Indices past the end are clamped to the last valid cell, so every load
    // is issued without a branch; only the LDS stores below are guarded.
    const int self = leaf_of_slot[p];
    int ai[NVA], aj[NVA], al[NVA], ri[NVR], rj[NVR], rl[NVR];
#pragma unroll
    for (int v = 0; v < NVA; v++) {  // q: three layers beyond each side
        const int g = min(tid + v * NT, 12 * MX - 1);
        const int sd = g / (3 * MX), k = g % (3 * MX);
        if (sd < 2) { aj[v] = k / 3; ai[v] = sd == 0 ? k % 3 - 3 : MX + k % 3; }
        else { ai[v] = k % MX; aj[v] = sd == 2 ? k / MX - 3 : MX + k / MX; }
        al[v] = leaf_at(side(ai[v]), side(aj[v]));
    }
#pragma unroll
    for (int v = 0; v < NVR; v++) {  // lambda_in: two ghost layers, corners included
        int rr;
        ghost_region_index<MX>(min(tid + v * NT, NG2 - 1), ri[v], rj[v], rr);
        rl[v] = leaf_at(side(ri[v]), side(rj[v]));
    }
    double2 qa[NVI], la[NVI];
#pragma unroll
    for (int v = 0; v < NVI; v++) {
        const int k = min(tid + v * NT, MX * MX / 2 - 1);
        qa[v] = *reinterpret_cast<const double2 *>(q_in + (size_t)self * PS + 2 * k);
        la[v] = *reinterpret_cast<const double2 *>(lam_in + (size_t)self * PS + 2 * k);
    }
    double av[NVA], rv[NVR];
#pragma unroll
    for (int v = 0; v < NVA; v++) {
        const int dx = side(ai[v]), dy = side(aj[v]);
        av[v] = q_in[(size_t)al[v] * PS + (aj[v] - dy * MX) * MX + ai[v] - dx * MX];
    }
#pragma unroll
    for (int v = 0; v < NVR; v++) {
        const int dx = side(ri[v]), dy = side(rj[v]);
        rv[v] = lam_in[(size_t)rl[v] * PS + (rj[v] - dy * MX) * MX + ri[v] - dx * MX];
    }
    // velocity factors at the mid-step time, as the forward step takes them
    {
        const int n = MX << l, gx0 = ix * MX, gy0 = iy * MX;
        if (c.velocity == 2) {
            const double ct = cos(M_PI * ((t + 0.5 * dt) * c.vel_invT));
            const double *vt = c.vt[l];
            const double *ex = vt + vt_ex(n, MB), *cxv = vt + vt_cx(n, MB);
            const double *ey = vt + vt_ey(n, MB), *cyv = vt + vt_cy(n, MB);
            for (int k = tid; k < MX + 4; k += NT) {
                if (k < MX + 3) { s.ue[k] = ex[gx0 + k - 1]; s.ve[k] = ey[gy0 + k - 1]; }
                s.uc[k] = cyv[gy0 + k - 2] * ct;
                s.vc[k] = -(cxv[gx0 + k - 2] * ct);
            }
        } else {
            for (int k = tid; k < MX + 4; k += NT) {
                if (k < MX + 3) { s.ue[k] = c.vel_u; s.ve[k] = c.vel_v; }
                s.uc[k] = 1.0;
                s.vc[k] = 1.0;
            }
        }
    }
#pragma unroll
    for (int v = 0; v < NVI; v++) {
        const int k = tid + v * NT;
        if (k < MX * MX / 2) {
            const int i = 2 * (k % (MX / 2)), j = k / (MX / 2);
            s.q[(j + 3) * A::QP + i + 3] = qa[v].x;
            s.q[(j + 3) * A::QP + i + 4] = qa[v].y;
            s.l[(j + 2) * A::LP + i + 2] = la[v].x;
            s.l[(j + 2) * A::LP + i + 3] = la[v].y;
        }
    }
#pragma unroll
    for (int v = 0; v < NVA; v++)
        if (tid + v * NT < 12 * MX) s.q[(aj[v] + 3) * A::QP + ai[v] + 3] = av[v];
#pragma unroll
    for (int v = 0; v < NVR; v++)
        if (tid + v * NT < NG2) s.l[(rj[v] + 2) * A::LP + ri[v] + 2] = rv[v];
    __syncthreads();
    double R[SEG];
    const int j = tid % MX, e0 = (tid / MX) * SEG;  // rows
    const int k0 = tid - NI, i = k0 % MX, c0 = (k0 / MX) * SEG;  // columns
    if (tid < NI) adjoint_line<MX, SEG, LIM, 0>(s, j, e0, lam, R);
    else if (tid < 2 * NI) adjoint_line<MX, SEG, LIM, 1>(s, i, c0, lam, R);
    __syncthreads();
    // rows: L + row part into the interior of lambda_in's tile (no sweep reads
    // it any more; one row item per cell), held in registers over the barrier
    if (tid < NI) {
        double *lr = &s.l[(j + 2) * A::LP + e0 + 2];
#pragma unroll
        for (int k = 0; k < SEG; k++) lr[k] = lr[k] + R[k];
    }
    __syncthreads();
    if (tid >= NI && tid < 2 * NI) {  // columns finish the cells (a row of lanes per store)
        double *lo = lam_out + (size_t)leaf_of_slot[p] * PS;
#pragma unroll
        for (int k = 0; k < SEG; k++) lo[(c0 + k) * MX + i] = s.l[(c0 + k + 2) * A::LP + i + 2] + R[k];
    }
}

// ------------------------------------------------------------------------
// persistent fused kernel: all level-steps of a coarse step in one launch
// ------------------------------------------------------------------------
constexpr long long kSpinLimit = 1ll << 22;

// Device-wide barrier for a co-resident grid.  Every wait is bounded: on
// timeout the error flag is raised and all later waits are skipped, so the
// kernel always drains.
__device__ void grid_barrier(DevState *st, unsigned nblocks) {
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned gen = __hip_atomic_load(&st->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const unsigned arrived =
            __hip_atomic_fetch_add(&st->bar_count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(&st->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(&st->bar_gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            long long spins = 0;
            while (__hip_atomic_load(&st->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > kSpinLimit ||
                    __hip_atomic_load(&st->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 1) {
                    __hip_atomic_fetch_or(&st->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    break;
                }
            }
        }
        __threadfence();
    }
    __syncthreads();
}

template <int MX, int EQ>
struct SmemOf { using type = ScalarSmem<MX>; };
template <int MX>
struct SmemOf<MX, 1> { using type = SweSmem<MX>; };
template <int MX>
struct SmemOf<MX, 2> { using type = MappedSmem<MX>; };  // scalar advection on a mapped grid

template <int MX, int NT, int EQ>
__global__ void __launch_bounds__(NT, (min_waves<MX, NT, EQ>())) persistent_kernel(Ctx c, const SchedEntry *sched, int nsched,
                                                        const LevelRange *lr, int ncoarse, DevState *st) {
    __shared__ typename SmemOf<MX, EQ>::type s;
    double t0 = st->t;
    const double dtc = st->dt_coarse;
    View w{st->curmask, -1, 1.0};
    const unsigned G = gridDim.x;
    // XCD-aware split: workgroup b runs on XCD b mod 8 and takes a stride of
    // that XCD's contiguous chunk (NXC chunks when fewer than 8 workgroups)
    const int NXC = G < 8 ? (int)G : 8;
    const int x = blockIdx.x % NXC, r = blockIdx.x / NXC;
    const int nbx = ((int)G - x + NXC - 1) / NXC;  // workgroups on this chunk
    uint32_t allmask = 0;
    int nall = 0;
    for (int l = 0; l < FC_MAXLEV; l++)
        if (lr->count[l] > 0) { allmask |= 1u << l; nall += lr->count[l]; }
    double cfl = 0.0;
    for (int cs = 0; cs < ncoarse; cs++) {
        for (int k = 0; k < nsched; k++) {
            const SchedEntry e = sched[k];
            int first, count;
            if (e.level < 0) { first = 0; count = nall; w.clevel = -1; w.alpha = 1.0; }
            else { first = lr->start[e.level]; count = lr->count[e.level]; w.clevel = e.level - 1; w.alpha = e.alpha; }
            if (count == 0) {
                if (e.level >= 0) w.curmask ^= 1u << e.level;
                continue;
            }
            const double t = t0 + e.off * dtc, dt = e.scale * dtc;
            const int c0 = (int)((long long)count * x / NXC), c1 = (int)((long long)count * (x + 1) / NXC);
            for (int pi = c0 + r; pi < c1; pi += nbx) {
                if constexpr (EQ == 0) advance_scalar_patch<MX, NT, true>(c, w, s, first + pi, e.level, t, dt, cfl);
                else if constexpr (EQ == 2) advance_mapped_patch<MX, NT, true>(c, w, s, first + pi, e.level, t, dt, cfl);
                else advance_swe_patch<MX, NT, true>(c, w, s, first + pi, dt, cfl);
                __syncthreads();
            }
            grid_barrier(st, G);
            w.curmask ^= (e.level < 0) ? allmask : (1u << e.level);
        }
        t0 = t0 + dtc;  // the same accumulation as the host's time
    }
    reduce_cfl<NT>(cfl, s.red, &st->cfl_bits);
    grid_barrier(st, G);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->t = t0;
        st->curmask = w.curmask;
    }
}

// ------------------------------------------------------------------------
// one level-step as its own kernel, for graph capture: the time, step and
// buffer parities come from device memory, so a graph captured once is
// replayed for every chunk of coarse steps (kernel boundaries provide the
// ordering and coherence between level-steps)
// ------------------------------------------------------------------------
// The node's constants (level range, buffer parities, coarse step, time
// offset and scale, time fraction) are baked in at capture; the graph is
// recaptured when a regrid changes the level populations or the coarse step
// changes.  Only the start time of the coarse step comes from device memory,
// read where the velocity factors need it.
struct StepArgs {
    int32_t level, first, count, cidx;
    uint32_t mask, pad;
    double off, scale, alpha, dtc;
};

template <int MX, int NT, int EQ, int SEGC = 0>
__global__ void __launch_bounds__(NT, (min_waves<MX, NT, EQ>())) level_step_kernel(Ctx c, StepArgs a, DevState *st) {
    __shared__ typename SmemOf<MX, EQ>::type s;
    const View w{a.mask, a.level < 0 ? -1 : a.level - 1, a.level < 0 ? 1.0 : a.alpha};
    const double dt = a.scale * a.dtc;
    double cfl = 0.0;
    const int p = a.first + xcd_remap(blockIdx.x, a.count);
    if constexpr (EQ == 0) {
        advance_scalar_patch<MX, NT, true, SEGC>(c, w, s, p, a.level, a.off * a.dtc, dt, cfl, &st->ts[a.cidx],
                                                 c.cflp + p);
        store_cfl_slot(c.cflp + p, s.red[15], cfl);
    } else if constexpr (EQ == 2) {
        const double old = cfl_slot_old(c.cflp + p);
        advance_mapped_patch<MX, NT, true>(c, w, s, p, a.level, a.off * a.dtc, dt, cfl, &st->ts[a.cidx]);
        store_cfl_slot(c.cflp + p, old, cfl);
    } else {
        const double old = cfl_slot_old(c.cflp + p);
        advance_swe_patch<MX, NT, true>(c, w, s, p, dt, cfl);
        store_cfl_slot(c.cflp + p, old, cfl);
    }
}

__device__ void fill_times(DevState *st) {
    double t = st->t;
    for (int q = 0; q <= FC_TCHUNK; q++) {
        st->ts[q] = t;
        t = t + st->dt_coarse;
    }
}

__global__ void finish_chunk_kernel(DevState *st, int ncoarse, uint32_t flip) {
    st->t = st->ts[ncoarse];
    st->curmask ^= flip;
    fill_times(st);
}

// ------------------------------------------------------------------------
// support kernels
// ------------------------------------------------------------------------
__global__ void init_tables_kernel(int n, int periodic_x, int periodic_y, double *vt) {
    const double h = 1.0 / (double)n;
    const double sig = sin(M_PI * h) / (M_PI * h);
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int ne = n + 2 * MB + 1, nc = n + 2 * MB;
    for (int ax = 0; ax < 2; ax++) {
        const int per = ax == 0 ? periodic_x : periodic_y;
        double *e = vt + (ax == 0 ? vt_ex(n, MB) : vt_ey(n, MB));
        double *cc = vt + (ax == 0 ? vt_cx(n, MB) : vt_cy(n, MB));
        if (k < ne) {
            int I = k - MB;
            if (per) I = ((I % n) + n) % n;
            const double sx = sin(M_PI * (I * h));
            e[k - MB] = sx * sx;
        }
        if (k < nc) {
            int I = k - MB;
            if (per) I = ((I % n) + n) % n;
            cc[k - MB] = sin(2.0 * M_PI * ((I + 0.5) * h)) * sig;
        }
    }
}

__global__ void set_state_kernel(DevState *st, double t, double dt, uint32_t curmask, int reset_cfl,
                                 unsigned long long *cflp, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k == 0) {
        st->t = t;
        st->dt_coarse = dt;
        st->curmask = curmask;
        st->bar_count = 0;
        if (reset_cfl) st->cfl_bits = 0ull;
        fill_times(st);
    }
    if (reset_cfl && cflp && k < n) cflp[k] = 0ull;
}

__global__ void zero_cfl_kernel(unsigned long long *cflp, int n) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) cflp[k] = 0ull;
}

__global__ void __launch_bounds__(256) export_cfl_kernel(const DevState *st, const unsigned long long *cflp, int n,
                                                            double *cfl, double cfl_max, int32_t *err) {
    __shared__ double red[4];
    double v = 0.0;
    for (int k = threadIdx.x; k < n; k += 256) v = fmax(v, __longlong_as_double((long long)cflp[k]));
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        if (st) m = fmax(m, __longlong_as_double((long long)st->cfl_bits));
        if (m > *cfl) *cfl = m;
        if (cfl_max > 0.0 && m > cfl_max) atomicOr(err, 16);
    }
}

// interiors of the n slots' current buffers <-> save[slot][F][mx][mx]
template <int MX>
__global__ void copy_interiors_kernel(Ctx c, int n, double *save, int restore) {
    constexpr int N = MX + 2 * MB;
    const long long tot = (long long)n * c.F * MX * MX;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < tot; k += (long long)gridDim.x * blockDim.x) {
        const int i = k % MX, j = (k / MX) % MX, f = (k / (MX * MX)) % c.F;
        const int p = (int)(k / ((long long)MX * MX * c.F));
        double *q = buf_of(c, view_of(c), c.info[p].level) + qidx(c.cap, N, f, p, i, j);
        if (restore) *q = save[k];
        else save[k] = *q;
    }
}

// interior data, input-leaf order [n][F][mx][mx] <-> store slots
template <int MX>
__global__ void set_interior_kernel(Ctx c, const int32_t *slot_of_leaf, int n, const double *src) {
    constexpr int N = MX + 2 * MB;
    const long long tot = (long long)n * c.F * MX * MX;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < tot; k += (long long)gridDim.x * blockDim.x) {
        const int i = k % MX, j = (k / MX) % MX, f = (k / (MX * MX)) % c.F;
        const int leaf = (int)(k / ((long long)MX * MX * c.F));
        const int p = slot_of_leaf[leaf];
        buf_of(c, view_of(c), c.info[p].level)[qidx(c.cap, N, f, p, i, j)] = src[k];
    }
}

template <int MX>
__global__ void get_interior_kernel(Ctx c, const int32_t *slot_of_leaf, int n, double *dst, int full) {
    constexpr int N = MX + 2 * MB;
    const int E = full ? N : MX, off = full ? MB : 0;
    const long long tot = (long long)n * c.F * E * E;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < tot; k += (long long)gridDim.x * blockDim.x) {
        const int i = k % E - off, j = (k / E) % E - off, f = (k / (E * E)) % c.F;
        const int leaf = (int)(k / ((long long)E * E * c.F));
        const int p = slot_of_leaf[leaf];
        dst[k] = buf_of(c, view_of(c), c.info[p].level)[qidx(c.cap, N, f, p, i, j)];
    }
}

// maximum that keeps a NaN: once either argument is NaN the result is NaN
__device__ __forceinline__ double nan_max(double a, double b) { return (a > b || a != a) ? a : b; }

// tagging: max over interior of |grad q|^2 with central differences / 2h; a
// NaN anywhere in the patch survives the reduction and raises bit 8 of the
// error flags
template <int MX>
__global__ void __launch_bounds__(256) tag_kernel(Ctx c, const int32_t *slot_of_leaf, int lmin, int lmax,
                                                  double tau_r, double tau_c, int8_t *tags, double *g2out) {
    constexpr int N = MX + 2 * MB;
    __shared__ double red[4];
    const int leaf = blockIdx.x;
    const int p = slot_of_leaf[leaf];
    const PatchInfo P = c.info[p];
    const double h = 1.0 / (double)(MX << P.level);
    const double *q = buf_of(c, view_of(c), P.level);
    double g2 = 0.0;
    for (int k = threadIdx.x; k < MX * MX; k += blockDim.x) {
        const int i = k % MX, j = k / MX;
        const double gx = (q[qidx(c.cap, N, 0, p, i + 1, j)] - q[qidx(c.cap, N, 0, p, i - 1, j)]) / (2.0 * h);
        const double gy = (q[qidx(c.cap, N, 0, p, i, j + 1)] - q[qidx(c.cap, N, 0, p, i, j - 1)]) / (2.0 * h);
        g2 = nan_max(g2, gx * gx + gy * gy);
    }
    for (int o = 32; o > 0; o >>= 1) g2 = nan_max(g2, __shfl_xor(g2, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = g2;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < (int)(blockDim.x >> 6); w++) m = nan_max(m, red[w]);
        int8_t tg = 0;
        if (m != m) atomicOr(c.err, 8);
        else if (m > tau_r * tau_r && P.level < lmax) tg = 1;
        else if (m <= tau_c * tau_c && P.level > lmin) tg = -1;
        tags[leaf] = tg;
        if (g2out) g2out[leaf] = m;
    }
}

// regrid: move every old patch (with ghosts) into buffer 0
template <int MX>
__global__ void consolidate_kernel(Ctx c) {
    constexpr int N = MX + 2 * MB;
    const int p = blockIdx.x;
    const int l = c.info[p].level;
    if (!((c.curmask >> l) & 1u)) return;
    for (int f = 0; f < c.F; f++)
        for (int k = threadIdx.x; k < N * N; k += blockDim.x) {
            const size_t a = (size_t)(f * c.cap + p) * N * N + k;
            c.q0[a] = c.q1[a];
        }
}

// regrid transfer: old data in buffer 0 (old slots), new data to buffer 1
template <int MX>
__global__ void transfer_kernel(Ctx c, const TransferRec *plan) {
    constexpr int N = MX + 2 * MB;
    const int p = blockIdx.x;
    const TransferRec tr = plan[p];
    for (int f = 0; f < c.F; f++)
        for (int k = threadIdx.x; k < MX * MX; k += blockDim.x) {
            const int i = k % MX, j = k / MX;
            double v;
            if (tr.kind == TR_COPY) {
                v = c.q0[qidx(c.cap, N, f, tr.src[0], i, j)];
            } else if (tr.kind == TR_REFINE) {
                const int ic = tr.cx * (MX / 2) + (i >> 1), jc = tr.cy * (MX / 2) + (j >> 1);
                const double dx = (i & 1) ? 1.0 : -1.0, dy = (j & 1) ? 1.0 : -1.0;
                const int s = tr.src[0];
                const double cc = c.q0[qidx(c.cap, N, f, s, ic, jc)];
                const double sx = minmod(c.q0[qidx(c.cap, N, f, s, ic + 1, jc)] - cc, cc - c.q0[qidx(c.cap, N, f, s, ic - 1, jc)]);
                const double sy = minmod(c.q0[qidx(c.cap, N, f, s, ic, jc + 1)] - cc, cc - c.q0[qidx(c.cap, N, f, s, ic, jc - 1)]);
                v = cc + 0.25 * (dx * sx + dy * sy);
            } else {
                const int cx = i >= MX / 2, cy = j >= MX / 2;
                const int s = tr.src[cx + 2 * cy];
                const int fi = 2 * i - cx * MX, fj = 2 * j - cy * MX;
                const double y0 = c.q0[qidx(c.cap, N, f, s, fi, fj)], y1 = c.q0[qidx(c.cap, N, f, s, fi + 1, fj)];
                const double y2 = c.q0[qidx(c.cap, N, f, s, fi, fj + 1)], y3 = c.q0[qidx(c.cap, N, f, s, fi + 1, fj + 1)];
                if (c.mapped) {
                    // area-weighted on a mapped grid; the new patch's cell
                    // (i, j) covers fine cells 2 (I, J) + {0, 1}
                    const PatchInfo P = c.info[p];
                    const int lf = P.level + 1, n = MX << lf;
                    const int I = 2 * (P.ix * MX + i), J = 2 * (P.iy * MX + j);
                    const double a0 = capacity_at(c, lf, n, I, J), a1 = capacity_at(c, lf, n, I + 1, J);
                    const double a2 = capacity_at(c, lf, n, I, J + 1), a3 = capacity_at(c, lf, n, I + 1, J + 1);
                    v = (a0 * y0 + a1 * y1 + a2 * y2 + a3 * y3) / (a0 + a1 + a2 + a3);
                } else {
                    v = 0.25 * (y0 + y1 + y2 + y3);
                }
            }
            c.q1[qidx(c.cap, N, f, p, i, j)] = v;
        }
}

// ------------------------------------------------------------------------
// adaptation on the device (Sec. 4.1, smooth refinement Sec. 4.2), on a map
// of the finest level L = max_level: n = 2^L cells per axis, cell (x, y) at
// index y n + x.  A leaf of level l covers the aligned block of 2^(L-l)
// cells per axis from (ix, iy) << (L-l).
// ------------------------------------------------------------------------
struct AdaptGrid {
    int L, n;            // finest level, cells per axis
    int px, py;          // periodic along x / y
    int lmin, lmax;
};

// owner[c] = the slot of the leaf covering finest cell c
__global__ void paint_owner_kernel(const PatchInfo *info, AdaptGrid g, int32_t *owner) {
    const int s = blockIdx.x;
    const PatchInfo P = info[s];
    const int b = 1 << (g.L - P.level), x0 = P.ix * b, y0 = P.iy * b;
    for (int k = threadIdx.x; k < b * b; k += blockDim.x) owner[(size_t)(y0 + k / b) * g.n + x0 + k % b] = s;
}

// target level of every leaf: its level plus its tag, within [lmin, lmax]
__global__ void target_kernel(const PatchInfo *info, const int32_t *slot_of_leaf, const int8_t *tags, int nleaf,
                              AdaptGrid g, int32_t *target) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nleaf) return;
    const int s = slot_of_leaf[k];
    target[s] = min(g.lmax, max(g.lmin, info[s].level + (int)tags[k]));
}

// finest cell of the level-lq quadrant (X, Y), wrapped where periodic; -1
// outside a wall
__device__ __forceinline__ long long quadrant_cell(const AdaptGrid &g, int lq, int X, int Y) {
    const int nq = 1 << lq;
    if (X < 0 || X >= nq) { if (!g.px) return -1; X = (X + nq) % nq; }
    if (Y < 0 || Y >= nq) { if (!g.py) return -1; Y = (Y + nq) % nq; }
    const int x = lq <= g.L ? X << (g.L - lq) : X >> (lq - g.L), y = lq <= g.L ? Y << (g.L - lq) : Y >> (lq - g.L);
    return (long long)y * g.n + x;
}

// T = the largest target over the leaf and the leaves touching it across a
// face or a corner (the ring of level-(l+1) quadrants around it); with
// smooth == 0 the leaf's own target
__global__ void smooth_kernel(const PatchInfo *info, int nslot, const int32_t *owner, const int32_t *target, AdaptGrid g,
                              int smooth, int32_t *T) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= nslot) return;
    int m = target[s];
    if (smooth) {
        const PatchInfo P = info[s];
        const int lq = P.level + 1;
        for (int dy = -1; dy <= 2; dy++)
            for (int dx = -1; dx <= 2; dx++) {
                if (dx >= 0 && dx <= 1 && dy >= 0 && dy <= 1) continue;
                const long long c = quadrant_cell(g, lq, 2 * P.ix + dx, 2 * P.iy + dy);
                if (c >= 0) m = max(m, target[owner[c]]);
            }
    }
    T[s] = m;
}

// New level of every leaf, painted over its cells: one finer if its T is
// above its level, one coarser if it and its three siblings are all leaves
// whose T is below their level, else unchanged.
__global__ void decide_kernel(const PatchInfo *info, const int32_t *owner, const int32_t *T, AdaptGrid g, int8_t *lev) {
    const int s = blockIdx.x;
    const PatchInfo P = info[s];
    const int l = P.level;
    int nl = l;
    if (T[s] > l && l < g.lmax) {
        nl = l + 1;
    } else if (T[s] < l && l > g.lmin) {
        bool all = true;
        for (int c = 0; c < 4; c++) {
            const int X = (P.ix & ~1) + (c & 1), Y = (P.iy & ~1) + (c >> 1);
            const int o = owner[quadrant_cell(g, l, X, Y)];
            const PatchInfo Q = info[o];
            all = all && Q.level == l && Q.ix == X && Q.iy == Y && T[o] < l;
        }
        if (all) nl = l - 1;
    }
    const int b = 1 << (g.L - l), x0 = P.ix * b, y0 = P.iy * b;
    for (int k = threadIdx.x; k < b * b; k += blockDim.x) lev[(size_t)(y0 + k / b) * g.n + x0 + k % b] = (int8_t)nl;
}

// One pass of 2:1 balance by refinement: every leaf of map `a` (found at the
// origin cell of its block) that touches a cell more than one level finer
// across a face or a corner is refined in map `b` (which starts as a copy of
// `a`); *changed is raised if any was.
__global__ void balance_kernel(const int8_t *a, int8_t *b, AdaptGrid g, int32_t *changed) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (long long)g.n * g.n) return;
    const int x = (int)(c % g.n), y = (int)(c / g.n), l = a[c], w = 1 << (g.L - l);
    if ((x & (w - 1)) || (y & (w - 1))) return;  // not the origin of a leaf
    bool refine = false;
    for (int k = -1; k <= w && !refine; k++) {
        // the perimeter just outside the block: rows y-1 and y+w, columns x-1 and x+w
        const int xs[4] = {x + k, x + k, x - 1, x + w}, ys[4] = {y - 1, y + w, y + k, y + k};
        for (int e = 0; e < 4; e++) {
            const long long q = quadrant_cell(g, g.L, xs[e], ys[e]);
            if (q >= 0 && a[q] > l + 1) refine = true;
        }
    }
    if (!refine || l >= g.lmax) return;
    for (int k = 0; k < w * w; k++) b[(size_t)(y + k / w) * g.n + x + k % w] = (int8_t)(l + 1);
    atomicOr(changed, 1);
}

// the leaves of map `a`: one per block origin, in no particular order
__global__ void extract_kernel(const int8_t *a, AdaptGrid g, int cap, int32_t *count, int32_t *out) {
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= (long long)g.n * g.n) return;
    const int x = (int)(c % g.n), y = (int)(c / g.n), l = a[c], sh = g.L - l, w = 1 << sh;
    if ((x & (w - 1)) || (y & (w - 1))) return;
    const int k = atomicAdd(count, 1);
    if (k < cap) {
        out[3 * k] = l;
        out[3 * k + 1] = x >> sh;
        out[3 * k + 2] = y >> sh;
    }
}

}  // namespace

// ------------------------------------------------------------------------
// launchers
// ------------------------------------------------------------------------
hipError_t launch_adapt_device(const Ctx &c, const int32_t *slot_of_leaf, const int8_t *tags, int nleaf, int L,
                               int periodic_x, int periodic_y, int lmin, int lmax, int smooth, int32_t *owner,
                               int32_t *target, int32_t *T, int8_t *lev_a, int8_t *lev_b, int32_t *flags,
                               hipStream_t s) {
    AdaptGrid g{L, 1 << L, periodic_x, periodic_y, lmin, lmax};
    const long long cells = (long long)g.n * g.n;
    const int cb = (int)((cells + 255) / 256);
    hipLaunchKernelGGL(paint_owner_kernel, dim3(nleaf), dim3(256), 0, s, c.info, g, owner);
    hipLaunchKernelGGL(target_kernel, dim3((nleaf + 255) / 256), dim3(256), 0, s, c.info, slot_of_leaf, tags, nleaf, g,
                       target);
    hipLaunchKernelGGL(smooth_kernel, dim3((nleaf + 255) / 256), dim3(256), 0, s, c.info, nleaf, owner, target, g,
                       smooth, T);
    hipLaunchKernelGGL(decide_kernel, dim3(nleaf), dim3(256), 0, s, c.info, owner, T, g, lev_a);
    (void)cb;
    (void)flags;
    (void)lev_b;
    return hipGetLastError();
}

hipError_t launch_balance_pass(const int8_t *a, int8_t *b, int L, int periodic_x, int periodic_y, int lmin, int lmax,
                               int32_t *changed, hipStream_t s) {
    AdaptGrid g{L, 1 << L, periodic_x, periodic_y, lmin, lmax};
    const long long cells = (long long)g.n * g.n;
    hipError_t e = hipMemcpyAsync(b, a, (size_t)cells, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(balance_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, a, b, g, changed);
    return hipGetLastError();
}

hipError_t launch_extract_leaves(const int8_t *a, int L, int cap, int32_t *count, int32_t *out, hipStream_t s) {
    AdaptGrid g{L, 1 << L, 0, 0, 0, 0};
    const long long cells = (long long)g.n * g.n;
    hipLaunchKernelGGL(extract_kernel, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, a, g, cap, count, out);
    return hipGetLastError();
}
hipError_t launch_init_capacity(int n, double alpha, double *K, hipStream_t s) {
    hipLaunchKernelGGL(init_capacity_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, alpha, K);
    return hipGetLastError();
}

hipError_t launch_init_tables(int level, int mx, int periodic_x, int periodic_y, double *vt, hipStream_t s) {
    const int n = mx << level;
    const int tot = n + 2 * MB + 1;
    hipLaunchKernelGGL(init_tables_kernel, dim3((tot + 255) / 256), dim3(256), 0, s, n, periodic_x, periodic_y, vt);
    return hipGetLastError();
}

hipError_t launch_set_state(DevState *st, double t, double dt, uint32_t curmask, int reset_cfl, unsigned long long *cflp,
                            int n, hipStream_t s) {
    const int nb = (n > 0 ? n : 1) + 255;
    hipLaunchKernelGGL(set_state_kernel, dim3(nb / 256), dim3(256), 0, s, st, t, dt, curmask, reset_cfl, cflp, n);
    return hipGetLastError();
}

hipError_t launch_zero_cfl(unsigned long long *cflp, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(zero_cfl_kernel, dim3((n + 255) / 256), dim3(256), 0, s, cflp, n);
    return hipGetLastError();
}

hipError_t launch_export_cfl(DevState *state, const unsigned long long *cflp, int n, double *cfl_dev,
                             double cfl_max, int32_t *err, hipStream_t s) {
    hipLaunchKernelGGL(export_cfl_kernel, dim3(1), dim3(256), 0, s, state, cflp, n, cfl_dev, cfl_max, err);
    return hipGetLastError();
}

hipError_t launch_copy_interiors(const Ctx &c, int mx, int n, double *save, int restore, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const long long tot = (long long)n * c.F * mx * mx;
    const int blocks = (int)((tot + 255) / 256 < 65536 ? (tot + 255) / 256 : 65536);
    switch (mx) {
        case 8: hipLaunchKernelGGL(copy_interiors_kernel<8>, dim3(blocks), dim3(256), 0, s, c, n, save, restore); break;
        case 16: hipLaunchKernelGGL(copy_interiors_kernel<16>, dim3(blocks), dim3(256), 0, s, c, n, save, restore); break;
        case 32: hipLaunchKernelGGL(copy_interiors_kernel<32>, dim3(blocks), dim3(256), 0, s, c, n, save, restore); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MX>
static hipError_t fill_mx(const Ctx &c, int first, int count, hipStream_t s) {
    if (c.F == 3) hipLaunchKernelGGL((fill_kernel<MX, 3>), dim3(count), dim3(256), 0, s, c, first);
    else if (c.mapped) hipLaunchKernelGGL((fill_kernel<MX, 1, true>), dim3(count), dim3(256), 0, s, c, first);
    else hipLaunchKernelGGL((fill_kernel<MX, 1>), dim3(count), dim3(256), 0, s, c, first);
    return hipGetLastError();
}

hipError_t launch_fill(const Ctx &c, int mx, int first, int count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    switch (mx) {
        case 8: return fill_mx<8>(c, first, count, s);
        case 16: return fill_mx<16>(c, first, count, s);
        case 32: return fill_mx<32>(c, first, count, s);
    }
    return hipErrorInvalidValue;
}

template <int MX, int NT, int SEGC>
static hipError_t adv_scalar(const Ctx &c, int first, int count, int level, double t, double dt, int fused,
                             hipStream_t s) {
    if (fused) hipLaunchKernelGGL((advance_scalar_kernel<MX, NT, true, SEGC>), dim3(count), dim3(NT), 0, s, c, first, count, level, t, dt);
    else hipLaunchKernelGGL((advance_scalar_kernel<MX, NT, false, SEGC>), dim3(count), dim3(NT), 0, s, c, first, count, level, t, dt);
    return hipGetLastError();
}

template <int MX, int NT>
static hipError_t adv_swe(const Ctx &c, int first, int count, double dt, int fused, hipStream_t s) {
    if (fused) hipLaunchKernelGGL((advance_swe_kernel<MX, NT, true>), dim3(count), dim3(NT), 0, s, c, first, count, dt);
    else hipLaunchKernelGGL((advance_swe_kernel<MX, NT, false>), dim3(count), dim3(NT), 0, s, c, first, count, dt);
    return hipGetLastError();
}

hipError_t launch_advance(const Ctx &c, LaunchCfg lc, int level, int first, int count, double t, double dt,
                          int fused, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (c.mapped) {
        // capacity form (fused: ghosts gathered, area-weighted)
#define ADM(MXV, NTV)                                                                                              \
    if (lc.mx == MXV && lc.nt == NTV) {                                                                            \
        if (fused)                                                                                                 \
            hipLaunchKernelGGL((advance_mapped_kernel<MXV, NTV, true>), dim3(count), dim3(NTV), 0, s, c, first, count, level, t, dt); \
        else                                                                                                       \
            hipLaunchKernelGGL((advance_mapped_kernel<MXV, NTV, false>), dim3(count), dim3(NTV), 0, s, c, first, count, level, t, dt); \
        return hipGetLastError();                                                                                  \
    }
        ADM(8, 64) ADM(8, 128) ADM(16, 64) ADM(16, 128) ADM(16, 256) ADM(32, 128) ADM(32, 256) ADM(32, 512)
#undef ADM
        return hipErrorInvalidValue;
    }
    if (c.eq == 0) {
#define ADV(MXV, NTV, SG) \
    if (lc.mx == MXV && lc.nt == NTV && lc.seg == SG) return adv_scalar<MXV, NTV, SG>(c, first, count, level, t, dt, fused, s);
        ADV(8, 64, 0) ADV(8, 128, 0) ADV(16, 64, 0) ADV(16, 128, 0) ADV(16, 256, 0) ADV(32, 128, 0) ADV(32, 256, 0)
        ADV(32, 512, 0)
        // long segments: twice the shortest that fits (see tile_long)
        ADV(16, 128, 8) ADV(16, 256, 8) ADV(32, 256, 16) ADV(32, 512, 8)
#undef ADV
    } else {
#define ADV(MXV, NTV) if (lc.mx == MXV && lc.nt == NTV) return adv_swe<MXV, NTV>(c, first, count, dt, fused, s);
        ADV(8, 64) ADV(8, 128) ADV(8, 192) ADV(16, 256) ADV(16, 384) ADV(16, 512) ADV(16, 640)
#undef ADV
    }
    return hipErrorInvalidValue;
}

// launch variants: scalar advection (64/128 threads at mx = 8; 64-256 at
// mx = 16; 128-512 at mx = 32), shallow water (64/128/192 at mx = 8,
// 256/384/512/640 at mx = 16)
static const void *persistent_select(LaunchCfg lc, int eq) {
#define PS(MXV, NTV, EQV) \
    if (lc.mx == MXV && lc.nt == NTV && eq == EQV) return reinterpret_cast<const void *>(&persistent_kernel<MXV, NTV, EQV>);
    PS(8, 64, 0) PS(8, 128, 0) PS(16, 64, 0) PS(16, 128, 0) PS(16, 256, 0) PS(32, 128, 0) PS(32, 256, 0) PS(32, 512, 0)
    PS(8, 64, 1) PS(8, 128, 1) PS(8, 192, 1) PS(16, 256, 1) PS(16, 384, 1) PS(16, 512, 1) PS(16, 640, 1)
    // eq 2: scalar advection on a mapped grid (capacity form)
    PS(8, 64, 2) PS(8, 128, 2) PS(16, 64, 2) PS(16, 128, 2) PS(16, 256, 2) PS(32, 128, 2) PS(32, 256, 2) PS(32, 512, 2)
#undef PS
    return nullptr;
}

// Workgroups of the persistent kernel that are certainly co-resident: the
// occupancy query, capped by an LDS count that rounds each workgroup's
// allocation up to 2 KiB (a kernel at the edge of the CU's LDS must not be
// counted one workgroup too many: its barrier would then wait on a workgroup
// that cannot start).
int persistent_max_grid(LaunchCfg lc, int eq) {
    const void *fn = persistent_select(lc, eq);
    if (!fn) return 0;
    int per_cu = 0, dev = 0, cus = 0, lds_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, lc.nt, 0) != hipSuccess) return 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess)
        return 0;
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, fn) != hipSuccess) return 0;
    const size_t lds = ((fa.sharedSizeBytes + 2047) / 2048) * 2048;
    if (lds > 0 && lds_cu > 0) {
        const int by_lds = (int)((size_t)lds_cu / lds);
        if (by_lds < per_cu) per_cu = by_lds;
    }
    return per_cu * cus;
}

static const void *level_step_select(LaunchCfg lc, int eq) {
#define PS(MXV, NTV, EQV) \
    if (lc.mx == MXV && lc.nt == NTV && eq == EQV && lc.seg == 0) \
        return reinterpret_cast<const void *>(&level_step_kernel<MXV, NTV, EQV>);
#define PL(MXV, NTV, SG) \
    if (lc.mx == MXV && lc.nt == NTV && eq == 0 && lc.seg == SG) \
        return reinterpret_cast<const void *>(&level_step_kernel<MXV, NTV, 0, SG>);
    PS(8, 64, 0) PS(8, 128, 0) PS(16, 64, 0) PS(16, 128, 0) PS(16, 256, 0) PS(32, 128, 0) PS(32, 256, 0) PS(32, 512, 0)
    PS(8, 64, 1) PS(8, 128, 1) PS(8, 192, 1) PS(16, 256, 1) PS(16, 384, 1) PS(16, 512, 1) PS(16, 640, 1)
    PL(16, 128, 8) PL(16, 256, 8) PL(32, 256, 16) PL(32, 512, 8)
    // eq 2: scalar advection on a mapped grid (capacity form)
    PS(8, 64, 2) PS(8, 128, 2) PS(16, 64, 2) PS(16, 128, 2) PS(16, 256, 2) PS(32, 128, 2) PS(32, 256, 2) PS(32, 512, 2)
#undef PL
#undef PS
    return nullptr;
}

hipError_t launch_level_step(const Ctx &c, LaunchCfg lc, const SchedEntry &e, int first, int count, int cidx,
                             uint32_t mask, double dt_coarse, DevState *st, hipStream_t s) {
    const void *fn = level_step_select(lc, c.mapped ? 2 : c.eq);
    if (!fn) return hipErrorInvalidValue;
    Ctx cc = c;
    StepArgs a{e.level, first, count, cidx, mask, 0u, e.off, e.scale, e.alpha, dt_coarse};
    void *args[] = {&cc, &a, &st};
    return hipLaunchKernel(fn, dim3(count > 0 ? count : 1), dim3(lc.nt), args, 0, s);
}

hipError_t launch_finish_chunk(DevState *st, int ncoarse, uint32_t flip, hipStream_t s) {
    hipLaunchKernelGGL(finish_chunk_kernel, dim3(1), dim3(1), 0, s, st, ncoarse, flip);
    return hipGetLastError();
}

hipError_t launch_persistent(const Ctx &c, LaunchCfg lc, const SchedEntry *sched, int nsched,
                             const LevelRange *ranges_dev, int ncoarse, DevState *state, int grid, hipStream_t s) {
    const void *fn = persistent_select(lc, c.mapped ? 2 : c.eq);
    if (!fn || grid <= 0 || ncoarse <= 0) return hipErrorInvalidValue;
    Ctx cc = c;
    void *args[] = {&cc, (void *)&sched, &nsched, (void *)&ranges_dev, &ncoarse, &state};
    return hipLaunchKernel(fn, dim3(grid), dim3(lc.nt), args, 0, s);
}

template <int MX>
static void setget(const Ctx &c, const int32_t *sl, int n, const double *src, double *dst, int full, hipStream_t s) {
    const long long tot = (long long)n * c.F * MX * MX;
    const int blocks = (int)((tot + 255) / 256 < 65536 ? (tot + 255) / 256 : 65536);
    if (src) hipLaunchKernelGGL(set_interior_kernel<MX>, dim3(blocks), dim3(256), 0, s, c, sl, n, src);
    else hipLaunchKernelGGL(get_interior_kernel<MX>, dim3(blocks), dim3(256), 0, s, c, sl, n, dst, full);
}

hipError_t launch_set_interior(const Ctx &c, int mx, const int32_t *slot_of_leaf, int n, const double *src,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    switch (mx) {
        case 8: setget<8>(c, slot_of_leaf, n, src, nullptr, 0, s); break;
        case 16: setget<16>(c, slot_of_leaf, n, src, nullptr, 0, s); break;
        case 32: setget<32>(c, slot_of_leaf, n, src, nullptr, 0, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_get_interior(const Ctx &c, int mx, const int32_t *slot_of_leaf, int n, double *dst, int full,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    switch (mx) {
        case 8: setget<8>(c, slot_of_leaf, n, nullptr, dst, full, s); break;
        case 16: setget<16>(c, slot_of_leaf, n, nullptr, dst, full, s); break;
        case 32: setget<32>(c, slot_of_leaf, n, nullptr, dst, full, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_tag(const Ctx &c, int mx, const int32_t *slot_of_leaf, int n, int lmin, int lmax, double tau_r,
                      double tau_c, int8_t *tags, double *g2, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    switch (mx) {
        case 8: hipLaunchKernelGGL(tag_kernel<8>, dim3(n), dim3(64), 0, s, c, slot_of_leaf, lmin, lmax, tau_r, tau_c, tags, g2); break;
        case 16: hipLaunchKernelGGL(tag_kernel<16>, dim3(n), dim3(256), 0, s, c, slot_of_leaf, lmin, lmax, tau_r, tau_c, tags, g2); break;
        case 32: hipLaunchKernelGGL(tag_kernel<32>, dim3(n), dim3(256), 0, s, c, slot_of_leaf, lmin, lmax, tau_r, tau_c, tags, g2); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_step_leaf(const Ctx &c, int mx, int level, int first, int count, double t, double dt,
                            const int32_t *leaf_of_slot, const double *q_in, double *q_out, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const LeafIO io{q_in, q_out, leaf_of_slot};
    if (!((c.complete >> level) & 1u)) return hipErrorInvalidValue;  // neighbour slots from the Morton index
    switch (mx) {
        case 8: hipLaunchKernelGGL((step_leaf_kernel<8, 64>), dim3(count), dim3(64), 0, s, c, first, count, level, t, dt, io); break;
        case 16: hipLaunchKernelGGL((step_leaf_kernel<16, 256>), dim3(count), dim3(256), 0, s, c, first, count, level, t, dt, io); break;
        case 32: hipLaunchKernelGGL((step_leaf_kernel<32, 256>), dim3(count), dim3(256), 0, s, c, first, count, level, t, dt, io); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int MX, int NT>
static void launch_adjoint_mx(const Ctx &c, int level, int first, int count, double t, double dt,
                              const int32_t *leaf_of_slot, const double *q_in, const double *lam_in, double *lam_out,
                              hipStream_t s) {
    switch (c.lim) {
        case 1: hipLaunchKernelGGL((adjoint_kernel<MX, NT, 1>), dim3(count), dim3(NT), 0, s, c, level, first, count, t, dt, leaf_of_slot, q_in, lam_in, lam_out); break;
        case 2: hipLaunchKernelGGL((adjoint_kernel<MX, NT, 2>), dim3(count), dim3(NT), 0, s, c, level, first, count, t, dt, leaf_of_slot, q_in, lam_in, lam_out); break;
        case 3: hipLaunchKernelGGL((adjoint_kernel<MX, NT, 3>), dim3(count), dim3(NT), 0, s, c, level, first, count, t, dt, leaf_of_slot, q_in, lam_in, lam_out); break;
        default: hipLaunchKernelGGL((adjoint_kernel<MX, NT, 0>), dim3(count), dim3(NT), 0, s, c, level, first, count, t, dt, leaf_of_slot, q_in, lam_in, lam_out); break;
    }
}

hipError_t launch_adjoint(const Ctx &c, int mx, int level, int first, int count, double t, double dt,
                          const int32_t *leaf_of_slot, const double *q_in, const double *lam_in, double *lam_out,
                          hipStream_t s) {
    if (count <= 0) return hipSuccess;
    if (!((c.complete >> level) & 1u)) return hipErrorInvalidValue;  // neighbour slots from the Morton index
    switch (mx) {
        case 8: launch_adjoint_mx<8, 64>(c, level, first, count, t, dt, leaf_of_slot, q_in, lam_in, lam_out, s); break;
        case 16: launch_adjoint_mx<16, 128>(c, level, first, count, t, dt, leaf_of_slot, q_in, lam_in, lam_out, s); break;
        case 32: launch_adjoint_mx<32, 256>(c, level, first, count, t, dt, leaf_of_slot, q_in, lam_in, lam_out, s); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_consolidate(const Ctx &c, int mx, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    switch (mx) {
        case 8: hipLaunchKernelGGL(consolidate_kernel<8>, dim3(n), dim3(256), 0, s, c); break;
        case 16: hipLaunchKernelGGL(consolidate_kernel<16>, dim3(n), dim3(256), 0, s, c); break;
        case 32: hipLaunchKernelGGL(consolidate_kernel<32>, dim3(n), dim3(256), 0, s, c); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_transfer(const Ctx &c, int mx, const TransferRec *plan, int n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    switch (mx) {
        case 8: hipLaunchKernelGGL(transfer_kernel<8>, dim3(n), dim3(64), 0, s, c, plan); break;
        case 16: hipLaunchKernelGGL(transfer_kernel<16>, dim3(n), dim3(256), 0, s, c, plan); break;
        case 32: hipLaunchKernelGGL(transfer_kernel<32>, dim3(n), dim3(256), 0, s, c, plan); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}
