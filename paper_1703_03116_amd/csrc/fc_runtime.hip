// fc_runtime.hip -- host runtime and C ABI of the AMR library (include/fc.h).
//
// Host side: leaf validation (tiling, 2:1 balance over faces and corners,
// Prop. 2.1 ghost width), store order (level, then Morton index inside a
// level, Sec. 2), per-patch neighbour records for the 20 neighbour cases of
// Sec. 2.3 (face: same / fine-lo / fine-hi / coarse, corner: same / fine /
// coarse, plus walls), the multirate level-step schedule, host adaptation
// (tag -> refine/coarsen -> balance, Sec. 4.1) and the regrid transfer plan.
// Device side: launches on the caller's stream; device memory is the
// caller's (two patch buffers and one workspace).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/fc.h"
#include "fc_internal.h"

// Per-slot Courant maxima of fc_advance_level_noalloc: a fixed array in
// device memory instead of the caller's workspace.  Host code must never pass
// `scratch` itself to a kernel (in host code the name is only a stand-in);
// it uses the device address that scratch_ptr() obtained for the current
// device.
constexpr int kNoallocSlots = 65536;  // 512 KiB on every device the library runs on
static __device__ __align__(256) unsigned long long scratch[kNoallocSlots];

namespace {

thread_local std::string g_err;

fc_status fail(fc_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

// A failed HIP call is reported to the caller and the runtime's sticky
// last-error state is cleared, so the caller's next HIP call does not see it.
#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) {                                                                   \
            (void)hipGetLastError();                                                              \
            return fail(FC_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));           \
        }                                                                                         \
    } while (0)

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
unsigned long long *g_scratch_ptr[kMaxDevices] = {};

fc_status scratch_ptr(unsigned long long **out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FC_ERR_HIP, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(FC_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        g_scratch_ptr[dev] = (unsigned long long *)p;
    }
    *out = g_scratch_ptr[dev];
    return FC_OK;
}

inline uint64_t key3(int l, int ix, int iy) {
    return ((uint64_t)(uint32_t)l << 56) | ((uint64_t)(uint32_t)iy << 28) | (uint64_t)(uint32_t)ix;
}

inline uint64_t morton(uint32_t x, uint32_t y) {
    uint64_t r = 0;
    for (int b = 0; b < 28; b++) r |= (uint64_t)((x >> b) & 1u) << (2 * b) | (uint64_t)((y >> b) & 1u) << (2 * b + 1);
    return r;
}

constexpr int MBK = 2;  // ghost layers the kernels use
// finest level of a store whose adaptation can run on the device (its
// level maps hold 4^max_level cells: 1 M at level 10, 6 MB of workspace)
constexpr int kAdaptMaxLevel = 10;
static_assert(sizeof(fc_leaf) == 3 * sizeof(int32_t), "leaf lists cross the ABI as (level, ix, iy) int32 triples");

// Leaves inside the library are in brick coordinates: a brick of nbx x nby
// unit blocks (one block: the unit square), level-l quadrant (ix, iy) with
// 0 <= ix < nbx 2^l, 0 <= iy < nby 2^l.  Blocks may have their own index
// orientation (Sec. 2.3); leaves cross the ABI in the blocks' own
// coordinates and are converted at the boundary (to_brick / to_own).
struct Mesh {
    int mx = 0;
    int nbx = 1, nby = 1;
    int bc[4] = {0, 0, 0, 0};
    std::vector<fc_leaf> lv;                 // store order
    std::unordered_map<uint64_t, int> at;    // (level, ix, iy) -> slot

    int find(int l, int ix, int iy) const {
        if (l < 0 || l > 30) return -1;
        if (ix < 0 || iy < 0 || ix >= (nbx << l) || iy >= (nby << l)) return -1;
        auto it = at.find(key3(l, ix, iy));
        return it == at.end() ? -1 : it->second;
    }
    bool covered_le(int lf, int X, int Y, int lcap) const {
        for (int l2 = lcap; l2 >= 0; l2--)
            if (find(l2, X >> (lf - l2), Y >> (lf - l2)) >= 0) return true;
        return false;
    }
    // 2:1 balance over faces and corners, with periodic wrap where periodic
    bool balanced_at(const fc_leaf &L) const {
        const int lf = L.level + 2, nfx = nbx << lf, nfy = nby << lf, x0 = L.ix * 4, y0 = L.iy * 4;
        for (int dy = -1; dy <= 1; dy++)
            for (int dx = -1; dx <= 1; dx++) {
                if (!dx && !dy) continue;
                const int xa = dx < 0 ? x0 - 1 : dx > 0 ? x0 + 4 : x0, xb = dx < 0 ? x0 - 1 : dx > 0 ? x0 + 4 : x0 + 3;
                const int ya = dy < 0 ? y0 - 1 : dy > 0 ? y0 + 4 : y0, yb = dy < 0 ? y0 - 1 : dy > 0 ? y0 + 4 : y0 + 3;
                for (int yy = ya; yy <= yb; yy++)
                    for (int xx = xa; xx <= xb; xx++) {
                        int X = xx, Y = yy;
                        if (X < 0 || X >= nfx) {
                            if (bc[X < 0 ? 0 : 1] != FC_BC_PERIODIC) continue;
                            X = (X + nfx) % nfx;
                        }
                        if (Y < 0 || Y >= nfy) {
                            if (bc[Y < 0 ? 2 : 3] != FC_BC_PERIODIC) continue;
                            Y = (Y + nfy) % nfy;
                        }
                        if (!covered_le(lf, X, Y, L.level + 1)) return false;
                    }
            }
        return true;
    }
    void index() {
        at.clear();
        at.reserve(lv.size() * 2);
        for (size_t k = 0; k < lv.size(); k++) at[key3(lv[k].level, lv[k].ix, lv[k].iy)] = (int)k;
    }
};

// Validate a leaf list (any order).  Returns FC_OK or an error status.
fc_status validate(const Mesh &m, const std::vector<fc_leaf> &L) {
    Mesh t;
    t.mx = m.mx;
    t.nbx = m.nbx;
    t.nby = m.nby;
    std::copy(m.bc, m.bc + 4, t.bc);
    t.lv = L;
    t.index();
    if (t.at.size() != L.size()) return fail(FC_ERR_COVER, "duplicate leaves");
    long double area = 0;
    for (const auto &q : L) {
        if (q.level < 0 || q.level > 20) return fail(FC_ERR_ARG, "leaf level out of range");
        if (q.ix < 0 || q.iy < 0 || q.ix >= (m.nbx << q.level) || q.iy >= (m.nby << q.level))
            return fail(FC_ERR_ARG, "leaf coordinates out of range");
        for (int a = 1; a <= q.level; a++)
            if (t.find(q.level - a, q.ix >> a, q.iy >> a) >= 0) return fail(FC_ERR_COVER, "overlapping leaves");
        area += ldexpl(1.0L, -2 * q.level);
    }
    if (fabsl(area - (long double)m.nbx * m.nby) > 1e-15L)
        return fail(FC_ERR_COVER, "leaves do not tile the unit square (the brick)");
    for (const auto &q : L)
        if (!t.balanced_at(q)) return fail(FC_ERR_UNBALANCED, "leaves are not 2:1 balanced");
    return FC_OK;
}

}  // namespace

struct fc_patchstore {
    fc_config cfg;
    int mx = 0, N = 0, F = 1;
    Mesh mesh;
    // brick of mesh.nbx x mesh.nby blocks: orientation code per block
    // (bx + nbx by); `multiblock` unless the brick is one block of code 0
    // (then the one-block fast paths are off)
    std::vector<int> ori;
    bool multiblock = false;
    std::vector<int32_t> slot_of_leaf, leaf_of_slot;  // input order <-> store order
    std::vector<PatchInfo> info;
    std::vector<NbrRec> nbr;
    LevelRange lr;
    uint32_t curmask = 0;
    double t = 0.0;
    int nt = 0;  // threads per patch of the advance kernels
    int seg = 0;  // scalar sweeps: cells per segment (0: the shortest that fits nt)
    // device
    double *q0 = nullptr, *q1 = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    size_t off_info = 0, off_nbr = 0, off_sl = 0, off_ls = 0, off_lr = 0, off_sched = 0, off_state = 0,
           off_plan = 0, off_tag = 0, off_cfl = 0, off_cflv = 0, off_save = 0, off_vt[FC_MAXLEV] = {0},
           off_mk[FC_MAXLEV] = {0};
    // adaptation on the device (max_level <= kAdaptMaxLevel): owner map, two
    // level maps of the finest level, per-slot target and maximum, leaf list,
    // flags (0: changed, 1: leaf count)
    size_t off_own = 0, off_lma = 0, off_lmb = 0, off_tgt = 0, off_tmax = 0, off_lout = 0, off_aflags = 0;
    bool dev_adapt = false;
    std::vector<SchedEntry> sched;
    int pgrid = 0;
    int pgrid_user = 0;  // grid override of the persistent kernel (0: occupancy)
    // Captured graphs, each for `n` coarse steps of one execution form.
    // Level-step graphs carry the buffer parities and the coarse step as node
    // constants, so they are keyed by (n, mask, dt); the persistent kernel
    // reads both from device memory and is keyed by (n, grid).  Every graph
    // is for the current launch variant; a regrid or a variant change drops
    // them all.  At most kMaxGraphs are kept (least recently used goes).
    struct Graph {
        hipGraphExec_t exec = nullptr;
        hipGraph_t graph = nullptr;
        int mode = 0, n = 0, grid = 0;
        uint32_t mask = 0;
        double dt = 0.0;
        uint64_t used = 0;
    };
    static constexpr int kMaxGraphs = 8;
    std::vector<Graph> graphs;
    uint64_t graph_clock = 0;
    hipStream_t cap_stream = nullptr;  // private stream the graph is captured on
};

namespace {

int nfields(const fc_config &c) { return c.equation == FC_EQ_SWE ? 3 : 1; }

// store order of a leaf list: by level, then by Morton index inside a level
std::vector<int> store_order(const std::vector<fc_leaf> &input) {
    std::vector<int> order(input.size());
    for (size_t k = 0; k < input.size(); k++) order[k] = (int)k;
    std::sort(order.begin(), order.end(), [&](int a, int b) {
        if (input[a].level != input[b].level) return input[a].level < input[b].level;
        return morton(input[a].ix, input[a].iy) < morton(input[b].ix, input[b].iy);
    });
    return order;
}

// ---- block orientations (Sec. 2.3) ----------------------------------------
// Code bits: 0 exchanges a block's two index directions, then 1 reverses the
// brick's first direction and 2 its second.  Own index (a, b) of a block with
// n cells (or quadrants) per side <-> brick index inside the block; both maps
// extend linearly beyond [0, n) (ghost cells).
inline void own_to_brick(int code, int n, int a, int b, int &x, int &y) {
    const int p = (code & 1) ? b : a, q = (code & 1) ? a : b;
    x = (code & 2) ? n - 1 - p : p;
    y = (code & 4) ? n - 1 - q : q;
}
inline void brick_to_own(int code, int n, int x, int y, int &a, int &b) {
    const int p = (code & 2) ? n - 1 - x : x, q = (code & 4) ? n - 1 - y : y;
    a = (code & 1) ? q : p;
    b = (code & 1) ? p : q;
}
int block_code(const fc_patchstore *ps, int l, int ix, int iy) {
    const int bx = ix >> l, by = iy >> l;
    if (ps->ori.empty() || bx < 0 || by < 0 || bx >= ps->mesh.nbx || by >= ps->mesh.nby) return 0;
    return ps->ori[bx + ps->mesh.nbx * by];
}
// a leaf in own coordinates -> brick coordinates, and back (same block)
fc_leaf to_brick(const fc_patchstore *ps, const fc_leaf &q) {
    const int n = 1 << q.level, bx = q.ix >> q.level, by = q.iy >> q.level;
    int x, y;
    own_to_brick(block_code(ps, q.level, q.ix, q.iy), n, q.ix - bx * n, q.iy - by * n, x, y);
    return fc_leaf{q.level, bx * n + x, by * n + y};
}
fc_leaf to_own(const fc_patchstore *ps, const fc_leaf &q) {
    const int n = 1 << q.level, bx = q.ix >> q.level, by = q.iy >> q.level;
    int a, b;
    brick_to_own(block_code(ps, q.level, q.ix, q.iy), n, q.ix - bx * n, q.iy - by * n, a, b);
    return fc_leaf{q.level, bx * n + a, by * n + b};
}
// Brick index of cell (i, j) of leaf P (brick coordinates), counted in P's
// own indices from its first cell, at the resolution of level r >= P.level.
void cell_to_brick(const fc_patchstore *ps, const fc_leaf &P, int r, int i, int j, int64_t &X, int64_t &Y) {
    const fc_leaf own = to_own(ps, P);
    const int l = P.level, sc = ps->mx << (r - l), n = ps->mx << r;
    const int bx = P.ix >> l, by = P.iy >> l;
    int x, y;
    own_to_brick(block_code(ps, l, P.ix, P.iy), n, (own.ix - (bx << l)) * sc + i, (own.iy - (by << l)) * sc + j, x, y);
    X = (int64_t)bx * n + x;
    Y = (int64_t)by * n + y;
}
// the inverse for leaf N: its own index of the level-r cell at brick index
// (X, Y) (in N's block or a linear extension of it)
void brick_to_cell(const fc_patchstore *ps, const fc_leaf &N, int r, int64_t X, int64_t Y, int &i, int &j) {
    const fc_leaf own = to_own(ps, N);
    const int l = N.level, sc = ps->mx << (r - l), n = ps->mx << r;
    const int bx = N.ix >> l, by = N.iy >> l;
    int a, b;
    brick_to_own(block_code(ps, l, N.ix, N.iy), n, (int)(X - (int64_t)bx * n), (int)(Y - (int64_t)by * n), a, b);
    i = a - (own.ix - (bx << l)) * sc;
    j = b - (own.iy - (by << l)) * sc;
}

// store order, level ranges, patch info and neighbour records
void build_metadata(fc_patchstore *ps, const std::vector<fc_leaf> &input) {
    const int n = (int)input.size();
    const std::vector<int> order = store_order(input);
    ps->mesh.lv.resize(n);
    ps->slot_of_leaf.assign(n, 0);
    ps->leaf_of_slot.assign(n, 0);
    for (int s = 0; s < n; s++) {
        ps->mesh.lv[s] = input[order[s]];
        ps->leaf_of_slot[s] = order[s];
        ps->slot_of_leaf[order[s]] = s;
    }
    ps->mesh.index();
    for (int l = 0; l < FC_MAXLEV; l++) { ps->lr.start[l] = 0; ps->lr.count[l] = 0; }
    for (int s = n - 1; s >= 0; s--) { ps->lr.start[ps->mesh.lv[s].level] = s; }
    for (int s = 0; s < n; s++) ps->lr.count[ps->mesh.lv[s].level]++;

    const int mx = ps->mx;
    const int *bc = ps->cfg.bc;
    ps->info.assign(n, PatchInfo{});
    ps->nbr.assign((size_t)n * FC_NREC, NbrRec{NB_NONE, 0, 0, 0});
    // representative cell of each record: faces W, E, S, N (two halves each), corners SW, SE, NW, NE
    const int rep[FC_NREC][2] = {{-1, 0}, {-1, mx / 2}, {mx, 0}, {mx, mx / 2}, {0, -1}, {mx / 2, -1},
                                 {0, mx}, {mx / 2, mx}, {-1, -1}, {mx, -1}, {-1, mx}, {mx, mx}};
    for (int s = 0; s < n; s++) {
        const fc_leaf P = ps->mesh.lv[s];
        const int nq = 1 << P.level;
        int walls = 0;
        if (P.ix == 0 && bc[0] == FC_BC_REFLECT) walls |= 1;
        if (P.ix == nq - 1 && bc[1] == FC_BC_REFLECT) walls |= 2;
        if (P.iy == 0 && bc[2] == FC_BC_REFLECT) walls |= 4;
        if (P.iy == nq - 1 && bc[3] == FC_BC_REFLECT) walls |= 8;  // (walls only on one block)
        ps->info[s] = PatchInfo{P.level, P.ix, P.iy, walls | (block_code(ps, P.level, P.ix, P.iy) << 8)};
    }
    for (int s = 0; s < n; s++) {
        const fc_leaf P = ps->mesh.lv[s];
        const int l = P.level;
        const int64_t W = (int64_t)ps->mesh.nbx * (mx << l), H = (int64_t)ps->mesh.nby * (mx << l);
        for (int r = 0; r < FC_NREC; r++) {
            const int ri = rep[r][0], rj = rep[r][1];
            int64_t X0, Y0;
            cell_to_brick(ps, P, l, ri, rj, X0, Y0);
            int64_t I = X0, J = Y0;
            bool wall = false;
            if (I < 0 || I >= W) { if (bc[I < 0 ? 0 : 1] == FC_BC_PERIODIC) I = (I + W) % W; else wall = true; }
            if (J < 0 || J >= H) { if (bc[J < 0 ? 2 : 3] == FC_BC_PERIODIC) J = (J + H) % H; else wall = true; }
            if (wall) continue;
            // point location: the level-l quadrant, its parent, or a child
            int kind = NB_NONE, id = -1;
            if ((id = ps->mesh.find(l, (int)(I / mx), (int)(J / mx))) >= 0) kind = NB_SAME;
            else if ((id = ps->mesh.find(l - 1, (int)(I / mx) >> 1, (int)(J / mx) >> 1)) >= 0) kind = NB_COARSE;
            else if ((id = ps->mesh.find(l + 1, (int)(2 * I / mx), (int)(2 * J / mx))) >= 0) kind = NB_FINE;
            else continue;  // cannot happen on a validated mesh
            // The index transform of eq. transform, P's own indices -> the
            // neighbour's own, taken through the brick's indices (with the
            // periodic image of the representative cell) at three points: a
            // fine neighbour's at the fine resolution, the others' at P's.
            const int sc = kind == NB_FINE ? 2 : 1, rr = l + sc - 1;
            const int64_t dX = (I - X0) * sc, dY = (J - Y0) * sc;
            const fc_leaf Nb = ps->mesh.lv[id];
            const int pi[3] = {sc * ri, sc * ri + 1, sc * ri}, pj[3] = {sc * rj, sc * rj, sc * rj + 1};
            int g[3][2];
            for (int t = 0; t < 3; t++) {
                int64_t X, Y;
                cell_to_brick(ps, P, rr, pi[t], pj[t], X, Y);
                brick_to_cell(ps, Nb, rr, X + dX, Y + dY, g[t][0], g[t][1]);
            }
            const int a00 = g[1][0] - g[0][0], a10 = g[1][1] - g[0][1];
            const int a01 = g[2][0] - g[0][0], a11 = g[2][1] - g[0][1];
            int code;
            if (a01 == 0 && a10 == 0 && std::abs(a00) == 1 && std::abs(a11) == 1)
                code = (a00 < 0 ? 2 : 0) | (a11 < 0 ? 4 : 0);
            else if (a00 == 0 && a11 == 0 && std::abs(a01) == 1 && std::abs(a10) == 1)
                code = 1 | (a01 < 0 ? 2 : 0) | (a10 < 0 ? 4 : 0);
            else
                continue;  // cannot happen: orientations compose to a signed permutation
            const int ta = (code & 1) ? pj[0] : pi[0], tb = (code & 1) ? pi[0] : pj[0];
            int fx = g[0][0] - ((code & 2) ? -ta : ta), fy = g[0][1] - ((code & 4) ? -tb : tb);
            if (kind == NB_FINE) {
                // the first of the four fine cells has the smallest index in
                // each direction: one less where A negates
                if (code & 2) fx -= 1;
                if (code & 4) fy -= 1;
            }
            ps->nbr[(size_t)s * FC_NREC + r] = NbrRec{kind | ((ps->info[id].walls & 15) << 4) | (code << 8), id, fx, fy};
        }
    }
}

// multirate recursion (coarse first): level l steps, then two half steps of l+1
void gen_sched(std::vector<SchedEntry> &out, int l, int lmax, double off, double scale, double alpha) {
    out.push_back(SchedEntry{l, 0, off, scale, alpha});
    if (l < lmax) {
        gen_sched(out, l + 1, lmax, off, 0.5 * scale, 0.0);
        gen_sched(out, l + 1, lmax, off + 0.5 * scale, 0.5 * scale, 0.5);
    }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

void layout_workspace(fc_patchstore *ps) {
    const size_t cap = (size_t)ps->cfg.capacity;
    size_t o = 0;
    ps->off_state = o; o = align256(o + sizeof(DevState));
    ps->off_lr = o; o = align256(o + sizeof(LevelRange));
    ps->off_sched = o; o = align256(o + sizeof(SchedEntry) * ps->sched.size());
    ps->off_info = o; o = align256(o + sizeof(PatchInfo) * cap);
    ps->off_nbr = o; o = align256(o + sizeof(NbrRec) * cap * FC_NREC);
    ps->off_sl = o; o = align256(o + sizeof(int32_t) * cap);
    ps->off_ls = o; o = align256(o + sizeof(int32_t) * cap);
    ps->off_plan = o; o = align256(o + sizeof(TransferRec) * cap);
    ps->off_tag = o; o = align256(o + sizeof(double) * cap);
    ps->off_cfl = o; o = align256(o + sizeof(double) * cap);
    ps->off_cflv = o; o = align256(o + sizeof(double));
    ps->off_save = o;  // interiors kept across a coarse step that may be rejected
    if (ps->cfg.cfl_max > 0) o = align256(o + sizeof(double) * cap * ps->F * ps->mx * ps->mx);
    ps->dev_adapt = ps->cfg.max_level <= kAdaptMaxLevel && !ps->multiblock;
    if (ps->dev_adapt) {
        const size_t cells = (size_t)1 << (2 * ps->cfg.max_level);
        ps->off_own = o; o = align256(o + sizeof(int32_t) * cells);
        ps->off_lma = o; o = align256(o + cells);
        ps->off_lmb = o; o = align256(o + cells);
        ps->off_tgt = o; o = align256(o + sizeof(int32_t) * cap);
        ps->off_tmax = o; o = align256(o + sizeof(int32_t) * cap);
        ps->off_lout = o; o = align256(o + 3 * sizeof(int32_t) * cap);
        ps->off_aflags = o; o = align256(o + 4 * sizeof(int32_t));
    }
    for (int l = 0; l < FC_MAXLEV; l++) {
        ps->off_vt[l] = o;
        if (l >= ps->cfg.min_level && l <= ps->cfg.max_level && ps->cfg.velocity == FC_VEL_SWIRL)
            o = align256(o + sizeof(double) * (size_t)vt_size(ps->mx << l, MBK));
    }
    for (int l = 0; l < FC_MAXLEV; l++) {
        ps->off_mk[l] = o;
        if (l >= ps->cfg.min_level && l <= ps->cfg.max_level && ps->cfg.map_alpha != 0.0)
            o = align256(o + sizeof(double) * (size_t)(ps->mx << l));
    }
    ps->ws_bytes = o;
}

unsigned long long *cflp(const fc_patchstore *ps) { return (unsigned long long *)(ps->ws + ps->off_cfl); }

Ctx make_ctx(const fc_patchstore *ps) {
    Ctx c;
    memset(&c, 0, sizeof(c));
    c.q0 = ps->q0; c.q1 = ps->q1;
    c.info = (const PatchInfo *)(ps->ws + ps->off_info);
    c.nbr = (const NbrRec *)(ps->ws + ps->off_nbr);
    c.cap = (int32_t)ps->cfg.capacity;
    c.F = ps->F; c.eq = ps->cfg.equation; c.lim = ps->cfg.limiter;
    c.curmask = ps->curmask;
    c.clevel = -1; c.alpha = 1.0;
    for (int l = 0; l < FC_MAXLEV; l++)
        c.vt[l] = (ps->cfg.velocity == FC_VEL_SWIRL && l >= ps->cfg.min_level && l <= ps->cfg.max_level)
                      ? (const double *)(ps->ws + ps->off_vt[l] ) : nullptr;
    c.velocity = ps->cfg.velocity;
    c.vel_u = ps->cfg.vel_params[0]; c.vel_v = ps->cfg.vel_params[1]; c.vel_T = ps->cfg.vel_params[0];
    c.vel_invT = ps->cfg.velocity == FC_VEL_SWIRL ? 1.0 / ps->cfg.vel_params[0] : 0.0;
    c.g = ps->cfg.gravity;
    c.err = (int32_t *)(ps->ws + ps->off_state + offsetof(DevState, err));
    c.cflp = cflp(ps);
    // Streaming stores for the advance output where they measured faster:
    // while both solution buffers fit the XCDs' L2 caches several times over
    // (<= 48 MiB: the end-of-launch write-back of dirty lines no longer
    // trails the last workgroup) and once they exceed the 256 MB Infinity
    // Cache (the next step reads from HBM anyway); in between, plain stores
    // keep the next step's input in the Infinity Cache.
    const double foot = 2.0 * 8.0 * (double)ps->F * (double)ps->N * ps->N * (double)ps->mesh.lv.size();
    c.stream_out = (foot <= 48.0 * 1048576.0 || foot >= 256.0 * 1048576.0) ? 1 : 0;
    c.mapped = ps->cfg.map_alpha != 0.0;
    for (int l = 0; l < FC_MAXLEV; l++)
        c.mk[l] = (c.mapped && l >= ps->cfg.min_level && l <= ps->cfg.max_level)
                      ? (const double *)(ps->ws + ps->off_mk[l]) : nullptr;
    const bool per = ps->cfg.bc[0] == FC_BC_PERIODIC && ps->cfg.bc[2] == FC_BC_PERIODIC;
    for (int l = 0; l < FC_MAXLEV; l++) {
        c.lstart[l] = ps->lr.start[l];
        if (per && !ps->multiblock && l < 16 && ps->lr.count[l] == (1 << (2 * l))) c.complete |= 1u << l;
    }
    return c;
}

DevState *dstate(fc_patchstore *ps) { return (DevState *)(ps->ws + ps->off_state); }
int32_t *derr(fc_patchstore *ps) { return (int32_t *)(ps->ws + ps->off_state + offsetof(DevState, err)); }

fc_status upload_metadata(fc_patchstore *ps, hipStream_t s) {
    const int n = (int)ps->mesh.lv.size();
    HIPCHK(hipMemcpyAsync(ps->ws + ps->off_info, ps->info.data(), sizeof(PatchInfo) * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ps->ws + ps->off_nbr, ps->nbr.data(), sizeof(NbrRec) * n * FC_NREC, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ps->ws + ps->off_sl, ps->slot_of_leaf.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ps->ws + ps->off_ls, ps->leaf_of_slot.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ps->ws + ps->off_lr, &ps->lr, sizeof(LevelRange), hipMemcpyHostToDevice, s));
    return FC_OK;
}

// launch variants (threads per patch) of the advance kernels (the mapped
// grid's capacity-form kernel shares the scalar kernel's work split and
// variants)
const int kVariantsScalar8[] = {64, 128}, kVariantsScalar16[] = {64, 128, 256}, kVariantsScalar32[] = {128, 256, 512};
const int kVariantsSwe8[] = {64, 128, 192}, kVariantsSwe16[] = {256, 384, 512, 640};

std::vector<int> variants(int mx, int eq) {
    if (eq == FC_EQ_SWE) {
        if (mx == 8) return {std::begin(kVariantsSwe8), std::end(kVariantsSwe8)};
        if (mx == 16) return {std::begin(kVariantsSwe16), std::end(kVariantsSwe16)};
        return {};
    }
    if (mx == 8) return {std::begin(kVariantsScalar8), std::end(kVariantsScalar8)};
    if (mx == 16) return {std::begin(kVariantsScalar16), std::end(kVariantsScalar16)};
    if (mx == 32) return {std::begin(kVariantsScalar32), std::end(kVariantsScalar32)};
    return {};
}
bool valid_nt(int mx, int nt, int eq = 0) {
    for (int v : variants(mx, eq))
        if (v == nt) return true;
    return false;
}
// shallow water: at mx = 8 every edge of the patch in one pass (192 = 3
// waves >= 180 edges); at mx = 16 eight waves (two workgroups per CU; the
// measured fastest on the dam break)
int default_nt(int mx, int eq) {
    if (eq == FC_EQ_SWE) return mx == 8 ? 192 : 512;
    return mx == 8 ? 64 : 256;
}
// The persistent kernel's device-wide barrier needs its whole grid resident;
// with three-wave workgroups (shallow water, 192 threads)
// the occupancy-derived grid was not (the bounded barrier timed out), so the
// persistent form runs the largest power-of-two variant not above the
// chosen one (all variants compute the same bits).
LaunchCfg persistent_cfg(const fc_patchstore *ps) {
    int nt = ps->nt;
    while (nt & (nt - 1)) nt &= nt - 1;
    return LaunchCfg{ps->mx, nt};
}

fc_status check_bound(const fc_patchstore *ps) {
    if (!ps) return fail(FC_ERR_ARG, "null store");
    if (!ps->ws || !ps->q0 || !ps->q1) return fail(FC_ERR_STATE, "store not bound to device memory");
    return FC_OK;
}

fc_status check_device_error(fc_patchstore *ps, hipStream_t s) {
    int32_t err = 0;
    HIPCHK(hipMemcpyAsync(&err, ps->ws + ps->off_state + offsetof(DevState, err), sizeof(err), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (err & 1) return fail(FC_ERR_HIP, "device-wide barrier timed out (grid not co-resident)");
    if (err & 2) return fail(FC_ERR_HIP, "interpolation stencil needed a third level (Prop. 2.1 violated)");
    if (err & 4) return fail(FC_ERR_STATE, "a captured graph did not cover a level's patches");
    if (err & 8) return fail(FC_ERR_NONFINITE, "the tagging reduction met a NaN");
    if (err & 16) return fail(FC_ERR_CFL, "a Courant number exceeded cfl_max");
    return FC_OK;
}

fc_status fill_levels(fc_patchstore *ps, int lo, int hi, double alpha, hipStream_t s) {
    Ctx c = make_ctx(ps);
    c.clevel = lo - 1;
    c.alpha = alpha;
    const int first = ps->lr.start[lo];
    int count = 0;
    for (int l = lo; l <= hi; l++) count += ps->lr.count[l];
    // levels are contiguous in the store, but an empty level has start 0
    int f0 = -1;
    for (int l = lo; l <= hi; l++)
        if (ps->lr.count[l] > 0) { f0 = ps->lr.start[l]; break; }
    (void)first;
    if (f0 < 0) return FC_OK;
    HIPCHK(launch_fill(c, ps->mx, f0, count, s));
    return FC_OK;
}

// rec: record the patches' Courant numbers in their slots
fc_status advance_one(fc_patchstore *ps, int level, double t, double dt, int fused_load, int clevel, double alpha,
                      bool rec, hipStream_t s) {
    if (ps->lr.count[level] > 0) {
        Ctx c = make_ctx(ps);
        c.clevel = clevel;
        c.alpha = alpha;
        if (!rec) c.cflp = nullptr;
        HIPCHK(launch_advance(c, LaunchCfg{ps->mx, ps->nt, ps->seg}, level, ps->lr.start[level], ps->lr.count[level], t, dt,
                              fused_load, s));
    }
    ps->curmask ^= 1u << level;
    return FC_OK;
}

void destroy_graph(fc_patchstore::Graph &g) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g.exec = nullptr;
    g.graph = nullptr;
}

void drop_graph(fc_patchstore *ps) {
    for (auto &g : ps->graphs) destroy_graph(g);
    ps->graphs.clear();
}

// end a capture on ps->cap_stream and instantiate it into `out`
fc_status finish_capture(fc_patchstore *ps, hipError_t e, fc_patchstore::Graph &out) {
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(ps->cap_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        (void)hipGetLastError();
        return fail(FC_ERR_HIP, "graph capture failed");
    }
    out.graph = g;
    hipError_t e3 = hipGraphInstantiate(&out.exec, g, nullptr, nullptr, 0);
    if (e3 != hipSuccess) {
        (void)hipGraphDestroy(g);
        out.graph = nullptr;
        out.exec = nullptr;
        (void)hipGetLastError();
        return fail(FC_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
    }
    return FC_OK;
}

// Capture one persistent launch of `ncoarse` coarse steps.  The kernel reads
// the time, step, buffer parities and level ranges from device memory, so one
// capture serves every replay.  Capture runs on a private stream (the null
// stream cannot be captured); replays go to the caller's stream.
fc_status capture(fc_patchstore *ps, fc_patchstore::Graph &out, int ncoarse, int grid) {
    if (!ps->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ps->cap_stream, hipStreamNonBlocking));
    Ctx c = make_ctx(ps);
    const SchedEntry *sched = (const SchedEntry *)(ps->ws + ps->off_sched);
    const LevelRange *lrd = (const LevelRange *)(ps->ws + ps->off_lr);
    HIPCHK(hipStreamBeginCapture(ps->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch_persistent(c, persistent_cfg(ps), sched, (int)ps->sched.size(), lrd, ncoarse,
                                     dstate(ps), grid, ps->cap_stream);
    return finish_capture(ps, e, out);
}


// Capture `ncoarse` coarse steps, starting from buffer parities `mask`, as
// one kernel per level-step (one workgroup per patch of the level, parities
// and level range baked in) plus a final node that advances the device time
// and parities.  A regrid drops the graph.
fc_status capture_levels(fc_patchstore *ps, fc_patchstore::Graph &out, int ncoarse, uint32_t mask, double dtc) {
    if (!ps->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ps->cap_stream, hipStreamNonBlocking));
    Ctx c = make_ctx(ps);
    uint32_t allmask = 0;
    int nall = 0;
    for (int l = 0; l < FC_MAXLEV; l++)
        if (ps->lr.count[l] > 0) { allmask |= 1u << l; nall += ps->lr.count[l]; }
    // A level-step of at most four patches per CU runs in one round of
    // workgroups, so its time is one workgroup's latency.  On a level that is
    // not complete (ghosts through neighbour records: two dependent loads,
    // coarse-fine averages and interpolations) scalar advection on 32x32
    // Cartesian patches takes it with 512 threads per patch (fewer ghost
    // cells per thread, twice the waves; measured 7.1-9.5 us against
    // 8.1-11.2 us for 256 threads over 1-1023 patches); a complete level
    // (one round of loads) and larger levels keep the chosen variant (a
    // complete level of 1024 patches: 9.8 us with 512 threads, 8.7 us with
    // 256).  Every variant gives the same bits.
    const LaunchCfg lc{ps->mx, ps->nt, ps->seg}, lc_small{ps->mx, 512, 0};
    int cus = 0, dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
        cus = 0;  // no small-level variant
        (void)hipGetLastError();
    }
    const bool small_ok = ps->mx == 32 && ps->cfg.equation == FC_EQ_ADVECTION && ps->cfg.map_alpha == 0.0;
    HIPCHK(hipStreamBeginCapture(ps->cap_stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    uint32_t flip = 0;
    for (int cs = 0; cs < ncoarse && e == hipSuccess; cs++)
        for (int k = 0; k < (int)ps->sched.size() && e == hipSuccess; k++) {
            const SchedEntry &en = ps->sched[k];
            const int first = en.level < 0 ? 0 : ps->lr.start[en.level];
            const int cnt = en.level < 0 ? nall : ps->lr.count[en.level];
            if (cnt > 0)
                e = launch_level_step(c,
                                      (small_ok && cnt <= 4 * cus && !(en.level >= 0 && ((c.complete >> en.level) & 1u)))
                                          ? lc_small : lc,
                                      en, first, cnt, cs, mask ^ flip, dtc, dstate(ps), ps->cap_stream);
            flip ^= en.level < 0 ? allmask : (1u << en.level);
        }
    if (e == hipSuccess) e = launch_finish_chunk(dstate(ps), ncoarse, flip, ps->cap_stream);
    return finish_capture(ps, e, out);
}
}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char *fc_last_error(void) { return g_err.c_str(); }

fc_status fc_patchstore_create(const fc_config *cfg, int64_t nleaves, const fc_leaf *leaves, fc_patchstore **out,
                               int64_t *perm_out) {
    return fc_patchstore_create_brick(cfg, 1, 1, nullptr, nleaves, leaves, out, perm_out);
}

fc_status fc_patchstore_create_brick(const fc_config *cfg, int32_t nbx, int32_t nby, const int32_t *orient,
                                     int64_t nleaves, const fc_leaf *leaves, fc_patchstore **out, int64_t *perm_out) {
    if (!cfg || !out || (nleaves > 0 && !leaves) || nleaves <= 0) return fail(FC_ERR_ARG, "bad arguments");
    *out = nullptr;
    if (nbx < 1 || nby < 1 || (int64_t)nbx * nby > (1 << 16)) return fail(FC_ERR_ARG, "brick needs 1 <= nbx, nby and nbx * nby <= 65536");
    bool multi = nbx * nby > 1;
    if (orient)
        for (int b = 0; b < nbx * nby; b++) {
            if (orient[b] < 0 || orient[b] > 7) return fail(FC_ERR_ARG, "orientation codes are 0 .. 7");
            if (orient[b] != 0) multi = true;
        }
    if (multi) {
        for (int s = 0; s < 4; s++)
            if (cfg->bc[s] != FC_BC_PERIODIC) return fail(FC_ERR_ARG, "a brick takes periodic sides");
        if (cfg->equation != FC_EQ_ADVECTION || cfg->velocity != FC_VEL_CONSTANT)
            return fail(FC_ERR_ARG, "a brick takes scalar advection at a constant velocity");
    }
    if (cfg->mx != 8 && cfg->mx != 16 && cfg->mx != 32) return fail(FC_ERR_ARG, "mx must be 8, 16 or 32");
    if (4 * cfg->mbc > cfg->mx || cfg->mbc < 2) return fail(FC_ERR_GHOST_WIDTH, "need 2 <= mbc <= mx/4 (Prop. 2.1)");
    if (cfg->mbc != 2) return fail(FC_ERR_ARG, "the kernels use exactly 2 ghost layers");
    if (cfg->equation != FC_EQ_ADVECTION && cfg->equation != FC_EQ_SWE) return fail(FC_ERR_ARG, "unknown equation");
    if (cfg->equation == FC_EQ_SWE && cfg->mx > 16) return fail(FC_ERR_ARG, "shallow water supports mx = 8 or 16");
    if (cfg->limiter < 0 || cfg->limiter > 3) return fail(FC_ERR_ARG, "unknown limiter");
    for (int s = 0; s < 4; s++)
        if (cfg->bc[s] != FC_BC_PERIODIC && cfg->bc[s] != FC_BC_REFLECT) return fail(FC_ERR_ARG, "unknown boundary condition");
    if ((cfg->bc[0] == FC_BC_PERIODIC) != (cfg->bc[1] == FC_BC_PERIODIC) ||
        (cfg->bc[2] == FC_BC_PERIODIC) != (cfg->bc[3] == FC_BC_PERIODIC))
        return fail(FC_ERR_ARG, "periodicity must match on opposite sides");
    if (cfg->min_level < 0 || cfg->max_level < cfg->min_level || cfg->max_level >= FC_MAXLEV - 1)
        return fail(FC_ERR_ARG, "bad level range");
    if (cfg->capacity < nleaves) return fail(FC_ERR_CAPACITY, "capacity below the number of leaves");
    {
        const int64_t n = cfg->mx + 2 * MBK, nf = cfg->equation == FC_EQ_SWE ? 3 : 1;
        if (nf * (int64_t)cfg->capacity * n * n > (int64_t)UINT32_MAX)
            return fail(FC_ERR_CAPACITY, "a patch buffer must stay below 2^32 doubles (32-bit cell indices)");
    }
    if (cfg->equation == FC_EQ_ADVECTION && cfg->velocity == FC_VEL_NONE) return fail(FC_ERR_ARG, "advection needs a velocity");
    if (cfg->velocity == FC_VEL_SWIRL && !(cfg->vel_params[0] > 0)) return fail(FC_ERR_ARG, "swirl period must be > 0");
    if (!(cfg->cfl_max >= 0.0)) return fail(FC_ERR_ARG, "cfl_max must be >= 0 (0: not checked)");
    if (!(fabs(cfg->map_alpha) < 0.5 / M_PI)) return fail(FC_ERR_ARG, "map_alpha must satisfy |alpha| < 1/(2 pi)");
    if (cfg->map_alpha != 0.0) {
        if (multi || nbx * nby > 1) return fail(FC_ERR_ARG, "a mapped grid takes one block");
        if (cfg->equation != FC_EQ_ADVECTION) return fail(FC_ERR_ARG, "a mapped grid takes scalar advection");
        for (int s = 0; s < 4; s++)
            if (cfg->bc[s] != FC_BC_PERIODIC) return fail(FC_ERR_ARG, "a mapped grid takes periodic sides");
    }
    std::vector<fc_leaf> L(leaves, leaves + nleaves);
    for (const auto &q : L) {
        if (q.level < cfg->min_level || q.level > cfg->max_level) return fail(FC_ERR_ARG, "leaf level outside [min_level, max_level]");
        if (q.ix < 0 || q.iy < 0 || q.ix >= (nbx << q.level) || q.iy >= (nby << q.level))
            return fail(FC_ERR_ARG, "leaf coordinates out of range");
    }
    fc_patchstore *ps = new fc_patchstore();
    ps->cfg = *cfg;
    ps->mx = cfg->mx;
    ps->N = cfg->mx + 2 * MBK;
    ps->F = nfields(*cfg);
    ps->mesh.mx = cfg->mx;
    ps->mesh.nbx = nbx;
    ps->mesh.nby = nby;
    std::copy(cfg->bc, cfg->bc + 4, ps->mesh.bc);
    if (orient) ps->ori.assign(orient, orient + nbx * nby);
    ps->multiblock = multi;
    for (auto &q : L) q = to_brick(ps, q);  // leaves arrive in the blocks' own coordinates
    fc_status st = validate(ps->mesh, L);
    if (st != FC_OK) {
        delete ps;
        return st;
    }
    build_metadata(ps, L);
    if (cfg->time_stepping == FC_STEP_GLOBAL) ps->sched.push_back(SchedEntry{-1, 0, 0.0, 1.0, 1.0});
    else gen_sched(ps->sched, cfg->min_level, cfg->max_level, 0.0, 1.0, 1.0);
    ps->nt = default_nt(ps->mx, cfg->equation);
    layout_workspace(ps);
    if (perm_out)
        for (int64_t k = 0; k < nleaves; k++) perm_out[k] = ps->slot_of_leaf[k];
    *out = ps;
    return FC_OK;
}

fc_status fc_patchstore_destroy(fc_patchstore *ps) {
    if (!ps) return FC_OK;
    drop_graph(ps);
    if (ps->cap_stream) (void)hipStreamDestroy(ps->cap_stream);
    delete ps;
    return FC_OK;
}

fc_status fc_patchstore_sizes(const fc_patchstore *ps, int64_t *q_doubles, int64_t *ws_bytes) {
    if (!ps) return fail(FC_ERR_ARG, "null store");
    if (q_doubles) *q_doubles = (int64_t)ps->F * ps->cfg.capacity * ps->N * ps->N;
    if (ws_bytes) *ws_bytes = (int64_t)ps->ws_bytes;
    return FC_OK;
}

fc_status fc_patchstore_bind(fc_patchstore *ps, double *q0, double *q1, void *workspace, void *stream) {
    if (!ps || !q0 || !q1 || !workspace) return fail(FC_ERR_ARG, "bad arguments");
    if (((uintptr_t)workspace & 255) != 0) return fail(FC_ERR_ARG, "workspace must be 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    drop_graph(ps);
    ps->q0 = q0;
    ps->q1 = q1;
    ps->ws = (char *)workspace;
    ps->curmask = 0;
    DevState st;
    memset(&st, 0, sizeof(st));
    st.t = ps->t;
    HIPCHK(hipMemcpyAsync(ps->ws + ps->off_state, &st, sizeof(st), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ps->ws + ps->off_sched, ps->sched.data(), sizeof(SchedEntry) * ps->sched.size(),
                          hipMemcpyHostToDevice, s));
    fc_status r = upload_metadata(ps, s);
    if (r != FC_OK) return r;
    if (ps->cfg.velocity == FC_VEL_SWIRL)
        for (int l = ps->cfg.min_level; l <= ps->cfg.max_level; l++)
            HIPCHK(launch_init_tables(l, ps->mx, ps->cfg.bc[0] == FC_BC_PERIODIC, ps->cfg.bc[2] == FC_BC_PERIODIC,
                                      (double *)(ps->ws + ps->off_vt[l]), s));
    if (ps->cfg.map_alpha != 0.0)
        for (int l = ps->cfg.min_level; l <= ps->cfg.max_level; l++)
            HIPCHK(launch_init_capacity(ps->mx << l, ps->cfg.map_alpha, (double *)(ps->ws + ps->off_mk[l]), s));
    ps->pgrid = persistent_max_grid(persistent_cfg(ps), ps->cfg.map_alpha != 0.0 ? 2 : ps->cfg.equation);
    HIPCHK(hipStreamSynchronize(s));
    return FC_OK;
}

fc_status fc_patchstore_info(const fc_patchstore *ps, int64_t *nleaves, int32_t *min_level, int32_t *max_level) {
    if (!ps) return fail(FC_ERR_ARG, "null store");
    if (nleaves) *nleaves = (int64_t)ps->mesh.lv.size();
    if (min_level) *min_level = ps->cfg.min_level;
    if (max_level) *max_level = ps->cfg.max_level;
    return FC_OK;
}

fc_status fc_patchstore_leaves(const fc_patchstore *ps, fc_leaf *out) {
    if (!ps || !out) return fail(FC_ERR_ARG, "bad arguments");
    for (size_t k = 0; k < ps->mesh.lv.size(); k++) out[k] = to_own(ps, ps->mesh.lv[k]);
    return FC_OK;
}

fc_status fc_patchstore_records(const fc_patchstore *ps, int32_t *out) {
    if (!ps || !out) return fail(FC_ERR_ARG, "bad arguments");
    for (size_t k = 0; k < ps->nbr.size(); k++) {
        const NbrRec &r = ps->nbr[k];
        out[4 * k] = r.type; out[4 * k + 1] = r.id; out[4 * k + 2] = r.fx; out[4 * k + 3] = r.fy;
    }
    return FC_OK;
}

fc_status fc_set_interior(fc_patchstore *ps, const double *src, void *stream) {
    fc_status r = check_bound(ps);
    if (r != FC_OK) return r;
    if (!src) return fail(FC_ERR_ARG, "null source");
    HIPCHK(launch_set_interior(make_ctx(ps), ps->mx, (const int32_t *)(ps->ws + ps->off_sl), (int)ps->mesh.lv.size(),
                               src, (hipStream_t)stream));
    return FC_OK;
}

fc_status fc_get_interior(fc_patchstore *ps, double *dst, void *stream) {
    fc_status r = check_bound(ps);
    if (r != FC_OK) return r;
    if (!dst) return fail(FC_ERR_ARG, "null destination");
    HIPCHK(launch_get_interior(make_ctx(ps), ps->mx, (const int32_t *)(ps->ws + ps->off_sl), (int)ps->mesh.lv.size(),
                               dst, 0, (hipStream_t)stream));
    return FC_OK;
}

fc_status fc_get_patches(fc_patchstore *ps, double *dst, void *stream) {
    fc_status r = check_bound(ps);
    if (r != FC_OK) return r;
    if (!dst) return fail(FC_ERR_ARG, "null destination");
    HIPCHK(launch_get_interior(make_ctx(ps), ps->mx, (const int32_t *)(ps->ws + ps->off_sl), (int)ps->mesh.lv.size(),
                               dst, 1, (hipStream_t)stream));
    return FC_OK;
}

fc_status fc_ghost_fill(fc_patchstore *ps, int32_t level_lo, int32_t level_hi, double alpha, void *stream) {
    fc_status r = check_bound(ps);
    if (r != FC_OK) return r;
    if (level_lo < ps->cfg.min_level || level_hi > ps->cfg.max_level || level_lo > level_hi)
        return fail(FC_ERR_ARG, "bad level range");
    if (!(alpha >= 0.0 && alpha <= 1.0)) return fail(FC_ERR_ARG, "alpha must lie in [0, 1]");
    return fill_levels(ps, level_lo, level_hi, alpha, (hipStream_t)stream);
}

fc_status fc_advance_level(fc_patchstore *ps, int32_t level, double t, double dt, double *cfl_dev, void *stream) {
    fc_status r = check_bound(ps);
    if (r != FC_OK) return r;
    if (level < ps->cfg.min_level || level > ps->cfg.max_level) return fail(FC_ERR_ARG, "bad level");
    if (!(dt > 0)) return fail(FC_ERR_ARG, "dt must be positive");
    hipStream_t s = (hipStream_t)stream;
    const int n = (int)ps->mesh.lv.size();
    if (cfl_dev) HIPCHK(launch_zero_cfl(cflp(ps), n, s));
    r = advance_one(ps, level, t, dt, 0, -1, 1.0, cfl_dev != nullptr, s);
    if (r == FC_OK && cfl_dev) HIPCHK(launch_export_cfl(nullptr, cflp(ps), n, cfl_dev, ps->cfg.cfl_max, derr(ps), s));
    return r;
}

fc_status fc_advance_level_noalloc(fc_patchstore *ps, int32_t level, double t, double dt, double *cfl_dev,
                                   void *stream) {
    if (!ps) return fail(FC_ERR_ARG, "null store");
    if (ps->cfg.capacity > kNoallocSlots)
        return fail(FC_ERR_CAPACITY, "store capacity above the 65536 slots of the fixed scratch array");
    fc_status r = check_bound(ps);
    if (r != FC_OK) return r;
    if (level < ps->cfg.min_level || level > ps->cfg.max_level) return fail(FC_ERR_ARG, "bad level");
    if (!(dt > 0)) return fail(FC_ERR_ARG, "dt must be positive");
    hipStream_t s = (hipStream_t)stream;
    const int n = (int)ps->mesh.lv.size();
    unsigned long long *slots = nullptr;
    if (cfl_dev) {
        r = scratch_ptr(&slots);
        if (r != FC_OK) return r;
        // the array keeps the previous call's maxima: clear the slots this
        // call reduces over (a kernel, so the call can be graph-captured)
        HIPCHK(launch_zero_cfl(slots, n, s));
    }
    if (ps->lr.count[level] > 0) {
        Ctx c = make_ctx(ps);
        c.cflp = slots;
        HIPCHK(launch_advance(c, LaunchCfg{ps->mx, ps->nt, ps->seg}, level, ps->lr.start[level], ps->lr.count[level], t, dt,
                              0, s));
    }
    ps->curmask ^= 1u << level;
    if (cfl_dev) HIPCHK(launch_export_cfl(nullptr, slots, n, cfl_dev, ps->cfg.cfl_max, derr(ps), s));
    return FC_OK;
}

fc_status fc_get_time(const fc_patchstore *ps, double *t) {
    if (!ps || !t) return fail(FC_ERR_ARG, "bad arguments");
    *t = ps->t;
    return FC_OK;
}

fc_status fc_set_time(fc_patchstore *ps, double t) {
    if (!ps) return fail(FC_ERR_ARG, "null store");
    ps->t = t;
    return FC_OK;
}

// Graph forms: replay (launch) or only capture (!launch) the graphs that
// `nsteps` coarse steps from the current parities need: as many chunks of
// FC_TCHUNK coarse steps as fit, then ONE graph for the remaining steps, so
// that any step count is a few replays.  Graphs are captured on demand and
// cached (see fc_patchstore::Graph).
static fc_status graph_steps(fc_patchstore *ps, double dt_coarse, int nsteps, int mode, int grid, bool launch,
                             hipStream_t s) {
    fc_status r = FC_OK;
    const int kChunk = FC_TCHUNK;
    uint32_t allm = 0, step_flip = 0;
    for (int l = 0; l < FC_MAXLEV; l++)
        if (ps->lr.count[l] > 0) allm |= 1u << l;
    for (const SchedEntry &e : ps->sched) step_flip ^= e.level < 0 ? allm : (1u << e.level);
    uint32_t mask = ps->curmask;  // parities at the start of the next replay
    const bool persistent = mode == FC_MODE_PERSISTENT_GRAPH;
    // the cached graph for n coarse steps from the current parities
    auto get = [&](int n, hipGraphExec_t &exec) -> fc_status {
        fc_patchstore::Graph *hit = nullptr;
        for (auto &g : ps->graphs) {
            if (g.mode != mode || g.n != n) continue;
            if (persistent ? g.grid == grid : (g.mask == mask && g.dt == dt_coarse)) { hit = &g; break; }
        }
        if (!hit) {
            if ((int)ps->graphs.size() >= fc_patchstore::kMaxGraphs) {
                size_t lru = 0;
                for (size_t k = 1; k < ps->graphs.size(); k++)
                    if (ps->graphs[k].used < ps->graphs[lru].used) lru = k;
                destroy_graph(ps->graphs[lru]);
                ps->graphs.erase(ps->graphs.begin() + lru);
            }
            fc_patchstore::Graph g;
            g.mode = mode; g.n = n; g.grid = grid; g.mask = mask; g.dt = dt_coarse;
            fc_status st = persistent ? capture(ps, g, n, grid) : capture_levels(ps, g, n, mask, dt_coarse);
            if (st != FC_OK) return st;
            ps->graphs.push_back(g);
            hit = &ps->graphs.back();
        }
        hit->used = ++ps->graph_clock;
        exec = hit->exec;
        return FC_OK;
    };
    for (int k = 0; k < nsteps;) {
        const int n = std::min(kChunk, nsteps - k);
        hipGraphExec_t exec = nullptr;
        if ((r = get(n, exec)) != FC_OK) return r;
        if (launch) HIPCHK(hipGraphLaunch(exec, s));
        if (n & 1) mask ^= step_flip;
        k += n;
    }
    return FC_OK;
}

fc_status fc_prepare_steps(fc_patchstore *ps, double dt_coarse, int32_t nsteps, int32_t mode, void *stream) {
    fc_status r = check_bound(ps);
    if (r != FC_OK) return r;
    if (!(dt_coarse > 0) || nsteps < 0) return fail(FC_ERR_ARG, "bad step arguments");
    if (mode == FC_MODE_PER_LEVEL || mode == FC_MODE_FUSED_LEVELS || mode == FC_MODE_FUSED) return FC_OK;
    if (mode != FC_MODE_FUSED_GRAPH && mode != FC_MODE_PERSISTENT_GRAPH) return fail(FC_ERR_ARG, "unknown mode");
    if (ps->pgrid <= 0) return fail(FC_ERR_HIP, "persistent kernel has no resident blocks");
    const int grid = ps->pgrid_user > 0 ? std::min(ps->pgrid_user, ps->pgrid) : ps->pgrid;
    return graph_steps(ps, dt_coarse, nsteps, mode, grid, false, (hipStream_t)stream);
}

// flag_cfl: a Courant number above cfl_max raises the device flag that
// fc_check_device reports (the adaptive driver decides on the host instead)
static fc_status advance_steps(fc_patchstore *ps, double dt_coarse, int32_t nsteps, int32_t mode, double *cfl_dev,
                               bool flag_cfl, hipStream_t s);

fc_status fc_advance_coarse_steps(fc_patchstore *ps, double dt_coarse, int32_t nsteps, int32_t mode, double *cfl_dev,
                                  void *stream) {
    return advance_steps(ps, dt_coarse, nsteps, mode, cfl_dev, true, (hipStream_t)stream);
}

static fc_status advance_steps(fc_patchstore *ps, double dt_coarse, int32_t nsteps, int32_t mode, double *cfl_dev,
                               bool flag_cfl, hipStream_t s) {
    fc_status r = check_bound(ps);
    if (r != FC_OK) return r;
    if (!(dt_coarse > 0) || nsteps < 0) return fail(FC_ERR_ARG, "bad step arguments");
    const bool cfl = cfl_dev != nullptr;
    const double cmax = flag_cfl ? ps->cfg.cfl_max : 0.0;
    const int nleaf = (int)ps->mesh.lv.size();
    if (cfl && (mode == FC_MODE_PER_LEVEL || mode == FC_MODE_FUSED_LEVELS))
        HIPCHK(launch_zero_cfl(cflp(ps), nleaf, s));
    if (mode == FC_MODE_PER_LEVEL) {
        for (int n = 0; n < nsteps; n++) {
            for (const SchedEntry &e : ps->sched) {
                const double t = ps->t + e.off * dt_coarse, dt = e.scale * dt_coarse;
                if (e.level < 0) {
                    r = fill_levels(ps, ps->cfg.min_level, ps->cfg.max_level, 1.0, s);
                    if (r != FC_OK) return r;
                    for (int l = ps->cfg.min_level; l <= ps->cfg.max_level; l++) {
                        r = advance_one(ps, l, t, dt, 0, -1, 1.0, cfl, s);
                        if (r != FC_OK) return r;
                    }
                } else {
                    if (ps->lr.count[e.level] > 0) {
                        r = fill_levels(ps, e.level, e.level, e.alpha, s);
                        if (r != FC_OK) return r;
                    }
                    r = advance_one(ps, e.level, t, dt, 0, e.level - 1, e.alpha, cfl, s);
                    if (r != FC_OK) return r;
                }
            }
            ps->t += dt_coarse;
        }
        if (cfl) HIPCHK(launch_export_cfl(nullptr, cflp(ps), nleaf, cfl_dev, cmax, derr(ps), s));
        return FC_OK;
    }
    if (mode == FC_MODE_FUSED_LEVELS) {
        // one launch per level-step of the kernel that gathers its ghosts
        for (int n = 0; n < nsteps; n++) {
            for (const SchedEntry &e : ps->sched) {
                const double t = ps->t + e.off * dt_coarse, dt = e.scale * dt_coarse;
                if (e.level < 0) {
                    Ctx c = make_ctx(ps);
                    if (!cfl) c.cflp = nullptr;
                    HIPCHK(launch_advance(c, LaunchCfg{ps->mx, ps->nt, ps->seg}, -1, 0, nleaf, t, dt, 1, s));
                    for (int l = 0; l < FC_MAXLEV; l++)
                        if (ps->lr.count[l] > 0) ps->curmask ^= 1u << l;
                } else {
                    r = advance_one(ps, e.level, t, dt, 1, e.level - 1, e.alpha, cfl, s);
                    if (r != FC_OK) return r;
                }
            }
            ps->t += dt_coarse;
        }
        if (cfl) HIPCHK(launch_export_cfl(nullptr, cflp(ps), nleaf, cfl_dev, cmax, derr(ps), s));
        return FC_OK;
    }
    if (mode != FC_MODE_FUSED && mode != FC_MODE_FUSED_GRAPH && mode != FC_MODE_PERSISTENT_GRAPH)
        return fail(FC_ERR_ARG, "unknown mode");
    if (ps->pgrid <= 0) return fail(FC_ERR_HIP, "persistent kernel has no resident blocks");
    const int grid = ps->pgrid_user > 0 ? std::min(ps->pgrid_user, ps->pgrid) : ps->pgrid;
    DevState *st = dstate(ps);
    HIPCHK(launch_set_state(st, ps->t, dt_coarse, ps->curmask, 1, cflp(ps), nleaf, s));
    Ctx c = make_ctx(ps);
    const SchedEntry *sched = (const SchedEntry *)(ps->ws + ps->off_sched);
    const LevelRange *lrd = (const LevelRange *)(ps->ws + ps->off_lr);
    // up to `kChunk` coarse steps per launch (persistent) or per graph replay
    const int kChunk = FC_TCHUNK;
    if (mode == FC_MODE_FUSED) {
        for (int k = 0; k < nsteps; k += kChunk) {
            const int m = std::min(kChunk, nsteps - k);
            HIPCHK(launch_persistent(c, persistent_cfg(ps), sched, (int)ps->sched.size(), lrd, m, st, grid, s));
        }
    } else {
        if ((r = graph_steps(ps, dt_coarse, nsteps, mode, grid, true, s)) != FC_OK) return r;
    }
    // host mirror of the device bookkeeping
    uint32_t allmask = 0;
    for (int l = 0; l < FC_MAXLEV; l++)
        if (ps->lr.count[l] > 0) allmask |= 1u << l;
    for (int k = 0; k < nsteps; k++) {
        for (const SchedEntry &e : ps->sched) ps->curmask ^= e.level < 0 ? allmask : (1u << e.level);
        ps->t += dt_coarse;
    }
    if (cfl_dev) HIPCHK(launch_export_cfl(st, cflp(ps), nleaf, cfl_dev, cmax, derr(ps), s));
    return FC_OK;
}

fc_status fc_advance_adaptive(fc_patchstore *ps, double t_end, double cfl_target, int32_t mode, double *dt_inout,
                              int32_t max_steps, int32_t *steps_out, int32_t *rejected_out, void *stream) {
    fc_status r = check_bound(ps);
    if (r != FC_OK) return r;
    if (!(ps->cfg.cfl_max > 0)) return fail(FC_ERR_STATE, "the store was created without cfl_max");
    if (!dt_inout || !(*dt_inout > 0) || !(cfl_target > 0) || cfl_target > ps->cfg.cfl_max || max_steps < 1)
        return fail(FC_ERR_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const int n = (int)ps->mesh.lv.size();
    double *save = (double *)(ps->ws + ps->off_save);
    double *cflv = (double *)(ps->ws + ps->off_cflv);
    double dt = *dt_inout;
    int steps = 0, rejected = 0, in_row = 0;
    if (steps_out) *steps_out = 0;
    if (rejected_out) *rejected_out = 0;
    while (steps < max_steps) {
        const double rem = t_end - ps->t;
        if (!(rem > 1e-14 * std::fabs(t_end))) break;
        const bool last = dt >= rem;
        const double dtu = last ? rem : dt;
        const uint32_t mask0 = ps->curmask;
        const double t0 = ps->t;
        HIPCHK(launch_copy_interiors(make_ctx(ps), ps->mx, n, save, 0, s));
        HIPCHK(launch_zero_cfl((unsigned long long *)cflv, 1, s));
        r = advance_steps(ps, dtu, 1, mode, cflv, false, s);
        if (r != FC_OK) return r;
        double c = 0.0;
        HIPCHK(hipMemcpyAsync(&c, cflv, sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (!(c <= ps->cfg.cfl_max)) {  // also NaN
            ps->curmask = mask0;
            ps->t = t0;
            HIPCHK(launch_copy_interiors(make_ctx(ps), ps->mx, n, save, 1, s));
            rejected++;
            if (rejected_out) *rejected_out = rejected;
            if (++in_row >= 8) {
                HIPCHK(hipStreamSynchronize(s));
                return fail(FC_ERR_CFL, "coarse step rejected eight times in a row (last Courant number " +
                                            std::to_string(c) + ")");
            }
            // a step that blew up (the later substeps of a long multirate
            // coarse step can) has no usable Courant number: halve it
            dt = std::isfinite(c) ? dtu * cfl_target / c : 0.5 * dtu;
            continue;
        }
        in_row = 0;
        steps++;
        if (steps_out) *steps_out = steps;
        if (last) ps->t = t_end;
        if (c > 0) dt = dtu * cfl_target / c;
    }
    *dt_inout = dt;
    return FC_OK;
}

fc_status fc_tag_refine(fc_patchstore *ps, double tau_refine, double tau_coarsen, int8_t *tags_dev, double *gmax2_dev,
                        void *stream) {
    fc_status r = check_bound(ps);
    if (r != FC_OK) return r;
    if (!tags_dev) return fail(FC_ERR_ARG, "null tags");
    HIPCHK(launch_tag(make_ctx(ps), ps->mx, (const int32_t *)(ps->ws + ps->off_sl), (int)ps->mesh.lv.size(),
                      ps->cfg.min_level, ps->cfg.max_level, tau_refine, tau_coarsen, tags_dev, gmax2_dev,
                      (hipStream_t)stream));
    return FC_OK;
}

fc_status fc_adapt(const fc_patchstore *ps, const int8_t *tags, int32_t smooth, fc_leaf *out, int64_t cap,
                   int64_t *n_out) {
    if (!ps || !tags || !out || !n_out) return fail(FC_ERR_ARG, "bad arguments");
    const int n = (int)ps->mesh.lv.size();
    const int lmin = ps->cfg.min_level, lmax = ps->cfg.max_level;
    // target level per slot (tags arrive in input-leaf order), and the
    // largest target over the leaf and every leaf touching it (Sec. 4.2)
    std::vector<int> target(n), T(n);
    for (int k = 0; k < n; k++) {
        const int s = ps->slot_of_leaf[k];
        target[s] = std::min(lmax, std::max(lmin, ps->mesh.lv[s].level + (int)tags[k]));
    }
    for (int s = 0; s < n; s++) {
        int m = target[s];
        if (smooth) {
            const fc_leaf L = ps->mesh.lv[s];
            const int lq = L.level + 1, nqx = ps->mesh.nbx << lq, nqy = ps->mesh.nby << lq;
            for (int dy = -1; dy <= 2; dy++)
                for (int dx = -1; dx <= 2; dx++) {
                    if (dx >= 0 && dx <= 1 && dy >= 0 && dy <= 1) continue;
                    int X = 2 * L.ix + dx, Y = 2 * L.iy + dy;
                    if (X < 0 || X >= nqx) { if (ps->cfg.bc[X < 0 ? 0 : 1] != FC_BC_PERIODIC) continue; X = (X + nqx) % nqx; }
                    if (Y < 0 || Y >= nqy) { if (ps->cfg.bc[Y < 0 ? 2 : 3] != FC_BC_PERIODIC) continue; Y = (Y + nqy) % nqy; }
                    for (int l2 = lq; l2 >= 0; l2--) {
                        const int o = ps->mesh.find(l2, X >> (lq - l2), Y >> (lq - l2));
                        if (o >= 0) { m = std::max(m, target[o]); break; }
                    }
                }
        }
        T[s] = m;
    }
    std::vector<fc_leaf> res;
    std::vector<char> done(n, 0);
    for (int s = 0; s < n; s++) {
        if (done[s]) continue;
        const fc_leaf L = ps->mesh.lv[s];
        if (T[s] < L.level && L.level > lmin) {
            const int px = L.ix >> 1, py = L.iy >> 1;
            int sib[4];
            bool ok = true;
            for (int c = 0; c < 4; c++) {
                sib[c] = ps->mesh.find(L.level, 2 * px + (c & 1), 2 * py + (c >> 1));
                if (sib[c] < 0 || !(T[sib[c]] < L.level)) ok = false;
            }
            if (ok) {
                for (int c = 0; c < 4; c++) done[sib[c]] = 1;
                res.push_back(fc_leaf{L.level - 1, px, py});
                continue;
            }
        }
        done[s] = 1;
        if (T[s] > L.level && L.level < lmax) {
            for (int c = 0; c < 4; c++) res.push_back(fc_leaf{L.level + 1, 2 * L.ix + (c & 1), 2 * L.iy + (c >> 1)});
        } else {
            res.push_back(L);
        }
    }
    // 2:1 balance by refinement (brick coordinates; quadtree families are
    // the same sets in a block's own coordinates)
    for (;;) {
        Mesh m;
        m.mx = ps->mx;
        m.nbx = ps->mesh.nbx;
        m.nby = ps->mesh.nby;
        std::copy(ps->cfg.bc, ps->cfg.bc + 4, m.bc);
        m.lv = res;
        m.index();
        std::vector<fc_leaf> nx;
        bool changed = false;
        for (const auto &L : res) {
            if (!m.balanced_at(L)) {
                changed = true;
                for (int c = 0; c < 4; c++) nx.push_back(fc_leaf{L.level + 1, 2 * L.ix + (c & 1), 2 * L.iy + (c >> 1)});
            } else {
                nx.push_back(L);
            }
        }
        res.swap(nx);
        if (!changed) break;
    }
    for (auto &q : res) q = to_own(ps, q);
    std::sort(res.begin(), res.end(), [](const fc_leaf &a, const fc_leaf &b) {
        if (a.level != b.level) return a.level < b.level;
        if (a.iy != b.iy) return a.iy < b.iy;
        return a.ix < b.ix;
    });
    if ((int64_t)res.size() > cap) return fail(FC_ERR_CAPACITY, "adapted leaf set exceeds the output capacity");
    std::copy(res.begin(), res.end(), out);
    *n_out = (int64_t)res.size();
    return FC_OK;
}

fc_status fc_adapt_device(fc_patchstore *ps, const int8_t *tags_dev, int32_t smooth, fc_leaf *out, int64_t cap,
                          int64_t *n_out, void *stream) {
    fc_status r = check_bound(ps);
    if (r != FC_OK) return r;
    if (!tags_dev || !out || !n_out) return fail(FC_ERR_ARG, "bad arguments");
    if (!ps->dev_adapt) return fail(FC_ERR_ARG, "adaptation on the device needs one block and max_level <= 10");
    hipStream_t s = (hipStream_t)stream;
    const int n = (int)ps->mesh.lv.size(), L = ps->cfg.max_level;
    const int perx = ps->cfg.bc[0] == FC_BC_PERIODIC, pery = ps->cfg.bc[2] == FC_BC_PERIODIC;
    int8_t *la = (int8_t *)(ps->ws + ps->off_lma), *lb = (int8_t *)(ps->ws + ps->off_lmb);
    int32_t *flags = (int32_t *)(ps->ws + ps->off_aflags);
    HIPCHK(launch_adapt_device(make_ctx(ps), (const int32_t *)(ps->ws + ps->off_sl), tags_dev, n, L, perx, pery,
                               ps->cfg.min_level, L, smooth, (int32_t *)(ps->ws + ps->off_own),
                               (int32_t *)(ps->ws + ps->off_tgt), (int32_t *)(ps->ws + ps->off_tmax), la, lb, flags, s));
    // 2:1 balance passes until no leaf is refined (each refinement is
    // forced by a leaf two levels finer, so the passes end within the level
    // span)
    bool settled = false;
    for (int it = 0; it <= L - ps->cfg.min_level + 2; it++) {
        HIPCHK(hipMemsetAsync(flags, 0, sizeof(int32_t), s));
        HIPCHK(launch_balance_pass(la, lb, L, perx, pery, ps->cfg.min_level, L, flags, s));
        int32_t changed = 0;
        HIPCHK(hipMemcpyAsync(&changed, flags, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        std::swap(la, lb);
        if (!changed) { settled = true; break; }
    }
    if (!settled) return fail(FC_ERR_STATE, "2:1 balance did not settle");
    const int capd = (int)ps->cfg.capacity;
    HIPCHK(hipMemsetAsync(flags + 1, 0, sizeof(int32_t), s));
    HIPCHK(launch_extract_leaves(la, L, capd, flags + 1, (int32_t *)(ps->ws + ps->off_lout), s));
    int32_t cnt = 0;
    HIPCHK(hipMemcpyAsync(&cnt, flags + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (cnt > capd || cnt > cap) return fail(FC_ERR_CAPACITY, "adapted leaf set exceeds the capacity");
    std::vector<fc_leaf> res((size_t)cnt);
    HIPCHK(hipMemcpyAsync(res.data(), ps->ws + ps->off_lout, sizeof(fc_leaf) * (size_t)cnt, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    std::sort(res.begin(), res.end(), [](const fc_leaf &a, const fc_leaf &b) {
        if (a.level != b.level) return a.level < b.level;
        if (a.iy != b.iy) return a.iy < b.iy;
        return a.ix < b.ix;
    });
    std::copy(res.begin(), res.end(), out);
    *n_out = (int64_t)cnt;
    return FC_OK;
}

fc_status fc_regrid(fc_patchstore *ps, int64_t nleaves, const fc_leaf *new_leaves, void *stream) {
    if (!ps) return fail(FC_ERR_ARG, "null store");
    if (!new_leaves || nleaves <= 0) return fail(FC_ERR_ARG, "bad arguments");
    if (nleaves > ps->cfg.capacity) return fail(FC_ERR_CAPACITY, "new leaf set exceeds capacity");
    std::vector<fc_leaf> L(new_leaves, new_leaves + nleaves);
    for (auto &q : L) {
        if (q.level < ps->cfg.min_level || q.level > ps->cfg.max_level) return fail(FC_ERR_ARG, "leaf level outside range");
        if (q.ix < 0 || q.iy < 0 || q.ix >= (ps->mesh.nbx << q.level) || q.iy >= (ps->mesh.nby << q.level))
            return fail(FC_ERR_ARG, "leaf coordinates out of range");
        q = to_brick(ps, q);  // own -> brick coordinates
    }
    fc_status r = validate(ps->mesh, L);
    if (r != FC_OK) return r;
    // The transfer plan, built against the new leaves in store order before
    // anything in the store changes: every new leaf must be an old leaf, a
    // child of one or the parent of four.  A leaf set that fails this leaves
    // the store as it was.
    const std::vector<int> order = store_order(L);
    const int n = (int)L.size();
    std::vector<TransferRec> plan(n);
    for (int p = 0; p < n; p++) {
        const fc_leaf q = L[order[p]];
        TransferRec tr{};
        int o;
        if ((o = ps->mesh.find(q.level, q.ix, q.iy)) >= 0) {
            tr.kind = TR_COPY; tr.src[0] = o;
        } else if ((o = ps->mesh.find(q.level - 1, q.ix >> 1, q.iy >> 1)) >= 0) {
            // the child's position in its parent's own indices
            const fc_leaf w = to_own(ps, q);
            tr.kind = TR_REFINE; tr.src[0] = o; tr.cx = w.ix & 1; tr.cy = w.iy & 1;
        } else {
            tr.kind = TR_COARSEN;
            const fc_leaf w = to_own(ps, q);
            for (int c = 0; c < 4; c++) {
                // child c at own position (c & 1, c >> 1) of the new parent
                const fc_leaf ch = to_brick(ps, fc_leaf{w.level + 1, 2 * w.ix + (c & 1), 2 * w.iy + (c >> 1)});
                tr.src[c] = ps->mesh.find(ch.level, ch.ix, ch.iy);
                if (tr.src[c] < 0) return fail(FC_ERR_ARG, "new leaf is neither old, child nor parent of old leaves");
            }
        }
        plan[p] = tr;
    }
    r = check_bound(ps);
    if (r != FC_OK) return r;
    hipStream_t s = (hipStream_t)stream;
    // every old patch (with the ghosts filled by the caller) into buffer 0
    Ctx old = make_ctx(ps);
    HIPCHK(launch_consolidate(old, ps->mx, (int)ps->mesh.lv.size(), s));
    build_metadata(ps, L);
    HIPCHK(hipMemcpyAsync(ps->ws + ps->off_plan, plan.data(), sizeof(TransferRec) * n, hipMemcpyHostToDevice, s));
    ps->curmask = ~0u;  // new data lives in buffer 1 for every level
    // the new slots' geometry first: the transfer reads it (area weights
    // of a mapped grid); consolidation, which read the old, is ahead in
    // the stream
    r = upload_metadata(ps, s);
    if (r != FC_OK) return r;
    Ctx nc = make_ctx(ps);
    HIPCHK(launch_transfer(nc, ps->mx, (const TransferRec *)(ps->ws + ps->off_plan), n, s));
    drop_graph(ps);     // level populations changed: recapture on next use
    HIPCHK(hipStreamSynchronize(s));
    return FC_OK;
}

// a uniform periodic level of scalar advection (the leaf-order step and its
// adjoint need every neighbour record to be a same-size one)
static fc_status check_uniform_periodic(fc_patchstore *ps, int32_t level, double dt) {
    fc_status r = check_bound(ps);
    if (r != FC_OK) return r;
    if (ps->cfg.equation != FC_EQ_ADVECTION) return fail(FC_ERR_ARG, "scalar advection only");
    if (ps->multiblock) return fail(FC_ERR_ARG, "one block of orientation code 0 only");
    if (ps->cfg.map_alpha != 0.0) return fail(FC_ERR_ARG, "a Cartesian grid only (map_alpha = 0)");
    if (level < ps->cfg.min_level || level > ps->cfg.max_level) return fail(FC_ERR_ARG, "bad level");
    if (ps->lr.count[level] != (int)ps->mesh.lv.size()) return fail(FC_ERR_ARG, "needs a uniform mesh at `level`");
    if (!(dt > 0)) return fail(FC_ERR_ARG, "dt must be positive");
    for (int k = 0; k < 4; k++)
        if (ps->cfg.bc[k] != FC_BC_PERIODIC) return fail(FC_ERR_ARG, "needs periodic boundaries");
    return FC_OK;
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

fc_status fc_step_uniform(fc_patchstore *ps, int32_t level, double t, double dt, const double *q_in, double *q_out,
                          void *stream) {
    fc_status r = check_uniform_periodic(ps, level, dt);
    if (r != FC_OK) return r;
    if (!q_in || !q_out) return fail(FC_ERR_ARG, "null array");
    if (q_in == q_out) return fail(FC_ERR_ARG, "q_out must be a separate array");
    if (!aligned16(q_in) || !aligned16(q_out)) return fail(FC_ERR_ARG, "arrays must be 16-byte aligned");
    const int32_t *ls = (const int32_t *)(ps->ws + ps->off_ls);
    Ctx c = make_ctx(ps);
    HIPCHK(launch_step_leaf(c, ps->mx, level, ps->lr.start[level], ps->lr.count[level], t, dt, ls, q_in, q_out,
                            (hipStream_t)stream));
    return FC_OK;
}

fc_status fc_adjoint_step(fc_patchstore *ps, int32_t level, double t, double dt, const double *q_in,
                          const double *lambda_in, double *lambda_out, void *stream) {
    fc_status r = check_uniform_periodic(ps, level, dt);
    if (r != FC_OK) return r;
    if (!q_in || !lambda_in || !lambda_out) return fail(FC_ERR_ARG, "null array");
    if (lambda_out == lambda_in || lambda_out == q_in) return fail(FC_ERR_ARG, "lambda_out must be a separate array");
    if (!aligned16(q_in) || !aligned16(lambda_in) || !aligned16(lambda_out))
        return fail(FC_ERR_ARG, "arrays must be 16-byte aligned");
    const int32_t *ls = (const int32_t *)(ps->ws + ps->off_ls);
    // transpose of copy + advance in one gather pass
    Ctx c = make_ctx(ps);
    HIPCHK(launch_adjoint(c, ps->mx, level, ps->lr.start[level], ps->lr.count[level], t, dt, ls, q_in, lambda_in, lambda_out,
                          (hipStream_t)stream));
    return FC_OK;
}

fc_status fc_check_device(fc_patchstore *ps, void *stream) {
    fc_status r = check_bound(ps);
    if (r != FC_OK) return r;
    return check_device_error(ps, (hipStream_t)stream);
}

fc_status fc_set_persistent_grid(fc_patchstore *ps, int32_t grid, int32_t *max_grid) {
    if (!ps) return fail(FC_ERR_ARG, "null store");
    if (grid < 0) return fail(FC_ERR_ARG, "grid must be >= 0");
    ps->pgrid_user = grid;
    if (max_grid) *max_grid = ps->pgrid;
    drop_graph(ps);
    return FC_OK;
}

fc_status fc_set_variant(fc_patchstore *ps, int32_t threads_per_patch) {
    if (!ps) return fail(FC_ERR_ARG, "null store");
    if (!valid_nt(ps->mx, threads_per_patch, ps->cfg.equation))
        return fail(FC_ERR_ARG, "unsupported threads per patch for this mx");
    ps->nt = threads_per_patch;
    ps->seg = 0;
    if (ps->ws) ps->pgrid = persistent_max_grid(persistent_cfg(ps), ps->cfg.map_alpha != 0.0 ? 2 : ps->cfg.equation);
    drop_graph(ps);
    return FC_OK;
}

// the long tile of the current variant, if the store's advance has tiles
static int store_tile_long(const fc_patchstore *ps, int nt) {
    return (ps->cfg.equation == FC_EQ_ADVECTION && ps->cfg.map_alpha == 0.0) ? tile_long(ps->mx, nt) : 0;
}

fc_status fc_set_tile(fc_patchstore *ps, int32_t seg_cells) {
    if (!ps) return fail(FC_ERR_ARG, "null store");
    const int def = tile_default(ps->mx, ps->nt), lg = store_tile_long(ps, ps->nt);
    if (seg_cells == 0 || seg_cells == def) ps->seg = 0;
    else if (lg != 0 && seg_cells == lg) ps->seg = lg;
    else return fail(FC_ERR_ARG, "unsupported segment length for this mx, thread count and equation");
    drop_graph(ps);
    return FC_OK;
}

fc_status fc_get_launch(const fc_patchstore *ps, int32_t *threads_per_patch, int32_t *seg_cells) {
    if (!ps) return fail(FC_ERR_ARG, "null store");
    if (threads_per_patch) *threads_per_patch = ps->nt;
    if (seg_cells) *seg_cells = ps->seg ? ps->seg : tile_default(ps->mx, ps->nt);
    return FC_OK;
}

fc_status fc_autotune(fc_patchstore *ps, int32_t *threads_out, void *stream) {
    fc_status r = check_bound(ps);
    if (r != FC_OK) return r;
    hipStream_t s = (hipStream_t)stream;
    // time the advance of the most populated level (the fused-load kernel;
    // on a mapped grid the capacity-form kernel), writing only the levels'
    // other buffers (the state is left unchanged), for every pair of threads
    // per patch and tile shape (segment length)
    const int fused = ps->cfg.map_alpha != 0.0 ? 0 : 1;
    int lbest = ps->cfg.min_level;
    for (int l = ps->cfg.min_level; l <= ps->cfg.max_level; l++)
        if (ps->lr.count[l] > ps->lr.count[lbest]) lbest = l;
    const double h = 1.0 / (double)(ps->mx << lbest);
    const double dt = 0.5 * h;
    std::vector<LaunchCfg> cl;
    for (int nt : variants(ps->mx, ps->cfg.equation)) {
        cl.push_back(LaunchCfg{ps->mx, nt, 0});
        const int lg = store_tile_long(ps, nt);
        if (lg) cl.push_back(LaunchCfg{ps->mx, nt, lg});
    }
    const int nc = (int)cl.size();
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    // three interleaved rounds of 10 launches per variant, the best round
    // counts; another variant replaces the default one only if it is at
    // least 5% faster, so that noise does not flip the choice from run to run
    std::vector<float> t(nc, 1e30f);
    for (int round = 0; round < 3; round++)
        for (int k = 0; k < nc; k++) {
            Ctx c = make_ctx(ps);
            c.cflp = nullptr;
            for (int w = 0; w < 2; w++)
                HIPCHK(launch_advance(c, cl[k], lbest, ps->lr.start[lbest], ps->lr.count[lbest], ps->t, dt, fused, s));
            HIPCHK(hipEventRecord(e0, s));
            for (int w = 0; w < 10; w++)
                HIPCHK(launch_advance(c, cl[k], lbest, ps->lr.start[lbest], ps->lr.count[lbest], ps->t, dt, fused, s));
            HIPCHK(hipEventRecord(e1, s));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            t[k] = std::min(t[k], ms);
        }
    const int dnt = default_nt(ps->mx, ps->cfg.equation);
    int kd = 0;
    for (int k = 0; k < nc; k++)
        if (cl[k].nt == dnt && cl[k].seg == 0) kd = k;
    int kb = kd;
    for (int k = 0; k < nc; k++)
        if (k != kd && t[k] < 0.95f * t[kd] && t[k] < t[kb]) kb = k;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    r = fc_set_variant(ps, cl[kb].nt);
    if (r != FC_OK) return r;
    r = fc_set_tile(ps, cl[kb].seg);
    if (r != FC_OK) return r;
    if (threads_out) *threads_out = cl[kb].nt;
    return FC_OK;
}

}  // extern "C"
