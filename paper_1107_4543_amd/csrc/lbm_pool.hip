// Pool of lattices advanced together: batched stepping with a recorded step
// loop (HIP graph), continuous membership, per-member step counts.
//
// Device side (carved from the caller's pool workspace):
//   [ PoolHeader ][ PoolMember x max_members ][ PoolTile x max_tiles ]
// Host side: a mirror of every member's progress.  Progress is deterministic
// (a chunk of kk steps advances each member by min(kk, remaining)), so the
// host always knows t_done without reading the device, and the device copy
// of t_done is advanced by a commit kernel at the end of every chunk.  Tables
// are rebuilt on the host and uploaded (stream-ordered) only when membership
// changes; the recorded graphs read them through fixed device pointers and
// stay valid.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <tuple>
#include <string>
#include <vector>

#include "lbm_internal.hpp"

namespace {

lbm_status pfail(lbm_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    lbm::set_error_text(buf);
    return s;
}

lbm_status phip(hipError_t e, const char *what) { return pfail(LBM_E_HIP, "%s: %s", what, hipGetErrorString(e)); }

size_t a256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Slot {
    lbm_lattice *lat = nullptr;
    int64_t t0 = 0, t_done = 0, t_target = 0;
    int64_t flips = 0;               // launches taken (buffer swaps) since added
    int cur0 = 0;
    bool finishing = false;          // reached t_target; waiting for poll
    hipEvent_t ev_in = nullptr;      // lattice stream -> pool stream
    hipEvent_t ev_done = nullptr;    // pool stream -> lattice stream
};

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

int class_of(const lbm_lattice *L) { return L->v.storage * 2 + L->v.compute; }

}  // namespace

struct lbm_pool {
    char *ws = nullptr;
    size_t ws_bytes = 0;
    hipStream_t stream = nullptr;
    int max_members = 0, max_tiles = 0;
    lbm::PoolHeader *d_hdr = nullptr;
    lbm::PoolMember *d_mem = nullptr;
    lbm::PoolTile *d_tiles = nullptr;
    size_t table_bytes = 0;
    void *stage = nullptr;           // pinned host staging of the tables
    hipEvent_t ev_stage = nullptr;
    bool stage_pending = false;
    bool dirty = true;
    unsigned range_mask = 0;         // table ranges (class * kChains + chain) with tiles
    int ntiles = 0;
    unsigned two_mask = 0;           // table ranges with two-wave strip tasks
    int max_range_tiles = 0;         // largest one-step tile range
    int max_range_tasks = 0;         // largest T-step task range
    int max_range_two = 0;           // largest two-wave task range
    lbm_pool_shape shape{256, 512, 4096, 256, 7, 96, 4, 32};
    std::vector<Slot> slots;
    std::vector<int> finishing;      // slot indices in completion order
    std::map<std::tuple<unsigned, unsigned, int, int, int, int, int, int>, GraphEntry> graphs;   // (range masks, steps, steps per T-step launch, one-step launches, grids)
};

namespace {

// Lattices narrower than the tile size are cut into bands of whole rows;
// rows longer than max(tile_cells, 1024) cells are cut into segments.
int tile_rows(const lbm_pool_shape &sh, const lbm_lattice *L)
{
    int r = sh.tile_cells / std::max(1, L->v.nx);
    return std::max(1, std::min(r, L->v.ny));
}

int tile_cols(const lbm_pool_shape &sh, const lbm_lattice *L)
{
    const int seg = std::max(sh.tile_cells, 1024);
    return L->v.nx <= seg ? L->v.nx : seg;
}

// T-step strip tasks: multi_strip_cols output columns by seg_rows rows.
int elem_bytes(const lbm_lattice *L)
{
    static const int bytes[4] = {8, 4, 2, 2};   // storage element size by lbm_storage
    return bytes[L->v.storage];
}

int strip_cols(const lbm_pool_shape &sh, const lbm_lattice *L)
{
    return lbm::multi_strip_cols(sh.steps_per_launch, elem_bytes(L));
}

// Shared-halo tables (flags bit 5): strip tasks of one workgroup each, as
// wide as its lanes allow: workgroups of kWgMaxWaves waves over a member's
// columns from x = 0, the columns left over in one more, narrower, four-wave
// strip -- or, with flags bit 6 (kWgTwo) in the shape, in one two-wave strip
// when they fit it.  The two-wave strips idle fewer lanes on narrow members
// but run as a second kernel beside the four-wave one: within the spread on
// the 256-lattice batch, and slower on a lone lattice with such columns
// (2048^2: 241k against 280k MLUPS), so they are not the default.
bool wg_table(const lbm_pool_shape &sh) { return sh.steps_per_launch > 1 && (sh.flags & lbm::kWgHalo) != 0; }

// The shape's kernel flags (the four-wave kernel's template flags): the
// table-layout bit kWgTwo removed.
int kernel_flags(const lbm_pool_shape &sh) { return sh.flags & ~lbm::kWgTwo; }

int task_cols(const lbm_pool_shape &sh, const lbm_lattice *L)
{
    return wg_table(sh) ? lbm::multi_strip_cols(sh.steps_per_launch, elem_bytes(L), 64 * lbm::kWgMaxWaves)
                        : strip_cols(sh, L);
}

// Strips of a member in a shared-halo table: n4 four-wave strips of w4
// columns (the last may be narrower), then two = 0 or 1 two-wave strip of
// the remaining columns.
struct WgStrips {
    int w4, n4, two;
};

WgStrips wg_strips(const lbm_pool_shape &sh, const lbm_lattice *L)
{
    WgStrips g;
    g.w4 = task_cols(sh, L);
    const int w2 = lbm::multi_strip_cols(sh.steps_per_launch, elem_bytes(L), 128);
    g.n4 = L->v.nx / g.w4;
    const int rem = L->v.nx - g.n4 * g.w4;
    g.two = (sh.flags & lbm::kWgTwo) && rem > 0 && rem <= w2;
    if (rem > 0 && !g.two) ++g.n4;
    return g;
}

// Segments of a member's strips: the ny rows cut into k = max(1, round(ny
// / seg_rows)) nearly equal segments (heights differ by at most one row), so
// that no member ends in a short segment that pays a whole pipeline start-up.
int segments_of(int seg_rows, const lbm_lattice *L)
{
    return std::max(1, (L->v.ny + seg_rows / 2) / seg_rows);
}

// Strips of a member's T-step tasks (four- and two-wave ones in a
// shared-halo table).
int strips_of(const lbm_pool_shape &sh, const lbm_lattice *L)
{
    if (wg_table(sh)) {
        const WgStrips g = wg_strips(sh, L);
        return g.n4 + g.two;
    }
    const int w = task_cols(sh, L);
    return (L->v.nx + w - 1) / w;
}

int tasks_of(const lbm_pool_shape &sh, const lbm_lattice *L)
{
    if (sh.steps_per_launch < 2) return 0;
    return strips_of(sh, L) * segments_of(sh.seg_rows, L);
}

// Table entries of one unfinished member: one-step tiles plus T-step tasks.
int onestep_tiles_of(const lbm_pool_shape &sh, const lbm_lattice *L)
{
    const int r = tile_rows(sh, L), c = tile_cols(sh, L);
    return ((L->v.ny + r - 1) / r) * ((L->v.nx + c - 1) / c);
}

int tiles_of(const lbm_pool_shape &sh, const lbm_lattice *L) { return onestep_tiles_of(sh, L) + tasks_of(sh, L); }

// Segment height of a pool's table: the shape's seg_rows, or -- when the
// unfinished members' strips cut at that height give fewer tasks than fill
// the device once (three four-wave workgroups per compute unit, the count a
// single lattice's default measured best with, or eight single waves; when
// every member has FP64 storage two workgroups, with seg_rows counting half
// as tall again, when every member has 16-bit storage four, with seg_rows
// counting three quarters as tall), as
// with a few small members or one job of a
// lightly loaded serving pool -- the shortest height whose tasks still fit
// in that one round (a task beyond it would run as a fourth workgroup on a
// unit and stretch the launch; a lone 4096^2 lattice gets 45 segments of 91
// rows per strip, 765 tasks, not 46 of 90, 782), at least 8 rows (as a
// single lattice's default shape: the pipeline then repeats its 2(T-1)
// start-up rows often, yet a full device still measured faster) and never
// above seg_rows, as long as the tile table holds them.
int table_seg_rows(const lbm_pool *P)
{
    const lbm_pool_shape &sh = P->shape;
    if (sh.steps_per_launch < 2) return sh.seg_rows;
    int64_t strip_rows = 0, onestep = 0;
    bool all_f64 = true, all_half = true;
    for (const Slot &sl : P->slots) {
        if (!sl.lat || sl.t_done >= sl.t_target) continue;
        strip_rows += (int64_t)strips_of(sh, sl.lat) * sl.lat->v.ny;
        onestep += onestep_tiles_of(sh, sl.lat);
        const int st = sl.lat->v.storage;
        all_f64 = all_f64 && st == LBM_STORE_F64;
        all_half = all_half && (st == LBM_STORE_F16 || st == LBM_STORE_BF16);
    }
    // Workgroups per compute unit, as a single lattice's default for the
    // storage type: FP64 workgroups hold about 250 registers per lane, so two
    // fit, with segments half as tall again as the shape's; 16-bit ones hold
    // at most 120, so four fit, with segments three quarters as tall
    int per_cu = 3, cap = sh.seg_rows;
    if (wg_table(sh) && all_f64) {
        per_cu = 2;
        cap = std::min(4096, sh.seg_rows * 3 / 2);
    } else if (wg_table(sh) && all_half) {
        per_cu = 4;
        cap = std::max(1, sh.seg_rows * 3 / 4);
    }
    const int64_t fill = (int64_t)lbm::device_cus() * (wg_table(sh) ? per_cu : 8);
    auto tasks_at = [&](int rows) {
        int64_t n = 0;
        for (const Slot &sl : P->slots)
            if (sl.lat && sl.t_done < sl.t_target) n += (int64_t)strips_of(sh, sl.lat) * segments_of(rows, sl.lat);
        return n;
    };
    // any height other than seg_rows must leave the table room (lbm_pool_add
    // counted every member's tasks at seg_rows)
    auto fits = [&](int rows) { return rows >= sh.seg_rows || onestep + tasks_at(rows) <= P->max_tiles; };
    if (tasks_at(cap) >= fill) return fits(cap) ? cap : sh.seg_rows;
    const int low = std::min(cap, 8);
    int seg = (int)std::max<int64_t>(low, std::min<int64_t>(cap, strip_rows / fill));
    while (seg < cap && tasks_at(seg) > fill) ++seg;
    return fits(seg) ? seg : (fits(cap) ? cap : sh.seg_rows);
}

void drop_graphs(lbm_pool *P)
{
    for (auto &kv : P->graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    P->graphs.clear();
}

// Rebuilds the member and tile tables on the host and uploads them.
lbm_status upload(lbm_pool *P)
{
    if (!P->dirty) return LBM_OK;
    hipError_t e;
    if (P->stage_pending) {
        if ((e = hipEventSynchronize(P->ev_stage)) != hipSuccess) return phip(e, "hipEventSynchronize");
        P->stage_pending = false;
    }
    char *base = (char *)P->stage;
    lbm::PoolHeader *hdr = (lbm::PoolHeader *)base;
    lbm::PoolMember *mem = (lbm::PoolMember *)(base + ((char *)P->d_mem - P->ws));
    lbm::PoolTile *tiles = (lbm::PoolTile *)(base + ((char *)P->d_tiles - P->ws));
    memset(base, 0, (size_t)((char *)P->d_tiles - P->ws));
    // Chains: the unfinished members of each class, largest first, each to
    // the chain of that class with the fewest cells so far.
    std::vector<int> chain(P->max_members, 0);
    {
        std::vector<std::pair<int64_t, int>> by_size;
        for (int i = 0; i < P->max_members; ++i) {
            const Slot &sl = P->slots[i];
            if (sl.lat && sl.t_done < sl.t_target) by_size.push_back({-(int64_t)sl.lat->v.nx * sl.lat->v.ny, i});
        }
        std::sort(by_size.begin(), by_size.end());
        int64_t load[lbm::kClasses][lbm::kChains] = {};
        for (const auto &e : by_size) {
            const int c = class_of(P->slots[e.second].lat);
            int best = 0;
            for (int k = 1; k < lbm::kChains; ++k)
                if (load[c][k] < load[c][best]) best = k;
            chain[e.second] = best;
            load[c][best] -= e.first;
        }
    }
    const int seg_rows = table_seg_rows(P);
    struct T { int range; int64_t cells; lbm::PoolTile t; };
    std::vector<T> all, tasks, twos;
    for (int i = 0; i < P->max_members; ++i) {
        const Slot &s = P->slots[i];
        lbm::PoolMember &m = mem[i];
        if (!s.lat) {
            m.cls = -1;
            continue;
        }
        const lbm_lattice *L = s.lat;
        m.buf[0] = L->buf[0];
        m.buf[1] = L->buf[1];
        m.nx = L->v.nx;
        m.ny = L->v.ny;
        m.pitch = L->v.pitch;
        m.cur0 = s.cur0;
        m.plane = L->v.plane;
        m.t_done = s.t_done;
        m.t_target = s.t_target;
        m.flips = s.flips;
        m.rf = lbm::relax_f32(L->v);
        m.rd = lbm::relax_f64(L->v);
        m.scale = (float)L->v.scale;
        m.inv_scale = (float)L->v.inv_scale;
        m.cls = class_of(L);
        if (s.t_done >= s.t_target) continue;        // finished: no tiles
        const int r = tile_rows(P->shape, L), cw = tile_cols(P->shape, L);
        for (int y0 = 0; y0 < L->v.ny; y0 += r)
            for (int x0 = 0; x0 < L->v.nx; x0 += cw) {
                T t{};
                t.range = m.cls * lbm::kChains + chain[i];
                t.t.member = i;
                t.t.y0 = y0;
                t.t.x0 = x0;
                t.t.nrows = std::min(r, L->v.ny - y0);
                t.t.ncols = std::min(cw, L->v.nx - x0);
                t.cells = (int64_t)t.t.nrows * t.t.ncols;
                all.push_back(t);
            }
        if (P->shape.steps_per_launch > 1) {
            // four-wave (or one-wave) strips, then a two-wave one
            const bool wg = wg_table(P->shape);
            const WgStrips g = wg ? wg_strips(P->shape, L) : WgStrips{0, 0, 0};
            const int w = task_cols(P->shape, L), k = segments_of(seg_rows, L);
            const int nfull = wg ? g.n4 : (L->v.nx + w - 1) / w;
            for (int sg = 0; sg < k; ++sg) {
                const int y0 = (int)((int64_t)L->v.ny * sg / k), y1 = (int)((int64_t)L->v.ny * (sg + 1) / k);
                for (int q = 0; q < nfull + g.two; ++q) {
                    T t{};
                    t.range = m.cls * lbm::kChains + chain[i];
                    t.t.member = i;
                    t.t.y0 = y0;
                    t.t.x0 = q * w;
                    t.t.nrows = y1 - y0;
                    t.t.ncols = std::min(w, L->v.nx - t.t.x0);
                    // a wave's (workgroup's) time follows its rows (every
                    // lane works, a partial strip or not)
                    t.cells = (int64_t)t.t.nrows * 64;
                    (q < nfull ? tasks : twos).push_back(t);
                }
            }
        }
    }
    // group by range, longest first (the hardware starts workgroups in
    // order, so the short tasks fill the end of the launch); one-step tiles,
    // then T-step tasks
    auto order = [](const T &a, const T &b) { return a.range != b.range ? a.range < b.range : a.cells > b.cells; };
    std::stable_sort(all.begin(), all.end(), order);
    std::stable_sort(tasks.begin(), tasks.end(), order);
    std::stable_sort(twos.begin(), twos.end(), order);
    const size_t ntot = all.size() + tasks.size() + twos.size();
    if ((int64_t)ntot > P->max_tiles) return pfail(LBM_E_NOMEM, "pool needs %zu tiles, has %d", ntot, P->max_tiles);
    static_assert(lbm::kRanges <= 32, "range mask bits");
    unsigned mask = 0;
    for (int c = 0; c < lbm::kRanges; ++c)
        hdr->begin[c] = hdr->end[c] = hdr->mbegin[c] = hdr->mend[c] = hdr->hbegin[c] = hdr->hend[c] = 0;
    for (size_t j = 0; j < all.size(); ++j) {
        tiles[j] = all[j].t;
        const int c = all[j].range;
        if (!(mask & (1u << c))) hdr->begin[c] = (int)j;
        hdr->end[c] = (int)j + 1;
        mask |= 1u << c;
    }
    unsigned tmask = 0;
    for (size_t j = 0; j < tasks.size(); ++j) {
        const int at = (int)(all.size() + j);
        tiles[at] = tasks[j].t;
        const int c = tasks[j].range;
        if (!(tmask & (1u << c))) hdr->mbegin[c] = at;
        hdr->mend[c] = at + 1;
        tmask |= 1u << c;
    }
    unsigned hmask = 0;
    for (size_t j = 0; j < twos.size(); ++j) {
        const int at = (int)(all.size() + tasks.size() + j);
        tiles[at] = twos[j].t;
        const int c = twos[j].range;
        if (!(hmask & (1u << c))) hdr->hbegin[c] = at;
        hdr->hend[c] = at + 1;
        hmask |= 1u << c;
    }
    P->ntiles = (int)ntot;
    P->max_range_tiles = P->max_range_tasks = P->max_range_two = 0;
    for (int c = 0; c < lbm::kRanges; ++c) {
        P->max_range_tiles = std::max(P->max_range_tiles, hdr->end[c] - hdr->begin[c]);
        P->max_range_tasks = std::max(P->max_range_tasks, hdr->mend[c] - hdr->mbegin[c]);
        P->max_range_two = std::max(P->max_range_two, hdr->hend[c] - hdr->hbegin[c]);
    }
    const size_t used = (size_t)((char *)P->d_tiles - P->ws) + sizeof(lbm::PoolTile) * (size_t)P->ntiles;
    if ((e = hipMemcpyAsync(P->ws, P->stage, used, hipMemcpyHostToDevice, P->stream)) != hipSuccess)
        return phip(e, "hipMemcpyAsync (pool tables)");
    if ((e = hipEventRecord(P->ev_stage, P->stream)) != hipSuccess) return phip(e, "hipEventRecord");
    P->stage_pending = true;
    P->range_mask = mask;
    P->two_mask = hmask;
    P->dirty = false;
    return LBM_OK;
}

// Workgroups per launch: the shape's grid, or fewer when the tables hold
// fewer tiles (rounded up to a power of two so that few graphs are needed).
int launch_grid(const lbm_pool *P)
{
    int g = 1;
    while (g < P->max_range_tiles && g < P->shape.grid) g *= 2;
    return std::min(g, P->shape.grid);
}

// Workgroups of a T-step launch: enough waves (workgroups, in a shared-halo
// table) for the largest range's tasks, rounded up to a power of two, at
// most the shape's grid.
int multi_grid(const lbm_pool *P)
{
    const int per = wg_table(P->shape) ? 1 : P->shape.waves;
    const int need = (P->max_range_tasks + per - 1) / per;
    int g = 1;
    while (g < need && g < P->shape.grid) g *= 2;
    return std::min(g, P->shape.grid);
}

// Workgroups of a two-wave launch: one per task of the largest range,
// rounded up to a power of two, at most the shape's grid.
int two_grid(const lbm_pool *P)
{
    int g = 1;
    while (g < P->max_range_two && g < P->shape.grid) g *= 2;
    return std::min(g, P->shape.grid);
}

// Records a step loop of `len` steps: the chunk schedule of
// lbm_internal.hpp (len / T T-step launches, then `nsingle` of its one-step
// launches) for every table range in `mask`, each launch depending only on
// the same range's previous launch: ranges hold disjoint members, so their
// chains may overlap on the device.  A T-step launch of a range with
// two-wave tasks (`two`) is two nodes, four- and two-wave workgroups, that
// run side by side.  The commit kernel follows every chain.  The one-step
// launches a member takes in the chunk come first, so nsingle only has to
// cover the largest such count among the members.  T is the chunk's steps
// per T-step launch (chunk_steps).
lbm_status get_graph(lbm_pool *P, unsigned mask, unsigned two, int len, int T, int nsingle, hipGraphExec_t *out)
{
    const int grid = launch_grid(P), mgrid = multi_grid(P), tgrid = two_grid(P);
    auto key = std::make_tuple(mask, two, len, T, nsingle, grid, mgrid, tgrid);
    auto it = P->graphs.find(key);
    if (it != P->graphs.end()) {
        *out = it->second.exec;
        return LBM_OK;
    }
    GraphEntry g;
    hipError_t e;
    if ((e = hipGraphCreate(&g.graph, 0)) != hipSuccess) return phip(e, "hipGraphCreate");
    std::vector<hipGraphNode_t> last[lbm::kRanges], cur;
    const lbm::PoolHeader *hdr = P->d_hdr;
    const lbm::PoolMember *mem = P->d_mem;
    const lbm::PoolTile *tiles = P->d_tiles;
    const int nmulti = lbm::chunk_multi_launches(len, T);
    for (int k = 0; k < nmulti + nsingle; ++k) {
        const bool multi = k < nmulti;
        for (int r = 0; r < lbm::kRanges; ++r) {
            if (!(mask & (1u << r))) continue;
            const int c = r / lbm::kChains;
            cur.clear();
            // kind 0: one-step, or T-step of one-wave / four-wave
            // workgroups; kind 1: T-step of two-wave workgroups
            for (int kind = 0; kind < (multi && (two & (1u << r)) ? 2 : 1); ++kind) {
                int range = r, idx = multi ? k : k - nmulti, kk = len, TT = T;
                void *margs[] = {(void *)&hdr, (void *)&mem, (void *)&tiles, (void *)&range, (void *)&idx};
                void *sargs[] = {(void *)&hdr, (void *)&mem, (void *)&tiles, (void *)&range, (void *)&idx, (void *)&kk,
                                 (void *)&TT};
                hipKernelNodeParams np{};
                np.func = !multi    ? lbm::pool_step_kernel(c)
                          : kind    ? lbm::pool_multi_kernel(c, T, kernel_flags(P->shape) | lbm::kWgTwo)
                                    : lbm::pool_multi_kernel(c, T, kernel_flags(P->shape));
                np.gridDim = dim3(!multi ? grid : kind ? tgrid : mgrid);
                np.blockDim = !multi ? dim3(P->shape.block) : dim3(64, kind ? 2 : P->shape.waves);
                np.sharedMemBytes = 0;
                np.kernelParams = multi ? margs : sargs;
                np.extra = nullptr;
                hipGraphNode_t n;
                if (!np.func || (e = hipGraphAddKernelNode(&n, g.graph, last[r].empty() ? nullptr : last[r].data(),
                                                           last[r].size(), &np)) != hipSuccess) {
                    (void)hipGraphDestroy(g.graph);
                    return np.func ? phip(e, "hipGraphAddKernelNode")
                                   : pfail(LBM_E_INVAL, "no pool kernel for this shape");
                }
                cur.push_back(n);
            }
            last[r] = cur;
        }
    }
    std::vector<hipGraphNode_t> prev;
    for (int r = 0; r < lbm::kRanges; ++r) prev.insert(prev.end(), last[r].begin(), last[r].end());
    lbm::PoolMember *memw = P->d_mem;
    int nmem = P->max_members, kk = len, TT = T;
    void *cargs[] = {(void *)&memw, (void *)&nmem, (void *)&kk, (void *)&TT};
    hipKernelNodeParams cp{};
    cp.func = lbm::pool_commit_kernel();
    cp.gridDim = dim3((nmem + 255) / 256);
    cp.blockDim = dim3(256);
    cp.kernelParams = cargs;
    hipGraphNode_t cn;
    if ((e = hipGraphAddKernelNode(&cn, g.graph, prev.empty() ? nullptr : prev.data(), prev.size(), &cp)) !=
        hipSuccess) {
        (void)hipGraphDestroy(g.graph);
        return phip(e, "hipGraphAddKernelNode (commit)");
    }
    if ((e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0)) != hipSuccess) {
        (void)hipGraphDestroy(g.graph);
        return phip(e, "hipGraphInstantiate");
    }
    P->graphs[key] = g;
    *out = g.exec;
    return LBM_OK;
}

// Steps per T-step launch in a chunk of kk steps: the shape's T, or for a
// chunk shorter than T (the end of a run) kk itself, so that the chunk is
// one pass of kk steps over the same strip tasks (their width fits any
// smaller T) when that kernel exists for every class present.
int chunk_steps(const lbm_pool *P, int kk)
{
    const int T = P->shape.steps_per_launch;
    if (T < 2 || kk >= T || kk < 2) return T;
    for (int r = 0; r < lbm::kRanges; ++r) {
        if (!(P->range_mask & (1u << r))) continue;
        if (!lbm::pool_multi_kernel(r / lbm::kChains, kk, kernel_flags(P->shape))) return T;
        if ((P->two_mask & (1u << r)) &&
            !lbm::pool_multi_kernel(r / lbm::kChains, kk, kernel_flags(P->shape) | lbm::kWgTwo))
            return T;
    }
    return kk;
}

// Advances every active member by min(kk, remaining) with one recorded loop
// of kk steps (kk <= graph_steps), holding as many one-step launches as the
// members need in it.
lbm_status run_chunk(lbm_pool *P, int kk)
{
    hipError_t e;
    hipGraphExec_t ex;
    const int T = chunk_steps(P, kk);
    int64_t need = 0;
    for (const Slot &s : P->slots) {
        if (!s.lat || s.finishing) continue;
        const int64_t rem = s.t_target - s.t_done;
        need = std::max(need, std::min<int64_t>(rem, kk) - lbm::member_multi(rem, kk, T) * T);
    }
    need = std::min<int64_t>(need, lbm::chunk_single_launches(kk, T));
    lbm_status st = get_graph(P, P->range_mask, P->two_mask, kk, T, (int)need, &ex);
    if (st != LBM_OK) return st;
    if ((e = hipGraphLaunch(ex, P->stream)) != hipSuccess) return phip(e, "hipGraphLaunch");
    for (int i = 0; i < P->max_members; ++i) {
        Slot &s = P->slots[i];
        if (!s.lat || s.finishing) continue;
        const int64_t rem = s.t_target - s.t_done;
        const int64_t span = std::min<int64_t>(rem, kk);
        const int64_t q = lbm::member_multi(rem, kk, T);
        s.t_done += span;
        s.flips += q + span - q * T;
        if (s.t_done >= s.t_target) {
            s.finishing = true;
            if ((e = hipEventRecord(s.ev_done, P->stream)) != hipSuccess) return phip(e, "hipEventRecord");
            P->finishing.push_back(i);
        }
    }
    return LBM_OK;
}

bool valid_shape(const lbm_pool_shape &s)
{
    const bool multi_ok = s.steps_per_launch == 1 ||
                          ((s.steps_per_launch == 2 || s.steps_per_launch == 4 || s.steps_per_launch == 5 ||
                            s.steps_per_launch == 6 || s.steps_per_launch == 7) && s.seg_rows >= 1 &&
                           s.seg_rows <= 4096 && s.waves >= 1 && s.waves <= 4 &&
                           (!(s.flags & lbm::kWgHalo) ||
                            (s.waves == lbm::kWgMaxWaves &&
                             lbm::pool_multi_kernel(LBM_STORE_F32 * 2 + LBM_COMPUTE_F32, s.steps_per_launch,
                                                    kernel_flags(s) | lbm::kWgTwo))) &&
                           (!(s.flags & lbm::kWgTwo) || (s.flags & lbm::kWgHalo)) &&
                           lbm::pool_multi_kernel(LBM_STORE_F32 * 2 + LBM_COMPUTE_F32, s.steps_per_launch,
                                                  kernel_flags(s)));
    return s.tile_cells >= 64 && s.tile_cells <= (1 << 22) && s.block >= 64 && s.block <= 1024 && s.block % 64 == 0 &&
           s.grid >= 1 && s.grid <= (1 << 20) && s.graph_steps >= 1 && s.graph_steps <= 1024 && multi_ok;
}

// Hands a member back to its lattice: host state and stream order.
lbm_status release(lbm_pool *P, int i)
{
    Slot &s = P->slots[i];
    lbm_lattice *L = s.lat;
    hipError_t e;
    if (!s.finishing) {
        if ((e = hipEventRecord(s.ev_done, P->stream)) != hipSuccess) return phip(e, "hipEventRecord");
    }
    if ((e = hipStreamWaitEvent(L->stream, s.ev_done, 0)) != hipSuccess) return phip(e, "hipStreamWaitEvent");
    L->t = s.t0 + s.t_done;
    L->cur = (int)((s.cur0 + s.flips) & 1);
    L->pool = nullptr;
    s.lat = nullptr;
    s.finishing = false;
    s.t_done = s.t_target = s.flips = 0;
    P->dirty = true;
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_pool_workspace_bytes(int32_t max_members, int32_t max_tiles)
{
    if (max_members < 1 || max_members > (1 << 20) || max_tiles < 1 || max_tiles > (1 << 26)) return 0;
    return a256(sizeof(lbm::PoolHeader)) + a256(sizeof(lbm::PoolMember) * (size_t)max_members) +
           a256(sizeof(lbm::PoolTile) * (size_t)max_tiles);
}

lbm_status lbm_pool_create(void *dev_ws, size_t ws_bytes, void *stream, int32_t max_members, int32_t max_tiles,
                           lbm_pool **out)
{
    if (!out) return pfail(LBM_E_INVAL, "out is NULL");
    *out = nullptr;
    const size_t need = lbm_pool_workspace_bytes(max_members, max_tiles);
    if (need == 0) return pfail(LBM_E_INVAL, "max_members in [1, 2^20] and max_tiles in [1, 2^26] required");
    if (!dev_ws || ((uintptr_t)dev_ws & 255u)) return pfail(LBM_E_INVAL, "workspace must be non-NULL and 256-byte aligned");
    if (ws_bytes < need) return pfail(LBM_E_NOMEM, "pool workspace has %zu bytes, needs %zu", ws_bytes, need);
    lbm_pool *P = new (std::nothrow) lbm_pool();
    if (!P) return pfail(LBM_E_NOMEM, "host allocation failed");
    P->ws = (char *)dev_ws;
    P->ws_bytes = ws_bytes;
    P->stream = (hipStream_t)stream;
    P->max_members = max_members;
    P->max_tiles = max_tiles;
    P->d_hdr = (lbm::PoolHeader *)P->ws;
    P->d_mem = (lbm::PoolMember *)(P->ws + a256(sizeof(lbm::PoolHeader)));
    P->d_tiles = (lbm::PoolTile *)((char *)P->d_mem + a256(sizeof(lbm::PoolMember) * (size_t)max_members));
    P->table_bytes = need;
    P->slots.resize(max_members);
    hipError_t e;
    lbm_status st = LBM_OK;
    if ((e = hipHostMalloc(&P->stage, need, hipHostMallocDefault)) != hipSuccess) st = phip(e, "hipHostMalloc");
    if (st == LBM_OK && (e = hipEventCreateWithFlags(&P->ev_stage, hipEventDisableTiming)) != hipSuccess)
        st = phip(e, "hipEventCreate");
    for (int i = 0; i < max_members && st == LBM_OK; ++i) {
        if ((e = hipEventCreateWithFlags(&P->slots[i].ev_in, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&P->slots[i].ev_done, hipEventDisableTiming)) != hipSuccess)
            st = phip(e, "hipEventCreate");
    }
    if (st != LBM_OK) {
        lbm_pool_destroy(P);
        return st;
    }
    *out = P;
    return LBM_OK;
}

lbm_status lbm_pool_destroy(lbm_pool *pool)
{
    if (!pool) return pfail(LBM_E_INVAL, "pool is NULL");
    // hand back members still in the pool (their stream waits for the pool)
    for (int i = 0; i < pool->max_members; ++i)
        if (pool->slots[i].lat) (void)release(pool, i);
    if (pool->stage_pending) (void)hipEventSynchronize(pool->ev_stage);
    drop_graphs(pool);
    for (Slot &s : pool->slots) {
        if (s.ev_in) (void)hipEventDestroy(s.ev_in);
        if (s.ev_done) (void)hipEventDestroy(s.ev_done);
    }
    if (pool->ev_stage) (void)hipEventDestroy(pool->ev_stage);
    if (pool->stage) (void)hipHostFree(pool->stage);
    delete pool;
    return LBM_OK;
}

lbm_status lbm_pool_add(lbm_pool *pool, lbm_lattice *lat, int64_t nsteps)
{
    if (!pool || !lat) return pfail(LBM_E_INVAL, "NULL argument");
    if (nsteps < 0) return pfail(LBM_E_INVAL, "nsteps must be >= 0");
    if (!lat->initialized) return pfail(LBM_E_STATE, "lattice must be initialised before joining a pool");
    if (lat->pool) return pfail(LBM_E_STATE, "lattice is already in a pool");
    int free_slot = -1, tiles = 0;
    for (int i = 0; i < pool->max_members; ++i) {
        const Slot &s = pool->slots[i];
        if (!s.lat) {
            if (free_slot < 0) free_slot = i;
        } else if (s.t_done < s.t_target) {
            tiles += tiles_of(pool->shape, s.lat);
        }
    }
    if (free_slot < 0) return pfail(LBM_E_NOMEM, "pool is full (%d members)", pool->max_members);
    if (tiles + tiles_of(pool->shape, lat) > pool->max_tiles)
        return pfail(LBM_E_NOMEM, "pool tile table is full (%d tiles)", pool->max_tiles);
    Slot &s = pool->slots[free_slot];
    hipError_t e;
    if ((e = hipEventRecord(s.ev_in, lat->stream)) != hipSuccess) return phip(e, "hipEventRecord");
    if ((e = hipStreamWaitEvent(pool->stream, s.ev_in, 0)) != hipSuccess) return phip(e, "hipStreamWaitEvent");
    s.lat = lat;
    s.t0 = lat->t;
    s.cur0 = lat->cur;
    s.t_done = 0;
    s.flips = 0;
    s.t_target = nsteps;
    s.finishing = false;
    lat->pool = pool;
    pool->dirty = true;
    if (nsteps == 0) {
        s.finishing = true;
        if ((e = hipEventRecord(s.ev_done, pool->stream)) != hipSuccess) return phip(e, "hipEventRecord");
        pool->finishing.push_back(free_slot);
    }
    return LBM_OK;
}

lbm_status lbm_pool_remove(lbm_pool *pool, lbm_lattice *lat)
{
    if (!pool || !lat) return pfail(LBM_E_INVAL, "NULL argument");
    if (lat->pool != pool) return pfail(LBM_E_STATE, "lattice is not in this pool");
    for (int i = 0; i < pool->max_members; ++i)
        if (pool->slots[i].lat == lat) {
            pool->finishing.erase(std::remove(pool->finishing.begin(), pool->finishing.end(), i),
                                  pool->finishing.end());
            return release(pool, i);
        }
    return pfail(LBM_E_STATE, "lattice not found in pool");
}

lbm_status lbm_pool_step(lbm_pool *pool, int64_t nsteps)
{
    if (!pool) return pfail(LBM_E_INVAL, "pool is NULL");
    if (nsteps < 0) return pfail(LBM_E_INVAL, "nsteps must be >= 0");
    while (nsteps > 0) {
        int64_t max_rem = 0;
        for (const Slot &s : pool->slots)
            if (s.lat && !s.finishing) max_rem = std::max(max_rem, s.t_target - s.t_done);
        if (max_rem == 0) break;
        lbm_status st = upload(pool);
        if (st != LBM_OK) return st;
        // the longest recorded loop that fits: T 2^m steps (only T-step
        // launches for members that stay); below T, the rest in one chunk
        // (one shorter pass, see chunk_steps); one step per launch: powers
        // of two
        const int64_t lim = std::min<int64_t>({nsteps, (int64_t)pool->shape.graph_steps, max_rem});
        const int T = pool->shape.steps_per_launch;
        int kk = 1;
        if (T > 1 && lim >= T) {
            kk = T;
            while ((int64_t)kk * 2 <= lim) kk *= 2;
        } else if (T > 1) {
            kk = (int)lim;
        } else {
            while ((int64_t)kk * 2 <= lim) kk *= 2;
        }
        if ((st = run_chunk(pool, kk)) != LBM_OK) return st;
        nsteps -= kk;
        // finished members keep their (now idle) tiles until the next upload
        for (const Slot &s : pool->slots)
            if (s.lat && s.finishing && s.t_done == s.t_target) {
                pool->dirty = true;
                break;
            }
    }
    return LBM_OK;
}

lbm_status lbm_pool_poll(lbm_pool *pool, lbm_lattice **done, int32_t cap, int32_t wait, int32_t *ndone)
{
    if (!pool || !ndone || cap < 0 || (cap > 0 && !done)) return pfail(LBM_E_INVAL, "bad argument");
    *ndone = 0;
    hipError_t e;
    if (wait && !pool->finishing.empty() && cap > 0) {
        if ((e = hipEventSynchronize(pool->slots[pool->finishing.front()].ev_done)) != hipSuccess)
            return phip(e, "hipEventSynchronize");
    }
    std::vector<int> keep;
    for (int i : pool->finishing) {
        if (*ndone >= cap) {
            keep.push_back(i);
            continue;
        }
        e = hipEventQuery(pool->slots[i].ev_done);
        if (e == hipErrorNotReady) {
            keep.push_back(i);
            continue;
        }
        if (e != hipSuccess) return phip(e, "hipEventQuery");
        lbm_lattice *L = pool->slots[i].lat;
        lbm_status st = release(pool, i);
        if (st != LBM_OK) return st;
        done[(*ndone)++] = L;
    }
    pool->finishing.swap(keep);
    return LBM_OK;
}

int32_t lbm_pool_members(const lbm_pool *pool)
{
    if (!pool) return -1;
    int n = 0;
    for (const Slot &s : pool->slots) n += s.lat != nullptr;
    return n;
}

int64_t lbm_pool_remaining(const lbm_pool *pool, const lbm_lattice *lat)
{
    if (!pool || !lat) return -1;
    for (const Slot &s : pool->slots)
        if (s.lat == lat) return s.t_target - s.t_done;
    return -1;
}

lbm_status lbm_pool_get_shape(const lbm_pool *pool, lbm_pool_shape *out)
{
    if (!pool || !out) return pfail(LBM_E_INVAL, "NULL argument");
    *out = pool->shape;
    return LBM_OK;
}

lbm_status lbm_pool_set_shape(lbm_pool *pool, const lbm_pool_shape *shape)
{
    if (!pool || !shape) return pfail(LBM_E_INVAL, "NULL argument");
    if (!valid_shape(*shape)) return pfail(LBM_E_INVAL, "invalid pool shape");
    int tiles = 0;
    for (const Slot &s : pool->slots)
        if (s.lat && s.t_done < s.t_target) tiles += tiles_of(*shape, s.lat);
    if (tiles > pool->max_tiles) return pfail(LBM_E_NOMEM, "shape needs %d tiles, pool has %d", tiles, pool->max_tiles);
    drop_graphs(pool);
    pool->shape = *shape;
    pool->dirty = true;
    return LBM_OK;
}

lbm_status lbm_pool_time_launches(lbm_pool *pool, int32_t reps, double *avg_us)
{
    if (!pool || reps < 1 || !avg_us) return pfail(LBM_E_INVAL, "bad argument");
    lbm_status st = upload(pool);
    if (st != LBM_OK) return st;
    hipEvent_t e0, e1;
    hipError_t e;
    if ((e = hipEventCreate(&e0)) != hipSuccess) return phip(e, "hipEventCreate");
    if ((e = hipEventCreate(&e1)) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return phip(e, "hipEventCreate");
    }
    // The first launch of a chunk without commit: every active member
    // recomputes its next state into its other buffer; the state itself
    // does not change.
    const int T = pool->shape.steps_per_launch;
    auto launch_all = [&]() -> hipError_t {
        for (int c = 0; c < lbm::kRanges; ++c) {
            if (!(pool->range_mask & (1u << c))) continue;
            hipError_t r = T > 1 ? lbm::launch_pool_multi(c, T, kernel_flags(pool->shape), pool->d_hdr, pool->d_mem,
                                                          pool->d_tiles, 0, multi_grid(pool), pool->shape.waves,
                                                          pool->stream)
                                 : lbm::launch_pool_step(c, pool->d_hdr, pool->d_mem, pool->d_tiles, 0, 1, 1,
                                                         launch_grid(pool), pool->shape.block, pool->stream);
            if (r == hipSuccess && T > 1 && (pool->two_mask & (1u << c)))
                r = lbm::launch_pool_multi(c, T, kernel_flags(pool->shape) | lbm::kWgTwo, pool->d_hdr, pool->d_mem,
                                           pool->d_tiles, 0, two_grid(pool), 2, pool->stream);
            if (r != hipSuccess) return r;
        }
        return hipSuccess;
    };
    e = launch_all();
    if (e == hipSuccess) e = hipEventRecord(e0, pool->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_all();
    if (e == hipSuccess) e = hipEventRecord(e1, pool->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return phip(e, "pool timing");
    *avg_us = 1000.0 * ms / reps;
    return LBM_OK;
}

lbm_status lbm_pool_tune(lbm_pool *pool, int32_t reps, lbm_pool_shape *best, double *best_us)
{
    if (!pool || reps < 1) return pfail(LBM_E_INVAL, "bad argument");
    const lbm_pool_shape keep = pool->shape;
    lbm_pool_shape best_s = keep;
    double best_t = INFINITY;
    auto consider = [&](const lbm_pool_shape &s) -> lbm_status {
        if (lbm_pool_set_shape(pool, &s) != LBM_OK) return LBM_OK;   // does not fit: skip
        double us;
        lbm_status st = lbm_pool_time_launches(pool, reps, &us);
        if (st != LBM_OK) return st;
        us /= s.steps_per_launch;                                      // per step
        if (us < best_t) {
            best_t = us;
            best_s = s;
        }
        return LBM_OK;
    };
    // one step per launch: tile, workgroup and grid sizes
    lbm_pool_shape single = keep;
    single.steps_per_launch = 1;
    double single_t = INFINITY;
    for (int cells : {256, 512, 1024, 2048, 4096, 16384})
        for (int block : {256, 512, 1024})
            for (int grid : {1024, 4096, 16384, 65536, 262144}) {
                lbm_pool_shape s = keep;
                s.steps_per_launch = 1;
                s.tile_cells = cells;
                s.block = block;
                s.grid = grid;
                const double before = best_t;
                lbm_status st = consider(s);
                if (st != LBM_OK) return st;
                if (best_t < before && best_t < single_t) {
                    single_t = best_t;
                    single = s;
                }
            }
    // several steps per launch (their left-over steps use the best one-step tiles)
    for (int T : {2, 4, 5, 6, 7})
        for (int seg : {32, 48, 64, 96, 128})
            for (int waves : {1, 4})
                for (int flags : {0, 2, 12, 32, 34, 96, 98})   // 32 and up: four waves only
                    for (int grid : {4096, 16384, 65536}) {
                        lbm_pool_shape s = single;
                        s.steps_per_launch = T;
                        s.seg_rows = seg;
                        s.waves = waves;
                        s.flags = flags;
                        s.grid = grid;
                        lbm_status st = consider(s);
                        if (st != LBM_OK) return st;
                    }
    lbm_status st = lbm_pool_set_shape(pool, &best_s);
    if (st != LBM_OK) return st;
    if (best) *best = best_s;
    if (best_us) *best_us = best_t;
    return LBM_OK;
}

}  // extern "C"
