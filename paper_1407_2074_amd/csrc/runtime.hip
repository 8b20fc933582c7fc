// Host side of the C ABI: octree manager (node states, homogeneity, change events, brick-pool
// slots) and launch orchestration.  All voxel work runs in the kernels of build_kernels.hip
// and render_kernels.hip; this file only decides what to launch.
#include "../../include/octree_rc.h"
#include "internal.h"
#include "page_cache.h"
#include "raycommon.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <string>
#include <vector>

using namespace octrc;

namespace {

enum NodeState : int8_t { kNone = -1, kEmpty = 0, kHomogLeaf = 1, kHomog = 2, kBrickState = 3 };

struct HCell {
    // statistics of the node's own level-L brick over its valid voxels
    double bmin[kMaxC] = {0, 0, 0, 0}, bmax[kMaxC] = {0, 0, 0, 0}, bsum[kMaxC] = {0, 0, 0, 0};
    // level-0 region: min / max, inserted voxels per channel, valid voxels
    double smin[kMaxC] = {0, 0, 0, 0}, smax[kMaxC] = {0, 0, 0, 0};
    uint64_t ins[kMaxC] = {0, 0, 0, 0};
    uint64_t nvalid0 = 0;
    uint64_t count = 0;          // valid level-L voxels of the brick
    bool inside = false;
    bool have_stats = false;
    // tree state
    int8_t exists = 0, populated = 0, complete = 0, has_children = 0, state = kNone;
    double avg[kMaxC] = {0, 0, 0, 0};
    // device side
    int32_t slot = -1;
    bool needs_gather = false;   // bordered brick in the slot is not current
    int32_t dev_kind = kAvg;     // last uploaded entry
    int32_t dev_slot = -1;
    float dev_avg[4] = {0, 0, 0, 0};
    float dev_miss[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    bool dev_valid = false;
};

struct Box {
    int32_t lo[3], hi[3];  // inclusive, level-local voxel coordinates
};

// A pinned host buffer paired with a device buffer, grown on demand.
struct Stage {
    void *host = nullptr;
    void *dev = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;  // last use of the host side by an async copy
};

struct RenderSlot {
    Stage st;
    float *part = nullptr;   // depth-segment results of split views ([nsplit][pixel] float4)
    size_t part_cap = 0;
    uint32_t *tmask = nullptr;  // per-view cell transparency masks of the launch
    size_t tmask_cap = 0;
    hipEvent_t k0 = nullptr, k1 = nullptr;   // around the render kernel, when timing is on
    bool k_pending = false;
    int64_t version = -1;   // node-table version the slot's last launch read
    hipEvent_t prep = nullptr;   // end of the launch's preparation on the handle's prep stream
    hipStream_t stream = nullptr;   // the stream of the slot's last launch (st.ev recorded on it)
};

// Default depth segments per ray for views without early termination or checkpoints: the
// longest rays set a launch's duration, and splitting them across waves shortens that
// critical path.  One segment per kSplitPositions positions of the longest possible ray (the
// volume diagonal over the step), at most kSplitMax (5 measured fastest for 1024x1024 views of
// a 512x512x256 octree with the longest tile groups dispatched first; short rays gain nothing
// and stay whole).
#ifndef OCTRC_SPLIT
#define OCTRC_SPLIT 5
#endif
constexpr int kSplitMax = OCTRC_SPLIT;
#ifndef OCTRC_SPLIT_POSITIONS
#define OCTRC_SPLIT_POSITIONS 256.0
#endif
constexpr double kSplitPositions = OCTRC_SPLIT_POSITIONS;

int auto_segments(const VolGeom &g, const oct_view &v)
{
    const double diag = std::sqrt((double)g.dims[0] * g.dims[0] + (double)g.dims[1] * g.dims[1] +
                                  (double)g.dims[2] * g.dims[2]);
    const double n = std::ceil(diag / v.step / kSplitPositions);
    return (int)std::max(1.0, std::min((double)kSplitMax, n));
}

constexpr int kRenderSlots = 8;

// Views per render_views_noalloc call and bytes of its device scratch (per GPU).
constexpr int kNoAllocMaxViews = 64;
constexpr int kNoAllocMaxOrder = 65536;   // tile groups of an ordered view (a 2048x2048 image)
constexpr size_t kScratchBytes = (size_t)16 << 20;

// Forward renders that filled a checkpoint workspace: the backward checks that the octree and
// the views are still those of the forward (ring of the last kCkptLog workspaces).
constexpr int kCkptLog = 64;
struct CkptRec {
    const void *ws = nullptr;
    int64_t version = -1;
    uint64_t views_hash = 0;
    int32_t n_views = 0;
};

}  // namespace

// Device scratch of render_views_noalloc: the view records, sample counters, transfer-function
// tables, transparency masks and tile-group orders of one launch.  Every GPU holds its own
// copy at its own address, which set-up looks up once per device (scratch_for_device); host
// code uses only that address, never this name.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

struct oct_handle {
    oct_create_params p{};
    VolGeom g{};
    int device = 0;
    size_t esz = 2;
    int64_t n_cells = 0;
    uint64_t brick_bytes = 0;
    int64_t n_slots = 0;
    // Uncapped pools hold n_cow slots more, so that an upload can rebuild a brick that renders
    // in flight still read into a fresh slot (copy on write) instead of waiting for them.
    int64_t n_cow = 0;
    void *master = nullptr;
    uint8_t *mask = nullptr;
    // Two node tables: renders read `table` (version `version`); an upload writes the other
    // one (a copy of the current one plus its changes), then the two swap and the version
    // grows.  Renders of older versions must end before a table or slot they read is reused.
    DevCell *table = nullptr;
    DevCell *table_alt = nullptr;
    int64_t version = 0;
    std::vector<std::pair<int32_t, int64_t>> deferred;   // (slot, first version without it)
    uint8_t *pool = nullptr;
    float *slot_range = nullptr;
    void *ins_stage = nullptr;   // device staging for host-pointer inserts
    size_t ins_stage_cap = 0;
    hipEvent_t ins_ev = nullptr;
    // cross-stream order: end of the last insert's kernels / of the last upload's device work
    hipEvent_t ev_insert = nullptr;
    hipEvent_t ev_upload = nullptr;
    // a render's view upload, tables and tile-group order run on this internal stream (default
    // priority), so they overlap the previous render; the render waits for their event
    hipStream_t prep = nullptr;
    Stage up;                    // upload: cell list / stats / deltas / jobs
    // rs[0 .. kRenderSlots) serve render_views and render_views_backward in turn;
    // rs[kRenderSlots] is render_views_noalloc's (host records allocated at creation)
    RenderSlot rs[kRenderSlots + 1];
    int next_rs = 0;
    void *scratch_dev = nullptr;     // this device's copy of `scratch`
    hipEvent_t na_copy = nullptr;    // end of the last noalloc call's record copy
    CkptRec ckpt_log[kCkptLog];
    int ckpt_next = 0;
    bool ktime = false;          // octree_render_timing: record the render kernels
    double ktime_ms = 0.0;
    uint64_t ktime_n = 0;
    // octree_build_timing: HIP events around the build kernels of each phase (insert,
    // downsample, statistics, gather) with the algorithmic bytes of each timed launch group
    bool btime = false;
    struct BuildTimed {
        int phase;
        hipEvent_t e0, e1;
        double bytes;
    };
    std::vector<BuildTimed> btimed;
    std::vector<hipEvent_t> bt_free;
    double bt_ms[4] = {0, 0, 0, 0}, bt_bytes[4] = {0, 0, 0, 0};
    void *bw_tmp = nullptr;      // adjoint: table-gradient accumulators (MIP views)
    size_t bw_tmp_cap = 0;
    float *vg_blk = nullptr;     // adjoint: blocked voxel-gradient scratch
    size_t vg_blk_cap = 0;
    // paging (capped pool): render flags per cell, missing-brick value bounds, LRU stamps
    bool capped = false;
    bool master_host = false;
    void *master_alloc = nullptr;  // host allocation when the master (or its host frames) lives in pinned memory
    // disk tier: page file with its RAM frames (master_alloc), the device page table (master)
    // and its pinned mirror, and the build-kernel batches in flight (sequence number, end
    // event) that the frames' pinning waits for
    PageCache *pc = nullptr;
    uint8_t *frames_dev = nullptr;   // the frames as the kernels address them
    bool frames_own = false;         // frames_dev is a device allocation (device frames)
    uint8_t *pg_stage = nullptr;     // device frames: pinned staging page for the file I/O
    hipStream_t pg_copy = nullptr;   // device frames: stream of the page copies and fills
    void **ptab_host = nullptr;
    hipEvent_t ptab_ev = nullptr;
    uint64_t pg_seq = 0;
    std::deque<std::pair<uint64_t, hipEvent_t>> pg_batches;
    std::vector<hipEvent_t> pg_free;
    uint8_t *flags = nullptr;
    uint8_t *flags_host = nullptr;
    float *miss_range = nullptr;
    uint64_t frame = 1;
    std::vector<uint64_t> last_used;
    // paging-only uploads (capped pool, no data changed since the last full upload, nothing
    // pending): which cells are brick nodes and which cell holds each slot, so that such an
    // upload touches the render flags, the resident slots and the cells it changes, not every
    // cell's host record
    bool paging_ready = false;
    std::vector<uint8_t> data_cell;
    std::vector<int64_t> slot_cell;
    uint64_t n_data = 0, n_resident = 0;
    // host brick store (host_bricks): one pinned entry per in-volume cell (channels unpadded),
    // mapped for the kernels; which entries hold their cell's current bordered brick; the
    // entries' value ranges on the device
    uint8_t *store = nullptr;
    uint8_t *store_dev = nullptr;
    uint64_t store_bytes = 0;
    std::vector<int32_t> store_idx;
    std::vector<uint8_t> store_ok;
    float *store_range = nullptr;
    std::vector<HCell> cells;
    std::vector<int32_t> free_slots;
    std::vector<std::vector<Box>> dirty;  // per level
    // transfer-function tables of recent views (control points -> table bytes)
    std::vector<std::pair<std::vector<float>, std::vector<uint8_t>>> table_cache;
    // tile-group dispatch orders of the last few ordered views (geometry key bytes -> order)
    std::vector<std::pair<std::vector<uint8_t>, std::vector<int32_t>>> order_cache;
    std::string err;
    float background_f = 0.0f;
};

static std::string g_create_err;

namespace {

int fail(oct_handle *h, int code, const std::string &msg)
{
    if (h) h->err = msg;
    else g_create_err = msg;
    return code;
}

#define HIPCHK(h, expr)                                                                     \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail((h), e_ == hipErrorOutOfMemory ? OCT_ENOMEM : OCT_EDEVICE,          \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                 \
    } while (0)

int64_t cell_index(const VolGeom &g, int L, int x, int y, int z)
{
    const int G = g.grid[L];
    return g.cell_off[L] + ((int64_t)z * G + y) * G + x;
}

// Calls may use different streams.  Device work is ordered as if every call had been issued
// on one stream in call order, with one relaxation: an upload's statistics pass (which reads
// only the mipmap) does not wait for renders issued before it, only its node-table and
// brick-pool writes do -- so the next batch's insertion and analysis overlap a render.
// Build timing: an event before a launch group (when enabled) and one after it, with the
// group's algorithmic bytes; summed when octree_build_timing is called.
hipEvent_t bt_event(oct_handle *h)
{
    if (!h->bt_free.empty()) {
        hipEvent_t e = h->bt_free.back();
        h->bt_free.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    return hipEventCreate(&e) == hipSuccess ? e : nullptr;
}

hipEvent_t bt_begin(oct_handle *h, hipStream_t s)
{
    if (!h->btime) return nullptr;
    hipEvent_t e = bt_event(h);
    if (e && hipEventRecord(e, s) != hipSuccess) return nullptr;
    return e;
}

void bt_end(oct_handle *h, hipEvent_t e0, hipStream_t s, int phase, double bytes)
{
    if (!e0) return;
    hipEvent_t e1 = bt_event(h);
    if (!e1 || hipEventRecord(e1, s) != hipSuccess) return;
    h->btimed.push_back({phase, e0, e1, bytes});
}

int wait_for(oct_handle *h, hipStream_t s, hipEvent_t ev)
{
    if (ev) HIPCHK(h, hipStreamWaitEvent(s, ev, 0));
    return OCT_OK;
}

// Adds a slot's recorded render-kernel time to the handle's totals (waits for it).
int collect_kernel_time(oct_handle *h, RenderSlot &r)
{
    if (!r.k_pending) return OCT_OK;
    HIPCHK(h, hipEventSynchronize(r.k1));
    float ms = 0.0f;
    HIPCHK(h, hipEventElapsedTime(&ms, r.k0, r.k1));
    h->ktime_ms += ms;
    h->ktime_n++;
    r.k_pending = false;
    return OCT_OK;
}

// A slot needs no wait when its last launch was on s itself (stream order; a stream is not
// destroyed while work on it is pending, so a later stream at the same address follows it) or
// has ended.  Each wait left out is a barrier the GPU does not process between launches.
static bool slot_pending_for(const RenderSlot &r, hipStream_t s)
{
    return r.st.ev && r.stream != s && hipEventQuery(r.st.ev) != hipSuccess;
}

int wait_for_renders(oct_handle *h, hipStream_t s)
{
    for (auto &r : h->rs)
        if (slot_pending_for(r, s)) HIPCHK(h, hipStreamWaitEvent(s, r.st.ev, 0));
    return OCT_OK;
}

// Device work on s after this call follows every render launch that read a node-table version
// below v.  A slot's earlier launches ended before it was reused (stage_reserve), so its last
// launch is the only one to wait for.
int wait_for_renders_before(oct_handle *h, hipStream_t s, int64_t v)
{
    for (auto &r : h->rs)
        if (r.version < v && slot_pending_for(r, s)) HIPCHK(h, hipStreamWaitEvent(s, r.st.ev, 0));
    return OCT_OK;
}

// Bytes of render_views_noalloc's host records (and of the same prefix of its scratch) for
// n views: the DevView records, the list of split views, the sample counters.
// Host records of a launch: views | split list, refinement list, per-view refinement wait
// counters | sample counters.
struct RecordLayout {
    size_t v_bytes, sv_off, sv_bytes, c_off, c_bytes;
    size_t rf_off, rw_off;   // offsets of the refinement list and wait counters
};
RecordLayout record_layout(size_t n_views, size_t n_split, size_t n_refine)
{
    RecordLayout l;
    l.v_bytes = n_views * sizeof(DevView);
    l.sv_off = (l.v_bytes + 255) & ~(size_t)255;
    l.rf_off = l.sv_off + n_split * sizeof(int32_t);
    l.rw_off = l.rf_off + n_refine * sizeof(int32_t);
    l.sv_bytes = (n_split + n_refine + n_views) * sizeof(int32_t);
    l.c_off = (l.sv_off + l.sv_bytes + 255) & ~(size_t)255;
    l.c_bytes = kCounterSlots * sizeof(RenderCounters);
    return l;
}

// Offset of the view tables behind a launch's host records (they are copied together).
size_t tables_offset(const RecordLayout &l) { return (l.c_off + l.c_bytes + 255) & ~(size_t)255; }

size_t noalloc_record_bytes()
{
    const RecordLayout l = record_layout(kNoAllocMaxViews, kNoAllocMaxViews, kNoAllocMaxViews);
    return ((tables_offset(l) + (size_t)kNoAllocMaxViews * view_tables_bytes(kMaxC) + 255) &
            ~(size_t)255) + (size_t)kNoAllocMaxOrder * 8;   // the order and its scratch
}

// Every view's transfer-function tables, built on the host into the launch's records.
// Every view's transfer-function tables, built on the host into the launch's records.  The
// tables depend only on the control points, so the last few distinct ones are kept (views of
// one request, or of one transfer function, share them); may_insert = false only looks up
// (the call allocates nothing then).
void fill_tables(oct_handle *h, const DevView *dvs, int n_views, uint8_t *dst, size_t tbytes,
                 bool may_insert)
{
    const int C = h->g.C;
    auto &cache = h->table_cache;
    for (int i = 0; i < n_views; i++) {
        uint8_t *t = dst + (size_t)i * tbytes;
        float key[kMaxC * 40];
        for (int c = 0; c < C; c++) {
            std::memcpy(key + c * 40, dvs[i].tf_pos[c], 8 * sizeof(float));
            std::memcpy(key + c * 40 + 8, dvs[i].tf_rgba[c], 32 * sizeof(float));
        }
        const size_t kb = (size_t)C * 40 * sizeof(float);
        bool hit = false;
        for (size_t e = 0; e < cache.size() && !hit; e++)
            if (!std::memcmp(cache[e].first.data(), key, kb)) {
                std::memcpy(t, cache[e].second.data(), tbytes);
                hit = true;
            }
        if (hit) continue;
        switch (C) {
        case 1: host_build_tables<1>(dvs[i], *(ViewTables<1> *)t); break;
        case 2: host_build_tables<2>(dvs[i], *(ViewTables<2> *)t); break;
        case 3: host_build_tables<3>(dvs[i], *(ViewTables<3> *)t); break;
        default: host_build_tables<4>(dvs[i], *(ViewTables<4> *)t); break;
        }
        if (may_insert) {
            if (cache.size() >= 64) cache.erase(cache.begin());
            cache.emplace_back(std::vector<float>(key, key + C * 40), std::vector<uint8_t>(t, t + tbytes));
        }
    }
}

// Views whose tile groups are dispatched longest first: the whole image of a launch's only
// view, when it has more than 1024 groups (above 512x512 pixels) -- there the longest rays set
// the launch's duration; smaller launches end soon either way.  Launches of several views or
// tile ranges (a serving mix) keep index order: they overlap other launches, which fill their
// tails.
bool view_ordered(const DevView &v, int n_views)
{
    const int tiles = v.tiles_x * ((v.height + OCT_TILE - 1) / OCT_TILE);
    return n_views == 1 && v.tile_begin == 0 && v.tile_end == tiles && v.groups > 1024;
}

// Dispatch order of a view's tile groups (read by item_of): groups sorted by the length, inside
// the volume box and the clip half-spaces, of the longest of their tile-centre rays (one ray
// per group above 4096 groups), longest first, in 32 length classes.  A stable counting sort
// keeps index order inside a class, so neighbouring groups of one class stay neighbours in the
// dispatch.  The order changes no result: every pixel depends only on its own ray.  `work`
// holds V.groups ints of scratch (lengths, then classes).
void build_group_order(const VolGeom &g, const DevView &V, int32_t *order, int32_t *work)
{
    constexpr int kCls = 32;
    const int G = V.groups;
    const int rays = G > 4096 ? 1 : kRenderTilesPerWg;
    float *len = (float *)work;
    float lmax = 0.0f;
    for (int gi = 0; gi < G; gi++) {
        float best = 0.0f;
        for (int q = 0; q < rays; q++) {
            const int t = std::min(group_tile(V, gi, rays == 1 ? 1 : q), V.tile_end - 1);
            const int px = std::min((t % V.tiles_x) * 8 + 4, V.width - 1);
            const int py = std::min((t / V.tiles_x) * 8 + 4, V.height - 1);
            const float sx = ((float)(2 * px + 1) / (float)V.width - 1.0f) * V.kx;
            const float sy = (1.0f - (float)(2 * py + 1) / (float)V.height) * V.ky;
            float d[3];
            for (int k = 0; k < 3; k++) d[k] = V.f[k] + sx * V.r[k] + sy * V.u[k];
            const float inv = 1.0f / std::sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            float t0 = 0.0f, t1 = INFINITY;
            for (int k = 0; k < 3; k++) {
                d[k] *= inv;
                const float o = V.eye[k];
                if (d[k] == 0.0f) {
                    if (o < 0.0f || o > (float)g.dims[k]) t1 = -1.0f;
                    continue;
                }
                const float ta = -o / d[k], tb = ((float)g.dims[k] - o) / d[k];
                t0 = std::max(t0, std::min(ta, tb));
                t1 = std::min(t1, std::max(ta, tb));
            }
            for (int c = 0; c < V.n_clip; c++) {
                const float *pl = V.clip[c];
                const float nd = pl[0] * d[0] + pl[1] * d[1] + pl[2] * d[2];
                const float no = pl[0] * V.eye[0] + pl[1] * V.eye[1] + pl[2] * V.eye[2];
                if (nd > 0.0f) t0 = std::max(t0, (pl[3] - no) / nd);
                else if (nd < 0.0f) t1 = std::min(t1, (pl[3] - no) / nd);
                else if (no < pl[3]) t1 = -1.0f;
            }
            best = std::max(best, t1 - t0);
        }
        len[gi] = best;
        lmax = std::max(lmax, best);
    }
    const float scale = lmax > 0.0f ? (float)kCls / lmax : 0.0f;
    int32_t *cls = work;   // replaces the lengths, entry by entry
    int start[kCls + 1] = {0};
    for (int gi = 0; gi < G; gi++) {   // class 0: the longest rays
        const int k = std::min(std::max((int)(len[gi] * scale), 0), kCls - 1);
        cls[gi] = kCls - 1 - k;
        start[cls[gi] + 1]++;
    }
    for (int c = 0; c < kCls; c++) start[c + 1] += start[c];
    for (int gi = 0; gi < G; gi++) order[start[cls[gi]]++] = gi;
}

// The geometry a group order depends on: a view repeated across launches (a stream of frames
// of one camera) reuses its order.
struct OrderKey {
    float eye[3], f[3], r[3], u[3], kx, ky;
    int32_t width, height, tiles_x, tile_begin, tile_end, groups, n_clip;
    float clip[3][4];
    int32_t dims[3];
};

OrderKey order_key(const VolGeom &g, const DevView &v)
{
    OrderKey k;
    std::memset(&k, 0, sizeof(k));
    for (int a = 0; a < 3; a++) {
        k.eye[a] = v.eye[a];
        k.f[a] = v.f[a];
        k.r[a] = v.r[a];
        k.u[a] = v.u[a];
        k.dims[a] = g.dims[a];
    }
    k.kx = v.kx;
    k.ky = v.ky;
    k.width = v.width;
    k.height = v.height;
    k.tiles_x = v.tiles_x;
    k.tile_begin = v.tile_begin;
    k.tile_end = v.tile_end;
    k.groups = v.groups;
    k.n_clip = v.n_clip;
    for (int c = 0; c < v.n_clip; c++)
        for (int q = 0; q < 4; q++) k.clip[c][q] = v.clip[c][q];
    return k;
}

// The group order of view v (from the cache when its geometry was ordered recently).
const std::vector<int32_t> &cached_group_order(oct_handle *h, const DevView &v)
{
    const OrderKey k = order_key(h->g, v);
    const uint8_t *kb = (const uint8_t *)&k;
    auto &cache = h->order_cache;
    for (size_t i = 0; i < cache.size(); i++)
        if (cache[i].first.size() == sizeof(k) && !std::memcmp(cache[i].first.data(), kb, sizeof(k))) {
            if (i) std::rotate(cache.begin(), cache.begin() + (std::ptrdiff_t)i, cache.begin() + (std::ptrdiff_t)i + 1);
            return cache[0].second;
        }
    std::vector<int32_t> ord((size_t)v.groups), work((size_t)v.groups);
    build_group_order(h->g, v, ord.data(), work.data());
    cache.insert(cache.begin(), {std::vector<uint8_t>(kb, kb + sizeof(k)), std::move(ord)});
    if (cache.size() > 4) cache.pop_back();
    return cache[0].second;
}

// Address of `scratch` on device `dev` (the current device), looked up once per device.
int scratch_for_device(int dev, void **out)
{
    static std::mutex mu;
    static void *addr[64] = {};
    if (dev < 0 || dev >= 64) return OCT_EDEVICE;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return OCT_EDEVICE;
        addr[dev] = p;
    }
    *out = addr[dev];
    return OCT_OK;
}

// FNV-1a over the bytes of a view list (oct_view has no padding: 4-byte fields only).
uint64_t views_hash(int32_t n_views, const oct_view *views)
{
    uint64_t x = 1469598103934665603ull;
    const uint8_t *b = (const uint8_t *)views;
    for (size_t i = 0; i < (size_t)n_views * sizeof(oct_view); i++) x = (x ^ b[i]) * 1099511628211ull;
    return x;
}

// Records that `ws` now holds the checkpoints of these views at the current table version.
void ckpt_log_put(oct_handle *h, const void *ws, int32_t n_views, const oct_view *views)
{
    CkptRec *r = nullptr;
    for (auto &e : h->ckpt_log)
        if (e.ws == ws) r = &e;
    if (!r) {
        r = &h->ckpt_log[h->ckpt_next];
        h->ckpt_next = (h->ckpt_next + 1) % kCkptLog;
    }
    r->ws = ws;
    r->version = h->version;
    r->views_hash = views_hash(n_views, views);
    r->n_views = n_views;
}

int stage_reserve(oct_handle *h, Stage &s, size_t bytes)
{
    if (s.ev) HIPCHK(h, hipEventSynchronize(s.ev));
    if (bytes <= s.cap) return OCT_OK;
    size_t cap = std::max<size_t>(bytes, 2 * s.cap);
    cap = std::max<size_t>(cap, 4096);
    if (s.host) HIPCHK(h, hipHostFree(s.host));
    if (s.dev) HIPCHK(h, hipFree(s.dev));
    s.host = nullptr;
    s.dev = nullptr;
    s.cap = 0;
    HIPCHK(h, hipHostMalloc(&s.host, cap, hipHostMallocDefault));
    HIPCHK(h, hipMalloc(&s.dev, cap));
    s.cap = cap;
    if (!s.ev) HIPCHK(h, hipEventCreateWithFlags(&s.ev, hipEventDisableTiming));
    return OCT_OK;
}

void stage_free(Stage &s)
{
    if (s.host) (void)hipHostFree(s.host);
    if (s.dev) (void)hipFree(s.dev);
    if (s.ev) (void)hipEventDestroy(s.ev);
    s = Stage{};
}

bool valid_params(const oct_create_params *p, std::string &why)
{
    for (int a = 0; a < 3; a++)
        if (p->dims[a] < 1 || p->dims[a] > (1 << 20)) { why = "dims out of range"; return false; }
    if (p->channels < 1 || p->channels > OCT_MAX_CHANNELS) { why = "channels must be 1..4"; return false; }
    if (p->brick_size < 2 || p->brick_size > 128 || (p->brick_size & 1)) {
        why = "brick_size must be even, 2..128";
        return false;
    }
    if (p->dtype != OCT_U16 && p->dtype != OCT_F32) { why = "dtype must be OCT_U16 or OCT_F32"; return false; }
    if (!std::isfinite(p->background) || !std::isfinite(p->homog_threshold) || p->homog_threshold < 0) {
        why = "background / threshold must be finite, threshold >= 0";
        return false;
    }
    if (p->dtype == OCT_U16 &&
        (p->background < 0 || p->background > 65535 || p->background != std::floor(p->background))) {
        why = "u16 background must be an integer in [0, 65535]";
        return false;
    }
    if (p->disk_frames != OCT_FRAMES_HOST && p->disk_frames != OCT_FRAMES_DEVICE) {
        why = "disk_frames must be OCT_FRAMES_HOST or OCT_FRAMES_DEVICE";
        return false;
    }
    if (p->host_bricks != 0 && p->host_bricks != 1) { why = "host_bricks must be 0 or 1"; return false; }
    if (p->host_bricks && !p->device_pool_bytes) {
        why = "host_bricks needs a capped device pool (device_pool_bytes)";
        return false;
    }
    if (p->master_on_host < OCT_MASTER_HBM || p->master_on_host > OCT_MASTER_DISK) {
        why = "master_on_host must be OCT_MASTER_HBM, _HOST or _DISK";
        return false;
    }
    if (p->master_on_host == OCT_MASTER_DISK) {
        const int pc = p->page_cells ? p->page_cells : 2;
        if (p->brick_size & (p->brick_size - 1)) {
            why = "the disk tier needs brick_size a power of two";
            return false;
        }
        if (pc < 2 || (pc & (pc - 1)) || (int64_t)pc * p->brick_size > 1024) {
            why = "page_cells must be a power of two >= 2 (at most 1024 voxels per page edge)";
            return false;
        }
        if (!p->disk_path || !p->disk_path[0]) {
            why = "the disk tier needs disk_path";
            return false;
        }
    } else if (p->page_cells || p->host_cache_bytes || p->disk_path || p->disk_frames) {
        why = "page_cells, host_cache_bytes, disk_path and disk_frames belong to the disk tier";
        return false;
    }
    return true;
}

void reset_host_state(oct_handle *h)
{
    const VolGeom &g = h->g;
    const int C = g.C;
    h->paging_ready = false;
    std::fill(h->store_ok.begin(), h->store_ok.end(), 0);
    for (auto &c : h->cells) c = HCell();
    for (int L = 0; L <= g.N; L++) {
        const int G = g.grid[L];
        for (int z = 0; z < G; z++)
            for (int y = 0; y < G; y++)
                for (int x = 0; x < G; x++) {
                    HCell &c = h->cells[cell_index(g, L, x, y, z)];
                    const int b[3] = {x, y, z};
                    uint64_t cnt = 1, n0 = 1;
                    for (int a = 0; a < 3; a++) {
                        const int64_t lo = (int64_t)b[a] * g.M;
                        const int64_t n = std::max<int64_t>(0, std::min<int64_t>(g.M, g.ext[L][a] - lo));
                        cnt *= (uint64_t)n;
                        const int64_t span = (int64_t)g.M << L;
                        const int64_t lo0 = (int64_t)b[a] * span;
                        const int64_t n0a = std::max<int64_t>(0, std::min<int64_t>(span, g.dims[a] - lo0));
                        n0 *= (uint64_t)n0a;
                    }
                    c.count = cnt;
                    c.nvalid0 = n0;
                    c.inside = cnt > 0;
                    for (int k = 0; k < C; k++) c.avg[k] = h->p.dtype == OCT_U16 ? h->p.background
                                                                                 : (double)h->background_f;
                }
    }
    h->cells[cell_index(g, g.N, 0, 0, 0)].exists = 1;
    h->cells[cell_index(g, g.N, 0, 0, 0)].state = kEmpty;
    h->free_slots.clear();
    for (int64_t s = h->n_slots + h->n_cow - 1; s >= 0; s--) h->free_slots.push_back((int32_t)s);
    h->deferred.clear();
    for (auto &d : h->dirty) d.clear();
}

// Full node table upload (creation / clear): every cell resolves to the background AVG.
int upload_full_table(oct_handle *h, hipStream_t s)
{
    const size_t bytes = sizeof(DevCell) * (size_t)h->n_cells;
    int rc = stage_reserve(h, h->up, bytes);
    if (rc) return rc;
    DevCell *t = (DevCell *)h->up.host;
    for (int64_t i = 0; i < h->n_cells; i++) {
        DevCell &c = t[i];
        std::memset(&c, 0, sizeof c);
        c.kind = kAvg;
        c.slot = -1;
        for (int k = 0; k < 4; k++) c.avg[k] = c.lo[k] = c.hi[k] = k < h->g.C ? h->background_f : 0.0f;
        HCell &hc = h->cells[i];
        hc.dev_kind = kAvg;
        hc.dev_slot = -1;
        for (int k = 0; k < 4; k++) hc.dev_avg[k] = c.avg[k];
        hc.dev_valid = true;
    }
    HIPCHK(h, hipMemcpyAsync(h->table, t, bytes, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipEventRecord(h->up.ev, s));
    return OCT_OK;
}

// ------------------------------------------------------------------ tree states
// Recompute every node's state from the cell statistics (top-down, as the oracle defines):
// populated / complete from the insertion counts, subtree min/max bottom-up, then the first
// complete node whose subtree is homogeneous in every channel becomes a leaf; otherwise a
// complete node with a homogeneous brick keeps its children; otherwise it holds a brick.
void recompute_states(oct_handle *h)
{
    const VolGeom &g = h->g;
    const int C = g.C;
    const double thr = h->p.homog_threshold;
    // bottom-up aggregates
    for (int L = 0; L <= g.N; L++) {
        const int G = g.grid[L];
        for (int z = 0; z < G; z++)
            for (int y = 0; y < G; y++)
                for (int x = 0; x < G; x++) {
                    HCell &c = h->cells[cell_index(g, L, x, y, z)];
                    if (!c.inside) continue;
                    if (L == 0) {
                        for (int k = 0; k < C; k++) {
                            c.smin[k] = c.bmin[k];
                            c.smax[k] = c.bmax[k];
                        }
                        continue;
                    }
                    bool first = true;
                    for (int k = 0; k < C; k++) c.ins[k] = 0;
                    for (int d = 0; d < 8; d++) {
                        const int cx = 2 * x + (d & 1), cy = 2 * y + ((d >> 1) & 1), cz = 2 * z + (d >> 2);
                        const HCell &ch = h->cells[cell_index(g, L - 1, cx, cy, cz)];
                        if (!ch.inside) continue;
                        for (int k = 0; k < C; k++) {
                            c.ins[k] += ch.ins[k];
                            c.smin[k] = first ? ch.smin[k] : std::min(c.smin[k], ch.smin[k]);
                            c.smax[k] = first ? ch.smax[k] : std::max(c.smax[k], ch.smax[k]);
                        }
                        first = false;
                    }
                }
    }
    // top-down states
    for (int L = g.N; L >= 0; L--) {
        const int G = g.grid[L];
        for (int z = 0; z < G; z++)
            for (int y = 0; y < G; y++)
                for (int x = 0; x < G; x++) {
                    HCell &c = h->cells[cell_index(g, L, x, y, z)];
                    const bool exists =
                        L == g.N ? true : h->cells[cell_index(g, L + 1, x / 2, y / 2, z / 2)].has_children;
                    c.exists = exists;
                    c.has_children = 0;
                    c.state = kNone;
                    bool any = false, all = c.inside;
                    for (int k = 0; k < C; k++) {
                        if (c.ins[k] > 0) any = true;
                        if (c.ins[k] != c.nvalid0) all = false;
                    }
                    c.populated = c.inside && any;
                    c.complete = c.inside && all;
                    if (!exists) continue;
                    if (!c.populated) {
                        c.state = kEmpty;
                        for (int k = 0; k < C; k++)
                            c.avg[k] = h->p.dtype == OCT_U16 ? h->p.background : (double)h->background_f;
                        continue;
                    }
                    for (int k = 0; k < C; k++) {
                        if (h->p.dtype == OCT_U16) {
                            const uint64_t s = (uint64_t)c.bsum[k];
                            c.avg[k] = (double)((2 * s + c.count) / (2 * c.count));
                        } else {
                            c.avg[k] = (double)(float)(c.bsum[k] / (double)c.count);
                        }
                    }
                    bool sub_h = c.complete, own_h = c.complete;
                    for (int k = 0; k < C; k++) {
                        if (!(c.smax[k] - c.smin[k] < thr)) sub_h = false;
                        if (!(c.bmax[k] - c.bmin[k] < thr)) own_h = false;
                    }
                    if (sub_h) {
                        c.state = kHomogLeaf;
                    } else {
                        c.has_children = L > 0;
                        c.state = own_h ? kHomog : kBrickState;
                    }
                }
    }
}

bool box_intersects(const Box &b, const int lo[3], const int hi[3])
{
    for (int a = 0; a < 3; a++)
        if (b.hi[a] < lo[a] || b.lo[a] > hi[a]) return false;
    return true;
}

// ------------------------------------------------------------------- disk tier
// Build kernels of the disk tier run in batches: a batch's pages are made resident (loaded,
// filled, or already in RAM), written into the device page table, and pinned until the batch's
// end event, which later evictions of their frames wait for.

// End of every batch up to `seq` (blocking) / without blocking, whether they have ended.
void pg_wait(oct_handle *h, uint64_t seq)
{
    while (!h->pg_batches.empty() && h->pg_batches.front().first <= seq) {
        (void)hipEventSynchronize(h->pg_batches.front().second);
        h->pg_free.push_back(h->pg_batches.front().second);
        h->pg_batches.pop_front();
    }
}

bool pg_done(oct_handle *h, uint64_t seq)
{
    while (!h->pg_batches.empty() && h->pg_batches.front().first <= seq &&
           hipEventQuery(h->pg_batches.front().second) == hipSuccess) {
        h->pg_free.push_back(h->pg_batches.front().second);
        h->pg_batches.pop_front();
    }
    return h->pg_batches.empty() || h->pg_batches.front().first > seq;
}

// Pages a batch may hold: half the frames, so that a batch finds frames whose previous batch
// has ended while the one before it still runs (at least the 9 of one downsample step).
int64_t pg_budget(const oct_handle *h) { return std::max<int64_t>(9, h->pc->n_frames() / 2); }

// Page range along each axis of level L's voxel box lo..hi (clamped to the level); false when
// the box is empty.
bool page_range(const VolGeom &g, int L, const int lo[3], const int hi[3], int a0[3], int a1[3])
{
    for (int a = 0; a < 3; a++) {
        const int l = std::max(lo[a], 0), u = std::min(hi[a], g.ext[L][a] - 1);
        if (u < l) return false;
        a0[a] = l >> g.plog;
        a1[a] = u >> g.plog;
    }
    return true;
}

int64_t count_box_pages(const VolGeom &g, int L, const int lo[3], const int hi[3])
{
    int a0[3], a1[3];
    if (!page_range(g, L, lo, hi, a0, a1)) return 0;
    return (int64_t)(a1[0] - a0[0] + 1) * (a1[1] - a0[1] + 1) * (a1[2] - a0[2] + 1);
}

void add_box_pages(const VolGeom &g, int L, const int lo[3], const int hi[3], uint8_t write,
                   std::vector<int64_t> &pages, std::vector<uint8_t> &writes)
{
    int a0[3], a1[3];
    if (!page_range(g, L, lo, hi, a0, a1)) return;
    for (int z = a0[2]; z <= a1[2]; z++)
        for (int y = a0[1]; y <= a1[1]; y++)
            for (int x = a0[0]; x <= a1[0]; x++) {
                pages.push_back(g.page_off[L] + ((int64_t)z * g.pgrid[L][1] + y) * g.pgrid[L][0] + x);
                writes.push_back(write);
            }
}

// Runs launch() as one batch on stream s with `pages` resident and mapped (writes[i]: the
// batch modifies pages[i]).
template <typename F>
int paged_batch(oct_handle *h, std::vector<int64_t> &pages, std::vector<uint8_t> &writes,
                hipStream_t s, F &&launch)
{
    if (pages.empty()) return launch();
    // distinct pages, a page written if any of its entries is
    std::vector<std::pair<int64_t, uint8_t>> pw(pages.size());
    for (size_t i = 0; i < pages.size(); i++) pw[i] = {pages[i], writes[i]};
    std::sort(pw.begin(), pw.end());
    pages.clear();
    writes.clear();
    for (const auto &e : pw) {
        if (!pages.empty() && pages.back() == e.first) writes.back() |= e.second;
        else {
            pages.push_back(e.first);
            writes.push_back(e.second);
        }
    }
    const uint64_t seq = ++h->pg_seq;
    std::string err;
    const int r = h->pc->acquire(pages.data(), (int)pages.size(), writes.data(), seq,
                                 [h](uint64_t q) { pg_wait(h, q); },
                                 [h](uint64_t q) { return pg_done(h, q); }, err);
    if (r == -1) return fail(h, OCT_ENOMEM, err);
    if (r < 0) return fail(h, OCT_EDEVICE, err);
    // the page table's entries for this batch; the mirror's previous copy must have been read
    HIPCHK(h, hipEventSynchronize(h->ptab_ev));
    for (int64_t p : pages)
        h->ptab_host[p] = h->frames_dev + (size_t)h->pc->frame_of(p) * h->pc->page_bytes();
    const int64_t lo = pages.front(), n = pages.back() - pages.front() + 1;
    HIPCHK(h, hipMemcpyAsync((void **)h->master + lo, h->ptab_host + lo, (size_t)n * sizeof(void *),
                             hipMemcpyHostToDevice, s));
    HIPCHK(h, hipEventRecord(h->ptab_ev, s));
    const int rc = launch();
    if (rc) return rc;
    hipEvent_t ev;
    if (!h->pg_free.empty()) {
        ev = h->pg_free.back();
        h->pg_free.pop_back();
    } else {
        HIPCHK(h, hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    }
    HIPCHK(h, hipEventRecord(ev, s));
    h->pg_batches.push_back({seq, ev});
    return OCT_OK;
}

// Bordered-brick gathers of jobs[j0 .. j1) (jobs_dev: the same jobs on the device) in runs
// whose source pages fit a batch.
int gather_paged(oct_handle *h, const std::vector<BrickJob> &jobs, int j0, int j1,
                 const BrickJob *jobs_dev, const DevCell *table, void *scratch, hipStream_t s)
{
    const VolGeom &g = h->g;
    const int M = g.M;
    const int64_t budget = pg_budget(h);
    for (int i0 = j0; i0 < j1;) {
        std::vector<int64_t> pages;
        std::vector<uint8_t> wr;
        int i1 = i0;
        for (; i1 < j1; i1++) {
            const BrickJob &jb = jobs[(size_t)i1];
            const int L = jb.level, G = g.grid[L];
            const int b[3] = {jb.bx, jb.by, jb.bz};
            // the kernel reads the mipmap only inside neighbours drawn from it (not AVG cells):
            // per axis, the clamped source indices of the job's sub-box split by neighbour
            // (o = 0: below the cell, 1: inside, 2: above)
            int rlo[3][3], rhi[3][3];
            for (int a = 0; a < 3; a++) {
                const int e = g.ext[L][a];
                const int glo = std::min(std::max(b[a] * M - 1 + jb.lo[a], 0), e - 1);
                const int ghi = std::min(std::max(b[a] * M - 1 + jb.hi[a], 0), e - 1);
                rlo[a][0] = glo;
                rhi[a][0] = std::min(ghi, b[a] * M - 1);
                rlo[a][1] = std::max(glo, b[a] * M);
                rhi[a][1] = std::min(ghi, b[a] * M + M - 1);
                rlo[a][2] = std::max(glo, b[a] * M + M);
                rhi[a][2] = ghi;
            }
            std::vector<int64_t> cp;
            std::vector<uint8_t> cw;
            for (int oz = 0; oz < 3; oz++)
                for (int oy = 0; oy < 3; oy++)
                    for (int ox = 0; ox < 3; ox++) {
                        const int o[3] = {ox, oy, oz};
                        int lo[3], hi[3], nb[3];
                        bool ok = true;
                        for (int a = 0; a < 3; a++) {
                            lo[a] = rlo[a][o[a]];
                            hi[a] = rhi[a][o[a]];
                            nb[a] = b[a] + o[a] - 1;
                            ok = ok && lo[a] <= hi[a] && nb[a] >= 0 && nb[a] < G;
                        }
                        if (ok && h->cells[(size_t)cell_index(g, L, nb[0], nb[1], nb[2])].dev_kind != kAvg)
                            add_box_pages(g, L, lo, hi, 0, cp, cw);
                    }
            std::sort(cp.begin(), cp.end());
            cp.erase(std::unique(cp.begin(), cp.end()), cp.end());
            int fresh = 0;
            for (int64_t q : cp) fresh += std::find(pages.begin(), pages.end(), q) == pages.end();
            if (i1 > i0 && (int64_t)pages.size() + fresh > budget) break;
            for (int64_t q : cp)
                if (std::find(pages.begin(), pages.end(), q) == pages.end()) {
                    pages.push_back(q);
                    wr.push_back(0);
                }
        }
        const int a0 = i0, n = i1 - i0;
        const int rc = paged_batch(h, pages, wr, s, [&]() -> int {
            HIPCHK(h, launch_gather(g, h->master, table, h->pool, h->brick_bytes, jobs_dev + a0, n,
                                    h->slot_range, h->background_f, scratch, h->store_dev,
                                    h->store_range, h->store_bytes, s));
            return OCT_OK;
        });
        if (rc) return rc;
        i0 = i1;
    }
    return OCT_OK;
}

// Splits the box lo..hi of level Lt into sub-boxes along whole pages of Lt (z rows, then y
// rows, then x columns) such that pages_of(sub-box) <= budget where possible (a single page
// column is taken as it is), and calls f(sub_lo, sub_hi) for each, in order.
template <typename Count, typename F>
int split_by_pages(const VolGeom &g, const int lo[3], const int hi[3], int64_t budget,
                   Count &&pages_of, F &&f)
{
    const int P = 1 << g.plog;
    auto rec = [&](auto &&self, int axis, const int *blo, const int *bhi) -> int {
        if (axis < 0 || pages_of(blo, bhi) <= budget) return f(blo, bhi);
        // greedy runs of whole page rows along `axis`
        int r = blo[axis];
        while (r <= bhi[axis]) {
            int sl[3] = {blo[0], blo[1], blo[2]}, sh[3] = {bhi[0], bhi[1], bhi[2]};
            sl[axis] = r;
            sh[axis] = std::min(bhi[axis], (r / P) * P + P - 1);   // one page row
            while (sh[axis] < bhi[axis]) {
                int th[3] = {sh[0], sh[1], sh[2]};
                th[axis] = std::min(bhi[axis], sh[axis] + P);
                if (pages_of(sl, th) > budget) break;
                sh[axis] = th[axis];
            }
            const int rc = pages_of(sl, sh) <= budget ? f(sl, sh) : self(self, axis - 1, sl, sh);
            if (rc) return rc;
            r = sh[axis] + 1;
        }
        return OCT_OK;
    };
    return rec(rec, 2, lo, hi);
}

}  // namespace

// =================================================================== C ABI

extern "C" {

int octree_create(const oct_create_params *params, void *stream, oct_handle **out)
{
    if (!params || !out) return fail(nullptr, OCT_EINVAL, "null argument");
    std::string why;
    if (!valid_params(params, why)) return fail(nullptr, OCT_EINVAL, why);
    oct_handle *h = new (std::nothrow) oct_handle();
    if (!h) return fail(nullptr, OCT_ENOMEM, "host allocation failed");
    h->p = *params;
    hipStream_t s = (hipStream_t)stream;
    auto bail = [&](int code) {
        g_create_err = h->err;
        octree_destroy(h);
        return code;
    };
    if (hipGetDevice(&h->device) != hipSuccess) {
        h->err = "no HIP device";
        return bail(OCT_EDEVICE);
    }
    VolGeom &g = h->g;
    g.C = params->channels;
    g.M = params->brick_size;
    g.dtype = params->dtype;
    for (int a = 0; a < 3; a++) g.dims[a] = params->dims[a];
    const int dmax = std::max(g.dims[0], std::max(g.dims[1], g.dims[2]));
    int N = 0;
    while (((int64_t)g.M << N) < dmax) N++;
    if (N + 2 > kMaxLevels) {
        h->err = "too many levels";
        return bail(OCT_EINVAL);
    }
    g.N = N;
    g.mlog2 = -1;
    for (int b = 1; b < 8; b++)
        if (g.M == (1 << b)) g.mlog2 = b;
    h->esz = params->dtype == OCT_U16 ? 2 : 4;
    h->background_f = (float)params->background;
    int64_t off = 0, coff = 0;
    int64_t in_volume_cells = 0;
    for (int L = 0; L <= N; L++) {
        int64_t nv = g.C;
        for (int a = 0; a < 3; a++) {
            g.ext[L][a] = (int32_t)(((int64_t)g.dims[a] + ((int64_t)1 << L) - 1) >> L);
            nv *= g.ext[L][a];
        }
        g.lvl_off[L] = off;
        off += nv;
        g.grid[L] = 1 << (N - L);
        g.cell_off[L] = (int32_t)coff;
        coff += (int64_t)g.grid[L] * g.grid[L] * g.grid[L];
        int64_t nb = 1;
        for (int a = 0; a < 3; a++) nb *= (g.ext[L][a] + g.M - 1) / g.M;
        in_volume_cells += nb;
    }
    g.lvl_off[N + 1] = off;
    h->n_cells = coff;
    const int S = g.M + 2;
    h->brick_bytes = ((uint64_t)S * S * S * 4 * h->esz + 255) & ~(uint64_t)255;
    h->n_slots = in_volume_cells;
    if (params->device_pool_bytes) {
        h->n_slots = std::min<int64_t>(h->n_slots, (int64_t)(params->device_pool_bytes / h->brick_bytes));
        h->capped = h->n_slots < in_volume_cells;
    }
    if (h->n_slots < 1) {
        h->err = "device_pool_bytes holds no brick";
        return bail(OCT_EINVAL);
    }
    if (!h->capped) {
        // copy-on-write headroom: the bricks of two brick layers across the largest face of
        // every level (what one slab insert makes dirty)
        int64_t cow = 8;
        for (int L = 0; L <= N; L++) {
            int64_t nb[3];
            for (int a = 0; a < 3; a++) nb[a] = (g.ext[L][a] + g.M - 1) / g.M;
            cow += 2 * std::max({nb[0] * nb[1], nb[0] * nb[2], nb[1] * nb[2]});
        }
        h->n_cow = std::min<int64_t>(cow, h->n_slots);
    }
    h->master_host = params->master_on_host == OCT_MASTER_HOST;
    h->cells.assign((size_t)h->n_cells, HCell());
    h->dirty.assign((size_t)N + 1, std::vector<Box>());

    auto dev_alloc = [&](void **ptr, size_t bytes) -> int {
        hipError_t e = hipMalloc(ptr, std::max<size_t>(bytes, 256));
        if (e != hipSuccess) {
            h->err = std::string("hipMalloc: ") + hipGetErrorString(e);
            return e == hipErrorOutOfMemory ? OCT_ENOMEM : OCT_EDEVICE;
        }
        return OCT_OK;
    };
    int rc;
    if (params->master_on_host == OCT_MASTER_DISK) {
        // pages of P^3 voxels (P = M * page_cells) per level, all channels
        const int P = g.M * (params->page_cells ? params->page_cells : 2);
        while ((1 << g.plog) < P) g.plog++;
        int64_t np = 0;
        for (int L = 0; L <= N; L++) {
            int64_t n3[3];
            for (int a = 0; a < 3; a++) n3[a] = (g.ext[L][a] + P - 1) / P;
            g.pgrid[L][0] = (int32_t)n3[0];
            g.pgrid[L][1] = (int32_t)n3[1];
            g.page_off[L] = np;
            np += n3[0] * n3[1] * n3[2];
        }
        g.page_off[N + 1] = np;
        const size_t page_bytes = (size_t)P * P * P * (size_t)g.C * h->esz;
        const int64_t n_frames = std::min<int64_t>((int64_t)(params->host_cache_bytes / page_bytes), np);
        if (n_frames < std::min<int64_t>(16, np) || n_frames > INT32_MAX) {
            h->err = "host_cache_bytes must hold at least 16 pages of " + std::to_string(page_bytes) +
                     " bytes (or every page)";
            return bail(OCT_EINVAL);
        }
        // frames (pinned and mapped for the kernels, or device memory with a pinned staging
        // page and a copy stream), the device page table and its host mirror
        const bool dev_frames = params->disk_frames == OCT_FRAMES_DEVICE;
        hipError_t e = hipSuccess;
        if (dev_frames) {
            if ((rc = dev_alloc((void **)&h->frames_dev, (size_t)n_frames * page_bytes))) return bail(rc);
            h->frames_own = true;
            e = hipHostMalloc((void **)&h->pg_stage, page_bytes, hipHostMallocDefault);
            if (e == hipSuccess) e = hipStreamCreateWithFlags(&h->pg_copy, hipStreamNonBlocking);
        } else {
            e = hipHostMalloc(&h->master_alloc, (size_t)n_frames * page_bytes, hipHostMallocMapped);
            if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&h->frames_dev, h->master_alloc, 0);
        }
        if (e == hipSuccess) e = hipHostMalloc((void **)&h->ptab_host, (size_t)np * sizeof(void *), hipHostMallocDefault);
        if (e != hipSuccess) {
            h->err = std::string("disk tier frames: ") + hipGetErrorString(e);
            return bail(e == hipErrorOutOfMemory ? OCT_ENOMEM : OCT_EDEVICE);
        }
        std::memset(h->ptab_host, 0, (size_t)np * sizeof(void *));
        if ((rc = dev_alloc(&h->master, (size_t)np * sizeof(void *)))) return bail(rc);
        if (hipMemcpy(h->master, h->ptab_host, (size_t)np * sizeof(void *), hipMemcpyHostToDevice) != hipSuccess ||
            hipEventCreateWithFlags(&h->ptab_ev, hipEventDisableTiming) != hipSuccess)
            return bail(OCT_EDEVICE);
        const bool u16 = params->dtype == OCT_U16;
        const double bg = params->background;
        h->pc = new (std::nothrow) PageCache();
        if (!h->pc) return bail(OCT_ENOMEM);
        std::string perr;
        auto host_fill = [u16, bg, page_bytes](uint8_t *f) {
            if (u16) std::fill_n((uint16_t *)f, page_bytes / 2, (uint16_t)bg);
            else std::fill_n((float *)f, page_bytes / 4, (float)bg);
        };
        bool opened;
        if (dev_frames) {
            // each copy or fill has finished when the callback returns: a frame is only
            // touched here while no device work uses it (the cache waits for that first)
            PageCache::FrameIO io;
            io.staging = h->pg_stage;
            io.load = [h, page_bytes](int f, const uint8_t *src) {
                return hipMemcpyAsync(h->frames_dev + (size_t)f * page_bytes, src, page_bytes,
                                      hipMemcpyHostToDevice, h->pg_copy) == hipSuccess &&
                       hipStreamSynchronize(h->pg_copy) == hipSuccess;
            };
            io.store = [h, page_bytes](int f, uint8_t *dst) {
                return hipMemcpyAsync(dst, h->frames_dev + (size_t)f * page_bytes, page_bytes,
                                      hipMemcpyDeviceToHost, h->pg_copy) == hipSuccess &&
                       hipStreamSynchronize(h->pg_copy) == hipSuccess;
            };
            io.fill = [h, page_bytes, u16, bg](int f) {
                uint8_t *p = h->frames_dev + (size_t)f * page_bytes;
                const hipError_t fe =
                    u16 ? launch_fill_u16((uint16_t *)p, (int64_t)(page_bytes / 2), (uint16_t)bg, h->pg_copy)
                        : launch_fill_f32((float *)p, (int64_t)(page_bytes / 4), (float)bg, h->pg_copy);
                return fe == hipSuccess && hipStreamSynchronize(h->pg_copy) == hipSuccess;
            };
            opened = h->pc->open(params->disk_path, np, page_bytes, std::move(io), (int)n_frames,
                                 host_fill, perr);
        } else {
            opened = h->pc->open(params->disk_path, np, page_bytes, (uint8_t *)h->master_alloc,
                                 (int)n_frames, host_fill, perr);
        }
        if (!opened) {
            h->err = perr;
            return bail(OCT_EINVAL);
        }
    } else if (h->master_host) {
        // pinned host memory, mapped for the kernels (they read and write it over the link)
        hipError_t e = hipHostMalloc(&h->master_alloc, std::max<size_t>((size_t)off * h->esz, 256),
                                     hipHostMallocMapped);
        if (e == hipSuccess) e = hipHostGetDevicePointer(&h->master, h->master_alloc, 0);
        if (e != hipSuccess) {
            h->err = std::string("pinned master: ") + hipGetErrorString(e);
            return bail(e == hipErrorOutOfMemory ? OCT_ENOMEM : OCT_EDEVICE);
        }
    } else if ((rc = dev_alloc(&h->master, (size_t)off * h->esz))) {
        return bail(rc);
    }
    if ((rc = dev_alloc((void **)&h->mask, (size_t)g.dims[0] * g.dims[1] * g.dims[2]))) return bail(rc);
    if ((rc = dev_alloc((void **)&h->table, sizeof(DevCell) * (size_t)h->n_cells))) return bail(rc);
    if ((rc = dev_alloc((void **)&h->table_alt, sizeof(DevCell) * (size_t)h->n_cells))) return bail(rc);
    // one spare slot past the pool: canonical dumps gather non-resident bricks into it
    const size_t pool_slots = (size_t)(h->n_slots + h->n_cow + 1);
    if ((rc = dev_alloc((void **)&h->pool, (size_t)h->brick_bytes * pool_slots))) return bail(rc);
    if ((rc = dev_alloc((void **)&h->slot_range, sizeof(float) * 8 * pool_slots))) return bail(rc);
    if ((rc = dev_alloc((void **)&h->flags, (size_t)h->n_cells))) return bail(rc);
    if ((rc = dev_alloc((void **)&h->miss_range, sizeof(float) * 8 * (size_t)h->n_cells))) return bail(rc);
    if (hipHostMalloc((void **)&h->flags_host, (size_t)h->n_cells, hipHostMallocDefault) != hipSuccess)
        return bail(OCT_ENOMEM);
    if (params->host_bricks) {
        if (!h->capped) {
            h->err = "host_bricks needs a device pool smaller than the octree's bricks";
            return bail(OCT_EINVAL);
        }
        h->store_bytes = ((uint64_t)S * S * S * (uint64_t)g.C * h->esz + 255) & ~(uint64_t)255;
        h->store_idx.assign((size_t)h->n_cells, -1);
        int32_t ne = 0;
        for (int L = 0; L <= N; L++) {
            int nb[3];
            for (int a = 0; a < 3; a++) nb[a] = (g.ext[L][a] + g.M - 1) / g.M;
            const int G = g.grid[L];
            for (int z = 0; z < nb[2]; z++)
                for (int y = 0; y < nb[1]; y++)
                    for (int x = 0; x < nb[0]; x++)
                        h->store_idx[(size_t)(g.cell_off[L] + ((int64_t)z * G + y) * G + x)] = ne++;
        }
        h->store_ok.assign((size_t)ne, 0);
        hipError_t e = hipHostMalloc((void **)&h->store, (size_t)ne * h->store_bytes, hipHostMallocMapped);
        if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&h->store_dev, h->store, 0);
        if (e != hipSuccess) {
            h->err = std::string("host brick store: ") + hipGetErrorString(e);
            return bail(e == hipErrorOutOfMemory ? OCT_ENOMEM : OCT_EDEVICE);
        }
        if ((rc = dev_alloc((void **)&h->store_range, sizeof(float) * 8 * (size_t)ne))) return bail(rc);
    }
    h->last_used.assign((size_t)h->n_cells, 0);
    if (hipStreamCreateWithFlags(&h->prep, hipStreamNonBlocking) != hipSuccess) return bail(OCT_EDEVICE);
    if (hipEventCreateWithFlags(&h->ins_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_insert, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&h->ev_upload, hipEventDisableTiming) != hipSuccess)
        return bail(OCT_EDEVICE);
    // render_views_noalloc: this device's scratch address, pinned host records for the largest
    // call, and its events -- everything it needs, so that the call itself allocates nothing
    if (scratch_for_device(h->device, &h->scratch_dev) != OCT_OK) {
        h->err = "hipGetSymbolAddress(scratch) failed";
        return bail(OCT_EDEVICE);
    }
    {
        RenderSlot &na = h->rs[kRenderSlots];
        na.st.cap = noalloc_record_bytes();
        if (hipHostMalloc(&na.st.host, na.st.cap, hipHostMallocDefault) != hipSuccess)
            return bail(OCT_ENOMEM);
        if (hipEventCreateWithFlags(&na.st.ev, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&h->na_copy, hipEventDisableTiming) != hipSuccess)
            return bail(OCT_EDEVICE);
    }
    if (octree_clear(h, stream) != OCT_OK) return bail(OCT_EDEVICE);
    (void)s;
    *out = h;
    return OCT_OK;
}

int octree_destroy(oct_handle *h)
{
    if (!h) return OCT_EINVAL;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    if (h->pc) {
        pg_wait(h, UINT64_MAX);
        delete h->pc;   // removes the page file
    }
    if (h->p.master_on_host == OCT_MASTER_DISK) {
        for (hipEvent_t e : h->pg_free) (void)hipEventDestroy(e);
        if (h->ptab_ev) (void)hipEventDestroy(h->ptab_ev);
        if (h->ptab_host) (void)hipHostFree(h->ptab_host);
        if (h->master) (void)hipFree(h->master);   // the device page table
        if (h->master_alloc) (void)hipHostFree(h->master_alloc);
        if (h->frames_own) (void)hipFree(h->frames_dev);
        if (h->pg_stage) (void)hipHostFree(h->pg_stage);
        if (h->pg_copy) (void)hipStreamDestroy(h->pg_copy);
    } else if (h->master_alloc) {
        (void)hipHostFree(h->master_alloc);   // the pinned master (master is its device address)
    } else if (h->master) {
        (void)hipFree(h->master);
    }
    if (h->flags) (void)hipFree(h->flags);
    if (h->flags_host) (void)hipHostFree(h->flags_host);
    if (h->store) (void)hipHostFree(h->store);
    if (h->store_range) (void)hipFree(h->store_range);
    if (h->miss_range) (void)hipFree(h->miss_range);
    if (h->mask) (void)hipFree(h->mask);
    if (h->table) (void)hipFree(h->table);
    if (h->table_alt) (void)hipFree(h->table_alt);
    if (h->pool) (void)hipFree(h->pool);
    if (h->slot_range) (void)hipFree(h->slot_range);
    if (h->ins_stage) (void)hipFree(h->ins_stage);
    if (h->bw_tmp) (void)hipFree(h->bw_tmp);
    if (h->vg_blk) (void)hipFree(h->vg_blk);
    for (const auto &r : h->btimed) {
        (void)hipEventDestroy(r.e0);
        (void)hipEventDestroy(r.e1);
    }
    for (hipEvent_t e : h->bt_free) (void)hipEventDestroy(e);
    if (h->ins_ev) (void)hipEventDestroy(h->ins_ev);
    if (h->ev_insert) (void)hipEventDestroy(h->ev_insert);
    if (h->ev_upload) (void)hipEventDestroy(h->ev_upload);
    if (h->na_copy) (void)hipEventDestroy(h->na_copy);
    if (h->prep) (void)hipStreamDestroy(h->prep);
    stage_free(h->up);
    for (auto &r : h->rs) {
        stage_free(r.st);
        if (r.part) (void)hipFree(r.part);
        if (r.tmask) (void)hipFree(r.tmask);
        if (r.prep) (void)hipEventDestroy(r.prep);
        if (r.k0) (void)hipEventDestroy(r.k0);
        if (r.k1) (void)hipEventDestroy(r.k1);
    }
    delete h;
    return OCT_OK;
}

int octree_clear(oct_handle *h, void *stream)
{
    if (!h) return OCT_EINVAL;
    HIPCHK(h, hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    int rc = wait_for(h, s, h->ev_insert);
    if (!rc) rc = wait_for(h, s, h->ev_upload);
    if (!rc) rc = wait_for_renders(h, s);
    if (rc) return rc;
    if (h->pc) {
        // every page back to the background: the frames are dropped once the batches using
        // them have ended (the renders never read the master)
        pg_wait(h, UINT64_MAX);
        h->pc->reset([h](uint64_t q) { pg_wait(h, q); });
    }
    HIPCHK(h, launch_clear(h->g, h->master, h->mask, h->p.background, s));
    HIPCHK(h, launch_fill_u8(h->flags, h->n_cells, 0, s));
    HIPCHK(h, launch_fill_f32(h->miss_range, h->n_cells * 8, h->background_f, s));
    reset_host_state(h);
    std::fill(h->last_used.begin(), h->last_used.end(), 0);
    h->frame = 1;
    h->version++;   // every earlier launch is now behind the version of the cleared table
    rc = upload_full_table(h, s);
    if (rc) return rc;
    HIPCHK(h, hipEventRecord(h->ev_insert, s));
    HIPCHK(h, hipEventRecord(h->ev_upload, s));
    return OCT_OK;
}

int octree_insert_block(oct_handle *h, int32_t channel, const int32_t origin[3],
                        const int32_t size[3], const void *data, int32_t data_is_device,
                        void *stream)
{
    if (!h || !origin || !size || !data) return fail(h, OCT_EINVAL, "null argument");
    const VolGeom &g = h->g;
    if (channel < -1 || channel >= g.C) return fail(h, OCT_EINVAL, "channel out of range");
    for (int a = 0; a < 3; a++) {
        if (size[a] < 1) return fail(h, OCT_EINVAL, "block size must be >= 1");
        if (origin[a] < 0 || (int64_t)origin[a] + size[a] > g.dims[a])
            return fail(h, OCT_ERANGE, "block outside the volume");
    }
    HIPCHK(h, hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    const int cb = channel < 0 ? g.C : 1;
    const size_t bytes = (size_t)cb * size[0] * size[1] * size[2] * h->esz;
    const void *src = data;
    if (!data_is_device) {
        HIPCHK(h, hipEventSynchronize(h->ins_ev));
        if (bytes > h->ins_stage_cap) {
            if (h->ins_stage) HIPCHK(h, hipFree(h->ins_stage));
            h->ins_stage = nullptr;
            h->ins_stage_cap = 0;
            HIPCHK(h, hipMalloc(&h->ins_stage, bytes));
            h->ins_stage_cap = bytes;
        }
        HIPCHK(h, hipMemcpyAsync(h->ins_stage, data, bytes, hipMemcpyHostToDevice, s));
        HIPCHK(h, hipStreamSynchronize(s));  // host data consumed before return
        src = h->ins_stage;
    }
    int rc = wait_for(h, s, h->ev_insert);     // overlapping inserts, and the last upload's
    if (!rc) rc = wait_for(h, s, h->ev_upload);  // gathers (they read the mipmap)
    if (rc) return rc;
    {
        const double nvox = (double)size[0] * size[1] * size[2];
        hipEvent_t e0 = bt_begin(h, s);
        const int64_t sp[3] = {size[0], (int64_t)size[0] * size[1], (int64_t)size[0] * size[1] * size[2]};
        if (h->pc) {
            // disk tier: level-0 page rows of the block, a batch each (as many as fit)
            const int lo[3] = {origin[0], origin[1], origin[2]};
            const int hi[3] = {origin[0] + size[0] - 1, origin[1] + size[1] - 1, origin[2] + size[2] - 1};
            rc = split_by_pages(
                g, lo, hi, pg_budget(h),
                [&](const int *a, const int *b) { return count_box_pages(g, 0, a, b); },
                [&](const int *a, const int *b) -> int {
                    std::vector<int64_t> pages;
                    std::vector<uint8_t> wr;
                    add_box_pages(g, 0, a, b, 1, pages, wr);
                    return paged_batch(h, pages, wr, s, [&]() -> int {
                        const int32_t o2[3] = {a[0], a[1], a[2]};
                        const int32_t n2[3] = {b[0] - a[0] + 1, b[1] - a[1] + 1, b[2] - a[2] + 1};
                        const int64_t off = (a[2] - origin[2]) * sp[1] + (a[1] - origin[1]) * sp[0] +
                                            (a[0] - origin[0]);
                        HIPCHK(h, launch_insert(g, h->master, h->mask,
                                                (const uint8_t *)src + off * (int64_t)h->esz, sp,
                                                channel, o2, n2, s));
                        return OCT_OK;
                    });
                });
            if (rc) return rc;
        } else {
            HIPCHK(h, launch_insert(g, h->master, h->mask, src, sp, channel, origin, size, s));
        }
        // block read + level-0 write per channel, inserted-channel mask read and written
        bt_end(h, e0, s, 0, nvox * (2.0 * cb * (double)h->esz + 2.0));
    }
    hipEvent_t e_ds = bt_begin(h, s);
    double ds_bytes = 0.0;
    Box b;
    for (int a = 0; a < 3; a++) {
        b.lo[a] = origin[a];
        b.hi[a] = origin[a] + size[a] - 1;
    }
    h->dirty[0].push_back(b);
    for (int L = 0; L < g.N; L++) {
        Box p;
        for (int a = 0; a < 3; a++) {
            p.lo[a] = b.lo[a] >> 1;
            p.hi[a] = b.hi[a] >> 1;
        }
        if (h->pc) {
            // disk tier: parent page rows with their children's pages, a batch each.  The
            // pages are taken for the x range widened to groups of four parents (the unit of
            // the four-parent kernel; page edges are multiples of four, so a widened sub-box
            // stays in its pages).
            auto widen = [&](const int *a, const int *b, int wl[3], int wh[3], int cl[3], int ch[3]) {
                for (int q = 0; q < 3; q++) {
                    wl[q] = a[q];
                    wh[q] = b[q];
                }
                wl[0] &= ~3;
                wh[0] = std::min(wh[0] | 3, g.ext[L + 1][0] - 1);
                for (int q = 0; q < 3; q++) {
                    cl[q] = 2 * wl[q];
                    ch[q] = 2 * wh[q] + 1;
                }
            };
            const int lo[3] = {p.lo[0], p.lo[1], p.lo[2]}, hi[3] = {p.hi[0], p.hi[1], p.hi[2]};
            int rc2 = split_by_pages(
                g, lo, hi, pg_budget(h),
                [&](const int *a, const int *b) {
                    int wl[3], wh[3], cl[3], ch[3];
                    widen(a, b, wl, wh, cl, ch);
                    return count_box_pages(g, L + 1, wl, wh) + count_box_pages(g, L, cl, ch);
                },
                [&](const int *a, const int *b) -> int {
                    int wl[3], wh[3], cl[3], ch[3];
                    widen(a, b, wl, wh, cl, ch);
                    std::vector<int64_t> pages;
                    std::vector<uint8_t> wr;
                    add_box_pages(g, L + 1, wl, wh, 1, pages, wr);
                    add_box_pages(g, L, cl, ch, 0, pages, wr);
                    return paged_batch(h, pages, wr, s, [&]() -> int {
                        const int32_t sl[3] = {a[0], a[1], a[2]}, sh[3] = {b[0], b[1], b[2]};
                        HIPCHK(h, launch_downsample(g, h->master, L, sl, sh, s));
                        return OCT_OK;
                    });
                });
            if (rc2) return rc2;
        } else {
            HIPCHK(h, launch_downsample(g, h->master, L, p.lo, p.hi, s));
        }
        double parents = 1.0, children = 1.0;
        for (int a = 0; a < 3; a++) {
            parents *= (double)(p.hi[a] - p.lo[a] + 1);
            children *= (double)(std::min(2 * p.hi[a] + 1, g.ext[L][a] - 1) - 2 * p.lo[a] + 1);
        }
        ds_bytes += (double)g.C * (double)h->esz * (parents + children);
        h->dirty[L + 1].push_back(p);
        b = p;
    }
    bt_end(h, e_ds, s, 1, ds_bytes);
    if (!data_is_device) HIPCHK(h, hipEventRecord(h->ins_ev, s));
    HIPCHK(h, hipEventRecord(h->ev_insert, s));
    return OCT_OK;
}

int octree_insert_slices(oct_handle *h, int32_t channel, int32_t z0, int32_t nz, const void *data,
                         int32_t data_is_device, void *stream)
{
    if (!h) return OCT_EINVAL;
    const int32_t o[3] = {0, 0, z0};
    const int32_t n[3] = {h->g.dims[0], h->g.dims[1], nz};
    return octree_insert_block(h, channel, o, n, data, data_is_device, stream);
}

// Upload of a capped pool when no data changed since the last full upload and nothing is
// pending: only residency changes.  Requested brick nodes get slots (coarser levels first; free
// slots, then slots the last renders did not use, least recently used first, then a used finer
// brick's slot for a coarser request), exactly as a full upload decides, but touching only the
// render flags, the resident slots and the cells that change.
static int upload_paging_only(oct_handle *h, uint64_t byte_budget, hipStream_t s,
                              std::vector<CellDelta> &deltas, std::vector<BrickJob> &jobs,
                              std::vector<CopyJob> &copies, uint64_t &requests_seen,
                              uint64_t &evictions, uint64_t &unserved)
{
    const VolGeom &g = h->g;
    const int C = g.C;
    HIPCHK(h, hipMemcpyAsync(h->flags_host, h->flags, (size_t)h->n_cells, hipMemcpyDeviceToHost, s));
    HIPCHK(h, launch_fill_u8(h->flags, h->n_cells, 0, s));
    HIPCHK(h, hipStreamSynchronize(s));
    const uint8_t *fl = h->flags_host;
    auto level_of = [&](int64_t ci) {
        int L = 0;
        while (L < g.N && ci >= g.cell_off[L + 1]) L++;
        return L;
    };
    // one pass over the flags, levels from the root down and cells in index order (the full
    // upload's scan order, which the requests keep): the cells used now, and the requests
    std::vector<int64_t> reqs;
    for (int L = g.N; L >= 0; L--) {
        const int64_t n = (int64_t)g.grid[L] * g.grid[L] * g.grid[L];
        const int64_t end = g.cell_off[L] + n;
        for (int64_t ci = g.cell_off[L]; ci < end; ci++) {
            if ((ci & 7) == 0 && ci + 8 <= end) {   // most cells are unflagged: skip zero words
                uint64_t w;
                std::memcpy(&w, fl + ci, 8);
                if (!w) {
                    ci += 7;
                    continue;
                }
            }
            if (fl[ci] == 1) h->last_used[(size_t)ci] = h->frame;
            else if (fl[ci] == 2 && h->data_cell[(size_t)ci] && h->cells[(size_t)ci].slot < 0)
                reqs.push_back(ci);
        }
    }
    requests_seen = reqs.size();
    // resident cells as (last use, level, cell) keys: the full upload's victim orders made total
    // are (last use, level, scan position) for cells not used now and (level, scan position)
    // for the others; inside a level the scan position is the cell index
    struct VKey {
        uint64_t used;
        int32_t level;
        int64_t ci;
        bool operator<(const VKey &o) const
        {
            if (used != o.used) return used < o.used;
            return level != o.level ? level < o.level : ci < o.ci;
        }
    };
    std::vector<VKey> idle, busy;
    for (int64_t ci : h->slot_cell)
        if (ci >= 0) {
            const uint64_t u = h->last_used[(size_t)ci];
            if (u == h->frame) busy.push_back(VKey{0, level_of(ci), ci});
            else idle.push_back(VKey{u, level_of(ci), ci});
        }
    // at most one victim per request that the budget admits: order only those
    uint64_t budget_left = byte_budget ? byte_budget : UINT64_MAX;
    const size_t admit = std::min<uint64_t>(reqs.size(), budget_left / h->brick_bytes);
    const size_t n_idle = std::min(idle.size(), admit);
    std::partial_sort(idle.begin(), idle.begin() + n_idle, idle.end());
    const size_t n_busy = std::min(busy.size(), admit - n_idle);
    std::partial_sort(busy.begin(), busy.begin() + n_busy, busy.end());
    std::vector<int64_t> changed;
    size_t vi = 0, bi = 0;
    for (int64_t ci : reqs) {
        if (budget_left < h->brick_bytes) {
            unserved++;
            continue;
        }
        HCell &c = h->cells[(size_t)ci];
        const int L = level_of(ci);
        if (h->free_slots.empty()) {
            int64_t victim;
            if (vi < n_idle) victim = idle[vi++].ci;
            else if (bi < n_busy && busy[bi].level < L) victim = busy[bi++].ci;
            else {
                unserved++;
                continue;
            }
            HCell &v = h->cells[(size_t)victim];
            h->free_slots.push_back(v.slot);
            h->slot_cell[(size_t)v.slot] = -1;
            v.slot = -1;
            v.needs_gather = false;
            changed.push_back(victim);
            evictions++;
            h->n_resident--;
        }
        c.slot = h->free_slots.back();
        h->free_slots.pop_back();
        h->slot_cell[(size_t)c.slot] = ci;
        const int G = g.grid[L];
        const int64_t li = ci - g.cell_off[L];
        const int32_t e = h->store ? h->store_idx[(size_t)ci] : -1;
        if (e >= 0 && h->store_ok[(size_t)e]) {
            copies.push_back(CopyJob{c.slot, e});
        } else {
            BrickJob j{};
            j.slot = c.slot;
            j.level = L;
            j.bx = (int)(li % G);
            j.by = (int)((li / G) % G);
            j.bz = (int)(li / ((int64_t)G * G));
            j.full = 1;
            j.store = e;
            if (e >= 0) h->store_ok[(size_t)e] = 1;
            for (int a = 0; a < 3; a++) j.hi[a] = g.M + 1;
            jobs.push_back(j);
        }
        budget_left -= h->brick_bytes;
        c.needs_gather = false;
        changed.push_back(ci);
        h->n_resident++;
    }
    h->frame++;
    // change events of the cells that changed residency: a resident brick is drawn from its
    // slot (skip range = its AVG here, the brick's range comes from the gather); a missing one
    // from its AVG with the value bound of the brick and its 26 neighbours
    for (int64_t ci : changed) {
        HCell &c = h->cells[(size_t)ci];
        const bool res = c.slot >= 0;
        float m[8];
        for (int k = 0; k < 4; k++) m[k] = m[4 + k] = c.dev_avg[k];
        if (!res) {
            const int L = level_of(ci), G = g.grid[L];
            const int64_t li = ci - g.cell_off[L];
            const int x = (int)(li % G), y = (int)((li / G) % G), z = (int)(li / ((int64_t)G * G));
            for (int dz = -1; dz <= 1; dz++)
                for (int dy = -1; dy <= 1; dy++)
                    for (int dx = -1; dx <= 1; dx++) {
                        const int nx = x + dx, ny = y + dy, nz = z + dz;
                        if (nx < 0 || ny < 0 || nz < 0 || nx >= G || ny >= G || nz >= G) continue;
                        const int64_t ni = cell_index(g, L, nx, ny, nz);
                        const HCell &nc = h->cells[(size_t)ni];
                        if (!nc.inside) continue;
                        const bool data = h->data_cell[(size_t)ni] != 0;
                        for (int k = 0; k < C; k++) {
                            const float lo = data ? (float)nc.bmin[k] : nc.dev_avg[k];
                            const float hi = data ? (float)nc.bmax[k] : nc.dev_avg[k];
                            m[k] = std::min(m[k], lo);
                            m[4 + k] = std::max(m[4 + k], hi);
                        }
                    }
        }
        const int32_t kind = res ? kBrick : kBrickMissing, slot = res ? c.slot : -1;
        bool diff = !c.dev_valid || c.dev_kind != kind || c.dev_slot != slot;
        for (int k = 0; k < 8 && !diff; k++) diff = c.dev_miss[k] != m[k];
        if (!diff) continue;
        CellDelta d{};
        d.index = (int32_t)ci;
        d.kind = kind;
        d.slot = slot;
        for (int k = 0; k < 4; k++) {
            d.avg[k] = c.dev_avg[k];
            d.lo[k] = m[k];
            d.hi[k] = m[4 + k];
        }
        deltas.push_back(d);
        c.dev_kind = kind;
        c.dev_slot = slot;
        for (int k = 0; k < 8; k++) c.dev_miss[k] = m[k];
        c.dev_valid = true;
    }
    return OCT_OK;
}

// Device side of an upload: change events into the other node table, gathers, skip bounds,
// then the tables swap.
static int upload_tail(oct_handle *h, hipStream_t s, int64_t V, bool in_place,
                const std::vector<CellDelta> &deltas, const std::vector<BrickJob> &jobs,
                const std::vector<CopyJob> &copies, uint64_t resident, uint64_t bricks_total, uint64_t pending, uint64_t requests_seen,
                uint64_t evictions, uint64_t unserved, oct_upload_stats *out)
{
    const VolGeom &g = h->g;
    const int C = g.C;
    const size_t d_bytes = deltas.size() * sizeof(CellDelta);
    const size_t j_off = (d_bytes + 255) & ~(size_t)255;
    const size_t j_bytes = jobs.size() * sizeof(BrickJob);
    const size_t c_off = (j_off + j_bytes + 255) & ~(size_t)255;    // copies from the store
    const size_t c_bytes = copies.size() * sizeof(CopyJob);
    const size_t gs_off = (c_off + c_bytes + 255) & ~(size_t)255;   // gather scratch
    if (d_bytes + j_bytes + c_bytes) {
        int rc = stage_reserve(h, h->up, gs_off + gather_scratch_bytes(g, (int)jobs.size()));
        // renders read the node table and the pool: those of the other table's version (and
        // older) end first, all of them when a brick they may read is rewritten in place
        if (!rc) rc = (h->capped || in_place) ? wait_for_renders(h, s) : wait_for_renders_before(h, s, V);
        if (rc) return rc;
        if (d_bytes) std::memcpy(h->up.host, deltas.data(), d_bytes);
        if (j_bytes) std::memcpy((uint8_t *)h->up.host + j_off, jobs.data(), j_bytes);
        if (c_bytes) std::memcpy((uint8_t *)h->up.host + c_off, copies.data(), c_bytes);
        HIPCHK(h, hipMemcpyAsync(h->up.dev, h->up.host, c_off + c_bytes, hipMemcpyHostToDevice, s));
        HIPCHK(h, hipEventRecord(h->up.ev, s));
        DevCell *next = h->table_alt;
        HIPCHK(h, hipMemcpyAsync(next, h->table, sizeof(DevCell) * (size_t)h->n_cells,
                                 hipMemcpyDeviceToDevice, s));
        HIPCHK(h, launch_apply_deltas(next, h->miss_range, (const CellDelta *)h->up.dev,
                                      (int)deltas.size(), s));
        hipEvent_t e0 = bt_begin(h, s);
        const BrickJob *jobs_dev = (const BrickJob *)((uint8_t *)h->up.dev + j_off);
        if (h->pc) {
            int rc2 = gather_paged(h, jobs, 0, (int)jobs.size(), jobs_dev, next,
                                   (uint8_t *)h->up.dev + gs_off, s);
            if (rc2) return rc2;
        } else {
            HIPCHK(h, launch_gather(g, h->master, next, h->pool, h->brick_bytes, jobs_dev,
                                    (int)jobs.size(), h->slot_range, h->background_f,
                                    (uint8_t *)h->up.dev + gs_off, h->store_dev, h->store_range,
                                    h->store_bytes, s));
        }
        HIPCHK(h, launch_copy_bricks(g, h->pool, h->brick_bytes,
                                     (const CopyJob *)((uint8_t *)h->up.dev + c_off),
                                     (int)copies.size(), h->store_dev, h->store_range,
                                     h->store_bytes, h->slot_range, s));
        if (e0) {
            // per bordered voxel of each job's sub-box: the padded pool voxel written and the
            // source level's C values read (plus the store entry written for stored bricks);
            // per copied brick: the entry read and the padded brick written
            double bytes = 0.0;
            const double s3 = (double)(g.M + 2) * (g.M + 2) * (g.M + 2);
            for (const BrickJob &jb : jobs) {
                double nv = 1.0;
                for (int a = 0; a < 3; a++) nv *= (double)(jb.hi[a] - jb.lo[a] + 1);
                bytes += nv * ((jb.slot >= 0 ? 4.0 : 0.0) + (double)C + (jb.store >= 0 ? (double)C : 0.0)) *
                         (double)h->esz;
            }
            bytes += (double)copies.size() * s3 * (4.0 + (double)C) * (double)h->esz;
            bt_end(h, e0, s, 3, bytes);
        }
        HIPCHK(h, launch_ranges(g, next, h->slot_range, h->miss_range, s));
        h->table_alt = h->table;
        h->table = next;
        h->version++;
    }
    HIPCHK(h, hipEventRecord(h->ev_upload, s));
    if (out) {
        out->bricks_gathered = jobs.size() + copies.size();
        out->bricks_from_store = copies.size();
        out->bricks_resident = resident;
        out->bricks_total = bricks_total;
        out->nodes_changed = deltas.size();
        out->bytes_written = (jobs.size() + copies.size()) * h->brick_bytes + d_bytes;
        out->requests_seen = requests_seen;
        out->evictions = evictions;
    }
    if (h->capped) return (pending || unserved) ? OCT_INCOMPLETE : OCT_OK;
    return resident < bricks_total ? OCT_INCOMPLETE : OCT_OK;
}

int brick_pool_upload(oct_handle *h, uint64_t byte_budget, void *stream, oct_upload_stats *out)
{
    if (!h) return OCT_EINVAL;
    HIPCHK(h, hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    const VolGeom &g = h->g;
    const int C = g.C, M = g.M;
    {
        int rc = wait_for(h, s, h->ev_insert);
        if (!rc) rc = wait_for(h, s, h->ev_upload);
        if (!rc && h->capped) rc = wait_for_renders(h, s);   // their flags are read first
        if (rc) return rc;
    }
    // This call writes table version V + 1.  Renders below version V are waited for before
    // its device writes (the other table held version V - 1), so slots that left the table at
    // version V or earlier can be reused now; slots leaving it now wait for the next call.
    const int64_t V = h->version;
    if (!h->capped) {
        size_t keep = 0;
        for (const auto &d : h->deferred) {
            if (d.second <= V) h->free_slots.push_back(d.first);
            else h->deferred[keep++] = d;
        }
        h->deferred.resize(keep);
    }
    // a slot the current table points at is read by renders in flight: released later
    auto release_slot = [&](const HCell &c) {
        if (!h->capped && c.dev_valid && c.dev_kind == kBrick && c.dev_slot == c.slot)
            h->deferred.push_back({c.slot, V + 1});
        else
            h->free_slots.push_back(c.slot);
    };
    bool in_place = false;   // a brick renders may read is rewritten in its slot
    bool dirty = false;
    for (const auto &d : h->dirty) dirty = dirty || !d.empty();
    std::vector<CellDelta> deltas;
    std::vector<BrickJob> jobs;
    std::vector<CopyJob> copies;
    uint64_t requests_seen = 0, evictions = 0, unserved = 0, resident = 0, pending = 0;
    uint64_t bricks_total = 0;
    if (h->capped && h->paging_ready && !dirty) {
        int rc = upload_paging_only(h, byte_budget, s, deltas, jobs, copies, requests_seen,
                                    evictions, unserved);
        if (rc) return rc;
        resident = h->n_resident;
        bricks_total = h->n_data;
        return upload_tail(h, s, V, in_place, deltas, jobs, copies, resident, bricks_total,
                           pending, requests_seen, evictions, unserved, out);
    }
    h->paging_ready = false;

    // ---- 1. cells whose level data changed, and cells whose bordered region touches a change
    std::vector<int32_t> stat_cells;  // (L, x, y, z) quadruples
    // per cell: bordered-brick sub-box touched by changed data (lo[3], hi[3]; lo > hi = none)
    std::vector<int32_t> border_box((size_t)h->n_cells * 6);
    for (int64_t i = 0; i < h->n_cells; i++) {
        int32_t *bb = &border_box[(size_t)i * 6];
        bb[0] = bb[1] = bb[2] = 1 << 30;
        bb[3] = bb[4] = bb[5] = -1;
    }
    std::vector<uint8_t> data_dirty((size_t)h->n_cells, 0);
    const int S = M + 2;
    for (int L = 0; L <= g.N; L++) {
        const int G = g.grid[L];
        for (const Box &b : h->dirty[L]) {
            int lo[3], hi[3];
            for (int a = 0; a < 3; a++) {
                lo[a] = std::max(0, (b.lo[a] - 1) / M);
                hi[a] = std::min(G - 1, (b.hi[a] + 1) / M);
            }
            for (int z = lo[2]; z <= hi[2]; z++)
                for (int y = lo[1]; y <= hi[1]; y++)
                    for (int x = lo[0]; x <= hi[0]; x++) {
                        const int64_t ci = cell_index(g, L, x, y, z);
                        if (!h->cells[ci].inside) continue;
                        // bordered positions l whose clamped source index lies in the box
                        const int cb[3] = {x, y, z};
                        int llo[3], lhi[3];
                        bool any = true;
                        for (int a = 0; a < 3; a++) {
                            llo[a] = S;
                            lhi[a] = -1;
                            for (int l = 0; l < S; l++) {
                                const int gi = std::min(std::max(cb[a] * M - 1 + l, 0), g.ext[L][a] - 1);
                                if (gi >= b.lo[a] && gi <= b.hi[a]) {
                                    llo[a] = std::min(llo[a], l);
                                    lhi[a] = std::max(lhi[a], l);
                                }
                            }
                            if (lhi[a] < 0) any = false;
                        }
                        if (any) {
                            int32_t *bb = &border_box[(size_t)ci * 6];
                            for (int a = 0; a < 3; a++) {
                                bb[a] = std::min(bb[a], llo[a]);
                                bb[3 + a] = std::max(bb[3 + a], lhi[a]);
                            }
                        }
                        const int clo[3] = {x * M, y * M, z * M};
                        const int chi[3] = {x * M + M - 1, y * M + M - 1, z * M + M - 1};
                        if (box_intersects(b, clo, chi) && !data_dirty[ci]) {
                            data_dirty[ci] = 1;
                            stat_cells.insert(stat_cells.end(), {L, x, y, z});
                        }
                    }
        }
        h->dirty[L].clear();
    }
    const int n_stat = (int)(stat_cells.size() / 4);

    // flags written by the renders since the last call (capped pool only), then cleared
    if (h->capped) {
        HIPCHK(h, hipMemcpyAsync(h->flags_host, h->flags, (size_t)h->n_cells, hipMemcpyDeviceToHost, s));
        HIPCHK(h, launch_fill_u8(h->flags, h->n_cells, 0, s));
        if (!n_stat) HIPCHK(h, hipStreamSynchronize(s));
        // synchronised by the statistics read-back below otherwise
    }

    // ---- 2. statistics of changed cells (one read-back)
    if (n_stat) {
        const size_t cl_bytes = stat_cells.size() * sizeof(int32_t);
        const size_t st_off = (cl_bytes + 255) & ~(size_t)255;
        const size_t st_bytes = (size_t)n_stat * sizeof(CellStat);
        const size_t sc_off = (st_off + st_bytes + 255) & ~(size_t)255;
        int rc = stage_reserve(h, h->up, sc_off + stats_scratch_bytes(g, n_stat));
        if (rc) return rc;
        std::memcpy(h->up.host, stat_cells.data(), cl_bytes);
        HIPCHK(h, hipMemcpyAsync(h->up.dev, h->up.host, cl_bytes, hipMemcpyHostToDevice, s));
        hipEvent_t e0 = bt_begin(h, s);
        const int32_t *cells_dev = (const int32_t *)h->up.dev;
        CellStat *stats_dev = (CellStat *)((uint8_t *)h->up.dev + st_off);
        if (h->pc) {
            // disk tier: runs of cells whose pages fit a batch (a cell lies in one page)
            const int64_t budget = pg_budget(h);
            for (int i0 = 0; i0 < n_stat;) {
                std::vector<int64_t> pages;
                std::vector<uint8_t> wr;
                int i1 = i0;
                for (; i1 < n_stat; i1++) {
                    const int L = stat_cells[4 * i1];
                    int lo[3], hi[3];
                    for (int a = 0; a < 3; a++) {
                        lo[a] = stat_cells[4 * i1 + 1 + a] * M;
                        hi[a] = lo[a] + M - 1;
                    }
                    std::vector<int64_t> cp;
                    std::vector<uint8_t> cw;
                    add_box_pages(g, L, lo, hi, 0, cp, cw);
                    bool fresh = false;
                    for (int64_t q : cp) fresh |= std::find(pages.begin(), pages.end(), q) == pages.end();
                    if (fresh && (int64_t)pages.size() + (int64_t)cp.size() > budget && i1 > i0) break;
                    for (size_t k = 0; k < cp.size(); k++)
                        if (std::find(pages.begin(), pages.end(), cp[k]) == pages.end()) {
                            pages.push_back(cp[k]);
                            wr.push_back(0);
                        }
                }
                const int a0 = i0, n = i1 - i0;
                rc = paged_batch(h, pages, wr, s, [&]() -> int {
                    HIPCHK(h, launch_stats(g, h->master, h->mask, cells_dev + 4 * a0, n,
                                           (uint8_t *)h->up.dev + sc_off, stats_dev + a0, s));
                    return OCT_OK;
                });
                if (rc) return rc;
                i0 = i1;
            }
        } else {
            HIPCHK(h, launch_stats(g, h->master, h->mask, cells_dev, n_stat,
                                   (uint8_t *)h->up.dev + sc_off, stats_dev, s));
        }
        if (e0) {
            // every valid voxel of each changed cell, all channels (plus the mask at level 0)
            double bytes = 0.0;
            for (int i = 0; i < n_stat; i++) {
                const int L = stat_cells[4 * i];
                double nv = 1.0;
                for (int a = 0; a < 3; a++) {
                    const int lo = stat_cells[4 * i + 1 + a] * M;
                    nv *= (double)std::max(0, std::min(lo + M, g.ext[L][a]) - lo);
                }
                bytes += nv * ((double)C * (double)h->esz + (L == 0 ? 1.0 : 0.0));
            }
            bt_end(h, e0, s, 2, bytes);
        }
        HIPCHK(h, hipMemcpyAsync((uint8_t *)h->up.host + st_off, (uint8_t *)h->up.dev + st_off, st_bytes,
                                 hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        const CellStat *st = (const CellStat *)((uint8_t *)h->up.host + st_off);
        for (int i = 0; i < n_stat; i++) {
            const int L = stat_cells[4 * i];
            HCell &c = h->cells[cell_index(g, L, stat_cells[4 * i + 1], stat_cells[4 * i + 2],
                                           stat_cells[4 * i + 3])];
            for (int k = 0; k < C; k++) {
                c.bmin[k] = st[i].mn[k];
                c.bmax[k] = st[i].mx[k];
                c.bsum[k] = st[i].sum[k];
                if (L == 0) c.ins[k] = st[i].ins[k];
            }
            c.have_stats = true;
        }
    }

    if (h->capped)
        for (int64_t i = 0; i < h->n_cells; i++)
            if (h->flags_host[i] == 1) h->last_used[i] = h->frame;

    // ---- 3. states, resolved entries and slots
    recompute_states(h);
    std::vector<int32_t> new_kind((size_t)h->n_cells);
    std::vector<float> new_avg((size_t)h->n_cells * 4);
    for (int L = g.N; L >= 0; L--) {
        const int G = g.grid[L];
        for (int z = 0; z < G; z++)
            for (int y = 0; y < G; y++)
                for (int x = 0; x < G; x++) {
                    const int64_t ci = cell_index(g, L, x, y, z);
                    HCell &c = h->cells[ci];
                    float *a = &new_avg[(size_t)ci * 4];
                    if (c.exists) {
                        for (int k = 0; k < 4; k++) a[k] = k < C ? (float)c.avg[k] : 0.0f;
                    } else {
                        const int64_t pi = cell_index(g, L + 1, x / 2, y / 2, z / 2);
                        for (int k = 0; k < 4; k++) a[k] = new_avg[(size_t)pi * 4 + k];
                    }
                    const bool brick = c.exists && c.state == kBrickState;
                    if (!brick && c.slot >= 0) {
                        release_slot(c);
                        c.slot = -1;
                        c.needs_gather = false;
                    }
                    // an uncapped pool gives every brick node a slot; a capped one pages on
                    // request (below)
                    if (!h->capped && brick && c.slot < 0 && !h->free_slots.empty()) {
                        c.slot = h->free_slots.back();
                        h->free_slots.pop_back();
                        c.needs_gather = true;
                    }
                    new_kind[ci] = brick ? kBrickMissing : kAvg;
                }
    }
    // neighbourhood changes: a brick's border holds R_L of its 26 neighbours
    auto rep_changed = [&](int64_t ci) {
        const HCell &c = h->cells[ci];
        const bool was_data = c.dev_kind != kAvg, is_data = new_kind[ci] != kAvg;
        if (was_data != is_data) return true;
        if (!is_data)
            for (int k = 0; k < C; k++)
                if (c.dev_avg[k] != new_avg[(size_t)ci * 4 + k]) return true;
        return false;
    };
    // near_change: the cell or one of its 26 neighbours (same level) changed kind or AVG.
    // Marked from the changed cells, usually few, instead of testing 27 cells per brick.
    std::vector<uint8_t> near_change((size_t)h->n_cells, 0);
    for (int L = 0; L <= g.N; L++) {
        const int G = g.grid[L];
        for (int z = 0; z < G; z++)
            for (int y = 0; y < G; y++)
                for (int x = 0; x < G; x++) {
                    if (!rep_changed(cell_index(g, L, x, y, z))) continue;
                    for (int nz = std::max(z - 1, 0); nz <= std::min(z + 1, G - 1); nz++)
                        for (int ny = std::max(y - 1, 0); ny <= std::min(y + 1, G - 1); ny++)
                            for (int nx = std::max(x - 1, 0); nx <= std::min(x + 1, G - 1); nx++)
                                near_change[cell_index(g, L, nx, ny, nz)] = 1;
                }
    }
    uint64_t budget_left = byte_budget ? byte_budget : UINT64_MAX;
    // a whole brick is copied from the host brick store when the store holds it, else gathered
    // (and, with a store, written to it too)
    auto push_job = [&](HCell &c, int L, int x, int y, int z, bool full, const int32_t *bb) {
        const int32_t e = h->store ? h->store_idx[(size_t)cell_index(g, L, x, y, z)] : -1;
        budget_left -= h->brick_bytes;
        c.needs_gather = false;
        if (full && e >= 0 && h->store_ok[(size_t)e]) {
            copies.push_back(CopyJob{c.slot, e});
            return;
        }
        BrickJob j{};
        j.slot = c.slot;
        j.level = L;
        j.bx = x;
        j.by = y;
        j.bz = z;
        j.full = full ? 1 : 0;
        j.store = full ? e : -1;
        if (full && e >= 0) h->store_ok[(size_t)e] = 1;
        for (int a = 0; a < 3; a++) {
            j.lo[a] = full ? 0 : bb[a];
            j.hi[a] = full ? S - 1 : bb[3 + a];
        }
        jobs.push_back(j);
    };
    for (int L = g.N; L >= 0; L--) {  // coarse levels first
        const int G = g.grid[L];
        for (int z = 0; z < G; z++)
            for (int y = 0; y < G; y++)
                for (int x = 0; x < G; x++) {
                    const int64_t ci = cell_index(g, L, x, y, z);
                    HCell &c = h->cells[ci];
                    if (new_kind[ci] == kAvg) continue;
                    bricks_total++;
                    const int32_t *bb = &border_box[(size_t)ci * 6];
                    const bool changed = near_change[ci] || (bb[3] >= 0 && bb[4] >= 0 && bb[5] >= 0);
                    if (h->store) {
                        // the store holds every brick's current bordered brick: a changed brick
                        // is gathered whole, into the store alone when it is not resident
                        const int32_t e = h->store_idx[(size_t)ci];
                        if (changed) h->store_ok[(size_t)e] = 0;
                        if (c.slot < 0) {
                            if (!h->store_ok[(size_t)e]) {
                                BrickJob j{};
                                j.slot = -1;
                                j.level = L;
                                j.bx = x;
                                j.by = y;
                                j.bz = z;
                                j.full = 1;
                                j.store = e;
                                for (int a = 0; a < 3; a++) j.hi[a] = S - 1;
                                jobs.push_back(j);
                                h->store_ok[(size_t)e] = 1;
                            }
                            continue;
                        }
                    }
                    if (c.slot < 0) continue;
                    // whole brick: new slot, deferred earlier, or a neighbour changed kind/AVG
                    // (and, with a store, any change: the store keeps whole bricks)
                    bool full = c.needs_gather || near_change[ci] || (h->store && changed);
                    const bool part = !full && bb[3] >= 0 && bb[4] >= 0 && bb[5] >= 0;
                    if (full || part) {
                        if (budget_left >= h->brick_bytes) {
                            if (!h->capped && c.dev_valid && c.dev_kind == kBrick &&
                                c.dev_slot == c.slot) {
                                if (!h->free_slots.empty()) {
                                    // copy on write: the whole brick into a fresh slot
                                    release_slot(c);
                                    c.slot = h->free_slots.back();
                                    h->free_slots.pop_back();
                                    full = true;
                                } else {
                                    in_place = true;
                                }
                            }
                            push_job(c, L, x, y, z, full, bb);
                        } else {
                            c.needs_gather = true;   // stale until gathered: rendered with AVG
                        }
                    }
                    if (!c.needs_gather) new_kind[ci] = kBrick;
                }
    }

    // ---- 4. paging ("Brick Upload from RAM to GPU"): requested bricks get slots, coarser
    // levels first; free slots first, then slots unused by the last renders (least recently
    // used first), and when those run out a coarser request may take a used finer brick.
    if (h->capped) {
        std::vector<int64_t> reqs, idle, busy;
        for (int L = g.N; L >= 0; L--) {
            const int64_t n = (int64_t)g.grid[L] * g.grid[L] * g.grid[L];
            for (int64_t i = 0; i < n; i++) {
                const int64_t ci = g.cell_off[L] + i;
                const HCell &c = h->cells[ci];
                if (new_kind[ci] == kAvg) continue;
                if (h->flags_host[ci] == 2 && c.slot < 0) reqs.push_back(ci);
                if (c.slot >= 0) (h->last_used[ci] == h->frame ? busy : idle).push_back(ci);
            }
        }
        requests_seen = reqs.size();
        auto level_of = [&](int64_t ci) {
            int L = 0;
            while (L < g.N && ci >= g.cell_off[L + 1]) L++;
            return L;
        };
        std::stable_sort(idle.begin(), idle.end(), [&](int64_t a, int64_t b) {
            if (h->last_used[a] != h->last_used[b]) return h->last_used[a] < h->last_used[b];
            return level_of(a) < level_of(b);
        });
        std::stable_sort(busy.begin(), busy.end(),
                         [&](int64_t a, int64_t b) { return level_of(a) < level_of(b); });
        size_t vi = 0, bi = 0;
        for (int64_t ci : reqs) {
            if (budget_left < h->brick_bytes) {
                unserved++;
                continue;
            }
            HCell &c = h->cells[ci];
            const int L = level_of(ci);
            int64_t victim = -1;
            if (h->free_slots.empty()) {
                if (vi < idle.size()) victim = idle[vi++];
                else if (bi < busy.size() && level_of(busy[bi]) < L) victim = busy[bi++];
                else {
                    unserved++;
                    continue;
                }
                HCell &v = h->cells[victim];
                h->free_slots.push_back(v.slot);
                v.slot = -1;
                v.needs_gather = false;
                new_kind[victim] = kBrickMissing;
                evictions++;
            }
            c.slot = h->free_slots.back();
            h->free_slots.pop_back();
            const int G = g.grid[L];
            const int64_t li = ci - g.cell_off[L];
            push_job(c, L, (int)(li % G), (int)((li / G) % G), (int)(li / ((int64_t)G * G)), true,
                     nullptr);
            new_kind[ci] = kBrick;
        }
        h->frame++;
    }

    // value bounds of missing bricks (their skip range): the brick and its 26 neighbours
    std::vector<float> miss((size_t)h->n_cells * 8, 0.0f);
    for (int L = g.N; L >= 0; L--) {
        const int G = g.grid[L];
        for (int z = 0; z < G; z++)
            for (int y = 0; y < G; y++)
                for (int x = 0; x < G; x++) {
                    const int64_t ci = cell_index(g, L, x, y, z);
                    float *m = &miss[(size_t)ci * 8];
                    for (int k = 0; k < 4; k++) m[k] = m[4 + k] = new_avg[(size_t)ci * 4 + k];
                    if (new_kind[ci] == kBrick) resident++;
                    if (new_kind[ci] != kBrickMissing) continue;
                    if (h->cells[ci].slot >= 0) pending++;
                    for (int dz = -1; dz <= 1; dz++)
                        for (int dy = -1; dy <= 1; dy++)
                            for (int dx = -1; dx <= 1; dx++) {
                                const int nx = x + dx, ny = y + dy, nz = z + dz;
                                if (nx < 0 || ny < 0 || nz < 0 || nx >= G || ny >= G || nz >= G) continue;
                                const int64_t ni = cell_index(g, L, nx, ny, nz);
                                const HCell &nc = h->cells[ni];
                                if (!nc.inside) continue;
                                for (int k = 0; k < C; k++) {
                                    const float lo = new_kind[ni] != kAvg ? (float)nc.bmin[k] : new_avg[(size_t)ni * 4 + k];
                                    const float hi = new_kind[ni] != kAvg ? (float)nc.bmax[k] : new_avg[(size_t)ni * 4 + k];
                                    m[k] = std::min(m[k], lo);
                                    m[4 + k] = std::max(m[4 + k], hi);
                                }
                            }
                }
    }

    // ---- 5. change events for the node table, then the gathers, then the skip bounds
    for (int64_t i = 0; i < h->n_cells; i++) {
        HCell &c = h->cells[i];
        const int32_t slot = new_kind[i] == kBrick ? c.slot : -1;
        const float *a = &new_avg[(size_t)i * 4];
        const float *m = &miss[(size_t)i * 8];
        bool diff = !c.dev_valid || c.dev_kind != new_kind[i] || c.dev_slot != slot;
        for (int k = 0; k < 4 && !diff; k++) diff = c.dev_avg[k] != a[k];
        for (int k = 0; k < 8 && !diff; k++) diff = c.dev_miss[k] != m[k];
        if (!diff) continue;
        CellDelta d{};
        d.index = (int32_t)i;
        d.kind = new_kind[i];
        d.slot = slot;
        for (int k = 0; k < 4; k++) {
            d.avg[k] = a[k];
            d.lo[k] = m[k];
            d.hi[k] = m[4 + k];
        }
        deltas.push_back(d);
        c.dev_kind = new_kind[i];
        c.dev_slot = slot;
        for (int k = 0; k < 4; k++) c.dev_avg[k] = a[k];
        for (int k = 0; k < 8; k++) c.dev_miss[k] = m[k];
        c.dev_valid = true;
    }
    if (h->capped) {
        // the state paging-only uploads start from
        h->data_cell.assign((size_t)h->n_cells, 0);
        h->slot_cell.assign((size_t)h->n_slots, -1);
        for (int64_t ci = 0; ci < h->n_cells; ci++) {
            h->data_cell[(size_t)ci] = new_kind[(size_t)ci] != kAvg;
            const int32_t sl = h->cells[(size_t)ci].slot;
            if (sl >= 0) h->slot_cell[(size_t)sl] = ci;
        }
        h->n_data = bricks_total;
        h->n_resident = resident;
        h->paging_ready = pending == 0;
    }
    return upload_tail(h, s, V, in_place, deltas, jobs, copies, resident, bricks_total, pending,
                       requests_seen, evictions, unserved, out);
}

// The render kernel a view runs in (views of one launch are grouped by class).
static int32_t view_class(const oct_view &v)
{
    if (v.n_xform > 0 || v.missing != OCT_MISSING_AVG) return kClassGeneral;
    return v.mode == OCT_MODE_MIP ? kClassMip : kClassDvr;
}

// Views whose adjoint render_views_backward computes (and whose forward may therefore fill a
// checkpoint workspace): DVR without channel transforms, MIP with or without them, both with
// missing bricks drawn as AVG.
static bool view_differentiable(const oct_view &v)
{
    if (v.missing != OCT_MISSING_AVG) return false;
    return v.mode == OCT_MODE_MIP || v.n_xform == 0;
}

// Checkpoint workspace: per view, [position][pixel] float32 transmittances then [pixel] int32
// end positions; the positions cover the longest possible ray (the box diagonal) plus the end
// position.  MIP views hold [pixel][4] int32 positions of the channel maxima instead.
static int view_npos(const oct_handle *h, const oct_view &v)
{
    const double diag = std::sqrt((double)h->g.dims[0] * h->g.dims[0] +
                                  (double)h->g.dims[1] * h->g.dims[1] +
                                  (double)h->g.dims[2] * h->g.dims[2]);
    const double nmax = std::ceil(diag / (double)v.step) + 2.0;
    return (int)nmax + 1;
}

// Depth segments of a view's rays; the forward, the differentiable forward and the adjoint
// agree on it: none with early termination, else the view's request or the automatic count.
static int view_segments(const oct_handle *h, const oct_view &v)
{
    if (view_class(v) == kClassGeneral) return 1;
    if (v.mode == OCT_MODE_MIP) {
        // maxima combine by max; no early termination applies
        if (v.depth_segments > 0) return std::min(v.depth_segments, kMaxSplit);
        return auto_segments(h->g, v);
    }
    if (!(v.ert_alpha >= 1.0f)) return 1;
    if (v.depth_segments > 0) return std::min(v.depth_segments, kMaxSplit);
    return auto_segments(h->g, v);
}

// Checkpoint workspace of one view: [position][pixel] float32 transmittance before each
// evaluated position (from the start of its depth segment) and, for rays not split, after the
// last one; [pixel] int32 end positions; then for a split view [segment][pixel] float4 (C, T)
// of every depth segment.
static size_t view_ckpt_part_offset(const oct_handle *h, const oct_view &v)
{
    const size_t npix = (size_t)v.width * v.height;
    return (npix * (size_t)view_npos(h, v) * 4 + npix * 4 + 15) & ~(size_t)15;
}

static size_t view_ckpt_bytes(const oct_handle *h, const oct_view &v)
{
    const size_t npix = (size_t)v.width * v.height;
    if (v.mode == OCT_MODE_MIP) return (npix * 16 + 255) & ~(size_t)255;
    size_t b = view_ckpt_part_offset(h, v);
    const int S = view_segments(h, v);
    if (S > 1) b += npix * (size_t)S * 16;
    return (b + 255) & ~(size_t)255;
}

size_t render_refine_bytes(const oct_handle *h, const oct_view *view)
{
    if (!h || !view || view->width < 1 || view->height < 1) return 0;
    return (size_t)view->width * view->height * sizeof(RefineState);
}

size_t render_ckpt_bytes(const oct_handle *h, int32_t n_views, const oct_view *views)
{
    if (!h || n_views < 0 || (n_views && !views)) return 0;
    size_t total = 0;
    for (int i = 0; i < n_views; i++) {
        if (views[i].width < 1 || views[i].height < 1 || !(views[i].step > 0.0f)) return 0;
        total += view_ckpt_bytes(h, views[i]);
    }
    return total;
}

static int build_view(oct_handle *h, const oct_view &v, float *image, DevView &dv)
{
    const VolGeom &g = h->g;
    if (v.width < 1 || v.height < 1 || v.width > 32768 || v.height > 32768)
        return fail(h, OCT_EINVAL, "view size out of range");
    if (!(v.step > 0.0f) || !std::isfinite(v.step)) return fail(h, OCT_EINVAL, "step must be > 0");
    if (!(v.fov_y_deg > 0.0f && v.fov_y_deg < 180.0f)) return fail(h, OCT_EINVAL, "fov out of range");
    if (v.n_clip < 0 || v.n_clip > OCT_MAX_CLIPS) return fail(h, OCT_EINVAL, "n_clip must be 0..3");
    if (v.lod < -1) return fail(h, OCT_EINVAL, "lod must be >= -1");
    if (v.tile_begin < 0 || v.tile_count < -1) return fail(h, OCT_EINVAL, "bad tile range");
    if (!(v.ert_alpha > 0.0f)) return fail(h, OCT_EINVAL, "ert_alpha must be > 0");
    if (v.depth_segments < 0 || v.depth_segments > kMaxSplit)
        return fail(h, OCT_EINVAL, "depth_segments must be 0..16");
    if (v.reserved) return fail(h, OCT_EINVAL, "reserved fields must be 0");
    if (v.mode != OCT_MODE_DVR && v.mode != OCT_MODE_MIP)
        return fail(h, OCT_EINVAL, "mode must be OCT_MODE_DVR or OCT_MODE_MIP");
    if (v.missing < OCT_MISSING_AVG || v.missing > OCT_MISSING_REFINE)
        return fail(h, OCT_EINVAL, "missing must be OCT_MISSING_AVG, _FALLBACK or _REFINE");
    if ((v.missing == OCT_MISSING_REFINE) != (v.refine_state != nullptr))
        return fail(h, OCT_EINVAL, "refine_state is required by, and only by, refinement views");
    if (v.n_xform != 0 && v.n_xform != g.C)
        return fail(h, OCT_EINVAL, "n_xform must be 0 or the channel count");
    for (int c = 0; c < v.n_xform; c++)
        for (int a = 0; a < 3; a++)
            for (int q = 0; q < 4; q++)
                if (!std::isfinite(v.xform[c][a][q]))
                    return fail(h, OCT_EINVAL, "channel transforms must be finite");
    if (!image) return fail(h, OCT_EINVAL, "null image");
    for (int c = 0; c < g.C; c++) {
        if (!(v.window[c][1] > v.window[c][0])) return fail(h, OCT_EINVAL, "window hi must exceed lo");
        for (int j = 0; j < 8; j++) {
            if (!(v.tf_pos[c][j] >= 0.0f && v.tf_pos[c][j] <= 1.0f))
                return fail(h, OCT_EINVAL, "tf positions must lie in [0,1]");
            if (j && v.tf_pos[c][j] < v.tf_pos[c][j - 1])
                return fail(h, OCT_EINVAL, "tf positions must ascend");
        }
    }
    // camera frame in double, rounded to float (the per-pixel part runs in the kernel)
    double e[3], f[3], up[3], r[3], u[3];
    for (int a = 0; a < 3; a++) {
        e[a] = (double)v.eye[a];
        f[a] = (double)v.target[a] - e[a];
        up[a] = (double)v.up[a];
    }
    double n = std::sqrt((f[0] * f[0] + f[1] * f[1]) + f[2] * f[2]);
    if (!(n > 0.0)) return fail(h, OCT_EINVAL, "eye equals target");
    for (int a = 0; a < 3; a++) f[a] = f[a] / n;
    r[0] = f[1] * up[2] - f[2] * up[1];
    r[1] = f[2] * up[0] - f[0] * up[2];
    r[2] = f[0] * up[1] - f[1] * up[0];
    n = std::sqrt((r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]);
    if (!(n > 0.0)) return fail(h, OCT_EINVAL, "up is parallel to the view direction");
    for (int a = 0; a < 3; a++) r[a] = r[a] / n;
    u[0] = r[1] * f[2] - r[2] * f[1];
    u[1] = r[2] * f[0] - r[0] * f[2];
    u[2] = r[0] * f[1] - r[1] * f[0];
    const double th = std::tan((double)v.fov_y_deg * (M_PI / 360.0));
    std::memset(&dv, 0, sizeof dv);
    for (int a = 0; a < 3; a++) {
        dv.eye[a] = v.eye[a];
        dv.f[a] = (float)f[a];
        dv.r[a] = (float)r[a];
        dv.u[a] = (float)u[a];
    }
    dv.kx = (float)(th * (double)v.width / (double)v.height);
    dv.ky = (float)th;
    dv.klod = (float)(2.0 * th / (double)v.height);
    dv.step = v.step;
    dv.ert = v.ert_alpha;
    dv.width = v.width;
    dv.height = v.height;
    dv.tiles_x = (v.width + OCT_TILE - 1) / OCT_TILE;
    dv.lod = v.lod;
    dv.n_clip = v.n_clip;
    dv.skip = v.no_skip ? 0 : 1;
    std::memcpy(dv.clip, v.clip, sizeof dv.clip);
    for (int c = 0; c < kMaxC; c++) {
        const bool on = c < g.C;
        dv.ulo[c] = on ? v.window[c][0] : 0.0f;
        dv.uscale[c] = on ? (float)(255.0 / ((double)v.window[c][1] - (double)v.window[c][0])) : 0.0f;
    }
    std::memcpy(dv.tf_pos, v.tf_pos, sizeof dv.tf_pos);
    std::memcpy(dv.tf_rgba, v.tf_rgba, sizeof dv.tf_rgba);
    dv.image = image;
    dv.mode = v.mode;
    dv.missing = v.missing;
    dv.xform_on = v.n_xform > 0 ? 1 : 0;
    if (dv.xform_on) std::memcpy(dv.xform, v.xform, sizeof dv.xform);
    dv.rstate = (RefineState *)v.refine_state;
    dv.vclass = view_class(v);
    return OCT_OK;
}

// Per-launch plan of a view list: the view records, their work items and depth segments.
struct LaunchPlan {
    int64_t n_items = 0;
    int64_t max_split_pixels = 0;
    int64_t max_refine_pixels = 0;
    int n_split = 0;
    int split_modes = 0;             // bit 0: a split DVR view, bit 1: a split MIP view
    int n_refine = 0;
    int n_skip = 0;
    size_t part_floats = 0;          // segment results of split views without checkpoints
    int32_t class_items[kNumClasses + 1] = {0, 0, 0, 0};
};

// Fills dvs[0 .. n_views) -- the views grouped by kernel class, in the caller's order inside a
// class (dvs[j].user_index is the caller's index) -- plus split[0 .. n_split) and
// refine[0 .. n_refine) (record indices of split and refinement views) for one forward launch.
// Views without checkpoints are split into depth segments only when `split_ok`; their segment
// results go at float offset part_at[j] of a buffer the caller assigns afterwards (dvs[j].part
// is left NULL for them).  With checkpoints the segment results live in the workspace, laid
// out in the caller's view order.
static int plan_launch(oct_handle *h, int32_t n_views, const oct_view *views,
                       float *const *images, void *ckpt_ws, bool split_ok, DevView *dvs,
                       int32_t *split, int32_t *refine, size_t *part_at, LaunchPlan &pl)
{
    // workspace offsets in the caller's order
    std::vector<size_t> ck_at((size_t)n_views, 0);
    {
        size_t ck_off = 0;
        for (int i = 0; i < n_views; i++) {
            ck_at[i] = ck_off;
            if (ckpt_ws) {
                if (!view_differentiable(views[i]))
                    return fail(h, OCT_EINVAL, "a checkpoint workspace needs views the adjoint "
                                               "supports (no refinement or full-frame fallback, "
                                               "no channel transforms in DVR)");
                if (views[i].width < 1 || views[i].height < 1 || !(views[i].step > 0.0f))
                    return fail(h, OCT_EINVAL, "view size out of range");
                ck_off += view_ckpt_bytes(h, views[i]);
            }
        }
    }
    int j = 0;
    for (int cls = 0; cls < kNumClasses; cls++) {
        pl.class_items[cls] = (int32_t)pl.n_items;
        for (int i = 0; i < n_views; i++) {
            if (view_class(views[i]) != cls) continue;
            DevView &dv = dvs[j];
            int rc = build_view(h, views[i], images[i], dv);
            if (rc) return rc;
            dv.user_index = i;
            const size_t npix = (size_t)views[i].width * views[i].height;
            uint8_t *ws = ckpt_ws ? (uint8_t *)ckpt_ws + ck_at[i] : nullptr;
            if (ws && views[i].mode == OCT_MODE_MIP) {
                dv.amax = (int32_t *)ws;
            } else if (ws) {
                dv.npos = view_npos(h, views[i]);
                dv.ckpt = (float *)ws;
                dv.nend = (int32_t *)(ws + npix * dv.npos * 4);
            }
            const int tiles = dv.tiles_x * ((views[i].height + OCT_TILE - 1) / OCT_TILE);
            const int tb = std::min(views[i].tile_begin, tiles);
            const int te = views[i].tile_count < 0 ? tiles : std::min(tiles, tb + views[i].tile_count);
            // early termination makes a later segment depend on the earlier ones: unsplit then;
            // a MIP adjoint needs each ray's positions of the maxima from one pass
            const bool mip_ck = ws && views[i].mode == OCT_MODE_MIP;
            const int nsplit = te > tb && !mip_ck && (ws || split_ok) ? view_segments(h, views[i]) : 1;
            dv.nsplit = nsplit;
            dv.tile_begin = tb;
            dv.tile_end = te;
            if (nsplit > 1) {
                if (ws) {
                    // the adjoint reads the segment partials back: they live in the workspace
                    dv.part = (float *)(ws + view_ckpt_part_offset(h, views[i]));
                } else {
                    part_at[j] = pl.part_floats;
                    pl.part_floats += (size_t)nsplit * npix * 4;
                }
                split[pl.n_split++] = j;
                pl.split_modes |= views[i].mode == OCT_MODE_MIP ? 2 : 1;
                pl.max_split_pixels = std::max<int64_t>(pl.max_split_pixels, (int64_t)npix);
            }
            if (views[i].missing == OCT_MISSING_REFINE) {
                refine[pl.n_refine++] = j;
                pl.max_refine_pixels = std::max<int64_t>(pl.max_refine_pixels, (int64_t)npix);
            }
            // the view's work items (the kernel derives each one from its index, item_of)
            const int groups = (te - tb + kRenderTilesPerWg - 1) / kRenderTilesPerWg;
            dv.item_begin = (int32_t)pl.n_items;
            dv.groups = groups;
            pl.n_items += (int64_t)groups * nsplit;
            pl.n_skip += dv.skip ? 1 : 0;
            j++;
        }
    }
    pl.class_items[kNumClasses] = (int32_t)pl.n_items;
    if (pl.n_items > INT32_MAX) return fail(h, OCT_EINVAL, "too many tiles in one launch");
    return OCT_OK;
}

// Sums the sample counters (and the refinement views' waiting rays) read back to the host.
static void collect_stats(const uint8_t *hp, const RecordLayout &l, int n_views,
                          oct_render_stats *out)
{
    const RenderCounters *rcnt = (const RenderCounters *)(hp + l.c_off);
    *out = oct_render_stats{};
    for (int i = 0; i < kCounterSlots; i++) {
        out->rays += rcnt[i].rays;
        out->positions_nominal += rcnt[i].nominal;
        out->positions_composited += rcnt[i].composited;
        out->positions_trilinear += rcnt[i].trilinear;
    }
    const int32_t *rw = (const int32_t *)(hp + l.rw_off);
    for (int i = 0; i < n_views; i++) out->rays_waiting += (uint64_t)rw[i];
}

int render_views(oct_handle *h, int32_t n_views, const oct_view *views, float *const *images,
                 void *ckpt_ws, void *stream, oct_render_stats *out)
{
    if (!h) return OCT_EINVAL;
    if (n_views < 0 || (n_views > 0 && (!views || !images))) return fail(h, OCT_EINVAL, "bad view list");
    HIPCHK(h, hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<DevView> dvs((size_t)n_views);
    std::vector<int32_t> split_views((size_t)n_views), refine_views((size_t)n_views);
    std::vector<size_t> part_at((size_t)n_views, 0);
    LaunchPlan pl;
    {
        int rc = plan_launch(h, n_views, views, images, ckpt_ws, true, dvs.data(), split_views.data(),
                             refine_views.data(), part_at.data(), pl);
        if (rc) return rc;
    }
    const RecordLayout l = record_layout((size_t)n_views, (size_t)pl.n_split, (size_t)pl.n_refine);
    const size_t tbytes = view_tables_bytes(h->g.C);
    const size_t t_off = tables_offset(l);
    // tile-group orders behind the tables (one copy with the records)
    const size_t o_off = (t_off + (size_t)n_views * tbytes + 255) & ~(size_t)255;
    size_t order_ints = 0;
    for (int i = 0; i < n_views; i++)
        if (view_ordered(dvs[i], n_views)) order_ints += (size_t)dvs[i].groups;
    const size_t rec_bytes = o_off + order_ints * 4;
    RenderSlot &rs = h->rs[h->next_rs];
    h->next_rs = (h->next_rs + 1) % kRenderSlots;
    int rc = stage_reserve(h, rs.st, rec_bytes);   // the slot is idle now
    rs.version = h->version;
    if (!rc) rc = collect_kernel_time(h, rs);
    if (rc) return rc;
    const size_t part_floats = pl.part_floats;
    if (part_floats * sizeof(float) > rs.part_cap) {
        if (rs.part) HIPCHK(h, hipFree(rs.part));
        rs.part = nullptr;
        rs.part_cap = 0;
        HIPCHK(h, hipMalloc(&rs.part, part_floats * sizeof(float)));
        rs.part_cap = part_floats * sizeof(float);
    }
    for (int k = 0; k < pl.n_split; k++) {
        const int32_t j = split_views[k];
        if (!dvs[j].part) dvs[j].part = rs.part + part_at[j];
    }
    const int64_t mwords = view_mask_words(h->n_cells);
    const int n_skip = pl.n_skip;
    if ((size_t)n_skip * mwords * 4 > rs.tmask_cap) {
        if (rs.tmask) HIPCHK(h, hipFree(rs.tmask));
        rs.tmask = nullptr;
        rs.tmask_cap = 0;
        HIPCHK(h, hipMalloc((void **)&rs.tmask, (size_t)n_skip * mwords * 4));
        rs.tmask_cap = (size_t)n_skip * mwords * 4;
    }
    for (int i = 0, j = 0; i < n_views; i++)
        dvs[i].tmask = dvs[i].skip ? rs.tmask + (size_t)(j++) * mwords : nullptr;
    uint8_t *hp = (uint8_t *)rs.st.host;
    uint8_t *dp = (uint8_t *)rs.st.dev;
    for (int i = 0, at = 0; i < n_views; i++) {
        dvs[i].group_order = nullptr;
        if (view_ordered(dvs[i], n_views)) {
            const std::vector<int32_t> &ord = cached_group_order(h, dvs[i]);
            std::memcpy(hp + o_off + (size_t)at * 4, ord.data(), ord.size() * 4);
            dvs[i].group_order = (int32_t *)(dp + o_off) + at;
            at += dvs[i].groups;
        }
        dvs[i].rwait = (int32_t *)(dp + l.rw_off) + i;
        dvs[i].tables = dp + t_off + (size_t)i * tbytes;
    }
    fill_tables(h, dvs.data(), n_views, hp + t_off, tbytes, true);
    std::memcpy(hp, dvs.data(), l.v_bytes);
    std::memcpy(hp + l.sv_off, split_views.data(), (size_t)pl.n_split * 4);
    std::memcpy(hp + l.rf_off, refine_views.data(), (size_t)pl.n_refine * 4);
    std::memset(hp + l.rw_off, 0, (size_t)n_views * 4);
    std::memset(hp + l.c_off, 0, l.c_bytes);
    // the copy runs on the prep stream (it overlaps the renders issued before this one): views,
    // lists, zeroed counters, tables and tile-group orders in one copy
    if (!rs.prep) HIPCHK(h, hipEventCreateWithFlags(&rs.prep, hipEventDisableTiming));
    HIPCHK(h, hipMemcpyAsync(rs.st.dev, hp, rec_bytes, hipMemcpyHostToDevice, h->prep));
    HIPCHK(h, hipEventRecord(rs.prep, h->prep));
    rc = wait_for(h, s, rs.prep);
    if (!rc) rc = wait_for(h, s, h->ev_upload);   // the node table and pool of the last upload
    if (rc) return rc;
    if (n_skip) HIPCHK(h, launch_view_mask(h->g, (const DevView *)dp, n_views, h->table, h->n_cells, s));
    if (h->ktime) {
        if (!rs.k0) HIPCHK(h, hipEventCreate(&rs.k0));
        if (!rs.k1) HIPCHK(h, hipEventCreate(&rs.k1));
        HIPCHK(h, hipEventRecord(rs.k0, s));
    }
    HIPCHK(h, launch_render(h->g, h->table, h->pool, h->brick_bytes, (const DevView *)dp,
                            n_views, pl.class_items, out ? (RenderCounters *)(dp + l.c_off) : nullptr,
                            h->capped ? h->flags : nullptr, s));
    if (h->ktime) {
        HIPCHK(h, hipEventRecord(rs.k1, s));
        rs.k_pending = true;
    }
    HIPCHK(h, launch_combine((const DevView *)dp, (const int32_t *)(dp + l.sv_off), pl.n_split,
                             h->g.C, pl.split_modes, pl.max_split_pixels, s));
    HIPCHK(h, launch_refine_finish((const DevView *)dp, (const int32_t *)(dp + l.rf_off),
                                   pl.n_refine, h->g.C, pl.max_refine_pixels, s));
    if (out) {
        HIPCHK(h, hipMemcpyAsync(hp + l.sv_off, dp + l.sv_off, l.c_off + l.c_bytes - l.sv_off,
                                 hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        collect_stats(hp, l, n_views, out);
    }
    HIPCHK(h, hipEventRecord(rs.st.ev, s));
    rs.stream = s;
    if (ckpt_ws) ckpt_log_put(h, ckpt_ws, n_views, views);
    return OCT_OK;
}

int render_views_noalloc(oct_handle *h, int32_t n_views, const oct_view *views,
                         float *const *images, void *ckpt_ws, void *stream, oct_render_stats *out)
{
    if (!h) return OCT_EINVAL;
    if (n_views < 0 || (n_views > 0 && (!views || !images))) return fail(h, OCT_EINVAL, "bad view list");
    if (n_views > kNoAllocMaxViews)
        return fail(h, OCT_ERANGE, "render_views_noalloc takes at most 64 views per call");
    if (!h->scratch_dev) return fail(h, OCT_EDEVICE, "no device scratch");
    HIPCHK(h, hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    RenderSlot &rs = h->rs[kRenderSlots];
    // the host records are reused: the previous call's copy of them must have finished
    HIPCHK(h, hipEventSynchronize(h->na_copy));
    uint8_t *hp = (uint8_t *)rs.st.host;
    DevView *dvs = (DevView *)hp;
    int32_t split[kNoAllocMaxViews], refine[kNoAllocMaxViews];
    LaunchPlan pl;
    int rc = plan_launch(h, n_views, views, images, ckpt_ws, false, dvs, split, refine, nullptr, pl);
    if (rc) return rc;
    const RecordLayout l = record_layout((size_t)n_views, (size_t)pl.n_split, (size_t)pl.n_refine);
    // scratch: records, tables and the tile-group order (one copy) | masks.  The order needs
    // room in the host records allotted at creation: a view of more groups keeps index order.
    const size_t tbytes = view_tables_bytes(h->g.C);
    const int64_t mwords = view_mask_words(h->n_cells);
    const size_t t_off = tables_offset(l);
    const size_t o_off = (t_off + (size_t)n_views * tbytes + 255) & ~(size_t)255;
    size_t order_ints = 0;
    for (int i = 0; i < n_views; i++)
        if (view_ordered(dvs[i], n_views) && dvs[i].groups <= kNoAllocMaxOrder)
            order_ints += (size_t)dvs[i].groups;
    const size_t rec_bytes = o_off + order_ints * 4;
    const size_t m_off = (rec_bytes + 255) & ~(size_t)255;
    const size_t need = m_off + (size_t)pl.n_skip * mwords * 4;
    if (need > kScratchBytes)
        return fail(h, OCT_ERANGE,
                    "render_views_noalloc: this launch needs " + std::to_string(need) +
                        " bytes of device scratch, the limit is " + std::to_string(kScratchBytes) +
                        " (fewer or smaller views per call, or render_views)");
    uint8_t *dp = (uint8_t *)h->scratch_dev;
    for (int i = 0, j = 0, at = 0; i < n_views; i++) {
        dvs[i].tables = dp + t_off + (size_t)i * tbytes;
        dvs[i].tmask = dvs[i].skip ? (uint32_t *)(dp + m_off) + (size_t)(j++) * mwords : nullptr;
        dvs[i].group_order = nullptr;
        if (view_ordered(dvs[i], n_views) && dvs[i].groups <= kNoAllocMaxOrder) {
            // built in the host records (no host allocation), its scratch behind it
            int32_t *ord = (int32_t *)(hp + o_off) + at;
            build_group_order(h->g, dvs[i], ord, ord + dvs[i].groups);
            dvs[i].group_order = (int32_t *)(dp + o_off) + at;
            at += dvs[i].groups;
        }
        dvs[i].rwait = (int32_t *)(dp + l.rw_off) + i;
    }
    fill_tables(h, dvs, n_views, hp + t_off, tbytes, false);
    std::memcpy(hp + l.sv_off, split, (size_t)pl.n_split * 4);
    std::memcpy(hp + l.rf_off, refine, (size_t)pl.n_refine * 4);
    std::memset(hp + l.rw_off, 0, (size_t)n_views * 4);
    std::memset(hp + l.c_off, 0, l.c_bytes);
    // the scratch is reused: this call's writes follow the previous call's launch; the node
    // table and pool are the last upload's
    rc = wait_for(h, s, rs.st.ev);
    if (!rc) rc = wait_for(h, s, h->ev_upload);
    if (rc) return rc;
    // an upload that rewrites what renders of an older table read waits for this slot's event,
    // which follows the previous launch too: keep the older version while that one may run
    rs.version = hipEventQuery(rs.st.ev) == hipSuccess ? h->version : std::min(rs.version, h->version);
    HIPCHK(h, hipMemcpyAsync(dp, hp, rec_bytes, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipEventRecord(h->na_copy, s));
    if (pl.n_skip)
        HIPCHK(h, launch_view_mask(h->g, (const DevView *)dp, n_views, h->table, h->n_cells, s));
    HIPCHK(h, launch_render(h->g, h->table, h->pool, h->brick_bytes, (const DevView *)dp, n_views,
                            pl.class_items, out ? (RenderCounters *)(dp + l.c_off) : nullptr,
                            h->capped ? h->flags : nullptr, s));
    HIPCHK(h, launch_combine((const DevView *)dp, (const int32_t *)(dp + l.sv_off), pl.n_split,
                             h->g.C, pl.split_modes, pl.max_split_pixels, s));
    HIPCHK(h, launch_refine_finish((const DevView *)dp, (const int32_t *)(dp + l.rf_off),
                                   pl.n_refine, h->g.C, pl.max_refine_pixels, s));
    if (out) {
        HIPCHK(h, hipMemcpyAsync(hp + l.sv_off, dp + l.sv_off, l.c_off + l.c_bytes - l.sv_off,
                                 hipMemcpyDeviceToHost, s));
        HIPCHK(h, hipStreamSynchronize(s));
        collect_stats(hp, l, n_views, out);
    }
    HIPCHK(h, hipEventRecord(rs.st.ev, s));
    rs.stream = s;
    if (ckpt_ws) ckpt_log_put(h, ckpt_ws, n_views, views);
    return OCT_OK;
}

int render_views_backward(oct_handle *h, int32_t n_views, const oct_view *views,
                          const float *const *dL_dimages, const void *ckpt_ws, float *dL_dctrl,
                          float *dL_dvoxels, void *stream)
{
    if (!h) return OCT_EINVAL;
    if (n_views < 1 || !views || !dL_dimages || !ckpt_ws || !dL_dctrl)
        return fail(h, OCT_EINVAL, "backward needs views, dL/dimages, the forward workspace and dL/dctrl");
    const VolGeom &g = h->g;
    {
        // the backward must see the octree and the views that the forward's record came from
        const CkptRec *r = nullptr;
        for (const auto &e : h->ckpt_log)
            if (e.ws == ckpt_ws) r = &e;
        if (!r)
            return fail(h, OCT_EINVAL, "the workspace was not filled by a render of this octree");
        if (r->version != h->version)
            return fail(h, OCT_EINVAL, "the octree changed (an upload or clear) since the forward "
                                       "render that filled the workspace");
        if (r->n_views != n_views || r->views_hash != views_hash(n_views, views))
            return fail(h, OCT_EINVAL, "the views differ from those of the forward render");
    }
    for (int i = 0; i < n_views; i++)
        if (!view_differentiable(views[i]))
            return fail(h, OCT_EINVAL, "the adjoint covers DVR without channel transforms and MIP, "
                                       "with missing bricks drawn as AVG");
    if (dL_dvoxels) {
        // voxel gradients flow through trilinear weights of level-0 bricks only
        for (int i = 0; i < n_views; i++)
            if (views[i].lod != 0) return fail(h, OCT_EINVAL, "voxel gradients need lod 0 views");
        const int G = g.grid[0];
        for (int z = 0; z < G; z++)
            for (int y = 0; y < G; y++)
                for (int x = 0; x < G; x++) {
                    const HCell &c = h->cells[cell_index(g, 0, x, y, z)];
                    if (c.inside && !(c.exists && c.state == kBrickState && c.dev_kind == kBrick))
                        return fail(h, OCT_EINVAL,
                                    "voxel gradients need every level-0 node to hold a current brick "
                                    "(threshold 0, everything inserted and uploaded)");
                }
    }
    HIPCHK(h, hipSetDevice(h->device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<DevView> dvs((size_t)n_views);
    std::vector<WgItem> items, mip_items;
    size_t ck_off = 0;
    const size_t dlut_floats = (size_t)g.C * 256 * 4;
    for (int i = 0; i < n_views; i++) {
        int rc = build_view(h, views[i], (float *)dL_dimages[i], dvs[i]);
        if (rc) return rc;
        const size_t npix = (size_t)views[i].width * views[i].height;
        dvs[i].image = nullptr;
        dvs[i].dimg = dL_dimages[i];
        dvs[i].user_index = i;
        if (views[i].mode == OCT_MODE_MIP) {
            // one lane per pixel through the samples at the recorded maxima
            dvs[i].amax = (int32_t *)((uint8_t *)ckpt_ws + ck_off);
            ck_off += view_ckpt_bytes(h, views[i]);
            const int tiles = dvs[i].tiles_x * ((views[i].height + OCT_TILE - 1) / OCT_TILE);
            const int tb = std::min(views[i].tile_begin, tiles);
            const int te = views[i].tile_count < 0 ? tiles : std::min(tiles, tb + views[i].tile_count);
            for (int t = tb; t < te; t += kRenderTilesPerWg) {
                WgItem w{};
                w.view = i;
                w.tile0 = t;
                w.ntiles = std::min(kRenderTilesPerWg, te - t);
                mip_items.push_back(w);
            }
            continue;
        }
        dvs[i].npos = view_npos(h, views[i]);
        dvs[i].ckpt = (float *)((uint8_t *)ckpt_ws + ck_off);
        dvs[i].nend = (int32_t *)((uint8_t *)ckpt_ws + ck_off + npix * dvs[i].npos * 4);
        ck_off += view_ckpt_bytes(h, views[i]);
        const int tiles = dvs[i].tiles_x * ((views[i].height + OCT_TILE - 1) / OCT_TILE);
        const int tb = std::min(views[i].tile_begin, tiles);
        const int te = views[i].tile_count < 0 ? tiles : std::min(tiles, tb + views[i].tile_count);
        // the forward's depth segments: each (tile group, segment) is walked by its own waves
        const int nsplit = te > tb ? view_segments(h, views[i]) : 1;
        dvs[i].nsplit = nsplit;
        if (nsplit > 1)
            dvs[i].part = (float *)((uint8_t *)ckpt_ws + ck_off - view_ckpt_bytes(h, views[i]) +
                                    view_ckpt_part_offset(h, views[i]));
        const int groups = (te - tb + kRenderTilesPerWg - 1) / kRenderTilesPerWg;
        for (int g0 = 0; g0 < groups; g0 += 8)   // segment order as in the forward
            for (int sg = 0; sg < nsplit; sg++)
                for (int gi = g0; gi < std::min(g0 + 8, groups); gi++) {
                    WgItem w{};
                    w.view = i;
                    w.tile0 = tb + gi * kRenderTilesPerWg;
                    w.ntiles = std::min(kRenderTilesPerWg, te - w.tile0);
                    w.seg = sg;
                    items.push_back(w);
                }
    }
    // device temporaries: per-view table gradients (MIP views)
    const size_t dl_bytes = ((size_t)n_views * dlut_floats * 4 + 255) & ~(size_t)255;
    if (dl_bytes > h->bw_tmp_cap) {
        // an earlier backward on any stream may still use the temporaries
        for (auto &r : h->rs)
            if (r.st.ev) HIPCHK(h, hipEventSynchronize(r.st.ev));
        HIPCHK(h, hipStreamSynchronize(s));
        if (h->bw_tmp) HIPCHK(h, hipFree(h->bw_tmp));
        h->bw_tmp = nullptr;
        h->bw_tmp_cap = 0;
        HIPCHK(h, hipMalloc(&h->bw_tmp, dl_bytes));
        h->bw_tmp_cap = dl_bytes;
    }
    float *dlut = (float *)h->bw_tmp;
    for (int i = 0; i < n_views; i++) dvs[i].dlut = dlut + (size_t)i * dlut_floats;
    // voxel gradients of DVR views first go to a scratch of 16-voxel blocks, added to
    // dL/dvoxels at the end: the corners that the lanes of a wave flush together then share
    // more 64-byte lines.  Lanes spread over the image plane and, by their entry points, along
    // the rays, so the block is 1 voxel along the axis closest to the first view's direction, 8
    // along the farthest and 2 along the other.  Volumes whose scratch would pass
    // kVoxBlockedMax go to dL/dvoxels directly.
    constexpr size_t kVoxBlockedMax = (size_t)4 << 30;
    int vg_shape = -1;
    if (dL_dvoxels && !items.empty()) {
        const float *f = dvs[(size_t)items[0].view].f;
        int ax[3] = {0, 1, 2};
        std::sort(ax, ax + 3, [&](int a, int b) {
            return std::fabs(f[a]) != std::fabs(f[b]) ? std::fabs(f[a]) > std::fabs(f[b]) : a < b;
        });
        int sh[3];
        sh[ax[0]] = 0;
        sh[ax[1]] = 1;
        sh[ax[2]] = 3;
        vg_shape = sh[0] + 8 * sh[1] + 64 * sh[2];
    }
    const size_t vg_bytes = vg_shape >= 0 ? voxgrad_blocked_floats(g, vg_shape) * sizeof(float) : 0;
    const bool vg_blocked = vg_shape >= 0 && vg_bytes <= kVoxBlockedMax;
    if (!vg_blocked) vg_shape = -1;
    if (vg_blocked && vg_bytes > h->vg_blk_cap) {
        for (auto &r : h->rs)
            if (r.st.ev) HIPCHK(h, hipEventSynchronize(r.st.ev));
        HIPCHK(h, hipStreamSynchronize(s));
        if (h->vg_blk) HIPCHK(h, hipFree(h->vg_blk));
        h->vg_blk = nullptr;
        h->vg_blk_cap = 0;
        HIPCHK(h, hipMalloc((void **)&h->vg_blk, vg_bytes));
        h->vg_blk_cap = vg_bytes;
    }

    const size_t n_dvr_items = items.size();
    items.insert(items.end(), mip_items.begin(), mip_items.end());
    const size_t v_bytes = dvs.size() * sizeof(DevView);
    const size_t i_off = (v_bytes + 255) & ~(size_t)255;
    const size_t i_bytes = items.size() * sizeof(WgItem);
    RenderSlot &rs = h->rs[h->next_rs];
    h->next_rs = (h->next_rs + 1) % kRenderSlots;
    int rc = stage_reserve(h, rs.st, i_off + i_bytes);
    if (!rc) rc = collect_kernel_time(h, rs);
    if (rc) return rc;
    rs.version = h->version;
    uint8_t *hp = (uint8_t *)rs.st.host;
    std::memcpy(hp, dvs.data(), v_bytes);
    std::memcpy(hp + i_off, items.data(), i_bytes);
    // the record copy runs on the prep stream, so that it overlaps the work queued before it
    if (!rs.prep) HIPCHK(h, hipEventCreateWithFlags(&rs.prep, hipEventDisableTiming));
    HIPCHK(h, hipMemcpyAsync(rs.st.dev, hp, i_off + i_bytes, hipMemcpyHostToDevice, h->prep));
    HIPCHK(h, hipEventRecord(rs.prep, h->prep));
    // the forward that wrote the checkpoints and every earlier backward (which shared the
    // table-gradient accumulators) may run on other streams: wait for
    // the last launch of every render slot (a slot's older launches ended before its reuse)
    rc = wait_for(h, s, rs.prep);
    if (!rc) rc = wait_for(h, s, h->ev_upload);
    if (!rc) rc = wait_for_renders(h, s);
    if (rc) return rc;
    if (!mip_items.empty()) HIPCHK(h, launch_fill_f32(dlut, (int64_t)n_views * dlut_floats, 0.0f, s));
    if (vg_blocked) HIPCHK(h, launch_fill_f32(h->vg_blk, (int64_t)(vg_bytes / sizeof(float)), 0.0f, s));
    uint8_t *dp = (uint8_t *)rs.st.dev;
    if (h->ktime && n_dvr_items) {
        if (!rs.k0) HIPCHK(h, hipEventCreate(&rs.k0));
        if (!rs.k1) HIPCHK(h, hipEventCreate(&rs.k1));
        HIPCHK(h, hipEventRecord(rs.k0, s));
    }
    HIPCHK(h, launch_render_backward(g, h->table, h->pool, h->brick_bytes, (const DevView *)dp,
                                     (const WgItem *)(dp + i_off), (int)n_dvr_items,
                                     vg_blocked ? h->vg_blk : dL_dvoxels, vg_shape, dL_dctrl, s));
    if (h->ktime && n_dvr_items) {
        HIPCHK(h, hipEventRecord(rs.k1, s));
        rs.k_pending = true;
    }
    HIPCHK(h, launch_render_backward_mip(g, h->table, h->pool, h->brick_bytes, (const DevView *)dp,
                                         (const WgItem *)(dp + i_off) + n_dvr_items,
                                         (int)mip_items.size(), dL_dvoxels, s));
    if (vg_blocked) HIPCHK(h, launch_voxgrad_unblock(g, vg_shape, h->vg_blk, dL_dvoxels, s));
    // MIP views accumulate table gradients (V.dlut); DVR views add to dL/dctrl directly
    if (!mip_items.empty()) HIPCHK(h, launch_lut_to_ctrl((const DevView *)dp, n_views, g.C, dL_dctrl, s));
    HIPCHK(h, hipEventRecord(rs.st.ev, s));
    rs.stream = s;
    return OCT_OK;
}

int octree_dump_canonical(oct_handle *h, void *buf, size_t cap, size_t *needed)
{
    if (!h || !needed) return OCT_EINVAL;
    HIPCHK(h, hipSetDevice(h->device));
    const VolGeom &g = h->g;
    const int C = g.C, M = g.M, S = M + 2;
    // pending inserts must be applied first so the dump reflects every inserted voxel
    for (int L = 0; L <= g.N; L++)
        if (!h->dirty[L].empty()) {
            int rc = brick_pool_upload(h, 0, nullptr, nullptr);
            if (rc < 0) return rc;
            break;
        }
    HIPCHK(h, hipDeviceSynchronize());
    int64_t n_nodes = 0, n_bricks = 0;
    for (int64_t i = 0; i < h->n_cells; i++)
        if (h->cells[i].exists) {
            n_nodes++;
            if (h->cells[i].state == kBrickState) n_bricks++;
        }
    const size_t bb = (size_t)S * S * S * C * h->esz;
    const size_t need = 64 + (size_t)n_nodes * 192 + (size_t)n_bricks * bb;
    *needed = need;
    if (!buf || cap < need) return fail(h, OCT_ERANGE, "dump buffer too small");
    uint8_t *o = (uint8_t *)buf;
    std::memset(o, 0, 64 + (size_t)n_nodes * 192);
    std::memcpy(o, "OCTDUMP1", 8);
    const int32_t hdr[9] = {g.dims[0], g.dims[1], g.dims[2], C, M, g.N, g.dtype, (int32_t)n_nodes,
                            (int32_t)n_bricks};
    std::memcpy(o + 8, hdr, sizeof hdr);
    uint8_t *rec = o + 64;
    uint8_t *bk = o + 64 + (size_t)n_nodes * 192;
    std::vector<uint8_t> slotbuf(h->brick_bytes);
    for (int L = g.N; L >= 0; L--) {
        const int G = g.grid[L];
        for (int z = 0; z < G; z++)
            for (int y = 0; y < G; y++)
                for (int x = 0; x < G; x++) {
                    const HCell &c = h->cells[cell_index(g, L, x, y, z)];
                    if (!c.exists) continue;
                    const bool resident = c.state == kBrickState && c.dev_kind == kBrick;
                    const int32_t head[8] = {L, x, y, z, c.state,
                                             (c.has_children ? 1 : 0) | (c.complete ? 2 : 0) |
                                                 (c.populated ? 4 : 0) | (resident ? 8 : 0),
                                             0, 0};
                    std::memcpy(rec, head, sizeof head);
                    double *d = (double *)(rec + 32);
                    for (int k = 0; k < C; k++) {
                        d[k] = c.avg[k];
                        if (c.populated) {
                            d[4 + k] = c.bmin[k];
                            d[8 + k] = c.bmax[k];
                            d[12 + k] = c.smin[k];
                            d[16 + k] = c.smax[k];
                        }
                    }
                    rec += 192;
                    if (c.state != kBrickState) continue;
                    int64_t slot = c.slot;
                    if (!resident) {
                        // gather the bordered brick into the spare slot past the pool
                        slot = h->n_slots + h->n_cow;
                        int rc = stage_reserve(h, h->up, 256 + gather_scratch_bytes(g, 1));
                        if (rc) return rc;
                        void *gscratch = (uint8_t *)h->up.dev + 256;
                        BrickJob j{};
                        j.slot = (int32_t)slot;
                        j.level = L;
                        j.bx = x;
                        j.by = y;
                        j.bz = z;
                        j.full = 1;
                        j.store = -1;
                        for (int a = 0; a < 3; a++) j.hi[a] = S - 1;
                        std::memcpy(h->up.host, &j, sizeof j);
                        HIPCHK(h, hipMemcpy(h->up.dev, h->up.host, sizeof j, hipMemcpyHostToDevice));
                        if (h->pc) {
                            const std::vector<BrickJob> one(1, j);
                            int rc2 = gather_paged(h, one, 0, 1, (const BrickJob *)h->up.dev,
                                                   h->table, gscratch, nullptr);
                            if (rc2) return rc2;
                        } else {
                            HIPCHK(h, launch_gather(g, h->master, h->table, h->pool, h->brick_bytes,
                                                    (const BrickJob *)h->up.dev, 1, h->slot_range,
                                                    h->background_f, gscratch, nullptr, nullptr, 0,
                                                    nullptr));
                        }
                        HIPCHK(h, hipDeviceSynchronize());
                    }
                    HIPCHK(h, hipMemcpy(slotbuf.data(), h->pool + (uint64_t)slot * h->brick_bytes,
                                        h->brick_bytes, hipMemcpyDeviceToHost));
                    for (int v = 0; v < S * S * S; v++)
                        for (int k = 0; k < C; k++) {
                            std::memcpy(bk, slotbuf.data() + ((size_t)v * 4 + k) * h->esz, h->esz);
                            bk += h->esz;
                        }
                }
    }
    return OCT_OK;
}

int octree_read_level(oct_handle *h, int32_t level, void *out, size_t cap, int32_t ext[3])
{
    if (!h || !out) return OCT_EINVAL;
    const VolGeom &g = h->g;
    if (level < 0 || level > g.N) return fail(h, OCT_EINVAL, "level out of range");
    HIPCHK(h, hipSetDevice(h->device));
    const size_t bytes = (size_t)(g.lvl_off[level + 1] - g.lvl_off[level]) * h->esz;
    if (ext)
        for (int a = 0; a < 3; a++) ext[a] = g.ext[level][a];
    if (cap < bytes) return fail(h, OCT_ERANGE, "buffer too small");
    HIPCHK(h, hipDeviceSynchronize());
    if (h->pc) {
        // disk tier: the level assembled page by page (RAM frame, file or background)
        const int P = 1 << g.plog, L = level;
        const int64_t ex = g.ext[L][0], ey = g.ext[L][1], ez = g.ext[L][2];
        std::vector<uint8_t> page(h->pc->page_bytes());
        const int64_t npz = (ez + P - 1) / P;
        for (int64_t pz = 0; pz < npz; pz++)
            for (int64_t py = 0; py < g.pgrid[L][1]; py++)
                for (int64_t px = 0; px < g.pgrid[L][0]; px++) {
                    const int64_t id = g.page_off[L] + (pz * g.pgrid[L][1] + py) * g.pgrid[L][0] + px;
                    std::string err;
                    if (!h->pc->read_page(id, page.data(), [h](uint64_t q) { pg_wait(h, q); }, err))
                        return fail(h, OCT_EDEVICE, err);
                    const int64_t nx = std::min<int64_t>(P, ex - px * P);
                    for (int c = 0; c < g.C; c++)
                        for (int64_t z = pz * P; z < std::min<int64_t>(ez, pz * P + P); z++)
                            for (int64_t y = py * P; y < std::min<int64_t>(ey, py * P + P); y++) {
                                const uint8_t *src = page.data() +
                                    ((((int64_t)c * P + (z - pz * P)) * P + (y - py * P)) * P) * (int64_t)h->esz;
                                uint8_t *dst = (uint8_t *)out +
                                    ((((int64_t)c * ez + z) * ey + y) * ex + px * P) * (int64_t)h->esz;
                                std::memcpy(dst, src, (size_t)nx * h->esz);
                            }
                }
        return OCT_OK;
    }
    HIPCHK(h, hipMemcpy(out, (uint8_t *)h->master + (size_t)g.lvl_off[level] * h->esz, bytes,
                        hipMemcpyDeviceToHost));
    return OCT_OK;
}

int octree_disk_stats(oct_handle *h, oct_disk_stats *out)
{
    if (!h || !out) return OCT_EINVAL;
    if (!h->pc) return fail(h, OCT_EINVAL, "the octree has no disk tier");
    const PageCache::Stats &st = h->pc->stats;
    out->pages = (uint64_t)h->pc->n_pages();
    out->frames = (uint64_t)h->pc->n_frames();
    out->hits = st.hits;
    out->loads = st.loads;
    out->fills = st.fills;
    out->writebacks = st.writebacks;
    out->evictions = st.evictions;
    out->waits = st.waits;
    out->bytes_read = st.bytes_read;
    out->bytes_written = st.bytes_written;
    return OCT_OK;
}

int octree_render_timing(oct_handle *h, int32_t enable, double *total_ms, uint64_t *launches)
{
    if (!h || (enable != 0 && enable != 1)) return h ? fail(h, OCT_EINVAL, "enable must be 0 or 1") : OCT_EINVAL;
    HIPCHK(h, hipSetDevice(h->device));
    for (auto &r : h->rs) {
        int rc = collect_kernel_time(h, r);
        if (rc) return rc;
    }
    if (total_ms) *total_ms = h->ktime_ms;
    if (launches) *launches = h->ktime_n;
    if (enable) {
        h->ktime_ms = 0.0;
        h->ktime_n = 0;
    }
    h->ktime = enable != 0;
    return OCT_OK;
}

int octree_build_timing(oct_handle *h, int32_t enable, double *ms, double *bytes)
{
    if (!h) return OCT_EINVAL;
    HIPCHK(h, hipSetDevice(h->device));
    for (const auto &r : h->btimed) {
        HIPCHK(h, hipEventSynchronize(r.e1));
        float t = 0.0f;
        HIPCHK(h, hipEventElapsedTime(&t, r.e0, r.e1));
        h->bt_ms[r.phase] += (double)t;
        h->bt_bytes[r.phase] += r.bytes;
        h->bt_free.push_back(r.e0);
        h->bt_free.push_back(r.e1);
    }
    h->btimed.clear();
    for (int k = 0; k < 4; k++) {
        if (ms) ms[k] = h->bt_ms[k];
        if (bytes) bytes[k] = h->bt_bytes[k];
    }
    h->btime = enable != 0;
    for (int k = 0; k < 4; k++) h->bt_ms[k] = h->bt_bytes[k] = 0.0;
    return OCT_OK;
}

int octree_info(const oct_handle *h, int32_t *levels, uint64_t *brick_bytes, uint64_t *pool_slots)
{
    if (!h) return OCT_EINVAL;
    if (levels) *levels = h->g.N + 1;
    if (brick_bytes) *brick_bytes = h->brick_bytes;
    if (pool_slots) *pool_slots = (uint64_t)h->n_slots;
    return OCT_OK;
}

const char *oct_last_error(const oct_handle *h)
{
    if (!h) return g_create_err.c_str();
    return h->err.c_str();
}

}  // extern "C"
