// Internal declarations shared by the runtime and the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace octrc {

constexpr int kMaxLevels = 16;
constexpr int kMaxC = 4;
constexpr int kMaxSplit = 16;   // depth segments per ray at most

// Kinds of a resolved node-table cell.  Every cell of the virtual complete tree has an entry:
// a cell whose node does not exist carries the AVG of its deepest existing ancestor, so a
// lookup never has to descend.
enum CellKind : int32_t { kAvg = 0, kBrick = 1, kBrickMissing = 2 };

// Device node-table entry, one per cell of every level (64 bytes, four 16-byte loads).
struct alignas(16) DevCell {
    int32_t kind;
    int32_t slot;
    int32_t pad0, pad1;
    float avg[4];   // AVG per channel (brick-less cells) -- value used for sampling
    float lo[4];    // lower bound of every value a sample inside the cell can take
    float hi[4];    // upper bound (bordered-brick range unioned over the subtree)
};
static_assert(sizeof(DevCell) == 64, "DevCell layout");

// Geometry of the volume, passed by value to kernels.
struct VolGeom {
    int32_t dims[3];
    int32_t C;
    int32_t M;
    int32_t N;
    int32_t dtype;
    int32_t mlog2;                 // log2(M) when M is a power of two, else -1
    int32_t ext[kMaxLevels][3];
    int64_t lvl_off[kMaxLevels];   // element offset of level L in the master buffer
    int32_t grid[kMaxLevels];      // cells per axis at level L = 2^(N-L)
    int32_t cell_off[kMaxLevels];  // offset of level L in the node table
    // disk tier (paged master): level L is cut into pages of P^3 voxels (P = 2^plog, a multiple
    // of M), pgrid[L] pages along x and y, page ids from page_off[L]; within a page the voxels
    // are planar per channel, [c][z][y][x].  plog = 0: the master is dense (lvl_off).
    int32_t plog;
    int32_t pgrid[kMaxLevels][2];
    int64_t page_off[kMaxLevels + 1];
};

// Where the build kernels find the master: dense levels, or the frame of each page (device
// addresses of the pinned RAM frames of the disk tier; only the pages of the current batch are
// valid).
template <typename T>
struct MasterRef {
    T *base;
    T *const *pages;
};

// Element (x, y, z) of channel c at level L; with kPaged, elements x .. x + k of a row stay in
// one page while x + k < the next multiple of P.
template <bool kPaged, typename T>
__host__ __device__ inline T *melem(const VolGeom &g, const MasterRef<T> &m, int L, int c, int x,
                                    int y, int z)
{
    if constexpr (kPaged) {
        const int pl = g.plog, pm = (1 << pl) - 1;
        const int64_t pid = g.page_off[L] +
                            ((int64_t)(z >> pl) * g.pgrid[L][1] + (y >> pl)) * g.pgrid[L][0] + (x >> pl);
        return m.pages[pid] + ((((int64_t)c << pl) + (z & pm)) << (2 * pl)) +
               ((int64_t)(y & pm) << pl) + (x & pm);
    } else {
        const int64_t plane = (int64_t)g.ext[L][0] * g.ext[L][1] * g.ext[L][2];
        return m.base + g.lvl_off[L] + (int64_t)c * plane +
               ((int64_t)z * g.ext[L][1] + y) * g.ext[L][0] + x;
    }
}

// Per-ray state of a refinement view (OCT_MISSING_REFINE), kept between passes: status 0 =
// not started (zero-filled memory), 1 = finished (acc is the result), 2 = waiting before
// position k for a missing brick.  acc = premultiplied colour and opacity (DVR) or the running
// per-channel maxima (MIP).
struct alignas(16) RefineState {
    float acc[4];
    int32_t k;
    int32_t status;
    int32_t pad[2];
};
static_assert(sizeof(RefineState) == 32, "RefineState layout");

// Render kernel classes: views are grouped by class in a launch (consecutive work items), and
// each class runs its own kernel, so the variants do not share one register allocation.
enum ViewClass : int32_t {
    kClassDvr = 0,      // emission-absorption, missing bricks drawn with AVG, no transforms
    kClassMip = 1,      // maximum intensity projection, otherwise as kClassDvr
    kClassGeneral = 2,  // channel transforms, full-frame fallback or refinement (either mode)
    kNumClasses = 3
};

// Per-view constants of one render launch (built on the host, read by every lane).
struct DevView {
    float eye[3];
    float f[3], r[3], u[3];
    float kx, ky, klod;
    float step;
    float ert;            // opacity at which a ray stops (>= 1: never)
    int32_t width, height, tiles_x;
    int32_t lod;          // fixed level, or -1 for the per-ray footprint level
    int32_t n_clip;
    int32_t skip;
    float clip[3][4];
    float ulo[kMaxC];     // u = (s - ulo) * uscale, u in [0, 255]
    float uscale[kMaxC];
    float tf_pos[kMaxC][8];
    float tf_rgba[kMaxC][8][4];
    float *image;
    // checkpoint workspace of this view (NULL: none): the transmittance before every
    // evaluated position k of every ray ([k][pixel], k < npos; from the start of the ray's depth
    // segment), after the last one (at k = the end position, rays not split), and the first
    // position not evaluated
    float *ckpt;
    int32_t *nend;
    int32_t npos;
    // forward without early termination or checkpoints: each ray is marched as nsplit depth
    // segments by different waves; segment s of a ray with n positions takes positions
    // [n s / nsplit, n (s+1) / nsplit) and writes (C, T) to part[s][pixel]; a combine pass
    // composites the segments front to back into the image
    int32_t nsplit;
    float *part;
    int32_t tile_begin, tile_end;   // tiles rendered by this launch (the combine pass's range)
    // forward launches: this view's work items are item_begin ... item_begin + groups * nsplit
    // - 1 of the grid (groups of kRenderTilesPerWg tiles; order in item_of)
    int32_t item_begin, groups;
    // [groups] the view's tile groups in dispatch order (longest estimated rays first), built
    // on the host and copied with the launch records.  NULL: index order
    int32_t *group_order;
    // adjoint only: dL/dimage of this view, dL/dtable accumulator [C][256][4]
    const float *dimg;
    float *dlut;
    // this view's transfer-function tables (value/slope and opacity prefix counts), built
    // on the host per launch and copied into LDS by every workgroup
    const void *tables;
    // views with skipping: one bit per node-table cell, set when the cell is transparent for
    // this view (built per launch by k_view_mask from the current table); NULL otherwise
    uint32_t *tmask;
    int32_t mode;        // OCT_MODE_DVR (0) or OCT_MODE_MIP (1)
    int32_t missing;     // OCT_MISSING_AVG (0), _FALLBACK (1) or _REFINE (2)
    int32_t xform_on;    // channel c samples at xform[c] applied to the position
    int32_t vclass;      // ViewClass
    int32_t user_index;  // position of the view in the caller's list
    float xform[kMaxC][3][4];
    RefineState *rstate; // refinement: [pixel] state kept between passes
    int32_t *rwait;      // refinement: rays of this view that waited in this launch
    // MIP with a checkpoint workspace: per pixel, per channel, the first position at which the
    // channel's maximum was reached (-1: no sample above the window's low end)
    int32_t *amax;
};

// One workgroup of a render launch: up to kRenderTilesPerWg tiles of one view (group_tile),
// one wave each.
#ifndef OCTRC_RENDER_WAVES
#define OCTRC_RENDER_WAVES 4
#endif
constexpr int kRenderTilesPerWg = OCTRC_RENDER_WAVES;
struct WgItem {
    int32_t view;
    int32_t tile0;
    int32_t ntiles;
    int32_t seg;      // depth segment of the rays (0 when the view is not split)
};

struct BrickJob {       // one bordered brick to (re)build, whole or a sub-box of it
    int32_t slot, level, bx, by, bz;
    int32_t full;       // 1: the sub-box is the whole bordered brick
    int32_t lo[3], hi[3];  // inclusive sub-box in bordered-brick coordinates 0..M+1
    int32_t store;      // whole bricks: also written to host brick store entry `store` (-1: no)
    int32_t pad[3];
};

// Host brick store (oct_create_params.host_bricks): entry e holds a bordered brick as C planes
// of (M+2)^3 elements (channels not padded), at e * store_bytes in pinned host memory; its
// value range (lo[4], hi[4]) in a device array.  A copy job moves entry `store` into `slot`.
struct CopyJob {
    int32_t slot, store;
};
static_assert(sizeof(BrickJob) == 64, "BrickJob layout");

struct CellStat {       // statistics of one cell over its valid voxels
    double mn[kMaxC], mx[kMaxC], sum[kMaxC];
    uint32_t ins[kMaxC];  // level 0 only: inserted voxels per channel
};

struct CellDelta {      // one change event applied to the node table
    int32_t index;
    int32_t kind;
    int32_t slot;
    int32_t pad;
    float avg[4];
    float lo[4], hi[4];  // kBrickMissing: bound of the brick's values (conservative skip range)
};
static_assert(sizeof(CellDelta) == 64, "CellDelta layout");

// Sample counters of a render launch, spread over kCounterSlots cache lines (a workgroup adds
// into slot blockIdx % kCounterSlots; the host sums the slots): one shared line would
// serialise the atomics of every wave of the launch.
constexpr int kCounterSlots = 64;
struct alignas(128) RenderCounters {
    unsigned long long rays, nominal, composited, trilinear;
};

// ---- launchers (build path) ----
// `master` is the dense master (g.plog == 0) or, for the disk tier, the device page table
// (void *[pages], the frame of every page the launch touches).
// Insert: the block's voxels in [C or 1][z][y][x] with row / slice / channel pitches
// src_pitch (elements); the region written is origin .. origin + size - 1.
hipError_t launch_insert(const VolGeom &g, void *master, uint8_t *mask, const void *src,
                         const int64_t src_pitch[3], int channel, const int32_t origin[3],
                         const int32_t size[3], hipStream_t s);
hipError_t launch_downsample(const VolGeom &g, void *master, int L, const int32_t lo[3],
                             const int32_t hi[3], hipStream_t s);
size_t stats_scratch_bytes(const VolGeom &g, int n);
hipError_t launch_stats(const VolGeom &g, const void *master, const uint8_t *mask,
                        const int32_t *cells /* (level, bx, by, bz) x n */, int n,
                        void *scratch /* stats_scratch_bytes */, CellStat *out, hipStream_t s);
hipError_t launch_apply_deltas(DevCell *table, float *miss_range, const CellDelta *d, int n,
                               hipStream_t s);
// scratch: gather_scratch_bytes(g, n) bytes of device memory (per-workgroup value ranges)
size_t gather_scratch_bytes(const VolGeom &g, int n);
// store / store_range / store_bytes: the host brick store (NULL when there is none).
hipError_t launch_gather(const VolGeom &g, const void *master, const DevCell *table,
                         void *pool, uint64_t brick_bytes, const BrickJob *jobs, int n,
                         float *slot_range, float background, void *scratch, uint8_t *store,
                         float *store_range, uint64_t store_bytes, hipStream_t s);
// Bricks from the host brick store into pool slots, with their value ranges.
hipError_t launch_copy_bricks(const VolGeom &g, void *pool, uint64_t brick_bytes,
                              const CopyJob *jobs, int n, const uint8_t *store,
                              const float *store_range, uint64_t store_bytes, float *slot_range,
                              hipStream_t s);
hipError_t launch_ranges(const VolGeom &g, DevCell *table, const float *slot_range,
                         const float *miss_range, hipStream_t s);
hipError_t launch_clear(const VolGeom &g, void *master, uint8_t *mask, double background,
                        hipStream_t s);
hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t s);
hipError_t launch_fill_u16(uint16_t *p, int64_t n, uint16_t v, hipStream_t s);
hipError_t launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s);

// ---- launchers (render path) ----
constexpr int kCkptStride = 64;   // depth segments of differentiable renders: whole blocks of this many positions

// flags (may be NULL): per node-table cell, set to 1 when a render interpolated the cell's
// resident brick and to 2 when it needed the cell's brick but found it missing.
// Views are ordered by class; class_items[k] .. class_items[k + 1] are the work items of class
// k (class_items[kNumClasses] = all items).
hipError_t launch_render(const VolGeom &g, const DevCell *table, const void *pool,
                         uint64_t brick_bytes, const DevView *views, int n_views,
                         const int32_t *class_items, RenderCounters *counters, uint8_t *flags,
                         hipStream_t s);
// Refinement views: when no ray of the view waited in this launch, write the states' results
// (DVR: the premultiplied colour; MIP: the classified, composited maxima) to the image.
hipError_t launch_refine_finish(const DevView *views, const int32_t *refine_views, int n_refine,
                                int C, int64_t max_pixels, hipStream_t s);
// Bytes of one view's tables for C channels (views[i].tables points at that many bytes, built
// on the host) and 32-bit words of one view's transparency mask over n_cells node-table cells
// (whole 64-cell groups).  Per launch, the mask kernel, after the last upload, fills the mask
// of every view with tmask != NULL from the node table `table`.
size_t view_tables_bytes(int C);
inline int64_t view_mask_words(int64_t n_cells) { return (n_cells + 63) / 64 * 2; }
hipError_t launch_view_mask(const VolGeom &g, const DevView *views, int n_views,
                            const DevCell *table, int64_t n_cells, hipStream_t s);
// Front-to-back composite of the depth segments of every split view into its image.
// modes: bit 0 = some split view is DVR, bit 1 = some split view is MIP.
hipError_t launch_combine(const DevView *views, const int32_t *split_views, int n_split,
                          int C, int modes, int64_t max_pixels, hipStream_t s);
// Adjoint of DVR views (from the transmittances their forward recorded); control-point
// gradients are added to dctrl [view][C][8][4] (views' user_index), voxel gradients (dvox not
// NULL) to dvox as [C][Dz][Dy][Dx] (shape < 0), or to a scratch of
// voxgrad_blocked_floats(g, shape) floats in blocks of 2^sx x 2^sy x 2^sz voxels (shape =
// sx + 8 sy + 64 sz) that launch_voxgrad_unblock then adds to dvox.
hipError_t launch_render_backward(const VolGeom &g, const DevCell *table, const void *pool,
                                  uint64_t brick_bytes, const DevView *views, const WgItem *items,
                                  int n_items, float *dvox, int shape, float *dctrl,
                                  hipStream_t s);
size_t voxgrad_blocked_floats(const VolGeom &g, int shape);
hipError_t launch_voxgrad_unblock(const VolGeom &g, int shape, const float *blk, float *dvox,
                                  hipStream_t s);
// Adjoint of MIP views: one lane per pixel, through the samples at the recorded maxima.
hipError_t launch_render_backward_mip(const VolGeom &g, const DevCell *table, const void *pool,
                                      uint64_t brick_bytes, const DevView *views,
                                      const WgItem *items, int n_items, float *dvox,
                                      hipStream_t s);
hipError_t launch_lut_to_ctrl(const DevView *views, int n_views, int C, float *dctrl,
                              hipStream_t s);

}  // namespace octrc
