/*
 * octree_rc.h -- C ABI of the MI355X (gfx950) multi-channel brick-octree ray caster.
 *
 * Method: Brix, Prassni & Hinrichs, "Visualization of Large Volumetric Multi-Channel Microscopy
 * Data Streams on Standard PCs".  A multi-channel volume is kept as a 3D mipmap of constant-size
 * bricks addressed by an octree that is built incrementally from inserted blocks (section
 * "Incremental Construction"), and rendered by front-to-back emission-absorption ray casting
 * with per-channel transfer functions (Algorithm 1, "Basic Ray-Casting").
 *
 * Conventions for every call:
 *  - Return value: OCT_OK (0) on success, OCT_INCOMPLETE (1) when the call succeeded but work
 *    remains (see brick_pool_upload), a negative OCT_E* code on failure.  No C++ exception
 *    crosses the ABI.  oct_last_error() gives a message for the last failure on a handle.
 *  - Invalid arguments return OCT_EINVAL before anything is changed.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Device work is
 *    enqueued on it in call order; calls that need results on the host say so.
 *  - Device pointers passed in are borrowed: they must stay valid until the stream has passed
 *    the call.  Host pointers are consumed before the call returns.
 *  - A handle is not thread-safe: calls on one handle must be serialised by the caller.
 *    Calls may use different streams: the library orders their device work as if all calls
 *    had been issued on one stream in call order (renders wait for the last upload; inserts
 *    for the last insert and upload; an upload for the last insert and upload, and -- only
 *    before it rewrites node table and brick pool -- for every render issued before it).
 *    Renders on different streams overlap each other, and an upload's statistics pass
 *    overlaps renders issued before it, so insertion of the next slices can proceed on one
 *    stream while another renders.
 *  - Coordinates: world space is level-0 voxel units; the volume occupies [0,Dx]x[0,Dy]x[0,Dz];
 *    voxel (x,y,z) has its centre at (x+1/2, y+1/2, z+1/2).  Volumes and blocks are planar per
 *    channel, [C][z][y][x], x fastest.
 */
#ifndef OCTREE_RC_H
#define OCTREE_RC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OCT_OK 0
#define OCT_INCOMPLETE 1
#define OCT_EINVAL (-1)
#define OCT_ENOMEM (-2)
#define OCT_ERANGE (-3)
#define OCT_EDEVICE (-4)
#define OCT_EBUSY (-5)

#define OCT_U16 0
#define OCT_F32 1
#define OCT_MAX_CHANNELS 4
#define OCT_MAX_CLIPS 3
#define OCT_TF_POINTS 8
#define OCT_TILE 8

/* oct_view.mode: how the samples of a ray are combined ("Basic Ray-Casting"). */
#define OCT_MODE_DVR 0   /* front-to-back emission-absorption (direct volume rendering)    */
#define OCT_MODE_MIP 1   /* maximum intensity projection: per channel the largest sample of
                            the ray is classified once; the C classified values are
                            composited in channel order; ert_alpha does not apply          */

/* oct_view.missing: how a sample is drawn whose brick is not in the device pool (capped
 * pools, "Brick Upload from RAM to GPU"). */
#define OCT_MISSING_AVG 0       /* the node's AVG ("Basic Ray-Casting")                     */
#define OCT_MISSING_FALLBACK 1  /* the resident brick of the first of the two coarser levels
                                   on the sample's path, else the AVG; all three bricks are
                                   requested ("Full-Frame Ray-Casting")                     */
#define OCT_MISSING_REFINE 2    /* the ray stops before the sample and waits in
                                   oct_view.refine_state; the next render_views of the same
                                   view resumes it; the image is written only by the pass in
                                   which no ray had to wait ("Refinement Ray-Casting")      */

typedef struct oct_handle oct_handle;

/* Volume description (section "CPU Data Structure", Eq. 1, and "Handling Volumes of Arbitrary
 * Dimensions"): the original dims are virtually extended to a cube M*2^N with the smallest N;
 * level L of the mipmap has valid extent ceil(D / 2^L) per axis.  Only the channel count and
 * the final resolution are needed up front ("Incremental Construction"). */
typedef struct {
    int32_t dims[3];            /* Dx, Dy, Dz of the original volume, each >= 1           */
    int32_t channels;           /* C, 1..4                                                */
    int32_t brick_size;         /* M, even, 2..128 (a brick holds M^3 voxels per channel)  */
    int32_t dtype;              /* OCT_U16 or OCT_F32                                      */
    double background;          /* value of not-yet-inserted voxels; an integer for u16   */
    double homog_threshold;     /* a node is homogeneous when max-min < threshold in every
                                   channel (strict); 0 keeps every brick                  */
    uint64_t device_pool_bytes; /* cap of the device brick pool; 0 = room for every brick.
                                   With a cap, bricks are paged in on request ("Data
                                   Transfer"): renders flag the brick nodes they used and
                                   the ones they needed but found missing (sampled with
                                   their AVG meanwhile); brick_pool_upload reads the flags
                                   and replaces least-recently-used slots, coarser levels
                                   first                                                  */
    int32_t master_on_host;     /* where the full-resolution mipmap lives:
                                   OCT_MASTER_HBM (0): device memory;
                                   OCT_MASTER_HOST (1): pinned host memory, read and
                                   written by the kernels over the host link;
                                   OCT_MASTER_DISK (2): the disk tier ("Brick Upload from
                                   Disk to RAM", Fig. 5): the levels are cut into pages of
                                   page_cells^3 cells, stored in the file disk_path; an LRU
                                   set of host_cache_bytes of them is held in frames (see
                                   disk_frames).  A page modified by insertion is written
                                   back before its frame is reused; a page that device work
                                   in flight still uses is not removed (the call waits for
                                   that work).  Needs M a power of two.                    */
    int32_t page_cells;         /* disk tier: cells per page edge, a power of two >= 2
                                   (0: 2); a page holds M*page_cells voxels per edge, all
                                   channels                                               */
    int32_t host_bricks;        /* 1: keep every whole bordered brick the library gathers in a
                                   host brick store (pinned host memory, channels unpadded;
                                   the paper's brick pool in RAM), so that a brick paged in
                                   again is copied as one contiguous block instead of being
                                   gathered from the mipmap.  Needs a capped device pool.   */
    int32_t disk_frames;        /* disk tier: where its page frames live.
                                   OCT_FRAMES_HOST (0): pinned host memory (the paper's RAM
                                   tier), read and written by the kernels over the host link;
                                   OCT_FRAMES_DEVICE (1): device memory; a page moves between
                                   the file and its frame through a pinned staging page, and
                                   the kernels read and write frames in HBM.  Must be 0
                                   without the disk tier.                                  */
    uint64_t host_cache_bytes;  /* disk tier: bytes of page frames (host or device memory,
                                   see disk_frames); must hold at least 16 pages (or every
                                   page)                                                  */
    const char *disk_path;      /* disk tier: the page file, created (truncated) by
                                   octree_create and removed by octree_destroy            */
} oct_create_params;

#define OCT_MASTER_HBM 0
#define OCT_MASTER_HOST 1
#define OCT_MASTER_DISK 2
#define OCT_FRAMES_HOST 0
#define OCT_FRAMES_DEVICE 1

/* Counters of the disk tier since octree_create (octree_disk_stats). */
typedef struct {
    uint64_t pages;             /* pages of the mipmap                                     */
    uint64_t frames;            /* RAM frames (pages held at once)                         */
    uint64_t hits;              /* page uses that found the page in RAM                    */
    uint64_t loads;             /* pages read from the file                                */
    uint64_t fills;             /* pages never written, set to the background in RAM       */
    uint64_t writebacks;        /* modified pages written to the file before eviction      */
    uint64_t evictions;         /* pages removed from RAM                                  */
    uint64_t waits;             /* evictions that waited for device work on the page       */
    uint64_t bytes_read;        /* file bytes read                                         */
    uint64_t bytes_written;     /* file bytes written                                      */
} oct_disk_stats;

/* One render request (Algorithm 1 and "Basic Ray-Casting").  Pinhole camera with square
 * pixels through pixel centres, row 0 at the top.  The image is premultiplied RGBA float32,
 * [height][width][4], not blended with any background. */
typedef struct {
    float eye[3], target[3], up[3];
    float fov_y_deg;            /* vertical field of view, (0, 180)                        */
    int32_t width, height;      /* image size, >= 1                                        */
    int32_t tile_begin;         /* first 8x8 tile (row-major over ceil(W/8) x ceil(H/8))   */
    int32_t tile_count;         /* number of tiles, -1 = to the end of the image           */
    float step;                 /* sample spacing in level-0 voxel units, > 0              */
    float ert_alpha;            /* stop a ray once its opacity >= ert_alpha; >= 1: never   */
    int32_t lod;                /* >= 0: fixed level (clamped to N); -1: per ray, the level
                                   whose voxel projects to about one pixel at the entry   */
    int32_t n_clip;             /* 0..3 clipping planes                                    */
    float clip[OCT_MAX_CLIPS][4]; /* (nx, ny, nz, d): keep points p with n.p >= d          */
    /* per-channel transfer function: 8 control points with ascending positions in [0,1] and
     * RGBA values; tabulated to 256 entries at x = k/255, linear in between, end values held */
    float tf_pos[OCT_MAX_CHANNELS][OCT_TF_POINTS];
    float tf_rgba[OCT_MAX_CHANNELS][OCT_TF_POINTS][4];
    float window[OCT_MAX_CHANNELS][2]; /* intensity (lo, hi) mapped to x = 0..1, hi > lo     */
    int32_t no_skip;            /* 1 disables empty-space skipping (same image, slower)    */
    int32_t depth_segments;     /* rays of a view without early termination (and without
                                   checkpoints) are marched as this many depth segments by
                                   different waves and composited afterwards, which shortens
                                   a launch's longest serial chain; 0 = automatic (one per
                                   256 positions of the volume diagonal, at most 5), 1 = one
                                   pass, at most 16.  Only compositing rounding differs
                                   between segment counts.                                */
    int32_t mode;               /* OCT_MODE_DVR or OCT_MODE_MIP                            */
    int32_t missing;            /* OCT_MISSING_AVG, _FALLBACK or _REFINE                   */
    int32_t n_xform;            /* 0, or C: channel c samples the volume at
                                   xform[c] (p) = M p + b instead of the ray position p
                                   ("Correction of Chromatic Aberration"); each row is
                                   evaluated as ((m0 p0 + m1 p1) + m2 p2) + b in float32   */
    int32_t reserved;           /* must be 0                                               */
    float xform[OCT_MAX_CHANNELS][3][4]; /* rows (m0, m1, m2, b) of each channel's map     */
    void *refine_state;         /* OCT_MISSING_REFINE only: device buffer of
                                   render_refine_bytes() bytes owned by the caller, zero-
                                   filled before the first pass of a new image and kept
                                   unchanged between the passes of one view               */
} oct_view;

typedef struct {
    uint64_t bricks_gathered;   /* bordered bricks (re)built by this call                  */
    uint64_t bricks_resident;   /* brick nodes with a current brick after the call         */
    uint64_t bricks_total;      /* brick nodes in the octree                               */
    uint64_t nodes_changed;     /* node-table entries rewritten (change events applied)    */
    uint64_t bytes_written;     /* device bytes written for bricks and node entries        */
    uint64_t requests_seen;     /* missing bricks the renders since the last call asked for */
    uint64_t evictions;         /* resident bricks replaced by this call                   */
    uint64_t bricks_from_store; /* of bricks_gathered: copied from the host brick store     */
} oct_upload_stats;

typedef struct {
    uint64_t rays;              /* pixels whose ray hits the clipped volume                */
    uint64_t positions_nominal; /* sample positions t_k < t1 over all rays                 */
    uint64_t positions_composited; /* positions actually sampled (not skipped, before ERT)  */
    uint64_t positions_trilinear;  /* of those, positions interpolated inside a brick       */
    uint64_t rays_waiting;      /* OCT_MISSING_REFINE views: rays stopped at a missing brick
                                   in this pass (their images were not written)            */
} oct_render_stats;

/* Creates the octree: the root node exists from the start and holds only the background
 * value, so the tree can be rendered at any time ("Incremental Construction").  Allocates the
 * device-resident mipmap, insertion mask, node table and brick pool.  *out receives the
 * handle (owned by the caller, released by octree_destroy).  Errors: OCT_EINVAL for a bad
 * parameter, OCT_ENOMEM when device memory runs out, OCT_EDEVICE on other HIP errors. */
int octree_create(const oct_create_params *params, void *stream, oct_handle **out);

/* Releases the handle and all memory it owns after synchronising its work. */
int octree_destroy(oct_handle *h);

/* Returns the octree to the state right after octree_create (background everywhere, only the
 * root node), keeping the allocations.  Enqueued on `stream`. */
int octree_clear(oct_handle *h, void *stream);

/* Inserts a cuboid block of voxels at an arbitrary position ("Incremental Construction",
 * step 1 and step 2): the block overwrites the level-0 voxels it covers (earlier values are
 * replaced) and every mipmap level above is re-half-sampled over the affected region,
 * integer mean rounded half up over the valid children (u16) or float32-rounded mean (f32).
 *   channel: 0..C-1 for one channel, or -1 for all channels at once
 *   origin:  x0, y0, z0 of the block; size: nx, ny, nz (each >= 1, block inside the volume)
 *   data:    planar [Cb][nz][ny][nx] in the volume's dtype, Cb = C or 1, x fastest
 *   data_is_device: 1 if `data` is device memory, 0 if host memory (copied before return)
 * Statistics, homogeneity decisions (step 3) and the node-table change events are applied
 * by the next brick_pool_upload.  Errors: OCT_EINVAL, OCT_ERANGE (block outside the volume),
 * OCT_EDEVICE. */
int octree_insert_block(oct_handle *h, int32_t channel, const int32_t origin[3],
                        const int32_t size[3], const void *data, int32_t data_is_device,
                        void *stream);

/* Slice-wise insertion, the streaming case of a slice-scanning microscope: inserts nz whole
 * z-slices starting at z0 (equivalent to octree_insert_block with origin (0,0,z0) and size
 * (Dx,Dy,nz)). */
int octree_insert_slices(oct_handle *h, int32_t channel, int32_t z0, int32_t nz,
                         const void *data, int32_t data_is_device, void *stream);

/* Applies everything inserted since the previous call to the render-side structures
 * ("Incremental Octree Updates on the GPU", "Filtering across Brick Boundaries", step 3 of
 * "Incremental Construction"): per-brick min/max/sum, homogeneity (only complete nodes are
 * merged), change events for created, deleted and updated nodes written into the device node
 * table, and bordered (M+2)^3 bricks gathered into the brick pool for every brick node whose
 * data or neighbourhood changed.  Synchronises `stream` once (statistics read-back).
 * byte_budget limits the bytes of bricks gathered by this call (0 = unlimited); when bricks
 * remain, the call returns OCT_INCOMPLETE and those nodes render with their AVG until a later
 * call gathers them.  With a capped pool (device_pool_bytes) brick nodes get slots only when
 * a render has requested them, coarser levels first, replacing the least recently used slots;
 * the call returns OCT_INCOMPLETE while requests remain unserved or gathers pending, and the
 * nodes concerned render with their AVG meanwhile.  `out` may be NULL.  Errors: OCT_ENOMEM
 * (a device or pinned allocation failed), OCT_EDEVICE. */
int brick_pool_upload(oct_handle *h, uint64_t byte_budget, void *stream, oct_upload_stats *out);

/* Renders n_views views in one launch (Algorithm 1 with accumulation-level intermixing of the
 * channels): each 8x8 tile of each view is one 64-lane wave.  images[i] is a device pointer
 * to [height][width][4] float32 for view i; only the tiles [tile_begin, tile_begin+count)
 * are written (for OCT_MISSING_REFINE views only by the pass in which no ray waited).
 * ckpt_ws: NULL, or a device workspace of render_ckpt_bytes() bytes that receives what
 * render_views_backward needs (the transmittance before every evaluated position; for MIP
 * views the position of each channel's maximum).  `out` (may be NULL) returns sample counts; passing it synchronises the
 * stream.  Views of any mode, missing-brick rule and transform may share a launch.
 * Errors: OCT_EINVAL (e.g. a refinement view without refine_state, n_xform other than 0 or
 * C, a refinement view with checkpoints), OCT_EDEVICE. */
int render_views(oct_handle *h, int32_t n_views, const oct_view *views, float *const *images,
                 void *ckpt_ws, void *stream, oct_render_stats *out);

/* render_views for callers that cannot allocate memory: code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation.  Same arguments, images and errors as
 * render_views, with these differences:
 *  - No allocation of any kind: the view records, sample counters, transfer-function tables,
 *    transparency masks and tile-group orders of the launch live in a fixed 16 MiB device
 *    scratch array that every GPU the library runs on holds until the process ends, and the
 *    host records in pinned memory that octree_create set aside.
 *  - At most 64 views per call; a launch whose tables, masks and orders do not fit the scratch
 *    returns OCT_ERANGE (before anything is enqueued) with the size it needed.
 *  - Views without a checkpoint workspace are marched in one pass (depth_segments is taken as
 *    1): the images equal render_views' images for the same views with depth_segments = 1 bit
 *    for bit, and other depth-segment counts within compositing rounding.  With ckpt_ws the
 *    call behaves as render_views (segment results live in the workspace).
 *  - All preparation runs on `stream` (no internal stream).  Successive calls on one handle are
 *    ordered by the library; calls on two handles of one GPU share that GPU's scratch, so
 *    calls that overlap in time on one GPU race and their results are undefined. */
int render_views_noalloc(oct_handle *h, int32_t n_views, const oct_view *views,
                         float *const *images, void *ckpt_ws, void *stream, oct_render_stats *out);

/* Bytes of checkpoint workspace render_views needs for these views (0 on bad arguments):
 * for a DVR view about 4 bytes per pixel per position of the longest possible ray (the volume
 * diagonal over the step, plus 3) plus 4 per pixel, and 16 per pixel per depth segment when
 * its rays are split (0.93 GB for 512x512 pixels over a 256^3 volume at step 0.5); for a MIP
 * view 16 per pixel. */
size_t render_ckpt_bytes(const oct_handle *h, int32_t n_views, const oct_view *views);

/* Bytes of refinement state for one view (32 per pixel; 0 on bad arguments).  The state holds
 * each ray's next position and its colour and opacity (or, for MIP, its running maxima) so far;
 * zero-filled memory starts every ray from its entry point. */
size_t render_refine_bytes(const oct_handle *h, const oct_view *view);

/* Adjoint of render_views for a scalar loss L(images): given dL/dimage per view (device,
 * [height][width][4] float32) and the workspace filled by the forward with the same views,
 * accumulates (adds) into
 *   dL_dctrl   device [n_views][C][8][4] float32: gradient w.r.t. tf_rgba (positions fixed)
 *   dL_dvoxels device [C][Dz][Dy][Dx] float32 or NULL: gradient w.r.t. the level-0 voxel
 *              values, defined for views with lod 0 on an octree whose level-0 nodes all hold
 *              bricks (threshold 0, everything inserted)
 * DVR views are differentiated through every position (walked back to front with the
 * transmittances the forward recorded); MIP views through the sample at which each channel first reaches its maximum
 * (with or without channel transforms).  DVR views with channel transforms and views whose
 * missing-brick rule is not OCT_MISSING_AVG are not differentiable here (OCT_EINVAL).
 * The workspace must have been filled by the last render_views call that used it, with the
 * same views, and no upload or clear that changed the octree may come between the two.
 * Voxel gradients of DVR views are first summed in a device scratch of the size of dL_dvoxels
 * (in 16-voxel blocks, allocated on first use and kept by the handle; volumes whose scratch
 * would pass 4 GiB are summed into dL_dvoxels directly), then added to dL_dvoxels.
 * Ordering: the backward follows every render and backward issued earlier on this handle, on
 * any stream (they share its table-gradient accumulators and gradient scratch).
 * Errors: OCT_EINVAL (e.g. voxel gradients requested where not defined, a workspace not filled
 * by a render of this handle, views that differ from the forward's, an octree changed since
 * the forward), OCT_EDEVICE. */
int render_views_backward(oct_handle *h, int32_t n_views, const oct_view *views,
                          const float *const *dL_dimages, const void *ckpt_ws, float *dL_dctrl,
                          float *dL_dvoxels, void *stream);

/* Canonical dump of the octree for parity checks (synchronises the device).
 * Layout (little endian): a 64-byte header "OCTDUMP1", int32 dims[3], C, M, N, dtype,
 * n_nodes, n_bricks; then one 192-byte record per existing node ordered by level descending,
 * then z, y, x: int32 level, bx, by, bz, state (0 empty, 1 homogeneous leaf, 2 homogeneous
 * with children, 3 brick), flags (1 has children, 2 complete, 4 populated, 8 resident), 0,
 * 0; float64 avg[4], bmin[4], bmax[4], smin[4], smax[4]; then the bordered (M+2)^3 brick of every brick
 * node in record order, channel-interleaved [z][y][x][C] in the dtype.  Flag 8 marks a brick
 * node whose brick is resident in the pool (renders interpolate it; a non-resident one is
 * sampled with its AVG).  Bricks that are not resident are gathered into a spare slot for
 * the dump.  With buf == NULL or cap too small only *needed is set and OCT_ERANGE returned. */
int octree_dump_canonical(oct_handle *h, void *buf, size_t cap, size_t *needed);

/* Counters of the disk tier ("Brick Upload from Disk to RAM"): page hits, loads from the
 * file, background fills, write-backs of modified pages, evictions and evictions that waited
 * for device work.  Errors: OCT_EINVAL for a null argument or a handle without the disk tier. */
int octree_disk_stats(oct_handle *h, oct_disk_stats *out);

/* Copies mipmap level `level` (planar [C][ez][ey][ex], dtype) to host memory `out` of `cap`
 * bytes; ext receives (ex, ey, ez).  Applies pending inserts first (synchronises). */
int octree_read_level(oct_handle *h, int32_t level, void *out, size_t cap, int32_t ext[3]);

/* Number of levels N+1 and the brick-pool slot size in bytes. */
int octree_info(const oct_handle *h, int32_t *levels, uint64_t *brick_bytes,
                uint64_t *pool_slots);

/* Render-kernel timing, for measurement.  Each call waits for the renders recorded so far and
 * returns in *total_ms / *launches (either may be NULL) their summed ray-casting kernel time
 * and count; then enable = 1 clears the totals and (re)starts recording -- every later
 * render_views records HIP events around its ray-casting kernel on the call's stream, and
 * every later render_views_backward around its kernel for DVR views -- and enable = 0 stops
 * recording.  The table and combine passes of a render are not included.
 * Errors: OCT_EINVAL, OCT_EDEVICE. */
int octree_render_timing(oct_handle *h, int32_t enable, double *total_ms, uint64_t *launches);

/* Build-kernel timing, for measurement.  Each call waits for the build work recorded so far and
 * returns in ms[4] its summed kernel time and in bytes[4] its algorithmic bytes, per phase:
 * [0] insertion into level 0 (block read, level-0 write, mask read and write), [1] half-sampling
 * of the levels above (children read, parents written), [2] statistics of the changed cells
 * (their valid voxels read, plus the mask at level 0), [3] bordered-brick gathers (the padded
 * pool voxels written and the source voxels read); either pointer may be NULL.  Then
 * enable = 1 clears the totals and (re)starts recording -- HIP events around those launches
 * on the calls' streams -- and enable = 0 stops it.  Errors: OCT_EINVAL, OCT_EDEVICE. */
int octree_build_timing(oct_handle *h, int32_t enable, double *ms, double *bytes);

/* Message describing the last failure on this handle (or of the last octree_create when h is
 * NULL); never NULL. */
const char *oct_last_error(const oct_handle *h);

#ifdef __cplusplus
}
#endif

#endif /* OCTREE_RC_H */
