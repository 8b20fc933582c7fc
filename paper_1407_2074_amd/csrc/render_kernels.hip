// Forward ray casting (Algorithm 1, "Basic Ray-Casting"), one 64-lane wave per 8x8 pixel tile
// (or per depth segment of a tile's rays), several tiles of one view per workgroup
// (kRenderTilesPerWg waves).
//
// Per launch, the host tabulates each view's transfer functions (256 RGBA value/slope pairs
// per channel, plus a prefix count of the entries with non-zero opacity) and the dispatch order
// of its tile groups, and k_view_mask turns the prefix counts into one bit per node-table cell: set when
// every value the cell can produce classifies to zero opacity in every channel.  Every render
// workgroup copies the value/slope table (and a small mask) into LDS; the mask drives the exact
// empty-space skipping (skipped positions would add exactly zero).
//
// Geometry follows the float32 operation sequence written in raycommon.h; this file is
// compiled without floating-point contraction.
#include "raycommon.h"

#include <float.h>

#include <algorithm>

namespace octrc {

namespace {

constexpr int kThreads = 64 * kRenderTilesPerWg;   // one wave per tile; the tiles share the tables

// Bit i of a view's transparency mask: from its LDS copy when one was staged (kLds), else
// from global memory.  (The choice is a template parameter: a run-time select between the two
// would make the compiler form generic pointers.)
template <bool kLds>
__device__ __forceinline__ bool mask_bit(const uint32_t *m, const uint32_t *lds, int i)
{
    uint32_t w;
    if constexpr (kLds) w = lds[i >> 5];
    else w = m[i >> 5];
    return (w >> (i & 31)) & 1u;
}

// Work item b of a forward launch.  The views' items are consecutive (item_begin); inside a
// view, tile groups go out in V.group_order (longest estimated rays first, so that the
// longest chains start early and short work fills the end of the launch), in blocks of 8
// groups, segment by segment, so that all segments of the j-th group land on XCD j mod 8
// (workgroups are dealt round-robin to the 8 XCDs; emitting a group's segments back to back
// would pin each segment to a fixed subset of XCDs whenever the segment count divides 8).

__device__ inline WgItem item_of(const DevView *__restrict__ views, int n_views, int b)
{
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {   // last view with item_begin <= b
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].item_begin <= b) lo = mid;
        else hi = mid - 1;
    }
    const DevView &V = views[lo];
    const int S = V.nsplit, j = b - V.item_begin;
    const int blk = j / (8 * S), r = j - blk * 8 * S;
    const int gcount = min(8, V.groups - 8 * blk);
    const int gs = 8 * blk + r % gcount;   // position in dispatch order
    const int gi = V.group_order ? V.group_order[gs] : gs;
    WgItem it;
    it.view = lo;
    // inside an XCD, consecutive workgroups go to its shader engines in turn: with an even
    // segment count the same segment of every group would land on the same engines (segments
    // differ in cost), so even counts rotate the segment order from block to block
    it.seg = (S & 1) ? r / gcount : (r / gcount + blk) % S;
    it.tile0 = V.tile_begin + gi * kRenderTilesPerWg;
    it.ntiles = min(kRenderTilesPerWg, V.tile_end - it.tile0);
    return it;
}

// kErt: the view may terminate rays early (otherwise the opacity test is left out of the
// march); kCount: sample counters are requested; kLdsMask: the transparency masks (mask_lds
// words each) are staged in LDS; kMip: maximum intensity projection instead of
// emission-absorption compositing.
//
// MIP keeps per channel the running maximum m_c, started at the window's low end lo_c (values
// at or below lo_c classify like lo_c, so max(lo_c, samples) gives the same image as the
// maximum of the samples), and the first position that raised it.  A cell whose upper value
// bound is at most m_c in every channel cannot change either, so its positions are skipped
// (the per-launch mask marks the cells bounded by lo_c; cells looked up are tested against the
// current m_c).  The result is the same with skipping on or off, bit for bit.
template <typename T, int C, bool kErt, bool kCount, bool kLdsMask, bool kMip = false>
__device__ __forceinline__ void
render_body(const VolGeom &g, const DevCell *__restrict__ table, const uint8_t *__restrict__ pool,
            uint64_t brick_bytes, const DevView *__restrict__ views, const WgItem &it,
            RenderCounters *counters, uint8_t *flags, LutTable<C> &tb, int mask_lds)
{

    // items stay in dispatch order: the hardware deals workgroups round-robin to the XCDs, which
    // spreads every part of the image over all of them (giving each XCD one contiguous band
    // measured 2x slower: the volume covers the bands unevenly)
    const DevView &V = views[it.view];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // a small transparency mask (mask_lds words, the same for every view of the launch) is
    // staged in LDS next to the table; the barrier of load_tables covers both copies
    extern __shared__ uint32_t smask[];
    if (kLdsMask && V.tmask)
        for (int i = threadIdx.x; i < mask_lds; i += kThreads) smask[i] = V.tmask[i];
    load_tables<kThreads>(V, tb);
    if (wave >= it.ntiles) return;  // no barrier below this point

    // uniform per-view constants, held in registers for the whole march
    float ulo[C], usc[C];
#pragma unroll
    for (int c = 0; c < C; c++) {
        usc[c] = V.uscale[c];
        ulo[c] = -V.ulo[c] * usc[c];   // table coordinate u = s * usc + ulo
    }
    const uint32_t *const tmask = V.tmask;
    const float step = V.step;
    // 1/step for position bounds (the exit of a skipped box, the inner range of an f32 cell),
    // which keep a margin of a whole step, far above the relative error of a product with the
    // rounded reciprocal
    const float rstep = 1.0f / step;
    const float ert_T = V.ert < 1.0f ? 1.0f - V.ert : -1.0f;
    const bool skip = V.skip != 0;
    float *const ckpt = V.ckpt;

    const int tile = group_tile(V, (it.tile0 - V.tile_begin) / kRenderTilesPerWg, wave);
    // lanes in Morton order over the 8x8 tile: each 16-lane quarter covers a 4x4 block
    const int mx = (lane & 1) | ((lane >> 1) & 2) | ((lane >> 2) & 4);
    const int my = ((lane >> 1) & 1) | ((lane >> 2) & 2) | ((lane >> 3) & 4);
    const int px_i = (tile % V.tiles_x) * 8 + mx;
    const int px_j = (tile / V.tiles_x) * 8 + my;
    const bool inside = px_i < V.width && px_j < V.height;
    const int64_t pix = (int64_t)px_j * V.width + px_i;
    const Ray ray = setup_ray(V, g, px_i, px_j, inside);
    const float *o = ray.o, *d = ray.d;
    const float t0 = ray.t0, t1 = ray.t1;
    const int L = ray.L;

    // ---- march
    const float scaleL = __builtin_ldexpf(1.0f, -L);
    const int S = g.M + 2;
    const int G = g.grid[L];
    const int coff = g.cell_off[L];
    const int csz = g.M << L;                          // cell edge in level-0 voxels
    const int csh = g.mlog2 >= 0 ? g.mlog2 + L : -1;   // log2(csz) when a power of two
    const float invd[3] = {d[0] != 0.0f ? 1.0f / d[0] : INFINITY,
                           d[1] != 0.0f ? 1.0f / d[1] : INFINITY,
                           d[2] != 0.0f ? 1.0f / d[2] : INFINITY};

    // positions t_k < t1 (the nominal count): from the estimate, settled with the exact test.
    // t_k grows with k, so the march tests k against it instead of comparing t_k with t1
    const bool split = V.nsplit > 1;
    int nominal = 0;
    if (ray.hit) {
        int kk = max((int)((t1 - t0) / step) - 2, 0);
        while (t0 + (float)kk * step < t1) kk++;
        nominal = kk;
    }
    // segment s of a split ray: positions [n s / S, n (s+1) / S) of its n positions; when
    // transmittances are recorded the bounds are whole 64-position blocks instead, blocks
    // [nb s / S, nb (s+1) / S) of nb = ceil(n / 64), as the adjoint walks them
    int k_begin = 0, k_end = nominal;
    if (split && ckpt) {
        const int nb = (nominal + kCkptStride - 1) / kCkptStride;
        k_begin = (int)(((int64_t)nb * it.seg) / V.nsplit) * kCkptStride;
        k_end = min((int)(((int64_t)nb * (it.seg + 1)) / V.nsplit) * kCkptStride, nominal);
    } else if (split) {
        k_begin = (int)(((int64_t)nominal * it.seg) / V.nsplit);
        k_end = (int)(((int64_t)nominal * (it.seg + 1)) / V.nsplit);
    }

    // transmittance and colour from the segment's start (the whole ray when not split)
    float Tr = 1.0f, Cr = 0.0f, Cg = 0.0f, Cb = 0.0f;
    int k = k_begin, composited = 0, trilinear = 0;
    const int64_t npix_ck = (int64_t)V.width * V.height;
    // How a position is found to lie in the cached cell. u16 bricks test the brick coordinates
    // of every position (few instructions, no per-cell set-up). f32 bricks keep the range of
    // positions k_lo..k_hi that lie at least 1/64 voxel inside the cell (and one step away from
    // its faces) and test the voxel only outside it: their march has no corner reuse and
    // measured 37 % slower with the coordinate test (0.88 vs 1.21 ms on 256^3 at 512^2).
    constexpr bool kCoordTest = sizeof(T) == 2;
    int blo[3] = {1, 1, 1}, bhi[3] = {0, 0, 0};  // cached cell, level-0 voxel box (inclusive)
    int k_lo = 1, k_hi = 0;
    bool brick = false;
    const uint8_t *base = nullptr;
    // brick coordinate of a position in the cached cell: p 2^-L - (cell origin - 1 border voxel
    // + 1/2 voxel); infinite while no cell is cached
    float bofs[3] = {INFINITY, INFINITY, INFINITY};
    const float lq_end = (float)g.M + 0.5f;
    const float imax = (float)(S - 2);                  // last corner-pair origin in the brick
    const uint32_t row8 = (uint32_t)S * 8u, slice8 = (uint32_t)(S * S) * 8u;
    float avg[C];
#pragma unroll
    for (int c = 0; c < C; c++) avg[c] = 0.0f;
    float mxv[C];    // MIP: running maxima (from the window's low end) and their positions
    int kmv[C];
#pragma unroll
    for (int c = 0; c < C; c++) {
        mxv[c] = V.ulo[c];
        kmv[c] = -1;
    }

    // skip the positions inside the box of cell (ax, ay, az) at level lev: jump to just before
    // its exit (one whole step of margin: every skipped position lies inside the box) and
    // forget the cached cell
    auto jump_box = [&](int lev, int ax, int ay, int az) {
        const int e = g.M << lev;
        const int bl[3] = {ax * e, ay * e, az * e};
        float te = INFINITY;
#pragma unroll
        for (int q = 0; q < 3; q++) {
            const float plane = d[q] > 0.0f ? (float)(bl[q] + e) : (float)bl[q];
            if (d[q] != 0.0f) te = fminf(te, (plane - o[q]) * invd[q]);
        }
        const float kf = floorf((te - t0) * rstep) - 1.0f;
        k = (kf > (float)(k + 1)) ? (int)fminf(kf, 2.0e9f) : k + 1;
        bofs[0] = INFINITY;   // no cell cached: the next position looks its cell up
        blo[0] = 1;
        bhi[0] = 0;
        k_lo = 1;
        k_hi = 0;
    };

    // the 8 corners of the last trilinear sample (bordered-brick byte offset last_off):
    // consecutive positions often fall between the same 8 voxels, and the loads are what the
    // texture data path is busiest with
    uint32_t last_off = 0xffffffffu;
    uint2 c000 = {0, 0}, c100 = {0, 0}, c010 = {0, 0}, c110 = {0, 0};
    uint2 c001 = {0, 0}, c101 = {0, 0}, c011 = {0, 0}, c111 = {0, 0};
    bool live = ray.hit;
    while (live) {
        if (k >= k_end) break;
        const float tk = t0 + (float)k * step;
        // transmittance before every evaluated position (positions skipped as transparent
        // keep it unchanged, and the adjoint carries it across them)
        if (ckpt) ckpt[(int64_t)k * npix_ck + pix] = Tr;
        float p[3];
#pragma unroll
        for (int q = 0; q < 3; q++) {
            const float m = tk * d[q];
            p[q] = o[q] + m;
        }
        // brick coordinates of the position in the cached cell (also those of the sample). The
        // cell holds the position's clamped voxel whenever all three lie in [1/2, M + 1/2):
        // the single rounding of p 2^-L - bofs is monotone and both bounds are floats, so a
        // coordinate can pass only if its exact value passes, or, just below 1/2, where the
        // position lies just below the volume's low face and its voxel is clamped into this
        // cell anyway. A position that fails (a new cell, or one clamped back into the same
        // cell from outside the volume) looks its cell up again, which gives the same sample.
        float lq[3];
        bool lookup = false;
        int v[3];   // the clamped voxel of the position (when looked up)
        if constexpr (kCoordTest) {
#pragma unroll
            for (int q = 0; q < 3; q++) lq[q] = __builtin_fmaf(p[q], scaleL, -bofs[q]);
            lookup = !(fminf(fminf(lq[0], lq[1]), lq[2]) >= 0.5f &&
                       fmaxf(fmaxf(lq[0], lq[1]), lq[2]) < lq_end);
            if (lookup)
#pragma unroll
                for (int q = 0; q < 3; q++)
                    v[q] = min(max((int)floorf(p[q]), 0), g.dims[q] - 1);
        } else if (k < k_lo || k > k_hi) {
#pragma unroll
            for (int q = 0; q < 3; q++) v[q] = min(max((int)floorf(p[q]), 0), g.dims[q] - 1);
            lookup = v[0] < blo[0] || v[0] > bhi[0] || v[1] < blo[1] || v[1] > bhi[1] ||
                     v[2] < blo[2] || v[2] > bhi[2];
        }
        if (lookup) {
            // the cell of the clamped voxel at level L
            int cx, cy, cz;
            if (csh >= 0) {
                cx = v[0] >> csh;
                cy = v[1] >> csh;
                cz = v[2] >> csh;
            } else {
                cx = v[0] / csz;
                cy = v[1] / csz;
                cz = v[2] / csz;
            }
            const int cidx = coff + (cz * G + cy) * G + cx;
            if (skip && mask_bit<kLdsMask>(tmask, smask, cidx)) {
                // widen to the largest transparent ancestor, jump to just before its exit
                int lev = L, ax = cx, ay = cy, az = cz;
                while (lev < g.N) {
                    const int pg = g.grid[lev + 1];
                    if (!mask_bit<kLdsMask>(tmask, smask, g.cell_off[lev + 1] +
                                             ((az >> 1) * pg + (ay >> 1)) * pg + (ax >> 1)))
                        break;
                    lev++;
                    ax >>= 1;
                    ay >>= 1;
                    az >>= 1;
                }
                jump_box(lev, ax, ay, az);
                continue;
            }
            const DevCell &cell = table[cidx];
            if constexpr (kMip) {
                if (skip) {
                    // no sample of this cell can raise a running maximum
                    const float4 ch4 = *(const float4 *)cell.hi;
                    const float chi[4] = {ch4.x, ch4.y, ch4.z, ch4.w};
                    bool below = true;
#pragma unroll
                    for (int c = 0; c < C; c++) below = below && chi[c] <= mxv[c];
                    if (below) {
                        jump_box(L, cx, cy, cz);
                        continue;
                    }
                }
            }
            bofs[0] = (float)(cx * g.M) - 0.5f;
            bofs[1] = (float)(cy * g.M) - 0.5f;
            bofs[2] = (float)(cz * g.M) - 0.5f;
            const int2 ks = *(const int2 *)&cell.kind;
            brick = ks.x == kBrick;
            if (flags && ks.x != kAvg) flags[cidx] = brick ? 1 : 2;  // used / requested
            if (brick) {
                last_off = 0xffffffffu;   // another brick: reload
                base = pool + (uint64_t)ks.y * brick_bytes;
            } else {
                const float4 av = *(const float4 *)cell.avg;
                const float a4[4] = {av.x, av.y, av.z, av.w};
#pragma unroll
                for (int c = 0; c < C; c++) avg[c] = a4[c];
            }
            if constexpr (kCoordTest) {
#pragma unroll
                for (int q = 0; q < 3; q++) lq[q] = __builtin_fmaf(p[q], scaleL, -bofs[q]);
            } else {
                blo[0] = cx * csz; bhi[0] = blo[0] + csz - 1;
                blo[1] = cy * csz; bhi[1] = blo[1] + csz - 1;
                blo[2] = cz * csz; bhi[2] = blo[2] + csz - 1;
                // positions safely inside the cell: the box shrunk by 1/64 voxel per face
                float tin = -INFINITY, tout = INFINITY;
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    if (d[q] != 0.0f) {
                        const float pa = ((float)blo[q] + 0.015625f - o[q]) * invd[q];
                        const float pb = ((float)(bhi[q] + 1) - 0.015625f - o[q]) * invd[q];
                        tin = fmaxf(tin, fminf(pa, pb));
                        tout = fminf(tout, fmaxf(pa, pb));
                    }
                }
                const float klo = ceilf((tin - t0) * rstep) + 1.0f;
                const float khi = floorf((tout - t0) * rstep) - 1.0f;
                k_lo = klo > (float)k ? (int)fminf(klo, 2.0e9f) : k;
                k_hi = khi > (float)k ? (int)fminf(khi, 2.0e9f) : -1;
            }
        }
        if constexpr (kCount) composited++;
        float s[C];
        if (brick) {
            if constexpr (kCount) trilinear++;
            float f[3];
            int ii[3];
            if constexpr (!kCoordTest)
#pragma unroll
                for (int q = 0; q < 3; q++) lq[q] = __builtin_fmaf(p[q], scaleL, -bofs[q]);
#pragma unroll
            for (int q = 0; q < 3; q++) {
                f[q] = __builtin_amdgcn_fractf(lq[q]);
                // inside the node, lq lies in [0.5, M + 0.5); the clamp only guards the
                // bordered brick against addressing outside itself (truncation of a
                // non-negative value is its floor)
                ii[q] = (int)__builtin_amdgcn_fmed3f(lq[q], 0.0f, imax);
            }
            // byte offset in the brick, 24-bit multiplies (a bordered brick is < 16 MiB)
            const uint32_t off = __umul24((uint32_t)ii[2], slice8) +
                                 __umul24((uint32_t)ii[1], row8) + ((uint32_t)ii[0] << 3);
            if constexpr (sizeof(T) == 2) {
                if (off != last_off) {
                    const uint8_t *a0 = base + off;
                    const uint8_t *a1 = a0 + slice8;
                    c000 = *(const uint2 *)(a0);
                    c100 = *(const uint2 *)(a0 + 8);
                    c010 = *(const uint2 *)(a0 + row8);
                    c110 = *(const uint2 *)(a0 + row8 + 8);
                    c001 = *(const uint2 *)(a1);
                    c101 = *(const uint2 *)(a1 + 8);
                    c011 = *(const uint2 *)(a1 + row8);
                    c111 = *(const uint2 *)(a1 + row8 + 8);
                    last_off = off;
                }
                const uint2 w000 = c000, w100 = c100, w010 = c010, w110 = c110;
                const uint2 w001 = c001, w101 = c101, w011 = c011, w111 = c111;
#pragma unroll
                for (int c = 0; c < C; c++) {
                    auto ch = [&](const uint2 &w) -> float {
                        const uint32_t word = (c < 2) ? w.x : w.y;
                        return (float)((c & 1) ? (word >> 16) : (word & 0xffffu));
                    };
                    const float c00 = lerpf(ch(w000), ch(w100), f[0]);
                    const float c10 = lerpf(ch(w010), ch(w110), f[0]);
                    const float c01 = lerpf(ch(w001), ch(w101), f[0]);
                    const float c11 = lerpf(ch(w011), ch(w111), f[0]);
                    s[c] = lerpf(lerpf(c00, c10, f[1]), lerpf(c01, c11, f[1]), f[2]);
                }
            } else {
                const float4 *a0 = (const float4 *)(base + 2u * off);   // 16-byte voxels
                const float4 *a1 = a0 + S * S;
                const float4 w000 = a0[0], w100 = a0[1], w010 = a0[S], w110 = a0[S + 1];
                const float4 w001 = a1[0], w101 = a1[1], w011 = a1[S], w111 = a1[S + 1];
#pragma unroll
                for (int c = 0; c < C; c++) {
                    auto ch = [&](const float4 &w) -> float {
                        return c == 0 ? w.x : c == 1 ? w.y : c == 2 ? w.z : w.w;
                    };
                    const float c00 = lerpf(ch(w000), ch(w100), f[0]);
                    const float c10 = lerpf(ch(w010), ch(w110), f[0]);
                    const float c01 = lerpf(ch(w001), ch(w101), f[0]);
                    const float c11 = lerpf(ch(w011), ch(w111), f[0]);
                    s[c] = lerpf(lerpf(c00, c10, f[1]), lerpf(c01, c11, f[1]), f[2]);
                }
            }
        } else {
#pragma unroll
            for (int c = 0; c < C; c++) s[c] = avg[c];
        }
        if constexpr (kMip) {
#pragma unroll
            for (int c = 0; c < C; c++)
                if (s[c] > mxv[c]) {
                    mxv[c] = s[c];
                    kmv[c] = k;
                }
        } else {
            // classification and front-to-back compositing, channels in order
#pragma unroll
            for (int c = 0; c < C; c++) {
                const Classified q = classify(s[c], ulo[c], usc[c], tb.lut[c]);
                const float al = __builtin_fmaf(q.fr, q.de.w, q.e0.w);
                const float wgt = Tr * al;
                Cr = __builtin_fmaf(wgt, __builtin_fmaf(q.fr, q.de.x, q.e0.x), Cr);
                Cg = __builtin_fmaf(wgt, __builtin_fmaf(q.fr, q.de.y, q.e0.y), Cg);
                Cb = __builtin_fmaf(wgt, __builtin_fmaf(q.fr, q.de.z, q.e0.z), Cb);
                Tr = Tr - wgt;
            }
        }
        if constexpr (kErt)
            if (Tr <= ert_T) live = false;  // early ray termination after this position
        k++;
    }

    if (kMip && inside) {
        if (split) {
            // this segment's maxima for the combine pass (-inf: the ray misses the volume)
            float m4[4] = {-INFINITY, -INFINITY, -INFINITY, -INFINITY};
            if (ray.hit)
#pragma unroll
                for (int c = 0; c < C; c++) m4[c] = mxv[c];
            const int64_t npix = (int64_t)V.width * V.height;
            *(float4 *)(V.part + ((int64_t)it.seg * npix + pix) * 4) =
                make_float4(m4[0], m4[1], m4[2], m4[3]);
        } else {
            if (ray.hit) {
                // the classified maxima, composited in channel order
#pragma unroll
                for (int c = 0; c < C; c++) {
                    const Classified q = classify(mxv[c], ulo[c], usc[c], tb.lut[c]);
                    const float wgt = Tr * __builtin_fmaf(q.fr, q.de.w, q.e0.w);
                    Cr = __builtin_fmaf(wgt, __builtin_fmaf(q.fr, q.de.x, q.e0.x), Cr);
                    Cg = __builtin_fmaf(wgt, __builtin_fmaf(q.fr, q.de.y, q.e0.y), Cg);
                    Cb = __builtin_fmaf(wgt, __builtin_fmaf(q.fr, q.de.z, q.e0.z), Cb);
                    Tr = Tr - wgt;
                }
            }
            *(float4 *)(V.image + pix * 4) = make_float4(Cr, Cg, Cb, 1.0f - Tr);
            if (V.amax) {
                int a4[4] = {-1, -1, -1, -1};
#pragma unroll
                for (int c = 0; c < C; c++) a4[c] = kmv[c];
                *(int4 *)(V.amax + pix * 4) = make_int4(a4[0], a4[1], a4[2], a4[3]);
            }
        }
    } else if (inside) {
        if (split) {
            // this segment's premultiplied colour and transmittance, for the combine pass
            const int64_t npix = (int64_t)V.width * V.height;
            *(float4 *)(V.part + ((int64_t)it.seg * npix + pix) * 4) = make_float4(Cr, Cg, Cb, Tr);
        } else {
            *(float4 *)(V.image + pix * 4) = make_float4(Cr, Cg, Cb, 1.0f - Tr);
        }
        // first position not evaluated: after early termination k, otherwise the end of the
        // ray (a skip may have jumped past it); a split ray (no early termination) ends at n
        const int n_end = ray.hit ? (live ? nominal : k) : 0;
        if (V.nend && it.seg == 0) V.nend[pix] = n_end;
        // and the transmittance after the last evaluated position (a split ray's segment keeps
        // it in its partial result)
        if (ckpt && !split) ckpt[(int64_t)n_end * npix_ck + pix] = Tr;
    }
    if (kCount && counters) {
        const bool first = it.seg == 0;   // rays and nominal positions counted once
        unsigned long long r = (ray.hit && first) ? 1ull : 0ull,
                           nn = first ? (unsigned long long)nominal : 0ull,
                           cc = (unsigned long long)composited, tt = (unsigned long long)trilinear;
        for (int off = 32; off > 0; off >>= 1) {
            r += __shfl_xor(r, off, 64);
            nn += __shfl_xor(nn, off, 64);
            cc += __shfl_xor(cc, off, 64);
            tt += __shfl_xor(tt, off, 64);
        }
        if (lane == 0) {
            RenderCounters *cs = counters + (blockIdx.x & (kCounterSlots - 1));
            atomicAdd(&cs->rays, r);
            atomicAdd(&cs->nominal, nn);
            atomicAdd(&cs->composited, cc);
            atomicAdd(&cs->trilinear, tt);
        }
    }
}

// One render work item: the march specialised for the view's early termination and for
// sample counters (both uniform over the workgroup); kMip: the MIP class (no termination).
template <typename T, int C, bool kLdsMask, bool kMip>
__device__ __forceinline__ void
render_item(const VolGeom &g, const DevCell *__restrict__ table, const uint8_t *__restrict__ pool,
            uint64_t brick_bytes, const DevView *__restrict__ views, int n_views, int item,
            RenderCounters *counters, uint8_t *flags, LutTable<C> &tb, int mask_lds)
{
    const WgItem it = item_of(views, n_views, item);
    if constexpr (kMip) {
        if (counters)
            render_body<T, C, false, true, kLdsMask, true>(g, table, pool, brick_bytes, views, it,
                                                           counters, flags, tb, mask_lds);
        else
            render_body<T, C, false, false, kLdsMask, true>(g, table, pool, brick_bytes, views,
                                                            it, counters, flags, tb, mask_lds);
    } else {
        if (counters)
            render_body<T, C, true, true, kLdsMask>(g, table, pool, brick_bytes, views, it,
                                                    counters, flags, tb, mask_lds);
        else if (views[it.view].ert < 1.0f)
            render_body<T, C, true, false, kLdsMask>(g, table, pool, brick_bytes, views, it,
                                                     counters, flags, tb, mask_lds);
        else
            render_body<T, C, false, false, kLdsMask>(g, table, pool, brick_bytes, views, it,
                                                      counters, flags, tb, mask_lds);
    }
}

// uint16 bricks: registers for 5 waves per SIMD (6 fit only with spills, measured 2 % slower);
// float32 bricks (twice the corner data) keep the compiler's choice.  item_base: the first
// work item of this kernel's view class.
#ifndef OCTRC_U16_WAVES_PER_EU
#define OCTRC_U16_WAVES_PER_EU 5
#endif
template <int C, bool kLdsMask, bool kMip>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(OCTRC_U16_WAVES_PER_EU)))
k_render_u16(VolGeom g, const DevCell *__restrict__ table, const uint8_t *__restrict__ pool,
             uint64_t brick_bytes, const DevView *__restrict__ views,
             int n_views, int item_base, RenderCounters *counters, uint8_t *flags, int mask_lds)
{
    __shared__ LutTable<C> tb;
    render_item<uint16_t, C, kLdsMask, kMip>(g, table, pool, brick_bytes, views, n_views,
                                             item_base + (int)blockIdx.x, counters, flags, tb,
                                             mask_lds);
}

template <int C, bool kLdsMask, bool kMip>
__global__ void __launch_bounds__(kThreads)
k_render_f32(VolGeom g, const DevCell *__restrict__ table, const uint8_t *__restrict__ pool,
             uint64_t brick_bytes, const DevView *__restrict__ views,
             int n_views, int item_base, RenderCounters *counters, uint8_t *flags, int mask_lds)
{
    __shared__ LutTable<C> tb;
    render_item<float, C, kLdsMask, kMip>(g, table, pool, brick_bytes, views, n_views,
                                          item_base + (int)blockIdx.x, counters, flags, tb,
                                          mask_lds);
}

// ---------------------------------------------------------------------------------------
// General march (class kClassGeneral): per-channel sample transforms ("Correction of
// Chromatic Aberration"), the full-frame fallback ("Full-Frame Ray-Casting") and refinement
// ("Refinement Ray-Casting"), in either compositing mode, one pass per ray.  A lookup group
// -- all channels at the ray position, or (kXf) each channel at its own transformed position
// -- caches the node-table cell of its last sample and how that cell is drawn.
enum : int { kDrawAvg = 0, kDrawBrick = 1, kDrawNone = 2, kDrawWait = 3 };

template <int C>
struct LookupGroup {
    int cidx = -1;               // cached cell at the ray's level
    int draw = kDrawAvg;
    float sscale = 1.0f;         // sampling level Ls: 2^-Ls
    float sb[3] = {0.0f, 0.0f, 0.0f};  // brick coordinate = p 2^-Ls - sb
    const uint8_t *base = nullptr;
    float avg[C];
};

template <typename T, int C, bool kXf, bool kLdsMask, bool kCount>
__device__ __forceinline__ void
render_general_body(const VolGeom &g, const DevCell *__restrict__ table,
                    const uint8_t *__restrict__ pool, uint64_t brick_bytes,
                    const DevView *__restrict__ views, const WgItem &it, RenderCounters *counters,
                    uint8_t *flags, LutTable<C> &tb, int mask_lds)
{
    const DevView &V = views[it.view];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    extern __shared__ uint32_t smask[];
    if (kLdsMask && V.tmask)
        for (int i = threadIdx.x; i < mask_lds; i += kThreads) smask[i] = V.tmask[i];
    load_tables<kThreads>(V, tb);
    if (wave >= it.ntiles) return;  // no barrier below this point

    float ulo[C], usc[C];
#pragma unroll
    for (int c = 0; c < C; c++) {
        usc[c] = V.uscale[c];
        ulo[c] = -V.ulo[c] * usc[c];
    }
    const uint32_t *const tmask = V.tmask;
    const float step = V.step, rstep = 1.0f / step;
    const bool mip = V.mode == 1;
    const int missing = V.missing;
    const float ert_T = (!mip && V.ert < 1.0f) ? 1.0f - V.ert : -1.0f;
    const bool skip = V.skip != 0;

    const int tile = group_tile(V, (it.tile0 - V.tile_begin) / kRenderTilesPerWg, wave);
    const int mx_ = (lane & 1) | ((lane >> 1) & 2) | ((lane >> 2) & 4);
    const int my_ = ((lane >> 1) & 1) | ((lane >> 2) & 2) | ((lane >> 3) & 4);
    const int px_i = (tile % V.tiles_x) * 8 + mx_;
    const int px_j = (tile / V.tiles_x) * 8 + my_;
    const bool inside = px_i < V.width && px_j < V.height;
    const int64_t pix = (int64_t)px_j * V.width + px_i;
    const Ray ray = setup_ray(V, g, px_i, px_j, inside);
    const float *o = ray.o, *d = ray.d;
    const float t0 = ray.t0, t1 = ray.t1;
    const int L = ray.L;
    const float scaleL = __builtin_ldexpf(1.0f, -L);
    const int S = g.M + 2;
    const float imax = (float)(S - 2);
    const float invd[3] = {d[0] != 0.0f ? 1.0f / d[0] : INFINITY,
                           d[1] != 0.0f ? 1.0f / d[1] : INFINITY,
                           d[2] != 0.0f ? 1.0f / d[2] : INFINITY};
    int nominal = 0;
    if (ray.hit) {
        int kk = max((int)((t1 - t0) / step) - 2, 0);
        while (t0 + (float)kk * step < t1) kk++;
        nominal = kk;
    }

    // accumulated state: DVR colour and transmittance, MIP running maxima (from the window's
    // low end) and the positions that set them
    float Tr = 1.0f, Cr = 0.0f, Cg = 0.0f, Cb = 0.0f;
    float mx[C];
    int kmx[C];
#pragma unroll
    for (int c = 0; c < C; c++) {
        mx[c] = V.ulo[c];
        kmx[c] = -1;
    }
    int k = 0;
    bool live = ray.hit && inside;
    RefineState *const rst = (missing == 2 && inside) ? V.rstate + pix : nullptr;
    int st_status = 0;   // refinement: the ray's state at the start of this pass
    if (rst) {
        const RefineState st = *rst;
        st_status = st.status;
        if (st.status == 1 || st.status == 3) {
            live = false;   // finished in an earlier pass: its result is kept in the state
        } else if (st.status == 2) {
            k = st.k;
            if (mip) {
#pragma unroll
                for (int c = 0; c < C; c++) mx[c] = st.acc[c];
            } else {
                Cr = st.acc[0];
                Cg = st.acc[1];
                Cb = st.acc[2];
                Tr = st.acc[3];
            }
        }
    }
    const bool done_before = st_status == 1 || st_status == 3;
    const bool first_pass = st_status == 0;   // rays and nominal positions counted once

    constexpr int NG = kXf ? C : 1;
    LookupGroup<C> grp[NG];
    bool waited = false;
    int composited = 0, trilinear = 0;

    auto cell_index = [&](int lev, const int v[3]) -> int {
        const int sh = g.mlog2 >= 0 ? g.mlog2 + lev : -1;
        const int e = g.M << lev;
        int cx, cy, cz;
        if (sh >= 0) {
            cx = v[0] >> sh;
            cy = v[1] >> sh;
            cz = v[2] >> sh;
        } else {
            cx = v[0] / e;
            cy = v[1] / e;
            cz = v[2] / e;
        }
        const int G = g.grid[lev];
        return g.cell_off[lev] + (cz * G + cy) * G + cx;
    };

    while (live && k < nominal) {
        const float tk = t0 + (float)k * step;
        float p[3];
#pragma unroll
        for (int q = 0; q < 3; q++) {
            const float m = tk * d[q];
            p[q] = o[q] + m;
        }
        bool jumped = false;
        bool any_brick = false;
#pragma unroll
        for (int gi = 0; gi < NG; gi++) {
            float pg[3];
            if constexpr (kXf) {
#pragma unroll
                for (int a = 0; a < 3; a++) {
                    const float *m = V.xform[gi][a];
                    const float s0 = m[0] * p[0];
                    const float s1 = m[1] * p[1];
                    const float s2 = m[2] * p[2];
                    const float u = s0 + s1;
                    const float w = u + s2;
                    pg[a] = w + m[3];
                }
            } else {
#pragma unroll
                for (int a = 0; a < 3; a++) pg[a] = p[a];
            }
            int v[3];
#pragma unroll
            for (int q = 0; q < 3; q++) v[q] = min(max((int)floorf(pg[q]), 0), g.dims[q] - 1);
            const int cidx = cell_index(L, v);
            LookupGroup<C> &G = grp[gi];
            if (cidx != G.cidx) {
                G.cidx = cidx;
                if (skip && mask_bit<kLdsMask>(tmask, smask, cidx)) {
                    G.draw = kDrawNone;
                    if constexpr (!kXf) {
                        // widen to the largest transparent ancestor, jump to just before its exit
                        int lev = L;
                        int a3[3];
                        const int e0 = g.M << L;
                        for (int q = 0; q < 3; q++) a3[q] = v[q] / e0;
                        while (lev < g.N) {
                            const int pg_ = g.grid[lev + 1];
                            if (!mask_bit<kLdsMask>(tmask, smask, g.cell_off[lev + 1] +
                                                     ((a3[2] >> 1) * pg_ + (a3[1] >> 1)) * pg_ +
                                                     (a3[0] >> 1)))
                                break;
                            lev++;
                            for (int q = 0; q < 3; q++) a3[q] >>= 1;
                        }
                        const int e = g.M << lev;
                        float te = INFINITY;
                        for (int q = 0; q < 3; q++) {
                            const float plane = d[q] > 0.0f ? (float)(a3[q] * e + e) : (float)(a3[q] * e);
                            if (d[q] != 0.0f) te = fminf(te, (plane - o[q]) * invd[q]);
                        }
                        const float kf = floorf((te - t0) * rstep) - 1.0f;
                        k = (kf > (float)(k + 1)) ? (int)fminf(kf, 2.0e9f) : k + 1;
                        G.cidx = -1;
                        jumped = true;
                    }
                    continue;
                }
                const DevCell &cell = table[cidx];
                const int kind = cell.kind;
                if (mip && skip && (kind != kBrickMissing || missing == 0)) {
                    // no sample of this cell can raise the group's running maxima
                    bool below = true;
#pragma unroll
                    for (int c = 0; c < C; c++)
                        if (!kXf || c == gi) below = below && cell.hi[c] <= mx[c];
                    if (below) {
                        G.draw = kDrawNone;
                        continue;
                    }
                }
                G.sscale = scaleL;
                G.base = nullptr;
                if (kind == kBrick) {
                    if (flags) flags[cidx] = 1;
                    G.draw = kDrawBrick;
                } else {
                    G.draw = kDrawAvg;
                    if (kind == kBrickMissing) {
                        if (flags) flags[cidx] = 2;
                        if (missing == 2) {
                            G.draw = kDrawWait;
                        } else if (missing == 1) {
                            // the resident brick of the first of the two coarser levels;
                            // missing ones among them are requested as well
                            for (int l = L + 1; l <= min(L + 2, g.N); l++) {
                                const int ci = cell_index(l, v);
                                const int2 ks = *(const int2 *)&table[ci].kind;
                                if (ks.x == kBrick && G.draw == kDrawAvg) {
                                    if (flags) flags[ci] = 1;
                                    G.draw = kDrawBrick;
                                    G.sscale = __builtin_ldexpf(1.0f, -l);
                                    const int e = g.M << l;
                                    for (int q = 0; q < 3; q++)
                                        G.sb[q] = (float)((v[q] / e) * g.M) - 0.5f;
                                    G.base = pool + (uint64_t)ks.y * brick_bytes;
                                } else if (ks.x == kBrickMissing && flags) {
                                    flags[ci] = 2;
                                }
                            }
                        }
                    }
                    if (G.draw == kDrawAvg)
#pragma unroll
                        for (int c = 0; c < C; c++) G.avg[c] = cell.avg[c];
                }
                if (G.draw == kDrawBrick && !G.base) {
                    const int e = g.M << L;
                    for (int q = 0; q < 3; q++) G.sb[q] = (float)((v[q] / e) * g.M) - 0.5f;
                    G.base = pool + (uint64_t)cell.slot * brick_bytes;
                }
            }
        }
        if (jumped) continue;
        bool wait = false;
#pragma unroll
        for (int gi = 0; gi < NG; gi++) wait = wait || grp[gi].draw == kDrawWait;
        if (wait) {
            waited = true;
            break;
        }
        // samples, one group at a time
        float s[C];
        bool on[C];
#pragma unroll
        for (int gi = 0; gi < NG; gi++) {
            const LookupGroup<C> &G = grp[gi];
            const int c_lo = kXf ? gi : 0, c_hi = kXf ? gi + 1 : C;
            for (int c = c_lo; c < c_hi; c++) on[c] = G.draw != kDrawNone;
            if (G.draw == kDrawAvg) {
                for (int c = c_lo; c < c_hi; c++) s[c] = G.avg[c];
            } else if (G.draw == kDrawBrick) {
                any_brick = true;
                float pg[3];
                if constexpr (kXf) {
#pragma unroll
                    for (int a = 0; a < 3; a++) {
                        const float *m = V.xform[gi][a];
                        const float s0 = m[0] * p[0];
                        const float s1 = m[1] * p[1];
                        const float s2 = m[2] * p[2];
                        const float u = s0 + s1;
                        const float w = u + s2;
                        pg[a] = w + m[3];
                    }
                } else {
#pragma unroll
                    for (int a = 0; a < 3; a++) pg[a] = p[a];
                }
                float f[3];
                int ii[3];
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    const float lq = __builtin_fmaf(pg[q], G.sscale, -G.sb[q]);
                    f[q] = __builtin_amdgcn_fractf(lq);
                    ii[q] = (int)__builtin_amdgcn_fmed3f(lq, 0.0f, imax);
                }
                const int64_t v0 = ((int64_t)(ii[2] * S + ii[1]) * S + ii[0]) * 4;
                const int64_t dy = (int64_t)S * 4, dz = (int64_t)S * S * 4;
                const T *b0 = (const T *)G.base;
                const int64_t off[8] = {v0, v0 + 4, v0 + dy, v0 + dy + 4,
                                        v0 + dz, v0 + dz + 4, v0 + dz + dy, v0 + dz + dy + 4};
                for (int c = c_lo; c < c_hi; c++) {
                    float w[8];
#pragma unroll
                    for (int q = 0; q < 8; q++) w[q] = (float)b0[off[q] + c];
                    const float c00 = lerpf(w[0], w[1], f[0]);
                    const float c10 = lerpf(w[2], w[3], f[0]);
                    const float c01 = lerpf(w[4], w[5], f[0]);
                    const float c11 = lerpf(w[6], w[7], f[0]);
                    s[c] = lerpf(lerpf(c00, c10, f[1]), lerpf(c01, c11, f[1]), f[2]);
                }
            }
        }
        if constexpr (kCount) {
            composited++;
            if (any_brick) trilinear++;
        }
        if (mip) {
#pragma unroll
            for (int c = 0; c < C; c++)
                if (on[c] && s[c] > mx[c]) {
                    mx[c] = s[c];
                    kmx[c] = k;
                }
        } else {
#pragma unroll
            for (int c = 0; c < C; c++) {
                if (!on[c]) continue;   // zero opacity: compositing would change nothing
                const Classified q = classify(s[c], ulo[c], usc[c], tb.lut[c]);
                const float wgt = Tr * __builtin_fmaf(q.fr, q.de.w, q.e0.w);
                Cr = __builtin_fmaf(wgt, __builtin_fmaf(q.fr, q.de.x, q.e0.x), Cr);
                Cg = __builtin_fmaf(wgt, __builtin_fmaf(q.fr, q.de.y, q.e0.y), Cg);
                Cb = __builtin_fmaf(wgt, __builtin_fmaf(q.fr, q.de.z, q.e0.z), Cb);
                Tr = Tr - wgt;
            }
            if (Tr <= ert_T) {
                k++;
                break;   // early ray termination after this position
            }
        }
        k++;
    }

    if (inside && !done_before) {
        float res[4];
        if (mip) {
            float a4[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int c = 0; c < C; c++) a4[c] = mx[c];
            for (int q = 0; q < 4; q++) res[q] = a4[q];
        } else {
            res[0] = Cr;
            res[1] = Cg;
            res[2] = Cb;
            res[3] = waited ? Tr : 1.0f - Tr;   // a waiting ray keeps its transmittance exactly
        }
        if (rst) {
            RefineState st;
            for (int q = 0; q < 4; q++) st.acc[q] = res[q];
            st.k = k;
            st.status = waited ? 2 : (ray.hit ? 1 : 3);
            st.pad[0] = st.pad[1] = 0;
            *rst = st;
        } else {
            if (mip && ray.hit) {
                Tr = 1.0f;
#pragma unroll
                for (int c = 0; c < C; c++) {
                    const Classified q = classify(mx[c], ulo[c], usc[c], tb.lut[c]);
                    const float wgt = Tr * __builtin_fmaf(q.fr, q.de.w, q.e0.w);
                    Cr = __builtin_fmaf(wgt, __builtin_fmaf(q.fr, q.de.x, q.e0.x), Cr);
                    Cg = __builtin_fmaf(wgt, __builtin_fmaf(q.fr, q.de.y, q.e0.y), Cg);
                    Cb = __builtin_fmaf(wgt, __builtin_fmaf(q.fr, q.de.z, q.e0.z), Cb);
                    Tr = Tr - wgt;
                }
                *(float4 *)(V.image + pix * 4) = make_float4(Cr, Cg, Cb, 1.0f - Tr);
            } else if (mip) {
                *(float4 *)(V.image + pix * 4) = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            } else {
                *(float4 *)(V.image + pix * 4) = make_float4(Cr, Cg, Cb, 1.0f - Tr);
            }
            if (mip && V.amax) {
                int a4[4] = {-1, -1, -1, -1};
#pragma unroll
                for (int c = 0; c < C; c++) a4[c] = kmx[c];
                *(int4 *)(V.amax + pix * 4) = make_int4(a4[0], a4[1], a4[2], a4[3]);
            }
        }
    }
    if (missing == 2) {
        const unsigned long long b = __ballot(waited);
        if (lane == 0 && b) atomicAdd(V.rwait, (int)__popcll(b));
    }
    if (kCount && counters) {
        unsigned long long r = (ray.hit && inside && first_pass) ? 1ull : 0ull,
                           nn = (inside && first_pass) ? (unsigned long long)nominal : 0ull,
                           cc = (unsigned long long)composited, tt = (unsigned long long)trilinear;
        for (int off = 32; off > 0; off >>= 1) {
            r += __shfl_xor(r, off, 64);
            nn += __shfl_xor(nn, off, 64);
            cc += __shfl_xor(cc, off, 64);
            tt += __shfl_xor(tt, off, 64);
        }
        if (lane == 0) {
            RenderCounters *cs = counters + (blockIdx.x & (kCounterSlots - 1));
            atomicAdd(&cs->rays, r);
            atomicAdd(&cs->nominal, nn);
            atomicAdd(&cs->composited, cc);
            atomicAdd(&cs->trilinear, tt);
        }
    }
}

template <typename T, int C, bool kLdsMask>
__global__ void __launch_bounds__(kThreads)
k_render_general(VolGeom g, const DevCell *__restrict__ table, const uint8_t *__restrict__ pool,
                 uint64_t brick_bytes, const DevView *__restrict__ views, int n_views,
                 int item_base, RenderCounters *counters, uint8_t *flags, int mask_lds)
{
    __shared__ LutTable<C> tb;
    const WgItem it = item_of(views, n_views, item_base + (int)blockIdx.x);
    const bool xf = views[it.view].xform_on != 0;
    if (counters) {
        if (xf)
            render_general_body<T, C, true, kLdsMask, true>(g, table, pool, brick_bytes, views, it,
                                                            counters, flags, tb, mask_lds);
        else
            render_general_body<T, C, false, kLdsMask, true>(g, table, pool, brick_bytes, views,
                                                             it, counters, flags, tb, mask_lds);
    } else {
        if (xf)
            render_general_body<T, C, true, kLdsMask, false>(g, table, pool, brick_bytes, views,
                                                             it, counters, flags, tb, mask_lds);
        else
            render_general_body<T, C, false, kLdsMask, false>(g, table, pool, brick_bytes, views,
                                                              it, counters, flags, tb, mask_lds);
    }
}

// Front-to-back composite of the depth segments: C = C_0 + T_0 (C_1 + T_1 (...)),
// T = T_0 T_1 ..., written as premultiplied (C, 1 - T) to the pixels of the rendered tiles.
// MIP views: the segments' per-channel maxima are combined by max and then classified and
// composited in channel order (-inf marks a ray that misses the volume: the pixel is 0).
// Segments are loaded two at a time and the kernel is held to 32 registers, so that it starts
// beside render waves of other launches (they leave 32 of a SIMD's 512).
// One instantiation per mode (kMip), each skipping the other mode's views, so that the DVR one
// keeps its few registers.
template <int C, bool kMip>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_num_vgpr(32)))
k_combine(const DevView *__restrict__ views, const int32_t *__restrict__ split_views)
{
    const DevView &V = views[split_views[blockIdx.y]];
    if ((V.mode == 1) != kMip) return;
    const int64_t npix = (int64_t)V.width * V.height;
    constexpr bool mip = kMip;
    const LutTable<C> *tab = (const LutTable<C> *)V.tables;
    for (int64_t pix = (int64_t)blockIdx.x * 256 + threadIdx.x; pix < npix;
         pix += (int64_t)gridDim.x * 256) {
        const int px = (int)(pix % V.width), py = (int)(pix / V.width);
        const int tile = (py >> 3) * V.tiles_x + (px >> 3);
        if (tile < V.tile_begin || tile >= V.tile_end) continue;
        const float4 *part = (const float4 *)V.part + pix;
        float4 acc = part[0];
        if constexpr (mip) {
            for (int s0 = 1; s0 < V.nsplit; s0 += 2) {
                float4 q[2];
#pragma unroll
                for (int k = 0; k < 2; k++)   // two segments' loads in flight
                    if (s0 + k < V.nsplit) q[k] = part[(int64_t)(s0 + k) * npix];
#pragma unroll
                for (int k = 0; k < 2; k++)
                    if (s0 + k < V.nsplit) {
                        acc.x = fmaxf(acc.x, q[k].x);
                        acc.y = fmaxf(acc.y, q[k].y);
                        acc.z = fmaxf(acc.z, q[k].z);
                        acc.w = fmaxf(acc.w, q[k].w);
                    }
            }
            float Cr = 0.0f, Cg = 0.0f, Cb = 0.0f, Tr = 1.0f;
            if (acc.x > -INFINITY) {
                const float m4[4] = {acc.x, acc.y, acc.z, acc.w};
#pragma unroll
                for (int c = 0; c < C; c++) {
                    const float usc = V.uscale[c], ub = -V.ulo[c] * usc;
                    const Classified cq = classify(m4[c], ub, usc, tab->lut[c]);
                    const float wgt = Tr * __builtin_fmaf(cq.fr, cq.de.w, cq.e0.w);
                    Cr = __builtin_fmaf(wgt, __builtin_fmaf(cq.fr, cq.de.x, cq.e0.x), Cr);
                    Cg = __builtin_fmaf(wgt, __builtin_fmaf(cq.fr, cq.de.y, cq.e0.y), Cg);
                    Cb = __builtin_fmaf(wgt, __builtin_fmaf(cq.fr, cq.de.z, cq.e0.z), Cb);
                    Tr = Tr - wgt;
                }
            }
            *(float4 *)(V.image + pix * 4) = make_float4(Cr, Cg, Cb, 1.0f - Tr);
            continue;
        }
        float T = acc.w;
        for (int s0 = 1; s0 < V.nsplit; s0 += 2) {
            float4 q[2];
#pragma unroll
            for (int k = 0; k < 2; k++)   // two segments' loads in flight
                if (s0 + k < V.nsplit) q[k] = part[(int64_t)(s0 + k) * npix];
#pragma unroll
            for (int k = 0; k < 2; k++)
                if (s0 + k < V.nsplit) {
                    acc.x = __builtin_fmaf(T, q[k].x, acc.x);
                    acc.y = __builtin_fmaf(T, q[k].y, acc.y);
                    acc.z = __builtin_fmaf(T, q[k].z, acc.z);
                    T = T * q[k].w;
                }
        }
        *(float4 *)(V.image + pix * 4) = make_float4(acc.x, acc.y, acc.z, 1.0f - T);
    }
}

// Refinement views whose rays all finished in this launch (no ray waited): the image takes
// the states' results -- DVR the premultiplied colour and opacity, MIP the classified maxima
// composited in channel order; rays that miss the volume give 0.
template <int C>
__global__ void __launch_bounds__(256)
k_refine_finish(const DevView *__restrict__ views, const int32_t *__restrict__ refine_views)
{
    const DevView &V = views[refine_views[blockIdx.y]];
    if (*V.rwait != 0) return;   // the previous image stays until every ray has finished
    const int64_t npix = (int64_t)V.width * V.height;
    const LutTable<C> *tab = (const LutTable<C> *)V.tables;
    for (int64_t pix = (int64_t)blockIdx.x * 256 + threadIdx.x; pix < npix;
         pix += (int64_t)gridDim.x * 256) {
        const int px = (int)(pix % V.width), py = (int)(pix / V.width);
        const int tile = (py >> 3) * V.tiles_x + (px >> 3);
        if (tile < V.tile_begin || tile >= V.tile_end) continue;
        const RefineState st = V.rstate[pix];
        float4 out = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if (st.status == 1) {
            if (V.mode == 1) {
                float Cr = 0.0f, Cg = 0.0f, Cb = 0.0f, Tr = 1.0f;
#pragma unroll
                for (int c = 0; c < C; c++) {
                    const float usc = V.uscale[c], ub = -V.ulo[c] * usc;
                    const Classified cq = classify(st.acc[c], ub, usc, tab->lut[c]);
                    const float wgt = Tr * __builtin_fmaf(cq.fr, cq.de.w, cq.e0.w);
                    Cr = __builtin_fmaf(wgt, __builtin_fmaf(cq.fr, cq.de.x, cq.e0.x), Cr);
                    Cg = __builtin_fmaf(wgt, __builtin_fmaf(cq.fr, cq.de.y, cq.e0.y), Cg);
                    Cb = __builtin_fmaf(wgt, __builtin_fmaf(cq.fr, cq.de.z, cq.e0.z), Cb);
                    Tr = Tr - wgt;
                }
                out = make_float4(Cr, Cg, Cb, 1.0f - Tr);
            } else {
                out = make_float4(st.acc[0], st.acc[1], st.acc[2], st.acc[3]);
            }
        }
        *(float4 *)(V.image + pix * 4) = out;
    }
}

// Transparency of every node-table cell for every view that skips: workgroup b of a view sets
// bits 256 b ... 256 b + 255 of V.tmask, one 64-bit ballot per wave.  Bit i is set when no
// sample drawn inside cell i can contribute:
//  - DVR: the cell's value range classifies to zero opacity in every channel (cell_transparent
//    with the view's opacity prefix counts from V.tables);
//  - MIP: the cell's upper bound is at most the window's low end in every channel (no sample
//    can raise a running maximum, which starts there);
//  - full-frame fallback views take the range of the cell's ancestor two levels up (or the
//    root): a missing brick is drawn from a coarser brick whose values that ancestor's range
//    covers, while its own range need not.
// Reads the current node table: after the last upload and after the launch records' copy.
template <int C>
__global__ void __launch_bounds__(256)
k_view_mask(VolGeom g, const DevView *__restrict__ views, const DevCell *__restrict__ table,
            int64_t n_cells)
{
    const DevView &V = views[blockIdx.y];
    if (!V.tmask) return;
    __shared__ int pref[C][257];
    const ViewTables<C> *tb = (const ViewTables<C> *)V.tables;
    for (int i = threadIdx.x; i < C * 257; i += 256) (&pref[0][0])[i] = (&tb->pref[0][0])[i];
    __syncthreads();
    float ulo[C], usc[C];
#pragma unroll
    for (int c = 0; c < C; c++) {
        usc[c] = V.uscale[c];
        ulo[c] = -V.ulo[c] * usc[c];
    }
    const int64_t cell = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool t = false;
    if (cell < n_cells) {
        int64_t src = cell;
        if (V.missing == 1) {
            int lev = 0;
            while (lev < g.N && cell >= g.cell_off[lev + 1]) lev++;
            const int G = g.grid[lev];
            const int64_t li = cell - g.cell_off[lev];
            int x = (int)(li % G), y = (int)((li / G) % G), z = (int)(li / ((int64_t)G * G));
            const int up = min(lev + 2, g.N);
            x >>= (up - lev);
            y >>= (up - lev);
            z >>= (up - lev);
            const int Gu = g.grid[up];
            src = g.cell_off[up] + ((int64_t)z * Gu + y) * Gu + x;
        }
        const DevCell &dc = table[src];
        if (V.mode == 1) {
            t = true;
#pragma unroll
            for (int c = 0; c < C; c++) t = t && dc.hi[c] <= V.ulo[c];
        } else {
            t = cell_transparent<C>(dc, ulo, usc, pref);
        }
    }
    const unsigned long long b = __ballot(t);
    const int64_t first = cell & ~(int64_t)63;   // first cell of this wave
    if ((threadIdx.x & 63) == 0 && first < n_cells) {
        V.tmask[first >> 5] = (uint32_t)b;
        V.tmask[(first >> 5) + 1] = (uint32_t)(b >> 32);
    }
}

template <typename T, int C>
void launch_c(hipStream_t s, const VolGeom &g, const DevCell *table, const uint8_t *p,
              uint64_t brick_bytes, const DevView *views, int n_views, const int32_t *class_items,
              RenderCounters *counters, uint8_t *flags)
{
    // masks of up to 1024 words (32768 cells: trees of up to five levels) go to LDS
    constexpr int64_t kMaskLdsWords = 1024;
    const int64_t words = view_mask_words((int64_t)g.cell_off[g.N] + 1);
    const int mask_lds = words <= kMaskLdsWords ? (int)words : 0;
    const size_t shm = (size_t)mask_lds * 4;
    const dim3 block(kThreads);
    for (int cls = 0; cls < kNumClasses; cls++) {
        const int base = class_items[cls], n = class_items[cls + 1] - base;
        if (n <= 0) continue;
        const dim3 grid((unsigned)n);
#define OCTRC_LAUNCH(KERNEL, LDS)                                                              \
    hipLaunchKernelGGL(KERNEL, grid, block, (LDS) ? shm : 0, s, g, table, p, brick_bytes, views, \
                       n_views, base, counters, flags, (LDS) ? mask_lds : 0)
        if (cls == kClassGeneral) {
            if (mask_lds) OCTRC_LAUNCH((k_render_general<T, C, true>), true);
            else OCTRC_LAUNCH((k_render_general<T, C, false>), false);
        } else if constexpr (sizeof(T) == 2) {
            if (cls == kClassMip) {
                if (mask_lds) OCTRC_LAUNCH((k_render_u16<C, true, true>), true);
                else OCTRC_LAUNCH((k_render_u16<C, false, true>), false);
            } else {
                if (mask_lds) OCTRC_LAUNCH((k_render_u16<C, true, false>), true);
                else OCTRC_LAUNCH((k_render_u16<C, false, false>), false);
            }
        } else {
            if (cls == kClassMip) {
                if (mask_lds) OCTRC_LAUNCH((k_render_f32<C, true, true>), true);
                else OCTRC_LAUNCH((k_render_f32<C, false, true>), false);
            } else {
                if (mask_lds) OCTRC_LAUNCH((k_render_f32<C, true, false>), true);
                else OCTRC_LAUNCH((k_render_f32<C, false, false>), false);
            }
        }
#undef OCTRC_LAUNCH
    }
}

template <typename T>
hipError_t launch_typed(const VolGeom &g, const DevCell *table, const void *pool,
                        uint64_t brick_bytes, const DevView *views, int n_views,
                        const int32_t *class_items, RenderCounters *counters, uint8_t *flags,
                        hipStream_t s)
{
    const uint8_t *p = (const uint8_t *)pool;
    switch (g.C) {
    case 1: launch_c<T, 1>(s, g, table, p, brick_bytes, views, n_views, class_items, counters, flags); break;
    case 2: launch_c<T, 2>(s, g, table, p, brick_bytes, views, n_views, class_items, counters, flags); break;
    case 3: launch_c<T, 3>(s, g, table, p, brick_bytes, views, n_views, class_items, counters, flags); break;
    default: launch_c<T, 4>(s, g, table, p, brick_bytes, views, n_views, class_items, counters, flags); break;
    }
    return hipGetLastError();
}

}  // namespace

size_t view_tables_bytes(int C)
{
    switch (C) {
    case 1: return sizeof(ViewTables<1>);
    case 2: return sizeof(ViewTables<2>);
    case 3: return sizeof(ViewTables<3>);
    default: return sizeof(ViewTables<4>);
    }
}

hipError_t launch_view_mask(const VolGeom &g, const DevView *views, int n_views,
                            const DevCell *table, int64_t n_cells, hipStream_t s)
{
    if (n_views <= 0 || n_cells <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n_cells + 255) / 256), (unsigned)n_views), block(256);
    switch (g.C) {
    case 1: hipLaunchKernelGGL(k_view_mask<1>, grid, block, 0, s, g, views, table, n_cells); break;
    case 2: hipLaunchKernelGGL(k_view_mask<2>, grid, block, 0, s, g, views, table, n_cells); break;
    case 3: hipLaunchKernelGGL(k_view_mask<3>, grid, block, 0, s, g, views, table, n_cells); break;
    default: hipLaunchKernelGGL(k_view_mask<4>, grid, block, 0, s, g, views, table, n_cells); break;
    }
    return hipGetLastError();
}

hipError_t launch_combine(const DevView *views, const int32_t *split_views, int n_split, int C,
                          int modes, int64_t max_pixels, hipStream_t s)
{
    if (n_split <= 0 || max_pixels <= 0) return hipSuccess;
    const unsigned gx = (unsigned)std::min<int64_t>((max_pixels + 255) / 256, 4096);
    const dim3 grid(gx, (unsigned)n_split), block(256);
    for (int m = 0; m < 2; m++) {   // DVR views, then MIP views (each kernel skips the others)
        if (!(modes & (1 << m))) continue;
        switch (C * 2 + m) {
        case 2: hipLaunchKernelGGL((k_combine<1, false>), grid, block, 0, s, views, split_views); break;
        case 3: hipLaunchKernelGGL((k_combine<1, true>), grid, block, 0, s, views, split_views); break;
        case 4: hipLaunchKernelGGL((k_combine<2, false>), grid, block, 0, s, views, split_views); break;
        case 5: hipLaunchKernelGGL((k_combine<2, true>), grid, block, 0, s, views, split_views); break;
        case 6: hipLaunchKernelGGL((k_combine<3, false>), grid, block, 0, s, views, split_views); break;
        case 7: hipLaunchKernelGGL((k_combine<3, true>), grid, block, 0, s, views, split_views); break;
        case 8: hipLaunchKernelGGL((k_combine<4, false>), grid, block, 0, s, views, split_views); break;
        default: hipLaunchKernelGGL((k_combine<4, true>), grid, block, 0, s, views, split_views); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_refine_finish(const DevView *views, const int32_t *refine_views, int n_refine,
                                int C, int64_t max_pixels, hipStream_t s)
{
    if (n_refine <= 0 || max_pixels <= 0) return hipSuccess;
    const unsigned gx = (unsigned)std::min<int64_t>((max_pixels + 255) / 256, 4096);
    const dim3 grid(gx, (unsigned)n_refine), block(256);
    switch (C) {
    case 1: hipLaunchKernelGGL(k_refine_finish<1>, grid, block, 0, s, views, refine_views); break;
    case 2: hipLaunchKernelGGL(k_refine_finish<2>, grid, block, 0, s, views, refine_views); break;
    case 3: hipLaunchKernelGGL(k_refine_finish<3>, grid, block, 0, s, views, refine_views); break;
    default: hipLaunchKernelGGL(k_refine_finish<4>, grid, block, 0, s, views, refine_views); break;
    }
    return hipGetLastError();
}

hipError_t launch_render(const VolGeom &g, const DevCell *table, const void *pool,
                         uint64_t brick_bytes, const DevView *views, int n_views,
                         const int32_t *class_items, RenderCounters *counters, uint8_t *flags,
                         hipStream_t s)
{
    if (class_items[kNumClasses] == 0) return hipSuccess;
    if (g.dtype == 0)
        return launch_typed<uint16_t>(g, table, pool, brick_bytes, views, n_views, class_items,
                                      counters, flags, s);
    return launch_typed<float>(g, table, pool, brick_bytes, views, n_views, class_items, counters,
                               flags, s);
}

}  // namespace octrc
