// Forward ray casting (Algorithm 1, "Basic Ray-Casting"), one 64-lane wave per 8x8 pixel tile
// (or per depth segment of a tile's rays), several tiles of one view per workgroup
// (kRenderTilesPerWg waves).
//
// Per launch, k_view_prep tabulates each view's transfer functions (256 RGBA value/slope pairs
// per channel, plus a prefix count of the entries with non-zero opacity) and orders its tile
// groups, and k_view_mask turns the prefix counts into one bit per node-table cell: set when
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

// Tile q of tile group gi. A whole image with an even number of tile rows and columns is
// grouped in 2x2 blocks of tiles (the four waves of a workgroup share L1); otherwise a group is
// four consecutive tiles of the view's row-major tile range.
__device__ inline int group_tile(const DevView &V, int gi, int q)
{
    const int ty = (V.height + 7) >> 3;
    if (kRenderTilesPerWg == 4 && V.tile_begin == 0 && V.tile_end == V.tiles_x * ty &&
        !(V.tiles_x & 1) && !(ty & 1)) {
        const int hx = V.tiles_x >> 1, gx = gi % hx, gy = gi / hx;
        return (2 * gy + (q >> 1)) * V.tiles_x + 2 * gx + (q & 1);
    }
    return V.tile_begin + gi * kRenderTilesPerWg + q;
}

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
// words each) are staged in LDS.
template <typename T, int C, bool kErt, bool kCount, bool kLdsMask>
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
    // checkpoints are written the bounds are whole 64-position blocks instead, blocks
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
    int k = k_begin, composited = 0, trilinear = 0, next_ck = k_begin;
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
        if (ckpt) {
            // transmittance before every 64th position (unchanged across skipped positions)
            for (; next_ck <= k; next_ck += kCkptStride)
                ckpt[pix * V.nseg + next_ck / kCkptStride] = Tr;
        }
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
                const int e = g.M << lev;
                const int bl[3] = {ax * e, ay * e, az * e};
                float te = INFINITY;
#pragma unroll
                for (int q = 0; q < 3; q++) {
                    const float plane = d[q] > 0.0f ? (float)(bl[q] + e) : (float)bl[q];
                    if (d[q] != 0.0f) te = fminf(te, (plane - o[q]) * invd[q]);
                }
                // one whole step of margin: every skipped position lies inside the box
                const float kf = floorf((te - t0) * rstep) - 1.0f;
                k = (kf > (float)(k + 1)) ? (int)fminf(kf, 2.0e9f) : k + 1;
                bofs[0] = INFINITY;   // no cell cached: the next position looks its cell up
                blo[0] = 1;
                bhi[0] = 0;
                k_lo = 1;
                k_hi = 0;
                continue;
            }
            const DevCell &cell = table[cidx];
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
        if constexpr (kErt)
            if (Tr <= ert_T) live = false;  // early ray termination after this position
        k++;
    }

    if (inside) {
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
        // checkpoint blocks that begin inside a final skipped run keep the transmittance of
        // the jump (split: up to the end of this segment's blocks)
        if (ckpt)
            for (; next_ck < min(n_end, k_end); next_ck += kCkptStride)
                ckpt[pix * V.nseg + next_ck / kCkptStride] = Tr;
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
// sample counters (both uniform over the workgroup).
template <typename T, int C, bool kLdsMask>
__device__ __forceinline__ void
render_item(const VolGeom &g, const DevCell *__restrict__ table, const uint8_t *__restrict__ pool,
            uint64_t brick_bytes, const DevView *__restrict__ views, int n_views,
            RenderCounters *counters, uint8_t *flags, LutTable<C> &tb, int mask_lds)
{
    const WgItem it = item_of(views, n_views, blockIdx.x);
    if (counters)
        render_body<T, C, true, true, kLdsMask>(g, table, pool, brick_bytes, views, it, counters,
                                                flags, tb, mask_lds);
    else if (views[it.view].ert < 1.0f)
        render_body<T, C, true, false, kLdsMask>(g, table, pool, brick_bytes, views, it, counters,
                                                 flags, tb, mask_lds);
    else
        render_body<T, C, false, false, kLdsMask>(g, table, pool, brick_bytes, views, it,
                                                  counters, flags, tb, mask_lds);
}

// uint16 bricks: registers for 5 waves per SIMD (6 fit only with spills, measured 2 % slower);
// float32 bricks (twice the corner data) keep the compiler's choice.
#ifndef OCTRC_U16_WAVES_PER_EU
#define OCTRC_U16_WAVES_PER_EU 5
#endif
template <int C, bool kLdsMask>
__global__ void __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(OCTRC_U16_WAVES_PER_EU)))
k_render_u16(VolGeom g, const DevCell *__restrict__ table, const uint8_t *__restrict__ pool,
             uint64_t brick_bytes, const DevView *__restrict__ views,
             int n_views, RenderCounters *counters, uint8_t *flags, int mask_lds)
{
    __shared__ LutTable<C> tb;
    render_item<uint16_t, C, kLdsMask>(g, table, pool, brick_bytes, views, n_views, counters,
                                       flags, tb, mask_lds);
}

template <int C, bool kLdsMask>
__global__ void __launch_bounds__(kThreads)
k_render_f32(VolGeom g, const DevCell *__restrict__ table, const uint8_t *__restrict__ pool,
             uint64_t brick_bytes, const DevView *__restrict__ views,
             int n_views, RenderCounters *counters, uint8_t *flags, int mask_lds)
{
    __shared__ LutTable<C> tb;
    render_item<float, C, kLdsMask>(g, table, pool, brick_bytes, views, n_views, counters, flags,
                                    tb, mask_lds);
}

// Front-to-back composite of the depth segments: C = C_0 + T_0 (C_1 + T_1 (...)),
// T = T_0 T_1 ..., written as premultiplied (C, 1 - T) to the pixels of the rendered tiles.
__global__ void __launch_bounds__(256)
k_combine(const DevView *__restrict__ views, const int32_t *__restrict__ split_views)
{
    const DevView &V = views[split_views[blockIdx.y]];
    const int64_t npix = (int64_t)V.width * V.height;
    for (int64_t pix = (int64_t)blockIdx.x * 256 + threadIdx.x; pix < npix;
         pix += (int64_t)gridDim.x * 256) {
        const int px = (int)(pix % V.width), py = (int)(pix / V.width);
        const int tile = (py >> 3) * V.tiles_x + (px >> 3);
        if (tile < V.tile_begin || tile >= V.tile_end) continue;
        // every segment's loads are issued before the first is used (at most kMaxSplit)
        float4 q[kMaxSplit];
#pragma unroll
        for (int sg = 0; sg < kMaxSplit; sg++)
            if (sg < V.nsplit) q[sg] = *(const float4 *)(V.part + ((int64_t)sg * npix + pix) * 4);
        float4 acc = q[0];
        float T = acc.w;
#pragma unroll
        for (int sg = 1; sg < kMaxSplit; sg++) {
            if (sg < V.nsplit) {
                acc.x = __builtin_fmaf(T, q[sg].x, acc.x);
                acc.y = __builtin_fmaf(T, q[sg].y, acc.y);
                acc.z = __builtin_fmaf(T, q[sg].z, acc.z);
                T = T * q[sg].w;
            }
        }
        *(float4 *)(V.image + pix * 4) = make_float4(acc.x, acc.y, acc.z, 1.0f - T);
    }
}

// Dispatch order of a view's tile groups (item_of): groups sorted by the length inside the
// volume box and the clip half-spaces of their longest tile-centre ray (one ray per group when
// the view has more than 4096 groups), longest first, in 32 length classes.  Each thread owns a
// contiguous run of groups, and a counting sort with per-thread class counts (scanned class by
// class over the threads) keeps index order inside a class, so neighbouring groups of one
// class stay neighbours in the dispatch.  One 256-thread workgroup; group_order[G ... 2G) is
// scratch.  Precision does not matter here (the order changes no result), hence the
// approximate reciprocals.
__device__ inline void view_group_order(const VolGeom &g, const DevView &V)
{
#ifndef OCTRC_ORDER_CLASSES
#define OCTRC_ORDER_CLASSES 32
#endif
    constexpr int kCls = OCTRC_ORDER_CLASSES;
    __shared__ int cnt[kCls][256];
    __shared__ int base[kCls];
    __shared__ float red[4];
    const int G = V.groups, tid = threadIdx.x;
    int32_t *order = V.group_order, *cls = V.group_order + G;
    const int chunk = (G + 255) / 256, lo = min(tid * chunk, G), hi = min(lo + chunk, G);
    const int rays = G > 4096 ? 1 : kRenderTilesPerWg;
    const float rw = __builtin_amdgcn_rcpf((float)V.width), rh = __builtin_amdgcn_rcpf((float)V.height);
    float lmax = 0.0f;
    for (int gi = lo; gi < hi; gi++) {
        float best = 0.0f;
        for (int q = 0; q < rays; q++) {
            const int t = min(group_tile(V, gi, rays == 1 ? 1 : q), V.tile_end - 1);
            const int px = min((t % V.tiles_x) * 8 + 4, V.width - 1);
            const int py = min((t / V.tiles_x) * 8 + 4, V.height - 1);
            const float sx = ((float)(2 * px + 1) * rw - 1.0f) * V.kx;
            const float sy = (1.0f - (float)(2 * py + 1) * rh) * V.ky;
            float d[3];
            for (int k = 0; k < 3; k++) d[k] = V.f[k] + sx * V.r[k] + sy * V.u[k];
            const float inv = rsqrtf(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            float t0 = 0.0f, t1 = INFINITY;
            for (int k = 0; k < 3; k++) {
                d[k] *= inv;
                const float o = V.eye[k];
                if (d[k] == 0.0f) {
                    if (o < 0.0f || o > (float)g.dims[k]) t1 = -1.0f;
                    continue;
                }
                const float rk = __builtin_amdgcn_rcpf(d[k]);
                const float ta = -o * rk, tb = ((float)g.dims[k] - o) * rk;
                t0 = fmaxf(t0, fminf(ta, tb));
                t1 = fminf(t1, fmaxf(ta, tb));
            }
            for (int c = 0; c < V.n_clip; c++) {
                const float *pl = V.clip[c];
                const float nd = pl[0] * d[0] + pl[1] * d[1] + pl[2] * d[2];
                const float no = pl[0] * V.eye[0] + pl[1] * V.eye[1] + pl[2] * V.eye[2];
                if (nd > 0.0f) t0 = fmaxf(t0, (pl[3] - no) * __builtin_amdgcn_rcpf(nd));
                else if (nd < 0.0f) t1 = fminf(t1, (pl[3] - no) * __builtin_amdgcn_rcpf(nd));
                else if (no < pl[3]) t1 = -1.0f;
            }
            best = fmaxf(best, t1 - t0);
        }
        cls[gi] = __float_as_int(best);
        lmax = fmaxf(lmax, best);
    }
    for (int c = 0; c < kCls; c++) cnt[c][tid] = 0;
    for (int o = 32; o > 0; o >>= 1) lmax = fmaxf(lmax, __shfl_xor(lmax, o, 64));
    if ((tid & 63) == 0) red[tid >> 6] = lmax;
    __syncthreads();
    lmax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    const float scale = lmax > 0.0f ? (float)kCls / lmax : 0.0f;
    for (int gi = lo; gi < hi; gi++) {
        const int c = kCls - 1 - min(max((int)(__int_as_float(cls[gi]) * scale), 0), kCls - 1);
        cls[gi] = c;   // class 0: the longest rays
        cnt[c][tid]++;
    }
    __syncthreads();
    if (tid < kCls) {   // exclusive prefix over the threads, per class
        int run = 0;
        for (int t = 0; t < 256; t++) {
            const int n = cnt[tid][t];
            cnt[tid][t] = run;
            run += n;
        }
        base[tid] = run;
    }
    __syncthreads();
    if (tid == 0) {
        int run = 0;
        for (int c = 0; c < kCls; c++) {
            const int n = base[c];
            base[c] = run;
            run += n;
        }
    }
    __syncthreads();
    for (int gi = lo; gi < hi; gi++) {
        const int c = cls[gi];
        order[base[c] + cnt[c][tid]++] = gi;
    }
}

// Per-launch view preparation in one grid (views along y): workgroup 0 of a view tabulates
// its transfer functions (value/slope table and opacity prefix counts) into V.tables,
// workgroup 1 sorts its tile groups into dispatch order.  Reads only the views.
template <int C>
__global__ void __launch_bounds__(256) k_view_prep(VolGeom g, const DevView *__restrict__ views)
{
    __shared__ ViewTables<C> tb;
    const DevView &V = views[blockIdx.y];
    if (blockIdx.x == 1) {
        if (V.group_order) view_group_order(g, V);
        return;
    }
    build_tables<C>(V, tb);   // ends with a barrier
    const uint4 *src = (const uint4 *)&tb;
    uint4 *dst = (uint4 *)V.tables;
    for (int i = threadIdx.x; i < (int)(sizeof(ViewTables<C>) / 16); i += 256) dst[i] = src[i];
}

// Transparency of every node-table cell for every view that skips: workgroup b of a view sets
// bits 256 b ... 256 b + 255 of V.tmask, bit i when cell i's value range classifies to zero
// opacity in every channel (cell_transparent with the view's opacity prefix counts from
// V.tables), one 64-bit ballot per wave.  Reads the current node table: after the last upload
// and after k_view_prep.
template <int C>
__global__ void __launch_bounds__(256)
k_view_mask(const DevView *__restrict__ views, const DevCell *__restrict__ table, int64_t n_cells)
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
    const bool t = cell < n_cells && cell_transparent<C>(table[cell], ulo, usc, pref);
    const unsigned long long b = __ballot(t);
    const int64_t first = cell & ~(int64_t)63;   // first cell of this wave
    if ((threadIdx.x & 63) == 0 && first < n_cells) {
        V.tmask[first >> 5] = (uint32_t)b;
        V.tmask[(first >> 5) + 1] = (uint32_t)(b >> 32);
    }
}

template <typename T, int C>
void launch_c(const dim3 &grid, const dim3 &block, hipStream_t s, const VolGeom &g,
              const DevCell *table, const uint8_t *p, uint64_t brick_bytes, const DevView *views,
              int n_views, RenderCounters *counters, uint8_t *flags)
{
    // masks of up to 1024 words (32768 cells: trees of up to five levels) go to LDS
    constexpr int64_t kMaskLdsWords = 1024;
    const int64_t words = view_mask_words((int64_t)g.cell_off[g.N] + 1);
    const int mask_lds = words <= kMaskLdsWords ? (int)words : 0;
    const size_t shm = (size_t)mask_lds * 4;
    if constexpr (sizeof(T) == 2) {
        if (mask_lds)
            hipLaunchKernelGGL((k_render_u16<C, true>), grid, block, shm, s, g, table, p,
                               brick_bytes, views, n_views, counters, flags, mask_lds);
        else
            hipLaunchKernelGGL((k_render_u16<C, false>), grid, block, 0, s, g, table, p,
                               brick_bytes, views, n_views, counters, flags, 0);
    } else {
        if (mask_lds)
            hipLaunchKernelGGL((k_render_f32<C, true>), grid, block, shm, s, g, table, p,
                               brick_bytes, views, n_views, counters, flags, mask_lds);
        else
            hipLaunchKernelGGL((k_render_f32<C, false>), grid, block, 0, s, g, table, p,
                               brick_bytes, views, n_views, counters, flags, 0);
    }
}

template <typename T>
hipError_t launch_typed(const VolGeom &g, const DevCell *table, const void *pool,
                        uint64_t brick_bytes, const DevView *views, int n_views, int n_items,
                        RenderCounters *counters, uint8_t *flags, hipStream_t s)
{
    const dim3 grid(n_items), block(kThreads);
    const uint8_t *p = (const uint8_t *)pool;
    switch (g.C) {
    case 1: launch_c<T, 1>(grid, block, s, g, table, p, brick_bytes, views, n_views, counters, flags); break;
    case 2: launch_c<T, 2>(grid, block, s, g, table, p, brick_bytes, views, n_views, counters, flags); break;
    case 3: launch_c<T, 3>(grid, block, s, g, table, p, brick_bytes, views, n_views, counters, flags); break;
    default: launch_c<T, 4>(grid, block, s, g, table, p, brick_bytes, views, n_views, counters, flags); break;
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

hipError_t launch_view_prep(const VolGeom &g, const DevView *views, int n_views, hipStream_t s)
{
    if (n_views <= 0) return hipSuccess;
    const dim3 grid(2, (unsigned)n_views), block(256);
    switch (g.C) {
    case 1: hipLaunchKernelGGL(k_view_prep<1>, grid, block, 0, s, g, views); break;
    case 2: hipLaunchKernelGGL(k_view_prep<2>, grid, block, 0, s, g, views); break;
    case 3: hipLaunchKernelGGL(k_view_prep<3>, grid, block, 0, s, g, views); break;
    default: hipLaunchKernelGGL(k_view_prep<4>, grid, block, 0, s, g, views); break;
    }
    return hipGetLastError();
}

hipError_t launch_view_mask(const DevView *views, int n_views, int C, const DevCell *table,
                            int64_t n_cells, hipStream_t s)
{
    if (n_views <= 0 || n_cells <= 0) return hipSuccess;
    const dim3 grid((unsigned)((n_cells + 255) / 256), (unsigned)n_views), block(256);
    switch (C) {
    case 1: hipLaunchKernelGGL(k_view_mask<1>, grid, block, 0, s, views, table, n_cells); break;
    case 2: hipLaunchKernelGGL(k_view_mask<2>, grid, block, 0, s, views, table, n_cells); break;
    case 3: hipLaunchKernelGGL(k_view_mask<3>, grid, block, 0, s, views, table, n_cells); break;
    default: hipLaunchKernelGGL(k_view_mask<4>, grid, block, 0, s, views, table, n_cells); break;
    }
    return hipGetLastError();
}

hipError_t launch_combine(const DevView *views, const int32_t *split_views, int n_split,
                          int64_t max_pixels, hipStream_t s)
{
    if (n_split <= 0 || max_pixels <= 0) return hipSuccess;
    const unsigned gx = (unsigned)std::min<int64_t>((max_pixels + 255) / 256, 4096);
    hipLaunchKernelGGL(k_combine, dim3(gx, (unsigned)n_split), dim3(256), 0, s, views,
                       split_views);
    return hipGetLastError();
}

hipError_t launch_render(const VolGeom &g, const DevCell *table, const void *pool,
                         uint64_t brick_bytes, const DevView *views, int n_views, int n_items,
                         RenderCounters *counters, uint8_t *flags, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    if (g.dtype == 0)
        return launch_typed<uint16_t>(g, table, pool, brick_bytes, views, n_views, n_items,
                                      counters, flags, s);
    return launch_typed<float>(g, table, pool, brick_bytes, views, n_views, n_items, counters,
                               flags, s);
}

}  // namespace octrc
