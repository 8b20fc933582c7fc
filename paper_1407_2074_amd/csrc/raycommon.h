// Device helpers shared by the forward and the adjoint ray casters: transfer-function tables
// in LDS, the float32 ray set-up, and node-table transparency tests.
//
// The files that include this header are compiled without floating-point contraction, and
// every intended fused multiply-add is written explicitly, so the ray geometry below follows
// its written operation sequence exactly: which voxel, node, level and sample count a ray
// gets is an exact function of the view.
#pragma once

#include "internal.h"

namespace octrc {

// Tile q of tile group gi. A whole image with an even number of tile rows and columns is
// grouped in 2x2 blocks of tiles (the four waves of a workgroup share L1); otherwise a group is
// four consecutive tiles of the view's row-major tile range.
__host__ __device__ inline int group_tile(const DevView &V, int gi, int q)
{
    const int ty = (V.height + 7) >> 3;
    if (kRenderTilesPerWg == 4 && V.tile_begin == 0 && V.tile_end == V.tiles_x * ty &&
        !(V.tiles_x & 1) && !(ty & 1)) {
        const int hx = V.tiles_x >> 1, gx = gi % hx, gy = gi / hx;
        return (2 * gy + (q >> 1)) * V.tiles_x + 2 * gx + (q & 1);
    }
    return V.tile_begin + gi * kRenderTilesPerWg + q;
}

__device__ inline float lerpf(float a, float b, float t) { return __builtin_fmaf(t, b - a, a); }

// Control-point segment and weight of table entry k (x = k/255): the entry is
// (1-f) * rgba[j] + f * rgba[j+1]; outside the first / last control point the end value is
// held (j = 0, f = 0 / j = 6, f = 1).  Host and device evaluate the same IEEE float32
// operations (no contraction), so tables built on either side are identical.
__host__ __device__ inline void tf_segment(const float *p, int k, int &j, float &f)
{
    const float x = (float)k / 255.0f;
    if (x <= p[0]) { j = 0; f = 0.0f; return; }
    if (x >= p[7]) { j = 6; f = 1.0f; return; }
    j = 0;
    while (j < 6 && !(x < p[j + 1])) j++;
    f = (x - p[j]) / (p[j + 1] - p[j]);
}

__host__ __device__ inline float4 tf_entry(const DevView &V, int c, int k)
{
    int j;
    float f;
    tf_segment(V.tf_pos[c], k, j, f);
    const float(*q)[4] = V.tf_rgba[c];
    const float w0 = 1.0f - f;
    return make_float4(w0 * q[j][0] + f * q[j + 1][0], w0 * q[j][1] + f * q[j + 1][1],
                       w0 * q[j][2] + f * q[j + 1][2], w0 * q[j][3] + f * q[j + 1][3]);
}

// Per-workgroup LDS tables of one view: entry k of channel c holds [0] the RGBA value and
// [1] the RGBA slope to entry k+1 (0 for k = 255), so a lookup with fraction f is one fused
// multiply-add per component; pref[c][k] counts the entries below k with non-zero opacity.
template <int C>
struct alignas(16) ViewTables {
    float4 lut[C][256][2];
    int pref[C][257];
    int wtot[C][4];
};

// The part of a view's tables the forward march reads (the value/slope table, which leads
// ViewTables): transparency comes from the per-launch cell mask instead of the prefix counts.
template <int C>
struct alignas(16) LutTable {
    float4 lut[C][256][2];
};

// Only the opacity prefix counts of build_tables (same entries, same counts); called by every
// thread of a 256-thread workgroup, ends with a barrier.
template <int C>
__device__ inline void build_prefix(const DevView &V, int (*pref)[257], int (*wtot)[4])
{
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
#pragma unroll
    for (int c = 0; c < C; c++) {
        const unsigned long long m = __ballot(tf_entry(V, c, tid).w != 0.0f);
        if (lane == 63) wtot[c][wave] = __popcll(m);
        pref[c][tid] = __popcll(m & ((1ull << lane) - 1ull));
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; c++) {
        int base = 0;
        for (int w = 0; w < wave; w++) base += wtot[c][w];
        pref[c][tid] += base;
        if (tid == 255) pref[c][256] = base + wtot[c][3];
    }
    __syncthreads();
}

// Called by every thread of the workgroup (blockDim >= 256); ends with a barrier.
template <int C>
__device__ inline void build_tables(const DevView &V, ViewTables<C> &tb)
{
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid < 256) {
#pragma unroll
        for (int c = 0; c < C; c++) {
            const float4 e = tf_entry(V, c, tid);
            tb.lut[c][tid][0] = e;
            const unsigned long long m = __ballot(e.w != 0.0f);
            if (lane == 63) tb.wtot[c][wave] = __popcll(m);
            tb.pref[c][tid] = __popcll(m & ((1ull << lane) - 1ull));  // wave-local for now
        }
    }
    __syncthreads();
    if (tid < 256) {
#pragma unroll
        for (int c = 0; c < C; c++) {
            int base = 0;
            for (int w = 0; w < wave; w++) base += tb.wtot[c][w];
            tb.pref[c][tid] += base;
            if (tid == 255) tb.pref[c][256] = base + tb.wtot[c][3];
            const float4 e0 = tb.lut[c][tid][0];
            const float4 e1 = tid < 255 ? tb.lut[c][tid + 1][0] : e0;
            tb.lut[c][tid][1] = make_float4(e1.x - e0.x, e1.y - e0.y, e1.z - e0.z, e1.w - e0.w);
        }
    }
    __syncthreads();
}

// A view's tables built on the host (the same entries, slopes and opacity prefix counts as
// build_tables), to be copied to the device with the launch's view records.
template <int C>
__host__ inline void host_build_tables(const DevView &V, ViewTables<C> &tb)
{
    for (int c = 0; c < C; c++) {
        float4 e[256];   // every entry once
        for (int k = 0; k < 256; k++) e[k] = tf_entry(V, c, k);
        int run = 0;
        for (int k = 0; k < 256; k++) {
            const float4 e0 = e[k], e1 = k < 255 ? e[k + 1] : e0;
            tb.lut[c][k][0] = e0;
            tb.lut[c][k][1] = make_float4(e1.x - e0.x, e1.y - e0.y, e1.z - e0.z, e1.w - e0.w);
            tb.pref[c][k] = run;
            run += e0.w != 0.0f ? 1 : 0;
        }
        tb.pref[c][256] = run;
        for (int w = 0; w < 4; w++) tb.wtot[c][w] = tb.pref[c][64 * w + 64] - tb.pref[c][64 * w];
    }
}

// The leading sizeof(Tab) bytes of V's tables (built on the host) copied into LDS by the
// whole workgroup (a multiple of 16 bytes, 16-byte loads); ends with a barrier.
template <int kThreadsPerWg, typename Tab>
__device__ inline void load_tables(const DevView &V, Tab &tb)
{
    static_assert(sizeof(Tab) % 16 == 0, "table copy in 16-byte words");
    const uint4 *src = (const uint4 *)V.tables;
    uint4 *dst = (uint4 *)&tb;
    for (int i = threadIdx.x; i < (int)(sizeof(Tab) / 16); i += kThreadsPerWg)
        dst[i] = src[i];
    __syncthreads();
}

// Table coordinate of intensity s: u = s * usc + ub with usc = 255 / (hi - lo), ub = -lo * usc.

// True when every value in [lo, hi] classifies to zero opacity in every channel: the table
// entries that interpolation may touch (with one entry of margin each side) are all zero.
template <int C>
__device__ inline bool range_transparent(const float *lo, const float *hi, const float *ub,
                                         const float *usc, const int (*pref)[257])
{
#pragma unroll
    for (int c = 0; c < C; c++) {
        float ul = __builtin_fmaf(lo[c], usc[c], ub[c]);
        float uh = __builtin_fmaf(hi[c], usc[c], ub[c]);
        ul = fminf(fmaxf(ul, 0.0f), 255.0f);
        uh = fminf(fmaxf(uh, 0.0f), 255.0f);
        const int il = max((int)ul - 1, 0);
        const int ih = min((int)uh + 2, 255);
        if (pref[c][ih + 1] - pref[c][il] != 0) return false;
    }
    return true;
}

template <int C>
__device__ inline bool cell_transparent(const DevCell &cell, const float *ub, const float *usc,
                                        const int (*pref)[257])
{
    const float4 clo = *(const float4 *)cell.lo, chi = *(const float4 *)cell.hi;
    const float lo4[4] = {clo.x, clo.y, clo.z, clo.w}, hi4[4] = {chi.x, chi.y, chi.z, chi.w};
    return range_transparent<C>(lo4, hi4, ub, usc, pref);
}

struct Ray {
    float o[3], d[3];
    float t0, t1;
    int L;
    bool hit;
};

// Pixel (i, j) of view V, every step one float32 operation:
//   a = (2i+1)/W, b = (2j+1)/H, sx = (a-1) kx, sy = (1-b) ky
//   dir_k = (f_k + sx r_k) + sy u_k, n2 = (dir_x^2 + dir_y^2) + dir_z^2, d = dir * (1/sqrt(n2))
//   [t0, t1] = [0, inf) cut by the slabs of the box [0, D] (ta = (0-o)/d, tb = (D-o)/d as
//   products with 1/d) and by the clip half-spaces n.p >= dist (nd = (nx dx + ny dy) + nz dz,
//   no likewise, t = (dist - no) / nd); a ray with d_k == 0 outside slab k, or with nd == 0
//   outside a half-space, or with t0 >= t1, is empty
//   LOD: fixed, or the binary exponent of w = t0 * klod clamped to [0, N]
__device__ inline Ray setup_ray(const DevView &V, const VolGeom &g, int px_i, int px_j,
                                bool inside)
{
    Ray r;
    const float a = (float)(2 * px_i + 1) / (float)V.width;
    const float b = (float)(2 * px_j + 1) / (float)V.height;
    const float sx = (a - 1.0f) * V.kx;
    const float sy = (1.0f - b) * V.ky;
    float dir[3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const float m1 = sx * V.r[k];
        const float s1 = V.f[k] + m1;
        const float m2 = sy * V.u[k];
        dir[k] = s1 + m2;
    }
    const float n2 = (dir[0] * dir[0] + dir[1] * dir[1]) + dir[2] * dir[2];
    const float inv = 1.0f / __builtin_sqrtf(n2);
    float t0 = 0.0f, t1 = INFINITY;
    bool hit = inside;
#pragma unroll
    for (int k = 0; k < 3; k++) {
        r.d[k] = dir[k] * inv;
        r.o[k] = V.eye[k];
        const float D = (float)g.dims[k];
        if (r.d[k] != 0.0f) {
            const float rk = 1.0f / r.d[k];
            const float ta = (0.0f - r.o[k]) * rk;
            const float tb = (D - r.o[k]) * rk;
            t0 = fmaxf(t0, fminf(ta, tb));
            t1 = fminf(t1, fmaxf(ta, tb));
        } else if (r.o[k] < 0.0f || r.o[k] > D) {
            hit = false;
        }
    }
    for (int c = 0; c < V.n_clip; c++) {
        const float *pl = V.clip[c];
        const float nd = (pl[0] * r.d[0] + pl[1] * r.d[1]) + pl[2] * r.d[2];
        const float no = (pl[0] * r.o[0] + pl[1] * r.o[1]) + pl[2] * r.o[2];
        const float num = pl[3] - no;
        if (nd > 0.0f) t0 = fmaxf(t0, num / nd);
        else if (nd < 0.0f) t1 = fminf(t1, num / nd);
        else if (no < pl[3]) hit = false;
    }
    if (!(t0 < t1)) hit = false;
    if (V.lod >= 0) {
        r.L = min(V.lod, g.N);
    } else {
        const float w = t0 * V.klod;
        r.L = (w > 0.0f && w < INFINITY) ? min(max(ilogbf(w), 0), g.N) : 0;
    }
    r.t0 = t0;
    r.t1 = t1;
    r.hit = hit;
    return r;
}

// Classification of intensity s in channel c: table cell i, fraction fr and the
// (value, slope) pair; u is clamped to [0, 255] (zero derivative outside the window).
struct Classified {
    float4 e0, de;   // entry i and slope to entry i+1
    float fr;
    int i;
    bool inside;     // u was not clamped
};

// u is clamped to [0, 255-] (the largest float below 255), so cell i = trunc(u) <= 254 and
// the fraction is u - i; at the top end entry 254 + (1 - 2^-16) * slope replaces entry 255.
__device__ inline Classified classify(float s, float ub, float usc, const float4 (*lut)[2])
{
    Classified r;
    const float u0 = __builtin_fmaf(s, usc, ub);
    r.inside = u0 > 0.0f && u0 < 255.0f;
    const float u = __builtin_amdgcn_fmed3f(u0, 0.0f, 254.99998474121094f);
    r.i = (int)u;
    r.fr = __builtin_amdgcn_fractf(u);
    r.e0 = lut[r.i][0];
    r.de = lut[r.i][1];
    return r;
}

}  // namespace octrc
