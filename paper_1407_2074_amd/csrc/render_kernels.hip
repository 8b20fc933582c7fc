// Forward ray casting (Algorithm 1, "Basic Ray-Casting"), one 64-lane wave per 8x8 pixel tile,
// four tiles of one view per 256-thread workgroup.
//
// Per workgroup the view's transfer functions are tabulated into LDS (256 RGBA entries per
// channel) together with a prefix count of the entries with non-zero opacity; the latter turns
// "is every sample in this node transparent?" into two LDS reads per channel, which drives the
// exact empty-space skipping.
//
// Geometry follows a fixed float32 operation sequence (this file is compiled without
// floating-point contraction, and every intended fused multiply-add is written explicitly):
// which voxel, node, level and sample count a ray gets is then an exact function of the view.
#include "internal.h"

#include <float.h>

namespace octrc {

namespace {

constexpr int kThreads = 256;

__device__ inline float lerpf(float a, float b, float t) { return __builtin_fmaf(t, b - a, a); }

// Tabulate one channel's transfer function: entry k at x = k/255, piecewise linear between
// the 8 control points, end values held outside.
__device__ inline float4 tf_entry(const DevView &V, int c, int k)
{
    const float x = (float)k / 255.0f;
    const float *p = V.tf_pos[c];
    const float(*q)[4] = V.tf_rgba[c];
    if (x <= p[0]) return make_float4(q[0][0], q[0][1], q[0][2], q[0][3]);
    if (x >= p[7]) return make_float4(q[7][0], q[7][1], q[7][2], q[7][3]);
    int j = 0;
    while (j < 6 && !(x < p[j + 1])) j++;
    const float f = (x - p[j]) / (p[j + 1] - p[j]);
    const float w0 = 1.0f - f;
    return make_float4(w0 * q[j][0] + f * q[j + 1][0], w0 * q[j][1] + f * q[j + 1][1],
                       w0 * q[j][2] + f * q[j + 1][2], w0 * q[j][3] + f * q[j + 1][3]);
}

template <int C>
__device__ inline bool cell_transparent(const float *lo, const float *hi, const DevView &V,
                                        const int (*pref)[257])
{
#pragma unroll
    for (int c = 0; c < C; c++) {
        float ul = (lo[c] - V.ulo[c]) * V.uscale[c];
        float uh = (hi[c] - V.ulo[c]) * V.uscale[c];
        ul = fminf(fmaxf(ul, 0.0f), 255.0f);
        uh = fminf(fmaxf(uh, 0.0f), 255.0f);
        const int il = max((int)ul - 1, 0);
        const int ih = min((int)uh + 2, 255);
        if (pref[c][ih + 1] - pref[c][il] != 0) return false;
    }
    return true;
}

template <typename T, int C>
__global__ void __launch_bounds__(kThreads)
k_render(VolGeom g, const DevCell *__restrict__ table, const uint8_t *__restrict__ pool,
         uint64_t brick_bytes, const DevView *__restrict__ views, const WgItem *__restrict__ items,
         RenderCounters *counters)
{
    __shared__ float4 s_lut[C][256];
    __shared__ int s_pref[C][257];
    __shared__ int s_wtot[C][4];

    const WgItem it = items[blockIdx.x];
    const DevView &V = views[it.view];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;

    // ---- per-view set-up: transfer-function tables and opacity prefix counts in LDS
#pragma unroll
    for (int c = 0; c < C; c++) {
        const float4 e = tf_entry(V, c, tid);
        s_lut[c][tid] = e;
        const unsigned long long m = __ballot(e.w != 0.0f);
        const int below = __popcll(m & ((1ull << lane) - 1ull));
        if (lane == 63) s_wtot[c][wave] = __popcll(m);
        s_pref[c][tid] = below;  // wave-local for now
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < C; c++) {
        int base = 0;
        for (int w = 0; w < wave; w++) base += s_wtot[c][w];
        s_pref[c][tid] += base;
        if (tid == 255) s_pref[c][256] = base + s_wtot[c][3];
    }
    __syncthreads();
    if (wave >= it.ntiles) return;  // no barrier below this point

    // ---- ray set-up (float32, no contraction)
    const int tile = it.tile0 + wave;
    const int px_i = (tile % V.tiles_x) * 8 + (lane & 7);
    const int px_j = (tile / V.tiles_x) * 8 + (lane >> 3);
    const bool inside = px_i < V.width && px_j < V.height;

    float o[3], d[3];
    float a = (float)(2 * px_i + 1) / (float)V.width;
    float b = (float)(2 * px_j + 1) / (float)V.height;
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
        d[k] = dir[k] * inv;
        o[k] = V.eye[k];
        const float D = (float)g.dims[k];
        if (d[k] != 0.0f) {
            const float rk = 1.0f / d[k];
            const float ta = (0.0f - o[k]) * rk;
            const float tb = (D - o[k]) * rk;
            t0 = fmaxf(t0, fminf(ta, tb));
            t1 = fminf(t1, fmaxf(ta, tb));
        } else if (o[k] < 0.0f || o[k] > D) {
            hit = false;
        }
    }
    for (int c = 0; c < V.n_clip; c++) {
        const float *pl = V.clip[c];
        const float nd = (pl[0] * d[0] + pl[1] * d[1]) + pl[2] * d[2];
        const float no = (pl[0] * o[0] + pl[1] * o[1]) + pl[2] * o[2];
        const float num = pl[3] - no;
        if (nd > 0.0f) t0 = fmaxf(t0, num / nd);
        else if (nd < 0.0f) t1 = fminf(t1, num / nd);
        else if (no < pl[3]) hit = false;
    }
    if (!(t0 < t1)) hit = false;
    int L;
    if (V.lod >= 0) {
        L = min(V.lod, g.N);
    } else {
        const float w = t0 * V.klod;
        L = (w > 0.0f && w < INFINITY) ? min(max(ilogbf(w), 0), g.N) : 0;
    }

    // ---- march
    const float step = V.step;
    const float ert_T = V.ert < 1.0f ? 1.0f - V.ert : -1.0f;
    const float scaleL = __builtin_ldexpf(1.0f, -L);
    const int S = g.M + 2;
    const int G = g.grid[L];
    const int coff = g.cell_off[L];
    const int csz = g.M << L;  // cell edge in level-0 voxels
    const float invd[3] = {d[0] != 0.0f ? 1.0f / d[0] : INFINITY,
                           d[1] != 0.0f ? 1.0f / d[1] : INFINITY,
                           d[2] != 0.0f ? 1.0f / d[2] : INFINITY};

    float Tr = 1.0f, Cr = 0.0f, Cg = 0.0f, Cb = 0.0f;
    int k = 0, composited = 0, trilinear = 0;
    int blo[3] = {1, 1, 1}, bhi[3] = {0, 0, 0};  // cached cell, level-0 voxel box (inclusive)
    int kind = kAvg;
    const uint8_t *base = nullptr;
    float org[3] = {0.0f, 0.0f, 0.0f};
    float arg[C][4];

    while (hit) {
        const float tk = t0 + (float)k * step;
        if (!(tk < t1)) break;
        float p[3];
        int v[3];
#pragma unroll
        for (int q = 0; q < 3; q++) {
            const float m = tk * d[q];
            p[q] = o[q] + m;
            v[q] = min(max((int)floorf(p[q]), 0), g.dims[q] - 1);
        }
        if (v[0] < blo[0] || v[0] > bhi[0] || v[1] < blo[1] || v[1] > bhi[1] || v[2] < blo[2] ||
            v[2] > bhi[2]) {
            int cx = v[0] / csz, cy = v[1] / csz, cz = v[2] / csz;
            const DevCell &cell = table[coff + (cz * G + cy) * G + cx];
            const float4 clo = *(const float4 *)cell.lo, chi = *(const float4 *)cell.hi;
            const float lo4[4] = {clo.x, clo.y, clo.z, clo.w}, hi4[4] = {chi.x, chi.y, chi.z, chi.w};
            if (V.skip && cell_transparent<C>(lo4, hi4, V, s_pref)) {
                // widen to the largest transparent ancestor, then jump to (just before) its exit
                int lev = L, ax = cx, ay = cy, az = cz;
                while (lev < g.N) {
                    const int pg = g.grid[lev + 1];
                    const DevCell &pc =
                        table[g.cell_off[lev + 1] + ((az >> 1) * pg + (ay >> 1)) * pg + (ax >> 1)];
                    const float4 plo = *(const float4 *)pc.lo, phi = *(const float4 *)pc.hi;
                    const float l4[4] = {plo.x, plo.y, plo.z, plo.w};
                    const float h4[4] = {phi.x, phi.y, phi.z, phi.w};
                    if (!cell_transparent<C>(l4, h4, V, s_pref)) break;
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
                const float kf = floorf((te - t0) / step) - 1.0f;
                k = (kf > (float)(k + 1)) ? (int)fminf(kf, 2.0e9f) : k + 1;
                blo[0] = 1;
                bhi[0] = 0;
                continue;
            }
            blo[0] = cx * csz; bhi[0] = blo[0] + csz - 1;
            blo[1] = cy * csz; bhi[1] = blo[1] + csz - 1;
            blo[2] = cz * csz; bhi[2] = blo[2] + csz - 1;
            kind = cell.kind;
            if (kind == kBrick) {
                base = pool + (uint64_t)cell.slot * brick_bytes;
                org[0] = (float)(cx * g.M - 1);
                org[1] = (float)(cy * g.M - 1);
                org[2] = (float)(cz * g.M - 1);
            } else {
#pragma unroll
                for (int c = 0; c < C; c++) {
                    float u = (cell.avg[c] - V.ulo[c]) * V.uscale[c];
                    u = fminf(fmaxf(u, 0.0f), 255.0f);
                    const float fi = fminf(floorf(u), 254.0f);
                    const float fr = u - fi;
                    const int i = (int)fi;
                    const float4 e0 = s_lut[c][i], e1 = s_lut[c][i + 1];
                    arg[c][0] = lerpf(e0.x, e1.x, fr);
                    arg[c][1] = lerpf(e0.y, e1.y, fr);
                    arg[c][2] = lerpf(e0.z, e1.z, fr);
                    arg[c][3] = lerpf(e0.w, e1.w, fr);
                }
            }
        }
        composited++;
        if (kind == kBrick) {
            trilinear++;
            float f[3];
            int ii[3];
#pragma unroll
            for (int q = 0; q < 3; q++) {
                const float qq = p[q] * scaleL - 0.5f;
                const float lq = qq - org[q];
                const float fl = floorf(lq);
                f[q] = lq - fl;
                // inside the node, lq lies in [0.5, M + 0.5); the clamp only guards the
                // bordered brick against addressing outside itself
                ii[q] = min(max((int)fl, 0), S - 2);
            }
            float s[C];
            if constexpr (sizeof(T) == 2) {
                const uint8_t *a0 = base + (uint64_t)(((ii[2] * S + ii[1]) * S + ii[0]) * 8);
                const uint8_t *a1 = a0 + (uint64_t)S * S * 8;
                const uint2 w000 = *(const uint2 *)(a0);
                const uint2 w100 = *(const uint2 *)(a0 + 8);
                const uint2 w010 = *(const uint2 *)(a0 + S * 8);
                const uint2 w110 = *(const uint2 *)(a0 + S * 8 + 8);
                const uint2 w001 = *(const uint2 *)(a1);
                const uint2 w101 = *(const uint2 *)(a1 + 8);
                const uint2 w011 = *(const uint2 *)(a1 + S * 8);
                const uint2 w111 = *(const uint2 *)(a1 + S * 8 + 8);
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
                const float4 *a0 = (const float4 *)(base) + ((ii[2] * S + ii[1]) * S + ii[0]);
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
#pragma unroll
            for (int c = 0; c < C; c++) {
                float u = (s[c] - V.ulo[c]) * V.uscale[c];
                u = fminf(fmaxf(u, 0.0f), 255.0f);
                const float fi = fminf(floorf(u), 254.0f);
                const float fr = u - fi;
                const int i = (int)fi;
                const float4 e0 = s_lut[c][i], e1 = s_lut[c][i + 1];
                const float al = lerpf(e0.w, e1.w, fr);
                const float wgt = Tr * al;
                Cr = __builtin_fmaf(wgt, lerpf(e0.x, e1.x, fr), Cr);
                Cg = __builtin_fmaf(wgt, lerpf(e0.y, e1.y, fr), Cg);
                Cb = __builtin_fmaf(wgt, lerpf(e0.z, e1.z, fr), Cb);
                Tr = Tr - wgt;
            }
        } else {
#pragma unroll
            for (int c = 0; c < C; c++) {
                const float wgt = Tr * arg[c][3];
                Cr = __builtin_fmaf(wgt, arg[c][0], Cr);
                Cg = __builtin_fmaf(wgt, arg[c][1], Cg);
                Cb = __builtin_fmaf(wgt, arg[c][2], Cb);
                Tr = Tr - wgt;
            }
        }
        if (Tr <= ert_T) break;
        k++;
    }

    if (inside) {
        float4 out = make_float4(Cr, Cg, Cb, 1.0f - Tr);
        *(float4 *)(V.image + ((int64_t)px_j * V.width + px_i) * 4) = out;
    }
    if (counters) {
        int nominal = 0;
        if (hit) {
            // positions t_k < t1: start from the estimate and settle with the exact test
            int kk = max((int)((t1 - t0) / step) - 2, 0);
            while (t0 + (float)kk * step < t1) kk++;
            nominal = kk;
        }
        unsigned long long r = hit ? 1ull : 0ull, nn = (unsigned long long)nominal,
                           cc = (unsigned long long)composited, tt = (unsigned long long)trilinear;
        for (int off = 32; off > 0; off >>= 1) {
            r += __shfl_xor(r, off, 64);
            nn += __shfl_xor(nn, off, 64);
            cc += __shfl_xor(cc, off, 64);
            tt += __shfl_xor(tt, off, 64);
        }
        if (lane == 0) {
            atomicAdd(&counters->rays, r);
            atomicAdd(&counters->nominal, nn);
            atomicAdd(&counters->composited, cc);
            atomicAdd(&counters->trilinear, tt);
        }
    }
}

template <typename T>
hipError_t launch_typed(const VolGeom &g, const DevCell *table, const void *pool,
                        uint64_t brick_bytes, const DevView *views, const WgItem *items,
                        int n_items, RenderCounters *counters, hipStream_t s)
{
    const dim3 grid(n_items), block(kThreads);
    const uint8_t *p = (const uint8_t *)pool;
    switch (g.C) {
    case 1: hipLaunchKernelGGL((k_render<T, 1>), grid, block, 0, s, g, table, p, brick_bytes, views, items, counters); break;
    case 2: hipLaunchKernelGGL((k_render<T, 2>), grid, block, 0, s, g, table, p, brick_bytes, views, items, counters); break;
    case 3: hipLaunchKernelGGL((k_render<T, 3>), grid, block, 0, s, g, table, p, brick_bytes, views, items, counters); break;
    default: hipLaunchKernelGGL((k_render<T, 4>), grid, block, 0, s, g, table, p, brick_bytes, views, items, counters); break;
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_render(const VolGeom &g, const DevCell *table, const void *pool,
                         uint64_t brick_bytes, const DevView *views, const WgItem *items,
                         int n_items, RenderCounters *counters, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    if (g.dtype == 0)
        return launch_typed<uint16_t>(g, table, pool, brick_bytes, views, items, n_items, counters, s);
    return launch_typed<float>(g, table, pool, brick_bytes, views, items, n_items, counters, s);
}

}  // namespace octrc
