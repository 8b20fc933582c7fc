// Construction kernels: block insertion, 2x2x2 half-sampling, per-cell statistics, node-table
// change events, bordered-brick gather and skip-range propagation.
//
// The master mipmap lives in HBM as dense planar levels ([C][ez][ey][ex] per level, level L
// valid extent ceil(D/2^L)), which makes insertion a coalesced copy and half-sampling a
// streaming pass; the renderer reads a separate pool of bordered, channel-interleaved bricks.
#include "internal.h"

#include <float.h>

#include <algorithm>

namespace octrc {

namespace {

constexpr int kThreads = 256;

template <typename T>
__device__ inline T *level_ptr(T *master, const VolGeom &g, int L, int c)
{
    const int64_t n = (int64_t)g.ext[L][0] * g.ext[L][1] * g.ext[L][2];
    return master + g.lvl_off[L] + (int64_t)c * n;
}

// ---------------------------------------------------------------------------------------
// Step 1 of incremental construction: copy a block into level 0 and record which channels
// of each voxel have been inserted (completeness tracking).
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_insert(VolGeom g, T *master, uint8_t *mask, const T *src, int channel, int x0, int y0, int z0,
         int nx, int ny, int nz)
{
    const int x = blockIdx.x * kThreads + threadIdx.x;
    if (x >= nx) return;
    const int cb = channel < 0 ? g.C : 1;
    const int64_t nvox0 = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
    for (int row = blockIdx.y; row < ny * nz; row += gridDim.y) {
        const int y = row % ny, z = row / ny;
        const int64_t lin = ((int64_t)(z0 + z) * g.dims[1] + (y0 + y)) * g.dims[0] + (x0 + x);
        uint32_t bits = 0;
        for (int c = 0; c < cb; c++) {
            const int ch = channel < 0 ? c : channel;
            master[g.lvl_off[0] + (int64_t)ch * nvox0 + lin] =
                src[(((int64_t)c * nz + z) * ny + y) * nx + x];
            bits |= 1u << ch;
        }
        mask[lin] = (uint8_t)(mask[lin] | bits);
    }
}

// ---------------------------------------------------------------------------------------
// Step 2: parent[i] = mean of the valid children 2i+d (d in {0,1}^3, 2i+d < ext_L).
// uint16: floor((2s + n) / (2n)) -- integer mean, halves rounded up; n is 1, 2, 4 or 8 so the
// division is a shift.  float32: the children are summed in double (exact for 8 floats of
// similar magnitude) and scaled by 1/n (a power of two), then rounded once to float.
__device__ inline uint32_t mean_rhu(uint32_t s, uint32_t n)
{
    const uint32_t sh = n == 8 ? 4u : n == 4 ? 3u : n == 2 ? 2u : 1u;  // log2(2n)
    return (2u * s + n) >> sh;
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_downsample(VolGeom g, T *master, int L, int lx, int ly, int lz, int hx, int hy, int hz)
{
    const int x = lx + blockIdx.x * kThreads + threadIdx.x;
    if (x > hx) return;
    const int ex = g.ext[L][0], ey = g.ext[L][1], ez = g.ext[L][2];
    const int px = g.ext[L + 1][0], py = g.ext[L + 1][1];
    const int ny = hy - ly + 1, nz = hz - lz + 1;
    const int cx0 = 2 * x, cx1 = min(2 * x + 1, ex - 1);
    const uint32_t nxv = (2 * x + 1 < ex) ? 2u : 1u;
    for (int row = blockIdx.y; row < ny * nz; row += gridDim.y) {
        const int y = ly + row % ny, z = lz + row / ny;
        const uint32_t nyv = (2 * y + 1 < ey) ? 2u : 1u, nzv = (2 * z + 1 < ez) ? 2u : 1u;
        const uint32_t n = nxv * nyv * nzv;
        for (int c = 0; c < g.C; c++) {
            const T *src = level_ptr(master, g, L, c);
            T *dst = level_ptr(master, g, L + 1, c);
            if constexpr (sizeof(T) == 2) {
                uint32_t s = 0;
                for (uint32_t dz = 0; dz < nzv; dz++)
                    for (uint32_t dy = 0; dy < nyv; dy++) {
                        const T *r = src + ((int64_t)(2 * z + dz) * ey + (2 * y + dy)) * ex;
                        s += r[cx0];
                        if (nxv == 2) s += r[cx1];
                    }
                dst[((int64_t)z * py + y) * px + x] = (T)mean_rhu(s, n);
            } else {
                double s = 0.0;
                for (uint32_t dz = 0; dz < nzv; dz++)
                    for (uint32_t dy = 0; dy < nyv; dy++) {
                        const T *r = src + ((int64_t)(2 * z + dz) * ey + (2 * y + dy)) * ex;
                        s += (double)r[cx0];
                        if (nxv == 2) s += (double)r[cx1];
                    }
                dst[((int64_t)z * py + y) * px + x] = (float)(s * (1.0 / (double)n));
            }
        }
    }
}

// ---------------------------------------------------------------------------------------
// Block-wide reductions over kWaves waves of 64 (scratch: kWaves values).
template <typename V, typename Op, int kWaves = kThreads / 64>
__device__ inline V block_reduce(V v, Op op, V *scratch)
{
    for (int o = 32; o > 0; o >>= 1) v = op(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0) scratch[w] = v;
    __syncthreads();
    V r = scratch[0];
    for (int i = 1; i < kWaves; i++) r = op(r, scratch[i]);
    return r;
}

struct MinOp { __device__ double operator()(double a, double b) const { return fmin(a, b); } };
struct MaxOp { __device__ double operator()(double a, double b) const { return fmax(a, b); } };
struct AddD { __device__ double operator()(double a, double b) const { return a + b; } };
struct AddU { __device__ unsigned long long operator()(unsigned long long a,
                                                       unsigned long long b) const { return a + b; } };

// Step 3 inputs: min / max / sum of a cell's valid voxels per channel (+ inserted counts at
// level 0).  Pass 1 spreads each listed cell over `nsub` workgroups (slabs of z-slices) that
// write partial results; pass 2 folds the partials of a cell in a fixed order, so the sums
// (integers for u16, doubles for f32) do not depend on scheduling.
struct StatPart {
    float mn[kMaxC], mx[kMaxC];
    double sum[kMaxC];
    uint32_t ins[kMaxC];
};

struct MinF { __device__ float operator()(float a, float b) const { return fminf(a, b); } };
struct MaxF { __device__ float operator()(float a, float b) const { return fmaxf(a, b); } };

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_stats_part(VolGeom g, const T *master, const uint8_t *mask, const int4 *cells, int nsub,
             StatPart *part)
{
    __shared__ float sf[kThreads / 64];
    __shared__ double sd[kThreads / 64];
    __shared__ unsigned long long su[kThreads / 64];
    const int4 cl = cells[blockIdx.x / nsub];
    const int sub = blockIdx.x % nsub;
    const int L = cl.x;
    const int b[3] = {cl.y, cl.z, cl.w};
    int lo[3], n[3];
    for (int a = 0; a < 3; a++) {
        lo[a] = b[a] * g.M;
        n[a] = min(g.M, g.ext[L][a] - lo[a]);
    }
    const int zc = (n[2] + nsub - 1) / nsub;
    const int zs = min(sub * zc, n[2]), ze = min(zs + zc, n[2]);
    const int rstep = kThreads / n[0];            // rows per pass (n[0] <= 128)
    const int x = threadIdx.x % n[0], r0 = threadIdx.x / n[0];
    const bool on = r0 < rstep;
    const int ex = g.ext[L][0], ey = g.ext[L][1];
    StatPart *o = part + blockIdx.x;
    for (int c = 0; c < g.C; c++) {
        const T *src = level_ptr(master, g, L, c);
        float mn = FLT_MAX, mx = -FLT_MAX;
        double sm = 0.0;
        uint32_t su_local = 0;
        if (on)
            for (int z = zs; z < ze; z++)
                for (int y = r0; y < n[1]; y += rstep) {
                    const T v = src[((int64_t)(lo[2] + z) * ey + (lo[1] + y)) * ex + (lo[0] + x)];
                    mn = fminf(mn, (float)v);
                    mx = fmaxf(mx, (float)v);
                    if constexpr (sizeof(T) == 2) su_local += v;
                    else sm += (double)v;
                }
        mn = block_reduce(mn, MinF{}, sf);
        mx = block_reduce(mx, MaxF{}, sf);
        if constexpr (sizeof(T) == 2)
            sm = (double)block_reduce((unsigned long long)su_local, AddU{}, su);
        else
            sm = block_reduce(sm, AddD{}, sd);
        if (threadIdx.x == 0) {
            o->mn[c] = mn;
            o->mx[c] = mx;
            o->sum[c] = sm;
        }
    }
    uint32_t cnt[kMaxC] = {0, 0, 0, 0};
    if (L == 0 && on)
        for (int z = zs; z < ze; z++)
            for (int y = r0; y < n[1]; y += rstep) {
                const uint32_t bits = mask[((int64_t)(lo[2] + z) * g.dims[1] + (lo[1] + y)) *
                                               g.dims[0] + (lo[0] + x)];
                for (int c = 0; c < kMaxC; c++) cnt[c] += (bits >> c) & 1u;
            }
    for (int c = 0; c < g.C; c++) {
        const unsigned long long t = block_reduce((unsigned long long)cnt[c], AddU{}, su);
        if (threadIdx.x == 0) o->ins[c] = (uint32_t)t;
    }
}

__global__ void __launch_bounds__(kThreads)
k_stats_fold(int n, int nsub, int C, const StatPart *part, CellStat *out)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    CellStat r;
    for (int c = 0; c < kMaxC; c++) {
        float mn = FLT_MAX, mx = -FLT_MAX;
        double sm = 0.0;
        uint32_t ins = 0;
        if (c < C)
            for (int k = 0; k < nsub; k++) {
                const StatPart &p = part[(int64_t)i * nsub + k];
                mn = fminf(mn, p.mn[c]);
                mx = fmaxf(mx, p.mx[c]);
                sm += p.sum[c];
                ins += p.ins[c];
            }
        r.mn[c] = c < C ? (double)mn : 0.0;
        r.mx[c] = c < C ? (double)mx : 0.0;
        r.sum[c] = sm;
        r.ins[c] = ins;
    }
    out[i] = r;
}

// ---------------------------------------------------------------------------------------
// Change events ("Incremental Octree Updates on the GPU"): rewrite the listed node-table
// entries.  The bounds lo/hi are recomputed afterwards by k_ranges.
__global__ void __launch_bounds__(kThreads)
k_apply_deltas(DevCell *table, float *miss_range, const CellDelta *d, int n)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    DevCell &c = table[d[i].index];
    c.kind = d[i].kind;
    c.slot = d[i].slot;
    for (int k = 0; k < 4; k++) {
        c.avg[k] = d[i].avg[k];
        miss_range[(int64_t)d[i].index * 8 + k] = d[i].lo[k];
        miss_range[(int64_t)d[i].index * 8 + 4 + k] = d[i].hi[k];
    }
}

// ---------------------------------------------------------------------------------------
// Bordered brick gather ("Filtering across Brick Boundaries"): slot <- R_L over
// [b*M-1, b*M+M]^3 with indices clamped to the valid extent, where R_L is the level-L data
// inside brick cells and the cell's AVG elsewhere.  Channels are interleaved and padded to
// four lanes, so one 8-byte (u16) or 16-byte (f32) load fetches a voxel of every channel.
// A job rebuilds the whole brick or only the sub-box its inserted data touched.  It also
// reduces the per-channel min/max of what it wrote: the slot's skip range is replaced by a
// whole-brick job and widened by a partial one (a superset stays a valid bound).
// One 256-thread workgroup per job; thread t owns (x, y) columns t, t + 256, ... of the job's
// sub-box and walks z, four slices per round so that several rows of loads are in flight
// (the job's rows are short, 34 voxels for 32^3 bricks: a thread-per-row walk is
// latency-bound).  Uploads run while renders occupy most wave slots of every CU: 4-wave
// workgroups fit beside them, 16-wave ones waited for whole CUs to drain.
#ifndef OCTRC_GATHER_THREADS
#define OCTRC_GATHER_THREADS 256
#endif
constexpr int kGatherThreads = OCTRC_GATHER_THREADS;

template <typename T>
__global__ void __launch_bounds__(kGatherThreads)
k_gather(VolGeom g, const T *master, const DevCell *table, uint8_t *pool, uint64_t brick_bytes,
         const BrickJob *jobs, float *slot_range, float background)
{
    __shared__ int s_kind[27];
    __shared__ float s_avg[27][4];
    __shared__ float sf[kGatherThreads / 64];
    const BrickJob job = jobs[blockIdx.x];
    const int L = job.level, M = g.M, S = M + 2, G = g.grid[L];
    const int b[3] = {job.bx, job.by, job.bz};
    if (threadIdx.x < 27) {
        const int dx = threadIdx.x % 3 - 1, dy = (threadIdx.x / 3) % 3 - 1, dz = threadIdx.x / 9 - 1;
        const int cx = b[0] + dx, cy = b[1] + dy, cz = b[2] + dz;
        int kind = kAvg;
        float avg[4] = {background, background, background, background};
        if (cx >= 0 && cy >= 0 && cz >= 0 && cx < G && cy < G && cz < G) {
            const DevCell &c = table[g.cell_off[L] + ((int64_t)cz * G + cy) * G + cx];
            kind = c.kind;
            for (int k = 0; k < 4; k++) avg[k] = c.avg[k];
        }
        s_kind[threadIdx.x] = kind;
        for (int k = 0; k < 4; k++) s_avg[threadIdx.x][k] = avg[k];
    }
    __syncthreads();
    const int ex = g.ext[L][0], ey = g.ext[L][1], ez = g.ext[L][2];
    const int64_t nlev = (int64_t)ex * ey * ez;
    const T *src = master + g.lvl_off[L];
    float mn[kMaxC], mx[kMaxC];
    for (int c = 0; c < kMaxC; c++) {
        mn[c] = FLT_MAX;
        mx[c] = -FLT_MAX;
    }
    T *dst = (T *)(pool + (uint64_t)job.slot * brick_bytes);
    const int nx = job.hi[0] - job.lo[0] + 1, ny = job.hi[1] - job.lo[1] + 1;
    for (int j = threadIdx.x; j < nx * ny; j += kGatherThreads) {
        const int x = job.lo[0] + j % nx, y = job.lo[1] + j / nx;
        // bordered position -> clamped level index, and which of the 3x3x3 neighbours holds it
        const int gx = min(max(b[0] * M - 1 + x, 0), ex - 1);
        const int ox = gx < b[0] * M ? 0 : (gx >= b[0] * M + M ? 2 : 1);
        const int gy = min(max(b[1] * M - 1 + y, 0), ey - 1);
        const int oy = gy < b[1] * M ? 0 : (gy >= b[1] * M + M ? 2 : 1);
        const int64_t row = (int64_t)gy * ex + gx;
#pragma unroll 4
        for (int z = job.lo[2]; z <= job.hi[2]; z++) {
            const int gz = min(max(b[2] * M - 1 + z, 0), ez - 1);
            const int oz = gz < b[2] * M ? 0 : (gz >= b[2] * M + M ? 2 : 1);
            const int nb = (oz * 3 + oy) * 3 + ox;
            T v[4];
            if (s_kind[nb] != kAvg) {
                const int64_t lin = (int64_t)gz * ey * ex + row;
                for (int c = 0; c < 4; c++) v[c] = c < g.C ? src[(int64_t)c * nlev + lin] : (T)0;
            } else {
                for (int c = 0; c < 4; c++) v[c] = c < g.C ? (T)s_avg[nb][c] : (T)0;
            }
            for (int c = 0; c < kMaxC; c++)
                if (c < g.C) {
                    mn[c] = fminf(mn[c], (float)v[c]);
                    mx[c] = fmaxf(mx[c], (float)v[c]);
                }
            const int64_t i = ((int64_t)z * S + y) * S + x;
            if constexpr (sizeof(T) == 2) {
                *(ushort4 *)(dst + i * 4) = make_ushort4(v[0], v[1], v[2], v[3]);
            } else {
                *(float4 *)(dst + i * 4) = make_float4(v[0], v[1], v[2], v[3]);
            }
        }
    }
    for (int c = 0; c < g.C; c++) {
        const float lo = block_reduce<float, MinF, kGatherThreads / 64>(mn[c], MinF{}, sf);
        const float hi = block_reduce<float, MaxF, kGatherThreads / 64>(mx[c], MaxF{}, sf);
        if (threadIdx.x == 0) {
            float *r = slot_range + (int64_t)job.slot * 8;
            r[c] = job.full ? lo : fminf(r[c], lo);
            r[4 + c] = job.full ? hi : fmaxf(r[4 + c], hi);
        }
    }
}

// ---------------------------------------------------------------------------------------
// Skip bounds, bottom-up one level per launch: a cell's [lo, hi] covers its own sampled
// values (bordered-brick range for a resident brick, a bound of the brick's values for a
// missing one -- so a missing brick is still requested unless it is surely empty -- and the
// AVG otherwise) and those of its eight children, so any ancestor whose range maps to zero
// opacity is empty at every LOD.
__global__ void __launch_bounds__(kThreads)
k_ranges(VolGeom g, DevCell *table, const float *slot_range, const float *miss_range, int L)
{
    const int G = g.grid[L];
    const int64_t n = (int64_t)G * G * G;
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    DevCell &c = table[g.cell_off[L] + i];
    float lo[4], hi[4];
    for (int k = 0; k < 4; k++) {
        if (c.kind == kBrick) {
            lo[k] = slot_range[(int64_t)c.slot * 8 + k];
            hi[k] = slot_range[(int64_t)c.slot * 8 + 4 + k];
        } else if (c.kind == kBrickMissing) {
            const int64_t ci = g.cell_off[L] + i;
            lo[k] = fminf(c.avg[k], miss_range[ci * 8 + k]);
            hi[k] = fmaxf(c.avg[k], miss_range[ci * 8 + 4 + k]);
        } else {
            lo[k] = hi[k] = c.avg[k];
        }
    }
    if (L > 0) {
        const int x = (int)(i % G), y = (int)((i / G) % G), z = (int)(i / ((int64_t)G * G));
        const int Gc = 2 * G;
        for (int d = 0; d < 8; d++) {
            const int cx = 2 * x + (d & 1), cy = 2 * y + ((d >> 1) & 1), cz = 2 * z + (d >> 2);
            const DevCell &ch = table[g.cell_off[L - 1] + ((int64_t)cz * Gc + cy) * Gc + cx];
            for (int k = 0; k < 4; k++) {
                lo[k] = fminf(lo[k], ch.lo[k]);
                hi[k] = fmaxf(hi[k], ch.hi[k]);
            }
        }
    }
    for (int k = 0; k < 4; k++) {
        c.lo[k] = lo[k];
        c.hi[k] = hi[k];
    }
}

template <typename T>
__global__ void __launch_bounds__(kThreads)
k_fill(T *p, int64_t n, T v)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * kThreads)
        p[i] = v;
}

inline unsigned ceil_div(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

hipError_t launch_insert(const VolGeom &g, void *master, uint8_t *mask, const void *src,
                         int channel, const int32_t o[3], const int32_t n[3], hipStream_t s)
{
    dim3 grid(ceil_div(n[0], kThreads), (unsigned)std::min<int64_t>((int64_t)n[1] * n[2], 65535));
    if (g.dtype == 0)
        hipLaunchKernelGGL(k_insert<uint16_t>, grid, dim3(kThreads), 0, s, g, (uint16_t *)master,
                           mask, (const uint16_t *)src, channel, o[0], o[1], o[2], n[0], n[1], n[2]);
    else
        hipLaunchKernelGGL(k_insert<float>, grid, dim3(kThreads), 0, s, g, (float *)master, mask,
                           (const float *)src, channel, o[0], o[1], o[2], n[0], n[1], n[2]);
    return hipGetLastError();
}

hipError_t launch_downsample(const VolGeom &g, void *master, int L, const int32_t lo[3],
                             const int32_t hi[3], hipStream_t s)
{
    const int64_t rows = (int64_t)(hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1);
    dim3 grid(ceil_div(hi[0] - lo[0] + 1, kThreads), (unsigned)std::min<int64_t>(rows, 65535));
    if (g.dtype == 0)
        hipLaunchKernelGGL(k_downsample<uint16_t>, grid, dim3(kThreads), 0, s, g,
                           (uint16_t *)master, L, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]);
    else
        hipLaunchKernelGGL(k_downsample<float>, grid, dim3(kThreads), 0, s, g, (float *)master, L,
                           lo[0], lo[1], lo[2], hi[0], hi[1], hi[2]);
    return hipGetLastError();
}

size_t stats_scratch_bytes(const VolGeom &g, int n)
{
    return (size_t)n * (size_t)std::max(1, g.M / 4) * sizeof(StatPart);
}

hipError_t launch_stats(const VolGeom &g, const void *master, const uint8_t *mask,
                        const int32_t *cells, int n, void *scratch, CellStat *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int nsub = std::max(1, g.M / 4);
    StatPart *part = (StatPart *)scratch;
    if (g.dtype == 0)
        hipLaunchKernelGGL(k_stats_part<uint16_t>, dim3(n * nsub), dim3(kThreads), 0, s, g,
                           (const uint16_t *)master, mask, (const int4 *)cells, nsub, part);
    else
        hipLaunchKernelGGL(k_stats_part<float>, dim3(n * nsub), dim3(kThreads), 0, s, g,
                           (const float *)master, mask, (const int4 *)cells, nsub, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stats_fold, dim3(ceil_div(n, kThreads)), dim3(kThreads), 0, s, n, nsub,
                       g.C, part, out);
    return hipGetLastError();
}

hipError_t launch_apply_deltas(DevCell *table, float *miss_range, const CellDelta *d, int n,
                               hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_apply_deltas, dim3(ceil_div(n, kThreads)), dim3(kThreads), 0, s, table,
                       miss_range, d, n);
    return hipGetLastError();
}

hipError_t launch_gather(const VolGeom &g, const void *master, const DevCell *table, void *pool,
                         uint64_t brick_bytes, const BrickJob *jobs, int n, float *slot_range,
                         float background, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    if (g.dtype == 0)
        hipLaunchKernelGGL(k_gather<uint16_t>, dim3(n), dim3(kGatherThreads), 0, s, g,
                           (const uint16_t *)master, table, (uint8_t *)pool, brick_bytes, jobs,
                           slot_range, background);
    else
        hipLaunchKernelGGL(k_gather<float>, dim3(n), dim3(kGatherThreads), 0, s, g, (const float *)master,
                           table, (uint8_t *)pool, brick_bytes, jobs, slot_range, background);
    return hipGetLastError();
}

hipError_t launch_ranges(const VolGeom &g, DevCell *table, const float *slot_range,
                         const float *miss_range, hipStream_t s)
{
    for (int L = 0; L <= g.N; L++) {
        const int64_t n = (int64_t)g.grid[L] * g.grid[L] * g.grid[L];
        hipLaunchKernelGGL(k_ranges, dim3(ceil_div(n, kThreads)), dim3(kThreads), 0, s, g, table,
                           slot_range, miss_range, L);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<uint8_t>, dim3((unsigned)std::min<int64_t>(ceil_div(n, kThreads), 65536)),
                       dim3(kThreads), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, int64_t n, float v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<float>, dim3((unsigned)std::min<int64_t>(ceil_div(n, kThreads), 65536)),
                       dim3(kThreads), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_clear(const VolGeom &g, void *master, uint8_t *mask, double background,
                        hipStream_t s)
{
    const int64_t n = g.lvl_off[g.N + 1];
    const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(n, kThreads), 65536);
    if (g.dtype == 0)
        hipLaunchKernelGGL(k_fill<uint16_t>, dim3(blocks), dim3(kThreads), 0, s, (uint16_t *)master,
                           n, (uint16_t)background);
    else
        hipLaunchKernelGGL(k_fill<float>, dim3(blocks), dim3(kThreads), 0, s, (float *)master, n,
                           (float)background);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nm = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
    hipLaunchKernelGGL(k_fill<uint8_t>, dim3((unsigned)std::min<int64_t>(ceil_div(nm, kThreads), 65536)),
                       dim3(kThreads), 0, s, mask, nm, (uint8_t)0);
    return hipGetLastError();
}

}  // namespace octrc
