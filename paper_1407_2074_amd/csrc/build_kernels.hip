// Construction kernels: block insertion, 2x2x2 half-sampling, per-cell statistics, node-table
// change events, bordered-brick gather and skip-range propagation.
//
// The master mipmap lives in HBM (or pinned host memory) as dense planar levels ([C][ez][ey][ex] per level, level L
// valid extent ceil(D/2^L)), which makes insertion a coalesced copy and half-sampling a
// streaming pass; the renderer reads a separate pool of bordered, channel-interleaved bricks.
#include "internal.h"

#include <float.h>

#include <algorithm>
#include <type_traits>

namespace octrc {

namespace {

constexpr int kThreads = 256;
constexpr int kXcds = 8;        // MI355X: 8 XCDs of 32 CUs, one L2 each

// Eight consecutive elements moved as 16-byte words (one for uint16, two for float32).
template <typename T> struct Pack8;
typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef unsigned int u32x2_t __attribute__((ext_vector_type(2)));
template <> struct Pack8<uint16_t> {
    uint4 w;
    __device__ static Pack8 load(const uint16_t *p) { return {*(const uint4 *)p}; }
    // streaming read (nontemporal hint): for data read once that should not displace what the
    // next kernels read from the caches
    __device__ static Pack8 load_nt(const uint16_t *p)
    {
        const u32x4_t v = __builtin_nontemporal_load((const u32x4_t *)p);
        return {make_uint4(v.x, v.y, v.z, v.w)};
    }
    __device__ void store(uint16_t *p) const { *(uint4 *)p = w; }
    __device__ void store_nt(uint16_t *p) const
    {
        const u32x4_t v = {w.x, w.y, w.z, w.w};
        __builtin_nontemporal_store(v, (u32x4_t *)p);
    }
    __device__ uint32_t at(int i) const
    {
        const uint32_t d = i < 2 ? w.x : i < 4 ? w.y : i < 6 ? w.z : w.w;
        return (i & 1) ? d >> 16 : d & 0xffffu;
    }
};
template <> struct Pack8<float> {
    float4 a, b;
    __device__ static Pack8 load(const float *p) { return {((const float4 *)p)[0], ((const float4 *)p)[1]}; }
    __device__ static Pack8 load_nt(const float *p)
    {
        const f32x4_t a = __builtin_nontemporal_load((const f32x4_t *)p);
        const f32x4_t b = __builtin_nontemporal_load((const f32x4_t *)p + 1);
        return {make_float4(a.x, a.y, a.z, a.w), make_float4(b.x, b.y, b.z, b.w)};
    }
    __device__ void store(float *p) const
    {
        ((float4 *)p)[0] = a;
        ((float4 *)p)[1] = b;
    }
    __device__ void store_nt(float *p) const
    {
        const f32x4_t u = {a.x, a.y, a.z, a.w}, v = {b.x, b.y, b.z, b.w};
        __builtin_nontemporal_store(u, (f32x4_t *)p);
        __builtin_nontemporal_store(v, (f32x4_t *)p + 1);
    }
    __device__ float at(int i) const
    {
        const float4 &q = i < 4 ? a : b;
        const int j = i & 3;
        return j == 0 ? q.x : j == 1 ? q.y : j == 2 ? q.z : q.w;
    }
};

// ---------------------------------------------------------------------------------------
// Step 1 of incremental construction: copy a block into level 0 and record which channels
// of each voxel have been inserted (completeness tracking).  Two forms: k_insert8 moves eight
// voxels per thread with 16-byte accesses (block origin, width and row pitches multiples of
// eight, 16-byte-aligned source and rows); k_insert takes any block, one voxel per thread.
// The source block has row / slice / channel pitches sp_y / sp_z / sp_c (elements).
// k_insert8 reads the source and writes level 0 as streaming (nontemporal) accesses: neither
// is read again by this launch (measured: 0.19 -> 0.15 ms for a 0.94 GB whole-volume insert).
template <typename T, bool kPaged>
__global__ void __launch_bounds__(kThreads)
k_insert8(VolGeom g, MasterRef<T> mr, uint8_t *__restrict__ mask, const T *__restrict__ src,
          int64_t sp_y, int64_t sp_z, int64_t sp_c, int channel, int x0, int y0, int z0, int nx,
          int ny, int nz)
{
    const int nq = nx >> 3;
    const int64_t items = (int64_t)nq * ny * nz;
    const int cb = channel < 0 ? g.C : 1;
    uint32_t bits = 0;
    for (int c = 0; c < cb; c++) bits |= 1u << (channel < 0 ? c : channel);
    const uint32_t bits4 = bits * 0x01010101u;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < items;
         i += (int64_t)gridDim.x * kThreads) {
        const int q = (int)(i % nq);
        const int64_t row = i / nq;
        const int y = (int)(row % ny), z = (int)(row / ny);
        const int64_t lin = ((int64_t)(z0 + z) * g.dims[1] + (y0 + y)) * g.dims[0] + x0 + 8 * q;
        const int64_t sl = (int64_t)z * sp_z + (int64_t)y * sp_y + 8 * q;
        Pack8<T> v[kMaxC];
#pragma unroll
        for (int c = 0; c < kMaxC; c++)
            if (c < cb) v[c] = Pack8<T>::load_nt(src + c * sp_c + sl);   // the source is read once
        uint2 m = *(const uint2 *)(mask + lin);
#pragma unroll
        for (int c = 0; c < kMaxC; c++)
            if (c < cb)
                v[c].store_nt(melem<kPaged>(g, mr, 0, channel < 0 ? c : channel, x0 + 8 * q, y0 + y, z0 + z));
        m.x |= bits4;
        m.y |= bits4;
        *(uint2 *)(mask + lin) = m;
    }
}

template <typename T, bool kPaged>
__global__ void __launch_bounds__(kThreads)
k_insert(VolGeom g, MasterRef<T> mr, uint8_t *mask, const T *src, int64_t sp_y, int64_t sp_z,
         int64_t sp_c, int channel, int x0, int y0, int z0, int nx, int ny, int nz)
{
    const int x = blockIdx.x * kThreads + threadIdx.x;
    if (x >= nx) return;
    const int cb = channel < 0 ? g.C : 1;
    for (int row = blockIdx.y; row < ny * nz; row += gridDim.y) {
        const int y = row % ny, z = row / ny;
        const int64_t lin = ((int64_t)(z0 + z) * g.dims[1] + (y0 + y)) * g.dims[0] + (x0 + x);
        uint32_t bits = 0;
        for (int c = 0; c < cb; c++) {
            const int ch = channel < 0 ? c : channel;
            *melem<kPaged>(g, mr, 0, ch, x0 + x, y0 + y, z0 + z) =
                src[c * sp_c + (int64_t)z * sp_z + (int64_t)y * sp_y + x];
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

// Four parents along x per thread from 16-byte child loads.  Needs level L's rows and both
// levels' channel planes aligned to eight (L) and four (L + 1) elements; the host checks.
// The x range is widened to whole groups of four: a parent outside the requested range is
// recomputed from unchanged children, which rewrites the value it already holds.  Each child is
// read by one thread only, so the child rows are streaming reads; the parents stay cached for
// the next level.
template <typename T, bool kPaged>
__global__ void __launch_bounds__(kThreads)
k_downsample4(VolGeom g, MasterRef<T> mr, int L, int qx0, int nq, int ly, int lz, int ny, int nz)
{
    const int ey = g.ext[L][1], ez = g.ext[L][2];
    const int64_t items = (int64_t)nq * ny * nz;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < items;
         i += (int64_t)gridDim.x * kThreads) {
        const int x4 = 4 * (qx0 + (int)(i % nq));
        const int64_t row = i / nq;
        const int y = ly + (int)(row % ny), z = lz + (int)(row / ny);
        const int nyv = (2 * y + 1 < ey) ? 2 : 1, nzv = (2 * z + 1 < ez) ? 2 : 1;
        const uint32_t sh = 2u + (nyv == 2) + (nzv == 2);        // log2(2n), n = 2 nyv nzv
        const uint32_t n = 2u * nyv * nzv;
        for (int c = 0; c < g.C; c++) {
            T *dst = melem<kPaged>(g, mr, L + 1, c, x4, y, z);
            Pack8<T> r[4];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                const int dz = k >> 1, dy = k & 1;
                if (dz < nzv && dy < nyv)
                    r[k] = Pack8<T>::load_nt(melem<kPaged>(g, mr, L, c, 2 * x4, 2 * y + dy, 2 * z + dz));
            }
            if constexpr (sizeof(T) == 2) {
                uint32_t s[4] = {0, 0, 0, 0};
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const int dz = k >> 1, dy = k & 1;
                    if (dz < nzv && dy < nyv)
#pragma unroll
                        for (int j = 0; j < 4; j++) s[j] += r[k].at(2 * j) + r[k].at(2 * j + 1);
                }
                uint2 o;
                o.x = ((2u * s[0] + n) >> sh) | (((2u * s[1] + n) >> sh) << 16);
                o.y = ((2u * s[2] + n) >> sh) | (((2u * s[3] + n) >> sh) << 16);
                *(uint2 *)dst = o;
            } else {
                double s[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int k = 0; k < 4; k++) {
                    const int dz = k >> 1, dy = k & 1;
                    if (dz < nzv && dy < nyv)
#pragma unroll
                        for (int j = 0; j < 4; j++)
                            s[j] += (double)r[k].at(2 * j) + (double)r[k].at(2 * j + 1);
                }
                const double inv = 1.0 / (double)n;
                *(float4 *)dst = make_float4((float)(s[0] * inv), (float)(s[1] * inv),
                                             (float)(s[2] * inv), (float)(s[3] * inv));
            }
        }
    }
}

template <typename T, bool kPaged>
__global__ void __launch_bounds__(kThreads)
k_downsample(VolGeom g, MasterRef<T> mr, int L, int lx, int ly, int lz, int hx, int hy, int hz)
{
    const int x = lx + blockIdx.x * kThreads + threadIdx.x;
    if (x > hx) return;
    const int ex = g.ext[L][0], ey = g.ext[L][1], ez = g.ext[L][2];
    const int ny = hy - ly + 1, nz = hz - lz + 1;
    const int cx0 = 2 * x, cx1 = min(2 * x + 1, ex - 1);
    const uint32_t nxv = (2 * x + 1 < ex) ? 2u : 1u;
    for (int row = blockIdx.y; row < ny * nz; row += gridDim.y) {
        const int y = ly + row % ny, z = lz + row / ny;
        const uint32_t nyv = (2 * y + 1 < ey) ? 2u : 1u, nzv = (2 * z + 1 < ez) ? 2u : 1u;
        const uint32_t n = nxv * nyv * nzv;
        for (int c = 0; c < g.C; c++) {
            T *dst = melem<kPaged>(g, mr, L + 1, c, x, y, z);
            if constexpr (sizeof(T) == 2) {
                uint32_t s = 0;
                for (uint32_t dz = 0; dz < nzv; dz++)
                    for (uint32_t dy = 0; dy < nyv; dy++) {
                        s += *melem<kPaged>(g, mr, L, c, cx0, 2 * y + dy, 2 * z + dz);
                        if (nxv == 2) s += *melem<kPaged>(g, mr, L, c, cx1, 2 * y + dy, 2 * z + dz);
                    }
                *dst = (T)mean_rhu(s, n);
            } else {
                double s = 0.0;
                for (uint32_t dz = 0; dz < nzv; dz++)
                    for (uint32_t dy = 0; dy < nyv; dy++) {
                        s += (double)*melem<kPaged>(g, mr, L, c, cx0, 2 * y + dy, 2 * z + dz);
                        if (nxv == 2)
                            s += (double)*melem<kPaged>(g, mr, L, c, cx1, 2 * y + dy, 2 * z + dz);
                    }
                *dst = (float)(s * (1.0 / (double)n));
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

// Cells of levels whose rows and channel planes are aligned to eight elements, with M a
// multiple of eight (a cell row is whole 8-element words; bit L of `vec_levels`), are read a
// 16-byte word per thread and step, every channel at once; other levels' cells one element per
// thread.  The block folds every statistic in one pass through LDS.
template <typename T, bool kPaged>
__global__ void __launch_bounds__(kThreads)
k_stats_part(VolGeom g, MasterRef<const T> mr, const uint8_t *__restrict__ mask,
             const int4 *cells, int nsub, int n_items, uint32_t vec_levels, StatPart *part)
{
    constexpr int kW = kThreads / 64;
    __shared__ float s_mn[kW][kMaxC], s_mx[kW][kMaxC];
    __shared__ unsigned long long s_su[kW][kMaxC];
    __shared__ double s_sd[kW][kMaxC];
    __shared__ uint32_t s_in[kW][kMaxC];
    // work item = cell * nsub + slab; workgroup b takes item (b % 8) * per + b / 8, so an XCD
    // works through a contiguous run of cells and x-neighbours, whose rows share 128-byte
    // lines, meet in its L2 (workgroups are dealt to the eight XCDs round robin)
    const int per = (int)(gridDim.x / kXcds);
    const int item = (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
    if (item >= n_items) return;
    const int4 cl = cells[item / nsub];
    const int sub = item % nsub;
    const int L = cl.x;
    const int b[3] = {cl.y, cl.z, cl.w};
    int lo[3], n[3];
    for (int a = 0; a < 3; a++) {
        lo[a] = b[a] * g.M;
        n[a] = min(g.M, g.ext[L][a] - lo[a]);
    }
    const int zc = (n[2] + nsub - 1) / nsub;
    const int zs = min(sub * zc, n[2]), ze = min(zs + zc, n[2]);
    const bool wide = (vec_levels >> L) & 1u;
    const int C = g.C;
    float mn[kMaxC], mx[kMaxC];
    uint32_t su[kMaxC], cnt[kMaxC];
    double sd[kMaxC];
    for (int c = 0; c < kMaxC; c++) {
        mn[c] = FLT_MAX;
        mx[c] = -FLT_MAX;
        su[c] = cnt[c] = 0;
        sd[c] = 0.0;
    }
    if (wide) {
        const int nq = n[0] >> 3;                    // 8-element words per cell row
        const int rows = (ze - zs) * n[1];
        for (int j = threadIdx.x; j < rows * nq; j += kThreads) {
            const int q = j % nq, r = j / nq;
            const int y = lo[1] + r % n[1], z = lo[2] + zs + r / n[1];
            const int64_t lin = ((int64_t)z * g.dims[1] + y) * g.dims[0] + lo[0] + 8 * q;   // mask (level 0)
            Pack8<T> v[kMaxC];
#pragma unroll
            for (int c = 0; c < kMaxC; c++)
                if (c < C) v[c] = Pack8<T>::load(melem<kPaged>(g, mr, L, c, lo[0] + 8 * q, y, z));
#pragma unroll
            for (int c = 0; c < kMaxC; c++)
                if (c < C)
#pragma unroll
                    for (int e = 0; e < 8; e++) {
                        const auto x = v[c].at(e);
                        mn[c] = fminf(mn[c], (float)x);
                        mx[c] = fmaxf(mx[c], (float)x);
                        if constexpr (sizeof(T) == 2) su[c] += x;
                        else sd[c] += (double)x;
                    }
            if (L == 0) {
                const uint2 m = *(const uint2 *)(mask + lin);
#pragma unroll
                for (int c = 0; c < kMaxC; c++) {
                    // bit c of each of the eight mask bytes, summed
                    const uint32_t a = (m.x >> c) & 0x01010101u, bb = (m.y >> c) & 0x01010101u;
                    cnt[c] += (uint32_t)__popc(a) + (uint32_t)__popc(bb);
                }
            }
        }
    } else {
        const int rstep = kThreads / n[0];            // rows per pass (n[0] <= 128)
        const int x = threadIdx.x % n[0], r0 = threadIdx.x / n[0];
        if (r0 < rstep)
            for (int z = zs; z < ze; z++)
                for (int y = r0; y < n[1]; y += rstep) {
                    const int64_t lin = ((int64_t)(lo[2] + z) * g.dims[1] + (lo[1] + y)) * g.dims[0] + (lo[0] + x);
                    for (int c = 0; c < C; c++) {
                        const T v = *melem<kPaged>(g, mr, L, c, lo[0] + x, lo[1] + y, lo[2] + z);
                        mn[c] = fminf(mn[c], (float)v);
                        mx[c] = fmaxf(mx[c], (float)v);
                        if constexpr (sizeof(T) == 2) su[c] += v;
                        else sd[c] += (double)v;
                    }
                    if (L == 0) {
                        const uint32_t bits = mask[lin];
                        for (int c = 0; c < kMaxC; c++) cnt[c] += (bits >> c) & 1u;
                    }
                }
    }
    // wave folds, then one LDS exchange for every statistic
    unsigned long long sul[kMaxC];
    for (int c = 0; c < kMaxC; c++) sul[c] = su[c];
    for (int o = 32; o > 0; o >>= 1)
        for (int c = 0; c < kMaxC; c++) {
            mn[c] = fminf(mn[c], __shfl_xor(mn[c], o, 64));
            mx[c] = fmaxf(mx[c], __shfl_xor(mx[c], o, 64));
            if constexpr (sizeof(T) == 2) sul[c] += __shfl_xor(sul[c], o, 64);
            else sd[c] += __shfl_xor(sd[c], o, 64);
            cnt[c] += __shfl_xor(cnt[c], o, 64);
        }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int c = 0; c < kMaxC; c++) {
            s_mn[w][c] = mn[c];
            s_mx[w][c] = mx[c];
            s_su[w][c] = sul[c];
            s_sd[w][c] = sd[c];
            s_in[w][c] = cnt[c];
        }
    __syncthreads();
    if (threadIdx.x < kMaxC) {
        const int c = threadIdx.x;
        float a = s_mn[0][c], z = s_mx[0][c];
        unsigned long long u = s_su[0][c];
        double d = s_sd[0][c];
        uint32_t k = s_in[0][c];
        for (int i = 1; i < kW; i++) {
            a = fminf(a, s_mn[i][c]);
            z = fmaxf(z, s_mx[i][c]);
            u += s_su[i][c];
            d += s_sd[i][c];
            k += s_in[i][c];
        }
        StatPart *o = part + item;
        if (c < C) {
            o->mn[c] = a;
            o->mx[c] = z;
            o->sum[c] = sizeof(T) == 2 ? (double)u : d;
        }
        o->ins[c] = k;
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
// Jobs are listed x-fastest, and x-neighbours read the same 64-byte segments of each other's
// border rows.  Workgroups are dealt to the eight XCDs (each with its own L2) round robin, so
// workgroup w takes job (w % 8) * per + w / 8 (per = jobs per XCD): an XCD works through a
// contiguous run of jobs and neighbours find the shared segments in its L2.
#ifndef OCTRC_GATHER_THREADS
#define OCTRC_GATHER_THREADS 256
#endif
constexpr int kGatherThreads = OCTRC_GATHER_THREADS;

// kStore: the launch writes whole bricks to the host brick store as well (its own
// instantiation, so the common one keeps its few registers).
template <typename T, bool kPaged, bool kStore>
__global__ void __launch_bounds__(kGatherThreads)
k_gather(VolGeom g, MasterRef<const T> mr, const DevCell *table, uint8_t *pool, uint64_t brick_bytes,
         const BrickJob *jobs, int n_items, int zsplit, float *part, float background,
         uint8_t *store, uint64_t store_bytes)
{
    __shared__ int s_kind[27];
    __shared__ float s_avg[27][4];
    __shared__ float sf[kGatherThreads / 64];
    const int per = (int)(gridDim.x / kXcds);
    const int item = (int)(blockIdx.x % kXcds) * per + (int)(blockIdx.x / kXcds);
    if (item >= n_items) return;
    const int jid = item / zsplit, zc = item % zsplit;
    const BrickJob job = jobs[jid];
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
    const int64_t slice = (int64_t)ex * ey, plane = slice * ez;   // dense master strides
    float mn[kMaxC], mx[kMaxC];
    for (int c = 0; c < kMaxC; c++) {
        mn[c] = FLT_MAX;
        mx[c] = -FLT_MAX;
    }
    // slot < 0: the brick goes to the host brick store only (it is not resident)
    T *dst = (!kStore || job.slot >= 0) ? (T *)(pool + (uint64_t)job.slot * brick_bytes) : nullptr;
    // whole bricks may also go to the host brick store: C planes of S^3 elements
    T *sto = (kStore && job.store >= 0) ? (T *)(store + (uint64_t)job.store * store_bytes) : nullptr;
    const int64_t S3 = (int64_t)S * S * S;
    const int nx = job.hi[0] - job.lo[0] + 1, ny = job.hi[1] - job.lo[1] + 1;
    // this workgroup's share of the job's slices
    const int zper = (job.hi[2] - job.lo[2] + zsplit) / zsplit;
    const int z_lo = job.lo[2] + zc * zper, z_hi = min(z_lo + zper - 1, job.hi[2]);
    for (int j = threadIdx.x; j < nx * ny; j += kGatherThreads) {
        const int x = job.lo[0] + j % nx, y = job.lo[1] + j / nx;
        // bordered position -> clamped level index, and which of the 3x3x3 neighbours holds it
        const int gx = min(max(b[0] * M - 1 + x, 0), ex - 1);
        const int ox = gx < b[0] * M ? 0 : (gx >= b[0] * M + M ? 2 : 1);
        const int gy = min(max(b[1] * M - 1 + y, 0), ey - 1);
        const int oy = gy < b[1] * M ? 0 : (gy >= b[1] * M + M ? 2 : 1);
        const T *col = kPaged ? nullptr : melem<false>(g, mr, L, 0, gx, gy, 0);   // dense: column base
#pragma unroll 4
        for (int z = z_lo; z <= z_hi; z++) {
            const int gz = min(max(b[2] * M - 1 + z, 0), ez - 1);
            const int oz = gz < b[2] * M ? 0 : (gz >= b[2] * M + M ? 2 : 1);
            const int nb = (oz * 3 + oy) * 3 + ox;
            T v[4];
            if (s_kind[nb] != kAvg) {
                if constexpr (kPaged) {
                    for (int c = 0; c < 4; c++) v[c] = c < g.C ? *melem<true>(g, mr, L, c, gx, gy, gz) : (T)0;
                } else {
                    const T *p = col + (int64_t)gz * slice;
                    for (int c = 0; c < 4; c++) v[c] = c < g.C ? p[(int64_t)c * plane] : (T)0;
                }
            } else {
                for (int c = 0; c < 4; c++) v[c] = c < g.C ? (T)s_avg[nb][c] : (T)0;
            }
            for (int c = 0; c < kMaxC; c++)
                if (c < g.C) {
                    mn[c] = fminf(mn[c], (float)v[c]);
                    mx[c] = fmaxf(mx[c], (float)v[c]);
                }
            const int64_t i = ((int64_t)z * S + y) * S + x;
            // streaming stores: this launch does not read the bricks it writes
            if (!kStore || dst) {
                if constexpr (sizeof(T) == 2) {
                    u32x2_t w;
                    w.x = (uint32_t)v[0] | ((uint32_t)v[1] << 16);
                    w.y = (uint32_t)v[2] | ((uint32_t)v[3] << 16);
                    __builtin_nontemporal_store(w, (u32x2_t *)(dst + i * 4));
                } else {
                    const f32x4_t w = {(float)v[0], (float)v[1], (float)v[2], (float)v[3]};
                    __builtin_nontemporal_store(w, (f32x4_t *)(dst + i * 4));
                }
            }
            if constexpr (kStore)
                if (sto)
                    for (int c = 0; c < kMaxC; c++)
                        if (c < g.C) sto[c * S3 + i] = v[c];
        }
    }
    for (int c = 0; c < g.C; c++) {
        const float lo = block_reduce<float, MinF, kGatherThreads / 64>(mn[c], MinF{}, sf);
        const float hi = block_reduce<float, MaxF, kGatherThreads / 64>(mx[c], MaxF{}, sf);
        if (threadIdx.x == 0) {
            part[(int64_t)item * 8 + c] = lo;
            part[(int64_t)item * 8 + 4 + c] = hi;
        }
    }
}

// The value range of what each job wrote, folded over its workgroups: the slot's skip range
// is replaced by a whole-brick job and widened by a partial one (a superset stays a valid
// bound).
__global__ void __launch_bounds__(kThreads)
k_gather_fold(const BrickJob *jobs, int n_jobs, int zsplit, int C, const float *part,
              float *slot_range, float *store_range)
{
    const int j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= n_jobs) return;
    const BrickJob &job = jobs[j];
    float *r = job.slot >= 0 ? slot_range + (int64_t)job.slot * 8 : nullptr;
    float *q = (store_range && job.store >= 0) ? store_range + (int64_t)job.store * 8 : nullptr;
    for (int c = 0; c < C; c++) {
        float lo = FLT_MAX, hi = -FLT_MAX;
        for (int k = 0; k < zsplit; k++) {
            lo = fminf(lo, part[((int64_t)j * zsplit + k) * 8 + c]);
            hi = fmaxf(hi, part[((int64_t)j * zsplit + k) * 8 + 4 + c]);
        }
        if (r) {
            r[c] = job.full ? lo : fminf(r[c], lo);
            r[4 + c] = job.full ? hi : fmaxf(r[4 + c], hi);
        }
        if (q) {   // stored whole bricks only
            q[c] = lo;
            q[4 + c] = hi;
        }
    }
}

// Bricks from the host brick store into pool slots: a thread moves eight voxels, reading 16
// bytes of each channel plane (whole, aligned words over the host link) and writing the
// channel-interleaved, padded voxels.  Workgroup b takes chunk b % chunks of job b / chunks.
template <typename T>
__global__ void __launch_bounds__(kThreads)
k_copy_bricks(int M, int C, uint8_t *pool, uint64_t brick_bytes, const CopyJob *jobs,
              int chunks, const uint8_t *store, uint64_t store_bytes)
{
    const int S = M + 2;
    const int64_t S3 = (int64_t)S * S * S;
    const CopyJob job = jobs[blockIdx.x / chunks];
    const int64_t v0 = ((int64_t)(blockIdx.x % chunks) * kThreads + threadIdx.x) * 8;
    if (v0 >= S3) return;
    const T *src = (const T *)(store + (uint64_t)job.store * store_bytes);
    T *dst = (T *)(pool + (uint64_t)job.slot * brick_bytes);
    Pack8<T> p[kMaxC];
#pragma unroll
    for (int c = 0; c < kMaxC; c++)
        if (c < C) p[c] = Pack8<T>::load(src + c * S3 + v0);
#pragma unroll
    for (int e = 0; e < 8; e++) {
        T v[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
        for (int c = 0; c < kMaxC; c++)
            if (c < C) v[c] = (T)p[c].at(e);
        if constexpr (sizeof(T) == 2)
            *(ushort4 *)(dst + (v0 + e) * 4) = make_ushort4(v[0], v[1], v[2], v[3]);
        else
            *(float4 *)(dst + (v0 + e) * 4) = make_float4(v[0], v[1], v[2], v[3]);
    }
}

__global__ void __launch_bounds__(kThreads)
k_copy_ranges(const CopyJob *jobs, int n, int C, const float *store_range, float *slot_range)
{
    const int j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= n) return;
    for (int c = 0; c < C; c++)
        for (int k = 0; k < 8; k += 4)
            slot_range[(int64_t)jobs[j].slot * 8 + k + c] = store_range[(int64_t)jobs[j].store * 8 + k + c];
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

// The master as the kernels see it: dense levels, or the device page table of the disk tier.
template <typename T>
static MasterRef<T> master_ref(const VolGeom &g, void *master)
{
    if (g.plog > 0) return MasterRef<T>{nullptr, (T *const *)master};
    return MasterRef<T>{(T *)master, nullptr};
}

// Calls f(T{}, std::bool_constant<paged>{}) for the master's element type and layout.
template <typename F>
static void by_type(const VolGeom &g, F &&f)
{
    if (g.dtype == 0) {
        if (g.plog > 0) f(uint16_t{}, std::true_type{});
        else f(uint16_t{}, std::false_type{});
    } else {
        if (g.plog > 0) f(float{}, std::true_type{});
        else f(float{}, std::false_type{});
    }
}

hipError_t launch_insert(const VolGeom &g, void *master, uint8_t *mask, const void *src,
                         const int64_t sp[3], int channel, const int32_t o[3], const int32_t n[3],
                         hipStream_t s)
{
    if ((int64_t)n[0] * n[1] * n[2] == 0) return hipSuccess;
    // 16-byte words: rows of the block, of the level-0 mask and of the master (or its pages)
    // start on multiples of eight elements
    const bool layout = g.plog > 0 ? g.plog >= 3
                                   : (g.lvl_off[0] % 8 == 0 && ((uintptr_t)master & 15) == 0);
    const bool wide = layout && o[0] % 8 == 0 && n[0] % 8 == 0 && g.dims[0] % 8 == 0 &&
                      sp[0] % 8 == 0 && sp[1] % 8 == 0 && sp[2] % 8 == 0 &&
                      ((uintptr_t)src & 15) == 0 && ((uintptr_t)mask & 15) == 0;
    by_type(g, [&](auto tv, auto paged) {
        using T = decltype(tv);
        constexpr bool kP = decltype(paged)::value;
        const MasterRef<T> mr = master_ref<T>(g, master);
        if (wide) {
            const int64_t items = (int64_t)(n[0] / 8) * n[1] * n[2];
            const dim3 grid((unsigned)std::min<int64_t>(ceil_div(items, kThreads), 1 << 20));
            hipLaunchKernelGGL((k_insert8<T, kP>), grid, dim3(kThreads), 0, s, g, mr, mask,
                               (const T *)src, sp[0], sp[1], sp[2], channel, o[0], o[1], o[2],
                               n[0], n[1], n[2]);
        } else {
            const dim3 grid(ceil_div(n[0], kThreads),
                            (unsigned)std::min<int64_t>((int64_t)n[1] * n[2], 65535));
            hipLaunchKernelGGL((k_insert<T, kP>), grid, dim3(kThreads), 0, s, g, mr, mask,
                               (const T *)src, sp[0], sp[1], sp[2], channel, o[0], o[1], o[2],
                               n[0], n[1], n[2]);
        }
    });
    return hipGetLastError();
}

// Level L's channel planes start on multiples of `a` elements and its rows are multiples of
// `a` elements long (dense master); with pages, rows of `a` elements stay inside a page row
// and only the extent matters.
static bool level_aligned(const VolGeom &g, int L, int a)
{
    if (g.plog > 0) return g.ext[L][0] % a == 0 && (1 << g.plog) % 8 == 0;
    const int64_t plane = (int64_t)g.ext[L][0] * g.ext[L][1] * g.ext[L][2];
    return g.ext[L][0] % a == 0 && g.lvl_off[L] % a == 0 && plane % a == 0;
}

hipError_t launch_downsample(const VolGeom &g, void *master, int L, const int32_t lo[3],
                             const int32_t hi[3], hipStream_t s)
{
    const int ny = hi[1] - lo[1] + 1, nz = hi[2] - lo[2] + 1;
    if (hi[0] < lo[0] || ny <= 0 || nz <= 0) return hipSuccess;
    const bool wide = level_aligned(g, L, 8) && level_aligned(g, L + 1, 4) &&
                      (g.plog > 0 || ((uintptr_t)master & 15) == 0);
    by_type(g, [&](auto tv, auto paged) {
        using T = decltype(tv);
        constexpr bool kP = decltype(paged)::value;
        const MasterRef<T> mr = master_ref<T>(g, master);
        if (wide) {
            const int q0 = lo[0] / 4, nq = hi[0] / 4 - q0 + 1;
            const int64_t items = (int64_t)nq * ny * nz;
            const dim3 grid((unsigned)std::min<int64_t>(ceil_div(items, kThreads), 1 << 20));
            hipLaunchKernelGGL((k_downsample4<T, kP>), grid, dim3(kThreads), 0, s, g, mr, L, q0,
                               nq, lo[1], lo[2], ny, nz);
        } else {
            const int64_t rows = (int64_t)ny * nz;
            const dim3 grid(ceil_div(hi[0] - lo[0] + 1, kThreads),
                            (unsigned)std::min<int64_t>(rows, 65535));
            hipLaunchKernelGGL((k_downsample<T, kP>), grid, dim3(kThreads), 0, s, g, mr, L, lo[0],
                               lo[1], lo[2], hi[0], hi[1], hi[2]);
        }
    });
    return hipGetLastError();
}

static int stats_nsub(const VolGeom &g) { return std::max(1, g.M / 8); }

size_t stats_scratch_bytes(const VolGeom &g, int n)
{
    return (size_t)n * (size_t)stats_nsub(g) * sizeof(StatPart);
}

hipError_t launch_stats(const VolGeom &g, const void *master, const uint8_t *mask,
                        const int32_t *cells, int n, void *scratch, CellStat *out, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int nsub = stats_nsub(g);
    uint32_t vec_levels = 0;
    if (g.M % 8 == 0 && (g.plog > 0 || ((uintptr_t)master & 15) == 0) && ((uintptr_t)mask & 15) == 0)
        for (int L = 0; L <= g.N; L++)
            if (level_aligned(g, L, 8)) vec_levels |= 1u << L;
    StatPart *part = (StatPart *)scratch;
    by_type(g, [&](auto tv, auto paged) {
        using T = decltype(tv);
        constexpr bool kP = decltype(paged)::value;
        const MasterRef<T> m0 = master_ref<T>(g, (void *)master);
        const MasterRef<const T> mr{m0.base, m0.pages};
        const int items = n * nsub;
        hipLaunchKernelGGL((k_stats_part<T, kP>), dim3((unsigned)(ceil_div(items, kXcds) * kXcds)),
                           dim3(kThreads), 0, s, g, mr, mask, (const int4 *)cells, nsub, items,
                           vec_levels, part);
    });
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

// Workgroups per job: a job's slices are split so that a whole-volume upload runs several
// rounds of workgroups (one workgroup per 34^3 job left the last round mostly empty).
static int gather_zsplit(const VolGeom &g) { return std::min(4, std::max(1, (g.M + 2) / 8)); }

size_t gather_scratch_bytes(const VolGeom &g, int n)
{
    return (size_t)n * (size_t)gather_zsplit(g) * 8 * sizeof(float);
}

hipError_t launch_gather(const VolGeom &g, const void *master, const DevCell *table, void *pool,
                         uint64_t brick_bytes, const BrickJob *jobs, int n, float *slot_range,
                         float background, void *scratch, uint8_t *store, float *store_range,
                         uint64_t store_bytes, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int zsplit = gather_zsplit(g), items = n * zsplit;
    const dim3 grid((unsigned)(ceil_div(items, kXcds) * kXcds));
    by_type(g, [&](auto tv, auto paged) {
        using T = decltype(tv);
        constexpr bool kP = decltype(paged)::value;
        const MasterRef<T> m0 = master_ref<T>(g, (void *)master);
        const MasterRef<const T> mr{m0.base, m0.pages};
        if (store)
            hipLaunchKernelGGL((k_gather<T, kP, true>), grid, dim3(kGatherThreads), 0, s, g, mr,
                               table, (uint8_t *)pool, brick_bytes, jobs, items, zsplit,
                               (float *)scratch, background, store, store_bytes);
        else
            hipLaunchKernelGGL((k_gather<T, kP, false>), grid, dim3(kGatherThreads), 0, s, g, mr,
                               table, (uint8_t *)pool, brick_bytes, jobs, items, zsplit,
                               (float *)scratch, background, store, store_bytes);
    });
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gather_fold, dim3(ceil_div(n, kThreads)), dim3(kThreads), 0, s, jobs, n,
                       zsplit, g.C, (const float *)scratch, slot_range, store_range);
    return hipGetLastError();
}

hipError_t launch_copy_bricks(const VolGeom &g, void *pool, uint64_t brick_bytes,
                              const CopyJob *jobs, int n, const uint8_t *store,
                              const float *store_range, uint64_t store_bytes, float *slot_range,
                              hipStream_t s)
{
    if (n == 0) return hipSuccess;
    const int64_t S = g.M + 2, words = S * S * S / 8;   // S is even: whole 8-voxel words
    const int chunks = (int)ceil_div(words, kThreads);
    if (g.dtype == 0)
        hipLaunchKernelGGL(k_copy_bricks<uint16_t>, dim3((unsigned)(n * chunks)), dim3(kThreads), 0, s,
                           g.M, g.C, (uint8_t *)pool, brick_bytes, jobs, chunks, store, store_bytes);
    else
        hipLaunchKernelGGL(k_copy_bricks<float>, dim3((unsigned)(n * chunks)), dim3(kThreads), 0, s,
                           g.M, g.C, (uint8_t *)pool, brick_bytes, jobs, chunks, store, store_bytes);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_copy_ranges, dim3(ceil_div(n, kThreads)), dim3(kThreads), 0, s, jobs, n,
                       g.C, store_range, slot_range);
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

hipError_t launch_fill_u16(uint16_t *p, int64_t n, uint16_t v, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<uint16_t>, dim3((unsigned)std::min<int64_t>(ceil_div(n, kThreads), 65536)),
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
    // a paged master is reset on the host (every page back to the background)
    if (g.plog == 0) {
        const int64_t n = g.lvl_off[g.N + 1];
        const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(n, kThreads), 65536);
        if (g.dtype == 0)
            hipLaunchKernelGGL(k_fill<uint16_t>, dim3(blocks), dim3(kThreads), 0, s,
                               (uint16_t *)master, n, (uint16_t)background);
        else
            hipLaunchKernelGGL(k_fill<float>, dim3(blocks), dim3(kThreads), 0, s, (float *)master,
                               n, (float)background);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t nm = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
    hipLaunchKernelGGL(k_fill<uint8_t>, dim3((unsigned)std::min<int64_t>(ceil_div(nm, kThreads), 65536)),
                       dim3(kThreads), 0, s, mask, nm, (uint8_t)0);
    return hipGetLastError();
}

}  // namespace octrc
