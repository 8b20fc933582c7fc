// Adjoint of the forward ray caster: gradients of a scalar image loss with respect to the
// transfer-function control-point RGBA values and to the level-0 voxel values.
//
// The forward stored, per ray, the transmittance T before every position it evaluated, T after
// the last one and the first position it did not evaluate (for a ray split into depth segments:
// T from the start of the segment, plus each segment's composite, from which a wave walking one
// segment gets the transmittance in front of it, its transmittance at the end and the
// colour/opacity behind it).  A lane walks its positions back to front.  A position the forward
// skipped is transparent in every channel, so T is the same before and after it; before any
// other position T is the recorded value.  With Bc / Ba the colour / opacity of everything
// behind an event (as seen with transmittance 1), an event e with transmittance T_e, opacity a_e
// and colour rgb_e receives
//     dL/drgb_e = gC * T_e * a_e
//     dL/da_e   = T_e * (gC . (rgb_e - Bc) + gA * (1 - Ba))
// and then Bc <- a_e rgb_e + (1 - a_e) Bc, Ba <- a_e + (1 - a_e) Ba,
// where (gC, gA) = dL/d(pixel RGBA).
// The event gradient flows into the two table entries it interpolated and through them into at
// most three consecutive transfer-function control points (summed per lane in registers over a
// window of three control points, added to an LDS accumulator per workgroup when an event leaves
// the window, which goes to dL/dctrl at the end) and, through
// the table slope and the trilinear weights, into the eight level-0 corner voxels: summed per
// lane in registers while the ray stays in one corner cube (a step to a face neighbour keeps
// the four shared corners) and added to memory with float atomics when corners leave.
// Every position is evaluated (no empty-space skipping): a zero-opacity sample still has a
// non-zero gradient with respect to the table.
#include "raycommon.h"

#include <float.h>
#include <limits.h>

namespace octrc {

namespace {

constexpr int kThreads = 64 * kRenderTilesPerWg;

// One sample position: intensity per channel and, for a brick sample, the trilinear corners.
template <int C>
struct Sample {
    float s[C];
    bool brick;
    int ii[3];      // lower corner in bordered-brick coordinates
    float f[3];     // trilinear fractions
    int org[3];     // level-L index of bordered-brick coordinate 0
};

template <typename T, int C>
struct Marcher {
    const VolGeom &g;
    const DevCell *table;
    const uint8_t *pool;
    uint64_t brick_bytes;
    int L, csz, G, coff;
    float scaleL;
    int blo[3] = {1, 1, 1}, bhi[3] = {0, 0, 0};
    bool brick = false;
    const uint8_t *base = nullptr;
    int org[3] = {0, 0, 0};
    float avg[C];
    __device__ Marcher(const VolGeom &g_, const DevCell *t, const uint8_t *p, uint64_t bb, int L_)
        : g(g_), table(t), pool(p), brick_bytes(bb), L(L_)
    {
        csz = g.M << L;
        G = g.grid[L];
        coff = g.cell_off[L];
        scaleL = __builtin_ldexpf(1.0f, -L);
        for (int c = 0; c < C; c++) avg[c] = 0.0f;
    }

    // Same decisions as the forward: the voxel holding p selects the level-L node; a brick
    // node is interpolated in its bordered brick (channels interleaved and padded to four: one
    // 8-byte (u16) or 16-byte (f32) load per corner, the eight issued together), any other node
    // gives its AVG.
    __device__ void sample(const float p[3], Sample<C> &out)
    {
        int v[3];
#pragma unroll
        for (int q = 0; q < 3; q++) v[q] = min(max((int)floorf(p[q]), 0), g.dims[q] - 1);
        if (v[0] < blo[0] || v[0] > bhi[0] || v[1] < blo[1] || v[1] > bhi[1] || v[2] < blo[2] ||
            v[2] > bhi[2]) {
            const int cx = v[0] / csz, cy = v[1] / csz, cz = v[2] / csz;
            const DevCell &cell = table[coff + (cz * G + cy) * G + cx];
            blo[0] = cx * csz; bhi[0] = blo[0] + csz - 1;
            blo[1] = cy * csz; bhi[1] = blo[1] + csz - 1;
            blo[2] = cz * csz; bhi[2] = blo[2] + csz - 1;
            brick = cell.kind == kBrick;
            if (brick) {
                base = pool + (uint64_t)cell.slot * brick_bytes;
                org[0] = cx * g.M - 1;
                org[1] = cy * g.M - 1;
                org[2] = cz * g.M - 1;
            } else {
                for (int c = 0; c < C; c++) avg[c] = cell.avg[c];
            }
        }
        out.brick = brick;
        if (!brick) {
            for (int c = 0; c < C; c++) out.s[c] = avg[c];
            return;
        }
        const int S = g.M + 2;
#pragma unroll
        for (int q = 0; q < 3; q++) {
            const float qq = p[q] * scaleL - 0.5f;
            const float lq = qq - (float)org[q];
            const float fl = floorf(lq);
            out.f[q] = lq - fl;
            out.ii[q] = min(max((int)fl, 0), S - 2);
            out.org[q] = org[q];
        }
        const uint32_t off = (uint32_t)((out.ii[2] * S + out.ii[1]) * S + out.ii[0]);
        const uint32_t dy = (uint32_t)S, dz = (uint32_t)(S * S);
        const uint32_t o8[8] = {off, off + 1, off + dy, off + dy + 1,
                                off + dz, off + dz + 1, off + dz + dy, off + dz + dy + 1};
        float w[8][C];
        if constexpr (sizeof(T) == 2) {
            const uint2 *b2 = (const uint2 *)base;
            uint2 q[8];
#pragma unroll
            for (int k = 0; k < 8; k++) q[k] = b2[o8[k]];   // all loads in flight first
#pragma unroll
            for (int k = 0; k < 8; k++)
#pragma unroll
                for (int c = 0; c < C; c++) {
                    const uint32_t word = (c < 2) ? q[k].x : q[k].y;
                    w[k][c] = (float)((c & 1) ? (word >> 16) : (word & 0xffffu));
                }
        } else {
            const float4 *b4 = (const float4 *)base;
            float4 q[8];
#pragma unroll
            for (int k = 0; k < 8; k++) q[k] = b4[o8[k]];
#pragma unroll
            for (int k = 0; k < 8; k++) {
                const float qv[4] = {q[k].x, q[k].y, q[k].z, q[k].w};
#pragma unroll
                for (int c = 0; c < C; c++) w[k][c] = qv[c];
            }
        }
#pragma unroll
        for (int c = 0; c < C; c++) {
            const float c00 = lerpf(w[0][c], w[1][c], out.f[0]);
            const float c10 = lerpf(w[2][c], w[3][c], out.f[0]);
            const float c01 = lerpf(w[4][c], w[5][c], out.f[0]);
            const float c11 = lerpf(w[6][c], w[7][c], out.f[0]);
            out.s[c] = lerpf(lerpf(c00, c10, out.f[1]), lerpf(c01, c11, out.f[1]), out.f[2]);
        }
    }
};

// Voxel gradients of one lane's current corner cube (lower corner k, level-0 indices), summed in
// registers while consecutive positions interpolate in the same cube; a step of one along an
// axis keeps the four corners the two cubes share, the others are added to memory.
// Blocked voxel-gradient scratch: [C] planes of blocks of 2^sx x 2^sy x 2^sz voxels (each
// shift 0..7), blocks x-fastest.  The shape code is sx + 8 sy + 64 sz.
struct BlockShape {
    int sx, sy, sz, sb;
    int64_t nbx, nby, plane;
    __host__ __device__ BlockShape(int code, const int32_t *dims)
        : sx(code & 7), sy((code >> 3) & 7), sz((code >> 6) & 7), sb(sx + sy + sz),
          nbx((dims[0] + (1 << sx) - 1) >> sx), nby((dims[1] + (1 << sy) - 1) >> sy),
          plane((nbx * nby * ((dims[2] + (1 << sz) - 1) >> sz)) << sb)
    {
    }
    __host__ __device__ int64_t index(int64_t x, int64_t y, int64_t z) const
    {
        return ((((z >> sz) * nby + (y >> sy)) * nbx + (x >> sx)) << sb) +
               ((((z & ((1 << sz) - 1)) << sy | (y & ((1 << sy) - 1))) << sx) | (x & ((1 << sx) - 1)));
    }
};

// The gradients go to dvox as [C][Dz][Dy][Dx] (shape code < 0), or to the blocked scratch,
// where the corners that the lanes of a wave flush together share more lines.
template <int C>
struct CubeAcc {
    float v[C][8];
    int kx = INT_MIN, ky = 0, kz = 0;
    float *dvox;
    int64_t nvox0;
    int dims[3];
    bool blocked;
    BlockShape bs;

    __device__ CubeAcc(float *d, int64_t n, const int32_t *dm, int shape)
        : dvox(d), nvox0(n), blocked(shape >= 0), bs(shape >= 0 ? shape : 0, dm)
    {
        dims[0] = dm[0];
        dims[1] = dm[1];
        dims[2] = dm[2];
#pragma unroll
        for (int c = 0; c < C; c++)
#pragma unroll
            for (int q = 0; q < 8; q++) v[c][q] = 0.0f;
    }

    template <int Q>
    __device__ __forceinline__ void flush_corner()
    {
        const int gx = min(max(kx + (Q & 1), 0), dims[0] - 1);
        const int gy = min(max(ky + ((Q >> 1) & 1), 0), dims[1] - 1);
        const int gz = min(max(kz + (Q >> 2), 0), dims[2] - 1);
        int64_t vi, pl;
        if (blocked) {
            vi = bs.index(gx, gy, gz);
            pl = bs.plane;
        } else {
            vi = ((int64_t)gz * dims[1] + gy) * dims[0] + gx;
            pl = nvox0;
        }
#pragma unroll
        for (int c = 0; c < C; c++) {
            if (v[c][Q] != 0.0f) atomicAdd(dvox + c * pl + vi, v[c][Q]);
            v[c][Q] = 0.0f;
        }
    }

    template <int Q = 0>
    __device__ __forceinline__ void flush_all()
    {
        if constexpr (Q < 8) {
            flush_corner<Q>();
            flush_all<Q + 1>();
        }
    }

    // a step of +1 (UP) or -1 along axis bit B: flush the face that leaves, move the other
    template <int B, bool UP, int Q = 0>
    __device__ __forceinline__ void shift_face()
    {
        if constexpr (Q < 8) {
            constexpr bool leaves = UP ? !(Q & B) : (Q & B);
            if constexpr (leaves) {
                constexpr int P = Q ^ B;   // the corner of the other face on this edge
                flush_corner<Q>();
#pragma unroll
                for (int c = 0; c < C; c++) {
                    v[c][Q] = v[c][P];
                    v[c][P] = 0.0f;
                }
            }
            shift_face<B, UP, Q + 1>();
        }
    }

    __device__ __forceinline__ void flush()
    {
        if (kx != INT_MIN) flush_all();
        kx = INT_MIN;
    }

    __device__ __forceinline__ void move_to(int nx, int ny, int nz)
    {
        const int dx = nx - kx, dy = ny - ky, dz = nz - kz;
        if (kx == INT_MIN || abs(dx) > 1 || abs(dy) > 1 || abs(dz) > 1) {
            flush();
        } else {
            if (dx == 1) { shift_face<1, true>(); kx += 1; }
            else if (dx == -1) { shift_face<1, false>(); kx -= 1; }
            if (dy == 1) { shift_face<2, true>(); ky += 1; }
            else if (dy == -1) { shift_face<2, false>(); ky -= 1; }
            if (dz == 1) { shift_face<4, true>(); kz += 1; }
            else if (dz == -1) { shift_face<4, false>(); kz -= 1; }
        }
        kx = nx;
        ky = ny;
        kz = nz;
    }
};

// kVox: voxel gradients are requested (otherwise their accumulators are not allocated).
template <typename T, int C, bool kVox>
__global__ void __launch_bounds__(kThreads)
k_render_backward(VolGeom g, const DevCell *__restrict__ table, const uint8_t *__restrict__ pool,
                  uint64_t brick_bytes, const DevView *__restrict__ views,
                  const WgItem *__restrict__ items, float *dvox, int vg_shape, float *dctrl)
{
    __shared__ ViewTables<C> tb;
    __shared__ float s_dctrl[C][8][4];
    __shared__ uint8_t s_segj[C][256];   // table entry k = (1 - f) ctrl[j] + f ctrl[j + 1], j < 8
    __shared__ float s_segf[C][256];

    const WgItem it = items[blockIdx.x];
    const DevView &V = views[it.view];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int i = threadIdx.x; i < C * 8 * 4; i += kThreads) (&s_dctrl[0][0][0])[i] = 0.0f;
    for (int i = threadIdx.x; i < C * 256; i += kThreads) {
        int j;
        float f;
        tf_segment(V.tf_pos[i >> 8], i & 255, j, f);
        s_segj[i >> 8][i & 255] = j;
        s_segf[i >> 8][i & 255] = f;
    }
    build_tables<C>(V, tb);   // ends with a barrier

    float ulo[C], usc[C];
    for (int c = 0; c < C; c++) {
        usc[c] = V.uscale[c];
        ulo[c] = -V.ulo[c] * usc[c];   // table coordinate u = s * usc + ulo
    }
    const float step = V.step;

    if (wave < it.ntiles) {
        const int tile = it.tile0 + wave;
        const int px_i = (tile % V.tiles_x) * 8 + (lane & 7);
        const int px_j = (tile / V.tiles_x) * 8 + (lane >> 3);
        const bool inside = px_i < V.width && px_j < V.height;
        const int64_t pix = (int64_t)px_j * V.width + px_i;
        const Ray ray = setup_ray(V, g, px_i, px_j, inside);
        const int n_end = ray.hit ? V.nend[pix] : 0;
        float gC[3] = {0.0f, 0.0f, 0.0f}, gA = 0.0f;
        if (inside) {
            const float4 gi = *(const float4 *)(V.dimg + pix * 4);
            gC[0] = gi.x;
            gC[1] = gi.y;
            gC[2] = gi.z;
            gA = gi.w;
        }
        const int64_t nvox0 = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
        Marcher<T, C> mb(g, table, pool, brick_bytes, ray.L);
        float Bc[3] = {0.0f, 0.0f, 0.0f}, Ba = 0.0f;
        CubeAcc<C> acc(dvox, nvox0, g.dims, vg_shape);
        // control-point gradients, through the table construction: an event interpolating
        // entries (i, i + 1) with weights (1 - fr, fr) reaches the control points of those two
        // entries (table entry k = (1 - f_k) ctrl[j_k] + f_k ctrl[j_k + 1]), i.e. at most three
        // consecutive control points.  Each lane sums them in registers over a window of three
        // control points (jb .. jb + 2) per channel and adds the window to the workgroup's LDS
        // accumulator only when an event falls outside it (a segment spans ~36 table entries)
        int jb[C];
        float wacc[C][3][4];
#pragma unroll
        for (int c = 0; c < C; c++) {
            jb[c] = -1;
#pragma unroll
            for (int j = 0; j < 3; j++)
#pragma unroll
                for (int q = 0; q < 4; q++) wacc[c][j][q] = 0.0f;
        }
        auto flush_window = [&](int c) {
#pragma unroll
            for (int j = 0; j < 3; j++)
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    if (wacc[c][j][q] != 0.0f) atomicAdd(&s_dctrl[c][jb[c] + j][q], wacc[c][j][q]);
                    wacc[c][j][q] = 0.0f;
                }
        };
        // the 64-position blocks this wave walks: all of the ray, or the blocks of its depth
        // segment (the forward split the ray the same way); then T_front holds the
        // transmittance in front of the segment and (Bc, Ba) start as the composite of the
        // segments behind it
        const int nb = (n_end + kCkptStride - 1) / kCkptStride;
        int b_lo = 0, b_hi = nb;
        float T_front = 1.0f;
        if (V.nsplit > 1) {
            b_lo = (int)(((int64_t)nb * it.seg) / V.nsplit);
            b_hi = (int)(((int64_t)nb * (it.seg + 1)) / V.nsplit);
            if (inside) {
                const int64_t npix = (int64_t)V.width * V.height;
                for (int j = 0; j < it.seg; j++) T_front *= V.part[((int64_t)j * npix + pix) * 4 + 3];
                float Tb = 1.0f;
                for (int j = V.nsplit - 1; j > it.seg; j--) {   // back to front
                    const float4 q = *(const float4 *)(V.part + ((int64_t)j * npix + pix) * 4);
                    Bc[0] = __builtin_fmaf(q.w, Bc[0], q.x);
                    Bc[1] = __builtin_fmaf(q.w, Bc[1], q.y);
                    Bc[2] = __builtin_fmaf(q.w, Bc[2], q.z);
                    Tb = Tb * q.w;
                }
                Ba = 1.0f - Tb;
            }
        }
        // positions of this wave, walked back to front; Tn: the transmittance after the
        // current position (after the walk's last position to begin with)
        const int64_t npix = (int64_t)V.width * V.height;
        const int k_lo = b_lo * kCkptStride, k_hi = min(b_hi * kCkptStride, n_end);
        float Tn = 0.0f;
        if (k_hi > k_lo)
            Tn = V.nsplit > 1 ? T_front * V.part[((int64_t)it.seg * npix + pix) * 4 + 3]
                              : V.ckpt[(int64_t)n_end * npix + pix];
        {
            for (int k = k_hi - 1; k >= k_lo; k--) {
                const float tk = ray.t0 + (float)k * step;
                if (!(tk < ray.t1)) continue;
                float p[3];
                for (int q = 0; q < 3; q++) {
                    const float m = tk * ray.d[q];
                    p[q] = ray.o[q] + m;
                }
                Sample<C> sm;
                mb.sample(p, sm);
                Classified cq[C];
                float rgba[C][4], Tc[C];
                if (kVox && sm.brick) {
                    // the corner cube of this sample (level-0 index of its lower corner)
                    const int kx = sm.org[0] + sm.ii[0], ky = sm.org[1] + sm.ii[1],
                              kz = sm.org[2] + sm.ii[2];
                    if (kx != acc.kx || ky != acc.ky || kz != acc.kz) acc.move_to(kx, ky, kz);
                }
                bool opaque = false;
                for (int c = 0; c < C; c++) {
                    cq[c] = classify(sm.s[c], ulo[c], usc[c], tb.lut[c]);
                    rgba[c][0] = __builtin_fmaf(cq[c].fr, cq[c].de.x, cq[c].e0.x);
                    rgba[c][1] = __builtin_fmaf(cq[c].fr, cq[c].de.y, cq[c].e0.y);
                    rgba[c][2] = __builtin_fmaf(cq[c].fr, cq[c].de.z, cq[c].e0.z);
                    rgba[c][3] = __builtin_fmaf(cq[c].fr, cq[c].de.w, cq[c].e0.w);
                    opaque |= rgba[c][3] != 0.0f;
                }
                // the transmittance before this position: recorded by the forward, or, for a
                // position transparent in every channel (the forward may have skipped it), the
                // one after it
                float Tp = opaque ? T_front * V.ckpt[(int64_t)k * npix + pix] : Tn;
                Tn = Tp;
                for (int c = 0; c < C; c++) {
                    Tc[c] = Tp;
                    Tp = Tp - Tp * rgba[c][3];
                }
                #pragma unroll
                for (int c = C - 1; c >= 0; c--) {
                    const float a = rgba[c][3];
                    float gq[4];
                    for (int q = 0; q < 3; q++) gq[q] = gC[q] * Tc[c] * a;
                    gq[3] = Tc[c] * (gC[0] * (rgba[c][0] - Bc[0]) + gC[1] * (rgba[c][1] - Bc[1]) +
                                     gC[2] * (rgba[c][2] - Bc[2]) + gA * (1.0f - Ba));
                    for (int q = 0; q < 3; q++) Bc[q] = a * rgba[c][q] + (1.0f - a) * Bc[q];
                    Ba = a + (1.0f - a) * Ba;
                    const float fr = cq[c].fr;
                    const int ja = s_segj[c][cq[c].i], jn = s_segj[c][cq[c].i + 1];
                    const float fa = s_segf[c][cq[c].i], fn = s_segf[c][cq[c].i + 1];
                    if (jb[c] < 0 || ja < jb[c] || jn + 1 > jb[c] + 2) {
                        if (jb[c] >= 0) flush_window(c);
                        jb[c] = min(ja, 5);
                    }
                    // weights of the window's three control points in this event
                    const float w0 = 1.0f - fr;
                    const int sa = ja - jb[c], sn = jn - jb[c];
                    float ws[3];
#pragma unroll
                    for (int j = 0; j < 3; j++)
                        ws[j] = (sa == j ? w0 * (1.0f - fa) : 0.0f) + (sa + 1 == j ? w0 * fa : 0.0f) +
                                (sn == j ? fr * (1.0f - fn) : 0.0f) + (sn + 1 == j ? fr * fn : 0.0f);
#pragma unroll
                    for (int j = 0; j < 3; j++)
#pragma unroll
                        for (int q = 0; q < 4; q++)
                            wacc[c][j][q] = __builtin_fmaf(ws[j], gq[q], wacc[c][j][q]);
                    if (kVox && sm.brick && cq[c].inside) {
                        const float4 de = cq[c].de;
                        const float gs = usc[c] * (gq[0] * de.x + gq[1] * de.y + gq[2] * de.z +
                                                   gq[3] * de.w);
                        if (gs != 0.0f) {
#pragma unroll
                            for (int corner = 0; corner < 8; corner++) {
                                const int dxx = corner & 1, dyy = (corner >> 1) & 1, dzz = corner >> 2;
                                const float wgt = (dxx ? sm.f[0] : 1.0f - sm.f[0]) *
                                                  (dyy ? sm.f[1] : 1.0f - sm.f[1]) *
                                                  (dzz ? sm.f[2] : 1.0f - sm.f[2]);
                                acc.v[c][corner] += gs * wgt;
                            }
                        }
                    }
                }
            }
        }
        if (kVox) acc.flush();
#pragma unroll
        for (int c = 0; c < C; c++)
            if (jb[c] >= 0) flush_window(c);
    }
    __syncthreads();
    float *out = dctrl + (int64_t)V.user_index * C * 32;
    for (int i = threadIdx.x; i < C * 8 * 4; i += kThreads) {
        const float v = (&s_dctrl[0][0][0])[i];
        if (v != 0.0f) atomicAdd(out + i, v);
    }
}

// Adjoint of a MIP view: a pixel is the channel-order composite of the classified maxima m_c,
// and m_c is the sample at the recorded position amax[c] (the first position reaching it; -1:
// no sample exceeded the window's low end, m_c = lo_c).  Per pixel the image gradient goes back
// through the compositing chain of the C events (as for one DVR position), into the two table
// entries each event interpolated (per-workgroup LDS accumulator), and, through the table slope
// and the trilinear weights of that one sample, into its eight level-0 corner voxels.  The
// sample is recomputed with the forward's operations (same cell, brick coordinates and
// interpolation order), so it equals the forward's maximum.
template <typename T, int C, bool kXf>
__device__ __forceinline__ void
mip_backward_body(const VolGeom &g, const DevCell *__restrict__ table,
                  const uint8_t *__restrict__ pool, uint64_t brick_bytes, const DevView &V,
                  const WgItem &it, const ViewTables<C> &tb, float (*s_dlut)[256][4], float *dvox)
{
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wave >= it.ntiles) return;
    const int tile = it.tile0 + wave;
    const int px_i = (tile % V.tiles_x) * 8 + (lane & 7);
    const int px_j = (tile / V.tiles_x) * 8 + (lane >> 3);
    const bool inside = px_i < V.width && px_j < V.height;
    if (!inside) return;
    const int64_t pix = (int64_t)px_j * V.width + px_i;
    const Ray ray = setup_ray(V, g, px_i, px_j, inside);
    if (!ray.hit) return;
    const float4 gi = *(const float4 *)(V.dimg + pix * 4);
    const int4 am4 = *(const int4 *)(V.amax + pix * 4);
    const int am[4] = {am4.x, am4.y, am4.z, am4.w};
    const int L = ray.L;
    const float scaleL = __builtin_ldexpf(1.0f, -L);
    const int S = g.M + 2;
    const float imax = (float)(S - 2);
    const int csz = g.M << L, G = g.grid[L];
    const int64_t nvox0 = (int64_t)g.dims[0] * g.dims[1] * g.dims[2];
    float sv[C], f[C][3], usc[C], ub[C];
    int org[C][3], ii[C][3];
    bool vox[C];
#pragma unroll
    for (int c = 0; c < C; c++) {
        usc[c] = V.uscale[c];
        ub[c] = -V.ulo[c] * usc[c];
        sv[c] = V.ulo[c];
        vox[c] = false;
        if (am[c] < 0) continue;
        const float tk = ray.t0 + (float)am[c] * V.step;
        float p[3];
        for (int q = 0; q < 3; q++) {
            const float m = tk * ray.d[q];
            p[q] = ray.o[q] + m;
        }
        if constexpr (kXf) {
            float pc[3];
            for (int a = 0; a < 3; a++) {
                const float *m = V.xform[c][a];
                const float s0 = m[0] * p[0];
                const float s1 = m[1] * p[1];
                const float s2 = m[2] * p[2];
                const float u = s0 + s1;
                const float w = u + s2;
                pc[a] = w + m[3];
            }
            for (int a = 0; a < 3; a++) p[a] = pc[a];
        }
        int v[3], cc[3];
        for (int q = 0; q < 3; q++) {
            v[q] = min(max((int)floorf(p[q]), 0), g.dims[q] - 1);
            cc[q] = v[q] / csz;
        }
        const DevCell &cell = table[g.cell_off[L] + (cc[2] * G + cc[1]) * G + cc[0]];
        if (cell.kind != kBrick) {
            sv[c] = cell.avg[c];
            continue;
        }
        const T *b0 = (const T *)(pool + (uint64_t)cell.slot * brick_bytes);
        for (int q = 0; q < 3; q++) {
            const float lq = __builtin_fmaf(p[q], scaleL, -((float)(cc[q] * g.M) - 0.5f));
            f[c][q] = __builtin_amdgcn_fractf(lq);
            ii[c][q] = (int)__builtin_amdgcn_fmed3f(lq, 0.0f, imax);
            org[c][q] = cc[q] * g.M - 1;
        }
        const int64_t v0 = ((int64_t)(ii[c][2] * S + ii[c][1]) * S + ii[c][0]) * 4 + c;
        const int64_t dy = (int64_t)S * 4, dz = (int64_t)S * S * 4;
        const float w000 = (float)b0[v0], w100 = (float)b0[v0 + 4];
        const float w010 = (float)b0[v0 + dy], w110 = (float)b0[v0 + dy + 4];
        const float w001 = (float)b0[v0 + dz], w101 = (float)b0[v0 + dz + 4];
        const float w011 = (float)b0[v0 + dz + dy], w111 = (float)b0[v0 + dz + dy + 4];
        const float c00 = lerpf(w000, w100, f[c][0]);
        const float c10 = lerpf(w010, w110, f[c][0]);
        const float c01 = lerpf(w001, w101, f[c][0]);
        const float c11 = lerpf(w011, w111, f[c][0]);
        sv[c] = lerpf(lerpf(c00, c10, f[c][1]), lerpf(c01, c11, f[c][1]), f[c][2]);
        vox[c] = dvox != nullptr && L == 0;
    }
    // forward chain over the C events, then back
    Classified cq[C];
    float rgba[C][4], Tc[C];
    float Tp = 1.0f;
#pragma unroll
    for (int c = 0; c < C; c++) {
        cq[c] = classify(sv[c], ub[c], usc[c], tb.lut[c]);
        rgba[c][0] = __builtin_fmaf(cq[c].fr, cq[c].de.x, cq[c].e0.x);
        rgba[c][1] = __builtin_fmaf(cq[c].fr, cq[c].de.y, cq[c].e0.y);
        rgba[c][2] = __builtin_fmaf(cq[c].fr, cq[c].de.z, cq[c].e0.z);
        rgba[c][3] = __builtin_fmaf(cq[c].fr, cq[c].de.w, cq[c].e0.w);
        Tc[c] = Tp;
        Tp = Tp - Tp * rgba[c][3];
    }
    const float gC[3] = {gi.x, gi.y, gi.z}, gA = gi.w;
    float Bc[3] = {0.0f, 0.0f, 0.0f}, Ba = 0.0f;
#pragma unroll
    for (int c = C - 1; c >= 0; c--) {
        const float a = rgba[c][3];
        float gq[4];
        for (int q = 0; q < 3; q++) gq[q] = gC[q] * Tc[c] * a;
        gq[3] = Tc[c] * (gC[0] * (rgba[c][0] - Bc[0]) + gC[1] * (rgba[c][1] - Bc[1]) +
                         gC[2] * (rgba[c][2] - Bc[2]) + gA * (1.0f - Ba));
        for (int q = 0; q < 3; q++) Bc[q] = a * rgba[c][q] + (1.0f - a) * Bc[q];
        Ba = a + (1.0f - a) * Ba;
        const float fr = cq[c].fr;
        for (int q = 0; q < 4; q++) {
            const float ga = (1.0f - fr) * gq[q], gb = fr * gq[q];
            if (ga != 0.0f) atomicAdd(&s_dlut[c][cq[c].i][q], ga);
            if (gb != 0.0f) atomicAdd(&s_dlut[c][cq[c].i + 1][q], gb);
        }
        if (vox[c] && cq[c].inside) {
            const float4 de = cq[c].de;
            const float gs = usc[c] * (gq[0] * de.x + gq[1] * de.y + gq[2] * de.z + gq[3] * de.w);
            if (gs != 0.0f) {
                for (int corner = 0; corner < 8; corner++) {
                    const int dxx = corner & 1, dyy = (corner >> 1) & 1, dzz = corner >> 2;
                    const float wgt = (dxx ? f[c][0] : 1.0f - f[c][0]) *
                                      (dyy ? f[c][1] : 1.0f - f[c][1]) *
                                      (dzz ? f[c][2] : 1.0f - f[c][2]);
                    const int gx = min(max(org[c][0] + ii[c][0] + dxx, 0), g.dims[0] - 1);
                    const int gy = min(max(org[c][1] + ii[c][1] + dyy, 0), g.dims[1] - 1);
                    const int gz = min(max(org[c][2] + ii[c][2] + dzz, 0), g.dims[2] - 1);
                    atomicAdd(dvox + c * nvox0 + ((int64_t)gz * g.dims[1] + gy) * g.dims[0] + gx,
                              gs * wgt);
                }
            }
        }
    }
}

template <typename T, int C>
__global__ void __launch_bounds__(kThreads)
k_render_backward_mip(VolGeom g, const DevCell *__restrict__ table,
                      const uint8_t *__restrict__ pool, uint64_t brick_bytes,
                      const DevView *__restrict__ views, const WgItem *__restrict__ items,
                      float *dvox)
{
    __shared__ ViewTables<C> tb;
    __shared__ float s_dlut[C][256][4];
    const WgItem it = items[blockIdx.x];
    const DevView &V = views[it.view];
    for (int i = threadIdx.x; i < C * 256 * 4; i += kThreads) (&s_dlut[0][0][0])[i] = 0.0f;
    build_tables<C>(V, tb);   // ends with a barrier
    if (V.xform_on)
        mip_backward_body<T, C, true>(g, table, pool, brick_bytes, V, it, tb, s_dlut, dvox);
    else
        mip_backward_body<T, C, false>(g, table, pool, brick_bytes, V, it, tb, s_dlut, dvox);
    __syncthreads();
    for (int i = threadIdx.x; i < C * 256 * 4; i += kThreads) {
        const float v = (&s_dlut[0][0][0])[i];
        if (v != 0.0f) atomicAdd(V.dlut + i, v);
    }
}

// dL/dctrl[v][c][j][q] += sum over table entries k of (weight of control point j in entry k)
// * dL/dtable[v][c][k][q]; the weights are those of the table construction.
__global__ void k_lut_to_ctrl(const DevView *views, int n_views, int C, float *dctrl)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int q = i & 3, j = (i >> 2) & 7, c = (i >> 5) % C, v = (i >> 5) / C;
    if (v >= n_views) return;
    const DevView &V = views[v];
    float acc = 0.0f;
    for (int k = 0; k < 256; k++) {
        int js;
        float f;
        tf_segment(V.tf_pos[c], k, js, f);
        const float gk = V.dlut[(c * 256 + k) * 4 + q];
        if (js == j) acc += (1.0f - f) * gk;
        if (js + 1 == j) acc += f * gk;
    }
    dctrl[(((int64_t)V.user_index * C + c) * 8 + j) * 4 + q] += acc;
}

template <typename T>
hipError_t launch_bw_typed(const VolGeom &g, const DevCell *table, const void *pool,
                           uint64_t brick_bytes, const DevView *views, const WgItem *items,
                           int n_items, float *dvox, int vg_shape, float *dctrl, hipStream_t s)
{
    const dim3 grid(n_items), block(kThreads);
    const uint8_t *p = (const uint8_t *)pool;
#define OCTRC_BW(TT, CC)                                                                          \
    do {                                                                                          \
        if (dvox)                                                                                 \
            hipLaunchKernelGGL((k_render_backward<TT, CC, true>), grid, block, 0, s, g, table, p,  \
                               brick_bytes, views, items, dvox, vg_shape, dctrl);                 \
        else                                                                                      \
            hipLaunchKernelGGL((k_render_backward<TT, CC, false>), grid, block, 0, s, g, table, p, \
                               brick_bytes, views, items, dvox, vg_shape, dctrl);                 \
    } while (0)
    switch (g.C) {
    case 1: OCTRC_BW(T, 1); break;
    case 2: OCTRC_BW(T, 2); break;
    case 3: OCTRC_BW(T, 3); break;
    default: OCTRC_BW(T, 4); break;
    }
#undef OCTRC_BW
    return hipGetLastError();
}

}  // namespace

hipError_t launch_render_backward(const VolGeom &g, const DevCell *table, const void *pool,
                                  uint64_t brick_bytes, const DevView *views, const WgItem *items,
                                  int n_items, float *dvox, int vg_shape, float *dctrl,
                                  hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    if (g.dtype == 0)
        return launch_bw_typed<uint16_t>(g, table, pool, brick_bytes, views, items, n_items, dvox,
                                         vg_shape, dctrl, s);
    return launch_bw_typed<float>(g, table, pool, brick_bytes, views, items, n_items, dvox,
                                  vg_shape, dctrl, s);
}

size_t voxgrad_blocked_floats(const VolGeom &g, int shape)
{
    return (size_t)BlockShape(shape, g.dims).plane * (size_t)g.C;
}

namespace {
// dvox[c][z][y][x] += the scratch's value of (x, y, z) in plane c; one block per thread (the
// block's values are contiguous, and neighbouring threads hold neighbouring blocks, which are
// neighbours along x in dvox)
__global__ void __launch_bounds__(256)
k_voxgrad_unblock(VolGeom g, int shape, const float *__restrict__ blk, float *__restrict__ dvox)
{
    const BlockShape bs(shape, g.dims);
    const int64_t nx = g.dims[0], ny = g.dims[1], nz = g.dims[2];
    const int64_t nvox0 = nx * ny * nz;
    const int64_t nblk = bs.plane >> bs.sb;
    const int per = 1 << bs.sb;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nblk * g.C;
         i += (int64_t)gridDim.x * 256) {
        const int64_t c = i / nblk, b = i - c * nblk;
        const int64_t bx = b % bs.nbx, by = (b / bs.nbx) % bs.nby, bz = b / (bs.nbx * bs.nby);
        const float *src = blk + c * bs.plane + (b << bs.sb);
        auto add = [&](int e, float v) {
            const int64_t x = (bx << bs.sx) + (e & ((1 << bs.sx) - 1));
            const int64_t y = (by << bs.sy) + ((e >> bs.sx) & ((1 << bs.sy) - 1));
            const int64_t z = (bz << bs.sz) + (e >> (bs.sx + bs.sy));
            if (x < nx && y < ny && z < nz) dvox[c * nvox0 + (z * ny + y) * nx + x] += v;
        };
        if (per == 16) {   // one 64-byte block: four 16-byte loads
            float4 q[4];
#pragma unroll
            for (int k = 0; k < 4; k++) q[k] = ((const float4 *)src)[k];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                add(4 * k, q[k].x);
                add(4 * k + 1, q[k].y);
                add(4 * k + 2, q[k].z);
                add(4 * k + 3, q[k].w);
            }
        } else {
            for (int e = 0; e < per; e++) add(e, src[e]);
        }
    }
}
}  // namespace

hipError_t launch_voxgrad_unblock(const VolGeom &g, int shape, const float *blk, float *dvox,
                                  hipStream_t s)
{
    const BlockShape bs(shape, g.dims);
    const int64_t n = (bs.plane >> bs.sb) * g.C;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_voxgrad_unblock, dim3((unsigned)std::min<int64_t>((n + 255) / 256, 1 << 20)),
                       dim3(256), 0, s, g, shape, blk, dvox);
    return hipGetLastError();
}

hipError_t launch_render_backward_mip(const VolGeom &g, const DevCell *table, const void *pool,
                                      uint64_t brick_bytes, const DevView *views,
                                      const WgItem *items, int n_items, float *dvox, hipStream_t s)
{
    if (n_items == 0) return hipSuccess;
    const dim3 grid(n_items), block(kThreads);
    const uint8_t *p = (const uint8_t *)pool;
#define OCTRC_MIPBW(T, CC) hipLaunchKernelGGL((k_render_backward_mip<T, CC>), grid, block, 0, s, g, \
                                              table, p, brick_bytes, views, items, dvox)
    if (g.dtype == 0) {
        switch (g.C) {
        case 1: OCTRC_MIPBW(uint16_t, 1); break;
        case 2: OCTRC_MIPBW(uint16_t, 2); break;
        case 3: OCTRC_MIPBW(uint16_t, 3); break;
        default: OCTRC_MIPBW(uint16_t, 4); break;
        }
    } else {
        switch (g.C) {
        case 1: OCTRC_MIPBW(float, 1); break;
        case 2: OCTRC_MIPBW(float, 2); break;
        case 3: OCTRC_MIPBW(float, 3); break;
        default: OCTRC_MIPBW(float, 4); break;
        }
    }
#undef OCTRC_MIPBW
    return hipGetLastError();
}

hipError_t launch_lut_to_ctrl(const DevView *views, int n_views, int C, float *dctrl, hipStream_t s)
{
    const int n = n_views * C * 32;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_lut_to_ctrl, dim3((n + 255) / 256), dim3(256), 0, s, views, n_views, C, dctrl);
    return hipGetLastError();
}

}  // namespace octrc
