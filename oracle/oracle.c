/*
 * CPU oracle for the multi-channel brick-octree ray caster (FP64, plain and slow on purpose).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include, link or call this
 * file; only the test-suite, the smoke check and the CPU-baseline leg of the benchmark use it.
 * It shares no code, header or table with the HIP path.
 *
 * It works on dense per-level arrays, not on bricks or a traversal: every quantity is written
 * as the definition the paper states (or the reading chosen where the paper is silent),
 * evaluated directly.
 *
 *   - Mipmap (Sec. "CPU Data Structure", Eq. 1; "Handling Volumes of Arbitrary Dimensions"):
 *     N = min n with M*2^n >= max(D); level L has valid extent ceil(D / 2^L); level L+1 is the
 *     half-sampling of level L over the valid children only (out-of-volume voxels are never
 *     used).  uint16: integer mean rounded half up, floor((2s+n)/(2n)); float32: the exact sum
 *     divided by n (n is a power of two) rounded once to float32.
 *   - Octree states ("CPU Data Structure", "Incremental Construction" steps 1-3,
 *     "Handling Multi-Channel Data"): a node is populated when any valid level-0 voxel of its
 *     region was inserted (any channel), complete when every valid voxel was inserted in every
 *     channel.  Populated nodes above level 0 have all eight children.  Top-down, the first
 *     complete node whose whole subtree satisfies max-min < threshold in every channel becomes a
 *     homogeneous leaf (its subtree is removed).  Otherwise a complete node whose own brick
 *     satisfies max-min < threshold in every channel is homogeneous but keeps its children; any
 *     other populated node holds a brick.  AVG is the rounded mean of the node's own level-L
 *     brick over its valid voxels.  Only complete nodes are ever made homogeneous (reading of
 *     the paper's mid-stream deletion, which would otherwise lose data of partly inserted
 *     bricks), so the tree depends only on the inserted data, not on how it was chunked.
 *   - Represented field R_L: V_L where the level-L node holding the voxel is a brick, else the
 *     AVG of the deepest existing node at level >= L containing it.  Bordered bricks
 *     ("Filtering across Brick Boundaries"): one voxel of overlap on every side, i.e. R_L at the
 *     neighbour index clamped to the valid extent.
 *   - Ray casting (Algorithm 1, "Basic Ray-Casting"): front-to-back emission-absorption along
 *     t_k = t0 + k*step while t_k < t1; the node holding the sample at the ray's LOD decides
 *     trilinear (brick) or AVG; per channel, in channel order, the sample is classified by a
 *     256-entry piecewise-linear RGBA table and composited ("accumulation level intermixing"),
 *     then early termination is tested once per position.
 *   - Maximum intensity projection ("Basic Ray-Casting": the traversal serves other compositing
 *     modes; Fig. 6, Table 1): per channel the largest sample along the ray is classified once,
 *     and the C classified values are composited in channel order like one DVR position.
 *     Early termination does not apply.
 *   - Missing bricks ("Basic Ray-Casting", "Full-Frame Ray-Casting"): a brick node whose brick
 *     is not resident is sampled with its AVG; under the full-frame fallback the resident brick
 *     of the first of the two coarser levels on the sample's path is interpolated instead, and
 *     only when neither is resident the AVG.
 *   - Chromatic-aberration correction ("Correction of Chromatic Aberration"): optionally each
 *     channel samples the volume at its own affine image of the ray position.
 *
 * Storage: level values are kept in the volume's data type (uint16 or float32), which holds
 * every value of the mipmap exactly (integer means for uint16, float32-rounded means for
 * float32), and R_L is evaluated at each lookup from the node states; nothing is stored twice.
 *
 * Precision: values, classification and compositing are FP64.  The geometric decisions (ray
 * direction, entry/exit parameter, clip planes, LOD, sample positions and the voxel/node a
 * sample falls into) are integer outcomes of floating-point arithmetic; both implementations
 * take them in IEEE float32 following one written operation sequence (each line below is one
 * correctly rounded float32 operation, no fused multiply-add), so that they agree exactly.
 * The trilinear weights are the float32 fractional parts of those positions, promoted to FP64.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXL 16
#define ORC_MAXC 4

typedef struct {
    int32_t dims[3];       /* Dx, Dy, Dz */
    int32_t channels;      /* 1..4 */
    int32_t brick;         /* M, even */
    int32_t dtype;         /* 0 = uint16, 1 = float32 */
    double background;
    double threshold;      /* strict '<'; 0 never merges */
} orc_params;

typedef struct {
    float eye[3], target[3], up[3];
    float fov_y_deg;
    int32_t width, height;
    float step;
    float ert_alpha;       /* >= 1: no early termination */
    int32_t lod;           /* -1: per-ray footprint */
    int32_t n_clip;
    float clip[3][4];      /* keep p with n.p >= d */
    float tf_pos[ORC_MAXC][8];
    float tf_rgba[ORC_MAXC][8][4];
    float window[ORC_MAXC][2];
    int32_t mode;          /* 0: emission-absorption (DVR), 1: maximum intensity projection */
    int32_t fullframe;     /* 1: missing bricks fall back to the two coarser levels */
    int32_t n_xform;       /* 0, or C: channel c samples at xform[c] applied to the position */
    float xform[ORC_MAXC][3][4];   /* rows (m_a0, m_a1, m_a2, b_a) of p' = M p + b */
} orc_view;

enum { ST_NONE = -1, ST_EMPTY = 0, ST_HOMOG_LEAF = 1, ST_HOMOG = 2, ST_BRICK = 3 };

typedef struct {
    int8_t exists, populated, complete, has_children, state;
    int8_t nonresident;    /* brick node whose brick is not in the render pool: sampled with AVG */
    double avg[ORC_MAXC], bmin[ORC_MAXC], bmax[ORC_MAXC], bsum[ORC_MAXC];
    double smin[ORC_MAXC], smax[ORC_MAXC];
    int64_t count;         /* valid level-L voxels in the node's brick */
} orc_node;

typedef struct {
    orc_params p;
    int N;
    int ext[ORC_MAXL][3];
    int G[ORC_MAXL];
    void *V[ORC_MAXL];     /* level values, planar [C][ez][ey][ex], in the data type */
    orc_node *nodes[ORC_MAXL];
    int poked;             /* a level-0 value was replaced in place (orc_poke_level0) */
} orc_tree;

/* ------------------------------------------------------------------ helpers */

static int64_t lvl_voxels(const orc_tree *t, int L)
{
    return (int64_t)t->ext[L][0] * t->ext[L][1] * t->ext[L][2];
}

static int64_t lvl_index(const orc_tree *t, int L, int c, int z, int y, int x)
{
    return (((int64_t)c * t->ext[L][2] + z) * t->ext[L][1] + y) * t->ext[L][0] + x;
}

/* Level-L value at planar index i (channel included), exact in FP64. */
static double vget(const orc_tree *t, int L, int64_t i)
{
    return t->p.dtype == 0 ? (double)((const uint16_t *)t->V[L])[i]
                           : (double)((const float *)t->V[L])[i];
}

/* Stores a value that the data type holds exactly (a mean of the mipmap or a replacement). */
static void vset(orc_tree *t, int L, int64_t i, double v)
{
    if (t->p.dtype == 0) ((uint16_t *)t->V[L])[i] = (uint16_t)v;
    else ((float *)t->V[L])[i] = (float)v;
}

static double lvl_get(const orc_tree *t, int L, int c, int z, int y, int x)
{
    return vget(t, L, lvl_index(t, L, c, z, y, x));
}

static orc_node *node_at(const orc_tree *t, int L, int bx, int by, int bz)
{
    int g = t->G[L];
    return &t->nodes[L][((int64_t)bz * g + by) * g + bx];
}

/* Round-half-up mean of an integer sum over n values (uint16 data). */
static double rhu_mean_int(double sum, int64_t n)
{
    uint64_t s = (uint64_t)sum;
    return (double)((2 * s + (uint64_t)n) / (2 * (uint64_t)n));
}

/* Mean for the data type: uint16 -> rounded half up; float32 -> float32(sum / n). */
static double type_mean(const orc_tree *t, double sum, int64_t n)
{
    if (t->p.dtype == 0) return rhu_mean_int(sum, n);
    return (double)(float)(sum / (double)n);
}

static int imin(int a, int b) { return a < b ? a : b; }
static int imax(int a, int b) { return a > b ? a : b; }

/* ------------------------------------------------------------------ build */

void orc_free(orc_tree *t);
int orc_num_threads(void);

/* Eq. 1: the octree has N+1 levels with N the smallest n for which M * 2^n covers the
 * largest dimension (the volume is extended virtually to M * 2^N per axis). */
int orc_tree_depth(const int32_t dims[3], int M)
{
    const int dmax = imax(dims[0], imax(dims[1], dims[2]));
    int N = 0;
    while ((int64_t)M << N < dmax) N++;
    return N;
}

/* Statistics of node (L, b) from the definitions ("CPU Data Structure"):
 *   own brick:  min, max and sum over the node's valid level-L voxels (AVG follows from them);
 *   subtree:    min and max over every value stored in the subtree -- the node's own brick and
 *               the subtrees of its children; at level 0 the subtree is the brick itself --
 *               and which of the region's valid level-0 voxels were inserted (any / all),
 *               which at level 0 is read from the mask and above is the union of the
 *               children's regions.  (Coarser values are means of finer ones, so this is also
 *               the minimum / maximum over the node's level-0 region.)
 * Children are computed before their parents (levels bottom-up). */
static void node_stats(orc_tree *t, const uint8_t *mask, int L, const int b[3])
{
    const orc_params *p = &t->p;
    const int C = p->channels, M = p->brick;
    orc_node *nd = node_at(t, L, b[0], b[1], b[2]);
    /* own brick at level L */
    int lo[3], hi[3];
    for (int a = 0; a < 3; a++) {
        lo[a] = b[a] * M;
        hi[a] = imin((b[a] + 1) * M, t->ext[L][a]);
    }
    int64_t cnt = 0;
    for (int c = 0; c < C; c++) {
        double mn = INFINITY, mx = -INFINITY, sm = 0.0;
        cnt = 0;
        for (int z = lo[2]; z < hi[2]; z++)
            for (int y = lo[1]; y < hi[1]; y++)
                for (int x = lo[0]; x < hi[0]; x++) {
                    double v = lvl_get(t, L, c, z, y, x);
                    mn = fmin(mn, v);
                    mx = fmax(mx, v);
                    sm += v;
                    cnt++;
                }
        nd->bmin[c] = cnt ? mn : 0.0;
        nd->bmax[c] = cnt ? mx : 0.0;
        nd->bsum[c] = sm;
    }
    nd->count = cnt;
    if (cnt == 0) {          /* outside the volume (virtual extension): no voxels */
        nd->populated = nd->complete = 0;
        for (int c = 0; c < C; c++) nd->smin[c] = nd->smax[c] = 0.0;
        return;
    }
    int any = 0, all = 1;
    double smin[ORC_MAXC], smax[ORC_MAXC];
    for (int c = 0; c < C; c++) {
        smin[c] = nd->bmin[c];
        smax[c] = nd->bmax[c];
    }
    if (L == 0) {
        for (int z = lo[2]; z < hi[2]; z++)
            for (int y = lo[1]; y < hi[1]; y++)
                for (int x = lo[0]; x < hi[0]; x++) {
                    const uint8_t m = mask[((int64_t)z * p->dims[1] + y) * p->dims[0] + x];
                    for (int c = 0; c < C; c++) {
                        int ins = (m >> c) & 1;
                        any |= ins;
                        all &= ins;
                    }
                }
    } else {
        for (int k = 0; k < 8; k++) {
            const orc_node *ch = node_at(t, L - 1, 2 * b[0] + (k & 1), 2 * b[1] + ((k >> 1) & 1),
                                         2 * b[2] + (k >> 2));
            if (ch->count == 0) continue;   /* a child outside the volume */
            any |= ch->populated;
            all &= ch->complete;
            for (int c = 0; c < C; c++) {
                smin[c] = fmin(smin[c], ch->smin[c]);
                smax[c] = fmax(smax[c], ch->smax[c]);
            }
        }
    }
    for (int c = 0; c < C; c++) {
        nd->smin[c] = smin[c];
        nd->smax[c] = smax[c];
    }
    nd->populated = (int8_t)any;
    nd->complete = (int8_t)all;
}

orc_tree *orc_build(const orc_params *p, const void *v0, const uint8_t *mask)
{
    if (p->channels < 1 || p->channels > ORC_MAXC || p->brick < 2 || (p->brick & 1)) return NULL;
    orc_tree *t = (orc_tree *)calloc(1, sizeof(orc_tree));
    t->p = *p;
    const int C = p->channels;
    const int N = orc_tree_depth(p->dims, p->brick);
    const size_t esz = p->dtype == 0 ? 2 : 4;
    t->N = N;
    for (int L = 0; L <= N; L++) {
        for (int a = 0; a < 3; a++)
            t->ext[L][a] = (int)(((int64_t)p->dims[a] + ((int64_t)1 << L) - 1) >> L);
        t->G[L] = 1 << (N - L);
        t->V[L] = malloc(esz * C * lvl_voxels(t, L));
        t->nodes[L] = (orc_node *)calloc((size_t)t->G[L] * t->G[L] * t->G[L], sizeof(orc_node));
        if (!t->V[L] || !t->nodes[L]) {
            orc_free(t);
            return NULL;
        }
    }

    /* Level 0: the inserted data (background where nothing was inserted is already in v0). */
    memcpy(t->V[0], v0, esz * C * lvl_voxels(t, 0));

    /* Levels 1..N: half-sampling of the valid children. */
    for (int L = 0; L < N; L++) {
        const int *e = t->ext[L], *e1 = t->ext[L + 1];
        for (int c = 0; c < C; c++)
#pragma omp parallel for schedule(static)
            for (int z = 0; z < e1[2]; z++)
                for (int y = 0; y < e1[1]; y++)
                    for (int x = 0; x < e1[0]; x++) {
                        double s = 0.0;
                        int64_t n = 0;
                        for (int dz = 0; dz < 2; dz++)
                            for (int dy = 0; dy < 2; dy++)
                                for (int dx = 0; dx < 2; dx++) {
                                    int cz = 2 * z + dz, cy = 2 * y + dy, cx = 2 * x + dx;
                                    if (cz >= e[2] || cy >= e[1] || cx >= e[0]) continue;
                                    s += lvl_get(t, L, c, cz, cy, cx);
                                    n++;
                                }
                        vset(t, L + 1, lvl_index(t, L + 1, c, z, y, x), type_mean(t, s, n));
                    }
    }

    /* Per-node statistics, level by level from the finest (nodes of one level are
     * independent). */
    for (int L = 0; L <= N; L++) {
        const int g = t->G[L];
        const int64_t g3 = (int64_t)g * g * g;
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t i = 0; i < g3; i++) {
            int b[3] = {(int)(i % g), (int)((i / g) % g), (int)(i / ((int64_t)g * g))};
            node_stats(t, mask, L, b);
        }
    }

    /* States, top-down from the root (the root always exists). */
    for (int L = N; L >= 0; L--) {
        int g = t->G[L];
        for (int bz = 0; bz < g; bz++)
            for (int by = 0; by < g; by++)
                for (int bx = 0; bx < g; bx++) {
                    orc_node *nd = node_at(t, L, bx, by, bz);
                    int exists = (L == N) ? 1 : node_at(t, L + 1, bx / 2, by / 2, bz / 2)->has_children;
                    nd->exists = (int8_t)exists;
                    nd->has_children = 0;
                    nd->state = ST_NONE;
                    if (!exists) continue;
                    if (!nd->populated) {
                        nd->state = ST_EMPTY;
                        for (int c = 0; c < C; c++)
                            nd->avg[c] = p->dtype == 0 ? p->background : (double)(float)p->background;
                        continue;
                    }
                    for (int c = 0; c < C; c++) nd->avg[c] = type_mean(t, nd->bsum[c], nd->count);
                    int sub_h = nd->complete, own_h = nd->complete;
                    for (int c = 0; c < C; c++) {
                        if (!(nd->smax[c] - nd->smin[c] < p->threshold)) sub_h = 0;
                        if (!(nd->bmax[c] - nd->bmin[c] < p->threshold)) own_h = 0;
                    }
                    if (sub_h) {
                        nd->state = ST_HOMOG_LEAF;
                    } else {
                        nd->has_children = (int8_t)(L > 0);
                        nd->state = own_h ? ST_HOMOG : ST_BRICK;
                    }
                }
    }
    return t;
}

/* Represented field R_L at voxel (x, y, z) of level L: V_L where the level-L node holding the
 * voxel is a brick, else the AVG of the deepest existing node at level >= L containing it.
 * Returns that node when the value is its AVG, NULL when it is V_L. */
static const orc_node *r_source(const orc_tree *t, int L, int x, int y, int z)
{
    const int M = t->p.brick;
    int bx = x / M, by = y / M, bz = z / M, l = L;
    const orc_node *nd = node_at(t, L, bx, by, bz);
    while (!nd->exists) {
        l++;
        bx >>= 1; by >>= 1; bz >>= 1;
        nd = node_at(t, l, bx, by, bz);
    }
    return (l == L && nd->state == ST_BRICK) ? NULL : nd;
}

void orc_free(orc_tree *t)
{
    if (!t) return;
    for (int L = 0; L <= t->N; L++) {
        free(t->V[L]);
        free(t->nodes[L]);
    }
    free(t);
}

int orc_num_levels(const orc_tree *t) { return t->N + 1; }

void orc_level_extent(const orc_tree *t, int L, int32_t *ext3)
{
    for (int a = 0; a < 3; a++) ext3[a] = t->ext[L][a];
}

/* Copy level L of the mipmap (planar [C][ez][ey][ex]) into out, in the data type. */
int orc_read_level(const orc_tree *t, int L, void *out)
{
    if (L < 0 || L > t->N || (t->poked && L > 0)) return -1;
    memcpy(out, t->V[L], (t->p.dtype == 0 ? 2 : 4) * t->p.channels * lvl_voxels(t, L));
    return 0;
}

/* ------------------------------------------------------------------ canonical dump
 * Layout (little endian):
 *   header, 64 bytes: "OCTDUMP1", int32 dims[3], C, M, N, dtype, n_nodes, n_bricks, pad to 64
 *   n_nodes records of 192 bytes, existing nodes ordered by (level descending, z, y, x):
 *     int32 level, bx, by, bz, state, flags (1 has_children | 2 complete | 4 populated), 0, 0
 *     float64 avg[4], bmin[4], bmax[4], smin[4], smax[4]   (unused channels are 0;
 *                                                          stats are 0 for unpopulated nodes)
 *   then, for every brick node in record order, its bordered brick: (M+2)^3 voxels, channel
 *   interleaved [z][y][x][c], in the data type (uint16 or float32).
 */
#define DUMP_HDR 64
#define DUMP_REC 192

size_t orc_dump(const orc_tree *t, void *buf, size_t cap)
{
    if (t->poked) return 0;
    const int C = t->p.channels, M = t->p.brick, S = M + 2;
    const size_t esz = t->p.dtype == 0 ? 2 : 4;
    int64_t n_nodes = 0, n_bricks = 0;
    for (int L = t->N; L >= 0; L--) {
        int64_t g3 = (int64_t)t->G[L] * t->G[L] * t->G[L];
        for (int64_t i = 0; i < g3; i++)
            if (t->nodes[L][i].exists) {
                n_nodes++;
                if (t->nodes[L][i].state == ST_BRICK) n_bricks++;
            }
    }
    size_t brick_bytes = (size_t)S * S * S * C * esz;
    size_t need = DUMP_HDR + (size_t)n_nodes * DUMP_REC + (size_t)n_bricks * brick_bytes;
    if (!buf || cap < need) return need;
    uint8_t *out = (uint8_t *)buf;
    memset(out, 0, DUMP_HDR + (size_t)n_nodes * DUMP_REC);
    memcpy(out, "OCTDUMP1", 8);
    int32_t hdr[9] = {t->p.dims[0], t->p.dims[1], t->p.dims[2], C, M, t->N, t->p.dtype,
                      (int32_t)n_nodes, (int32_t)n_bricks};
    memcpy(out + 8, hdr, sizeof hdr);
    uint8_t *rec = out + DUMP_HDR;
    uint8_t *bricks = out + DUMP_HDR + (size_t)n_nodes * DUMP_REC;
    for (int L = t->N; L >= 0; L--) {
        int g = t->G[L];
        for (int bz = 0; bz < g; bz++)
            for (int by = 0; by < g; by++)
                for (int bx = 0; bx < g; bx++) {
                    const orc_node *nd = node_at(t, L, bx, by, bz);
                    if (!nd->exists) continue;
                    int32_t head[8] = {L, bx, by, bz, nd->state,
                                       (nd->has_children ? 1 : 0) | (nd->complete ? 2 : 0) |
                                           (nd->populated ? 4 : 0) |
                                           (nd->state == ST_BRICK && !nd->nonresident ? 8 : 0),
                                       0, 0};
                    memcpy(rec, head, sizeof head);
                    double *d = (double *)(rec + 32);
                    for (int c = 0; c < C; c++) {
                        d[c] = nd->avg[c];
                        if (nd->populated) {
                            d[4 + c] = nd->bmin[c];
                            d[8 + c] = nd->bmax[c];
                            d[12 + c] = nd->smin[c];
                            d[16 + c] = nd->smax[c];
                        }
                    }
                    rec += DUMP_REC;
                    if (nd->state != ST_BRICK) continue;
                    const int *e = t->ext[L];
                    for (int z = 0; z < S; z++)
                        for (int y = 0; y < S; y++)
                            for (int x = 0; x < S; x++) {
                                int gz = imin(imax(bz * M - 1 + z, 0), e[2] - 1);
                                int gy = imin(imax(by * M - 1 + y, 0), e[1] - 1);
                                int gx = imin(imax(bx * M - 1 + x, 0), e[0] - 1);
                                const orc_node *src = r_source(t, L, gx, gy, gz);
                                for (int c = 0; c < C; c++) {
                                    double v = src ? src->avg[c] : lvl_get(t, L, c, gz, gy, gx);
                                    if (esz == 2) {
                                        uint16_t u = (uint16_t)v;
                                        memcpy(bricks, &u, 2);
                                    } else {
                                        float f = (float)v;
                                        memcpy(bricks, &f, 4);
                                    }
                                    bricks += esz;
                                }
                            }
                }
    }
    return need;
}

/* ------------------------------------------------------------------ transfer function
 * Per channel, a 256-entry RGBA table: entry k holds the piecewise-linear interpolation of the
 * 8 control points at x = k/255; outside the first/last control point the end value is held.
 * Classification of an intensity s: x = clamp((s - lo) / (hi - lo), 0, 1), u = 255 x,
 * i = min(floor(u), 254), value = lerp(entry i, entry i+1, u - i).
 */
typedef struct {
    double lut[ORC_MAXC][256][4];
} orc_luts;

/* Weight of control point j in entry k (the table is linear in the control RGBA). */
static void lut_weights(const float *pos, int k, int *j0, double *w0, double *w1)
{
    double x = (double)k / 255.0;
    if (x <= (double)pos[0]) { *j0 = 0; *w0 = 1.0; *w1 = 0.0; return; }
    if (x >= (double)pos[7]) { *j0 = 6; *w0 = 0.0; *w1 = 1.0; return; }
    int j = 0;
    while (j < 6 && !(x < (double)pos[j + 1])) j++;
    double f = (x - (double)pos[j]) / ((double)pos[j + 1] - (double)pos[j]);
    *j0 = j;
    *w0 = 1.0 - f;
    *w1 = f;
}

static void build_luts(const orc_view *v, int C, orc_luts *L)
{
    for (int c = 0; c < C; c++)
        for (int k = 0; k < 256; k++) {
            int j;
            double w0, w1;
            lut_weights(v->tf_pos[c], k, &j, &w0, &w1);
            for (int q = 0; q < 4; q++)
                L->lut[c][k][q] = w0 * (double)v->tf_rgba[c][j][q] + w1 * (double)v->tf_rgba[c][j + 1][q];
        }
}

/* ------------------------------------------------------------------ ray geometry (float32)
 * Camera frame, computed once per view in double and rounded to float32:
 *   f = (target - eye) / |target - eye|, r = (f x up) / |f x up|, u = r x f,
 *   th = tan(fov_y / 2), kx = th * W / H, ky = th, klod = 2 th / H.
 * Per pixel (i, j), each step one float32 operation, no fused multiply-add:
 *   a = (2i+1) / W;  b = (2j+1) / H;  sx = (a - 1) * kx;  sy = (1 - b) * ky
 *   dir_k = (f_k + sx * r_k) + sy * u_k;  n2 = (dir_x^2 + dir_y^2) + dir_z^2
 *   inv = 1 / sqrt(n2);  d_k = dir_k * inv;  o = eye
 *   box [0, D]: t0 = 0, t1 = +inf; per axis with d_k != 0: rk = 1 / d_k, ta = (0 - o_k) * rk,
 *     tb = (D_k - o_k) * rk, t0 = max(t0, min(ta, tb)), t1 = min(t1, max(ta, tb));
 *     with d_k == 0 the ray misses when o_k < 0 or o_k > D_k
 *   clip (n, d): nd = (n_x d_x + n_y d_y) + n_z d_z, no = (n_x o_x + n_y o_y) + n_z o_z,
 *     num = d - no; nd > 0: t0 = max(t0, num / nd); nd < 0: t1 = min(t1, num / nd);
 *     nd == 0: misses when no < d
 *   the pixel is empty unless t0 < t1
 *   LOD: fixed lod, or w = t0 * klod and L = clamp(floor(log2 w), 0, N) (L = 0 when w <= 0);
 *     floor(log2 w) is the binary exponent of w, exact
 *   sample k: t = t0 + float(k) * step, continue while t < t1; p_k = o_k + t * d_k
 *   voxel v_k = clamp(floor(p_k), 0, D_k - 1); node at level L: (v_k >> L) / M
 *   brick sample: q_k = p_k * 2^-L - 0.5 (exact), corner i0 = floor(q_k), weight f = q_k - i0
 */
typedef struct {
    float eye[3], f[3], r[3], u[3];
    float kx, ky, klod;
} orc_cam;

static void cam_setup(const orc_view *v, orc_cam *cm)
{
    double e[3], fw[3], rt[3], up[3], uu[3];
    for (int a = 0; a < 3; a++) {
        e[a] = (double)v->eye[a];
        fw[a] = (double)v->target[a] - e[a];
        up[a] = (double)v->up[a];
    }
    double n = sqrt((fw[0] * fw[0] + fw[1] * fw[1]) + fw[2] * fw[2]);
    for (int a = 0; a < 3; a++) fw[a] = fw[a] / n;
    rt[0] = fw[1] * up[2] - fw[2] * up[1];
    rt[1] = fw[2] * up[0] - fw[0] * up[2];
    rt[2] = fw[0] * up[1] - fw[1] * up[0];
    n = sqrt((rt[0] * rt[0] + rt[1] * rt[1]) + rt[2] * rt[2]);
    for (int a = 0; a < 3; a++) rt[a] = rt[a] / n;
    uu[0] = rt[1] * fw[2] - rt[2] * fw[1];
    uu[1] = rt[2] * fw[0] - rt[0] * fw[2];
    uu[2] = rt[0] * fw[1] - rt[1] * fw[0];
    double th = tan((double)v->fov_y_deg * (M_PI / 360.0));
    for (int a = 0; a < 3; a++) {
        cm->eye[a] = v->eye[a];
        cm->f[a] = (float)fw[a];
        cm->r[a] = (float)rt[a];
        cm->u[a] = (float)uu[a];
    }
    cm->kx = (float)(th * (double)v->width / (double)v->height);
    cm->ky = (float)th;
    cm->klod = (float)(2.0 * th / (double)v->height);
}

typedef struct {
    float o[3], d[3];
    float t0, t1;
    int L;
    int hit;
} orc_ray;

static void ray_setup(const orc_tree *t, const orc_view *v, const orc_cam *cm, int i, int j,
                      orc_ray *ry)
{
    float a = (float)(2 * i + 1) / (float)v->width;
    float b = (float)(2 * j + 1) / (float)v->height;
    float sx = (a - 1.0f) * cm->kx;
    float sy = (1.0f - b) * cm->ky;
    float dir[3];
    for (int k = 0; k < 3; k++) {
        float m1 = sx * cm->r[k];
        float s1 = cm->f[k] + m1;
        float m2 = sy * cm->u[k];
        dir[k] = s1 + m2;
    }
    float q0 = dir[0] * dir[0], q1 = dir[1] * dir[1], q2 = dir[2] * dir[2];
    float n2 = (q0 + q1) + q2;
    float inv = 1.0f / sqrtf(n2);
    for (int k = 0; k < 3; k++) {
        ry->d[k] = dir[k] * inv;
        ry->o[k] = cm->eye[k];
    }
    float t0 = 0.0f, t1 = INFINITY;
    int hit = 1;
    for (int k = 0; k < 3; k++) {
        float D = (float)t->p.dims[k];
        if (ry->d[k] != 0.0f) {
            float rk = 1.0f / ry->d[k];
            float ta = (0.0f - ry->o[k]) * rk;
            float tb = (D - ry->o[k]) * rk;
            t0 = fmaxf(t0, fminf(ta, tb));
            t1 = fminf(t1, fmaxf(ta, tb));
        } else if (ry->o[k] < 0.0f || ry->o[k] > D) {
            hit = 0;
        }
    }
    for (int c = 0; c < v->n_clip && c < 3; c++) {
        const float *pl = v->clip[c];
        float nd = (pl[0] * ry->d[0] + pl[1] * ry->d[1]) + pl[2] * ry->d[2];
        float no = (pl[0] * ry->o[0] + pl[1] * ry->o[1]) + pl[2] * ry->o[2];
        float num = pl[3] - no;
        if (nd > 0.0f) t0 = fmaxf(t0, num / nd);
        else if (nd < 0.0f) t1 = fminf(t1, num / nd);
        else if (no < pl[3]) hit = 0;
    }
    if (!(t0 < t1)) hit = 0;
    ry->t0 = t0;
    ry->t1 = t1;
    ry->hit = hit;
    int L;
    if (v->lod >= 0) {
        L = imin(v->lod, t->N);
    } else {
        float w = t0 * cm->klod;
        if (w > 0.0f && isfinite(w)) {
            L = ilogbf(w);
            L = imax(0, imin(L, t->N));
        } else {
            L = 0;
        }
    }
    ry->L = L;
}

/* ------------------------------------------------------------------ sampling */

/* What channel samples at a float32 position read: trilinear interpolation in R at level Ls
 * (the ray's LOD, or a coarser level under the full-frame fallback), or one node's AVG. */
typedef struct {
    int trilinear;             /* 1: trilinear in R_Ls, 0: constant */
    int Ls;                    /* level of the interpolated field */
    int64_t idx[8];            /* corner voxel indices within one channel of level Ls */
    double w[8];               /* trilinear weights */
    const orc_node *src[8];    /* corner value: NULL = V_Ls at idx, else that node's AVG */
    const orc_node *cnode;     /* constant case: the node whose AVG is the value */
    int avg_fallback;          /* a non-resident brick node approximated by its AVG */
} orc_sample_geo;

/* Trilinear set-up in R at level Ls: q = p 2^-Ls - 1/2 (exact), corner i0 = floor(q), weight
 * f = q - i0 (float32), corner indices clamped to the valid extent. */
static void trilinear_geo(const orc_tree *t, int Ls, const float p[3], orc_sample_geo *g)
{
    const int *e = t->ext[Ls];
    float scale = ldexpf(1.0f, -Ls);
    int i0[3];
    double f[3];
    for (int a = 0; a < 3; a++) {
        float q = p[a] * scale - 0.5f;
        float fl = floorf(q);
        i0[a] = (int)fl;
        f[a] = (double)(q - fl);
    }
    g->trilinear = 1;
    g->Ls = Ls;
    int k = 0;
    for (int dz = 0; dz < 2; dz++)
        for (int dy = 0; dy < 2; dy++)
            for (int dx = 0; dx < 2; dx++, k++) {
                int x = imax(0, imin(i0[0] + dx, e[0] - 1));
                int y = imax(0, imin(i0[1] + dy, e[1] - 1));
                int z = imax(0, imin(i0[2] + dz, e[2] - 1));
                g->idx[k] = ((int64_t)z * e[1] + y) * e[0] + x;
                g->src[k] = r_source(t, Ls, x, y, z);
                g->w[k] = (dx ? f[0] : 1.0 - f[0]) * (dy ? f[1] : 1.0 - f[1]) * (dz ? f[2] : 1.0 - f[2]);
            }
}

/* The node at the ray's LOD L holding the position's clamped voxel decides: a resident brick
 * is interpolated; a brick that is not resident is approximated by its AVG ("Basic
 * Ray-Casting"), or, under the full-frame fallback, by the resident brick of level L+1, else
 * of level L+2, on the position's path ("Full-Frame Ray-Casting"); any other node (and any
 * cell whose node does not exist) contributes the AVG of the deepest existing node. */
static void sample_geo(const orc_tree *t, int L, const float p[3], int fullframe,
                       orc_sample_geo *g)
{
    const int M = t->p.brick;
    int v[3], b[3];
    for (int a = 0; a < 3; a++) {
        int vi = (int)floorf(p[a]);
        vi = imax(0, imin(vi, t->p.dims[a] - 1));
        v[a] = vi;
        b[a] = (vi >> L) / M;
    }
    g->avg_fallback = 0;
    const orc_node *nd = node_at(t, L, b[0], b[1], b[2]);
    if (nd->exists && nd->state == ST_BRICK) {
        if (!nd->nonresident) {
            trilinear_geo(t, L, p, g);
            return;
        }
        if (fullframe)
            for (int l = L + 1; l <= L + 2 && l <= t->N; l++) {
                const orc_node *up = node_at(t, l, (v[0] >> l) / M, (v[1] >> l) / M, (v[2] >> l) / M);
                if (up->state == ST_BRICK && !up->nonresident) {
                    trilinear_geo(t, l, p, g);
                    return;
                }
            }
        g->trilinear = 0;
        g->cnode = nd;
        g->avg_fallback = 1;
        return;
    }
    int l = L;
    while (!nd->exists) {
        l++;
        b[0] >>= 1; b[1] >>= 1; b[2] >>= 1;
        nd = node_at(t, l, b[0], b[1], b[2]);
    }
    g->trilinear = 0;
    g->cnode = nd;
}

static double sample_value(const orc_tree *t, int c, const orc_sample_geo *g)
{
    if (!g->trilinear) return g->cnode->avg[c];
    const int64_t off = (int64_t)c * lvl_voxels(t, g->Ls);
    double s = 0.0;
    for (int k = 0; k < 8; k++)
        s += g->w[k] * (g->src[k] ? g->src[k]->avg[c] : vget(t, g->Ls, off + g->idx[k]));
    return s;
}

/* Position at which channel c is sampled ("Correction of Chromatic Aberration"): the ray
 * position itself, or its image under the channel's affine map, each row as float32
 * ((m0 p0 + m1 p1) + m2 p2) + b, every operation rounded once, no fused multiply-add. */
static void channel_position(const orc_view *v, int c, const float p[3], float pc[3])
{
    if (v->n_xform == 0) {
        for (int a = 0; a < 3; a++) pc[a] = p[a];
        return;
    }
    for (int a = 0; a < 3; a++) {
        const float *m = v->xform[c][a];
        float s0 = m[0] * p[0];
        float s1 = m[1] * p[1];
        float s2 = m[2] * p[2];
        float u = s0 + s1;
        float w = u + s2;
        pc[a] = w + m[3];
    }
}

/* The per-channel sample geometry of one ray position (shared by all channels when the view
 * has no channel transforms).  Returns the number of AVG fallbacks among the C samples. */
static int position_geo(const orc_tree *t, const orc_view *v, int L, const float p[3],
                        orc_sample_geo *g /* [C] */)
{
    const int C = t->p.channels;
    int nfb = 0;
    if (v->n_xform == 0) {
        sample_geo(t, L, p, v->fullframe, &g[0]);
        for (int c = 1; c < C; c++) g[c] = g[0];
        return g[0].avg_fallback ? C : 0;
    }
    for (int c = 0; c < C; c++) {
        float pc[3];
        channel_position(v, c, p, pc);
        sample_geo(t, L, pc, v->fullframe, &g[c]);
        nfb += g[c].avg_fallback;
    }
    return nfb;
}

/* Classification: returns rgba; *slot_i / *slot_f give the table cell, *dudx the slope
 * factor du/ds (0 where x is clamped). */
static void classify(const orc_luts *lu, const orc_view *v, int c, double s, double rgba[4],
                     int *slot_i, double *slot_f, double *duds)
{
    double lo = (double)v->window[c][0], hi = (double)v->window[c][1];
    double x = (s - lo) / (hi - lo);
    double dxds = 1.0 / (hi - lo);
    if (x <= 0.0) { x = 0.0; dxds = 0.0; }
    if (x >= 1.0) { x = 1.0; dxds = 0.0; }
    double u = 255.0 * x;
    int i = (int)floor(u);
    if (i > 254) i = 254;
    double fr = u - (double)i;
    for (int q = 0; q < 4; q++)
        rgba[q] = lu->lut[c][i][q] + fr * (lu->lut[c][i + 1][q] - lu->lut[c][i][q]);
    if (slot_i) *slot_i = i;
    if (slot_f) *slot_f = fr;
    if (duds) *duds = 255.0 * dxds;
}

/* ------------------------------------------------------------------ render
 * images: [n_views] pointers to [H][W][4] double (premultiplied RGBA, row 0 at the top).
 * Optional per-view [H][W] outputs:
 *   nsamp   int32: positions t_k < t1 (nominal samples);
 *   margin  double: DVR with early termination: the smallest |A - ert| over the termination
 *           tests of the ray; MIP: the smallest gap, over the channels, between the largest
 *           sample and the largest sample at any other position (0 = a tie); +inf otherwise.
 *           Both detect rays whose discrete outcome floating point could decide differently;
 *   navg    int32: channel samples that approximated a non-resident brick by its AVG.
 */
static int render_rows(const orc_tree *t, int n_views, const orc_view *views,
                       double *const *images, int32_t *const *nsamp, double *const *margin,
                       int32_t *const *navg, int row_begin, int row_end, int row_step,
                       int col_begin, int col_end);

static int view_ok(const orc_tree *t, const orc_view *v)
{
    if (v->width <= 0 || v->height <= 0) return 0;
    if (v->mode != 0 && v->mode != 1) return 0;
    if (v->n_xform != 0 && v->n_xform != t->p.channels) return 0;
    if (t->poked && v->lod != 0) return 0;
    return 1;
}

int orc_render(const orc_tree *t, int n_views, const orc_view *views, double *const *images,
               int32_t *const *nsamp, double *const *margin)
{
    return render_rows(t, n_views, views, images, nsamp, margin, NULL, 0, 1 << 30, 1, 0, 1 << 30);
}

/* One view with every optional output (any of them may be NULL). */
int orc_render_aux(const orc_tree *t, const orc_view *view, double *image, int32_t *nsamp,
                   double *margin, int32_t *navg)
{
    return render_rows(t, 1, view, &image, &nsamp, &margin, &navg, 0, 1 << 30, 1, 0, 1 << 30);
}

/* Same as orc_render for the rows row_begin, row_begin + row_step, ... only (other rows are
 * left untouched): a bounded sample of a large frame. */
int orc_render_rows(const orc_tree *t, const orc_view *view, double *image, int32_t *nsamp,
                    int row_begin, int row_step)
{
    if (row_begin < 0 || row_step < 1) return -1;
    return render_rows(t, 1, view, &image, &nsamp, NULL, NULL, row_begin, 1 << 30, row_step, 0,
                       1 << 30);
}

/* Same as orc_render for the pixels x0 <= i < x1, y0 <= j < y1 of the [H][W] image only (the
 * others are left untouched): the rays a local change of the volume can reach. */
int orc_render_window(const orc_tree *t, const orc_view *view, double *image, int x0, int y0,
                      int x1, int y1)
{
    if (x0 < 0 || y0 < 0 || x1 < x0 || y1 < y0) return -1;
    return render_rows(t, 1, view, &image, NULL, NULL, NULL, y0, y1, 1, x0, x1);
}

/* The pixels listed in px ([n][2] = column, row) of one view, written to out[n][4] (a sparse
 * sample of a large frame), with their nominal counts and margins when asked for. */
int orc_render_pixels(const orc_tree *t, const orc_view *view, const int32_t *px, int64_t n,
                      double *out, int32_t *nsamp, double *margin);

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* One ray: its premultiplied RGBA, nominal count, margin and AVG-fallback count. */
static void cast_ray(const orc_tree *t, const orc_view *v, const orc_cam *cm,
                     const orc_luts *lu, int i, int j, double px[4], int32_t *ns_out,
                     double *margin_out, int32_t *navg_out)
{
    const int C = t->p.channels;
    orc_ray ry;
    ray_setup(t, v, cm, i, j, &ry);
    double Cr = 0, Cg = 0, Cb = 0, A = 0, margin = INFINITY;
    int32_t ns = 0, nfb = 0;
    double mx1[ORC_MAXC], mx2[ORC_MAXC];   /* MIP: largest sample, largest at another position */
    for (int c = 0; c < C; c++) mx1[c] = mx2[c] = -INFINITY;
    const int mip = v->mode == 1;
    const int ert = !mip && v->ert_alpha < 1.0f;
    if (ry.hit) {
        for (int k = 0;; k++) {
            float tk = ry.t0 + (float)k * v->step;
            if (!(tk < ry.t1)) break;
            ns++;
            if (ert && A >= (double)v->ert_alpha) continue;
            float p[3];
            for (int a = 0; a < 3; a++) {
                float m = tk * ry.d[a];
                p[a] = ry.o[a] + m;
            }
            orc_sample_geo g[ORC_MAXC];
            nfb += position_geo(t, v, ry.L, p, g);
            for (int c = 0; c < C; c++) {
                double s = sample_value(t, c, &g[c]);
                if (mip) {
                    if (s > mx1[c]) {
                        mx2[c] = mx1[c];
                        mx1[c] = s;
                    } else if (s > mx2[c]) {
                        mx2[c] = s;
                    }
                    continue;
                }
                double rgba[4];
                classify(lu, v, c, s, rgba, NULL, NULL, NULL);
                double wgt = (1.0 - A) * rgba[3];
                Cr += wgt * rgba[0];
                Cg += wgt * rgba[1];
                Cb += wgt * rgba[2];
                A += wgt;
            }
            if (ert) {
                double m = fabs(A - (double)v->ert_alpha);
                if (m < margin) margin = m;
            }
        }
        if (mip && ns > 0) {
            for (int c = 0; c < C; c++) {
                double rgba[4];
                classify(lu, v, c, mx1[c], rgba, NULL, NULL, NULL);
                double wgt = (1.0 - A) * rgba[3];
                Cr += wgt * rgba[0];
                Cg += wgt * rgba[1];
                Cb += wgt * rgba[2];
                A += wgt;
                double gap = mx1[c] - mx2[c];
                if (gap < margin) margin = gap;
            }
        }
    }
    px[0] = Cr; px[1] = Cg; px[2] = Cb; px[3] = A;
    if (ns_out) *ns_out = ns;
    if (margin_out) *margin_out = margin;
    if (navg_out) *navg_out = nfb;
}

static int render_rows(const orc_tree *t, int n_views, const orc_view *views,
                       double *const *images, int32_t *const *nsamp, double *const *margin,
                       int32_t *const *navg, int row_begin, int row_end, int row_step,
                       int col_begin, int col_end)
{
    const int C = t->p.channels;
    for (int vi = 0; vi < n_views; vi++)
        if (!view_ok(t, &views[vi])) return -1;
    for (int vi = 0; vi < n_views; vi++) {
        const orc_view *v = &views[vi];
        orc_luts *lu = (orc_luts *)malloc(sizeof(orc_luts));
        build_luts(v, C, lu);
        orc_cam cm;
        cam_setup(v, &cm);
        const int W = v->width, H = v->height;
        const int j_end = row_end < H ? row_end : H, i_end = col_end < W ? col_end : W;
#pragma omp parallel for schedule(dynamic, 1)
        for (int j = row_begin; j < j_end; j += row_step)
            for (int i = col_begin; i < i_end; i++) {
                const int64_t q = (int64_t)j * W + i;
                cast_ray(t, v, &cm, lu, i, j, images[vi] + q * 4, nsamp ? &nsamp[vi][q] : NULL,
                         margin ? &margin[vi][q] : NULL, navg ? &navg[vi][q] : NULL);
            }
        free(lu);
    }
    return 0;
}

int orc_render_pixels(const orc_tree *t, const orc_view *view, const int32_t *px, int64_t n,
                      double *out, int32_t *nsamp, double *margin)
{
    if (!view_ok(t, view)) return -1;
    for (int64_t q = 0; q < n; q++)
        if (px[2 * q] < 0 || px[2 * q] >= view->width || px[2 * q + 1] < 0 ||
            px[2 * q + 1] >= view->height)
            return -1;
    orc_luts *lu = (orc_luts *)malloc(sizeof(orc_luts));
    build_luts(view, t->p.channels, lu);
    orc_cam cm;
    cam_setup(view, &cm);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < n; q++)
        cast_ray(t, view, &cm, lu, px[2 * q], px[2 * q + 1], out + q * 4,
                 nsamp ? nsamp + q : NULL, margin ? margin + q : NULL, NULL);
    free(lu);
    return 0;
}

/* ------------------------------------------------------------------ adjoint
 * Loss gradient by reverse-mode differentiation of the forward above, per ray, in FP64.
 * Inputs dL/dI per view [H][W][4].  Outputs (accumulated, caller zeroes):
 *   dctrl  [n_views][C][8][4]: gradient w.r.t. the control-point RGBA (positions fixed),
 *   dvox   [C][Dz][Dy][Dx] or NULL: gradient w.r.t. the level-0 voxel values, defined when the
 *          field sampled at level 0 is V_0 itself (every node a brick: threshold 0, everything
 *          inserted, LOD 0), through the trilinear weights of the clamped corner indices.
 * Compositing events e = (position, channel) in order: with T_e = 1 - A_e,
 *   C_{e+1} = C_e + T_e a_e rgb_e,  A_{e+1} = A_e + T_e a_e.
 * Walking back: g_rgb_e = gC T_e a_e, g_a_e = gC.rgb_e T_e + gA_{e+1} T_e,
 *   gA_e = gA_{e+1} (1 - a_e) - a_e gC.rgb_e.
 * MIP: the events are the C classified maxima; the maximum of channel c is the sample at the
 * first position where it is reached (the gradient of a maximum is taken at its arg max), so
 * its value gradient flows through that sample's trilinear weights.
 */
typedef struct {
    double A;              /* alpha before the event */
    double rgba[4];
    int slot_i;
    double slot_f, duds;
    orc_sample_geo g;      /* the sample's geometry (its channel's) */
    int c;
} orc_event;

/* Adds the gradient of one ray's events (in compositing order) into the thread's table
 * accumulator tl and into dvox. */
static void backprop_events(const orc_tree *t, const orc_luts *lu, const orc_event *ev, size_t ne,
                            const double gI[4], double *tl, double *dvox)
{
    const int64_t nv0 = lvl_voxels(t, 0);
    double gC[3] = {gI[0], gI[1], gI[2]}, gA = gI[3];
    for (size_t n = ne; n-- > 0;) {
        const orc_event *e = &ev[n];
        double T = 1.0 - e->A, a = e->rgba[3];
        double gcr = gC[0] * e->rgba[0] + gC[1] * e->rgba[1] + gC[2] * e->rgba[2];
        double g_rgba[4];
        for (int q = 0; q < 3; q++) g_rgba[q] = gC[q] * T * a;
        g_rgba[3] = gcr * T + gA * T;
        gA = gA * (1.0 - a) - a * gcr;
        /* into the table cell */
        double *d0 = tl + ((int64_t)e->c * 256 + e->slot_i) * 4;
        double *d1 = d0 + 4;
        double gs = 0.0;
        const double *l0 = lu->lut[e->c][e->slot_i], *l1 = lu->lut[e->c][e->slot_i + 1];
        for (int q = 0; q < 4; q++) {
            d0[q] += (1.0 - e->slot_f) * g_rgba[q];
            d1[q] += e->slot_f * g_rgba[q];
            gs += g_rgba[q] * (l1[q] - l0[q]);
        }
        gs *= e->duds;
        if (dvox && e->g.trilinear && e->g.Ls == 0) {
            double *dv = dvox + (int64_t)e->c * nv0;
            for (int k = 0; k < 8; k++) {
                if (e->g.src[k]) continue;   /* an AVG, not a voxel value */
                const double add = gs * e->g.w[k];
#pragma omp atomic
                dv[e->g.idx[k]] += add;
            }
        }
    }
}

int orc_render_grad(const orc_tree *t, int n_views, const orc_view *views,
                    const double *const *dL_dI, double *dctrl, double *dvox)
{
    const int C = t->p.channels;
    for (int vi = 0; vi < n_views; vi++)
        if (!view_ok(t, &views[vi])) return -1;
    for (int vi = 0; vi < n_views; vi++) {
        const orc_view *v = &views[vi];
        const int mip = v->mode == 1;
        const int ert = !mip && v->ert_alpha < 1.0f;
        orc_luts *lu = (orc_luts *)malloc(sizeof(orc_luts));
        build_luts(v, C, lu);
        orc_cam cm;
        cam_setup(v, &cm);
        const int W = v->width, H = v->height;
        double *dlut = (double *)calloc((size_t)C * 256 * 4, sizeof(double));
        /* rays are independent; their contributions are added with atomic updates (only the
         * order of the FP64 sums depends on the threads) */
#pragma omp parallel
        {
        size_t cap = 1024;
        orc_event *ev = (orc_event *)malloc(cap * sizeof(orc_event));
        double *tl = (double *)calloc((size_t)C * 256 * 4, sizeof(double));  /* this thread's */
#pragma omp for schedule(dynamic, 1)
        for (int j = 0; j < H; j++)
            for (int i = 0; i < W; i++) {
                const double *gI = dL_dI[vi] + ((int64_t)j * W + i) * 4;
                if (gI[0] == 0.0 && gI[1] == 0.0 && gI[2] == 0.0 && gI[3] == 0.0)
                    continue;  /* this ray contributes exactly zero */
                orc_ray ry;
                ray_setup(t, v, &cm, i, j, &ry);
                if (!ry.hit) continue;
                size_t ne = 0;
                double A = 0.0;
                double mx[ORC_MAXC];
                orc_sample_geo amax[ORC_MAXC];
                for (int c = 0; c < C; c++) mx[c] = -INFINITY;
                for (int k = 0;; k++) {
                    float tk = ry.t0 + (float)k * v->step;
                    if (!(tk < ry.t1)) break;
                    if (ert && A >= (double)v->ert_alpha) break;
                    float p[3];
                    for (int a = 0; a < 3; a++) {
                        float m = tk * ry.d[a];
                        p[a] = ry.o[a] + m;
                    }
                    orc_sample_geo g[ORC_MAXC];
                    position_geo(t, v, ry.L, p, g);
                    for (int c = 0; c < C; c++) {
                        double s = sample_value(t, c, &g[c]);
                        if (mip) {
                            if (s > mx[c]) {   /* the first position reaching the maximum */
                                mx[c] = s;
                                amax[c] = g[c];
                            }
                            continue;
                        }
                        if (ne == cap) {
                            cap *= 2;
                            ev = (orc_event *)realloc(ev, cap * sizeof(orc_event));
                        }
                        orc_event *e = &ev[ne++];
                        classify(lu, v, c, s, e->rgba, &e->slot_i, &e->slot_f, &e->duds);
                        e->A = A;
                        e->c = c;
                        e->g = g[c];
                        A += (1.0 - A) * e->rgba[3];
                    }
                }
                if (mip)
                    for (int c = 0; c < C; c++) {
                        orc_event *e = &ev[ne++];
                        classify(lu, v, c, mx[c], e->rgba, &e->slot_i, &e->slot_f, &e->duds);
                        e->A = A;
                        e->c = c;
                        e->g = amax[c];
                        A += (1.0 - A) * e->rgba[3];
                    }
                backprop_events(t, lu, ev, ne, gI, tl, dvox);
            }
        free(ev);
#pragma omp critical
        for (int k = 0; k < C * 256 * 4; k++) dlut[k] += tl[k];
        free(tl);
        }
        /* table entries -> control points */
        for (int c = 0; c < C; c++)
            for (int k = 0; k < 256; k++) {
                int jj;
                double w0, w1;
                lut_weights(v->tf_pos[c], k, &jj, &w0, &w1);
                for (int q = 0; q < 4; q++) {
                    double g = dlut[((int64_t)c * 256 + k) * 4 + q];
                    dctrl[(((int64_t)vi * C + c) * 8 + jj) * 4 + q] += w0 * g;
                    dctrl[(((int64_t)vi * C + c) * 8 + jj + 1) * 4 + q] += w1 * g;
                }
            }
        free(dlut);
        free(lu);
    }
    return 0;
}

/* Per-pixel ray set-up for tests: out[H][W][8] = o[3], d[3], t0, t1; lod_hit[H][W][2]. */
int orc_rays(const orc_tree *t, const orc_view *v, float *out, int32_t *lod_hit)
{
    orc_cam cm;
    cam_setup(v, &cm);
    for (int j = 0; j < v->height; j++)
        for (int i = 0; i < v->width; i++) {
            orc_ray ry;
            ray_setup(t, v, &cm, i, j, &ry);
            float *o = out + ((int64_t)j * v->width + i) * 8;
            for (int a = 0; a < 3; a++) {
                o[a] = ry.o[a];
                o[3 + a] = ry.d[a];
            }
            o[6] = ry.t0;
            o[7] = ry.t1;
            lod_hit[((int64_t)j * v->width + i) * 2] = ry.L;
            lod_hit[((int64_t)j * v->width + i) * 2 + 1] = ry.hit;
        }
    return 0;
}

/* Out-of-core rendering ("Brick Upload from RAM to GPU"): a brick node whose brick is not
 * resident is sampled with its AVG by the renderer (Algorithm 1, the request branch).  The
 * residency set is an input: the GPU path reports it.  The bordered bricks of resident
 * neighbours are unaffected (R_L does not depend on residency). */
int orc_set_nonresident(orc_tree *t, int L, int bx, int by, int bz, int nonresident)
{
    if (L < 0 || L > t->N) return -1;
    int g = t->G[L];
    if (bx < 0 || by < 0 || bz < 0 || bx >= g || by >= g || bz >= g) return -1;
    node_at(t, L, bx, by, bz)->nonresident = (int8_t)(nonresident != 0);
    return 0;
}

/* Per-node view for tests: state and flags of node (L, bx, by, bz); -1 state if absent. */
int orc_node_info(const orc_tree *t, int L, int bx, int by, int bz, int32_t *state,
                  int32_t *flags, double *avg)
{
    if (L < 0 || L > t->N) return -1;
    int g = t->G[L];
    if (bx < 0 || by < 0 || bz < 0 || bx >= g || by >= g || bz >= g) return -1;
    const orc_node *nd = node_at(t, L, bx, by, bz);
    *state = nd->exists ? nd->state : ST_NONE;
    *flags = (nd->has_children ? 1 : 0) | (nd->complete ? 2 : 0) | (nd->populated ? 4 : 0);
    for (int c = 0; c < t->p.channels; c++) avg[c] = nd->avg[c];
    return 0;
}

/* Replaces the level-0 value of voxel (x, y, z), channel c, in place, for finite differences
 * with respect to a voxel: valid only where level 0 is sampled as the data itself, i.e. when
 * the homogeneity threshold is 0 and the level-0 node holding the voxel is a brick.  Then
 * R_0 = V_0 there and a view at LOD 0 reads nothing else that depends on the voxel.  Upper
 * levels, node statistics and the dump keep describing the built volume, so afterwards the
 * tree refuses everything but LOD-0 renders and gradients (they return -1). */
int orc_poke_level0(orc_tree *t, int c, int x, int y, int z, double value)
{
    if (c < 0 || c >= t->p.channels || t->p.threshold != 0.0) return -1;
    if (x < 0 || y < 0 || z < 0 || x >= t->ext[0][0] || y >= t->ext[0][1] || z >= t->ext[0][2])
        return -1;
    const int M = t->p.brick;
    const orc_node *nd = node_at(t, 0, x / M, y / M, z / M);
    if (!nd->exists || nd->state != ST_BRICK) return -1;
    if (t->p.dtype == 0 ? !(value >= 0.0 && value <= 65535.0 && value == floor(value))
                        : (double)(float)value != value)
        return -1;   /* the data type must hold the replacement exactly */
    vset(t, 0, lvl_index(t, 0, c, z, y, x), value);
    t->poked = 1;
    return 0;
}
