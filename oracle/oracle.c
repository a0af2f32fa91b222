/*
 * CPU oracle for block-merged ray marching (City-on-Web, arXiv 2312.16457).
 *
 * TEST INFRASTRUCTURE ONLY -- see oracle.h.  Written for plain readability:
 * one ray at a time, every sample tested by its definition, no blocking,
 * no skipping structure beyond the occupancy bit the method itself defines.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off (no fast-math), so every float
 * operation below is one correctly rounded IEEE fp32 operation.
 */
#include "oracle.h"

#include <stdlib.h>
#include <string.h>
#include <tgmath.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NCH 8

/* Type of the continuous per-sample arithmetic (interpolation, decode,
 * activations, compositing).  double for the oracle.  A build with
 * -DORC_REAL=float exists only to time the same code in single precision
 * (the benchmark's CPU baseline); its decisions are the same fp32 ones.  The
 * MLP, the adjoint's sums and everything at the interface stay double. */
#ifndef ORC_REAL
#define ORC_REAL double
#endif
typedef ORC_REAL real;

/* ---------------------------------------------------------------------- */
/* Discrete decisions in exact fp32                                         */
/* ---------------------------------------------------------------------- */

/* Pixel ray r(t) = o + t d (Sec. 3): o is the eye; d is the normalised
 * camera-to-world rotation of the pixel-centre direction (x, y, 1). */
static void ray_dir(const orc_view* v, int i, int j, float d[3]) {
    float x = ((float)i + 0.5f - v->cx) / v->fx;
    float y = ((float)j + 0.5f - v->cy) / v->fy;
    float u[3];
    for (int c = 0; c < 3; ++c) {
        float a = v->R[3 * c + 0] * x;
        float b = v->R[3 * c + 1] * y;
        u[c] = (a + b) + v->R[3 * c + 2];
    }
    float n = sqrtf((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
    for (int c = 0; c < 3; ++c) d[c] = u[c] / n;
}

static void position(const float o[3], const float d[3], float t, float p[3]) {
    for (int c = 0; c < 3; ++c) {
        float td = t * d[c];
        p[c] = o[c] + td;
    }
}

static int inside(const float p[3], const float lo[3], const float hi[3]) {
    for (int c = 0; c < 3; ++c)
        if (!(lo[c] <= p[c] && p[c] < hi[c])) return 0;
    return 1;
}

/* slab intersection in fp32 with the closed box; t_near clamped at 0 */
static int slab32(const float o[3], const float d[3], const float lo[3], const float hi[3],
                  float* tn, float* tf) {
    float t0 = 0.0f, t1 = INFINITY;
    for (int c = 0; c < 3; ++c) {
        if (d[c] == 0.0f) {
            if (o[c] < lo[c] || o[c] > hi[c]) return 0;
            continue;
        }
        float inv = 1.0f / d[c];
        float a = (lo[c] - o[c]) * inv;
        float b = (hi[c] - o[c]) * inv;
        float mn = a < b ? a : b, mx = a < b ? b : a;
        if (mn > t0) t0 = mn;
        if (mx < t1) t1 = mx;
    }
    *tn = t0;
    *tf = t1;
    return t0 < t1;
}

/* Texels (or cells) along axis c of a block: the per-unit-length resolution
 * times the block's extent on that axis (a whole power of two). */
static int dim(const orc_block* b, int res, int c) { return res * (int)(b->hi[c] - b->lo[c]); }

/* Contraction of the implementation details (MERF's, in the max norm):
 * identity inside the unit cube; outside it a coordinate below the norm is
 * divided by the norm and the one(s) attaining it become (2 - 1/|x_j|)
 * sign(x_j), so all of space lands in the cube of radius 2.  The condition
 * "x_j equals the norm" is read on |x_j| (the sign factor shows negative
 * coordinates are meant too). */
void orc_contract(const double* x, double* y) {
    double m = 0.0;
    for (int c = 0; c < 3; ++c) m = fabs(x[c]) > m ? fabs(x[c]) : m;
    for (int c = 0; c < 3; ++c) {
        if (m <= 1.0)
            y[c] = x[c];
        else if (fabs(x[c]) == m)
            y[c] = (2.0 - 1.0 / fabs(x[c])) * (x[c] / fabs(x[c]));
        else
            y[c] = x[c] / m;
    }
}

/* fp32 decision sequence of the contraction for the box [lo, hi): the
 * box-normalised coordinate x = (p - centre) (2 / extent) is contracted and
 * mapped to texture space, q = (contract(x) + 2) (extent / 4), so the block's
 * texels cover the contracted cube and the box itself its middle half per
 * axis.  Returns max_c |x_c|. */
static float contract32(const float lo[3], const float hi[3], const float p[3], float q[3]) {
    float x[3], m = 0.0f;
    for (int c = 0; c < 3; ++c) {
        float ext = hi[c] - lo[c];
        float ctr = lo[c] + 0.5f * ext;
        x[c] = (p[c] - ctr) * (2.0f / ext);
        float a = fabsf(x[c]);
        if (a > m) m = a;
    }
    for (int c = 0; c < 3; ++c) {
        float y = x[c];
        if (m > 1.0f) y = fabsf(x[c]) == m ? copysignf(2.0f - 1.0f / m, x[c]) : x[c] / m;
        q[c] = (y + 2.0f) * (0.25f * (hi[c] - lo[c]));
    }
    return m;
}

/* local (texture-space) coordinate of a sample in block b: p - lo, or the
 * contracted coordinate for a contracted block */
float orc_local_q(const orc_block* b, const float* p, float* q) {
    if (b->contracted) return contract32(b->lo, b->hi, p, q);
    for (int c = 0; c < 3; ++c) q[c] = p[c] - b->lo[c];
    return 0.0f;
}

/* occupancy cell of a sample in block b (fp32 local coordinate) */
static int occ_cell(const orc_block* b, const float p[3], float q[3]) {
    int cell[3];
    orc_local_q(b, p, q);
    for (int c = 0; c < 3; ++c) {
        float s = q[c] * (float)b->O;
        int k = (int)floorf(s);
        if (k < 0) k = 0;
        if (k > dim(b, b->O, c) - 1) k = dim(b, b->O, c) - 1;
        cell[c] = k;
    }
    return (cell[2] * dim(b, b->O, 1) + cell[1]) * dim(b, b->O, 0) + cell[0];
}

/* ---------------------------------------------------------------------- */
/* Texture access                                                           */
/* ---------------------------------------------------------------------- */

static real texel(const orc_block* b, int tex, long idx, int ch) {
    if (b->dtype == ORC_U8) {
        const unsigned char* src = tex == 0 ? b->g8 : b->p8[tex - 1];
        return (real)src[idx * NCH + ch] * (real)b->scale[tex][ch] + (real)b->offset[tex][ch];
    }
    const double* src = tex == 0 ? b->gf : b->pf[tex - 1];
    return (real)src[idx * NCH + ch];
}

/* texel value as the fp32 decision sees it: fl(fl(q*s)+o), or the stored value */
static float texel32(const orc_block* b, int tex, long idx, int ch) {
    if (b->dtype == ORC_U8) {
        const unsigned char* src = tex == 0 ? b->g8 : b->p8[tex - 1];
        float m = (float)src[idx * NCH + ch] * b->scale[tex][ch];
        return m + b->offset[tex][ch];
    }
    const double* src = tex == 0 ? b->gf : b->pf[tex - 1];
    return (float)src[idx * NCH + ch];
}

static int clampi(int a, int lo, int hi) { return a < lo ? lo : (a > hi ? hi : a); }

/* cell-centred linear interpolation taps with clamp-to-edge: u = q*R - 1/2
 * for R texels per unit length, D texels along the axis */
static void lin_taps(real q, int R, int D, int idx[2], real w[2]) {
    real u = q * (real)R - (real)0.5;
    real f0 = floor(u);
    real f = u - f0;
    int a = (int)f0;
    idx[0] = clampi(a, 0, D - 1);
    idx[1] = clampi(a + 1, 0, D - 1);
    w[0] = (real)1 - f;
    w[1] = f;
}

typedef struct tap {
    int tex;
    long idx;
    double w;
} tap;

/* raw features = grid trilinear + three bilinear planes, summed ((G+XY)+XZ)+YZ.
 * taps (20 entries) receive the texel index and interpolation weight of each
 * texture sample, for the adjoint. */
static void eval_raw(const orc_block* b, const float q32[3], real raw[NCH], tap* taps) {
    real q[3] = {q32[0], q32[1], q32[2]};
    int gi[3][2], pi[3][2];
    real gw[3][2], pw[3][2];
    for (int c = 0; c < 3; ++c) {
        lin_taps(q[c], b->R, dim(b, b->R, c), gi[c], gw[c]);
        lin_taps(q[c], b->Rp, dim(b, b->Rp, c), pi[c], pw[c]);
    }
    real part[4][NCH];
    memset(part, 0, sizeof(part));
    int nt = 0;
    /* grid [z][y][x] */
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                long idx = ((long)gi[2][dz] * dim(b, b->R, 1) + gi[1][dy]) * dim(b, b->R, 0) + gi[0][dx];
                real w = gw[2][dz] * gw[1][dy] * gw[0][dx];
                for (int ch = 0; ch < NCH; ++ch) part[0][ch] += w * texel(b, 0, idx, ch);
                if (taps) taps[nt++] = (tap){0, idx, w};
            }
    /* planes: xy -> (x, y), xz -> (x, z), yz -> (y, z); index [v][u] */
    static const int axes[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int pl = 0; pl < 3; ++pl) {
        int au = axes[pl][0], av = axes[pl][1];
        for (int dv = 0; dv < 2; ++dv)
            for (int du = 0; du < 2; ++du) {
                long idx = (long)pi[av][dv] * dim(b, b->Rp, au) + pi[au][du];
                real w = pw[av][dv] * pw[au][du];
                for (int ch = 0; ch < NCH; ++ch) part[1 + pl][ch] += w * texel(b, 1 + pl, idx, ch);
                if (taps) taps[nt++] = (tap){1 + pl, idx, w};
            }
    }
    for (int ch = 0; ch < NCH; ++ch) raw[ch] = ((part[0][ch] + part[1][ch]) + part[2][ch]) + part[3][ch];
}

static real sigm(real x) { return (real)1 / ((real)1 + exp(-x)); }

/* ---------------------------------------------------------------------- */
/* Occupancy: conservative max-bound of the interpolated density           */
/* ---------------------------------------------------------------------- */

int orc_occupancy(const orc_block* b, unsigned char* out) {
    const float thresh = (float)log(0.01); /* density 0.01 in pre-activation units */
    int O = b->O, R = b->R, Rp = b->Rp;
    if (O <= 0 || R % O || Rp % O) return -1;
    int s = R / O, sp = Rp / O;
    int G[3], P[3], C[3];
    for (int a = 0; a < 3; ++a) {
        G[a] = dim(b, R, a);
        P[a] = dim(b, Rp, a);
        C[a] = dim(b, O, a);
    }
    /* cells are independent: split the z layers over threads */
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int cz = 0; cz < C[2]; ++cz)
        for (int cy = 0; cy < C[1]; ++cy)
            for (int cx = 0; cx < C[0]; ++cx) {
                int c3[3] = {cx, cy, cz};
                int glo[3], ghi[3], plo[3], phi[3];
                for (int a = 0; a < 3; ++a) {
                    glo[a] = clampi(c3[a] * s - 1, 0, G[a] - 1);
                    ghi[a] = clampi((c3[a] + 1) * s, 0, G[a] - 1);
                    plo[a] = clampi(c3[a] * sp - 1, 0, P[a] - 1);
                    phi[a] = clampi((c3[a] + 1) * sp, 0, P[a] - 1);
                }
                float mg = -INFINITY;
                for (int z = glo[2]; z <= ghi[2]; ++z)
                    for (int y = glo[1]; y <= ghi[1]; ++y)
                        for (int x = glo[0]; x <= ghi[0]; ++x) {
                            float v = texel32(b, 0, ((long)z * G[1] + y) * G[0] + x, 0);
                            if (v > mg) mg = v;
                        }
                static const int axes[3][2] = {{0, 1}, {0, 2}, {1, 2}};
                float mp[3];
                for (int pl = 0; pl < 3; ++pl) {
                    int au = axes[pl][0], av = axes[pl][1];
                    float m = -INFINITY;
                    for (int vv = plo[av]; vv <= phi[av]; ++vv)
                        for (int uu = plo[au]; uu <= phi[au]; ++uu) {
                            float val = texel32(b, 1 + pl, (long)vv * P[au] + uu, 0);
                            if (val > m) m = val;
                        }
                    mp[pl] = m;
                }
                float bound = ((mg + mp[0]) + mp[1]) + mp[2];
                out[(cz * C[1] + cy) * C[0] + cx] = bound > thresh ? 1 : 0;
            }
    return 0;
}

/* Height of a block's content (Appendix D, the z of the rectangle the viewer
 * tests): the top face of its highest occupied cell, the floor when empty.  A
 * contracted block's texture z is the contracted coordinate, not world z, and
 * the block owns space above its box: its box top. */
double orc_ztop(const orc_block* b, const unsigned char* occ) {
    if (b->contracted) return (double)b->hi[2];
    int nz = dim(b, b->O, 2), nxy = dim(b, b->O, 0) * dim(b, b->O, 1), top = -1;
    for (int z = 0; z < nz; ++z)
        for (int i = 0; i < nxy; ++i)
            if (occ[z * nxy + i]) top = z;
    double ext = (double)b->hi[2] - (double)b->lo[2];
    return (double)b->lo[2] + (double)(top + 1) / (double)nz * ext;
}

/* Level `level` of the multi-level occupancy grid psi (Sec. 3, rendering
 * stage, and Sec. 4.5 "Baking": the binary grid downsampled by max-pooling).
 * Level 0 is the grid itself.  Cell x of level l stands for the base cells i
 * with i_a >> l == x_a on every axis a, so the level has max(C_a >> l, 1)
 * cells along axis a (C_a the base count), and the cell is occupied iff one of
 * its base cells is. */
int orc_occupancy_level(const orc_block* b, const unsigned char* occ, int level, unsigned char* out) {
    if (level < 0 || level > 30) return -1;
    int C[3], L[3];
    for (int a = 0; a < 3; ++a) {
        C[a] = dim(b, b->O, a);
        L[a] = C[a] >> level;
        if (L[a] < 1) L[a] = 1;
    }
    memset(out, 0, (size_t)L[0] * L[1] * L[2]);
    for (int z = 0; z < C[2]; ++z)
        for (int y = 0; y < C[1]; ++y)
            for (int x = 0; x < C[0]; ++x)
                if (occ[((size_t)z * C[1] + y) * C[0] + x])
                    out[((size_t)(z >> level) * L[1] + (y >> level)) * L[0] + (x >> level)] = 1;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Sample enumeration                                                      */
/* ---------------------------------------------------------------------- */

typedef struct sample {
    int set_pos;   /* position in the view's set */
    long k;        /* global (mode 1) or per-block (mode 0) step index */
    float q[3];    /* fp32 local coordinate */
    double delta;
    int occupied;
} sample;

static int cmp_tin(const void* a, const void* b) {
    const double* x = (const double*)a;
    const double* y = (const double*)b;
    if (x[0] < y[0]) return -1;
    if (x[0] > y[0]) return 1;
    return x[1] < y[1] ? -1 : (x[1] > y[1]);
}

/* The ray's interval inside the footprint's column (x and y only; the
 * slab32 sequence on two axes, t clamped at 0). */
static int slab_xy(const float o[3], const float d[3], const float lo[3], const float hi[3], float* tn,
                   float* tf) {
    float t0 = 0.0f, t1 = INFINITY;
    for (int c = 0; c < 2; ++c) {
        if (d[c] == 0.0f) {
            if (o[c] < lo[c] || o[c] > hi[c]) return 0;
            continue;
        }
        float inv = 1.0f / d[c];
        float a = (lo[c] - o[c]) * inv;
        float b = (hi[c] - o[c]) * inv;
        float mn = a < b ? a : b, mx = a < b ? b : a;
        if (mn > t0) t0 = mn;
        if (mx < t1) t1 = mx;
    }
    *tn = t0;
    *tf = t1;
    return t0 < t1;
}

/* One exterior segment of a ray, [t_start, t_end), outside the footprint
 * [X0, X1) x [Y0, Y1) of the scene.  A point there belongs to the block
 * column nearest in the max norm (Eq. "blocks"); where several tie, to the
 * one the clamped unit cell names: (clamp(floor(x - X0)), clamp(floor(y - Y0))).
 * Steps are uniform in contracted space to first order: from t the next
 * sample lies ext_delta m^2 further, m = max(1, |x|_inf) of the point's
 * coordinate normalised to its owner cell (unit in x and y, the scene's
 * height in z), whose contraction has radial derivative 1/m^2.  The first
 * sample sits half a base step in; a sample is taken (listed) when its point
 * lies outside the footprint, its owner is a contracted block of the view's
 * set and m <= 1 / ext_delta; the post-exit segment (post = 1) ends at the
 * first point beyond that far limit, and every segment after ext_max_steps
 * steps. */
static long ext_phase(const orc_block* blocks, const unsigned char* const* occ, const int* set, int nset,
                      const orc_params* p, const float o[3], const float d[3], const float slo[3],
                      const float shi[3], float t_start, float t_end, int post, sample* out, long n, long cap) {
    const float nxm = (shi[0] - slo[0]) - 1.0f, nym = (shi[1] - slo[1]) - 1.0f;
    const float far = 1.0f / p->ext_delta;
    float t = t_start + 0.5f * p->ext_delta;
    float m_prev = INFINITY;
    for (int st = 0; st < p->ext_max_steps; ++st) {
        if (!post && !(t < t_end)) break;
        float pt[3];
        position(o, d, t, pt);
        float fx = floorf(pt[0] - slo[0]), fy = floorf(pt[1] - slo[1]);
        fx = fx < 0.0f ? 0.0f : (fx > nxm ? nxm : fx);
        fy = fy < 0.0f ? 0.0f : (fy > nym ? nym : fy);
        const float clo[3] = {slo[0] + fx, slo[1] + fy, slo[2]};
        const float chi[3] = {clo[0] + 1.0f, clo[1] + 1.0f, shi[2]};
        float q[3];
        float m = contract32(clo, chi, pt, q);
        if (m < 1.0f) m = 1.0f;
        const float w = (p->ext_delta * m) * m;
        /* beyond the far limit: the segment after the column ends there; the
         * one before it ends once m grows past it (m is convex along a ray
         * outside the column, so it never comes back) */
        const int rising = m > m_prev;
        m_prev = m;
        if (m > far) {
            if (post || rising) break;
        } else if (!(slo[0] <= pt[0] && pt[0] < shi[0] && slo[1] <= pt[1] && pt[1] < shi[1])) {
            int s_hit = -1;
            for (int s = 0; s < nset; ++s) {
                const orc_block* b = &blocks[set[s]];
                if (b->contracted && b->lo[0] == clo[0] && b->lo[1] == clo[1]) {
                    s_hit = s;
                    break;
                }
            }
            if (s_hit >= 0 && n < cap) {
                sample* sm = &out[n++];
                sm->set_pos = s_hit;
                sm->k = -1;
                sm->delta = w;
                int cell = occ_cell(&blocks[set[s_hit]], pt, sm->q);
                sm->occupied = occ[set[s_hit]][cell] != 0;
            }
        }
        t = t + w;
    }
    return n;
}

/* Samples of one exterior segment of a ray, for tests: texture-space
 * coordinates (3 per sample) and step lengths, at most cap. */
long orc_ext_samples(const orc_block* blocks, int nblocks, const unsigned char* const* occ, const int* set,
                     int nset, const orc_params* p, const float* o, const float* d, float t_start, float t_end,
                     int post, float* q_out, double* delta_out, long cap) {
    float slo[3] = {INFINITY, INFINITY, INFINITY}, shi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < nblocks; ++b)
        for (int c = 0; c < 3; ++c) {
            if (blocks[b].lo[c] < slo[c]) slo[c] = blocks[b].lo[c];
            if (blocks[b].hi[c] > shi[c]) shi[c] = blocks[b].hi[c];
        }
    sample* buf = (sample*)malloc(sizeof(sample) * (cap > 0 ? cap : 1));
    long n = ext_phase(blocks, occ, set, nset, p, o, d, slo, shi, t_start, t_end, post, buf, 0, cap);
    for (long i = 0; i < n; ++i) {
        for (int c = 0; c < 3; ++c) q_out[3 * i + c] = buf[i].q[c];
        delta_out[i] = buf[i].delta;
    }
    free(buf);
    return n;
}

/* Enumerate the samples of one ray in compositing order (front to back).
 * Returns the number written (<= cap).  Empty samples (no block in the set,
 * or outside every block) are not listed; unoccupied ones are, with
 * occupied = 0. */
static long enumerate(const orc_block* blocks, int nblocks, const unsigned char* const* occ,
                      const orc_view* v, const int* set, int nset, const orc_params* p,
                      int i, int j, sample* out, long cap, float dir[3]) {
    float d[3];
    ray_dir(v, i, j, d);
    if (dir) memcpy(dir, d, sizeof(d));
    const float* o = v->eye;
    long n = 0;
    if (p->mode == 0) {
        /* per-block chord, n_steps midpoints; blocks in order of entry t */
        double* ord = (double*)malloc(sizeof(double) * 4 * (nset > 0 ? nset : 1));
        int nh = 0;
        for (int s = 0; s < nset; ++s) {
            const orc_block* b = &blocks[set[s]];
            float tn, tf;
            if (!slab32(o, d, b->lo, b->hi, &tn, &tf)) continue;
            ord[4 * nh + 0] = tn;
            ord[4 * nh + 1] = b->block_id;
            ord[4 * nh + 2] = s;
            ord[4 * nh + 3] = tf;
            ++nh;
        }
        qsort(ord, nh, sizeof(double) * 4, cmp_tin);
        for (int h = 0; h < nh; ++h) {
            int s = (int)ord[4 * h + 2];
            const orc_block* b = &blocks[set[s]];
            float tn = (float)ord[4 * h + 0], tf = (float)ord[4 * h + 3];
            float dr = (tf - tn) / (float)p->n_steps;
            for (int k = 0; k < p->n_steps; ++k) {
                float t = tn + ((float)k + 0.5f) * dr;
                float pt[3];
                position(o, d, t, pt);
                if (!inside(pt, b->lo, b->hi)) continue;
                if (n >= cap) break;
                sample* sm = &out[n++];
                sm->set_pos = s;
                sm->k = k;
                sm->delta = dr;
                int cell = occ_cell(b, pt, sm->q);
                sm->occupied = occ[set[s]][cell] != 0;
            }
        }
        free(ord);
        return n;
    }
    /* mode 1: camera-anchored grid t_k = (k + 1/2) delta; window of max_steps
     * steps from the first sample inside the scene box */
    float slo[3] = {INFINITY, INFINITY, INFINITY}, shi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < nblocks; ++b)
        for (int c = 0; c < 3; ++c) {
            if (blocks[b].lo[c] < slo[c]) slo[c] = blocks[b].lo[c];
            if (blocks[b].hi[c] > shi[c]) shi[c] = blocks[b].hi[c];
        }
    /* exterior of the footprint (contracted boundary blocks): the part of the
     * ray before it enters the footprint's column, then, after the blocks,
     * the part after it leaves it */
    int ext = 0;
    if (p->ext_delta > 0.0f && p->ext_max_steps > 0)
        for (int s = 0; s < nset; ++s) ext |= blocks[set[s]].contracted;
    float fin = INFINITY, fout = INFINITY;
    if (ext) {
        if (!slab_xy(o, d, slo, shi, &fin, &fout)) fin = fout = INFINITY;
        n = ext_phase(blocks, occ, set, nset, p, o, d, slo, shi, 0.0f, fin, 0, out, n, cap);
    }
    long k_end = -1; /* end of the window of max_steps steps, when the ray enters the box */
    do {
        /* scan bound from an fp64 slab test of the box grown by 1e-3 */
        double tfar = INFINITY, tnear = 0.0;
        int miss = 0;
        for (int c = 0; c < 3; ++c) {
            double lo = (double)slo[c] - 1e-3, hi = (double)shi[c] + 1e-3, oc = o[c], dc = d[c];
            if (dc == 0.0) {
                if (oc < lo || oc > hi) miss = 1;
                continue;
            }
            double a = (lo - oc) / dc, bb = (hi - oc) / dc;
            double mn = a < bb ? a : bb, mx = a < bb ? bb : a;
            if (mn > tnear) tnear = mn;
            if (mx < tfar) tfar = mx;
        }
        if (miss || !(tnear <= tfar)) break;
        long kmax = (long)ceil(tfar / (double)p->delta) + 8;
        long k0 = -1;
        for (long k = 0; k <= kmax; ++k) {
            float t = ((float)k + 0.5f) * p->delta;
            float pt[3];
            position(o, d, t, pt);
            if (inside(pt, slo, shi)) {
                k0 = k;
                break;
            }
        }
        if (k0 < 0) break;
        k_end = k0 + p->max_steps;
        for (long k = k0; k < k0 + p->max_steps; ++k) {
            float t = ((float)k + 0.5f) * p->delta;
            float pt[3];
            position(o, d, t, pt);
            int s_hit = -1;
            for (int s = 0; s < nset; ++s)
                if (inside(pt, blocks[set[s]].lo, blocks[set[s]].hi)) {
                    s_hit = s;
                    break;
                }
            if (s_hit < 0) continue;
            if (n >= cap) break;
            sample* sm = &out[n++];
            sm->set_pos = s_hit;
            sm->k = k;
            sm->delta = p->delta;
            int cell = occ_cell(&blocks[set[s_hit]], pt, sm->q);
            sm->occupied = occ[set[s_hit]][cell] != 0;
        }
    } while (0);
    /* the cap truncates the ray: when the window ends before the ray leaves
     * the column, nothing behind it (the exterior beyond the column included)
     * is sampled */
    const int capped = k_end >= 0 && ((float)k_end + 0.5f) * p->delta < fout;
    if (ext && fout < INFINITY && !capped)
        n = ext_phase(blocks, occ, set, nset, p, o, d, slo, shi, fout, INFINITY, 1, out, n, cap);
    return n;
}

static long sample_cap(const orc_params* p, int nset) {
    if (p->mode == 0) return (long)p->n_steps * (nset > 0 ? nset : 1);
    return (long)p->max_steps + (p->ext_delta > 0.0f && p->ext_max_steps > 0 ? 2L * p->ext_max_steps : 0L);
}

/* ---------------------------------------------------------------------- */
/* Deferred MLP (Eq. "deferred")                                            */
/* ---------------------------------------------------------------------- */

/* Input of the deferred MLP (Eq. deferred): [C_d, F, PE(d)], with PE(d) =
 * [d, sin(2^0 d), cos(2^0 d), ..., sin(2^(L-1) d), cos(2^(L-1) d)] taken per
 * component (L = 0: the direction alone).  10 + 6L inputs. */
#define MLP_MAX_IN 34

int orc_posenc(const double* d, int L, double* out) {
    if (L < 0 || L > 4) return -1;
    for (int c = 0; c < 3; ++c) out[c] = d[c];
    for (int l = 0; l < L; ++l) {
        const double f = ldexp(1.0, l);
        for (int c = 0; c < 3; ++c) {
            out[3 + 6 * l + c] = sin(f * d[c]);
            out[6 + 6 * l + c] = cos(f * d[c]);
        }
    }
    return 3 + 6 * L;
}

static int mlp_input(const double A[7], const float d[3], int L, double* x) {
    const double dd[3] = {d[0], d[1], d[2]};
    for (int c = 0; c < 7; ++c) x[c] = A[c];
    return 7 + orc_posenc(dd, L, x + 7);
}

/* parameter layout: W1 [16][ni], b1 [16], W2 [16][16], b2 [16], W3 [3][16], b3 [3] */
typedef struct mlp_shape {
    int ni;
    long W1, b1, W2, b2, W3, b3, n;
} mlp_shape;

static mlp_shape mlp_shape_of(int L) {
    mlp_shape s;
    s.ni = 10 + 6 * L;
    s.W1 = 0;
    s.b1 = 16L * s.ni;
    s.W2 = s.b1 + 16;
    s.b2 = s.W2 + 256;
    s.W3 = s.b2 + 16;
    s.b3 = s.W3 + 48;
    s.n = s.b3 + 3;
    return s;
}

long orc_mlp_params(int L) { return mlp_shape_of(L).n; }

typedef struct mlp_trace {
    double x[MLP_MAX_IN], pre1[16], h1[16], pre2[16], h2[16], z[3], s[3];
} mlp_trace;

static void mlp_fwd(const double* w, const mlp_shape* sh, const double* x, mlp_trace* tr) {
    const int ni = sh->ni;
    const double *W1 = w + sh->W1, *b1 = w + sh->b1, *W2 = w + sh->W2, *b2 = w + sh->b2, *W3 = w + sh->W3,
                 *b3 = w + sh->b3;
    memcpy(tr->x, x, sizeof(double) * ni);
    for (int o = 0; o < 16; ++o) {
        double a = b1[o];
        for (int i = 0; i < ni; ++i) a += W1[o * ni + i] * x[i];
        tr->pre1[o] = a;
        tr->h1[o] = a > 0.0 ? a : 0.0;
    }
    for (int o = 0; o < 16; ++o) {
        double a = b2[o];
        for (int i = 0; i < 16; ++i) a += W2[o * 16 + i] * tr->h1[i];
        tr->pre2[o] = a;
        tr->h2[o] = a > 0.0 ? a : 0.0;
    }
    for (int o = 0; o < 3; ++o) {
        double a = b3[o];
        for (int i = 0; i < 16; ++i) a += W3[o * 16 + i] * tr->h2[i];
        tr->z[o] = a;
        tr->s[o] = sigm(a);
    }
}

void orc_field(const orc_block* b, int n, const float* pts, double* raw) {
    for (int k = 0; k < n; ++k) {
        float q[3];
        for (int c = 0; c < 3; ++c) q[c] = pts[3 * k + c] - b->lo[c];
        real r8[NCH];
        eval_raw(b, q, r8, NULL);
        for (int ch = 0; ch < NCH; ++ch) raw[NCH * k + ch] = r8[ch];
    }
}

void orc_mlp(const double* mlp, const double* x, double* out) {
    orc_mlp_pe(mlp, 0, x, out);
}

int orc_mlp_pe(const double* mlp, int L, const double* x, double* out) {
    if (L < 0 || L > 4) return -1;
    const mlp_shape sh = mlp_shape_of(L);
    mlp_trace tr;
    mlp_fwd(mlp, &sh, x, &tr);
    for (int c = 0; c < 3; ++c) out[c] = tr.s[c];
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Rendering                                                               */
/* ---------------------------------------------------------------------- */

typedef struct pt_val {
    real sigma, v[7];
} pt_val;

static void shade(const orc_block* b, const float q[3], pt_val* pv, real raw[NCH], tap* taps) {
    eval_raw(b, q, raw, taps);
    pv->sigma = exp(raw[0]);
    for (int c = 0; c < 7; ++c) pv->v[c] = sigm(raw[1 + c]);
}

static void render_one(const orc_block* blocks, int nblocks, const unsigned char* const* occ,
                       const orc_view* v, const int* set, int nset, const orc_params* p,
                       const double* mlp, int i, int j, int composite, sample* buf, long cap,
                       double rgb[3], double* trans, double aux[8], long long* ne,
                       long long* nm, int* ook) {
    float d[3];
    long n = enumerate(blocks, nblocks, occ, v, set, nset, p, i, j, buf, cap, d);
    /* block runs in ray order */
    int* run_pos = (int*)malloc(sizeof(int) * (n + 1));
    int nrun = 0, ordered = 1;
    long long eval = 0;
    for (long s = 0; s < n; ++s) {
        if (s == 0 || buf[s].set_pos != buf[s - 1].set_pos) {
            for (int r = 0; r < nrun; ++r)
                if (run_pos[r] == buf[s].set_pos) ordered = 0; /* block re-entered */
            if (nrun > 0 && buf[s].set_pos < run_pos[nrun - 1]) ordered = 0;
            run_pos[nrun++] = buf[s].set_pos;
        }
        eval += buf[s].occupied;
    }
    /* early ray termination: the ray stops after the first evaluated sample
     * at which its transmittance falls below t_min (applied in ray order, so
     * to the monolithic and the merged composite alike) */
    const double t_min = p->t_min;
    long n_used = n; /* samples up to and including the terminating one */
    real A[7] = {0}, T = 1;
    if (composite == ORC_MONOLITHIC) {
        eval = 0;
        for (long s = 0; s < n; ++s) {
            if (!buf[s].occupied) continue;
            pt_val pv;
            real raw[NCH];
            shade(&blocks[set[buf[s].set_pos]], buf[s].q, &pv, raw, NULL);
            real sd = pv.sigma * (real)buf[s].delta;
            real alpha = -expm1(-sd);
            real w = T * alpha;
            for (int c = 0; c < 7; ++c) A[c] += w * pv.v[c];
            T *= exp(-sd);
            ++eval;
            if (t_min > 0.0 && T < t_min) {
                n_used = s + 1;
                break;
            }
        }
    } else if (composite == ORC_MERGED || composite == ORC_BLOCK_MLP) {
        /* per-block composite (Eq. "volume rendering inside blocks"), merged
         * front to back in ray order (Eq. "volume rendering across blocks")
         * with the block transmittance carried as the product of (1 - alpha_i).
         * ORC_BLOCK_MLP shades each block with its own deferred MLP first and
         * merges the colours C^k instead of (C_d^k, F^k) */
        eval = 0;
        long s = 0;
        int stop = 0;
        double Cb[3] = {0, 0, 0};
        while (s < n && !stop) {
            const int run = buf[s].set_pos;
            real Ak[7] = {0}, Tk = 1;
            for (; s < n && buf[s].set_pos == run; ++s) {
                if (!buf[s].occupied) continue;
                pt_val pv;
                real raw[NCH];
                shade(&blocks[set[run]], buf[s].q, &pv, raw, NULL);
                real sd = pv.sigma * (real)buf[s].delta;
                real alpha = -expm1(-sd);
                real w = Tk * alpha;
                for (int c = 0; c < 7; ++c) Ak[c] += w * pv.v[c];
                Tk *= exp(-sd);
                ++eval;
                if (t_min > 0.0 && T * Tk < t_min) {
                    n_used = s + 1;
                    stop = 1;
                    break;
                }
            }
            if (composite == ORC_BLOCK_MLP) {
                const mlp_shape sh = mlp_shape_of(p->pe);
                double x[MLP_MAX_IN], Ak64[7];
                for (int c = 0; c < 7; ++c) Ak64[c] = Ak[c];
                mlp_input(Ak64, d, p->pe, x);
                mlp_trace tr;
                mlp_fwd(mlp + sh.n * (long)set[run], &sh, x, &tr);
                for (int c = 0; c < 3; ++c) Cb[c] += T * (Ak[c] + tr.s[c]);
            }
            for (int c = 0; c < 7; ++c) A[c] += T * Ak[c];
            T *= Tk;
        }
        if (composite == ORC_BLOCK_MLP) {
            free(run_pos);
            for (int c = 0; c < 3; ++c) rgb[c] = Cb[c];
            *trans = T;
            for (int c = 0; c < 8; ++c) aux[c] = 0.0;
            for (int c = 0; c < 3; ++c) aux[c] = Cb[c];
            aux[7] = T;
            *ne = eval;
            *nm = n_used;
            *ook = ordered;
            return;
        }
    } else {
        /* negative controls: per-block composites combined some other way */
        double* Ak = (double*)calloc((size_t)(nrun + 1) * 8, sizeof(double));
        int r = -1;
        for (long s = 0; s < n; ++s) {
            if (s == 0 || buf[s].set_pos != buf[s - 1].set_pos) {
                ++r;
                Ak[r * 8 + 7] = 1.0;
            }
            if (!buf[s].occupied) continue;
            pt_val pv;
            real raw[NCH];
            shade(&blocks[set[buf[s].set_pos]], buf[s].q, &pv, raw, NULL);
            double sd = pv.sigma * buf[s].delta;
            double alpha = -expm1(-sd);
            double w = Ak[r * 8 + 7] * alpha;
            for (int c = 0; c < 7; ++c) Ak[r * 8 + c] += w * pv.v[c];
            Ak[r * 8 + 7] *= exp(-sd);
        }
        if (composite == ORC_ALPHA_NORM) {
            double asum = 0.0;
            for (int q = 0; q < nrun; ++q) asum += 1.0 - Ak[q * 8 + 7];
            for (int q = 0; q < nrun; ++q) {
                double wgt = asum > 0.0 ? (1.0 - Ak[q * 8 + 7]) / asum : 0.0;
                for (int c = 0; c < 7; ++c) A[c] += wgt * Ak[q * 8 + c];
                T *= Ak[q * 8 + 7];
            }
        } else {
            int* ordr = (int*)malloc(sizeof(int) * (nrun + 1));
            for (int q = 0; q < nrun; ++q) ordr[q] = composite == ORC_REVERSED ? nrun - 1 - q : q;
            if (composite == ORC_BY_ID) /* insertion sort of runs by block id */
                for (int a = 1; a < nrun; ++a)
                    for (int b = a; b > 0; --b) {
                        int ia = blocks[set[run_pos[ordr[b]]]].block_id;
                        int ib = blocks[set[run_pos[ordr[b - 1]]]].block_id;
                        if (ia < ib) {
                            int t = ordr[b];
                            ordr[b] = ordr[b - 1];
                            ordr[b - 1] = t;
                        }
                    }
            for (int q = 0; q < nrun; ++q) {
                int rr = ordr[q];
                for (int c = 0; c < 7; ++c) A[c] += T * Ak[rr * 8 + c];
                T *= Ak[rr * 8 + 7];
            }
            free(ordr);
        }
        free(Ak);
    }
    free(run_pos);
    const mlp_shape sh = mlp_shape_of(p->pe);
    double x[MLP_MAX_IN], A64[7];
    for (int c = 0; c < 7; ++c) A64[c] = A[c];
    mlp_input(A64, d, p->pe, x);
    mlp_trace tr;
    mlp_fwd(mlp, &sh, x, &tr);
    for (int c = 0; c < 3; ++c) rgb[c] = A[c] + tr.s[c];
    *trans = T;
    for (int c = 0; c < 7; ++c) aux[c] = A[c];
    aux[7] = T;
    *ne = eval;
    *nm = n_used;
    *ook = ordered;
}

/* Contracted blocks are boundary columns: one unit in x and y, the scene's
 * full height in z (the exterior's owner cells have that shape). */
static int contracted_ok(const orc_block* blocks, int nblocks, const orc_params* p) {
    if (!(p->ext_delta >= 0.0f && p->ext_delta < INFINITY) || p->ext_max_steps < 0) return 0;
    float zlo = INFINITY, zhi = -INFINITY;
    for (int b = 0; b < nblocks; ++b) {
        if (blocks[b].lo[2] < zlo) zlo = blocks[b].lo[2];
        if (blocks[b].hi[2] > zhi) zhi = blocks[b].hi[2];
    }
    for (int b = 0; b < nblocks; ++b) {
        const orc_block* k = &blocks[b];
        if (k->contracted && (k->hi[0] - k->lo[0] != 1.0f || k->hi[1] - k->lo[1] != 1.0f || k->lo[2] != zlo ||
                              k->hi[2] != zhi))
            return 0;
    }
    return 1;
}

int orc_render(const orc_block* blocks, int nblocks, const unsigned char* const* occ,
               const orc_view* v, const int* set, int nset, const orc_params* p,
               const double* mlp, const int* pix, int npix, int composite,
               double* rgb, double* trans, double* aux, long long* n_eval,
               long long* n_march, int* order_ok, int nthreads) {
    if (p->pe < 0 || p->pe > 4) return -1;
    if (!contracted_ok(blocks, nblocks, p)) return -1;
    long cap = sample_cap(p, nset);
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
#endif
    {
        sample* buf = (sample*)malloc(sizeof(sample) * cap);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
        for (int q = 0; q < npix; ++q) {
            double c3[3], t, a8[8];
            long long ne, nm;
            int ok;
            render_one(blocks, nblocks, occ, v, set, nset, p, mlp, pix[2 * q], pix[2 * q + 1],
                       composite, buf, cap, c3, &t, a8, &ne, &nm, &ok);
            if (rgb) memcpy(rgb + 3 * q, c3, sizeof(c3));
            if (trans) trans[q] = t;
            if (aux) memcpy(aux + 8 * q, a8, sizeof(a8));
            if (n_eval) n_eval[q] = ne;
            if (n_march) n_march[q] = nm;
            if (order_ok) order_ok[q] = ok;
        }
        free(buf);
    }
    (void)nthreads;
    return 0;
}

/* Texels the evaluated samples of the given pixels read (the compulsory
 * texture bytes of a frame, Sec. 4.5 "Baking": the textures a renderer must
 * fetch at least once): for every sample in an occupied cell, the eight grid
 * taps and four taps per plane of the interpolation (clamped indices, as in
 * eval_raw), marked with 1 in marks[4 e + t] (e the entry in `blocks`, t =
 * 0 grid, 1-3 the xy, xz, yz planes; byte arrays of the textures' texel
 * counts, NULL to skip).  Without early termination only (t_min = 0): the
 * samples a terminated ray skips depend on its shading.  Returns 0, or -1
 * for t_min > 0 or contracted blocks. */
static void mark_taps(const orc_block* b, const float q32[3], unsigned char* const* mk) {
    int gi[3][2], pi[3][2];
    real gw[3][2], pw[3][2];
    for (int c = 0; c < 3; ++c) {
        lin_taps((real)q32[c], b->R, dim(b, b->R, c), gi[c], gw[c]);
        lin_taps((real)q32[c], b->Rp, dim(b, b->Rp, c), pi[c], pw[c]);
    }
    if (mk[0])
        for (int dz = 0; dz < 2; ++dz)
            for (int dy = 0; dy < 2; ++dy)
                for (int dx = 0; dx < 2; ++dx) {
                    long idx = ((long)gi[2][dz] * dim(b, b->R, 1) + gi[1][dy]) * dim(b, b->R, 0) + gi[0][dx];
#ifdef _OPENMP
#pragma omp atomic write
#endif
                    mk[0][idx] = 1;
                }
    static const int axes[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    for (int pl = 0; pl < 3; ++pl) {
        if (!mk[1 + pl]) continue;
        int au = axes[pl][0], av = axes[pl][1];
        for (int dv = 0; dv < 2; ++dv)
            for (int du = 0; du < 2; ++du) {
                long idx = (long)pi[av][dv] * dim(b, b->Rp, au) + pi[au][du];
#ifdef _OPENMP
#pragma omp atomic write
#endif
                mk[1 + pl][idx] = 1;
            }
    }
}

int orc_touched_texels(const orc_block* blocks, int nblocks, const unsigned char* const* occ, const orc_view* v,
                       const int* set, int nset, const orc_params* p, const int* pix, long npix,
                       unsigned char* const* marks, int nthreads) {
    if (p->t_min > 0.0f) return -1;
    for (int s = 0; s < nset; ++s)
        if (blocks[set[s]].contracted) return -1;
    long cap = sample_cap(p, nset);
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads)
#endif
    {
        sample* buf = (sample*)malloc(sizeof(sample) * cap);
#ifdef _OPENMP
#pragma omp for schedule(dynamic, 64)
#endif
        for (long q = 0; q < npix; ++q) {
            long n = enumerate(blocks, nblocks, occ, v, set, nset, p, pix[2 * q], pix[2 * q + 1], buf, cap, NULL);
            for (long k = 0; k < n; ++k) {
                if (!buf[k].occupied) continue;
                int e = set[buf[k].set_pos];
                mark_taps(&blocks[e], buf[k].q, marks + 4 * e);
            }
        }
        free(buf);
    }
    (void)nthreads;
    return 0;
}

int orc_ray_blocks(const orc_block* blocks, int nblocks, const orc_view* v, const int* set,
                   int nset, const orc_params* p, int i, int j, int* out, int cap) {
    /* occupancy is irrelevant for the order: use an all-occupied mask */
    unsigned char one = 1;
    const unsigned char** occ = (const unsigned char**)malloc(sizeof(void*) * nblocks);
    unsigned char** full = (unsigned char**)malloc(sizeof(void*) * nblocks);
    for (int b = 0; b < nblocks; ++b) {
        long o3 = (long)dim(&blocks[b], blocks[b].O, 0) * dim(&blocks[b], blocks[b].O, 1) * dim(&blocks[b], blocks[b].O, 2);
        full[b] = (unsigned char*)malloc(o3);
        memset(full[b], one, o3);
        occ[b] = full[b];
    }
    long cap_s = sample_cap(p, nset);
    sample* buf = (sample*)malloc(sizeof(sample) * cap_s);
    long n = enumerate(blocks, nblocks, occ, v, set, nset, p, i, j, buf, cap_s, NULL);
    int m = 0;
    for (long s = 0; s < n; ++s)
        if ((s == 0 || buf[s].set_pos != buf[s - 1].set_pos) && m < cap) out[m++] = set[buf[s].set_pos];
    free(buf);
    for (int b = 0; b < nblocks; ++b) free(full[b]);
    free(full);
    free(occ);
    return m;
}

/* ---------------------------------------------------------------------- */
/* Adjoint (fp64)                                                          */
/* ---------------------------------------------------------------------- */

/* entropy of a block's opacity and its derivative in the opacity */
static const double OPAC_EPS = 1e-6;
static double opac_h(double alpha) {
    double a = alpha < OPAC_EPS ? OPAC_EPS : (alpha > 1.0 - OPAC_EPS ? 1.0 - OPAC_EPS : alpha);
    return -(a * log(a) + (1.0 - a) * log(1.0 - a));
}
static double opac_dh(double alpha) {
    if (!(alpha > OPAC_EPS && alpha < 1.0 - OPAC_EPS)) return 0.0; /* clamped */
    return log((1.0 - alpha) / alpha);
}

int orc_adjoint(const orc_block* blocks, int nblocks, const unsigned char* const* occ,
                const orc_view* v, const int* set, int nset, const orc_params* p,
                const double* mlp, const int* pix, int npix, const double* grad_rgb,
                const double* grad_trans, const double* w_opacity, double* const* grad_grid,
                double* const* grad_plane, double* grad_mlp) {
    int any_ct = 0;
    for (int s = 0; s < nset; ++s) {
        if (blocks[set[s]].dtype != ORC_F64) return -1;
        any_ct |= blocks[set[s]].contracted;
    }
    if (p->pe < 0 || p->pe > 4) return -1;
    /* contracted blocks: the samples are those of the forward (the exterior
     * segments in ray order around the blocks, each with its own step), so
     * the single-chain adjoint below applies unchanged; the opacity term is
     * defined per block run and an exterior segment splits a block's run,
     * so it is not taken with them */
    if (!contracted_ok(blocks, nblocks, p)) return -1;
    if (any_ct && w_opacity) return -1;
    long cap = sample_cap(p, nset);
    sample* buf = (sample*)malloc(sizeof(sample) * cap);
    pt_val* pv = (pt_val*)malloc(sizeof(pt_val) * cap);
    tap* taps = (tap*)malloc(sizeof(tap) * 20 * cap);
    double* wts = (double*)malloc(sizeof(double) * cap);
    double* Tb = (double*)malloc(sizeof(double) * (cap + 1));
    double* suf = (double*)malloc(sizeof(double) * 7 * (cap + 1));
    long* ev = (long*)malloc(sizeof(long) * cap);
    const mlp_shape sh = mlp_shape_of(p->pe);
    const double *W1 = mlp + sh.W1, *W2 = mlp + sh.W2, *W3 = mlp + sh.W3;
    for (int q = 0; q < npix; ++q) {
        float d[3];
        long n = enumerate(blocks, nblocks, occ, v, set, nset, p, pix[2 * q], pix[2 * q + 1], buf,
                           cap, d);
        /* forward over the monolithic sequence (equal to the merged one) */
        long m = 0;
        double T = 1.0, A[7] = {0};
        for (long s = 0; s < n; ++s) {
            if (!buf[s].occupied) continue;
            real raw[NCH];
            shade(&blocks[set[buf[s].set_pos]], buf[s].q, &pv[m], raw, &taps[20 * m]);
            double sd = pv[m].sigma * buf[s].delta;
            double alpha = -expm1(-sd);
            Tb[m] = T;
            wts[m] = T * alpha;
            for (int c = 0; c < 7; ++c) A[c] += wts[m] * pv[m].v[c];
            T *= exp(-sd);
            ev[m] = s;
            ++m;
            if (p->t_min > 0.0f && T < (double)p->t_min) break; /* early termination */
        }
        Tb[m] = T;
        /* opacity term: per block (run) T^k over its evaluated samples;
         * d/dsigma_i of -h(1 - T^k) weight = w dh/dalpha delta_i T^k */
        double* opg = (double*)calloc((size_t)(m + 1), sizeof(double));
        if (w_opacity && w_opacity[q] != 0.0) {
            long s0 = 0;
            while (s0 < m) {
                long s1 = s0;
                int run = buf[ev[s0]].set_pos;
                double Tk = 1.0;
                while (s1 < m && buf[ev[s1]].set_pos == run) {
                    Tk *= exp(-pv[s1].sigma * buf[ev[s1]].delta);
                    ++s1;
                }
                double g = w_opacity[q] * opac_dh(1.0 - Tk);
                for (long s = s0; s < s1; ++s) opg[s] = g * buf[ev[s]].delta * Tk;
                s0 = s1;
            }
        }
        /* suffix sums S_i = sum_{j>i} w_j v_j */
        for (int c = 0; c < 7; ++c) suf[7 * m + c] = 0.0;
        if (m > 0)
            for (int c = 0; c < 7; ++c) suf[7 * (m - 1) + c] = 0.0;
        for (long s = m - 2; s >= 0; --s)
            for (int c = 0; c < 7; ++c) suf[7 * s + c] = suf[7 * (s + 1) + c] + wts[s + 1] * pv[s + 1].v[c];
        /* MLP backward */
        double x[MLP_MAX_IN];
        mlp_input(A, d, p->pe, x);
        mlp_trace tr;
        mlp_fwd(mlp, &sh, x, &tr);
        const double* g = grad_rgb + 3 * q;
        double dz[3], dh2[16], dh1[16], dx[7];
        for (int o = 0; o < 3; ++o) dz[o] = g[o] * tr.s[o] * (1.0 - tr.s[o]);
        for (int i = 0; i < 16; ++i) {
            double a = 0.0;
            for (int o = 0; o < 3; ++o) a += W3[o * 16 + i] * dz[o];
            dh2[i] = tr.pre2[i] > 0.0 ? a : 0.0;
        }
        for (int i = 0; i < 16; ++i) {
            double a = 0.0;
            for (int o = 0; o < 16; ++o) a += W2[o * 16 + i] * dh2[o];
            dh1[i] = tr.pre1[i] > 0.0 ? a : 0.0;
        }
        for (int i = 0; i < 7; ++i) { /* the direction inputs are constants */
            double a = 0.0;
            for (int o = 0; o < 16; ++o) a += W1[o * sh.ni + i] * dh1[o];
            dx[i] = a;
        }
        if (grad_mlp) {
            for (int o = 0; o < 16; ++o) {
                for (int i = 0; i < sh.ni; ++i) grad_mlp[sh.W1 + o * sh.ni + i] += dh1[o] * tr.x[i];
                grad_mlp[sh.b1 + o] += dh1[o];
                for (int i = 0; i < 16; ++i) grad_mlp[sh.W2 + o * 16 + i] += dh2[o] * tr.h1[i];
                grad_mlp[sh.b2 + o] += dh2[o];
            }
            for (int o = 0; o < 3; ++o) {
                for (int i = 0; i < 16; ++i) grad_mlp[sh.W3 + o * 16 + i] += dz[o] * tr.h2[i];
                grad_mlp[sh.b3 + o] += dz[o];
            }
        }
        double u[7];
        for (int c = 0; c < 7; ++c) u[c] = dx[c] + (c < 3 ? g[c] : 0.0);
        double gT = grad_trans ? grad_trans[q] : 0.0;
        /* per-sample adjoint */
        for (long s = 0; s < m; ++s) {
            const sample* sm = &buf[ev[s]];
            double delta = sm->delta;
            double uv = 0.0, us = 0.0;
            for (int c = 0; c < 7; ++c) {
                uv += u[c] * pv[s].v[c];
                us += u[c] * suf[7 * s + c];
            }
            double dsig = delta * (Tb[s + 1] * uv - us) - delta * T * gT + opg[s];
            double draw[NCH];
            draw[0] = pv[s].sigma * dsig;
            for (int c = 0; c < 7; ++c) {
                double sv = pv[s].v[c];
                draw[1 + c] = wts[s] * u[c] * sv * (1.0 - sv);
            }
            int b = set[sm->set_pos];
            for (int t = 0; t < 20; ++t) {
                const tap* tp = &taps[20 * s + t];
                double* dst = tp->tex == 0 ? grad_grid[b] : grad_plane[3 * b + tp->tex - 1];
                if (!dst) continue;
                for (int ch = 0; ch < NCH; ++ch) dst[tp->idx * NCH + ch] += tp->w * draw[ch];
            }
        }
        free(opg);
    }
    free(buf);
    free(pv);
    free(taps);
    free(wts);
    free(Tb);
    free(suf);
    free(ev);
    (void)nblocks;
    return 0;
}

/* Adjoint of the per-block deferred composite.  Per block k (in ray order)
 * with local composite (A^k, T^k), prefix transmittance P_k and colour
 * C^k = A^k[0..2] + sigmoid(Phi^k(A^k, d)):
 *   C = sum_k P_k C^k, T = prod_k T^k,
 *   dL/dA^k = P_k (g on C_d) + P_k J_Phi^T (g * s (1 - s)),
 *   T^k dL/dT^k = g . R_k + gT T with R_k = sum_{k'>k} P_k' C^k',
 * and inside block k the single-chain adjoint with u = dL/dA^k. */
int orc_adjoint_block_mlp(const orc_block* blocks, int nblocks, const unsigned char* const* occ,
                          const orc_view* v, const int* set, int nset, const orc_params* p,
                          const double* mlp, const int* pix, int npix, const double* grad_rgb,
                          const double* grad_trans, const double* w_opacity, double* const* grad_grid,
                          double* const* grad_plane, double* grad_mlp) {
    for (int s = 0; s < nset; ++s)
        if (blocks[set[s]].dtype != ORC_F64 || blocks[set[s]].contracted) return -1;
    if (p->pe < 0 || p->pe > 4) return -1;
    const mlp_shape sh = mlp_shape_of(p->pe);
    long cap = sample_cap(p, nset);
    sample* buf = (sample*)malloc(sizeof(sample) * cap);
    pt_val* pv = (pt_val*)malloc(sizeof(pt_val) * cap);
    tap* taps = (tap*)malloc(sizeof(tap) * 20 * cap);
    double* Tl = (double*)malloc(sizeof(double) * (cap + 1)); /* local T before each sample */
    long* ev = (long*)malloc(sizeof(long) * cap);
    int nb_max = nset + 1;
    long* rb = (long*)malloc(sizeof(long) * (nb_max + 1)); /* first evaluated sample of each run */
    int* rpos = (int*)malloc(sizeof(int) * nb_max);
    double* Ak = (double*)malloc(sizeof(double) * 7 * nb_max);
    double* Tk = (double*)malloc(sizeof(double) * nb_max);
    double* Pk = (double*)malloc(sizeof(double) * nb_max);
    double* Ck = (double*)malloc(sizeof(double) * 3 * nb_max);
    mlp_trace* tr = (mlp_trace*)malloc(sizeof(mlp_trace) * nb_max);
    for (int q = 0; q < npix; ++q) {
        float d[3];
        long n = enumerate(blocks, nblocks, occ, v, set, nset, p, pix[2 * q], pix[2 * q + 1], buf, cap, d);
        /* forward, run by run, with early termination */
        int nr = 0;
        long m = 0;
        double P = 1.0;
        long s = 0;
        int stop = 0;
        while (s < n && !stop) {
            const int run = buf[s].set_pos;
            rpos[nr] = run;
            rb[nr] = m;
            double A[7] = {0}, T = 1.0;
            for (; s < n && buf[s].set_pos == run; ++s) {
                if (!buf[s].occupied) continue;
                real raw[NCH];
                shade(&blocks[set[run]], buf[s].q, &pv[m], raw, &taps[20 * m]);
                double sd = pv[m].sigma * buf[s].delta;
                double alpha = -expm1(-sd);
                Tl[m] = T;
                for (int c = 0; c < 7; ++c) A[c] += T * alpha * pv[m].v[c];
                T *= exp(-sd);
                ev[m++] = s;
                if (p->t_min > 0.0f && P * T < (double)p->t_min) {
                    stop = 1;
                    break;
                }
            }
            for (int c = 0; c < 7; ++c) Ak[7 * nr + c] = A[c];
            Tk[nr] = T;
            Pk[nr] = P;
            double x[MLP_MAX_IN];
            mlp_input(A, d, p->pe, x);
            mlp_fwd(mlp + sh.n * (long)set[run], &sh, x, &tr[nr]);
            for (int c = 0; c < 3; ++c) Ck[3 * nr + c] = A[c] + tr[nr].s[c];
            P *= T;
            ++nr;
        }
        rb[nr] = m;
        const double Ttot = P;
        const double* g = grad_rgb + 3 * q;
        const double gT = grad_trans ? grad_trans[q] : 0.0;
        double R[3] = {0, 0, 0}; /* sum over later blocks of P_k' C^k' */
        for (int k = nr - 1; k >= 0; --k) {
            const double* Wk = mlp + sh.n * (long)set[rpos[k]];
            const double *W1 = Wk + sh.W1, *W2 = Wk + sh.W2, *W3 = Wk + sh.W3;
            double dz[3], dh2[16], dh1[16], dx[7];
            for (int o = 0; o < 3; ++o) dz[o] = Pk[k] * g[o] * tr[k].s[o] * (1.0 - tr[k].s[o]);
            for (int i = 0; i < 16; ++i) {
                double a = 0.0;
                for (int o = 0; o < 3; ++o) a += W3[o * 16 + i] * dz[o];
                dh2[i] = tr[k].pre2[i] > 0.0 ? a : 0.0;
            }
            for (int i = 0; i < 16; ++i) {
                double a = 0.0;
                for (int o = 0; o < 16; ++o) a += W2[o * 16 + i] * dh2[o];
                dh1[i] = tr[k].pre1[i] > 0.0 ? a : 0.0;
            }
            for (int i = 0; i < 7; ++i) { /* the direction inputs are constants */
                double a = 0.0;
                for (int o = 0; o < 16; ++o) a += W1[o * sh.ni + i] * dh1[o];
                dx[i] = a;
            }
            if (grad_mlp) {
                double* gm = grad_mlp + sh.n * (long)set[rpos[k]];
                for (int o = 0; o < 16; ++o) {
                    for (int i = 0; i < sh.ni; ++i) gm[sh.W1 + o * sh.ni + i] += dh1[o] * tr[k].x[i];
                    gm[sh.b1 + o] += dh1[o];
                    for (int i = 0; i < 16; ++i) gm[sh.W2 + o * 16 + i] += dh2[o] * tr[k].h1[i];
                    gm[sh.b2 + o] += dh2[o];
                }
                for (int o = 0; o < 3; ++o) {
                    for (int i = 0; i < 16; ++i) gm[sh.W3 + o * 16 + i] += dz[o] * tr[k].h2[i];
                    gm[sh.b3 + o] += dz[o];
                }
            }
            double u[7];
            for (int c = 0; c < 7; ++c) u[c] = dx[c] + (c < 3 ? Pk[k] * g[c] : 0.0);
            const double tT = g[0] * R[0] + g[1] * R[1] + g[2] * R[2] + gT * Ttot; /* T^k dL/dT^k */
            /* opacity term of this block: w h'(1 - T^k) T^k per unit step */
            double gop = 0.0;
            if (w_opacity && w_opacity[q] != 0.0) gop = w_opacity[q] * opac_dh(1.0 - Tk[k]) * Tk[k];
            /* inside the block: suffix sums of w_j v_j */
            double S[7] = {0, 0, 0, 0, 0, 0, 0};
            for (long e = rb[k + 1] - 1; e >= rb[k]; --e) {
                const sample* sm = &buf[ev[e]];
                double delta = sm->delta;
                double alpha = -expm1(-pv[e].sigma * delta);
                double w = Tl[e] * alpha;
                double Tn = Tl[e] * exp(-pv[e].sigma * delta);
                double uv = 0.0, us = 0.0;
                for (int c = 0; c < 7; ++c) {
                    uv += u[c] * pv[e].v[c];
                    us += u[c] * S[c];
                }
                double dsig = delta * (Tn * uv - us) - delta * tT + delta * gop;
                double draw[NCH];
                draw[0] = pv[e].sigma * dsig;
                for (int c = 0; c < 7; ++c) draw[1 + c] = w * u[c] * pv[e].v[c] * (1.0 - pv[e].v[c]);
                int b = set[sm->set_pos];
                for (int t = 0; t < 20; ++t) {
                    const tap* tp = &taps[20 * e + t];
                    double* dst = tp->tex == 0 ? grad_grid[b] : grad_plane[3 * b + tp->tex - 1];
                    if (!dst) continue;
                    for (int ch = 0; ch < NCH; ++ch) dst[tp->idx * NCH + ch] += tp->w * draw[ch];
                }
                for (int c = 0; c < 7; ++c) S[c] += w * pv[e].v[c];
            }
            for (int c = 0; c < 3; ++c) R[c] += Pk[k] * Ck[3 * k + c];
        }
    }
    free(buf);
    free(pv);
    free(taps);
    free(Tl);
    free(ev);
    free(rb);
    free(rpos);
    free(Ak);
    free(Tk);
    free(Pk);
    free(Ck);
    free(tr);
    (void)nblocks;
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Regularisers of the training objective (Sec. 4.3)                       */
/* ---------------------------------------------------------------------- */

int orc_opacity(const orc_block* blocks, int nblocks, const unsigned char* const* occ,
                const orc_view* v, const int* set, int nset, const orc_params* p,
                const int* pix, int npix, double* loss) {
    long cap = sample_cap(p, nset);
    sample* buf = (sample*)malloc(sizeof(sample) * cap);
    for (int q = 0; q < npix; ++q) {
        float d[3];
        long n = enumerate(blocks, nblocks, occ, v, set, nset, p, pix[2 * q], pix[2 * q + 1], buf, cap, d);
        double L = 0.0, T = 1.0;
        long s = 0;
        int stop = 0;
        while (s < n && !stop) {
            int run = buf[s].set_pos;
            double Tk = 1.0;
            for (; s < n && buf[s].set_pos == run; ++s) {
                if (!buf[s].occupied) continue;
                pt_val pv;
                real raw[NCH];
                shade(&blocks[set[run]], buf[s].q, &pv, raw, NULL);
                Tk *= exp(-pv.sigma * buf[s].delta);
                if (p->t_min > 0.0f && T * Tk < (double)p->t_min) {
                    stop = 1;
                    break;
                }
            }
            L += opac_h(1.0 - Tk);
            T *= Tk;
        }
        loss[q] = L;
    }
    free(buf);
    return 0;
}

double orc_sparsity(const orc_block* blocks, int nblocks, const unsigned char* const* occ,
                    const int* set, int nset, const float* pts, int n, double delta, double weight,
                    double* alpha_out, double* const* grad_grid, double* const* grad_plane) {
    double loss = 0.0;
    tap taps[20];
    for (int i = 0; i < n; ++i) {
        const float* pt = pts + 3 * i;
        if (alpha_out) alpha_out[i] = 0.0;
        int s_hit = -1;
        for (int s = 0; s < nset; ++s)
            if (inside(pt, blocks[set[s]].lo, blocks[set[s]].hi)) {
                s_hit = s;
                break;
            }
        if (s_hit < 0) continue;
        const orc_block* b = &blocks[set[s_hit]];
        float q[3];
        int cell = occ_cell(b, pt, q);
        if (!occ[set[s_hit]][cell]) continue; /* density is zero in unoccupied cells */
        real raw[NCH];
        eval_raw(b, q, raw, taps);
        double sigma = exp(raw[0]);
        double alpha = -expm1(-sigma * delta);
        if (alpha_out) alpha_out[i] = alpha;
        loss += weight / n * alpha;
        double draw0 = weight / n * delta * exp(-sigma * delta) * sigma;
        int bi = set[s_hit];
        for (int t = 0; t < 20; ++t) {
            double* const* tab = taps[t].tex == 0 ? grad_grid : grad_plane;
            double* dst = !tab ? NULL : (taps[t].tex == 0 ? tab[bi] : tab[3 * bi + taps[t].tex - 1]);
            if (dst) dst[taps[t].idx * NCH] += taps[t].w * draw0;
        }
    }
    (void)nblocks;
    return loss;
}

/* ---------------------------------------------------------------------- */
/* Selection (viewer: dynamic loading, LOD, depth sorting)                 */
/* ---------------------------------------------------------------------- */

static int culled(const orc_view* v, const double lo[3], const double hi[3]) {
    double Rm[9], e[3];
    for (int k = 0; k < 9; ++k) Rm[k] = v->R[k];
    for (int k = 0; k < 3; ++k) e[k] = v->eye[k];
    double xw0 = v->x0, xw1 = (double)v->x0 + v->w, yw0 = v->y0, yw1 = (double)v->y0 + v->h;
    double fx = v->fx, fy = v->fy, cx = v->cx, cy = v->cy;
    double planes[5][3] = {
        {fx, 0.0, cx - xw0}, {-fx, 0.0, xw1 - cx}, {0.0, fy, cy - yw0}, {0.0, -fy, yw1 - cy}, {0.0, 0.0, 1.0}};
    double X[8][3], nX[8];
    for (int c = 0; c < 8; ++c) {
        double P[3] = {(c & 1) ? hi[0] : lo[0], (c & 2) ? hi[1] : lo[1], (c & 4) ? hi[2] : lo[2]};
        double w[3] = {P[0] - e[0], P[1] - e[1], P[2] - e[2]};
        for (int a = 0; a < 3; ++a) X[c][a] = Rm[0 * 3 + a] * w[0] + Rm[1 * 3 + a] * w[1] + Rm[2 * 3 + a] * w[2];
        nX[c] = sqrt(X[c][0] * X[c][0] + X[c][1] * X[c][1] + X[c][2] * X[c][2]);
    }
    for (int pl = 0; pl < 5; ++pl) {
        double* n = planes[pl];
        double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        int all_out = 1;
        for (int c = 0; c < 8 && all_out; ++c) {
            double s = (n[0] * X[c][0] + n[1] * X[c][1] + n[2] * X[c][2]) / nn;
            if (!(s < -1e-5 * nX[c])) all_out = 0;
        }
        if (all_out) return 1;
    }
    return 0;
}

int orc_select(const orc_view* v, int nent, const int* ids, const int* lods, const float* lo,
               const float* hi, const double* ztop, const int* contracted, const double* thresholds,
               int n_thr, int cull, int* out, int cap) {
    int n = 0;
    double* key = (double*)malloc(sizeof(double) * (nent + 1));
    for (int e = 0; e < nent; ++e) {
        if (lods[e] != 0) continue; /* one decision per block, made from its finest level */
        double c[3] = {0.5 * ((double)lo[3 * e] + (double)hi[3 * e]),
                       0.5 * ((double)lo[3 * e + 1] + (double)hi[3 * e + 1]), ztop[e]};
        double dx = (double)v->eye[0] - c[0], dy = (double)v->eye[1] - c[1], dz = (double)v->eye[2] - c[2];
        double dist = sqrt(dx * dx + dy * dy + dz * dz);
        int lod = -1;
        for (int l = 0; l < n_thr; ++l)
            if (dist < thresholds[l]) {
                lod = l;
                break;
            }
        /* a contracted block also owns the space beyond its outer faces, out to
         * infinity: the far cut and the frustum test of its box do not apply */
        if (lod < 0 && contracted[e]) lod = n_thr - 1;
        if (lod < 0) continue; /* beyond the far cut */
        int chosen = -1;
        for (int f = 0; f < nent; ++f)
            if (ids[f] == ids[e] && lods[f] == lod) chosen = f;
        if (chosen < 0) {
            free(key);
            return -2;
        }
        if (cull && !contracted[e]) {
            double blo[3] = {lo[3 * chosen], lo[3 * chosen + 1], lo[3 * chosen + 2]};
            double bhi[3] = {hi[3 * chosen], hi[3 * chosen + 1], ztop[chosen]};
            if (culled(v, blo, bhi)) continue;
        }
        if (n >= cap) break;
        out[n] = chosen;
        key[n] = sqrt(dx * dx + dy * dy);
        ++n;
    }
    /* insertion sort by xy distance, ties to the lower block id */
    for (int a = 1; a < n; ++a)
        for (int b = a; b > 0; --b) {
            int swap = key[b] < key[b - 1] || (key[b] == key[b - 1] && ids[out[b]] < ids[out[b - 1]]);
            if (!swap) break;
            double tk = key[b];
            key[b] = key[b - 1];
            key[b - 1] = tk;
            int to = out[b];
            out[b] = out[b - 1];
            out[b - 1] = to;
        }
    free(key);
    return n;
}

/* Quadtree LOD selection (Appendix D "Dynamic Loading" with the merged LOD
 * assets of Sec. 4.5 "Baking": an entry of LOD l covers 2^l x 2^l blocks).
 * Coarse to fine: an entry of LOD l > 0 is drawn when every visible entry of
 * LOD l - 1 inside it lies at distance >= thresholds[l - 1] (vacuously when
 * none is visible); otherwise its visible children are examined in turn.
 * Distance: eye to (centre x, centre y, highest finest-level top inside the
 * entry).  Culling: the entry's box [lo, (hi_x, hi_y, its own ztop)].  Order:
 * the coarsest entries by xy distance of their centres (ties: lower id), and
 * inside an entry its children nearest quadrant first, then the two quadrants
 * beside it (lower id first), then the opposite one: a straight ray crosses
 * each of the two centre lines at most once, so it never meets them in
 * another order.  A coarsest entry at distance >= thresholds[L] (when given)
 * is not drawn. */
typedef struct qt_state {
    const orc_view* v;
    int nent;
    const int *ids, *lods;
    const float *lo, *hi;
    const double *ztop, *thr;
    const int* contracted;
    int n_thr, cull, *out, cap, n;
} qt_state;

/* the entry's footprint holds a contracted finest-level entry */
static int qt_pinned(const qt_state* q, int e);

static int xy_inside(const qt_state* q, int f, int e) {
    return q->lo[3 * f] >= q->lo[3 * e] && q->hi[3 * f] <= q->hi[3 * e] && q->lo[3 * f + 1] >= q->lo[3 * e + 1] &&
           q->hi[3 * f + 1] <= q->hi[3 * e + 1];
}

static double qt_dist(const qt_state* q, int e) {
    double zf = -INFINITY;
    for (int f = 0; f < q->nent; ++f)
        if (q->lods[f] == 0 && xy_inside(q, f, e) && q->ztop[f] > zf) zf = q->ztop[f];
    double cx = 0.5 * ((double)q->lo[3 * e] + (double)q->hi[3 * e]);
    double cy = 0.5 * ((double)q->lo[3 * e + 1] + (double)q->hi[3 * e + 1]);
    double dx = (double)q->v->eye[0] - cx, dy = (double)q->v->eye[1] - cy, dz = (double)q->v->eye[2] - zf;
    return sqrt(dx * dx + dy * dy + dz * dz);
}

static int qt_pinned(const qt_state* q, int e) {
    for (int f = 0; f < q->nent; ++f)
        if (q->lods[f] == 0 && q->contracted[f] && xy_inside(q, f, e)) return 1;
    return 0;
}

static int qt_visible(const qt_state* q, int e) {
    if (!q->cull || qt_pinned(q, e)) return 1;
    double blo[3] = {q->lo[3 * e], q->lo[3 * e + 1], q->lo[3 * e + 2]};
    double bhi[3] = {q->hi[3 * e], q->hi[3 * e + 1], q->ztop[e]};
    return !culled(q->v, blo, bhi);
}

static void qt_emit(qt_state* q, int e) {
    if (q->n < q->cap) q->out[q->n] = e;
    ++q->n;
}

static void qt_visit(qt_state* q, int e) {
    int l = q->lods[e];
    if (l == 0) {
        qt_emit(q, e);
        return;
    }
    int kid[64], rank[64], nk = 0, all_far = 1;
    double cx = 0.5 * ((double)q->lo[3 * e] + (double)q->hi[3 * e]);
    double cy = 0.5 * ((double)q->lo[3 * e + 1] + (double)q->hi[3 * e + 1]);
    int ex = (double)q->v->eye[0] >= cx, ey = (double)q->v->eye[1] >= cy;
    for (int f = 0; f < q->nent && nk < 64; ++f) {
        if (q->lods[f] != l - 1 || !xy_inside(q, f, e) || !qt_visible(q, f)) continue;
        if (qt_dist(q, f) < q->thr[l - 1]) all_far = 0;
        double fx = 0.5 * ((double)q->lo[3 * f] + (double)q->hi[3 * f]);
        double fy = 0.5 * ((double)q->lo[3 * f + 1] + (double)q->hi[3 * f + 1]);
        rank[nk] = ((fx >= cx) != ex) + ((fy >= cy) != ey);
        kid[nk++] = f;
    }
    if (all_far && !qt_pinned(q, e)) {
        qt_emit(q, e);
        return;
    }
    for (int r = 0; r <= 2; ++r) {
        /* children of this rank, lower id first */
        int used[64] = {0};
        for (;;) {
            int best = -1;
            for (int k = 0; k < nk; ++k)
                if (!used[k] && rank[k] == r && (best < 0 || q->ids[kid[k]] < q->ids[kid[best]])) best = k;
            if (best < 0) break;
            used[best] = 1;
            qt_visit(q, kid[best]);
        }
    }
}

int orc_select_quadtree(const orc_view* v, int nent, const int* ids, const int* lods, const float* lo,
                        const float* hi, const double* ztop, const int* contracted, const double* thresholds,
                        int n_thr, int cull, int* out, int cap) {
    int L = 0;
    for (int e = 0; e < nent; ++e)
        if (lods[e] > L) L = lods[e];
    if (n_thr < L) return -3;
    qt_state q = {v, nent, ids, lods, lo, hi, ztop, thresholds, contracted, n_thr, cull, out, cap, 0};
    int* roots = (int*)malloc(sizeof(int) * (nent + 1));
    double* key = (double*)malloc(sizeof(double) * (nent + 1));
    int nr = 0;
    for (int e = 0; e < nent; ++e) {
        if (lods[e] != L || !qt_visible(&q, e)) continue;
        if (n_thr > L && qt_dist(&q, e) >= thresholds[L] && !qt_pinned(&q, e)) continue;
        double cx = 0.5 * ((double)lo[3 * e] + (double)hi[3 * e]), cy = 0.5 * ((double)lo[3 * e + 1] + (double)hi[3 * e + 1]);
        double dx = (double)v->eye[0] - cx, dy = (double)v->eye[1] - cy;
        roots[nr] = e;
        key[nr++] = sqrt(dx * dx + dy * dy);
    }
    for (int a = 1; a < nr; ++a)
        for (int b = a; b > 0; --b) {
            int swap = key[b] < key[b - 1] || (key[b] == key[b - 1] && ids[roots[b]] < ids[roots[b - 1]]);
            if (!swap) break;
            double tk = key[b];
            key[b] = key[b - 1];
            key[b - 1] = tk;
            int tr = roots[b];
            roots[b] = roots[b - 1];
            roots[b - 1] = tr;
        }
    for (int r = 0; r < nr; ++r) qt_visit(&q, roots[r]);
    free(roots);
    free(key);
    return q.n > cap ? cap : q.n;
}
