// Device kernels of the block-merged ray-march renderer for gfx950
// (City-on-Web, arXiv 2312.16457).
//
// Compiled with -ffp-contract=off and correctly rounded fp32 divide/sqrt:
// every discrete decision (ray direction, sample position, sample -> block,
// occupancy cell) is one fixed sequence of IEEE fp32 operations, so it is
// reproducible bit for bit by any other IEEE implementation of the same
// sequence.  Continuous arithmetic uses explicit fmaf where fusion is wanted.
#include <hip/hip_runtime.h>

#include "cow_internal.h"

namespace cow {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// exact fp32 decision sequences
// ---------------------------------------------------------------------------

// Pixel ray r(t) = o + t d (Sec. 3): d is the normalised camera-to-world
// rotation of (x, y, 1), x = (i + 1/2 - cx) / fx, y = (j + 1/2 - cy) / fy.
__device__ inline void ray_direction(const DevView* v, int i, int j, float d[3]) {
    float x = ((float)i + 0.5f - v->cx) / v->fx;
    float y = ((float)j + 0.5f - v->cy) / v->fy;
    float u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float a = v->R[3 * c + 0] * x;
        float b = v->R[3 * c + 1] * y;
        u[c] = (a + b) + v->R[3 * c + 2];
    }
    float n = sqrtf((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) d[c] = u[c] / n;
}

// camera-anchored step k: t_k = (k + 1/2) delta, exact for k < 2^23 when
// delta is a power of two
__device__ inline float step_t(int k, float delta) { return ((float)k + 0.5f) * delta; }

// sample coordinate fl(o + fl(t d))
__device__ inline float coord(float o, float t, float d) {
    float td = t * d;
    return o + td;
}

// Least k in [0, kMaxStep] for which pred(k) holds, pred monotone
// false -> true; kMaxStep + 1 when it never holds.  Exact whatever the guess
// (the guess only sets the cost): gallop from it, then bisect.
template <class Pred>
__device__ inline int first_true(Pred pred, int guess) {
    guess = guess < 0 ? 0 : (guess > kMaxStep ? kMaxStep : guess);
    int lo, hi;  // pred(lo) false (lo may be -1), pred(hi) true (hi may be kMaxStep + 1)
    if (pred(guess)) {
        hi = guess;
        int step = 1;
        for (;;) {
            int c = hi - step;
            if (c < 0) {
                lo = -1;
                break;
            }
            if (!pred(c)) {
                lo = c;
                break;
            }
            hi = c;
            step <<= 1;
        }
    } else {
        lo = guess;
        int step = 1;
        for (;;) {
            int c = lo + step;
            if (c > kMaxStep) {
                hi = kMaxStep + 1;
                break;
            }
            if (pred(c)) {
                hi = c;
                break;
            }
            lo = c;
            step <<= 1;
        }
    }
    while (hi - lo > 1) {
        int mid = lo + ((hi - lo) >> 1);
        if (pred(mid))
            hi = mid;
        else
            lo = mid;
    }
    return hi;
}

__device__ inline int guess_index(float g) {
    if (!(g > 0.0f)) return 0;
    if (g > (float)kMaxStep) return kMaxStep;
    return (int)ceilf(g);
}

// Step indices k >= 0 whose fp32 sample position lies in the half-open box
// [lo, hi) on every axis: the interval [*ka, *kb) (empty when *ka >= *kb).
// Each axis predicate is monotone in k because t_k and both roundings are
// monotone, so the set is an intersection of prefixes and suffixes.
__device__ inline void box_interval(const float o[3], const float d[3], float delta, float inv_delta,
                                    const float lo[3], const float hi[3], int* ka, int* kb) {
    int a = 0, b = kMaxStep + 1;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float oc = o[c], dc = d[c], l = lo[c], h = hi[c];
        if (dc == 0.0f) {
            if (!(l <= oc && oc < h)) b = 0;
            continue;
        }
        const float r = __builtin_amdgcn_rcpf(dc);
        const int gl = guess_index(((l - oc) * r) * inv_delta - 0.5f);
        const int gh = guess_index(((h - oc) * r) * inv_delta - 0.5f);
        if (dc > 0.0f) {
            int e = first_true([&](int k) { return coord(oc, step_t(k, delta), dc) >= l; }, gl);
            int x = first_true([&](int k) { return coord(oc, step_t(k, delta), dc) >= h; }, gh);
            a = e > a ? e : a;
            b = x < b ? x : b;
        } else {
            int e = first_true([&](int k) { return coord(oc, step_t(k, delta), dc) < h; }, gh);
            int x = first_true([&](int k) { return coord(oc, step_t(k, delta), dc) < l; }, gl);
            a = e > a ? e : a;
            b = x < b ? x : b;
        }
    }
    *ka = a;
    *kb = b;
}

// slab test against the closed box, t_near clamped at 0 (chord mode)
__device__ inline bool slab_exact(const float o[3], const float d[3], const float lo[3],
                                  const float hi[3], float* tn, float* tf) {
    float t0 = 0.0f, t1 = INFINITY;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        if (d[c] == 0.0f) {
            if (o[c] < lo[c] || o[c] > hi[c]) return false;
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

__device__ inline int occ_index(const DevBlock* B, const float q[3]) {
    const int O = B->O;
    const float Of = (float)O;
    int cell[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        int k = (int)floorf(q[c] * Of);
        k = k < 0 ? 0 : k;
        cell[c] = k > O - 1 ? O - 1 : k;
    }
    return (cell[2] * O + cell[1]) * O + cell[0];
}

// ---------------------------------------------------------------------------
// feature gather: trilinear grid + three bilinear planes
// ---------------------------------------------------------------------------

struct Lin {
    int i0, i1;
    float w0, w1;
};

// cell-centred, clamp-to-edge linear taps: u = q R - 1/2
__device__ inline Lin lin_taps(float q, int R) {
    float u = q * (float)R - 0.5f;
    float fl = floorf(u);
    int a = (int)fl;
    Lin t;
    t.w1 = u - fl;
    t.w0 = 1.0f - t.w1;
    t.i0 = a < 0 ? 0 : a;
    t.i1 = a + 1 > R - 1 ? R - 1 : a + 1;
    return t;
}

__device__ inline float ub(uint2 v, int c) {
    uint32_t w = c < 4 ? v.x : v.y;
    return (float)((w >> (8 * (c & 3))) & 0xffu);
}

// weighted sum over n uint8 texels, per channel
template <int N>
__device__ inline void accum_u8(const uint2 (&t)[N], const float (&w)[N], float acc[8]) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        float s = w[0] * ub(t[0], c);
#pragma unroll
        for (int k = 1; k < N; ++k) s = fmaf(w[k], ub(t[k], c), s);
        acc[c] = s;
    }
}

// texel offsets and weights of one sample: 8 grid, then xy, xz, yz (4 each)
struct Taps {
    int idx[20];
    float w[20];
};

__device__ inline void sample_taps(int R, int Rp, const float q[3], Taps& T) {
    Lin gx = lin_taps(q[0], R), gy = lin_taps(q[1], R), gz = lin_taps(q[2], R);
    Lin px = lin_taps(q[0], Rp), py = lin_taps(q[1], Rp), pz = lin_taps(q[2], Rp);
    const int zi[2] = {gz.i0, gz.i1}, yi[2] = {gy.i0, gy.i1}, xi[2] = {gx.i0, gx.i1};
    const float zw[2] = {gz.w0, gz.w1}, yw[2] = {gy.w0, gy.w1}, xw[2] = {gx.w0, gx.w1};
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            const int row = (zi[dz] * R + yi[dy]) * R;
            const float wzy = zw[dz] * yw[dy];
#pragma unroll
            for (int dx = 0; dx < 2; ++dx) {
                T.idx[dz * 4 + dy * 2 + dx] = row + xi[dx];
                T.w[dz * 4 + dy * 2 + dx] = wzy * xw[dx];
            }
        }
    // planes index [v][u]: xy (u=x, v=y), xz (u=x, v=z), yz (u=y, v=z)
    const Lin U[3] = {px, px, py}, V[3] = {py, pz, pz};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const int v0 = V[p].i0 * Rp, v1 = V[p].i1 * Rp;
        T.idx[8 + 4 * p + 0] = v0 + U[p].i0;
        T.idx[8 + 4 * p + 1] = v0 + U[p].i1;
        T.idx[8 + 4 * p + 2] = v1 + U[p].i0;
        T.idx[8 + 4 * p + 3] = v1 + U[p].i1;
        T.w[8 + 4 * p + 0] = V[p].w0 * U[p].w0;
        T.w[8 + 4 * p + 1] = V[p].w0 * U[p].w1;
        T.w[8 + 4 * p + 2] = V[p].w1 * U[p].w0;
        T.w[8 + 4 * p + 3] = V[p].w1 * U[p].w1;
    }
}

// Buffer resources: the texture base lives in scalar registers and each
// texel fetch carries only a 32-bit byte offset; the hardware range check
// returns zero outside [0, bytes).
__device__ inline __amdgpu_buffer_rsrc_t tex_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ inline uint2 ld8(__amdgpu_buffer_rsrc_t r, int idx) {
    auto v = __builtin_amdgcn_raw_buffer_load_b64(r, idx * 8, 0, 0);
    return make_uint2(v[0], v[1]);
}

__device__ inline float4 ld16(__amdgpu_buffer_rsrc_t r, int byte_off) {
    auto v = __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 0);
    return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]),
                       __uint_as_float(v[3]));
}

// raw pre-activation features ((G + XY) + XZ) + YZ of a uint8 block
template <bool SPARSE>
__device__ inline void raw_u8(const DevBlock* B, const float q[3], int cell, float raw[8]) {
    Taps T;
    sample_taps(B->R, B->Rp, q, T);
    const int R = B->R, Rp = B->Rp;
    const uint32_t pbytes = (uint32_t)Rp * Rp * 8;
    uint2 g[8], p0[4], p1[4], p2[4];
    float wg[8], w0[4], w1[4], w2[4];
    if (SPARSE) {
        // brick of (s+2)^3 texels around the sample's occupancy cell: texel
        // j of an axis holds grid index clamp(c s - 1 + j)
        const int O = B->O, s = R / O, s2 = s + 2;
        const int cx = cell % O, cy = (cell / O) % O, cz = cell / (O * O);
        const int slot = B->brick_slot[cell];
        const int bsz = s2 * s2 * s2;
        const __amdgpu_buffer_rsrc_t rb = tex_rsrc(B->bricks, B->brick_bytes);
        const Lin gx = lin_taps(q[0], R), gy = lin_taps(q[1], R), gz = lin_taps(q[2], R);
        const int xs[2] = {gx.i0 - (cx * s - 1), gx.i1 - (cx * s - 1)};
        const int ys[2] = {gy.i0 - (cy * s - 1), gy.i1 - (cy * s - 1)};
        const int zs[2] = {gz.i0 - (cz * s - 1), gz.i1 - (cz * s - 1)};
#pragma unroll
        for (int k = 0; k < 8; ++k)
            g[k] = ld8(rb, slot * bsz + (zs[k >> 2] * s2 + ys[(k >> 1) & 1]) * s2 + xs[k & 1]);
    } else {
        const __amdgpu_buffer_rsrc_t rg = tex_rsrc(B->grid, (uint32_t)R * R * R * 8);
#pragma unroll
        for (int k = 0; k < 8; ++k) g[k] = ld8(rg, T.idx[k]);
    }
    const __amdgpu_buffer_rsrc_t r0 = tex_rsrc(B->plane[0], pbytes);
    const __amdgpu_buffer_rsrc_t r1 = tex_rsrc(B->plane[1], pbytes);
    const __amdgpu_buffer_rsrc_t r2 = tex_rsrc(B->plane[2], pbytes);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        p0[k] = ld8(r0, T.idx[8 + k]);
        p1[k] = ld8(r1, T.idx[12 + k]);
        p2[k] = ld8(r2, T.idx[16 + k]);
        w0[k] = T.w[8 + k];
        w1[k] = T.w[12 + k];
        w2[k] = T.w[16 + k];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) wg[k] = T.w[k];
    // fold each texture into raw as soon as it is summed: ((G + XY) + XZ) + YZ
    float acc[8];
    accum_u8<8>(g, wg, acc);
#pragma unroll
    for (int c = 0; c < 8; ++c) raw[c] = fmaf(acc[c], B->scale[0][c], B->offset[0][c]);
    accum_u8<4>(p0, w0, acc);
#pragma unroll
    for (int c = 0; c < 8; ++c) raw[c] += fmaf(acc[c], B->scale[1][c], B->offset[1][c]);
    accum_u8<4>(p1, w1, acc);
#pragma unroll
    for (int c = 0; c < 8; ++c) raw[c] += fmaf(acc[c], B->scale[2][c], B->offset[2][c]);
    accum_u8<4>(p2, w2, acc);
#pragma unroll
    for (int c = 0; c < 8; ++c) raw[c] += fmaf(acc[c], B->scale[3][c], B->offset[3][c]);
}

// fp32 block: texel = two 16-byte halves (channels 0-3, 4-7); textures are
// summed one at a time to bound the registers held by loads in flight
__device__ inline void raw_f32(const DevBlock* B, const float q[3], float raw[8], const Taps& T) {
    const int R = B->R, Rp = B->Rp;
    const __amdgpu_buffer_rsrc_t rs[4] = {tex_rsrc(B->grid, (uint32_t)R * R * R * 32),
                                          tex_rsrc(B->plane[0], (uint32_t)Rp * Rp * 32),
                                          tex_rsrc(B->plane[1], (uint32_t)Rp * Rp * 32),
                                          tex_rsrc(B->plane[2], (uint32_t)Rp * Rp * 32)};
    float part[4][8];
#pragma unroll
    for (int tex = 0; tex < 4; ++tex) {
        const int k0 = tex == 0 ? 0 : 4 + 4 * tex, n = tex == 0 ? 8 : 4;
        float a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < n; ++k) {
            const float4 lo = ld16(rs[tex], T.idx[k0 + k] * 32);
            const float4 hi = ld16(rs[tex], T.idx[k0 + k] * 32 + 16);
            const float w = T.w[k0 + k];
            a[0] = fmaf(w, lo.x, a[0]);
            a[1] = fmaf(w, lo.y, a[1]);
            a[2] = fmaf(w, lo.z, a[2]);
            a[3] = fmaf(w, lo.w, a[3]);
            a[4] = fmaf(w, hi.x, a[4]);
            a[5] = fmaf(w, hi.y, a[5]);
            a[6] = fmaf(w, hi.z, a[6]);
            a[7] = fmaf(w, hi.w, a[7]);
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) part[tex][c] = a[c];
    }
#pragma unroll
    for (int c = 0; c < 8; ++c) raw[c] = ((part[0][c] + part[1][c]) + part[2][c]) + part[3][c];
}

__device__ inline float sigmoidf_(float x) { return __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }

// ---------------------------------------------------------------------------
// forward march: per-block composite + front-to-back merge
// ---------------------------------------------------------------------------

struct RayState {
    float o[3], d[3];
    float A[7], T;
    int64_t n_eval, n_march;
    int w0, w1;  // grid-mode window [k0, k0 + max_steps)
    bool hit;
};

// Composite the samples of one block for one lane (Eqs. "alpha
// accumulation", "combined accumulation", "volume rendering inside blocks"):
// Ak = sum_i T_i alpha_i (c_i, f_i), Tk = prod_i (1 - alpha_i).
template <int DT, int MODE, bool SPARSE>
__device__ inline void march_block(const MarchArgs& a, const DevBlock* B, RayState& s, float Ak[7],
                                   float& Tk) {
    int ka = 0, kb = 0;
    float tn = 0.0f, dr = 0.0f;
    if (MODE == 1) {
        if (s.hit) {
            box_interval(s.o, s.d, a.delta, 1.0f / a.delta, B->lo, B->hi, &ka, &kb);
            ka = ka > s.w0 ? ka : s.w0;
            kb = kb < s.w1 ? kb : s.w1;
        }
    } else {
        float tf;
        if (s.hit && slab_exact(s.o, s.d, B->lo, B->hi, &tn, &tf)) {
            dr = (tf - tn) / (float)a.n_steps;
            kb = a.n_steps;
        }
    }
    if (!__any(ka < kb)) return;
    const float delta = MODE == 1 ? a.delta : dr;
    int k = ka;
    int64_t marched = 0;
    for (;;) {
        bool have = false;
        float q[3];
        int cell = 0;
        while (k < kb) {
            const float t = MODE == 1 ? step_t(k, a.delta) : tn + ((float)k + 0.5f) * dr;
            float p[3];
            bool in = true;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                p[c] = coord(s.o[c], t, s.d[c]);
                if (MODE == 0) in = in && (B->lo[c] <= p[c] && p[c] < B->hi[c]);
                q[c] = p[c] - B->lo[c];
            }
            if (in) {
                ++marched;
                cell = occ_index(B, q);
                if (B->occ[cell]) {
                    have = true;
                    break;
                }
            }
            ++k;
        }
        if (!__any(have)) break;
        if (have) {
            float raw[8];
            if (DT == 0) {
                raw_u8<SPARSE>(B, q, cell, raw);
            } else {
                Taps T;
                sample_taps(B->R, B->Rp, q, T);
                raw_f32(B, q, raw, T);
            }
            const float sigma = __expf(raw[0]);
            const float e = __expf(-sigma * delta);
            const float w = Tk * (1.0f - e);
#pragma unroll
            for (int c = 0; c < 7; ++c) Ak[c] = fmaf(w, sigmoidf_(raw[1 + c]), Ak[c]);
            Tk *= e;
            ++s.n_eval;
            ++k;
        }
    }
    s.n_march += marched;
}

__device__ inline void xcd_packet(int* packet_out, int waves, int wave) {
    const int nb = gridDim.x, b = blockIdx.x;
    const int x = b & 7, q = nb >> 3, r = nb & 7;
    const int lb = x * q + (x < r ? x : r) + (b >> 3);
    *packet_out = lb * waves + wave;
}

__device__ inline const DevView* find_view_by_tile(const MarchArgs& a, int packet) {
    int lo = 0, hi = a.n_views - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.views[mid].tile_begin <= packet)
            lo = mid;
        else
            hi = mid - 1;
    }
    return a.views + lo;
}

template <int MODE, int DT, bool SPARSE>
__device__ void march_packet(const MarchArgs& a, const DevView* V, int tile, int lane) {
    const int tw = a.tile_w, th = a.tile_h;
    const int tx = tile % V->tiles_x, ty = tile / V->tiles_x;
    const int px = V->x0 + tx * tw + (lane % tw);
    const int py = V->y0 + ty * th + (lane / tw);
    const bool active = px < V->x0 + V->w && py < V->y0 + V->h;
    RayState s;
    ray_direction(V, px, py, s.d);
    s.o[0] = V->eye[0];
    s.o[1] = V->eye[1];
    s.o[2] = V->eye[2];
    s.n_eval = 0;
    s.n_march = 0;
    s.hit = active;
    s.w0 = 0;
    s.w1 = 0;
    if (MODE == 1 && active) {
        int ka, kb;
        box_interval(s.o, s.d, a.delta, 1.0f / a.delta, a.scene_lo, a.scene_hi, &ka, &kb);
        s.hit = ka < kb;
        s.w0 = ka;
        s.w1 = ka + a.max_steps;
    }
    const int64_t pix = V->pix_begin + (int64_t)(py - V->y0) * V->w + (px - V->x0);
    int r0 = 0, r1 = V->set_n;
    if (a.only_set_pos >= 0) {
        r0 = a.only_set_pos;
        r1 = a.only_set_pos + 1;
    }
#pragma unroll
    for (int c = 0; c < 7; ++c) s.A[c] = 0.0f;
    s.T = 1.0f;
    if (a.only_set_pos > 0 && active) {  // per-block baseline: continue the running blend
        const float4 lo4 = reinterpret_cast<const float4*>(a.aux)[2 * pix];
        const float4 hi4 = reinterpret_cast<const float4*>(a.aux)[2 * pix + 1];
        s.A[0] = lo4.x, s.A[1] = lo4.y, s.A[2] = lo4.z, s.A[3] = lo4.w;
        s.A[4] = hi4.x, s.A[5] = hi4.y, s.A[6] = hi4.z, s.T = hi4.w;
        if (a.counts) {
            s.n_eval = a.counts[2 * pix];
            s.n_march = a.counts[2 * pix + 1];
        }
    }
    for (int r = r0; r < r1; ++r) {
        const int e = __builtin_amdgcn_readfirstlane(a.refs[V->set_begin + r]);
        const DevBlock* B = a.blocks + e;
        float Ak[7] = {0, 0, 0, 0, 0, 0, 0}, Tk = 1.0f;
        march_block<DT, MODE, SPARSE>(a, B, s, Ak, Tk);
        // merge (Eq. "volume rendering across blocks"), T^k carried directly
#pragma unroll
        for (int c = 0; c < 7; ++c) s.A[c] = fmaf(s.T, Ak[c], s.A[c]);
        s.T *= Tk;
    }
    if (active) {
        float4* aux4 = reinterpret_cast<float4*>(a.aux);
        aux4[2 * pix] = make_float4(s.A[0], s.A[1], s.A[2], s.A[3]);
        aux4[2 * pix + 1] = make_float4(s.A[4], s.A[5], s.A[6], s.T);
        a.trans[pix] = s.T;
        if (a.counts) {
            a.counts[2 * pix] = s.n_eval;
            a.counts[2 * pix + 1] = s.n_march;
        }
    }
}

// all blocks of one launch share a texture dtype (checked on the host)
template <int MODE, int DT, bool SPARSE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4)))
void march_fwd_kernel(MarchArgs a) {
    const int lane = threadIdx.x & 63;
    const int waves = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (a.persistent) {
        for (;;) {
            int p = 0;
            if (lane == 0) p = atomicAdd(a.work_counter, 1);
            p = __builtin_amdgcn_readfirstlane(__shfl(p, 0));
            if (p >= a.total_tiles) break;
            const DevView* V = find_view_by_tile(a, p);
            march_packet<MODE, DT, SPARSE>(a, V, p - V->tile_begin, lane);
        }
        return;
    }
    int packet;
    xcd_packet(&packet, waves, wave);
    packet = __builtin_amdgcn_readfirstlane(packet);
    if (packet >= a.total_tiles) return;
    if (a.only_view >= 0) {
        const DevView* V = a.views + a.only_view;
        march_packet<MODE, DT, SPARSE>(a, V, packet, lane);
        return;
    }
    const DevView* V = find_view_by_tile(a, packet);
    march_packet<MODE, DT, SPARSE>(a, V, packet - V->tile_begin, lane);
}

hipError_t launch_march(const MarchArgs& a, int waves, hipStream_t s) {
    int total = a.total_tiles;
    if (a.only_view >= 0) total = a.total_tiles;  // tiles of that view only
    if (total <= 0) return hipSuccess;
    dim3 block(64 * waves);
    dim3 grid;
    if (a.persistent) {
        int dev = 0, cus = 256;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        const int per_cu = 16 / waves;  // four waves per SIMD
        grid = dim3(cus * per_cu);
    } else {
        grid = dim3((total + waves - 1) / waves);
    }
    const int dt = a.blocks_dtype;
    if (a.mode == 1) {
        if (dt == 1)
            hipLaunchKernelGGL((march_fwd_kernel<1, 1, false>), grid, block, 0, s, a);
        else if (a.use_sparse)
            hipLaunchKernelGGL((march_fwd_kernel<1, 0, true>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((march_fwd_kernel<1, 0, false>), grid, block, 0, s, a);
    } else {
        if (dt == 1)
            hipLaunchKernelGGL((march_fwd_kernel<0, 1, false>), grid, block, 0, s, a);
        else if (a.use_sparse)
            hipLaunchKernelGGL((march_fwd_kernel<0, 0, true>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((march_fwd_kernel<0, 0, false>), grid, block, 0, s, a);
    }
    return hipGetLastError();
}

__global__ void reset_counter_kernel(int32_t* c) {
    if (threadIdx.x == 0) c[0] = 0;
}

hipError_t launch_reset_counter(int32_t* counter, hipStream_t s) {
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, counter);
    return hipGetLastError();
}

__global__ void clear_aux_kernel(float4* aux, int64_t n_pix) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_pix) {
        aux[2 * i] = make_float4(0.f, 0.f, 0.f, 0.f);
        aux[2 * i + 1] = make_float4(0.f, 0.f, 0.f, 1.f);
    }
}

hipError_t launch_clear_aux(float* aux, int64_t n_pix, hipStream_t s) {
    if (n_pix <= 0) return hipSuccess;
    hipLaunchKernelGGL(clear_aux_kernel, dim3((unsigned)((n_pix + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<float4*>(aux), n_pix);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// occupancy (conservative max-bound rule)
// ---------------------------------------------------------------------------

__device__ inline float texel0(const DevBlock* B, int tex, int idx) {
    const void* base = tex == 0 ? B->grid : B->plane[tex - 1];
    if (B->dtype == 0) {
        const float q = (float)reinterpret_cast<const uint8_t*>(base)[(size_t)idx * 8];
        const float m = q * B->scale[tex][0];
        return m + B->offset[tex][0];
    }
    return reinterpret_cast<const float*>(base)[(size_t)idx * 8];
}

__global__ void occupancy_kernel(const DevBlock* blocks, int entry) {
    const DevBlock* B = blocks + entry;
    const int O = B->O, R = B->R, Rp = B->Rp;
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= O * O * O) return;
    const int c3[3] = {cell % O, (cell / O) % O, cell / (O * O)};
    const int s = R / O, sp = Rp / O;
    int glo[3], ghi[3], plo[3], phi[3];
    for (int a = 0; a < 3; ++a) {
        glo[a] = max(c3[a] * s - 1, 0);
        ghi[a] = min((c3[a] + 1) * s, R - 1);
        plo[a] = max(c3[a] * sp - 1, 0);
        phi[a] = min((c3[a] + 1) * sp, Rp - 1);
    }
    float mg = -INFINITY;
    for (int z = glo[2]; z <= ghi[2]; ++z)
        for (int y = glo[1]; y <= ghi[1]; ++y)
            for (int x = glo[0]; x <= ghi[0]; ++x) mg = fmaxf(mg, texel0(B, 0, (z * R + y) * R + x));
    const int au[3] = {0, 0, 1}, av[3] = {1, 2, 2};
    float mp[3];
    for (int p = 0; p < 3; ++p) {
        float m = -INFINITY;
        for (int v = plo[av[p]]; v <= phi[av[p]]; ++v)
            for (int u = plo[au[p]]; u <= phi[au[p]]; ++u) m = fmaxf(m, texel0(B, 1 + p, v * Rp + u));
        mp[p] = m;
    }
    // density 0.01 in pre-activation units: fp32 nearest to ln(0.01)
    const float thresh = -0x1.26bb1cp+2f;
    const float bound = ((mg + mp[0]) + mp[1]) + mp[2];
    const_cast<uint8_t*>(B->occ)[cell] = bound > thresh ? 1 : 0;
}

hipError_t launch_occupancy(const DevBlock* blocks, int entry, int O, hipStream_t s) {
    const int n = O * O * O;
    hipLaunchKernelGGL(occupancy_kernel, dim3((n + 63) / 64), dim3(64), 0, s, blocks, entry);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sparse bricks: copy each occupied cell's interpolation support
// ---------------------------------------------------------------------------

__global__ void pack_bricks_kernel(const DevBlock* blocks, int entry) {
    const DevBlock* B = blocks + entry;
    const int O = B->O, R = B->R, s = R / O, s2 = s + 2;
    const int cell = blockIdx.x;
    const int slot = B->brick_slot[cell];
    if (slot < 0) return;
    const int cx = cell % O, cy = (cell / O) % O, cz = cell / (O * O);
    const uint2* G = reinterpret_cast<const uint2*>(B->grid);
    uint2* dst = reinterpret_cast<uint2*>(const_cast<uint8_t*>(B->bricks)) + (size_t)slot * (s2 * s2 * s2);
    for (int t = threadIdx.x; t < s2 * s2 * s2; t += blockDim.x) {
        const int bx = t % s2, by = (t / s2) % s2, bz = t / (s2 * s2);
        const int x = min(max(cx * s - 1 + bx, 0), R - 1);
        const int y = min(max(cy * s - 1 + by, 0), R - 1);
        const int z = min(max(cz * s - 1 + bz, 0), R - 1);
        dst[t] = G[(z * R + y) * R + x];
    }
}

hipError_t launch_pack_bricks(const DevBlock* blocks, int entry, int O, int, const int32_t*,
                              hipStream_t st) {
    hipLaunchKernelGGL(pack_bricks_kernel, dim3(O * O * O), dim3(256), 0, st, blocks, entry);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// deferred MLP on MFMA: x = [C_d, F, d] -> 16 -> 16 -> 3, C = C_d + sigmoid(z)
// ---------------------------------------------------------------------------
//
// v_mfma_f32_16x16x4f32 computes D[16][16] += A[16][4] B[4][16]; lane l
// supplies A[l%16][l/16] and B[l/16][l%16] and holds D[4(l/16)+r][l%16].
// Each layer is computed transposed, H^T = W X^T, with pixels along the 16
// columns; for layers 2 and 3 the K index of (step s, lane group g) is 4g+s,
// so the B operand is exactly the lane's own previous-layer output.

__device__ inline int64_t view_of_pixel(const DevView* views, int n_views, int64_t p) {
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].pix_begin <= p)
            lo = mid;
        else
            hi = mid - 1;
    }
    return lo;
}

__device__ inline void pixel_direction(const DevView* views, int n_views, int64_t p, float d[3]) {
    const DevView* V = views + view_of_pixel(views, n_views, p);
    const int64_t li = p - V->pix_begin;
    const int ly = (int)(li / V->w), lx = (int)(li - (int64_t)ly * V->w);
    ray_direction(V, V->x0 + lx, V->y0 + ly, d);
}

__global__ __launch_bounds__(256) void mlp_fwd_kernel(MlpArgs a) {
    __shared__ float W[kMlpParams + 1];
    __shared__ float X[4][64][11];
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) W[i] = a.mlp[i];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 64;
    const int64_t pix = base + lane;
    float x[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (pix < a.n_pix) {
        const float4 lo = reinterpret_cast<const float4*>(a.aux)[2 * pix];
        const float4 hi = reinterpret_cast<const float4*>(a.aux)[2 * pix + 1];
        x[0] = lo.x, x[1] = lo.y, x[2] = lo.z, x[3] = lo.w, x[4] = hi.x, x[5] = hi.y, x[6] = hi.z;
        pixel_direction(a.views, a.n_views, pix, x + 7);
    }
#pragma unroll
    for (int k = 0; k < 10; ++k) X[wave][lane][k] = x[k];
    __syncthreads();
    const float *W1 = W, *b1 = W + 160, *W2 = W + 176, *b2 = W + 432, *W3 = W + 448, *b3 = W + 496;
    const int j = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        floatx4 h = {b1[4 * g + 0], b1[4 * g + 1], b1[4 * g + 2], b1[4 * g + 3]};
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int k = g + 4 * s;
            const float av = k < 10 ? W1[j * 10 + k] : 0.0f;
            const float bv = k < 10 ? X[wave][16 * t + j][k] : 0.0f;
            h = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, h, 0, 0, 0);
        }
        floatx4 h2 = {b2[4 * g + 0], b2[4 * g + 1], b2[4 * g + 2], b2[4 * g + 3]};
#pragma unroll
        for (int s = 0; s < 4; ++s)
            h2 = __builtin_amdgcn_mfma_f32_16x16x4f32(W2[j * 16 + 4 * g + s], fmaxf(h[s], 0.0f), h2, 0, 0, 0);
        floatx4 z = {0.0f, 0.0f, 0.0f, 0.0f};
        if (g == 0) z = floatx4{b3[0], b3[1], b3[2], 0.0f};
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const float av = j < 3 ? W3[j * 16 + 4 * g + s] : 0.0f;
            z = __builtin_amdgcn_mfma_f32_16x16x4f32(av, fmaxf(h2[s], 0.0f), z, 0, 0, 0);
        }
        const int64_t p = base + 16 * t + j;
        if (g == 0 && p < a.n_pix) {
            const float* xp = X[wave][16 * t + j];
            a.rgb[3 * p + 0] = xp[0] + sigmoidf_(z[0]);
            a.rgb[3 * p + 1] = xp[1] + sigmoidf_(z[1]);
            a.rgb[3 * p + 2] = xp[2] + sigmoidf_(z[2]);
        }
    }
}

hipError_t launch_mlp(const MlpArgs& a, hipStream_t s) {
    if (a.n_pix <= 0) return hipSuccess;
    const int64_t blocks = (a.n_pix + 255) / 256;
    hipLaunchKernelGGL(mlp_fwd_kernel, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace cow

namespace cow {

// ---------------------------------------------------------------------------
// backward: deferred MLP (recompute from aux), then the march adjoint
// ---------------------------------------------------------------------------
//
// MLP backward, one pixel per lane: recompute h1, h2, z, then
//   dz = g * s (1 - s),  dh2 = (W3^T dz) [pre2 > 0],  dh1 = (W2^T dh2) [pre1 > 0],
//   u = W1^T dh1 (first 7 inputs) + g on the C_d inputs (C = C_d + ...).
// Weight gradients are sums over pixels of outer products, i.e. GEMMs with
// the pixels as the reduction dimension: each wave runs them on MFMA with
// K = 4 pixels per instruction and keeps the accumulators across its
// grid-stride loop; one set of atomics per workgroup at the end.

__global__ __launch_bounds__(256) void mlp_bwd_kernel(MlpBwdArgs a) {
    __shared__ float W[kMlpParams + 1];
    __shared__ float S_dh1[4][64][17];
    __shared__ float S_x[4][64][17];
    __shared__ float S_dh2[4][64][17];
    __shared__ float S_h1[4][64][17];
    __shared__ float S_dz[4][64][4];
    __shared__ float S_h2[4][64][17];
    __shared__ float S_red[4][kMlpParams + 1];
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) W[i] = a.mlp[i];
    __syncthreads();
    const float *W1 = W, *b1 = W + 160, *W2 = W + 176, *b2 = W + 432, *W3 = W + 448, *b3 = W + 496;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = lane & 15, g = lane >> 4;
    floatx4 acc1 = {0, 0, 0, 0}, acc2 = {0, 0, 0, 0}, acc3 = {0, 0, 0, 0};
    float bias_acc = 0.0f;  // lanes 0..15: db2[lane]; lanes 16..18: db3[lane-16]
    const int64_t n_chunks = (a.n_pix + 63) / 64;
    for (int64_t chunk = (int64_t)blockIdx.x * 4 + wave; chunk < n_chunks; chunk += (int64_t)gridDim.x * 4) {
        const int64_t pix = chunk * 64 + lane;
        const bool act = pix < a.n_pix;
        float x[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0}, gr[3] = {0, 0, 0};
        if (act) {
            const float4 lo = reinterpret_cast<const float4*>(a.aux)[2 * pix];
            const float4 hi = reinterpret_cast<const float4*>(a.aux)[2 * pix + 1];
            x[0] = lo.x, x[1] = lo.y, x[2] = lo.z, x[3] = lo.w, x[4] = hi.x, x[5] = hi.y, x[6] = hi.z;
            pixel_direction(a.views, a.n_views, pix, x + 7);
            gr[0] = a.grad_rgb[3 * pix], gr[1] = a.grad_rgb[3 * pix + 1], gr[2] = a.grad_rgb[3 * pix + 2];
        }
        float pre1[16], h1[16], pre2[16], h2[16], dz[3], dh2[16], dh1[16];
        for (int o = 0; o < 16; ++o) {
            float s = b1[o];
            for (int i = 0; i < 10; ++i) s = fmaf(W1[o * 10 + i], x[i], s);
            pre1[o] = s;
            h1[o] = fmaxf(s, 0.0f);
        }
        for (int o = 0; o < 16; ++o) {
            float s = b2[o];
            for (int i = 0; i < 16; ++i) s = fmaf(W2[o * 16 + i], h1[i], s);
            pre2[o] = s;
            h2[o] = fmaxf(s, 0.0f);
        }
        for (int o = 0; o < 3; ++o) {
            float s = b3[o];
            for (int i = 0; i < 16; ++i) s = fmaf(W3[o * 16 + i], h2[i], s);
            const float sg = sigmoidf_(s);
            dz[o] = act ? gr[o] * sg * (1.0f - sg) : 0.0f;
        }
        for (int i = 0; i < 16; ++i) {
            float s = 0.0f;
            for (int o = 0; o < 3; ++o) s = fmaf(W3[o * 16 + i], dz[o], s);
            dh2[i] = pre2[i] > 0.0f ? s : 0.0f;
        }
        for (int i = 0; i < 16; ++i) {
            float s = 0.0f;
            for (int o = 0; o < 16; ++o) s = fmaf(W2[o * 16 + i], dh2[o], s);
            dh1[i] = pre1[i] > 0.0f ? s : 0.0f;
        }
        if (act) {
            float u[8];
            for (int i = 0; i < 7; ++i) {
                float s = 0.0f;
                for (int o = 0; o < 16; ++o) s = fmaf(W1[o * 10 + i], dh1[o], s);
                u[i] = s + (i < 3 ? gr[i] : 0.0f);
            }
            u[7] = 0.0f;
            float4* u4 = reinterpret_cast<float4*>(a.u);
            u4[2 * pix] = make_float4(u[0], u[1], u[2], u[3]);
            u4[2 * pix + 1] = make_float4(u[4], u[5], u[6], u[7]);
        }
        // stage per-pixel vectors for the outer-product GEMMs
        for (int i = 0; i < 16; ++i) {
            S_dh1[wave][lane][i] = dh1[i];
            S_dh2[wave][lane][i] = dh2[i];
            S_h1[wave][lane][i] = h1[i];
            S_h2[wave][lane][i] = h2[i];
            S_x[wave][lane][i] = i < 10 ? x[i] : (i == 10 && act ? 1.0f : 0.0f);
        }
        for (int i = 0; i < 3; ++i) S_dz[wave][lane][i] = dz[i];
        S_dz[wave][lane][3] = 0.0f;
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        for (int s = 0; s < 16; ++s) {
            const int p = 4 * s + g;  // pixel of this lane's K slot
            acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(S_dh1[wave][p][j], S_x[wave][p][j], acc1, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_16x16x4f32(S_dh2[wave][p][j], S_h1[wave][p][j], acc2, 0, 0, 0);
            const float a3 = j < 3 ? S_dz[wave][p][j] : 0.0f;
            acc3 = __builtin_amdgcn_mfma_f32_16x16x4f32(a3, S_h2[wave][p][j], acc3, 0, 0, 0);
        }
        if (lane < 16) {
            float s = 0.0f;
            for (int p = 0; p < 64; ++p) s += S_dh2[wave][p][lane];
            bias_acc += s;
        } else if (lane < 19) {
            float s = 0.0f;
            for (int p = 0; p < 64; ++p) s += S_dz[wave][p][lane - 16];
            bias_acc += s;
        }
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
    }
    // per-wave partial gradients -> LDS -> workgroup sum -> global atomics
    float* red = S_red[wave];
    for (int r = 0; r < 4; ++r) {
        const int i = 4 * g + r;
        if (j < 10) red[i * 10 + j] = acc1[r];
        if (j == 10) red[160 + i] = acc1[r];
        red[176 + i * 16 + j] = acc2[r];
        if (i < 3) red[448 + i * 16 + j] = acc3[r];
    }
    if (lane < 16) red[432 + lane] = bias_acc;
    if (lane >= 16 && lane < 19) red[496 + lane - 16] = bias_acc;
    __syncthreads();
    for (int i = threadIdx.x; i < kMlpParams; i += blockDim.x) {
        const float s = ((S_red[0][i] + S_red[1][i]) + S_red[2][i]) + S_red[3][i];
        atomicAdd(a.grad_mlp + i, s);
    }
}

hipError_t launch_mlp_bwd(const MlpBwdArgs& a, hipStream_t s) {
    if (a.n_pix <= 0) return hipSuccess;
    const int64_t chunks = (a.n_pix + 63) / 64;
    int64_t groups = (chunks + 3) / 4;
    if (groups > 1024) groups = 1024;
    hipLaunchKernelGGL(mlp_bwd_kernel, dim3((unsigned)groups), dim3(256), 0, s, a);
    return hipGetLastError();
}

// March adjoint, one ray per lane, samples recomputed in the forward order.
// With v_k = (c_k, f_k), u = dL/dA, A the ray's final (C_d, F), A_{<=k} the
// running prefix and T_{k+1} the transmittance after sample k:
//   dL/dsigma_k = delta (T_{k+1} u.v_k - u.(A - A_{<=k})) - delta T_N dL/dT_N
//   dL/draw_0   = sigma_k dL/dsigma_k
//   dL/draw_c   = w_k u_c s (1 - s)        (c >= 1, s = sigmoid(raw_c))
// then each texel receives its interpolation weight times dL/draw (fp32
// atomics).  The block merge is the same monolithic sequence in block order
// (Appendix A), so one running prefix serves all blocks.
template <int MODE>
__device__ void march_bwd_packet(const BwdArgs& ba, const DevView* V, int tile, int lane) {
    const MarchArgs& a = ba.m;
    const int tw = a.tile_w, th = a.tile_h;
    const int tx = tile % V->tiles_x, ty = tile / V->tiles_x;
    const int px = V->x0 + tx * tw + (lane % tw);
    const int py = V->y0 + ty * th + (lane / tw);
    const bool active = px < V->x0 + V->w && py < V->y0 + V->h;
    RayState s;
    ray_direction(V, px, py, s.d);
    s.o[0] = V->eye[0];
    s.o[1] = V->eye[1];
    s.o[2] = V->eye[2];
    s.hit = active;
    s.w0 = 0;
    s.w1 = 0;
    if (MODE == 1 && active) {
        int ka, kb;
        box_interval(s.o, s.d, a.delta, 1.0f / a.delta, a.scene_lo, a.scene_hi, &ka, &kb);
        s.hit = ka < kb;
        s.w0 = ka;
        s.w1 = ka + a.max_steps;
    }
    const int64_t pix = V->pix_begin + (int64_t)(py - V->y0) * V->w + (px - V->x0);
    float Af[7] = {0, 0, 0, 0, 0, 0, 0}, TN = 1.0f, u[7] = {0, 0, 0, 0, 0, 0, 0}, gT = 0.0f;
    if (active) {
        const float4 lo = reinterpret_cast<const float4*>(a.aux)[2 * pix];
        const float4 hi = reinterpret_cast<const float4*>(a.aux)[2 * pix + 1];
        Af[0] = lo.x, Af[1] = lo.y, Af[2] = lo.z, Af[3] = lo.w, Af[4] = hi.x, Af[5] = hi.y, Af[6] = hi.z;
        TN = hi.w;
        const float4 ulo = reinterpret_cast<const float4*>(ba.u)[2 * pix];
        const float4 uhi = reinterpret_cast<const float4*>(ba.u)[2 * pix + 1];
        u[0] = ulo.x, u[1] = ulo.y, u[2] = ulo.z, u[3] = ulo.w, u[4] = uhi.x, u[5] = uhi.y, u[6] = uhi.z;
        if (ba.grad_trans) gT = ba.grad_trans[pix];
    }
    float Ap[7] = {0, 0, 0, 0, 0, 0, 0}, Tg = 1.0f;
    const float tn_term = TN * gT;
    for (int r = 0; r < V->set_n; ++r) {
        const int e = __builtin_amdgcn_readfirstlane(a.refs[V->set_begin + r]);
        const DevBlock* B = a.blocks + e;
        float* gg = ba.grad_grid[e];
        float* gp0 = ba.grad_plane[3 * e + 0];
        float* gp1 = ba.grad_plane[3 * e + 1];
        float* gp2 = ba.grad_plane[3 * e + 2];
        int ka = 0, kb = 0;
        float tn = 0.0f, dr = 0.0f;
        if (MODE == 1) {
            if (s.hit) {
                box_interval(s.o, s.d, a.delta, 1.0f / a.delta, B->lo, B->hi, &ka, &kb);
                ka = ka > s.w0 ? ka : s.w0;
                kb = kb < s.w1 ? kb : s.w1;
            }
        } else {
            float tf;
            if (s.hit && slab_exact(s.o, s.d, B->lo, B->hi, &tn, &tf)) {
                dr = (tf - tn) / (float)a.n_steps;
                kb = a.n_steps;
            }
        }
        if (!__any(ka < kb)) continue;
        const float delta = MODE == 1 ? a.delta : dr;
        int k = ka;
        for (;;) {
            bool have = false;
            float q[3];
            while (k < kb) {
                const float t = MODE == 1 ? step_t(k, a.delta) : tn + ((float)k + 0.5f) * dr;
                float p[3];
                bool in = true;
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    p[c] = coord(s.o[c], t, s.d[c]);
                    if (MODE == 0) in = in && (B->lo[c] <= p[c] && p[c] < B->hi[c]);
                    q[c] = p[c] - B->lo[c];
                }
                if (in && B->occ[occ_index(B, q)]) {
                    have = true;
                    break;
                }
                ++k;
            }
            if (!__any(have)) break;
            if (have) {
                Taps T;
                sample_taps(B->R, B->Rp, q, T);
                float raw[8];
                raw_f32(B, q, raw, T);
                const float sigma = __expf(raw[0]);
                const float e = __expf(-sigma * delta);
                const float w = Tg * (1.0f - e);
                float v[7];
                float uv = 0.0f, us = 0.0f;
#pragma unroll
                for (int c = 0; c < 7; ++c) {
                    v[c] = sigmoidf_(raw[1 + c]);
                    Ap[c] = fmaf(w, v[c], Ap[c]);
                    uv = fmaf(u[c], v[c], uv);
                    us = fmaf(u[c], Af[c] - Ap[c], us);
                }
                const float Tn = Tg * e;
                const float dsig = delta * (Tn * uv - us) - delta * tn_term;
                float draw[8];
                draw[0] = sigma * dsig;
#pragma unroll
                for (int c = 0; c < 7; ++c) draw[1 + c] = w * u[c] * v[c] * (1.0f - v[c]);
                if (gg) {
#pragma unroll
                    for (int t8 = 0; t8 < 8; ++t8) {
                        float* dst = gg + (size_t)T.idx[t8] * 8;
#pragma unroll
                        for (int c = 0; c < 8; ++c) atomicAdd(dst + c, T.w[t8] * draw[c]);
                    }
                }
                float* planes[3] = {gp0, gp1, gp2};
#pragma unroll
                for (int pl = 0; pl < 3; ++pl) {
                    if (!planes[pl]) continue;
#pragma unroll
                    for (int t4 = 0; t4 < 4; ++t4) {
                        float* dst = planes[pl] + (size_t)T.idx[8 + 4 * pl + t4] * 8;
                        const float wt = T.w[8 + 4 * pl + t4];
#pragma unroll
                        for (int c = 0; c < 8; ++c) atomicAdd(dst + c, wt * draw[c]);
                    }
                }
                Tg = Tn;
                ++k;
            }
        }
    }
}

template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2)))
void march_bwd_kernel(BwdArgs ba) {
    const MarchArgs& a = ba.m;
    const int lane = threadIdx.x & 63;
    const int waves = blockDim.x >> 6;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int packet;
    xcd_packet(&packet, waves, wave);
    packet = __builtin_amdgcn_readfirstlane(packet);
    if (packet >= a.total_tiles) return;
    const DevView* V = find_view_by_tile(a, packet);
    march_bwd_packet<MODE>(ba, V, packet - V->tile_begin, lane);
}

hipError_t launch_march_bwd(const BwdArgs& a, int waves, hipStream_t s) {
    if (a.m.total_tiles <= 0) return hipSuccess;
    dim3 block(64 * waves), grid((a.m.total_tiles + waves - 1) / waves);
    if (a.m.mode == 1)
        hipLaunchKernelGGL(march_bwd_kernel<1>, grid, block, 0, s, a);
    else
        hipLaunchKernelGGL(march_bwd_kernel<0>, grid, block, 0, s, a);
    return hipGetLastError();
}

}  // namespace cow
