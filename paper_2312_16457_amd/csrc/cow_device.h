// Device helpers shared by the forward and backward march kernels:
// exact fp32 decision sequences, the step-interval search, texture taps,
// and wave-uniform block / view descriptors held in scalar registers.
//
// Every translation unit that includes this is compiled with
// -ffp-contract=off and correctly rounded fp32 divide/sqrt, so each decision
// below is one fixed sequence of IEEE fp32 operations; continuous arithmetic
// asks for fusion explicitly with fmaf.
#pragma once

#include <hip/hip_runtime.h>

#include "cow_internal.h"

namespace cow {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// wave-uniform values: readfirstlane puts them in scalar registers, so a
// buffer resource built from them needs no per-lane waterfall
// ---------------------------------------------------------------------------
__device__ inline int ufl(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ inline float uff(float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); }
template <class T>
__device__ inline T* ufp(T* p) {
    const uint64_t v = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return reinterpret_cast<T*>(((uint64_t)hi << 32) | lo);
}

// Buffer resource: base in scalar registers, 32-bit byte offsets per lane,
// hardware range check (reads outside [0, bytes) return zero).
__device__ inline __amdgpu_buffer_rsrc_t tex_rsrc(const void* base, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ inline uint2 ld8(__amdgpu_buffer_rsrc_t r, int byte_off) {
    auto v = __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0);
    return make_uint2(v[0], v[1]);
}

__device__ inline float ld4(__amdgpu_buffer_rsrc_t r, int byte_off) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, byte_off, 0, 0));
}

__device__ inline float4 ld16(__amdgpu_buffer_rsrc_t r, int byte_off) {
    auto v = __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 0);
    return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]),
                       __uint_as_float(v[3]));
}

// ---------------------------------------------------------------------------
// view (camera) of a ray packet
// ---------------------------------------------------------------------------
struct ViewU {
    float eye[3], R[9], fx, fy, cx, cy;
    int x0, y0, w, h, tiles_x, set_begin, set_n;
    int64_t pix_begin;
};

__device__ inline void load_view(const DevView* V, ViewU& v) {
    for (int c = 0; c < 3; ++c) v.eye[c] = uff(V->eye[c]);
    for (int c = 0; c < 9; ++c) v.R[c] = uff(V->R[c]);
    v.fx = uff(V->fx), v.fy = uff(V->fy), v.cx = uff(V->cx), v.cy = uff(V->cy);
    v.x0 = ufl(V->x0), v.y0 = ufl(V->y0), v.w = ufl(V->w), v.h = ufl(V->h);
    v.tiles_x = ufl(V->tiles_x), v.set_begin = ufl(V->set_begin), v.set_n = ufl(V->set_n);
    const uint64_t pb = (uint64_t)V->pix_begin;
    v.pix_begin = (int64_t)(((uint64_t)(uint32_t)ufl((int)(pb >> 32)) << 32) | (uint32_t)ufl((int)pb));
}

// Pixel ray r(t) = o + t d (Sec. 3): d is the normalised camera-to-world
// rotation of (x, y, 1), x = (i + 1/2 - cx) / fx, y = (j + 1/2 - cy) / fy.
template <class V>
__device__ inline void ray_direction(const V& v, int i, int j, float d[3]) {
    float x = ((float)i + 0.5f - v.cx) / v.fx;
    float y = ((float)j + 0.5f - v.cy) / v.fy;
    float u[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float a = v.R[3 * c + 0] * x;
        float b = v.R[3 * c + 1] * y;
        u[c] = (a + b) + v.R[3 * c + 2];
    }
    float n = sqrtf((u[0] * u[0] + u[1] * u[1]) + u[2] * u[2]);
#pragma unroll
    for (int c = 0; c < 3; ++c) d[c] = u[c] / n;
}

// ---------------------------------------------------------------------------
// camera-anchored steps and their block intervals
// ---------------------------------------------------------------------------

// t_k = (k + 1/2) delta, exact for k < 2^23 when delta is a power of two
__device__ inline float step_t(int k, float delta) { return ((float)k + 0.5f) * delta; }

// sample coordinate fl(o + fl(t d))
__device__ inline float coord(float o, float t, float d) {
    float td = t * d;
    return o + td;
}

// Least k in [0, kMaxStep] with pred(k), pred monotone false -> true;
// kMaxStep + 1 if none.  Exact whatever the guess: gallop from it, bisect.
template <class Pred>
__device__ inline int first_true(Pred pred, int guess) {
    guess = guess < 0 ? 0 : (guess > kMaxStep ? kMaxStep : guess);
    int lo, hi;  // pred(lo) false (lo may be -1), pred(hi) true (hi may be kMaxStep + 1)
    if (pred(guess)) {
        hi = guess;
        int step = 1;
        for (;;) {
            const int c = hi - step;
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
            const int c = lo + step;
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
        const int mid = lo + ((hi - lo) >> 1);
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
// [lo, hi) on every axis: [*ka, *kb) (empty when *ka >= *kb).  Each axis
// predicate is monotone in k (t_k and both roundings are monotone), so the
// set is an intersection of prefixes and suffixes.
__device__ inline void box_interval(const float o[3], const float d[3], float delta, const float lo[3],
                                          const float hi[3], int* ka, int* kb) {
    const float inv_delta = 1.0f / delta;
    int a = 0, b = kMaxStep + 1;
    for (int c = 0; c < 3; ++c) {
        const float oc = o[c], dc = d[c], l = lo[c], h = hi[c];
        if (dc == 0.0f) {
            if (!(l <= oc && oc < h)) b = 0;
            continue;
        }
        const float r = __builtin_amdgcn_rcpf(dc);
        const int gl = guess_index(((l - oc) * r) * inv_delta - 0.5f);
        const int gh = guess_index(((h - oc) * r) * inv_delta - 0.5f);
        int e, x;
        if (dc > 0.0f) {
            e = first_true([&](int k) { return coord(oc, step_t(k, delta), dc) >= l; }, gl);
            x = first_true([&](int k) { return coord(oc, step_t(k, delta), dc) >= h; }, gh);
        } else {
            e = first_true([&](int k) { return coord(oc, step_t(k, delta), dc) < h; }, gh);
            x = first_true([&](int k) { return coord(oc, step_t(k, delta), dc) < l; }, gl);
        }
        a = e > a ? e : a;
        b = x < b ? x : b;
    }
    *ka = a;
    *kb = b;
}

// slab test against the closed box, t_near clamped at 0 (chord mode)
__device__ inline bool slab_exact(const float o[3], const float d[3], const float lo[3], const float hi[3],
                                  float* tn, float* tf) {
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

// ---------------------------------------------------------------------------
// one (block, LOD) of the march, wave-uniform
// ---------------------------------------------------------------------------
struct BlockU {
    __amdgpu_buffer_rsrc_t tex[4];  // grid, xy, xz, yz
    uint64_t tp[4];                 // the same textures' addresses (uint8 path, global loads)
    __amdgpu_buffer_rsrc_t brick;   // packed grid bricks (sparse)
    const uint8_t* occ;
    uint64_t skip;                  // address of the per-cell skip levels (0 occupied, else 1 + the
                                    // coarsest empty level), read with global loads
    const int32_t* slot;
    int R, Rp, O;                   // texels (cells) per unit length
    int gd[3], pd[3], od[3];        // texels (cells) along x, y, z
    int lgx, lgy, lpx, lpy, lox, loy;  // log2 of the row lengths used in indexing
    float lo[3], hi[3];
    const float* dec;               // uint8 decode: DevBlock::dsc, then dosum (40 floats)
    int contracted;                 // texture space is the contracted cube of the box
};

__device__ inline uint32_t grid_texels(const BlockU& b) { return (uint32_t)b.gd[0] * b.gd[1] * b.gd[2]; }
// planes xy, xz, yz: (u, v) = (x, y), (x, z), (y, z)
__device__ inline uint32_t plane_texels(const BlockU& b, int p) {
    return p == 0 ? (uint32_t)b.pd[0] * b.pd[1] : (p == 1 ? (uint32_t)b.pd[0] * b.pd[2] : (uint32_t)b.pd[1] * b.pd[2]);
}

constexpr float kLog2e = 1.44269504088896341f;

template <int DT>
__device__ inline void load_block(const DevBlock* B, BlockU& b) {
    b.R = ufl(B->R), b.Rp = ufl(B->Rp), b.O = ufl(B->O);
    for (int c = 0; c < 3; ++c) b.gd[c] = ufl(B->gd[c]), b.pd[c] = ufl(B->pd[c]), b.od[c] = ufl(B->od[c]);
    b.lgx = 31 - __builtin_clz((unsigned)b.gd[0]), b.lgy = 31 - __builtin_clz((unsigned)b.gd[1]);
    b.lpx = 31 - __builtin_clz((unsigned)b.pd[0]), b.lpy = 31 - __builtin_clz((unsigned)b.pd[1]);
    b.lox = 31 - __builtin_clz((unsigned)b.od[0]), b.loy = 31 - __builtin_clz((unsigned)b.od[1]);
    for (int c = 0; c < 3; ++c) b.lo[c] = uff(B->lo[c]), b.hi[c] = uff(B->hi[c]);
    const uint32_t texel = DT == 0 ? 8u : 32u;
    b.tex[0] = tex_rsrc(ufp(B->grid), grid_texels(b) * texel);
    for (int p = 0; p < 3; ++p) b.tex[1 + p] = tex_rsrc(ufp(B->plane[p]), plane_texels(b, p) * texel);
    b.tp[0] = reinterpret_cast<uint64_t>(ufp(B->grid));
    for (int p = 0; p < 3; ++p) b.tp[1 + p] = reinterpret_cast<uint64_t>(ufp(B->plane[p]));
    b.occ = ufp(B->occ);
    b.skip = reinterpret_cast<uint64_t>(ufp(B->skip));
    b.slot = ufp(B->brick_slot);
    b.brick = tex_rsrc(ufp(B->bricks), (uint32_t)ufl((int)B->brick_bytes));
    // raw_u8 returns log2(e) raw_0 and -log2(e) raw_c (c >= 1), the arguments
    // of exp2 in the activations, so the factor rides in the decode scales and
    // offsets formed at load (DevBlock::dsc, dosum); 2^24 undoes the fp16-subnormal
    // byte unpacking (bytes_even_h2, bytes_odd_h2)
    b.dec = ufp(&B->dsc[0][0]);
    b.contracted = ufl(B->contracted);
}

// Contraction (implementation details, after MERF) of the box [lo, hi) in
// fp32, the decision sequence: x = (p - centre) (2 / extent); inside the unit
// cube x itself, else x_c / m for a coordinate below m = |x|_inf and
// (2 - 1/m) sign(x_c) for one attaining it; texture space q = (y + 2) (extent / 4).
// Returns m.
__device__ inline float contract_q(const float lo[3], const float hi[3], const float p[3], float q[3]) {
    float x[3], m = 0.0f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const float ext = hi[c] - lo[c];
        const float ctr = lo[c] + 0.5f * ext;
        x[c] = (p[c] - ctr) * (2.0f / ext);
        m = fmaxf(m, fabsf(x[c]));
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float y = x[c];
        if (m > 1.0f) y = fabsf(x[c]) == m ? copysignf(2.0f - 1.0f / m, x[c]) : x[c] / m;
        q[c] = (y + 2.0f) * (0.25f * (hi[c] - lo[c]));
    }
    return m;
}

__device__ inline int occ_cell(const BlockU& b, const float q[3], int cell[3]) {
    const float Of = (float)b.O;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        // truncation equals the floor for q O >= 0, and both clamp to 0 below
        int k = (int)(q[c] * Of);
        k = k < 0 ? 0 : k;
        cell[c] = k > b.od[c] - 1 ? b.od[c] - 1 : k;
    }
    return (((cell[2] << b.loy) + cell[1]) << b.lox) + cell[0];
}

__device__ inline int occ_cell(const BlockU& b, const float q[3]) {
    int cell[3];
    return occ_cell(b, q, cell);
}

// ---------------------------------------------------------------------------
// feature gather: trilinear grid + three bilinear planes
// ---------------------------------------------------------------------------
// Clamp-to-edge linear interpolation along one axis over cell-centred
// texels (u = q R - 1/2), written as a pair of adjacent texels p, p + 1:
// weights (1 - f, f) at p = floor(u) inside the texture, all weight on
// texel 0 below the first centre and on texel R - 1 beyond the last.  The
// pair is contiguous in memory along x (grid) and u (planes), so one 16-byte
// load fetches both uint8 texels.  Needs R >= 2.
struct Lin {
    int p;
    float w0, w1;  // weights of texels p and p + 1
};

// R texels per unit length, D texels along the axis.  Clamping u to
// [0, D - 1] first gives both edge cases directly: p = 0 with f = 0 below,
// p = D - 2 with f = 1 above; inside, f = u - floor(u).
__device__ inline Lin lin_pair(float q, int R, int D) {
    // u = q R - 1/2 in one rounding (q R is exact, R a power of two), as
    // v_fmaak_f32 (a two-operand encoding with the constant as a literal):
    // the compiler's choice, v_fma_f32 with an inline constant, is a
    // three-operand instruction that issues at about 4.3 cycles against 2.7
    float u;
    asm("v_fmaak_f32 %0, %1, %2, 0xbf000000" : "=v"(u) : "v"(q), "v"((float)R));
    const float uc = __builtin_amdgcn_fmed3f(u, 0.0f, (float)(D - 1));
    const int a = (int)uc;
    Lin t;
    t.p = a < D - 2 ? a : D - 2;
    const float f = uc - (float)t.p;
    t.w0 = 1.0f - f;
    t.w1 = f;
    return t;
}

// The taps of one sample as ten pairs: 0-3 the grid rows (z0,y0), (z0,y1),
// (z1,y0), (z1,y1); 4-9 the plane rows xy v0, v1, xz v0, v1, yz v0, v1.
// w[2j] and w[2j + 1] weight texels pidx[j] and pidx[j] + 1.
struct Taps {
    int pidx[10];
    float w[20];
};

__device__ inline int pair_tex(int j) { return j < 4 ? 0 : 1 + (j - 4) / 2; }

__device__ inline void sample_taps(const BlockU& b, const float q[3], Taps& T) {
    const int R = b.R, Rp = b.Rp;
    const Lin gx = lin_pair(q[0], R, b.gd[0]), gy = lin_pair(q[1], R, b.gd[1]), gz = lin_pair(q[2], R, b.gd[2]);
    const Lin px = lin_pair(q[0], Rp, b.pd[0]), py = lin_pair(q[1], Rp, b.pd[1]), pz = lin_pair(q[2], Rp, b.pd[2]);
    const float zw[2] = {gz.w0, gz.w1}, yw[2] = {gy.w0, gy.w1};
#pragma unroll
    for (int dz = 0; dz < 2; ++dz)
#pragma unroll
        for (int dy = 0; dy < 2; ++dy) {
            const int j = dz * 2 + dy;
            const float wzy = zw[dz] * yw[dy];
            T.pidx[j] = ((((gz.p + dz) << b.lgy) + gy.p + dy) << b.lgx) + gx.p;
            T.w[2 * j] = wzy * gx.w0;
            T.w[2 * j + 1] = wzy * gx.w1;
        }
    // planes are indexed [v][u]: xy (u=x, v=y), xz (u=x, v=z), yz (u=y, v=z)
    const Lin U[3] = {px, px, py}, V[3] = {py, pz, pz};
    const int lrow[3] = {b.lpx, b.lpx, b.lpy};  // row length of each plane: its u extent
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const int j = 4 + 2 * p;
        T.pidx[j] = (V[p].p << lrow[p]) + U[p].p;
        T.pidx[j + 1] = ((V[p].p + 1) << lrow[p]) + U[p].p;
        T.w[2 * j + 0] = V[p].w0 * U[p].w0;
        T.w[2 * j + 1] = V[p].w0 * U[p].w1;
        T.w[2 * j + 2] = V[p].w1 * U[p].w0;
        T.w[2 * j + 3] = V[p].w1 * U[p].w1;
    }
}

__device__ inline uint4 ld16u(__amdgpu_buffer_rsrc_t r, int byte_off) {
    auto v = __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, 0, 0);
    return make_uint4(v[0], v[1], v[2], v[3]);
}

// 16 bytes at a wave-uniform base address plus a 32-bit lane offset: a
// global load with the base in two scalar registers (a buffer resource takes
// four).  The address is rebuilt as a global-space pointer from its integer
// value; through a generic pointer the compiler would emit a flat load.
// one byte at a wave-uniform base address plus a 32-bit lane offset (global load)
__device__ inline uint32_t ld1g(uint64_t base, uint32_t byte_off) {
    return *(const __attribute__((address_space(1))) uint8_t*)(base + byte_off);
}

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(1))) u32x4_t gu32x4_t;
__device__ inline uint4 ld16g(uint64_t base, uint32_t byte_off) {
    const u32x4_t v = *(const gu32x4_t*)(base + byte_off);
    return make_uint4(v[0], v[1], v[2], v[3]);
}

// Two bytes of a word as two fp16 subnormals, byte * 2^-24 exactly:
// v_fma_mix_f32 then multiplies them by fp32 weights with no separate
// conversion, and the 2^24 comes back, exactly, in the decode scale.  Bytes 0
// and 2 need only a mask (a 2-cycle VOP2 instruction); bytes 1 and 3 a byte
// permute (4 cycles).
typedef _Float16 h2_t __attribute__((ext_vector_type(2)));
__device__ inline h2_t bytes_even_h2(uint32_t w) { return __builtin_bit_cast(h2_t, w & 0x00ff00ffu); }
__device__ inline h2_t bytes_odd_h2(uint32_t w) {
    return __builtin_bit_cast(h2_t, __builtin_amdgcn_perm(0u, w, 0x0c030c01u));
}

// s[c] += w * byte c of one uint8 texel (two words), scaled by 2^-24
__device__ inline void fold_texel(uint32_t x, uint32_t y, float w, float s[kNch]) {
    const h2_t a = bytes_even_h2(x), b = bytes_odd_h2(x), c = bytes_even_h2(y), d = bytes_odd_h2(y);
    s[0] = fmaf(w, (float)a.x, s[0]);
    s[1] = fmaf(w, (float)b.x, s[1]);
    s[2] = fmaf(w, (float)a.y, s[2]);
    s[3] = fmaf(w, (float)b.y, s[3]);
    s[4] = fmaf(w, (float)c.x, s[4]);
    s[5] = fmaf(w, (float)d.x, s[5]);
    s[6] = fmaf(w, (float)c.y, s[6]);
    s[7] = fmaf(w, (float)d.y, s[7]);
}

typedef const __attribute__((address_space(4))) float cfloat;

// raw[c] += scale[c] * (sum over N pairs of w q[c]) for one texture (FIRST:
// raw[c] = the product, a two-operand multiply)
template <int N, bool FIRST = false>
__device__ inline void fold_u8(const uint4 (&t)[N], const float* w, const cfloat* sc, float raw[kNch]) {
    float s[kNch] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < N; ++k) {
        fold_texel(t[k].x, t[k].y, w[2 * k], s);
        fold_texel(t[k].z, t[k].w, w[2 * k + 1], s);
    }
#pragma unroll
    for (int c = 0; c < kNch; ++c) raw[c] = FIRST ? s[c] * sc[c] : fmaf(s[c], sc[c], raw[c]);
}

// Pre-activation features of a uint8 block at local coordinate q, in the
// exp2 domain of the activations: raw[0] = log2(e) x density logit, raw[c] =
// -log2(e) x feature logit (c >= 1); each is the sum over the four textures
// of scale * interpolated q, plus the offsets.  Interpolating the bytes and
// decoding once equals decoding every texel because the weights of each
// texture sum to one.
template <bool SPARSE>
__device__ inline void raw_u8(const BlockU& b, const float q[3], int cell, float raw[kNch]) {
    Taps T;
    sample_taps(b, q, T);
    uint4 g[4], p0[2], p1[2], p2[2];
    if (SPARSE) {
        // brick of (s+2)^3 texels around the sample's occupancy cell; texel j
        // of an axis holds grid index clamp(c s - 1 + j), so the pair at grid
        // index p sits at brick index p - (c s - 1) and the next one
        const int O = b.O, s = b.R / O, s2 = s + 2;
        const int cx = cell & (b.od[0] - 1), cy = (cell >> b.lox) & (b.od[1] - 1), cz = cell >> (b.lox + b.loy);
        const int base = b.slot[cell] * (s2 * s2 * s2);
        const Lin gx = lin_pair(q[0], b.R, b.gd[0]), gy = lin_pair(q[1], b.R, b.gd[1]), gz = lin_pair(q[2], b.R, b.gd[2]);
        const int xs = gx.p - (cx * s - 1), ys = gy.p - (cy * s - 1), zs = gz.p - (cz * s - 1);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            g[j] = ld16u(b.brick, 8 * (base + ((zs + (j >> 1)) * s2 + ys + (j & 1)) * s2 + xs));
    } else {
        // the other three grid rows lie one row (8 B x gd[0]), one slice
        // (8 B x gd[0] gd[1]) and both further than row 0: wave-uniform
        // strides added to one offset (two-operand adds)
        const uint32_t g0 = 8u * (uint32_t)T.pidx[0], gr = 8u << b.lgx, gs = 8u << (b.lgx + b.lgy);
        g[0] = ld16g(b.tp[0], g0);
        g[1] = ld16g(b.tp[0], g0 + gr);
        g[2] = ld16g(b.tp[0], g0 + gs);
        g[3] = ld16g(b.tp[0], g0 + (gs + gr));
    }
    // the second row of each plane footprint is one row (8 B x its u extent) further
    const uint32_t rx = 8u << b.lpx, ry = 8u << b.lpy;
    const uint32_t o0 = 8u * (uint32_t)T.pidx[4], o1 = 8u * (uint32_t)T.pidx[6], o2 = 8u * (uint32_t)T.pidx[8];
    p0[0] = ld16g(b.tp[1], o0);
    p0[1] = ld16g(b.tp[1], o0 + rx);
    p1[0] = ld16g(b.tp[2], o1);
    p1[1] = ld16g(b.tp[2], o1 + rx);
    p2[0] = ld16g(b.tp[3], o2);
    p2[1] = ld16g(b.tp[3], o2 + ry);
    // every load of the sample is issued before the first is consumed, so
    // the sample pays one memory latency
    __builtin_amdgcn_sched_barrier(0);
    // The decode constants are read sample by sample with scalar loads (the
    // block table is constant during a launch), eight at a time beside the
    // texture that uses them: each group's pointer is an opaque copy that
    // depends on the previous group's result, so the loads can neither leave
    // the march loop (the 40 wave-uniform values would then hold 40 vector
    // registers) nor gather at its top (40 scalar registers at once).  The
    // offsets come last: (((G + XY) + XZ) + YZ) + offsets, every step a
    // two-operand multiply or add with a scalar operand except the three
    // multiply-adds.
    const float* dg = b.dec;
    asm volatile("" : "+s"(dg));
    fold_u8<4, true>(g, T.w, (const cfloat*)dg, raw);
    asm volatile("" : "+s"(dg) : "v"(raw[0]));
    fold_u8<2>(p0, T.w + 8, (const cfloat*)dg + kNch, raw);
    asm volatile("" : "+s"(dg) : "v"(raw[0]));
    fold_u8<2>(p1, T.w + 12, (const cfloat*)dg + 2 * kNch, raw);
    asm volatile("" : "+s"(dg) : "v"(raw[0]));
    fold_u8<2>(p2, T.w + 16, (const cfloat*)dg + 3 * kNch, raw);
    asm volatile("" : "+s"(dg) : "v"(raw[0]));
    const cfloat* off = (const cfloat*)dg + 4 * kNch;
#pragma unroll
    for (int c = 0; c < kNch; ++c) raw[c] += off[c];
}

// fp32 block: a texel pair is 64 contiguous bytes (channels 0-3, 4-7 of each
// texel).  All 40 loads are issued before any is consumed, so one sample's
// memory latency is paid once; the four textures are then summed
// ((G + XY) + XZ) + YZ.  SPLIT: the grid's 16 loads are summed before the
// planes' 24 are issued (the same sums in the same order, 64 fewer registers
// in flight, for kernels whose other state needs them).
template <bool SPLIT = false>
__device__ inline void raw_f32(const BlockU& b, const Taps& T, float raw[kNch]) {
    float4 lo[20], hi[20];
    auto load = [&](int j) {
        const __amdgpu_buffer_rsrc_t r = b.tex[pair_tex(j)];
        const int off = 32 * T.pidx[j];
        lo[2 * j] = ld16(r, off);
        hi[2 * j] = ld16(r, off + 16);
        lo[2 * j + 1] = ld16(r, off + 32);
        hi[2 * j + 1] = ld16(r, off + 48);
    };
    auto sum = [&](int tex) {
        const int k0 = tex == 0 ? 0 : 4 + 4 * tex, n = tex == 0 ? 8 : 4;
        float a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int k = k0; k < k0 + n; ++k) {
            const float w = T.w[k];
            a[0] = fmaf(w, lo[k].x, a[0]);
            a[1] = fmaf(w, lo[k].y, a[1]);
            a[2] = fmaf(w, lo[k].z, a[2]);
            a[3] = fmaf(w, lo[k].w, a[3]);
            a[4] = fmaf(w, hi[k].x, a[4]);
            a[5] = fmaf(w, hi[k].y, a[5]);
            a[6] = fmaf(w, hi[k].z, a[6]);
            a[7] = fmaf(w, hi[k].w, a[7]);
        }
#pragma unroll
        for (int c = 0; c < 8; ++c) raw[c] = tex == 0 ? a[c] : raw[c] + a[c];
    };
    if (SPLIT) {
#pragma unroll
        for (int j = 0; j < 4; ++j) load(j);
        sum(0);
#pragma unroll
        for (int j = 4; j < 10; ++j) load(j);
#pragma unroll
        for (int tex = 1; tex < 4; ++tex) sum(tex);
    } else {
#pragma unroll
        for (int j = 0; j < 10; ++j) load(j);
#pragma unroll
        for (int tex = 0; tex < 4; ++tex) sum(tex);
    }
}

// Density channel alone of an fp32 block: the same operations, in the same
// order, as channel 0 of raw_f32, so the two agree bit for bit.
__device__ inline float raw0_f32(const BlockU& b, const Taps& T) {
    float v[20];
#pragma unroll
    for (int j = 0; j < 10; ++j) {
        const __amdgpu_buffer_rsrc_t r = b.tex[pair_tex(j)];
        v[2 * j] = ld4(r, 32 * T.pidx[j]);
        v[2 * j + 1] = ld4(r, 32 * T.pidx[j] + 32);
    }
    float raw = 0.0f;
#pragma unroll
    for (int tex = 0; tex < 4; ++tex) {
        const int k0 = tex == 0 ? 0 : 4 + 4 * tex, n = tex == 0 ? 8 : 4;
        float a = 0.0f;
#pragma unroll
        for (int k = k0; k < k0 + n; ++k) a = fmaf(T.w[k], v[k], a);
        raw = tex == 0 ? a : raw + a;
    }
    return raw;
}

// ---------------------------------------------------------------------------
// activations and opacity
// ---------------------------------------------------------------------------
__device__ inline float sigmoidf_(float x) { return __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }

// density and activated features from raw_u8's exp2-domain values:
// sigma = 2^(log2(e) raw_0), sigmoid(raw_c) = 1 / (1 + 2^(-log2(e) raw_c))
__device__ inline float density_u8(const float rawx[kNch]) { return __builtin_amdgcn_exp2f(rawx[0]); }
__device__ inline float feature_u8(const float rawx[kNch], int c) {
    return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(rawx[c]));
}

// alpha = 1 - exp(-x) for x = sigma delta >= 0 (Eq. "alpha accumulation"),
// without the cancellation of forming 1 - exp(-x) when x is small: a
// five-term series below 1/16 (truncation < 2e-9 relative).
__device__ inline float alpha_of(float x) {
    float t = fmaf(-x, 1.0f / 120.0f, 1.0f / 24.0f);
    t = fmaf(-x, t, 1.0f / 6.0f);
    t = fmaf(-x, t, 0.5f);
    t = fmaf(-x, t, 1.0f);
    const float series = x * t;
    return x < 0.0625f ? series : 1.0f - __expf(-x);
}

// Input of the deferred MLP (Eq. "deferred"): [C_d, F, PE(d)] with PE(d) =
// [d, sin(2^l d), cos(2^l d) for l < L], per component; the scaled arguments
// are exact (powers of two), sinf/cosf the accurate library versions.
template <int L>
__device__ inline void mlp_input(const float A[7], const float d[3], float* x) {
#pragma unroll
    for (int c = 0; c < 7; ++c) x[c] = A[c];
#pragma unroll
    for (int c = 0; c < 3; ++c) x[7 + c] = d[c];
#pragma unroll
    for (int l = 0; l < L; ++l)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float t = (float)(1 << l) * d[c];
            x[10 + 6 * l + c] = sinf(t);
            x[13 + 6 * l + c] = cosf(t);
        }
}

// One block's deferred shading for one lane (Eq. "deferred" per block):
// C = C_d + sigmoid(Phi(C_d, F, PE(d))), Phi NI -> 16 -> 16 -> 3 with ReLU,
// the weights laid out as in MlpShape<L> and read through a wave-uniform
// pointer (scalar loads).
template <int L>
__device__ inline void block_shade(const float* w, const float A[7], const float d[3], float C[3]) {
    using S = MlpShape<L>;
    float x[S::NI], h1[16], h2[16];
    mlp_input<L>(A, d, x);
#pragma unroll
    for (int o = 0; o < 16; ++o) {
        float a = w[S::B1 + o];
#pragma unroll
        for (int i = 0; i < S::NI; ++i) a = fmaf(w[o * S::NI + i], x[i], a);
        h1[o] = fmaxf(a, 0.0f);
    }
#pragma unroll
    for (int o = 0; o < 16; ++o) {
        float a = w[S::B2 + o];
#pragma unroll
        for (int i = 0; i < 16; ++i) a = fmaf(w[S::W2 + o * 16 + i], h1[i], a);
        h2[o] = fmaxf(a, 0.0f);
    }
#pragma unroll
    for (int o = 0; o < 3; ++o) {
        float a = w[S::B3 + o];
#pragma unroll
        for (int i = 0; i < 16; ++i) a = fmaf(w[S::W3 + o * 16 + i], h2[i], a);
        C[o] = A[o] + sigmoidf_(a);
    }
}

__device__ inline float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    return v;
}

// Adjoint of block_shade for one lane: C = A + sigmoid(Phi(A, PE(d)))
// weighted by P in the merge, g = dL/dC of the ray.  Returns C and u = dL/dA
// (with P folded in; the direction inputs are constants).  With want_gw, the
// gradient of the weights is summed over the wave and added once to gw
// (wave-collective: every lane calls it, an inactive lane with zero weight).
// wp and gwp are wave-uniform; the function is not inlined, so its arguments
// arrive in vector registers and are made scalar again here (one buffer
// resource for the weight-gradient atomics, no per-lane waterfall).
template <int L>
__device__ __attribute__((noinline)) void block_shade_adjoint(const float* wp, const float A[7], const float d[3],
                                                              float P, const float g[3], bool active, float C[3],
                                                              float u[7], float* gwp, int lane) {
    using S = MlpShape<L>;
    const float* w = ufp(wp);
    const bool want_gw = ufl(gwp != nullptr);
    float x[S::NI], h1[16], h2[16], s[3];
    mlp_input<L>(A, d, x);
#pragma unroll
    for (int o = 0; o < 16; ++o) {
        float a = w[S::B1 + o];
#pragma unroll
        for (int i = 0; i < S::NI; ++i) a = fmaf(w[o * S::NI + i], x[i], a);
        h1[o] = fmaxf(a, 0.0f);
    }
#pragma unroll
    for (int o = 0; o < 16; ++o) {
        float a = w[S::B2 + o];
#pragma unroll
        for (int i = 0; i < 16; ++i) a = fmaf(w[S::W2 + o * 16 + i], h1[i], a);
        h2[o] = fmaxf(a, 0.0f);
    }
#pragma unroll
    for (int o = 0; o < 3; ++o) {
        float a = w[S::B3 + o];
#pragma unroll
        for (int i = 0; i < 16; ++i) a = fmaf(w[S::W3 + o * 16 + i], h2[i], a);
        s[o] = sigmoidf_(a);
        C[o] = A[o] + s[o];
    }
    const float wP = active ? P : 0.0f;
    float dz[3], dh2[16], dh1[16];
#pragma unroll
    for (int o = 0; o < 3; ++o) dz[o] = wP * g[o] * s[o] * (1.0f - s[o]);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        float a = 0.0f;
#pragma unroll
        for (int o = 0; o < 3; ++o) a = fmaf(w[S::W3 + o * 16 + i], dz[o], a);
        dh2[i] = h2[i] > 0.0f ? a : 0.0f;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        float a = 0.0f;
#pragma unroll
        for (int o = 0; o < 16; ++o) a = fmaf(w[S::W2 + o * 16 + i], dh2[o], a);
        dh1[i] = h1[i] > 0.0f ? a : 0.0f;
    }
#pragma unroll
    for (int c = 0; c < 7; ++c) {
        float a = c < 3 ? wP * g[c] : 0.0f;
#pragma unroll
        for (int o = 0; o < 16; ++o) a = fmaf(w[o * S::NI + c], dh1[o], a);
        u[c] = a;
    }
    if (!want_gw) return;
    // weight gradient, in the weights' own layout: lane (i % 64) keeps the
    // wave sum of entry i in acc[i / 64]
    constexpr int NQ = (S::N + 63) / 64;
    float acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0f;
#define COW_RED(idx, val)                                   \
    {                                                       \
        const float t_ = wave_sum(val);                     \
        if (lane == ((idx) & 63)) acc[(idx) >> 6] = t_;     \
    }
#pragma unroll
    for (int o = 0; o < 16; ++o) {
#pragma unroll
        for (int i = 0; i < S::NI; ++i) COW_RED(o * S::NI + i, dh1[o] * x[i]);
        COW_RED(S::B1 + o, dh1[o]);
    }
#pragma unroll
    for (int o = 0; o < 16; ++o) {
#pragma unroll
        for (int i = 0; i < 16; ++i) COW_RED(S::W2 + o * 16 + i, dh2[o] * h1[i]);
        COW_RED(S::B2 + o, dh2[o]);
    }
#pragma unroll
    for (int o = 0; o < 3; ++o) {
#pragma unroll
        for (int i = 0; i < 16; ++i) COW_RED(S::W3 + o * 16 + i, dz[o] * h2[i]);
        COW_RED(S::B3 + o, dz[o]);
    }
#undef COW_RED
    const __amdgpu_buffer_rsrc_t gw = tex_rsrc(ufp(gwp), 4u * (uint32_t)S::N);
#pragma unroll
    for (int q = 0; q < NQ; ++q)
        if (q * 64 + lane < S::N) __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(acc[q], gw, 4 * (q * 64 + lane), 0, 0);
}

// Binary entropy of a block's opacity a = 1 - Tk (Eq. "opacity loss"), with
// a clamped to [1e-6, 1 - 1e-6] so that both logarithms stay finite; 1 - a
// is taken as Tk itself (no cancellation).  The derivative in a is
// log((1 - a) / a), zero where the clamp holds.
constexpr float kOpacityEps = 1e-6f;
__device__ inline float opacity_entropy(float Tk) {
    const float lo = kOpacityEps, hi = 1.0f - kOpacityEps;
    const float a = fminf(fmaxf(1.0f - Tk, lo), hi);
    const float b = fminf(fmaxf(Tk, lo), hi);
    return -(a * logf(a) + b * logf(b));
}
__device__ inline float opacity_dentropy(float Tk) {
    const float a = 1.0f - Tk;
    return (a > kOpacityEps && a < 1.0f - kOpacityEps) ? logf(Tk / a) : 0.0f;
}

// ---------------------------------------------------------------------------
// packets: which tile of which view a wave marches
// ---------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the 8 XCDs.  Hand each XCD
// chunks of 16 consecutive workgroups' packets (neighbouring pixels share its
// L2), with the chunks interleaved over the XCDs so that every XCD draws from
// the whole image (a contiguous range per XCD leaves the XCDs of sky rows idle).
__device__ inline int xcd_packet(int waves, int wave) {
    const int nb = gridDim.x, b = blockIdx.x, C = 16;
    const int nfull = nb / (8 * C) * (8 * C);
    int lb = b;  // tail workgroups keep their own index (still a bijection)
    if (b < nfull) {
        const int x = b & 7, j = b >> 3;
        lb = ((j / C) * 8 + x) * C + (j % C);
    }
    return lb * waves + wave;
}

// Persistent launches: one work counter per XCD.  XCD x owns interleaved
// chunks of kXcdChunk consecutive packets (chunk j belongs to XCD j mod 8;
// 256 packets are four blocks of 8 x 8 tiles, so the packets an XCD runs
// together cover a compact patch of one view), takes them in order from its own counter,
// and once they run out takes the other XCDs' packets through their
// counters.  Every packet is taken exactly once; a wave gets -1 when all
// eight counters are exhausted, so every wave reaches the exit.
constexpr int kXcds = 8, kXcdChunk = 256;
__device__ inline int64_t xcd_packet_of(int x, int i) {
    return ((int64_t)(i / kXcdChunk) * kXcds + x) * kXcdChunk + (i % kXcdChunk);
}
// lane 0 of a wave calls this; workgroups are dispatched round-robin over the
// XCDs, so blockIdx.x mod 8 is the workgroup's XCD
__device__ inline int take_packet(int32_t* counters, int total) {
    const int home = blockIdx.x & (kXcds - 1);
    for (int s = 0; s < kXcds; ++s) {
        const int x = (home + s) & (kXcds - 1);
        const int i = atomicAdd(counters + x, 1);
        // xcd_packet_of grows with i, so one index past the end exhausts x
        if (i < total) {  // xcd_packet_of(x, i) >= i
            const int64_t p = xcd_packet_of(x, i);
            if (p < total) return (int)p;
        }
    }
    return -1;
}

__device__ inline const DevView* find_view_by_tile(const DevView* views, int n_views, int packet) {
    int lo = 0, hi = n_views - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (views[mid].tile_begin <= packet)
            lo = mid;
        else
            hi = mid - 1;
    }
    return views + lo;
}

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
    ray_direction(*V, V->x0 + lx, V->y0 + ly, d);
}

// A ray packet: lane -> pixel of a tile_w x tile_h tile of the view's crop.
struct Ray {
    float o[3], d[3];
    int64_t pix;
    bool active;
};

// Packet index -> tile of a view's tx_n x ty_n tile grid, in blocks of 8 x 8
// tiles (raster order inside a block, blocks in raster order; the blocks of
// the last row and column are cut to fit).  Consecutive packets then cover a
// compact patch of the image, and the packets one XCD runs together (chunks
// of consecutive packets) share more texels in its L2 than a strip along one
// tile row would.
__device__ inline void tile_xy(int tile, int tx_n, int ty_n, int& tx, int& ty) {
    constexpr int kB = 8;
    const int bys = (ty_n - 1) / kB, row_tiles = kB * tx_n;  // last block row; tiles in a full block row
    int r = tile / row_tiles;
    r = r < bys ? r : bys;
    int q = tile - r * row_tiles;
    const int h = r < bys ? kB : ty_n - kB * bys;
    const int bxs = (tx_n - 1) / kB;
    int c = q / (h * kB);
    c = c < bxs ? c : bxs;
    q -= c * h * kB;
    const int w = c < bxs ? kB : tx_n - kB * bxs;
    ty = r * kB + q / w;
    tx = c * kB + q % w;
}

__device__ inline void packet_ray(const MarchArgs& a, const ViewU& v, int tile, int lane, Ray& r) {
    const int tw = a.tile_w, th = a.tile_h;
    int tx, ty;
    tile_xy(tile, v.tiles_x, (v.h + th - 1) / th, tx, ty);
    const int px = v.x0 + tx * tw + (lane % tw);
    const int py = v.y0 + ty * th + (lane / tw);
    r.active = px < v.x0 + v.w && py < v.y0 + v.h;
    ray_direction(v, px, py, r.d);
    r.o[0] = v.eye[0];
    r.o[1] = v.eye[1];
    r.o[2] = v.eye[2];
    r.pix = v.pix_begin + (int64_t)(py - v.y0) * v.w + (px - v.x0);
}

// Samples of one block for one lane: grid mode, the block's step interval
// clipped to the ray's window; chord mode, n_steps midpoints of the chord.
struct Span {
    int ka, kb;
    float tn, dr, delta;
};

// Per-block composites handed from the forward to the backward: slot j of
// pixel pix holds (A^k[0..6], T^k) of the j-th block of the view's set, T^k =
// -1 for a block the ray marches no sample in.
__device__ inline void put_block_aux(const MarchArgs& a, int64_t pix, int j, const float A[7], float T) {
    float4* p = reinterpret_cast<float4*>(a.block_aux + ((size_t)pix * a.block_aux_n + j) * 8);
    p[0] = make_float4(A[0], A[1], A[2], A[3]);
    p[1] = make_float4(A[4], A[5], A[6], T);
}

// Returns whether the ray marched a sample in the block; A and T are then its
// composite, else zero and 1.
__device__ inline bool get_block_aux(const MarchArgs& a, int64_t pix, int j, float A[7], float& T) {
    const float4* p = reinterpret_cast<const float4*>(a.block_aux + ((size_t)pix * a.block_aux_n + j) * 8);
    const float4 lo = p[0], hi = p[1];
    A[0] = lo.x, A[1] = lo.y, A[2] = lo.z, A[3] = lo.w, A[4] = hi.x, A[5] = hi.y, A[6] = hi.z;
    T = hi.w < 0.0f ? 1.0f : hi.w;
    return hi.w >= 0.0f;
}

template <int MODE>
__device__ inline Span block_span(const MarchArgs& a, const BlockU& b, const Ray& r, bool hit, int w0, int w1) {
    Span s{0, 0, 0.0f, 0.0f, a.delta};
    if (!hit) return s;
    if (MODE == 1) {
        box_interval(r.o, r.d, a.delta, b.lo, b.hi, &s.ka, &s.kb);
        s.ka = s.ka > w0 ? s.ka : w0;
        s.kb = s.kb < w1 ? s.kb : w1;
    } else {
        float tf;
        if (slab_exact(r.o, r.d, b.lo, b.hi, &s.tn, &tf)) {
            s.dr = (tf - s.tn) / (float)a.n_steps;
            s.delta = s.dr;
            s.kb = a.n_steps;
        }
    }
    return s;
}

// First step index after k whose sample lies outside the level-l cell of the
// occupancy pyramid that holds sample k (base cell indices ci), or kb if every
// sample up to the span's end stays inside.  On each axis the base cell index
// of a sample, trunc((fl(o + fl(t d)) - lo) O) clamped to the grid, is
// monotone in k, so "outside the cell" is a monotone predicate: walking from
// a guess (the analytic crossing of the cell's exit face) down while the
// sample before is outside and up while the sample is inside ends at its
// least k exactly, usually after one or two evaluations.  Every sample
// skipped lies in an empty pyramid cell, hence in an empty base cell, so the
// evaluated samples are those of a one-step-at-a-time march.
__device__ inline int level_exit(const BlockU& b, const Ray& r, float delta, int k, int kb, const int ci[3], int l) {
    const float Of = (float)b.O;
    // An opaque zero keeps the guess's reciprocals inside the jump: hoisted
    // out of the march loop they would hold registers across it.
    float z = 0.0f;
    asm volatile("" : "+v"(z));
    float lim[3];
    int dir[3];  // +1: leaves once u >= lim; -1: once u < lim; 0: cannot leave across this axis
    float tx = INFINITY;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const int a0 = (ci[c] >> l) << l, a1 = a0 + (1 << l);
        dir[c] = 0;
        lim[c] = 0.0f;
        if (r.d[c] > 0.0f && a1 < b.od[c]) {
            dir[c] = 1;
            lim[c] = (float)a1;
        } else if (r.d[c] < 0.0f && a0 > 0) {
            dir[c] = -1;
            lim[c] = (float)a0;
        }
        if (dir[c] != 0) {
            const float face = b.lo[c] + lim[c] * __builtin_amdgcn_rcpf(Of + z);
            tx = fminf(tx, (face - r.o[c]) * __builtin_amdgcn_rcpf(r.d[c] + z));
        }
    }
    if (dir[0] == 0 && dir[1] == 0 && dir[2] == 0) return kb;  // the cell spans the rest of the block
    auto outside = [&](int j) {
        const float t = step_t(j, delta);
        bool out = false;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float u = (coord(r.o[c], t, r.d[c]) - b.lo[c]) * Of;
            out = out || (dir[c] > 0 && u >= lim[c]) || (dir[c] < 0 && u < lim[c]);
        }
        return out;
    };
    // start at the guess, clamped to (k, kb]; walk down while the sample
    // before is already outside, then up while the sample is still inside:
    // the result is the least outside index in (k, kb), else kb
    int kx = guess_index(tx * __builtin_amdgcn_rcpf(delta + z) - 0.5f);
    kx = kx > k + 1 ? (kx < kb ? kx : kb) : k + 1;
    while (kx > k + 1 && outside(kx - 1)) --kx;
    while (kx < kb && !outside(kx)) ++kx;
    return kx;
}

// Advance k to the next occupied sample of the span (or to kb).  Loads the
// occupancy byte only when the sample's cell differs from the cached one.  In
// grid mode an empty cell is left in one jump to the first sample outside the
// coarsest empty pyramid cell around it (unless flat); the jumped samples count
// as marched, as a one-step march would count them.
// CT: the launch may hold contracted blocks, whose samples map to texture
// space through the contraction and step one at a time.
template <int MODE, bool CT = false>
__device__ inline bool next_occupied(const BlockU& b, const Ray& r, const Span& sp, int kb, float delta, bool flat,
                                     int& k, float q[3], int& cell, int& cur_cell, bool& cur_occ, int64_t& marched) {
    if (CT && b.contracted) flat = true;
    while (k < kb) {
        const float t = MODE == 1 ? step_t(k, delta) : sp.tn + ((float)k + 0.5f) * sp.dr;
        bool in = true;
        float pw[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float p = coord(r.o[c], t, r.d[c]);
            if (MODE == 0) in = in && (b.lo[c] <= p && p < b.hi[c]);
            q[c] = p - b.lo[c];
            pw[c] = p;
        }
        if (CT && b.contracted) contract_q(b.lo, b.hi, pw, q);
        if (in) {
            ++marched;
            int ci[3];
            cell = occ_cell(b, q, ci);
            if (cell != cur_cell) {
                cur_cell = cell;
                const int s = ld1g(b.skip, (uint32_t)cell);
                cur_occ = s == 0;
                if (MODE == 1 && s != 0 && !flat) {
                    const int kx = level_exit(b, r, delta, k, kb, ci, s - 1);
                    marched += kx - k - 1;
                    k = kx;
                    continue;
                }
            }
            if (cur_occ) return true;
        }
        ++k;
    }
    return false;
}

// Composite the samples of one block for one lane (Eqs. "alpha
// accumulation", "combined accumulation", "volume rendering inside
// blocks"): Ak = sum_i T_i alpha_i (c_i, f_i), Tk = prod_i (1 - alpha_i).
// Lanes advance independently through their own spans; a wave iterates
// while any lane still has an occupied sample.
// With early termination (t_min > 0) a lane stops after the first sample at
// which its transmittance T_before * Tk falls below t_min.
// JUMPS = false steps one sample at a time whatever the launch asks (the
// adjoint: its register budget has no room for the jump code, and its
// per-sample atomics dwarf the cost of an empty step).
template <int DT, int MODE, bool SPARSE, bool JUMPS = true, bool CT = false>
__device__ inline void march_block(const MarchArgs& a, const BlockU& b, const Ray& r, const Span& sp,
                                   float T_before, float Ak[7], float& Tk, int64_t& n_eval, int64_t& n_march) {
    int k = sp.ka, kb = sp.kb;
    int cur_cell = -1;
    bool cur_occ = false;
    for (;;) {
        float q[3];
        int cell = 0;
        const bool have =
            next_occupied<MODE, CT>(b, r, sp, kb, sp.delta, !JUMPS || a.flat_occ != 0, k, q, cell, cur_cell, cur_occ,
                                    n_march);
        if (!__any(have)) break;
        if (have) {
            float raw[8], v[7], sigma;
            if (DT == 0) {
                raw_u8<SPARSE>(b, q, cell, raw);
                sigma = density_u8(raw);
#pragma unroll
                for (int c = 0; c < 7; ++c) v[c] = feature_u8(raw, 1 + c);
            } else {
                Taps T;
                sample_taps(b, q, T);
                raw_f32(b, T, raw);
                sigma = __expf(raw[0]);
#pragma unroll
                for (int c = 0; c < 7; ++c) v[c] = sigmoidf_(raw[1 + c]);
            }
            const float alpha = alpha_of(sigma * sp.delta);
            const float w = Tk * alpha;
#pragma unroll
            for (int c = 0; c < 7; ++c) Ak[c] = fmaf(w, v[c], Ak[c]);
            Tk *= 1.0f - alpha;
            ++n_eval;
            ++k;
            if (T_before * Tk < a.t_min) kb = k;  // early ray termination
        }
    }
}

// Transmittance prod(1 - alpha_i) of one block for one lane of an fp32
// march, density channel only, with the forward's early-termination rule:
// the value the forward's composite of the block forms.  A lane with
// want == false marches nothing and gets 1.
template <int MODE>
__device__ inline float block_trans_f32(const BlockU& b, const Ray& r, const Span& sp, float T_before,
                                        float t_min, bool flat, bool want) {
    int k = sp.ka, kb = want ? sp.kb : sp.ka;
    int cur_cell = -1;
    bool cur_occ = false;
    int64_t unused = 0;
    float Tk = 1.0f;
    for (;;) {
        float q[3];
        int cell = 0;
        const bool have = next_occupied<MODE>(b, r, sp, kb, sp.delta, flat, k, q, cell, cur_cell, cur_occ, unused);
        if (!__any(have)) break;
        if (have) {
            Taps T;
            sample_taps(b, q, T);
            const float sigma = __expf(raw0_f32(b, T));
            Tk *= 1.0f - alpha_of(sigma * sp.delta);
            ++k;
            if (T_before * Tk < t_min) kb = k;
        }
    }
    return Tk;
}

// The ray's interval inside the footprint's column: the exact slab test on
// x and y only, t clamped at 0.
__device__ inline bool slab_xy(const float o[3], const float d[3], const float lo[3], const float hi[3], float* tn,
                               float* tf) {
    float t0 = 0.0f, t1 = INFINITY;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        if (d[c] == 0.0f) {
            if (o[c] < lo[c] || o[c] > hi[c]) return false;
            continue;
        }
        const float inv = 1.0f / d[c];
        const float a = (lo[c] - o[c]) * inv;
        const float b = (hi[c] - o[c]) * inv;
        const float mn = a < b ? a : b, mx = a < b ? b : a;
        if (mn > t0) t0 = mn;
        if (mx < t1) t1 = mx;
    }
    *tn = t0;
    *tf = t1;
    return t0 < t1;
}

// Walk of one exterior segment [t_start, t_end) of a lane's ray outside the
// scene's footprint, sampled in the contracted representation of the
// boundary block that owns each point (implementation details; Eq. "blocks"
// in the max norm, ties to the clamped unit cell).  From t the next point
// lies ext_delta m^2 further, m = max(1, |x|_inf) in the owner cell's
// normalised coordinate: about uniform steps in contracted space.  A point is
// sampled when it lies outside the footprint, within the far limit
// m <= 1/ext_delta, and its owner is a contracted block of the view's set;
// the segment after the column (post) ends at the far limit.  The forward
// and the adjoint take the same walk, so they see the same samples.
struct ExtWalk {
    float t, t_end, m_prev, cur_fx, cur_fy;
    int st;     // steps taken
    int owner;  // entry of the owner of the current cell, -1: none
    bool live, post;
};

__device__ inline void ext_begin(const MarchArgs& a, float t_start, float t_end, bool post, bool want, ExtWalk& W) {
    W.t = t_start + 0.5f * a.ext_delta;
    W.t_end = t_end;
    W.m_prev = INFINITY;
    W.cur_fx = W.cur_fy = -1.0f;
    W.st = 0;
    W.owner = -1;
    W.live = want;
    W.post = post;
}

// Advance to the segment's next sample: its texture coordinate q in the
// owner's textures (owner in W.owner) and its step w.  False once the lane's
// segment has ended (W.live is cleared by the caller on early termination).
__device__ inline bool ext_next(const MarchArgs& a, const ViewU& v, const Ray& r, ExtWalk& W, float q[3], float& w,
                                int64_t& n_march) {
    const float slo[3] = {a.scene_lo[0], a.scene_lo[1], a.scene_lo[2]};
    const float shi[3] = {a.scene_hi[0], a.scene_hi[1], a.scene_hi[2]};
    const float nxm = (shi[0] - slo[0]) - 1.0f, nym = (shi[1] - slo[1]) - 1.0f;
    const float far = 1.0f / a.ext_delta;
    while (W.live && W.st < a.ext_max_steps) {
        if (!W.post && !(W.t < W.t_end)) {
            W.live = false;
            break;
        }
        float p[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) p[c] = coord(r.o[c], W.t, r.d[c]);
        float fx = floorf(p[0] - slo[0]), fy = floorf(p[1] - slo[1]);
        fx = fx < 0.0f ? 0.0f : (fx > nxm ? nxm : fx);
        fy = fy < 0.0f ? 0.0f : (fy > nym ? nym : fy);
        const float clo[3] = {slo[0] + fx, slo[1] + fy, slo[2]};
        const float chi[3] = {clo[0] + 1.0f, clo[1] + 1.0f, shi[2]};
        float m = contract_q(clo, chi, p, q);
        if (m < 1.0f) m = 1.0f;
        w = (a.ext_delta * m) * m;
        ++W.st;
        W.t = W.t + w;
        // beyond the far limit: the segment after the column ends there,
        // the one before it once m grows past it (m is convex along a ray
        // outside the column: it never comes back)
        const bool rising = m > W.m_prev;
        W.m_prev = m;
        if (m > far) {
            if (W.post || rising) W.live = false;
            continue;
        }
        if (slo[0] <= p[0] && p[0] < shi[0] && slo[1] <= p[1] && p[1] < shi[1]) continue;
        if (fx != W.cur_fx || fy != W.cur_fy) {  // owner of the cell: a contracted block of the set
            W.cur_fx = fx, W.cur_fy = fy, W.owner = -1;
            for (int j = 0; j < v.set_n; ++j) {
                const int e = ufl(a.refs[v.set_begin + j]);
                const DevBlock* B = a.blocks + e;
                if (ufl(B->contracted) && uff(B->lo[0]) == clo[0] && uff(B->lo[1]) == clo[1]) {
                    W.owner = e;
                    break;
                }
            }
        }
        if (W.owner < 0) continue;
        ++n_march;
        return true;
    }
    return false;
}

}  // namespace cow
