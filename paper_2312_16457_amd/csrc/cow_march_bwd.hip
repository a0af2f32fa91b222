// March adjoint of the block-merged render for gfx950 (City-on-Web,
// arXiv 2312.16457): per-ray recomputation of the samples, fp32 atomic
// scatter of texel gradients.
#include <hip/hip_runtime.h>

#include "cow_device.h"

namespace cow {

// One ray per lane, samples recomputed in the forward order.  With
// v_k = (c_k, f_k), u = dL/dA, A the ray's final (C_d, F), A_{<=k} the
// running prefix and T_{k+1} the transmittance after sample k:
//   dL/dsigma_k = delta (T_{k+1} u.v_k - u.(A - A_{<=k})) - delta T_N dL/dT_N
//   dL/draw_0   = sigma_k dL/dsigma_k
//   dL/draw_c   = w_k u_c s (1 - s)        (c >= 1, s = sigmoid(raw_c))
// and each texel receives its interpolation weight times dL/draw.  The
// opacity regulariser H = sum_k h(1 - T^k) with per-ray weight g adds
// g h'(1 - T^k) delta_i T^k to dL/dsigma_i for every sample i of block k;
// T^k comes from a density-only pre-march of the block.  The
// merged composite equals the monolithic one over the same sequence
// (Appendix A), so one running prefix serves all blocks in order.
// Texel-gradient scatter, one collective step per wave.  Each interpolation
// tap pair (texels p and p + 1 along the fastest axis) of a lane is 16
// contiguous floats (8 channels each).  The lanes stage
// their pairs in LDS and read them back transposed, so that one atomic
// instruction covers four lanes' 64-byte runs instead of 64 scattered texels:
// far fewer cache-line requests for the L2 atomic units, whose request rate
// bounds the adjoint.
struct ScatterLds {
    // 16 values; the pair's byte offset in its pair-slot buffer, 64 p (-1:
    // none); the lanes whose values ride along in this row (two slots, -1:
    // none).  Rows of 19 floats leave the LDS room for two workgroups of four
    // waves per CU; a third follower slot (rows of 20) leaves room for one.
    float v[64][19];
    // lanes of one step that scatter the same pair: (p << 6 | first lane) by
    // a hash of p, -1 between steps
    int merge[256];
};

// ordering point for one wave's LDS traffic: no memory operation moves across
// it (a wave's LDS operations complete in order)
__device__ inline void wave_fence() {
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline void scatter_lds_init(ScatterLds& L, int lane) {
    for (int i = lane; i < 256; i += 64) L.merge[i] = -1;
    wave_fence();
}

// Add vals[16] (texel p channels 0-7, texel p + 1 channels 0-7) for the pair
// at texel index p (-1: nothing from this lane) of one gradient texture into
// slot p of its pair-slot buffer (64 bytes per texel, at byte 64 p): every
// pair is one aligned 64-byte segment whatever its parity, and one buffer
// resource serves every row of an atomic instruction.  The fold after the
// march adds slot p's first texel and slot p - 1's second texel into
// gradient texel p.  Neighbouring rays often scatter the same pair in the
// same step (a sixth of the plane pairs on the differentiable workload), so
// a lane whose pair another lane entered first in a small LDS table hands
// its row to that lane's row (up to two such lanes per row, each taking a
// follower slot by compare-and-swap): the scatter adds the rows' values and
// sends one request for them.  Further repeats keep their rows.
__device__ inline void scatter_pair(ScatterLds& L, int lane, const float vals[16], int p,
                                    const __amdgpu_buffer_rsrc_t& ga) {
    float* row = L.v[lane];
#pragma unroll
    for (int c = 0; c < 16; ++c) row[c] = vals[c];
    // a multiple of 64 below 2^32 (fewer than 2^26 texels), so never -1
    row[16] = __int_as_float(p < 0 ? -1 : (int)((uint32_t)p << 6));
    row[17] = __int_as_float(-1);
    row[18] = __int_as_float(-1);
    wave_fence();
    const bool merge = p >= 0 && p < (1 << 25);  // the table packs p and a lane into 31 bits
    int h = 0;
    if (merge) {
        h = (int)(((uint32_t)p * 2654435761u) >> 24);
        int expected = -1;
        if (!__hip_atomic_compare_exchange_strong(&L.merge[h], &expected, (p << 6) | lane, __ATOMIC_RELAXED,
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) &&
            (expected >> 6) == p) {
            for (int f = 17; f <= 18; ++f) {
                int none = -1;
                int* slot = reinterpret_cast<int*>(&L.v[expected & 63][f]);
                if (__hip_atomic_compare_exchange_strong(slot, &none, lane, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_WAVEFRONT)) {
                    row[16] = __int_as_float(-1);  // sent with the first lane's row
                    break;
                }
            }
        }
    }
    wave_fence();
    const int e = lane & 15, sub = lane >> 4;
#pragma unroll 4
    for (int j = 0; j < 16; ++j) {
        // the four rows of one instruction come from lanes far apart in the
        // 8 x 8 packet (pixel (x, y) of lane 8y + x: x shifted by 3 and y by 2
        // per row): two rows of one instruction on the same segment cost the
        // L2 five requests instead of two
        const int src = (((j & 7) + 3 * sub) & 7) + 8 * ((j >> 3) + 2 * sub);
        const int ov = __float_as_int(L.v[src][16]);
        const int f1 = __float_as_int(L.v[src][17]), f2 = __float_as_int(L.v[src][18]);
        float val = L.v[src][e];
        if (f1 >= 0) val += L.v[f1][e];
        if (f2 >= 0) val += L.v[f2][e];
        if (ov != -1) __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(val, ga, (int)((uint32_t)ov + 4u * e), 0, 0);
    }
    wave_fence();
    if (merge) L.merge[h] = -1;
}

// Plane pairs (taps 4-9) of one sample: scattered at once.
__device__ inline void scatter_planes(ScatterLds& L, int lane, const Taps& T, const float draw[8],
                                      float* const gptr[4], const __amdgpu_buffer_rsrc_t ga[4], bool have) {
#pragma unroll
    for (int pr = 4; pr < 10; ++pr) {
        const int tex = pair_tex(pr);
        if (!gptr[tex]) continue;
        float vals[16];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            vals[c] = T.w[2 * pr] * draw[c];
            vals[8 + c] = T.w[2 * pr + 1] * draw[c];
        }
        scatter_pair(L, lane, vals, have ? T.pidx[pr] : -1, ga[tex]);
    }
}

// Grid pairs (taps 0-3): the samples of a wave's rays fall between far fewer
// distinct grid texels than they visit.  Consecutive samples of a ray share
// a 128^3 grid cell for about 2.7 steps of 1/512, so a lane sums its cell's
// gradient in registers while the cell stays the same (GridAcc); and
// neighbouring rays of a packet pass about half a cell apart, so when its
// cell changes the lane adds the sum into a small direct-mapped cache of
// texel pairs in LDS shared by the wave, and a pair goes to memory only when
// another pair takes its slot or the block ends.  The slot of the pair at
// grid texel (x, y, z) is (x + 5 y + 19 z) mod 128, so the four pairs of a
// cell never share a slot.  Pairs leaving the cache wait in a queue of 64
// rows and go out through the transposed scatter when it fills or the block
// ends.  Only the summation order differs from a per-sample scatter.
constexpr int kGridSlots = 128;
struct GridLds {
    int tag[kGridSlots];      // texel index of the pair a slot holds, -1: empty
    float v[kGridSlots][17];  // its 16 values (row padded against bank conflicts)
};
struct OutQueue {
    float v[64][17];  // 16 values of a pair leaving the cache
    int p[64];        // its texel index
};

__device__ inline void grid_cache_clear(GridLds& G, int lane) {
    for (int s = lane; s < kGridSlots; s += 64) G.tag[s] = -1;
    wave_fence();
}

__device__ inline int grid_slot(int pid, int lgx, int lgy) {
    const int x = pid & ((1 << lgx) - 1), y = (pid >> lgx) & ((1 << lgy) - 1), z = pid >> (lgx + lgy);
    return (x + 5 * y + 19 * z) & (kGridSlots - 1);
}

// Scatter the q queued pairs (q is wave-uniform): rows 4j..4j+3 per atomic
// instruction, 16 lanes per row, as in scatter_pair.
__device__ inline void queue_flush(OutQueue& Q, int lane, int& q, const __amdgpu_buffer_rsrc_t& ga) {
    wave_fence();
    const int e = lane & 15, sub = lane >> 4;
    for (int j = 0; 4 * j < q; ++j) {
        const int src = 4 * j + sub;
        if (src < q) {
            const uint32_t p = (uint32_t)Q.p[src];
            const float val = Q.v[src][e];
            __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(val, ga, (int)((p << 6) + 4u * e), 0, 0);
        }
    }
    wave_fence();
    q = 0;
}

// Row of this lane's entry among the lanes with `out`, after flushing the
// queue if they do not all fit.
__device__ inline int queue_row(OutQueue& Q, int lane, int& q, bool out, const __amdgpu_buffer_rsrc_t& ga) {
    const uint64_t m = __ballot(out);
    const int n = __popcll(m);
    if (q + n > 64) queue_flush(Q, lane, q, ga);
    const int row = q + __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
    q += n;
    return row;
}

// Add one grid pair per lane (texel index pid, values val(c); want ==
// false: none) into the wave's cache, in three ordered phases: a pair that
// holds its slot adds to it; the others try to take the slot (the first in
// lane order wins, queues the pair the slot held, if any, and writes its own
// values); the rest add to the slot if the winner holds their pair too, else
// queue their own values.
template <class Val>
__device__ inline void grid_cache_add(GridLds& G, OutQueue& Q, int lane, int& q, int pid, bool want, int lgx, int lgy,
                                      const __amdgpu_buffer_rsrc_t& ga, Val val) {
    const int slot = want ? grid_slot(pid, lgx, lgy) : 0;
    const int t = want ? G.tag[slot] : -2;
    const bool hit = want && t == pid;
    if (hit) {
#pragma unroll
        for (int c = 0; c < 16; ++c)
            __hip_atomic_fetch_add(&G.v[slot][c], val(c), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
    const bool miss = want && !hit;
    if (!__any(miss)) return;
    wave_fence();
    bool won = false;
    if (miss) {
        int expected = t;
        won = __hip_atomic_compare_exchange_strong(&G.tag[slot], &expected, pid, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                   __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
    const bool ev = won && t >= 0;
    const int row = queue_row(Q, lane, q, ev, ga);
    if (ev) {
#pragma unroll
        for (int c = 0; c < 16; ++c) Q.v[row][c] = G.v[slot][c];
        Q.p[row] = t;
    }
    if (won) {
#pragma unroll
        for (int c = 0; c < 16; ++c) G.v[slot][c] = val(c);
    }
    wave_fence();
    bool fb = false;
    if (miss && !won) {
        if (G.tag[slot] == pid) {
#pragma unroll
            for (int c = 0; c < 16; ++c)
                __hip_atomic_fetch_add(&G.v[slot][c], val(c), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        } else {
            fb = true;
        }
    }
    const int row2 = queue_row(Q, lane, q, fb, ga);
    if (fb) {
#pragma unroll
        for (int c = 0; c < 16; ++c) Q.v[row2][c] = val(c);
        Q.p[row2] = pid;
    }
    wave_fence();
}

// a lane's pending grid cell: its four pairs' gradient summed over the
// ray's consecutive samples in the cell
struct GridAcc {
    int cell;        // texel index of pair 0 of the pending cell, -1: none
    float v[4][16];  // pending gradient of the cell's four pairs
};

__device__ inline void grid_acc_push(GridLds& G, OutQueue& Q, int lane, int& q, GridAcc& g, bool push, int lgx,
                                     int lgy, const __amdgpu_buffer_rsrc_t& ga) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int pid = g.cell + ((((j >> 1) << lgy) + (j & 1)) << lgx);
        grid_cache_add(G, Q, lane, q, pid, push, lgx, lgy, ga, [&](int c) { return g.v[j][c]; });
    }
    if (push) {
        g.cell = -1;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int c = 0; c < 16; ++c) g.v[j][c] = 0.0f;
    }
}

// send every pair the cache and the queue hold and empty both (the block's end)
__device__ inline void grid_cache_flush(GridLds& G, OutQueue& Q, int lane, int& q, const __amdgpu_buffer_rsrc_t& ga) {
    for (int s0 = 0; s0 < kGridSlots; s0 += 64) {
        const int s = s0 + lane;
        const int t = G.tag[s];
        const int row = queue_row(Q, lane, q, t >= 0, ga);
        if (t >= 0) {
#pragma unroll
            for (int c = 0; c < 16; ++c) Q.v[row][c] = G.v[s][c];
            Q.p[row] = t;
        }
    }
    if (q > 0) queue_flush(Q, lane, q, ga);
    grid_cache_clear(G, lane);
}

// Local composite (Ae, Te) of one exterior segment, as the forward forms it
// (the same walk, samples and early-termination rule; Tm the merged
// transmittance before the segment).
__device__ inline void bwd_exterior_total(const BwdArgs& ba, const ViewU& v, const Ray& r, float t_start,
                                          float t_end, bool post, bool want, float Tm, float Ae[7], float& Te) {
    const MarchArgs& a = ba.m;
    ExtWalk W;
    ext_begin(a, t_start, t_end, post, want, W);
#pragma unroll
    for (int c = 0; c < 7; ++c) Ae[c] = 0.0f;
    Te = 1.0f;
    int64_t unused = 0;
    for (;;) {
        float q[3] = {0.0f, 0.0f, 0.0f}, w = 0.0f;
        const bool have = ext_next(a, v, r, W, q, w, unused);
        if (!__any(have)) break;
        bool pending = have;
        while (__any(pending)) {
            const uint64_t mask = __ballot(pending);
            const int first = __ffsll((unsigned long long)mask) - 1;
            const int eu = ufl(__shfl(W.owner, first));
            BlockU b;
            load_block<1>(a.blocks + eu, b);
            if (pending && W.owner == eu) {
                pending = false;
                const int cell = occ_cell(b, q);
                if (ld1g(b.skip, (uint32_t)cell) == 0) {
                    Taps T;
                    sample_taps(b, q, T);
                    float raw[8];
                    raw_f32<true>(b, T, raw);
                    const float alpha = alpha_of(__expf(raw[0]) * w);
                    const float wt = Te * alpha;
#pragma unroll
                    for (int c = 0; c < 7; ++c) Ae[c] = fmaf(wt, sigmoidf_(raw[1 + c]), Ae[c]);
                    Te *= 1.0f - alpha;
                    if (Tm * Te < a.t_min) W.live = false;
                }
            }
        }
    }
}

// Adjoint of one exterior segment of a lane's ray (contracted boundary
// blocks): the samples of the forward's walk, in its order, each with its
// own step w as its delta, join the running prefix (Ap, Tg) of the single
// chain; dL/draw of a sample is scattered into the pair slots of the block
// that owns it.  Lanes may have different owners: each round serves one
// owner, whose wave-uniform descriptors address its textures.  Tm is the
// merged transmittance before the segment as the forward forms it (its
// early-termination decision uses Tm Te), multiplied by the segment's Te at
// the end.  The light after sample i, A - A_{<=i}, is formed locally as
// Tm (Ae - Ae_{<=i}) + rest, from the segment's own composite Ae and the
// light after the segment (rest), not as the ray's A minus the running
// prefix: that difference carries fp32 rounding of the whole ray's light,
// which the exterior's long steps (delta up to ext_delta m^2) would multiply
// into the gradient of samples behind opaque content.  Each part is clamped
// to where it lies exactly: features are in (0, 1), so the light after a
// sample is at most the transmittance after it.
__device__ inline void bwd_exterior(const BwdArgs& ba, const ViewU& v, const Ray& r, float t_start, float t_end,
                                    bool post, bool want, const float u[7], const float Ae_tot[7],
                                    const float rest[7], float tn_term, float Ap[7], float& Tg, float& Tm,
                                    ScatterLds& lds, int lane) {
    const MarchArgs& a = ba.m;
    ExtWalk W;
    ext_begin(a, t_start, t_end, post, want, W);
    float Te = 1.0f, Ael[7] = {0, 0, 0, 0, 0, 0, 0};
    int64_t unused = 0;
    for (;;) {
        float q[3] = {0.0f, 0.0f, 0.0f}, w = 0.0f;
        const bool have = ext_next(a, v, r, W, q, w, unused);
        if (!__any(have)) break;
        bool pending = have;
        while (__any(pending)) {
            const uint64_t mask = __ballot(pending);
            const int first = __ffsll((unsigned long long)mask) - 1;
            const int eu = ufl(__shfl(W.owner, first));
            BlockU b;
            load_block<1>(a.blocks + eu, b);
            Taps T;
            float draw[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            bool sampled = false;
            if (pending && W.owner == eu) {
                pending = false;
                const int cell = occ_cell(b, q);
                if (ld1g(b.skip, (uint32_t)cell) == 0) {
                    sampled = true;
                    sample_taps(b, q, T);
                    float raw[8];
                    raw_f32<true>(b, T, raw);
                    const float sigma = __expf(raw[0]);
                    const float alpha = alpha_of(sigma * w);
                    const float wt = Tg * alpha, wl = Te * alpha;
                    const float Tel = Te * (1.0f - alpha);  // the segment's transmittance after the sample
                    float vv[7];
                    float uv = 0.0f, us = 0.0f;
#pragma unroll
                    for (int c = 0; c < 7; ++c) {
                        vv[c] = sigmoidf_(raw[1 + c]);
                        Ap[c] = fmaf(wt, vv[c], Ap[c]);  // the ray's prefix, for the blocks after the segment
                        Ael[c] = fmaf(wl, vv[c], Ael[c]);
                        const float after = fmaf(Tm, fminf(fmaxf(Ae_tot[c] - Ael[c], 0.0f), Tel), rest[c]);
                        uv = fmaf(u[c], vv[c], uv);
                        us = fmaf(u[c], after, us);
                    }
                    const float Tn = Tg * (1.0f - alpha);
                    const float dsig = w * (Tn * uv - us) - w * tn_term;
                    draw[0] = sigma * dsig;
#pragma unroll
                    for (int c = 0; c < 7; ++c) draw[1 + c] = wt * u[c] * vv[c] * (1.0f - vv[c]);
                    Tg = Tn;
                    Te = Tel;
                    if (Tm * Te < a.t_min) W.live = false;  // early ray termination, as in the forward
                }
            }
            // the owner's ten pairs, from the lanes it serves this round
            float* gptr[4] = {ufp(ba.grad_grid[eu]), ufp(ba.grad_plane[3 * eu + 0]), ufp(ba.grad_plane[3 * eu + 1]),
                              ufp(ba.grad_plane[3 * eu + 2])};
            __amdgpu_buffer_rsrc_t ga[4];
            ga[0] = tex_rsrc(ufp(ba.slots[4 * eu]), grid_texels(b) * 64u);
            for (int t = 1; t < 4; ++t) ga[t] = tex_rsrc(ufp(ba.slots[4 * eu + t]), plane_texels(b, t - 1) * 64u);
#pragma unroll
            for (int pr = 0; pr < 10; ++pr) {
                const int tex = pair_tex(pr);
                if (!gptr[tex]) continue;
                float vals[16];
#pragma unroll
                for (int c = 0; c < 8; ++c) {  // a lane without a sample this round sends nothing
                    vals[c] = sampled ? T.w[2 * pr] * draw[c] : 0.0f;
                    vals[8 + c] = sampled ? T.w[2 * pr + 1] * draw[c] : 0.0f;
                }
                scatter_pair(lds, lane, vals, sampled ? T.pidx[pr] : -1, ga[tex]);
            }
        }
    }
    Tm *= Te;
}

// BMLP: per-block deferred MLPs before the merge.  Per block k with prefix
// transmittance P, a first pass composites the block (A^k, T^k); the lane
// then runs the block's MLP adjoint for u = dL/dA^k and takes
// T^k dL/dT^k = g . R_k + gT T, with R_k = C - (colour merged up to block k)
// the light of the later blocks; the sample adjoint inside the block is the
// single-chain one with these per-block u and transmittance term.
template <int MODE, bool OPAC, bool BMLP, bool CT>
__device__ __attribute__((always_inline)) inline void march_bwd_packet(const BwdArgs& ba, const DevView* V, int tile,
                                                                       int lane, ScatterLds& lds, GridLds& glds,
                                                                       OutQueue& gq) {
    // the exterior's adjoint reads the ray's A from aux: one MLP after the merge
    static_assert(!(CT && (OPAC || BMLP || MODE != 1)), "contracted blocks: grid mode, one MLP, no opacity term");
    const MarchArgs& a = ba.m;
    ViewU v;
    load_view(V, v);
    Ray r;
    packet_ray(a, v, tile, lane, r);
    bool hit = r.active;
    int w0 = 0, w1 = 0;
    if (MODE == 1 && r.active) {
        int ka, kb;
        const float slo[3] = {a.scene_lo[0], a.scene_lo[1], a.scene_lo[2]};
        const float shi[3] = {a.scene_hi[0], a.scene_hi[1], a.scene_hi[2]};
        box_interval(r.o, r.d, a.delta, slo, shi, &ka, &kb);
        hit = ka < kb;
        w0 = ka;
        w1 = ka + a.max_steps;
    }
    float Af[7] = {0, 0, 0, 0, 0, 0, 0}, TN = 1.0f, u[7] = {0, 0, 0, 0, 0, 0, 0}, gT = 0.0f;
    float Cf[3] = {0, 0, 0}, g[3] = {0, 0, 0}, Cpre[3] = {0, 0, 0};  // per-block MLPs only
    if (r.active) {
        const float4 lo = reinterpret_cast<const float4*>(a.aux)[2 * r.pix];
        const float4 hi = reinterpret_cast<const float4*>(a.aux)[2 * r.pix + 1];
        TN = hi.w;
        if (BMLP) {  // aux = (C, 0, 0, 0, 0, T)
            Cf[0] = lo.x, Cf[1] = lo.y, Cf[2] = lo.z;
            for (int c = 0; c < 3; ++c) g[c] = ba.grad_rgb[3 * r.pix + c];
        } else {
            Af[0] = lo.x, Af[1] = lo.y, Af[2] = lo.z, Af[3] = lo.w, Af[4] = hi.x, Af[5] = hi.y, Af[6] = hi.z;
            const float4 ulo = reinterpret_cast<const float4*>(ba.u)[2 * r.pix];
            const float4 uhi = reinterpret_cast<const float4*>(ba.u)[2 * r.pix + 1];
            u[0] = ulo.x, u[1] = ulo.y, u[2] = ulo.z, u[3] = ulo.w, u[4] = uhi.x, u[5] = uhi.y, u[6] = uhi.z;
        }
        if (ba.grad_trans) gT = ba.grad_trans[r.pix];
    }
    const float w_op = ((OPAC || BMLP) && r.active && ba.w_opacity) ? ba.w_opacity[r.pix] : 0.0f;
    float Ap[7] = {0, 0, 0, 0, 0, 0, 0}, Tg = 1.0f;
    float T_blk = 1.0f;  // merged transmittance before the block, as the forward forms it
    float tn_term = TN * gT;
    int64_t unused = 0;
    float fin = INFINITY, fout = INFINITY;  // the ray's interval in the footprint's column
    if (CT && a.ext_delta > 0.0f) {
        const float slo[3] = {a.scene_lo[0], a.scene_lo[1], a.scene_lo[2]};
        const float shi[3] = {a.scene_hi[0], a.scene_hi[1], a.scene_hi[2]};
        if (!slab_xy(r.o, r.d, slo, shi, &fin, &fout)) fin = fout = INFINITY;
        float Ae[7], Te, rest[7];
        bwd_exterior_total(ba, v, r, 0.0f, fin, false, r.active, T_blk, Ae, Te);
#pragma unroll
        for (int c = 0; c < 7; ++c) rest[c] = fminf(fmaxf(Af[c] - Ae[c], 0.0f), Te);  // light after the segment
        bwd_exterior(ba, v, r, 0.0f, fin, false, r.active, u, Ae, rest, tn_term, Ap, Tg, T_blk, lds, lane);
    }
    for (int j = 0; j < v.set_n; ++j) {
        const int e = ufl(a.refs[v.set_begin + j]);
        BlockU b;
        load_block<1>(a.blocks + e, b);
        // the textures whose gradient the caller wants (null: none), and their
        // pair-slot buffers as buffer resources: base in scalar registers,
        // no-return buffer_atomic_add_f32 with a 32-bit offset per lane
        float* gptr[4] = {ufp(ba.grad_grid[e]), ufp(ba.grad_plane[3 * e + 0]), ufp(ba.grad_plane[3 * e + 1]),
                          ufp(ba.grad_plane[3 * e + 2])};
        __amdgpu_buffer_rsrc_t ga[4];
        ga[0] = tex_rsrc(ufp(ba.slots[4 * e]), grid_texels(b) * 64u);
        for (int t = 1; t < 4; ++t) ga[t] = tex_rsrc(ufp(ba.slots[4 * e + t]), plane_texels(b, t - 1) * 64u);
        const bool alive = hit && !(T_blk < a.t_min);
        const Span sp = block_span<MODE>(a, b, r, alive, w0, w1);
        if (!__any(sp.ka < sp.kb)) continue;
        float g_op = 0.0f;  // dL/dsigma_i of the opacity term, per unit step length
        if (BMLP) {
            float Tkf = 1.0f;
            int64_t ne = 0, nm = 0;
#pragma unroll
            for (int c = 0; c < 7; ++c) Af[c] = 0.0f;
            if (a.block_aux) {  // the block's composite as the forward formed it
                if (r.active) nm = get_block_aux(a, r.pix, j, Af, Tkf) ? 1 : 0;
            } else {
                march_block<1, MODE, false, false>(a, b, r, sp, T_blk, Af, Tkf, ne, nm);
            }
            float Ck[3];
            const int np = mlp_params(a.pe);  // weights per block: 499, or 883 with four PE frequencies
            float* gwp = ba.grad_block_mlp ? ufp(ba.grad_block_mlp) + (size_t)e * np : nullptr;
            if (a.pe == 4)
                block_shade_adjoint<4>(ufp(a.block_mlp) + (size_t)e * np, Af, r.d, T_blk, g, nm > 0, Ck, u, gwp, lane);
            else
                block_shade_adjoint<0>(ufp(a.block_mlp) + (size_t)e * np, Af, r.d, T_blk, g, nm > 0, Ck, u, gwp, lane);
            float R = gT * TN;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (nm > 0) Cpre[c] = fmaf(T_blk, Ck[c], Cpre[c]);
                R = fmaf(g[c], Cf[c] - Cpre[c], R);
            }
            tn_term = R;
            if (w_op != 0.0f) g_op = w_op * opacity_dentropy(Tkf) * Tkf;
#pragma unroll
            for (int c = 0; c < 7; ++c) Ap[c] = 0.0f;
            Tg = 1.0f;
        } else if (OPAC && __any(w_op != 0.0f)) {
            float Tkf = 1.0f;
            if (a.block_aux) {
                float Ab[7];
                if (r.active) (void)get_block_aux(a, r.pix, j, Ab, Tkf);
            } else {
                Tkf = block_trans_f32<MODE>(b, r, sp, T_blk, a.t_min, true, w_op != 0.0f);
            }
            g_op = w_op * opacity_dentropy(Tkf) * Tkf;
        }
        int k = sp.ka, kb = sp.kb;
        int cur_cell = -1;
        bool cur_occ = false;
        float Tk = 1.0f;  // block-local transmittance, for the same termination decision as the forward
        const bool want_grid = gptr[0] != nullptr;
        int nq = 0;  // pairs waiting in the wave's queue
        GridAcc gacc;
        gacc.cell = -1;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int c = 0; c < 16; ++c) gacc.v[j][c] = 0.0f;
        if (want_grid) grid_cache_clear(glds, lane);
        for (;;) {
            float q[3];
            int cell = 0;
            // one step at a time (see march_block): the same samples as the forward's jumps
            const bool have =
                next_occupied<MODE, CT>(b, r, sp, kb, sp.delta, true, k, q, cell, cur_cell, cur_occ, unused);
            if (!__any(have)) break;
            Taps T;
            float draw[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (have) {
                sample_taps(b, q, T);
                float raw[8];
                raw_f32<true>(b, T, raw);
                const float sigma = __expf(raw[0]);
                const float alpha = alpha_of(sigma * sp.delta);
                const float w = Tg * alpha;
                float vv[7];
                float uv = 0.0f, us = 0.0f;
#pragma unroll
                for (int c = 0; c < 7; ++c) {
                    vv[c] = sigmoidf_(raw[1 + c]);
                    Ap[c] = fmaf(w, vv[c], Ap[c]);
                    uv = fmaf(u[c], vv[c], uv);
                    us = fmaf(u[c], Af[c] - Ap[c], us);
                }
                const float Tn = Tg * (1.0f - alpha);
                const float dsig = sp.delta * (Tn * uv - us) - sp.delta * tn_term + sp.delta * g_op;
                draw[0] = sigma * dsig;
#pragma unroll
                for (int c = 0; c < 7; ++c) draw[1 + c] = w * u[c] * vv[c] * (1.0f - vv[c]);
                Tg = Tn;
                ++k;
                Tk *= 1.0f - alpha;
                if (T_blk * Tk < a.t_min) kb = k;  // early ray termination, as in the forward
            }
            // collectives over the wave: lanes without a sample take part with nothing to add
            scatter_planes(lds, lane, T, draw, gptr, ga, have);
            if (want_grid) {
                const int cell_now = have ? T.pidx[0] : -1;
                const bool push = have && gacc.cell >= 0 && cell_now != gacc.cell;
                if (__any(push)) grid_acc_push(glds, gq, lane, nq, gacc, push, b.lgx, b.lgy, ga[0]);
                if (have) {
                    gacc.cell = cell_now;
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int c = 0; c < 8; ++c) {
                            gacc.v[j][c] = fmaf(T.w[2 * j], draw[c], gacc.v[j][c]);
                            gacc.v[j][8 + c] = fmaf(T.w[2 * j + 1], draw[c], gacc.v[j][8 + c]);
                        }
                }
            }
        }
        if (want_grid) {
            if (__any(gacc.cell >= 0))
                grid_acc_push(glds, gq, lane, nq, gacc, gacc.cell >= 0, b.lgx, b.lgy, ga[0]);
            grid_cache_flush(glds, gq, lane, nq, ga[0]);
        }
        T_blk *= Tk;
    }
    if (CT && a.ext_delta > 0.0f) {
        // the cap truncates the ray, as in the forward
        const bool capped = MODE == 1 && hit && step_t(w1, a.delta) < fout;
        const bool want = r.active && fout < INFINITY && !capped && !(T_blk < a.t_min);
        float Ae[7], Te;
        const float rest[7] = {0, 0, 0, 0, 0, 0, 0};  // nothing after the last segment
        bwd_exterior_total(ba, v, r, fout, INFINITY, true, want, T_blk, Ae, Te);
        bwd_exterior(ba, v, r, fout, INFINITY, true, want, u, Ae, rest, tn_term, Ap, Tg, T_blk, lds, lane);
    }
}

// OPAC: with the opacity regulariser's pre-march (a separate instance keeps
// the plain adjoint's register budget)
template <int MODE, bool OPAC, bool BMLP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void march_bwd_kernel(BwdArgs ba) {
    const MarchArgs& a = ba.m;
    __shared__ ScatterLds lds[4];
    __shared__ GridLds glds[4];
    __shared__ OutQueue gq[4];
    const int lane = threadIdx.x & 63;
    const int waves = blockDim.x >> 6;
    const int wave = ufl(threadIdx.x >> 6);
    scatter_lds_init(lds[wave], lane);
    int p = a.persistent ? 0 : ufl(xcd_packet(waves, wave));  // one call site, as in the forward
    for (;;) {
        if (a.persistent) {
            int q = -1;
            if (lane == 0) q = take_packet(a.work_counter, a.total_tiles);
            p = ufl(__shfl(q, 0));
            if (p < 0) return;
        }
        if (p >= a.total_tiles) return;
        const DevView* V = find_view_by_tile(a.views, a.n_views, p);
        march_bwd_packet<MODE, OPAC, BMLP, false>(ba, V, p - ufl(V->tile_begin), lane, lds[wave], glds[wave], gq[wave]);
        if (!a.persistent) return;
    }
}

// Contracted boundary blocks (their samples read through the contraction,
// the exterior segments around the blocks): grid mode, one MLP after the
// merge, no opacity term.  A kernel of its own, the same packet walk, so the
// plain adjoint carries none of its code.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void march_bwd_ct_kernel(BwdArgs ba) {
    const MarchArgs& a = ba.m;
    __shared__ ScatterLds lds[4];
    __shared__ GridLds glds[4];
    __shared__ OutQueue gq[4];
    const int lane = threadIdx.x & 63;
    const int waves = blockDim.x >> 6;
    const int wave = ufl(threadIdx.x >> 6);
    scatter_lds_init(lds[wave], lane);
    int p = a.persistent ? 0 : ufl(xcd_packet(waves, wave));  // one call site, as in the forward
    for (;;) {
        if (a.persistent) {
            int q = -1;
            if (lane == 0) q = take_packet(a.work_counter, a.total_tiles);
            p = ufl(__shfl(q, 0));
            if (p < 0) return;
        }
        if (p >= a.total_tiles) return;
        const DevView* V = find_view_by_tile(a.views, a.n_views, p);
        march_bwd_packet<1, false, false, true>(ba, V, p - ufl(V->tile_begin), lane, lds[wave], glds[wave], gq[wave]);
        if (!a.persistent) return;
    }
}

// blockIdx.y: job; grid-stride over the job's slots (four float4 each)
__global__ __launch_bounds__(256) void slots_zero_kernel(const FoldJob* jobs) {
    const FoldJob j = jobs[blockIdx.y];
    float4* sl = reinterpret_cast<float4*>(j.slots);
    const int64_t n = 4 * j.n_texels;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        sl[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// gradient texel x += first texel of slot x + second texel of slot x - 1;
// grid-stride over the gradient's float4 (two per texel)
__global__ __launch_bounds__(256) void slots_fold_kernel(const FoldJob* jobs) {
    const FoldJob j = jobs[blockIdx.y];
    float4* g = reinterpret_cast<float4*>(j.grad);
    const float4* sl = reinterpret_cast<const float4*>(j.slots);
    const int64_t n = 2 * j.n_texels;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = i >> 1, h = i & 1;
        const float4 a = g[i], b = sl[4 * x + h];
        const float4 c = x > 0 ? sl[4 * (x - 1) + 2 + h] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        g[i] = make_float4(a.x + (b.x + c.x), a.y + (b.y + c.y), a.z + (b.z + c.z), a.w + (b.w + c.w));
    }
}

static dim3 fold_grid(int n_jobs, int64_t max_texels) {
    const int64_t blocks = (4 * max_texels + 255) / 256;
    return dim3((unsigned)(blocks < 2048 ? blocks : 2048), (unsigned)n_jobs);
}

hipError_t launch_slots_zero(const FoldJob* jobs, int n_jobs, int64_t max_texels, hipStream_t s) {
    if (n_jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(slots_zero_kernel, fold_grid(n_jobs, max_texels), dim3(256), 0, s, jobs);
    return hipGetLastError();
}

hipError_t launch_slots_fold(const FoldJob* jobs, int n_jobs, int64_t max_texels, hipStream_t s) {
    if (n_jobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(slots_fold_kernel, fold_grid(n_jobs, max_texels), dim3(256), 0, s, jobs);
    return hipGetLastError();
}

hipError_t launch_march_bwd(const BwdArgs& a, int waves, hipStream_t s) {
    if (a.m.total_tiles <= 0) return hipSuccess;
    dim3 block(64 * waves), grid((a.m.total_tiles + waves - 1) / waves);
    if (a.m.persistent) {
        int dev = 0, cus = 256;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        grid = dim3(cus * (16 / waves));
    }
    const bool op = a.w_opacity != nullptr, bm = a.m.block_mlp != nullptr;
    const size_t shm = 0;
#define COW_LAUNCH(M, O, B) hipLaunchKernelGGL((march_bwd_kernel<M, O, B>), grid, block, shm, s, a)
    if (a.m.contract) {  // grid mode, one MLP after the merge, no opacity term (checked on the host)
        hipLaunchKernelGGL(march_bwd_ct_kernel, grid, block, shm, s, a);
    } else if (a.m.mode == 1) {
        if (bm)
            COW_LAUNCH(1, false, true);
        else if (op)
            COW_LAUNCH(1, true, false);
        else
            COW_LAUNCH(1, false, false);
    } else {
        if (bm)
            COW_LAUNCH(0, false, true);
        else if (op)
            COW_LAUNCH(0, true, false);
        else
            COW_LAUNCH(0, false, false);
    }
#undef COW_LAUNCH
    return hipGetLastError();
}

}  // namespace cow
