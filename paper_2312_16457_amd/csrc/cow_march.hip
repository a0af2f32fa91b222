// Forward march (per-block composite + front-to-back merge), occupancy
// build and sparse-brick packing for gfx950 (City-on-Web, arXiv 2312.16457).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "cow_device.h"

namespace cow {

// One exterior segment of a lane's ray (see ExtWalk), composited into
// (Ae, Te) and merged into (A, T) at the end (Eq. "volume rendering across
// blocks").  Lanes of a wave may sample different owners: each round
// evaluates one owner for all lanes that need it, the textures addressed
// through that block's wave-uniform descriptors.
template <int DT, bool SPARSE>
__device__ inline void march_exterior(const MarchArgs& a, const ViewU& v, const Ray& r, float t_start, float t_end,
                                      bool post, bool want, float A[7], float& T, int64_t& n_eval, int64_t& n_march) {
    ExtWalk W;
    ext_begin(a, t_start, t_end, post, want, W);
    float Ae[7] = {0, 0, 0, 0, 0, 0, 0}, Te = 1.0f;
    for (;;) {
        float q[3] = {0.0f, 0.0f, 0.0f}, w = 0.0f;
        const bool have = ext_next(a, v, r, W, q, w, n_march);
        if (!__any(have)) break;
        bool pending = have;
        bool occupied = false;
        float sigma = 0.0f, val[7] = {0, 0, 0, 0, 0, 0, 0};
        while (__any(pending)) {
            const uint64_t mask = __ballot(pending);
            const int first = __ffsll((unsigned long long)mask) - 1;
            const int eu = ufl(__shfl(W.owner, first));
            BlockU b;
            load_block<DT>(a.blocks + eu, b);
            if (pending && W.owner == eu) {
                pending = false;
                const int cell = occ_cell(b, q);
                occupied = ld1g(b.skip, (uint32_t)cell) == 0;
                if (occupied) {
                    float raw[8];
                    if (DT == 0) {
                        raw_u8<SPARSE>(b, q, cell, raw);
                        sigma = density_u8(raw);
#pragma unroll
                        for (int c = 0; c < 7; ++c) val[c] = feature_u8(raw, 1 + c);
                    } else {
                        Taps Tp;
                        sample_taps(b, q, Tp);
                        raw_f32(b, Tp, raw);
                        sigma = __expf(raw[0]);
#pragma unroll
                        for (int c = 0; c < 7; ++c) val[c] = sigmoidf_(raw[1 + c]);
                    }
                }
            }
        }
        if (have && occupied) {
            const float alpha = alpha_of(sigma * w);
            const float wt = Te * alpha;
#pragma unroll
            for (int c = 0; c < 7; ++c) Ae[c] = fmaf(wt, val[c], Ae[c]);
            Te *= 1.0f - alpha;
            ++n_eval;
            if (T * Te < a.t_min) W.live = false;  // early ray termination
        }
    }
#pragma unroll
    for (int c = 0; c < 7; ++c) A[c] = fmaf(T, Ae[c], A[c]);
    T *= Te;
}

// PE: positional-encoding frequencies of the per-block MLPs' direction input
// (a kernel of its own, so the plain kernels carry none of its code)
// CT: the launch holds contracted blocks (the contraction kernel)
template <int MODE, int DT, bool SPARSE, int PE = 0, bool CT = false>
__device__ __attribute__((always_inline)) inline void march_packet(const MarchArgs& a, const DevView* V, int tile,
                                                                   int lane) {
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
    int r0 = 0, r1 = v.set_n;
    if (a.only_set_pos >= 0) r0 = a.only_set_pos, r1 = a.only_set_pos + 1;
    float A[7] = {0, 0, 0, 0, 0, 0, 0}, T = 1.0f, H = 0.0f;
    int64_t n_eval = 0, n_march = 0;
    if (a.only_set_pos > 0 && r.active) {  // per-block baseline: continue the running blend
        const float4 lo4 = reinterpret_cast<const float4*>(a.aux)[2 * r.pix];
        const float4 hi4 = reinterpret_cast<const float4*>(a.aux)[2 * r.pix + 1];
        A[0] = lo4.x, A[1] = lo4.y, A[2] = lo4.z, A[3] = lo4.w;
        A[4] = hi4.x, A[5] = hi4.y, A[6] = hi4.z, T = hi4.w;
        if (a.counts) n_eval = a.counts[2 * r.pix], n_march = a.counts[2 * r.pix + 1];
        if (a.opacity) H = a.opacity[r.pix];
    }
    float fin = INFINITY, fout = INFINITY;  // the ray's interval in the footprint's column
    if (CT && a.ext_delta > 0.0f) {
        const float slo[3] = {a.scene_lo[0], a.scene_lo[1], a.scene_lo[2]};
        const float shi[3] = {a.scene_hi[0], a.scene_hi[1], a.scene_hi[2]};
        if (!slab_xy(r.o, r.d, slo, shi, &fin, &fout)) fin = fout = INFINITY;
        march_exterior<DT, SPARSE>(a, v, r, 0.0f, fin, false, r.active, A, T, n_eval, n_march);
    }
    for (int j = r0; j < r1; ++j) {
        const int e = ufl(a.refs[v.set_begin + j]);
        BlockU b;
        load_block<DT>(a.blocks + e, b);
        const bool alive = hit && !(T < a.t_min);  // a terminated ray takes no more samples
        const Span sp = block_span<MODE>(a, b, r, alive, w0, w1);
        float Ak[7] = {0, 0, 0, 0, 0, 0, 0}, Tk = 1.0f;
        // per-block composites for the backward (float32 blocks only, the
        // adjoint's input; the uint8 kernels carry none of this code)
        if (!__any(sp.ka < sp.kb)) {
            if (DT == 1 && a.block_aux && r.active) put_block_aux(a, r.pix, j, Ak, -1.0f);
            continue;
        }
        const int64_t marched_before = n_march;
        march_block<DT, MODE, SPARSE, true, CT>(a, b, r, sp, T, Ak, Tk, n_eval, n_march);
        if (DT == 1 && a.block_aux && r.active) put_block_aux(a, r.pix, j, Ak, n_march > marched_before ? Tk : -1.0f);
        // opacity regulariser: entropy of the block's opacity 1 - Tk, for
        // every block the ray marches (Eq. "opacity loss")
        if (a.opacity && n_march > marched_before) H += opacity_entropy(Tk);
        if (a.block_mlp) {
            // per-block deferred shading before the merge: every block the
            // ray marches adds its colour C^k under the prefix transmittance
            if (n_march > marched_before) {
                float Ck[3];
                block_shade<PE>(ufp(a.block_mlp) + (size_t)e * MlpShape<PE>::N, Ak, r.d, Ck);
#pragma unroll
                for (int c = 0; c < 3; ++c) A[c] = fmaf(T, Ck[c], A[c]);
            }
        } else {
            // merge front to back (Eq. "volume rendering across blocks"), with
            // the block's transmittance prod(1 - alpha_i) carried directly
#pragma unroll
            for (int c = 0; c < 7; ++c) A[c] = fmaf(T, Ak[c], A[c]);
        }
        T *= Tk;
    }
    if (CT && a.ext_delta > 0.0f) {
        // the cap truncates the ray: a window that ends before the ray leaves
        // the column leaves the exterior behind it unsampled
        const bool capped = MODE == 1 && hit && step_t(w1, a.delta) < fout;
        march_exterior<DT, SPARSE>(a, v, r, fout, INFINITY, true,
                                   r.active && fout < INFINITY && !capped && !(T < a.t_min), A, T, n_eval, n_march);
    }
    if (r.active) {
        float4* aux4 = reinterpret_cast<float4*>(a.aux);
        aux4[2 * r.pix] = make_float4(A[0], A[1], A[2], A[3]);
        aux4[2 * r.pix + 1] = make_float4(A[4], A[5], A[6], T);
        a.trans[r.pix] = T;
        if (a.block_mlp) {  // A[0..2] is the colour; A[3..6] stay zero
            a.rgb[3 * r.pix + 0] = A[0];
            a.rgb[3 * r.pix + 1] = A[1];
            a.rgb[3 * r.pix + 2] = A[2];
        }
        if (a.opacity) a.opacity[r.pix] = H;
        if (a.counts) {
            a.counts[2 * r.pix] = n_eval;
            a.counts[2 * r.pix + 1] = n_march;
        }
    }
}

// All blocks of one launch share a texture dtype (checked on the host).  The
// uint8 kernel runs four waves per SIMD.  The fp32 one keeps its 40 texel
// loads (160 registers) in flight with one: it is bound by the traffic its
// L2 misses make, and with fewer rays in flight per XCD more of the texels
// that neighbouring samples share are still cached (20% faster than two
// waves per SIMD on the differentiable 4x4-block workload).
template <int MODE, int DT, bool SPARSE, int PE = 0, bool CT = false>
__device__ inline void march_fwd_body(const MarchArgs& a) {
    const int lane = threadIdx.x & 63;
    const int waves = blockDim.x >> 6;
    const int wave = ufl(threadIdx.x >> 6);
    // One call site of march_packet, so that it stays inlined with the
    // arguments in scalar registers: a persistent wave takes packets from the
    // counter until it runs dry, otherwise a wave marches its one packet.
    int p = a.persistent ? 0 : ufl(xcd_packet(waves, wave));
    for (;;) {
        if (a.persistent) {
            int q = -1;
            if (lane == 0) q = take_packet(a.work_counter, a.total_tiles);
            p = ufl(__shfl(q, 0));
            if (p < 0) return;
        }
        if (p >= a.total_tiles) return;
        const DevView* V;
        int tile;
        if (a.only_view >= 0) {  // per-block baseline: one view per launch
            V = a.views + a.only_view;
            tile = p;
        } else {
            V = find_view_by_tile(a.views, a.n_views, p);
            tile = p - ufl(V->tile_begin);
        }
        march_packet<MODE, DT, SPARSE, PE, CT>(a, V, tile, lane);
        if (!a.persistent) return;
    }
}

template <int MODE, bool SPARSE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void march_fwd_kernel(MarchArgs a) {
    march_fwd_body<MODE, 0, SPARSE>(a);
}

template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void march_fwd_f32_kernel(MarchArgs a) {
    march_fwd_body<MODE, 1, false>(a);
}

// per-block deferred MLPs over [C_d, F, PE(d)] with four frequencies
template <int MODE, int DT, bool SPARSE>
__global__ __launch_bounds__(256) void march_fwd_pe_kernel(MarchArgs a) {
    march_fwd_body<MODE, DT, SPARSE, 4>(a);
}

// grid mode with contracted boundary blocks and their exterior
template <int DT, bool SPARSE>
__global__ __launch_bounds__(256) void march_fwd_ct_kernel(MarchArgs a) {
    march_fwd_body<1, DT, SPARSE, 0, true>(a);
}

hipError_t launch_march(const MarchArgs& a, int waves, hipStream_t s) {
    if (a.total_tiles <= 0) return hipSuccess;
    dim3 block(64 * waves);
    dim3 grid;
    if (a.persistent) {
        int dev = 0, cus = 256;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        // as many waves as fit at once: four per SIMD, one for the plain fp32 kernel
        const bool one = a.blocks_dtype == 1 && !a.contract && !(a.block_mlp && a.pe == 4);
        grid = dim3(cus * ((one ? 4 : 16) / waves));
    } else {
        grid = dim3((a.total_tiles + waves - 1) / waves);
    }
    const int dt = a.blocks_dtype;
    if (a.contract) {  // grid mode, one MLP after the merge (checked on the host)
        if (dt == 1)
            hipLaunchKernelGGL((march_fwd_ct_kernel<1, false>), grid, block, 0, s, a);
        else if (a.use_sparse)
            hipLaunchKernelGGL((march_fwd_ct_kernel<0, true>), grid, block, 0, s, a);
        else
            hipLaunchKernelGGL((march_fwd_ct_kernel<0, false>), grid, block, 0, s, a);
        return hipGetLastError();
    }
    if (a.block_mlp && a.pe == 4) {
#define COW_LAUNCH_PE(M, D, S) hipLaunchKernelGGL((march_fwd_pe_kernel<M, D, S>), grid, block, 0, s, a)
        if (dt == 1) {
            if (a.mode == 1)
                COW_LAUNCH_PE(1, 1, false);
            else
                COW_LAUNCH_PE(0, 1, false);
        } else if (a.mode == 1) {
            if (a.use_sparse)
                COW_LAUNCH_PE(1, 0, true);
            else
                COW_LAUNCH_PE(1, 0, false);
        } else {
            if (a.use_sparse)
                COW_LAUNCH_PE(0, 0, true);
            else
                COW_LAUNCH_PE(0, 0, false);
        }
#undef COW_LAUNCH_PE
        return hipGetLastError();
    }
#define COW_LAUNCH(M, S) hipLaunchKernelGGL((march_fwd_kernel<M, S>), grid, block, 0, s, a)
    if (dt == 1) {
        if (a.mode == 1)
            hipLaunchKernelGGL(march_fwd_f32_kernel<1>, grid, block, 0, s, a);
        else
            hipLaunchKernelGGL(march_fwd_f32_kernel<0>, grid, block, 0, s, a);
    } else if (a.mode == 1) {
        if (a.use_sparse)
            COW_LAUNCH(1, true);
        else
            COW_LAUNCH(1, false);
    } else {
        if (a.use_sparse)
            COW_LAUNCH(0, true);
        else
            COW_LAUNCH(0, false);
    }
#undef COW_LAUNCH
    return hipGetLastError();
}

__global__ void reset_counter_kernel(int32_t* c) {
    if (threadIdx.x < kXcds) c[threadIdx.x] = 0;  // one work counter per XCD
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
// occupancy: conservative max-bound of the interpolated density
// ---------------------------------------------------------------------------

// density-channel texel as the decision sees it: fl(fl(q s) + o), or the
// stored fp32 value
__device__ inline float texel0(const DevBlock* B, int tex, int idx) {
    const void* base = tex == 0 ? B->grid : B->plane[tex - 1];
    if (B->dtype == 0) {
        const float q = (float)reinterpret_cast<const uint8_t*>(base)[(size_t)idx * 8];
        const float m = q * B->scale[tex][0];
        return m + B->offset[tex][0];
    }
    return reinterpret_cast<const float*>(base)[(size_t)idx * 8];
}

// A cell is occupied iff the largest density texel of each texture over the
// cell's interpolation support, summed ((G + XY) + XZ) + YZ, exceeds ln 0.01:
// every sample of an unoccupied cell then has density <= 0.01 (interpolation
// is a convex combination and exp is monotone), and such cells are skipped.
__global__ void occupancy_kernel(const DevBlock* blocks, int entry) {
    const DevBlock* B = blocks + entry;
    const int O = B->O, R = B->R, Rp = B->Rp;
    const int ox = B->od[0], oy = B->od[1], oz = B->od[2];
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= ox * oy * oz) return;
    const int c3[3] = {cell % ox, (cell / ox) % oy, cell / (ox * oy)};
    const int s = R / O, sp = Rp / O;
    int glo[3], ghi[3], plo[3], phi[3];
    for (int a = 0; a < 3; ++a) {
        glo[a] = max(c3[a] * s - 1, 0);
        ghi[a] = min((c3[a] + 1) * s, B->gd[a] - 1);
        plo[a] = max(c3[a] * sp - 1, 0);
        phi[a] = min((c3[a] + 1) * sp, B->pd[a] - 1);
    }
    const int gx = B->gd[0], gy = B->gd[1];
    float mg = -INFINITY;
    for (int z = glo[2]; z <= ghi[2]; ++z)
        for (int y = glo[1]; y <= ghi[1]; ++y)
            for (int x = glo[0]; x <= ghi[0]; ++x) mg = fmaxf(mg, texel0(B, 0, (z * gy + y) * gx + x));
    const int au[3] = {0, 0, 1}, av[3] = {1, 2, 2};
    float mp[3];
    for (int p = 0; p < 3; ++p) {
        float m = -INFINITY;
        const int row = B->pd[au[p]];
        for (int v = plo[av[p]]; v <= phi[av[p]]; ++v)
            for (int u = plo[au[p]]; u <= phi[au[p]]; ++u) m = fmaxf(m, texel0(B, 1 + p, v * row + u));
        mp[p] = m;
    }
    const float thresh = -0x1.26bb1cp+2f;  // fp32 nearest to ln(0.01)
    const float bound = ((mg + mp[0]) + mp[1]) + mp[2];
    const_cast<uint8_t*>(B->occ)[cell] = bound > thresh ? 1 : 0;
}

hipError_t launch_occupancy(const DevBlock* blocks, int entry, int n_cells, hipStream_t s) {
    const int n = n_cells;
    hipLaunchKernelGGL(occupancy_kernel, dim3((n + 63) / 64), dim3(64), 0, s, blocks, entry);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// multi-level occupancy (Sec. 3, the grids psi; Sec. 4.5: downsampled by
// max-pooling)
// ---------------------------------------------------------------------------
__device__ inline int level_dim(int n, int l) { return max(n >> l, 1); }

__device__ inline const uint8_t* pyramid_level(const DevBlock* B, int l) {
    if (l == 0) return B->occ;
    const uint8_t* p = B->occ_pyr;
    for (int j = 1; j < l; ++j)
        p += (size_t)level_dim(B->od[0], j) * level_dim(B->od[1], j) * level_dim(B->od[2], j);
    return p;
}

// Level l from level l - 1: cell x is the OR of the cells y with y >> 1 == x,
// at most 2 x 2 x 2 of them (fewer where the finer level is one cell wide).
__global__ void occ_pool_kernel(const DevBlock* blocks, int entry, int l) {
    const DevBlock* B = blocks + entry;
    const int nx = level_dim(B->od[0], l), ny = level_dim(B->od[1], l), nz = level_dim(B->od[2], l);
    const int fx = level_dim(B->od[0], l - 1), fy = level_dim(B->od[1], l - 1), fz = level_dim(B->od[2], l - 1);
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= nx * ny * nz) return;
    const int x = cell % nx, y = (cell / nx) % ny, z = cell / (nx * ny);
    const uint8_t* src = pyramid_level(B, l - 1);
    int any = 0;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx) {
                const int cx = 2 * x + dx, cy = 2 * y + dy, cz = 2 * z + dz;
                if (cx < fx && cy < fy && cz < fz) any |= src[((size_t)cz * fy + cy) * fx + cx];
            }
    const_cast<uint8_t*>(pyramid_level(B, l))[cell] = any ? 1 : 0;
}

// Per base cell: 0 if occupied, else 1 + the coarsest level whose cell holding
// it is empty.  The levels are nested (an empty cell's parent may be occupied,
// never the reverse), so the first occupied level ends the climb.
__global__ void occ_skip_kernel(const DevBlock* blocks, int entry) {
    const DevBlock* B = blocks + entry;
    const int ox = B->od[0], oy = B->od[1], oz = B->od[2];
    const int cell = blockIdx.x * blockDim.x + threadIdx.x;
    if (cell >= ox * oy * oz) return;
    const int x = cell % ox, y = (cell / ox) % oy, z = cell / (ox * oy);
    int s = 0;
    if (!B->occ[cell]) {
        s = 1;
        for (int l = 1; l <= B->n_levels; ++l) {
            const int nx = level_dim(ox, l), ny = level_dim(oy, l);
            const size_t c = ((size_t)(z >> l) * ny + (y >> l)) * nx + (x >> l);
            if (pyramid_level(B, l)[c]) break;
            s = l + 1;
        }
    }
    const_cast<uint8_t*>(B->skip)[cell] = (uint8_t)s;
}

hipError_t launch_occupancy_pyramid(const DevBlock* blocks, int entry, int n_levels, const int od[3],
                                    hipStream_t s) {
    for (int l = 1; l <= n_levels; ++l) {
        const int n = std::max(od[0] >> l, 1) * std::max(od[1] >> l, 1) * std::max(od[2] >> l, 1);
        hipLaunchKernelGGL(occ_pool_kernel, dim3((n + 63) / 64), dim3(64), 0, s, blocks, entry, l);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int n = od[0] * od[1] * od[2];
    hipLaunchKernelGGL(occ_skip_kernel, dim3((n + 63) / 64), dim3(64), 0, s, blocks, entry);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sparse grid: copy each occupied cell's interpolation support to a brick
// ---------------------------------------------------------------------------
__global__ void pack_bricks_kernel(const DevBlock* blocks, int entry) {
    const DevBlock* B = blocks + entry;
    const int O = B->O, R = B->R, s = R / O, s2 = s + 2;
    const int ox = B->od[0], oy = B->od[1];
    const int gx = B->gd[0], gy = B->gd[1], gz = B->gd[2];
    const int cell = blockIdx.x;
    const int slot = B->brick_slot[cell];
    if (slot < 0) return;
    const int cx = cell % ox, cy = (cell / ox) % oy, cz = cell / (ox * oy);
    const uint2* G = reinterpret_cast<const uint2*>(B->grid);
    uint2* dst = reinterpret_cast<uint2*>(const_cast<uint8_t*>(B->bricks)) + (size_t)slot * (s2 * s2 * s2);
    for (int t = threadIdx.x; t < s2 * s2 * s2; t += blockDim.x) {
        const int bx = t % s2, by = (t / s2) % s2, bz = t / (s2 * s2);
        const int x = min(max(cx * s - 1 + bx, 0), gx - 1);
        const int y = min(max(cy * s - 1 + by, 0), gy - 1);
        const int z = min(max(cz * s - 1 + bz, 0), gz - 1);
        dst[t] = G[((size_t)z * gy + y) * gx + x];
    }
}

hipError_t launch_pack_bricks(const DevBlock* blocks, int entry, int n_cells, int, const int32_t*, hipStream_t st) {
    hipLaunchKernelGGL(pack_bricks_kernel, dim3(n_cells), dim3(256), 0, st, blocks, entry);
    return hipGetLastError();
}

}  // namespace cow
