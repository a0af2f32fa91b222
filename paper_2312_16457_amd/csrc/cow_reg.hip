// Sparsity regulariser of the training objective for gfx950 (City-on-Web,
// arXiv 2312.16457, Sec. 4.3): mean opacity at given points and its
// gradient into the density channel of the textures.
#include <hip/hip_runtime.h>

#include "cow_device.h"

namespace cow {

// One point per lane.  The entry a point falls in is found against every
// entry's box (first match wins); the wave then visits the entries its lanes
// hit one at a time, so that each entry's descriptor stays wave-uniform in
// scalar registers as in the march.
template <int DT>
__global__ __launch_bounds__(256) void sparsity_kernel(SparsityArgs s) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < s.n;
    float p[3] = {0.0f, 0.0f, 0.0f};
    if (valid)
        for (int c = 0; c < 3; ++c) p[c] = s.pts[3 * i + c];
    int first = -1;
    for (int j = 0; j < s.n_set; ++j) {
        const DevBlock* B = s.blocks + ufl(s.set[j]);
        bool in = valid && first < 0;
        for (int c = 0; c < 3; ++c) in = in && (uff(B->lo[c]) <= p[c] && p[c] < uff(B->hi[c]));
        if (in) first = j;
    }
    float alpha = 0.0f;
    for (int j = 0; j < s.n_set; ++j) {
        if (!__any(first == j)) continue;
        const int e = ufl(s.set[j]);
        BlockU b;
        load_block<DT>(s.blocks + e, b);
        if (first != j) continue;
        // texture coordinate: p - lo, or the contracted coordinate of a
        // contracted boundary block (its box fills the middle half of its
        // textures), as the march reads it
        float q[3];
        if (b.contracted)
            contract_q(b.lo, b.hi, p, q);
        else
            for (int c = 0; c < 3; ++c) q[c] = p[c] - b.lo[c];
        const int cell = occ_cell(b, q);
        if (b.occ[cell] == 0) continue;  // the render's density is zero here
        Taps T;
        float sigma;
        if (DT == 0) {
            float raw[kNch];
            raw_u8<false>(b, q, cell, raw);
            sigma = density_u8(raw);
        } else {
            sample_taps(b, q, T);
            sigma = __expf(raw0_f32(b, T));
        }
        alpha = alpha_of(sigma * s.delta);
        if (DT == 1 && s.grad_grid) {
            // d(scale alpha)/draw_0 = scale delta sigma exp(-sigma delta),
            // scattered through range-checked buffer atomics
            const float g = s.scale * s.delta * sigma * (1.0f - alpha);
            float* gp[4] = {ufp(s.grad_grid[e]), ufp(s.grad_plane[3 * e]), ufp(s.grad_plane[3 * e + 1]),
                            ufp(s.grad_plane[3 * e + 2])};
            __amdgpu_buffer_rsrc_t gr[4];
            gr[0] = tex_rsrc(gp[0], grid_texels(b) * 32u);
            for (int t = 1; t < 4; ++t) gr[t] = tex_rsrc(gp[t], plane_texels(b, t - 1) * 32u);
#pragma unroll
            for (int k = 0; k < 20; ++k) {
                const int tex = pair_tex(k >> 1);
                if (gp[tex])
                    __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(T.w[k] * g, gr[tex], 32 * (T.pidx[k >> 1] + (k & 1)),
                                                                    0, 0);
            }
        }
    }
    if (valid && s.alpha) s.alpha[i] = alpha;
    // wave sum of this wave's share of the loss, one atomic per wave
    float part = valid ? s.scale * alpha : 0.0f;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) part += __shfl_xor(part, off);
    if ((threadIdx.x & 63) == 0 && part != 0.0f) atomicAdd(s.loss, part);
}

hipError_t launch_sparsity(const SparsityArgs& a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    const dim3 block(256), grid((unsigned)((a.n + 255) / 256));
    if (a.dtype == 0)
        hipLaunchKernelGGL(sparsity_kernel<0>, grid, block, 0, st, a);
    else
        hipLaunchKernelGGL(sparsity_kernel<1>, grid, block, 0, st, a);
    return hipGetLastError();
}

}  // namespace cow
