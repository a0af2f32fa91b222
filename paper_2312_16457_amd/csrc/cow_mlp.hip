// Deferred MLP of the render path (Eq. "deferred"): forward on MFMA after
// the merge, and its backward (recompute from aux, MFMA outer-product GEMMs
// for the weight gradients) for gfx950.
#include <hip/hip_runtime.h>

#include "cow_device.h"

namespace cow {

// ---------------------------------------------------------------------------
// deferred MLP on MFMA: x = [C_d, F, PE(d)] -> 16 -> 16 -> 3, C = C_d + sigmoid(z)
// ---------------------------------------------------------------------------
//
// v_mfma_f32_16x16x4f32 computes D[16][16] += A[16][4] B[4][16]; lane l
// supplies A[l%16][l/16] and B[l/16][l%16] and holds D[4(l/16)+r][l%16].
// Each layer is computed transposed, H^T = W X^T, with pixels along the 16
// columns; for layers 2 and 3 the K index of (step s, lane group g) is 4g+s,
// so the B operand is exactly the lane's own previous-layer output.

template <int L>
__global__ __launch_bounds__(256) void mlp_fwd_kernel(MlpArgs a) {
    using S = MlpShape<L>;
    constexpr int NI = S::NI, KS = (NI + 3) / 4;  // first-layer inputs, MFMA steps over them
    __shared__ float W[S::N + 1];
    __shared__ float X[4][64][NI + 1];
    for (int i = threadIdx.x; i < S::N; i += blockDim.x) W[i] = a.mlp[i];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t base = ((int64_t)blockIdx.x * 4 + wave) * 64;
    const int64_t pix = base + lane;
    float x[NI];
#pragma unroll
    for (int k = 0; k < NI; ++k) x[k] = 0.0f;
    if (pix < a.n_pix) {
        const float4 lo = reinterpret_cast<const float4*>(a.aux)[2 * pix];
        const float4 hi = reinterpret_cast<const float4*>(a.aux)[2 * pix + 1];
        const float A[7] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z};
        float d[3];
        pixel_direction(a.views, a.n_views, pix, d);
        mlp_input<L>(A, d, x);
    }
#pragma unroll
    for (int k = 0; k < NI; ++k) X[wave][lane][k] = x[k];
    __syncthreads();
    const float *W1 = W, *b1 = W + S::B1, *W2 = W + S::W2, *b2 = W + S::B2, *W3 = W + S::W3, *b3 = W + S::B3;
    const int j = lane & 15, g = lane >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        floatx4 h = {b1[4 * g + 0], b1[4 * g + 1], b1[4 * g + 2], b1[4 * g + 3]};
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            const int k = g + 4 * s;
            const float av = k < NI ? W1[j * NI + k] : 0.0f;
            const float bv = k < NI ? X[wave][16 * t + j][k] : 0.0f;
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
    if (a.pe == 4)
        hipLaunchKernelGGL(mlp_fwd_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(mlp_fwd_kernel<0>, dim3((unsigned)blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

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

template <int L>
__global__ __launch_bounds__(256) void mlp_bwd_kernel(MlpBwdArgs a) {
    using S = MlpShape<L>;
    constexpr int NI = S::NI;
    constexpr int XT = (NI + 1 + 15) / 16, XW = 16 * XT;  // column tiles of [x, 1] for dW1 and db1
    __shared__ float W[S::N + 1];
    __shared__ float S_dh1[4][64][17];
    __shared__ float S_x[4][64][XW + 1];
    __shared__ float S_dh2[4][64][17];
    __shared__ float S_h1[4][64][17];
    __shared__ float S_dz[4][64][4];
    __shared__ float S_h2[4][64][17];
    __shared__ float S_red[4][S::N + 1];
    for (int i = threadIdx.x; i < S::N; i += blockDim.x) W[i] = a.mlp[i];
    __syncthreads();
    const float *W1 = W, *b1 = W + S::B1, *W2 = W + S::W2, *b2 = W + S::B2, *W3 = W + S::W3, *b3 = W + S::B3;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = lane & 15, g = lane >> 4;
    floatx4 acc1[XT], acc2 = {0, 0, 0, 0}, acc3 = {0, 0, 0, 0};
#pragma unroll
    for (int t = 0; t < XT; ++t) acc1[t] = floatx4{0, 0, 0, 0};
    float bias_acc = 0.0f;  // lanes 0..15: db2[lane]; lanes 16..18: db3[lane-16]
    const int64_t n_chunks = (a.n_pix + 63) / 64;
    for (int64_t chunk = (int64_t)blockIdx.x * 4 + wave; chunk < n_chunks; chunk += (int64_t)gridDim.x * 4) {
        const int64_t pix = chunk * 64 + lane;
        const bool act = pix < a.n_pix;
        float x[NI], gr[3] = {0, 0, 0};
#pragma unroll
        for (int k = 0; k < NI; ++k) x[k] = 0.0f;
        if (act) {
            const float4 lo = reinterpret_cast<const float4*>(a.aux)[2 * pix];
            const float4 hi = reinterpret_cast<const float4*>(a.aux)[2 * pix + 1];
            const float A[7] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z};
            float d[3];
            pixel_direction(a.views, a.n_views, pix, d);
            mlp_input<L>(A, d, x);
            gr[0] = a.grad_rgb[3 * pix], gr[1] = a.grad_rgb[3 * pix + 1], gr[2] = a.grad_rgb[3 * pix + 2];
        }
        float pre1[16], h1[16], pre2[16], h2[16], dz[3], dh2[16], dh1[16];
#pragma unroll
        for (int o = 0; o < 16; ++o) {
            float s = b1[o];
#pragma unroll
            for (int i = 0; i < NI; ++i) s = fmaf(W1[o * NI + i], x[i], s);
            pre1[o] = s;
            h1[o] = fmaxf(s, 0.0f);
        }
#pragma unroll
        for (int o = 0; o < 16; ++o) {
            float s = b2[o];
            #pragma unroll
            for (int i = 0; i < 16; ++i) s = fmaf(W2[o * 16 + i], h1[i], s);
            pre2[o] = s;
            h2[o] = fmaxf(s, 0.0f);
        }
#pragma unroll
        for (int o = 0; o < 3; ++o) {
            float s = b3[o];
            #pragma unroll
            for (int i = 0; i < 16; ++i) s = fmaf(W3[o * 16 + i], h2[i], s);
            const float sg = sigmoidf_(s);
            dz[o] = act ? gr[o] * sg * (1.0f - sg) : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            float s = 0.0f;
            #pragma unroll
            for (int o = 0; o < 3; ++o) s = fmaf(W3[o * 16 + i], dz[o], s);
            dh2[i] = pre2[i] > 0.0f ? s : 0.0f;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            float s = 0.0f;
            #pragma unroll
            for (int o = 0; o < 16; ++o) s = fmaf(W2[o * 16 + i], dh2[o], s);
            dh1[i] = pre1[i] > 0.0f ? s : 0.0f;
        }
        if (act) {
            float u[8];
#pragma unroll
            for (int i = 0; i < 7; ++i) {  // the direction inputs are constants
                float s = 0.0f;
                #pragma unroll
                for (int o = 0; o < 16; ++o) s = fmaf(W1[o * NI + i], dh1[o], s);
                u[i] = s + (i < 3 ? gr[i] : 0.0f);
            }
            u[7] = 0.0f;
            float4* u4 = reinterpret_cast<float4*>(a.u);
            u4[2 * pix] = make_float4(u[0], u[1], u[2], u[3]);
            u4[2 * pix + 1] = make_float4(u[4], u[5], u[6], u[7]);
        }
        // stage per-pixel vectors for the outer-product GEMMs
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            S_dh1[wave][lane][i] = dh1[i];
            S_dh2[wave][lane][i] = dh2[i];
            S_h1[wave][lane][i] = h1[i];
            S_h2[wave][lane][i] = h2[i];
        }
#pragma unroll
        for (int i = 0; i < XW; ++i) S_x[wave][lane][i] = i < NI ? x[i] : (i == NI && act ? 1.0f : 0.0f);
#pragma unroll
        for (int i = 0; i < 3; ++i) S_dz[wave][lane][i] = dz[i];
        S_dz[wave][lane][3] = 0.0f;
        __builtin_amdgcn_s_waitcnt(0);
        __builtin_amdgcn_wave_barrier();
        for (int s = 0; s < 16; ++s) {
            const int p = 4 * s + g;  // pixel of this lane's K slot
            const float dh1p = S_dh1[wave][p][j];
#pragma unroll
            for (int t = 0; t < XT; ++t)
                acc1[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(dh1p, S_x[wave][p][16 * t + j], acc1[t], 0, 0, 0);
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
#pragma unroll
        for (int t = 0; t < XT; ++t) {
            const int col = 16 * t + j;
            if (col < NI) red[i * NI + col] = acc1[t][r];
            if (col == NI) red[S::B1 + i] = acc1[t][r];
        }
        red[S::W2 + i * 16 + j] = acc2[r];
        if (i < 3) red[S::W3 + i * 16 + j] = acc3[r];
    }
    if (lane < 16) red[S::B2 + lane] = bias_acc;
    if (lane >= 16 && lane < 19) red[S::B3 + lane - 16] = bias_acc;
    __syncthreads();
    for (int i = threadIdx.x; i < S::N; i += blockDim.x) {
        const float s = ((S_red[0][i] + S_red[1][i]) + S_red[2][i]) + S_red[3][i];
        atomicAdd(a.grad_mlp + i, s);
    }
}

hipError_t launch_mlp_bwd(const MlpBwdArgs& a, hipStream_t s) {
    if (a.n_pix <= 0) return hipSuccess;
    const int64_t chunks = (a.n_pix + 63) / 64;
    int64_t groups = (chunks + 3) / 4;
    if (groups > 1024) groups = 1024;
    if (a.pe == 4)
        hipLaunchKernelGGL(mlp_bwd_kernel<4>, dim3((unsigned)groups), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(mlp_bwd_kernel<0>, dim3((unsigned)groups), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace cow
