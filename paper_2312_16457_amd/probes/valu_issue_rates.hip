// Vector-ALU issue rates on gfx950: a measurement aid, not part of the
// render path.  Each lane runs eight independent chains of one instruction
// kind (inline assembly, so the loop holds exactly that instruction, 32 of
// them per loop trip), 2048 workgroups of 256 lanes (eight waves per SIMD);
// the kernel time from HIP events gives cycles per wave64 instruction per
// SIMD at the given clock (the nominal 2.4 GHz unless another is passed; at a
// lower real clock the true cycle counts are proportionally smaller).  It also checks the
// semantic the byte-select (SDWA) form of v_mul_f32 is used for: with fp32
// denormal inputs preserved, src1_sel:BYTE_k reads byte k of a word as the
// fp32 denormal b 2^-149, so w 2^125 times it is w b 2^-24, rounded once.
//
// Build and run (from the repository root):
//   hipcc --offload-arch=gfx950 -O3 -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o valu_issue_rates paper_2312_16457_amd/probes/valu_issue_rates.hip
//   ./valu_issue_rates [clock_GHz]
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#define CHECK(x)                                                                      \
    do {                                                                              \
        hipError_t e_ = (x);                                                          \
        if (e_ != hipSuccess) {                                                       \
            fprintf(stderr, "%s: %s\n", #x, hipGetErrorString(e_));                   \
            exit(1);                                                                  \
        }                                                                             \
    } while (0)

constexpr int kChains = 8;
constexpr int kThreads = 256;
constexpr int kBlocks = 2048;

#define OP1(asmstr) asm volatile(asmstr : "+v"(a[c]))
#define OP2(asmstr) asm volatile(asmstr : "+v"(a[c]) : "v"(b))

template <int K>
__global__ void __launch_bounds__(kThreads) issue_kernel(float* out, int iters, float seed) {
    float a[kChains];
    const unsigned bw = 0x3f7f1f40u ^ (threadIdx.x * 2654435761u);
    const float b = __uint_as_float((bw & 0x007fffffu) | 0x3f000000u);  // in [0.5, 1)
#pragma unroll
    for (int c = 0; c < kChains; ++c) a[c] = seed + 1e-3f * (float)(threadIdx.x + c);
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < kChains; ++c) {
            if (K == 0) OP2("v_mul_f32 %0, %0, %1");
            if (K == 1) OP2("v_fmac_f32 %0, %1, %1");
            if (K == 2) OP2("v_fma_f32 %0, %1, %1, %0");
            if (K == 3) OP2("v_fma_mix_f32 %0, %1, %1, %0 op_sel_hi:[0,1,0]");
            if (K == 4) OP2("v_mov_b32_sdwa %0, %1 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:BYTE_1");
            if (K == 5) OP2("v_mul_f32_sdwa %0, %1, %0 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2");
            if (K == 6) OP2("v_perm_b32 %0, %0, %1, %1");
            if (K == 7) OP2("v_and_b32 %0, 0xff00ff, %0");
            if (K == 8) OP1("v_cvt_i32_f32 %0, %0");
            if (K == 9) OP1("v_floor_f32 %0, %0");
            if (K == 10) OP1("v_fract_f32 %0, %0");
            if (K == 11) OP2("v_med3_f32 %0, %0, 0, %1");
            if (K == 12) OP2("v_add_lshl_u32 %0, %0, %1, 3");
            if (K == 13) OP2("v_add_u32 %0, %0, %1");
            if (K == 14) OP1("v_exp_f32 %0, %0");
            if (K == 15) OP1("v_rcp_f32 %0, %0");
            if (K == 16) OP2("v_fmaak_f32 %0, %1, %0, 0xbf000000");
            if (K == 17) OP2("v_sub_f32 %0, %1, %0");
            if (K == 18) OP1("v_cvt_f32_ubyte1 %0, %0");
            if (K == 19) OP2("v_xor_b32 %0, %0, %1");
        }
    }
    float s = 0.0f;
#pragma unroll
    for (int c = 0; c < kChains; ++c) s += a[c];
    out[blockIdx.x * kThreads + threadIdx.x] = s;
}

// (w 2^125) * byte k of word, through the byte-select form, k = 0..3
__global__ void sdwa_check_kernel(const unsigned* words, const float* w, float* out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned x = words[i];
    const float ws = w[i] * 0x1p125f;
    float r0, r1, r2, r3;
    asm volatile("v_mul_f32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_0"
                 : "=v"(r0) : "v"(ws), "v"(x));
    asm volatile("v_mul_f32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_1"
                 : "=v"(r1) : "v"(ws), "v"(x));
    asm volatile("v_mul_f32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_2"
                 : "=v"(r2) : "v"(ws), "v"(x));
    asm volatile("v_mul_f32_sdwa %0, %1, %2 dst_sel:DWORD dst_unused:UNUSED_PAD src0_sel:DWORD src1_sel:BYTE_3"
                 : "=v"(r3) : "v"(ws), "v"(x));
    out[4 * i + 0] = r0;
    out[4 * i + 1] = r1;
    out[4 * i + 2] = r2;
    out[4 * i + 3] = r3;
}

template <int K>
float time_kind(float* out, int iters) {
    hipEvent_t e0, e1;
    CHECK(hipEventCreate(&e0));
    CHECK(hipEventCreate(&e1));
    hipLaunchKernelGGL(issue_kernel<K>, dim3(kBlocks), dim3(kThreads), 0, 0, out, iters, 1.0f);
    CHECK(hipEventRecord(e0, 0));
    hipLaunchKernelGGL(issue_kernel<K>, dim3(kBlocks), dim3(kThreads), 0, 0, out, iters, 1.0f);
    CHECK(hipEventRecord(e1, 0));
    CHECK(hipEventSynchronize(e1));
    float ms = 0.0f;
    CHECK(hipEventElapsedTime(&ms, e0, e1));
    CHECK(hipEventDestroy(e0));
    CHECK(hipEventDestroy(e1));
    return ms;
}

template <int K>
void report(const char* name, float* out, int iters, double ghz, int simds) {
    const float ms = time_kind<K>(out, iters);
    const double waves = (double)kBlocks * kThreads / 64.0;
    const double instr_per_simd = waves * iters * 4 * kChains / simds;
    printf("| `%s` | %.2f |\n", name, ms * 1e-3 * ghz * 1e9 / instr_per_simd);
}

int main(int argc, char** argv) {
    const double ghz = argc > 1 ? atof(argv[1]) : 2.4;
    hipDeviceProp_t prop;
    CHECK(hipGetDeviceProperties(&prop, 0));
    const int simds = prop.multiProcessorCount * 4;
    // semantics of the byte-select form
    const int n = 1 << 16;
    unsigned* hw = (unsigned*)malloc(n * 4);
    float* hwt = (float*)malloc(n * 4);
    unsigned s = 12345u;
    for (int i = 0; i < n; ++i) {
        s = s * 1664525u + 1013904223u;
        hw[i] = s;
        s = s * 1664525u + 1013904223u;
        hwt[i] = (float)(s >> 8) / 16777216.0f;
    }
    unsigned* dw;
    float *dwt, *dout;
    CHECK(hipMalloc(&dw, n * 4));
    CHECK(hipMalloc(&dwt, n * 4));
    CHECK(hipMalloc(&dout, (size_t)4 * n * 4));
    CHECK(hipMemcpy(dw, hw, n * 4, hipMemcpyHostToDevice));
    CHECK(hipMemcpy(dwt, hwt, n * 4, hipMemcpyHostToDevice));
    hipLaunchKernelGGL(sdwa_check_kernel, dim3(n / 256), dim3(256), 0, 0, dw, dwt, dout);
    float* ho = (float*)malloc((size_t)4 * n * 4);
    CHECK(hipMemcpy(ho, dout, (size_t)4 * n * 4, hipMemcpyDeviceToHost));
    long bad = 0;
    for (int i = 0; i < n; ++i)
        for (int k = 0; k < 4; ++k) {
            const float b = (float)((hw[i] >> (8 * k)) & 0xffu);
            // reference: w b 2^-24 rounded once to fp32 (the product is exact in fp64)
            const float ref = (float)((double)hwt[i] * (double)b * 0x1p-24);
            if (memcmp(&ref, &ho[4 * i + k], 4) != 0) ++bad;
        }
    printf("byte-select check: %ld of %d products differ from w b 2^-24 rounded once\n", bad, 4 * n);
    // issue rates
    float* out;
    CHECK(hipMalloc(&out, (size_t)kBlocks * kThreads * 4));
    const int iters = 1024;
    printf("| Instruction | Cycles per wave64 instruction per SIMD (kernel time at %.2f GHz) |\n|---|---|\n", ghz);
    report<0>("v_mul_f32 (VOP2)", out, iters, ghz, simds);
    report<1>("v_fmac_f32 (VOP2)", out, iters, ghz, simds);
    report<2>("v_fma_f32 (VOP3)", out, iters, ghz, simds);
    report<3>("v_fma_mix_f32 (VOP3P)", out, iters, ghz, simds);
    report<4>("v_mov_b32_sdwa, byte select (VOP1 + SDWA)", out, iters, ghz, simds);
    report<5>("v_mul_f32_sdwa, byte select (VOP2 + SDWA)", out, iters, ghz, simds);
    report<6>("v_perm_b32 (VOP3)", out, iters, ghz, simds);
    report<7>("v_and_b32 (VOP2, literal)", out, iters, ghz, simds);
    report<8>("v_cvt_i32_f32 (VOP1)", out, iters, ghz, simds);
    report<9>("v_floor_f32 (VOP1)", out, iters, ghz, simds);
    report<10>("v_fract_f32 (VOP1)", out, iters, ghz, simds);
    report<11>("v_med3_f32 (VOP3)", out, iters, ghz, simds);
    report<12>("v_add_lshl_u32 (VOP3)", out, iters, ghz, simds);
    report<13>("v_add_u32 (VOP2)", out, iters, ghz, simds);
    report<14>("v_exp_f32", out, iters, ghz, simds);
    report<15>("v_rcp_f32", out, iters, ghz, simds);
    report<16>("v_fmaak_f32 (VOP2, literal)", out, iters, ghz, simds);
    report<17>("v_sub_f32 (VOP2)", out, iters, ghz, simds);
    report<18>("v_cvt_f32_ubyte1 (VOP1)", out, iters, ghz, simds);
    report<19>("v_xor_b32 (VOP2)", out, iters, ghz, simds);
    CHECK(hipFree(out));
    CHECK(hipFree(dw));
    CHECK(hipFree(dwt));
    CHECK(hipFree(dout));
    free(hw);
    free(hwt);
    free(ho);
    return bad == 0 ? 0 : 2;
}
