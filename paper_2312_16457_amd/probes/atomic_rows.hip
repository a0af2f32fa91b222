// Rate of 64-lane fp32 atomic adds on one MI355X by the 64-byte segments
// they touch (a measurement aid for the adjoint's scatter, not part of the
// render path).  Each wave instruction adds 1.0 to four rows of 16 floats,
// 16 lanes per row, the way the adjoint's transposed scatter does; the rows
// are chosen by a hash over a buffer of the given footprint.  Patterns:
//   aligned    four rows on four 64-byte-aligned segments
//   straddle   every row 32 bytes off alignment (two segments each)
//   duplicate  rows 0 and 1, 2 and 3 of an instruction on the same segment
// The kernel time comes from HIP events; the L2's request count for each
// launch from rocprofv3 (TCC_ATOMIC_sum), run on this program.  After each
// launch the program checks that the buffer holds every add exactly.
//
//   hipcc --offload-arch=gfx950 -O3 -munsafe-fp-atomics \
//         -Xclang -target-feature -Xclang -packed-fp32-ops \
//         -o atomic_rows paper_2312_16457_amd/probes/atomic_rows.hip
//   ./atomic_rows
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <vector>

#define CHECK(x)                                                                     \
    do {                                                                             \
        hipError_t e_ = (x);                                                         \
        if (e_ != hipSuccess) {                                                      \
            fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, hipGetErrorString(e_)); \
            exit(1);                                                                 \
        }                                                                            \
    } while (0)

enum { kAligned = 0, kStraddle = 1, kDuplicate = 2 };

__device__ inline uint32_t mix(uint32_t h) {
    h ^= h >> 16;
    h *= 0x7feb352dU;
    h ^= h >> 15;
    h *= 0x846ca68bU;
    h ^= h >> 16;
    return h;
}

// nseg: segments the rows may start at; the buffer holds nseg + 1 segments,
// so a straddling row stays inside it
__global__ void rows_kernel(float* buf, uint32_t nseg, int iters, int mode) {
    const __amdgpu_buffer_rsrc_t r =
        __builtin_amdgcn_make_buffer_rsrc(buf, (short)0, (int)((nseg + 1) * 64u), 0x00020000);
    const int lane = threadIdx.x & 63, e = lane & 15, sub = lane >> 4;
    const uint32_t wave = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    const int row = mode == kDuplicate ? (sub >> 1) : sub;
    for (int i = 0; i < iters; ++i) {
        const uint32_t seg = mix(wave * 0x9e3779b9U + (uint32_t)i * 0x85ebca6bU + (uint32_t)row * 0xc2b2ae35U) % nseg;
        const int off = (int)(seg * 64u) + (mode == kStraddle ? 32 : 0) + 4 * e;
        __builtin_amdgcn_raw_ptr_buffer_atomic_fadd_f32(1.0f, r, off, 0, 0);
    }
}

__global__ void sum_kernel(const float* buf, size_t n, unsigned long long* out) {
    unsigned long long s = 0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        s += (unsigned long long)buf[i];
    atomicAdd(out, s);
}

int main() {
    const int blocks = 4096, threads = 256, iters = 256;
    const long long rows = (long long)blocks * (threads / 64) * iters * 4;
    const uint32_t footprints_mib[] = {1, 64, 2560};
    const char* names[] = {"aligned", "straddle", "duplicate"};
    printf("| footprint | pattern | rows | segments touched | ms | G segments/s |\n|---|---|---|---|---|---|\n");
    for (uint32_t mib : footprints_mib) {
        const uint32_t nseg = (uint32_t)((size_t)mib * 1024 * 1024 / 64) - 1;
        const size_t n = (size_t)(nseg + 1) * 16;
        float* buf;
        unsigned long long* d_sum;
        CHECK(hipMalloc(&buf, n * sizeof(float)));
        CHECK(hipMalloc(&d_sum, sizeof(unsigned long long)));
        hipEvent_t e0, e1;
        CHECK(hipEventCreate(&e0));
        CHECK(hipEventCreate(&e1));
        for (int mode = 0; mode < 3; ++mode) {
            CHECK(hipMemset(buf, 0, n * sizeof(float)));
            // warm-up launch (its adds are counted in the check below)
            hipLaunchKernelGGL(rows_kernel, dim3(blocks), dim3(threads), 0, 0, buf, nseg, iters, mode);
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(e0, 0));
            hipLaunchKernelGGL(rows_kernel, dim3(blocks), dim3(threads), 0, 0, buf, nseg, iters, mode);
            CHECK(hipGetLastError());
            CHECK(hipEventRecord(e1, 0));
            CHECK(hipEventSynchronize(e1));
            float ms = 0.0f;
            CHECK(hipEventElapsedTime(&ms, e0, e1));
            CHECK(hipMemset(d_sum, 0, sizeof(unsigned long long)));
            hipLaunchKernelGGL(sum_kernel, dim3(1024), dim3(256), 0, 0, buf, n, d_sum);
            CHECK(hipGetLastError());
            unsigned long long got = 0;
            CHECK(hipMemcpy(&got, d_sum, sizeof(got), hipMemcpyDeviceToHost));
            const unsigned long long want = 2ull * (unsigned long long)rows * 16ull;
            if (got != want) {
                fprintf(stderr, "check failed: %s at %u MiB: %llu adds, expected %llu\n", names[mode], mib, got, want);
                return 2;
            }
            const double segs = (double)rows * (mode == kStraddle ? 2.0 : 1.0);
            printf("| %u MiB | %s | %lld | %.0f | %.3f | %.2f |\n", mib, names[mode], rows, segs, ms,
                   segs / (ms * 1e-3) / 1e9);
        }
        CHECK(hipEventDestroy(e0));
        CHECK(hipEventDestroy(e1));
        CHECK(hipFree(d_sum));
        CHECK(hipFree(buf));
    }
    return 0;
}
