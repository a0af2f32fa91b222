// Texel-gather microbenchmark: the memory side of the forward march with its
// arithmetic taken away, to measure how fast the texture path can deliver
// the march's access pattern.  Rays of a pinhole view step through a tiled
// field of blocks (x, y and z wrap around, so every lane takes the same number
// of samples); each sample issues the ten texel-pair loads of the march
// (four grid rows, two rows of each plane) at the same cell-centred,
// clamp-to-edge indices, and folds the loaded words into one XOR per lane.
// The result is the achievable gather rate for that pattern at the given
// texture footprint; the march's own gather rate is quoted against it.
#include <hip/hip_runtime.h>


#include "cow.h"
#include "cow_device.h"

namespace cow {

struct GatherArgs {
    DevView v;                // camera and crop (tiles_x set)
    const unsigned char* tex; // n_blocks consecutive blocks
    int64_t block_bytes;      // (R^3 + 3 Rp^2) * texel bytes
    int32_t nbx, nby;         // block field, x fastest
    int32_t R, Rp, lR, lRp;
    int32_t f32;              // texel = 8 uint8 (16-byte pair) or 8 fp32 (64-byte pair)
    int32_t steps, n_tiles;
    float delta;
    uint32_t* sink;           // [n_tiles][64]
};

__device__ inline uint32_t xor4(uint4 a) { return (a.x ^ a.y) ^ (a.z ^ a.w); }

__device__ inline int wrap(int i, int n) {
    const int m = i % n;
    return m < 0 ? m + n : m;
}

__device__ inline uint32_t gather_pair(const unsigned char* base, int64_t texel_off, bool f32) {
    if (!f32) return xor4(*reinterpret_cast<const uint4*>(base + 8 * texel_off));
    const uint4* p = reinterpret_cast<const uint4*>(base + 32 * texel_off);
    return (xor4(p[0]) ^ xor4(p[1])) ^ (xor4(p[2]) ^ xor4(p[3]));
}

__global__ __launch_bounds__(256) void gather_kernel(GatherArgs a) {
    const int lane = threadIdx.x & 63;
    const int tile = xcd_packet(blockDim.x >> 6, threadIdx.x >> 6);
    if (tile >= a.n_tiles) return;
    const int tx = tile % a.v.tiles_x, ty = tile / a.v.tiles_x;
    const int px = a.v.x0 + tx * 8 + (lane & 7), py = a.v.y0 + ty * 8 + (lane >> 3);
    float d[3];
    ray_direction(a.v, px, py, d);
    const bool f32 = a.f32 != 0;
    const int64_t plane_off = (int64_t)a.R * a.R * a.R;
    const int64_t plane_sz = (int64_t)a.Rp * a.Rp;
    uint32_t acc = 0;
    for (int k = 0; k < a.steps; ++k) {
        const float t = ((float)k + 0.5f) * a.delta;
        float q[3];
        int cell[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float p = fmaf(t, d[c], a.v.eye[c]);
            const float fl = floorf(p);
            cell[c] = (int)fl;
            q[c] = p - fl;
        }
        const int blk = wrap(cell[1], a.nby) * a.nbx + wrap(cell[0], a.nbx);
        const unsigned char* base = a.tex + (int64_t)blk * a.block_bytes;
        const Lin gx = lin_pair(q[0], a.R, a.R), gy = lin_pair(q[1], a.R, a.R), gz = lin_pair(q[2], a.R, a.R);
        const Lin ux = lin_pair(q[0], a.Rp, a.Rp), uy = lin_pair(q[1], a.Rp, a.Rp), uz = lin_pair(q[2], a.Rp, a.Rp);
        uint32_t x = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t pidx = ((((int64_t)(gz.p + (j >> 1)) << a.lR) + gy.p + (j & 1)) << a.lR) + gx.p;
            x ^= gather_pair(base, pidx, f32);
        }
        const Lin U[3] = {ux, ux, uy}, V[3] = {uy, uz, uz};
#pragma unroll
        for (int pl = 0; pl < 3; ++pl)
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int64_t pidx = plane_off + pl * plane_sz + ((int64_t)(V[pl].p + j) << a.lRp) + U[pl].p;
                x ^= gather_pair(base, pidx, f32);
            }
        acc ^= x;
    }
    a.sink[(int64_t)tile * 64 + lane] = acc;
}

}  // namespace cow

namespace {
int log2i(int x) {
    int l = 0;
    while ((1 << l) < x) ++l;
    return l;
}
bool pow2(int x) { return x >= 2 && (x & (x - 1)) == 0; }
}  // namespace

extern "C" COW_API cow_status cow_gather_probe(const cow_view* view, const void* tex, size_t tex_bytes,
                                               int blocks_x, int blocks_y, int grid_res, int plane_res,
                                               int dtype, int steps, float delta, uint32_t* sink,
                                               float* ms_out, hipStream_t stream) {
    if (!view || !tex || !sink || !ms_out) return COW_E_INVALID;
    if (blocks_x < 1 || blocks_y < 1 || steps < 1 || !(delta > 0.0f)) return COW_E_INVALID;
    if (!pow2(grid_res) || !pow2(plane_res) || grid_res > 1024 || plane_res > 8192) return COW_E_INVALID;
    if (dtype != COW_U8 && dtype != COW_F32) return COW_E_INVALID;
    if (view->crop_w < 1 || view->crop_h < 1 || view->crop_w % 8 || view->crop_h % 8) return COW_E_INVALID;
    const int64_t texel = dtype == COW_U8 ? 8 : 32;
    const int64_t block_bytes =
        ((int64_t)grid_res * grid_res * grid_res + 3 * (int64_t)plane_res * plane_res) * texel;
    if ((int64_t)blocks_x * blocks_y * block_bytes > (int64_t)tex_bytes) return COW_E_INVALID;
    cow::GatherArgs a{};
    for (int c = 0; c < 3; ++c) a.v.eye[c] = view->eye[c];
    for (int c = 0; c < 9; ++c) a.v.R[c] = view->R[c];
    a.v.fx = view->fx, a.v.fy = view->fy, a.v.cx = view->cx, a.v.cy = view->cy;
    a.v.x0 = view->crop_x0, a.v.y0 = view->crop_y0, a.v.w = view->crop_w, a.v.h = view->crop_h;
    a.v.tiles_x = view->crop_w / 8;
    a.n_tiles = a.v.tiles_x * (view->crop_h / 8);
    a.tex = static_cast<const unsigned char*>(tex);
    a.block_bytes = block_bytes;
    a.nbx = blocks_x, a.nby = blocks_y;
    a.R = grid_res, a.Rp = plane_res, a.lR = log2i(grid_res), a.lRp = log2i(plane_res);
    a.f32 = dtype == COW_F32;
    a.steps = steps, a.delta = delta;
    a.sink = sink;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return COW_E_HIP;
    const dim3 block(256), grid((a.n_tiles + 3) / 4);
    cow_status st = COW_OK;
    if (hipEventRecord(e0, stream) != hipSuccess) st = COW_E_HIP;
    if (st == COW_OK) {
        hipLaunchKernelGGL(cow::gather_kernel, grid, block, 0, stream, a);
        if (hipGetLastError() != hipSuccess || hipEventRecord(e1, stream) != hipSuccess ||
            hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(ms_out, e0, e1) != hipSuccess)
            st = COW_E_HIP;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}
