// Device-side tables shared by the host library (cow_host.cpp) and the
// kernels (the .hip sources).  Plain structs, copied to device memory once per
// cow_load_blocks (DevBlock) or per cow_render call (DevView, refs).
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace cow {

constexpr int kNch = 8;
constexpr int kMlpParams = 499;  // deferred MLP over 10 inputs
// Deferred MLP over [C_d, F, PE(d)] with L frequencies of positional encoding
// (L = 0: the direction alone): 10 + 6L inputs, weights W1 [16][NI], b1 [16],
// W2 [16][16], b2 [16], W3 [3][16], b3 [3].
template <int L>
struct MlpShape {
    static constexpr int NI = 10 + 6 * L, W1 = 0, B1 = 16 * NI, W2 = B1 + 16, B2 = W2 + 256, W3 = B2 + 16,
                         B3 = W3 + 48, N = B3 + 3;
};
constexpr int kMlpParamsMax = MlpShape<4>::N;  // 883
inline constexpr int mlp_params(int L) { return 499 + 96 * L; }
// largest camera-anchored step index; t_k = (k + 1/2) delta is exact in fp32
// below 2^23
constexpr int32_t kMaxStep = (1 << 23) - 2;

struct DevBlock {
    float lo[3], hi[3];
    int32_t R, Rp, O, dtype;   // grid, plane, occupancy texels (cells) per unit length
    int32_t gd[3], pd[3], od[3];  // texels (cells) along x, y, z: resolution x extent
    const void* grid;
    const void* plane[3];
    const uint8_t* occ;        // [Oz][Oy][Ox] binary occupancy
    // multi-level occupancy: levels 1..n_levels of the max-pooled pyramid,
    // consecutive, level l [Lz][Ly][Lx] with L_a = max(od_a >> l, 1)
    const uint8_t* occ_pyr;
    // [Oz][Oy][Ox]: 0 for an occupied cell, else 1 + the coarsest level whose
    // cell holding it is empty (the level the march may skip at)
    const uint8_t* skip;
    int32_t n_levels;
    const int32_t* brick_slot; // [O][O][O] -> brick index or -1 (sparse grids)
    const uint8_t* bricks;     // [n][(s+2)^3][8] uint8
    uint32_t brick_bytes;      // size of this block's part of the brick atlas
    float scale[4][kNch];
    float offset[4][kNch];
    // uint8 decode in the exp2 domain of the activations, formed at load:
    // dsc[t][c] = scale[t][c] 2^24 (+log2 e for c = 0, -log2 e otherwise),
    // dosum[c] = (((offset[0][c] + offset[1][c]) + offset[2][c]) + offset[3][c]) (+-log2 e)
    float dsc[4][kNch];
    float dosum[kNch];
    int32_t contracted;        // texture space is the contracted cube (boundary block)
};

struct DevView {
    float eye[3];
    float R[9];
    float fx, fy, cx, cy;
    int32_t x0, y0, w, h;
    int32_t tiles_x, tile_begin, n_tiles;
    int32_t set_begin, set_n;
    int64_t pix_begin;
};

struct MarchArgs {
    const DevBlock* blocks;
    const DevView* views;
    int32_t n_views;
    const int32_t* refs;       // per view, ordered entry indices
    int32_t total_tiles;
    int32_t tile_w, tile_h;    // tile_w * tile_h == 64
    int32_t mode, n_steps, max_steps;
    float delta;
    float t_min;               // early ray termination threshold (0: off)
    float scene_lo[3], scene_hi[3];
    int32_t use_sparse;
    int32_t flat_occ;          // 1: step through empty cells one sample at a time (no pyramid skips)
    int32_t blocks_dtype;      // COW_U8 / COW_F32, the same for every block of the launch
    float* aux;                // [P][8] (C_d, F, T)
    float* trans;              // [P]
    int64_t* counts;           // [P][2] or null
    float* opacity;            // [P] per-ray block-opacity entropy, or null
    const float* block_mlp;    // [entries][mlp_params(pe)] per-block deferred MLPs, or null (one MLP after the merge)
    int32_t pe;                // positional-encoding frequencies of the deferred MLPs' direction input (0 or 4)
    float* rgb;                // [P][3], written by the march when block_mlp is set
    int32_t* work_counter;     // persistent mode: one counter per XCD (8 ints)
    int32_t persistent;
    // per-block baseline: only this view and this one set position
    int32_t only_view, only_set_pos;
    // exterior of contracted boundary blocks: step scale (0: none), steps per segment
    float ext_delta;
    int32_t ext_max_steps;
    int32_t contract;          // some block of the call is contracted: the contraction kernel
    // per-block composites (A^k, T^k) per pixel and set position, [P][block_aux_n][8], or null
    float* block_aux;
    int32_t block_aux_n;
};

struct MlpArgs {
    const DevView* views;
    int32_t n_views;
    int64_t n_pix;
    const float* mlp;          // [mlp_params(pe)]
    const float* aux;
    float* rgb;
    float* trans;
    int32_t pe;                // positional-encoding frequencies (0 or 4)
};

struct MlpBwdArgs {
    const DevView* views;
    int32_t n_views;
    int64_t n_pix;
    const float* mlp;
    const float* aux;
    const float* grad_rgb;
    float* u;                  // [P][8]: dL/d(C_d, F) in 0..6
    float* grad_mlp;           // [mlp_params(pe)], accumulated
    int32_t pe;                // positional-encoding frequencies (0 or 4)
};

struct BwdArgs {
    MarchArgs m;
    const float* u;            // [P][8]
    const float* grad_trans;   // [P] or null
    const float* w_opacity;    // [P] dL/d(per-ray opacity entropy), or null
    const float* grad_rgb;     // [P][3], read directly with per-block MLPs (m.block_mlp)
    float* grad_block_mlp;     // [entries][mlp_params(pe)], accumulated, or null
    float* const* grad_grid;   // device array of per-entry pointers
    float* const* grad_plane;  // device array, 3 per entry
    // Pair-slot buffers: the march adds the gradient of texel pair (p, p + 1)
    // into slot p of its texture's buffer (16 floats, at byte 64 p), one
    // aligned 64-byte segment per pair whatever the parity of p (in the
    // gradient itself an odd pair would straddle two); the slots are folded
    // into the gradient after the march.  Device array, 4 per entry (grid,
    // xy, xz, yz; null: none).
    float* const* slots;
};

// zero the pair slots, then (after the march) add slot x's first texel and
// slot x - 1's second texel into gradient texel x
struct FoldJob {
    float* grad;      // [n_texels][8]
    float* slots;     // [n_texels][2][8]
    int64_t n_texels;
};

// sparsity regulariser at given points
struct SparsityArgs {
    const DevBlock* blocks;
    const int32_t* set;        // entry indices, first match wins
    int32_t n_set;
    int32_t dtype;             // COW_U8 / COW_F32, the same for every entry of the set
    const float* pts;          // [n][3]
    int64_t n;
    float delta;
    float scale;               // weight / n
    float* alpha;              // [n] or null
    float* loss;               // [1], accumulated
    float* const* grad_grid;   // device array of per-entry pointers, or null
    float* const* grad_plane;  // device array, 3 per entry, or null
};

// launchers
hipError_t launch_occupancy(const DevBlock* blocks, int entry, int n_cells, hipStream_t s);
hipError_t launch_occupancy_pyramid(const DevBlock* blocks, int entry, int n_levels, const int od[3], hipStream_t s);
hipError_t launch_march(const MarchArgs& a, int waves_per_group, hipStream_t s);
hipError_t launch_reset_counter(int32_t* counter, hipStream_t s);
hipError_t launch_clear_aux(float* aux, int64_t n_pix, hipStream_t s);
hipError_t launch_mlp(const MlpArgs& a, hipStream_t s);
hipError_t launch_mlp_bwd(const MlpBwdArgs& a, hipStream_t s);
hipError_t launch_march_bwd(const BwdArgs& a, int waves_per_group, hipStream_t s);
hipError_t launch_slots_zero(const FoldJob* jobs, int n_jobs, int64_t max_texels, hipStream_t s);
hipError_t launch_slots_fold(const FoldJob* jobs, int n_jobs, int64_t max_texels, hipStream_t s);
hipError_t launch_sparsity(const SparsityArgs& a, hipStream_t s);
hipError_t launch_pack_bricks(const DevBlock* blocks, int entry, int n_cells, int s_cells,
                              const int32_t* slot_host_unused, hipStream_t st);

}  // namespace cow
