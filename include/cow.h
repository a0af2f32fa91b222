/*
 * cow.h -- C ABI of the MI355X block-merged ray-march renderer
 * (City-on-Web, arXiv 2312.16457).
 *
 * What it computes.  A scene is partitioned on the ground plane into
 * axis-aligned unit blocks (Sec. 4.1, Eq. "blocks"); a sample point belongs
 * to the block whose half-open box [lo, hi) contains it.  Each (block, LOD)
 * holds a MERF-style baked representation (Sec. 3, Sec. 4.1 "Rendering
 * Stage"): a low-res 3D feature grid, three high-res feature planes (xy, xz,
 * yz) and an occupancy grid.  For every pixel ray the library
 *   1. composites the samples of each block front to back (Eqs. "alpha
 *      accumulation", "combined accumulation", "volume rendering inside
 *      blocks"), giving per-block (C_d^k, F^k, T^k);
 *   2. merges the blocks in depth order, A <- A + T * A^k, T <- T * T^k
 *      (Eq. "volume rendering across blocks"; Appendix A shows
 *      1 - alpha^k = prod_i (1 - alpha_i^k), so T^k is carried directly);
 *   3. shades once with the tiny deferred MLP, C = C_d + sigmoid(Phi(C_d, F, d))
 *      (Eq. "deferred"), with the unit world-space view direction d.
 *
 * Conventions.
 *   Texture layouts are channels-last with 8 channels (0: pre-activation
 *   density, exp; 1-3: diffuse, sigmoid; 4-7: specular features, sigmoid):
 *     grid  [R][R][R][8]  indexed [z][y][x][c]
 *     plane xy [Rp][Rp][8] indexed [y][x][c]; xz [z][x][c]; yz [z][y][c]
 *   Texels are cell-centred with clamp-to-edge; raw features are
 *   ((grid + xy) + xz) + yz.  uint8 texels decode to q * scale + offset per
 *   (texture, channel), texture 0 = grid, 1 = xy, 2 = xz, 3 = yz.
 *   Cameras use OpenCV axes; R is camera-to-world, row-major, with columns
 *   (right, down, forward).  Pixel (i, j) has direction
 *   normalize(R [(i + 1/2 - cx)/fx, (j + 1/2 - cy)/fy, 1]).
 *   MLP weights: float[499] = W1[16][10], b1[16], W2[16][16], b2[16],
 *   W3[3][16], b3[3] (row-major, out x in); input x = [C_d(3), F(4), d(3)],
 *   or with params->pe_freqs = 4 float[883] over x = [C_d(3), F(4), PE(d)(27)].
 *
 * Memory ownership.  Every device buffer is owned by the caller.  The library
 * keeps non-owning pointers to the textures passed to cow_load_blocks until
 * the next cow_load_blocks or cow_destroy; the caller keeps them alive and
 * may change their values (occupancy is not recomputed).  Workspaces are
 * caller-allocated device memory sized by cow_query_workspace.
 *
 * Streams and threads.  Device work is enqueued on the given HIP stream and
 * the call returns; outputs are valid after the stream synchronises.  A
 * context is used from one host thread at a time.
 *
 * Errors.  Every entry point returns a cow_status.  Arguments are validated
 * before anything is enqueued, so a failed call has no device side effects;
 * cow_last_error gives the reason.  No C++ exception crosses this boundary.
 */
#ifndef COW_H
#define COW_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define COW_API __attribute__((visibility("default")))

typedef enum cow_status {
    COW_OK = 0,
    COW_E_INVALID = 1,     /* bad argument (null pointer, size, range, NaN camera ...) */
    COW_E_NOT_LOADED = 2,  /* a (block, LOD) in a set is not loaded */
    COW_E_WORKSPACE = 3,   /* workspace smaller than cow_query_workspace asked for */
    COW_E_UNSUPPORTED = 4, /* e.g. backward through uint8 textures */
    COW_E_HIP = 5,         /* HIP runtime error; text in cow_last_error */
    COW_E_INTERNAL = 6
} cow_status;

enum { COW_U8 = 0, COW_F32 = 1 };

/* sampling modes */
enum {
    COW_MODE_CHORD = 0, /* n_steps midpoints over each block's ray chord (single-block scenes) */
    COW_MODE_GRID = 1   /* t_k = (k + 1/2) delta from the eye; max_steps steps from scene entry */
};

/* render flags */
enum {
    COW_F_NONE = 0,
    COW_F_GRAPH = 1,       /* replay a cached hipGraph of the launch sequence */
    COW_F_PERSISTENT = 2,  /* persistent workgroups pulling ray packets from a counter */
    COW_F_PER_BLOCK = 4,   /* baseline: one launch per view per block, blended in order */
    COW_F_SPARSE = 8,      /* read uint8 grids from the packed brick atlas (cow_pack_bricks) */
    COW_F_FLAT_OCC = 16    /* baseline: step through empty space one sample at a time instead of
                              jumping over empty cells of the occupancy pyramid (same results) */
};

typedef struct cow_ctx cow_ctx;

typedef struct cow_block_desc {
    int32_t block_id, lod;
    float aabb_min[3], aabb_max[3]; /* extent E_a = max - min on each axis: a whole power of two
                                       (1 to 64); unit cubes for plain blocks, 2^l x 2^l x 1 for a
                                       merged LOD-l asset */
    int32_t grid_res, plane_res, occ_res; /* texels (cells) per unit length, powers of two,
                                       occ_res divides both; a texture holds res * E_a texels
                                       along axis a: G_a = grid_res E_a, P_a = plane_res E_a */
    int32_t dtype;                  /* COW_U8 or COW_F32 */
    const void* grid;               /* device, [G_z][G_y][G_x][8] */
    const void* plane[3];           /* device, xy: [P_y][P_x][8], xz: [P_z][P_x][8], yz: [P_z][P_y][8] */
    float scale[4][8];              /* uint8 decode; ignored for COW_F32 */
    float offset[4][8];
    /* COW_BLOCK_CONTRACTED: a boundary block with an unbounded representation
     * (implementation details, the contraction equation, after MERF).  Its
     * textures and occupancy cover the contracted cube [-2, 2]^3 of the
     * box-normalised coordinate x = (p - centre) (2 / extent), mapped to the
     * block's texture space by q = (contract(x) + 2) (extent / 4): the box
     * fills the middle half of every axis, the rest of space the outer
     * shell.  Such a block must be one unit wide in x and y and span the full
     * height of the loaded scene (it owns the space beyond its outer faces,
     * see cow_render_params.ext_delta).  0 for a plain block. */
    int32_t flags;
} cow_block_desc;

enum { COW_BLOCK_CONTRACTED = 1 };

typedef struct cow_view {
    int32_t W, H;                   /* image size */
    int32_t crop_x0, crop_y0, crop_w, crop_h; /* rendered window */
    float eye[3];
    float R[9];
    float fx, fy, cx, cy;
} cow_view;

typedef struct cow_block_ref {
    int32_t block_id, lod;
} cow_block_ref;

typedef struct cow_block_set {
    const cow_block_ref* refs;      /* host array, any order */
    int32_t n;
} cow_block_set;

typedef struct cow_lod_policy {
    double thresholds[3];           /* LOD l where distance < thresholds[l]; beyond the last: dropped */
    int32_t n_thresholds;
    int32_t cull;                   /* nonzero: frustum culling */
    int32_t quadtree;               /* nonzero: LOD l entries are merged assets over 2^l x 2^l blocks
                                       (see cow_select_blocks) */
} cow_lod_policy;

typedef struct cow_render_params {
    int32_t mode;                   /* COW_MODE_CHORD or COW_MODE_GRID */
    int32_t n_steps;                /* chord mode */
    float delta;                    /* grid mode step length (world units) */
    int32_t max_steps;              /* grid mode cap, counted from scene entry */
    float t_min;                    /* early ray termination: a ray stops after the first evaluated
                                       sample at which its transmittance drops below t_min (0: off) */
    int32_t flags;                  /* COW_F_* */
    int64_t* counts;                /* device [P][2] (evaluated, marched) per pixel, or NULL */
    /* Opacity regulariser (Sec. 4.3, Eq. "opacity loss"): the entropy
     * -(a log a + (1 - a) log(1 - a)) of each block's opacity a = 1 - T^k,
     * with a clamped to [1e-6, 1 - 1e-6], summed over the blocks in which the
     * ray marches at least one sample (up to its early termination). */
    float* opacity;                 /* cow_render: device [P] per-ray entropy sum, or NULL */
    const float* opacity_weight;    /* cow_render_backward: device [P] dL/d(that sum), or NULL */
    /* Per-block deferred shading (Sec. 4.2, the across-block equation as
     * written): every block the ray marches at least one sample in is shaded
     * with its own MLP, C^k = C_d^k + sigmoid(Phi^k(C_d^k, F^k, d)), and
     * C = sum_k prod_{j<k} T^j C^k.  Device [loaded entries][499] in load
     * order, or NULL for one MLP after the merge.  When set, the mlp argument
     * of cow_render / cow_render_backward is unused (may be NULL) and aux
     * holds (C, 0, 0, 0, 0, T). */
    const float* block_mlp;
    float* grad_block_mlp;          /* cow_render_backward: device [entries][499], accumulated, or NULL */
    /* Positional encoding of the direction input of the deferred MLPs (Eq.
     * deferred: Phi(C_d, F, PE(d))): PE(d) = [d, sin(2^l d), cos(2^l d) for
     * l < pe_freqs], per component, so the MLP takes 10 + 6 pe_freqs inputs and
     * holds 499 + 96 pe_freqs weights (W1 [16][10 + 6 pe_freqs], then b1, W2,
     * b2, W3, b3 as above); every "499" of this header then reads 883.  0 (the
     * direction alone) or 4; 1-3 give COW_E_UNSUPPORTED, other values
     * COW_E_INVALID. */
    int32_t pe_freqs;
    /* Exterior of contracted boundary blocks (grid mode).  Outside the
     * footprint of the loaded scene (the union of the blocks' x-y extents) a
     * point belongs to the block column nearest in the max norm (Eq. "blocks"),
     * ties going to the one named by clamping the point's unit cell into the
     * footprint; when that block is contracted and in the view's set, the
     * ray samples it there.  Two segments per ray: from the camera to the
     * footprint's column, and from the column's exit on.  Steps start half of
     * ext_delta in and grow as ext_delta m^2, m = max(1, |x|_inf) of the
     * point's coordinate normalised to its owner cell, which keeps them about
     * uniform in contracted space; a point with m > 1 / ext_delta is beyond
     * the far limit (the segment after the column ends there); each segment
     * takes at most ext_max_steps steps.  Exterior samples composite in ray
     * order with the blocks (before them, then after them) and count in
     * counts like any sample.  ext_delta = 0 (or ext_max_steps = 0): no
     * exterior sampling.  A call whose sets hold a contracted block must use
     * grid mode, one MLP after the merge, no opacity output and no per-block
     * launches (else COW_E_UNSUPPORTED).  cow_render_backward takes
     * contracted blocks under the same rule and without the opacity term
     * (the exterior's samples, each with its own step, join the chain in ray
     * order and scatter into their owner's textures), COW_E_UNSUPPORTED
     * otherwise.  cow_sparsity reads a point in a contracted block's box
     * through the contraction; it samples no exterior. */
    float ext_delta;
    int32_t ext_max_steps;
    /* Per-block composites handed from the forward to the backward.  Device
     * [P][block_aux_n][8] float, 16-byte aligned, or NULL.  cow_render and
     * cow_render_noalloc write, for each pixel and the j-th block of its
     * view's set in the order the call composites the set, (A^k, T^k): the
     * block's own composite of (C_d, F) (Eq. "volume rendering inside
     * blocks") and its transmittance prod(1 - alpha_i), with T^k = -1 for a
     * block in which the ray marches no sample.  cow_render_backward, given
     * the buffer its forward wrote for the same views and sets, takes A^k and
     * T^k from it instead of marching each block a second time for them (the
     * per-block MLPs' adjoint, the opacity gradient); the gradients are the
     * same.  block_aux_n: slots per pixel, at least the largest set size of
     * the call's views (COW_E_INVALID otherwise).  COW_F32 blocks only, like
     * the backward (COW_E_UNSUPPORTED for a call over uint8 blocks). */
    float* block_aux;
    int32_t block_aux_n;
} cow_render_params;

/* Create a context bound to HIP device `device` (host state only). */
COW_API cow_status cow_create(cow_ctx** out, int device);
COW_API cow_status cow_destroy(cow_ctx* ctx);

/* Reason for the last failure on this context; valid until the next call. */
COW_API const char* cow_last_error(const cow_ctx* ctx);

/* Workspace sizes in bytes for loading `blocks` and for render / backward
 * calls of up to max_views views and max_pixels pixels in total.  The
 * backward size includes a pair-slot buffer for every float32 texture (64
 * bytes per texel): the adjoint adds the gradient of each pair of adjacent
 * texels into the slot of its first texel, one aligned 64-byte segment per
 * pair, and folds the slots into the caller's gradients at the end of the
 * call. */
COW_API cow_status cow_query_workspace(cow_ctx* ctx, const cow_block_desc* blocks, int n_blocks,
                               int max_views, int64_t max_pixels, size_t* load_bytes,
                               size_t* render_bytes, size_t* backward_bytes);

/* Register the blocks and build each one's occupancy grid (conservative
 * max-bound rule: a cell is occupied iff the sum over the four textures of
 * the largest density-channel texel in the cell's interpolation support
 * exceeds ln 0.01, Sec. 4.5 "Baking") into load_ws.  Replaces any previous
 * load.  Synchronises `stream` once (z_top of each block is read back). */
COW_API cow_status cow_load_blocks(cow_ctx* ctx, const cow_block_desc* blocks, int n, void* load_ws,
                           size_t load_bytes, hipStream_t stream);

/* Copy one loaded block's occupancy [Oz][Oy][Ox] (z, y, x; O per unit length
 * times the extent on each axis) to host memory. */
COW_API cow_status cow_get_occupancy(cow_ctx* ctx, int block_id, int lod, uint8_t* host_out, size_t n);

/* Multi-level occupancy (Sec. 3, the grids psi; Sec. 4.5 "Baking": the
 * binary grid downsampled by max-pooling), built by cow_load_blocks.  Level 0
 * is the grid of cow_get_occupancy; level l >= 1 holds L_a = max(O_a >> l, 1)
 * cells along axis a, [Lz][Ly][Lx], and its cell x is occupied (1) iff a base
 * cell i with i_a >> l == x_a on every axis is.  Levels run up to log2 of the
 * longest axis, where one cell remains.  Grid-mode marches jump over every
 * sample that lies in an empty cell of the coarsest empty level around it.
 * Copies level `level` to host memory (n >= its cell count); COW_E_INVALID
 * for a level outside that range. */
COW_API cow_status cow_get_occupancy_level(cow_ctx* ctx, int block_id, int lod, int level, uint8_t* host_out,
                                           size_t n);

/* Per-view selection (Appendix D, "Dynamic Loading", "Depth sorting"):
 * LOD by the distance from the eye to (centre_x, centre_y, z_top of the
 * finest level), frustum culling of [x0,x1]x[y0,y1]x[z_lo, z_top(LOD)],
 * front-to-back order by xy distance to the block centre (ties: lower id).
 * With policy->quadtree (merged LOD assets, Sec. 4.5 "Baking": an entry of
 * LOD l covers 2^l x 2^l blocks, aligned to its size): from the coarsest LOD
 * down, an entry of LOD l > 0 is drawn when every visible LOD l-1 entry
 * inside it is at distance >= thresholds[l-1] (vacuously when none is
 * visible), else its visible children are examined; the distance uses the
 * highest LOD-0 top inside the entry; thresholds[L] for the coarsest LOD L,
 * when given, drops far coarsest entries; order: coarsest entries by xy
 * distance, inside an entry its children by quadrant (the eye's, the two
 * beside it, the opposite; ties: lower id).  n_thresholds must be >= L.
 * Contracted boundary blocks (COW_BLOCK_CONTRACTED) also own the unbounded
 * space beyond their outer faces: z_top of such a block is its box top; a
 * block whose LOD-0 entry is contracted is never culled and, beyond the far
 * cut, takes LOD n_thresholds - 1 instead of being dropped; in quadtree mode
 * an entry whose footprint holds a contracted LOD-0 entry is never culled,
 * never dropped and never drawn merged (its children are examined).
 * All decisions in fp64.  Writes up to cap refs; *n_out = count. */
COW_API cow_status cow_select_blocks(cow_ctx* ctx, const cow_view* view, const cow_lod_policy* policy,
                             cow_block_ref* out, int cap, int* n_out);

/* Sparse grid (Sec. 4.5 "block-sparse format"): pack the uint8 grid of every
 * loaded uint8 block into bricks covering the interpolation support of its
 * occupied cells.  cow_query_bricks gives the size after cow_load_blocks.
 * Renders with COW_F_SPARSE then read the grid from the bricks (results are
 * bitwise identical to the dense grid). */
COW_API cow_status cow_query_bricks(cow_ctx* ctx, size_t* brick_bytes);
COW_API cow_status cow_pack_bricks(cow_ctx* ctx, void* brick_ws, size_t brick_bytes, hipStream_t stream);

/* Render n_views views: per pixel ray, the samples of each block composited
 * front to back (Sec. 3, Eqs. "alpha accumulation" and "combined
 * accumulation"; Appendix A, Eq. "volume rendering inside blocks"), the
 * blocks merged in depth order (Sec. 4.2, Eq. "volume rendering across
 * blocks", with T^k carried as prod(1 - alpha_i) by Appendix A) and the
 * result shaded by the deferred MLP (Sec. 3, Eq. "deferred").  Pixels are
 * the views' crops concatenated in view order, row-major within each crop (P
 * in total).  sets[v] lists the (block, LOD) entries view v renders; the
 * library orders them front to back by xy distance (Appendix D, "Depth
 * sorting").  mlp: device float[499].  Outputs (device): rgb [P][3], trans
 * [P], aux [P][8] = (C_d, F, T) or NULL (required before a backward). */
COW_API cow_status cow_render(cow_ctx* ctx, const cow_view* views, int n_views, const cow_block_set* sets,
                      const cow_render_params* params, const float* mlp, float* rgb, float* trans,
                      float* aux, void* ws, size_t ws_bytes, hipStream_t stream);

/* cow_render for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and results as cow_render, with no workspace argument.  The
 * per-call view and block-set tables and the persistent launch's counters
 * live in a fixed scratch array inside the library, one per GPU (about 128
 * KiB of device memory each, held until the process ends; its address is
 * taken when the first context is created on that GPU).  The call makes no
 * device or pinned-host allocation.  Limits: at most 256 views and 16384
 * set entries per call (COW_E_INVALID beyond), aux must be given (it is the
 * only per-pixel scratch cow_render would otherwise take from its
 * workspace; COW_E_INVALID if NULL), and COW_F_GRAPH is refused
 * (COW_E_UNSUPPORTED: instantiating a graph allocates).  Every call on one
 * GPU shares that GPU's scratch: calls on different streams of one GPU that
 * overlap in time race on it and must be ordered by the caller. */
COW_API cow_status cow_render_noalloc(cow_ctx* ctx, const cow_view* views, int n_views, const cow_block_set* sets,
                                      const cow_render_params* params, const float* mlp, float* rgb, float* trans,
                                      float* aux, hipStream_t stream);

/* Adjoint of cow_render for COW_F32 blocks: the gradients that training
 * through the block-merged render needs (Sec. 4.2, the block-based rendering
 * used in training for consistency between training and rendering), by the
 * chain rule through the deferred MLP, the merge across blocks and the
 * per-block composite, with each ray's samples recomputed.  grad_rgb [P][3] and grad_trans
 * [P] (nullable) are dL/d outputs, as is params->opacity_weight (nullable);
 * aux is the forward's aux.  Gradients are
 * ACCUMULATED into grad_grid[e] / grad_plane[3e + k] for loaded entry e (in
 * load order; NULL entries skipped) and into grad_mlp[499]; fp32 atomics, so
 * summation order varies run to run.  Per-ray samples are recomputed.
 * Gradient buffers and ws must be 16-byte aligned (COW_E_INVALID otherwise).
 * The atomics go to the pair-slot buffers in ws (see cow_query_workspace),
 * which are added into the gradients at the end of the call; with ws 64-byte
 * aligned every texel pair is one 64-byte atomic segment.
 * With params->block_mlp the weights' gradient goes to
 * params->grad_block_mlp instead (grad_mlp and mlp unused, may be NULL): each
 * lane re-composites a block, runs that block's MLP adjoint, and the wave's
 * sum of the 499 weight gradients is added once per block and wave.
 * Contracted boundary blocks: grid mode, one MLP after the merge, no
 * opacity_weight (COW_E_UNSUPPORTED otherwise); their exterior samples are
 * those of the forward with the same ext_delta and ext_max_steps. */
COW_API cow_status cow_render_backward(cow_ctx* ctx, const cow_view* views, int n_views,
                               const cow_block_set* sets, const cow_render_params* params,
                               const float* mlp, const float* aux, const float* grad_rgb,
                               const float* grad_trans, float* const* grad_grid,
                               float* const* grad_plane, float* grad_mlp, void* ws,
                               size_t ws_bytes, hipStream_t stream);

/* Sparsity regulariser (Sec. 4.3, Eq. "sparse loss"): the mean opacity
 * alpha_i = 1 - exp(-sigma(p_i) delta) at n points, times weight.  sigma is
 * the render's density: the point takes the first entry of `set` whose
 * half-open box holds it (read through the contraction in a contracted
 * boundary block), and is zero in an unoccupied cell or outside every
 * entry.  pts: device float [n][3] (world).  alpha: device float [n] or NULL.
 * loss: device float [1]; weight / n * sum alpha_i is ADDED to it (fp32
 * atomics, order unspecified).  grad_grid / grad_plane: host tables of device
 * pointers per loaded entry as in cow_render_backward, or NULL for no
 * gradient; only the density channel (0) receives gradient, accumulated;
 * gradients need COW_F32 entries.  ws: device workspace of at least
 * 256 + 4 * set->n + 32 * (loaded entries) bytes (the backward workspace of
 * cow_query_workspace always suffices). */
COW_API cow_status cow_sparsity(cow_ctx* ctx, const cow_block_set* set, const float* pts, int64_t n, float delta,
                                float weight, float* alpha, float* loss, float* const* grad_grid,
                                float* const* grad_plane, void* ws, size_t ws_bytes, hipStream_t stream);

/* Time the launch configurations (ray-packet shape, waves per workgroup,
 * persistent or not) on this workload and keep the fastest for later
 * renders; the fastest of the short trials replaces the configuration in
 * force only if longer interleaved runs of both show it at least 1% faster.
 * Reads/writes a JSON cache at cache_path (nullable).  The choice never
 * changes results. */
COW_API cow_status cow_autotune(cow_ctx* ctx, const cow_view* views, int n_views, const cow_block_set* sets,
                        const cow_render_params* params, const float* mlp, void* ws,
                        size_t ws_bytes, const char* cache_path, hipStream_t stream);

/* Current launch configuration (packet width in pixels, waves per
 * workgroup, persistent flag) and an explicit override.  persistent: 1 =
 * waves take packets from per-XCD work counters until they run out, 0 = one
 * wave per packet, -1 (the default) = by texture type: 1 for COW_F32 launches
 * (forward and adjoint), 0 for COW_U8.  The configuration never changes
 * results. */
COW_API cow_status cow_get_config(cow_ctx* ctx, int* tile_w, int* waves, int* persistent);
COW_API cow_status cow_set_config(cow_ctx* ctx, int tile_w, int waves, int persistent);

/* Instrumentation: when enabled, HIP events bracket the march kernel of
 * each cow_render / cow_render_backward on the call's stream; the last
 * call's forward and backward march durations in milliseconds. */
COW_API cow_status cow_set_timing(cow_ctx* ctx, int enable);
COW_API cow_status cow_last_timing(cow_ctx* ctx, float* fwd_march_ms, float* bwd_march_ms);

/* Texel-gather microbenchmark (a measurement aid, not a step of the render):
 * the forward march's memory accesses without its arithmetic.  Each 8x8 tile
 * of view's crop is one wave; a lane marches `steps` camera-anchored samples
 * t_k = (k + 1/2) delta along its pixel ray through a field of
 * blocks_x x blocks_y unit blocks that repeats in x, y and z, and per sample
 * loads the ten texel pairs the march loads (four grid rows, two rows per
 * plane; cell-centred, clamp-to-edge).  tex: device, blocks_x * blocks_y
 * blocks of (grid_res^3 + 3 plane_res^2) texels of 8 bytes (COW_U8) or 32
 * bytes (COW_F32) each, block (x, y) at index y * blocks_x + x, each laid
 * out grid then the xy, xz, yz planes ([z][y][x] and [v][u], channels last).
 * sink: device uint32 [tiles][64], one XOR of the loaded words per lane.
 * ms_out (host): kernel time from HIP events; the call synchronises the
 * stream.  Gathered bytes = tiles * 64 * steps * (160 or 640).
 * COW_E_INVALID for a crop that is not a multiple of 8, non-power-of-two
 * resolutions, or tex_bytes too small. */
COW_API cow_status cow_gather_probe(const cow_view* view, const void* tex, size_t tex_bytes, int blocks_x,
                                    int blocks_y, int grid_res, int plane_res, int dtype, int steps, float delta,
                                    uint32_t* sink, float* ms_out, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif
