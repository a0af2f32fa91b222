/*
 * CPU oracle for block-merged ray marching (City-on-Web, arXiv 2312.16457).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the slow, plainly written definition the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load it; the renderer itself never does.
 * It shares no code, header or constant table with the HIP library.
 *
 * Discrete decisions (ray direction, sample positions, sample -> block,
 * occupancy cell, occupancy bit) are taken in IEEE fp32 exactly as specified
 * below; all continuous arithmetic (interpolation, activations, compositing,
 * MLP, adjoint) is fp64.
 */
#ifndef CITYWEB_ORACLE_H
#define CITYWEB_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_U8 = 0, ORC_F64 = 1 };

typedef struct orc_block {
    int block_id, lod;
    float lo[3], hi[3];      /* AABB; samples belong to [lo, hi) (half-open) */
    int R, Rp, O;            /* grid, plane and occupancy texels (cells) per unit length; a
                                block spans hi - lo (whole powers of two per axis), so its
                                grid holds R*(hi-lo) texels along each axis */
    int dtype;               /* ORC_U8 or ORC_F64 */
    const unsigned char* g8; /* [R][R][R][8]  z,y,x,ch */
    const unsigned char* p8[3];
    const double* gf;        /* same layouts, fp64 values */
    const double* pf[3];
    float scale[4][8];       /* uint8 decode q*scale+offset (tex 0 grid, 1 xy, 2 xz, 3 yz) */
    float offset[4][8];
    int contracted;          /* boundary block whose representation covers the contracted cube
                                [-2,2]^3 of its box-normalised coordinate (MERF contraction) */
} orc_block;

typedef struct orc_view {
    int W, H, x0, y0, w, h;  /* image size and crop window */
    float eye[3];
    float R[9];              /* camera-to-world, row-major; columns right, down, forward */
    float fx, fy, cx, cy;
} orc_view;

typedef struct orc_params {
    int mode;                /* 0: n_steps midpoints over each block chord; 1: global grid */
    int n_steps;
    float delta;             /* mode 1 step length */
    int max_steps;           /* mode 1 cap counted from scene entry */
    float t_min;             /* stop a ray after the first evaluated sample with T < t_min (0: off) */
    int pe;                  /* deferred MLP input: [C_d, F, PE(d)] with L = pe frequencies (0-4) */
    float ext_delta;         /* mode 1, contracted blocks: exterior step scale (0: no exterior) */
    int ext_max_steps;       /* exterior steps per ray segment outside the footprint */
} orc_params;

enum {
    ORC_MERGED = 0,          /* per-block composite, merged in per-ray entry order */
    ORC_MONOLITHIC = 1,      /* one composite over the whole sample sequence */
    ORC_REVERSED = 2,        /* negative control: merge in reverse entry order */
    ORC_BY_ID = 3,           /* negative control: merge in block-id order */
    ORC_ALPHA_NORM = 4,      /* negative control: blend blocks with alpha^k / sum alpha^j */
    ORC_BLOCK_MLP = 5        /* per-block deferred shading before the merge (Eq. across as
                                written): mlp holds one 499-weight MLP per entry of `blocks`;
                                C = sum_k prod_{j<k} T^j (C_d^k + sigmoid(Phi^k(C_d^k, F^k, d)))
                                over the blocks the ray marches at least one sample in;
                                aux = (C, 0, 0, 0, 0, T) */
};

/* positional encoding of a direction (Eq. deferred): [d, sin(2^l d), cos(2^l d) for
 * l < L], per component; writes and returns 3 + 6L values (-1 for L outside 0-4) */
int orc_posenc(const double* d, int L, double* out);

/* parameter count of the deferred MLP over 10 + 6L inputs: W1 [16][10+6L], b1 [16],
 * W2 [16][16], b2 [16], W3 [3][16], b3 [3] (499 for L = 0) */
long orc_mlp_params(int L);
/* contraction of the implementation details (MERF): x -> contract(x), fp64 */
void orc_contract(const double* x, double* y);
/* fp32 texture-space coordinate of world point p in block b (decision
 * sequence; contracted blocks map through the contraction); returns the max
 * norm of the box-normalised coordinate (0 for plain blocks) */
float orc_local_q(const orc_block* b, const float* p, float* q);
/* the samples of one exterior segment [t_start, t_end) of the ray (o, d):
 * texture-space coordinates and step lengths; returns their number (<= cap) */
long orc_ext_samples(const orc_block* blocks, int nblocks, const unsigned char* const* occ, const int* set,
                     int nset, const orc_params* p, const float* o, const float* d, float t_start, float t_end,
                     int post, float* q_out, double* delta_out, long cap);

/* occupancy bits [O][O][O] (z,y,x) of one block by the conservative max-bound rule */
int orc_occupancy(const orc_block* b, unsigned char* out);

/* level `level` >= 0 of the max-pooled occupancy pyramid: [Lz][Ly][Lx] with
 * L_a = max(C_a >> level, 1), C_a the base cell count along axis a */
int orc_occupancy_level(const orc_block* b, const unsigned char* occ, int level, unsigned char* out);

/* top of the highest occupied cell (world z) */
double orc_ztop(const orc_block* b, const unsigned char* occ);

/* Render pixels (absolute image coordinates pix[2n], pix[2n+1]) of one view.
 * blocks: every registered block (defines the scene box); occ[b]: its fixed
 * occupancy; set: indices into blocks of the (block, LOD) entries that the
 * view renders.  Any output pointer may be NULL. */
int orc_render(const orc_block* blocks, int nblocks, const unsigned char* const* occ,
               const orc_view* v, const int* set, int nset, const orc_params* p,
               const double* mlp, const int* pix, int npix, int composite,
               double* rgb, double* trans, double* aux, long long* n_eval,
               long long* n_march, int* order_ok, int nthreads);

/* Entry order of blocks along one ray (block indices into `blocks`); returns count */
int orc_ray_blocks(const orc_block* blocks, int nblocks, const orc_view* v, const int* set,
                   int nset, const orc_params* p, int i, int j, int* out, int cap);

/* fp64 adjoint.  grad_rgb[npix*3], grad_trans[npix] and w_opacity[npix] (the
 * weight of each ray's block-opacity entropy, see orc_opacity) are nullable.
 * Gradients are ACCUMULATED into grad_grid[b] / grad_plane[3b+k] (NULL
 * entries skipped) for every b in the set and into grad_mlp[499] (nullable).
 * fp64 blocks only. */
int orc_adjoint(const orc_block* blocks, int nblocks, const unsigned char* const* occ,
                const orc_view* v, const int* set, int nset, const orc_params* p,
                const double* mlp, const int* pix, int npix, const double* grad_rgb,
                const double* grad_trans, const double* w_opacity, double* const* grad_grid,
                double* const* grad_plane, double* grad_mlp);

/* fp64 adjoint of the ORC_BLOCK_MLP composite: mlp[nblocks*499] per entry;
 * gradients ACCUMULATED into grad_grid / grad_plane as in orc_adjoint and
 * into grad_mlp[nblocks*499] (nullable).  grad_trans, w_opacity nullable. */
int orc_adjoint_block_mlp(const orc_block* blocks, int nblocks, const unsigned char* const* occ,
                          const orc_view* v, const int* set, int nset, const orc_params* p,
                          const double* mlp, const int* pix, int npix, const double* grad_rgb,
                          const double* grad_trans, const double* w_opacity, double* const* grad_grid,
                          double* const* grad_plane, double* grad_mlp);

/* Block-opacity entropy of each ray (Eq. "opacity loss"):
 * -sum_k (a log a + (1 - a) log(1 - a)), a = clamp(1 - T^k, 1e-6, 1 - 1e-6),
 * over the blocks in which the ray marches at least one sample. */
int orc_opacity(const orc_block* blocks, int nblocks, const unsigned char* const* occ,
                const orc_view* v, const int* set, int nset, const orc_params* p,
                const int* pix, int npix, double* loss);

/* L1 sparsity of opacity at given points (Eq. "sparse loss"):
 * loss = weight / n * sum_i alpha(p_i), alpha = 1 - exp(-sigma(p_i) delta),
 * sigma the render's density (zero in unoccupied cells, zero outside the
 * set's blocks; a point takes the first entry of the set whose half-open
 * box holds it).  Returns the loss; writes alpha[n] (nullable); accumulates
 * its gradient into the density channel of grad_grid / grad_plane (fp64
 * blocks, NULL skipped). */
double orc_sparsity(const orc_block* blocks, int nblocks, const unsigned char* const* occ,
                    const int* set, int nset, const float* pts, int n, double delta, double weight,
                    double* alpha, double* const* grad_grid, double* const* grad_plane);

/* Per-view block selection: LOD by eye-to-centre distance, frustum culling,
 * front-to-back order by xy distance.  Inputs per distinct block entry k:
 * ids[k], lods[k], lo/hi[3k..], ztop[k], contracted[k].  A block whose finest
 * entry is contracted (it owns the unbounded space beyond its outer faces) is
 * never culled, and beyond the far cut takes LOD n_thr - 1 instead of being
 * dropped.  Writes chosen entry indices in order.
 * Returns the count, or -2 if a chosen (block, LOD) is not among the entries. */
int orc_select(const orc_view* v, int nent, const int* ids, const int* lods, const float* lo,
               const float* hi, const double* ztop, const int* contracted, const double* thresholds,
               int n_thr, int cull, int* out, int cap);

/* Quadtree selection over merged LOD entries (an entry of LOD l covers
 * 2^l x 2^l blocks): coarse to fine, an entry of LOD l > 0 is drawn when
 * every visible LOD l-1 entry inside it is at distance >= thresholds[l-1];
 * front-to-back order by recursive quadrants.  n_thr >= the coarsest LOD
 * (-3 otherwise); thresholds[L], when given, drops far coarsest entries.  An
 * entry whose footprint holds a contracted finest-level entry is never
 * culled, never dropped and never drawn merged (its children are examined).
 * Returns the count of chosen entry indices written to out. */
int orc_select_quadtree(const orc_view* v, int nent, const int* ids, const int* lods, const float* lo,
                        const float* hi, const double* ztop, const int* contracted, const double* thresholds,
                        int n_thr, int cull, int* out, int cap);

/* Texels read by the evaluated samples of pixels pix[npix][2] (the compulsory
 * texture bytes of a frame): marks[4 e + t] (t = 0 grid, 1-3 the xy, xz, yz
 * planes; NULL to skip) receive 1 at every texel index the interpolation of
 * an occupied sample of entry e taps (clamped, as the render's field).
 * t_min = 0 and plain blocks only (-1 otherwise); 0 on success. */
int orc_touched_texels(const orc_block* blocks, int nblocks, const unsigned char* const* occ, const orc_view* v,
                       const int* set, int nset, const orc_params* p, const int* pix, long npix,
                       unsigned char* const* marks, int nthreads);

/* pre-activation features at n world points of block b (points outside the
 * block are evaluated by the same clamped rule): raw[8n] */
void orc_field(const orc_block* b, int n, const float* pts, double* raw);

/* the MLP alone: x[10] -> out[3] = sigmoid(z) (before adding C_d) */
void orc_mlp(const double* mlp, const double* x, double* out);
/* the same with 10 + 6L inputs x = [C_d, F, PE(d)]; -1 for L outside 0-4 */
int orc_mlp_pe(const double* mlp, int L, const double* x, double* out);

#ifdef __cplusplus
}
#endif
#endif
