// Host side of the C ABI (include/cow.h): validation, block registry,
// per-view selection and ordering, workspace layout, launch sequencing,
// hipGraph replay, autotuning and timing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "cow.h"
#include "cow_internal.h"

// digest of the library's sources, set by the build (tune-cache key)
#ifndef COW_SOURCE_DIGEST
#define COW_SOURCE_DIGEST "unversioned"
#endif

using cow::DevBlock;
using cow::DevView;

namespace {

// Scratch of cow_render_noalloc: the per-call view and block-set tables and
// the persistent launch's counters, for callers that cannot allocate device
// memory.  One copy per GPU, held until the process ends; its device address
// is looked up once per device (hipGetSymbolAddress) when a context is
// created there.  In host code the name is only a stand-in, never an address.
constexpr size_t kScratchBytes = 128 * 1024;
constexpr int kNoAllocMaxViews = 256;
constexpr int kNoAllocMaxRefs = 16384;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// the device address of `scratch` on `device`, which must be current
hipError_t scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch[device] = ptr;
    }
    *out = g_scratch[device];
    return hipSuccess;
}

constexpr size_t kAlign = 256;
constexpr int kMaxViews = 1 << 16;
constexpr int kMaxBlocks = 1 << 16;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Entry {
    cow_block_desc desc;
    size_t occ_off = 0, slot_off = 0;
    int n_bricks = 0;
    double ztop = 0.0;
};

struct GraphEntry {
    std::vector<unsigned char> key;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

// one pinned host buffer for table uploads and the event that marks the end
// of the copy that last read it
struct Staging {
    unsigned char* buf = nullptr;
    size_t bytes = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
};
constexpr int kStagingSlots = 4;
constexpr size_t kStagingInitial = 1 << 18;  // per slot, allocated by cow_create

// default launch: 8x8 ray packets, four waves per workgroup, XCD-chunked
// packet order; persistent -1 picks by texture type: fp32 launches (forward
// and adjoint) take packets from the per-XCD work counters, uint8 launches
// are one wave per packet (each measured fastest on its 4x4-block workload;
// the autotuner may change any of it)
struct TuneCfg {
    int tile_w = 8, waves = 4, persistent = -1;
};

int persistent_for(const TuneCfg& t, int dtype) { return t.persistent < 0 ? (dtype == COW_F32 ? 1 : 0) : t.persistent; }

}  // namespace

struct cow_ctx {
    int device = 0;
    int n_cus = 256;
    std::string arch;
    std::vector<Entry> entries;
    unsigned char* load_ws = nullptr;
    size_t load_bytes = 0;
    DevBlock* d_blocks = nullptr;
    std::vector<DevBlock> h_blocks;
    float scene_lo[3] = {0, 0, 0}, scene_hi[3] = {0, 0, 0};
    bool loaded = false;
    int dtype = COW_U8;
    bool mixed_dtype = false;
    // sparse bricks
    bool bricks_packed = false;
    size_t brick_bytes = 0;
    // pinned staging for table uploads: a ring of slots, each reused only
    // once the copy that last read it has finished, so the host can run
    // several calls ahead of the device
    Staging staging[kStagingSlots];
    int staging_next = 0;
    // graphs are captured on this stream (the caller's may be the null
    // stream, which cannot capture) and launched on the caller's
    hipStream_t capture_stream = nullptr;
    // launch configuration
    TuneCfg cfg;
    // instrumentation
    bool timing = false;
    hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
    bool have_fwd = false, have_bwd = false;
    std::vector<GraphEntry> graphs;
    // this device's copy of the cow_render_noalloc scratch
    unsigned char* scratch = nullptr;
    std::string err;
};

namespace {

cow_status fail(cow_ctx* c, cow_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

#define HIP_TRY(ctx, expr)                                                                   \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(ctx, COW_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

bool is_pow2(int x) { return x > 0 && (x & (x - 1)) == 0; }

bool finite_view(const cow_view& v) {
    for (int i = 0; i < 3; ++i)
        if (!std::isfinite(v.eye[i])) return false;
    for (int i = 0; i < 9; ++i)
        if (!std::isfinite(v.R[i])) return false;
    return std::isfinite(v.fx) && std::isfinite(v.fy) && std::isfinite(v.cx) && std::isfinite(v.cy) &&
           v.fx != 0.0f && v.fy != 0.0f;
}

// extent of a block along axis a (a whole power of two, checked at load)
int extent(const cow_block_desc& d, int a) { return (int)(d.aabb_max[a] - d.aabb_min[a]); }
// texels (cells) along x, y, z: resolution per unit length times extent
void dims(const cow_block_desc& d, int res, int out[3]) {
    for (int a = 0; a < 3; ++a) out[a] = res * extent(d, a);
}
size_t grid_texels(const cow_block_desc& d) {
    int g[3];
    dims(d, d.grid_res, g);
    return (size_t)g[0] * g[1] * g[2];
}
// planes xy, xz, yz: (u, v) = (x, y), (x, z), (y, z)
size_t plane_texels(const cow_block_desc& d, int p) {
    int q[3];
    dims(d, d.plane_res, q);
    return p == 0 ? (size_t)q[0] * q[1] : (p == 1 ? (size_t)q[0] * q[2] : (size_t)q[1] * q[2]);
}
size_t occ_cells(const cow_block_desc& d) {
    int o[3];
    dims(d, d.occ_res, o);
    return (size_t)o[0] * o[1] * o[2];
}
// levels above the base of the max-pooled occupancy pyramid: log2 of the
// longest axis, so the top level is one cell
int occ_levels(const cow_block_desc& d) {
    int o[3];
    dims(d, d.occ_res, o);
    const int m = std::max(o[0], std::max(o[1], o[2]));
    int l = 0;
    while ((1 << l) < m) ++l;
    return l;
}
size_t occ_level_cells(const cow_block_desc& d, int l) {
    int o[3];
    dims(d, d.occ_res, o);
    return (size_t)std::max(o[0] >> l, 1) * std::max(o[1] >> l, 1) * std::max(o[2] >> l, 1);
}
size_t occ_pyramid_cells(const cow_block_desc& d) {
    size_t n = 0;
    for (int l = 1; l <= occ_levels(d); ++l) n += occ_level_cells(d, l);
    return n;
}
// per entry: [base][levels 1..L][skip levels], each base-sized part aligned
size_t occ_region(const cow_block_desc& d) {
    return align_up(occ_cells(d)) + align_up(occ_pyramid_cells(d)) + align_up(occ_cells(d));
}

cow_status validate_desc(cow_ctx* c, const cow_block_desc& d) {
    char buf[256];
    snprintf(buf, sizeof buf, "block %d lod %d: ", d.block_id, d.lod);
    std::string who(buf);
    if (d.lod < 0) return fail(c, COW_E_INVALID, who + "negative LOD");
    if (d.dtype != COW_U8 && d.dtype != COW_F32) return fail(c, COW_E_INVALID, who + "unknown dtype");
    if (!is_pow2(d.grid_res) || !is_pow2(d.plane_res) || !is_pow2(d.occ_res))
        return fail(c, COW_E_INVALID, who + "resolutions must be powers of two");
    if (d.grid_res % d.occ_res || d.plane_res % d.occ_res || d.occ_res > d.grid_res)
        return fail(c, COW_E_INVALID, who + "occupancy resolution must divide grid and plane resolution");
    if (d.grid_res < 2 || d.plane_res < 2)
        return fail(c, COW_E_INVALID, who + "grid and plane resolution must be at least 2");
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(d.aabb_min[a]) || !std::isfinite(d.aabb_max[a]))
            return fail(c, COW_E_INVALID, who + "non-finite AABB");
        const float e = d.aabb_max[a] - d.aabb_min[a];
        if (!(e >= 1.0f && e <= 64.0f) || e != (float)(int)e || !is_pow2((int)e))
            return fail(c, COW_E_INVALID, who + "block extents must be whole powers of two (1 to 64)");
    }
    int g[3], q[3];
    dims(d, d.grid_res, g);
    dims(d, d.plane_res, q);
    for (int a = 0; a < 3; ++a)
        if (g[a] > 1024 || q[a] > 8192)
            return fail(c, COW_E_INVALID, who + "resolution too large for 32-bit texel offsets");
    const size_t tex = d.dtype == COW_U8 ? 8 : 32;
    if (grid_texels(d) * tex >= (1ull << 31) || plane_texels(d, 0) * tex >= (1ull << 31) ||
        plane_texels(d, 1) * tex >= (1ull << 31) || plane_texels(d, 2) * tex >= (1ull << 31))
        return fail(c, COW_E_INVALID, who + "texture larger than 2 GiB");
    if (d.flags & ~COW_BLOCK_CONTRACTED) return fail(c, COW_E_INVALID, who + "unknown block flags");
    if ((d.flags & COW_BLOCK_CONTRACTED) && (d.aabb_max[0] - d.aabb_min[0] != 1.0f || d.aabb_max[1] - d.aabb_min[1] != 1.0f))
        return fail(c, COW_E_INVALID, who + "a contracted block must be one unit wide in x and y");
    if (!d.grid || !d.plane[0] || !d.plane[1] || !d.plane[2])
        return fail(c, COW_E_INVALID, who + "null texture pointer");
    if (d.dtype == COW_U8)
        for (int t = 0; t < 4; ++t)
            for (int ch = 0; ch < 8; ++ch)
                if (!std::isfinite(d.scale[t][ch]) || !std::isfinite(d.offset[t][ch]) ||
                    std::fabs(d.scale[t][ch]) > 1e30f)
                    return fail(c, COW_E_INVALID, who + "non-finite or too large scale/offset");
    return COW_OK;
}

// load workspace layout: [DevBlock table][occupancy grids, pyramids and skip
// levels][brick slot tables]
size_t load_layout(const cow_block_desc* b, int n, std::vector<size_t>* occ_off,
                   std::vector<size_t>* slot_off) {
    size_t off = align_up(sizeof(DevBlock) * (size_t)n);
    for (int i = 0; i < n; ++i) {
        if (occ_off) occ_off->push_back(off);
        off += occ_region(b[i]);
    }
    for (int i = 0; i < n; ++i) {
        if (slot_off) slot_off->push_back(off);
        off += align_up(occ_cells(b[i]) * 4);
    }
    return off;
}

// The next staging slot, at least `bytes` long: waits only for the copy
// that last read this slot (kStagingSlots calls back), and grows the slot
// when it is too small (the only allocation on the render path).
cow_status take_staging(cow_ctx* c, size_t bytes, Staging** out, bool may_grow = true) {
    Staging& st = c->staging[c->staging_next];
    c->staging_next = (c->staging_next + 1) % kStagingSlots;
    if (st.pending) {
        HIP_TRY(c, hipEventSynchronize(st.done));
        st.pending = false;
    }
    if (bytes > st.bytes) {
        if (!may_grow) return fail(c, COW_E_INTERNAL, "staging slot too small for a call that may not allocate");
        if (st.buf) HIP_TRY(c, hipHostFree(st.buf));
        st.buf = nullptr;
        st.bytes = 0;
        const size_t want = std::max(bytes, kStagingInitial);
        HIP_TRY(c, hipHostMalloc((void**)&st.buf, want, hipHostMallocDefault));
        st.bytes = want;
    }
    *out = &st;
    return COW_OK;
}

// mark a slot busy until the work enqueued on s so far (its copy) is done
cow_status release_staging(cow_ctx* c, Staging* st, hipStream_t s) {
    HIP_TRY(c, hipEventRecord(st->done, s));
    st->pending = true;
    return COW_OK;
}

int find_entry(const cow_ctx* c, int block_id, int lod) {
    for (size_t i = 0; i < c->entries.size(); ++i)
        if (c->entries[i].desc.block_id == block_id && c->entries[i].desc.lod == lod) return (int)i;
    return -1;
}

// ---------------------------------------------------------------------------
// per-call tables
// ---------------------------------------------------------------------------

struct CallTables {
    std::vector<DevView> views;
    std::vector<int32_t> refs;
    int64_t n_pix = 0;
    int32_t total_tiles = 0;
};

// xy distance from the eye to the block's footprint centre (Appendix D,
// "Depth sorting"), fp64
double xy_dist(const cow_view& v, const cow_block_desc& d) {
    const double cx = 0.5 * ((double)d.aabb_min[0] + (double)d.aabb_max[0]);
    const double cy = 0.5 * ((double)d.aabb_min[1] + (double)d.aabb_max[1]);
    const double dx = (double)v.eye[0] - cx, dy = (double)v.eye[1] - cy;
    return std::sqrt(dx * dx + dy * dy);
}

// Front-to-back order of a set of ground squares of mixed power-of-two sizes
// (merged LOD assets, each aligned to a multiple of its own size): recursive
// quadrant subdivision of an aligned square that covers the set.  Inside a
// square the quadrant on the eye's side of both centre lines goes first, the
// two quadrants beside it next and the opposite one last: a straight ray
// crosses each centre line at most once, so it can only meet the quadrants
// in an order consistent with this (the xy-distance order of equal squares
// does not extend to mixed sizes).
struct QuadOrder {
    const cow_ctx* c;
    double ex, ey;
    std::vector<int> in, out;
    void visit(double x0, double y0, double S) {
        std::vector<int> here;
        for (int e : in) {
            const cow_block_desc& d = c->entries[e].desc;
            if (d.aabb_min[0] >= x0 && d.aabb_max[0] <= x0 + S && d.aabb_min[1] >= y0 && d.aabb_max[1] <= y0 + S)
                here.push_back(e);
        }
        if (here.empty()) return;
        for (int e : here) {
            const cow_block_desc& d = c->entries[e].desc;
            if (d.aabb_min[0] == x0 && d.aabb_min[1] == y0 && d.aabb_max[0] - d.aabb_min[0] == S &&
                d.aabb_max[1] - d.aabb_min[1] == S) {
                out.push_back(e);  // the square itself is an entry (a partition holds nothing else here)
                return;
            }
        }
        if (S <= 1.0) return;
        const double h = 0.5 * S, cx = x0 + h, cy = y0 + h;
        const int qx = ex >= cx, qy = ey >= cy;
        const int seq[4][2] = {{qx, qy}, {1 - qx, qy}, {qx, 1 - qy}, {1 - qx, 1 - qy}};
        for (auto& q : seq) visit(x0 + q[0] * h, y0 + q[1] * h, h);
    }
};

cow_status build_tables(cow_ctx* c, const cow_view* views, int n_views, const cow_block_set* sets,
                        int tile_w, CallTables* T) {
    const int tile_h = 64 / tile_w;
    T->views.resize(n_views);
    T->refs.clear();
    T->n_pix = 0;
    T->total_tiles = 0;
    std::vector<int> seen(c->entries.size(), -1);
    for (int vi = 0; vi < n_views; ++vi) {
        const cow_view& v = views[vi];
        char who[64];
        snprintf(who, sizeof who, "view %d: ", vi);
        if (v.W <= 0 || v.H <= 0 || v.W > 65536 || v.H > 65536)
            return fail(c, COW_E_INVALID, std::string(who) + "image size out of range");
        if (v.crop_x0 < 0 || v.crop_y0 < 0 || v.crop_w < 0 || v.crop_h < 0 ||
            (int64_t)v.crop_x0 + v.crop_w > v.W || (int64_t)v.crop_y0 + v.crop_h > v.H)
            return fail(c, COW_E_INVALID, std::string(who) + "crop outside the image");
        if (!finite_view(v)) return fail(c, COW_E_INVALID, std::string(who) + "non-finite or singular camera");
        const cow_block_set& s = sets[vi];
        if (s.n < 0 || (s.n > 0 && !s.refs)) return fail(c, COW_E_INVALID, std::string(who) + "bad block set");
        std::vector<std::pair<double, int>> order;
        std::vector<int> ids;
        for (int r = 0; r < s.n; ++r) {
            const int e = find_entry(c, s.refs[r].block_id, s.refs[r].lod);
            if (e < 0) {
                char b[128];
                snprintf(b, sizeof b, "%s(block %d, lod %d) is not loaded", who, s.refs[r].block_id,
                         s.refs[r].lod);
                return fail(c, COW_E_NOT_LOADED, b);
            }
            for (int id : ids)
                if (id == s.refs[r].block_id)
                    return fail(c, COW_E_INVALID, std::string(who) + "a block appears twice in one set");
            ids.push_back(s.refs[r].block_id);
            order.push_back({xy_dist(v, c->entries[e].desc), e});
        }
        // the set's footprints must not overlap (a sample belongs to one entry)
        bool mixed = false;
        for (size_t a = 0; a < order.size(); ++a) {
            const cow_block_desc& da = c->entries[order[a].second].desc;
            const cow_block_desc& d0 = c->entries[order[0].second].desc;
            for (int k = 0; k < 2; ++k)
                if (da.aabb_max[k] - da.aabb_min[k] != d0.aabb_max[k] - d0.aabb_min[k]) mixed = true;
            for (size_t b = a + 1; b < order.size(); ++b) {
                const cow_block_desc& db = c->entries[order[b].second].desc;
                bool apart = false;
                for (int k = 0; k < 3; ++k)
                    apart = apart || da.aabb_max[k] <= db.aabb_min[k] || db.aabb_max[k] <= da.aabb_min[k];
                if (!apart) return fail(c, COW_E_INVALID, std::string(who) + "two entries of a set overlap");
            }
        }
        if (!mixed) {
            // equal squares: front to back by xy distance (their columns are the
            // Voronoi cells of their centres), ties to the lower block id
            std::stable_sort(order.begin(), order.end(), [&](const auto& a, const auto& b) {
                if (a.first != b.first) return a.first < b.first;
                return c->entries[a.second].desc.block_id < c->entries[b.second].desc.block_id;
            });
        } else {
            QuadOrder q{c, (double)v.eye[0], (double)v.eye[1], {}, {}};
            double lo[2] = {INFINITY, INFINITY}, hi[2] = {-INFINITY, -INFINITY}, big = 1.0;
            for (auto& o : order) {
                const cow_block_desc& d = c->entries[o.second].desc;
                q.in.push_back(o.second);
                for (int k = 0; k < 2; ++k) lo[k] = std::min(lo[k], (double)d.aabb_min[k]), hi[k] = std::max(hi[k], (double)d.aabb_max[k]);
                big = std::max(big, (double)(d.aabb_max[0] - d.aabb_min[0]));
            }
            // smallest aligned power-of-two square holding every footprint
            double S = big, x0 = 0, y0 = 0;
            for (;; S *= 2) {
                x0 = std::floor(lo[0] / S) * S, y0 = std::floor(lo[1] / S) * S;
                if (hi[0] <= x0 + S && hi[1] <= y0 + S) break;
            }
            q.visit(x0, y0, S);
            if (q.out.size() != order.size())
                return fail(c, COW_E_INVALID,
                            std::string(who) + "entries of mixed sizes must be squares aligned to their own size");
            for (size_t k = 0; k < order.size(); ++k) order[k].second = q.out[k];
        }
        DevView& d = T->views[vi];
        memset(&d, 0, sizeof d);
        for (int i = 0; i < 3; ++i) d.eye[i] = v.eye[i];
        for (int i = 0; i < 9; ++i) d.R[i] = v.R[i];
        d.fx = v.fx, d.fy = v.fy, d.cx = v.cx, d.cy = v.cy;
        d.x0 = v.crop_x0, d.y0 = v.crop_y0, d.w = v.crop_w, d.h = v.crop_h;
        d.tiles_x = (v.crop_w + tile_w - 1) / tile_w;
        const int tiles_y = (v.crop_h + tile_h - 1) / tile_h;
        d.n_tiles = d.tiles_x * tiles_y;
        d.tile_begin = T->total_tiles;
        d.pix_begin = T->n_pix;
        d.set_begin = (int32_t)T->refs.size();
        d.set_n = s.n;
        for (auto& o : order) T->refs.push_back(o.second);
        T->n_pix += (int64_t)v.crop_w * v.crop_h;
        if ((int64_t)T->total_tiles + d.n_tiles > (1ll << 30))
            return fail(c, COW_E_INVALID, "too many ray packets in one call");
        T->total_tiles += d.n_tiles;
    }
    return COW_OK;
}

struct RenderWs {
    DevView* views;
    int32_t* refs;
    float* aux;
    int32_t* counter;
    float** grad_ptrs;
    float* u;
    float* grad_mlp_scratch;
    cow::FoldJob* jobs;
    unsigned char* slots;
    size_t bytes;
};

// pair-slot buffer of a gradient texture of n texels: one 64-byte slot per
// texel, the pair that starts there
size_t slot_bytes(int64_t n_texels) { return align_up((size_t)n_texels * 64); }

// pair-slot buffers of every float32 entry: grid, then the three planes
size_t slots_total(const cow_block_desc* d, int64_t n) {
    size_t t = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (d[i].dtype != COW_F32) continue;
        t += slot_bytes((int64_t)grid_texels(d[i]));
        for (int p = 0; p < 3; ++p) t += slot_bytes((int64_t)plane_texels(d[i], p));
    }
    return t;
}

// render workspace: [views][refs][aux scratch][counter][grad pointers][u][mlp grad scratch][fold jobs][pair slots]
size_t render_ws_layout(int64_t n_views, int64_t n_refs, int64_t n_pix, bool need_aux, bool backward,
                        int64_t n_entries, size_t slots, unsigned char* base, RenderWs* w) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off += align_up(bytes);
        return base ? (void*)(base + o) : nullptr;
    };
    RenderWs r{};
    r.views = (DevView*)take(sizeof(DevView) * (size_t)std::max<int64_t>(n_views, 1));
    r.refs = (int32_t*)take(4 * (size_t)std::max<int64_t>(n_refs, 1));
    r.aux = need_aux ? (float*)take(32 * (size_t)n_pix) : nullptr;
    r.counter = (int32_t*)take(64);
    if (backward) {
        // gradient pointers (4 per entry), then pair-slot pointers (4 per entry)
        r.grad_ptrs = (float**)take(sizeof(float*) * 8 * (size_t)std::max<int64_t>(n_entries, 1));
        r.u = (float*)take(32 * (size_t)n_pix);
        r.grad_mlp_scratch = (float*)take(4 * cow::kMlpParamsMax);
        r.jobs = (cow::FoldJob*)take(sizeof(cow::FoldJob) * 4 * (size_t)std::max<int64_t>(n_entries, 1));
        r.slots = (unsigned char*)take(slots);
    }
    r.bytes = off;
    if (w) *w = r;
    return off;
}

cow_status validate_params(cow_ctx* c, const cow_render_params* p) {
    if (!p) return fail(c, COW_E_INVALID, "null params");
    if (p->mode == COW_MODE_CHORD) {
        if (p->n_steps < 1 || p->n_steps > (1 << 16)) return fail(c, COW_E_INVALID, "n_steps out of range");
    } else if (p->mode == COW_MODE_GRID) {
        if (!(p->delta > 0.0f) || !std::isfinite(p->delta) || p->delta < 1e-6f)
            return fail(c, COW_E_INVALID, "delta must be a positive finite step");
        if (p->max_steps < 1 || p->max_steps > (1 << 22)) return fail(c, COW_E_INVALID, "max_steps out of range");
    } else {
        return fail(c, COW_E_INVALID, "unknown mode");
    }
    if (!(p->t_min >= 0.0f && p->t_min < 1.0f)) return fail(c, COW_E_INVALID, "t_min must be in [0, 1)");
    if (p->pe_freqs < 0 || p->pe_freqs > 4) return fail(c, COW_E_INVALID, "pe_freqs must be in [0, 4]");
    if (p->pe_freqs != 0 && p->pe_freqs != 4)
        return fail(c, COW_E_UNSUPPORTED, "the deferred MLP kernels are built for 0 or 4 encoding frequencies");
    if (!(p->ext_delta >= 0.0f && p->ext_delta <= 1.0f)) return fail(c, COW_E_INVALID, "ext_delta must be in [0, 1]");
    if (p->ext_max_steps < 0 || p->ext_max_steps > (1 << 16)) return fail(c, COW_E_INVALID, "ext_max_steps out of range");
    return COW_OK;
}

// whether a call's sets hold a contracted block
bool any_contracted(const cow_ctx* c, const std::vector<int32_t>& refs) {
    for (int32_t e : refs)
        if (c->entries[e].desc.flags & COW_BLOCK_CONTRACTED) return true;
    return false;
}

// the per-block composites buffer holds a slot for every set position of every view
cow_status check_block_aux(cow_ctx* c, const CallTables& T, const cow_render_params* p) {
    if (!p->block_aux) return COW_OK;
    if ((uintptr_t)p->block_aux % 16) return fail(c, COW_E_INVALID, "block_aux must be 16-byte aligned");
    for (const DevView& v : T.views)
        if (v.set_n > p->block_aux_n) return fail(c, COW_E_INVALID, "block_aux_n is below a view's set size");
    return COW_OK;
}

cow_status check_dtypes(cow_ctx* c, const CallTables& T, int* dtype) {
    int dt = -1;
    for (int32_t e : T.refs) {
        const int d = c->entries[e].desc.dtype;
        if (dt < 0) dt = d;
        if (d != dt) return fail(c, COW_E_UNSUPPORTED, "one render call must use blocks of a single dtype");
    }
    *dtype = dt < 0 ? c->dtype : dt;
    return COW_OK;
}

cow_status upload_tables(cow_ctx* c, const CallTables& T, const RenderWs& w, hipStream_t s, bool may_grow = true) {
    const size_t vb = sizeof(DevView) * T.views.size(), rb = 4 * T.refs.size();
    Staging* sl = nullptr;
    cow_status st = take_staging(c, align_up(vb) + rb + 64, &sl, may_grow);
    if (st != COW_OK) return st;
    memcpy(sl->buf, T.views.data(), vb);
    memcpy(sl->buf + align_up(vb), T.refs.data(), rb);
    if (vb) HIP_TRY(c, hipMemcpyAsync(w.views, sl->buf, vb, hipMemcpyHostToDevice, s));
    if (rb) HIP_TRY(c, hipMemcpyAsync(w.refs, sl->buf + align_up(vb), rb, hipMemcpyHostToDevice, s));
    return release_staging(c, sl, s);
}

cow::MarchArgs march_args(cow_ctx* c, const CallTables& T, const RenderWs& w,
                          const cow_render_params* p, int dtype, float* aux, float* trans) {
    cow::MarchArgs a{};
    a.blocks = c->d_blocks;
    a.views = w.views;
    a.n_views = (int32_t)T.views.size();
    a.refs = w.refs;
    a.total_tiles = T.total_tiles;
    a.tile_w = c->cfg.tile_w;
    a.tile_h = 64 / c->cfg.tile_w;
    a.mode = p->mode;
    a.n_steps = p->n_steps;
    a.max_steps = p->max_steps;
    a.t_min = p->t_min;
    a.delta = p->delta;
    for (int i = 0; i < 3; ++i) a.scene_lo[i] = c->scene_lo[i], a.scene_hi[i] = c->scene_hi[i];
    a.use_sparse = (p->flags & COW_F_SPARSE) ? 1 : 0;
    a.flat_occ = (p->flags & COW_F_FLAT_OCC) ? 1 : 0;
    a.blocks_dtype = dtype;
    a.aux = aux;
    a.trans = trans;
    a.counts = p->counts;
    a.opacity = p->opacity;
    a.block_mlp = p->block_mlp;
    a.pe = p->pe_freqs;
    a.rgb = nullptr;
    a.work_counter = w.counter;
    a.persistent = persistent_for(c->cfg, dtype);
    a.only_view = -1;
    a.only_set_pos = -1;
    a.contract = any_contracted(c, T.refs) ? 1 : 0;
    a.ext_delta = a.contract && p->ext_max_steps > 0 ? p->ext_delta : 0.0f;
    a.ext_max_steps = a.ext_delta > 0.0f ? p->ext_max_steps : 0;
    a.block_aux = p->block_aux;
    a.block_aux_n = p->block_aux_n;
    return a;
}

// the launch sequence of one forward render (what a graph captures)
cow_status enqueue_forward(cow_ctx* c, const CallTables& T, const cow::MarchArgs& a0,
                           const cow::MlpArgs& m, bool per_block, hipStream_t s) {
    if (per_block) {
        // baseline: one launch per view per block, each blending its block
        // into the view's running (A, T) in depth order (the paper's
        // one-shader-per-block viewer, Sec. 4.2)
        for (size_t v = 0; v < T.views.size(); ++v) {
            const DevView& dv = T.views[v];
            if (dv.n_tiles == 0) continue;
            cow::MarchArgs a = a0;
            a.persistent = 0;
            a.only_view = (int32_t)v;
            a.total_tiles = dv.n_tiles;
            const int nb = dv.set_n;
            for (int r = 0; r < std::max(nb, 1); ++r) {
                a.only_set_pos = nb == 0 ? -1 : r;
                HIP_TRY(c, cow::launch_march(a, c->cfg.waves, s));
            }
        }
    } else {
        if (a0.persistent) HIP_TRY(c, cow::launch_reset_counter(a0.work_counter, s));
        if (c->timing) HIP_TRY(c, hipEventRecord(c->ev[0], s));
        HIP_TRY(c, cow::launch_march(a0, c->cfg.waves, s));
        if (c->timing) HIP_TRY(c, hipEventRecord(c->ev[1], s));
    }
    if (!a0.block_mlp) HIP_TRY(c, cow::launch_mlp(m, s));  // per-block shading ran in the march
    return COW_OK;
}

cow_status run_graph(cow_ctx* c, const CallTables& T, const cow::MarchArgs& a, const cow::MlpArgs& m,
                     bool per_block, hipStream_t s) {
    std::vector<unsigned char> key(sizeof a + sizeof m + 8);
    memcpy(key.data(), &a, sizeof a);
    memcpy(key.data() + sizeof a, &m, sizeof m);
    const int64_t extra = (per_block ? 1 : 0) | ((int64_t)c->cfg.waves << 8);
    memcpy(key.data() + sizeof a + sizeof m, &extra, 8);
    for (auto& g : c->graphs)
        if (g.key == key) {
            HIP_TRY(c, hipGraphLaunch(g.exec, s));
            return COW_OK;
        }
    const bool timing = c->timing;
    c->timing = false;  // events are not recorded inside a captured graph
    if (!c->capture_stream) HIP_TRY(c, hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
    hipStream_t cs = c->capture_stream;
    HIP_TRY(c, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    cow_status st = enqueue_forward(c, T, a, m, per_block, cs);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &graph);
    c->timing = timing;
    if (st != COW_OK) return st;
    if (e != hipSuccess) return fail(c, COW_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    GraphEntry g;
    g.key = key;
    g.graph = graph;
    HIP_TRY(c, hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0));
    if (c->graphs.size() >= 16) {
        (void)hipGraphExecDestroy(c->graphs.front().exec);
        (void)hipGraphDestroy(c->graphs.front().graph);
        c->graphs.erase(c->graphs.begin());
    }
    c->graphs.push_back(g);
    HIP_TRY(c, hipGraphLaunch(g.exec, s));
    return COW_OK;
}

void drop_graphs(cow_ctx* c) {
    for (auto& g : c->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        (void)hipGraphDestroy(g.graph);
    }
    c->graphs.clear();
}

// ---------------------------------------------------------------------------
// selection (fp64)
// ---------------------------------------------------------------------------

// A box is culled when all eight corners lie strictly outside one of the
// frustum side planes or behind the camera plane, with a relative margin of
// 1e-5 that absorbs the fp32 rounding of the rays.
bool box_outside_frustum(const cow_view& v, const double lo[3], const double hi[3]) {
    double Rm[9], e[3];
    for (int k = 0; k < 9; ++k) Rm[k] = v.R[k];
    for (int k = 0; k < 3; ++k) e[k] = v.eye[k];
    const double x0 = v.crop_x0, x1 = (double)v.crop_x0 + v.crop_w;
    const double y0 = v.crop_y0, y1 = (double)v.crop_y0 + v.crop_h;
    const double fx = v.fx, fy = v.fy, cx = v.cx, cy = v.cy;
    const double n[5][3] = {{fx, 0, cx - x0}, {-fx, 0, x1 - cx}, {0, fy, cy - y0}, {0, -fy, y1 - cy}, {0, 0, 1}};
    double X[8][3], len[8];
    for (int k = 0; k < 8; ++k) {
        const double P[3] = {(k & 1) ? hi[0] : lo[0], (k & 2) ? hi[1] : lo[1], (k & 4) ? hi[2] : lo[2]};
        const double w[3] = {P[0] - e[0], P[1] - e[1], P[2] - e[2]};
        for (int a = 0; a < 3; ++a) X[k][a] = Rm[a] * w[0] + Rm[3 + a] * w[1] + Rm[6 + a] * w[2];
        len[k] = std::sqrt(X[k][0] * X[k][0] + X[k][1] * X[k][1] + X[k][2] * X[k][2]);
    }
    for (int p = 0; p < 5; ++p) {
        const double nn = std::sqrt(n[p][0] * n[p][0] + n[p][1] * n[p][1] + n[p][2] * n[p][2]);
        bool all_out = true;
        for (int k = 0; k < 8 && all_out; ++k) {
            const double sd = (n[p][0] * X[k][0] + n[p][1] * X[k][1] + n[p][2] * X[k][2]) / nn;
            if (!(sd < -1e-5 * len[k])) all_out = false;
        }
        if (all_out) return true;
    }
    return false;
}

// Quadtree selection (Appendix D "Dynamic Loading" over the merged assets of
// Sec. 4.5: an entry of LOD l covers 2^l x 2^l blocks).  From the coarsest
// LOD down: an entry of LOD l > 0 is drawn when every visible LOD l-1 entry
// inside it is at least thresholds[l-1] from the eye (vacuously when none is
// visible), otherwise its visible children are examined.  Distance: eye to
// (centre x, centre y, highest LOD-0 top inside the entry), fp64; culling of
// [lo, (hi_x, hi_y, the entry's own top)].  Order: the coarsest entries by xy
// distance (ties: lower id), inside an entry its children by quadrant (the
// eye's quadrant, the two beside it, the opposite one; ties: lower id).
struct QuadSelect {
    cow_ctx* c;
    const cow_view* v;
    const cow_lod_policy* pol;
    std::vector<std::vector<int>> kids;
    std::vector<double> zfine;
    std::vector<char> pinned;  // holds a contracted finest-level block: always opened, never culled
    std::vector<int> out;

    static bool inside_xy(const cow_block_desc& a, const cow_block_desc& b) {
        return a.aabb_min[0] >= b.aabb_min[0] && a.aabb_max[0] <= b.aabb_max[0] && a.aabb_min[1] >= b.aabb_min[1] &&
               a.aabb_max[1] <= b.aabb_max[1];
    }
    double centre(int e, int k) const {
        const cow_block_desc& d = c->entries[e].desc;
        return 0.5 * ((double)d.aabb_min[k] + (double)d.aabb_max[k]);
    }
    double dist(int e) const {
        const double dx = (double)v->eye[0] - centre(e, 0), dy = (double)v->eye[1] - centre(e, 1);
        const double dz = (double)v->eye[2] - zfine[e];
        return std::sqrt(dx * dx + dy * dy + dz * dz);
    }
    bool visible(int e) const {
        if (!pol->cull || pinned[e]) return true;
        const cow_block_desc& d = c->entries[e].desc;
        const double lo[3] = {d.aabb_min[0], d.aabb_min[1], d.aabb_min[2]};
        const double hi[3] = {d.aabb_max[0], d.aabb_max[1], c->entries[e].ztop};
        return !box_outside_frustum(*v, lo, hi);
    }
    void visit(int e) {
        const int l = c->entries[e].desc.lod;
        if (l == 0) {
            out.push_back(e);
            return;
        }
        std::vector<std::pair<int, int>> seen;  // (rank, entry)
        bool far = true;
        const bool ex = (double)v->eye[0] >= centre(e, 0), ey = (double)v->eye[1] >= centre(e, 1);
        for (int f : kids[e]) {
            if (!visible(f)) continue;
            if (dist(f) < pol->thresholds[l - 1]) far = false;
            const int rank = ((centre(f, 0) >= centre(e, 0)) != ex) + ((centre(f, 1) >= centre(e, 1)) != ey);
            seen.push_back({rank, f});
        }
        if (far && !pinned[e]) {
            out.push_back(e);
            return;
        }
        std::stable_sort(seen.begin(), seen.end(), [&](const auto& a, const auto& b) {
            if (a.first != b.first) return a.first < b.first;
            return c->entries[a.second].desc.block_id < c->entries[b.second].desc.block_id;
        });
        for (auto& k : seen) visit(k.second);
    }
};

cow_status select_quadtree(cow_ctx* c, const cow_view* v, const cow_lod_policy* pol, cow_block_ref* out, int cap,
                           int* n_out) {
    const int ne = (int)c->entries.size();
    int L = 0;
    for (auto& e : c->entries) L = std::max(L, e.desc.lod);
    if (pol->n_thresholds < L) return fail(c, COW_E_INVALID, "quadtree selection needs a threshold per finer LOD");
    QuadSelect q{c, v, pol, std::vector<std::vector<int>>(ne), std::vector<double>(ne, -INFINITY),
                 std::vector<char>(ne, 0), {}};
    for (int e = 0; e < ne; ++e) {
        const cow_block_desc& d = c->entries[e].desc;
        for (int f = 0; f < ne; ++f) {
            const cow_block_desc& g = c->entries[f].desc;
            if (!QuadSelect::inside_xy(g, d)) continue;
            if (g.lod == 0) q.zfine[e] = std::max(q.zfine[e], c->entries[f].ztop);
            if (g.lod == 0 && (g.flags & COW_BLOCK_CONTRACTED)) q.pinned[e] = 1;
            if (d.lod > 0 && g.lod == d.lod - 1) q.kids[e].push_back(f);
        }
    }
    std::vector<std::pair<double, int>> roots;
    for (int e = 0; e < ne; ++e) {
        if (c->entries[e].desc.lod != L || !q.visible(e)) continue;
        if (pol->n_thresholds > L && q.dist(e) >= pol->thresholds[L] && !q.pinned[e]) continue;
        const double dx = (double)v->eye[0] - q.centre(e, 0), dy = (double)v->eye[1] - q.centre(e, 1);
        roots.push_back({std::sqrt(dx * dx + dy * dy), e});
    }
    std::stable_sort(roots.begin(), roots.end(), [&](const auto& a, const auto& b) {
        if (a.first != b.first) return a.first < b.first;
        return c->entries[a.second].desc.block_id < c->entries[b.second].desc.block_id;
    });
    for (auto& r : roots) q.visit(r.second);
    const int n = (int)q.out.size();
    for (int i = 0; i < n && i < cap; ++i) {
        out[i].block_id = c->entries[q.out[i]].desc.block_id;
        out[i].lod = c->entries[q.out[i]].desc.lod;
    }
    *n_out = std::min(n, cap);
    if (n > cap) return fail(c, COW_E_INVALID, "output capacity too small");
    return COW_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

cow_status cow_create(cow_ctx** out, int device) {
    if (!out) return COW_E_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return COW_E_HIP;
    if (device < 0 || device >= n || device >= kMaxDevices) return COW_E_INVALID;
    cow_ctx* c = new (std::nothrow) cow_ctx();
    if (!c) return COW_E_INTERNAL;
    c->device = device;
    hipDeviceProp_t prop;
    if (hipSetDevice(device) != hipSuccess || hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete c;
        return COW_E_HIP;
    }
    c->n_cus = prop.multiProcessorCount;
    c->arch = prop.gcnArchName;
    for (auto& st : c->staging) {
        if (hipEventCreateWithFlags(&st.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void**)&st.buf, kStagingInitial, hipHostMallocDefault) != hipSuccess) {
            cow_destroy(c);
            return COW_E_HIP;
        }
        st.bytes = kStagingInitial;
    }
    void* sp = nullptr;
    if (scratch_address(device, &sp) != hipSuccess) {
        cow_destroy(c);
        return COW_E_HIP;
    }
    c->scratch = (unsigned char*)sp;
    *out = c;
    return COW_OK;
}

cow_status cow_destroy(cow_ctx* c) {
    if (!c) return COW_E_INVALID;
    (void)hipSetDevice(c->device);
    for (auto& st : c->staging)
        if (st.pending) (void)hipEventSynchronize(st.done);
    drop_graphs(c);
    for (auto& st : c->staging) {
        if (st.buf) (void)hipHostFree(st.buf);
        if (st.done) (void)hipEventDestroy(st.done);
    }
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    for (auto& e : c->ev)
        if (e) (void)hipEventDestroy(e);
    delete c;
    return COW_OK;
}

const char* cow_last_error(const cow_ctx* c) { return c ? c->err.c_str() : "null context"; }

cow_status cow_query_workspace(cow_ctx* c, const cow_block_desc* blocks, int n_blocks, int max_views,
                               int64_t max_pixels, size_t* load_bytes, size_t* render_bytes,
                               size_t* backward_bytes) {
    if (!c) return COW_E_INVALID;
    if (n_blocks < 0 || n_blocks > kMaxBlocks || (n_blocks > 0 && !blocks))
        return fail(c, COW_E_INVALID, "bad block list");
    if (max_views < 0 || max_views > kMaxViews || max_pixels < 0)
        return fail(c, COW_E_INVALID, "bad view/pixel limits");
    for (int i = 0; i < n_blocks; ++i) {
        cow_status s = validate_desc(c, blocks[i]);
        if (s != COW_OK) return s;
    }
    if (load_bytes) *load_bytes = load_layout(blocks, n_blocks, nullptr, nullptr);
    const int64_t refs = (int64_t)max_views * std::max(n_blocks, 1);
    if (render_bytes) *render_bytes = render_ws_layout(max_views, refs, max_pixels, true, false, n_blocks, 0, nullptr, nullptr);
    if (backward_bytes)
        *backward_bytes = render_ws_layout(max_views, refs, max_pixels, true, true, n_blocks,
                                           slots_total(blocks, n_blocks), nullptr, nullptr);
    return COW_OK;
}

cow_status cow_load_blocks(cow_ctx* c, const cow_block_desc* blocks, int n, void* load_ws,
                           size_t load_bytes, hipStream_t stream) {
    if (!c) return COW_E_INVALID;
    if (n <= 0 || n > kMaxBlocks || !blocks) return fail(c, COW_E_INVALID, "need at least one block");
    for (int i = 0; i < n; ++i) {
        cow_status s = validate_desc(c, blocks[i]);
        if (s != COW_OK) return s;
    }
    // unique (block, LOD); all LODs of a block share its AABB's lower corner;
    // the entries of one LOD have disjoint boxes (a ground partition,
    // Sec. 4.1); entries of different LODs may overlap (a merged LOD asset
    // covers several finer blocks)
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            const auto &a = blocks[i], &b = blocks[j];
            if (a.block_id == b.block_id) {
                if (a.lod == b.lod) return fail(c, COW_E_INVALID, "duplicate (block, LOD)");
                for (int k = 0; k < 3; ++k)
                    if (a.aabb_min[k] != b.aabb_min[k])
                        return fail(c, COW_E_INVALID, "LODs of one block must share its AABB");
            } else if (a.lod == b.lod) {
                bool overlap = true;
                for (int k = 0; k < 3; ++k)
                    overlap = overlap && a.aabb_min[k] < b.aabb_max[k] && b.aabb_min[k] < a.aabb_max[k];
                if (overlap) return fail(c, COW_E_INVALID, "blocks overlap");
            }
        }
    {  // contracted blocks span the scene's full height
        float zlo = INFINITY, zhi = -INFINITY;
        for (int i = 0; i < n; ++i) zlo = std::min(zlo, blocks[i].aabb_min[2]), zhi = std::max(zhi, blocks[i].aabb_max[2]);
        for (int i = 0; i < n; ++i)
            if ((blocks[i].flags & COW_BLOCK_CONTRACTED) && (blocks[i].aabb_min[2] != zlo || blocks[i].aabb_max[2] != zhi))
                return fail(c, COW_E_INVALID, "a contracted block must span the scene's full height");
    }
    std::vector<size_t> occ_off, slot_off;
    const size_t need = load_layout(blocks, n, &occ_off, &slot_off);
    if (!load_ws || load_bytes < need) return fail(c, COW_E_WORKSPACE, "load workspace too small");
    HIP_TRY(c, hipSetDevice(c->device));
    drop_graphs(c);
    c->entries.clear();
    c->loaded = false;
    c->bricks_packed = false;
    c->load_ws = (unsigned char*)load_ws;
    c->load_bytes = load_bytes;
    c->d_blocks = (DevBlock*)load_ws;
    c->h_blocks.assign(n, DevBlock{});
    c->mixed_dtype = false;
    c->dtype = blocks[0].dtype;
    for (int k = 0; k < 3; ++k) c->scene_lo[k] = INFINITY, c->scene_hi[k] = -INFINITY;
    for (int i = 0; i < n; ++i) {
        Entry e;
        e.desc = blocks[i];
        e.occ_off = occ_off[i];
        e.slot_off = slot_off[i];
        c->entries.push_back(e);
        DevBlock& d = c->h_blocks[i];
        for (int k = 0; k < 3; ++k) {
            d.lo[k] = blocks[i].aabb_min[k];
            d.hi[k] = blocks[i].aabb_max[k];
            c->scene_lo[k] = std::min(c->scene_lo[k], d.lo[k]);
            c->scene_hi[k] = std::max(c->scene_hi[k], d.hi[k]);
        }
        d.R = blocks[i].grid_res;
        d.Rp = blocks[i].plane_res;
        d.O = blocks[i].occ_res;
        dims(blocks[i], d.R, d.gd);
        dims(blocks[i], d.Rp, d.pd);
        dims(blocks[i], d.O, d.od);
        d.dtype = blocks[i].dtype;
        d.contracted = (blocks[i].flags & COW_BLOCK_CONTRACTED) ? 1 : 0;
        if (d.dtype != c->dtype) c->mixed_dtype = true;
        d.grid = blocks[i].grid;
        for (int k = 0; k < 3; ++k) d.plane[k] = blocks[i].plane[k];
        d.occ = c->load_ws + occ_off[i];
        d.occ_pyr = d.occ + align_up(occ_cells(blocks[i]));
        d.skip = d.occ_pyr + align_up(occ_pyramid_cells(blocks[i]));
        d.n_levels = occ_levels(blocks[i]);
        d.brick_slot = nullptr;
        d.bricks = nullptr;
        for (int t = 0; t < 4; ++t)
            for (int ch = 0; ch < 8; ++ch) {
                d.scale[t][ch] = d.dtype == COW_U8 ? blocks[i].scale[t][ch] : 1.0f;
                d.offset[t][ch] = d.dtype == COW_U8 ? blocks[i].offset[t][ch] : 0.0f;
            }
        // fp32 products, rounded once each as on the device
        const float log2e = 1.44269504088896341f;
        for (int ch = 0; ch < 8; ++ch) {
            const float sgn = ch == 0 ? log2e : -log2e;
            for (int t = 0; t < 4; ++t) d.dsc[t][ch] = d.scale[t][ch] * (16777216.0f * sgn);
            d.dosum[ch] = (((d.offset[0][ch] + d.offset[1][ch]) + d.offset[2][ch]) + d.offset[3][ch]) * sgn;
        }
    }
    const size_t tb = sizeof(DevBlock) * (size_t)n;
    Staging* sl = nullptr;
    cow_status st = take_staging(c, tb, &sl);
    if (st != COW_OK) return st;
    memcpy(sl->buf, c->h_blocks.data(), tb);
    HIP_TRY(c, hipMemcpyAsync(c->d_blocks, sl->buf, tb, hipMemcpyHostToDevice, stream));
    st = release_staging(c, sl, stream);
    if (st != COW_OK) return st;
    for (int i = 0; i < n; ++i) {
        HIP_TRY(c, cow::launch_occupancy(c->d_blocks, i, (int)occ_cells(blocks[i]), stream));
        HIP_TRY(c, cow::launch_occupancy_pyramid(c->d_blocks, i, c->h_blocks[i].n_levels, c->h_blocks[i].od, stream));
    }
    // z_top of each entry from its occupancy (top of the highest occupied cell)
    size_t tot = 0;
    for (int i = 0; i < n; ++i) tot += occ_cells(blocks[i]);
    std::vector<unsigned char> occ(tot);
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
        HIP_TRY(c, hipMemcpyAsync(occ.data() + off, c->load_ws + occ_off[i], occ_cells(blocks[i]),
                                  hipMemcpyDeviceToHost, stream));
        off += occ_cells(blocks[i]);
    }
    HIP_TRY(c, hipStreamSynchronize(stream));
    off = 0;
    for (int i = 0; i < n; ++i) {
        int o[3];
        dims(blocks[i], blocks[i].occ_res, o);
        const size_t layer = (size_t)o[0] * o[1];
        int top = -1;
        for (int z = 0; z < o[2]; ++z)
            for (size_t k = 0; k < layer; ++k)
                if (occ[off + (size_t)z * layer + k]) top = z;
        const double ext = (double)blocks[i].aabb_max[2] - (double)blocks[i].aabb_min[2];
        c->entries[i].ztop = (double)blocks[i].aabb_min[2] + (double)(top + 1) / o[2] * ext;
        // a contracted block's texture z is the contracted coordinate, not
        // world z, and it owns the space above its box: its box top
        if (blocks[i].flags & COW_BLOCK_CONTRACTED) c->entries[i].ztop = (double)blocks[i].aabb_max[2];
        off += occ_cells(blocks[i]);
    }
    c->loaded = true;
    return COW_OK;
}

cow_status cow_get_occupancy(cow_ctx* c, int block_id, int lod, uint8_t* host_out, size_t n) {
    if (!c) return COW_E_INVALID;
    if (!host_out) return fail(c, COW_E_INVALID, "null output");
    const int e = find_entry(c, block_id, lod);
    if (e < 0) return fail(c, COW_E_NOT_LOADED, "block not loaded");
    const size_t cells = occ_cells(c->entries[e].desc);
    if (n < cells) return fail(c, COW_E_INVALID, "output too small");
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipDeviceSynchronize());
    HIP_TRY(c, hipMemcpy(host_out, c->load_ws + c->entries[e].occ_off, cells, hipMemcpyDeviceToHost));
    return COW_OK;
}

cow_status cow_get_occupancy_level(cow_ctx* c, int block_id, int lod, int level, uint8_t* host_out, size_t n) {
    if (!c) return COW_E_INVALID;
    if (!host_out) return fail(c, COW_E_INVALID, "null output");
    const int e = find_entry(c, block_id, lod);
    if (e < 0) return fail(c, COW_E_NOT_LOADED, "block not loaded");
    const cow_block_desc& d = c->entries[e].desc;
    if (level < 0 || level > occ_levels(d)) return fail(c, COW_E_INVALID, "no such occupancy level");
    const size_t cells = occ_level_cells(d, level);
    if (n < cells) return fail(c, COW_E_INVALID, "output too small");
    size_t off = c->entries[e].occ_off;
    if (level > 0) {
        off += align_up(occ_cells(d));
        for (int l = 1; l < level; ++l) off += occ_level_cells(d, l);
    }
    HIP_TRY(c, hipSetDevice(c->device));
    HIP_TRY(c, hipDeviceSynchronize());
    HIP_TRY(c, hipMemcpy(host_out, c->load_ws + off, cells, hipMemcpyDeviceToHost));
    return COW_OK;
}

cow_status cow_select_blocks(cow_ctx* c, const cow_view* v, const cow_lod_policy* pol, cow_block_ref* out,
                             int cap, int* n_out) {
    if (!c) return COW_E_INVALID;
    if (!v || !pol || !n_out || (cap > 0 && !out)) return fail(c, COW_E_INVALID, "null argument");
    if (!c->loaded) return fail(c, COW_E_NOT_LOADED, "no blocks loaded");
    if (!finite_view(*v)) return fail(c, COW_E_INVALID, "non-finite or singular camera");
    if (pol->n_thresholds < 1 || pol->n_thresholds > 3) return fail(c, COW_E_INVALID, "1 to 3 thresholds");
    if (pol->quadtree) return select_quadtree(c, v, pol, out, cap, n_out);
    struct Pick {
        double key;
        int id, entry;
    };
    std::vector<Pick> picks;
    for (size_t e = 0; e < c->entries.size(); ++e) {
        const cow_block_desc& d = c->entries[e].desc;
        if (d.lod != 0) continue;  // decide once per block, from its finest level
        const double cx = 0.5 * ((double)d.aabb_min[0] + (double)d.aabb_max[0]);
        const double cy = 0.5 * ((double)d.aabb_min[1] + (double)d.aabb_max[1]);
        const double dx = (double)v->eye[0] - cx, dy = (double)v->eye[1] - cy;
        const double dz = (double)v->eye[2] - c->entries[e].ztop;
        const double dist = std::sqrt(dx * dx + dy * dy + dz * dz);
        int lod = -1;
        for (int l = 0; l < pol->n_thresholds; ++l)
            if (dist < pol->thresholds[l]) {
                lod = l;
                break;
            }
        // a contracted boundary block also owns the unbounded space beyond
        // its outer faces: never dropped by the far cut (its coarsest level
        // the policy names instead) and never culled
        const bool contracted = (d.flags & COW_BLOCK_CONTRACTED) != 0;
        if (lod < 0 && contracted) lod = pol->n_thresholds - 1;
        if (lod < 0) continue;  // beyond the far cut
        const int chosen = find_entry(c, d.block_id, lod);
        if (chosen < 0) return fail(c, COW_E_NOT_LOADED, "selected LOD is not loaded");
        if (pol->cull && !contracted) {
            const cow_block_desc& cd = c->entries[chosen].desc;
            const double lo[3] = {cd.aabb_min[0], cd.aabb_min[1], cd.aabb_min[2]};
            const double hi[3] = {cd.aabb_max[0], cd.aabb_max[1], c->entries[chosen].ztop};
            if (box_outside_frustum(*v, lo, hi)) continue;
        }
        picks.push_back({std::sqrt(dx * dx + dy * dy), d.block_id, chosen});
    }
    std::stable_sort(picks.begin(), picks.end(), [](const Pick& a, const Pick& b) {
        if (a.key != b.key) return a.key < b.key;
        return a.id < b.id;
    });
    const int n = (int)picks.size();
    for (int i = 0; i < n && i < cap; ++i) {
        out[i].block_id = c->entries[picks[i].entry].desc.block_id;
        out[i].lod = c->entries[picks[i].entry].desc.lod;
    }
    *n_out = std::min(n, cap);
    if (n > cap) return fail(c, COW_E_INVALID, "output capacity too small");
    return COW_OK;
}

cow_status cow_query_bricks(cow_ctx* c, size_t* brick_bytes) {
    if (!c || !brick_bytes) return COW_E_INVALID;
    if (!c->loaded) return fail(c, COW_E_NOT_LOADED, "no blocks loaded");
    size_t total = 0;
    std::vector<unsigned char> occ;
    for (auto& e : c->entries) {
        if (e.desc.dtype != COW_U8) continue;
        const size_t cells = occ_cells(e.desc);
        occ.resize(cells);
        HIP_TRY(c, hipDeviceSynchronize());
        HIP_TRY(c, hipMemcpy(occ.data(), c->load_ws + e.occ_off, cells, hipMemcpyDeviceToHost));
        size_t nb = 0;
        for (unsigned char o : occ) nb += o != 0;
        const size_t s2 = (size_t)(e.desc.grid_res / e.desc.occ_res) + 2;
        total += align_up(nb * s2 * s2 * s2 * 8);
    }
    *brick_bytes = total;
    return COW_OK;
}

cow_status cow_pack_bricks(cow_ctx* c, void* brick_ws, size_t brick_bytes, hipStream_t stream) {
    if (!c) return COW_E_INVALID;
    if (!c->loaded) return fail(c, COW_E_NOT_LOADED, "no blocks loaded");
    size_t need = 0;
    cow_status st = cow_query_bricks(c, &need);
    if (st != COW_OK) return st;
    if (need > 0 && (!brick_ws || brick_bytes < need)) return fail(c, COW_E_WORKSPACE, "brick workspace too small");
    HIP_TRY(c, hipSetDevice(c->device));
    drop_graphs(c);
    size_t off = 0;
    std::vector<unsigned char> occ;
    std::vector<int32_t> slots;
    for (size_t i = 0; i < c->entries.size(); ++i) {
        Entry& e = c->entries[i];
        if (e.desc.dtype != COW_U8) continue;
        const size_t cells = occ_cells(e.desc);
        occ.resize(cells);
        slots.assign(cells, -1);
        HIP_TRY(c, hipMemcpy(occ.data(), c->load_ws + e.occ_off, cells, hipMemcpyDeviceToHost));
        int nb = 0;
        for (size_t k = 0; k < cells; ++k)
            if (occ[k]) slots[k] = nb++;
        e.n_bricks = nb;
        HIP_TRY(c, hipMemcpy(c->load_ws + e.slot_off, slots.data(), cells * 4, hipMemcpyHostToDevice));
        DevBlock& d = c->h_blocks[i];
        d.brick_slot = (const int32_t*)(c->load_ws + e.slot_off);
        d.bricks = (const uint8_t*)brick_ws + off;
        const size_t s2 = (size_t)(e.desc.grid_res / e.desc.occ_res) + 2;
        const size_t bytes = (size_t)nb * s2 * s2 * s2 * 8;
        if (bytes >= (1ull << 31)) return fail(c, COW_E_INVALID, "brick atlas of one block exceeds 2 GiB");
        d.brick_bytes = (uint32_t)bytes;
        off += align_up(bytes);
    }
    HIP_TRY(c, hipMemcpy(c->d_blocks, c->h_blocks.data(), sizeof(DevBlock) * c->h_blocks.size(),
                         hipMemcpyHostToDevice));
    for (size_t i = 0; i < c->entries.size(); ++i)
        if (c->entries[i].desc.dtype == COW_U8)
            HIP_TRY(c, cow::launch_pack_bricks(c->d_blocks, (int)i, (int)occ_cells(c->entries[i].desc), 0, nullptr, stream));
    c->bricks_packed = true;
    return COW_OK;
}

// noalloc: the tables live in this device's scratch array instead of ws
// (cow_render_noalloc), which bounds the views and set entries of a call,
// needs the caller's aux and rules out graph replay (instantiating a graph
// allocates)
static cow_status render_impl(cow_ctx* c, const cow_view* views, int n_views, const cow_block_set* sets,
                              const cow_render_params* p, const float* mlp, float* rgb, float* trans,
                              float* aux, void* ws, size_t ws_bytes, hipStream_t s, bool noalloc = false) {
    if (!c) return COW_E_INVALID;
    if (!c->loaded) return fail(c, COW_E_NOT_LOADED, "no blocks loaded");
    if (!views || !sets || n_views < 1 || n_views > kMaxViews) return fail(c, COW_E_INVALID, "bad views");
    cow_status st = validate_params(c, p);
    if (st != COW_OK) return st;
    if ((!mlp && !p->block_mlp) || !rgb || !trans) return fail(c, COW_E_INVALID, "null mlp or output");
    if (noalloc) {
        if (!aux) return fail(c, COW_E_INVALID, "cow_render_noalloc needs the aux output");
        if (n_views > kNoAllocMaxViews)
            return fail(c, COW_E_INVALID, "cow_render_noalloc: more than 256 views in one call");
        int64_t refs = 0;
        for (int v = 0; v < n_views; ++v) refs += sets[v].n > 0 ? sets[v].n : 0;
        if (refs > kNoAllocMaxRefs)
            return fail(c, COW_E_INVALID, "cow_render_noalloc: more than 16384 set entries in one call");
        if (p->flags & COW_F_GRAPH)
            return fail(c, COW_E_UNSUPPORTED, "cow_render_noalloc does not replay graphs (instantiation allocates)");
        ws = c->scratch;
        ws_bytes = kScratchBytes;
    }
    if ((p->flags & COW_F_SPARSE) && !c->bricks_packed) return fail(c, COW_E_INVALID, "bricks not packed");
    CallTables T;
    st = build_tables(c, views, n_views, sets, c->cfg.tile_w, &T);
    if (st != COW_OK) return st;
    st = check_block_aux(c, T, p);
    if (st != COW_OK) return st;
    int dtype;
    st = check_dtypes(c, T, &dtype);
    if (st != COW_OK) return st;
    if (p->block_aux && dtype != COW_F32)
        return fail(c, COW_E_UNSUPPORTED, "block_aux is the backward's input: float32 blocks only");
    if ((p->flags & COW_F_SPARSE) && dtype != COW_U8) return fail(c, COW_E_UNSUPPORTED, "sparse bricks hold uint8 grids only");
    if (any_contracted(c, T.refs) && (p->mode != COW_MODE_GRID || p->block_mlp || p->opacity || (p->flags & COW_F_PER_BLOCK)))
        return fail(c, COW_E_UNSUPPORTED, "contracted blocks render in grid mode with one MLP after the merge, "
                                          "without opacity output or per-block launches");
    RenderWs w;
    const size_t need = render_ws_layout(n_views, (int64_t)T.refs.size(), T.n_pix, aux == nullptr, false,
                                         (int64_t)c->entries.size(), 0, (unsigned char*)ws, &w);
    if (!ws || ws_bytes < need) return fail(c, COW_E_WORKSPACE, "render workspace too small");
    if (T.n_pix == 0) return COW_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    st = upload_tables(c, T, w, s, !noalloc);
    if (st != COW_OK) return st;
    float* aux_out = aux ? aux : w.aux;
    cow::MarchArgs a = march_args(c, T, w, p, dtype, aux_out, trans);
    a.rgb = rgb;
    cow::MlpArgs m{};
    m.views = w.views;
    m.n_views = n_views;
    m.n_pix = T.n_pix;
    m.mlp = mlp;
    m.aux = aux_out;
    m.rgb = rgb;
    m.trans = trans;
    m.pe = p->pe_freqs;
    const bool per_block = (p->flags & COW_F_PER_BLOCK) != 0;
    if (!per_block) a.persistent = a.persistent || (p->flags & COW_F_PERSISTENT) ? 1 : 0;
    c->have_fwd = c->timing && !(p->flags & COW_F_GRAPH) && !per_block;
    if (p->flags & COW_F_GRAPH) return run_graph(c, T, a, m, per_block, s);
    return enqueue_forward(c, T, a, m, per_block, s);
}

cow_status cow_render(cow_ctx* c, const cow_view* views, int n_views, const cow_block_set* sets,
                      const cow_render_params* p, const float* mlp, float* rgb, float* trans, float* aux,
                      void* ws, size_t ws_bytes, hipStream_t s) {
    try {
        return render_impl(c, views, n_views, sets, p, mlp, rgb, trans, aux, ws, ws_bytes, s);
    } catch (...) {
        return fail(c, COW_E_INTERNAL, "internal error");
    }
}

cow_status cow_render_noalloc(cow_ctx* c, const cow_view* views, int n_views, const cow_block_set* sets,
                              const cow_render_params* p, const float* mlp, float* rgb, float* trans, float* aux,
                              hipStream_t s) {
    try {
        return render_impl(c, views, n_views, sets, p, mlp, rgb, trans, aux, nullptr, 0, s, true);
    } catch (...) {
        return fail(c, COW_E_INTERNAL, "internal error");
    }
}

cow_status cow_render_backward(cow_ctx* c, const cow_view* views, int n_views, const cow_block_set* sets,
                               const cow_render_params* p, const float* mlp, const float* aux,
                               const float* grad_rgb, const float* grad_trans, float* const* grad_grid,
                               float* const* grad_plane, float* grad_mlp, void* ws, size_t ws_bytes,
                               hipStream_t s) try {
    if (!c) return COW_E_INVALID;
    if (!c->loaded) return fail(c, COW_E_NOT_LOADED, "no blocks loaded");
    if (!views || !sets || n_views < 1 || n_views > kMaxViews) return fail(c, COW_E_INVALID, "bad views");
    cow_status st = validate_params(c, p);
    if (st != COW_OK) return st;
    if ((!mlp && !p->block_mlp) || !aux || !grad_rgb || !grad_grid || !grad_plane)
        return fail(c, COW_E_INVALID, "null mlp, aux, grad_rgb or gradient table");
    CallTables T;
    st = build_tables(c, views, n_views, sets, c->cfg.tile_w, &T);
    if (st != COW_OK) return st;
    st = check_block_aux(c, T, p);
    if (st != COW_OK) return st;
    for (int32_t e : T.refs)
        if (c->entries[e].desc.dtype != COW_F32)
            return fail(c, COW_E_UNSUPPORTED, "backward needs float32 textures");
    if (any_contracted(c, T.refs) && (p->mode != COW_MODE_GRID || p->block_mlp || p->opacity_weight))
        return fail(c, COW_E_UNSUPPORTED, "the adjoint of contracted blocks runs in grid mode with one MLP after "
                                          "the merge and no opacity term");
    RenderWs w;
    std::vector<cow_block_desc> descs;
    for (const Entry& en : c->entries) descs.push_back(en.desc);
    const size_t need = render_ws_layout(n_views, (int64_t)T.refs.size(), T.n_pix, false, true,
                                         (int64_t)c->entries.size(), slots_total(descs.data(), (int64_t)descs.size()),
                                         (unsigned char*)ws, &w);
    if (!ws || ws_bytes < need) return fail(c, COW_E_WORKSPACE, "backward workspace too small");
    if ((uintptr_t)ws % 16) return fail(c, COW_E_INVALID, "the backward workspace must be 16-byte aligned");
    const size_t ne = c->entries.size();
    for (size_t e = 0; e < ne; ++e) {
        if ((uintptr_t)grad_grid[e] % 16) return fail(c, COW_E_INVALID, "gradient buffers must be 16-byte aligned");
        for (int k = 0; k < 3; ++k)
            if ((uintptr_t)grad_plane[3 * e + k] % 16)
                return fail(c, COW_E_INVALID, "gradient buffers must be 16-byte aligned");
    }
    if (T.n_pix == 0) return COW_OK;
    HIP_TRY(c, hipSetDevice(c->device));
    // views, refs, the per-entry gradient and pair-slot pointer tables and the
    // fold jobs (the textures of the entries this call renders) in one upload
    std::vector<float*> ptrs(8 * ne, nullptr);
    std::vector<char> used(ne, 0);
    for (int32_t e : T.refs) used[e] = 1;
    std::vector<cow::FoldJob> jobs;
    int64_t max_texels = 0;
    size_t sl_off = 0;
    for (size_t e = 0; e < ne; ++e) {
        ptrs[e] = grad_grid[e];
        for (int k = 0; k < 3; ++k) ptrs[ne + 3 * e + k] = grad_plane[3 * e + k];
        if (descs[e].dtype != COW_F32) continue;
        for (int t = 0; t < 4; ++t) {
            const int64_t n = (int64_t)(t == 0 ? grid_texels(descs[e]) : plane_texels(descs[e], t - 1));
            float* g = t == 0 ? grad_grid[e] : grad_plane[3 * e + t - 1];
            float* sl = (float*)(w.slots + sl_off);
            sl_off += slot_bytes(n);
            if (!g || !used[e]) continue;
            ptrs[4 * ne + 4 * e + t] = sl;
            jobs.push_back(cow::FoldJob{g, sl, n});
            max_texels = std::max(max_texels, n);
        }
    }
    const size_t vb = sizeof(DevView) * T.views.size(), rb = 4 * T.refs.size(), pb = sizeof(float*) * ptrs.size();
    const size_t jb = sizeof(cow::FoldJob) * jobs.size();
    const size_t o_ref = align_up(vb), o_ptr = o_ref + align_up(rb), o_job = o_ptr + align_up(pb);
    Staging* sl = nullptr;
    st = take_staging(c, o_job + jb, &sl);
    if (st != COW_OK) return st;
    memcpy(sl->buf, T.views.data(), vb);
    memcpy(sl->buf + o_ref, T.refs.data(), rb);
    memcpy(sl->buf + o_ptr, ptrs.data(), pb);
    if (jb) memcpy(sl->buf + o_job, jobs.data(), jb);
    HIP_TRY(c, hipMemcpyAsync(w.views, sl->buf, vb, hipMemcpyHostToDevice, s));
    if (rb) HIP_TRY(c, hipMemcpyAsync(w.refs, sl->buf + o_ref, rb, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(w.grad_ptrs, sl->buf + o_ptr, pb, hipMemcpyHostToDevice, s));
    if (jb) HIP_TRY(c, hipMemcpyAsync(w.jobs, sl->buf + o_job, jb, hipMemcpyHostToDevice, s));
    st = release_staging(c, sl, s);
    if (st != COW_OK) return st;
    HIP_TRY(c, cow::launch_slots_zero(w.jobs, (int)jobs.size(), max_texels, s));
    cow::MlpBwdArgs mb{};
    mb.views = w.views;
    mb.n_views = n_views;
    mb.n_pix = T.n_pix;
    mb.mlp = mlp;
    mb.aux = aux;
    mb.grad_rgb = grad_rgb;
    mb.u = w.u;
    mb.grad_mlp = grad_mlp ? grad_mlp : w.grad_mlp_scratch;
    mb.pe = p->pe_freqs;
    if (!p->block_mlp) HIP_TRY(c, cow::launch_mlp_bwd(mb, s));  // per-block MLPs: adjoint inside the march
    cow::BwdArgs ba{};
    ba.m = march_args(c, T, w, p, COW_F32, const_cast<float*>(aux), nullptr);
    ba.m.counts = nullptr;
    ba.m.opacity = nullptr;
    ba.u = w.u;
    ba.grad_trans = grad_trans;
    ba.w_opacity = p->opacity_weight;
    ba.grad_rgb = grad_rgb;
    ba.grad_block_mlp = p->grad_block_mlp;
    ba.grad_grid = w.grad_ptrs;
    ba.grad_plane = w.grad_ptrs + ne;
    ba.slots = w.grad_ptrs + 4 * ne;
    c->have_bwd = c->timing;
    if (ba.m.persistent) HIP_TRY(c, cow::launch_reset_counter(ba.m.work_counter, s));
    if (c->timing) HIP_TRY(c, hipEventRecord(c->ev[2], s));
    HIP_TRY(c, cow::launch_march_bwd(ba, c->cfg.waves, s));
    if (c->timing) HIP_TRY(c, hipEventRecord(c->ev[3], s));
    HIP_TRY(c, cow::launch_slots_fold(w.jobs, (int)jobs.size(), max_texels, s));
    return COW_OK;
} catch (...) {
    return fail(c, COW_E_INTERNAL, "internal error");
}

cow_status cow_sparsity(cow_ctx* c, const cow_block_set* set, const float* pts, int64_t n, float delta,
                        float weight, float* alpha, float* loss, float* const* grad_grid,
                        float* const* grad_plane, void* ws, size_t ws_bytes, hipStream_t s) try {
    if (!c) return COW_E_INVALID;
    if (!c->loaded) return fail(c, COW_E_NOT_LOADED, "no blocks loaded");
    if (!set || set->n < 0 || (set->n > 0 && !set->refs)) return fail(c, COW_E_INVALID, "bad block set");
    if (n < 0 || (n > 0 && !pts) || !loss) return fail(c, COW_E_INVALID, "null points or loss");
    if (n > (int64_t)1 << 31) return fail(c, COW_E_INVALID, "too many points");
    if (!(delta > 0.0f) || !std::isfinite(delta)) return fail(c, COW_E_INVALID, "delta must be positive and finite");
    if (!std::isfinite(weight)) return fail(c, COW_E_INVALID, "weight must be finite");
    if ((grad_grid == nullptr) != (grad_plane == nullptr))
        return fail(c, COW_E_INVALID, "gradient tables must be both given or both NULL");
    std::vector<int32_t> idx((size_t)set->n);
    int dtype = -1;
    for (int r = 0; r < set->n; ++r) {
        const int e = find_entry(c, set->refs[r].block_id, set->refs[r].lod);
        if (e < 0) return fail(c, COW_E_INVALID, "set names a (block, lod) that is not loaded");
        idx[r] = e;
        const int d = c->entries[e].desc.dtype;
        if (dtype >= 0 && d != dtype) return fail(c, COW_E_UNSUPPORTED, "one call must use blocks of a single dtype");
        dtype = d;
    }
    if (grad_grid && dtype == COW_U8) return fail(c, COW_E_UNSUPPORTED, "gradients need float32 textures");
    const size_t ne = c->entries.size();
    const size_t ib = align_up(4 * (size_t)std::max(set->n, 1)), pb = sizeof(float*) * 4 * ne;
    if (!ws || ws_bytes < ib + pb) return fail(c, COW_E_WORKSPACE, "sparsity workspace too small");
    if (n == 0 || set->n == 0) {
        if (n > 0 && alpha) HIP_TRY(c, hipMemsetAsync(alpha, 0, sizeof(float) * (size_t)n, s));
        return COW_OK;
    }
    HIP_TRY(c, hipSetDevice(c->device));
    std::vector<float*> ptrs(4 * ne, nullptr);
    if (grad_grid)
        for (size_t e = 0; e < ne; ++e) {
            ptrs[e] = grad_grid[e];
            for (int k = 0; k < 3; ++k) ptrs[ne + 3 * e + k] = grad_plane[3 * e + k];
        }
    Staging* sl = nullptr;
    cow_status st = take_staging(c, ib + pb, &sl);
    if (st != COW_OK) return st;
    memcpy(sl->buf, idx.data(), 4 * idx.size());
    memcpy(sl->buf + ib, ptrs.data(), pb);
    unsigned char* d = (unsigned char*)ws;
    HIP_TRY(c, hipMemcpyAsync(d, sl->buf, ib + pb, hipMemcpyHostToDevice, s));
    st = release_staging(c, sl, s);
    if (st != COW_OK) return st;
    cow::SparsityArgs a{};
    a.blocks = c->d_blocks;
    a.set = (const int32_t*)d;
    a.n_set = set->n;
    a.dtype = dtype;
    a.pts = pts;
    a.n = n;
    a.delta = delta;
    a.scale = (float)((double)weight / (double)n);
    a.alpha = alpha;
    a.loss = loss;
    a.grad_grid = grad_grid ? (float* const*)(d + ib) : nullptr;
    a.grad_plane = grad_grid ? (float* const*)(d + ib) + ne : nullptr;
    HIP_TRY(c, cow::launch_sparsity(a, s));
    return COW_OK;
} catch (...) {
    return fail(c, COW_E_INTERNAL, "internal error");
}

cow_status cow_get_config(cow_ctx* c, int* tile_w, int* waves, int* persistent) {
    if (!c) return COW_E_INVALID;
    if (tile_w) *tile_w = c->cfg.tile_w;
    if (waves) *waves = c->cfg.waves;
    if (persistent) *persistent = c->cfg.persistent;
    return COW_OK;
}

cow_status cow_set_config(cow_ctx* c, int tile_w, int waves, int persistent) {
    if (!c) return COW_E_INVALID;
    if (!(tile_w == 1 || tile_w == 2 || tile_w == 4 || tile_w == 8 || tile_w == 16 || tile_w == 32 || tile_w == 64))
        return fail(c, COW_E_INVALID, "tile width must be a power of two dividing 64");
    if (!(waves == 1 || waves == 2 || waves == 4)) return fail(c, COW_E_INVALID, "waves per workgroup: 1, 2 or 4");
    c->cfg.tile_w = tile_w;
    c->cfg.waves = waves;
    c->cfg.persistent = persistent < 0 ? -1 : persistent ? 1 : 0;
    drop_graphs(c);
    return COW_OK;
}

cow_status cow_set_timing(cow_ctx* c, int enable) {
    if (!c) return COW_E_INVALID;
    HIP_TRY(c, hipSetDevice(c->device));
    if (enable)
        for (auto& e : c->ev)
            if (!e) HIP_TRY(c, hipEventCreate(&e));
    c->timing = enable != 0;
    c->have_fwd = c->have_bwd = false;
    return COW_OK;
}

cow_status cow_last_timing(cow_ctx* c, float* fwd_ms, float* bwd_ms) {
    if (!c) return COW_E_INVALID;
    if (fwd_ms) {
        *fwd_ms = -1.0f;
        if (c->have_fwd) {
            HIP_TRY(c, hipEventSynchronize(c->ev[1]));
            HIP_TRY(c, hipEventElapsedTime(fwd_ms, c->ev[0], c->ev[1]));
        }
    }
    if (bwd_ms) {
        *bwd_ms = -1.0f;
        if (c->have_bwd) {
            HIP_TRY(c, hipEventSynchronize(c->ev[3]));
            HIP_TRY(c, hipEventElapsedTime(bwd_ms, c->ev[2], c->ev[3]));
        }
    }
    return COW_OK;
}

cow_status cow_autotune(cow_ctx* c, const cow_view* views, int n_views, const cow_block_set* sets,
                        const cow_render_params* p, const float* mlp, void* ws, size_t ws_bytes,
                        const char* cache_path, hipStream_t s) try {
    if (!c) return COW_E_INVALID;
    if (!c->loaded) return fail(c, COW_E_NOT_LOADED, "no blocks loaded");
    cow_status st = validate_params(c, p);
    if (st != COW_OK) return st;
    if (!views || !sets || n_views < 1) return fail(c, COW_E_INVALID, "bad views");
    int64_t n_pix = 0, n_refs = 0;
    for (int v = 0; v < n_views; ++v) {
        n_pix += (int64_t)views[v].crop_w * views[v].crop_h;
        n_refs += sets[v].n;
    }
    // cache key: device, workload shape, and the digest of the library's
    // sources (a rebuilt kernel may prefer another configuration)
    char key[256];
    snprintf(key, sizeof key, "%s|cu%d|v%d|p%lld|r%lld|m%d|s%d|f%d|dt%d|src%s", c->arch.c_str(), c->n_cus, n_views,
             (long long)n_pix, (long long)n_refs, p->mode, p->max_steps, p->flags & COW_F_SPARSE, c->dtype,
             COW_SOURCE_DIGEST);
    // cache: one JSON object per line
    if (cache_path) {
        FILE* f = fopen(cache_path, "r");
        if (f) {
            char line[512];
            while (fgets(line, sizeof line, f)) {
                char k[256];
                int tw, wv, ps;
                if (sscanf(line, " {\"key\": \"%255[^\"]\", \"tile_w\": %d, \"waves\": %d, \"persistent\": %d}", k,
                           &tw, &wv, &ps) == 4 &&
                    strcmp(k, key) == 0) {
                    fclose(f);
                    return cow_set_config(c, tw, wv, ps);
                }
            }
            fclose(f);
        }
    }
    // outputs live in the tail of the workspace beyond what render needs
    const int64_t need_render = (int64_t)render_ws_layout(n_views, n_refs, n_pix, true, false,
                                                          (int64_t)c->entries.size(), 0, nullptr, nullptr);
    const int64_t need = need_render + (int64_t)align_up(16 * n_pix) + 256;
    if (!ws || (int64_t)ws_bytes < need) return fail(c, COW_E_WORKSPACE, "autotune needs render workspace + 16 B per pixel");
    float* rgb = (float*)((unsigned char*)ws + need_render);
    float* trans = rgb + 3 * n_pix;
    const TuneCfg saved = c->cfg;
    const bool saved_timing = c->timing;
    // events and the context's configuration are restored on every exit
    struct Guard {
        cow_ctx* c;
        TuneCfg cfg;
        bool timing;
        hipEvent_t e[2] = {nullptr, nullptr};
        ~Guard() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
            c->timing = timing;
        }
    } guard{c, saved, saved_timing};
    HIP_TRY(c, hipEventCreate(&guard.e[0]));
    HIP_TRY(c, hipEventCreate(&guard.e[1]));
    cow_render_params q = *p;
    q.flags &= COW_F_SPARSE;
    q.counts = nullptr;
    // one warm-up render and three timed ones in configuration t; any failure
    // ends the sweep with that status and the previous configuration restored
    auto trial = [&](const TuneCfg& t, float* ms, int reps) -> cow_status {
        c->cfg = t;
        c->timing = false;
        cow_status r = render_impl(c, views, n_views, sets, &q, mlp, rgb, trans, nullptr, ws, ws_bytes, s);
        if (r != COW_OK) return r;
        HIP_TRY(c, hipEventRecord(guard.e[0], s));
        for (int it = 0; it < reps; ++it) {
            r = render_impl(c, views, n_views, sets, &q, mlp, rgb, trans, nullptr, ws, ws_bytes, s);
            if (r != COW_OK) return r;
        }
        HIP_TRY(c, hipEventRecord(guard.e[1], s));
        HIP_TRY(c, hipEventSynchronize(guard.e[1]));
        HIP_TRY(c, hipEventElapsedTime(ms, guard.e[0], guard.e[1]));
        return COW_OK;
    };
    float best = INFINITY;
    TuneCfg best_cfg = saved;
    const int tws[] = {8, 16, 4, 32};
    const int wvs[] = {4, 2, 1};
    for (int persistent = 0; persistent < 2; ++persistent)
        for (int tw : tws)
            for (int wv : wvs) {
                const TuneCfg t{tw, wv, persistent};
                float ms = 0.0f;
                st = trial(t, &ms, 3);
                if (st != COW_OK) {
                    c->cfg = saved;
                    drop_graphs(c);
                    return st;
                }
                if (ms < best) {
                    best = ms;
                    best_cfg = t;
                }
            }
    // a short trial is noisy: the pick replaces the configuration the call
    // found only if longer runs of both, interleaved, show it 1% faster
    const bool same = best_cfg.tile_w == saved.tile_w && best_cfg.waves == saved.waves &&
                      best_cfg.persistent == saved.persistent;
    if (!same) {
        float t_best = 0.0f, t_saved = 0.0f;
        for (int round = 0; round < 2; ++round) {
            float a = 0.0f, b = 0.0f;
            st = trial(best_cfg, &a, 8);
            if (st == COW_OK) st = trial(saved, &b, 8);
            if (st != COW_OK) {
                c->cfg = saved;
                drop_graphs(c);
                return st;
            }
            t_best += a;
            t_saved += b;
        }
        if (!(t_best < 0.99f * t_saved)) best_cfg = saved;
    }
    c->cfg = best_cfg;
    drop_graphs(c);
    if (cache_path) {
        FILE* f = fopen(cache_path, "a");
        if (f) {
            fprintf(f, "{\"key\": \"%s\", \"tile_w\": %d, \"waves\": %d, \"persistent\": %d}\n", key,
                    best_cfg.tile_w, best_cfg.waves, best_cfg.persistent);
            fclose(f);
        }
    }
    return COW_OK;
} catch (...) {
    return fail(c, COW_E_INTERNAL, "internal error");
}

}  // extern "C"
