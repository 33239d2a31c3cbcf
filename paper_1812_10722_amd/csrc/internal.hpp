// Internal declarations of the LSPR library: error handling, device buffers, the geometry
// handle and the launchers each translation unit provides.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "lspr.h"

namespace lspr {

struct Error : std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define LSPR_HIP(call)                                                                      \
    do {                                                                                    \
        hipError_t err_ = (call);                                                           \
        if (err_ != hipSuccess)                                                             \
            throw ::lspr::Error(err_ == hipErrorOutOfMemory ? LSPR_E_NOMEM : LSPR_E_DEVICE, \
                                std::string(#call) + ": " + hipGetErrorString(err_));       \
    } while (0)

#define LSPR_REQUIRE(cond, code, msg)                                  \
    do {                                                               \
        if (!(cond)) throw ::lspr::Error((code), std::string(msg));    \
    } while (0)

// Allocation context of the calling thread.  Without a pool DevBuf allocates with hipMalloc and
// frees with hipFree.  A thread that installs a memory pool allocates stream-ordered from it on
// `stream` and frees stream-ordered on the same stream, so that requests sharing the device do
// not synchronise the whole device on every free (the request server does this per worker; the
// C entry points install the library's own pool for their call, see PoolScope).  While
// `free_on` is set, pooled frees go to `free_stream` instead (a stream valid for the call).
// live / peak count the bytes held by DevBufs allocated on this thread.
struct AllocCtx {
    hipMemPool_t pool = nullptr;
    hipStream_t stream = nullptr;
    bool free_on = false;
    hipStream_t free_stream = nullptr;
    bool keep_big = false;  // large blocks of `pool` go to the block cache when released
    int64_t live = 0, peak = 0;
};
AllocCtx& alloc_ctx();

// The library's memory pool on the current device (created on first use; keeps up to 64 GiB of
// freed memory for reuse instead of returning it at every synchronisation).
hipMemPool_t library_pool();

// Cache of large released blocks of the library pool.  Returning a pool allocation of several
// GB costs the host about 1.3 ms per GB, and obtaining it again a few tenths of a ms, so blocks
// of at least BIG_BLOCK bytes are kept (up to 128 GiB per pool, larger blocks first: both tile
// stores of a 100k-panel geometry, or the FP64 store of a 491k-panel one) and handed to the next
// request
// of a size they cover.  A kept block is reusable once an event recorded on its last stream
// has completed; the taker's stream waits for that event.
constexpr size_t BIG_BLOCK = 32ull << 20;
// A cached block of `pool` of at least `bytes` (and not much larger), ordered after its last
// use on `s`; nullptr if none.  *got receives the block's size.
void* big_block_take(hipMemPool_t pool, size_t bytes, hipStream_t s, size_t* got);
// Keeps `p` (a block of `bytes` from `pool`, last used on `s`); false if the cache is full.
bool big_block_put(hipMemPool_t pool, void* p, size_t bytes, hipStream_t s);
// Frees every cached block of `pool` (after their last uses); true if there was any.
bool big_block_flush(hipMemPool_t pool);
// Bytes `pool` holds for reuse: cached blocks and reserved memory not in use (0 for no pool).
size_t reusable_bytes(hipMemPool_t pool);

// Installs the library pool and `stream` for allocations, and `stream` for frees, for the
// lifetime of the object, unless the thread already has a pool (the request server's).
struct PoolScope {
    AllocCtx saved;
    bool active = false;
    explicit PoolScope(hipStream_t stream) {
        AllocCtx& c = alloc_ctx();
        if (c.pool != nullptr) return;
        saved = c;
        c.pool = library_pool();
        c.stream = stream;
        c.free_on = true;
        c.free_stream = stream;
        c.keep_big = true;
        active = true;
    }
    ~PoolScope() {
        if (!active) return;
        AllocCtx& c = alloc_ctx();
        const int64_t live = c.live, peak = c.peak;
        c = saved;
        c.live = live;
        c.peak = peak;
    }
    PoolScope(const PoolScope&) = delete;
    PoolScope& operator=(const PoolScope&) = delete;
};

// Owning device allocation.  Moves, never copies.
template <class T>
struct DevBuf {
    T* p = nullptr;
    size_t n = 0;
    hipStream_t free_stream = nullptr;
    bool pooled = false;
    hipMemPool_t keep_pool = nullptr;  // set: the block goes back to the block cache
    size_t block = 0;                  // bytes of the underlying block
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    DevBuf(DevBuf&& o) noexcept { take(o); }
    DevBuf& operator=(DevBuf&& o) noexcept {
        if (this != &o) { release(); take(o); }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        AllocCtx& c = alloc_ctx();
        const size_t b = count * sizeof(T);
        if (c.pool) {
            block = b;
            void* q = nullptr;
            if (c.keep_big && b >= BIG_BLOCK) {
                keep_pool = c.pool;
                q = big_block_take(c.pool, b, c.stream, &block);
            }
            if (q == nullptr) {
                hipError_t e = hipMallocFromPoolAsync(&q, b, c.pool, c.stream);
                if (e == hipErrorOutOfMemory && c.keep_big) {
                    (void)hipGetLastError();  // clear the recorded failure before retrying
                    if (big_block_flush(c.pool))
                        e = hipMallocFromPoolAsync(&q, b, c.pool, c.stream);
                }
                LSPR_HIP(e);
                block = b;
            }
            p = static_cast<T*>(q);
            free_stream = c.stream;
            pooled = true;
        } else {
            LSPR_HIP(hipMalloc(reinterpret_cast<void**>(&p), b));
            pooled = false;
        }
        n = count;
        c.live += static_cast<int64_t>(b);
        if (c.live > c.peak) c.peak = c.live;
    }
    // grow-only reallocation for workspaces
    void reserve(size_t count) { if (count > n) alloc(count); }
    void release() {
        if (p) {
            if (pooled) {
                const AllocCtx& c = alloc_ctx();
                hipStream_t fs = c.free_on ? c.free_stream : free_stream;
                if (keep_pool == nullptr || !big_block_put(keep_pool, p, block, fs))
                    (void)hipFreeAsync(p, fs);
            }
            else (void)hipFree(p);
            alloc_ctx().live -= static_cast<int64_t>(bytes());
        }
        p = nullptr;
        n = 0;
        pooled = false;
        keep_pool = nullptr;
        block = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
    T* get() const { return p; }

  private:
    void take(DevBuf& o) {
        p = o.p; n = o.n; free_stream = o.free_stream; pooled = o.pooled;
        keep_pool = o.keep_pool; block = o.block;
        o.p = nullptr; o.n = 0; o.pooled = false; o.keep_pool = nullptr; o.block = 0;
    }
};

// Stream-ordered copy that returns when it has completed (host buffers may be temporaries).
inline void copy_sync(void* dst, const void* src, size_t bytes, hipMemcpyKind kind,
                      hipStream_t s) {
    if (bytes == 0) return;
    LSPR_HIP(hipMemcpyAsync(dst, src, bytes, kind, s));
    LSPR_HIP(hipStreamSynchronize(s));
}

// Pinned (page-locked) host staging buffers, shared by all threads and reused: a transfer from
// or to pinned memory is one DMA, where pageable memory goes through the runtime's own staging
// at a few GB/s.  A buffer is put back only once no transfer uses it.
struct PinnedBuf {
    uint8_t* p = nullptr;
    size_t cap = 0;
};
// A free buffer of at least `bytes` (a new one, a multiple of 1 MiB, if none is free).
PinnedBuf pinned_take(size_t bytes);
void pinned_put(PinnedBuf b);

// Batched host-to-device uploads of set-up code.  add() copies host data into one pinned
// buffer (so temporaries may be passed); flush() moves the buffer to the device in one
// transfer and queues a device-to-device copy to each destination on `s`, so the host waits
// once rather than once per destination.  The device staging block is kept until the next
// flush or the object's end, both of which first wait for `s`.
class Uploads {
  public:
    explicit Uploads(hipStream_t s) : s_(s) {}
    ~Uploads() {
        if (stage_.p) (void)hipStreamSynchronize(s_);
        if (buf_.p) pinned_put(buf_);
    }
    Uploads(const Uploads&) = delete;
    Uploads& operator=(const Uploads&) = delete;
    template <class T>
    void add(T* dst, const T* src, size_t count) {
        const size_t bytes = count * sizeof(T);
        if (bytes == 0) return;
        const size_t at = (used_ + 255) & ~static_cast<size_t>(255);
        reserve(at + bytes);
        std::memcpy(buf_.p + at, src, bytes);
        items_.push_back({dst, at, bytes});
        used_ = at + bytes;
    }
    void flush() {
        if (items_.empty()) return;
        if (stage_.p) {
            LSPR_HIP(hipStreamSynchronize(s_));
            stage_.release();
        }
        stage_.alloc(used_);
        copy_sync(stage_.p, buf_.p, used_, hipMemcpyHostToDevice, s_);  // buf_ free again
        for (const Item& it : items_)
            LSPR_HIP(hipMemcpyAsync(it.dst, stage_.p + it.at, it.bytes, hipMemcpyDeviceToDevice,
                                    s_));
        items_.clear();
        used_ = 0;
    }

  private:
    struct Item {
        void* dst;
        size_t at, bytes;
    };
    void reserve(size_t n) {
        if (n <= buf_.cap) return;
        const PinnedBuf nb = pinned_take(n > 2 * buf_.cap ? n : 2 * buf_.cap);
        if (used_) std::memcpy(nb.p, buf_.p, used_);
        if (buf_.p) pinned_put(buf_);
        buf_ = nb;
    }
    hipStream_t s_;
    PinnedBuf buf_;
    size_t used_ = 0;
    std::vector<Item> items_;
    DevBuf<uint8_t> stage_;
};

// Batched device-to-host downloads: add() records a destination; fetch() gathers the sources
// into one device block (device-to-device copies queued on `s`), reads it back in one transfer
// into a pinned buffer and fills every destination.  The sources must be ready in the stream
// order of `s`.
class Downloads {
  public:
    explicit Downloads(hipStream_t s) : s_(s) {}
    template <class T>
    void add(T* dst, const T* src, size_t count) {
        const size_t bytes = count * sizeof(T);
        if (bytes == 0) return;
        const size_t at = (total_ + 255) & ~static_cast<size_t>(255);
        items_.push_back({dst, src, at, bytes});
        total_ = at + bytes;
    }
    void fetch() {
        if (items_.empty()) return;
        DevBuf<uint8_t> stage(total_);
        for (const Item& it : items_)
            LSPR_HIP(hipMemcpyAsync(stage.p + it.at, it.src, it.bytes, hipMemcpyDeviceToDevice,
                                    s_));
        const PinnedBuf host = pinned_take(total_);
        try {
            copy_sync(host.p, stage.p, total_, hipMemcpyDeviceToHost, s_);
        } catch (...) {
            (void)hipStreamSynchronize(s_);  // no transfer into the buffer once it is put back
            pinned_put(host);
            throw;
        }
        for (const Item& it : items_) std::memcpy(it.dst, host.p + it.at, it.bytes);
        pinned_put(host);
        items_.clear();
        total_ = 0;
    }

  private:
    struct Item {
        void* dst;
        const void* src;
        size_t at, bytes;
    };
    hipStream_t s_;
    std::vector<Item> items_;
    size_t total_ = 0;
};

// Octree box, one per node of every surface's tree.  Boxes of one surface are stored level by
// level; the children of a box are contiguous.
struct Box {
    double cx, cy, cz;  // expansion centre: centre of the bounding box of the box's nodes
    double rb;          // max |node - centre| over its quadrature nodes (MAC radius)
    double rv;          // max |vertex - centre| over its panels (near-singular guard radius)
    double lmax;        // max representative length L = sqrt(2 A) of its panels
    int32_t start, end; // panel range [start, end) in sorted order
    int32_t child, nchild;
    int32_t level, surf;
    int32_t next;       // the box after this one's subtree in depth-first order (-1: none)
};

// Group of consecutive targets (panel centroids of one surface, sorted order) that share
// interaction lists.
struct Chunk {
    double cx, cy, cz;  // centre of the bounding box of its centroids
    double r;           // max |centroid - centre|
    int32_t start, end;
    int32_t surf, pad;
};

// A P2M work item: panels [start, end) of expanded box `box`, whose moments are row block
// `mslot` of the moment array (expanded boxes only, in box order); slot < 0 writes the box's
// moments directly, otherwise partial moments go to scratch slot `slot`.
struct P2MSeg {
    int32_t box, start, end, slot, mslot;
};
// Boxes assembled from several segments: moments = sum of scratch slots [slot0, slot1).
struct P2MRed {
    int32_t box, slot0, slot1, mslot;
};

// One left factor of the matrix-core far-field product, stored in MFMA operand order.
// kind 0: expansion (Taylor coefficients; B rows = moments rows b_row0 .. b_row0 + b_rows);
// kind 1: direct tile (double-layer then single-layer kernel values; B rows = density rows of
// panels b_row0 .. b_row0 + b_rows).  nstep K-steps of 4 rows; the left factor starts at
// element 256 a_blk of the tile store (every tile is a multiple of 256 elements).  16 bytes, so
// a kernel fetches a descriptor with one 128-bit load.
struct TileDesc {
    int16_t kind, nstep;
    int32_t a_blk;
    int32_t b_row0, b_rows;
    __host__ __device__ int64_t a_off() const { return static_cast<int64_t>(a_blk) * 256; }
};
static_assert(sizeof(TileDesc) == 16, "tile descriptors are fetched as one 128-bit load");

// A work item of the one-operator matrix-core far-field kernel: tiles [t0, t1) of a chunk.
// slot < 0: the whole chunk, whose sums the kernel writes itself; slot >= 0: a piece of a
// chunk cut into several (never across its own-surface/other-surface boundary), whose FP64
// partial sums go to scratch block `slot` for k_far_reduce.
struct FarItem {
    int32_t chunk, t0, t1, slot;
};
// A chunk cut into pieces: its partial sums are scratch blocks [slot0, slot1), the first
// `nself` of them over own-surface tiles; they are added in block order.
struct FarRed {
    int32_t chunk, slot0, slot1, nself;
};

// One entry of a chunk's direct-sum list: source panels [start, end) of one surface.
struct Range {
    int32_t start, end;
};

struct Geometry {
    // parameters
    int S = 0, N = 0;
    int K = 4, Kf = 19, Nk = 9;
    double threshold = 0.5;
    int method = LSPR_TREECODE, P = 6, ncrit = 16, precision = LSPR_FP32;
    double theta = 0.5;
    int tchunk = 64;
    int n_terms = 0;   // expansion terms per column (Taylor terms kept after folding)
    int max_depth = 0;
    std::vector<int> surf_start;  // S+1 offsets of each surface's panels in sorted order
    std::vector<int> surf_root;   // root box of each surface's tree
    double origin[3] = {0, 0, 0}; // centre of the global bounding cube
    double half = 1.0;            // half side of the global bounding cube

    // per panel, sorted order
    DevBuf<double> tri;     // [N][9] vertex coordinates
    DevBuf<double> cen;     // [N][3] centroid
    DevBuf<double> nrm;     // [N][3] unit outward normal
    DevBuf<double> area;    // [N]
    DevBuf<int32_t> surf;   // [N] surface id
    DevBuf<int32_t> perm;   // [N] sorted index -> caller's panel index
    DevBuf<int32_t> iperm;  // [N] caller's panel index -> sorted index
    DevBuf<uint64_t> morton; // [N] sorted keys: surface id << 48 | 48-bit Morton code
    // far-field source record per panel (geometry.hip, k_permute), in FP32 and/or FP64 as the
    // geometry's precision needs: (n_x, n_y, n_z, A) then (y_g - c, w_g) per far-rule node g
    DevBuf<float> src32;
    DevBuf<double> src64;
    bool need32 = true, need64 = false;  // precisions of the products this geometry runs
    int m2p_min_panels = 0;  // boxes with fewer panels are summed directly (cost criterion)
    // tree and lists
    int n_boxes = 0, n_leaves = 0;
    DevBuf<Box> boxes;
    DevBuf<double> far_rule;   // [K][4] barycentric coordinates and weight of the far rule
    std::vector<int32_t> mom_boxes;  // boxes that appear in some expansion list (ascending)
    std::vector<int32_t> mom_slot_h; // [n_boxes] index of each box in mom_boxes, -1 if absent
    int64_t mom_panels = 0;          // panels summed over those boxes
    int n_seg = 0, n_slots = 0, n_red = 0;
    // matrix-core tiles (FP32 geometries)
    int64_t n_tiles = 0;
    int64_t tile_steps = 0, max_chunk_steps = 0;  // K-steps in all, and of the busiest chunk
    int64_t tile_elems = 0;  // elements of one tile store (the left factors of one precision)
    DevBuf<TileDesc> tiles;
    DevBuf<int32_t> tile_off, tile_self;
    DevBuf<int32_t> chunk_order;  // workgroup -> chunk of the matrix-core kernel (-1: none)
    int n_order = 0;              // entries of chunk_order (a multiple of 8)
    // Work items of the one-operator far-field kernel, one set per launch class (0: up to 16
    // wavelengths, 1: 17 to 32, 2: more): chunks heavier than a share of the mean are cut into
    // pieces of about that cost, so that no workgroup holds the launch's tail alone.
    struct FarPlan {
        DevBuf<FarItem> items;
        DevBuf<int32_t> order;  // workgroup -> item (-1: none); a multiple of 8 entries
        DevBuf<FarRed> red;     // chunks cut into pieces
        int n_order = 0, n_red = 0, n_slots = 0;
        size_t bytes() const { return items.bytes() + order.bytes() + red.bytes(); }
    };
    FarPlan far_plan[3];
    // largest piece, as a fraction of the mean chunk cost, per launch class (0: no pieces), and
    // the share of each XCD run's cost, at its end, cut into pieces of a quarter of that size.
    // Measured on the 32768-panel sphere (busiest chunk 1.95 x the mean): a per-workgroup clock
    // trace showed the launches' slots full until the last items started and a tail of about
    // one item's length; cutting only the chunks above the mean and the last fifth of each
    // run's work finer is 4-8 % faster than pieces of 0.25-0.35 x the mean everywhere, with
    // fewer partial sums to add (times flat within 3 % for splits of 1-2, tails of 0.2-0.3 and
    // tail pieces of 0.15-0.25 x the mean)
    double far_split[3] = {1.0, 1.0, 1.0};
    double far_tail[3] = {0.2, 0.2, 0.2};
    DevBuf<float> tileA;      // FP32 left factors (need32)
    DevBuf<double> tileA64;   // FP64 left factors (need64), same element offsets
    DevBuf<P2MSeg> p2m_seg;
    DevBuf<float> p2mA;          // FP32 folded node polynomials per P2M segment (matrix cores)
    DevBuf<double> p2mA64;       // FP64 ones, same element offsets
    DevBuf<int64_t> p2m_aoff;    // [n_seg] offset of each segment's block in p2mA / p2mA64
    DevBuf<P2MRed> p2m_red;
    DevBuf<int32_t> mom_slot;    // [n_boxes] moment row block of each box (-1: not expanded)
    int n_chunks = 0;
    DevBuf<Chunk> chunks;
    std::vector<int> chunk_h_surf;
    DevBuf<int32_t> m2p_off;   // [n_chunks + 1]
    DevBuf<int32_t> m2p_box;   // [n_m2p]
    DevBuf<int32_t> m2p_self;  // [n_chunks] entries of the own surface come first: count
    DevBuf<int32_t> p2p_off;   // [n_chunks + 1]
    DevBuf<Range> p2p_rng;     // [n_p2p]
    DevBuf<int32_t> p2p_self;  // [n_chunks]
    int64_t n_m2p = 0, n_p2p = 0, p2p_pairs = 0, m2p_pairs = 0;
    // host copies the set-up steps hand on to each other (released once the geometry is
    // built): panel range of each box, list offsets, own-surface counts and expansion boxes
    std::vector<Range> box_rng_h, p2p_rng_h;
    std::vector<int32_t> m2p_off_h, p2p_off_h, m2p_self_h, p2p_self_h, m2p_box_h;
    std::vector<P2MSeg> p2m_seg_h;
    // near-singular corrections (CSR over targets, sorted order) and singular self terms
    DevBuf<int64_t> near_off64; // [N + 1]
    DevBuf<int32_t> near_col;  // [n_near]
    DevBuf<double> near_dv;    // [n_near] fine - coarse single-layer entry
    DevBuf<double> near_dk;    // [n_near] fine - coarse double-layer entry
    DevBuf<double> vself;      // [N] semi-analytic V_ii
    int64_t n_near = 0;
    // geometry part of the right-hand side: u[s][d][i] = sum_{j in s} V_ij (-n_j,d)
    DevBuf<double> rhs_u;      // [S][3][N]
    // workspaces reused by the operator
    DevBuf<uint8_t> ws_dens, ws_mom, ws_out, ws_part, ws_fpart;
    // While set, the operator takes those workspaces from this caller-provided region instead
    // (lspr_apply_noalloc), so a product allocates nothing.
    struct Arena {
        uint8_t* base = nullptr;
        size_t cap = 0, used = 0;
    };
    Arena* arena = nullptr;
    // point charges: charge_u[i] = sum over the charges inside panel i's surface of
    // q_k / (4 pi |c_i - r_k|) (sorted order; empty without charges); ws_inv_eps: 1 / eps_s
    // [column][surface] of the current batch, filled with the ratios
    DevBuf<double> charge_u;
    DevBuf<double2> ws_inv_eps;
    hipStream_t stream = nullptr;
    bool allow_mfma = true;  // products use matrix cores (precomputed tiles)
    bool stream_narrow = false;  // products of up to 16 wavelengths stream their operands
                                 // (k_far_stream) instead of staging them in LDS
    bool pair_ops = false;  // products of more than 16 wavelengths stage each left factor once
                            // for both operators (eight-wave workgroups)
    bool pair_narrow = false;  // the same for products of up to 16 wavelengths
    bool four_wave = false;  // products in four-wave workgroups (register staging)
    double tile_budget_bytes = 0.0;  // largest tile store kept (0: 55 % of free device memory)
    // near-singular corrections and V_ii folded into the direct tiles of that precision (the
    // matrix-core products then need no separate near-field pass)
    bool near_in_tiles32 = false, near_in_tiles64 = false;

    size_t device_bytes() const;
};

// Bytes of region `bytes` taken from an arena (256-byte aligned pieces, in call order).
inline size_t arena_piece(size_t bytes) { return (bytes + 255) & ~static_cast<size_t>(255); }
// A workspace of `bytes` for the operator: from the geometry's arena when one is set (an
// error if it is exhausted), else the grow-only buffer `own`.
inline uint8_t* workspace(Geometry& g, DevBuf<uint8_t>& own, size_t bytes) {
    if (g.arena != nullptr) {
        Geometry::Arena& a = *g.arena;
        const size_t piece = arena_piece(bytes);
        LSPR_REQUIRE(a.used + piece <= a.cap, LSPR_E_INVALID, "scratch region exhausted");
        uint8_t* p = a.base + a.used;
        a.used += piece;
        return p;
    }
    own.reserve(bytes);
    return own.p;
}

// Column layout of one block matrix-vector product.  The real operators act on 2*ncol real
// columns: ncol "K columns" (real and imaginary parts of phi) and ncol "V columns" (of
// sigma = (eps_s / eps_m) psi).  Every column count is padded to a multiple of cpt.
struct Cols {
    int ncol = 0;  // real columns per operator (2 * wavelengths)
    int cpt = 0;   // columns per thread per operator
    int pad = 0;   // ncol rounded up to cpt
    bool mfma = false;  // matrix-core far-field kernel
    int prec = LSPR_FP32;  // LSPR_FP32 or LSPR_FP64 products
};

// ---------------------------------------------------------------- quadrature (quadrature.cpp)
// Returns false when no rule with n points exists.
bool triangle_rule(int n, std::vector<double>& bary, std::vector<double>& w);
void gauss_legendre(int n, std::vector<double>& t, std::vector<double>& w);

// ---------------------------------------------------------------- geometry (geometry.hip)
void build_geometry(Geometry& g, const lspr_surface* surfaces, int n_surf);

// ---------------------------------------------------------------- tree (tree.hip)
void build_tree(Geometry& g);
void build_lists(Geometry& g);
void build_near_table(Geometry& g);

// ---------------------------------------------------------------- operator (operator.hip)
// Raw layer sums for a packed density: dens [N][2*pad] in the precision c.prec (K columns
// then V columns, sorted panel order).  out_self/out_all [N][2*pad] FP64 receive, per target,
// the K and V sums over its own surface and over all surfaces, including the near-singular
// and singular corrections, without the 1/(4 pi) factor.
void apply_raw(Geometry& g, const Cols& c, const void* dens, double* out_self, double* out_all,
               hipStream_t s);
void precompute_rhs(Geometry& g);
// Host part of the matrix-core tiles: descriptors, the tiles of each chunk, workgroup order and
// the direct tiles sorted for the near-field fold.  Reads only host copies of the lists (and
// sizes), so it may run on another host thread while the device builds the near-singular table.
struct TilePlan {
    std::vector<TileDesc> tiles;
    std::vector<int32_t> toff, tself;            // per chunk: first tile, own-surface tiles
    std::vector<int32_t> m2p_tile, m2p_chunk;    // per expansion entry: its tile and chunk
    std::vector<int32_t> p2p_tile, p2p_chunk;    // per direct tile: its tile and chunk
    std::vector<int32_t> order;                  // workgroup -> chunk
    struct Items {                               // one launch class's work items
        std::vector<FarItem> items;
        std::vector<int32_t> order;
        std::vector<FarRed> red;
        int n_slots = 0;
    } far[3];                                    // per launch class
    std::vector<int32_t> dto, dtr, dti;          // per chunk: direct tiles by first panel
    int64_t aoff = 0;                            // elements of one tile store
    int64_t tile_steps = 0, max_chunk_steps = 0;
};
// Fills P (its vectors keep their capacity).
void plan_tiles(const Geometry& g, TilePlan& P);
void plan_items(const std::vector<TileDesc>& tl, const std::vector<int32_t>& off,
                const std::vector<int32_t>& self, double split, double tail, bool cut_self,
                TilePlan::Items& W);
// Tile plans kept for reuse: a plan refilled in place keeps its host memory mapped from one
// geometry to the next, instead of fresh pages being faulted in on every set-up.
std::unique_ptr<TilePlan> take_plan();
void put_plan(std::unique_ptr<TilePlan> p);
// Scratch bytes the far-field pieces of a product of pad columns per operator write.
size_t far_part_bytes(const Geometry& g, int pad);
// Elements of one tile store, from the host lists (the size plan_tiles will find).
int64_t estimate_tile_elems(const Geometry& g);
// Geometry-only left factors of the matrix-core far-field product, in each needed precision.
void build_tiles(Geometry& g, const TilePlan& plan);

}  // namespace lspr
