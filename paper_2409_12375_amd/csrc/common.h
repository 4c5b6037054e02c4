// Internal helpers shared by the library's translation units: status
// plumbing, device buffers, and the tree / plan structures.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/xrl.h"

namespace xrl {

void set_error(const char *fmt, ...);

// Exception used internally; converted to a status at the ABI boundary.
struct Error {
    xrl_status code;
    std::string msg;
};

[[noreturn]] void fail(xrl_status code, const char *fmt, ...);

#define XRL_HIP(call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            ::xrl::fail(e_ == hipErrorOutOfMemory ? XRL_E_OOM : XRL_E_HIP, "%s: %s (%s:%d)", \
                        #call, hipGetErrorString(e_), __FILE__, __LINE__);                \
    } while (0)

#define XRL_CHECK(cond, code, ...)                   \
    do {                                             \
        if (!(cond)) ::xrl::fail(code, __VA_ARGS__); \
    } while (0)

// Run `body` and convert any xrl::Error to a status (the ABI never throws).
template <class F>
xrl_status guarded(F &&body)
{
    try {
        body();
        return XRL_OK;
    } catch (const Error &e) {
        set_error("%s", e.msg.c_str());
        return e.code;
    } catch (const std::bad_alloc &) {
        set_error("host allocation failed");
        return XRL_E_OOM;
    } catch (...) {
        set_error("unexpected internal error");
        return XRL_E_HIP;
    }
}

// Device allocation: through the installed xrl_allocator if any (the
// stream of the current entry point is passed on), else hipMalloc/hipFree.
// A buffer remembers the allocator that made it and is released through it,
// after the device has finished with it (hipFree waits the same way).
struct AllocSrc {
    void (*free)(void *, void *) = nullptr;
    void *ctx = nullptr;
};
void *dev_alloc(size_t bytes, AllocSrc &src);
void dev_free(void *p, const AllocSrc &src);

// The stream handed to the allocator for allocations made in this thread
// while an entry point runs (set for the entry point's duration).
struct AllocStream {
    hipStream_t prev;
    explicit AllocStream(hipStream_t s);
    ~AllocStream();
};

// Owning device buffer.
template <class T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    AllocSrc src;
    DevBuf() = default;
    explicit DevBuf(size_t count) { alloc(count); }
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n), src(o.src)
    {
        o.p = nullptr;
        o.n = 0;
    }
    DevBuf &operator=(DevBuf &&o) noexcept
    {
        if (this != &o) {
            release();
            p = o.p;
            n = o.n;
            src = o.src;
            o.p = nullptr;
            o.n = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void alloc(size_t count)
    {
        release();
        if (count) p = (T *)dev_alloc(count * sizeof(T), src);
        n = count;
    }
    void release()
    {
        if (p) dev_free(p, src);
        p = nullptr;
        n = 0;
    }
    void upload(const T *h, size_t count, hipStream_t s)
    {
        if (count > n) alloc(count);
        if (count) XRL_HIP(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
    }
    void upload(const std::vector<T> &h, hipStream_t s) { upload(h.data(), h.size(), s); }
    std::vector<T> download(hipStream_t s, size_t count = (size_t)-1) const
    {
        if (count == (size_t)-1) count = n;
        std::vector<T> h(count);
        if (count) {
            XRL_HIP(hipMemcpyAsync(h.data(), p, count * sizeof(T), hipMemcpyDeviceToHost, s));
            XRL_HIP(hipStreamSynchronize(s));
        }
        return h;
    }
    size_t bytes() const { return n * sizeof(T); }
};

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Morton helpers (21 bits per axis, 63-bit codes).
__host__ __device__ inline uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0x1fffffull;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}
__host__ __device__ inline uint32_t compact3(uint64_t x)
{
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
    x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x1fffffull;
    return (uint32_t)x;
}
__host__ __device__ inline uint64_t morton3(uint32_t ix, uint32_t iy, uint32_t iz)
{
    return spread3(ix) | (spread3(iy) << 1) | (spread3(iz) << 2);
}

constexpr int kMaxDepth = 21;
constexpr int kMaxLeaf = 128;

}  // namespace xrl

// --------------------------------------------------------------------------
// Tree: one mesh, panels sorted in Morton order of their centroids.
// --------------------------------------------------------------------------
struct xrl_tree {
    int64_t N = 0, nv = 0;  // elements (triangles), vertices
    int64_t Np = 0;         // user panels (N unless four-sided panels were split)
    xrl::DevBuf<int32_t> elem_panel;  // [N] element (input order) -> user panel; empty: identity
    int max_leaf = 64, max_depth = 21;
    double root_c[3] = {0, 0, 0};
    double root_size = 0;
    int depth = 0;
    int n_overfull = 0;
    // sorted panel data (device)
    xrl::DevBuf<int32_t> perm;    // sorted position -> original panel index
    xrl::DevBuf<double> pv;       // [N][9] vertices of each panel
    xrl::DevBuf<int32_t> pvid;    // [N][3] vertex ids of each panel
    xrl::DevBuf<double> cen;      // [N][3] centroids
    xrl::DevBuf<double> area;     // [N]
    xrl::DevBuf<double> diam;     // [N] longest edge
    xrl::DevBuf<uint64_t> code;   // [N] sorted Morton codes
    // boxes, level-major, sorted by key within a level (host copies; small)
    std::vector<int64_t> level_off;  // [depth+2]
    std::vector<uint64_t> box_key;   // key at its own level
    std::vector<int32_t> box_level, box_parent, box_child0, box_nchild, box_beg, box_end;
};

// --------------------------------------------------------------------------
// One translation pass (M2L over all levels, or M2M / L2L at one level):
// (target box, source box, operator) triples sorted by operator, plus the
// per-target reduction lists over the sorted positions.
// --------------------------------------------------------------------------
struct TransPass {
    int64_t n_pairs = 0, n_groups = 0, n_red = 0;
    std::vector<int32_t> h_gbeg;      // [n_groups+1]
    xrl::DevBuf<int32_t> src;         // [n_pairs] source box, operator-sorted
    xrl::DevBuf<int32_t> goff;        // [n_groups] operator index
    xrl::DevBuf<int32_t> gbeg;        // [n_groups+1]
    xrl::DevBuf<int32_t> red_tgt;     // [n_red] target boxes
    xrl::DevBuf<int32_t> red_ptr;     // [n_red+1]
    xrl::DevBuf<int32_t> red_slot;    // [n_pairs] sorted position of each pair, target order
    xrl::DevBuf<int32_t> ts_src;      // [n_pairs] source box of each pair, target order
    xrl::DevBuf<int32_t> ts_op;       // [n_pairs] target order: operator index << 3 | reflection bits
    xrl::DevBuf<int32_t> ts_op_full;  // [n_pairs] target order: plain operator index << 3 (M2L only)
    xrl::DevBuf<int32_t> ts_order;    // [n_red] target indices, most pairs first (ties in target order)
    xrl::DevBuf<int32_t> ts_tgt;      // [n_pairs] target box of each pair, target order
    int64_t n_ps = 0;                 // runs of consecutive pairs (target order) with the same source
    xrl::DevBuf<int32_t> ps_beg;      // [n_ps+1] first pair of each run
    mutable std::vector<std::pair<int64_t, xrl::DevBuf<int32_t>>> item_cache;  // key: (engine, cols)
};

// --------------------------------------------------------------------------
// Plan: one or more trees, interaction lists, operators, near field.
// --------------------------------------------------------------------------
struct xrl_plan {
    int p = 8, K = 81;
    int precision = XRL_PREC_MIXED;
    int m2l_engine = XRL_M2L_MFMA;
    int max_cols = 1;  // complex columns
    std::vector<xrl_tree *> trees;
    std::vector<int64_t> panel_off;  // [ntrees+1] global element offsets (sorted blocks)
    std::vector<int64_t> user_off;   // [ntrees+1] global user panel offsets
    int64_t N = 0;                   // elements (the FMM's and the near field's points)
    int64_t Nu = 0;                  // user panels (rows of x and y)
    // global boxes (level-major across trees)
    int64_t B = 0;
    int depth = 0;
    std::vector<int64_t> level_off;  // [depth+2]
    std::vector<int32_t> h_box_beg, h_box_end, h_box_parent, h_box_child0, h_box_nchild, h_box_level,
        h_box_tree;
    std::vector<int32_t> h_leaf_box;
    xrl::DevBuf<int32_t> box_beg, box_end, box_parent, box_child0, box_nchild, box_level, box_octant;
    xrl::DevBuf<double> box_center;  // [B][3]
    xrl::DevBuf<double> box_h;       // [B] side length
    xrl::DevBuf<double> box_rad;     // [B] panel-inclusive radius
    xrl::DevBuf<int32_t> leaf_box;   // [n_leaves]
    int64_t n_leaves = 0;
    // global sorted panels
    xrl::DevBuf<int32_t> perm;    // global sorted element -> global user panel index
    xrl::DevBuf<int32_t> iperm;   // [Nu] user panel -> sorted position of its (first) element
    xrl::DevBuf<int32_t> iperm2;  // [Nu] second element of a four-sided panel, -1 (empty: none)
    xrl::DevBuf<double> pv;      // [N][9]
    xrl::DevBuf<int32_t> pvid;   // [N][3] (vertex ids offset per tree)
    xrl::DevBuf<double> cen, area, diam;
    xrl::DevBuf<int32_t> panel_leaf;  // [N] leaf index (into leaf_box) of each sorted panel
    // translation passes
    int64_t n_m2l = 0;
    int64_t n_demoted = 0;  // V candidates applied directly (radii do not separate)
    xrl::DevBuf<int32_t> m2l_pair_t, m2l_pair_s;  // [n] target and source box of each pair, per-target order
    xrl::DevBuf<double> m2l_ratio;                // [n] (r_t + r_s) / |c_t - c_s| of each pair, same order
    double theta = XRL_DEFAULT_THETA;  // separation criterion of the V-list pairs
    TransPass m2l;
    std::vector<TransPass> m2m, l2l;   // per level
    // L2L per level without the leaf targets: the FP32 matrix-core L2P
    // applies the parent's local to a leaf's panels itself (mom_l2l32)
    std::vector<TransPass> l2l_inner;
    mutable xrl::DevBuf<float> os_tmp32;
    mutable xrl::DevBuf<double> os_tmp64;
    double max_sep_ratio = 0;
    // operators (FP64 master + FP32 copy), real (p+1)^2 x (p+1)^2, row = output
    xrl::DevBuf<double> op_m2m64, op_l2l64, op_m2l64;  // [8][K][K], [8][K][K], [343][KP][KK]
    xrl::DevBuf<float> op_m2m32, op_l2l32, op_m2l32;
    // M2L operators k-major for the vector-ALU GEMM [343][KK][KP]
    xrl::DevBuf<float> op_m2l32k;
    xrl::DevBuf<double> op_m2l64k;
    // operators in MFMA fragment order [n_op][KP/16][KK/4][64] and k-major
    // [n_op][KK][KP] for the vector-ALU GEMM (M2L: 343 slots, M2M/L2L: 8)
    xrl::DevBuf<double> op_m2l64f, op_m2m64f, op_l2l64f, op_m2m64k, op_l2l64k;
    xrl::DevBuf<float> op_m2l32f, op_m2m32f, op_l2l32f, op_m2m32k, op_l2l32k;
    // Operators for the target-stationary kernel in vector fragment order
    // [op][row tile][k step / VEC][lane][VEC] (VEC = 16 bytes / element):
    // M2L for the 64 offsets with non-negative components (every other offset
    // is one of these under coordinate reflections), M2M and L2L (8 each).
    xrl::DevBuf<double> op_m2lc64v, op_m2m64v, op_l2l64v, op_m2l64v;
    xrl::DevBuf<float> op_m2lc32v, op_m2m32v, op_l2l32v, op_m2l32v;
    // last operator row (K - 1) of the same operators, [op][k % 4][k / 4]
    // (padded to the vector length), for orders with K = 16 n + 1 whose last
    // row is applied on the vector ALU instead of a 16-row MFMA tile
    xrl::DevBuf<double> op_m2m64t, op_l2l64t, op_m2l64t, op_m2lc64t;
    xrl::DevBuf<float> op_m2m32t, op_l2l32t, op_m2l32t, op_m2lc32t;
    // form of the target-stationary M2L (XRL_TUNE_TS_KERNEL)
    int ts_kernel = 0;
    int ts_min_cols = 16;  // MFMA engine: target-stationary from this many real columns on
    int p2p_form = 0;  // P2P above 16 FP32 columns: 0 MFMA, 1 scalar densities, 2 LDS-staged (XRL_TUNE_P2P_FORM)
    int leaf_mfma = 1;       // P2M and L2P above 16 FP32 columns on MFMA (1) or the vector ALU (0)
    int leaf_l2l = 1;        // matrix-core L2P applies the leaves' L2L itself (XRL_TUNE_LEAF_L2L)
    int valu_col = 1;        // vector-ALU offset-stationary form (XRL_TUNE_VALU_FORM)
    int tr_m2m = 2;          // <= 8 pairs per target: one wave per row tile (1), per target (0), by level size (2)
    int ps_l2l = 1;          // passes with one source per target: source-stationary (1) or lean (0)
    int ts_order = 1;        // target-stationary launch order: 1 most pairs first, 0 target order
    int ts_narrow_cols = 1;  // FP32 target-stationary: 1..4 columns past the last full tile on 4x4 MFMA blocks
    mutable int64_t scratch_budget = 0;  // bytes for the offset-stationary per-pair scratch (0: not set)
    int KP = 96, KK = 84;  // padded row / k dims of the M2L operator tiles
    // moment table per sorted panel, scaled to its leaf: [N][K]
    xrl::DevBuf<double> mom64;
    xrl::DevBuf<float> mom32;
    // [N][K] per panel of a leaf at level >= 3: its weighted moment row
    // through the L2L operator of its leaf's octant, (1/h) sum_i Q[i] w_i
    // T[i][j], so that L2P takes the parent's local directly (FP32 plans)
    xrl::DevBuf<float> mom_l2l32;
    // near field: per leaf a list of source rows; block [rows][tpad]
    std::vector<int32_t> h_near_rows;  // [n_leaves+1]
    xrl::DevBuf<int32_t> near_rows;    // [n_leaves+1]
    xrl::DevBuf<int32_t> near_src;     // [n_rows]
    xrl::DevBuf<int64_t> near_val_off; // [n_leaves+1] value offsets
    xrl::DevBuf<int32_t> leaf_tpad;    // [n_leaves]
    int64_t n_near_rows = 0, n_near_entries = 0, n_near_pairs = 0;
    xrl::DevBuf<double> near64;
    xrl::DevBuf<float> near32;
    bool assembled = false;
    // work buffers for the matvec (sorted order, real columns)
    mutable xrl::DevBuf<double> xs64, ys64, M64, L64;
    mutable xrl::DevBuf<float> xs32, ys32, M32, L32;
    mutable int64_t work_cols = 0;
    // profiling
    bool profiling = false;
    // ring of per-matvec event sets (recorded without any host wait; read
    // and averaged by xrl_plan_get_phase_ms)
    static constexpr int kProfRing = 256;
    mutable std::vector<std::vector<hipEvent_t>> prof_ev;
    mutable int64_t prof_count = 0;
    // epilogue scalars of the current call, [alpha re, im][beta re, im] per
    // column (plan-owned, so no call allocates or waits for them)
    mutable xrl::DevBuf<double> ep_dev;
    // HIP graph of the whole matvec for one argument set (graph mode)
    bool use_graph = false;
    mutable hipStream_t cap_stream = nullptr;
    mutable hipGraphExec_t gexec = nullptr;
    struct GraphKey {
        const void *x = nullptr;
        void *y = nullptr;
        int64_t ldx = 0, ldy = 0;
        int ncols = 0, dtype = 0, alpha = 0, beta = 0;
        bool operator==(const GraphKey &o) const
        {
            return x == o.x && y == o.y && ldx == o.ldx && ldy == o.ldy && ncols == o.ncols && dtype == o.dtype &&
                   alpha == o.alpha && beta == o.beta;
        }
    };
    mutable GraphKey gkey;
    mutable int64_t graph_launches = 0;
};
