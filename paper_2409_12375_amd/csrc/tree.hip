// Octree on panel centroids (the FMM of Sec. II-C runs on panel centroids):
// panel geometry, Morton codes, radix sort (our own, sort.h) and
// level-by-level splitting, on the device.

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <memory>
#include <mutex>

#include "common.h"
#include "sort.h"

namespace xrl {

static thread_local std::string g_last_error;

void set_error(const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void fail(xrl_status code, const char *fmt, ...)
{
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Error{code, std::string(buf)};
}

// ------------------------------------------------------------------ device memory
static std::mutex g_alloc_mu;
static xrl_allocator g_alloc{};  // hooks NULL: hipMalloc / hipFree
static thread_local hipStream_t t_alloc_stream = nullptr;

AllocStream::AllocStream(hipStream_t s) : prev(t_alloc_stream) { t_alloc_stream = s; }
AllocStream::~AllocStream() { t_alloc_stream = prev; }

void *dev_alloc(size_t bytes, AllocSrc &src)
{
    xrl_allocator a;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        a = g_alloc;
    }
    void *p = nullptr;
    if (a.alloc) {
        p = a.alloc(bytes, (void *)t_alloc_stream, a.ctx);
        XRL_CHECK(p, XRL_E_OOM, "device allocation of %zu bytes refused by the installed allocator", bytes);
        XRL_CHECK(((uintptr_t)p & 255) == 0, XRL_E_INVALID_ARG,
                  "the installed allocator returned a pointer not aligned to 256 bytes");
        src.free = a.free;
        src.ctx = a.ctx;
    } else {
        XRL_HIP(hipMalloc(&p, bytes));
        src = AllocSrc{};
    }
    return p;
}

void dev_free(void *p, const AllocSrc &src)
{
    if (src.free) {
        // every use of the buffer is enqueued before its release; wait for
        // them, as hipFree does, before the allocator may hand it out again
        (void)hipDeviceSynchronize();
        src.free(p, src.ctx);
    } else {
        (void)hipFree(p);
    }
}

// Per panel (input order): vertices, centroid, area, longest edge; error
// flags: bit 0 vertex index out of range, bit 1 degenerate or non-finite.
__global__ void k_panel_geometry(const double *__restrict__ V, int64_t nv, const int32_t *__restrict__ T,
                                 int64_t N, double *__restrict__ cen, double *__restrict__ area,
                                 double *__restrict__ diam, int *__restrict__ flags)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= N) return;
    int32_t i0 = T[3 * k], i1 = T[3 * k + 1], i2 = T[3 * k + 2];
    if (i0 < 0 || i1 < 0 || i2 < 0 || i0 >= nv || i1 >= nv || i2 >= nv) {
        atomicOr(flags, 1);
        cen[3 * k] = cen[3 * k + 1] = cen[3 * k + 2] = 0.0;
        area[k] = 0.0;
        diam[k] = 0.0;
        return;
    }
    double a[3], b[3], c[3];
    for (int d = 0; d < 3; ++d) {
        a[d] = V[3 * (int64_t)i0 + d];
        b[d] = V[3 * (int64_t)i1 + d];
        c[d] = V[3 * (int64_t)i2 + d];
    }
    double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double e3[3] = {c[0] - b[0], c[1] - b[1], c[2] - b[2]};
    double cx = e1[1] * e2[2] - e1[2] * e2[1];
    double cy = e1[2] * e2[0] - e1[0] * e2[2];
    double cz = e1[0] * e2[1] - e1[1] * e2[0];
    double A = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
    double l1 = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    double l2 = sqrt(e2[0] * e2[0] + e2[1] * e2[1] + e2[2] * e2[2]);
    double l3 = sqrt(e3[0] * e3[0] + e3[1] * e3[1] + e3[2] * e3[2]);
    double D = fmax(l1, fmax(l2, l3));
    for (int d = 0; d < 3; ++d) cen[3 * k + d] = (a[d] + b[d] + c[d]) / 3.0;
    area[k] = A;
    diam[k] = D;
    if (!(A > 1e-14 * D * D) || !isfinite(A) || !isfinite(D)) atomicOr(flags, 2);
}

// Partial bounding box of centroids: out[block][6] = (min xyz, max xyz).
__global__ void k_bbox(const double *__restrict__ cen, int64_t N, double *__restrict__ out)
{
    __shared__ double s[256][6];
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < N;
         k += (int64_t)gridDim.x * blockDim.x)
        for (int d = 0; d < 3; ++d) {
            mn[d] = fmin(mn[d], cen[3 * k + d]);
            mx[d] = fmax(mx[d], cen[3 * k + d]);
        }
    for (int d = 0; d < 3; ++d) {
        s[threadIdx.x][d] = mn[d];
        s[threadIdx.x][3 + d] = mx[d];
    }
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int d = 0; d < 3; ++d) {
                s[threadIdx.x][d] = fmin(s[threadIdx.x][d], s[threadIdx.x + w][d]);
                s[threadIdx.x][3 + d] = fmax(s[threadIdx.x][3 + d], s[threadIdx.x + w][3 + d]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < 6; ++d) out[6 * blockIdx.x + d] = s[0][d];
}

__global__ void k_morton(const double *__restrict__ cen, int64_t N, double x0, double y0, double z0,
                         double inv_h, uint64_t *__restrict__ code, int32_t *__restrict__ idx)
{
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= N) return;
    const double o[3] = {x0, y0, z0};
    uint32_t q[3];
    for (int d = 0; d < 3; ++d) {
        double f = (cen[3 * k + d] - o[d]) * inv_h;  // in [0, 2^21)
        long long v = (long long)floor(f);
        v = v < 0 ? 0 : (v > 2097151 ? 2097151 : v);
        q[d] = (uint32_t)v;
    }
    code[k] = morton3(q[0], q[1], q[2]);
    idx[k] = (int32_t)k;
}

__global__ void k_gather_panels(const int32_t *__restrict__ perm, int64_t N, const double *__restrict__ V,
                                const int32_t *__restrict__ T, const double *__restrict__ cen_in,
                                const double *__restrict__ area_in, const double *__restrict__ diam_in,
                                double *__restrict__ pv, int32_t *__restrict__ pvid, double *__restrict__ cen,
                                double *__restrict__ area, double *__restrict__ diam)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    int64_t k = perm[i];
    for (int j = 0; j < 3; ++j) {
        int32_t v = T[3 * k + j];
        pvid[3 * i + j] = v;
        for (int d = 0; d < 3; ++d) pv[9 * i + 3 * j + d] = V[3 * (int64_t)v + d];
        cen[3 * i + j] = cen_in[3 * k + j];
    }
    area[i] = area_in[k];
    diam[i] = diam_in[k];
}

// Coincident panels: two panels with the same centroid have the same Morton
// code, so they are neighbours in the sorted order.  Within each run of equal
// codes (bounded scan), a panel is flagged if a later one has the same three
// vertex indices or the same three vertex positions (bit 2 of flags).
__global__ void k_duplicates(const uint64_t *__restrict__ code, const int32_t *__restrict__ pvid,
                             const double *__restrict__ pv, int64_t N, int *__restrict__ flags)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    int32_t a[3] = {pvid[3 * i], pvid[3 * i + 1], pvid[3 * i + 2]};
    for (int64_t j = i + 1; j < N && j <= i + 256 && code[j] == code[i]; ++j) {
        bool same_ids = true, same_pos = true;
        for (int u = 0; u < 3; ++u) {
            bool id_found = false, pos_found = false;
            for (int v = 0; v < 3; ++v) {
                id_found |= pvid[3 * j + v] == a[u];
                pos_found |= pv[9 * j + 3 * v] == pv[9 * i + 3 * u] && pv[9 * j + 3 * v + 1] == pv[9 * i + 3 * u + 1] &&
                             pv[9 * j + 3 * v + 2] == pv[9 * i + 3 * u + 2];
            }
            same_ids &= id_found;
            same_pos &= pos_found;
        }
        if (same_ids || same_pos) {
            atomicOr(flags, 4);
            return;
        }
    }
}

// Root box: every element, at level 0.
__global__ void k_root_box(int32_t N, uint64_t *key, int32_t *level, int32_t *parent, int32_t *child0,
                           int32_t *nchild, int32_t *beg, int32_t *end)
{
    key[0] = 0;
    level[0] = 0;
    parent[0] = -1;
    child0[0] = -1;
    nchild[0] = 0;
    beg[0] = 0;
    end[0] = N;
}

// Boxes lo .. lo + n - 1 of one level: a box with more than max_leaf
// elements splits (below the maximum depth; at it, it is counted in *over).
// For a splitting box: the 9 boundaries of its child ranges in the sorted
// code array (lower bounds of the 8 child digits, then its end) and the
// number of nonempty children; 0 children for the others.
__global__ void k_split_level(const uint64_t *__restrict__ code, int32_t lo, int32_t n, int level, bool can_split,
                              int max_leaf, const uint64_t *__restrict__ key, const int32_t *__restrict__ beg,
                              const int32_t *__restrict__ end, int32_t *__restrict__ bounds,
                              int32_t *__restrict__ nch, int32_t *__restrict__ over)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = lo + i;
    nch[i] = 0;
    if (end[b] - beg[b] <= max_leaf) return;
    if (!can_split) {
        atomicAdd(over, 1);
        return;
    }
    const int shift_child = 3 * (kMaxDepth - level - 1);
    int cnt = 0;
    int32_t prev = beg[b];
    for (int d = 0; d < 8; ++d) {
        int32_t l = beg[b], h = end[b];
        const uint64_t target = ((key[b] << 3) | (uint64_t)d) << shift_child;
        while (l < h) {
            const int32_t mid = l + (h - l) / 2;
            if (code[mid] < target)
                l = mid + 1;
            else
                h = mid;
        }
        bounds[9 * (int64_t)i + d] = l;
        if (d > 0) cnt += l > prev;
        prev = l;
    }
    bounds[9 * (int64_t)i + 8] = end[b];
    cnt += end[b] > prev;
    nch[i] = cnt;
}

// The children of the splitting boxes of one level, from position
// first + coff[i] on (nonempty octants in order).
__global__ void k_make_children(int32_t lo, int32_t n, int32_t first, int level, const int32_t *__restrict__ bounds,
                                const int32_t *__restrict__ nch, const int32_t *__restrict__ coff, uint64_t *key,
                                int32_t *blevel, int32_t *parent, int32_t *child0, int32_t *nchild, int32_t *beg,
                                int32_t *end)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || nch[i] == 0) return;
    const int32_t b = lo + i, c0 = first + coff[i];
    child0[b] = c0;
    nchild[b] = nch[i];
    int k = 0;
    for (int d = 0; d < 8; ++d) {
        const int32_t cb = bounds[9 * (int64_t)i + d], ce = bounds[9 * (int64_t)i + d + 1];
        if (ce <= cb) continue;
        const int32_t c = c0 + k++;
        key[c] = (key[b] << 3) | (uint64_t)d;
        blevel[c] = level + 1;
        parent[c] = b;
        child0[c] = -1;
        nchild[c] = 0;
        beg[c] = cb;
        end[c] = ce;
    }
}

// Hybrid meshes: one element per triangle row, two per four-sided panel
// (a, b, c, d) -> (a, b, c), (a, c, d).
__global__ void k_elem_count(const int32_t *__restrict__ Q, int64_t N, int32_t *__restrict__ cnt)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p < N) cnt[p] = Q[4 * p + 3] >= 0 ? 2 : 1;
}

__global__ void k_split_panels(const int32_t *__restrict__ Q, int64_t N, const int64_t *__restrict__ off,
                               int32_t *__restrict__ T, int32_t *__restrict__ elem_panel)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= N) return;
    const int32_t a = Q[4 * p], b = Q[4 * p + 1], c = Q[4 * p + 2], d = Q[4 * p + 3];
    const int64_t e = off[p];
    T[3 * e] = a;
    T[3 * e + 1] = b;
    T[3 * e + 2] = c;
    elem_panel[e] = (int32_t)p;
    if (d >= 0) {
        T[3 * e + 3] = a;
        T[3 * e + 4] = c;
        T[3 * e + 5] = d;
        elem_panel[e + 1] = (int32_t)p;
    }
}

}  // namespace xrl

using namespace xrl;

extern "C" const char *xrl_last_error(void) { return g_last_error.c_str(); }
extern "C" const char *xrl_version(void) { return "xrl-mi355x 0.1 (gfx950)"; }

extern "C" xrl_status xrl_tree_build(const xrl_mesh_desc *mesh, int32_t max_leaf, int32_t max_depth,
                                     void *stream, xrl_tree **out)
{
    return guarded([&] {
        XRL_CHECK(mesh && out, XRL_E_INVALID_ARG, "xrl_tree_build: null mesh or out");
        *out = nullptr;
        XRL_CHECK(mesh->vertices && mesh->tris, XRL_E_INVALID_ARG, "xrl_tree_build: null arrays");
        XRL_CHECK(mesh->n_panels >= 1 && mesh->n_panels < (int64_t(1) << 31) && mesh->n_vertices >= 3 &&
                      mesh->n_vertices < (int64_t(1) << 31),
                  XRL_E_INVALID_ARG, "xrl_tree_build: bad sizes (n_panels=%lld, n_vertices=%lld)",
                  (long long)mesh->n_panels, (long long)mesh->n_vertices);
        XRL_CHECK(max_leaf >= 1 && max_leaf <= kMaxLeaf, XRL_E_INVALID_ARG,
                  "xrl_tree_build: max_leaf must be in 1..%d (got %d)", kMaxLeaf, max_leaf);
        XRL_CHECK(max_depth >= 1 && max_depth <= kMaxDepth, XRL_E_INVALID_ARG,
                  "xrl_tree_build: max_depth must be in 1..21 (got %d)", max_depth);
        const int vpp = mesh->verts_per_panel == 0 ? 3 : mesh->verts_per_panel;
        XRL_CHECK(vpp == 3 || vpp == 4, XRL_E_INVALID_ARG, "xrl_tree_build: verts_per_panel must be 3 or 4 (got %d)",
                  mesh->verts_per_panel);
        hipStream_t s = (hipStream_t)stream;
        const AllocStream alloc_scope(s);
        const int64_t Np = mesh->n_panels, nv = mesh->n_vertices;
        auto t = std::make_unique<xrl_tree>();
        t->Np = Np;
        t->nv = nv;
        t->max_leaf = max_leaf;
        t->max_depth = max_depth;
        DevBuf<double> V(3 * nv);
        hipMemcpyKind kind = mesh->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        XRL_HIP(hipMemcpyAsync(V.p, mesh->vertices, V.bytes(), kind, s));
        DevBuf<int32_t> T;
        int64_t N = Np;
        if (vpp == 3) {
            T.alloc(3 * Np);
            XRL_HIP(hipMemcpyAsync(T.p, mesh->tris, T.bytes(), kind, s));
        } else {
            // elements: the triangles of every panel, in panel order
            DevBuf<int32_t> Q(4 * Np), cnt(Np);
            DevBuf<int64_t> off(Np), tot(1);
            XRL_HIP(hipMemcpyAsync(Q.p, mesh->tris, Q.bytes(), kind, s));
            k_elem_count<<<cdiv(Np, 256), 256, 0, s>>>(Q.p, Np, cnt.p);
            XRL_HIP(hipGetLastError());
            exclusive_scan<int32_t, int64_t>(cnt.p, Np, off.p, tot.p, s);
            N = tot.download(s)[0];
            XRL_CHECK(N < (int64_t(1) << 31), XRL_E_INVALID_ARG, "xrl_tree_build: more than 2^31 elements");
            T.alloc(3 * N);
            t->elem_panel.alloc(N);
            k_split_panels<<<cdiv(Np, 256), 256, 0, s>>>(Q.p, Np, off.p, T.p, t->elem_panel.p);
            XRL_HIP(hipGetLastError());
        }
        t->N = N;
        DevBuf<double> cen0(3 * N), area0(N), diam0(N);
        DevBuf<int> flags(1);
        XRL_HIP(hipMemsetAsync(flags.p, 0, sizeof(int), s));
        const int bs = 256;
        k_panel_geometry<<<cdiv(N, bs), bs, 0, s>>>(V.p, nv, T.p, N, cen0.p, area0.p, diam0.p, flags.p);
        XRL_HIP(hipGetLastError());
        int hflag = flags.download(s)[0];
        XRL_CHECK(!(hflag & 1), XRL_E_INVALID_ARG, "xrl_tree_build: vertex index out of range");
        XRL_CHECK(!(hflag & 2), XRL_E_DEGENERATE_PANEL,
                  "xrl_tree_build: degenerate or non-finite panel (area <= 1e-14 diam^2)");
        // bounding cube of the centroids
        int nb = (int)std::min<int64_t>(1024, cdiv(N, bs));
        DevBuf<double> part(6 * nb);
        k_bbox<<<nb, bs, 0, s>>>(cen0.p, N, part.p);
        XRL_HIP(hipGetLastError());
        auto hp = part.download(s);
        double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
        for (int b = 0; b < nb; ++b)
            for (int d = 0; d < 3; ++d) {
                mn[d] = std::min(mn[d], hp[6 * b + d]);
                mx[d] = std::max(mx[d], hp[6 * b + 3 + d]);
            }
        double ext = std::max({mx[0] - mn[0], mx[1] - mn[1], mx[2] - mn[2]});
        double scale = std::max({std::fabs(mn[0]), std::fabs(mn[1]), std::fabs(mn[2]), std::fabs(mx[0]),
                                 std::fabs(mx[1]), std::fabs(mx[2]), 1e-300});
        double side = ext * (1.0 + 1e-6) + 1e-9 * scale;
        if (!(side > 0)) side = 1.0;
        for (int d = 0; d < 3; ++d) t->root_c[d] = 0.5 * (mn[d] + mx[d]);
        t->root_size = side;
        // Morton codes and sort
        DevBuf<uint64_t> code(N), code_tmp(N);
        DevBuf<int32_t> idx_tmp(N);
        t->perm.alloc(N);
        const double inv_h = double(1 << kMaxDepth) / side;
        k_morton<<<cdiv(N, bs), bs, 0, s>>>(cen0.p, N, t->root_c[0] - 0.5 * side, t->root_c[1] - 0.5 * side,
                                            t->root_c[2] - 0.5 * side, inv_h, code.p, t->perm.p);
        XRL_HIP(hipGetLastError());
        // stable: equal codes keep their input order
        radix_sort_pairs(code.p, t->perm.p, code_tmp.p, idx_tmp.p, N, 63, s);
        t->pv.alloc(9 * N);
        t->pvid.alloc(3 * N);
        t->cen.alloc(3 * N);
        t->area.alloc(N);
        t->diam.alloc(N);
        k_gather_panels<<<cdiv(N, bs), bs, 0, s>>>(t->perm.p, N, V.p, T.p, cen0.p, area0.p, diam0.p, t->pv.p,
                                                   t->pvid.p, t->cen.p, t->area.p, t->diam.p);
        XRL_HIP(hipGetLastError());
        k_duplicates<<<cdiv(N, bs), bs, 0, s>>>(code.p, t->pvid.p, t->pv.p, N, flags.p);
        XRL_HIP(hipGetLastError());
        XRL_CHECK(!(flags.download(s)[0] & 4), XRL_E_DEGENERATE_PANEL,
                  "xrl_tree_build: two panels share their three vertices (coincident panels)");
        // level-by-level split, on the device: the boxes of one level that
        // hold more than max_leaf elements split into their nonempty octant
        // children, appended in parent order (then octant order) as the next
        // level; the arrays grow by doubling
        struct Boxes {
            DevBuf<uint64_t> key;
            DevBuf<int32_t> level, parent, child0, nchild, beg, end;
        } bx, grow;
        int64_t cap = 0, B = 1;
        auto reserve = [&](int64_t need) {
            if (need <= cap) return;
            const int64_t nc = std::max<int64_t>({need, 2 * cap, 1024});
            grow.key.alloc(nc);
            grow.level.alloc(nc);
            grow.parent.alloc(nc);
            grow.child0.alloc(nc);
            grow.nchild.alloc(nc);
            grow.beg.alloc(nc);
            grow.end.alloc(nc);
            if (B > 0 && cap > 0) {
                auto cp = [&](auto &dst, auto &src) {
                    XRL_HIP(hipMemcpyAsync(dst.p, src.p, B * sizeof(*src.p), hipMemcpyDeviceToDevice, s));
                };
                cp(grow.key, bx.key);
                cp(grow.level, bx.level);
                cp(grow.parent, bx.parent);
                cp(grow.child0, bx.child0);
                cp(grow.nchild, bx.nchild);
                cp(grow.beg, bx.beg);
                cp(grow.end, bx.end);
            }
            std::swap(bx, grow);
            cap = nc;
        };
        reserve(1);
        k_root_box<<<1, 1, 0, s>>>((int32_t)N, bx.key.p, bx.level.p, bx.parent.p, bx.child0.p, bx.nchild.p, bx.beg.p,
                                   bx.end.p);
        XRL_HIP(hipGetLastError());
        t->level_off = {0};
        DevBuf<int32_t> over(1), nch, coff, ctot(1), bounds;
        XRL_HIP(hipMemsetAsync(over.p, 0, sizeof(int32_t), s));
        for (int level = 0;; ++level) {
            const int64_t lo = t->level_off.back(), hi = B, n = hi - lo;
            t->level_off.push_back(hi);
            nch.alloc(n);
            coff.alloc(n);
            bounds.alloc(9 * n);
            k_split_level<<<(unsigned)cdiv(n, 128), 128, 0, s>>>(code.p, (int32_t)lo, (int32_t)n, level,
                                                                level < max_depth, max_leaf, bx.key.p, bx.beg.p,
                                                                bx.end.p, bounds.p, nch.p, over.p);
            XRL_HIP(hipGetLastError());
            exclusive_scan<int32_t, int32_t>(nch.p, n, coff.p, ctot.p, s);
            const int64_t nc = ctot.download(s)[0];
            if (nc == 0) break;
            XRL_CHECK(hi + nc < (int64_t(1) << 31), XRL_E_UNSUPPORTED, "xrl_tree_build: more than 2^31 boxes");
            reserve(hi + nc);
            k_make_children<<<(unsigned)cdiv(n, 128), 128, 0, s>>>((int32_t)lo, (int32_t)n, (int32_t)hi, level,
                                                                   bounds.p, nch.p, coff.p, bx.key.p, bx.level.p,
                                                                   bx.parent.p, bx.child0.p, bx.nchild.p, bx.beg.p,
                                                                   bx.end.p);
            XRL_HIP(hipGetLastError());
            B = hi + nc;
        }
        t->n_overfull = over.download(s)[0];
        // host copies of the box arrays (the plan merges the boxes of its trees)
        t->box_key = bx.key.download(s, B);
        t->box_level = bx.level.download(s, B);
        t->box_parent = bx.parent.download(s, B);
        t->box_child0 = bx.child0.download(s, B);
        t->box_nchild = bx.nchild.download(s, B);
        t->box_beg = bx.beg.download(s, B);
        t->box_end = bx.end.download(s, B);
        // level_off holds [depth + 2] entries: the start of every level and the total
        t->depth = (int)t->level_off.size() - 2;
        t->code = std::move(code);
        XRL_HIP(hipStreamSynchronize(s));
        *out = t.release();
    });
}

extern "C" void xrl_tree_destroy(xrl_tree *tree) { delete tree; }

extern "C" xrl_status xrl_tree_get_info(const xrl_tree *t, xrl_tree_info *info)
{
    return guarded([&] {
        XRL_CHECK(t && info, XRL_E_INVALID_ARG, "xrl_tree_get_info: null argument");
        info->n_panels = t->Np;
        info->n_elements = t->N;
        info->n_boxes = (int64_t)t->box_key.size();
        int64_t nl = 0;
        for (size_t b = 0; b < t->box_nchild.size(); ++b) nl += t->box_nchild[b] == 0;
        info->n_leaves = nl;
        info->depth = t->depth;
        info->n_overfull_leaves = t->n_overfull;
        for (int d = 0; d < 3; ++d) info->root_center[d] = t->root_c[d];
        info->root_size = t->root_size;
    });
}

extern "C" xrl_status xrl_set_allocator(const xrl_allocator *a)
{
    return xrl::guarded([&] {
        if (a) XRL_CHECK(a->alloc && a->free, XRL_E_INVALID_ARG, "xrl_set_allocator: both hooks are required");
        std::lock_guard<std::mutex> lk(xrl::g_alloc_mu);
        xrl::g_alloc = a ? *a : xrl_allocator{};
    });
}
