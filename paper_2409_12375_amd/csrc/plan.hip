// FMM plan: global boxes over one or more trees, interaction lists (on the
// device), translation operators, per-panel moment tables.
//
// Lists of the adaptive octree (U, V, W, X; the classical adaptive FMM that
// Sec. II-C refers to for the panel-based FMM):
//   V(b)  boxes at b's level that are children of the colleagues of b's
//         parent and not adjacent to b                      -> M2L
//   U(T)  leaves adjacent to leaf T (any level, T included)  -> direct
//   W(T)  descendants D of T's colleagues with D not adjacent to T and
//         D's parent adjacent to T                           -> direct (all panels of D)
//   X(B)  leaves C coarser than B, adjacent to B's parent, not adjacent to B
//                                                            -> direct to every
//         leaf below B
// so the near field of a target leaf is U(T), W(T) and X of T and of all its
// ancestors, each given as a contiguous range of Morton-sorted panels.

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <exception>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>

#include "common.h"
#include "scan.h"
#include "sort.h"
#include "harmonics.h"

namespace xrl {

void build_m2m(int p, double *out);
void build_l2l(int p, double *out);
void build_m2l(int p, int ox, int oy, int oz, double *out);
void gauss_legendre01(int n, double *x, double *w);

struct BoxView {
    const uint64_t *key;
    const int32_t *level, *parent, *child0, *nchild, *tree;
    const int64_t *seg;  // [(depth+1) * (ntrees+1)]
    int ntrees;
};

__device__ inline void box_coords(uint64_t key, int32_t c[3])
{
    c[0] = (int32_t)compact3(key);
    c[1] = (int32_t)compact3(key >> 1);
    c[2] = (int32_t)compact3(key >> 2);
}

// Closed cubes of boxes (level la, coords a) and (lb, b) intersect.
__device__ inline bool adjacent(int la, const int32_t *a, int lb, const int32_t *b)
{
    const int f = la > lb ? la : lb;
    const int sa = f - la, sb = f - lb;
    for (int d = 0; d < 3; ++d) {
        const int64_t alo = (int64_t)a[d] << sa, ahi = (int64_t)(a[d] + 1) << sa;
        const int64_t blo = (int64_t)b[d] << sb, bhi = (int64_t)(b[d] + 1) << sb;
        if (alo > bhi || blo > ahi) return false;
    }
    return true;
}

__device__ inline int32_t find_box(const BoxView &bv, int level, int tree, uint64_t key)
{
    int64_t lo = bv.seg[level * (bv.ntrees + 1) + tree], hi = bv.seg[level * (bv.ntrees + 1) + tree + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (bv.key[mid] < key)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo < bv.seg[level * (bv.ntrees + 1) + tree + 1] && bv.key[lo] == key) return (int32_t)lo;
    return -1;
}

// Same-level neighbours (27 slots, -1 when absent; slot 13 is the box itself).
__global__ void k_colleagues(BoxView bv, int64_t B, int32_t *__restrict__ coll)
{
    int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int l = bv.level[b], t = bv.tree[b];
    int32_t c[3];
    box_coords(bv.key[b], c);
    const int32_t lim = 1 << l;
    int slot = 0;
    for (int dz = -1; dz <= 1; ++dz)
        for (int dy = -1; dy <= 1; ++dy)
            for (int dx = -1; dx <= 1; ++dx, ++slot) {
                const int32_t x = c[0] + dx, y = c[1] + dy, z = c[2] + dz;
                int32_t r = -1;
                if (x >= 0 && y >= 0 && z >= 0 && x < lim && y < lim && z < lim)
                    r = (slot == 13) ? (int32_t)b : find_box(bv, l, t, morton3(x, y, z));
                coll[27 * b + slot] = r;
            }
}

// V-lists: count (src == nullptr) or fill.  A candidate pair whose
// panel-inclusive radii do not separate (rad_t + rad_s >= theta |c_t - c_s|)
// cannot be translated with a convergent expansion; it is emitted to the
// demoted list instead and applied directly as near field.
__global__ void k_vlist(BoxView bv, int64_t B, const int32_t *__restrict__ coll, const double *__restrict__ center,
                        const double *__restrict__ rad, double theta, int32_t *__restrict__ cnt,
                        int32_t *__restrict__ dcnt, const int64_t *__restrict__ off, const int64_t *__restrict__ doff,
                        int32_t *__restrict__ src, int32_t *__restrict__ code, int32_t *__restrict__ dsrc)
{
    int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= B) return;
    const int l = bv.level[b];
    int n = 0, nd = 0;
    if (l >= 2) {
        const int32_t p = bv.parent[b];
        int32_t cb[3];
        box_coords(bv.key[b], cb);
        for (int s = 0; s < 27; ++s) {
            const int32_t q = coll[27 * p + s];
            if (q < 0) continue;
            for (int i = 0; i < bv.nchild[q]; ++i) {
                const int32_t c = bv.child0[q] + i;
                int32_t cc[3];
                box_coords(bv.key[c], cc);
                const int ox = cb[0] - cc[0], oy = cb[1] - cc[1], oz = cb[2] - cc[2];
                if (ox >= -1 && ox <= 1 && oy >= -1 && oy <= 1 && oz >= -1 && oz <= 1) continue;
                const double dx = center[3 * b] - center[3 * c], dy = center[3 * b + 1] - center[3 * c + 1],
                             dz = center[3 * b + 2] - center[3 * c + 2];
                if (rad[b] + rad[c] >= theta * sqrt(dx * dx + dy * dy + dz * dz)) {
                    if (src) dsrc[doff[b] + nd] = c;
                    ++nd;
                    continue;
                }
                if (src) {
                    src[off[b] + n] = c;
                    code[off[b] + n] = (ox + 3) + 7 * (oy + 3) + 49 * (oz + 3);
                }
                ++n;
            }
        }
    }
    if (!src) {
        cnt[b] = n;
        dcnt[b] = nd;
    }
}

// Near-field source boxes of every leaf (U, W, X): count or fill.
__global__ void k_nearlist(BoxView bv, const int32_t *__restrict__ leaves, int64_t nleaf,
                           const int32_t *__restrict__ coll, int32_t *__restrict__ cnt,
                           const int64_t *__restrict__ off, int32_t *__restrict__ out)
{
    int64_t li = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (li >= nleaf) return;
    const int32_t T = leaves[li];
    const int lT = bv.level[T];
    int32_t cT[3];
    box_coords(bv.key[T], cT);
    int n = 0;
    auto emit = [&](int32_t box) {
        if (out) out[off[li] + n] = box;
        ++n;
    };
    // U (same level and finer) and W: colleagues and the descent below them
    int32_t stack[8 * kMaxDepth + 8];
    for (int s = 0; s < 27; ++s) {
        const int32_t C = coll[27 * T + s];
        if (C < 0) continue;
        if (bv.nchild[C] == 0) {
            emit(C);
            continue;
        }
        int sp = 0;
        for (int i = 0; i < bv.nchild[C]; ++i) stack[sp++] = bv.child0[C] + i;
        while (sp > 0) {
            const int32_t D = stack[--sp];
            int32_t cD[3];
            box_coords(bv.key[D], cD);
            if (adjacent(lT, cT, bv.level[D], cD)) {
                if (bv.nchild[D] == 0)
                    emit(D);  // U, finer
                else
                    for (int i = 0; i < bv.nchild[D]; ++i) stack[sp++] = bv.child0[D] + i;
            } else {
                emit(D);  // W
            }
        }
    }
    // U (coarser): leaf colleagues of proper ancestors adjacent to T
    for (int32_t A = bv.parent[T]; A >= 0; A = bv.parent[A]) {
        for (int s = 0; s < 27; ++s) {
            if (s == 13) continue;
            const int32_t Q = coll[27 * A + s];
            if (Q < 0 || bv.nchild[Q] != 0) continue;
            int32_t cQ[3];
            box_coords(bv.key[Q], cQ);
            if (adjacent(lT, cT, bv.level[Q], cQ)) emit(Q);
        }
    }
    // X of T and of every ancestor Bx: leaves Q coarser than Bx, adjacent to
    // parent(Bx), not adjacent to Bx
    for (int32_t Bx = T; bv.parent[Bx] >= 0; Bx = bv.parent[Bx]) {
        const int32_t P = bv.parent[Bx];
        int32_t cB[3], cP[3];
        box_coords(bv.key[Bx], cB);
        box_coords(bv.key[P], cP);
        const int lB = bv.level[Bx], lP = bv.level[P];
        for (int32_t A = P; A >= 0; A = bv.parent[A]) {
            for (int s = 0; s < 27; ++s) {
                if (s == 13) continue;
                const int32_t Q = coll[27 * A + s];
                if (Q < 0 || bv.nchild[Q] != 0) continue;
                int32_t cQ[3];
                box_coords(bv.key[Q], cQ);
                const int lQ = bv.level[Q];
                if (adjacent(lP, cP, lQ, cQ) && !adjacent(lB, cB, lQ, cQ)) emit(Q);
            }
        }
    }
    if (!out) cnt[li] = n;
}

// Source boxes of each leaf's near field: its U, W and X boxes (nbox) and
// the sources of the pairs demoted to the near field at the leaf or at any
// of its ancestors (every leaf below a demoted target takes the source's
// panels), sorted by their first panel so the rows come in Morton order.
// Count pass (soff NULL), then fill pass.
__global__ void k_leaf_sources(const int32_t *__restrict__ leaves, int64_t nleaf, const int32_t *__restrict__ parent,
                               const int64_t *__restrict__ noff, const int32_t *__restrict__ nbox,
                               const int64_t *__restrict__ doff, const int32_t *__restrict__ dsrc,
                               const int32_t *__restrict__ beg, const int32_t *__restrict__ end,
                               const int64_t *__restrict__ soff, int32_t *__restrict__ cnt,
                               int32_t *__restrict__ nrow, int32_t *__restrict__ sbox)
{
    const int64_t li = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (li >= nleaf) return;
    const int32_t T = leaves[li];
    if (!soff) {
        int64_t n = noff[li + 1] - noff[li], r = 0;
        for (int64_t j = noff[li]; j < noff[li + 1]; ++j) r += end[nbox[j]] - beg[nbox[j]];
        for (int32_t A = T; A >= 0; A = parent[A]) {
            n += doff[A + 1] - doff[A];
            for (int64_t j = doff[A]; j < doff[A + 1]; ++j) r += end[dsrc[j]] - beg[dsrc[j]];
        }
        cnt[li] = (int32_t)n;
        nrow[li] = (int32_t)min(r, (int64_t)INT32_MAX);
        return;
    }
    int32_t *out = sbox + soff[li];
    int n = 0;
    auto put = [&](int32_t b) {
        // insertion by first panel (lists hold tens of boxes)
        int i = n++;
        while (i > 0 && beg[out[i - 1]] > beg[b]) {
            out[i] = out[i - 1];
            --i;
        }
        out[i] = b;
    };
    for (int64_t j = noff[li]; j < noff[li + 1]; ++j) put(nbox[j]);
    for (int32_t A = T; A >= 0; A = parent[A])
        for (int64_t j = doff[A]; j < doff[A + 1]; ++j) put(dsrc[j]);
}

// Rows of each leaf's block: the panels of its source boxes in order
// (one workgroup per leaf).
__global__ void k_leaf_rows(int64_t nleaf, const int64_t *__restrict__ soff, const int32_t *__restrict__ sbox,
                            const int32_t *__restrict__ beg, const int32_t *__restrict__ end,
                            const int32_t *__restrict__ rows_ptr, int32_t *__restrict__ src)
{
    const int64_t li = blockIdx.x;
    if (li >= nleaf) return;
    int32_t at = rows_ptr[li];
    for (int64_t j = soff[li]; j < soff[li + 1]; ++j) {
        const int32_t b0 = beg[sbox[j]], nb = end[sbox[j]] - b0;
        for (int32_t k = threadIdx.x; k < nb; k += blockDim.x) src[at + k] = b0 + k;
        at += nb;
    }
}

// Per leaf: block padding (targets rounded up to 4, so that a row starts
// on 16 bytes for the vector loads of the vector-ALU forms) and its value
// count.
__global__ void k_leaf_blocks(int64_t nleaf, const int32_t *__restrict__ leaves, const int32_t *__restrict__ beg,
                              const int32_t *__restrict__ end, const int32_t *__restrict__ nrow,
                              int32_t *__restrict__ tpad, int64_t *__restrict__ nval, int64_t *__restrict__ npair)
{
    const int64_t li = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (li >= nleaf) return;
    const int32_t nt = end[leaves[li]] - beg[leaves[li]];
    tpad[li] = 4 * ((nt + 3) / 4);
    nval[li] = (int64_t)nrow[li] * tpad[li];
    npair[li] = (int64_t)nrow[li] * nt;
}

// Panel-inclusive radius of every box about its centre.
__global__ void k_box_radius(int64_t B, const int32_t *__restrict__ beg, const int32_t *__restrict__ end,
                             const double *__restrict__ center, const double *__restrict__ pv,
                             double *__restrict__ rad)
{
    int64_t b = blockIdx.x;
    if (b >= B) return;
    __shared__ double red[256];
    double r = 0;
    const double cx = center[3 * b], cy = center[3 * b + 1], cz = center[3 * b + 2];
    for (int64_t k = beg[b] + threadIdx.x; k < end[b]; k += blockDim.x)
        for (int j = 0; j < 3; ++j) {
            const double dx = pv[9 * k + 3 * j] - cx, dy = pv[9 * k + 3 * j + 1] - cy, dz = pv[9 * k + 3 * j + 2] - cz;
            r = fmax(r, sqrt(dx * dx + dy * dy + dz * dz));
        }
    red[threadIdx.x] = r;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) rad[b] = red[0];
}

// Moment table: for every sorted panel k in leaf box b(k),
//   Q_k = int_{S_k} conj(Rn_m((y - c_b)/h_b)) dy  in real storage,
// exact with an n x n conical Gauss rule for degree <= 2n - 2 >= p.
template <int P>
__global__ void k_moments(int64_t N, const double *__restrict__ pv, const int32_t *__restrict__ panel_leaf,
                          const int32_t *__restrict__ leaf_box, const double *__restrict__ center,
                          const double *__restrict__ hbox, const double *__restrict__ area, int nq,
                          const double *__restrict__ gx, const double *__restrict__ gw, double *__restrict__ mom64,
                          float *__restrict__ mom32)
{
    constexpr int K = (P + 1) * (P + 1);
    constexpr int NC = (P + 1) * (P + 2) / 2;
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k >= N) return;
    const int32_t b = leaf_box[panel_leaf[k]];
    const double ih = 1.0 / hbox[b];
    double v[9];
    for (int i = 0; i < 9; ++i) v[i] = pv[9 * k + i];
    double acc[K];
    for (int i = 0; i < K; ++i) acc[i] = 0;
    const double A2 = 2.0 * area[k];
    double re[NC], im[NC];
    for (int i = 0; i < nq; ++i)
        for (int j = 0; j < nq; ++j) {
            const double s = gx[i], t = gx[j];
            const double w = gw[i] * gw[j] * A2 * s;
            double u[3];
            for (int d = 0; d < 3; ++d)
                u[d] = (v[d] + s * (v[3 + d] - v[d]) + s * t * (v[6 + d] - v[3 + d]) - center[3 * b + d]) * ih;
            regular_harmonics<P, double>(u[0], u[1], u[2], re, im);
            for (int n = 0; n <= P; ++n) {
                acc[ridx(n, 0, 0)] += w * re[n * (n + 1) / 2];
                for (int m = 1; m <= n; ++m) {
                    acc[ridx(n, m, 0)] += w * re[n * (n + 1) / 2 + m];
                    acc[ridx(n, m, 1)] -= w * im[n * (n + 1) / 2 + m];
                }
            }
        }
    for (int i = 0; i < K; ++i) {
        mom64[(size_t)k * K + i] = acc[i];
        mom32[(size_t)k * K + i] = (float)acc[i];
    }
}

// Operator layouts, from the padded FP64 tables pad[op][KP][KK] (row =
// output coefficient) on the device; one thread per output element.
//   fragment order (16x16x4 MFMA A operand): [op][rt][ks][lane],
//     lane = row % 16 + 16 (k % 4), row = 16 rt + lane % 16, k = 4 ks + lane / 16
//   k-major (vector ALU): [op][k][row]
//   vector fragment order: [op][rt][ks / vec][lane][ks % vec], zero past the
//     last k step
//   last row (K - 1) by k lane group: [op][kq][ks] padded to a multiple of vec
template <typename TO>
__global__ void k_lay_frag(const double *__restrict__ pad, int64_t n, int KP, int KK, TO *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int nks = KK / 4, nrt = KP / 16;
    const int lane = (int)(i & 63);
    const int64_t q = i >> 6;
    const int ks = (int)(q % nks), rt = (int)((q / nks) % nrt);
    const int64_t c = q / ((int64_t)nks * nrt);
    out[i] = (TO)pad[(c * KP + rt * 16 + (lane & 15)) * KK + 4 * ks + (lane >> 4)];
}

template <typename TO>
__global__ void k_lay_kmaj(const double *__restrict__ pad, int64_t n, int KP, int KK, TO *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int r = (int)(i % KP), k = (int)((i / KP) % KK);
    const int64_t c = i / ((int64_t)KP * KK);
    out[i] = (TO)pad[(c * KP + r) * KK + k];
}

template <typename TO>
__global__ void k_lay_vec(const double *__restrict__ pad, int64_t n, int KP, int KK, int vec, TO *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int nks = KK / 4, nrt = KP / 16, nkv = (nks + vec - 1) / vec;
    const int e = (int)(i % vec);
    const int lane = (int)((i / vec) & 63);
    const int64_t q = i / vec / 64;
    const int kv = (int)(q % nkv), rt = (int)((q / nkv) % nrt);
    const int64_t c = q / ((int64_t)nkv * nrt);
    const int ks = kv * vec + e;
    out[i] = ks < nks ? (TO)pad[(c * KP + rt * 16 + (lane & 15)) * KK + 4 * ks + (lane >> 4)] : TO(0);
}

template <typename TO>
__global__ void k_lay_last(const double *__restrict__ pad, int64_t n, int KP, int KK, int K, int vec,
                           TO *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int nks = KK / 4, w = ((nks + vec - 1) / vec) * vec;
    const int ks = (int)(i % w), kq = (int)((i / w) % 4);
    const int64_t c = i / ((int64_t)w * 4);
    out[i] = ks < nks ? (TO)pad[(c * KP + K - 1) * KK + 4 * ks + kq] : TO(0);
}

__global__ void k_to_f32(const double *__restrict__ in, int64_t n, float *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)in[i];
}

__global__ void k_fill(int32_t *__restrict__ p, int64_t n, int32_t v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// elem_panel_t (NULL for a tree of triangles): element -> panel of the tree;
// the two elements of a four-sided panel are consecutive in input order, the
// first goes to iperm, the second to iperm2.
__global__ void k_concat_panels(int64_t n, int64_t off, int32_t user_off, int32_t vid_off,
                                const int32_t *__restrict__ perm_t, const int32_t *__restrict__ elem_panel_t,
                                const double *__restrict__ pv_t, const int32_t *__restrict__ pvid_t,
                                const double *__restrict__ cen_t, const double *__restrict__ area_t,
                                const double *__restrict__ diam_t, int32_t *__restrict__ perm,
                                int32_t *__restrict__ iperm, int32_t *__restrict__ iperm2, double *__restrict__ pv,
                                int32_t *__restrict__ pvid, double *__restrict__ cen, double *__restrict__ area,
                                double *__restrict__ diam)
{
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t g = off + i;
    const int32_t oe = perm_t[i];
    if (elem_panel_t) {
        const int32_t up = elem_panel_t[oe];
        const int32_t u = user_off + up;
        perm[g] = u;
        if (oe > 0 && elem_panel_t[oe - 1] == up)
            iperm2[u] = (int32_t)g;
        else
            iperm[u] = (int32_t)g;
    } else {
        const int32_t u = user_off + oe;
        perm[g] = u;
        iperm[u] = (int32_t)g;
    }
    for (int j = 0; j < 9; ++j) pv[9 * g + j] = pv_t[9 * i + j];
    for (int j = 0; j < 3; ++j) {
        pvid[3 * g + j] = vid_off + pvid_t[3 * i + j];
        cen[3 * g + j] = cen_t[3 * i + j];
    }
    area[g] = area_t[i];
    diam[g] = diam_t[i];
}

__global__ void k_panel_leaf(int64_t nleaf, const int32_t *__restrict__ leaf_box, const int32_t *__restrict__ beg,
                             const int32_t *__restrict__ end, int32_t *__restrict__ panel_leaf)
{
    int64_t li = blockIdx.x;
    if (li >= nleaf) return;
    const int32_t b = leaf_box[li];
    for (int32_t k = beg[b] + threadIdx.x; k < end[b]; k += blockDim.x) panel_leaf[k] = (int32_t)li;
}

// M2L offset slot (ox+3) + 7 (oy+3) + 49 (oz+3) -> index of the offset
// (|ox|, |oy|, |oz|) in the 64-entry table of non-negative offsets, shifted
// left by 3, with the reflection bits (1: x, 2: y, 4: z) of the signs.
static int32_t m2l_reflected_code(int32_t slot)
{
    const int ox = slot % 7 - 3, oy = (slot / 7) % 7 - 3, oz = slot / 49 - 3;
    const int canon = std::abs(ox) + 4 * std::abs(oy) + 16 * std::abs(oz);
    return canon << 3 | (ox < 0 ? 1 : 0) | (oy < 0 ? 2 : 0) | (oz < 0 ? 4 : 0);
}

// ---------------------------------------------------------------- passes
// A translation pass from its (target, source, operator) triples, grouped
// by target (targets ascending, the pairs of a target contiguous), built on
// the device:
//   operator order (offset-stationary kernels): the triples stably sorted by
//     operator, the groups of one operator, and each pair's sorted position;
//   target order (target-stationary kernels): the runs of one target, the
//     pairs of each run stably sorted by reflection bits (so the
//     accumulator of a reflected table changes frame at most seven times
//     per target), the runs of one source in that order, and the targets
//     with the most pairs first (ties in target order).

// flag[j] = 1 where a[j] starts a run of equal values
__global__ void k_run_flags(int64_t n, const int32_t *__restrict__ a, int32_t *__restrict__ flag)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j < n) flag[j] = (j == 0 || a[j] != a[j - 1]) ? 1 : 0;
}

// beg[pos[j]] = j for every run start j, and beg[runs] = n
__global__ void k_run_starts(int64_t n, const int32_t *__restrict__ flag, const int32_t *__restrict__ pos,
                             int32_t *__restrict__ beg)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    if (flag[j]) beg[pos[j]] = (int32_t)j;
    if (j == n - 1) beg[pos[j] + flag[j]] = (int32_t)n;
}

// out[i] = a[idx[i]]
__global__ void k_gather_i32(int64_t n, const int32_t *__restrict__ idx, const int32_t *__restrict__ a,
                             int32_t *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) out[i] = a[idx[i]];
}

__global__ void k_code_keys(int64_t n, const int32_t *__restrict__ code, uint64_t *__restrict__ key,
                            int32_t *__restrict__ idx)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    key[j] = (uint64_t)code[j];
    idx[j] = (int32_t)j;
}

// operator order: sorted source, operator and position of every pair
__global__ void k_pass_osort(int64_t n, const int32_t *__restrict__ ord, const int32_t *__restrict__ src,
                             const int32_t *__restrict__ code, int32_t *__restrict__ osrc,
                             int32_t *__restrict__ ocode, int32_t *__restrict__ slot)
{
    const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int32_t o = ord[j];
    osrc[j] = src[o];
    ocode[j] = code[o];
    slot[o] = (int32_t)j;
}

// target order: one thread per target run [rp[i], rp[i+1]), its pairs by
// reflection bits (eight stable passes over the run)
__global__ void k_pass_tsort(int64_t nrun, const int32_t *__restrict__ rp, const int32_t *__restrict__ rt,
                             const int32_t *__restrict__ src, const int32_t *__restrict__ code,
                             const int32_t *__restrict__ ts_code, int32_t *__restrict__ tsrc,
                             int32_t *__restrict__ tcode, int32_t *__restrict__ ttgt,
                             int32_t *__restrict__ tfull)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nrun) return;
    const int32_t a = rp[i], b = rp[i + 1], t = rt[i];
    int32_t p = a;
    for (int f = 0; f < 8; ++f)
        for (int32_t j = a; j < b; ++j) {
            const int32_t c8 = ts_code ? ts_code[j] : code[j] << 3;
            if ((c8 & 7) != f) continue;
            tsrc[p] = src[j];
            tcode[p] = c8;
            ttgt[p] = t;
            if (tfull) tfull[p] = code[j] << 3;
            ++p;
        }
}

// pairs per run and their maximum
__global__ void k_run_counts(int64_t nrun, const int32_t *__restrict__ rp, int32_t *__restrict__ cnt,
                             int32_t *__restrict__ maxc)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nrun) return;
    const int32_t c = rp[i + 1] - rp[i];
    cnt[i] = c;
    atomicMax(maxc, c);
}

__global__ void k_heavy_keys(int64_t nrun, const int32_t *__restrict__ cnt, const int32_t *__restrict__ maxc,
                             uint64_t *__restrict__ key, int32_t *__restrict__ idx)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nrun) return;
    key[i] = (uint64_t)(*maxc - cnt[i]);
    idx[i] = (int32_t)i;
}

static int bit_width(uint64_t v)
{
    int b = 0;
    while (v >> b) ++b;
    return std::max(b, 1);
}

// Starts of the runs of equal values of a[0..n) into beg (n + 1 entries,
// the first runs + 1 used); returns the number of runs.
static int64_t run_starts(const int32_t *a, int64_t n, DevBuf<int32_t> &beg, hipStream_t s)
{
    DevBuf<int32_t> flag(n), pos(n), tot(1);
    k_run_flags<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(n, a, flag.p);
    XRL_HIP(hipGetLastError());
    exclusive_scan<int32_t, int32_t>(flag.p, n, pos.p, tot.p, s);
    beg.alloc(n + 1);
    k_run_starts<<<(unsigned)cdiv(n, 256), 256, 0, s>>>(n, flag.p, pos.p, beg.p);
    XRL_HIP(hipGetLastError());
    return tot.download(s)[0];
}

// The pass of n triples (device arrays tgt, src, code; ts_code: operator
// code of each pair for the target-stationary kernel, or null for code << 3,
// no reflection); ncode bounds the codes.
static void build_pass(TransPass &T, int64_t n, const int32_t *tgt, const int32_t *src, const int32_t *code,
                       int ncode, hipStream_t s, const int32_t *ts_code = nullptr)
{
    T.n_pairs = n;
    T.n_groups = T.n_red = T.n_ps = 0;
    T.h_gbeg.assign(1, 0);
    if (n == 0) return;
    XRL_CHECK(n < (int64_t(1) << 31), XRL_E_UNSUPPORTED, "xrl_fmm_plan: a translation pass of %lld pairs",
              (long long)n);
    const unsigned g = (unsigned)cdiv(n, 256);
    // operator order
    {
        DevBuf<uint64_t> key(n), ktmp(n);
        DevBuf<int32_t> ord(n), otmp(n), ocode(n);
        k_code_keys<<<g, 256, 0, s>>>(n, code, key.p, ord.p);
        XRL_HIP(hipGetLastError());
        radix_sort_pairs(key.p, ord.p, ktmp.p, otmp.p, n, bit_width((uint64_t)ncode), s);
        T.src.alloc(n);
        T.red_slot.alloc(n);
        k_pass_osort<<<g, 256, 0, s>>>(n, ord.p, src, code, T.src.p, ocode.p, T.red_slot.p);
        XRL_HIP(hipGetLastError());
        T.n_groups = run_starts(ocode.p, n, T.gbeg, s);
        T.goff.alloc(T.n_groups);
        k_gather_i32<<<(unsigned)cdiv(T.n_groups, 256), 256, 0, s>>>(T.n_groups, T.gbeg.p, ocode.p, T.goff.p);
        XRL_HIP(hipGetLastError());
        T.h_gbeg = T.gbeg.download(s, T.n_groups + 1);
    }
    // target order
    T.n_red = run_starts(tgt, n, T.red_ptr, s);
    const int64_t nr = T.n_red;
    const unsigned gr = (unsigned)cdiv(nr, 256);
    T.red_tgt.alloc(nr);
    k_gather_i32<<<gr, 256, 0, s>>>(nr, T.red_ptr.p, tgt, T.red_tgt.p);
    XRL_HIP(hipGetLastError());
    T.ts_src.alloc(n);
    T.ts_op.alloc(n);
    T.ts_tgt.alloc(n);
    if (ts_code)
        T.ts_op_full.alloc(n);
    else
        T.ts_op_full.release();
    k_pass_tsort<<<gr, 256, 0, s>>>(nr, T.red_ptr.p, T.red_tgt.p, src, code, ts_code, T.ts_src.p, T.ts_op.p,
                                    T.ts_tgt.p, ts_code ? T.ts_op_full.p : nullptr);
    XRL_HIP(hipGetLastError());
    T.n_ps = run_starts(T.ts_src.p, n, T.ps_beg, s);
    // targets with the most pairs first, ties in target order
    DevBuf<int32_t> cnt(nr), maxc(1), hidx(nr), htmp(nr);
    DevBuf<uint64_t> hkey(nr), hktmp(nr);
    XRL_HIP(hipMemsetAsync(maxc.p, 0, sizeof(int32_t), s));
    k_run_counts<<<gr, 256, 0, s>>>(nr, T.red_ptr.p, cnt.p, maxc.p);
    XRL_HIP(hipGetLastError());
    const int32_t mc = maxc.download(s)[0];
    k_heavy_keys<<<gr, 256, 0, s>>>(nr, cnt.p, maxc.p, hkey.p, hidx.p);
    XRL_HIP(hipGetLastError());
    radix_sort_pairs(hkey.p, hidx.p, hktmp.p, htmp.p, nr, bit_width((uint64_t)mc), s);
    T.ts_order = std::move(hidx);
}

// M2L offset slot (ox+3) + 7 (oy+3) + 49 (oz+3) of every V-list pair -> the
// code of the target-stationary kernel: index of the offset (|ox|, |oy|,
// |oz|) in the 64-entry table of non-negative offsets, shifted left by 3,
// with the reflection bits (1: x, 2: y, 4: z) of the signs.
__global__ void k_m2l_pairs(int64_t B, const int64_t *__restrict__ voff, const int32_t *__restrict__ vsrc,
                            const int32_t *__restrict__ vcode, const double *__restrict__ center,
                            const double *__restrict__ rad, int32_t *__restrict__ tgt, int32_t *__restrict__ rcode,
                            double *__restrict__ ratio, unsigned long long *__restrict__ max_ratio_bits)
{
    const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b >= B) return;
    double mx = 0;
    for (int64_t j = voff[b]; j < voff[b + 1]; ++j) {
        tgt[j] = (int32_t)b;
        const int32_t slot = vcode[j];
        const int ox = slot % 7 - 3, oy = (slot / 7) % 7 - 3, oz = slot / 49 - 3;
        const int canon = abs(ox) + 4 * abs(oy) + 16 * abs(oz);
        rcode[j] = canon << 3 | (ox < 0 ? 1 : 0) | (oy < 0 ? 2 : 0) | (oz < 0 ? 4 : 0);
        const int32_t sb = vsrc[j];
        double d2 = 0;
        for (int d = 0; d < 3; ++d) {
            const double dd = center[3 * b + d] - center[3 * (int64_t)sb + d];
            d2 += dd * dd;
        }
        const double r = (rad[b] + rad[sb]) / sqrt(d2);
        ratio[j] = r;
        mx = fmax(mx, r);
    }
    // non-negative doubles order as their bit patterns
    if (mx > 0) atomicMax(max_ratio_bits, (unsigned long long)__double_as_longlong(mx));
}

// M2M pairs of one level (parent b <- child, operator: the child's octant),
// from each parent's first position pos[b - lo]
__global__ void k_m2m_pairs(int32_t lo, int32_t nb, const int32_t *__restrict__ child0,
                            const int32_t *__restrict__ nchild, const int32_t *__restrict__ octant,
                            const int32_t *__restrict__ pos, int32_t *__restrict__ tgt, int32_t *__restrict__ src,
                            int32_t *__restrict__ code)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    const int32_t b = lo + i;
    for (int32_t c = 0; c < nchild[b]; ++c) {
        const int32_t ch = child0[b] + c;
        tgt[pos[i] + c] = b;
        src[pos[i] + c] = ch;
        code[pos[i] + c] = octant[ch];
    }
}

// flag[i] = 1 for the boxes lo + i with children
__global__ void k_inner_flags(int32_t lo, int32_t nb, const int32_t *__restrict__ nchild, int32_t *__restrict__ flag)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nb) flag[i] = nchild[lo + i] > 0 ? 1 : 0;
}

// L2L pairs of the boxes with children of one level, in box order
__global__ void k_l2l_inner_pairs(int32_t lo, int32_t nb, const int32_t *__restrict__ flag,
                                  const int32_t *__restrict__ pos, const int32_t *__restrict__ parent,
                                  const int32_t *__restrict__ octant, int32_t *__restrict__ tgt,
                                  int32_t *__restrict__ src, int32_t *__restrict__ code)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb || !flag[i]) return;
    tgt[pos[i]] = lo + i;
    src[pos[i]] = parent[lo + i];
    code[pos[i]] = octant[lo + i];
}

// Moment rows through the L2L operator: out[t][j] = (1/h) sum_i Q[t][i] w_i
// T_o[i][j] for the panels t of a leaf at level >= 3 (o: the leaf's
// octant, w_i = 1 for the m = 0 coefficient of each degree, 2 otherwise),
// zero for the others.  L2P of the leaf's panels then adds
// sum_j out[t][j] L_parent[j], which is L2P of T_o L_parent.
__global__ void k_mom_l2l(int64_t N, int K, const int32_t *__restrict__ panel_leaf,
                          const int32_t *__restrict__ leaf_box, const int32_t *__restrict__ box_level,
                          const int32_t *__restrict__ box_octant, const double *__restrict__ box_h,
                          const double *__restrict__ mom, const double *__restrict__ l2l, float *__restrict__ out)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= N * K) return;
    const int64_t t = e / K;
    const int j = (int)(e - t * K);
    const int32_t b = leaf_box[panel_leaf[t]];
    if (box_level[b] < 3) {
        out[e] = 0.f;
        return;
    }
    const double *T = l2l + (int64_t)box_octant[b] * K * K;
    const double *q = mom + t * K;
    double acc = 0;
    for (int n = 0, i = 0; i < K; ++n)
        for (int m = 0; m <= 2 * n; ++m, ++i) acc += q[i] * (m == 0 ? 1.0 : 2.0) * T[(int64_t)i * K + j];
    out[e] = (float)(acc / box_h[b]);
}

// L2L pairs of one level (child b <- its parent, operator: the octant of b)
__global__ void k_l2l_pairs(int32_t lo, int32_t nb, const int32_t *__restrict__ parent,
                            const int32_t *__restrict__ octant, int32_t *__restrict__ tgt, int32_t *__restrict__ src,
                            int32_t *__restrict__ code)
{
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    tgt[i] = lo + i;
    src[i] = parent[lo + i];
    code[i] = octant[lo + i];
}

}  // namespace xrl

using namespace xrl;

// fn(i, scratch) for i in [0, n) on up to 16 host threads, each with its own
// scratch vector of `scratch` doubles; the calls are independent.
template <class F>
static void for_each_parallel(int n, F fn, size_t scratch)
{
    const int nt = std::max(1, std::min<int>({n, 16, (int)std::thread::hardware_concurrency()}));
    std::atomic<int> next{0};
    std::mutex mu;
    std::exception_ptr err;  // the first failure, rethrown on the calling thread
    auto work = [&] {
        try {
            std::vector<double> buf(scratch);
            for (int i = next++; i < n; i = next++) fn(i, buf);
        } catch (...) {
            std::lock_guard<std::mutex> lk(mu);
            if (!err) err = std::current_exception();
            next = n;
        }
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(work);
    work();
    for (auto &th : pool) th.join();
    if (err) std::rethrow_exception(err);
}

static void build_plan(xrl_plan *P, hipStream_t s)
{
    const int ntrees = (int)P->trees.size();
    // ---------------- global panels
    P->panel_off.assign(ntrees + 1, 0);
    P->user_off.assign(ntrees + 1, 0);
    std::vector<int64_t> vid_off(ntrees + 1, 0);
    bool hybrid = false;
    for (int t = 0; t < ntrees; ++t) {
        P->panel_off[t + 1] = P->panel_off[t] + P->trees[t]->N;
        P->user_off[t + 1] = P->user_off[t] + P->trees[t]->Np;
        vid_off[t + 1] = vid_off[t] + P->trees[t]->nv;
        hybrid |= P->trees[t]->elem_panel.p != nullptr;
    }
    XRL_CHECK(P->panel_off[ntrees] < (int64_t(1) << 31) && vid_off[ntrees] < (int64_t(1) << 31), XRL_E_UNSUPPORTED,
              "xrl_fmm_plan: more than 2^31 panels or vertices in one plan");
    const int64_t N = P->N = P->panel_off[ntrees];
    const int64_t Nu = P->Nu = P->user_off[ntrees];
    P->perm.alloc(N);
    P->iperm.alloc(Nu);
    if (hybrid) {
        P->iperm2.alloc(Nu);
        k_fill<<<cdiv(Nu, 256), 256, 0, s>>>(P->iperm2.p, Nu, -1);
        XRL_HIP(hipGetLastError());
    } else {
        P->iperm2.release();
    }
    P->pv.alloc(9 * N);
    P->pvid.alloc(3 * N);
    P->cen.alloc(3 * N);
    P->area.alloc(N);
    P->diam.alloc(N);
    for (int t = 0; t < ntrees; ++t) {
        const xrl_tree *T = P->trees[t];
        k_concat_panels<<<cdiv(T->N, 256), 256, 0, s>>>(T->N, P->panel_off[t], (int32_t)P->user_off[t],
                                                        (int32_t)vid_off[t], T->perm.p, T->elem_panel.p, T->pv.p,
                                                        T->pvid.p, T->cen.p, T->area.p, T->diam.p, P->perm.p,
                                                        P->iperm.p, P->iperm2.p, P->pv.p, P->pvid.p, P->cen.p,
                                                        P->area.p, P->diam.p);
        XRL_HIP(hipGetLastError());
    }
    // ---------------- global boxes, level-major across trees
    int depth = 0;
    for (auto *T : P->trees) depth = std::max(depth, T->depth);
    P->depth = depth;
    std::vector<std::vector<int32_t>> newid(ntrees);
    std::vector<int64_t> seg((depth + 1) * (ntrees + 1), 0);
    int64_t B = 0;
    P->level_off.assign(depth + 2, 0);
    for (int l = 0; l <= depth; ++l) {
        P->level_off[l] = B;
        for (int t = 0; t < ntrees; ++t) {
            const xrl_tree *T = P->trees[t];
            if (newid[t].empty()) newid[t].assign(T->box_key.size(), -1);
            seg[l * (ntrees + 1) + t] = B;
            if (l <= T->depth)
                for (int64_t b = T->level_off[l]; b < T->level_off[l + 1]; ++b) newid[t][b] = (int32_t)B++;
        }
        seg[l * (ntrees + 1) + ntrees] = B;
    }
    P->level_off[depth + 1] = B;
    P->B = B;
    std::vector<uint64_t> key(B);
    std::vector<int32_t> level(B), parent(B), child0(B), nchild(B), beg(B), end(B), tree(B);
    std::vector<double> center(3 * B), hsz(B);
    for (int t = 0; t < ntrees; ++t) {
        const xrl_tree *T = P->trees[t];
        for (size_t b = 0; b < T->box_key.size(); ++b) {
            const int32_t g = newid[t][b];
            key[g] = T->box_key[b];
            level[g] = T->box_level[b];
            parent[g] = T->box_parent[b] >= 0 ? newid[t][T->box_parent[b]] : -1;
            child0[g] = T->box_child0[b] >= 0 ? newid[t][T->box_child0[b]] : -1;
            nchild[g] = T->box_nchild[b];
            beg[g] = (int32_t)(P->panel_off[t] + T->box_beg[b]);
            end[g] = (int32_t)(P->panel_off[t] + T->box_end[b]);
            tree[g] = t;
            const double h = T->root_size / double(1 << level[g]);
            hsz[g] = h;
            const uint64_t k = key[g];
            const uint32_t c[3] = {compact3(k), compact3(k >> 1), compact3(k >> 2)};
            for (int d = 0; d < 3; ++d) center[3 * g + d] = T->root_c[d] - 0.5 * T->root_size + (c[d] + 0.5) * h;
        }
    }
    P->h_box_beg = beg;
    P->h_box_end = end;
    P->h_box_parent = parent;
    P->h_box_child0 = child0;
    P->h_box_nchild = nchild;
    P->h_box_level = level;
    P->h_box_tree = tree;
    std::vector<int32_t> leaves, octant(B);
    for (int64_t b = 0; b < B; ++b) {
        octant[b] = (int32_t)(key[b] & 7);
        if (nchild[b] == 0) {
            leaves.push_back((int32_t)b);
            XRL_CHECK(end[b] - beg[b] <= kMaxLeaf, XRL_E_UNSUPPORTED,
                      "xrl_fmm_plan: a leaf holds %d > %d panels (coincident centroids at max depth)",
                      end[b] - beg[b], kMaxLeaf);
        }
    }
    P->h_leaf_box = leaves;
    P->n_leaves = (int64_t)leaves.size();
    DevBuf<uint64_t> dkey;
    dkey.upload(key, s);
    DevBuf<int32_t> dtree;
    dtree.upload(tree, s);
    DevBuf<int64_t> dseg;
    dseg.upload(seg, s);
    P->box_level.upload(level, s);
    P->box_parent.upload(parent, s);
    P->box_child0.upload(child0, s);
    P->box_nchild.upload(nchild, s);
    P->box_beg.upload(beg, s);
    P->box_end.upload(end, s);
    P->box_octant.upload(octant, s);
    P->box_center.upload(center, s);
    P->box_h.upload(hsz, s);
    P->leaf_box.upload(leaves, s);
    P->box_rad.alloc(B);
    k_box_radius<<<B, 256, 0, s>>>(B, P->box_beg.p, P->box_end.p, P->box_center.p, P->pv.p, P->box_rad.p);
    XRL_HIP(hipGetLastError());
    P->panel_leaf.alloc(N);
    k_panel_leaf<<<P->n_leaves, 64, 0, s>>>(P->n_leaves, P->leaf_box.p, P->box_beg.p, P->box_end.p,
                                             P->panel_leaf.p);
    XRL_HIP(hipGetLastError());
    BoxView bv{dkey.p, P->box_level.p, P->box_parent.p, P->box_child0.p, P->box_nchild.p, dtree.p, dseg.p, ntrees};
    // ---------------- colleagues
    DevBuf<int32_t> coll(27 * (size_t)B);
    k_colleagues<<<cdiv(B, 128), 128, 0, s>>>(bv, B, coll.p);
    XRL_HIP(hipGetLastError());
    // ---------------- V lists (and pairs demoted to the near field)
    DevBuf<int32_t> vcnt(B), dcnt(B);
    const double theta = P->theta;
    k_vlist<<<cdiv(B, 128), 128, 0, s>>>(bv, B, coll.p, P->box_center.p, P->box_rad.p, theta, vcnt.p, dcnt.p,
                                         nullptr, nullptr, nullptr, nullptr, nullptr);
    XRL_HIP(hipGetLastError());
    DevBuf<int64_t> dvoff(B + 1), ddoff(B + 1), vtot(1), dtot(1);
    exclusive_scan<int32_t, int64_t>(vcnt.p, B, dvoff.p, vtot.p, s);
    exclusive_scan<int32_t, int64_t>(dcnt.p, B, ddoff.p, dtot.p, s);
    XRL_HIP(hipMemcpyAsync(dvoff.p + B, vtot.p, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    XRL_HIP(hipMemcpyAsync(ddoff.p + B, dtot.p, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    const int64_t nV = vtot.download(s)[0], nD = dtot.download(s)[0];
    P->n_m2l = nV;
    P->n_demoted = nD;
    DevBuf<int32_t> vsrc(std::max<int64_t>(nV, 1)), vcode(std::max<int64_t>(nV, 1)), dsrc(std::max<int64_t>(nD, 1));
    k_vlist<<<cdiv(B, 128), 128, 0, s>>>(bv, B, coll.p, P->box_center.p, P->box_rad.p, theta, vcnt.p, dcnt.p,
                                         dvoff.p, ddoff.p, vsrc.p, vcode.p, dsrc.p);
    XRL_HIP(hipGetLastError());
    // ---------------- near lists (source boxes), then rows, all on the device
    const int64_t nl = P->n_leaves;
    for (int64_t li = 0; li < nl; ++li)
        XRL_CHECK(end[leaves[li]] - beg[leaves[li]] <= kMaxLeaf, XRL_E_UNSUPPORTED,
                  "xrl_fmm_plan: a leaf at the maximum depth holds %d panels (more than %d); "
                  "the mesh has (nearly) coincident panel centroids",
                  end[leaves[li]] - beg[leaves[li]], kMaxLeaf);
    DevBuf<int32_t> ncnt(std::max<int64_t>(nl, 1));
    k_nearlist<<<cdiv(nl, 64), 64, 0, s>>>(bv, P->leaf_box.p, nl, coll.p, ncnt.p, nullptr, nullptr);
    XRL_HIP(hipGetLastError());
    DevBuf<int64_t> dnoff(nl + 1), tot(1);
    exclusive_scan<int32_t, int64_t>(ncnt.p, nl, dnoff.p, tot.p, s);
    XRL_HIP(hipMemcpyAsync(dnoff.p + nl, tot.p, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    const int64_t n_nbox = tot.download(s)[0];
    DevBuf<int32_t> nbox(std::max<int64_t>(n_nbox, 1));
    k_nearlist<<<cdiv(nl, 64), 64, 0, s>>>(bv, P->leaf_box.p, nl, coll.p, ncnt.p, dnoff.p, nbox.p);
    XRL_HIP(hipGetLastError());
    // with the demoted pairs: boxes and rows per leaf
    DevBuf<int32_t> scnt(std::max<int64_t>(nl, 1)), nrow(std::max<int64_t>(nl, 1));
    k_leaf_sources<<<cdiv(nl, 64), 64, 0, s>>>(P->leaf_box.p, nl, P->box_parent.p, dnoff.p, nbox.p, ddoff.p, dsrc.p,
                                                P->box_beg.p, P->box_end.p, nullptr, scnt.p, nrow.p, nullptr);
    XRL_HIP(hipGetLastError());
    DevBuf<int64_t> soff(nl + 1), rows64(nl + 1);
    exclusive_scan<int32_t, int64_t>(scnt.p, nl, soff.p, tot.p, s);
    XRL_HIP(hipMemcpyAsync(soff.p + nl, tot.p, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    const int64_t n_sbox = tot.download(s)[0];
    DevBuf<int32_t> sbox(std::max<int64_t>(n_sbox, 1));
    k_leaf_sources<<<cdiv(nl, 64), 64, 0, s>>>(P->leaf_box.p, nl, P->box_parent.p, dnoff.p, nbox.p, ddoff.p, dsrc.p,
                                                P->box_beg.p, P->box_end.p, soff.p, scnt.p, nrow.p, sbox.p);
    XRL_HIP(hipGetLastError());
    exclusive_scan<int32_t, int64_t>(nrow.p, nl, rows64.p, tot.p, s);
    const int64_t n_rows = tot.download(s)[0];
    XRL_CHECK(n_rows < (int64_t(1) << 31), XRL_E_UNSUPPORTED, "xrl_fmm_plan: near-field row count overflows int32");
    std::vector<int64_t> h_rows64 = rows64.download(s, nl);
    std::vector<int32_t> rows_ptr(nl + 1);
    for (int64_t li = 0; li < nl; ++li) rows_ptr[li] = (int32_t)h_rows64[li];
    rows_ptr[nl] = (int32_t)n_rows;
    P->near_rows.upload(rows_ptr, s);
    P->near_src.alloc(std::max<int64_t>(n_rows, 1));
    k_leaf_rows<<<(unsigned)std::max<int64_t>(nl, 1), 256, 0, s>>>(nl, soff.p, sbox.p, P->box_beg.p, P->box_end.p,
                                                                    P->near_rows.p, P->near_src.p);
    XRL_HIP(hipGetLastError());
    // block padding and value offsets
    P->leaf_tpad.alloc(std::max<int64_t>(nl, 1));
    DevBuf<int64_t> nval(std::max<int64_t>(nl, 1)), npair(std::max<int64_t>(nl, 1)), tot2(1);
    k_leaf_blocks<<<cdiv(nl, 256), 256, 0, s>>>(nl, P->leaf_box.p, P->box_beg.p, P->box_end.p, nrow.p,
                                                P->leaf_tpad.p, nval.p, npair.p);
    XRL_HIP(hipGetLastError());
    P->near_val_off.alloc(nl + 1);
    exclusive_scan<int64_t, int64_t>(nval.p, nl, P->near_val_off.p, tot.p, s);
    XRL_HIP(hipMemcpyAsync(P->near_val_off.p + nl, tot.p, sizeof(int64_t), hipMemcpyDeviceToDevice, s));
    DevBuf<int64_t> pscan(std::max<int64_t>(nl, 1));
    exclusive_scan<int64_t, int64_t>(npair.p, nl, pscan.p, tot2.p, s);
    P->h_near_rows = rows_ptr;
    P->n_near_rows = n_rows;
    P->n_near_entries = tot.download(s)[0];
    P->n_near_pairs = tot2.download(s)[0];
    // ---------------- translation passes: M2L (all levels), M2M and L2L per
    // level, on the device
    {
        DevBuf<int32_t> mtgt(std::max<int64_t>(nV, 1)), mrc(std::max<int64_t>(nV, 1));
        DevBuf<unsigned long long> mx(1);
        P->m2l_ratio.alloc(std::max<int64_t>(nV, 1));
        XRL_HIP(hipMemsetAsync(mx.p, 0, sizeof(unsigned long long), s));
        k_m2l_pairs<<<cdiv(B, 128), 128, 0, s>>>(B, dvoff.p, vsrc.p, vcode.p, P->box_center.p, P->box_rad.p, mtgt.p,
                                                 mrc.p, P->m2l_ratio.p, mx.p);
        XRL_HIP(hipGetLastError());
        build_pass(P->m2l, nV, mtgt.p, vsrc.p, vcode.p, 343, s, mrc.p);
        const unsigned long long mb = mx.download(s)[0];
        double maxsep;
        std::memcpy(&maxsep, &mb, sizeof maxsep);
        P->max_sep_ratio = maxsep;
        // the pairs in per-target order, for export
        P->m2l_pair_t = std::move(mtgt);
        P->m2l_pair_s = std::move(vsrc);
        P->m2m.clear();
        P->l2l.clear();
        P->l2l_inner.clear();
        P->m2m.resize(depth + 1);
        P->l2l.resize(depth + 1);
        P->l2l_inner.resize(depth + 1);
        for (int l = 0; l <= depth; ++l) {
            const int32_t lo = (int32_t)P->level_off[l], nb = (int32_t)(P->level_off[l + 1] - P->level_off[l]);
            if (nb == 0) continue;
            // M2M: parent b <- each child
            DevBuf<int32_t> pos(nb), ptot(1);
            exclusive_scan<int32_t, int32_t>(P->box_nchild.p + lo, nb, pos.p, ptot.p, s);
            const int32_t n1 = ptot.download(s)[0];
            if (n1 > 0) {
                DevBuf<int32_t> t1(n1), s1(n1), c1(n1);
                k_m2m_pairs<<<cdiv(nb, 128), 128, 0, s>>>(lo, nb, P->box_child0.p, P->box_nchild.p, P->box_octant.p,
                                                          pos.p, t1.p, s1.p, c1.p);
                XRL_HIP(hipGetLastError());
                build_pass(P->m2m[l], n1, t1.p, s1.p, c1.p, 8, s);
            }
            // L2L: child b <- its parent (locals are zero above level 2); and
            // the same without the leaf targets
            if (l >= 3) {
                DevBuf<int32_t> t2(nb), s2(nb), c2(nb);
                k_l2l_pairs<<<cdiv(nb, 128), 128, 0, s>>>(lo, nb, P->box_parent.p, P->box_octant.p, t2.p, s2.p, c2.p);
                XRL_HIP(hipGetLastError());
                build_pass(P->l2l[l], nb, t2.p, s2.p, c2.p, 8, s);
                DevBuf<int32_t> flag(nb), ipos(nb), itot(1);
                k_inner_flags<<<cdiv(nb, 128), 128, 0, s>>>(lo, nb, P->box_nchild.p, flag.p);
                XRL_HIP(hipGetLastError());
                exclusive_scan<int32_t, int32_t>(flag.p, nb, ipos.p, itot.p, s);
                const int32_t ni = itot.download(s)[0];
                if (ni > 0) {
                    DevBuf<int32_t> t3(ni), s3(ni), c3(ni);
                    k_l2l_inner_pairs<<<cdiv(nb, 128), 128, 0, s>>>(lo, nb, flag.p, ipos.p, P->box_parent.p,
                                                                    P->box_octant.p, t3.p, s3.p, c3.p);
                    XRL_HIP(hipGetLastError());
                    build_pass(P->l2l_inner[l], ni, t3.p, s3.p, c3.p, 8, s);
                }
            }
        }
    }
    std::vector<int32_t> grp_off;
    if (P->m2l.n_groups > 0) grp_off = P->m2l.goff.download(s, P->m2l.n_groups);
    // ---------------- operators
    const int p = P->p, K = P->K;
    std::vector<double> m2m(8 * (size_t)K * K), l2l(8 * (size_t)K * K);
    build_m2m(p, m2m.data());
    build_l2l(p, l2l.data());
    P->KP = (int)cdiv(K, 16) * 16;
    P->KK = (int)cdiv(K, 4) * 4;
    std::vector<double> m2l(343 * (size_t)P->KP * P->KK, 0.0);
    std::vector<int> used_codes;
    {
        std::vector<char> used(343, 0);
        for (int c : grp_off) used[c] = 1;
        for (int c = 0; c < 343; ++c)
            if (used[c]) used_codes.push_back(c);
    }
    // the operators of the offsets in use, each an independent FP64
    // construction, on the host's cores
    for_each_parallel((int)used_codes.size(), [&](int i, std::vector<double> &scratch) {
        const int c = used_codes[i];
        const int ox = c % 7 - 3, oy = (c / 7) % 7 - 3, oz = c / 49 - 3;
        build_m2l(p, ox, oy, oz, scratch.data());
        for (int r = 0; r < K; ++r)
            for (int k = 0; k < K; ++k) m2l[((size_t)c * P->KP + r) * P->KK + k] = scratch[(size_t)r * K + k];
    }, (size_t)K * K);
    auto to32 = [](const std::vector<double> &v) {
        std::vector<float> f(v.size());
        for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
        return f;
    };
    const int nrt = P->KP / 16, nks = P->KK / 4;
    auto grid = [](int64_t n) { return (unsigned)cdiv(n, 256); };
    // fragment order and k-major order, FP64 and FP32, from a padded table
    // already on the device
    auto layouts = [&](const double *pad, int nop, DevBuf<double> &f64, DevBuf<float> &f32, DevBuf<double> &k64,
                       DevBuf<float> &k32) {
        const int64_t n = (int64_t)nop * P->KP * P->KK;
        f64.alloc(n);
        f32.alloc(n);
        k64.alloc(n);
        k32.alloc(n);
        k_lay_frag<double><<<grid(n), 256, 0, s>>>(pad, n, P->KP, P->KK, f64.p);
        k_lay_frag<float><<<grid(n), 256, 0, s>>>(pad, n, P->KP, P->KK, f32.p);
        k_lay_kmaj<double><<<grid(n), 256, 0, s>>>(pad, n, P->KP, P->KK, k64.p);
        k_lay_kmaj<float><<<grid(n), 256, 0, s>>>(pad, n, P->KP, P->KK, k32.p);
        XRL_HIP(hipGetLastError());
    };
    // vector fragment order (pairs of k steps in FP64, quads in FP32) and the
    // last-row tables
    auto vec_layouts = [&](const double *pad, int nop, DevBuf<double> &v64, DevBuf<float> &v32, DevBuf<double> &t64,
                           DevBuf<float> &t32) {
        for (int vec : {2, 4}) {
            const int nkv = (nks + vec - 1) / vec;
            const int64_t nt = (int64_t)nop * 4 * nkv * vec, nv = (int64_t)nop * nrt * nkv * 64 * vec;
            if (vec == 2) {
                t64.alloc(nt);
                v64.alloc(nv);
                k_lay_last<double><<<grid(nt), 256, 0, s>>>(pad, nt, P->KP, P->KK, K, vec, t64.p);
                k_lay_vec<double><<<grid(nv), 256, 0, s>>>(pad, nv, P->KP, P->KK, vec, v64.p);
            } else {
                t32.alloc(nt);
                v32.alloc(nv);
                k_lay_last<float><<<grid(nt), 256, 0, s>>>(pad, nt, P->KP, P->KK, K, vec, t32.p);
                k_lay_vec<float><<<grid(nv), 256, 0, s>>>(pad, nv, P->KP, P->KK, vec, v32.p);
            }
            XRL_HIP(hipGetLastError());
        }
    };
    auto padded = [&](const std::vector<double> &dense, int nop) {
        std::vector<double> out((size_t)nop * P->KP * P->KK, 0.0);
        for (int c = 0; c < nop; ++c)
            for (int r = 0; r < K; ++r)
                for (int k = 0; k < K; ++k)
                    out[((size_t)c * P->KP + r) * P->KK + k] = dense[((size_t)c * K + r) * K + k];
        return out;
    };
    P->op_m2m64.upload(m2m, s);
    P->op_l2l64.upload(l2l, s);
    P->op_m2l64.upload(m2l, s);  // padded [343][KP][KK]
    P->op_m2m32.upload(to32(m2m), s);
    P->op_l2l32.upload(to32(l2l), s);
    P->op_m2l32.alloc(P->op_m2l64.n);
    k_to_f32<<<grid((int64_t)P->op_m2l64.n), 256, 0, s>>>(P->op_m2l64.p, (int64_t)P->op_m2l64.n, P->op_m2l32.p);
    XRL_HIP(hipGetLastError());
    layouts(P->op_m2l64.p, 343, P->op_m2l64f, P->op_m2l32f, P->op_m2l64k, P->op_m2l32k);
    {
        // the non-negative offsets that some used offset reflects onto
        std::vector<double> m2lc(64 * (size_t)P->KP * P->KK, 0.0);
        std::vector<char> cu(64, 0);
        for (int c : grp_off) cu[m2l_reflected_code(c) >> 3] = 1;
        std::vector<int> canon;
        for (int c = 0; c < 64; ++c)
            if (cu[c]) canon.push_back(c);
        for_each_parallel((int)canon.size(), [&](int i, std::vector<double> &scratch) {
            const int c = canon[i];
            build_m2l(p, c % 4, (c / 4) % 4, c / 16, scratch.data());
            for (int r = 0; r < K; ++r)
                for (int k = 0; k < K; ++k) m2lc[((size_t)c * P->KP + r) * P->KK + k] = scratch[(size_t)r * K + k];
        }, (size_t)K * K);
        DevBuf<double> dm2lc;
        dm2lc.upload(m2lc, s);
        vec_layouts(dm2lc.p, 64, P->op_m2lc64v, P->op_m2lc32v, P->op_m2lc64t, P->op_m2lc32t);
        vec_layouts(P->op_m2l64.p, 343, P->op_m2l64v, P->op_m2l32v, P->op_m2l64t, P->op_m2l32t);
        DevBuf<double> pm2m, pl2l;
        pm2m.upload(padded(m2m, 8), s);
        pl2l.upload(padded(l2l, 8), s);
        vec_layouts(pm2m.p, 8, P->op_m2m64v, P->op_m2m32v, P->op_m2m64t, P->op_m2m32t);
        vec_layouts(pl2l.p, 8, P->op_l2l64v, P->op_l2l32v, P->op_l2l64t, P->op_l2l32t);
        layouts(pm2m.p, 8, P->op_m2m64f, P->op_m2m32f, P->op_m2m64k, P->op_m2m32k);
        layouts(pl2l.p, 8, P->op_l2l64f, P->op_l2l32f, P->op_l2l64k, P->op_l2l32k);
        XRL_HIP(hipStreamSynchronize(s));  // the padded staging tables are released here
    }
    // ---------------- moments
    const int nq = (p + 3) / 2;  // 2 nq - 2 >= p
    std::vector<double> gx(nq), gw(nq);
    gauss_legendre01(nq, gx.data(), gw.data());
    DevBuf<double> dgx, dgw;
    dgx.upload(gx, s);
    dgw.upload(gw, s);
    P->mom64.alloc((size_t)N * K);
    P->mom32.alloc((size_t)N * K);
#define XRL_MOM(PP)                                                                                          \
    case PP:                                                                                                 \
        k_moments<PP><<<cdiv(N, 64), 64, 0, s>>>(N, P->pv.p, P->panel_leaf.p, P->leaf_box.p, P->box_center.p, \
                                                 P->box_h.p, P->area.p, nq, dgx.p, dgw.p, P->mom64.p,      \
                                                 P->mom32.p);                                              \
        break;
    switch (p) {
        XRL_MOM(2)
        XRL_MOM(4)
        XRL_MOM(6)
        XRL_MOM(8)
        XRL_MOM(10)
        XRL_MOM(12)
        default: fail(XRL_E_UNSUPPORTED, "xrl_fmm_plan: order %d not compiled (2,4,6,8,10,12)", p);
    }
#undef XRL_MOM
    XRL_HIP(hipGetLastError());
    if (P->precision != XRL_PREC_FP64 && N > 0) {
        P->mom_l2l32.alloc((size_t)N * K);
        k_mom_l2l<<<(unsigned)cdiv(N * K, 256), 256, 0, s>>>(N, K, P->panel_leaf.p, P->leaf_box.p, P->box_level.p,
                                                             P->box_octant.p, P->box_h.p, P->mom64.p,
                                                             P->op_l2l64.p, P->mom_l2l32.p);
        XRL_HIP(hipGetLastError());
    } else {
        P->mom_l2l32.release();
    }
    XRL_HIP(hipStreamSynchronize(s));
}

extern "C" xrl_status xrl_fmm_plan(xrl_tree *const *trees, int32_t n_trees, const xrl_plan_opts *opts,
                                   void *stream, xrl_plan **out)
{
    return guarded([&] {
        XRL_CHECK(trees && opts && out && n_trees >= 1, XRL_E_INVALID_ARG, "xrl_fmm_plan: bad arguments");
        *out = nullptr;
        for (int t = 0; t < n_trees; ++t) XRL_CHECK(trees[t], XRL_E_INVALID_ARG, "xrl_fmm_plan: null tree %d", t);
        XRL_CHECK(opts->order >= 2 && opts->order <= 12 && opts->order % 2 == 0, XRL_E_UNSUPPORTED,
                  "xrl_fmm_plan: order must be even in 2..12 (got %d)", opts->order);
        XRL_CHECK(opts->precision >= 0 && opts->precision <= 2, XRL_E_INVALID_ARG, "xrl_fmm_plan: bad precision");
        XRL_CHECK(opts->m2l_engine >= 0 && opts->m2l_engine <= 4, XRL_E_INVALID_ARG, "xrl_fmm_plan: bad engine");
        XRL_CHECK(opts->max_cols >= 1 && opts->max_cols <= 4096, XRL_E_INVALID_ARG,
                  "xrl_fmm_plan: max_cols must be in 1..4096");
        XRL_CHECK(opts->theta == 0.0 || (opts->theta >= 0.5 && opts->theta <= 1.0), XRL_E_INVALID_ARG,
                  "xrl_fmm_plan: theta must be 0 (default) or in [0.5, 1] (got %g)", opts->theta);
        auto P = std::make_unique<xrl_plan>();
        P->p = opts->order;
        P->K = (P->p + 1) * (P->p + 1);
        P->precision = opts->precision;
        P->m2l_engine = opts->m2l_engine == XRL_M2L_AUTO
                            ? (opts->precision == XRL_PREC_FP32 ? XRL_M2L_VALU : XRL_M2L_MFMA)
                            : opts->m2l_engine;
        if (P->m2l_engine == XRL_M2L_VALU) {
            // the vector-ALU plan (the plain FP32 method) keeps every phase
            // off the matrix cores
            P->p2p_form = 2;
            P->leaf_mfma = 0;
        }
        P->max_cols = opts->max_cols;
        P->theta = opts->theta == 0.0 ? XRL_DEFAULT_THETA : opts->theta;
        P->trees.assign(trees, trees + n_trees);
        const AllocStream alloc_scope((hipStream_t)stream);
        build_plan(P.get(), (hipStream_t)stream);
        *out = P.release();
    });
}

extern "C" void xrl_plan_destroy(xrl_plan *plan)
{
    if (!plan) return;
    for (auto &set : plan->prof_ev)
        for (auto &e : set) (void)hipEventDestroy(e);
    if (plan->gexec) (void)hipGraphExecDestroy(plan->gexec);
    if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
    delete plan;
}

extern "C" xrl_status xrl_plan_get_info(const xrl_plan *P, xrl_plan_info *info)
{
    return guarded([&] {
        XRL_CHECK(P && info, XRL_E_INVALID_ARG, "xrl_plan_get_info: null argument");
        info->n_panels = P->Nu;
        info->n_elements = P->N;
        info->n_boxes = P->B;
        info->n_leaves = P->n_leaves;
        info->n_m2l_pairs = P->n_m2l;
        info->n_near_rows = P->n_near_rows;
        info->n_near_entries = P->n_near_entries;
        info->n_near_pairs = P->n_near_pairs;
        info->order = P->p;
        info->precision = P->precision;
        info->max_sep_ratio = P->max_sep_ratio;
        info->n_demoted_pairs = P->n_demoted;
        info->theta = P->theta;
    });
}

extern "C" xrl_status xrl_plan_export(const xrl_plan *P, int32_t item, void *buf, int64_t *nbytes)
{
    return guarded([&] {
        XRL_CHECK(P && nbytes, XRL_E_INVALID_ARG, "xrl_plan_export: null argument");
        std::vector<int32_t> v;
        switch (item) {
            case 0: v = const_cast<xrl_plan *>(P)->perm.download(0); break;
            case 1:
                v.resize(2 * P->B);
                for (int64_t b = 0; b < P->B; ++b) {
                    v[2 * b] = P->h_box_beg[b];
                    v[2 * b + 1] = P->h_box_end[b];
                }
                break;
            case 2: v = P->h_box_level; break;
            case 3: v = P->h_near_rows; break;
            case 4: v = const_cast<xrl_plan *>(P)->near_src.download(0); break;
            case 5: {
                const auto t = P->m2l_pair_t.download(0, P->n_m2l), src = P->m2l_pair_s.download(0, P->n_m2l);
                v.resize(2 * P->n_m2l);
                for (int64_t q = 0; q < P->n_m2l; ++q) {
                    v[2 * q] = t[q];
                    v[2 * q + 1] = src[q];
                }
                break;
            }
            case 6: v = P->h_leaf_box; break;
            case 7: v = P->h_box_parent; break;
            case 9: v = const_cast<xrl_plan *>(P)->leaf_tpad.download(0); break;
            case 8:
            case 10: {
                // near-field values as float64 (layout: items 3, 4, 9), or the
                // separation ratio of every M2L pair (order of item 5)
                std::vector<double> d;
                if (item == 10)
                    d = P->m2l_ratio.download(0, P->n_m2l);
                else if (P->near64.p)
                    d = const_cast<xrl_plan *>(P)->near64.download(0, P->n_near_entries);
                else {
                    auto f = const_cast<xrl_plan *>(P)->near32.download(0, P->n_near_entries);
                    d.assign(f.begin(), f.end());
                }
                const int64_t nb = (int64_t)(d.size() * sizeof(double));
                if (buf) {
                    XRL_CHECK(*nbytes >= nb, XRL_E_INVALID_ARG, "xrl_plan_export: buffer too small");
                    std::memcpy(buf, d.data(), nb);
                }
                *nbytes = nb;
                return;
            }
            default: fail(XRL_E_INVALID_ARG, "xrl_plan_export: unknown item %d", item);
        }
        const int64_t nb = (int64_t)(v.size() * sizeof(int32_t));
        if (buf) {
            XRL_CHECK(*nbytes >= nb, XRL_E_INVALID_ARG, "xrl_plan_export: buffer too small");
            std::memcpy(buf, v.data(), nb);
        }
        *nbytes = nb;
    });
}
