// Near-field assembly: the panel-panel entries P_kl of eq. (6) (second term,
// without j*omega*mu0/4pi) for every pair in the near lists, filled once and
// reused by every matvec (Sec. II-C, last paragraph; Sec. II-D).
//
// Pair classes (k target, l source, r = |c_k - c_l| / max(diam_k, diam_l)):
//   self          k == l: closed form of the double integral over a flat
//                 triangle, (4A^2/3) sum_e ln(Pr / (Pr - 2 l_e)) / l_e
//                 (Arcioni-Bressan-Perregrini 1997, Eibert-Hansen 1995).
//   touching      a shared vertex: outer tensor Gauss rule on S_k in coordinates
//                 collapsed at the shared vertex, both directions through the
//                 sigmoidal map u^3/(u^3+(1-u)^3) (Sidi 1993); inner integral
//                 exact (potential of a uniform triangle, Wilton et al. 1984).
//   near-singular r < r_near: outer conical Gauss rule on 1, 4 or 16
//                 sub-triangles of S_k, inner integral exact.  Optionally the
//                 learned surrogate with quadrature fall-back.
//   regular       product of two triangle rules: in FP32 the symmetric rules
//                 of Dunavant (1985), 12 points (degree 6) below r_mid and
//                 6 points (degree 4) above; in FP64 conical Gauss rules,
//                 5x5 or 4x4 points.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "nfcommon.h"

namespace xrl {



template <typename T>
__device__ inline T dot3(const T *a, const T *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// int_{triangle v} 1/|r - r'| dS' for a uniform unit density (the closed form
// of Wilton et al. 1984), with the source geometry set up once per triangle
// and the edge terms in forms free of cancellation:
//   per edge (a -> b, unit direction s, length L, outward in-plane normal m):
//   t0 = (a - r).m, s- = (a - r).s, s+ = s- + L, R-/+ = |r - a|, |r - b|,
//   phi = sum t0 ln(f+/f-) - |h| sum [atan(t0 s+/(R0^2 + |h| R+)) - atan(t0 s-/(R0^2 + |h| R-))]
// with f = R + s (or R0^2/(R - s) behind the foot of r), R0^2 = t0^2 + h^2.
// ln(f+/f-) is taken as log1p of L (S + s- + s+)/(S (R- + s-)) (S = R- + R+)
// when both ends lie on the same side of the foot (the ratio tends to 1 far
// from the edge); the arc-tangent terms of the three edges add up to the
// solid angle of the triangle, taken at once.
template <typename T>
struct TriPot {
    T n[3], a[3][3], s[3][3], m[3][3], L[3];
    __device__ void init(const T *v)
    {
        T e1[3], e2[3];
        for (int d = 0; d < 3; ++d) {
            e1[d] = v[3 + d] - v[d];
            e2[d] = v[6 + d] - v[d];
        }
        n[0] = e1[1] * e2[2] - e1[2] * e2[1];
        n[1] = e1[2] * e2[0] - e1[0] * e2[2];
        n[2] = e1[0] * e2[1] - e1[1] * e2[0];
        const T inn = T(1) / sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        for (int d = 0; d < 3; ++d) n[d] *= inn;
        for (int i = 0; i < 3; ++i) {
            const T *p = v + 3 * i, *q = v + 3 * ((i + 1) % 3);
            T e[3] = {q[0] - p[0], q[1] - p[1], q[2] - p[2]};
            L[i] = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
            const T il = T(1) / L[i];
            for (int d = 0; d < 3; ++d) {
                a[i][d] = p[d];
                s[i][d] = e[d] * il;
            }
            m[i][0] = s[i][1] * n[2] - s[i][2] * n[1];
            m[i][1] = s[i][2] * n[0] - s[i][0] * n[2];
            m[i][2] = s[i][0] * n[1] - s[i][1] * n[0];
        }
    }
    __device__ T operator()(const T *r) const
    {
        const T eps = sizeof(T) == 4 ? T(1e-5) : T(1e-12);
        T dd[3][3], R[3];
        for (int i = 0; i < 3; ++i) {
            for (int d = 0; d < 3; ++d) dd[i][d] = a[i][d] - r[d];
            R[i] = sqrt(dd[i][0] * dd[i][0] + dd[i][1] * dd[i][1] + dd[i][2] * dd[i][2]);
        }
        const T h = -(n[0] * dd[0][0] + n[1] * dd[0][1] + n[2] * dd[0][2]);
        const T ah = fabs(h);
        T phi = 0;
        for (int i = 0; i < 3; ++i) {
            const T t0 = dd[i][0] * m[i][0] + dd[i][1] * m[i][1] + dd[i][2] * m[i][2];
            if (fabs(t0) <= eps * L[i]) continue;
            const T sm = dd[i][0] * s[i][0] + dd[i][1] * s[i][1] + dd[i][2] * s[i][2];
            const T sp = sm + L[i];
            const T Rm = R[i], Rp = R[(i + 1) % 3];
            const T R0s = t0 * t0 + h * h;
            const T S = Rm + Rp;
            // ln(f+/f-) = log1p(z), z >= 0 in all three cases (one
            // transcendental whichever side of the foot the edge lies on)
            T z;
            if (sm >= 0)
                z = L[i] * (S + sm + sp) / (S * (Rm + sm));
            else if (sp <= 0)
                z = L[i] * (S - sm - sp) / (S * (Rp - sp));
            else
                z = (Rp + sp) * (Rm - sm) / R0s - T(1);
            phi += t0 * log1p(z);
        }
        // the arc-tangent terms of the three edges sum to the solid angle of
        // the triangle seen from r: one atan2 (Van Oosterom and Strackee 1983)
        // (in the triangle's plane the term vanishes)
        const T *d0 = dd[0], *d1 = dd[1], *d2 = dd[2];
        const T num = d0[0] * (d1[1] * d2[2] - d1[2] * d2[1]) + d0[1] * (d1[2] * d2[0] - d1[0] * d2[2]) +
                      d0[2] * (d1[0] * d2[1] - d1[1] * d2[0]);
        const T den = R[0] * R[1] * R[2] + (d0[0] * d1[0] + d0[1] * d1[1] + d0[2] * d1[2]) * R[2] +
                      (d0[0] * d2[0] + d0[1] * d2[1] + d0[2] * d2[2]) * R[1] +
                      (d1[0] * d2[0] + d1[1] * d2[1] + d1[2] * d2[2]) * R[0];
        if (ah > eps * (L[0] + L[1] + L[2])) phi -= ah * fabs(T(2) * atan2(num, den));
        return phi;
    }
};

__device__ inline double self_term(const double *v)
{
    double l[3];
    for (int i = 0; i < 3; ++i) {
        const double *a = v + 3 * i, *b = v + 3 * ((i + 1) % 3);
        const double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
        l[i] = sqrt(dx * dx + dy * dy + dz * dz);
    }
    const double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
    const double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
    const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                 cz = e1[0] * e2[1] - e1[1] * e2[0];
    const double A = 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
    const double pr = l[0] + l[1] + l[2];
    double s = 0;
    for (int e = 0; e < 3; ++e) s += log(pr / (pr - 2 * l[e])) / l[e];
    return 4.0 * A * A / 3.0 * s;
}

template <typename T>
__device__ inline T tri_area2(const T *v)
{
    const T e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
    const T e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
    const T cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2], cz = e1[0] * e2[1] - e1[1] * e2[0];
    return sqrt(cx * cx + cy * cy + cz * cz);
}

// Touching pair: target vertices reordered so that tv[0] is a shared vertex
// and, when the panels share an edge (edge), tv[1] is its other end, so
// that the shared side is t = 0 of the collapsed coordinates.
template <typename T>
__device__ T touching_pair(const T *tv, const T *sv, const NFRules &R, bool edge)
{
    TriPot<T> pot;
    pot.init(sv);
    const T A2 = tri_area2(tv);
    T acc = 0;
    if (R.touch_graded) {
        const int ns = edge ? R.n_gse : R.n_gs;
        const double *sx = edge ? R.gse_x : R.gs_x, *sw = edge ? R.gse_w : R.gs_w;
        for (int i = 0; i < ns; ++i) {
            const T s = (T)sx[i];
            T inner = 0;
            for (int j = 0; j < R.n_gt; ++j) {
                const T t = (T)R.gt_x[j];
                T x[3];
                for (int d = 0; d < 3; ++d) x[d] = tv[d] + s * (tv[3 + d] - tv[d]) + s * t * (tv[6 + d] - tv[3 + d]);
                inner += (T)R.gt_w[j] * pot(x);
            }
            acc += (T)sw[i] * s * inner;
        }
        return acc * A2;
    }
    for (int i = 0; i < R.n_touch; ++i) {
        const T s = (T)R.tx[i];
        T inner = 0;
        for (int j = 0; j < R.n_touch; ++j) {
            const T t = (T)R.tx[j];
            T x[3];
            for (int d = 0; d < 3; ++d) x[d] = tv[d] + s * (tv[3 + d] - tv[d]) + s * t * (tv[6 + d] - tv[3 + d]);
            inner += (T)R.tw[j] * pot(x);
        }
        acc += (T)R.tw[i] * s * inner;
    }
    return acc * A2;
}

// Conical rule on triangle v with the potential of a source triangle.
template <typename T>
__device__ T conical_outer(const T *v, const TriPot<T> &pot, const NFRules &R, int c)
{
    const T A2 = tri_area2(v);
    T acc = 0;
    if (R.ns_sym[c]) {
        // symmetric rule: barycentric points, weights summing to one
        for (int q = 0; q < 16; ++q) {
            const double *b = R.ns16_b[q];
            T x[3];
            for (int d = 0; d < 3; ++d) x[d] = (T)b[0] * v[d] + (T)b[1] * v[3 + d] + (T)b[2] * v[6 + d];
            acc += (T)R.ns16_w[q] * pot(x);
        }
        return acc * A2 * T(0.5);
    }
    for (int i = 0; i < R.ns_n[c]; ++i) {
        const T s = (T)R.nx[c][i];
        T inner = 0;
        for (int j = 0; j < R.ns_n[c]; ++j) {
            const T t = (T)R.nx[c][j];
            T x[3];
            for (int d = 0; d < 3; ++d) x[d] = v[d] + s * (v[3 + d] - v[d]) + s * t * (v[6 + d] - v[3 + d]);
            inner += (T)R.nw[c][j] * pot(x);
        }
        acc += (T)R.nw[c][i] * s * inner;
    }
    return acc * A2;
}

// Near-singular pair of class c: the outer triangle split into 4^lev
// sub-triangles by midpoint subdivision (child c of (a,b,c): 0 corner a,
// 1 corner b, 2 corner c, 3 middle), the class's conical rule on each.
template <typename T>
__device__ T near_pair(const T *tv, const T *sv, int c, const NFRules &R)
{
    const int lev = R.ns_lev[c];
    TriPot<T> pot;
    pot.init(sv);
    T acc = 0;
    const int nsub = 1 << (2 * lev);
    for (int q = 0; q < nsub; ++q) {
        T v[9];
        for (int i = 0; i < 9; ++i) v[i] = tv[i];
        for (int l = lev - 1; l >= 0; --l) {
            const int c = (q >> (2 * l)) & 3;
            T m01[3], m12[3], m20[3];
            for (int d = 0; d < 3; ++d) {
                m01[d] = T(0.5) * (v[d] + v[3 + d]);
                m12[d] = T(0.5) * (v[3 + d] + v[6 + d]);
                m20[d] = T(0.5) * (v[6 + d] + v[d]);
            }
            for (int d = 0; d < 3; ++d) {
                if (c == 0) { v[3 + d] = m01[d]; v[6 + d] = m20[d]; }
                else if (c == 1) { v[d] = m01[d]; v[6 + d] = m12[d]; }
                else if (c == 2) { v[d] = m20[d]; v[3 + d] = m12[d]; }
                else { v[d] = m12[d]; v[3 + d] = m20[d]; v[6 + d] = m01[d]; }
            }
        }
        acc += conical_outer(v, pot, R, c);
    }
    return acc;
}

// Product of two NQ x NQ conical rules (compile-time size: the source points
// stay in registers).
template <typename T, int NQ>
__device__ T regular_pair(const T *tv, const T *sv, const double *gx, const double *gw)
{
    const T At = tri_area2(tv), As = tri_area2(sv);
    T py[NQ * NQ][3], pw[NQ * NQ];
#pragma unroll
    for (int i = 0; i < NQ; ++i)
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            const T s = (T)gx[i], t = (T)gx[j];
#pragma unroll
            for (int d = 0; d < 3; ++d) py[i * NQ + j][d] = sv[d] + s * (sv[3 + d] - sv[d]) + s * t * (sv[6 + d] - sv[3 + d]);
            pw[i * NQ + j] = (T)gw[i] * (T)gw[j] * s;
        }
    T acc = 0;
#pragma unroll
    for (int i = 0; i < NQ; ++i)
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            const T s = (T)gx[i], t = (T)gx[j];
            T x[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) x[d] = tv[d] + s * (tv[3 + d] - tv[d]) + s * t * (tv[6 + d] - tv[3 + d]);
            T inner = 0;
#pragma unroll
            for (int q = 0; q < NQ * NQ; ++q) {
                const T dx = x[0] - py[q][0], dy = x[1] - py[q][1], dz = x[2] - py[q][2];
                inner += pw[q] * rsqrt(dx * dx + dy * dy + dz * dz);
            }
            acc += (T)gw[i] * (T)gw[j] * s * inner;
        }
    return acc * At * As;
}



__device__ inline int shared_vertex(const int32_t *ik, const int32_t *il)
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (ik[a] == il[b]) return a;
    return -1;
}

// Class of an entry from the squared distance ratio d2 = (|c_k - c_l| /
// max(diam_k, diam_l))^2; the counting pass and the filling pass call this
// with bit-identical arguments, so they agree on every entry.
template <typename T>
__device__ inline int entry_class(bool self, bool touch, T d2, T rn2)
{
    if (self) return kSelf;
    if (touch) return kQTouch;
    if (d2 < rn2) return d2 < T(0.5625) ? kQNs2 : (d2 < T(2.25) ? kQNs1 : kQNs0);
    return kRegular;
}

__device__ inline double ratio2_64(const NFArgs &a, int32_t k, int32_t l)
{
    const double dx = a.cen[3 * k] - a.cen[3 * l], dy = a.cen[3 * k + 1] - a.cen[3 * l + 1],
                 dz = a.cen[3 * k + 2] - a.cen[3 * l + 2];
    const double dm = fmax(a.diam[k], a.diam[l]);
    return (dx * dx + dy * dy + dz * dz) / (dm * dm);
}

__device__ inline float ratio2_32(float4 ck, float4 cl)
{
    const float dx = ck.x - cl.x, dy = ck.y - cl.y, dz = ck.z - cl.z;
    const float dm = fmaxf(ck.w, cl.w);
    return fmaf(dx, dx, fmaf(dy, dy, dz * dz)) / (dm * dm);
}

// Centroid relative to the plan's reference point, and diameter, in FP32:
// the same four floats for a panel in every leaf, so the FP32 class of
// (k, l) and of (l, k) is the same.
__device__ inline float4 meta32(const NFArgs &a, int32_t k)
{
    return make_float4((float)(a.cen[3 * k] - a.cref[0]), (float)(a.cen[3 * k + 1] - a.cref[1]),
                       (float)(a.cen[3 * k + 2] - a.cref[2]), (float)a.diam[k]);
}

__device__ inline bool share_vertex4(int4 ik, int4 il)
{
    return ik.x == il.x || ik.x == il.y || ik.x == il.z || ik.y == il.x || ik.y == il.y || ik.y == il.z ||
           ik.z == il.x || ik.z == il.y || ik.z == il.z;
}

// Mirror of a source row.  The source rows of a leaf are a sorted union of
// whole boxes and a leaf's panels are one range of panels, so the panels of
// leaf T (kb .. kb + nt - 1) are either all source rows of leaf(l), on
// consecutive rows, or none of them is.  Returns the value index of the
// entry (target l, source kb) in the block of leaf(l), with that block's row
// stride (its tpad, at most 128) in bits 48..55, or -1 when T's panels are
// not source rows of leaf(l).
constexpr int64_t kMirMask = (1ll << 48) - 1;

__device__ inline int64_t row_mirror(const NFArgs &a, int32_t kb, int32_t nt, int32_t l)
{
    const int32_t li = a.panel_leaf[l];
    const int32_t end = a.near_rows[li + 1];
    int32_t lo = a.near_rows[li], hi = end;
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (a.near_src[mid] < kb)
            lo = mid + 1;
        else
            hi = mid;
    }
    if (lo + nt > end || a.near_src[lo] != kb || a.near_src[lo + nt - 1] != kb + nt - 1) return -1;
    const int64_t tp = a.leaf_tpad[li];
    return (tp << 48) | (a.val_off[li] + (int64_t)(lo - a.near_rows[li]) * tp + (l - a.box_beg[a.leaf_box[li]]));
}

// Value index of the entry (target l, source kb + j) from the row's mirror,
// or -1.
__device__ inline int64_t mirror_of(int64_t rm, int32_t j)
{
    return rm < 0 ? -1 : (rm & kMirMask) + (int64_t)j * (rm >> 48);
}

// Counting pass: per leaf, the number of entries of each queue (touching,
// near-singular classes 0..2), cnt[4 li + q]; also the mirror of every source
// row (a.row_mir) for the filling passes.  FP32 classifies as the FP32
// filling pass does (centroids relative to the plan's reference point),
// FP64 as the FP64 one.  A pair (k, l) with k > l whose mirror is stored is
// not queued here: it is integrated as (l, k) and written to both blocks.
template <bool FP64>
__global__ __launch_bounds__(256) void k_nf_count(NFArgs a, int64_t *__restrict__ cnt)
{
    const int64_t li = blockIdx.x;
    if (li >= a.n_leaves) return;
    __shared__ int s_cnt[kNQueues];
    __shared__ unsigned long long s_all[2];
    // each chunk of source rows: centroid (relative), diameter; vertex ids,
    // panel index; the row's mirror
    __shared__ float4 tcd[kMaxLeaf], scd[256];
    __shared__ int4 tid[kMaxLeaf], sid[256];
    __shared__ int64_t smir[256];
    const int32_t Tb = a.leaf_box[li];
    const int32_t kb = a.box_beg[Tb], nt = a.box_end[Tb] - kb;
    const int32_t r0 = a.near_rows[li], nr = a.near_rows[li + 1] - r0;
    if (threadIdx.x < kNQueues) s_cnt[threadIdx.x] = 0;
    if (threadIdx.x < 2) s_all[threadIdx.x] = 0;
    int my[kNQueues] = {0, 0, 0, 0};
    unsigned long long all[2] = {0, 0};
    const float rn2f = (float)(a.r_near * a.r_near);
    auto tally = [&](int c, int32_t k, int32_t l, int64_t rm) {
        if (c < kNQueues) {
            ++all[c == kQTouch ? 0 : 1];
            if (k < l || rm < 0) ++my[c];
        }
    };
    if constexpr (!FP64) {
        for (int j = threadIdx.x; j < nt; j += blockDim.x) {
            const int32_t k = kb + j;
            tcd[j] = meta32(a, k);
            tid[j] = make_int4(a.pvid[3 * k], a.pvid[3 * k + 1], a.pvid[3 * k + 2], k);
        }
    }
    for (int rc = 0; rc < nr; rc += 256) {
        const int nrc = min(256, nr - rc);
        __syncthreads();  // the previous chunk is no longer read
        for (int r = threadIdx.x; r < nrc; r += blockDim.x) {
            const int32_t l = a.near_src[r0 + rc + r];
            const int64_t rm = row_mirror(a, kb, nt, l);
            smir[r] = rm;
            a.row_mir[r0 + rc + r] = rm;
            if constexpr (!FP64) {
                scd[r] = meta32(a, l);
                sid[r] = make_int4(a.pvid[3 * l], a.pvid[3 * l + 1], a.pvid[3 * l + 2], l);
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nrc * nt; e += blockDim.x) {
            const int r = e / nt, j = e - r * nt;
            if constexpr (FP64) {
                const int32_t k = kb + j, l = a.near_src[r0 + rc + r];
                const int4 ik = make_int4(a.pvid[3 * k], a.pvid[3 * k + 1], a.pvid[3 * k + 2], k);
                const int4 il = make_int4(a.pvid[3 * l], a.pvid[3 * l + 1], a.pvid[3 * l + 2], l);
                tally(entry_class<double>(k == l, share_vertex4(ik, il), ratio2_64(a, k, l), a.r_near * a.r_near), k,
                      l, smir[r]);
            } else {
                const int4 ik = tid[j], il = sid[r];
                tally(entry_class<float>(ik.w == il.w, share_vertex4(ik, il), ratio2_32(tcd[j], scd[r]), rn2f), ik.w,
                      il.w, smir[r]);
            }
        }
    }
    __syncthreads();
    for (int q = 0; q < kNQueues; ++q)
        if (my[q]) atomicAdd(&s_cnt[q], my[q]);
    if (all[0]) atomicAdd(&s_all[0], all[0]);
    if (all[1]) atomicAdd(&s_all[1], all[1]);
    __syncthreads();
    if (threadIdx.x < kNQueues) cnt[4 * li + threadIdx.x] = s_cnt[threadIdx.x];
    // stored entries per class (both orientations), for the statistics
    if (threadIdx.x == 0) {
        atomicAdd(&a.counters[1], s_all[0]);
        atomicAdd(&a.counters[2], s_all[1]);
    }
}

// Pass 1 in FP64: one workgroup per target leaf; self and regular entries
// computed, the others written to their queue at the leaf's offset (slots
// within a leaf from LDS counters).  P_kl = P_lk: an entry with k < l whose
// mirror is stored is computed once and written to both blocks, the entry
// with k > l is left to the leaf that holds (l, k).
template <typename V, bool FP64>
__global__ __launch_bounds__(256) void k_nf_main(NFArgs a, NFRules R, V *__restrict__ val)
{
    const int64_t li = blockIdx.x;
    if (li >= a.n_leaves) return;
    __shared__ unsigned long long s_cnt[3];
    __shared__ unsigned long long s_q[kNQueues];
    const int32_t T = a.leaf_box[li];
    const int32_t kb = a.box_beg[T], nt = a.box_end[T] - kb;
    const int32_t r0 = a.near_rows[li], nr = a.near_rows[li + 1] - r0;
    const int tpad = a.leaf_tpad[li];
    const int64_t vo = a.val_off[li];
    if (threadIdx.x == 0) s_cnt[0] = s_cnt[1] = s_cnt[2] = 0;
    if (threadIdx.x < kNQueues) s_q[threadIdx.x] = (unsigned long long)a.q_off[4 * li + threadIdx.x];
    __syncthreads();
    unsigned long long c_self = 0, c_reg = 0, c_fine = 0;
    for (int64_t e = threadIdx.x; e < (int64_t)nr * tpad; e += blockDim.x) {
        const int32_t r = (int32_t)(e / tpad), j = (int32_t)(e - (int64_t)r * tpad);
        if (j >= nt) {
            val[vo + e] = V(0);
            continue;
        }
        const int32_t k = kb + j, l = a.near_src[r0 + r];
        const int4 ik = make_int4(a.pvid[3 * k], a.pvid[3 * k + 1], a.pvid[3 * k + 2], k);
        const int4 il = make_int4(a.pvid[3 * l], a.pvid[3 * l + 1], a.pvid[3 * l + 2], l);
        const double d2 = ratio2_64(a, k, l);
        const int c = entry_class<double>(k == l, share_vertex4(ik, il), d2, a.r_near * a.r_near);
        if (c == kSelf) {
            val[vo + e] = (V)self_term(a.pv + 9 * (int64_t)k);
            ++c_self;
            continue;
        }
        // the mirror entry (target l, source k); with k > l and the mirror
        // stored, this entry is written when (l, k) is computed
        const int64_t mir = mirror_of(a.row_mir[r0 + r], j);
        if (c < kNQueues) {
            if (k < l || mir < 0) {
                const int64_t pos = (int64_t)atomicAdd(&s_q[c], 1ull);
                a.work[pos] = vo + e;
                a.work_meta[2 * pos] = k;
                a.work_meta[2 * pos + 1] = l;
                a.work_mirror[pos] = k < l ? mir : -1;
                val[vo + e] = V(0);
            }
            continue;
        }
        ++c_reg;
        const bool fine = d2 < a.r_mid * a.r_mid;
        c_fine += fine;
        if (k > l && mir >= 0) continue;
        double tv[9], svv[9];
        for (int i = 0; i < 9; ++i) {
            tv[i] = a.pv[9 * (int64_t)k + i];
            svv[i] = a.pv[9 * (int64_t)l + i];
        }
        const V v = (V)(fine ? regular_pair<double, 5>(tv, svv, R.rx4, R.rw4)
                             : regular_pair<double, 4>(tv, svv, R.rx3, R.rw3));
        val[vo + e] = v;
        if (mir >= 0) val[mir] = v;
    }
    // class counters: LDS first, one global atomic per workgroup
    if (c_self) atomicAdd(&s_cnt[0], c_self);
    if (c_reg) atomicAdd(&s_cnt[1], c_reg);
    if (c_fine) atomicAdd(&s_cnt[2], c_fine);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&a.counters[0], s_cnt[0]);
        atomicAdd(&a.counters[3], s_cnt[1]);
        atomicAdd(&a.counters[4], s_cnt[2]);
    }
}

// Pass 1 in FP32 (plain FP32 and mixed modes): one workgroup per target leaf.
// The quadrature points of both product rules (the 12- and 6-point symmetric
// triangle rules) and the areas of the leaf's targets and of a chunk of
// source rows are staged in LDS, in FP32 relative to the leaf's first
// centroid; every lane takes one (row, target) entry of the
// chunk at a time: the self entry in FP64 by the closed form, touching and
// near-singular entries queued for pass 2, regular entries by the product
// rule (sum of w_i w_j / |x_i - y_j|), padding entries set to zero.
// P_kl = P_lk: a regular entry with k < l whose mirror is stored is computed
// once and written to both blocks (the classification is bitwise the same
// in both leaves, see meta32); the entry with k > l is left to leaf(l).
constexpr int kRegHi = 12, kRegLo = 6;
constexpr int kRegPts = kRegHi + kRegLo;  // points per panel: the 12-point rule, then the 6-point rule
constexpr int kRowChunk = 16;
static_assert(kRowChunk <= 256 && kMaxLeaf <= 256, "a regular entry is packed as row << 8 | target in 16 bits");

// A quadrature point in FP32 relative to the leaf's first centroid; the
// weight of point q of panel k is the rule weight times the panel's area, so
// the points carry positions only and each panel one area.
struct P3 {
    float x, y, z;
};

__device__ inline void stage_point(const double *__restrict__ pv, int32_t k, const double *c0, const NFRules &R, int q,
                                   P3 *__restrict__ out)
{
    const double *v = pv + 9 * (int64_t)k;
    const double *b = R.sym_b[q];
    P3 o;
    o.x = (float)(b[0] * v[0] + b[1] * v[3] + b[2] * v[6] - c0[0]);
    o.y = (float)(b[0] * v[1] + b[1] * v[4] + b[2] * v[7] - c0[1]);
    o.z = (float)(b[0] * v[2] + b[1] * v[5] + b[2] * v[8] - c0[2]);
    *out = o;
}

__device__ inline float area32(const double *__restrict__ pv, int32_t k)
{
    const double *v = pv + 9 * (int64_t)k;
    const double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
    const double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
    const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                 cz = e1[0] * e2[1] - e1[1] * e2[0];
    return (float)(0.5 * sqrt(cx * cx + cy * cy + cz * cz));
}

// sum_i w_i sum_j w_j / |x_i - y_j| over the NQ points of one rule (weights
// R.sym_w[off ..], summing to one; the caller multiplies by both areas): the
// source points and weights go to registers once, the target points stream
// from LDS.
template <int NQ>
__device__ inline float product_rule(const P3 *__restrict__ xp, const P3 *__restrict__ yp, const NFRules &R, int off)
{
    P3 y[NQ];
    float w[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) {
        y[j] = yp[j];
        w[j] = (float)R.sym_w[off + j];
    }
    float acc = 0.f;
#pragma unroll 2
    for (int i = 0; i < NQ; ++i) {
        const P3 x = xp[i];
        float inner = 0.f;
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            const float dx = x.x - y[j].x, dy = x.y - y[j].y, dz = x.z - y[j].z;
            inner = fmaf(w[j], rsqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz))), inner);
        }
        acc = fmaf((float)R.sym_w[off + i], inner, acc);
    }
    return acc;
}

__global__ __launch_bounds__(256) void k_nf_leaf32(NFArgs a, NFRules R, float *__restrict__ val)
{
    const int64_t li = blockIdx.x;
    if (li >= a.n_leaves) return;
    __shared__ P3 tp[kMaxLeaf * kRegPts];
    __shared__ P3 spt[kRowChunk * kRegPts];
    __shared__ float tar[kMaxLeaf], sar[kRowChunk];  // panel areas
    __shared__ float4 tcd[kMaxLeaf], scd[kRowChunk];  // centroid (relative), diameter
    __shared__ int4 tid[kMaxLeaf], sid[kRowChunk];    // vertex ids, panel index
    __shared__ int64_t smir[kRowChunk];               // mirror of each row of the chunk
    __shared__ unsigned long long s_cnt[3];
    __shared__ unsigned long long s_q[kNQueues];  // next free position of this leaf in each queue
    // regular entries of the current chunk, compacted by rule (4 x 4 from the
    // front, 3 x 3 from the back) so that the lanes of a wave all run the
    // same rule: entry = row << 8 | target
    __shared__ uint16_t s_reg[kRowChunk * kMaxLeaf];
    __shared__ int s_n4, s_n3;
    const int32_t Tb = a.leaf_box[li];
    const int32_t kb = a.box_beg[Tb], nt = a.box_end[Tb] - kb;
    const int32_t r0 = a.near_rows[li], nr = a.near_rows[li + 1] - r0;
    const int tpad = a.leaf_tpad[li];
    const int64_t vo = a.val_off[li];
    const double c0[3] = {a.cen[3 * (int64_t)kb], a.cen[3 * (int64_t)kb + 1], a.cen[3 * (int64_t)kb + 2]};
    if (threadIdx.x == 0) s_cnt[0] = s_cnt[1] = s_cnt[2] = 0;
    if (threadIdx.x < kNQueues) s_q[threadIdx.x] = (unsigned long long)a.q_off[4 * li + threadIdx.x];
    for (int e = threadIdx.x; e < nt * kRegPts; e += blockDim.x)
        stage_point(a.pv, kb + e / kRegPts, c0, R, e % kRegPts, &tp[e]);
    for (int j = threadIdx.x; j < nt; j += blockDim.x) {
        const int32_t k = kb + j;
        tar[j] = area32(a.pv, k);
        tcd[j] = meta32(a, k);
        tid[j] = make_int4(a.pvid[3 * k], a.pvid[3 * k + 1], a.pvid[3 * k + 2], k);
    }
    unsigned long long c_self = 0, c_reg = 0, c_fine = 0;
    const float rn2 = (float)(a.r_near * a.r_near), rm2 = (float)(a.r_mid * a.r_mid);
    for (int rc = 0; rc < nr; rc += kRowChunk) {
        const int nrc = min(kRowChunk, nr - rc);
        __syncthreads();  // the previous chunk's points are no longer read
        for (int e = threadIdx.x; e < nrc * kRegPts; e += blockDim.x)
            stage_point(a.pv, a.near_src[r0 + rc + e / kRegPts], c0, R, e % kRegPts, &spt[e]);
        for (int r = threadIdx.x; r < nrc; r += blockDim.x) {
            const int32_t l = a.near_src[r0 + rc + r];
            sar[r] = area32(a.pv, l);
            scd[r] = meta32(a, l);
            sid[r] = make_int4(a.pvid[3 * l], a.pvid[3 * l + 1], a.pvid[3 * l + 2], l);
            smir[r] = a.row_mir[r0 + rc + r];
        }
        __syncthreads();
        if (threadIdx.x == 0) s_n4 = s_n3 = 0;
        __syncthreads();
        for (int e = threadIdx.x; e < nrc * tpad; e += blockDim.x) {
            const int r = e / tpad, j = e - r * tpad;
            const int64_t out = vo + (int64_t)(rc + r) * tpad + j;
            if (j >= nt) {
                val[out] = 0.f;
                continue;
            }
            const int4 ik = tid[j], il = sid[r];
            const float d2 = ratio2_32(tcd[j], scd[r]);
            const int c = entry_class<float>(ik.w == il.w, share_vertex4(ik, il), d2, rn2);
            if (c == kSelf) {
                val[out] = (float)self_term(a.pv + 9 * (int64_t)ik.w);
                ++c_self;
                continue;
            }
            // the mirror entry (target l, source k); with k > l and the
            // mirror stored, this entry is written when (l, k) is computed
            const int32_t k = ik.w, l = il.w;
            const int64_t mir = mirror_of(smir[r], j);
            if (c < kNQueues) {
                if (k < l || mir < 0) {
                    const int64_t pos = (int64_t)atomicAdd(&s_q[c], 1ull);
                    a.work[pos] = out;
                    a.work_meta[2 * pos] = k;
                    a.work_meta[2 * pos + 1] = l;
                    a.work_mirror[pos] = k < l ? mir : -1;
                    val[out] = 0.f;
                }
                continue;
            }
            const bool fine = d2 < rm2;
            ++c_reg;
            c_fine += fine;
            if (k > l && mir >= 0) continue;
            if (fine)
                s_reg[atomicAdd(&s_n4, 1)] = r << 8 | j;
            else
                s_reg[kRowChunk * kMaxLeaf - 1 - atomicAdd(&s_n3, 1)] = r << 8 | j;
        }
        __syncthreads();
        const int n4 = s_n4, n3 = s_n3;
        // the value, and its mirror where stored (then k < l)
        auto store = [&](int r, int j, float v) {
            val[vo + (int64_t)(rc + r) * tpad + j] = v;
            const int64_t mir = mirror_of(smir[r], j);
            if (mir >= 0) val[mir] = v;
        };
        for (int q = threadIdx.x; q < n4; q += blockDim.x) {
            const int rj = s_reg[q], r = rj >> 8, j = rj & 255;
            store(r, j, tar[j] * sar[r] * product_rule<kRegHi>(&tp[j * kRegPts], &spt[r * kRegPts], R, 0));
        }
        for (int q = threadIdx.x; q < n3; q += blockDim.x) {
            const int rj = s_reg[kRowChunk * kMaxLeaf - 1 - q], r = rj >> 8, j = rj & 255;
            store(r, j,
                  tar[j] * sar[r] *
                      product_rule<kRegLo>(&tp[j * kRegPts + kRegHi], &spt[r * kRegPts + kRegHi], R, kRegHi));
        }
    }
    // padding rows of a leaf without rows do not exist; class counters: LDS
    // first, one global atomic per workgroup
    __syncthreads();
    if (c_self) atomicAdd(&s_cnt[0], c_self);
    if (c_reg) atomicAdd(&s_cnt[1], c_reg);
    if (c_fine) atomicAdd(&s_cnt[2], c_fine);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&a.counters[0], s_cnt[0]);
        atomicAdd(&a.counters[3], s_cnt[1]);
        atomicAdd(&a.counters[4], s_cnt[2]);
    }
}

// Pass 2: the entries of one queue, one per thread.  Entry t of the launch
// is queue position list[t] (a fall-back or audit list) or base + t.
// Touching pairs: the graded rule collapsed at the shared vertex.  Near-
// singular pairs of rule class c: P_kl = P_lk, so the outer rule runs over
// the smaller panel and the closed-form potential belongs to the larger one,
// whose evaluation points then lie within a few of its diameters (far from a
// small triangle its edge terms cancel in FP32).
template <typename V, typename C>
__global__ __launch_bounds__(64) void k_nf_special(NFArgs a, NFRules R, int queue, int64_t base, int64_t count,
                                                   V *__restrict__ val, const int64_t *__restrict__ list,
                                                   double *__restrict__ alt_out)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= count) return;
    const int64_t pos = list ? list[t] : base + t;
    const int32_t k = a.work_meta[2 * pos], l = a.work_meta[2 * pos + 1];
    // coordinates relative to the target centroid
    C tv[9], sv[9];
    C v;
    if (queue == kQTouch) {
        const int32_t *ik = a.pvid + 3 * (int64_t)k, *il = a.pvid + 3 * (int64_t)l;
        const int s0 = shared_vertex(ik, il);
        // a second shared vertex (the panels share an edge) goes second
        int ord[3] = {s0, (s0 + 1) % 3, (s0 + 2) % 3};
        const auto shared = [&](int i) { return ik[i] == il[0] || ik[i] == il[1] || ik[i] == il[2]; };
        const bool edge = shared(ord[1]) || shared(ord[2]);
        if (!shared(ord[1]) && shared(ord[2])) {
            ord[1] = (s0 + 2) % 3;
            ord[2] = (s0 + 1) % 3;
        }
        for (int j = 0; j < 3; ++j)
            for (int d = 0; d < 3; ++d) tv[3 * j + d] = (C)(a.pv[9 * (int64_t)k + 3 * ord[j] + d] - a.cen[3 * k + d]);
        for (int q = 0; q < 9; ++q) sv[q] = (C)(a.pv[9 * (int64_t)l + q] - a.cen[3 * k + q % 3]);
        v = touching_pair<C>(tv, sv, R, edge);
    } else {
        const int32_t o = a.diam[l] < a.diam[k] ? l : k, in = o == k ? l : k;
        for (int q = 0; q < 9; ++q) {
            tv[q] = (C)(a.pv[9 * (int64_t)o + q] - a.cen[3 * k + q % 3]);
            sv[q] = (C)(a.pv[9 * (int64_t)in + q] - a.cen[3 * k + q % 3]);
        }
        v = near_pair<C>(tv, sv, queue - kQNs0, R);
    }
    if (alt_out) {
        alt_out[t] = (double)v;
    } else {
        val[a.work[pos]] = (V)v;
        if (a.work_mirror[pos] >= 0) val[a.work_mirror[pos]] = (V)v;
    }
}

// Claim n slots of a global counter for the lanes of a workgroup that pass
// `take`: one global atomic per workgroup; returns this lane's slot or -1.
__device__ inline int64_t block_claim(bool take, unsigned long long *ctr)
{
    __shared__ unsigned int s_n;
    __shared__ unsigned long long s_base;
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    const unsigned int mine = take ? atomicAdd(&s_n, 1u) : 0u;
    __syncthreads();
    if (threadIdx.x == 0) s_base = s_n ? atomicAdd(ctr, (unsigned long long)s_n) : 0ull;
    __syncthreads();
    return take ? (int64_t)(s_base + mine) : -1;
}

// Surrogate decision for entry i of the rule-class-0 near-singular queue
// (position base + i): accept P = cheap (1 + out0) when every feature lies
// in the training range and out1 <= bound, else list the entry for
// quadrature.  Every audit_every-th accepted entry is also listed for an
// audit against quadrature.
template <typename V>
__global__ __launch_bounds__(256) void k_ns_accept(NFArgs a, int64_t base, int64_t n, const float *__restrict__ feat,
                                                   const double *__restrict__ cheap, const float *__restrict__ out,
                                                   const float *__restrict__ lo, const float *__restrict__ hi,
                                                   float bound, int audit_every, V *__restrict__ val,
                                                   int64_t *__restrict__ fb, unsigned long long *__restrict__ fbn,
                                                   int64_t *__restrict__ aud, double *__restrict__ aud_val,
                                                   unsigned long long *__restrict__ audn)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool live = i < n;
    bool ok = false;
    double v = 0;
    if (live) {
        ok = out[2 * i + 1] <= bound && isfinite(out[2 * i]);
        for (int q = 0; q < 18 && ok; ++q) ok = feat[18 * i + q] >= lo[q] && feat[18 * i + q] <= hi[q];
        if (ok) {
            v = cheap[i] * (1.0 + (double)out[2 * i]);
            val[a.work[base + i]] = (V)v;
            if (a.work_mirror[base + i] >= 0) val[a.work_mirror[base + i]] = (V)v;
        }
    }
    const int64_t f = block_claim(live && !ok, fbn);
    if (f >= 0) fb[f] = base + i;
    const int64_t d = block_claim(live && ok && audit_every > 0 && i % audit_every == 0, audn);
    if (d >= 0) {
        aud[d] = base + i;
        aud_val[d] = v;
    }
}

__global__ void k_audit_err(const double *__restrict__ ref, const double *__restrict__ got, int64_t n,
                            double *__restrict__ rel)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) rel[i] = fabs(got[i] - ref[i]) / fabs(ref[i]);
}

}  // namespace xrl

using namespace xrl;

extern "C" xrl_status xrl_nearfield_assemble(xrl_plan *P, const xrl_nf_opts *opts, void *stream,
                                             xrl_nf_stats *stats)
{
    return guarded([&] {
        XRL_CHECK(P, XRL_E_INVALID_ARG, "xrl_nearfield_assemble: null plan");
        hipStream_t s = (hipStream_t)stream;
        const AllocStream alloc_scope(s);
        xrl_nf_opts o{2.0, 4.0, nullptr, 0};
        if (opts) o = *opts;
        XRL_CHECK(o.r_near > 0 && o.r_mid >= o.r_near, XRL_E_INVALID_ARG,
                  "xrl_nearfield_assemble: need 0 < r_near <= r_mid");
        if (o.surrogate)
            XRL_CHECK(o.surrogate->hidden == 64 || o.surrogate->hidden == 128, XRL_E_UNSUPPORTED,
                      "xrl_nearfield_assemble: surrogate hidden width must be 64 or 128");
        hipEvent_t e0, e1;
        XRL_HIP(hipEventCreate(&e0));
        XRL_HIP(hipEventCreate(&e1));
        XRL_HIP(hipEventRecord(e0, s));
        const bool fp64 = P->precision == XRL_PREC_FP64;
        NFRules R{};
        R.n_touch = fp64 ? 32 : 24;
        // near-singular rules: FP64 keeps 6 x 6 points on 1, 4, 16
        // sub-triangles (error <= 2e-9 against the oracle on the package's
        // pairs); the FP32 storage modes take 5 x 5 on 1 and 4 and 6 x 6 on 4
        // sub-triangles (error <= 2.2e-7, below FP32 arithmetic)
        // (classes 0 and 1 of the FP32 storage modes on the 16-point
        // symmetric rule of Dunavant (1985), exact to degree 8 like the 5 x 5
        // conical rule, with 16 points instead of 25: within 6e-8 of the
        // oracle on the package's pairs)
        const int nsn[2][3] = {{5, 5, 6}, {6, 6, 6}}, nsl[2][3] = {{0, 1, 1}, {0, 1, 2}};
        for (int c = 0; c < 3; ++c) {
            R.ns_n[c] = nsn[fp64][c];
            R.ns_lev[c] = nsl[fp64][c];
            R.ns_sym[c] = !fp64 && c < 2;
            gauss_legendre01(R.ns_n[c], R.nx[c], R.nw[c]);
        }
        {
            int q = 0;
            auto put = [&](double a, double b, double c, double w) {
                R.ns16_b[q][0] = a;
                R.ns16_b[q][1] = b;
                R.ns16_b[q][2] = c;
                R.ns16_w[q++] = w;
            };
            put(1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0, 0.144315607677787);
            const double a3[3][2] = {{0.459292588292723, 0.095091634267285},
                                     {0.170569307751760, 0.103217370534718},
                                     {0.050547228317031, 0.032458497623198}};
            for (auto &g : a3) {
                const double a = g[0], c = 1.0 - 2.0 * a;
                put(a, a, c, g[1]);
                put(a, c, a, g[1]);
                put(c, a, a, g[1]);
            }
            const double a = 0.008394777409958, b = 0.263112829634638, c = 1.0 - a - b, w = 0.027230314174435;
            put(a, b, c, w);
            put(a, c, b, w);
            put(b, a, c, w);
            put(b, c, a, w);
            put(c, a, b, w);
            put(c, b, a, w);
        }
        R.n_hi = fp64 ? 5 : 4;
        R.n_lo = fp64 ? 4 : 3;
        gauss_legendre01(R.n_touch, R.gx, R.gw);
        // graded touching rules of the FP32 storage modes: Gauss-Legendre
        // nodes u through u -> u^2 (weights times 2u)
        R.touch_graded = !fp64;
        R.n_gs = 12;
        R.n_gse = 16;
        R.n_gt = 12;
        auto graded = [](int n, double *x, double *w) {
            double u[16], gw[16];
            gauss_legendre01(n, u, gw);
            for (int i = 0; i < n; ++i) {
                x[i] = u[i] * u[i];
                w[i] = gw[i] * 2.0 * u[i];
            }
        };
        graded(R.n_gs, R.gs_x, R.gs_w);
        graded(R.n_gse, R.gse_x, R.gse_w);
        graded(R.n_gt, R.gt_x, R.gt_w);
        for (int i = 0; i < R.n_touch; ++i) {
            // sigmoidal map s(u) = u^3 / (u^3 + (1-u)^3), clustering the nodes
            // at both ends of each collapsed coordinate
            const double u = R.gx[i], u3 = u * u * u, v3 = (1 - u) * (1 - u) * (1 - u);
            R.tx[i] = u3 / (u3 + v3);
            R.tw[i] = R.gw[i] * 3.0 * u * u * (1 - u) * (1 - u) / ((u3 + v3) * (u3 + v3));
        }
        // symmetric rules for the triangle (Dunavant 1985): orbits of the
        // barycentric point (a, a, 1 - 2a) (3 points) and (a, b, 1 - a - b)
        // (6 points); degree 6 with 12 points, degree 4 with 6 points
        {
            int q = 0;
            auto orbit3 = [&](double a, double w) {
                const double c = 1.0 - 2.0 * a;
                const double p[3][3] = {{a, a, c}, {a, c, a}, {c, a, a}};
                for (auto &b : p) {
                    for (int d = 0; d < 3; ++d) R.sym_b[q][d] = b[d];
                    R.sym_w[q++] = w;
                }
            };
            auto orbit6 = [&](double a, double b, double w) {
                const double c = 1.0 - a - b;
                const double p[6][3] = {{a, b, c}, {a, c, b}, {b, a, c}, {b, c, a}, {c, a, b}, {c, b, a}};
                for (auto &t : p) {
                    for (int d = 0; d < 3; ++d) R.sym_b[q][d] = t[d];
                    R.sym_w[q++] = w;
                }
            };
            orbit3(0.063089014491502228, 0.050844906370206817);
            orbit3(0.24928674517091042, 0.11678627572637937);
            orbit6(0.053145049844816947, 0.31035245103378440, 0.082851075618373575);
            orbit3(0.44594849091596489, 0.22338158967801147);
            orbit3(0.091576213509770743, 0.10995174365532187);
        }
        gauss_legendre01(R.n_hi, R.rx4, R.rw4);
        gauss_legendre01(R.n_lo, R.rx3, R.rw3);
        if (fp64) {
            P->near32.release();
            P->near64.alloc(std::max<int64_t>(P->n_near_entries, 1));
        } else {
            P->near64.release();
            P->near32.alloc(std::max<int64_t>(P->n_near_entries, 1));
        }
        DevBuf<unsigned long long> cnt(5);
        XRL_HIP(hipMemsetAsync(cnt.p, 0, cnt.bytes(), s));
        NFArgs a{P->leaf_box.p, P->box_beg.p, P->box_end.p, P->near_rows.p, P->near_src.p, P->leaf_tpad.p,
                 P->pvid.p,     P->near_val_off.p, P->pv.p, P->cen.p, P->diam.p, o.r_near, o.r_mid,
                 P->n_leaves,   cnt.p,       nullptr,  nullptr, nullptr, nullptr, nullptr, P->panel_leaf.p,
                 {P->trees[0]->root_c[0], P->trees[0]->root_c[1], P->trees[0]->root_c[2]}};
        DevBuf<int64_t> rowmir(std::max<int64_t>(P->n_near_rows, 1));
        a.row_mir = rowmir.p;
        // counting pass, then every leaf's first position in each queue
        // (queues stored one after another: touching, near-singular 0, 1, 2)
        const int64_t L = P->n_leaves;
        DevBuf<int64_t> lcnt(std::max<int64_t>(4 * L, 4)), qoff(std::max<int64_t>(4 * L, 4));
        std::vector<int64_t> qbase(kNQueues + 1, 0);
        if (L > 0) {
            if (fp64)
                k_nf_count<true><<<L, 256, 0, s>>>(a, lcnt.p);
            else
                k_nf_count<false><<<L, 256, 0, s>>>(a, lcnt.p);
            XRL_HIP(hipGetLastError());
            std::vector<int64_t> hc = lcnt.download(s, 4 * L), ho(4 * L);
            for (int q = 0; q < kNQueues; ++q) {
                int64_t tot = 0;
                for (int64_t li = 0; li < L; ++li) tot += hc[4 * li + q];
                qbase[q + 1] = qbase[q] + tot;
            }
            for (int q = 0; q < kNQueues; ++q) {
                int64_t run = qbase[q];
                for (int64_t li = 0; li < L; ++li) {
                    ho[4 * li + q] = run;
                    run += hc[4 * li + q];
                }
            }
            qoff.upload(ho, s);
        }
        const int64_t nq = qbase[kNQueues];
        DevBuf<int64_t> work(std::max<int64_t>(nq, 1));
        DevBuf<int32_t> meta(2 * std::max<int64_t>(nq, 1));
        DevBuf<int64_t> mirror(std::max<int64_t>(nq, 1));
        a.work = work.p;
        a.work_meta = meta.p;
        a.work_mirror = mirror.p;
        a.q_off = qoff.p;
        if (L > 0) {
            if (fp64)
                k_nf_main<double, true><<<L, 256, 0, s>>>(a, R, P->near64.p);
            else
                k_nf_leaf32<<<L, 256, 0, s>>>(a, R, P->near32.p);
            XRL_HIP(hipGetLastError());
        }
        // mixed precision: FP64 for the touching (adjacent-panel) pairs and
        // for the audit reference of the surrogate, FP32 (relative to the
        // target centroid, exact inner potential) for the near-singular
        // pairs that are not adjacent
        auto special = [&](int queue, int64_t base, int64_t count, const int64_t *list, double *alt) {
            if (count == 0) return;
            if (P->precision == XRL_PREC_FP64)
                k_nf_special<double, double><<<cdiv(count, 64), 64, 0, s>>>(a, R, queue, base, count, P->near64.p,
                                                                            list, alt);
            else if (P->precision == XRL_PREC_MIXED && (queue == kQTouch || alt))
                k_nf_special<float, double><<<cdiv(count, 64), 64, 0, s>>>(a, R, queue, base, count, P->near32.p,
                                                                           list, alt);
            else
                k_nf_special<float, float><<<cdiv(count, 64), 64, 0, s>>>(a, R, queue, base, count, P->near32.p,
                                                                          list, alt);
            XRL_HIP(hipGetLastError());
        };
        for (int q = 0; q < kNQueues; ++q)
            if (!(o.surrogate && q == kQNs0)) special(q, qbase[q], qbase[q + 1] - qbase[q], nullptr, nullptr);
        int64_t n_acc = 0, n_fb = 0;
        double aud_max = 0, aud_rms = 0;
        // the surrogate takes the rule-class-0 near-singular pairs (r >= 1.5):
        // closer pairs fail its error bound almost always, so evaluating the
        // network there would only add to the quadrature
        const int64_t nns = qbase[kQNs0 + 1] - qbase[kQNs0];
        if (o.surrogate && nns > 0) {
            MlpDevice mlp;
            mlp_prepare_host(mlp, o.surrogate, s);
            DevBuf<float> feat(18 * nns), out(2 * nns), lo, hi;
            DevBuf<double> cheap(nns), aud_val(nns), aud_ref(nns), rel(nns);
            DevBuf<int64_t> fb(nns), aud(nns);
            DevBuf<unsigned long long> fbn(2);
            lo.upload(o.surrogate->feat_lo, 18, s);
            hi.upload(o.surrogate->feat_hi, 18, s);
            XRL_HIP(hipMemsetAsync(fbn.p, 0, fbn.bytes(), s));
            ns_features(a, qbase[kQNs0], nns, feat.p, cheap.p, s);
            mlp_infer(mlp, feat.p, nns, out.p, s);
            if (fp64)
                k_ns_accept<double><<<cdiv(nns, 256), 256, 0, s>>>(a, qbase[kQNs0], nns, feat.p, cheap.p, out.p, lo.p,
                                                                  hi.p, o.surrogate->log10_err_bound, o.audit_every,
                                                                  P->near64.p, fb.p, fbn.p, aud.p, aud_val.p,
                                                                  fbn.p + 1);
            else
                k_ns_accept<float><<<cdiv(nns, 256), 256, 0, s>>>(a, qbase[kQNs0], nns, feat.p, cheap.p, out.p, lo.p,
                                                                 hi.p, o.surrogate->log10_err_bound, o.audit_every,
                                                                 P->near32.p, fb.p, fbn.p, aud.p, aud_val.p,
                                                                 fbn.p + 1);
            XRL_HIP(hipGetLastError());
            auto hn = fbn.download(s);
            n_fb = (int64_t)hn[0];
            n_acc = nns - n_fb;
            special(kQNs0, 0, n_fb, fb.p, nullptr);
            const int64_t na = (int64_t)hn[1];
            if (na > 0) {
                special(kQNs0, 0, na, aud.p, aud_ref.p);
                k_audit_err<<<cdiv(na, 256), 256, 0, s>>>(aud_ref.p, aud_val.p, na, rel.p);
                auto hr = rel.download(s, na);
                double ss = 0;
                for (double r : hr) {
                    aud_max = std::max(aud_max, r);
                    ss += r * r;
                }
                aud_rms = std::sqrt(ss / na);
            }
        }
        XRL_HIP(hipEventRecord(e1, s));
        XRL_HIP(hipEventSynchronize(e1));
        float ms = 0;
        XRL_HIP(hipEventElapsedTime(&ms, e0, e1));
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        auto hc = cnt.download(s);
        P->assembled = true;
        if (stats) {
            std::memset(stats, 0, sizeof *stats);
            stats->n_entries = P->n_near_entries;
            stats->n_self = (int64_t)hc[0];
            stats->n_touching = (int64_t)hc[1];
            stats->n_near_singular = (int64_t)hc[2];
            stats->n_regular = (int64_t)hc[3];
            stats->n_regular_fine = (int64_t)hc[4];
            stats->n_mlp_accepted = n_acc;
            stats->n_mlp_fallback = o.surrogate ? n_fb : 0;
            stats->audit_max_rel_err = aud_max;
            stats->audit_rms_rel_err = aud_rms;
            stats->ms = ms;
        }
    });
}
