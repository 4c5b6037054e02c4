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
//   regular       product of two conical Gauss rules (4x4 or 3x3 points per
//                 triangle in FP32; 5x5 or 4x4 in FP64).
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
// from the edge) and the two arc tangents as one atan2 of their difference,
// whose numerator uses s+ R- - s- R+ = R0^2 L (s+ + s-)/(s+ R- + s- R+).
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
            T lg;
            if (sm >= 0)
                lg = log1p(L[i] * (S + sm + sp) / (S * (Rm + sm)));
            else if (sp <= 0)
                lg = log1p(L[i] * (S - sm - sp) / (S * (Rp - sp)));
            else
                lg = log((Rp + sp) * (Rm - sm) / R0s);
            phi += t0 * lg;
            if (ah > eps * L[i]) {
                const T D = sp * sm > 0 ? R0s * L[i] * (sp + sm) / (sp * Rm + sm * Rp) : sp * Rm - sm * Rp;
                const T Dp = R0s + ah * Rp, Dm = R0s + ah * Rm;
                phi -= ah * atan2(t0 * (R0s * L[i] + ah * D), Dp * Dm + t0 * t0 * sp * sm);
            }
        }
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

// Touching pair: target vertices reordered so that tv[0] is a shared vertex.
template <typename T>
__device__ T touching_pair(const T *tv, const T *sv, const NFRules &R)
{
    TriPot<T> pot;
    pot.init(sv);
    const T A2 = tri_area2(tv);
    T acc = 0;
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



// Queue slot for a special entry: touching pairs fill the queue from the
// front (which = 0), near-singular pairs from the back (which = 1).  One
// atomic per wave and queue (lanes counted with a ballot), not one per entry.
__device__ inline int64_t queue_slot(const NFArgs &a, int which)
{
    int64_t pos = -1;
    for (int q = 0; q < 2; ++q) {
        const unsigned long long mask = __ballot(which == q);
        if (mask == 0) continue;
        const int lane = __lane_id();
        const int leader = __ffsll((long long)mask) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(&a.work_n[q], (unsigned long long)__popcll(mask));
        base = __shfl(base, leader);
        if (which == q) {
            const unsigned long long rank = __popcll(mask & ((1ull << lane) - 1ull));
            pos = q == 0 ? (int64_t)(base + rank) : a.work_cap - 1 - (int64_t)(base + rank);
        }
    }
    return pos;
}

__device__ inline int shared_vertex(const int32_t *ik, const int32_t *il)
{
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            if (ik[a] == il[b]) return a;
    return -1;
}

// Pass 1: one workgroup per target leaf; self and regular entries computed,
// touching and near-singular entries queued.
template <typename V, bool FP64>
__global__ __launch_bounds__(256) void k_nf_main(NFArgs a, NFRules R, V *__restrict__ val)
{
    const int64_t li = blockIdx.x;
    if (li >= a.n_leaves) return;
    const int32_t T = a.leaf_box[li];
    const int32_t kb = a.box_beg[T], nt = a.box_end[T] - kb;
    const int32_t r0 = a.near_rows[li], nr = a.near_rows[li + 1] - r0;
    const int tpad = a.leaf_tpad[li];
    const int64_t vo = a.val_off[li];
    unsigned long long c_self = 0, c_reg = 0;
    for (int64_t e = threadIdx.x; e < (int64_t)nr * tpad; e += blockDim.x) {
        const int32_t r = (int32_t)(e / tpad), j = (int32_t)(e - (int64_t)r * tpad);
        if (j >= nt) {
            val[vo + e] = V(0);
            continue;
        }
        const int32_t k = kb + j, l = a.near_src[r0 + r];
        if (k == l) {
            val[vo + e] = (V)self_term(a.pv + 9 * (int64_t)k);
            ++c_self;
            continue;
        }
        const int sv = shared_vertex(a.pvid + 3 * (int64_t)k, a.pvid + 3 * (int64_t)l);
        const double dx = a.cen[3 * k] - a.cen[3 * l], dy = a.cen[3 * k + 1] - a.cen[3 * l + 1],
                     dz = a.cen[3 * k + 2] - a.cen[3 * l + 2];
        const double rr = sqrt(dx * dx + dy * dy + dz * dz) / fmax(a.diam[k], a.diam[l]);
        if (sv >= 0 || rr < a.r_near) {
            const int which = sv >= 0 ? 0 : 1;
            const int64_t pos = queue_slot(a, which);
            if (pos >= 0 && pos < a.work_cap) {
                a.work[pos] = vo + e;
                a.work_meta[2 * pos] = k;
                a.work_meta[2 * pos + 1] = l;
            }
            val[vo + e] = V(0);
            continue;
        }
        ++c_reg;
        if (FP64) {
            double tv[9], svv[9];
            for (int i = 0; i < 9; ++i) {
                tv[i] = a.pv[9 * (int64_t)k + i];
                svv[i] = a.pv[9 * (int64_t)l + i];
            }
            val[vo + e] = (V)(rr < a.r_mid ? regular_pair<double, 5>(tv, svv, R.rx4, R.rw4)
                                           : regular_pair<double, 4>(tv, svv, R.rx3, R.rw3));
        } else {
            // FP32 arithmetic relative to the target centroid
            float tv[9], svv[9];
            for (int i = 0; i < 9; ++i) {
                tv[i] = (float)(a.pv[9 * (int64_t)k + i] - a.cen[3 * k + i % 3]);
                svv[i] = (float)(a.pv[9 * (int64_t)l + i] - a.cen[3 * k + i % 3]);
            }
            val[vo + e] = (V)(rr < a.r_mid ? regular_pair<float, 4>(tv, svv, R.rx4, R.rw4)
                                           : regular_pair<float, 3>(tv, svv, R.rx3, R.rw3));
        }
    }
    // class counters: LDS first, one global atomic per workgroup
    __shared__ unsigned long long s_cnt[2];
    if (threadIdx.x == 0) s_cnt[0] = s_cnt[1] = 0;
    __syncthreads();
    if (c_self) atomicAdd(&s_cnt[0], c_self);
    if (c_reg) atomicAdd(&s_cnt[1], c_reg);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&a.counters[0], s_cnt[0]);
        atomicAdd(&a.counters[3], s_cnt[1]);
    }
}

// Pass 1 in FP32 (plain FP32 and mixed modes): one workgroup per target leaf.
// The quadrature points of both product rules (4 x 4 and 3 x 3 conical Gauss
// points per triangle, weights times twice the area) of the leaf's targets
// and of a chunk of source rows are staged in LDS, in FP32 relative to the
// leaf's first centroid; every lane takes one (row, target) entry of the
// chunk at a time: the self entry in FP64 by the closed form, touching and
// near-singular entries queued for pass 2, regular entries by the product
// rule (sum of w_i w_j / |x_i - y_j|), padding entries set to zero.
constexpr int kRegPts = 16 + 9;  // points per panel: the 4 x 4 rule, then the 3 x 3 rule
constexpr int kRowChunk = 16;

__device__ inline void stage_points(const double *__restrict__ pv, int32_t k, const double *c0, const NFRules &R,
                                    int q, float4 *__restrict__ out)
{
    const double *v = pv + 9 * (int64_t)k;
    const double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
    const double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
    const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                 cz = e1[0] * e2[1] - e1[1] * e2[0];
    const double A2 = sqrt(cx * cx + cy * cy + cz * cz);
    double s, t, w;
    if (q < 16) {
        s = R.rx4[q / 4];
        t = R.rx4[q % 4];
        w = R.rw4[q / 4] * R.rw4[q % 4] * s * A2;
    } else {
        s = R.rx3[(q - 16) / 3];
        t = R.rx3[(q - 16) % 3];
        w = R.rw3[(q - 16) / 3] * R.rw3[(q - 16) % 3] * s * A2;
    }
    float4 o;
    o.x = (float)(v[0] + s * (v[3] - v[0]) + s * t * (v[6] - v[3]) - c0[0]);
    o.y = (float)(v[1] + s * (v[4] - v[1]) + s * t * (v[7] - v[4]) - c0[1]);
    o.z = (float)(v[2] + s * (v[5] - v[2]) + s * t * (v[8] - v[5]) - c0[2]);
    o.w = (float)w;
    *out = o;
}

template <int NQ>
__device__ inline float product_rule(const float4 *__restrict__ xp, const float4 *__restrict__ yp)
{
    float acc = 0.f;
    for (int i = 0; i < NQ; ++i) {
        const float4 x = xp[i];
        float inner = 0.f;
#pragma unroll
        for (int j = 0; j < NQ; ++j) {
            const float4 y = yp[j];
            const float dx = x.x - y.x, dy = x.y - y.y, dz = x.z - y.z;
            inner = fmaf(y.w, rsqrtf(fmaf(dx, dx, fmaf(dy, dy, dz * dz))), inner);
        }
        acc = fmaf(x.w, inner, acc);
    }
    return acc;
}

__global__ __launch_bounds__(256) void k_nf_leaf32(NFArgs a, NFRules R, float *__restrict__ val)
{
    const int64_t li = blockIdx.x;
    if (li >= a.n_leaves) return;
    __shared__ float4 tp[kMaxLeaf * kRegPts];
    __shared__ float4 spt[kRowChunk * kRegPts];
    __shared__ float4 tcd[kMaxLeaf], scd[kRowChunk];  // centroid (relative), diameter
    __shared__ int4 tid[kMaxLeaf], sid[kRowChunk];    // vertex ids, panel index
    __shared__ unsigned long long s_cnt[2];
    const int32_t Tb = a.leaf_box[li];
    const int32_t kb = a.box_beg[Tb], nt = a.box_end[Tb] - kb;
    const int32_t r0 = a.near_rows[li], nr = a.near_rows[li + 1] - r0;
    const int tpad = a.leaf_tpad[li];
    const int64_t vo = a.val_off[li];
    const double c0[3] = {a.cen[3 * (int64_t)kb], a.cen[3 * (int64_t)kb + 1], a.cen[3 * (int64_t)kb + 2]};
    if (threadIdx.x == 0) s_cnt[0] = s_cnt[1] = 0;
    for (int e = threadIdx.x; e < nt * kRegPts; e += blockDim.x)
        stage_points(a.pv, kb + e / kRegPts, c0, R, e % kRegPts, &tp[e]);
    for (int j = threadIdx.x; j < nt; j += blockDim.x) {
        const int32_t k = kb + j;
        tcd[j] = make_float4((float)(a.cen[3 * k] - c0[0]), (float)(a.cen[3 * k + 1] - c0[1]),
                             (float)(a.cen[3 * k + 2] - c0[2]), (float)a.diam[k]);
        tid[j] = make_int4(a.pvid[3 * k], a.pvid[3 * k + 1], a.pvid[3 * k + 2], k);
    }
    unsigned long long c_self = 0, c_reg = 0;
    const float rn2 = (float)(a.r_near * a.r_near), rm2 = (float)(a.r_mid * a.r_mid);
    for (int rc = 0; rc < nr; rc += kRowChunk) {
        const int nrc = min(kRowChunk, nr - rc);
        __syncthreads();  // the previous chunk's points are no longer read
        for (int e = threadIdx.x; e < nrc * kRegPts; e += blockDim.x)
            stage_points(a.pv, a.near_src[r0 + rc + e / kRegPts], c0, R, e % kRegPts, &spt[e]);
        for (int r = threadIdx.x; r < nrc; r += blockDim.x) {
            const int32_t l = a.near_src[r0 + rc + r];
            scd[r] = make_float4((float)(a.cen[3 * l] - c0[0]), (float)(a.cen[3 * l + 1] - c0[1]),
                                 (float)(a.cen[3 * l + 2] - c0[2]), (float)a.diam[l]);
            sid[r] = make_int4(a.pvid[3 * l], a.pvid[3 * l + 1], a.pvid[3 * l + 2], l);
        }
        __syncthreads();
        for (int e = threadIdx.x; e < nrc * tpad; e += blockDim.x) {
            const int r = e / tpad, j = e - r * tpad;
            const int64_t out = vo + (int64_t)(rc + r) * tpad + j;
            if (j >= nt) {
                val[out] = 0.f;
                continue;
            }
            const int4 ik = tid[j], il = sid[r];
            if (ik.w == il.w) {
                val[out] = (float)self_term(a.pv + 9 * (int64_t)ik.w);
                ++c_self;
                continue;
            }
            const bool touch = ik.x == il.x || ik.x == il.y || ik.x == il.z || ik.y == il.x || ik.y == il.y ||
                               ik.y == il.z || ik.z == il.x || ik.z == il.y || ik.z == il.z;
            const float4 ck = tcd[j], cl = scd[r];
            const float dx = ck.x - cl.x, dy = ck.y - cl.y, dz = ck.z - cl.z;
            const float dm = fmaxf(ck.w, cl.w);
            const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz)) / (dm * dm);
            if (touch || d2 < rn2) {
                const int64_t pos = queue_slot(a, touch ? 0 : 1);
                if (pos >= 0 && pos < a.work_cap) {
                    a.work[pos] = out;
                    a.work_meta[2 * pos] = ik.w;
                    a.work_meta[2 * pos + 1] = il.w;
                }
                val[out] = 0.f;
                continue;
            }
            ++c_reg;
            val[out] = d2 < rm2 ? product_rule<16>(&tp[j * kRegPts], &spt[r * kRegPts])
                                : product_rule<9>(&tp[j * kRegPts + 16], &spt[r * kRegPts + 16]);
        }
    }
    // padding rows of a leaf without rows do not exist; class counters: LDS
    // first, one global atomic per workgroup
    __syncthreads();
    if (c_self) atomicAdd(&s_cnt[0], c_self);
    if (c_reg) atomicAdd(&s_cnt[1], c_reg);
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(&a.counters[0], s_cnt[0]);
        atomicAdd(&a.counters[3], s_cnt[1]);
    }
}

// Pass 2: queued touching (which = 0, from the front of the queue) or
// near-singular (which = 1, from the back) entries, one per thread.
// Rule class of a near-singular pair: r < 0.75 (2), r < 1.5 (1), r < r_near (0).
__device__ inline int ns_level(const NFArgs &a, int32_t k, int32_t l)
{
    const double dx = a.cen[3 * k] - a.cen[3 * l], dy = a.cen[3 * k + 1] - a.cen[3 * l + 1],
                 dz = a.cen[3 * k + 2] - a.cen[3 * l + 2];
    const double rr = sqrt(dx * dx + dy * dy + dz * dz) / fmax(a.diam[k], a.diam[l]);
    return rr < 0.75 ? 2 : (rr < 1.5 ? 1 : 0);
}

// Near-singular entries bucketed by subdivision level, so that each launch
// of pass 2 runs one level (lanes of a wave then do equal work).  Entry i of
// the batch is queue position list[i] (or cap - 1 - i without a list).
// Pass 0 counts per level (one atomic per wave and level); pass 1 writes i
// into order[] at the running offset of its level.
__global__ void k_ns_bucket(NFArgs a, int64_t count, const int64_t *__restrict__ list, int pass,
                            unsigned long long *__restrict__ ctr, int64_t *__restrict__ order, int64_t off1,
                            int64_t off2)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int lev = -1;
    if (i < count) {
        const int64_t pos = list ? list[i] : a.work_cap - 1 - i;
        lev = ns_level(a, a.work_meta[2 * pos], a.work_meta[2 * pos + 1]);
    }
    for (int q = 0; q < 3; ++q) {
        const unsigned long long mask = __ballot(lev == q);
        if (mask == 0) continue;
        const int lane = __lane_id();
        const int leader = __ffsll((long long)mask) - 1;
        unsigned long long base = 0;
        if (lane == leader) base = atomicAdd(&ctr[q], (unsigned long long)__popcll(mask));
        base = __shfl(base, leader);
        const int64_t off = q == 0 ? 0 : (q == 1 ? off1 : off2);
        if (pass == 1 && lev == q) order[off + (int64_t)(base + __popcll(mask & ((1ull << lane) - 1ull)))] = i;
    }
}

template <typename V, typename C>
__global__ __launch_bounds__(64) void k_nf_special(NFArgs a, NFRules R, int which, int64_t count,
                                                   V *__restrict__ val, const int64_t *__restrict__ list,
                                                   const int64_t *__restrict__ order, double *__restrict__ alt_out)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= count) return;
    const int64_t i = order ? order[t] : t;
    const int64_t pos = list ? list[i] : (which == 0 ? i : a.work_cap - 1 - i);
    const int32_t k = a.work_meta[2 * pos], l = a.work_meta[2 * pos + 1];
    // coordinates relative to the target centroid
    C tv[9], sv[9];
    if (which == 0) {
        const int s0 = shared_vertex(a.pvid + 3 * (int64_t)k, a.pvid + 3 * (int64_t)l);
        for (int j = 0; j < 3; ++j)
            for (int d = 0; d < 3; ++d) tv[3 * j + d] = (C)(a.pv[9 * (int64_t)k + 3 * ((s0 + j) % 3) + d] - a.cen[3 * k + d]);
        for (int q = 0; q < 9; ++q) sv[q] = (C)(a.pv[9 * (int64_t)l + q] - a.cen[3 * k + q % 3]);
        const C v = touching_pair<C>(tv, sv, R);
        if (alt_out)
            alt_out[i] = (double)v;
        else
            val[a.work[pos]] = (V)v;
    } else {
        // P_kl = P_lk: the outer rule runs over the smaller panel and the
        // closed-form potential belongs to the larger one, so the points
        // where it is evaluated lie within a few of its diameters (far from
        // a small triangle its edge terms cancel in FP32)
        const int32_t o = a.diam[l] < a.diam[k] ? l : k, in = o == k ? l : k;
        for (int q = 0; q < 9; ++q) {
            tv[q] = (C)(a.pv[9 * (int64_t)o + q] - a.cen[3 * k + q % 3]);
            sv[q] = (C)(a.pv[9 * (int64_t)in + q] - a.cen[3 * k + q % 3]);
        }
        const C v = near_pair<C>(tv, sv, ns_level(a, k, l), R);
        if (alt_out)
            alt_out[i] = (double)v;
        else
            val[a.work[pos]] = (V)v;
    }
}

// Surrogate decision for queued near-singular entry i (queue position
// cap - 1 - i): accept P = cheap (1 + out0) when every feature lies in the
// training range and out1 <= bound, else queue the entry for quadrature.
// Every audit_every-th accepted entry is also queued for an audit.
template <typename V>
__global__ void k_ns_accept(NFArgs a, int64_t n, const float *__restrict__ feat, const double *__restrict__ cheap,
                            const float *__restrict__ out, const float *__restrict__ lo, const float *__restrict__ hi,
                            float bound, int audit_every, V *__restrict__ val, int64_t *__restrict__ fb,
                            unsigned long long *__restrict__ fbn, int64_t *__restrict__ aud,
                            double *__restrict__ aud_val, unsigned long long *__restrict__ audn)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t pos = a.work_cap - 1 - i;
    bool ok = out[2 * i + 1] <= bound && isfinite(out[2 * i]);
    for (int q = 0; q < 18 && ok; ++q) ok = feat[18 * i + q] >= lo[q] && feat[18 * i + q] <= hi[q];
    if (ok) {
        const double v = cheap[i] * (1.0 + (double)out[2 * i]);
        val[a.work[pos]] = (V)v;
        if (audit_every > 0 && i % audit_every == 0) {
            const unsigned long long j = atomicAdd(audn, 1ull);
            aud[j] = pos;
            aud_val[j] = v;
        }
    } else {
        const unsigned long long j = atomicAdd(fbn, 1ull);
        fb[j] = pos;
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
        xrl_nf_opts o{2.0, 6.0, nullptr, 0};
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
        const int nsn[2][3] = {{5, 5, 6}, {6, 6, 6}}, nsl[2][3] = {{0, 1, 1}, {0, 1, 2}};
        for (int c = 0; c < 3; ++c) {
            R.ns_n[c] = nsn[fp64][c];
            R.ns_lev[c] = nsl[fp64][c];
            gauss_legendre01(R.ns_n[c], R.nx[c], R.nw[c]);
        }
        R.n_hi = fp64 ? 5 : 4;
        R.n_lo = fp64 ? 4 : 3;
        gauss_legendre01(R.n_touch, R.gx, R.gw);
        for (int i = 0; i < R.n_touch; ++i) {
            // sigmoidal map s(u) = u^3 / (u^3 + (1-u)^3), clustering the nodes
            // at both ends of each collapsed coordinate
            const double u = R.gx[i], u3 = u * u * u, v3 = (1 - u) * (1 - u) * (1 - u);
            R.tx[i] = u3 / (u3 + v3);
            R.tw[i] = R.gw[i] * 3.0 * u * u * (1 - u) * (1 - u) / ((u3 + v3) * (u3 + v3));
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
        // queue capacity: touching + near-singular entries (bounded by all pairs)
        const int64_t cap = std::max<int64_t>(1, std::min<int64_t>(P->n_near_pairs, 160 * P->N));
        DevBuf<int64_t> work(cap);
        DevBuf<int32_t> meta(2 * cap);
        DevBuf<unsigned long long> cnt(4), wn(2);
        XRL_HIP(hipMemsetAsync(cnt.p, 0, cnt.bytes(), s));
        XRL_HIP(hipMemsetAsync(wn.p, 0, wn.bytes(), s));
        NFArgs a{P->leaf_box.p, P->box_beg.p, P->box_end.p, P->near_rows.p, P->near_src.p, P->leaf_tpad.p,
                 P->pvid.p,     P->near_val_off.p, P->pv.p, P->cen.p, P->diam.p, o.r_near, o.r_mid,
                 P->n_leaves,   cnt.p,       work.p,   meta.p,  wn.p,    cap};
        if (P->n_leaves > 0) {
            if (fp64)
                k_nf_main<double, true><<<P->n_leaves, 256, 0, s>>>(a, R, P->near64.p);
            else
                k_nf_leaf32<<<P->n_leaves, 256, 0, s>>>(a, R, P->near32.p);
            XRL_HIP(hipGetLastError());
        }
        auto hw = wn.download(s);
        XRL_CHECK((int64_t)(hw[0] + hw[1]) <= cap, XRL_E_OOM,
                  "xrl_nearfield_assemble: special-pair queue overflow (%llu + %llu > %lld)",
                  (unsigned long long)hw[0], (unsigned long long)hw[1], (long long)cap);
        // mixed precision: FP64 for the touching (adjacent-panel) pairs and
        // for the audit reference of the surrogate, FP32 (relative to the
        // target centroid, exact inner potential) for the near-singular
        // pairs that are not adjacent
        auto launch = [&](int which, int64_t count, const int64_t *list, const int64_t *order, double *alt) {
            if (count == 0) return;
            if (P->precision == XRL_PREC_FP64)
                k_nf_special<double, double><<<cdiv(count, 64), 64, 0, s>>>(a, R, which, count, P->near64.p, list,
                                                                            order, alt);
            else if (P->precision == XRL_PREC_MIXED && (which == 0 || alt))
                k_nf_special<float, double><<<cdiv(count, 64), 64, 0, s>>>(a, R, which, count, P->near32.p, list,
                                                                           order, alt);
            else
                k_nf_special<float, float><<<cdiv(count, 64), 64, 0, s>>>(a, R, which, count, P->near32.p, list,
                                                                          order, alt);
            XRL_HIP(hipGetLastError());
        };
        // touching entries in queue order; near-singular entries one
        // subdivision level per launch
        auto special = [&](int which, int64_t count, const int64_t *list, double *alt) {
            if (count == 0) return;
            if (which == 0) {
                launch(0, count, list, nullptr, alt);
                return;
            }
            DevBuf<unsigned long long> ctr(6);
            DevBuf<int64_t> order(count);
            XRL_HIP(hipMemsetAsync(ctr.p, 0, ctr.bytes(), s));
            k_ns_bucket<<<cdiv(count, 256), 256, 0, s>>>(a, count, list, 0, ctr.p, nullptr, 0, 0);
            XRL_HIP(hipGetLastError());
            auto n = ctr.download(s, 3);
            const int64_t off[3] = {0, (int64_t)n[0], (int64_t)(n[0] + n[1])};
            k_ns_bucket<<<cdiv(count, 256), 256, 0, s>>>(a, count, list, 1, ctr.p + 3, order.p, off[1], off[2]);
            XRL_HIP(hipGetLastError());
            for (int q = 2; q >= 0; --q) launch(1, (int64_t)n[q], list, order.p + off[q], alt);
            XRL_HIP(hipStreamSynchronize(s));  // order[] lives until the launches are done
        };
        special(0, (int64_t)hw[0], nullptr, nullptr);
        int64_t n_acc = 0, n_fb = (int64_t)hw[1];
        double aud_max = 0, aud_rms = 0;
        if (o.surrogate && hw[1] > 0) {
            const int64_t nns = (int64_t)hw[1];
            MlpDevice mlp;
            mlp_prepare_host(mlp, o.surrogate, s);
            DevBuf<float> feat(18 * nns), out(2 * nns), lo, hi;
            DevBuf<double> cheap(nns), aud_val(nns), aud_ref(nns), rel(nns);
            DevBuf<int64_t> fb(nns), aud(nns);
            DevBuf<unsigned long long> fbn(2);
            lo.upload(o.surrogate->feat_lo, 18, s);
            hi.upload(o.surrogate->feat_hi, 18, s);
            XRL_HIP(hipMemsetAsync(fbn.p, 0, fbn.bytes(), s));
            ns_features(a, nns, feat.p, cheap.p, s);
            mlp_infer(mlp, feat.p, nns, out.p, s);
            if (fp64)
                k_ns_accept<double><<<cdiv(nns, 256), 256, 0, s>>>(a, nns, feat.p, cheap.p, out.p, lo.p, hi.p,
                                                                  o.surrogate->log10_err_bound, o.audit_every,
                                                                  P->near64.p, fb.p, fbn.p, aud.p, aud_val.p,
                                                                  fbn.p + 1);
            else
                k_ns_accept<float><<<cdiv(nns, 256), 256, 0, s>>>(a, nns, feat.p, cheap.p, out.p, lo.p, hi.p,
                                                                 o.surrogate->log10_err_bound, o.audit_every,
                                                                 P->near32.p, fb.p, fbn.p, aud.p, aud_val.p,
                                                                 fbn.p + 1);
            XRL_HIP(hipGetLastError());
            auto hn = fbn.download(s);
            n_fb = (int64_t)hn[0];
            n_acc = nns - n_fb;
            special(1, n_fb, fb.p, nullptr);
            const int64_t na = (int64_t)hn[1];
            if (na > 0) {
                special(1, na, aud.p, aud_ref.p);
                k_audit_err<<<cdiv(na, 256), 256, 0, s>>>(aud_ref.p, aud_val.p, na, rel.p);
                auto hr = rel.download(s, na);
                double ss = 0;
                for (double r : hr) {
                    aud_max = std::max(aud_max, r);
                    ss += r * r;
                }
                aud_rms = std::sqrt(ss / na);
            }
        } else {
            special(1, (int64_t)hw[1], nullptr, nullptr);
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
            stats->n_touching = (int64_t)hw[0];
            stats->n_near_singular = (int64_t)hw[1];
            stats->n_regular = (int64_t)hc[3];
            stats->n_mlp_accepted = n_acc;
            stats->n_mlp_fallback = o.surrogate ? n_fb : 0;
            stats->audit_max_rel_err = aud_max;
            stats->audit_rms_rel_err = aud_rms;
            stats->ms = ms;
        }
    });
}
