// The FMM-accelerated panel matvec y = P x (eq. (9): FMM applies P to the
// panel densities I_pt, Sec. II-C).  Densities and potentials are complex;
// P is real, so a complex column is carried as two real columns.
//
// Phases (all on the caller's stream):
//   gather   user order, complex -> Morton order, real columns   xs[N][C]
//   P2P      y  = P_near x (stored near-field blocks)             ys[N][C]
//   P2M      M_leaf = sum_k Q_k x_k (exact panel moments)         M[B][K][C]
//   M2M      parents from children, deepest level first  } grouped GEMMs, one
//   M2L      L_t = sum_{s in V(t)} T_{o(t,s)} M_s         } operator per group,
//   L2L      children from parents, top level first      } MFMA or vector ALU
//   L2P      y += (1/h) sum_i w_i Q_k[i] L_leaf[i]  (Galerkin-tested local)
//   scatter  y_user = alpha_c y + beta_c A .* x_user
#include <algorithm>
#include <cmath>
#include <functional>
#include <mutex>
#include <type_traits>

#include "common.h"

namespace xrl {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- gather / scatter
// One thread per complex density: one load of the (re, im) pair when the
// caller's array is aligned to a pair (PAIR), else two scalar loads.
template <typename TI, typename TW, bool PAIR>
__global__ void k_gather_x(int64_t N, const int32_t *__restrict__ perm, const TI *__restrict__ x, int64_t ldx,
                           int ncols, TW *__restrict__ xs)
{
    typedef TI TI2 __attribute__((ext_vector_type(2)));
    typedef TW TW2 __attribute__((ext_vector_type(2)));
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N * ncols;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = e / ncols;
        const int c = (int)(e - i * ncols);
        const int64_t u = perm[i];
        TI re, im;
        if constexpr (PAIR) {
            const TI2 v = reinterpret_cast<const TI2 *>(x)[u * ldx + c];
            re = v[0];
            im = v[1];
        } else {
            re = x[2 * (u * ldx + c)];
            im = x[2 * (u * ldx + c) + 1];
        }
        reinterpret_cast<TW2 *>(xs)[e] = TW2{(TW)re, (TW)im};
    }
}

// One thread per (user panel, column): the potential of the panel's element
// (or the sum over the two elements of a four-sided panel, iperm2 >= 0),
// then the epilogue with the panel's area.
template <typename TO, typename TW>
__global__ void k_scatter_y(int64_t Nu, const int32_t *__restrict__ iperm, const int32_t *__restrict__ iperm2,
                            const TW *__restrict__ ys, const double *__restrict__ area, const TO *__restrict__ x,
                            int64_t ldx, TO *__restrict__ y, int64_t ldy, int ncols, const double *__restrict__ alpha,
                            const double *__restrict__ beta)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < Nu * ncols;
         e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t u = e / ncols;
    const int c = (int)(e - u * ncols);
    const int64_t i = iperm[u];
    double pr = (double)ys[i * 2 * ncols + 2 * c], pi = (double)ys[i * 2 * ncols + 2 * c + 1];
    double A = area[i];
    if (iperm2) {
        const int64_t i2 = iperm2[u];
        if (i2 >= 0) {
            pr += (double)ys[i2 * 2 * ncols + 2 * c];
            pi += (double)ys[i2 * 2 * ncols + 2 * c + 1];
            A += area[i2];
        }
    }
    double ar = 1, ai = 0, br = 0, bi = 0;
    if (alpha) {
        ar = alpha[2 * c];
        ai = alpha[2 * c + 1];
    }
    double yr = ar * pr - ai * pi, yi = ar * pi + ai * pr;
    if (beta) {
        br = beta[2 * c];
        bi = beta[2 * c + 1];
        const double xr = (double)x[2 * (u * ldx + c)], xi = (double)x[2 * (u * ldx + c) + 1];
        yr += A * (br * xr - bi * xi);
        yi += A * (br * xi + bi * xr);
    }
    y[2 * (u * ldy + c)] = (TO)yr;
    y[2 * (u * ldy + c) + 1] = (TO)yi;
    }
}

// Raw buffer loads: a wave-uniform base goes into the (scalar) resource,
// the lane part into one vector offset and a uniform per-step part into the
// scalar offset, so the address arithmetic stays off the vector ALU.  An
// access whose vector offset lies past the record count returns zeros
// instead of reading memory.
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

template <int W>
struct Words {
    uint32_t w[W];
};

template <int W>
__device__ inline Words<W> buf_load_words(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    Words<W> o;
    if constexpr (W == 1) {
        o.w[0] = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
    } else if constexpr (W == 2) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
        o.w[0] = v[0];
        o.w[1] = v[1];
    } else if constexpr (W == 3) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b96(r, voff, soff, 0);
        o.w[0] = v[0];
        o.w[1] = v[1];
        o.w[2] = v[2];
    } else if constexpr (W == 4) {
        const auto v = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
        o.w[0] = v[0];
        o.w[1] = v[1];
        o.w[2] = v[2];
        o.w[3] = v[3];
    } else {
        const Words<4> a = buf_load_words<4>(r, voff, soff);
        const Words<W - 4> b = buf_load_words<W - 4>(r, voff + 16, soff);
        for (int i = 0; i < 4; ++i) o.w[i] = a.w[i];
        for (int i = 0; i < W - 4; ++i) o.w[4 + i] = b.w[i];
    }
    return o;
}

// A value of type V (a whole number of 32-bit words) by one buffer load.
template <typename V>
__device__ inline V buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff)
{
    static_assert(sizeof(V) % 4 == 0, "word-sized values only");
    return __builtin_bit_cast(V, buf_load_words<sizeof(V) / 4>(r, voff, soff));
}

// ---------------------------------------------------------------- P2P
// One workgroup per (target leaf, column tile).  The stored block of a leaf
// is [rows][tpad] (tpad a multiple of 4); a thread owns VEC consecutive
// targets of one row (one 16-byte load) and the tpad/VEC threads of a row
// group stride over the rows (threads past the last whole group idle).
// Source indices and the source densities of a chunk of 256 rows are staged
// in LDS first, so the value stream is the only global load in the inner
// loop.  The row groups are summed in a fixed order at the end.
template <typename T, int CT>
__global__ __launch_bounds__(256) void k_p2p(const int32_t *__restrict__ leaf_box, const int32_t *__restrict__ box_beg,
                                             const int32_t *__restrict__ box_end, const int32_t *__restrict__ near_rows,
                                             const int32_t *__restrict__ near_src, const int32_t *__restrict__ leaf_tpad,
                                             const int64_t *__restrict__ val_off, const T *__restrict__ val,
                                             const T *__restrict__ xs, T *__restrict__ ys, int C)
{
    constexpr int VEC = 16 / sizeof(T);
    constexpr int ROWS = 256;
    using V4 = typename std::conditional<sizeof(T) == 4, f32x4, double __attribute__((ext_vector_type(2)))>::type;
    __shared__ T sx[ROWS * CT];
    __shared__ T red[256 * VEC * CT];
    const int64_t li = blockIdx.x;
    const int c0 = blockIdx.y * CT;
    const int32_t tb = leaf_box[li];
    const int32_t kb = box_beg[tb], nt = box_end[tb] - kb;
    const int32_t r0 = near_rows[li], nr = near_rows[li + 1] - r0;
    const int G = leaf_tpad[li];
    const int tpr = G / VEC;          // threads per row
    const int groups = 256 / tpr;     // rows in flight per pass
    const int jv = (threadIdx.x % tpr) * VEC, grp = threadIdx.x / tpr;
    const T *vb = val + val_off[li];
    T acc[VEC][CT];
#pragma unroll
    for (int v = 0; v < VEC; ++v)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[v][c] = 0;
    for (int32_t rc = 0; rc < nr; rc += ROWS) {
        const int nrc = min(ROWS, nr - rc);
        __syncthreads();
        for (int i = threadIdx.x; i < nrc * CT; i += 256) {
            const int r = i / CT, c = i - r * CT;
            sx[i] = (c0 + c < C) ? xs[(int64_t)near_src[r0 + rc + r] * C + c0 + c] : T(0);
        }
        __syncthreads();
#pragma unroll 4
        for (int r = grp < groups ? grp : nrc; r < nrc; r += groups) {
            const V4 v = *reinterpret_cast<const V4 *>(vb + (int64_t)(rc + r) * G + jv);
            const T *xr = sx + r * CT;
#pragma unroll
            for (int c = 0; c < CT; ++c) {
                const T xv = xr[c];
#pragma unroll
                for (int e = 0; e < VEC; ++e) acc[e][c] += v[e] * xv;
            }
        }
    }
    if (grp < groups)
#pragma unroll
        for (int e = 0; e < VEC; ++e)
#pragma unroll
            for (int c = 0; c < CT; ++c) red[(grp * G + jv + e) * CT + c] = acc[e][c];
    __syncthreads();
    for (int idx = threadIdx.x; idx < nt * CT; idx += 256) {
        const int jj = idx / CT, c = idx - jj * CT;
        if (c0 + c >= C) continue;
        T sum = 0;
        for (int g = 0; g < groups; ++g) sum += red[(g * G + jj) * CT + c];
        ys[(int64_t)(kb + jj) * C + c0 + c] = sum;
    }
}

// Wide-column form (FP32, C > 16): one workgroup per (leaf, tile of up to
// CT columns), so the value stream of a leaf is read once for every 48
// columns.  A thread owns VT consecutive targets of a row (one vector
// load) and all CT columns; the row groups are summed through LDS in chunks
// of RC columns, in a fixed order.
template <int CT>
__global__ __launch_bounds__(256) void k_p2p_wide(const int32_t *__restrict__ leaf_box,
                                                  const int32_t *__restrict__ box_beg,
                                                  const int32_t *__restrict__ box_end,
                                                  const int32_t *__restrict__ near_rows,
                                                  const int32_t *__restrict__ near_src,
                                                  const int32_t *__restrict__ leaf_tpad,
                                                  const int64_t *__restrict__ val_off, const float *__restrict__ val,
                                                  const float *__restrict__ xs, float *__restrict__ ys, int C)
{
    constexpr int VT = 2, ROWS = 64, RC = 12;
    __shared__ __align__(16) float sx[ROWS * CT];
    __shared__ float red[256 * VT * RC];
    const int64_t li = blockIdx.x;
    const int c0 = blockIdx.y * CT;
    const int32_t tb = leaf_box[li];
    const int32_t kb = box_beg[tb], nt = box_end[tb] - kb;
    const int32_t r0 = near_rows[li], nr = near_rows[li + 1] - r0;
    const int G = leaf_tpad[li];
    const int tpr = G / VT, groups = 256 / tpr;
    const int jv = (threadIdx.x % tpr) * VT, grp = threadIdx.x / tpr;
    const bool in_group = grp < groups;  // threads past the last whole row group idle
    const float *vb = val + val_off[li];
    float acc[VT][CT];
#pragma unroll
    for (int v = 0; v < VT; ++v)
#pragma unroll
        for (int c = 0; c < CT; ++c) acc[v][c] = 0.f;
    // the source densities and the block values of the next chunk are
    // fetched into registers while the current chunk is multiplied out, so
    // every thread keeps a whole chunk of loads in flight
    typedef float fv_t __attribute__((ext_vector_type(VT)));
    constexpr int PER = ROWS * CT / 256;
    constexpr int RMAX = ROWS * kMaxLeaf / (256 * VT);  // rows per thread and chunk at the widest block
    float xn[PER];
    fv_t vn[RMAX], vc[RMAX];
    auto fetch = [&](int rc) {
        const int nrc = min(ROWS, nr - rc);
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = threadIdx.x + 256 * q, r = i / CT, c = i - r * CT;
            xn[q] = (r < nrc && c0 + c < C) ? xs[(int64_t)near_src[r0 + rc + r] * C + c0 + c] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < RMAX; ++q) {
            const int r = grp + q * groups;
            vn[q] = (in_group && r < nrc) ? *reinterpret_cast<const fv_t *>(vb + (int64_t)(rc + r) * G + jv)
                                          : fv_t(0.f);
        }
    };
    if (nr > 0) fetch(0);
    for (int32_t rc = 0; rc < nr; rc += ROWS) {
        const int nrc = min(ROWS, nr - rc);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) sx[threadIdx.x + 256 * q] = xn[q];
#pragma unroll
        for (int q = 0; q < RMAX; ++q) vc[q] = vn[q];
        __syncthreads();
        if (rc + ROWS < nr) fetch(rc + ROWS);
#pragma unroll
        for (int q = 0; q < RMAX; ++q) {
            const int r = grp + q * groups;
            if (!in_group || r >= nrc) break;
            const fv_t v = vc[q];
            const f32x4 *xr = reinterpret_cast<const f32x4 *>(sx + r * CT);
#pragma unroll
            for (int c4 = 0; c4 < CT / 4; ++c4) {
                const f32x4 xv = xr[c4];
#pragma unroll
                for (int e = 0; e < 4; ++e)
#pragma unroll
                    for (int t = 0; t < VT; ++t) acc[t][4 * c4 + e] += v[t] * xv[e];
            }
        }
    }
#pragma unroll
    for (int cc = 0; cc < CT; cc += RC) {
        __syncthreads();
        if (in_group)
#pragma unroll
            for (int v = 0; v < VT; ++v)
#pragma unroll
                for (int c = 0; c < RC; ++c)
                    if (cc + c < CT) red[(grp * G + jv + v) * RC + c] = acc[v][cc + c];
        __syncthreads();
        for (int idx = threadIdx.x; idx < nt * RC; idx += 256) {
            const int jj = idx / RC, c = idx - jj * RC;
            if (cc + c >= CT || c0 + cc + c >= C) continue;
            float sum = 0.f;
            for (int g = 0; g < groups; ++g) sum += red[(g * G + jj) * RC + c];
            ys[(int64_t)(kb + jj) * C + c0 + cc + c] = sum;
        }
    }
}

// Scalar-density form (FP32, C > 16): one wave per (leaf, tile of CT
// columns), lane = target of the leaf block.  A source row's densities are
// the same for every lane, so they come in through scalar loads and enter
// the FMAs as SGPR operands: no LDS traffic, and each lane's block value
// (one coalesced 4-byte load per row) feeds CT FMAs.  Lanes past the block
// width idle (the price for leaves of 16 or 32 targets).
template <int CT>
__global__ __launch_bounds__(64) void k_p2p_sx(const int32_t *__restrict__ leaf_box,
                                               const int32_t *__restrict__ box_beg,
                                               const int32_t *__restrict__ box_end,
                                               const int32_t *__restrict__ near_rows,
                                               const int32_t *__restrict__ near_src,
                                               const int32_t *__restrict__ leaf_tpad,
                                               const int64_t *__restrict__ val_off, const float *__restrict__ val,
                                               const float *__restrict__ xs, float *__restrict__ ys, int C)
{
    const int li = blockIdx.x;
    const int c0 = blockIdx.y * CT;
    const int lane = threadIdx.x;
    const int32_t tb = leaf_box[li];
    const int32_t kb = box_beg[tb], nt = box_end[tb] - kb;
    const int32_t r0 = near_rows[li], nr = near_rows[li + 1] - r0;
    const int G = leaf_tpad[li];
    const int ncol = min(CT, C - c0);
    // blocks wider than a wave: one pass per 64 targets
    for (int t0 = 0; t0 < G; t0 += 64) {
    const int t = t0 + lane;
    const bool act = t < G;
    const float *vb = val + val_off[li] + (act ? t : 0);
    float acc[CT];
#pragma unroll
    for (int c = 0; c < CT; ++c) acc[c] = 0.f;
    if (ncol == CT) {
#pragma unroll 2
        for (int r = 0; r < nr; ++r) {
            const float *xr = xs + (int64_t)near_src[r0 + r] * C + c0;
            const float v = act ? vb[(int64_t)r * G] : 0.f;
#pragma unroll
            for (int c = 0; c < CT; ++c) acc[c] += v * xr[c];
        }
    } else {
        for (int r = 0; r < nr; ++r) {
            const float *xr = xs + (int64_t)near_src[r0 + r] * C + c0;
            const float v = act ? vb[(int64_t)r * G] : 0.f;
#pragma unroll
            for (int c = 0; c < CT; ++c)
                if (c < ncol) acc[c] += v * xr[c];
        }
    }
    if (t < nt) {
        float *yo = ys + (int64_t)(kb + t) * C + c0;
#pragma unroll
        for (int c = 0; c < CT; ++c)
            if (c < ncol) yo[c] = acc[c];
    }
    }
}

// Matrix-core form (FP32, C > 16): the near field of a leaf is the dense
// product Y[t][c] = sum over rows r of V[r][t] X[src_r][c], so it runs on
// the 16x16x4 MFMA with the densities as A (16 columns x 4 rows) and the
// stored block as B (4 rows x 16 targets).  One wave per (leaf, item of WT
// column tiles, plus XC = 4 narrow columns on 4x4x1 blocks as in the
// target-stationary translation).  A lane (li, kq) takes row 4 ks + kq of
// every k step: targets li, 16 + li, ..., 16 (E - 1) + li of it, E =
// ceil(G / 16) for the block width G (one word each; target 16 e + li goes
// to target tile e), and WT consecutive densities (column cb + WT li + ct to
// column tile ct).  Targets past G read the start of the next row and feed
// only results that are not stored; rows past the block read as zeros
// (range-checked buffer loads, one word each, so the check is exact), and
// so do their source indices, which then point at source 0: every product
// with a missing row is zero.
template <int WT, int XC, int E>
__device__ inline void p2p_mfma_leaf(int lane, int nr, int G, const float *__restrict__ vb,
                                     const int32_t *__restrict__ srcs, const float *__restrict__ xs, int C, int cb,
                                     float *__restrict__ ys, int64_t kb, int nt)
{
    constexpr int U = 4;  // k steps per stage
    using VE = Words<E>;  // a row's values of the lane's E targets
    struct BV {
        float v[WT];
    };
    struct Stage {
        VE v[U];
        BV b[U];
        float xn[U];
    };
    const int li = lane & 15, kq = lane >> 4;
    f32x4 acc[E][WT], accx[XC ? E : 1];
#pragma unroll
    for (int e = 0; e < E; ++e) {
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) acc[e][ct] = f32x4{0, 0, 0, 0};
        if (XC || e == 0) accx[XC ? e : 0] = f32x4{0, 0, 0, 0};
    }
    const auto rv = buf_rsrc(vb, (uint32_t)nr * G * 4);
    const auto rs = buf_rsrc(srcs, (uint32_t)nr * 4);
    const int xo = cb + WT * li, xno = cb + 16 * WT + (li & 3);
    // source rows of a stage, fetched two stages ahead, so that the
    // densities they index can be requested as soon as the stage is due
    struct Src {
        int r[U];
    };
    auto load_src = [&](int ks0, Src &sr) {
#pragma unroll
        for (int u = 0; u < U; ++u) sr.r[u] = buf_load<int>(rs, (4 * (ks0 + u) + kq) * 4, 0);
    };
    auto load = [&](int ks0, const Src &sr, Stage &st) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int r = 4 * (ks0 + u) + kq;
#pragma unroll
            for (int e = 0; e < E; ++e) st.v[u].w[e] = buf_load_words<1>(rv, (r * G + 16 * e + li) * 4, 0).w[0];
            const float *xr = xs + (int64_t)sr.r[u] * C;
            st.b[u] = *reinterpret_cast<const BV *>(xr + xo);
            if constexpr (XC > 0) st.xn[u] = xr[xno];
        }
    };
    auto comp = [&](const Stage &st) {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const float bv = __uint_as_float(st.v[u].w[e]);
#pragma unroll
                for (int ct = 0; ct < WT; ++ct)
                    acc[e][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(st.b[u].v[ct], bv, acc[e][ct], 0, 0, 0);
                if constexpr (XC > 0) accx[e] = __builtin_amdgcn_mfma_f32_4x4x1f32(st.xn[u], bv, accx[e], 0, 0, 0);
            }
    };
    // whole trips of 2 U k steps (the rows past the block read as zeros), so
    // the loop has one exit and the accumulators stay where the MFMAs put
    // them
    const int ntrip = (nr + 8 * U - 1) / (8 * U);
    Stage s0, s1;
    Src ra, rb;
    load_src(0, ra);
    load(0, ra, s0);
    load_src(U, rb);
    for (int q = 0; q < ntrip; ++q) {
        const int ks = 2 * U * q;
        load_src(ks + 2 * U, ra);
        load(ks + U, rb, s1);
        comp(s0);
        load_src(ks + 3 * U, rb);
        load(ks + 2 * U, ra, s0);
        comp(s1);
    }
    // D[i][j] of tile (e, ct) at lane j + 16 q, element i - 4 q: column
    // cb + WT i + ct, target 16 e + j
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int t = 16 * e + li;
#pragma unroll
        for (int ct = 0; ct < WT; ++ct)
#pragma unroll
            for (int e4 = 0; e4 < 4; ++e4) {
                const int col = cb + WT * (4 * kq + e4) + ct;
                if (t < nt && col < C) ys[(kb + t) * C + col] = acc[e][ct][e4];
            }
        if constexpr (XC > 0) {
            // block accumulators: lane (li, kq) holds target 16 e + li and
            // narrow columns 0..3 in elements 0..3 for its k-subset; after the
            // sum over the four k-subsets it stores column kq
            f32x4 v = accx[e];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v[i] += __shfl_xor(v[i], 16);
                v[i] += __shfl_xor(v[i], 32);
            }
            const float mine = kq == 0 ? v[0] : kq == 1 ? v[1] : kq == 2 ? v[2] : v[3];
            const int col = cb + 16 * WT + kq;
            if (t < nt && col < C) ys[(kb + t) * C + col] = mine;
        }
    }
}

// three full column tiles (C = 48) fit three waves per SIMD (168 registers)
template <int WT, int XC>
constexpr int p2p_min_waves()
{
    return WT == 3 && XC == 0 ? 3 : 1;
}

template <int WT, int XC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(p2p_min_waves<WT, XC>()))) void k_p2p_mfma(
    int items_per_leaf, const int32_t *__restrict__ leaf_box,
                                                 const int32_t *__restrict__ box_beg,
                                                 const int32_t *__restrict__ box_end,
                                                 const int32_t *__restrict__ near_rows,
                                                 const int32_t *__restrict__ near_src,
                                                 const int32_t *__restrict__ leaf_tpad,
                                                 const int64_t *__restrict__ val_off, const float *__restrict__ val,
                                                 const float *__restrict__ xs, float *__restrict__ ys, int C)
{
    const int w = blockIdx.x;
    const int li = w / items_per_leaf;
    const int cb = (w - li * items_per_leaf) * 16 * WT;
    const int lane = threadIdx.x;
    const int32_t tb = leaf_box[li];
    const int32_t kb = box_beg[tb], nt = box_end[tb] - kb;
    const int32_t r0 = near_rows[li], nr = near_rows[li + 1] - r0;
    const float *vb = val + val_off[li];
    const int G = leaf_tpad[li];  // 4..128
    const int32_t *sr = near_src + r0;
    switch ((G + 15) >> 4) {
        case 1: p2p_mfma_leaf<WT, XC, 1>(lane, nr, G, vb, sr, xs, C, cb, ys, kb, nt); break;
        case 2: p2p_mfma_leaf<WT, XC, 2>(lane, nr, G, vb, sr, xs, C, cb, ys, kb, nt); break;
        case 3: p2p_mfma_leaf<WT, XC, 3>(lane, nr, G, vb, sr, xs, C, cb, ys, kb, nt); break;
        case 4: p2p_mfma_leaf<WT, XC, 4>(lane, nr, G, vb, sr, xs, C, cb, ys, kb, nt); break;
        case 5: p2p_mfma_leaf<WT, XC, 5>(lane, nr, G, vb, sr, xs, C, cb, ys, kb, nt); break;
        case 6: p2p_mfma_leaf<WT, XC, 6>(lane, nr, G, vb, sr, xs, C, cb, ys, kb, nt); break;
        case 7: p2p_mfma_leaf<WT, XC, 7>(lane, nr, G, vb, sr, xs, C, cb, ys, kb, nt); break;
        default: p2p_mfma_leaf<WT, XC, 8>(lane, nr, G, vb, sr, xs, C, cb, ys, kb, nt); break;
    }
}

// ---------------------------------------------------------------- P2M
// One workgroup per (leaf, tile of CT columns):
//     M[b][i][c] = sum over the leaf's panels k of mom[k][i] x[k][c].
// The panels' moment rows and densities are staged in LDS in chunks of NP
// panels (any leaf size); a thread owns one coefficient i and four
// consecutive columns, so each staged moment feeds four FMAs.
constexpr int kP2MPanels = 32;
constexpr int kMaxK = 169;  // (p + 1)^2 at the largest supported order, 12

template <typename T, int CT>
__global__ __launch_bounds__(256) void k_p2m(const int32_t *__restrict__ leaf_box, const int32_t *__restrict__ box_beg,
                                             const int32_t *__restrict__ box_end, const T *__restrict__ mom,
                                             const T *__restrict__ xs, T *__restrict__ M, int C, int K)
{
    constexpr int NP = kP2MPanels, NQ = CT / 4;
    constexpr int MAXO = (kMaxK * NQ + 255) / 256;  // outputs (of four columns) per thread
    using V4 = typename std::conditional<sizeof(T) == 4, f32x4, f64x4>::type;
    __shared__ T smom[NP * kMaxK];
    __shared__ __align__(16) T sx[NP * CT];
    const int32_t b = leaf_box[blockIdx.x];
    const int c0 = blockIdx.y * CT;
    const int32_t kb = box_beg[b], nt = box_end[b] - kb;
    V4 acc[MAXO];
#pragma unroll
    for (int o = 0; o < MAXO; ++o) acc[o] = V4{0, 0, 0, 0};
    for (int kc = 0; kc < nt; kc += NP) {
        const int nk = min(NP, nt - kc);
        __syncthreads();
        for (int idx = threadIdx.x; idx < nk * K; idx += 256) smom[idx] = mom[(int64_t)(kb + kc) * K + idx];
        for (int idx = threadIdx.x; idx < nk * CT; idx += 256) {
            const int k = idx / CT, c = idx - k * CT;
            sx[idx] = (c0 + c < C) ? xs[(int64_t)(kb + kc + k) * C + c0 + c] : T(0);
        }
        __syncthreads();
#pragma unroll
        for (int o = 0; o < MAXO; ++o) {
            const int idx = threadIdx.x + 256 * o;
            if (idx >= K * NQ) break;
            const int i = idx / NQ, q = idx - i * NQ;
            for (int k = 0; k < nk; ++k) {
                const T m = smom[k * K + i];
                const V4 xv = *reinterpret_cast<const V4 *>(sx + k * CT + 4 * q);
                acc[o] += m * xv;
            }
        }
    }
#pragma unroll
    for (int o = 0; o < MAXO; ++o) {
        const int idx = threadIdx.x + 256 * o;
        if (idx >= K * NQ) break;
        const int i = idx / NQ, q = idx - i * NQ;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = c0 + 4 * q + e;
            if (c < C) M[((int64_t)b * K + i) * C + c] = acc[o][e];
        }
    }
}

// Matrix-core form (FP32, C > 16): per leaf, M[i][c] = sum over the
// leaf's panels t of Q[t][i] X[t][c], the moment table as A (16
// coefficients x 4 panels, a coalesced row segment per panel) and the
// densities as B (loaded once per item and reused for every coefficient
// tile); narrow columns (XC = 4) on 4x4x1 blocks.  Panels past the leaf read
// as zeros (range-checked buffer loads), so do coefficients past the last
// panel's row; rows past K are not stored.
template <int ORD, int WT, int XC>
__global__ __launch_bounds__(64) void k_p2m_mfma(int items_per_leaf, const int32_t *__restrict__ leaf_box,
                                                 const int32_t *__restrict__ box_beg,
                                                 const int32_t *__restrict__ box_end, const float *__restrict__ mom,
                                                 const float *__restrict__ xs, float *__restrict__ M, int C)
{
    constexpr int K = (ORD + 1) * (ORD + 1), NRT = (K + 15) / 16;
    struct BV {
        float v[WT];
    };
    // operands of one k step: the moments of panel 4 ks + kq for every
    // coefficient tile, and its densities
    struct Step {
        float a[NRT];
        BV b;
        float x;
    };
    const int w = blockIdx.x;
    const int li_leaf = w / items_per_leaf;
    const int cb = (w - li_leaf * items_per_leaf) * 16 * WT, cn = cb + 16 * WT;
    const int lane = threadIdx.x, li = lane & 15, kq = lane >> 4;
    const int32_t b = leaf_box[li_leaf];
    const int32_t kb = box_beg[b], nt = box_end[b] - kb;
    const auto rx = buf_rsrc(xs + (int64_t)kb * C, (uint32_t)(nt * C * 4));
    const auto rq = buf_rsrc(mom + (int64_t)kb * K, (uint32_t)(nt * K * 4));
    auto load = [&](int ks, Step &st) {
        const int t = 4 * ks + kq;
#pragma unroll
        for (int it = 0; it < NRT; ++it) st.a[it] = buf_load<float>(rq, (t * K + 16 * it + li) * 4, 0);
        st.b = buf_load<BV>(rx, (t * C + cb + WT * li) * 4, 0);
        if constexpr (XC > 0) st.x = buf_load<float>(rx, (t * C + cn + (li & 3)) * 4, 0);
    };
    f32x4 acc[NRT][WT], accx[XC ? NRT : 1];
#pragma unroll
    for (int it = 0; it < NRT; ++it) {
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) acc[it][ct] = f32x4{0, 0, 0, 0};
        if (XC || it == 0) accx[XC ? it : 0] = f32x4{0, 0, 0, 0};
    }
    auto comp = [&](const Step &st) {
#pragma unroll
        for (int it = 0; it < NRT; ++it) {
#pragma unroll
            for (int ct = 0; ct < WT; ++ct)
                acc[it][ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(st.a[it], st.b.v[ct], acc[it][ct], 0, 0, 0);
            if constexpr (XC > 0) accx[it] = __builtin_amdgcn_mfma_f32_4x4x1f32(st.a[it], st.x, accx[it], 0, 0, 0);
        }
    };
    // a ring of four k steps in flight (one wave per leaf: the loads of the
    // next steps cover each step's latency); steps past the leaf read zeros
    // (range-checked loads) and are not computed
    const int nks = (nt + 3) / 4;
    Step s0, s1, s2, s3;
    load(0, s0);
    load(1, s1);
    load(2, s2);
    load(3, s3);
    for (int ks = 0; ks < nks; ks += 4) {
        comp(s0);
        load(ks + 4, s0);
        if (ks + 1 < nks) comp(s1);
        load(ks + 5, s1);
        if (ks + 2 < nks) comp(s2);
        load(ks + 6, s2);
        if (ks + 3 < nks) comp(s3);
        load(ks + 7, s3);
    }
    float *Mb = M + (int64_t)b * K * C;
#pragma unroll
    for (int it = 0; it < NRT; ++it) {
        // D[i][j] at lane j + 16 q, element i - 4 q: coefficient 16 it + i,
        // column cb + WT j + ct
#pragma unroll
        for (int ct = 0; ct < WT; ++ct)
#pragma unroll
            for (int e4 = 0; e4 < 4; ++e4) {
                const int i = 16 * it + 4 * kq + e4, col = cb + WT * li + ct;
                if (i < K && col < C) Mb[i * C + col] = acc[it][ct][e4];
            }
        if constexpr (XC > 0) {
            f32x4 v = accx[it];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v[i] += __shfl_xor(v[i], 16);
                v[i] += __shfl_xor(v[i], 32);
            }
            const float mine = kq == 0 ? v[0] : kq == 1 ? v[1] : kq == 2 ? v[2] : v[3];
            const int i = 16 * it + 4 * (li >> 2) + kq, col = cn + (li & 3);
            if (i < K && col < C) Mb[i * C + col] = mine;
        }
    }
}

// ---------------------------------------------------------------- L2P
template <typename T, int CT>
__global__ __launch_bounds__(256) void k_l2p(const int32_t *__restrict__ leaf_box, const int32_t *__restrict__ box_beg,
                                             const int32_t *__restrict__ box_end, const double *__restrict__ hbox,
                                             const T *__restrict__ mom, const T *__restrict__ L, T *__restrict__ ys,
                                             int C, int K)
{
    extern __shared__ unsigned char smem_raw[];
    T *sl = reinterpret_cast<T *>(smem_raw);  // [K][CT]
    const int32_t b = leaf_box[blockIdx.x];
    const int c0 = blockIdx.y * CT;
    const int32_t kb = box_beg[b], nt = box_end[b] - kb;
    const T ih = T(1.0 / hbox[b]);
    for (int idx = threadIdx.x; idx < K * CT; idx += blockDim.x) {
        const int i = idx / CT, c = idx - i * CT;
        int n = 0;
        while ((n + 1) * (n + 1) <= i) ++n;
        const T w = (i == n * n) ? T(1) : T(2);
        sl[idx] = (c0 + c < C) ? w * ih * L[((int64_t)b * K + i) * C + c0 + c] : T(0);
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < nt * CT; idx += blockDim.x) {
        const int k = idx / CT, c = idx - k * CT;
        if (c0 + c >= C) continue;
        const T *q = mom + (int64_t)(kb + k) * K;
        T acc = 0;
        for (int i = 0; i < K; ++i) acc += q[i] * sl[i * CT + c];
        ys[(int64_t)(kb + k) * C + c0 + c] += acc;
    }
}

// Matrix-core form (FP32, C > 16): per leaf, y[t][c] += sum over i of
// Q[t][i] (w_i / h) L[i][c], the moment table as A (16 targets x 4
// coefficients) and the weighted local expansion as B.  Lane (li, kq) takes
// the NKS consecutive coefficients NKS kq .. NKS kq + NKS - 1, so its moments
// are contiguous; coefficients past K get a zero moment (their local row is
// clamped to K - 1).  The expansion fragments are loaded and weighted once
// per item and reused for every 16-target tile; narrow columns (XC = 4) on
// 4x4x1 blocks as in the translations.  Moment rows past the leaf read as
// zeros (range-checked buffer loads).
// FUSE: the leaf's local holds its M2L part only (L2L skipped the leaves);
// for a leaf at level >= 3 the wave adds sum_j Q'[t][j] L_parent[j][c], Q'
// the moment rows through the leaf's L2L operator (momp), as a second
// contraction with the parent's local as B.
//
// Waves per SIMD asked of the compiler: two (at most 256 registers) where
// that costs no spills (below order 8; at order 8 the fused items of up to
// 48 columns, e.g. 263 registers otherwise at two tiles and four narrow
// columns), else no bound: the wider fused items would spill to scratch.
template <int ORD, int WT, int XC, bool FUSE>
constexpr int l2p_min_waves()
{
    return ORD < 8 || (ORD == 8 && (!FUSE || 16 * WT + XC <= 48)) ? 2 : 1;
}

template <int ORD, int WT, int XC, bool FUSE>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(l2p_min_waves<ORD, WT, XC, FUSE>()))) void k_l2p_mfma(int items_per_leaf, const int32_t *__restrict__ leaf_box,
                                                 const int32_t *__restrict__ box_beg,
                                                 const int32_t *__restrict__ box_end,
                                                 const double *__restrict__ hbox, const float *__restrict__ mom,
                                                 const float *__restrict__ L, float *__restrict__ ys, int C,
                                                 const float *__restrict__ momp, const int32_t *__restrict__ box_parent,
                                                 const int32_t *__restrict__ box_level)
{
    constexpr int K = (ORD + 1) * (ORD + 1), NKS = (K + 3) / 4;
    struct BV {
        float v[WT];
    };
    const int w = blockIdx.x;
    const int li_leaf = w / items_per_leaf;
    const int cb = (w - li_leaf * items_per_leaf) * 16 * WT, cn = cb + 16 * WT;
    const int lane = threadIdx.x, li = lane & 15, kq = lane >> 4;
    const int32_t b = leaf_box[li_leaf];
    const int32_t kb = box_beg[b], nt = box_end[b] - kb;
    const float ih = (float)(1.0 / hbox[b]);
    // weighted local fragments: row k = NKS kq + ks (clamped), weight 1 for
    // the m = 0 coefficient of each degree (k = n^2), 2 otherwise
    const auto rl = buf_rsrc(L + (int64_t)b * K * C, (uint32_t)((K * C + 256) * 4));
    float bl[NKS][WT], bx[XC ? NKS : 1];
    bool valid[NKS];
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
        const int k = NKS * kq + ks;
        valid[ks] = k < K;
        const int kc = k < K ? k : K - 1;
        int n = (int)sqrtf((float)kc + 0.5f);
        const float wk = (n * n == kc ? 1.f : 2.f) * ih;
        const BV v = buf_load<BV>(rl, (kc * C + cb + WT * li) * 4, 0);
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) bl[ks][ct] = v.v[ct] * wk;
        if constexpr (XC > 0) bx[ks] = buf_load<float>(rl, (kc * C + cn + (li & 3)) * 4, 0) * wk;
    }
    // the parent's local (unweighted: the weights are in Q')
    const bool fz = FUSE && box_level[b] >= 3;
    float bp[FUSE ? NKS : 1][WT], bpx[FUSE && XC ? NKS : 1];
    if constexpr (FUSE) {
        if (fz) {
            const auto rp = buf_rsrc(L + (int64_t)box_parent[b] * K * C, (uint32_t)((K * C + 256) * 4));
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks) {
                const int k = NKS * kq + ks;
                const int kc = k < K ? k : K - 1;
                const BV v = buf_load<BV>(rp, (kc * C + cb + WT * li) * 4, 0);
#pragma unroll
                for (int ct = 0; ct < WT; ++ct) bp[ks][ct] = v.v[ct];
                if constexpr (XC > 0) bpx[ks] = buf_load<float>(rp, (kc * C + cn + (li & 3)) * 4, 0);
            }
        }
    }
    const auto rq = buf_rsrc(mom + (int64_t)kb * K, (uint32_t)(nt * K * 4));
    const auto rq2 = buf_rsrc(FUSE ? momp + (int64_t)kb * K : mom, (uint32_t)(fz ? nt * K * 4 : 0));
    const int ntt = (nt + 15) / 16;
    // a 16-target tile's moments and the values it adds to, fetched one
    // tile ahead
    struct Tile {
        float a[NKS];
        float a2[FUSE ? NKS : 1];
        float old[WT][4];
        float ox;
    };
    auto load_tile = [&](int tt, Tile &T) {
        const int qo = ((16 * tt + li) * K + NKS * kq) * 4;
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) T.a[ks] = buf_load<float>(rq, qo + 4 * ks, 0);
        if constexpr (FUSE)
            if (fz)
#pragma unroll
                for (int ks = 0; ks < NKS; ++ks) T.a2[ks] = buf_load<float>(rq2, qo + 4 * ks, 0);
#pragma unroll
        for (int ct = 0; ct < WT; ++ct)
#pragma unroll
            for (int e4 = 0; e4 < 4; ++e4) {
                const int t = 16 * tt + 4 * kq + e4, col = cb + WT * li + ct;
                T.old[ct][e4] = (t < nt && col < C) ? ys[(int64_t)(kb + t) * C + col] : 0.f;
            }
        if constexpr (XC > 0) {
            const int t = 16 * tt + 4 * (li >> 2) + kq, col = cn + (li & 3);
            T.ox = (t < nt && col < C) ? ys[(int64_t)(kb + t) * C + col] : 0.f;
        }
    };
    Tile tn;
    if (ntt > 0) load_tile(0, tn);
    for (int tt = 0; tt < ntt; ++tt) {
        const Tile tc = tn;
        if (tt + 1 < ntt) load_tile(tt + 1, tn);
        float a[NKS];
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) a[ks] = valid[ks] ? tc.a[ks] : 0.f;
        f32x4 acc[WT], accx = {0, 0, 0, 0};
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) acc[ct] = f32x4{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
#pragma unroll
            for (int ct = 0; ct < WT; ++ct) acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ks], bl[ks][ct], acc[ct], 0, 0, 0);
            if constexpr (XC > 0) accx = __builtin_amdgcn_mfma_f32_4x4x1f32(a[ks], bx[ks], accx, 0, 0, 0);
        }
        if constexpr (FUSE) {
            if (fz) {
#pragma unroll
                for (int ks = 0; ks < NKS; ++ks) {
                    const float a2 = valid[ks] ? tc.a2[ks] : 0.f;
#pragma unroll
                    for (int ct = 0; ct < WT; ++ct)
                        acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(a2, bp[ks][ct], acc[ct], 0, 0, 0);
                    if constexpr (XC > 0) accx = __builtin_amdgcn_mfma_f32_4x4x1f32(a2, bpx[ks], accx, 0, 0, 0);
                }
            }
        }
        // D[i][j] at lane j + 16 q, element i - 4 q: target 16 tt + i,
        // column cb + WT j + ct
#pragma unroll
        for (int ct = 0; ct < WT; ++ct)
#pragma unroll
            for (int e4 = 0; e4 < 4; ++e4) {
                const int t = 16 * tt + 4 * kq + e4, col = cb + WT * li + ct;
                if (t < nt && col < C) ys[(int64_t)(kb + t) * C + col] = tc.old[ct][e4] + acc[ct][e4];
            }
        if constexpr (XC > 0) {
            // lane (li, kq): column cn + (li & 3), targets 16 tt + 4 (li / 4) + i
            // in element i for its coefficient subset; after the sum over
            // the four subsets it stores element i = kq
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                accx[i] += __shfl_xor(accx[i], 16);
                accx[i] += __shfl_xor(accx[i], 32);
            }
            const float mine = kq == 0 ? accx[0] : kq == 1 ? accx[1] : kq == 2 ? accx[2] : accx[3];
            const int t = 16 * tt + 4 * (li >> 2) + kq, col = cn + (li & 3);
            if (t < nt && col < C) ys[(int64_t)(kb + t) * C + col] = tc.ox + mine;
        }
    }
}

// ---------------------------------------------------------------- M2L
// Offset-stationary batched GEMM.  All V-list pairs with the same integer
// offset share one operator T_o, so for every offset group
//     D_g[KP][pairs x cols] = T_o[KP][KK] * [M_s1 | M_s2 | ...]
// is one dense product with the operator held in registers (MFMA) or LDS
// (vector ALU).  Column n of a group is (pair n / Cc, column n % Cc).  D is
// written per pair to a scratch array tmp[pair][Cc][KP] and a second kernel
// sums the pairs of every target in a fixed order (deterministic, no
// atomics).
//
// MFMA 16x16x4 operand layout on a 64-lane wave (checked by the GPU tests):
// A[i][k]: lane = i + 16 k;  B[k][j]: lane = j + 16 k;
// D[i][j]: lane = j + 16 q, element e, with i = 4 q + e for f32 and
//          i = q + 4 e for f64.
// op_frag holds each operator in fragment order [o][row tile][k step][lane].
template <typename T>
__device__ inline void mfma_16x16x4(T a, T b, typename std::conditional<sizeof(T) == 4, f32x4, f64x4>::type &d);
template <>
__device__ inline void mfma_16x16x4<float>(float a, float b, f32x4 &d)
{
    d = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, d, 0, 0, 0);
}
template <>
__device__ inline void mfma_16x16x4<double>(double a, double b, f64x4 &d)
{
    d = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, d, 0, 0, 0);
}

template <typename T>
__device__ inline int mfma_row(int q, int e)
{
    return sizeof(T) == 4 ? 4 * q + e : q + 4 * e;
}

template <int ORD>
struct M2LDims {
    static constexpr int K = (ORD + 1) * (ORD + 1);
    static constexpr int NRT = (K + 15) / 16;  // 16-row tiles
    static constexpr int NKS = (K + 3) / 4;    // 4-deep k steps
    static constexpr int KP = NRT * 16;
    static constexpr int KK = NKS * 4;
};

// One wave per work item (group g, column tiles [ct0, ct1)).
template <typename T, int ORD>
__global__ __launch_bounds__(256) void k_m2l_os_mfma(const int32_t *__restrict__ items, int n_items,
                                                     const int32_t *__restrict__ gbeg, const int32_t *__restrict__ goff,
                                                     const int32_t *__restrict__ src, const T *__restrict__ op_frag,
                                                     const T *__restrict__ M, int C, int c0, int Cc,
                                                     T *__restrict__ tmp)
{
    using D = M2LDims<ORD>;
    using VT = typename std::conditional<sizeof(T) == 4, f32x4, f64x4>::type;
    constexpr int RB = sizeof(T) == 4 ? D::NRT : 2;  // row tiles of the operator held in registers
    const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (w >= n_items) return;
    const int lane = threadIdx.x & 63, li = lane & 15, kq = lane >> 4;
    const int g = items[3 * w], ct0 = items[3 * w + 1], ct1 = items[3 * w + 2];
    const int pb = gbeg[g], ncols = (gbeg[g + 1] - pb) * Cc;
    const T *Tf = op_frag + (int64_t)goff[g] * D::NRT * D::NKS * 64 + lane;
    for (int r0 = 0; r0 < D::NRT; r0 += RB) {
        T a[RB][D::NKS];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int ks = 0; ks < D::NKS; ++ks) a[rb][ks] = (r0 + rb < D::NRT) ? Tf[((r0 + rb) * D::NKS + ks) * 64] : T(0);
        // B fragments of the first column tile; the next tile's loads are
        // issued before the current tile's MFMAs
        T b[D::NKS], bn[D::NKS];
        auto load_b = [&](int ct, T *dst) {
            const int n = ct * 16 + li;
            const int p = n / Cc, c = n - p * Cc;
            const bool valid = n < ncols && ct < ct1;
            const T *Mp = M + (int64_t)(valid ? src[pb + p] : 0) * D::K * C + c0 + c;
#pragma unroll
            for (int ks = 0; ks < D::NKS; ++ks) {
                const int kk = 4 * ks + kq;
                dst[ks] = (valid && kk < D::K) ? Mp[(int64_t)kk * C] : T(0);
            }
        };
        load_b(ct0, b);
        for (int ct = ct0; ct < ct1; ++ct) {
            load_b(ct + 1, bn);
            const int n = ct * 16 + li;
            const int p = n / Cc, c = n - p * Cc;
            const bool valid = n < ncols;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                if (r0 + rb >= D::NRT) break;
                VT d = {0, 0, 0, 0};
#pragma unroll
                for (int ks = 0; ks < D::NKS; ++ks) mfma_16x16x4<T>(a[rb][ks], b[ks], d);
                if (valid) {
                    T *out = tmp + ((int64_t)(pb + p) * Cc + c) * D::KP + (r0 + rb) * 16;
                    if (sizeof(T) == 4) {
                        *reinterpret_cast<VT *>(out + 4 * kq) = d;
                    } else {
#pragma unroll
                        for (int e = 0; e < 4; ++e) out[mfma_row<T>(kq, e)] = d[e];
                    }
                }
            }
#pragma unroll
            for (int ks = 0; ks < D::NKS; ++ks) b[ks] = bn[ks];
        }
    }
}

// One workgroup per work item (group g, columns [n0, n1), at most 64):
// operator (k-major) and the gathered multipoles staged in LDS, every thread
// owns NRT rows x 4 columns of the product.
template <typename T, int ORD>
__global__ __launch_bounds__(256) void k_m2l_os_valu(const int32_t *__restrict__ items,
                                                     const int32_t *__restrict__ gbeg, const int32_t *__restrict__ goff,
                                                     const int32_t *__restrict__ src, const T *__restrict__ op_k,
                                                     const T *__restrict__ M, int C, int c0, int Cc,
                                                     T *__restrict__ tmp)
{
    using D = M2LDims<ORD>;
    constexpr int NC = 64, TC = 4;
    __shared__ T sA[D::KK * D::KP];
    __shared__ T sB[D::KK * NC];
    const int g = items[3 * blockIdx.x], n0 = items[3 * blockIdx.x + 1], n1 = items[3 * blockIdx.x + 2];
    const int pb = gbeg[g];
    const T *Ao = op_k + (int64_t)goff[g] * D::KK * D::KP;
    for (int i = threadIdx.x; i < D::KK * D::KP; i += 256) sA[i] = Ao[i];
    for (int i = threadIdx.x; i < D::KK * NC; i += 256) {
        const int k = i / NC, j = i - k * NC, n = n0 + j;
        T v = T(0);
        if (n < n1 && k < D::K) {
            const int p = n / Cc, c = n - p * Cc;
            v = M[((int64_t)src[pb + p] * D::K + k) * C + c0 + c];
        }
        sB[i] = v;
    }
    __syncthreads();
    const int tr = threadIdx.x >> 4, tc = threadIdx.x & 15;
    T acc[D::NRT][TC];
#pragma unroll
    for (int i = 0; i < D::NRT; ++i)
#pragma unroll
        for (int j = 0; j < TC; ++j) acc[i][j] = 0;
    for (int k = 0; k < D::K; ++k) {
        T a[D::NRT], b[TC];
#pragma unroll
        for (int i = 0; i < D::NRT; ++i) a[i] = sA[k * D::KP + tr * D::NRT + i];
#pragma unroll
        for (int j = 0; j < TC; ++j) b[j] = sB[k * NC + tc * TC + j];
#pragma unroll
        for (int i = 0; i < D::NRT; ++i)
#pragma unroll
            for (int j = 0; j < TC; ++j) acc[i][j] += a[i] * b[j];
    }
#pragma unroll
    for (int j = 0; j < TC; ++j) {
        const int n = n0 + tc * TC + j;
        if (n >= n1) continue;
        const int p = n / Cc, c = n - p * Cc;
        T *out = tmp + ((int64_t)(pb + p) * Cc + c) * D::KP + tr * D::NRT;
#pragma unroll
        for (int i = 0; i < D::NRT; ++i) out[i] = acc[i][j];
    }
}

// Offset-stationary translation on the vector ALU, one column per thread
// (FP32): the group's operator, k-major, in LDS and read as broadcasts (every
// lane of a wave reads the same address), all K output rows of the thread's
// column in registers, its multipole column streamed from memory one chunk
// of p + 1 coefficients ahead (K = (p + 1)^2 is a whole number of chunks).
// Per coefficient: K FMAs for about K / 4 broadcast reads.
template <int ORD>
__global__ __launch_bounds__(256) void k_m2l_os_col(const int32_t *__restrict__ items,
                                                    const int32_t *__restrict__ gbeg, const int32_t *__restrict__ goff,
                                                    const int32_t *__restrict__ src, const float *__restrict__ op_k,
                                                    const float *__restrict__ M, int C, int c0, int Cc,
                                                    float *__restrict__ tmp)
{
    using D = M2LDims<ORD>;
    constexpr int K = D::K, KC = ORD + 1, NCH = ORD + 1;
    __shared__ float4 sA4[K * D::KP / 4];
    const float *sA = reinterpret_cast<const float *>(sA4);
    const int g = items[3 * blockIdx.x], n0 = items[3 * blockIdx.x + 1], n1 = items[3 * blockIdx.x + 2];
    const int pb = gbeg[g];
    const float4 *Ao = reinterpret_cast<const float4 *>(op_k + (int64_t)goff[g] * D::KK * D::KP);
    for (int i = threadIdx.x; i < K * D::KP / 4; i += 256) sA4[i] = Ao[i];
    const int n = n0 + (int)threadIdx.x;
    const bool active = n < n1;
    int p = 0, c = 0;
    const float *mcol = M;
    if (active) {
        p = n / Cc;
        c = n - p * Cc;
        mcol = M + (int64_t)src[pb + p] * K * C + c0 + c;
    }
    float acc[K];
#pragma unroll
    for (int r = 0; r < K; ++r) acc[r] = 0.f;
    float bcur[KC], bnext[KC];
#pragma unroll
    for (int j = 0; j < KC; ++j) bcur[j] = active ? mcol[(int64_t)j * C] : 0.f;
    __syncthreads();
    for (int ch = 0; ch < NCH; ++ch) {
        if (ch + 1 < NCH) {
#pragma unroll
            for (int j = 0; j < KC; ++j) bnext[j] = active ? mcol[(int64_t)((ch + 1) * KC + j) * C] : 0.f;
        }
#pragma unroll
        for (int j = 0; j < KC; ++j) {
            const float *a = sA + (ch * KC + j) * D::KP;
            const float b = bcur[j];
#pragma unroll
            for (int r = 0; r < K; ++r) acc[r] = fmaf(a[r], b, acc[r]);
        }
#pragma unroll
        for (int j = 0; j < KC; ++j) bcur[j] = bnext[j];
    }
    if (active) {
        float *out = tmp + ((int64_t)(pb + p) * Cc + c) * D::KP;
#pragma unroll
        for (int r = 0; r < K; ++r) out[r] = acc[r];
    }
}

// Target-stationary translation for wide column blocks: one wave per item
// (target, WT consecutive 16-column tiles).  The wave visits the pairs of its
// target in their list order and accumulates T_o M_s in registers, so there
// is no scratch array and no second pass, and the sum order is fixed.  Per
// pair the source expansion is read once (its rows are contiguous runs of C
// values, so the WT tiles of one wave cover whole cache lines) and the
// operator is streamed one 16-row tile of fragments at a time.
//
// Launch: one wave (64 threads) per workgroup, in target order, so that a
// SIMD whose target has few pairs takes the next item at once instead of
// idling until the longest target of a larger workgroup is done.  (Giving
// each XCD one contiguous range of targets, for L2 locality, was measured
// slower: the pair counts of spatial regions differ, and the XCD with the
// densest range finishes last.)

// Widest item (column tiles) whose accumulators, double-buffered B
// fragments and the two operator ring buffers stay within about 480
// registers.
template <typename T, int ORD>
constexpr int ts_max_tiles()
{
    using D = M2LDims<ORD>;
    constexpr int r = sizeof(T) / 4, vec = 16 / sizeof(T);
    constexpr int a = 2 * ((D::NRT + 2) / 3) * ((D::NKS + vec - 1) / vec) * vec;
    int w = 4;
    while (w > 1 && (D::NRT * 4 * w + 2 * D::NKS * w + a) * r > 480) --w;
    return w;
}

// Sign of the real coefficient k under the reflections x -> -x, y -> -y and
// z -> -z (bits 0, 1, 2 set where the sign flips).  With the normalised
// harmonics R_n^m ~ P_n^m(cos theta) e^{i m phi}: x -> -x takes phi to
// pi - phi, (-1)^m times the conjugate; y -> -y takes phi to -phi, the
// conjugate; z -> -z takes cos theta to -cos theta, (-1)^(n+m).  Multipole
// and local coefficients both change this way, so the M2L operator of a
// reflected offset is S T S with S = diag(signs).
__device__ inline int reflection_signs(int k)
{
    int n = (int)sqrtf((float)k);
    while (n * n > k) --n;
    while ((n + 1) * (n + 1) <= k) ++n;
    const int d = k - n * n, m = (d + 1) >> 1, im = (d > 0 && !(d & 1)) ? 1 : 0;
    return ((m & 1) ^ im) | (im << 1) | (((n + m) & 1) << 2);
}

template <typename T>
__device__ inline T flip_sign(T v, uint32_t bit)
{
    if constexpr (sizeof(T) == 4) {
        return __int_as_float(__float_as_int(v) ^ (int)(bit << 31));
    } else {
        return __longlong_as_double(__double_as_longlong(v) ^ (long long)((uint64_t)bit << 63));
    }
}

// REFL: the operator code of a pair is (index of the non-negative offset
// |o|) << 3 | reflection bits, and T_o = S T_|o| S is applied by flipping
// the signs of the B fragments (columns) and of the A fragments (rows), so
// only 64 operators (L2-resident) are streamed instead of 316.
//
// XC = 4 (FP32): the item also owns the (up to) four columns after its WT
// tiles and applies the operator to them with the 16-block 4x4x1 MFMA on
// the operator fragments already in registers, instead of a further 16x16x4
// tile that would be at most a quarter useful (C = 36: two tiles plus 4x4
// blocks, a quarter of the MFMA cycles less per pair).  Lane (li, kq) holds
// operator row 16 rt + li at k = 4 ks + kq and loads density column
// cx + (li & 3) of row 4 ks + kq, so block b = lane / 4 sees rows
// 16 rt + 4 (li / 4) + 0..3 times the four columns at one k; each block sums
// its k-subset, and the four k-subsets are added across lanes once per
// target.
template <typename T, int ORD, int WT, bool REFL, int XC = 0>
__global__ __launch_bounds__(64) void k_trans_ts(int n_items, int items_per_tgt, const int32_t *__restrict__ order,
                                                  const int32_t *__restrict__ red_tgt,
                                                  const int32_t *__restrict__ red_ptr,
                                                  const int32_t *__restrict__ ts_src,
                                                  const int32_t *__restrict__ ts_op, const T *__restrict__ op_vec,
                                                  const T *__restrict__ op_tail, const T *__restrict__ in, int C,
                                                  int accumulate, T *__restrict__ out)
{
    using D = M2LDims<ORD>;
    using VT = typename std::conditional<sizeof(T) == 4, f32x4, f64x4>::type;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int NKV = (D::NKS + VEC - 1) / VEC;
    using AV = T __attribute__((ext_vector_type(VEC)));
    static_assert(XC == 0 || (XC == 4 && sizeof(T) == 4), "4x4-block columns: four, FP32 only");
    // K = 16 n + 1 (orders 6 and 8): the last operator row is applied on the
    // vector ALU from the B fragments already in registers (21 FMAs per
    // column tile and pair), instead of a 16-row MFMA tile that is 15/16
    // padding; the four k-subsets of a column are summed across lanes once
    // per target
    constexpr bool TAIL = D::K % 16 == 1;
    constexpr int NRTM = TAIL ? D::K / 16 : D::NRT;  // row tiles on MFMA
    const int w = blockIdx.x;
    if (w >= n_items) return;
    const int lane = threadIdx.x & 63, li = lane & 15, kq = lane >> 4;
    // targets in launch order (order: a permutation of the target list,
    // those with the most pairs first, so that no long target starts last)
    const int slot = w / items_per_tgt;
    const int ti = order ? order[slot] : slot;
    const int cb = (w - slot * items_per_tgt) * WT * 16;  // first column of the item
    const int t = red_tgt[ti], j0 = red_ptr[ti], j1 = red_ptr[ti + 1];
    // Columns are interleaved over the WT tiles: lane li feeds column
    // cb + WT li + ct to tile ct, so its B values of one coefficient row are
    // WT consecutive floats, one vector load.  Loads are unconditional: a
    // column past C runs into the next row (or the slack after the array)
    // and only feeds a discarded output column; the coefficient row of the
    // last k step is clamped to K - 1, where the operator column is zero.
    const int boff = kq * C + cb + WT * li;
    const int blast = min(4 * (D::NKS - 1) + kq, D::K - 1) * C - 4 * (D::NKS - 1) * C - kq * C;
    const int cx = cb + WT * 16;  // first vector-ALU column (XC > 0)
    const int xoff = kq * C + cx + (li & 3);
    struct BV {
        T v[WT];
    };
    VT acc[NRTM][WT];
#pragma unroll
    for (int rt = 0; rt < NRTM; ++rt)
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) acc[rt][ct] = VT{0, 0, 0, 0};
    T tacc[WT];
#pragma unroll
    for (int ct = 0; ct < WT; ++ct) tacc[ct] = T(0);
    VT accx[XC ? NRTM : 1], taccx = VT{0, 0, 0, 0};
#pragma unroll
    for (int rt = 0; rt < (XC ? NRTM : 1); ++rt) accx[rt] = VT{0, 0, 0, 0};
    // Reflection sign masks of this lane, per axis a: bit ks of col[a] for
    // the coefficient 4 ks + kq it feeds as B, bit 4 rt + e of acm[a] for the
    // accumulator element (rt, e), whose row is 16 rt + mfma_row(kq, e).
    // Bit 4 rt + i of axm[a]: the same for element i of the 4x4-block
    // accumulator of row tile rt, whose row is 16 rt + 4 (li / 4) + i.
    uint64_t col[3] = {0, 0, 0}, acm[3] = {0, 0, 0}, axm[3] = {0, 0, 0};
    if constexpr (REFL) {
        for (int ks = 0; ks < D::NKS; ++ks) {
            const int kk = 4 * ks + kq;
            const int sg = kk < D::K ? reflection_signs(kk) : 0;
            for (int a = 0; a < 3; ++a) col[a] |= (uint64_t)((sg >> a) & 1) << ks;
        }
        for (int rt = 0; rt < D::NRT; ++rt) {
            for (int e = 0; e < 4; ++e) {
                const int r = 16 * rt + mfma_row<T>(kq, e);
                const int sg = r < D::K ? reflection_signs(r) : 0;
                for (int a = 0; a < 3; ++a) acm[a] |= (uint64_t)((sg >> a) & 1) << (4 * rt + e);
            }
            for (int i = 0; i < 4; ++i) {
                const int r = 16 * rt + 4 * (li >> 2) + i;
                const int sg = r < D::K ? reflection_signs(r) : 0;
                for (int a = 0; a < 3; ++a) axm[a] |= (uint64_t)((sg >> a) & 1) << (4 * rt + i);
            }
        }
    }
    auto mask_of = [&](const uint64_t (&m)[3], int rf) {
        uint64_t x = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
            if (rf >> a & 1) x ^= m[a];
        return x;
    };
    // T_o = S T_|o| S for a reflected offset.  The column sign goes on the B
    // fragments; the row sign is carried by the accumulator, which holds
    // S_f (sum so far) for the reflection f of the pairs being summed: the
    // pairs of a target come sorted by reflection, and the accumulator is
    // re-signed (S_f S_g = S_(f^g)) only when the reflection changes.
    auto flip_acc = [&](int d) {
        const uint64_t m = mask_of(acm, d);
#pragma unroll
        for (int rt = 0; rt < NRTM; ++rt)
#pragma unroll
            for (int ct = 0; ct < WT; ++ct)
#pragma unroll
                for (int e = 0; e < 4; ++e) acc[rt][ct][e] = flip_sign(acc[rt][ct][e], (uint32_t)(m >> (4 * rt + e)) & 1u);
        if constexpr (XC > 0) {
            const uint64_t mx = mask_of(axm, d);
#pragma unroll
            for (int rt = 0; rt < NRTM; ++rt)
#pragma unroll
                for (int i = 0; i < 4; ++i) accx[rt][i] = flip_sign(accx[rt][i], (uint32_t)(mx >> (4 * rt + i)) & 1u);
        }
        if constexpr (TAIL) {  // the last row, summed on the vector ALU
            const int sg = reflection_signs(D::K - 1);
            int f = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a)
                if (d >> a & 1) f ^= (sg >> a) & 1;
#pragma unroll
            for (int ct = 0; ct < WT; ++ct) tacc[ct] = flip_sign(tacc[ct], (uint32_t)f);
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (XC) taccx[i] = flip_sign(taccx[i], (uint32_t)f);
        }
    };
    // Software pipeline over (pair, row-tile group) steps; the next pair's B
    // fragments are issued at the first group of the current pair, and
    // loads complete in issue order, so each wait covers only what the next
    // step needs.  FP32 with the full operator table up to order 8: one
    // register buffer per operator row tile, the next pair's tile issued
    // right after the current pair's, as many steps ahead as there are
    // tiles less one.  Otherwise (FP64 has twice the registers per tile,
    // reflections need their sign masks, higher orders more tiles): three
    // groups of row tiles through a ring of two buffers, each group's loads
    // issued two steps before its MFMAs, so that the accumulators stay in
    // their registers as far as they fit.
    constexpr bool TILE_RING = sizeof(T) == 4 && !REFL && ORD <= 8;
    constexpr int GR = TILE_RING ? 1 : (NRTM + 2) / 3;  // row tiles per group
    // per-pair operands (B fragments, 4x4-block densities, last operator
    // row), in two sets that alternate between the two pairs of a trip, so
    // the next pair's loads land in place without copies
    struct PB {
        T b[WT][D::NKS];
        T x[XC ? D::NKS : 1];
        AV t[TAIL ? NKV : 1];
    };
    PB p0, p1;
    auto xmfma = [&](VT &d, T a, T x) {
        if constexpr (XC > 0) d = __builtin_amdgcn_mfma_f32_4x4x1f32(a, x, d, 0, 0, 0);
    };
    auto load_t = [&](int code, PB &d) {
        if constexpr (TAIL) {
            const auto rs = buf_rsrc(op_tail + (int64_t)(code >> 3) * 4 * NKV * VEC, 4 * NKV * VEC * sizeof(T));
#pragma unroll
            for (int kv = 0; kv < NKV; ++kv) d.t[kv] = buf_load<AV>(rs, (kq * NKV + kv) * VEC * (int)sizeof(T), 0);
        }
    };
    auto tail_fma = [&](const PB &p) {
        if constexpr (TAIL) {
#pragma unroll
            for (int ks = 0; ks < D::NKS; ++ks)
#pragma unroll
                for (int ct = 0; ct < WT; ++ct) tacc[ct] += p.t[ks / VEC][ks % VEC] * p.b[ct][ks];
            if constexpr (XC > 0)
#pragma unroll
                for (int ks = 0; ks < D::NKS; ++ks) xmfma(taccx, p.t[ks / VEC][ks % VEC], p.x[ks]);
        }
    };
    // the source record and the 256 elements after it (columns past C and
    // the clamped last k step read at most that far)
    const uint32_t mbytes = (uint32_t)((D::K * C + 256) * sizeof(T));
    // live = false: a record of zero bytes, every load of it returns zero
    auto load_b = [&](int j, PB &d, bool live = true) {
        const auto rs = buf_rsrc(in + (int64_t)ts_src[j] * D::K * C, live ? mbytes : 0u);
#pragma unroll
        for (int ks = 0; ks < D::NKS; ++ks) {
            const int lofs = ks == D::NKS - 1 ? blast : 0;  // lane part of the clamp
            const int sofs = 4 * ks * C * (int)sizeof(T);
            const BV v = buf_load<BV>(rs, (boff + lofs) * (int)sizeof(T), sofs);
#pragma unroll
            for (int ct = 0; ct < WT; ++ct) d.b[ct][ks] = v.v[ct];
            if constexpr (XC > 0) d.x[ks] = buf_load<T>(rs, (xoff + lofs) * (int)sizeof(T), sofs);
        }
    };
    constexpr uint32_t obytes = D::NRT * NKV * 64 * 16;  // one operator in vector fragment order
    auto load_g = [&](int code, int g, AV (&dst)[GR][NKV]) {
        const auto rs = buf_rsrc(op_vec + (int64_t)(code >> 3) * D::NRT * NKV * 64 * VEC, obytes);
#pragma unroll
        for (int r = 0; r < GR; ++r)
            if (g * GR + r < NRTM)
#pragma unroll
                for (int kv = 0; kv < NKV; ++kv) dst[r][kv] = buf_load<AV>(rs, lane * 16, ((g * GR + r) * NKV + kv) * 1024);
    };
    // column signs of a reflected offset, applied in place once the loads
    // have landed
    auto flip_b = [&](int code, PB &d) {
        if constexpr (REFL) {
            const uint64_t cm = mask_of(col, code & 7);
#pragma unroll
            for (int ks = 0; ks < D::NKS; ++ks) {
#pragma unroll
                for (int ct = 0; ct < WT; ++ct) d.b[ct][ks] = flip_sign(d.b[ct][ks], (uint32_t)(cm >> ks) & 1u);
                if constexpr (XC > 0) d.x[ks] = flip_sign(d.x[ks], (uint32_t)(cm >> ks) & 1u);
            }
        }
    };
    // K = 4 n + 1 (every even order): the last k step holds one operator
    // column, K - 1, a rank-one update.  On the FP32 per-tile path it goes
    // to 4x4 blocks instead of a 16x16x4 tile that is 3/4 padding: block b
    // takes rows 4 (b / 4) .. + 3 and columns 4 (b % 4) .. + 3 of the tile,
    // so its A value at lane (li, kq) is operator row 16 rt + 4 kq + li % 4
    // (one word of the tile's last fragment, the one lane 4 kq + li % 4
    // holds, loaded on its own with the tile), its B value is the density
    // row K - 1 already loaded for that step, and its result lands in the
    // 16x16 accumulator's own lane layout (lane (li, kq), element e: row
    // 4 kq + e, column li), so it accumulates in place.  Taken at order 8
    // with more than 16 columns, where the wave holds over 256 registers
    // anyway: the loaded values would cost the narrower forms their second
    // wave.
    constexpr bool RANK1 = TILE_RING && D::K % 4 == 1 && ORD == 8 && WT * 16 + XC > 16;
    constexpr int NKM = RANK1 ? D::NKS - 1 : D::NKS;  // k steps on 16x16x4
    T ra[RANK1 ? NRTM : 1];
    auto load_a1 = [&](int code, int rt) {
        if constexpr (RANK1) {
            const auto rs = buf_rsrc(op_vec + (int64_t)(code >> 3) * D::NRT * NKV * 64 * VEC, obytes);
            ra[rt] = buf_load<T>(rs, (4 * kq + (li & 3)) * 16, (rt * NKV + NKV - 1) * 1024);
        }
    };
    auto compute = [&](int g, AV (&av)[GR][NKV], const PB &p) {
#pragma unroll
        for (int r = 0; r < GR; ++r) {
            if (g * GR + r >= NRTM) break;
            // the rank-one blocks go first, on accumulators last written a
            // pair ago, so that they wait on no MFMA chain
            if constexpr (RANK1)
#pragma unroll
                for (int ct = 0; ct < WT; ++ct)
                    acc[g * GR + r][ct] = __builtin_amdgcn_mfma_f32_4x4x1f32(ra[g * GR + r], p.b[ct][D::NKS - 1], acc[g * GR + r][ct], 0, 0, 0);
#pragma unroll
            for (int ks = 0; ks < D::NKS; ++ks) {
                if (ks < NKM)
#pragma unroll
                    for (int ct = 0; ct < WT; ++ct)
                        mfma_16x16x4<T>(av[r][ks / VEC][ks % VEC], p.b[ct][ks], acc[g * GR + r][ct]);
                if constexpr (XC > 0) xmfma(accx[g * GR + r], av[r][ks / VEC][ks % VEC], p.x[ks]);
            }
        }
    };
    auto clampj = [&](int j) { return j < j1 ? j : j1 - 1; };
    int frame = 0;
    auto reframe = [&](int code) {
        if constexpr (REFL) {
            if ((code & 7) != frame) {
                flip_acc((code & 7) ^ frame);
                frame = code & 7;
            }
        }
    };
    // Two pairs per trip, so that the buffer of each step and the operand
    // set of each pair are static.  With one buffer per tile a target with
    // an odd number of pairs ends on a phantom pair: the operator of its
    // last pair applied to densities that load as zeros.  That trip has no
    // branch, so the compiler cannot move the next pair's loads down to
    // their first use, which would undo the prefetch; the prologue issues
    // its loads in the order of the trip's, so that the waits of the first
    // step hold for every trip.  The ring of two keeps the branch around
    // the second pair (both operand sets live at once would not fit).
    if constexpr (TILE_RING) {
        AV rb[NRTM][GR][NKV];
        // one pair: tile rt computed, then the same tile of the next pair
        // (code cn) loaded into its buffer; the next pair's operands go
        // out after the first tile
        auto pair = [&](const PB &p, int cn, PB &pn, int jn, bool live) {
            __builtin_amdgcn_sched_barrier(0);
            compute(0, rb[0], p);
            tail_fma(p);
            __builtin_amdgcn_sched_barrier(0);
            load_b(jn, pn, live);
            load_t(cn, pn);
            load_g(cn, 0, rb[0]);
            load_a1(cn, 0);
#pragma unroll
            for (int rt = 1; rt < NRTM; ++rt) {
                __builtin_amdgcn_sched_barrier(0);
                compute(rt, rb[rt], p);
                __builtin_amdgcn_sched_barrier(0);
                load_g(cn, rt, rb[rt]);
                load_a1(cn, rt);
            }
            __builtin_amdgcn_sched_barrier(0);
            flip_b(cn, pn);
        };
        if (j0 < j1) {
            int c0 = ts_op[j0], c1 = ts_op[clampj(j0 + 1)];
            load_b(j0, p0);
            load_t(c0, p0);
            load_g(c0, 0, rb[0]);
            load_a1(c0, 0);
#pragma unroll
            for (int rt = 1; rt < NRTM; ++rt) {
                __builtin_amdgcn_sched_barrier(0);
                load_g(c0, rt, rb[rt]);
                load_a1(c0, rt);
            }
            __builtin_amdgcn_sched_barrier(0);
            flip_b(c0, p0);
            for (int j = j0; j < j1; j += 2) {
                const int c2 = ts_op[clampj(j + 2)];
                reframe(c0);
                pair(p0, c1, p1, clampj(j + 1), j + 1 < j1);
                reframe(c1);
                pair(p1, c2, p0, clampj(j + 2), true);
                c0 = c2;
                c1 = ts_op[clampj(j + 3)];
            }
            if constexpr (REFL)
                if (frame) flip_acc(frame);
        }
    } else if (j0 < j1) {
        AV r0[GR][NKV], r1[GR][NKV];
        int c0 = ts_op[j0], c1 = ts_op[clampj(j0 + 1)];
        load_b(j0, p0);
        load_t(c0, p0);
        load_g(c0, 0, r0);
        load_g(c0, 1, r1);
        flip_b(c0, p0);
        for (int j = j0; j < j1; j += 2) {
            const int c2 = ts_op[clampj(j + 2)];
            reframe(c0);
            __builtin_amdgcn_sched_barrier(0);
            compute(0, r0, p0);
            tail_fma(p0);
            __builtin_amdgcn_sched_barrier(0);
            load_b(clampj(j + 1), p1, j + 1 < j1);
            load_t(c1, p1);
            load_g(c0, 2, r0);
            __builtin_amdgcn_sched_barrier(0);
            compute(1, r1, p0);
            __builtin_amdgcn_sched_barrier(0);
            load_g(c1, 0, r1);
            __builtin_amdgcn_sched_barrier(0);
            compute(2, r0, p0);
            __builtin_amdgcn_sched_barrier(0);
            load_g(c1, 1, r0);
            __builtin_amdgcn_sched_barrier(0);
            flip_b(c1, p1);
            if (j + 1 < j1) {
                reframe(c1);
                __builtin_amdgcn_sched_barrier(0);
                compute(0, r1, p1);
                tail_fma(p1);
                __builtin_amdgcn_sched_barrier(0);
                load_b(clampj(j + 2), p0);
                load_t(c2, p0);
                load_g(c1, 2, r1);
                __builtin_amdgcn_sched_barrier(0);
                compute(1, r0, p1);
                __builtin_amdgcn_sched_barrier(0);
                load_g(c2, 0, r0);
                __builtin_amdgcn_sched_barrier(0);
                compute(2, r1, p1);
                __builtin_amdgcn_sched_barrier(0);
                load_g(c2, 1, r1);
                __builtin_amdgcn_sched_barrier(0);
                flip_b(c2, p0);
            }
            c0 = c2;
            c1 = ts_op[clampj(j + 3)];
        }
        if constexpr (REFL)
            if (frame) flip_acc(frame);
    }
#pragma unroll
    for (int rt = 0; rt < NRTM; ++rt)
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) {
            const int col = cb + WT * li + ct;
            if (col >= C) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = rt * 16 + mfma_row<T>(kq, e);
                if (row >= D::K) continue;
                T *o = out + ((int64_t)t * D::K + row) * C + col;
                *o = accumulate ? *o + acc[rt][ct][e] : acc[rt][ct][e];
            }
        }
    if constexpr (TAIL) {
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) {
            T v = tacc[ct];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            const int col = cb + WT * li + ct;
            if (kq == 0 && col < C) {
                T *o = out + ((int64_t)t * D::K + D::K - 1) * C + col;
                *o = accumulate ? *o + v : v;
            }
        }
    }
    if constexpr (XC > 0) {
        // 4x4 block accumulators: lane (li, kq) holds column cx + (li & 3),
        // rows 16 rt + 4 (li / 4) + i in element i, for its k-subset; after
        // the sum over the four k-subsets it stores element i = kq
        const int col = cx + (li & 3);
#pragma unroll
        for (int rt = 0; rt < NRTM; ++rt) {
            VT v = accx[rt];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                v[i] += __shfl_xor(v[i], 16);
                v[i] += __shfl_xor(v[i], 32);
            }
            const T mine = kq == 0 ? v[0] : kq == 1 ? v[1] : kq == 2 ? v[2] : v[3];
            const int row = 16 * rt + 4 * (li >> 2) + kq;
            if (col < C && row < D::K) {
                T *o = out + ((int64_t)t * D::K + row) * C + col;
                *o = accumulate ? *o + mine : mine;
            }
        }
        if constexpr (TAIL) {  // every row of a block holds the last operator row
            T v = taccx[0];
            v += __shfl_xor(v, 16);
            v += __shfl_xor(v, 32);
            if (kq == 0 && li < 4 && col < C) {
                T *o = out + ((int64_t)t * D::K + D::K - 1) * C + col;
                *o = accumulate ? *o + v : v;
            }
        }
    }
}

// Lean form of the target-stationary kernel for the full operator table:
// no software pipeline, one operator row tile ahead, registers capped for
// two waves per SIMD so that the other wave covers each wait.
template <typename T, int ORD, int WT>
__global__ __launch_bounds__(64, 2) void k_trans_ts_lean(int n_items, int items_per_tgt,
                                                          const int32_t *__restrict__ red_tgt,
                                                          const int32_t *__restrict__ red_ptr,
                                                          const int32_t *__restrict__ ts_src,
                                                          const int32_t *__restrict__ ts_op,
                                                          const T *__restrict__ op_vec, const T *__restrict__ in,
                                                          int C, int accumulate, T *__restrict__ out)
{
    using D = M2LDims<ORD>;
    using VT = typename std::conditional<sizeof(T) == 4, f32x4, f64x4>::type;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int NKV = (D::NKS + VEC - 1) / VEC;
    using AV = T __attribute__((ext_vector_type(VEC)));
    struct BV {
        T v[WT];
    };
    const int w = blockIdx.x;
    if (w >= n_items) return;
    const int lane = threadIdx.x & 63, li = lane & 15, kq = lane >> 4;
    const int ti = w / items_per_tgt;
    const int cb = (w - ti * items_per_tgt) * WT * 16;
    const int t = red_tgt[ti], j0 = red_ptr[ti], j1 = red_ptr[ti + 1];
    const int boff = kq * C + cb + WT * li;
    const int blast = min(4 * (D::NKS - 1) + kq, D::K - 1) * C - 4 * (D::NKS - 1) * C - kq * C;
    VT acc[D::NRT][WT];
#pragma unroll
    for (int rt = 0; rt < D::NRT; ++rt)
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) acc[rt][ct] = VT{0, 0, 0, 0};
    for (int j = j0; j < j1; ++j) {
        const T *Ms = in + (int64_t)ts_src[j] * D::K * C;
        const AV *Tv = reinterpret_cast<const AV *>(op_vec) + (int64_t)(ts_op[j] >> 3) * D::NRT * NKV * 64 + lane;
        T b[WT][D::NKS];
#pragma unroll
        for (int ks = 0; ks < D::NKS; ++ks) {
            const int rofs = 4 * ks * C + (ks == D::NKS - 1 ? blast : 0);
            const BV v = *reinterpret_cast<const BV *>(Ms + rofs + boff);
#pragma unroll
            for (int ct = 0; ct < WT; ++ct) b[ct][ks] = v.v[ct];
        }
        AV an[NKV];
#pragma unroll
        for (int kv = 0; kv < NKV; ++kv) an[kv] = Tv[kv * 64];
#pragma unroll
        for (int rt = 0; rt < D::NRT; ++rt) {
            AV ac[NKV];
#pragma unroll
            for (int kv = 0; kv < NKV; ++kv) ac[kv] = an[kv];
            if (rt + 1 < D::NRT)
#pragma unroll
                for (int kv = 0; kv < NKV; ++kv) an[kv] = Tv[((rt + 1) * NKV + kv) * 64];
#pragma unroll
            for (int ks = 0; ks < D::NKS; ++ks)
#pragma unroll
                for (int ct = 0; ct < WT; ++ct) mfma_16x16x4<T>(ac[ks / VEC][ks % VEC], b[ct][ks], acc[rt][ct]);
        }
    }
#pragma unroll
    for (int rt = 0; rt < D::NRT; ++rt)
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) {
            const int col = cb + WT * li + ct;
            if (col >= C) continue;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = rt * 16 + mfma_row<T>(kq, e);
                if (row >= D::K) continue;
                T *o = out + ((int64_t)t * D::K + row) * C + col;
                *o = accumulate ? *o + acc[rt][ct][e] : acc[rt][ct][e];
            }
        }
}

// Source-stationary translation for passes where each target has one
// source and a source feeds several targets (L2L: a parent's local to its
// children).  One wave per (run of pairs with the same source, 16-row tile
// of the result, item of WT column tiles [+ XC narrow columns]): the source
// fragments are loaded once and stay in registers; the wave walks the pairs
// of the run with the next pair's operator tile (and the target values it
// adds to) in flight, and adds each finished tile into its target.  Short
// waves in large numbers: the passes are level by level, and the small
// levels are bound by the length of one wave.  The operator is the padded
// [NRT][KP] form (the last row in the last tile); the tables of a pass are
// few and stay in the L2.
template <typename T, int ORD, int WT, int XC>
__global__ __launch_bounds__(64) void k_trans_ps(int n_items, int items_per_run, const int32_t *__restrict__ ps_beg,
                                                 const int32_t *__restrict__ ts_tgt,
                                                 const int32_t *__restrict__ ts_src,
                                                 const int32_t *__restrict__ ts_op, const T *__restrict__ op_vec,
                                                 const T *__restrict__ in, int C, int accumulate, T *__restrict__ out)
{
    using D = M2LDims<ORD>;
    using VT = typename std::conditional<sizeof(T) == 4, f32x4, f64x4>::type;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int NKV = (D::NKS + VEC - 1) / VEC;
    using AV = T __attribute__((ext_vector_type(VEC)));
    static_assert(XC == 0 || (XC == 4 && sizeof(T) == 4), "4x4-block columns: four, FP32 only");
    struct BV {
        T v[WT];
    };
    const int w = blockIdx.x;
    if (w >= n_items) return;
    const int g = w / (items_per_run * D::NRT);
    const int rem = w - g * items_per_run * D::NRT;
    const int rt = rem / items_per_run;
    const int cb = (rem - rt * items_per_run) * WT * 16, cx = cb + WT * 16;
    const int lane = threadIdx.x & 63, li = lane & 15, kq = lane >> 4;
    const int j0 = ps_beg[g], j1 = ps_beg[g + 1];
    // source fragments (columns interleaved over the tiles as in the
    // target-stationary kernel; the last k step's row clamped to K - 1,
    // where the operator column is zero)
    const int boff = kq * C + cb + WT * li, xoff = kq * C + cx + (li & 3);
    const int blast = min(4 * (D::NKS - 1) + kq, D::K - 1) * C - 4 * (D::NKS - 1) * C - kq * C;
    const auto rm = buf_rsrc(in + (int64_t)ts_src[j0] * D::K * C, (uint32_t)((D::K * C + 256) * sizeof(T)));
    T b[WT][D::NKS], bx[XC ? D::NKS : 1];
#pragma unroll
    for (int ks = 0; ks < D::NKS; ++ks) {
        const int lofs = ks == D::NKS - 1 ? blast : 0;
        const int sofs = 4 * ks * C * (int)sizeof(T);
        const BV v = buf_load<BV>(rm, (boff + lofs) * (int)sizeof(T), sofs);
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) b[ct][ks] = v.v[ct];
        if constexpr (XC > 0) bx[ks] = buf_load<T>(rm, (xoff + lofs) * (int)sizeof(T), sofs);
    }
    constexpr uint32_t obytes = D::NRT * NKV * 64 * 16;
    auto load_a = [&](int step, AV (&dst)[NKV]) {
        const int j = j0 + step;
        const auto ro = buf_rsrc(op_vec + (int64_t)(ts_op[j] >> 3) * D::NRT * NKV * 64 * VEC, obytes);
#pragma unroll
        for (int kv = 0; kv < NKV; ++kv) dst[kv] = buf_load<AV>(ro, lane * 16, (rt * NKV + kv) * 1024);
    };
    // the target values a step adds to, fetched one step ahead with its
    // operator tile (the rows of different steps never overlap)
    struct Old {
        T v[WT][4];
        T x;
    };
    auto load_old = [&](int step, Old &o) {
        const int j = j0 + step;
        const T *tp = out + (int64_t)ts_tgt[j] * D::K * C;
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) {
            const int col = cb + WT * li + ct;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = rt * 16 + mfma_row<T>(kq, e);
                o.v[ct][e] = (accumulate && col < C && row < D::K) ? tp[row * C + col] : T(0);
            }
        }
        if constexpr (XC > 0) {
            const int row = 16 * rt + 4 * (li >> 2) + kq, col = cx + (li & 3);
            o.x = (accumulate && col < C && row < D::K) ? tp[row * C + col] : T(0);
        } else {
            o.x = T(0);
        }
    };
    const int nsteps = j1 - j0;
    AV an[NKV];
    Old on;
    load_a(0, an);
    load_old(0, on);
    for (int step = 0; step < nsteps; ++step) {
        AV a[NKV];
#pragma unroll
        for (int kv = 0; kv < NKV; ++kv) a[kv] = an[kv];
        const Old oc = on;
        if (step + 1 < nsteps) {
            load_a(step + 1, an);
            load_old(step + 1, on);
        }
        const int t = ts_tgt[j0 + step];
        VT acc[WT], accx = VT{0, 0, 0, 0};
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) acc[ct] = VT{0, 0, 0, 0};
#pragma unroll
        for (int ks = 0; ks < D::NKS; ++ks) {
#pragma unroll
            for (int ct = 0; ct < WT; ++ct) mfma_16x16x4<T>(a[ks / VEC][ks % VEC], b[ct][ks], acc[ct]);
            if constexpr (XC > 0) accx = __builtin_amdgcn_mfma_f32_4x4x1f32(a[ks / VEC][ks % VEC], bx[ks], accx, 0, 0, 0);
        }
#pragma unroll
        for (int ct = 0; ct < WT; ++ct) {
            const int col = cb + WT * li + ct;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int row = rt * 16 + mfma_row<T>(kq, e);
                if (col < C && row < D::K) out[((int64_t)t * D::K + row) * C + col] = oc.v[ct][e] + acc[ct][e];
            }
        }
        if constexpr (XC > 0) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                accx[i] += __shfl_xor(accx[i], 16);
                accx[i] += __shfl_xor(accx[i], 32);
            }
            const T mine = kq == 0 ? accx[0] : kq == 1 ? accx[1] : kq == 2 ? accx[2] : accx[3];
            const int row = 16 * rt + 4 * (li >> 2) + kq, col = cx + (li & 3);
            if (col < C && row < D::K) out[((int64_t)t * D::K + row) * C + col] = oc.x + mine;
        }
    }
}

// Row-tile form of the target-stationary translation for passes with few
// pairs per target (M2M: a parent's multipole from its children).  One wave
// per (target, 16-row tile of the result, item of WT column tiles [+ XC
// narrow columns]) sums the target's pairs in list order in registers, the
// next pair's source fragments and operator tile in flight, and stores its
// tile once.  As for the source-stationary form: short waves in large
// numbers for passes that run level by level.
template <typename T, int ORD, int WT, int XC>
__global__ __launch_bounds__(64) void k_trans_tr(int n_items, int items_per_tgt, const int32_t *__restrict__ red_tgt,
                                                 const int32_t *__restrict__ red_ptr,
                                                 const int32_t *__restrict__ ts_src,
                                                 const int32_t *__restrict__ ts_op, const T *__restrict__ op_vec,
                                                 const T *__restrict__ in, int C, int accumulate, T *__restrict__ out)
{
    using D = M2LDims<ORD>;
    using VT = typename std::conditional<sizeof(T) == 4, f32x4, f64x4>::type;
    constexpr int VEC = 16 / sizeof(T);
    constexpr int NKV = (D::NKS + VEC - 1) / VEC;
    using AV = T __attribute__((ext_vector_type(VEC)));
    static_assert(XC == 0 || (XC == 4 && sizeof(T) == 4), "4x4-block columns: four, FP32 only");
    struct BV {
        T v[WT];
    };
    struct Step {
        AV a[NKV];
        T b[WT][D::NKS];
        T x[XC ? D::NKS : 1];
    };
    const int w = blockIdx.x;
    if (w >= n_items) return;
    const int ti = w / (items_per_tgt * D::NRT);
    const int rem = w - ti * items_per_tgt * D::NRT;
    const int rt = rem / items_per_tgt;
    const int cb = (rem - rt * items_per_tgt) * WT * 16, cx = cb + WT * 16;
    const int lane = threadIdx.x & 63, li = lane & 15, kq = lane >> 4;
    const int t = red_tgt[ti], j0 = red_ptr[ti], j1 = red_ptr[ti + 1];
    const int boff = kq * C + cb + WT * li, xoff = kq * C + cx + (li & 3);
    const int blast = min(4 * (D::NKS - 1) + kq, D::K - 1) * C - 4 * (D::NKS - 1) * C - kq * C;
    const uint32_t mbytes = (uint32_t)((D::K * C + 256) * sizeof(T));
    constexpr uint32_t obytes = D::NRT * NKV * 64 * 16;
    auto load = [&](int j, Step &st) {
        const auto rm = buf_rsrc(in + (int64_t)ts_src[j] * D::K * C, mbytes);
#pragma unroll
        for (int ks = 0; ks < D::NKS; ++ks) {
            const int lofs = ks == D::NKS - 1 ? blast : 0;
            const int sofs = 4 * ks * C * (int)sizeof(T);
            const BV v = buf_load<BV>(rm, (boff + lofs) * (int)sizeof(T), sofs);
#pragma unroll
            for (int ct = 0; ct < WT; ++ct) st.b[ct][ks] = v.v[ct];
            if constexpr (XC > 0) st.x[ks] = buf_load<T>(rm, (xoff + lofs) * (int)sizeof(T), sofs);
        }
        const auto ro = buf_rsrc(op_vec + (int64_t)(ts_op[j] >> 3) * D::NRT * NKV * 64 * VEC, obytes);
#pragma unroll
        for (int kv = 0; kv < NKV; ++kv) st.a[kv] = buf_load<AV>(ro, lane * 16, (rt * NKV + kv) * 1024);
    };
    VT acc[WT], accx = VT{0, 0, 0, 0};
#pragma unroll
    for (int ct = 0; ct < WT; ++ct) acc[ct] = VT{0, 0, 0, 0};
    auto comp = [&](const Step &st) {
#pragma unroll
        for (int ks = 0; ks < D::NKS; ++ks) {
#pragma unroll
            for (int ct = 0; ct < WT; ++ct) mfma_16x16x4<T>(st.a[ks / VEC][ks % VEC], st.b[ct][ks], acc[ct]);
            if constexpr (XC > 0)
                accx = __builtin_amdgcn_mfma_f32_4x4x1f32(st.a[ks / VEC][ks % VEC], st.x[ks], accx, 0, 0, 0);
        }
    };
    // two pairs per trip (static operand sets), the next one in flight
    if (j0 < j1) {
        Step s0, s1;
        load(j0, s0);
        for (int j = j0; j < j1; j += 2) {
            if (j + 1 < j1) load(j + 1, s1);
            comp(s0);
            if (j + 1 >= j1) break;
            if (j + 2 < j1) load(j + 2, s0);
            comp(s1);
        }
    }
#pragma unroll
    for (int ct = 0; ct < WT; ++ct) {
        const int col = cb + WT * li + ct;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int row = rt * 16 + mfma_row<T>(kq, e);
            if (col < C && row < D::K) {
                T *o = out + ((int64_t)t * D::K + row) * C + col;
                *o = accumulate ? *o + acc[ct][e] : acc[ct][e];
            }
        }
    }
    if constexpr (XC > 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            accx[i] += __shfl_xor(accx[i], 16);
            accx[i] += __shfl_xor(accx[i], 32);
        }
        const T mine = kq == 0 ? accx[0] : kq == 1 ? accx[1] : kq == 2 ? accx[2] : accx[3];
        const int row = 16 * rt + 4 * (li >> 2) + kq, col = cx + (li & 3);
        if (col < C && row < D::K) {
            T *o = out + ((int64_t)t * D::K + row) * C + col;
            *o = accumulate ? *o + mine : mine;
        }
    }
}

// out[t][row][c0 + c] (=|+=) sum over the pairs of t (fixed order) of
// tmp[slot][c][row].
template <typename T, int ORD>
__global__ __launch_bounds__(256) void k_pass_reduce(const int32_t *__restrict__ red_tgt,
                                                     const int32_t *__restrict__ red_ptr,
                                                     const int32_t *__restrict__ red_slot, const T *__restrict__ tmp,
                                                     int C, int c0, int Cc, int accumulate, T *__restrict__ out)
{
    using D = M2LDims<ORD>;
    __shared__ int64_t sbase[512];
    const int ti = blockIdx.x;
    const int32_t t = red_tgt[ti], j0 = red_ptr[ti], np = red_ptr[ti + 1] - j0;
    for (int j = threadIdx.x; j < np && j < 512; j += 256) sbase[j] = (int64_t)red_slot[j0 + j] * Cc * D::KP;
    __syncthreads();
    for (int idx = threadIdx.x; idx < Cc * D::K; idx += 256) {
        const int c = idx / D::K, row = idx - c * D::K;
        const T *tp = tmp + (int64_t)c * D::KP + row;
        T s0 = 0, s1 = 0, s2 = 0, s3 = 0;
        int j = 0;
        const int nl = np < 512 ? np : 512;
        for (; j + 4 <= nl; j += 4) {
            s0 += tp[sbase[j]];
            s1 += tp[sbase[j + 1]];
            s2 += tp[sbase[j + 2]];
            s3 += tp[sbase[j + 3]];
        }
        for (; j < nl; ++j) s0 += tp[sbase[j]];
        for (; j < np; ++j) s0 += tp[(int64_t)red_slot[j0 + j] * Cc * D::KP];
        const T s = (s0 + s1) + (s2 + s3);
        T *o = out + ((int64_t)t * D::K + row) * C + c0 + c;
        *o = accumulate ? *o + s : s;
    }
}

// Work items of one column chunk width Cc (cached per engine and width).
static const int32_t *pass_items(const TransPass &T, bool mfma, int Cc, int *n_items, hipStream_t s, int width = 64)
{
    const int64_t key = (mfma ? 1000000 : 0) + (int64_t)width * 10000000 + Cc;
    for (auto &kv : T.item_cache)
        if (kv.first == key) {
            *n_items = (int)(kv.second.n / 3);
            return kv.second.p;
        }
    std::vector<int32_t> it;
    for (int64_t g = 0; g < T.n_groups; ++g) {
        const int64_t ncols = (int64_t)(T.h_gbeg[g + 1] - T.h_gbeg[g]) * Cc;
        if (mfma) {
            const int64_t nct = cdiv(ncols, 16), WT = 8;
            for (int64_t c = 0; c < nct; c += WT) it.insert(it.end(), {(int32_t)g, (int32_t)c, (int32_t)std::min(nct, c + WT)});
        } else {
            for (int64_t c = 0; c < ncols; c += width)
                it.insert(it.end(), {(int32_t)g, (int32_t)c, (int32_t)std::min(ncols, c + width)});
        }
    }
    T.item_cache.emplace_back(key, DevBuf<int32_t>());
    auto &buf = T.item_cache.back().second;
    buf.upload(it, s);
    XRL_HIP(hipStreamSynchronize(s));
    *n_items = (int)(it.size() / 3);
    return buf.p;
}

// One translation pass: grouped GEMM into the scratch array, then the
// per-target reduction into `out` (overwrite or accumulate).
// op_vec: the operators of the target-stationary kernel (vector fragment
// order); refl: its codes carry reflection bits (M2L) or not (M2M, L2L).
template <typename T, int ORD>
static void pass_launch(const xrl_plan *P, const TransPass &TP, const T *op_frag, const T *op_k, const T *op_vec,
                        const T *op_tail, bool refl, const T *in, T *out, int accumulate, DevBuf<T> *tmp, int C,
                        hipStream_t s, bool force_ts, const T *op_full = nullptr, const T *op_full_tail = nullptr)
{
    using D = M2LDims<ORD>;
    if (TP.n_pairs == 0) return;
    const int eng = P->m2l_engine;
    // MFMA: M2M and L2L (few pairs per target) always target-stationary;
    // M2L target-stationary from ts_min_cols real columns on (always when
    // force_ts: the caller has no per-pair scratch to give)
    if (force_ts || eng == XRL_M2L_MFMA_TS || (eng == XRL_M2L_MFMA && (!refl || C >= P->ts_min_cols))) {
        // tiles per wave: the widest (up to the register budget) that wastes
        // the fewest padded tiles; in FP32, one to four columns past the last
        // full tile go to 4x4 MFMA blocks of the same wave instead of a tile
        // one source per target (L2L): source-stationary; few pairs per
        // target otherwise (or asked for): the lean form
        const bool ss = !refl && TP.n_pairs == TP.n_red && P->ps_l2l;
        // at most eight pairs per target (M2M): one wave per row tile when
        // the level has fewer targets than the chip has SIMDs (tr_m2m = 2),
        // always (1) or never (0)
        const bool tr = !refl && !ss && TP.n_pairs <= 8 * TP.n_red &&
                        (P->tr_m2m == 1 || (P->tr_m2m == 2 && TP.n_red < 1024));
        const bool lean = !ss && !tr && (refl ? P->ts_kernel == 2 : TP.n_pairs < 2 * TP.n_red);
        const int ntiles = (int)cdiv(C, 16);
        const int wmax = ts_max_tiles<T, ORD>();
        // (up to two full tiles: with three, the accumulators of the extra
        // blocks no longer fit the registers)
        const bool xc = !lean && sizeof(T) == 4 && P->ts_narrow_cols && C > 16 && C % 16 >= 1 && C % 16 <= 4 &&
                        ntiles - 1 <= std::min(wmax, 2);
        int WT = 1;
        if (xc)
            WT = ntiles - 1;
        else
            for (int w = 1; w <= wmax; ++w)
                if (cdiv(ntiles, w) * w <= cdiv(ntiles, WT) * WT) WT = w;
        const int ipt = xc ? 1 : (int)cdiv(ntiles, WT);
        const int64_t n_items = TP.n_red * ipt;
        XRL_CHECK(n_items < (int64_t(1) << 31), XRL_E_UNSUPPORTED, "xrl_fmm_matvec: too many translation items");
        const unsigned nb = (unsigned)n_items;
        const int32_t *ord = P->ts_order ? TP.ts_order.p : nullptr;
        auto go = [&](auto wt, auto xcols) {
            constexpr int W = decltype(wt)::value, X = decltype(xcols)::value;
            if (refl && P->ts_kernel == 1)
                k_trans_ts<T, ORD, W, true, X><<<nb, 64, 0, s>>>((int)n_items, ipt, ord, TP.red_tgt.p, TP.red_ptr.p,
                                                                 TP.ts_src.p, TP.ts_op.p, op_vec, op_tail, in, C,
                                                                 accumulate, out);
            else if (tr)
                k_trans_tr<T, ORD, W, X><<<(unsigned)(TP.n_red * ipt * M2LDims<ORD>::NRT), 64, 0, s>>>(
                    (int)(TP.n_red * ipt * M2LDims<ORD>::NRT), ipt, TP.red_tgt.p, TP.red_ptr.p, TP.ts_src.p,
                    TP.ts_op.p, op_vec, in, C, accumulate, out);
            else if (ss)
                k_trans_ps<T, ORD, W, X><<<(unsigned)(TP.n_ps * ipt * M2LDims<ORD>::NRT), 64, 0, s>>>(
                    (int)(TP.n_ps * ipt * M2LDims<ORD>::NRT), ipt, TP.ps_beg.p, TP.ts_tgt.p, TP.ts_src.p, TP.ts_op.p, op_vec, in, C,
                    accumulate, out);
            else if (lean)
                k_trans_ts_lean<T, ORD, W><<<nb, 64, 0, s>>>((int)n_items, ipt, TP.red_tgt.p, TP.red_ptr.p,
                                                              TP.ts_src.p, refl ? TP.ts_op_full.p : TP.ts_op.p,
                                                              refl ? op_full : op_vec, in, C, accumulate, out);
            else if (refl)
                k_trans_ts<T, ORD, W, false, X><<<nb, 64, 0, s>>>((int)n_items, ipt, ord, TP.red_tgt.p, TP.red_ptr.p,
                                                                  TP.ts_src.p, TP.ts_op_full.p, op_full, op_full_tail,
                                                                  in, C, accumulate, out);
            else
                k_trans_ts<T, ORD, W, false, X><<<nb, 64, 0, s>>>((int)n_items, ipt, ord, TP.red_tgt.p, TP.red_ptr.p,
                                                                  TP.ts_src.p, TP.ts_op.p, op_vec, op_tail, in, C,
                                                                  accumulate, out);
        };
        using I0 = std::integral_constant<int, 0>;
        auto go_w = [&](auto wt) {
            if constexpr (sizeof(T) == 4) {
                if (xc) {
                    go(wt, std::integral_constant<int, 4>());
                    return;
                }
            }
            go(wt, I0());
        };
        if (WT == 1) go_w(std::integral_constant<int, 1>());
        if constexpr (ts_max_tiles<T, ORD>() >= 2)
            if (WT == 2) go_w(std::integral_constant<int, 2>());
        if constexpr (ts_max_tiles<T, ORD>() >= 3)
            if (WT == 3) go(std::integral_constant<int, 3>(), I0());
        if constexpr (ts_max_tiles<T, ORD>() >= 4)
            if (WT == 4) go(std::integral_constant<int, 4>(), I0());
        XRL_HIP(hipGetLastError());
        return;
    }
    const bool mfma = eng != XRL_M2L_VALU;
    XRL_CHECK(tmp, XRL_E_UNSUPPORTED, "xrl_fmm_matvec: offset-stationary translations need the per-pair scratch");
    // column chunk so that the per-pair scratch stays within the plan's
    // scratch budget (a quarter of the device memory free at the first
    // translation, at least 4 GiB; fixed from then on, so that a captured
    // graph sees the same chunks)
    if (P->scratch_budget == 0) {
        size_t fr = 0, tot = 0;
        XRL_HIP(hipMemGetInfo(&fr, &tot));
        P->scratch_budget = std::max<int64_t>(int64_t(4) << 30, (int64_t)(fr / 4));
    }
    const int64_t per_col = TP.n_pairs * (int64_t)D::KP * (int64_t)sizeof(T);
    const int Cc = (int)std::max<int64_t>(1, std::min<int64_t>(C, P->scratch_budget / per_col));
    if (tmp->n < (size_t)(TP.n_pairs * (int64_t)Cc * D::KP)) tmp->alloc(TP.n_pairs * (int64_t)Cc * D::KP);
    for (int c0 = 0; c0 < C; c0 += Cc) {
        const int cc = std::min(Cc, C - c0);
        int n_items = 0;
        // the column-per-thread vector-ALU kernel: FP32, K = (p+1)^2 registers
        constexpr bool col = sizeof(T) == 4 && ORD <= 8;
        const int32_t *items = pass_items(TP, mfma, cc, &n_items, s, !mfma && col && P->valu_col ? 256 : 64);
        if (mfma) {
            k_m2l_os_mfma<T, ORD><<<(unsigned)cdiv(n_items, 4), 256, 0, s>>>(
                items, n_items, TP.gbeg.p, TP.goff.p, TP.src.p, op_frag, in, C, c0, cc, tmp->p);
        } else {
            // the LDS-staged operator of the vector-ALU kernel fits up to order 8
            if constexpr (col) {
                if (P->valu_col)
                    k_m2l_os_col<ORD><<<(unsigned)n_items, 256, 0, s>>>(items, TP.gbeg.p, TP.goff.p, TP.src.p,
                                                                         (const float *)op_k, (const float *)in, C, c0,
                                                                         cc, (float *)tmp->p);
                else
                    k_m2l_os_valu<T, ORD><<<(unsigned)n_items, 256, 0, s>>>(items, TP.gbeg.p, TP.goff.p, TP.src.p,
                                                                            op_k, in, C, c0, cc, tmp->p);
            } else if constexpr (ORD <= 8 && (sizeof(T) == 4 || ORD <= 6))
                k_m2l_os_valu<T, ORD><<<(unsigned)n_items, 256, 0, s>>>(items, TP.gbeg.p, TP.goff.p, TP.src.p, op_k,
                                                                        in, C, c0, cc, tmp->p);
            else
                fail(XRL_E_UNSUPPORTED, "xrl_fmm_matvec: the vector-ALU translations support order <= 8 "
                                        "(<= 6 in FP64)");
        }
        XRL_HIP(hipGetLastError());
        k_pass_reduce<T, ORD><<<(unsigned)TP.n_red, 256, 0, s>>>(TP.red_tgt.p, TP.red_ptr.p, TP.red_slot.p, tmp->p, C,
                                                                 c0, cc, accumulate, out);
        XRL_HIP(hipGetLastError());
    }
}

// ---------------------------------------------------------------- driver
template <typename T>
__global__ void k_fill_zero(T *__restrict__ p, int64_t n)
{
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = T(0);
}

template <typename T>
static void p2p_launch(const xrl_plan *P, const T *val, const T *xs, T *ys, int C, hipStream_t s)
{
    if (P->n_leaves == 0) return;
    if constexpr (sizeof(T) == 4) {
        if (C > 16 && P->p2p_form == 0) {
            // column items: WT 16-column tiles (+ four narrow columns when
            // 1..4 columns are left past the last full tile)
            const int ntiles = (int)cdiv(C, 16);
            const bool xc = C % 16 >= 1 && C % 16 <= 4 && ntiles - 1 <= 4;
            int WT = 1;
            if (xc)
                WT = ntiles - 1;
            else
                for (int w = 1; w <= 4; ++w)
                    if (cdiv(ntiles, w) * w <= cdiv(ntiles, WT) * WT) WT = w;
            const int ipl = xc ? 1 : (int)cdiv(ntiles, WT);
            const int64_t n_items = P->n_leaves * ipl;
            XRL_CHECK(n_items < (int64_t(1) << 31), XRL_E_UNSUPPORTED, "xrl_fmm_matvec: too many P2P items");
            auto mf = [&](auto wt, auto xcols) {
                constexpr int W = decltype(wt)::value, X = decltype(xcols)::value;
                k_p2p_mfma<W, X><<<(unsigned)n_items, 64, 0, s>>>(ipl, P->leaf_box.p, P->box_beg.p, P->box_end.p,
                                                                 P->near_rows.p, P->near_src.p, P->leaf_tpad.p,
                                                                 P->near_val_off.p, val, xs, ys, C);
            };
            auto mw = [&](auto wt) {
                if (xc)
                    mf(wt, std::integral_constant<int, 4>());
                else
                    mf(wt, std::integral_constant<int, 0>());
            };
            if (WT == 1) mw(std::integral_constant<int, 1>());
            if (WT == 2) mw(std::integral_constant<int, 2>());
            if (WT == 3) mw(std::integral_constant<int, 3>());
            if (WT == 4) mw(std::integral_constant<int, 4>());
            XRL_HIP(hipGetLastError());
            return;
        }
        if (C > 16 && P->p2p_form == 1) {
            auto sx = [&](auto ctc) {
                constexpr int CT = decltype(ctc)::value;
                dim3 grid((unsigned)P->n_leaves, (unsigned)cdiv(C, CT));
                k_p2p_sx<CT><<<grid, 64, 0, s>>>(P->leaf_box.p, P->box_beg.p, P->box_end.p, P->near_rows.p,
                                                 P->near_src.p, P->leaf_tpad.p, P->near_val_off.p, val, xs, ys, C);
            };
            int ct = 24;
            for (int w : {32, 36, 48})
                if (cdiv(C, w) * w <= cdiv(C, ct) * ct) ct = w;
            if (ct == 24)
                sx(std::integral_constant<int, 24>());
            else if (ct == 32)
                sx(std::integral_constant<int, 32>());
            else if (ct == 36)
                sx(std::integral_constant<int, 36>());
            else
                sx(std::integral_constant<int, 48>());
            XRL_HIP(hipGetLastError());
            return;
        }
        if (C > 16) {
            auto wide = [&](auto ctc) {
                constexpr int CT = decltype(ctc)::value;
                dim3 grid((unsigned)P->n_leaves, (unsigned)cdiv(C, CT));
                k_p2p_wide<CT><<<grid, 256, 0, s>>>(P->leaf_box.p, P->box_beg.p, P->box_end.p, P->near_rows.p,
                                                    P->near_src.p, P->leaf_tpad.p, P->near_val_off.p, val, xs, ys, C);
            };
            // the tile width (24, 32 or 36) with the least padding, the
            // widest among equals
            int ct = 24;
            for (int w : {32, 36})
                if (cdiv(C, w) * w <= cdiv(C, ct) * ct) ct = w;
            if (ct == 24)
                wide(std::integral_constant<int, 24>());
            else if (ct == 32)
                wide(std::integral_constant<int, 32>());
            else
                wide(std::integral_constant<int, 36>());
            XRL_HIP(hipGetLastError());
            return;
        }
    }
    auto go = [&](auto ctc) {
        constexpr int CT = decltype(ctc)::value;
        dim3 grid((unsigned)P->n_leaves, (unsigned)cdiv(C, CT));
        k_p2p<T, CT><<<grid, 256, 0, s>>>(P->leaf_box.p, P->box_beg.p, P->box_end.p, P->near_rows.p, P->near_src.p,
                                          P->leaf_tpad.p, P->near_val_off.p, val, xs, ys, C);
    };
    if (C <= 2)
        go(std::integral_constant<int, 2>());
    else if (C <= 4)
        go(std::integral_constant<int, 4>());
    else if (C <= 8)
        go(std::integral_constant<int, 8>());
    else
        go(std::integral_constant<int, 16>());
    XRL_HIP(hipGetLastError());
}

template <typename T>
struct Ops {
    const T *near, *mom, *m2m_f, *m2m_k, *l2l_f, *l2l_k, *m2l_f, *m2l_k;
    const T *m2m_v, *l2l_v, *m2l_v;  // target-stationary operators (M2L: non-negative offsets)
    const T *m2l_full;               // target-stationary M2L operators of every offset
    const T *m2m_t, *l2l_t, *m2l_full_t, *m2l_t;  // their last rows (orders with K = 16 n + 1)
};

template <typename T, int ORD>
static void translations(const xrl_plan *P, const Ops<T> &op, T *M, T *L, DevBuf<T> *tmp, int C, hipStream_t s,
                         bool force_ts, const std::function<void(int)> &mark, bool leaf_l2l_in_l2p)
{
    using D = M2LDims<ORD>;
    mark(3);
    for (int l = P->depth - 1; l >= 0; --l)
        pass_launch<T, ORD>(P, P->m2m[l], op.m2m_f, op.m2m_k, op.m2m_v, op.m2m_t, false, M, M, 0, tmp, C, s,
                            force_ts);
    // zero every local expansion (a fill kernel, so the sequence stays
    // capturable into a HIP graph without memset nodes)
    const int64_t nL = P->B * (int64_t)D::K * C;
    k_fill_zero<T><<<(unsigned)std::min<int64_t>(cdiv(nL, 256), 65536), 256, 0, s>>>(L, nL);
    XRL_HIP(hipGetLastError());
    mark(4);
    pass_launch<T, ORD>(P, P->m2l, op.m2l_f, op.m2l_k, op.m2l_v, op.m2l_t, true, M, L, 0, tmp, C, s, force_ts,
                        op.m2l_full, op.m2l_full_t);
    mark(5);
    // (without the leaf targets when L2P applies the leaves' L2L itself)
    const std::vector<TransPass> &l2l = leaf_l2l_in_l2p ? P->l2l_inner : P->l2l;
    for (int l = 3; l <= P->depth; ++l)
        pass_launch<T, ORD>(P, l2l[l], op.l2l_f, op.l2l_k, op.l2l_v, op.l2l_t, false, L, L, 1, tmp, C, s, force_ts);
    mark(6);
}

// Enqueue one matvec on stream s: kernels only (no allocation, no host
// synchronisation once the work buffers exist), so the same sequence can be
// captured into a HIP graph.  The epilogue scalars are read from the plan's
// ep_dev buffer when has_alpha / has_beta.
// Work arrays of one matvec (sorted panel order, real columns): densities
// and potentials [N][C] + 256, expansions [B][K][C] + 256 elements each.  The
// slack after the densities: P2P reads (and discards) the padded columns of
// the last source row; after the expansions: the target-stationary kernel
// reads (and discards) up to 16 WT columns past the last record.
template <typename T>
struct Work {
    T *xs, *ys, *M, *L;
    DevBuf<T> *tmp;  // per-pair scratch of the offset-stationary translations (null: target-stationary only)
    const double *alpha, *beta;  // epilogue scalars on the device ([2 C_complex] each) or null
    bool force_ts;
    bool profile;  // record the phase events of the plan's profiling ring
};
inline int64_t work_dens_elems(const xrl_plan *P, int C) { return P->N * (int64_t)C + 256; }
inline int64_t work_exp_elems(const xrl_plan *P, int C) { return P->B * (int64_t)P->K * C + 256; }

template <typename T>
static void run_matvec(const xrl_plan *P, const void *x, int64_t ldx, int ncols, int dtype, void *y, int64_t ldy,
                       hipStream_t s, const Work<T> &wk, const Ops<T> &op)
{
    const int C = 2 * ncols;
    const int K = P->K;
    const int64_t N = P->N;
    const bool prof = wk.profile;
    std::function<void(int)> mark = [&](int i) {
        if (prof) XRL_HIP(hipEventRecord(P->prof_ev[P->prof_count % xrl_plan::kProfRing][i], s));
    };
    mark(0);
    const int bs = 256;
    const unsigned gx = (unsigned)std::min<int64_t>(cdiv(N * ncols, bs), 1 << 20);
    const size_t pair = dtype == XRL_C64 ? 2 * sizeof(float) : 2 * sizeof(double);
    const bool aligned = (uintptr_t)x % pair == 0;
    if (dtype == XRL_C64) {
        if (aligned)
            k_gather_x<float, T, true><<<gx, bs, 0, s>>>(N, P->perm.p, (const float *)x, ldx, ncols, wk.xs);
        else
            k_gather_x<float, T, false><<<gx, bs, 0, s>>>(N, P->perm.p, (const float *)x, ldx, ncols, wk.xs);
    } else {
        if (aligned)
            k_gather_x<double, T, true><<<gx, bs, 0, s>>>(N, P->perm.p, (const double *)x, ldx, ncols, wk.xs);
        else
            k_gather_x<double, T, false><<<gx, bs, 0, s>>>(N, P->perm.p, (const double *)x, ldx, ncols, wk.xs);
    }
    XRL_HIP(hipGetLastError());
    mark(1);
    p2p_launch<T>(P, op.near, wk.xs, wk.ys, C, s);
    mark(2);
    // column tile of P2M / L2P: the narrowest of 8, 16, 24, 32, 48 (FP32) or
    // 8, 16 (FP64) that holds all columns, else the widest
    auto moment_tiles = [&](auto fn) {
        if (C <= 8) return fn(std::integral_constant<int, 8>());
        if (sizeof(T) == 8 || C <= 16) return fn(std::integral_constant<int, 16>());
        if constexpr (sizeof(T) == 4) {
            if (C <= 24) return fn(std::integral_constant<int, 24>());
            if (C <= 32) return fn(std::integral_constant<int, 32>());
            return fn(std::integral_constant<int, 48>());
        }
    };
    // the FP32 matrix-core L2P applies the leaves' L2L itself (Q' table)
    const bool fuse_l2l = sizeof(T) == 4 && P->n_leaves > 0 && C > 16 && P->leaf_mfma && P->leaf_l2l &&
                          P->mom_l2l32.p != nullptr && (int)P->l2l_inner.size() == P->depth + 1;
    bool p2m_done = false;
    if constexpr (sizeof(T) == 4) {
        if (P->n_leaves > 0 && C > 16 && P->leaf_mfma) {
            const int ntiles = (int)cdiv(C, 16);
            const bool xc = C % 16 >= 1 && C % 16 <= 4 && ntiles - 1 <= 4;
            int WT = 1;
            if (xc)
                WT = ntiles - 1;
            else
                for (int w = 1; w <= 4; ++w)
                    if (cdiv(ntiles, w) * w <= cdiv(ntiles, WT) * WT) WT = w;
            const int ipl = xc ? 1 : (int)cdiv(ntiles, WT);
            const int64_t n_items = P->n_leaves * ipl;
            XRL_CHECK(n_items < (int64_t(1) << 31), XRL_E_UNSUPPORTED, "xrl_fmm_matvec: too many P2M items");
            auto go = [&](auto ordc, auto wt, auto xcols) {
                constexpr int O = decltype(ordc)::value, W = decltype(wt)::value, X = decltype(xcols)::value;
                k_p2m_mfma<O, W, X><<<(unsigned)n_items, 64, 0, s>>>(ipl, P->leaf_box.p, P->box_beg.p, P->box_end.p,
                                                                    (const float *)op.mom, (const float *)wk.xs,
                                                                    (float *)wk.M, C);
            };
            auto go_w = [&](auto ordc) {
                auto gx = [&](auto wt) {
                    if (xc)
                        go(ordc, wt, std::integral_constant<int, 4>());
                    else
                        go(ordc, wt, std::integral_constant<int, 0>());
                };
                if (WT == 1) gx(std::integral_constant<int, 1>());
                if (WT == 2) gx(std::integral_constant<int, 2>());
                if (WT == 3) gx(std::integral_constant<int, 3>());
                if (WT == 4) gx(std::integral_constant<int, 4>());
            };
            switch (P->p) {
                case 2: go_w(std::integral_constant<int, 2>()); break;
                case 4: go_w(std::integral_constant<int, 4>()); break;
                case 6: go_w(std::integral_constant<int, 6>()); break;
                case 8: go_w(std::integral_constant<int, 8>()); break;
                case 10: go_w(std::integral_constant<int, 10>()); break;
                default: go_w(std::integral_constant<int, 12>()); break;
            }
            XRL_HIP(hipGetLastError());
            p2m_done = true;
        }
    }
    if (P->n_leaves > 0 && !p2m_done) {
        moment_tiles([&](auto ctc) {
            constexpr int CT = decltype(ctc)::value;
            k_p2m<T, CT><<<dim3((unsigned)P->n_leaves, (unsigned)cdiv(C, CT)), 256, 0, s>>>(
                P->leaf_box.p, P->box_beg.p, P->box_end.p, op.mom, wk.xs, wk.M, C, K);
        });
        XRL_HIP(hipGetLastError());
    }
    switch (P->p) {
        case 2: translations<T, 2>(P, op, wk.M, wk.L, wk.tmp, C, s, wk.force_ts, mark, fuse_l2l); break;
        case 4: translations<T, 4>(P, op, wk.M, wk.L, wk.tmp, C, s, wk.force_ts, mark, fuse_l2l); break;
        case 6: translations<T, 6>(P, op, wk.M, wk.L, wk.tmp, C, s, wk.force_ts, mark, fuse_l2l); break;
        case 8: translations<T, 8>(P, op, wk.M, wk.L, wk.tmp, C, s, wk.force_ts, mark, fuse_l2l); break;
        case 10: translations<T, 10>(P, op, wk.M, wk.L, wk.tmp, C, s, wk.force_ts, mark, fuse_l2l); break;
        default: translations<T, 12>(P, op, wk.M, wk.L, wk.tmp, C, s, wk.force_ts, mark, fuse_l2l); break;
    }
    bool l2p_done = false;
    if constexpr (sizeof(T) == 4) {
        if (P->n_leaves > 0 && C > 16 && P->leaf_mfma) {
            // column items as in P2P: WT 16-column tiles, or the tiles plus
            // four narrow columns
            const int ntiles = (int)cdiv(C, 16);
            const bool xc = C % 16 >= 1 && C % 16 <= 4 && ntiles - 1 <= 4;
            int WT = 1;
            if (xc)
                WT = ntiles - 1;
            else
                for (int w = 1; w <= 4; ++w)
                    if (cdiv(ntiles, w) * w <= cdiv(ntiles, WT) * WT) WT = w;
            const int ipl = xc ? 1 : (int)cdiv(ntiles, WT);
            const int64_t n_items = P->n_leaves * ipl;
            XRL_CHECK(n_items < (int64_t(1) << 31), XRL_E_UNSUPPORTED, "xrl_fmm_matvec: too many L2P items");
            auto go = [&](auto ordc, auto wt, auto xcols) {
                constexpr int O = decltype(ordc)::value, W = decltype(wt)::value, X = decltype(xcols)::value;
                if (fuse_l2l)
                    k_l2p_mfma<O, W, X, true><<<(unsigned)n_items, 64, 0, s>>>(
                        ipl, P->leaf_box.p, P->box_beg.p, P->box_end.p, P->box_h.p, (const float *)op.mom,
                        (const float *)wk.L, (float *)wk.ys, C, P->mom_l2l32.p, P->box_parent.p, P->box_level.p);
                else
                    k_l2p_mfma<O, W, X, false><<<(unsigned)n_items, 64, 0, s>>>(
                        ipl, P->leaf_box.p, P->box_beg.p, P->box_end.p, P->box_h.p, (const float *)op.mom,
                        (const float *)wk.L, (float *)wk.ys, C, nullptr, nullptr, nullptr);
            };
            auto go_w = [&](auto ordc) {
                auto gx = [&](auto wt) {
                    if (xc)
                        go(ordc, wt, std::integral_constant<int, 4>());
                    else
                        go(ordc, wt, std::integral_constant<int, 0>());
                };
                if (WT == 1) gx(std::integral_constant<int, 1>());
                if (WT == 2) gx(std::integral_constant<int, 2>());
                if (WT == 3) gx(std::integral_constant<int, 3>());
                if (WT == 4) gx(std::integral_constant<int, 4>());
            };
            switch (P->p) {
                case 2: go_w(std::integral_constant<int, 2>()); break;
                case 4: go_w(std::integral_constant<int, 4>()); break;
                case 6: go_w(std::integral_constant<int, 6>()); break;
                case 8: go_w(std::integral_constant<int, 8>()); break;
                case 10: go_w(std::integral_constant<int, 10>()); break;
                default: go_w(std::integral_constant<int, 12>()); break;
            }
            XRL_HIP(hipGetLastError());
            l2p_done = true;
        }
    }
    if (P->n_leaves > 0 && !l2p_done) {
        const int CT = (sizeof(T) == 8 || C <= 8) ? 8 : 16;
        const unsigned ntile = (unsigned)cdiv(C, CT);
        const size_t sm = (size_t)K * CT * sizeof(T);
        if (CT == 8)
            k_l2p<T, 8><<<dim3((unsigned)P->n_leaves, ntile), 256, sm, s>>>(P->leaf_box.p, P->box_beg.p, P->box_end.p,
                                                                            P->box_h.p, op.mom, wk.L, wk.ys, C, K);
        else
            k_l2p<T, 16><<<dim3((unsigned)P->n_leaves, ntile), 256, sm, s>>>(P->leaf_box.p, P->box_beg.p, P->box_end.p,
                                                                             P->box_h.p, op.mom, wk.L, wk.ys, C, K);
        XRL_HIP(hipGetLastError());
    }
    mark(7);
    const double *da = wk.alpha, *db = wk.beta;
    const unsigned gy = (unsigned)std::min<int64_t>(cdiv(P->Nu * ncols, bs), 1 << 20);
    if (dtype == XRL_C64)
        k_scatter_y<float, T><<<gy, bs, 0, s>>>(P->Nu, P->iperm.p, P->iperm2.p, wk.ys, P->area.p, (const float *)x,
                                                ldx, (float *)y, ldy, ncols, da, db);
    else
        k_scatter_y<double, T><<<gy, bs, 0, s>>>(P->Nu, P->iperm.p, P->iperm2.p, wk.ys, P->area.p,
                                                 (const double *)x, ldx, (double *)y, ldy, ncols, da, db);
    XRL_HIP(hipGetLastError());
    mark(8);
    if (prof) ++P->prof_count;
}

}  // namespace xrl

using namespace xrl;

// Epilogue scalars to the plan's device buffer (ordered on s before the
// kernels that read them).
static void upload_epilogue(const xrl_plan *P, int ncols, const double *alpha, const double *beta, hipStream_t s)
{
    if (!alpha && !beta) return;
    std::vector<double> h(4 * (size_t)ncols, 0.0);
    for (int c = 0; c < ncols; ++c) {
        h[2 * c] = alpha ? alpha[2 * c] : 1.0;
        h[2 * c + 1] = alpha ? alpha[2 * c + 1] : 0.0;
        h[2 * ncols + 2 * c] = beta ? beta[2 * c] : 0.0;
        h[2 * ncols + 2 * c + 1] = beta ? beta[2 * c + 1] : 0.0;
    }
    if (P->ep_dev.n < h.size()) P->ep_dev.alloc(4 * (size_t)P->max_cols);
    XRL_HIP(hipMemcpyAsync(P->ep_dev.p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, s));
}

static Ops<double> ops64(const xrl_plan *P)
{
    return Ops<double>{P->near64.p, P->mom64.p, P->op_m2m64f.p, P->op_m2m64k.p, P->op_l2l64f.p, P->op_l2l64k.p,
                       P->op_m2l64f.p, P->op_m2l64k.p, P->op_m2m64v.p, P->op_l2l64v.p, P->op_m2lc64v.p,
                       P->op_m2l64v.p, P->op_m2m64t.p, P->op_l2l64t.p, P->op_m2l64t.p, P->op_m2lc64t.p};
}
static Ops<float> ops32(const xrl_plan *P)
{
    return Ops<float>{P->near32.p, P->mom32.p, P->op_m2m32f.p, P->op_m2m32k.p, P->op_l2l32f.p, P->op_l2l32k.p,
                      P->op_m2l32f.p, P->op_m2l32k.p, P->op_m2m32v.p, P->op_l2l32v.p, P->op_m2lc32v.p,
                      P->op_m2l32v.p, P->op_m2m32t.p, P->op_l2l32t.p, P->op_m2l32t.p, P->op_m2lc32t.p};
}

// The plan-owned work arrays, grown (hipMalloc) to the call's column count.
template <typename T>
static Work<T> plan_work(const xrl_plan *P, int C, bool ha, bool hb, bool profile, DevBuf<T> &xs, DevBuf<T> &ys,
                         DevBuf<T> &M, DevBuf<T> &L, DevBuf<T> &tmp)
{
    if (xs.n < (size_t)work_dens_elems(P, C)) {
        xs.alloc(work_dens_elems(P, C));
        ys.alloc(work_dens_elems(P, C));
    }
    if (M.n < (size_t)work_exp_elems(P, C)) {
        M.alloc(work_exp_elems(P, C));
        L.alloc(work_exp_elems(P, C));
    }
    const double *da = (ha || hb) ? P->ep_dev.p : nullptr;
    const double *db = hb ? P->ep_dev.p + C : nullptr;
    return Work<T>{xs.p, ys.p, M.p, L.p, &tmp, da, db, false, profile && P->profiling};
}

// profile: record the plan's phase events when its profiling is on (the
// caller has made the ring slot); the solver's inner products pass false.
static void enqueue_matvec(const xrl_plan *P, const void *x, int64_t ldx, int n_cols, int dtype, void *y, int64_t ldy,
                           bool ha, bool hb, hipStream_t s, bool profile = true)
{
    xrl_plan *Pm = const_cast<xrl_plan *>(P);
    const int C = 2 * n_cols;
    if (P->precision == XRL_PREC_FP64)
        run_matvec<double>(P, x, ldx, n_cols, dtype, y, ldy, s,
                           plan_work<double>(P, C, ha, hb, profile, Pm->xs64, Pm->ys64, Pm->M64, Pm->L64,
                                             Pm->os_tmp64),
                           ops64(P));
    else
        run_matvec<float>(P, x, ldx, n_cols, dtype, y, ldy, s,
                          plan_work<float>(P, C, ha, hb, profile, Pm->xs32, Pm->ys32, Pm->M32, Pm->L32, Pm->os_tmp32),
                          ops32(P));
}

// Graph mode: the first call with a new argument set runs eagerly (which
// sizes the work buffers and builds the work lists), then captures the same
// kernel sequence on the plan's capture stream and instantiates it; later
// calls with the same arguments replay it with one hipGraphLaunch.
static void graph_matvec(const xrl_plan *P, const void *x, int64_t ldx, int n_cols, int dtype, void *y, int64_t ldy,
                         bool ha, bool hb, hipStream_t s)
{
    xrl_plan::GraphKey k;
    k.x = x;
    k.y = y;
    k.ldx = ldx;
    k.ldy = ldy;
    k.ncols = n_cols;
    k.dtype = dtype;
    k.alpha = ha;
    k.beta = hb;
    if (P->gexec && k == P->gkey) {
        XRL_HIP(hipGraphLaunch(P->gexec, s));
        ++P->graph_launches;
        return;
    }
    if (P->gexec) {
        XRL_HIP(hipGraphExecDestroy(P->gexec));
        P->gexec = nullptr;
    }
    enqueue_matvec(P, x, ldx, n_cols, dtype, y, ldy, ha, hb, s);
    XRL_HIP(hipStreamSynchronize(s));
    if (!P->cap_stream) XRL_HIP(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    XRL_HIP(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeThreadLocal));
    try {
        enqueue_matvec(P, x, ldx, n_cols, dtype, y, ldy, ha, hb, P->cap_stream);
    } catch (...) {
        (void)hipStreamEndCapture(P->cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    XRL_HIP(hipStreamEndCapture(P->cap_stream, &g));
    const hipError_t e = hipGraphInstantiate(&P->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    XRL_HIP(e);
    P->gkey = k;
}

extern "C" xrl_status xrl_fmm_matvec(const xrl_plan *P, const void *x, int64_t ldx, int32_t n_cols, int32_t dtype,
                                     void *y, int64_t ldy, const xrl_epilogue *ep, void *stream)
{
    return guarded([&] {
        XRL_CHECK(P && x && y, XRL_E_INVALID_ARG, "xrl_fmm_matvec: null argument");
        XRL_CHECK(P->assembled, XRL_E_STATE, "xrl_fmm_matvec: call xrl_nearfield_assemble first");
        XRL_CHECK(n_cols >= 1 && n_cols <= P->max_cols, XRL_E_INVALID_ARG,
                  "xrl_fmm_matvec: n_cols must be in 1..max_cols (%d), got %d", P->max_cols, n_cols);
        XRL_CHECK(ldx >= n_cols && ldy >= n_cols, XRL_E_INVALID_ARG, "xrl_fmm_matvec: ldx/ldy < n_cols");
        XRL_CHECK(dtype == XRL_C64 || dtype == XRL_C128, XRL_E_INVALID_ARG, "xrl_fmm_matvec: bad dtype %d", dtype);
        XRL_CHECK(x != y, XRL_E_INVALID_ARG, "xrl_fmm_matvec: x and y must not alias");
        hipStream_t s = (hipStream_t)stream;
        const AllocStream alloc_scope(s);
        xrl_plan *Pm = const_cast<xrl_plan *>(P);
        if (Pm->profiling) {
            auto &ring = Pm->prof_ev;
            const size_t slot = (size_t)(Pm->prof_count % xrl_plan::kProfRing);
            if (ring.size() <= slot) {
                ring.emplace_back(XRL_N_PHASES + 1, nullptr);
                for (auto &e : ring.back()) XRL_HIP(hipEventCreate(&e));
            }
        }
        const double *al = ep ? ep->alpha : nullptr, *be = ep ? ep->beta : nullptr;
        upload_epilogue(P, n_cols, al, be, s);
        if (P->use_graph && !P->profiling)
            graph_matvec(P, x, ldx, n_cols, dtype, y, ldy, al != nullptr, be != nullptr, s);
        else
            enqueue_matvec(P, x, ldx, n_cols, dtype, y, ldy, al != nullptr, be != nullptr, s);
    });
}

// ---------------------------------------------------------------- matvec without allocation
// The work arrays of xrl_fmm_matvec_noalloc live in this fixed device array
// (each device that runs the library holds its own copy until the process
// ends).  Host code never uses the name `scratch` itself, only the address
// hipGetSymbolAddress returns for the current device.
static constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[kMaxDevices] = {};

// This device's address of `scratch`, looked up once per device.
static unsigned char *scratch_ptr()
{
    int dev = -1;
    XRL_HIP(hipGetDevice(&dev));
    XRL_CHECK(dev >= 0 && dev < kMaxDevices, XRL_E_UNSUPPORTED, "xrl_fmm_matvec_noalloc: device %d out of range",
              dev);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        XRL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        XRL_CHECK(p, XRL_E_HIP, "xrl_fmm_matvec_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = (unsigned char *)p;
    }
    return g_scratch_ptr[dev];
}

__global__ void k_fill_pairs(double *__restrict__ p, int n, double re, double im)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        p[2 * i] = re;
        p[2 * i + 1] = im;
    }
}

template <typename T>
static void noalloc_matvec(const xrl_plan *P, const void *x, int64_t ldx, int n_cols, int dtype, void *y,
                           int64_t ldy, const double *alpha, const double *beta, hipStream_t s)
{
    const int C = 2 * n_cols;
    auto up = [](size_t b) { return (b + 255) & ~size_t(255); };
    const size_t ep_b = up(4 * (size_t)n_cols * sizeof(double));
    const size_t dens_b = up((size_t)work_dens_elems(P, C) * sizeof(T));
    const size_t exp_b = up((size_t)work_exp_elems(P, C) * sizeof(T));
    const size_t need = ep_b + 2 * dens_b + 2 * exp_b;
    XRL_CHECK(need <= kScratchBytes, XRL_E_INVALID_ARG,
              "xrl_fmm_matvec_noalloc: this plan and column count need %zu bytes of work arrays, more than the "
              "%zu-byte scratch (use xrl_fmm_matvec)",
              need, kScratchBytes);
    unsigned char *base = scratch_ptr();
    double *ep = (double *)base;
    const bool has = alpha || beta;
    if (has) {
        // alpha (default 1) in [0, 2 n_cols), beta (default 0) after it
        if (alpha)
            XRL_HIP(hipMemcpyAsync(ep, alpha, 2 * (size_t)n_cols * sizeof(double), hipMemcpyHostToDevice, s));
        else
            k_fill_pairs<<<(unsigned)cdiv(n_cols, 256), 256, 0, s>>>(ep, n_cols, 1.0, 0.0);
        if (beta)
            XRL_HIP(hipMemcpyAsync(ep + C, beta, 2 * (size_t)n_cols * sizeof(double), hipMemcpyHostToDevice, s));
        XRL_HIP(hipGetLastError());
    }
    unsigned char *q = base + ep_b;
    Work<T> wk;
    wk.xs = (T *)q;
    wk.ys = (T *)(q + dens_b);
    wk.M = (T *)(q + 2 * dens_b);
    wk.L = (T *)(q + 2 * dens_b + exp_b);
    wk.tmp = nullptr;
    wk.alpha = has ? ep : nullptr;
    wk.beta = beta ? ep + C : nullptr;
    wk.force_ts = true;
    wk.profile = false;
    if constexpr (sizeof(T) == 8)
        run_matvec<double>(P, x, ldx, n_cols, dtype, y, ldy, s, wk, ops64(P));
    else
        run_matvec<float>(P, x, ldx, n_cols, dtype, y, ldy, s, wk, ops32(P));
}

extern "C" xrl_status xrl_fmm_matvec_noalloc(const xrl_plan *P, const void *x, int64_t ldx, int32_t n_cols,
                                             int32_t dtype, void *y, int64_t ldy, const xrl_epilogue *ep,
                                             void *stream)
{
    return guarded([&] {
        XRL_CHECK(P && x && y, XRL_E_INVALID_ARG, "xrl_fmm_matvec_noalloc: null argument");
        XRL_CHECK(P->assembled, XRL_E_STATE, "xrl_fmm_matvec_noalloc: call xrl_nearfield_assemble first");
        XRL_CHECK(n_cols >= 1 && n_cols <= P->max_cols, XRL_E_INVALID_ARG,
                  "xrl_fmm_matvec_noalloc: n_cols must be in 1..max_cols (%d), got %d", P->max_cols, n_cols);
        XRL_CHECK(ldx >= n_cols && ldy >= n_cols, XRL_E_INVALID_ARG, "xrl_fmm_matvec_noalloc: ldx/ldy < n_cols");
        XRL_CHECK(dtype == XRL_C64 || dtype == XRL_C128, XRL_E_INVALID_ARG, "xrl_fmm_matvec_noalloc: bad dtype %d",
                  dtype);
        XRL_CHECK(x != y, XRL_E_INVALID_ARG, "xrl_fmm_matvec_noalloc: x and y must not alias");
        const double *al = ep ? ep->alpha : nullptr, *be = ep ? ep->beta : nullptr;
        if (P->precision == XRL_PREC_FP64)
            noalloc_matvec<double>(P, x, ldx, n_cols, dtype, y, ldy, al, be, (hipStream_t)stream);
        else
            noalloc_matvec<float>(P, x, ldx, n_cols, dtype, y, ldy, al, be, (hipStream_t)stream);
    });
}

// Eager matvec for the solver: every Arnoldi step hands over a new vector,
// so graph mode (one captured graph per argument set) would capture anew at
// each step; this path never uses the graph.
xrl_status xrl_matvec_eager(const xrl_plan *P, const void *x, int64_t ldx, int32_t n_cols, int32_t dtype, void *y,
                            int64_t ldy, const xrl_epilogue *ep, void *stream)
{
    return guarded([&] {
        XRL_CHECK(P && x && y && P->assembled && n_cols >= 1 && n_cols <= P->max_cols, XRL_E_INVALID_ARG,
                  "gmres matvec: bad arguments");
        hipStream_t s = (hipStream_t)stream;
        const AllocStream alloc_scope(s);
        const double *al = ep ? ep->alpha : nullptr, *be = ep ? ep->beta : nullptr;
        upload_epilogue(P, n_cols, al, be, s);
        enqueue_matvec(P, x, ldx, n_cols, dtype, y, ldy, al != nullptr, be != nullptr, s, false);
    });
}

extern "C" xrl_status xrl_plan_set_graph(xrl_plan *P, int32_t on)
{
    return guarded([&] {
        XRL_CHECK(P, XRL_E_INVALID_ARG, "xrl_plan_set_graph: null plan");
        P->use_graph = on != 0;
        if (!P->use_graph && P->gexec) {
            XRL_HIP(hipGraphExecDestroy(P->gexec));
            P->gexec = nullptr;
        }
    });
}

// Kernel-shape autotuner: times every translation form that applies to the
// plan's precision on the caller's arguments and keeps the fastest.
extern "C" xrl_status xrl_plan_autotune(xrl_plan *P, const void *x, int64_t ldx, int32_t n_cols, int32_t dtype,
                                        void *y, int64_t ldy, int32_t reps, void *stream, xrl_tune_result *res)
{
    return guarded([&] {
        XRL_CHECK(P && x && y && res && reps >= 1, XRL_E_INVALID_ARG, "xrl_plan_autotune: bad arguments");
        XRL_CHECK(P->assembled, XRL_E_STATE, "xrl_plan_autotune: call xrl_nearfield_assemble first");
        XRL_CHECK(n_cols >= 1 && n_cols <= P->max_cols && ldx >= n_cols && ldy >= n_cols &&
                      (dtype == XRL_C64 || dtype == XRL_C128) && x != y,
                  XRL_E_INVALID_ARG, "xrl_plan_autotune: bad matvec arguments");
        hipStream_t s = (hipStream_t)stream;
        const AllocStream alloc_scope(s);
        *res = xrl_tune_result{};
        struct Cand {
            int engine, ts_kernel;
        };
        std::vector<Cand> cands;
        if (P->m2l_engine == XRL_M2L_VALU) {
            cands.push_back({XRL_M2L_VALU, P->ts_kernel});
        } else {
            // the offset-stationary form only while its per-pair scratch
            // holds the columns in at most two chunks
            const int64_t per_col = P->m2l.n_pairs * (int64_t)P->KP * (P->precision == XRL_PREC_FP64 ? 8 : 4);
            const int64_t budget = P->scratch_budget ? P->scratch_budget : int64_t(4) << 30;
            const int64_t cc = std::max<int64_t>(1, budget / std::max<int64_t>(1, per_col));
            if (cdiv(2 * (int64_t)n_cols, cc) <= 2) cands.push_back({XRL_M2L_MFMA_OS, 0});
            for (int k = 0; k < 3; ++k) cands.push_back({XRL_M2L_MFMA_TS, k});
        }
        hipEvent_t e0, e1;
        XRL_HIP(hipEventCreate(&e0));
        XRL_HIP(hipEventCreate(&e1));
        const bool prof = P->profiling, graph = P->use_graph;
        P->profiling = false;
        P->use_graph = false;
        double best = 1e300;
        Cand pick = cands[0];
        try {
            for (size_t i = 0; i < cands.size() && i < 8; ++i) {
                P->m2l_engine = cands[i].engine;
                P->ts_kernel = cands[i].ts_kernel;
                enqueue_matvec(P, x, ldx, n_cols, dtype, y, ldy, false, false, s);  // warm-up
                XRL_HIP(hipEventRecord(e0, s));
                for (int r = 0; r < reps; ++r) enqueue_matvec(P, x, ldx, n_cols, dtype, y, ldy, false, false, s);
                XRL_HIP(hipEventRecord(e1, s));
                XRL_HIP(hipEventSynchronize(e1));
                float ms = 0;
                XRL_HIP(hipEventElapsedTime(&ms, e0, e1));
                res->ms[i] = ms / reps;
                res->engine[i] = cands[i].engine;
                res->ts_kernel[i] = cands[i].ts_kernel;
                res->n_tried = (int32_t)(i + 1);
                if (ms / reps < best) {
                    best = ms / reps;
                    pick = cands[i];
                }
            }
        } catch (...) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            P->profiling = prof;
            P->use_graph = graph;
            throw;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        P->profiling = prof;
        P->use_graph = graph;
        P->m2l_engine = pick.engine;
        P->ts_kernel = pick.ts_kernel;
        res->best_p2p_form = P->p2p_form;
        if (P->precision != XRL_PREC_FP64 && n_cols > 8) {  // more than 16 real FP32 columns
            hipEvent_t f0, f1;
            XRL_HIP(hipEventCreate(&f0));
            XRL_HIP(hipEventCreate(&f1));
            double bp = 1e300;
            for (int f = 0; f < 3; ++f) {
                P->p2p_form = f;
                enqueue_matvec(P, x, ldx, n_cols, dtype, y, ldy, false, false, s);
                XRL_HIP(hipEventRecord(f0, s));
                for (int r = 0; r < reps; ++r) enqueue_matvec(P, x, ldx, n_cols, dtype, y, ldy, false, false, s);
                XRL_HIP(hipEventRecord(f1, s));
                XRL_HIP(hipEventSynchronize(f1));
                float ms = 0;
                XRL_HIP(hipEventElapsedTime(&ms, f0, f1));
                res->p2p_ms[f] = ms / reps;
                res->n_p2p_tried = f + 1;
                if (ms / reps < bp) {
                    bp = ms / reps;
                    res->best_p2p_form = f;
                }
            }
            (void)hipEventDestroy(f0);
            (void)hipEventDestroy(f1);
            P->p2p_form = res->best_p2p_form;
        }
        if (P->gexec) {  // a captured graph holds the old kernel shapes
            XRL_HIP(hipGraphExecDestroy(P->gexec));
            P->gexec = nullptr;
        }
        res->best_engine = pick.engine;
        res->best_ts_kernel = pick.ts_kernel;
        res->best_ms = best;
    });
}

// Self-test of the MFMA operand layout: D[16][16] = A[16][4] B[4][16] through
// the same 16x16x4 helper the M2L kernel uses (row-major host arrays).
template <typename T>
__global__ void k_mfma_probe(const T *A, const T *B, T *D)
{
    using VT = typename std::conditional<sizeof(T) == 4, f32x4, f64x4>::type;
    const int lane = threadIdx.x;
    const int i = lane & 15, k = lane >> 4;
    VT d = {0, 0, 0, 0};
    mfma_16x16x4<T>(A[i * 4 + k], B[k * 16 + i], d);
    for (int e = 0; e < 4; ++e) D[mfma_row<T>(k, e) * 16 + i] = d[e];
}

extern "C" xrl_status xrl_selftest_mfma(int32_t dtype, const void *A, const void *B, void *D)
{
    return guarded([&] {
        XRL_CHECK(A && B && D && (dtype == 4 || dtype == 8), XRL_E_INVALID_ARG, "xrl_selftest_mfma: bad arguments");
        const size_t e = dtype;
        DevBuf<char> dA(64 * e), dB(64 * e), dD(256 * e);
        XRL_HIP(hipMemcpy(dA.p, A, 64 * e, hipMemcpyHostToDevice));
        XRL_HIP(hipMemcpy(dB.p, B, 64 * e, hipMemcpyHostToDevice));
        if (dtype == 4)
            k_mfma_probe<float><<<1, 64>>>((const float *)dA.p, (const float *)dB.p, (float *)dD.p);
        else
            k_mfma_probe<double><<<1, 64>>>((const double *)dA.p, (const double *)dB.p, (double *)dD.p);
        XRL_HIP(hipGetLastError());
        XRL_HIP(hipMemcpy(D, dD.p, 256 * e, hipMemcpyDeviceToHost));
    });
}

// 16 blocks of 4x4x1: lane l = 4 b + r supplies A[b][r] and B[b][r] and
// receives D_b[i][r] in element i.
__global__ void k_mfma4_probe(const float *A, const float *B, float *D)
{
    const int l = threadIdx.x;
    f32x4 d = {0, 0, 0, 0};
    d = __builtin_amdgcn_mfma_f32_4x4x1f32(A[l], B[l], d, 0, 0, 0);
    for (int i = 0; i < 4; ++i) D[((l >> 2) * 4 + i) * 4 + (l & 3)] = d[i];
}

extern "C" xrl_status xrl_selftest_mfma_4x4(const float *A, const float *B, float *D)
{
    return guarded([&] {
        XRL_CHECK(A && B && D, XRL_E_INVALID_ARG, "xrl_selftest_mfma_4x4: bad arguments");
        DevBuf<float> dA(64), dB(64), dD(256);
        XRL_HIP(hipMemcpy(dA.p, A, 64 * sizeof(float), hipMemcpyHostToDevice));
        XRL_HIP(hipMemcpy(dB.p, B, 64 * sizeof(float), hipMemcpyHostToDevice));
        k_mfma4_probe<<<1, 64>>>(dA.p, dB.p, dD.p);
        XRL_HIP(hipGetLastError());
        XRL_HIP(hipMemcpy(D, dD.p, 256 * sizeof(float), hipMemcpyDeviceToHost));
    });
}

extern "C" xrl_status xrl_plan_set_profiling(xrl_plan *P, int32_t on)
{
    return guarded([&] {
        XRL_CHECK(P, XRL_E_INVALID_ARG, "xrl_plan_set_profiling: null plan");
        P->profiling = on != 0;
        P->prof_count = 0;
    });
}

extern "C" xrl_status xrl_plan_set_tuning(xrl_plan *P, int32_t key, int32_t value)
{
    return guarded([&] {
        XRL_CHECK(P, XRL_E_INVALID_ARG, "xrl_plan_set_tuning: null plan");
        switch (key) {
            case XRL_TUNE_TS_KERNEL:
                XRL_CHECK(value >= 0 && value <= 2, XRL_E_INVALID_ARG, "xrl_plan_set_tuning: kernel form must be 0..2");
                P->ts_kernel = value;
                break;
            case XRL_TUNE_P2P_FORM:
                XRL_CHECK(value >= 0 && value <= 2, XRL_E_INVALID_ARG, "xrl_plan_set_tuning: P2P form must be 0..2");
                P->p2p_form = value;
                break;
            case XRL_TUNE_TS_MIN_COLS:
                XRL_CHECK(value >= 1, XRL_E_INVALID_ARG, "xrl_plan_set_tuning: min columns must be >= 1");
                P->ts_min_cols = value;
                break;
            case XRL_TUNE_L2L_FORM:
                XRL_CHECK(value == 0 || value == 1, XRL_E_INVALID_ARG, "xrl_plan_set_tuning: L2L form must be 0 or 1");
                P->ps_l2l = value;
                break;
            case XRL_TUNE_LEAF_FORM:
                XRL_CHECK(value == 0 || value == 1, XRL_E_INVALID_ARG, "xrl_plan_set_tuning: leaf form must be 0 or 1");
                P->leaf_mfma = value;
                break;
            case XRL_TUNE_VALU_FORM:
                XRL_CHECK(value == 0 || value == 1, XRL_E_INVALID_ARG, "xrl_plan_set_tuning: vector-ALU form must be 0 or 1");
                P->valu_col = value;
                break;
            case XRL_TUNE_LEAF_L2L:
                XRL_CHECK(value == 0 || value == 1, XRL_E_INVALID_ARG, "xrl_plan_set_tuning: leaf L2L must be 0 or 1");
                P->leaf_l2l = value;
                break;
            case XRL_TUNE_M2M_FORM:
                XRL_CHECK(value >= 0 && value <= 2, XRL_E_INVALID_ARG, "xrl_plan_set_tuning: M2M form must be 0..2");
                P->tr_m2m = value;
                break;
            case XRL_TUNE_TS_ORDER:
                XRL_CHECK(value == 0 || value == 1, XRL_E_INVALID_ARG, "xrl_plan_set_tuning: order must be 0 or 1");
                P->ts_order = value;
                break;
            case XRL_TUNE_TS_NARROW_COLS:
                XRL_CHECK(value == 0 || value == 1, XRL_E_INVALID_ARG,
                          "xrl_plan_set_tuning: narrow columns must be 0 or 1");
                P->ts_narrow_cols = value;
                break;
            default: fail(XRL_E_INVALID_ARG, "xrl_plan_set_tuning: unknown key %d", key);
        }
        // a captured graph holds the old kernel forms: drop it, the next
        // graph-mode matvec captures the new ones
        if (P->gexec) {
            XRL_HIP(hipGraphExecDestroy(P->gexec));
            P->gexec = nullptr;
        }
    });
}

extern "C" xrl_status xrl_plan_get_phase_ms(const xrl_plan *P, double *ms)
{
    return guarded([&] {
        XRL_CHECK(P && ms, XRL_E_INVALID_ARG, "xrl_plan_get_phase_ms: null argument");
        for (int i = 0; i < XRL_N_PHASES; ++i) ms[i] = 0;
        const int64_t n = std::min<int64_t>(P->prof_count, xrl_plan::kProfRing);
        for (int64_t q = 0; q < n; ++q) {
            const auto &ev = P->prof_ev[(size_t)((P->prof_count - 1 - q) % xrl_plan::kProfRing)];
            XRL_HIP(hipEventSynchronize(ev[XRL_N_PHASES]));
            // public phase order: gather, P2P, P2M, M2M, M2L, L2L, L2P, scatter
            for (int i = 0; i < XRL_N_PHASES; ++i) {
                float t = 0;
                XRL_HIP(hipEventElapsedTime(&t, ev[i], ev[i + 1]));
                ms[i] += t / (double)n;
            }
        }
    });
}
