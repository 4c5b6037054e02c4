// Learned surrogate for near-singular panel pairs of the near field.
//
// A pair (target triangle, source triangle) is described by 18 features: the
// six vertices in a frame attached to the source (centroid at the origin,
// longest edge along +x, normal along +z, third vertex at y > 0), scaled by
// the source diameter, source vertices in that canonical order and target
// vertices sorted by x.  A multilayer perceptron 18 -> H -> H -> 2 with SiLU
// activations gives y; the surrogate outputs are
//     out0 = y0 / rho^4 = P_kl / P_kl^cheap - 1   (P^cheap: 3 x 3 conical Gauss
//            product; rho: target-centroid distance in source diameters)
//     out1 = y1 = log10 of the absolute error of out0,
// so P_kl = P^cheap (1 + out0) when out1 is below the bound and the features
// lie inside the training range; otherwise the pair falls back to quadrature.
//
// Training runs on the GPU with the kernels below (FP32 forward, backward,
// Adam); inference inside the assembly runs the three layers on BF16 MFMA
// (16x16x16, FP32 accumulation).
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "nfcommon.h"

namespace xrl {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef short s16x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ features
__device__ inline double tri_area2_d(const double *v)
{
    const double e1[3] = {v[3] - v[0], v[4] - v[1], v[5] - v[2]};
    const double e2[3] = {v[6] - v[0], v[7] - v[1], v[8] - v[2]};
    const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                 cz = e1[0] * e2[1] - e1[1] * e2[0];
    return sqrt(cx * cx + cy * cy + cz * cz);
}

// 3 x 3 conical Gauss on both triangles (81 kernel evaluations), FP64.
__device__ double cheap_value(const double *tv, const double *sv, const CheapRule &R)
{
    double py[9][3], pw[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double s = R.x[i], t = R.x[j];
            for (int d = 0; d < 3; ++d) py[3 * i + j][d] = sv[d] + s * (sv[3 + d] - sv[d]) + s * t * (sv[6 + d] - sv[3 + d]);
            pw[3 * i + j] = R.w[i] * R.w[j] * s;
        }
    double acc = 0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            const double s = R.x[i], t = R.x[j];
            double x[3];
            for (int d = 0; d < 3; ++d) x[d] = tv[d] + s * (tv[3 + d] - tv[d]) + s * t * (tv[6 + d] - tv[3 + d]);
            double inner = 0;
            for (int q = 0; q < 9; ++q) {
                const double dx = x[0] - py[q][0], dy = x[1] - py[q][1], dz = x[2] - py[q][2];
                inner += pw[q] / sqrt(dx * dx + dy * dy + dz * dz);
            }
            acc += R.w[i] * R.w[j] * s * inner;
        }
    return acc * tri_area2_d(tv) * tri_area2_d(sv);
}

__device__ void pair_features(const double *tv, const double *sv, float *f)
{
    // longest source edge a -> b, third vertex c
    int ia = 0;
    double best = -1;
    for (int e = 0; e < 3; ++e) {
        const double *p = sv + 3 * e, *q = sv + 3 * ((e + 1) % 3);
        const double l2 = (q[0] - p[0]) * (q[0] - p[0]) + (q[1] - p[1]) * (q[1] - p[1]) + (q[2] - p[2]) * (q[2] - p[2]);
        if (l2 > best) {
            best = l2;
            ia = e;
        }
    }
    const double *a = sv + 3 * ia, *b = sv + 3 * ((ia + 1) % 3), *c = sv + 3 * ((ia + 2) % 3);
    const double d = sqrt(best);
    // direction of the longest edge: the foot of the third vertex lies in its
    // first half (fixes the frame whatever the input vertex order)
    if ((c[0] - a[0]) * (b[0] - a[0]) + (c[1] - a[1]) * (b[1] - a[1]) + (c[2] - a[2]) * (b[2] - a[2]) > 0.5 * best) {
        const double *tmp = a;
        a = b;
        b = tmp;
    }
    double ex[3] = {(b[0] - a[0]) / d, (b[1] - a[1]) / d, (b[2] - a[2]) / d};
    const double ac[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double ez[3] = {ex[1] * ac[2] - ex[2] * ac[1], ex[2] * ac[0] - ex[0] * ac[2], ex[0] * ac[1] - ex[1] * ac[0]};
    const double nz = sqrt(ez[0] * ez[0] + ez[1] * ez[1] + ez[2] * ez[2]);
    for (int k = 0; k < 3; ++k) ez[k] /= nz;
    // e_y = e_z x e_x puts c at y > 0 by construction
    double ey[3] = {ez[1] * ex[2] - ez[2] * ex[1], ez[2] * ex[0] - ez[0] * ex[2], ez[0] * ex[1] - ez[1] * ex[0]};
    // centroid summed in the canonical vertex order (same rounding whatever
    // the input order)
    const double cen[3] = {(a[0] + b[0] + c[0]) / 3, (a[1] + b[1] + c[1]) / 3, (a[2] + b[2] + c[2]) / 3};
    auto map = [&](const double *p, float *o) {
        const double q[3] = {(p[0] - cen[0]) / d, (p[1] - cen[1]) / d, (p[2] - cen[2]) / d};
        o[0] = (float)(q[0] * ex[0] + q[1] * ex[1] + q[2] * ex[2]);
        o[1] = (float)(q[0] * ey[0] + q[1] * ey[1] + q[2] * ey[2]);
        o[2] = (float)(q[0] * ez[0] + q[1] * ez[1] + q[2] * ez[2]);
    };
    map(a, f + 0);
    map(b, f + 3);
    map(c, f + 6);
    float t[3][3];
    for (int i = 0; i < 3; ++i) map(tv + 3 * i, t[i]);
    int o0 = 0, o1 = 1, o2 = 2;  // sort target vertices
    // lexicographic (x, y, z) with a tolerance, so coincident coordinates
    // computed in a different order still tie
    auto less = [&](int i, int j) {
        for (int k = 0; k < 3; ++k) {
            if (t[i][k] < t[j][k] - 1e-6f) return true;
            if (t[i][k] > t[j][k] + 1e-6f) return false;
        }
        return false;
    };
    if (less(o1, o0)) { int s = o0; o0 = o1; o1 = s; }
    if (less(o2, o1)) { int s = o1; o1 = o2; o2 = s; }
    if (less(o1, o0)) { int s = o0; o0 = o1; o1 = s; }
    const int ord[3] = {o0, o1, o2};
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) f[9 + 3 * i + k] = t[ord[i]][k];
}

__global__ void k_pair_features(const double *__restrict__ tk, const double *__restrict__ tl, int64_t n, CheapRule R,
                                float *__restrict__ feat, double *__restrict__ cheap)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    double tv[9], sv[9];
    for (int q = 0; q < 9; ++q) {
        tv[q] = tk[9 * i + q];
        sv[q] = tl[9 * i + q];
    }
    pair_features(tv, sv, feat + 18 * i);
    if (cheap) cheap[i] = cheap_value(tv, sv, R);
}

// ------------------------------------------------------------------ FP32 MLP kernels
// C[M][N] = op(A)[M][K] op(B)[K][N] (+ beta C), row-major storage, op = optional
// transpose; 16 x 16 output tile per workgroup, K in steps of 16 through LDS.
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const float *__restrict__ A, int lda, int ta,
                                              const float *__restrict__ B, int ldb, int tb, float *__restrict__ C,
                                              int ldc, float beta)
{
    __shared__ float sa[16][17], sb[16][17];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int row = blockIdx.y * 16 + ty, col = blockIdx.x * 16 + tx;
    float acc = 0;
    for (int k0 = 0; k0 < K; k0 += 16) {
        const int ka = k0 + tx, kb = k0 + ty;
        const int ar = blockIdx.y * 16 + ty, bc = blockIdx.x * 16 + tx;
        sa[ty][tx] = (ar < M && ka < K) ? (ta ? A[(int64_t)ka * lda + ar] : A[(int64_t)ar * lda + ka]) : 0.f;
        sb[ty][tx] = (kb < K && bc < N) ? (tb ? B[(int64_t)bc * ldb + kb] : B[(int64_t)kb * ldb + bc]) : 0.f;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 16; ++k) acc += sa[ty][k] * sb[k][tx];
        __syncthreads();
    }
    if (row < M && col < N) {
        float *c = C + (int64_t)row * ldc + col;
        *c = beta != 0.f ? beta * *c + acc : acc;
    }
}

__device__ inline float sigm(float z) { return 1.f / (1.f + expf(-z)); }

// Fixed output scaling of the first output: rho^-4, rho = distance of the
// target centroid from the source centroid in source diameters (features
// 9..17 are the target vertices in that frame).  The cheap rule's relative
// error falls roughly as this power, so the network learns an O(1) quantity.
__device__ inline float out_scale(const float *f)
{
    const float cx = (f[9] + f[12] + f[15]) * (1.f / 3.f);
    const float cy = (f[10] + f[13] + f[16]) * (1.f / 3.f);
    const float cz = (f[11] + f[14] + f[17]) * (1.f / 3.f);
    const float r2 = cx * cx + cy * cy + cz * cz;
    return 1.f / (r2 * r2);
}

// Y[i][0] *= out_scale(X[i])
__global__ void k_scale_out(float *__restrict__ Y, const float *__restrict__ X, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) Y[2 * i] *= out_scale(X + 18 * i);
}

// Z += bias (per column); H = SiLU(Z)
__global__ void k_bias_silu(float *__restrict__ Z, float *__restrict__ H, const float *__restrict__ b, int64_t rows,
                            int cols, int act)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= rows * cols) return;
    const float z = Z[i] + b[i % cols];
    Z[i] = z;
    if (H) H[i] = act ? z * sigm(z) : z;
}

// dZ = dH * SiLU'(Z)
__global__ void k_silu_back(const float *__restrict__ Z, float *__restrict__ dH, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float s = sigm(Z[i]);
    dH[i] *= s * (1.f + Z[i] * (1.f - s));
}

// out[c] = sum_r X[r][c], one workgroup per column, fixed-order tree
__global__ __launch_bounds__(256) void k_colsum(const float *__restrict__ X, int64_t rows, int cols, float *__restrict__ out)
{
    __shared__ float s[256];
    const int c = blockIdx.x;
    float a = 0;
    for (int64_t r = threadIdx.x; r < rows; r += 256) a += X[r * cols + c];
    s[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) s[threadIdx.x] += s[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = s[0];
}

struct LossArgs {
    float lam;     // weight of the calibration term
    float mu, sig; // log10-error target scaling: (log10(err) - mu) / sig
    float scale;   // raw out0 = scale * y0
};

// Y[B][2] -> dY, per-sample loss terms into part[B][2]; the calibration
// target is the log10 error of the scaled first output, scale * out_scale * y0
__global__ void k_loss(const float *__restrict__ Y, const float *__restrict__ t, const float *__restrict__ X, int64_t B,
                       LossArgs a, float *__restrict__ dY, float *__restrict__ part)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= B) return;
    const float e0 = Y[2 * i] - t[i];
    const float err = fabsf(e0) * a.scale * out_scale(X + 18 * i);
    const float lt = (log10f(err + 1e-12f) - a.mu) / a.sig;  // detached target
    const float e1 = Y[2 * i + 1] - lt;
    dY[2 * i] = 2.f * e0 / (float)B;
    dY[2 * i + 1] = 2.f * a.lam * e1 / (float)B;
    part[2 * i] = e0 * e0;
    part[2 * i + 1] = e1 * e1;
}

__global__ void k_gather_rows(const float *__restrict__ X, const float *__restrict__ t, const int32_t *__restrict__ idx,
                              int64_t B, float *__restrict__ Xb, float *__restrict__ tb)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= B) return;
    const int64_t j = idx[i];
    for (int k = 0; k < 18; ++k) Xb[18 * i + k] = X[18 * j + k];
    tb[i] = t[j];
}

__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int64_t n, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    m[i] = b1 * m[i] + (1.f - b1) * gi;
    v[i] = b2 * v[i] + (1.f - b2) * gi * gi;
    p[i] -= lr * (m[i] / c1) / (sqrtf(v[i] / c2) + eps);
}

struct MlpView {
    int H;
    float *w1, *b1, *w2, *b2, *w3, *b3;
};
inline MlpView mlp_view(float *w, int H)
{
    MlpView v;
    v.H = H;
    v.w1 = w;
    v.b1 = v.w1 + 18 * H;
    v.w2 = v.b1 + H;
    v.b2 = v.w2 + H * H;
    v.w3 = v.b2 + H;
    v.b3 = v.w3 + 2 * H;
    return v;
}
inline int64_t mlp_size(int H) { return (int64_t)H * H + 22 * (int64_t)H + 2; }

struct MlpWork {
    DevBuf<float> Z1, H1, Z2, H2, Y, dY, dH2, dH1, part;
    void ensure(int64_t B, int H)
    {
        if (Z1.n < (size_t)(B * H)) {
            Z1.alloc(B * H);
            H1.alloc(B * H);
            Z2.alloc(B * H);
            H2.alloc(B * H);
            dH2.alloc(B * H);
            dH1.alloc(B * H);
        }
        if (Y.n < (size_t)(2 * B)) {
            Y.alloc(2 * B);
            dY.alloc(2 * B);
            part.alloc(2 * B);
        }
    }
};

static void gemm(hipStream_t s, int M, int N, int K, const float *A, int lda, int ta, const float *B, int ldb, int tb,
                 float *C, int ldc, float beta = 0.f)
{
    dim3 grid((unsigned)cdiv(N, 16), (unsigned)cdiv(M, 16));
    k_gemm<<<grid, 256, 0, s>>>(M, N, K, A, lda, ta, B, ldb, tb, C, ldc, beta);
    XRL_HIP(hipGetLastError());
}

static void mlp_forward(hipStream_t s, MlpView w, const float *X, int64_t B, MlpWork &k)
{
    const int H = w.H;
    gemm(s, (int)B, H, 18, X, 18, 0, w.w1, 18, 1, k.Z1.p, H);
    k_bias_silu<<<cdiv(B * H, 256), 256, 0, s>>>(k.Z1.p, k.H1.p, w.b1, B, H, 1);
    gemm(s, (int)B, H, H, k.H1.p, H, 0, w.w2, H, 1, k.Z2.p, H);
    k_bias_silu<<<cdiv(B * H, 256), 256, 0, s>>>(k.Z2.p, k.H2.p, w.b2, B, H, 1);
    gemm(s, (int)B, 2, H, k.H2.p, H, 0, w.w3, H, 1, k.Y.p, 2);
    k_bias_silu<<<cdiv(B * 2, 256), 256, 0, s>>>(k.Y.p, nullptr, w.b3, B, 2, 0);
    XRL_HIP(hipGetLastError());
}

// loss and gradient (packed like the weights) of one batch
static void mlp_backward(hipStream_t s, MlpView w, MlpView g, const float *X, const float *t, int64_t B, LossArgs la,
                         MlpWork &k)
{
    const int H = w.H;
    k_loss<<<cdiv(B, 256), 256, 0, s>>>(k.Y.p, t, X, B, la, k.dY.p, k.part.p);
    gemm(s, 2, H, (int)B, k.dY.p, 2, 1, k.H2.p, H, 0, g.w3, H);
    k_colsum<<<2, 256, 0, s>>>(k.dY.p, B, 2, g.b3);
    gemm(s, (int)B, H, 2, k.dY.p, 2, 0, w.w3, H, 0, k.dH2.p, H);
    k_silu_back<<<cdiv(B * H, 256), 256, 0, s>>>(k.Z2.p, k.dH2.p, B * H);
    gemm(s, H, H, (int)B, k.dH2.p, H, 1, k.H1.p, H, 0, g.w2, H);
    k_colsum<<<H, 256, 0, s>>>(k.dH2.p, B, H, g.b2);
    gemm(s, (int)B, H, H, k.dH2.p, H, 0, w.w2, H, 0, k.dH1.p, H);
    k_silu_back<<<cdiv(B * H, 256), 256, 0, s>>>(k.Z1.p, k.dH1.p, B * H);
    gemm(s, H, 18, (int)B, k.dH1.p, H, 1, X, 18, 0, g.w1, 18);
    k_colsum<<<H, 256, 0, s>>>(k.dH1.p, B, H, g.b1);
    XRL_HIP(hipGetLastError());
}

// ------------------------------------------------------------------ BF16 MFMA inference
__device__ inline short f2bf(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7fffu + ((u >> 16) & 1u);  // round to nearest even
    return (short)(u >> 16);
}

// Weights prepared for inference: bf16 [H][32] (W1, k padded), [H][H] (W2),
// [16][H] (W3, rows padded), FP32 biases.
struct MlpBf16 {
    int H;
    const short *w1, *w2, *w3;
    const float *b1, *b2, *b3;
};

// One wave per 16 samples.  16x16x16 bf16 MFMA operand layout: A[i][k] at
// lane i + 16 (k / 4), element k % 4; B[k][j] at lane j + 16 (k / 4),
// element k % 4; D as the f32 16x16x4 (row 4 q + e, column lane % 16).
template <int H>
__global__ __launch_bounds__(256) void k_mlp_infer(MlpBf16 w, const float *__restrict__ X, int64_t n,
                                                   float *__restrict__ out)
{
    // LDS rows padded so that the 16 rows a wave reads at once start in
    // different banks: W1 rows 40 shorts (20 words apart), W2, W3 and the
    // hidden layer H + 8 shorts (H/2 + 4 words apart)
    constexpr int S1 = 40, SH = H + 8;
    extern __shared__ unsigned char smem_raw[];
    short *sw1 = reinterpret_cast<short *>(smem_raw);  // [H][S1]
    short *sw2 = sw1 + H * S1;                          // [H][SH]
    short *sw3 = sw2 + H * SH;                          // [16][SH]
    short *sh = sw3 + 16 * SH;                          // per wave [16][SH]
    for (int i = threadIdx.x; i < H * 32; i += 256) sw1[(i / 32) * S1 + i % 32] = w.w1[i];
    for (int i = threadIdx.x; i < H * H; i += 256) sw2[(i / H) * SH + i % H] = w.w2[i];
    for (int i = threadIdx.x; i < 16 * H; i += 256) sw3[(i / H) * SH + i % H] = w.w3[i];
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, kq = lane >> 4;
    short *hbuf = sh + wave * 16 * SH;
    const int64_t nchunks = (n + 15) / 16;
    // SiLU on the hardware exponential and reciprocal: its result is rounded
    // to BF16 at once, far coarser than their error
    auto silu_bf = [](float z) { return f2bf(z * __builtin_amdgcn_rcpf(1.f + __expf(-z))); };
    // each wave works on its own 16 samples and its own slice of LDS; a
    // wave's LDS accesses complete in order, so only a wave barrier (no
    // instruction, a fence for the compiler) separates writing the hidden
    // layer and reading it back across lanes
    for (int64_t base = (int64_t)blockIdx.x * 4; base < nchunks; base += (int64_t)gridDim.x * 4) {
        const int64_t ch = base + wave;
        const bool active = ch < nchunks;
        const int64_t s0 = ch * 16;
        // layer 1: A = X[16][32] (features padded with zeros)
        s16x4 ax[2];
        for (int ks = 0; ks < 2; ++ks)
            for (int e = 0; e < 4; ++e) {
                const int k = 16 * ks + 4 * kq + e;
                const int64_t sidx = s0 + li;
                ax[ks][e] = f2bf((active && k < 18 && sidx < n) ? X[sidx * 18 + k] : 0.f);
            }
        for (int ct = 0; ct < H / 16; ++ct) {
            f32x4 d = {0, 0, 0, 0};
            for (int ks = 0; ks < 2; ++ks) {
                const s16x4 b = *reinterpret_cast<const s16x4 *>(sw1 + (16 * ct + li) * S1 + 16 * ks + 4 * kq);
                d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ax[ks], b, d, 0, 0, 0);
            }
            for (int e = 0; e < 4; ++e) {
                const int r = 4 * kq + e, c = 16 * ct + li;
                hbuf[r * SH + c] = silu_bf(d[e] + w.b1[c]);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // layer 2
        f32x4 d2[H / 16];
        for (int ct = 0; ct < H / 16; ++ct) d2[ct] = f32x4{0, 0, 0, 0};
        for (int ks = 0; ks < H / 16; ++ks) {
            const s16x4 a = *reinterpret_cast<const s16x4 *>(hbuf + li * SH + 16 * ks + 4 * kq);
            for (int ct = 0; ct < H / 16; ++ct) {
                const s16x4 b = *reinterpret_cast<const s16x4 *>(sw2 + (16 * ct + li) * SH + 16 * ks + 4 * kq);
                d2[ct] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, d2[ct], 0, 0, 0);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int ct = 0; ct < H / 16; ++ct)
            for (int e = 0; e < 4; ++e) {
                const int r = 4 * kq + e, c = 16 * ct + li;
                hbuf[r * SH + c] = silu_bf(d2[ct][e] + w.b2[c]);
            }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // layer 3 (2 outputs, rows of W3 padded to 16)
        f32x4 d3 = {0, 0, 0, 0};
        for (int ks = 0; ks < H / 16; ++ks) {
            const s16x4 a = *reinterpret_cast<const s16x4 *>(hbuf + li * SH + 16 * ks + 4 * kq);
            const s16x4 b = *reinterpret_cast<const s16x4 *>(sw3 + li * SH + 16 * ks + 4 * kq);
            d3 = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, d3, 0, 0, 0);
        }
        if (active && li < 2)
            for (int e = 0; e < 4; ++e) {
                const int64_t sidx = s0 + 4 * kq + e;
                if (sidx < n) out[2 * sidx + li] = (d3[e] + w.b3[li]) * (li == 0 ? out_scale(X + sidx * 18) : 1.f);
            }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

__global__ void k_to_bf16_pad(const float *__restrict__ src, int rows, int cols, int rows_p, int cols_p,
                              short *__restrict__ dst)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows_p * cols_p) return;
    const int r = i / cols_p, c = i - r * cols_p;
    dst[i] = (r < rows && c < cols) ? f2bf(src[r * cols + c]) : (short)0;
}

static MlpBf16 bf16_view(const MlpDevice &m)
{
    MlpView v = mlp_view(const_cast<float *>(m.w32.p), m.H);
    return MlpBf16{m.H, m.w1.p, m.w2.p, m.w3.p, v.b1, v.b2, v.b3};
}

static void mlp_prepare(MlpDevice &m, const float *w_packed_dev, int H, hipStream_t s)
{
    m.H = H;
    m.w32.alloc(mlp_size(H));
    XRL_HIP(hipMemcpyAsync(m.w32.p, w_packed_dev, m.w32.bytes(), hipMemcpyDeviceToDevice, s));
    MlpView v = mlp_view(m.w32.p, H);
    m.w1.alloc((size_t)H * 32);
    m.w2.alloc((size_t)H * H);
    m.w3.alloc((size_t)16 * H);
    k_to_bf16_pad<<<cdiv(H * 32, 256), 256, 0, s>>>(v.w1, H, 18, H, 32, m.w1.p);
    k_to_bf16_pad<<<cdiv(H * H, 256), 256, 0, s>>>(v.w2, H, H, H, H, m.w2.p);
    k_to_bf16_pad<<<cdiv(16 * H, 256), 256, 0, s>>>(v.w3, 2, H, 16, H, m.w3.p);
    XRL_HIP(hipGetLastError());
}

void mlp_infer(const MlpDevice &m, const float *X, int64_t n, float *out, hipStream_t s)
{
    XRL_CHECK(m.H == 128 || m.H == 64, XRL_E_UNSUPPORTED, "surrogate: hidden width must be 64 or 128");
    if (n == 0) return;
    const size_t sm = (size_t)(m.H * 40 + (m.H + 16 + 4 * 16) * (m.H + 8)) * sizeof(short);
    const unsigned grid = (unsigned)std::min<int64_t>(cdiv(cdiv(n, 16), 4), 4096);
    if (m.H == 128)
        k_mlp_infer<128><<<grid, 256, sm, s>>>(bf16_view(m), X, n, out);
    else
        k_mlp_infer<64><<<grid, 256, sm, s>>>(bf16_view(m), X, n, out);
    XRL_HIP(hipGetLastError());
}

void mlp_prepare_host(MlpDevice &m, const xrl_mlp *h, hipStream_t s)
{
    const int H = h->hidden;
    std::vector<float> packed(mlp_size(H));
    size_t o = 0;
    auto put = [&](const float *p, size_t n) {
        std::memcpy(packed.data() + o, p, n * sizeof(float));
        o += n;
    };
    put(h->w1, 18 * (size_t)H);
    put(h->b1, H);
    put(h->w2, (size_t)H * H);
    put(h->b2, H);
    put(h->w3, 2 * (size_t)H);
    put(h->b3, 2);
    DevBuf<float> tmp;
    tmp.upload(packed, s);
    mlp_prepare(m, tmp.p, H, s);
    XRL_HIP(hipStreamSynchronize(s));
}

__global__ void k_ns_features(NFArgs a, int64_t base, int64_t n, CheapRule R, float *__restrict__ feat,
                              double *__restrict__ cheap)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t pos = base + i;
    const int32_t k = a.work_meta[2 * pos], l = a.work_meta[2 * pos + 1];
    double tv[9], sv[9];
    for (int q = 0; q < 9; ++q) {
        tv[q] = a.pv[9 * (int64_t)k + q] - a.cen[3 * k + q % 3];
        sv[q] = a.pv[9 * (int64_t)l + q] - a.cen[3 * k + q % 3];
    }
    pair_features(tv, sv, feat + 18 * i);
    cheap[i] = cheap_value(tv, sv, R);
}

void ns_features(const NFArgs &a, int64_t base, int64_t n, float *feat, double *cheap, hipStream_t s)
{
    if (n == 0) return;
    CheapRule R;
    gauss_legendre01(3, R.x, R.w);
    k_ns_features<<<cdiv(n, 128), 128, 0, s>>>(a, base, n, R, feat, cheap);
    XRL_HIP(hipGetLastError());
}

}  // namespace xrl

using namespace xrl;

extern "C" xrl_status xrl_surrogate_features(const double *tri_k, const double *tri_l, int64_t n, float *feat,
                                             double *cheap, void *stream)
{
    return guarded([&] {
        XRL_CHECK(tri_k && tri_l && feat && n >= 0, XRL_E_INVALID_ARG, "xrl_surrogate_features: bad arguments");
        CheapRule R;
        gauss_legendre01(3, R.x, R.w);
        if (n > 0) {
            k_pair_features<<<cdiv(n, 128), 128, 0, (hipStream_t)stream>>>(tri_k, tri_l, n, R, feat, cheap);
            XRL_HIP(hipGetLastError());
        }
    });
}

__global__ void k_bf16_probe(const float *A, const float *B, float *D)
{
    const int lane = threadIdx.x, li = lane & 15, kq = lane >> 4;
    s16x4 a, b;
    for (int e = 0; e < 4; ++e) {
        a[e] = f2bf(A[li * 16 + 4 * kq + e]);
        b[e] = f2bf(B[(4 * kq + e) * 16 + li]);
    }
    f32x4 d = {0, 0, 0, 0};
    d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, d, 0, 0, 0);
    for (int e = 0; e < 4; ++e) D[(4 * kq + e) * 16 + li] = d[e];
}

extern "C" xrl_status xrl_selftest_mfma_bf16(const float *A, const float *B, float *D)
{
    return guarded([&] {
        XRL_CHECK(A && B && D, XRL_E_INVALID_ARG, "xrl_selftest_mfma_bf16: null argument");
        DevBuf<float> dA(256), dB(256), dD(256);
        XRL_HIP(hipMemcpy(dA.p, A, 1024, hipMemcpyHostToDevice));
        XRL_HIP(hipMemcpy(dB.p, B, 1024, hipMemcpyHostToDevice));
        k_bf16_probe<<<1, 64>>>(dA.p, dB.p, dD.p);
        XRL_HIP(hipGetLastError());
        XRL_HIP(hipMemcpy(D, dD.p, 1024, hipMemcpyDeviceToHost));
    });
}

extern "C" xrl_status xrl_mlp_loss_grad(const float *w, int32_t hidden, const float *X, const float *t, int64_t n,
                                        const float *loss_args, float *loss, float *grad, void *stream)
{
    return guarded([&] {
        XRL_CHECK(w && X && t && n >= 1 && hidden >= 1 && loss_args && loss && grad, XRL_E_INVALID_ARG,
                  "xrl_mlp_loss_grad: bad arguments");
        hipStream_t s = (hipStream_t)stream;
        const AllocStream alloc_scope(s);
        MlpWork k;
        k.ensure(n, hidden);
        MlpView wv = mlp_view(const_cast<float *>(w), hidden), gv = mlp_view(grad, hidden);
        LossArgs la{loss_args[0], loss_args[1], loss_args[2], loss_args[3]};
        mlp_forward(s, wv, X, n, k);
        mlp_backward(s, wv, gv, X, t, n, la, k);
        auto part = k.part.download(s, 2 * n);
        double l0 = 0, l1 = 0;
        for (int64_t i = 0; i < n; ++i) {
            l0 += part[2 * i];
            l1 += part[2 * i + 1];
        }
        loss[0] = (float)(l0 / n);
        loss[1] = (float)(l1 / n);
    });
}

extern "C" xrl_status xrl_mlp_forward(const float *w, int32_t hidden, const float *X, int64_t n, int32_t bf16,
                                      float *out, void *stream)
{
    return guarded([&] {
        XRL_CHECK(w && X && out && n >= 0 && hidden >= 1, XRL_E_INVALID_ARG, "xrl_mlp_forward: bad arguments");
        hipStream_t s = (hipStream_t)stream;
        const AllocStream alloc_scope(s);
        if (n == 0) return;
        if (bf16) {
            MlpDevice m;
            mlp_prepare(m, w, hidden, s);
            mlp_infer(m, X, n, out, s);
            XRL_HIP(hipStreamSynchronize(s));
        } else {
            MlpWork k;
            k.ensure(n, hidden);
            mlp_forward(s, mlp_view(const_cast<float *>(w), hidden), X, n, k);
            k_scale_out<<<cdiv(n, 256), 256, 0, s>>>(k.Y.p, X, n);
            XRL_HIP(hipMemcpyAsync(out, k.Y.p, 2 * n * sizeof(float), hipMemcpyDeviceToDevice, s));
            XRL_HIP(hipStreamSynchronize(s));
        }
    });
}

extern "C" xrl_status xrl_mlp_train(const float *X, const float *t, int64_t n, const xrl_mlp_train_opts *o, float *w,
                                    float *loss_hist, void *stream)
{
    return guarded([&] {
        XRL_CHECK(X && t && o && w && n >= 1 && o->hidden >= 1 && o->batch >= 1 && o->epochs >= 1, XRL_E_INVALID_ARG,
                  "xrl_mlp_train: bad arguments");
        hipStream_t s = (hipStream_t)stream;
        const AllocStream alloc_scope(s);
        const int H = o->hidden;
        const int64_t B = std::min<int64_t>(o->batch, n);
        const int64_t P = mlp_size(H);
        DevBuf<float> g(P), m(P), v(P), Xb(18 * B), tb(B);
        XRL_HIP(hipMemsetAsync(m.p, 0, m.bytes(), s));
        XRL_HIP(hipMemsetAsync(v.p, 0, v.bytes(), s));
        MlpWork k;
        k.ensure(B, H);
        MlpView wv = mlp_view(w, H), gv = mlp_view(g.p, H);
        LossArgs la{o->calib_weight, o->log_mu, o->log_sigma, o->target_scale};
        std::mt19937_64 rng(o->seed);
        std::vector<int32_t> perm(n);
        DevBuf<int32_t> dperm(n);
        int64_t step = 0;
        const int64_t nb = n / B;
        DevBuf<float> ep_loss(2 * std::max<int64_t>(nb, 1));
        for (int ep = 0; ep < o->epochs; ++ep) {
            for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
            std::shuffle(perm.begin(), perm.end(), rng);
            dperm.upload(perm, s);
            const float lr = o->lr * (o->lr_decay > 0 ? std::pow(o->lr_decay, (float)ep) : 1.f);
            for (int64_t bi = 0; bi < nb; ++bi) {
                k_gather_rows<<<cdiv(B, 256), 256, 0, s>>>(X, t, dperm.p + bi * B, B, Xb.p, tb.p);
                mlp_forward(s, wv, Xb.p, B, k);
                mlp_backward(s, wv, gv, Xb.p, tb.p, B, la, k);
                k_colsum<<<2, 256, 0, s>>>(k.part.p, B, 2, ep_loss.p + 2 * bi);
                ++step;
                const float c1 = 1.f - std::pow(o->beta1, (float)step), c2 = 1.f - std::pow(o->beta2, (float)step);
                k_adam<<<cdiv(P, 256), 256, 0, s>>>(w, g.p, m.p, v.p, P, lr, o->beta1, o->beta2, o->eps, c1, c2);
                XRL_HIP(hipGetLastError());
            }
            auto hl = ep_loss.download(s, 2 * nb);
            double l0 = 0;
            for (int64_t bi = 0; bi < nb; ++bi) l0 += hl[2 * bi];
            l0 /= (double)nb * (double)B;
            if (loss_hist) loss_hist[ep] = (float)l0;
        }
        XRL_HIP(hipStreamSynchronize(s));
    });
}
