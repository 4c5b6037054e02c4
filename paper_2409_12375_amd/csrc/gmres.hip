// Restarted GMRES for (beta_c diag(A) + alpha_c P) x_c = b_c over several
// right-hand sides that share every FMM matvec (Sec. III: multiple
// right-hand-side GMRES, restart 50, relative residual 1e-4 / 1e-6).
// Arnoldi vectors, the Gram-Schmidt projections (classical, applied twice)
// and the Givens least-squares update are FP64 whatever the plan's precision.
#include <cmath>
#include <complex>
#include <cstring>
#include <functional>
#include <vector>

#include "common.h"

namespace xrl {

using cplx = std::complex<double>;

// partial[(i * nb + block) * R + c] = sum_n conj(V_i[n][c]) w[n][c] over this
// block's share of n.  V_i = V + i * N * R (complex128 interleaved).
__global__ __launch_bounds__(256) void k_dots(const double *__restrict__ V, int64_t N, int R,
                                              const double *__restrict__ w, double *__restrict__ partial)
{
    __shared__ double sr[256], si[256];
    const int i = blockIdx.y, nb = gridDim.x;
    const double *Vi = V + 2 * (int64_t)i * N * R;
    for (int c = 0; c < R; ++c) {
        double ar = 0, ai = 0;
        for (int64_t n = blockIdx.x * 256 + threadIdx.x; n < N; n += (int64_t)nb * 256) {
            const double vr = Vi[2 * (n * R + c)], vi = Vi[2 * (n * R + c) + 1];
            const double xr = w[2 * (n * R + c)], xi = w[2 * (n * R + c) + 1];
            ar += vr * xr + vi * xi;
            ai += vr * xi - vi * xr;
        }
        sr[threadIdx.x] = ar;
        si[threadIdx.x] = ai;
        __syncthreads();
        for (int s = 128; s > 0; s >>= 1) {
            if ((int)threadIdx.x < s) {
                sr[threadIdx.x] += sr[threadIdx.x + s];
                si[threadIdx.x] += si[threadIdx.x + s];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            partial[2 * (((int64_t)i * nb + blockIdx.x) * R + c)] = sr[0];
            partial[2 * (((int64_t)i * nb + blockIdx.x) * R + c) + 1] = si[0];
        }
        __syncthreads();
    }
}

// w[n][c] -= sum_{i<m} h[i][c] V_i[n][c]
__global__ void k_project(const double *__restrict__ V, int64_t N, int R, int m, const double *__restrict__ h,
                          double *__restrict__ w)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= N * R) return;
    const int c = (int)(e % R);
    double ar = w[2 * e], ai = w[2 * e + 1];
    for (int i = 0; i < m; ++i) {
        const double hr = h[2 * (i * R + c)], hi = h[2 * (i * R + c) + 1];
        const double vr = V[2 * ((int64_t)i * N * R + e)], vi = V[2 * ((int64_t)i * N * R + e) + 1];
        ar -= hr * vr - hi * vi;
        ai -= hr * vi + hi * vr;
    }
    w[2 * e] = ar;
    w[2 * e + 1] = ai;
}

// out[n][c] = s_c * in[n][c] (s real per column); out may alias in.
__global__ void k_scale_cols(const double *__restrict__ in, int64_t N, int R, const double *__restrict__ s,
                             double *__restrict__ out)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= N * R) return;
    const double f = s[e % R];
    out[2 * e] = f * in[2 * e];
    out[2 * e + 1] = f * in[2 * e + 1];
}

// out = a - b
__global__ void k_sub(const double *__restrict__ a, const double *__restrict__ b, int64_t n, double *__restrict__ out)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < n) out[e] = a[e] - b[e];
}

// Widen / narrow complex64 <-> complex128 (interleaved, n complex values).
__global__ void k_widen(const float *__restrict__ in, int64_t n, double *__restrict__ out)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < 2 * n) out[e] = (double)in[e];
}
__global__ void k_narrow(const double *__restrict__ in, int64_t n, float *__restrict__ out)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e < 2 * n) out[e] = (float)in[e];
}

}  // namespace xrl

using namespace xrl;

// Eager matvec of the operator (fmm.hip): never replays a captured graph.
xrl_status xrl_matvec_eager(const xrl_plan *P, const void *x, int64_t ldx, int32_t n_cols, int32_t dtype, void *y,
                            int64_t ldy, const xrl_epilogue *ep, void *stream);

namespace {

struct Solver {
    std::function<void(const double *, double *)> apply;  // y = A x on [N][R] complex128
    int64_t N;
    int R;
    hipStream_t s;
    int nb;
    DevBuf<double> partial, hdev, sdev;

    // dots[i][c] = <V_i, w>_c for i < m
    std::vector<cplx> dots(const double *V, int m, const double *w)
    {
        if (partial.n < (size_t)(2 * m * nb * R)) partial.alloc(2 * (size_t)m * nb * R);
        k_dots<<<dim3(nb, m), 256, 0, s>>>(V, N, R, w, partial.p);
        XRL_HIP(hipGetLastError());
        auto h = partial.download(s, 2 * (size_t)m * nb * R);
        std::vector<cplx> out((size_t)m * R, 0.0);
        for (int i = 0; i < m; ++i)
            for (int b = 0; b < nb; ++b)
                for (int c = 0; c < R; ++c)
                    out[(size_t)i * R + c] += cplx(h[2 * (((size_t)i * nb + b) * R + c)], h[2 * (((size_t)i * nb + b) * R + c) + 1]);
        return out;
    }
    void project(const double *V, int m, const std::vector<cplx> &h, double *w)
    {
        std::vector<double> hh(2 * (size_t)m * R);
        for (size_t i = 0; i < (size_t)m * R; ++i) {
            hh[2 * i] = h[i].real();
            hh[2 * i + 1] = h[i].imag();
        }
        hdev.upload(hh, s);
        k_project<<<cdiv(N * R, 256), 256, 0, s>>>(V, N, R, m, hdev.p, w);
        XRL_HIP(hipGetLastError());
    }
    void scale(const double *in, const std::vector<double> &f, double *out)
    {
        sdev.upload(f, s);
        k_scale_cols<<<cdiv(N * R, 256), 256, 0, s>>>(in, N, R, sdev.p, out);
        XRL_HIP(hipGetLastError());
    }
    std::vector<double> norms(const double *w)
    {
        auto d = dots(w, 1, w);
        std::vector<double> n(R);
        for (int c = 0; c < R; ++c) n[c] = std::sqrt(std::max(0.0, d[c].real()));
        return n;
    }
};

}  // namespace

namespace xrl {

// Restarted GMRES on R systems of length N that share every application of
// the operator: b, x device [N][R] complex128 (x: initial guess in, solution
// out).  Classical Gram-Schmidt applied twice and Givens rotations, all in
// FP64.  Returns the number of right-hand sides that reached rtol.
int gmres_core(const std::function<void(const double *, double *)> &apply, int64_t N, int R, const double *Bv,
               double *X, int restart, double rtol, int max_iter, hipStream_t stream, xrl_gmres_stats *stats)
{
    Solver S;
    S.apply = apply;
    S.N = N;
    S.R = R;
    S.s = stream;
    S.nb = (int)std::max<int64_t>(1, std::min<int64_t>(64, cdiv(S.N, 256)));
    const int64_t NR2 = 2 * N * R;
    const int m = restart;
    DevBuf<double> V((size_t)(m + 1) * NR2), w(NR2), r(NR2);
    std::vector<double> bnorm = S.norms(Bv);
    for (auto &v : bnorm)
        if (v == 0) v = 1;
    int total = 0, restarts = 0;
    std::vector<double> relres(R, 1.0);
    while (true) {
        // r = b - A x
        S.apply(X, w.p);
        k_sub<<<cdiv(NR2, 256), 256, 0, S.s>>>(Bv, w.p, NR2, r.p);
        XRL_HIP(hipGetLastError());
        std::vector<double> beta = S.norms(r.p);
        bool done = true;
        for (int c = 0; c < R; ++c) {
            relres[c] = beta[c] / bnorm[c];
            if (relres[c] > rtol) done = false;
        }
        if (done || total >= max_iter) break;
        std::vector<double> inv(R);
        for (int c = 0; c < R; ++c) inv[c] = beta[c] > 0 ? 1.0 / beta[c] : 0.0;
        S.scale(r.p, inv, V.p);
        // Hessenberg (column-major per RHS), Givens rotations, rhs g
        std::vector<cplx> H((size_t)(m + 1) * m * R, 0.0), cs((size_t)m * R), sn((size_t)m * R),
            gv((size_t)(m + 1) * R, 0.0);
        auto Hat = [&](int i, int j, int c) -> cplx & { return H[((size_t)j * (m + 1) + i) * R + c]; };
        for (int c = 0; c < R; ++c) gv[c] = beta[c];
        int k = 0;
        for (int j = 0; j < m && total < max_iter; ++j) {
            double *Vj = V.p + (size_t)j * NR2;
            S.apply(Vj, w.p);
            std::vector<cplx> h1 = S.dots(V.p, j + 1, w.p);
            S.project(V.p, j + 1, h1, w.p);
            std::vector<cplx> h2 = S.dots(V.p, j + 1, w.p);
            S.project(V.p, j + 1, h2, w.p);
            std::vector<double> hn = S.norms(w.p);
            std::vector<double> f(R);
            for (int c = 0; c < R; ++c) {
                for (int i = 0; i <= j; ++i) Hat(i, j, c) = h1[(size_t)i * R + c] + h2[(size_t)i * R + c];
                Hat(j + 1, j, c) = hn[c];
                f[c] = hn[c] > 1e-300 ? 1.0 / hn[c] : 0.0;
            }
            S.scale(w.p, f, V.p + (size_t)(j + 1) * NR2);
            ++total;
            k = j + 1;
            bool all = true;
            for (int c = 0; c < R; ++c) {
                for (int i = 0; i < j; ++i) {  // previous rotations
                    cplx a = Hat(i, j, c), bb = Hat(i + 1, j, c);
                    Hat(i, j, c) = std::conj(cs[(size_t)i * R + c]) * a + std::conj(sn[(size_t)i * R + c]) * bb;
                    Hat(i + 1, j, c) = -sn[(size_t)i * R + c] * a + cs[(size_t)i * R + c] * bb;
                }
                cplx a = Hat(j, j, c), bb = Hat(j + 1, j, c);
                const double den = std::sqrt(std::norm(a) + std::norm(bb));
                cplx cc = den > 0 ? a / den : 1.0, ss = den > 0 ? bb / den : 0.0;
                cs[(size_t)j * R + c] = cc;
                sn[(size_t)j * R + c] = ss;
                Hat(j, j, c) = std::conj(cc) * a + std::conj(ss) * bb;
                Hat(j + 1, j, c) = 0;
                cplx g0 = gv[(size_t)j * R + c];
                gv[(size_t)j * R + c] = std::conj(cc) * g0;
                gv[(size_t)(j + 1) * R + c] = -ss * g0;
                const double est = std::abs(gv[(size_t)(j + 1) * R + c]) / bnorm[c];
                if (est > rtol && hn[c] > 1e-300) all = false;
            }
            if (all) break;
        }
        // x += V y per RHS, y from the triangular solve
        std::vector<cplx> y((size_t)k * R, 0.0);
        for (int c = 0; c < R; ++c)
            for (int i = k - 1; i >= 0; --i) {
                cplx acc = gv[(size_t)i * R + c];
                for (int q = i + 1; q < k; ++q) acc -= Hat(i, q, c) * y[(size_t)q * R + c];
                y[(size_t)i * R + c] = Hat(i, i, c) != 0.0 ? acc / Hat(i, i, c) : 0.0;
            }
        std::vector<cplx> negy(y.size());
        for (size_t i = 0; i < y.size(); ++i) negy[i] = -y[i];
        S.project(V.p, k, negy, X);
        ++restarts;
    }
    double mx = 0;
    int conv = 0;
    for (int c = 0; c < R; ++c) {
        mx = std::max(mx, relres[c]);
        conv += relres[c] <= rtol;
    }
    if (stats) {
        stats->iterations = total;
        stats->restarts = restarts;
        stats->converged = conv;
        stats->max_rel_residual = mx;
    }
    XRL_HIP(hipStreamSynchronize(S.s));
    return conv;
}

}  // namespace xrl

extern "C" xrl_status xrl_gmres_solve(const xrl_plan *P, const xrl_epilogue *op, const void *b, void *x,
                                      int32_t n_rhs, int32_t dtype, int32_t restart, double rtol, int32_t max_iter,
                                      void *stream, xrl_gmres_stats *stats)
{
    xrl_status result = XRL_OK;
    xrl_status g = guarded([&] {
        XRL_CHECK(P && b && x && n_rhs >= 1 && restart >= 1 && restart <= 1000 && rtol > 0 && max_iter >= 1,
                  XRL_E_INVALID_ARG, "xrl_gmres_solve: bad arguments");
        XRL_CHECK(dtype == XRL_C64 || dtype == XRL_C128, XRL_E_INVALID_ARG, "xrl_gmres_solve: bad dtype %d", dtype);
        XRL_CHECK(n_rhs <= P->max_cols, XRL_E_INVALID_ARG, "xrl_gmres_solve: n_rhs > plan max_cols");
        XRL_CHECK(P->assembled, XRL_E_STATE, "xrl_gmres_solve: call xrl_nearfield_assemble first");
        hipStream_t s = (hipStream_t)stream;
        const AllocStream alloc_scope(s);
        const int64_t N = P->Nu, R = n_rhs, NR2 = 2 * N * R;
        const xrl_epilogue ep = op ? *op : xrl_epilogue{nullptr, nullptr};
        // complex64 right-hand sides and solutions are widened to complex128
        // for the iteration and the solution narrowed back at the end
        DevBuf<double> b64, x64;
        double *X = (double *)x;
        const double *Bv = (const double *)b;
        if (dtype == XRL_C64) {
            b64.alloc(NR2);
            x64.alloc(NR2);
            k_widen<<<cdiv(NR2, 256), 256, 0, s>>>((const float *)b, N * R, b64.p);
            k_widen<<<cdiv(NR2, 256), 256, 0, s>>>((const float *)x, N * R, x64.p);
            XRL_HIP(hipGetLastError());
            X = x64.p;
            Bv = b64.p;
        }
        auto apply = [&](const double *xx, double *yy) {
            xrl_status st = xrl_matvec_eager(P, xx, R, (int32_t)R, XRL_C128, yy, R, &ep, s);
            if (st != XRL_OK) throw Error{st, std::string("gmres matvec: ") + xrl_last_error()};
        };
        const int conv = gmres_core(apply, N, (int)R, Bv, X, restart, rtol, max_iter, s, stats);
        if (dtype == XRL_C64) {
            k_narrow<<<cdiv(NR2, 256), 256, 0, s>>>(X, N * R, (float *)x);
            XRL_HIP(hipGetLastError());
            XRL_HIP(hipStreamSynchronize(s));
        }
        if (conv < R) {
            set_error("xrl_gmres_solve: %d of %d right-hand sides did not reach rtol %.3g (max %.3g)", (int)R - conv,
                      (int)R, rtol, stats ? stats->max_rel_residual : 0.0);
            result = XRL_E_NOT_CONVERGED;
        }
    });
    return g != XRL_OK ? g : result;
}
