// Host construction (FP64) of the FMM translation operators and of the
// Gauss rules used by the device kernels.
//
// Expansions (Sec. II-C applies the FMM to the panel potential of eq. (6)):
//   multipole of a box with centre c:  M_n^m = int conj(R_n^m(y - c)) x(y) dy,
//   potential far from the box:         sum_{n,m} M_n^m I_n^m(r - c),
//   local expansion about c:            sum_{n,m} L_n^m R_n^m(r - c),
// with the unnormalised harmonics
//       R_n^m(u) = u^n P_n^m e^{im phi} / (n+m)!,   I_n^m(u) = (n-m)! P_n^m e^{im phi} / u^{n+1}
// (negative m by X_n^{-m} = (-1)^m conj(X_n^m)), for which
//       1/|x - y| = sum conj(R_n^m(y)) I_n^m(x)            (|y| < |x|)
//       R_n^m(a + b) = sum_{j,k} R_j^k(a) R_{n-j}^{m-k}(b)
//       I_n^m(d + r) = sum_{j,k} (-1)^{j+k} R_j^k(r) I_{n+j}^{m-k}(d)   (|r| < |d|)
// and the stored coefficients are scaled to the box size and normalised by
// s_nm = sqrt((n+|m|)!(n-|m|)!):
//       Mh_n^m = s_nm M_n^m / h^n,   Lh_n^m = h^{n+1} L_n^m / s_nm,
// which makes every operator independent of the level.
#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <complex>
#include <vector>

#include "common.h"
#include "harmonics.h"

namespace xrl {

using cd = std::complex<double>;

static double fact(int n)
{
    double f = 1;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}
static double snm(int n, int m)
{
    m = std::abs(m);
    return std::sqrt(fact(n + m) * fact(n - m));
}

// s_nm for every (n, m) up to degree P, index n*n + n + m.
static std::vector<double> snm_table(int P)
{
    std::vector<double> t((P + 1) * (P + 1));
    for (int n = 0; n <= P; ++n)
        for (int m = -n; m <= n; ++m) t[n * n + n + m] = snm(n, m);
    return t;
}

// Nonzero coefficients (n, m, value) of an expansion, in (n, m) order: a
// real unit vector has at most two, so the operators built by probing cost
// O(K) per column instead of O(K^2).
struct Term {
    int n, m;
    cd v;
};
static std::vector<Term> nonzeros(const std::vector<cd> &c, int p)
{
    std::vector<Term> t;
    for (int n = 0; n <= p; ++n)
        for (int m = -n; m <= n; ++m)
            if (c[n * n + n + m] != cd(0.0)) t.push_back({n, m, c[n * n + n + m]});
    return t;
}

// Associated Legendre P_n^m(c), m >= 0, with the Condon-Shortley phase.
static void legendre(int P, double c, std::vector<double> &out)
{
    out.assign((P + 1) * (P + 1), 0.0);
    auto at = [&](int n, int m) -> double & { return out[n * (P + 1) + m]; };
    double s = std::sqrt(std::max(0.0, 1 - c * c));
    at(0, 0) = 1;
    for (int m = 1; m <= P; ++m) at(m, m) = -(2 * m - 1) * s * at(m - 1, m - 1);
    for (int m = 0; m < P; ++m) at(m + 1, m) = (2 * m + 1) * c * at(m, m);
    for (int m = 0; m <= P; ++m)
        for (int n = m + 2; n <= P; ++n) at(n, m) = ((2 * n - 1) * c * at(n - 1, m) - (n + m - 1) * at(n - 2, m)) / (n - m);
}

struct Harm {
    int P;
    std::vector<cd> v;  // [(P+1)^2], index n*n + n + m, m in [-n, n]
    cd operator()(int n, int m) const
    {
        if (n < 0 || std::abs(m) > n || n > P) return 0.0;
        return v[n * n + n + m];
    }
};

// Unnormalised regular (irregular=false) or irregular harmonics at u.
static Harm harmonics(int P, const double u[3], bool irregular)
{
    Harm H;
    H.P = P;
    H.v.assign((P + 1) * (P + 1), 0.0);
    double r = std::sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double c = r > 0 ? u[2] / r : 1.0;
    double phi = std::atan2(u[1], u[0]);
    std::vector<double> L;
    legendre(P, c, L);
    for (int n = 0; n <= P; ++n)
        for (int m = 0; m <= n; ++m) {
            double mag = irregular ? fact(n - m) * L[n * (P + 1) + m] / std::pow(r, n + 1)
                                   : std::pow(r, n) * L[n * (P + 1) + m] / fact(n + m);
            cd val = std::polar(1.0, m * phi) * mag;
            H.v[n * n + n + m] = val;
            if (m > 0) H.v[n * n + n - m] = ((m & 1) ? -1.0 : 1.0) * std::conj(val);
        }
    return H;
}

// Real-field coefficient vector <-> real storage.
static std::vector<cd> from_real(int p, const double *x)
{
    std::vector<cd> c((p + 1) * (p + 1));
    for (int n = 0; n <= p; ++n) {
        c[n * n + n] = x[ridx(n, 0, 0)];
        for (int m = 1; m <= n; ++m) {
            cd v(x[ridx(n, m, 0)], x[ridx(n, m, 1)]);
            c[n * n + n + m] = v;
            c[n * n + n - m] = ((m & 1) ? -1.0 : 1.0) * std::conj(v);
        }
    }
    return c;
}
static void to_real(int p, const std::vector<cd> &c, double *x)
{
    for (int n = 0; n <= p; ++n) {
        x[ridx(n, 0, 0)] = c[n * n + n].real();
        for (int m = 1; m <= n; ++m) {
            x[ridx(n, m, 0)] = c[n * n + n + m].real();
            x[ridx(n, m, 1)] = c[n * n + n + m].imag();
        }
    }
}
// Dense real operator: out = A in, A[K][K] row-major (row = output index),
// built by applying `apply` to the K real unit vectors.
template <class F>
static void probe(int p, F apply, double *A)
{
    const int K = (p + 1) * (p + 1);
    std::vector<double> e(K), out(K);
    for (int i = 0; i < K; ++i) {
        std::fill(e.begin(), e.end(), 0.0);
        e[i] = 1.0;
        std::vector<cd> cin = from_real(p, e.data());
        std::vector<cd> cout = apply(cin);
        to_real(p, cout, out.data());
        for (int r = 0; r < K; ++r) A[r * K + i] = out[r];
    }
}

// Octant digit d (bit0 x, bit1 y, bit2 z) -> child centre minus parent centre
// in units of the parent side.
static void octant_shift(int d, double *u)
{
    for (int a = 0; a < 3; ++a) u[a] = ((d >> a) & 1) ? 0.25 : -0.25;
}

void build_m2m(int p, double *out /* [8][K][K] */)
{
    const int K = (p + 1) * (p + 1);
    for (int d = 0; d < 8; ++d) {
        double u[3];
        octant_shift(d, u);
        Harm R = harmonics(p, u, false);
        const std::vector<double> sn = snm_table(p);
        probe(
            p,
            [&](const std::vector<cd> &M) {
                std::vector<cd> O((p + 1) * (p + 1), 0.0);
                const std::vector<Term> nz = nonzeros(M, p);
                for (int n = 0; n <= p; ++n)
                    for (int m = -n; m <= n; ++m) {
                        cd acc = 0;
                        for (const Term &t : nz)
                            if (t.n <= n)
                                acc += sn[n * n + n + m] / sn[t.n * t.n + t.n + t.m] * std::conj(R(n - t.n, m - t.m)) *
                                       std::pow(0.5, t.n) * t.v;
                        O[n * n + n + m] = acc;
                    }
                return O;
            },
            out + (size_t)d * K * K);
    }
}

void build_l2l(int p, double *out /* [8][K][K] */)
{
    const int K = (p + 1) * (p + 1);
    for (int d = 0; d < 8; ++d) {
        double u[3];
        octant_shift(d, u);
        Harm R = harmonics(p, u, false);
        const std::vector<double> sn = snm_table(p);
        probe(
            p,
            [&](const std::vector<cd> &L) {
                std::vector<cd> O((p + 1) * (p + 1), 0.0);
                const std::vector<Term> nz = nonzeros(L, p);
                for (int j = 0; j <= p; ++j)
                    for (int k = -j; k <= j; ++k) {
                        cd acc = 0;
                        for (const Term &t : nz)
                            if (t.n >= j)
                                acc += sn[t.n * t.n + t.n + t.m] / sn[j * j + j + k] * R(t.n - j, t.m - k) *
                                       std::pow(0.5, j + 1) * t.v;
                        O[j * j + j + k] = acc;
                    }
                return O;
            },
            out + (size_t)d * K * K);
    }
}

// M2L for integer offset (target centre - source centre) / h = (ox, oy, oz).
void build_m2l(int p, int ox, int oy, int oz, double *out /* [K][K] */)
{
    double u[3] = {(double)ox, (double)oy, (double)oz};
    Harm I = harmonics(2 * p, u, true);
    const std::vector<double> sn = snm_table(p);
    probe(
        p,
        [&](const std::vector<cd> &M) {
            std::vector<cd> O((p + 1) * (p + 1), 0.0);
            const std::vector<Term> nz = nonzeros(M, p);
            for (int j = 0; j <= p; ++j)
                for (int k = -j; k <= j; ++k) {
                    cd acc = 0;
                    for (const Term &t : nz)
                        acc += t.v * I(t.n + j, t.m - k) / (sn[j * j + j + k] * sn[t.n * t.n + t.n + t.m]);
                    O[j * j + j + k] = (((j + k) & 1) ? -1.0 : 1.0) * acc;
                }
            return O;
        },
        out);
}

// Gauss-Legendre on [0,1] by the Golub-Welsch construction: eigenvalues of
// the symmetric tridiagonal Jacobi matrix (off-diagonal k/sqrt(4k^2-1)) are
// the nodes, squared first eigenvector components the weights.  Cyclic
// Jacobi rotations on the dense matrix (n is small).
void gauss_legendre01(int n, double *x, double *w)
{
    std::vector<double> A(n * n, 0.0), Vm(n * n, 0.0);
    for (int i = 0; i < n; ++i) Vm[i * n + i] = 1.0;
    for (int k = 1; k < n; ++k) {
        double b = k / std::sqrt(4.0 * k * k - 1.0);
        A[(k - 1) * n + k] = A[k * n + k - 1] = b;
    }
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += A[i * n + j] * A[i * n + j];
        if (off < 1e-32) break;
        for (int pi = 0; pi < n; ++pi)
            for (int q = pi + 1; q < n; ++q) {
                double apq = A[pi * n + q];
                if (std::fabs(apq) < 1e-300) continue;
                double theta = (A[q * n + q] - A[pi * n + pi]) / (2 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1));
                double c = 1 / std::sqrt(t * t + 1), s = t * c;
                for (int k = 0; k < n; ++k) {
                    double akp = A[k * n + pi], akq = A[k * n + q];
                    A[k * n + pi] = c * akp - s * akq;
                    A[k * n + q] = s * akp + c * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = A[pi * n + k], aqk = A[q * n + k];
                    A[pi * n + k] = c * apk - s * aqk;
                    A[q * n + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = Vm[k * n + pi], vkq = Vm[k * n + q];
                    Vm[k * n + pi] = c * vkp - s * vkq;
                    Vm[k * n + q] = s * vkp + c * vkq;
                }
            }
    }
    std::vector<std::pair<double, double>> nw(n);
    for (int i = 0; i < n; ++i) nw[i] = {A[i * n + i], 2.0 * Vm[i] * Vm[i]};  // Vm[0][i]
    std::sort(nw.begin(), nw.end());
    for (int i = 0; i < n; ++i) {
        x[i] = 0.5 * (nw[i].first + 1.0);
        w[i] = 0.5 * nw[i].second;
    }
}

}  // namespace xrl

extern "C" xrl_status xrl_m2l_operator(int32_t order, int32_t ox, int32_t oy, int32_t oz, double *out)
{
    return xrl::guarded([&] {
        XRL_CHECK(out, XRL_E_INVALID_ARG, "xrl_m2l_operator: null output");
        XRL_CHECK(order >= 2 && order <= 12 && order % 2 == 0, XRL_E_UNSUPPORTED,
                  "xrl_m2l_operator: order must be even in 2..12 (got %d)", order);
        const int a = std::max(std::abs(ox), std::max(std::abs(oy), std::abs(oz)));
        XRL_CHECK(a >= 2 && a <= 3, XRL_E_INVALID_ARG, "xrl_m2l_operator: offset must lie in [-3,3]^3 outside [-1,1]^3");
        xrl::build_m2l(order, ox, oy, oz, out);
    });
}
