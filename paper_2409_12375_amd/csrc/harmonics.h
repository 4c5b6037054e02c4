// Solid harmonics for the Laplace FMM on panel centroids.
//
// Normalised regular solid harmonics (m >= 0)
//     Rn_m(u) = sqrt((n-m)!/(n+m)!) |u|^n P_n^m(cos theta) e^{i m phi}
// with P_n^m carrying the Condon-Shortley phase, so |Rn_m(u)| <= |u|^n.
// They obey (classical solid-harmonic recurrences)
//     R_m^m = -(x + i y) sqrt((2m-1)/(2m)) R_{m-1}^{m-1}
//     R_n^m = [(2n-1) z R_{n-1}^m - sqrt((n+m-1)(n-m-1)) |u|^2 R_{n-2}^m] / sqrt((n+m)(n-m)).
//
// Real storage of a coefficient vector of a real field (X_n^{-m} =
// (-1)^m conj(X_n^m)): index n^2 for m = 0, n^2 + 2m - 1 (real part) and
// n^2 + 2m (imaginary part) for m >= 1; (p+1)^2 reals in total.
#pragma once

#include <hip/hip_runtime.h>

namespace xrl {

// Complex normalised regular harmonics up to degree P, m >= 0, stored at
// n(n+1)/2 + m.  T is float or double.
template <int P, typename T>
__host__ __device__ inline void regular_harmonics(T x, T y, T z, T *re, T *im)
{
    const T r2 = x * x + y * y + z * z;
    re[0] = T(1);
    im[0] = T(0);
    for (int m = 0; m <= P; ++m) {
        const int mm = m * (m + 1) / 2 + m;  // index of (m, m)
        if (m > 0) {
            const int pm = (m - 1) * m / 2 + (m - 1);
            const T f = -sqrt(T(2 * m - 1) / T(2 * m));
            const T pr = re[pm], pi = im[pm];
            re[mm] = f * (x * pr - y * pi);
            im[mm] = f * (x * pi + y * pr);
        }
        if (m + 1 <= P) {
            const int i1 = (m + 1) * (m + 2) / 2 + m;
            const T f = T(2 * m + 1) * z / sqrt(T(2 * m + 1));
            re[i1] = f * re[mm];
            im[i1] = f * im[mm];
        }
        for (int n = m + 2; n <= P; ++n) {
            const int i0 = n * (n + 1) / 2 + m;
            const int i1 = (n - 1) * n / 2 + m;
            const int i2 = (n - 2) * (n - 1) / 2 + m;
            const T a = T(2 * n - 1) * z;
            const T b = sqrt(T((n + m - 1) * (n - m - 1))) * r2;
            const T inv = T(1) / sqrt(T((n + m) * (n - m)));
            re[i0] = (a * re[i1] - b * re[i2]) * inv;
            im[i0] = (a * im[i1] - b * im[i2]) * inv;
        }
    }
}

// Real-storage index of (n, m, part).
__host__ __device__ inline int ridx(int n, int m, int part) { return m == 0 ? n * n : n * n + 2 * m - 1 + part; }

}  // namespace xrl
