/*
 * Plain FP64 CPU oracle for the Galerkin 1/R panel operator of the XRL method
 * (arXiv 2409.12375, Sec. II-A, eq. (6), second term; Sec. II-C, eq. (9)).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference against
 * which the GPU path is checked.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no code, header, table
 * or constant generator with the GPU library.
 *
 * What it computes (pulse basis w_k = 1 on panel S_k, eq. (4)/(6)):
 *
 *     P_kl = \int_{S_k} \int_{S_l} 1/|r - r'| dS' dS      (no mu0/4pi factor,
 *            the paper extracts j*omega*mu0/(4*pi) before the integral, Sec. II-D)
 *     y[k][c] = sum_l P_kl x[l][c]                          (direct O(N^2))
 *
 * Entry evaluation by pair class (k = target, l = source):
 *   self      k == l       closed form of the double integral over one flat
 *                          triangle (Arcioni, Bressan, Perregrini 1997;
 *                          Eibert, Hansen 1995).
 *   touching  shared vertex index
 *                          outer tensor Gauss rule on S_k in collapsed
 *                          coordinates with a sigmoidal change of variables
 *                          that clusters points on the shared edge/vertex;
 *                          inner integral exact (Wilton et al. 1984).  The
 *                          rule is refined until two successive values agree
 *                          to 1e-12.
 *   near      r < 4        outer 10 x 10 conical Gauss rule on S_k, split
 *                          into 4 sub-triangles when r < 2 and 16 when r < 1;
 *                          inner integral exact.
 *   far       r >= 4       product of two conical Gauss rules, n x n points per
 *                          triangle, n = 4 (r < 30) or 3 (r >= 30).
 *   with r = |c_k - c_l| / max(diam_k, diam_l).
 *
 * Gauss-Legendre nodes come from Newton's method on the three-term Legendre
 * recurrence.  Nothing is tabulated.
 *
 * Parity: every routine is pinned by the CPU test-suite (closed forms, an
 * independent polar-angle integration of the point potential, symmetry of P,
 * the monopole limit, the discretised-sphere potential, positive definiteness).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXGL 64

/* ------------------------------------------------------------------ */
/* small vector helpers                                                 */
/* ------------------------------------------------------------------ */
static void sub3(const double *a, const double *b, double *o) { o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2]; }
static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double *a) { return sqrt(dot3(a, a)); }
static double dist3(const double *a, const double *b) { double d[3]; sub3(a, b, d); return norm3(d); }

/* ------------------------------------------------------------------ */
/* Gauss-Legendre on [0,1] by Newton iteration on P_n                    */
/* ------------------------------------------------------------------ */
void orc_gauss_legendre01(int n, double *x, double *w)
{
    for (int i = 0; i < n; ++i) {
        /* initial guess near the i-th root of P_n */
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        double pn = 1.0, pnm1 = 1.0;
        for (int it = 0; it < 100; ++it) {
            /* P_n(z) and P_{n-1}(z) by (k) P_k = (2k-1) z P_{k-1} - (k-1) P_{k-2} */
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            pn = p1;
            pnm1 = p0;
            double dp = n * (z * pn - pnm1) / (z * z - 1.0);
            double dz = pn / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        double dp = n * (z * p1 - p0) / (z * z - 1.0);
        double wi = 2.0 / ((1.0 - z * z) * dp * dp);
        /* map [-1,1] -> [0,1]; roots come out descending, store ascending */
        x[n - 1 - i] = 0.5 * (1.0 + z);
        w[n - 1 - i] = 0.5 * wi;
    }
}

/* ------------------------------------------------------------------ */
/* Triangle geometry                                                   */
/* ------------------------------------------------------------------ */
static double tri_area(const double *t)
{
    double e1[3], e2[3], c[3];
    sub3(t + 3, t, e1);
    sub3(t + 6, t, e2);
    cross3(e1, e2, c);
    return 0.5 * norm3(c);
}
static double tri_diam(const double *t)
{
    double a = dist3(t, t + 3), b = dist3(t + 3, t + 6), c = dist3(t + 6, t);
    double m = a > b ? a : b;
    return m > c ? m : c;
}
static void tri_centroid(const double *t, double *c)
{
    for (int d = 0; d < 3; ++d) c[d] = (t[d] + t[3 + d] + t[6 + d]) / 3.0;
}

/* Per-panel area, centroid, unit normal (right-hand rule on the vertex
 * order) and diameter (longest edge). */
void orc_panel_geometry(const double *V, const int32_t *T, int64_t N,
                        double *area, double *centroid, double *normal, double *diam)
{
    for (int64_t k = 0; k < N; ++k) {
        double t[9];
        for (int j = 0; j < 3; ++j)
            for (int d = 0; d < 3; ++d) t[3 * j + d] = V[3 * (int64_t)T[3 * k + j] + d];
        double e1[3], e2[3], c[3];
        sub3(t + 3, t, e1);
        sub3(t + 6, t, e2);
        cross3(e1, e2, c);
        double nn = norm3(c);
        area[k] = 0.5 * nn;
        for (int d = 0; d < 3; ++d) normal[3 * k + d] = c[d] / nn;
        tri_centroid(t, centroid + 3 * k);
        diam[k] = tri_diam(t);
    }
}

/* ------------------------------------------------------------------ */
/* Self term: closed form of int_T int_T 1/|r-r'| for a flat triangle   */
/*   (4 A^2 / 3) * sum_e (1/l_e) ln( Pr / (Pr - 2 l_e) ),  Pr = perimeter */
/* ------------------------------------------------------------------ */
double orc_self(const double *t)
{
    double l[3] = {dist3(t, t + 3), dist3(t + 3, t + 6), dist3(t + 6, t)};
    double pr = l[0] + l[1] + l[2];
    double A = tri_area(t);
    double s = 0.0;
    for (int e = 0; e < 3; ++e) s += log(pr / (pr - 2.0 * l[e])) / l[e];
    return 4.0 * A * A / 3.0 * s;
}

/* ------------------------------------------------------------------ */
/* Exact potential of a unit-density flat triangle at point r           */
/*   phi(r) = int_T 1/|r - r'| dS'   (Wilton, Rao, Glisson et al. 1984) */
/* ------------------------------------------------------------------ */
/* R + l computed without cancellation when l < 0:  R + l = (R^2 - l^2)/(R - l) */
static double rpl(double R, double l, double R0sq)
{
    return (l >= 0.0) ? (R + l) : (R0sq / (R - l));
}

double orc_point_potential(const double *t, const double *r)
{
    double e1[3], e2[3], n[3];
    sub3(t + 3, t, e1);
    sub3(t + 6, t, e2);
    cross3(e1, e2, n);
    double nn = norm3(n);
    for (int d = 0; d < 3; ++d) n[d] /= nn;
    double rv[3];
    sub3(r, t, rv);
    double h = dot3(n, rv);
    double ah = fabs(h);
    double rho[3] = {r[0] - h * n[0], r[1] - h * n[1], r[2] - h * n[2]};
    double scale = tri_diam(t);
    double phi = 0.0;
    for (int i = 0; i < 3; ++i) {
        const double *va = t + 3 * i;
        const double *vb = t + 3 * ((i + 1) % 3);
        double le[3];
        sub3(vb, va, le);
        double len = norm3(le);
        for (int d = 0; d < 3; ++d) le[d] /= len;
        double u[3];
        cross3(le, n, u); /* outward in-plane edge normal for right-handed order */
        double dva[3], dvb[3];
        sub3(va, rho, dva);
        sub3(vb, rho, dvb);
        double P0 = dot3(dva, u);
        double lm = dot3(dva, le), lp = dot3(dvb, le);
        double R0sq = P0 * P0 + h * h;
        double Rm = dist3(r, va), Rp = dist3(r, vb);
        if (fabs(P0) > 1e-14 * scale) {
            double num = rpl(Rp, lp, R0sq), den = rpl(Rm, lm, R0sq);
            phi += P0 * log(num / den);
            if (ah > 1e-14 * scale) {
                phi -= ah * (atan(P0 * lp / (R0sq + ah * Rp)) - atan(P0 * lm / (R0sq + ah * Rm)));
            }
        }
    }
    return phi;
}

/* ------------------------------------------------------------------ */
/* Quadrature building blocks                                           */
/* ------------------------------------------------------------------ */
/* Conical (collapsed) product rule on a triangle: x = v0 + s (v1 - v0) + s t (v2 - v1),
 * Jacobian 2 A s.  With n Gauss points per direction it is exact for total
 * degree 2n - 2. */
typedef struct {
    int n;
    double x[ORC_MAXGL], w[ORC_MAXGL];
} gl_rule;

static gl_rule gl_cache[ORC_MAXGL + 1];
static int gl_ready = 0;

/* Fill the rule cache once (called before any parallel region). */
void orc_init(void)
{
    if (gl_ready) return;
    for (int n = 1; n <= ORC_MAXGL; ++n) {
        gl_cache[n].n = n;
        orc_gauss_legendre01(n, gl_cache[n].x, gl_cache[n].w);
    }
    gl_ready = 1;
}

static void gl_make(gl_rule *g, int n)
{
    if (!gl_ready) orc_init();
    *g = gl_cache[n];
}

/* Fill pts[np][3], wts[np] with the conical rule on triangle t. Returns np. */
static int conical_points(const double *t, const gl_rule *g, double *pts, double *wts)
{
    double A2 = 2.0 * tri_area(t);
    int m = 0;
    for (int i = 0; i < g->n; ++i)
        for (int j = 0; j < g->n; ++j) {
            double s = g->x[i], u = g->x[j];
            for (int d = 0; d < 3; ++d)
                pts[3 * m + d] = t[d] + s * (t[3 + d] - t[d]) + s * u * (t[6 + d] - t[3 + d]);
            wts[m] = g->w[i] * g->w[j] * A2 * s;
            ++m;
        }
    return m;
}

/* int_{T} f(x) dx with f = potential of triangle src, one conical rule */
static double outer_rule(const double *tgt, const double *src, const gl_rule *g)
{
    double pts[3 * ORC_MAXGL * ORC_MAXGL / 4], wts[ORC_MAXGL * ORC_MAXGL / 4];
    int np = conical_points(tgt, g, pts, wts);
    double s = 0.0;
    for (int q = 0; q < np; ++q) s += wts[q] * orc_point_potential(src, pts + 3 * q);
    return s;
}

static void split4(const double *t, double c[4][9])
{
    double m01[3], m12[3], m20[3];
    for (int d = 0; d < 3; ++d) {
        m01[d] = 0.5 * (t[d] + t[3 + d]);
        m12[d] = 0.5 * (t[3 + d] + t[6 + d]);
        m20[d] = 0.5 * (t[6 + d] + t[d]);
    }
    for (int d = 0; d < 3; ++d) {
        c[0][d] = t[d];      c[0][3 + d] = m01[d];    c[0][6 + d] = m20[d];
        c[1][d] = m01[d];    c[1][3 + d] = t[3 + d];  c[1][6 + d] = m12[d];
        c[2][d] = m20[d];    c[2][3 + d] = m12[d];    c[2][6 + d] = t[6 + d];
        c[3][d] = m12[d];    c[3][3 + d] = m20[d];    c[3][6 + d] = m01[d];
    }
}

/* Outer integration over tgt split uniformly into 4^levels sub-triangles,
 * each with an n x n conical rule; the inner integral over src is exact. */
static double subdiv_outer(const double *tgt, const double *src, const gl_rule *g, int levels)
{
    if (levels == 0) return outer_rule(tgt, src, g);
    double c[4][9];
    split4(tgt, c);
    double acc = 0.0;
    for (int i = 0; i < 4; ++i) acc += subdiv_outer(c[i], src, g, levels - 1);
    return acc;
}

/* Sigmoidal map of [0,1] onto itself, clustering points at both ends:
 *   psi(u) = u^q / (u^q + (1-u)^q). */
static void sigmoid(double u, int q, double *psi, double *dpsi)
{
    double a = pow(u, q), b = pow(1.0 - u, q);
    *psi = a / (a + b);
    *dpsi = q * pow(u, q - 1) * pow(1.0 - u, q - 1) / ((a + b) * (a + b));
}

/* Outer rule for a target triangle whose vertex t[0..2] is the collapse
 * point: x = t0 + s (t1 - t0) + s u (t2 - t1).  Both s and u go through the
 * sigmoidal map, so the rule clusters on every edge and on every vertex of
 * the target triangle. n points per direction. */
static double sigmoid_outer(const double *tgt, const double *src, int n, int q)
{
    gl_rule g;
    gl_make(&g, n);
    double A2 = 2.0 * tri_area(tgt);
    double acc = 0.0;
    for (int i = 0; i < n; ++i) {
        double s, ds;
        sigmoid(g.x[i], q, &s, &ds);
        for (int j = 0; j < n; ++j) {
            double u, du;
            sigmoid(g.x[j], q, &u, &du);
            double x[3];
            for (int d = 0; d < 3; ++d)
                x[d] = tgt[d] + s * (tgt[3 + d] - tgt[d]) + s * u * (tgt[6 + d] - tgt[3 + d]);
            acc += g.w[i] * g.w[j] * ds * du * A2 * s * orc_point_potential(src, x);
        }
    }
    return acc;
}

/* Touching pair: rotate the target's vertex order so that a shared vertex is
 * the collapse point, then refine the sigmoidal tensor rule until two
 * successive values agree to 1e-12 relative. */
static double touching_pair(const double *tgt, const double *src, int shared_local)
{
    double t[9];
    for (int j = 0; j < 3; ++j)
        for (int d = 0; d < 3; ++d) t[3 * j + d] = tgt[3 * ((shared_local + j) % 3) + d];
    double prev = sigmoid_outer(t, src, 12, 4);
    for (int n = 20; n <= 60; n += 8) {
        double cur = sigmoid_outer(t, src, n, 4);
        if (fabs(cur - prev) <= 1e-12 * fabs(cur)) return cur;
        prev = cur;
    }
    return prev;
}

/* Public: semi-analytic value of int_{tgt} phi_src with the sigmoidal rule
 * collapsed at target vertex `collapse` (used by tests for the self term). */
double orc_semianalytic_sigmoid(const double *tgt, const double *src, int collapse, int n)
{
    double t[9];
    for (int j = 0; j < 3; ++j)
        for (int d = 0; d < 3; ++d) t[3 * j + d] = tgt[3 * ((collapse + j) % 3) + d];
    return sigmoid_outer(t, src, n, 4);
}

/* Public: semi-analytic value of int_{tgt} phi_src with an n x n conical
 * rule on each of 4^levels sub-triangles of tgt. */
double orc_semianalytic_subdiv(const double *tgt, const double *src, int n, int levels)
{
    gl_rule g;
    gl_make(&g, n);
    return subdiv_outer(tgt, src, &g, levels);
}

/* Far pair: product conical rule, n x n points on each triangle. */
double orc_far_pair(const double *tk, const double *tl, int n)
{
    gl_rule g;
    gl_make(&g, n);
    double pk[3 * 64], wk[64], pl[3 * 64], wl[64];
    int nk = conical_points(tk, &g, pk, wk), nl = conical_points(tl, &g, pl, wl);
    double acc = 0.0;
    for (int a = 0; a < nk; ++a)
        for (int b = 0; b < nl; ++b) acc += wk[a] * wl[b] / dist3(pk + 3 * a, pl + 3 * b);
    return acc;
}

/* Public: conical rule on the reference triangle (0,0),(1,0),(0,1) applied
 * to the monomial x^a y^b (tests check the exactness degree 2n - 2). */
double orc_conical_monomial(int n, int a, int b)
{
    gl_rule g;
    gl_make(&g, n);
    double t[9] = {0, 0, 0, 1, 0, 0, 0, 1, 0};
    double pts[3 * ORC_MAXGL * ORC_MAXGL / 4], wts[ORC_MAXGL * ORC_MAXGL / 4];
    int np = conical_points(t, &g, pts, wts);
    double acc = 0.0;
    for (int q = 0; q < np; ++q) acc += wts[q] * pow(pts[3 * q], a) * pow(pts[3 * q + 1], b);
    return acc;
}

/* ------------------------------------------------------------------ */
/* One operator entry P_kl from vertex coordinates and vertex indices  */
/* ------------------------------------------------------------------ */
double orc_entry(const double *tk, const int32_t *ik, const double *tl, const int32_t *il, int same)
{
    if (same) return orc_self(tk);
    int shared = -1;
    for (int a = 0; a < 3 && shared < 0; ++a)
        for (int b = 0; b < 3; ++b)
            if (ik[a] == il[b]) { shared = a; break; }
    if (shared >= 0) return touching_pair(tk, tl, shared);
    double ck[3], cl[3];
    tri_centroid(tk, ck);
    tri_centroid(tl, cl);
    double dk = tri_diam(tk), dl = tri_diam(tl);
    double r = dist3(ck, cl) / (dk > dl ? dk : dl);
    if (r < 4.0) return orc_semianalytic_subdiv(tk, tl, 10, r < 1.0 ? 2 : (r < 2.0 ? 1 : 0));
    return orc_far_pair(tk, tl, r < 30.0 ? 4 : 3);
}

/* Entry by panel index (convenience for tests). */
double orc_entry_idx(const double *V, const int32_t *T, int64_t k, int64_t l)
{
    double tk[9], tl[9];
    for (int j = 0; j < 3; ++j)
        for (int d = 0; d < 3; ++d) {
            tk[3 * j + d] = V[3 * (int64_t)T[3 * k + j] + d];
            tl[3 * j + d] = V[3 * (int64_t)T[3 * l + j] + d];
        }
    return orc_entry(tk, T + 3 * k, tl, T + 3 * l, k == l);
}

/* ------------------------------------------------------------------ */
/* Direct matvec over a set of target rows                              */
/*   y[i][c] = sum_l P_{rows[i], l} x[l][c],  x is [N][C] row-major      */
/* Returns the number of threads used.                                  */
/* ------------------------------------------------------------------ */
int orc_matvec_rows(const double *V, const int32_t *T, int64_t N,
                    const double *x, int64_t C, const int64_t *rows, int64_t nrows,
                    double *y, int nthreads)
{
    int used = 1;
    orc_init();
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
    {
#pragma omp single
        used = omp_get_num_threads();
    }
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nrows; ++i) {
        int64_t k = rows[i];
        double *acc = (double *)calloc((size_t)C, sizeof(double));
        for (int64_t l = 0; l < N; ++l) {
            double p = orc_entry_idx(V, T, k, l);
            for (int64_t c = 0; c < C; ++c) acc[c] += p * x[l * C + c];
        }
        for (int64_t c = 0; c < C; ++c) y[i * C + c] = acc[c];
        free(acc);
    }
    return used;
}

/* P_kl for an explicit list of (k, l) index pairs (training labels). */
void orc_pairs(const double *V, const int32_t *T, const int64_t *ks, const int64_t *ls, int64_t n, double *out,
               int nthreads)
{
    orc_init();
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) out[i] = orc_entry_idx(V, T, ks[i], ls[i]);
}

/* Dense operator block P[rows][cols] (tests on small meshes). */
void orc_dense(const double *V, const int32_t *T, const int64_t *rows, int64_t nr,
               const int64_t *cols, int64_t nc, double *P, int nthreads)
{
    orc_init();
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = 0; i < nr; ++i)
        for (int64_t j = 0; j < nc; ++j) P[i * nc + j] = orc_entry_idx(V, T, rows[i], cols[j]);
}
