// Loop analysis around the panel operator: the PEEC graph of the mesh and
// the centroid-midpoint maps A_1, A_2, A_3 (Sec. II-A, Algorithm 1), a loop
// basis M (Sec. II-B, eq. (7)), the surface impedance of eq. (3), the loop
// operator of eq. (8)/(9) applied through the FMM, and the diagonal-of-P
// preconditioner of eq. (10)/(11) with a sparse LDL^T factorisation.
//
// PEEC graph: panel centroids are nodes; a mesh edge shared by panels i < j
// is a branch whose global current runs from i to j.  Algorithm 1: row e of
// A_t holds rho_{i,e} = m_e - c_i (the vector points along the current) at
// column i and -rho_{j,e} at column j, component t.  Loops (rows of M, +-1
// per branch): one fan of panels around every mesh vertex except one vertex
// per connected surface, plus the handle loops of a tree-cotree split (two
// per handle of the surface); together they span the branch currents that
// satisfy current continuity at every panel (eq. (2)).
//
// The loop operator applied to loop currents I_l (R columns, one frequency
// each: alpha = j omega mu0 / 4 pi, beta = Z_s):
//     I_edge = M^T I_l,  I_pt = A_t^T I_edge (t = 1..3),
//     Y_t = beta .* area .* I_pt + alpha P I_pt     (the FMM matvec, 3R columns)
//     V_l = M sum_t A_t Y_t.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>
#include <exception>
#include <functional>
#include <numeric>
#include <memory>
#include <thread>
#include <vector>

#include "common.h"

using cplx = std::complex<double>;

struct xrl_loops {
    int64_t Np = 0, Ne = 0, Nl = 0, nv = 0;
    int64_t n_vertex_loops = 0, n_global_loops = 0, n_components = 0;
    std::vector<int32_t> h_pairs;  // [Ne][2] panels (i < j)
    std::vector<int32_t> h_verts;  // [Ne][2] mesh vertices of the edge
    std::vector<double> h_rho;     // [Ne][6] rho_i, rho_j
    std::vector<int32_t> h_mptr, h_midx;  // M, CSR over loops
    std::vector<int8_t> h_msgn;
    std::vector<int32_t> h_pedge;  // [Np][4] branch of each side of a panel (-1: no fourth side)
    std::vector<double> h_pcoef;   // [Np][4][3] A_t(e, p) of each side
    std::vector<double> h_area;    // [Np]
    xrl::DevBuf<int32_t> pairs, pedge, mptr, midx, mtptr, mtidx;
    xrl::DevBuf<int8_t> msgn, mtsgn;
    xrl::DevBuf<double> rho, pcoef;
};

// Eager matvec of the operator (fmm.hip): never replays a captured graph.
xrl_status xrl_matvec_eager(const xrl_plan *P, const void *x, int64_t ldx, int32_t n_cols, int32_t dtype, void *y,
                            int64_t ldy, const xrl_epilogue *ep, void *stream);

namespace xrl {

constexpr int kSides = 4;  // sides of a panel, at most (triangles leave the fourth empty)

int gmres_core(const std::function<void(const double *, double *)> &apply, int64_t N, int R, const double *Bv,
               double *X, int restart, double rtol, int max_iter, hipStream_t stream, xrl_gmres_stats *stats);

// ------------------------------------------------------------------ kernels
// out[row][c] = sum over the row's entries of sign * in[col][c]  (complex128,
// R columns): M (rows = loops) or M^T (rows = branches).
__global__ void k_signed_csr(int64_t nrows, const int32_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                             const int8_t *__restrict__ sgn, const double *__restrict__ in, int R,
                             double *__restrict__ out)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= nrows * R) return;
    const int64_t row = e / R;
    const int c = (int)(e - row * R);
    double re = 0, im = 0;
    for (int32_t q = ptr[row]; q < ptr[row + 1]; ++q) {
        const double s = sgn[q];
        re += s * in[2 * ((int64_t)idx[q] * R + c)];
        im += s * in[2 * ((int64_t)idx[q] * R + c) + 1];
    }
    out[2 * e] = re;
    out[2 * e + 1] = im;
}

// Panel currents I_p[p][3 c + t] = sum over the panel's sides k (three or
// four) of A_t(e_k, p) I_edge[e_k][c]  (A_t^T applied, complex128).
__global__ void k_edge_to_panel(int64_t Np, const int32_t *__restrict__ pedge, const double *__restrict__ pcoef,
                                const double *__restrict__ ie, int R, double *__restrict__ ip)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= Np * R) return;
    const int64_t p = e / R;
    const int c = (int)(e - p * R);
    double acc[3][2] = {{0, 0}, {0, 0}, {0, 0}};
    for (int k = 0; k < kSides; ++k) {
        const int32_t b = pedge[kSides * p + k];
        if (b < 0) continue;
        const double re = ie[2 * ((int64_t)b * R + c)], im = ie[2 * ((int64_t)b * R + c) + 1];
        for (int t = 0; t < 3; ++t) {
            const double a = pcoef[3 * (kSides * p + k) + t];
            acc[t][0] += a * re;
            acc[t][1] += a * im;
        }
    }
    for (int t = 0; t < 3; ++t) {
        ip[2 * (p * 3 * R + 3 * c + t)] = acc[t][0];
        ip[2 * (p * 3 * R + 3 * c + t) + 1] = acc[t][1];
    }
}

// Branch voltages V_edge[e][c] = sum_t A_t(e, i) Y[i][3c+t] + A_t(e, j) Y[j][3c+t]
// = rho_i . Y_i - rho_j . Y_j  (A_t applied, complex128).
__global__ void k_panel_to_edge(int64_t Ne, const int32_t *__restrict__ pairs, const double *__restrict__ rho,
                                const double *__restrict__ y, int R, double *__restrict__ ve)
{
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= Ne * R) return;
    const int64_t b = e / R;
    const int c = (int)(e - b * R);
    const int64_t i = pairs[2 * b], j = pairs[2 * b + 1];
    double re = 0, im = 0;
    for (int t = 0; t < 3; ++t) {
        const double ri = rho[6 * b + t], rj = rho[6 * b + 3 + t];
        re += ri * y[2 * (i * 3 * R + 3 * c + t)] - rj * y[2 * (j * 3 * R + 3 * c + t)];
        im += ri * y[2 * (i * 3 * R + 3 * c + t) + 1] - rj * y[2 * (j * 3 * R + 3 * c + t) + 1];
    }
    ve[2 * e] = re;
    ve[2 * e + 1] = im;
}

// Stored near-field entry of sorted elements (sk, sl): the block row of sl
// in the near list of sk's leaf, column of sk; NaN if it is not stored.
struct NearTable {
    const int32_t *panel_leaf, *leaf_box, *box_beg, *near_rows, *near_src, *leaf_tpad;
    const int64_t *val_off;
    const float *v32;
    const double *v64;
    __device__ double operator()(int32_t sk, int32_t sl) const
    {
        const int32_t li = panel_leaf[sk];
        int32_t lo = near_rows[li], hi = near_rows[li + 1];
        while (lo < hi) {
            const int32_t mid = lo + (hi - lo) / 2;
            if (near_src[mid] < sl)
                lo = mid + 1;
            else
                hi = mid;
        }
        if (lo >= near_rows[li + 1] || near_src[lo] != sl) return NAN;
        const int64_t at = val_off[li] + (int64_t)(lo - near_rows[li]) * leaf_tpad[li] + (sk - box_beg[leaf_box[li]]);
        return v64 ? v64[at] : (double)v32[at];
    }
};

// P_kl for user panels (k, l) that are near neighbours: the sum over the
// elements of both panels (one each for triangles, two for a four-sided
// panel, iperm2 >= 0).
__global__ void k_near_lookup(int64_t n, const int32_t *__restrict__ qk, const int32_t *__restrict__ ql,
                              const int32_t *__restrict__ iperm, const int32_t *__restrict__ iperm2, NearTable tab,
                              double *__restrict__ out)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t k[2] = {iperm[qk[i]], iperm2 ? iperm2[qk[i]] : -1};
    const int32_t l[2] = {iperm[ql[i]], iperm2 ? iperm2[ql[i]] : -1};
    double v = 0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            if (k[a] >= 0 && l[b] >= 0) v += tab(k[a], l[b]);
    out[i] = v;
}

// ------------------------------------------------------------------ loop search
// Panels as [Np][4] vertex indices, -1 as the fourth of a triangle.
static inline int sides(const int32_t *Q, int64_t p) { return Q[kSides * p + 3] >= 0 ? 4 : 3; }

static void build_edges(const int32_t *Q, int64_t Np, int64_t nv, xrl_loops &L)
{
    std::vector<std::pair<uint64_t, int32_t>> key;
    key.reserve(kSides * Np);
    for (int64_t p = 0; p < Np; ++p) {
        const int ns = sides(Q, p);
        for (int a = 0; a < ns; ++a) {
            const uint32_t u = (uint32_t)Q[kSides * p + a], w = (uint32_t)Q[kSides * p + (a + 1) % ns];
            key.push_back({((uint64_t)std::min(u, w) << 32) | std::max(u, w), (int32_t)(kSides * p + a)});
        }
    }
    std::sort(key.begin(), key.end());
    L.h_pedge.assign(kSides * Np, -1);
    for (size_t q = 0; q < key.size();) {
        size_t r = q;
        while (r < key.size() && key[r].first == key[q].first) ++r;
        XRL_CHECK(r - q == 2, XRL_E_UNSUPPORTED,
                  "xrl_loops_build: an edge belongs to %d panels (loop analysis needs a closed conforming mesh)",
                  (int)(r - q));
        const int32_t s0 = key[q].second, s1 = key[q + 1].second;
        const int32_t p0 = s0 / kSides, p1 = s1 / kSides;
        XRL_CHECK(p0 != p1, XRL_E_DEGENERATE_PANEL, "xrl_loops_build: panel %d repeats an edge", p0);
        const int32_t e = (int32_t)(L.h_pairs.size() / 2);
        L.h_pairs.push_back(std::min(p0, p1));
        L.h_pairs.push_back(std::max(p0, p1));
        L.h_verts.push_back((int32_t)(key[q].first >> 32));
        L.h_verts.push_back((int32_t)(key[q].first & 0xffffffffu));
        L.h_pedge[s0] = e;
        L.h_pedge[s1] = e;
        q = r;
    }
    L.Ne = (int64_t)L.h_pairs.size() / 2;
}

// Fan loop around mesh vertex v: walk the panels around v, crossing at each
// step the edge at v not crossed last; sign +1 where the walk follows the
// branch's global direction.
static bool vertex_fan(int32_t v, const std::vector<int32_t> &vp_ptr, const std::vector<int32_t> &vp,
                       const int32_t *Q, const xrl_loops &L, std::vector<std::pair<int32_t, int8_t>> &loop)
{
    loop.clear();
    const int32_t n = vp_ptr[v + 1] - vp_ptr[v];
    if (n < 3) return false;
    const int32_t start = vp[vp_ptr[v]];
    int32_t cur = start, came = -1;
    for (int step = 0; step < n; ++step) {
        int32_t next_e = -1;
        const int ns = sides(Q, cur);
        for (int a = 0; a < ns && next_e < 0; ++a) {
            const int32_t u = Q[kSides * cur + a], w = Q[kSides * cur + (a + 1) % ns];
            if (u != v && w != v) continue;
            const int32_t e = L.h_pedge[kSides * cur + a];
            if (e != came) next_e = e;
        }
        if (next_e < 0) return false;
        const int32_t i = L.h_pairs[2 * next_e], j = L.h_pairs[2 * next_e + 1];
        const int32_t nxt = i == cur ? j : i;
        loop.push_back({next_e, (int8_t)(i == cur ? 1 : -1)});
        came = next_e;
        cur = nxt;
        if (cur == start) return (int32_t)loop.size() == n;
    }
    return false;
}

static void build_loops(const int32_t *Q, xrl_loops &L)
{
    const int64_t Np = L.Np, Ne = L.Ne, nv = L.nv;
    // panels around each vertex
    std::vector<int32_t> vp_ptr(nv + 1, 0);
    for (int64_t q = 0; q < kSides * Np; ++q)
        if (Q[q] >= 0) ++vp_ptr[Q[q] + 1];
    for (int64_t v = 0; v < nv; ++v) vp_ptr[v + 1] += vp_ptr[v];
    std::vector<int32_t> vp(vp_ptr[nv]);
    {
        std::vector<int32_t> fill(vp_ptr.begin(), vp_ptr.end() - 1);
        for (int64_t p = 0; p < Np; ++p)
            for (int a = 0; a < sides(Q, p); ++a) vp[fill[Q[kSides * p + a]]++] = (int32_t)p;
    }
    // connected surfaces (BFS over branches)
    std::vector<std::vector<int32_t>> adj_e(Np);
    for (int64_t e = 0; e < Ne; ++e) {
        adj_e[L.h_pairs[2 * e]].push_back((int32_t)e);
        adj_e[L.h_pairs[2 * e + 1]].push_back((int32_t)e);
    }
    std::vector<int32_t> comp(Np, -1);
    int32_t nc = 0;
    for (int64_t p0 = 0; p0 < Np; ++p0) {
        if (comp[p0] >= 0) continue;
        std::vector<int32_t> q{(int32_t)p0};
        comp[p0] = nc;
        for (size_t h = 0; h < q.size(); ++h)
            for (int32_t e : adj_e[q[h]]) {
                const int32_t o = L.h_pairs[2 * e] == q[h] ? L.h_pairs[2 * e + 1] : L.h_pairs[2 * e];
                if (comp[o] < 0) {
                    comp[o] = nc;
                    q.push_back(o);
                }
            }
        ++nc;
    }
    L.n_components = nc;
    // vertex fans: all used vertices but the last of each surface
    std::vector<int32_t> last_v(nc, -1);
    for (int64_t v = 0; v < nv; ++v)
        if (vp_ptr[v + 1] > vp_ptr[v]) last_v[comp[vp[vp_ptr[v]]]] = (int32_t)v;
    L.h_mptr.assign(1, 0);
    std::vector<std::pair<int32_t, int8_t>> loop;
    auto add = [&](const std::vector<std::pair<int32_t, int8_t>> &lp) {
        for (auto &q : lp) {
            L.h_midx.push_back(q.first);
            L.h_msgn.push_back(q.second);
        }
        L.h_mptr.push_back((int32_t)L.h_midx.size());
    };
    for (int64_t v = 0; v < nv; ++v) {
        if (vp_ptr[v + 1] == vp_ptr[v]) continue;
        if (last_v[comp[vp[vp_ptr[v]]]] == v) continue;
        XRL_CHECK(vertex_fan((int32_t)v, vp_ptr, vp, Q, L, loop), XRL_E_UNSUPPORTED,
                  "xrl_loops_build: the panels around vertex %lld do not form one fan (non-manifold mesh)",
                  (long long)v);
        add(loop);
    }
    L.n_vertex_loops = (int64_t)L.h_mptr.size() - 1;
    // handle loops (tree-cotree): a spanning tree of the mesh's vertex graph,
    // a spanning tree of the PEEC graph over the branches whose edge is not
    // in it; each branch left over closes one loop through the second tree
    std::vector<char> in_tree(Ne, 0);
    {
        std::vector<std::vector<std::pair<int32_t, int32_t>>> vadj(nv);  // (neighbour, branch)
        for (int64_t e = 0; e < Ne; ++e) {
            vadj[L.h_verts[2 * e]].push_back({L.h_verts[2 * e + 1], (int32_t)e});
            vadj[L.h_verts[2 * e + 1]].push_back({L.h_verts[2 * e], (int32_t)e});
        }
        std::vector<char> seen(nv, 0);
        for (int64_t v0 = 0; v0 < nv; ++v0) {
            if (seen[v0] || vadj[v0].empty()) continue;
            std::vector<int32_t> q{(int32_t)v0};
            seen[v0] = 1;
            for (size_t h = 0; h < q.size(); ++h)
                for (auto &nb : vadj[q[h]])
                    if (!seen[nb.first]) {
                        seen[nb.first] = 1;
                        in_tree[nb.second] = 1;
                        q.push_back(nb.first);
                    }
        }
    }
    std::vector<int32_t> par(Np, -1), par_e(Np, -1), depth(Np, 0);
    std::vector<char> in_cotree(Ne, 0), done(Np, 0);
    for (int64_t p0 = 0; p0 < Np; ++p0) {
        if (done[p0]) continue;
        std::vector<int32_t> q{(int32_t)p0};
        done[p0] = 1;
        for (size_t h = 0; h < q.size(); ++h)
            for (int32_t e : adj_e[q[h]]) {
                if (in_tree[e]) continue;
                const int32_t o = L.h_pairs[2 * e] == q[h] ? L.h_pairs[2 * e + 1] : L.h_pairs[2 * e];
                if (done[o]) continue;
                done[o] = 1;
                par[o] = q[h];
                par_e[o] = e;
                depth[o] = depth[q[h]] + 1;
                in_cotree[e] = 1;
                q.push_back(o);
            }
    }
    for (int64_t e = 0; e < Ne; ++e) {
        if (in_tree[e] || in_cotree[e]) continue;
        // branch e from i to j, then back from j to i through the cotree
        loop.clear();
        int32_t a = L.h_pairs[2 * e], b = L.h_pairs[2 * e + 1];
        loop.push_back({(int32_t)e, 1});
        std::vector<std::pair<int32_t, int8_t>> up_b, up_a;  // j -> lca, then lca -> i (reversed)
        while (depth[b] > depth[a]) {
            const int32_t f = par_e[b];
            up_b.push_back({f, (int8_t)(L.h_pairs[2 * f] == b ? 1 : -1)});
            b = par[b];
        }
        while (depth[a] > depth[b]) {
            const int32_t f = par_e[a];
            up_a.push_back({f, (int8_t)(L.h_pairs[2 * f] == a ? -1 : 1)});  // walked par -> a
            a = par[a];
        }
        while (a != b) {
            const int32_t fb = par_e[b], fa = par_e[a];
            up_b.push_back({fb, (int8_t)(L.h_pairs[2 * fb] == b ? 1 : -1)});
            up_a.push_back({fa, (int8_t)(L.h_pairs[2 * fa] == a ? -1 : 1)});
            b = par[b];
            a = par[a];
        }
        for (auto &q : up_b) loop.push_back(q);
        for (auto it = up_a.rbegin(); it != up_a.rend(); ++it) loop.push_back(*it);
        add(loop);
    }
    L.Nl = (int64_t)L.h_mptr.size() - 1;
    L.n_global_loops = L.Nl - L.n_vertex_loops;
    XRL_CHECK(L.Nl == Ne - Np + nc, XRL_E_UNSUPPORTED,
              "xrl_loops_build: %lld loops found for a cycle space of dimension %lld", (long long)L.Nl,
              (long long)(Ne - Np + nc));
}

// ------------------------------------------------------------------ sparse LDL^T (complex symmetric)
// Envelope factorisation after a reverse Cuthill-McKee ordering:
// A = L D L^T without pivoting (A = R + jX with R, X symmetric positive
// definite, as the preconditioners of eq. (10) are, has no zero pivot).
static inline cplx zmulh(cplx a, cplx b)
{
    return cplx(a.real() * b.real() - a.imag() * b.imag(), a.real() * b.imag() + a.imag() * b.real());
}

// sum_{k in [k0, k1)} a[k] b[k] (complex), four independent partial sums so
// that the multiply-adds pipeline
static inline cplx zdot(const cplx *a, const cplx *b, int64_t k0, int64_t k1)
{
    double r[4] = {0, 0, 0, 0}, m[4] = {0, 0, 0, 0};
    int64_t k = k0;
    for (; k + 4 <= k1; k += 4)
        for (int u = 0; u < 4; ++u) {
            const cplx x = a[k + u], y = b[k + u];
            r[u] += x.real() * y.real() - x.imag() * y.imag();
            m[u] += x.real() * y.imag() + x.imag() * y.real();
        }
    for (; k < k1; ++k) {
        r[0] += a[k].real() * b[k].real() - a[k].imag() * b[k].imag();
        m[0] += a[k].real() * b[k].imag() + a[k].imag() * b[k].real();
    }
    return cplx((r[0] + r[1]) + (r[2] + r[3]), (m[0] + m[1]) + (m[2] + m[3]));
}

struct SparseLDL {
    int64_t n = 0;
    std::vector<int64_t> perm, first, off;  // permuted row i: columns first[i]..i-1 at env[off[i]..]
    std::vector<cplx> env, d, rinv;         // rinv = 1 / d

    void factor(int64_t nn, const std::vector<std::vector<std::pair<int64_t, cplx>>> &rows)
    {
        n = nn;
        // reverse Cuthill-McKee from a minimum-degree start per component
        perm.assign(n, -1);
        std::vector<int64_t> order;
        order.reserve(n);
        std::vector<char> seen(n, 0);
        std::vector<int64_t> byd(n);
        std::iota(byd.begin(), byd.end(), 0);
        std::sort(byd.begin(), byd.end(), [&](int64_t a, int64_t b) { return rows[a].size() < rows[b].size(); });
        for (int64_t s0 : byd) {
            if (seen[s0]) continue;
            size_t h = order.size();
            order.push_back(s0);
            seen[s0] = 1;
            for (; h < order.size(); ++h) {
                std::vector<int64_t> nb;
                for (auto &q : rows[order[h]])
                    if (!seen[q.first]) {
                        seen[q.first] = 1;
                        nb.push_back(q.first);
                    }
                std::sort(nb.begin(), nb.end(),
                          [&](int64_t a, int64_t b) { return rows[a].size() < rows[b].size(); });
                order.insert(order.end(), nb.begin(), nb.end());
            }
        }
        std::reverse(order.begin(), order.end());
        std::vector<int64_t> pos(n);
        for (int64_t i = 0; i < n; ++i) pos[order[i]] = i;
        perm = order;  // permuted i -> original
        first.assign(n, 0);
        for (int64_t i = 0; i < n; ++i) {
            int64_t f = i;
            for (auto &q : rows[order[i]]) f = std::min(f, pos[q.first]);
            first[i] = f;
        }
        off.assign(n + 1, 0);
        for (int64_t i = 0; i < n; ++i) off[i + 1] = off[i] + (i - first[i]);
        env.assign(off[n], cplx(0));
        d.assign(n, cplx(0));
        rinv.assign(n, cplx(0));
        for (int64_t i = 0; i < n; ++i)
            for (auto &q : rows[order[i]]) {
                const int64_t j = pos[q.first];
                if (j < i)
                    env[off[i] + (j - first[i])] += q.second;
                else if (j == i)
                    d[i] += q.second;
            }
        // row by row: L_ij = (A_ij - sum_k L_ik D_k L_jk) / D_j, D_i = A_ii - sum_k L_ik^2 D_k
        // (complex products written out: the library's complex multiply
        // handles infinities and NaNs through a slow call; the values here
        // are finite); W_k = L_ik D_k of the current row, kept beside it
        std::vector<cplx> w(n);
        for (int64_t i = 0; i < n; ++i) {
            cplx *li = env.data() + off[i];
            const int64_t fi = first[i];
            for (int64_t j = fi; j < i; ++j) {
                const int64_t k0 = std::max(fi, first[j]);
                const cplx acc = li[j - fi] - zdot(w.data(), env.data() + off[j] - first[j], k0, j);
                const double ar = acc.real(), ai = acc.imag();
                const cplx r = rinv[j];
                const cplx l(ar * r.real() - ai * r.imag(), ar * r.imag() + ai * r.real());
                li[j - fi] = l;
                w[j] = zmulh(l, d[j]);
            }
            const cplx dd = d[i] - zdot(w.data(), li - fi, fi, i);
            const double dr = dd.real(), di = dd.imag();
            XRL_CHECK(std::abs(dd) > 0, XRL_E_UNSUPPORTED, "preconditioner: zero pivot");
            d[i] = dd;
            const double q = dr * dr + di * di;
            rinv[i] = cplx(dr / q, -di / q);
        }
    }
    // x = A^-1 b in place (original order)
    void solve(cplx *b) const
    {
        std::vector<cplx> y(n);
        for (int64_t i = 0; i < n; ++i) y[i] = b[perm[i]];
        for (int64_t i = 0; i < n; ++i) y[i] -= zdot(env.data() + off[i] - first[i], y.data(), first[i], i);
        for (int64_t i = 0; i < n; ++i) y[i] = zmulh(y[i], rinv[i]);
        for (int64_t i = n - 1; i >= 0; --i) {
            const double yr = y[i].real(), yi = y[i].imag();
            const cplx *li = env.data() + off[i] - first[i];
            for (int64_t k = first[i]; k < i; ++k)
                y[k] = cplx(y[k].real() - (li[k].real() * yr - li[k].imag() * yi),
                            y[k].imag() - (li[k].real() * yi + li[k].imag() * yr));
        }
        for (int64_t i = 0; i < n; ++i) b[perm[i]] = y[i];
    }
};

// fn(c) for c in [0, n) on n host threads (the columns of the
// preconditioner are independent); the first failure is rethrown here.
template <class F>
static void for_each_column(int n, F fn)
{
    std::vector<std::exception_ptr> err(n);
    std::vector<std::thread> pool;
    for (int c = 1; c < n; ++c)
        pool.emplace_back([&, c] {
            try {
                fn(c);
            } catch (...) {
                err[c] = std::current_exception();
            }
        });
    try {
        if (n > 0) fn(0);
    } catch (...) {
        err[0] = std::current_exception();
    }
    for (auto &t : pool) t.join();
    for (auto &e : err)
        if (e) std::rethrow_exception(e);
}

// Q = M B M^T for an edge-space sparse B given per row (host).
static std::vector<std::vector<std::pair<int64_t, cplx>>> loop_product(
    const xrl_loops &L, const std::vector<std::vector<std::pair<int64_t, cplx>>> &B)
{
    // M^T as lists: loops through each branch
    std::vector<std::vector<std::pair<int32_t, int8_t>>> mt(L.Ne);
    for (int64_t l = 0; l < L.Nl; ++l)
        for (int32_t q = L.h_mptr[l]; q < L.h_mptr[l + 1]; ++q) mt[L.h_midx[q]].push_back({(int32_t)l, L.h_msgn[q]});
    std::vector<std::vector<std::pair<int64_t, cplx>>> Q(L.Nl);
    std::vector<cplx> rowB(L.Ne, 0.0), rowQ(L.Nl, 0.0);
    std::vector<int64_t> touchedB, touchedQ;
    std::vector<char> markB(L.Ne, 0), markQ(L.Nl, 0);
    for (int64_t l = 0; l < L.Nl; ++l) {
        for (int32_t q = L.h_mptr[l]; q < L.h_mptr[l + 1]; ++q) {
            const int32_t e = L.h_midx[q];
            const double s = L.h_msgn[q];
            for (auto &be : B[e]) {
                if (!markB[be.first]) {
                    markB[be.first] = 1;
                    touchedB.push_back(be.first);
                }
                rowB[be.first] += s * be.second;
            }
        }
        for (int64_t e : touchedB) {
            for (auto &ml : mt[e]) {
                if (!markQ[ml.first]) {
                    markQ[ml.first] = 1;
                    touchedQ.push_back(ml.first);
                }
                rowQ[ml.first] += (double)ml.second * rowB[e];
            }
            rowB[e] = 0;
            markB[e] = 0;
        }
        touchedB.clear();
        for (int64_t m : touchedQ) {
            if (rowQ[m] != 0.0) Q[l].push_back({m, rowQ[m]});
            rowQ[m] = 0;
            markQ[m] = 0;
        }
        touchedQ.clear();
    }
    return Q;
}

}  // namespace xrl

using namespace xrl;

extern "C" xrl_status xrl_loops_build(const xrl_mesh_desc *mesh, void *stream, xrl_loops **out)
{
    return guarded([&] {
        XRL_CHECK(mesh && out && mesh->vertices && mesh->tris, XRL_E_INVALID_ARG, "xrl_loops_build: null argument");
        XRL_CHECK(!mesh->on_device, XRL_E_UNSUPPORTED, "xrl_loops_build: the mesh must be on the host");
        XRL_CHECK(mesh->n_panels >= 1 && mesh->n_panels < (int64_t(1) << 31) && mesh->n_vertices >= 3 &&
                      mesh->n_vertices < (int64_t(1) << 31),
                  XRL_E_INVALID_ARG, "xrl_loops_build: bad sizes");
        *out = nullptr;
        hipStream_t s = (hipStream_t)stream;
        const AllocStream alloc_scope(s);
        const int vpp = mesh->verts_per_panel == 0 ? 3 : mesh->verts_per_panel;
        XRL_CHECK(vpp == 3 || vpp == 4, XRL_E_INVALID_ARG, "xrl_loops_build: verts_per_panel must be 3 or 4");
        auto L = std::make_unique<xrl_loops>();
        L->Np = mesh->n_panels;
        L->nv = mesh->n_vertices;
        const double *V = mesh->vertices;
        // panels as [Np][4], -1 as the fourth index of a triangle
        std::vector<int32_t> Qv(kSides * L->Np, -1);
        for (int64_t p = 0; p < L->Np; ++p)
            for (int a = 0; a < vpp; ++a) Qv[kSides * p + a] = mesh->tris[vpp * p + a];
        const int32_t *Q = Qv.data();
        for (int64_t p = 0; p < L->Np; ++p)
            for (int a = 0; a < sides(Q, p); ++a)
                XRL_CHECK(Q[kSides * p + a] >= 0 && Q[kSides * p + a] < L->nv, XRL_E_INVALID_ARG,
                          "xrl_loops_build: vertex index out of range");
        build_edges(Q, L->Np, L->nv, *L);
        // area centroids (a four-sided panel: the triangles (a, b, c) and
        // (a, c, d) weighted by area), rho vectors of Algorithm 1 and the
        // per-panel side coefficients
        std::vector<double> c(3 * L->Np, 0.0);
        L->h_area.assign(L->Np, 0.0);
        auto tri_area = [&](const double *a, const double *b, const double *d) {
            const double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]}, e2[3] = {d[0] - a[0], d[1] - a[1], d[2] - a[2]};
            const double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2],
                         cz = e1[0] * e2[1] - e1[1] * e2[0];
            return 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
        };
        for (int64_t p = 0; p < L->Np; ++p) {
            const int nt = sides(Q, p) - 2;
            for (int t = 0; t < nt; ++t) {
                const double *a = V + 3 * Q[kSides * p], *b = V + 3 * Q[kSides * p + 1 + t],
                             *d = V + 3 * Q[kSides * p + 2 + t];
                const double ar = tri_area(a, b, d);
                L->h_area[p] += ar;
                for (int k = 0; k < 3; ++k) c[3 * p + k] += ar * (a[k] + b[k] + d[k]) / 3.0;
            }
            for (int k = 0; k < 3; ++k) c[3 * p + k] /= L->h_area[p];
        }
        L->h_rho.resize(6 * L->Ne);
        for (int64_t e = 0; e < L->Ne; ++e) {
            const double *u = V + 3 * L->h_verts[2 * e], *w = V + 3 * L->h_verts[2 * e + 1];
            for (int side = 0; side < 2; ++side) {
                const int32_t p = L->h_pairs[2 * e + side];
                for (int k = 0; k < 3; ++k) L->h_rho[6 * e + 3 * side + k] = 0.5 * (u[k] + w[k]) - c[3 * p + k];
            }
        }
        L->h_pcoef.assign(3 * kSides * L->Np, 0.0);
        for (int64_t p = 0; p < L->Np; ++p)
            for (int k = 0; k < sides(Q, p); ++k) {
                const int32_t e = L->h_pedge[kSides * p + k];
                const bool is_i = L->h_pairs[2 * e] == p;
                for (int t = 0; t < 3; ++t)
                    L->h_pcoef[3 * (kSides * p + k) + t] = is_i ? L->h_rho[6 * e + t] : -L->h_rho[6 * e + 3 + t];
            }
        build_loops(Q, *L);
        // M^T (CSR over branches)
        std::vector<int32_t> mtptr(L->Ne + 1, 0), mtidx(L->h_midx.size());
        std::vector<int8_t> mtsgn(L->h_midx.size());
        for (int32_t e : L->h_midx) ++mtptr[e + 1];
        for (int64_t e = 0; e < L->Ne; ++e) mtptr[e + 1] += mtptr[e];
        {
            std::vector<int32_t> fill(mtptr.begin(), mtptr.end() - 1);
            for (int64_t l = 0; l < L->Nl; ++l)
                for (int32_t q = L->h_mptr[l]; q < L->h_mptr[l + 1]; ++q) {
                    const int32_t at = fill[L->h_midx[q]]++;
                    mtidx[at] = (int32_t)l;
                    mtsgn[at] = L->h_msgn[q];
                }
        }
        L->pairs.upload(L->h_pairs, s);
        L->rho.upload(L->h_rho, s);
        L->pedge.upload(L->h_pedge, s);
        L->pcoef.upload(L->h_pcoef, s);
        L->mptr.upload(L->h_mptr, s);
        L->midx.upload(L->h_midx, s);
        L->msgn.upload(L->h_msgn, s);
        L->mtptr.upload(mtptr, s);
        L->mtidx.upload(mtidx, s);
        L->mtsgn.upload(mtsgn, s);
        XRL_HIP(hipStreamSynchronize(s));
        *out = L.release();
    });
}

extern "C" void xrl_loops_destroy(xrl_loops *L) { delete L; }

extern "C" xrl_status xrl_loops_get_info(const xrl_loops *L, xrl_loops_info *info)
{
    return guarded([&] {
        XRL_CHECK(L && info, XRL_E_INVALID_ARG, "xrl_loops_get_info: null argument");
        info->n_panels = L->Np;
        info->n_edges = L->Ne;
        info->n_loops = L->Nl;
        info->n_vertex_loops = L->n_vertex_loops;
        info->n_global_loops = L->n_global_loops;
        info->n_components = L->n_components;
        info->nnz_loop_matrix = (int64_t)L->h_midx.size();
    });
}

extern "C" xrl_status xrl_loops_export(const xrl_loops *L, int32_t item, void *buf, int64_t *nbytes)
{
    return guarded([&] {
        XRL_CHECK(L && nbytes, XRL_E_INVALID_ARG, "xrl_loops_export: null argument");
        std::vector<int32_t> v;
        switch (item) {
            case 0: v = L->h_pairs; break;
            case 1: v = L->h_verts; break;
            case 2:
                v.reserve(3 * L->h_midx.size());
                for (int64_t l = 0; l < L->Nl; ++l)
                    for (int32_t q = L->h_mptr[l]; q < L->h_mptr[l + 1]; ++q) {
                        v.push_back((int32_t)l);
                        v.push_back(L->h_midx[q]);
                        v.push_back(L->h_msgn[q]);
                    }
                break;
            default: fail(XRL_E_INVALID_ARG, "xrl_loops_export: unknown item %d", item);
        }
        const int64_t nb = (int64_t)(v.size() * sizeof(int32_t));
        if (buf) {
            XRL_CHECK(*nbytes >= nb, XRL_E_INVALID_ARG, "xrl_loops_export: buffer too small");
            std::memcpy(buf, v.data(), nb);
        }
        *nbytes = nb;
    });
}

extern "C" xrl_status xrl_surface_impedance(double sigma, double thickness, const double *freq, int32_t n, double *zs)
{
    return guarded([&] {
        XRL_CHECK(sigma > 0 && thickness > 0 && freq && zs && n >= 0, XRL_E_INVALID_ARG,
                  "xrl_surface_impedance: bad arguments");
        const double pi = 3.14159265358979323846, mu0 = 4e-7 * pi;
        const double r_dc = 2.0 / (sigma * thickness), r_rf = std::sqrt(pi * mu0 / sigma);
        for (int32_t i = 0; i < n; ++i) {
            XRL_CHECK(freq[i] > 0, XRL_E_INVALID_ARG, "xrl_surface_impedance: frequency must be positive");
            const cplx z = cplx(1, 1) * r_rf * std::sqrt(freq[i]);
            // 1 - exp(-z / r_dc) = -expm1(-z / r_dc), taken without cancellation at low frequency
            const cplx u = -z / r_dc;
            const cplx em1 = std::abs(u) < 1e-3 ? u * (1.0 + u * (0.5 + u / 6.0)) : std::exp(u) - 1.0;
            const cplx v = z / (-em1);
            zs[2 * i] = v.real();
            zs[2 * i + 1] = v.imag();
        }
    });
}

namespace {

// Edge-space operator on R columns: V_edge = sum_t A_t (beta area + alpha P) A_t^T I_edge.
struct EdgeOp {
    const xrl_loops *L;
    const xrl_plan *P;
    int R;
    hipStream_t s;
    std::vector<double> alpha3, beta3;  // per FMM column (3 R): the column's scalars
    xrl_epilogue ep{};
    DevBuf<double> ip, yp;
    void init(const xrl_epilogue *op)
    {
        alpha3.assign(2 * 3 * (size_t)R, 0.0);
        beta3.assign(2 * 3 * (size_t)R, 0.0);
        for (int c = 0; c < R; ++c)
            for (int t = 0; t < 3; ++t) {
                alpha3[2 * (3 * c + t)] = op && op->alpha ? op->alpha[2 * c] : 1.0;
                alpha3[2 * (3 * c + t) + 1] = op && op->alpha ? op->alpha[2 * c + 1] : 0.0;
                beta3[2 * (3 * c + t)] = op && op->beta ? op->beta[2 * c] : 0.0;
                beta3[2 * (3 * c + t) + 1] = op && op->beta ? op->beta[2 * c + 1] : 0.0;
            }
        ep.alpha = alpha3.data();
        ep.beta = beta3.data();
        ip.alloc(2 * L->Np * 3 * (size_t)R);
        yp.alloc(2 * L->Np * 3 * (size_t)R);
    }
    void apply(const double *ie, double *ve)
    {
        const int64_t Np = L->Np, Ne = L->Ne;
        k_edge_to_panel<<<cdiv(Np * R, 256), 256, 0, s>>>(Np, L->pedge.p, L->pcoef.p, ie, R, ip.p);
        XRL_HIP(hipGetLastError());
        const xrl_status st = xrl_matvec_eager(P, ip.p, 3 * R, 3 * R, XRL_C128, yp.p, 3 * R, &ep, s);
        if (st != XRL_OK) throw Error{st, std::string("loop operator: ") + xrl_last_error()};
        k_panel_to_edge<<<cdiv(Ne * R, 256), 256, 0, s>>>(Ne, L->pairs.p, L->rho.p, yp.p, R, ve);
        XRL_HIP(hipGetLastError());
    }
};

void check_pair(const xrl_loops *L, const xrl_plan *P, int R, const char *who)
{
    XRL_CHECK(L && P, XRL_E_INVALID_ARG, "%s: null handle", who);
    XRL_CHECK(P->assembled, XRL_E_STATE, "%s: call xrl_nearfield_assemble first", who);
    XRL_CHECK(P->Nu == L->Np, XRL_E_INVALID_ARG, "%s: plan has %lld panels, loops %lld", who, (long long)P->Nu,
              (long long)L->Np);
    XRL_CHECK(R >= 1 && 3 * R <= P->max_cols, XRL_E_INVALID_ARG,
              "%s: 3 x n_cols (%d) must not exceed the plan's max_cols (%d)", who, 3 * R, P->max_cols);
}

}  // namespace

extern "C" xrl_status xrl_edge_matvec(const xrl_loops *L, const xrl_plan *P, const xrl_epilogue *op,
                                      const void *i_edge, void *v_edge, int32_t n_cols, void *stream)
{
    return guarded([&] {
        check_pair(L, P, n_cols, "xrl_edge_matvec");
        XRL_CHECK(i_edge && v_edge && i_edge != v_edge, XRL_E_INVALID_ARG, "xrl_edge_matvec: bad buffers");
        const AllocStream alloc_scope((hipStream_t)stream);
        EdgeOp E{L, P, n_cols, (hipStream_t)stream};
        E.init(op);
        E.apply((const double *)i_edge, (double *)v_edge);
        XRL_HIP(hipStreamSynchronize(E.s));
    });
}

extern "C" xrl_status xrl_loop_gmres_solve(const xrl_loops *L, const xrl_plan *P, const xrl_epilogue *op,
                                           const void *v_edge, void *i_edge, int32_t n_rhs, int32_t precond,
                                           int32_t restart, double rtol, int32_t max_iter, void *stream,
                                           xrl_gmres_stats *stats)
{
    xrl_status result = XRL_OK;
    xrl_status g = guarded([&] {
        check_pair(L, P, n_rhs, "xrl_loop_gmres_solve");
        XRL_CHECK(v_edge && i_edge && restart >= 1 && restart <= 1000 && rtol > 0 && max_iter >= 1 && precond >= 0 &&
                      precond <= 2,
                  XRL_E_INVALID_ARG, "xrl_loop_gmres_solve: bad arguments");
        hipStream_t s = (hipStream_t)stream;
        const AllocStream alloc_scope(s);
        const int R = n_rhs;
        const int64_t Nl = L->Nl, Ne = L->Ne;
        EdgeOp E{L, P, R, s};
        E.init(op);
        DevBuf<double> vl(2 * Nl * (size_t)R), il(2 * Nl * (size_t)R), ie(2 * Ne * (size_t)R),
            ve(2 * Ne * (size_t)R), tmp(2 * Nl * (size_t)R);
        // V_l = M V_edge (eq. (7))
        k_signed_csr<<<cdiv(Nl * R, 256), 256, 0, s>>>(Nl, L->mptr.p, L->midx.p, L->msgn.p, (const double *)v_edge, R,
                                                       vl.p);
        XRL_HIP(hipGetLastError());
        XRL_HIP(hipMemsetAsync(il.p, 0, il.bytes(), s));
        // eq. (8): Z_loop I_l = M sum_t A_t (beta area + alpha P) A_t^T M^T I_l
        auto op_loop = [&](const double *x, double *y) {
            k_signed_csr<<<cdiv(Ne * R, 256), 256, 0, s>>>(Ne, L->mtptr.p, L->mtidx.p, L->mtsgn.p, x, R, ie.p);
            XRL_HIP(hipGetLastError());
            E.apply(ie.p, ve.p);
            k_signed_csr<<<cdiv(Nl * R, 256), 256, 0, s>>>(Nl, L->mptr.p, L->midx.p, L->msgn.p, ve.p, R, y);
            XRL_HIP(hipGetLastError());
        };
        std::vector<SparseLDL> Qf;
        if (precond) {
            // eq. (10): Q = M sum_t A_t (beta area + alpha P_d) A_t^T M^T
            // (diagonal of P); or the diagonal-of-L form: the surface part
            // with the diagonal of the branch interaction matrix
            // sum_t A_t P A_t^T.  The diagonal of P and the entries of
            // adjacent panels come from the assembled near field.
            const int64_t Np = L->Np;
            std::vector<int32_t> qk, ql;
            for (int64_t p = 0; p < Np; ++p) {
                qk.push_back((int32_t)p);
                ql.push_back((int32_t)p);
            }
            if (precond == 2)
                for (int64_t e = 0; e < Ne; ++e) {
                    qk.push_back(L->h_pairs[2 * e]);
                    ql.push_back(L->h_pairs[2 * e + 1]);
                }
            DevBuf<int32_t> dk, dl;
            dk.upload(qk, s);
            dl.upload(ql, s);
            DevBuf<double> dv(qk.size());
            const NearTable tab{P->panel_leaf.p, P->leaf_box.p, P->box_beg.p, P->near_rows.p, P->near_src.p,
                                P->leaf_tpad.p, P->near_val_off.p, P->near32.p, P->near64.p};
            k_near_lookup<<<cdiv((int64_t)qk.size(), 256), 256, 0, s>>>((int64_t)qk.size(), dk.p, dl.p, P->iperm.p,
                                                                        P->iperm2.p, tab, dv.p);
            XRL_HIP(hipGetLastError());
            std::vector<double> pv = dv.download(s);
            for (double v : pv) XRL_CHECK(std::isfinite(v), XRL_E_STATE, "preconditioner: near entry missing");
            Qf.resize(R);
            for_each_column(R, [&](int c) {
                const cplx al(E.alpha3[6 * c], E.alpha3[6 * c + 1]), be(E.beta3[6 * c], E.beta3[6 * c + 1]);
                std::vector<std::vector<std::pair<int64_t, cplx>>> B(Ne);
                auto addB = [&](int64_t e, int64_t f, cplx v) {
                    for (auto &q : B[e])
                        if (q.first == f) {
                            q.second += v;
                            return;
                        }
                    B[e].push_back({f, v});
                };
                for (int64_t p = 0; p < Np; ++p) {
                    const cplx w = be * L->h_area[p] + (precond == 1 ? al * pv[p] : cplx(0));
                    for (int k = 0; k < kSides; ++k)
                        for (int m = 0; m < kSides; ++m) {
                            const int32_t ek = L->h_pedge[kSides * p + k], em = L->h_pedge[kSides * p + m];
                            if (ek < 0 || em < 0) continue;
                            double dot = 0;
                            for (int t = 0; t < 3; ++t)
                                dot += L->h_pcoef[3 * (kSides * p + k) + t] * L->h_pcoef[3 * (kSides * p + m) + t];
                            addB(ek, em, w * dot);
                        }
                }
                if (precond == 2)
                    for (int64_t e = 0; e < Ne; ++e) {
                        const int32_t i = L->h_pairs[2 * e], j = L->h_pairs[2 * e + 1];
                        const double *ri = &L->h_rho[6 * e], *rj = &L->h_rho[6 * e + 3];
                        const double ii = ri[0] * ri[0] + ri[1] * ri[1] + ri[2] * ri[2];
                        const double jj = rj[0] * rj[0] + rj[1] * rj[1] + rj[2] * rj[2];
                        const double ij = ri[0] * rj[0] + ri[1] * rj[1] + ri[2] * rj[2];
                        addB(e, e, al * (ii * pv[i] + jj * pv[j] - 2.0 * ij * pv[Np + e]));
                    }
                Qf[c].factor(Nl, loop_product(*L, B));
            });
        }
        // right preconditioning: GMRES on Z_loop Q^-1 u = V_l, I_l = Q^-1 u
        std::vector<cplx> hbuf;
        auto apply_qinv = [&](const double *x, double *y) {
            hbuf.resize((size_t)Nl * R);
            XRL_HIP(hipMemcpyAsync(hbuf.data(), x, hbuf.size() * sizeof(cplx), hipMemcpyDeviceToHost, s));
            XRL_HIP(hipStreamSynchronize(s));
            for_each_column(R, [&](int c) {
                std::vector<cplx> col(Nl);
                for (int64_t l = 0; l < Nl; ++l) col[l] = hbuf[(size_t)l * R + c];
                Qf[c].solve(col.data());
                for (int64_t l = 0; l < Nl; ++l) hbuf[(size_t)l * R + c] = col[l];
            });
            XRL_HIP(hipMemcpyAsync(y, hbuf.data(), hbuf.size() * sizeof(cplx), hipMemcpyHostToDevice, s));
            XRL_HIP(hipStreamSynchronize(s));
        };
        std::function<void(const double *, double *)> A = op_loop;
        if (precond)
            A = [&](const double *x, double *y) {
                apply_qinv(x, tmp.p);
                op_loop(tmp.p, y);
            };
        const int conv = gmres_core(A, Nl, R, vl.p, il.p, restart, rtol, max_iter, s, stats);
        if (precond) {
            apply_qinv(il.p, tmp.p);
            XRL_HIP(hipMemcpyAsync(il.p, tmp.p, il.bytes(), hipMemcpyDeviceToDevice, s));
        }
        // I_edge = M^T I_l
        k_signed_csr<<<cdiv(Ne * R, 256), 256, 0, s>>>(Ne, L->mtptr.p, L->mtidx.p, L->mtsgn.p, il.p, R,
                                                       (double *)i_edge);
        XRL_HIP(hipGetLastError());
        XRL_HIP(hipStreamSynchronize(s));
        if (conv < R) {
            set_error("xrl_loop_gmres_solve: %d of %d right-hand sides did not reach rtol %.3g", R - conv, R, rtol);
            result = XRL_E_NOT_CONVERGED;
        }
    });
    return g != XRL_OK ? g : result;
}
