"""Plain FP64 reference of the loop formulation around the panel operator
(TEST INFRASTRUCTURE ONLY: tests may import this module, the library never
does).

What it computes, from the paper (arXiv 2409.12375):
  * the PEEC graph of a closed, conforming triangle mesh: panel centroids
    are nodes, each edge shared by two panels is a branch (Sec. II-A);
  * the centroid-midpoint maps A_1, A_2, A_3 (N_e x N_p) of Algorithm 1:
    row e (the branch between panels i and j, global current from i to j)
    holds rho_{i,e} = m_e - c_i with + (the vector points along the current)
    and rho_{j,e} = m_e - c_j with - (it points against it), component t;
  * the branch-panel incidence D (N_p x N_e) of current continuity, eq. (2)
    (Kirchhoff's current law at every panel node): a loop basis M spans the
    null space of D;
  * the surface impedance Z_s of eq. (3) (double-plane model);
  * the edge-space impedance Z_e = sum_t A_t (beta diag(area) + alpha P) A_t^T
    (eq. (5) with eq. (6): beta = Z_s, alpha = j omega mu0 / 4 pi);
  * the solution of the loop system eq. (7)-(8) expressed in edge currents,
    I_edge = M^T (M Z_e M^T)^-1 M V_edge, which does not depend on which loop
    basis M spans the null space of D: here M is replaced by an orthonormal
    basis Q of that null space (numpy SVD), so the reference needs no loop
    search of its own.
Panels are triangles ([N][3]) or, on hybrid meshes (Sec. II-A, Fig. 1),
triangles and four-sided panels ([N][4], a negative fourth index marks a
triangle); Algorithm 1 is the same for both, with c_p the area centroid of
panel p and one branch per side.
Dense numpy, small meshes only.
"""
import numpy as np

MU0 = 4e-7 * np.pi


def mesh_edges(T):
    """Branches of the PEEC graph: every mesh edge with the two panels that
    share it, (i, j) with i < j (the global current runs from i to j), and
    the edge's vertex pair.  The mesh must be closed and conforming: each
    edge belongs to exactly two panels."""
    T = np.asarray(T)
    owner = {}
    for p, poly in enumerate(T.tolist()):
        poly = [v for v in poly if v >= 0]
        for a in range(len(poly)):
            u, v = poly[a], poly[(a + 1) % len(poly)]
            owner.setdefault((min(u, v), max(u, v)), []).append(p)
    keys = sorted(owner)
    pairs, verts = [], []
    for key in keys:
        ps = owner[key]
        if len(ps) != 2:
            raise ValueError("edge %s belongs to %d panels (closed conforming mesh required)" % (key, len(ps)))
        pairs.append((min(ps), max(ps)))
        verts.append(key)
    return np.array(pairs, dtype=np.int64), np.array(verts, dtype=np.int64)


def centroids(V, T):
    """Area centroid of every panel: the vertex mean of a triangle; for a
    four-sided panel (a, b, c, d) the area-weighted mean of the centroids of
    its triangles (a, b, c) and (a, c, d)."""
    V = np.asarray(V, dtype=np.float64)
    T = np.asarray(T)
    if T.shape[1] == 3:
        return V[T].mean(axis=1)
    c = np.empty((len(T), 3))
    for p, q in enumerate(T.tolist()):
        if q[3] < 0:
            c[p] = V[q[:3]].mean(axis=0)
            continue
        t1, t2 = V[[q[0], q[1], q[2]]], V[[q[0], q[2], q[3]]]
        a1 = 0.5 * np.linalg.norm(np.cross(t1[1] - t1[0], t1[2] - t1[0]))
        a2 = 0.5 * np.linalg.norm(np.cross(t2[1] - t2[0], t2[2] - t2[0]))
        c[p] = (a1 * t1.mean(axis=0) + a2 * t2.mean(axis=0)) / (a1 + a2)
    return c


def cm_maps(V, T, pairs, verts):
    """A_1, A_2, A_3 of Algorithm 1 as dense [3][N_e][N_p] arrays."""
    V = np.asarray(V, dtype=np.float64)
    T = np.asarray(T)
    c = centroids(V, T)
    m = 0.5 * (V[verts[:, 0]] + V[verts[:, 1]])
    Ne, Np = len(pairs), len(T)
    A = np.zeros((3, Ne, Np))
    for e, (i, j) in enumerate(pairs):
        A[:, e, i] += m[e] - c[i]
        A[:, e, j] -= m[e] - c[j]
    return A


def incidence(pairs, n_panels):
    """D[p][e]: +1 where branch e leaves panel p, -1 where it enters."""
    D = np.zeros((n_panels, len(pairs)))
    for e, (i, j) in enumerate(pairs):
        D[i, e] += 1.0
        D[j, e] -= 1.0
    return D


def cycle_space(D, tol=1e-10):
    """Orthonormal basis Q [N_e][r] of the null space of D (the span of
    every loop basis)."""
    u, s, vt = np.linalg.svd(D)
    rank = int(np.sum(s > tol * s.max()))
    return vt[rank:].T


def surface_impedance(f, sigma, thickness):
    """Eq. (3): Z_s = (1+j) R_RF sqrt(f) / (1 - exp(-(1+j) R_RF sqrt(f) / R_DC)),
    R_DC = 2 / (sigma thickness), R_RF = sqrt(pi mu0 / sigma)."""
    f = np.asarray(f, dtype=np.float64)
    r_dc = 2.0 / (sigma * thickness)
    r_rf = np.sqrt(np.pi * MU0 / sigma)
    z = (1 + 1j) * r_rf * np.sqrt(f)
    return z / (-np.expm1(-z / r_dc))


def edge_impedance(P, area, A, alpha, beta):
    """Z_e = sum_t A_t (beta diag(area) + alpha P) A_t^T (dense)."""
    K = beta * np.diag(area) + alpha * P
    return sum(A[t] @ K @ A[t].T for t in range(3))


def loop_solution_edges(Ze, Q, V_edge):
    """I_edge = Q (Q^T Z_e Q)^-1 Q^T V_edge (loop-basis independent)."""
    return Q @ np.linalg.solve(Q.T @ Ze @ Q, Q.T @ V_edge)
