"""Pins of the loop-formulation reference (oracle/loops.py) against what the
paper and the mathematics fix, on the CPU:

* Algorithm 1's maps reproduce the panel-integrated current of a uniform
  tangential current density exactly (a closed-form identity of the
  centroid-midpoint transformation: the edge midpoint rule integrates the
  flux of a linear field exactly), which fixes the sign convention, the
  vector rho = m_e - c_p and the indexing;
* the cycle space of the PEEC graph has dimension V - c + 2 g (Euler's
  formula for closed surfaces): 0 handles for spheres, 1 for a torus;
* an explicit integer loop basis built here from vertex fans gives the same
  edge currents as the null-space basis (the loop solution does not depend
  on the basis);
* eq. (3) reaches R_DC at low frequency and (1+j) R_RF sqrt(f) at high
  frequency;
* sum_t A_t P A_t^T is positive definite on the cycle space (Sec. II-D).
"""
import numpy as np
import pytest

import oracle as O
from oracle import hybrid as H
from oracle import loops as LO
from paper_2409_12375_amd import inputs as I


def torus(n_major=16, n_minor=8, R=1.0, r=0.35):
    """Closed genus-1 triangle mesh (quads of a torus split in two)."""
    V = []
    for i in range(n_major):
        u = 2 * np.pi * i / n_major
        for j in range(n_minor):
            v = 2 * np.pi * j / n_minor
            V.append([(R + r * np.cos(v)) * np.cos(u), (R + r * np.cos(v)) * np.sin(u), r * np.sin(v)])
    T = []
    for i in range(n_major):
        for j in range(n_minor):
            a = i * n_minor + j
            b = ((i + 1) % n_major) * n_minor + j
            c = ((i + 1) % n_major) * n_minor + (j + 1) % n_minor
            d = i * n_minor + (j + 1) % n_minor
            T += [[a, b, c], [a, c, d]]
    return np.array(V), np.array(T, dtype=np.int32)


@pytest.mark.parametrize("hybrid", [False, True])
def test_cm_maps_reproduce_uniform_current(hybrid):
    """For every panel p and a constant tangential density J on it, edge
    currents equal to the outward fluxes J . nu_e l_e give
    (A_t^T I_edge)[p] = J_t * area_p (the edge midpoint rule integrates the
    flux of (x - c)_t J exactly on any straight-sided panel, triangle or
    quadrilateral, with c its area centroid)."""
    V, T = I.bar(2, 2, 6, size=(1.0, 1.0, 3.0), jitter=0.1 if hybrid else 0.05, hybrid=hybrid)
    pairs, verts = LO.mesh_edges(T)
    A = LO.cm_maps(V, T, pairs, verts)
    if hybrid:
        area, cen = H.panel_geometry(V, T)
        Tt, owner = H.split(T)
        nrm = O.panel_geometry(V, Tt)[2][np.searchsorted(owner, np.arange(len(T)))]
    else:
        area, cen, nrm, _ = O.panel_geometry(V, T)
    rng = np.random.default_rng(0)
    edge_of = {tuple(vv): e for e, vv in enumerate(verts.tolist())}
    for p in rng.choice(len(T), 40, replace=False):
        J = rng.standard_normal(3)
        J -= nrm[p] * (J @ nrm[p])  # tangential to panel p
        I_edge = np.zeros(len(pairs))
        tri = [v for v in T[p] if v >= 0]
        for a in range(len(tri)):
            u, w = tri[a], tri[(a + 1) % len(tri)]
            e = edge_of[(min(u, w), max(u, w))]
            ev = V[w] - V[u]
            nu = np.cross(ev, nrm[p])
            nu /= np.linalg.norm(nu)
            if nu @ (0.5 * (V[u] + V[w]) - cen[p]) < 0:
                nu = -nu  # outward from panel p
            flux = (J @ nu) * np.linalg.norm(ev)
            I_edge[e] = flux if pairs[e][0] == p else -flux  # global direction i -> j
        got = np.array([A[t].T @ I_edge for t in range(3)])[:, p]
        assert np.allclose(got, J * area[p], rtol=1e-12, atol=1e-12 * np.abs(J).max() * area[p])
    # a panel's rho vectors sum to n (vertex mean - c): zero on a triangle
    # (the midpoints average to the centroid), not on a general quadrilateral
    for p in range(len(T)):
        col = A[:, :, p]
        sgn = np.where(pairs[:, 0] == p, 1.0, np.where(pairs[:, 1] == p, -1.0, 0.0))
        tri = [v for v in T[p] if v >= 0]
        expect = len(tri) * (V[tri].mean(axis=0) - cen[p])
        assert np.allclose((col * sgn[None, :]).sum(axis=1), expect, atol=1e-12)


@pytest.mark.parametrize("mesh,genus", [("sphere", 0), ("bar", 0), ("hybrid bar", 0), ("torus", 1)])
def test_cycle_space_dimension_is_euler(mesh, genus):
    if mesh == "sphere":
        V, T = I.icosphere(2)
    elif mesh == "bar":
        V, T = I.bar(2, 2, 5, size=(1.0, 1.0, 3.0))
    elif mesh == "hybrid bar":
        V, T = I.bar(2, 2, 5, size=(1.0, 1.0, 3.0), hybrid=True)
    else:
        V, T = torus()
    pairs, verts = LO.mesh_edges(T)
    D = LO.incidence(pairs, len(T))
    Q = LO.cycle_space(D)
    nv = len(np.unique(T[T >= 0]))
    assert Q.shape[1] == nv - 1 + 2 * genus
    assert np.abs(D @ Q).max() < 1e-12


def vertex_loops(T, pairs, verts):
    """Integer loop basis from vertex fans (independent construction): the
    panels around each vertex, walked across the edges at that vertex; all
    vertices but the last."""
    edge_of = {tuple(v): e for e, v in enumerate(verts.tolist())}
    around = {}
    for p, tri in enumerate(T.tolist()):
        for v in tri:
            around.setdefault(v, []).append(p)
    rows = []
    for v in sorted(around)[:-1]:
        ps = around[v]
        start = ps[0]
        row = np.zeros(len(pairs))
        cur, came = start, None
        for _ in range(len(ps)):
            tri = T[cur].tolist()
            others = [w for w in tri if w != v]
            nxt_e = None
            for w in others:
                e = edge_of[(min(v, w), max(v, w))]
                if e != came:
                    nxt_e = e
                    break
            i, j = pairs[nxt_e]
            nxt = j if i == cur else i
            row[nxt_e] += 1.0 if i == cur else -1.0
            came, cur = nxt_e, nxt
            if cur == start:
                break
        rows.append(row)
    return np.array(rows)


def test_loop_solution_does_not_depend_on_the_basis():
    V, T = I.icosphere(2, radius=0.5)
    N = len(T)
    pairs, verts = LO.mesh_edges(T)
    A = LO.cm_maps(V, T, pairs, verts)
    D = LO.incidence(pairs, N)
    Q = LO.cycle_space(D)
    M = vertex_loops(T, pairs, verts)
    assert np.abs(M @ D.T).max() == 0 and np.linalg.matrix_rank(M) == Q.shape[1]
    P = O.dense(V, T)
    area = O.panel_geometry(V, T)[0]
    f = 1e9
    Ze = LO.edge_impedance(P, area, A, 1j * 2 * np.pi * f * LO.MU0 / (4 * np.pi),
                           LO.surface_impedance(f, 5.96e7, 35e-6))
    Vedge = np.random.default_rng(1).standard_normal(len(pairs))
    I_q = LO.loop_solution_edges(Ze, Q, Vedge)
    I_m = M.T @ np.linalg.solve(M @ Ze @ M.T, M @ Vedge)
    assert np.linalg.norm(I_q - I_m) <= 1e-10 * np.linalg.norm(I_m)


def test_surface_impedance_limits():
    sigma, th = 5.96e7, 35e-6
    r_dc = 2.0 / (sigma * th)
    r_rf = np.sqrt(np.pi * LO.MU0 / sigma)
    z_lo = LO.surface_impedance(1e-6, sigma, th)
    assert abs(z_lo - r_dc) <= 1e-6 * r_dc
    f = 1e14
    z_hi = LO.surface_impedance(f, sigma, th)
    assert abs(z_hi - (1 + 1j) * r_rf * np.sqrt(f)) <= 1e-9 * abs(z_hi)
    # between the limits: the real part grows monotonically with frequency
    fs = np.logspace(3, 11, 40)
    assert np.all(np.diff(LO.surface_impedance(fs, sigma, th).real) > 0)


def test_edge_operator_positive_on_cycle_space():
    V, T = I.icosphere(2)
    pairs, verts = LO.mesh_edges(T)
    A = LO.cm_maps(V, T, pairs, verts)
    Q = LO.cycle_space(LO.incidence(pairs, len(T)))
    P = O.dense(V, T)
    L = sum(A[t] @ P @ A[t].T for t in range(3))
    ev = np.linalg.eigvalsh(Q.T @ L @ Q)
    assert ev.min() > 0
