"""Pins of the hybrid-mesh reference (oracle/hybrid.py, rectangles and
triangles, Sec. II-A, Fig. 1) against what the mathematics fixes, on the CPU:

* the self term of an a x b rectangle equals its closed form
  4 int_0^a int_0^b (a-u)(b-v)/sqrt(u^2+v^2) du dv, written out here from
  four elementary integrals (not the oracle's triangle formulas);
* the mutual terms of rectangles that share an edge or a corner follow from
  the same closed form by additivity: a 2a x b rectangle is two a x b ones,
  so I(2a, b) = 2 I(a, b) + 2 M_edge, and a 2a x 2b one gives the corner term;
* the entries do not depend on which diagonal splits a four-sided panel;
* a mesh of triangles given in the [N][4] form gives the triangle oracle's
  matrix; the matvec equals the dense product.
"""
import numpy as np
import pytest

import oracle as O
from oracle import hybrid as H
from paper_2409_12375_amd import inputs as I


def rect_self(a, b):
    d = np.hypot(a, b)
    j0 = a * np.log((b + d) / a) + b * np.log((a + d) / b)  # int int 1/r
    ju = b * d / 2 + a * a / 2 * np.log((b + d) / a) - b * b / 2  # int int u/r
    jv = a * d / 2 + b * b / 2 * np.log((a + d) / b) - a * a / 2  # int int v/r
    juv = (d ** 3 - a ** 3 - b ** 3) / 3  # int int u v/r
    return 4.0 * (a * b * j0 - a * jv - b * ju + juv)


def rotation(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((3, 3)))
    return q


def grid_panels(nx, ny, a, b, seed):
    """nx x ny rectangles of a x b as four-sided panels, rotated and moved."""
    Rm = rotation(seed)
    shift = np.random.default_rng(seed + 1).standard_normal(3)
    V = np.array([[i * a, j * b, 0.0] for j in range(ny + 1) for i in range(nx + 1)]) @ Rm.T + shift
    vid = lambda i, j: j * (nx + 1) + i  # noqa: E731
    T = np.array([[vid(i, j), vid(i + 1, j), vid(i + 1, j + 1), vid(i, j + 1)]
                  for j in range(ny) for i in range(nx)], dtype=np.int32)
    return V, T


def test_closed_form_reference_values():
    # unit square: (4/3)(1 - sqrt 2) + 4 ln(1 + sqrt 2), the classical value
    assert abs(rect_self(1.0, 1.0) - (4.0 / 3.0 * (1 - np.sqrt(2)) + 4 * np.log(1 + np.sqrt(2)))) < 1e-14
    # homogeneity of degree 3
    assert abs(rect_self(2.0, 1.0) - 8 * rect_self(1.0, 0.5)) < 1e-12


@pytest.mark.parametrize("a,b", [(1.0, 1.0), (2.0, 0.5), (0.3, 1.7)])
def test_rectangle_self_term_matches_closed_form(a, b):
    V, T = grid_panels(1, 1, a, b, seed=3)
    ref = rect_self(a, b)
    assert abs(H.dense(V, T)[0, 0] - ref) <= 1e-9 * ref
    # the other diagonal
    T2 = T[:, [1, 2, 3, 0]]
    assert abs(H.dense(V, T2)[0, 0] - ref) <= 1e-9 * ref


@pytest.mark.parametrize("a,b", [(1.0, 1.0), (0.7, 0.4)])
def test_edge_and_corner_neighbours_from_the_closed_form(a, b):
    V, T = grid_panels(2, 2, a, b, seed=5)  # panels 0 1 / 2 3
    P = H.dense(V, T)
    s = rect_self(a, b)
    m_x = rect_self(2 * a, b) / 2 - s  # neighbours along the a side
    m_y = rect_self(a, 2 * b) / 2 - s
    m_c = (rect_self(2 * a, 2 * b) - 4 * s - 4 * m_x - 4 * m_y) / 4
    tol = 1e-9 * rect_self(2 * a, 2 * b)
    assert np.abs(np.diag(P) - s).max() <= tol
    assert abs(P[0, 1] - m_x) <= tol and abs(P[2, 3] - m_x) <= tol
    assert abs(P[0, 2] - m_y) <= tol and abs(P[1, 3] - m_y) <= tol
    assert abs(P[0, 3] - m_c) <= tol and abs(P[1, 2] - m_c) <= tol
    assert np.abs(P - P.T).max() <= tol


def test_split_diagonal_does_not_change_entries():
    """Planar quadrilaterals (a jittered hybrid bar face): splitting every
    four-sided panel along its other diagonal leaves P unchanged."""
    V, T = I.bar(2, 2, 4, size=(1.0, 1.0, 2.0), jitter=0.15, hybrid=True)
    T2 = T.copy()
    q = T[:, 3] >= 0
    T2[q] = T[q][:, [1, 2, 3, 0]]
    P1, P2 = H.dense(V, T), H.dense(V, T2)
    assert np.abs(P1 - P2).max() <= 1e-9 * np.abs(P1).max()


def test_triangles_in_the_four_index_form():
    V, T = I.bar(2, 2, 3, size=(1.0, 1.0, 1.5))
    T4 = np.concatenate([T, np.full((len(T), 1), -1)], 1)
    assert np.array_equal(H.dense(V, T4), O.dense(V, T))


def test_hybrid_matvec_equals_dense():
    V, T = I.bar(2, 2, 6, size=(1.0, 1.0, 3.0), hybrid=True)
    x = I.densities(len(T), 2)
    y, _ = H.matvec(V, T, x)
    assert np.abs(y - H.dense(V, T) @ x).max() <= 1e-12 * np.abs(y).max()
    rows = np.array([0, 5, 17, 63])
    yr, _ = H.matvec(V, T, x, rows=rows)
    assert np.abs(yr - y[rows]).max() <= 1e-12 * np.abs(y).max()
    # areas and centroids: the rectangles of the long faces are 0.5 x 0.5
    area, cen = H.panel_geometry(V, T)
    assert abs(area.sum() - (4 * 3.0 + 2 * 1.0)) < 1e-12
