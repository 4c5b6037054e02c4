"""Plain FP64 reference of the panel operator on hybrid meshes of triangles and
rectangles (TEST INFRASTRUCTURE ONLY: tests may import this module, the
library never does).

What it computes, from the paper (arXiv 2409.12375): Sec. II-A discretises
the conductor surface into a hybrid mesh of triangles and rectangles (Fig. 1,
Fig. 2) and puts one pulse function on each panel, so the Galerkin entry of
eq. (6) (second term) between panels k and l is the double integral of 1/R
over the two panel surfaces, whatever their shape.

A four-sided panel (a, b, c, d) is the union of the triangles (a, b, c) and
(a, c, d).  The double integral is additive over a partition of either
surface, so

    P_kl = sum over triangles s of k, sum over triangles t of l of P_st,

with P_st the triangle entries of the FP64 oracle (oracle.c): P = S P_tri S^T
with S the 0/1 panel-triangle membership.  Panel area and centroid are the
sums and the area-weighted centroid of its triangles.

Panels are given as an int array [N][4]; a row whose last index is negative
is a triangle.
"""
import numpy as np

import oracle as O


def split(T4):
    """Triangles of every panel, in panel order, and the owning panel of each
    triangle."""
    T4 = np.asarray(T4)
    if T4.shape[1] == 3:
        return np.ascontiguousarray(T4, dtype=np.int32), np.arange(len(T4))
    tris, owner = [], []
    for p, q in enumerate(T4.tolist()):
        tris.append(q[:3])
        owner.append(p)
        if q[3] >= 0:
            tris.append([q[0], q[2], q[3]])
            owner.append(p)
    return np.array(tris, dtype=np.int32), np.array(owner)


def panel_geometry(V, T4):
    """Area and area-weighted centroid of every panel."""
    Tt, owner = split(T4)
    a, c, _, _ = O.panel_geometry(V, Tt)
    n = len(T4)
    area = np.bincount(owner, weights=a, minlength=n)
    cen = np.stack([np.bincount(owner, weights=a * c[:, d], minlength=n) for d in range(3)], 1) / area[:, None]
    return area, cen


def membership(T4):
    """S [N_panels][N_triangles]."""
    Tt, owner = split(T4)
    S = np.zeros((len(T4), len(Tt)))
    S[owner, np.arange(len(Tt))] = 1.0
    return S


def dense(V, T4):
    """P = S P_tri S^T (small meshes only)."""
    Tt, owner = split(T4)
    S = membership(T4)
    return S @ O.dense(V, Tt) @ S.T


def matvec(V, T4, x, rows=None, nthreads=0):
    """y[rows] = P[rows, :] x for panel densities x [N] or [N][C] (real or
    complex).  Returns (y, threads_used)."""
    Tt, owner = split(T4)
    n = len(T4)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    x = np.asarray(x)
    xt = x[owner]  # each triangle carries its panel's density (pulse basis)
    want = np.isin(owner, rows)
    trows = np.nonzero(want)[0]
    yt, th = O.matvec(V, Tt, xt, rows=trows, nthreads=nthreads)
    yt = np.asarray(yt).reshape(len(trows), -1)
    pos = {p: i for i, p in enumerate(rows.tolist())}
    y = np.zeros((len(rows), yt.shape[1]), dtype=yt.dtype)
    np.add.at(y, [pos[p] for p in owner[trows].tolist()], yt)
    return (y[:, 0] if x.ndim == 1 else y), th

