"""Seeded synthetic inputs: triangle surface meshes and panel densities.

This module holds only input generation (geometry and random numbers).  It
contains none of the operator's arithmetic, so both the GPU path and the CPU
oracle can be fed from it.

The paper's structures (a wire, two square coils, a BGA package and an HBPOP
package, Sec. III) are proprietary or not given; these generators stand in for
them with the same kind of geometry: conductor surfaces meshed into flat
triangles (Sec. II-A), with quasi-uniform panel size.

Every generator returns ``(V, T)``: vertices [nv][3] float64 and triangles
[N][3] int32 (indexed, conforming where the surface is connected).
Geometry seed 2409 (+ mesh index), density seed 12375, numpy PCG64.
"""
import numpy as np

GEOM_SEED = 2409
DENS_SEED = 12375


class _Welder:
    """Collects vertices, merging coincident ones (quantised coordinates)."""

    def __init__(self, tol=1e-9):
        self.tol = tol
        self.map = {}
        self.pts = []

    def add(self, p):
        key = tuple(int(round(c / self.tol)) for c in p)
        idx = self.map.get(key)
        if idx is None:
            idx = len(self.pts)
            self.map[key] = idx
            self.pts.append(np.asarray(p, dtype=np.float64))
        return idx

    def add_many(self, P):
        return np.array([self.add(p) for p in P], dtype=np.int64)

    def vertices(self):
        return np.array(self.pts, dtype=np.float64).reshape(-1, 3)


def _grid_tris(idx, flip=False):
    """Split every quad of an index grid idx[i][j] into two triangles."""
    a = idx[:-1, :-1].ravel()
    b = idx[1:, :-1].ravel()
    c = idx[1:, 1:].ravel()
    d = idx[:-1, 1:].ravel()
    if flip:
        t1 = np.stack([a, c, b], 1)
        t2 = np.stack([a, d, c], 1)
    else:
        t1 = np.stack([a, b, c], 1)
        t2 = np.stack([a, c, d], 1)
    return np.concatenate([t1, t2])


def _grid_quads(idx, flip=False):
    """Every cell of an index grid idx[i][j] as one four-sided panel."""
    a = idx[:-1, :-1].ravel()
    b = idx[1:, :-1].ravel()
    c = idx[1:, 1:].ravel()
    d = idx[:-1, 1:].ravel()
    return np.stack([a, d, c, b] if flip else [a, b, c, d], 1)


def densities(n_panels, n_cols, dtype=np.complex128, seed=DENS_SEED):
    """iid N(0,1) real and imaginary parts, shape [N][n_cols] (panel-major)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    re = rng.standard_normal((n_panels, n_cols))
    im = rng.standard_normal((n_panels, n_cols))
    return (re + 1j * im).astype(dtype)


# --------------------------------------------------------------------------
# straight bar
# --------------------------------------------------------------------------
def bar(nx=4, ny=4, nz=126, size=(1.0, 1.0, 20.0), jitter=0.05, seed=GEOM_SEED, hybrid=False):
    """Surface of the box [0,sx]x[0,sy]x[0,sz] with nx*ny*nz surface cells per
    direction, every quad split in two.  N = 4*(nx*nz + ny*nz + nx*ny).
    Defaults: 1 x 1 x 20 bar, 4096 triangles.

    Vertex jitter is uniform in +-jitter of the local cell size, only along
    the directions in which the vertex is free to move without leaving its
    face (vertices on bar edges slide along the edge, corners stay fixed), so
    the mesh stays flat and conforming.

    hybrid=True: the four long faces keep their cells as four-sided panels
    (rectangles without jitter, planar quadrilaterals with it) and the end
    caps are split into triangles; T is then [N][4] with -1 as the fourth
    index of a triangle, N = 2*(nx*nz + ny*nz) + 4*nx*ny."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sx, sy, sz = size
    n = (nx, ny, nz)
    h = (sx / nx, sy / ny, sz / nz)
    index = {}
    pts = []

    def vid(i, j, k):
        key = (i, j, k)
        v = index.get(key)
        if v is None:
            v = len(pts)
            index[key] = v
            p = [i * h[0], j * h[1], k * h[2]]
            for d, q in enumerate((i, j, k)):
                if 0 < q < n[d]:
                    p[d] += rng.uniform(-jitter, jitter) * h[d]
            pts.append(p)
        return v

    tris = []

    def face(axis, side):
        a1, a2 = [d for d in range(3) if d != axis]
        fixed = 0 if side == 0 else n[axis]
        idx = np.empty((n[a1] + 1, n[a2] + 1), dtype=np.int64)
        for u in range(n[a1] + 1):
            for v in range(n[a2] + 1):
                c = [0, 0, 0]
                c[axis] = fixed
                c[a1] = u
                c[a2] = v
                idx[u, v] = vid(*c)
        # outward normal: e_a1 x e_a2 = +e_axis for (axis,a1,a2) cyclic
        cyc = (a1 - axis) % 3 == 1
        flip = (side == 0) == cyc
        if hybrid and axis != 2:
            tris.append(_grid_quads(idx, flip=flip))
        else:
            t = _grid_tris(idx, flip=flip)
            tris.append(np.concatenate([t, np.full((len(t), 1), -1)], 1) if hybrid else t)

    for axis in range(3):
        for side in (0, 1):
            face(axis, side)
    T = np.concatenate(tris).astype(np.int32)
    return np.array(pts, dtype=np.float64), T


# --------------------------------------------------------------------------
# icosphere
# --------------------------------------------------------------------------
def torus(n_major=24, n_minor=12, R=1.0, r=0.35):
    """Closed genus-1 surface (a ring conductor): quads of a torus split in
    two, consistently oriented."""
    i, j = np.meshgrid(np.arange(n_major), np.arange(n_minor), indexing="ij")
    u = 2 * np.pi * i / n_major
    v = 2 * np.pi * j / n_minor
    V = np.stack([(R + r * np.cos(v)) * np.cos(u), (R + r * np.cos(v)) * np.sin(u), r * np.sin(v)], -1).reshape(-1, 3)
    a = (i * n_minor + j).ravel()
    b = (((i + 1) % n_major) * n_minor + j).ravel()
    c = (((i + 1) % n_major) * n_minor + (j + 1) % n_minor).ravel()
    d = (i * n_minor + (j + 1) % n_minor).ravel()
    T = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)]).astype(np.int32)
    return V, T


def icosphere(level, radius=1.0, center=(0.0, 0.0, 0.0)):
    """Regular icosahedron, each face split into 4 `level` times, vertices
    projected onto the sphere.  N = 20 * 4**level."""
    t = (1.0 + 5 ** 0.5) / 2.0
    V = [[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t],
         [0, -1, -t], [0, 1, -t], [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]]
    V = [np.array(v, dtype=np.float64) / np.linalg.norm(v) for v in V]
    F = [[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4],
         [11, 10, 2], [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8],
         [3, 8, 9], [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = V[a] + V[b]
                V.append(m / np.linalg.norm(m))
                cache[key] = len(V) - 1
            return cache[key]

        nF = []
        for a, b, c in F:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nF += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        F = nF
    Vout = np.array(V) * radius + np.asarray(center, dtype=np.float64)
    return Vout, np.array(F, dtype=np.int32)


# --------------------------------------------------------------------------
# swept rectangular tube along a planar polyline (square spiral coils)
# --------------------------------------------------------------------------
def _rect_ring(nw, nt):
    """Boundary of the unit cross-section [-1,1]x[-1,1] (u in-plane, v along z)
    with nw cells along u and nt along v, counter-clockwise.  Returns [M][2]."""
    pts = []
    for i in range(nw):
        pts.append((-1 + 2 * i / nw, -1))
    for j in range(nt):
        pts.append((1, -1 + 2 * j / nt))
    for i in range(nw):
        pts.append((1 - 2 * i / nw, 1))
    for j in range(nt):
        pts.append((-1, 1 - 2 * j / nt))
    return np.array(pts)


def swept_trace(poly, width, thick, z0, nw, nt, ds, welder):
    """Mesh the surface of a trace of rectangular cross-section width x thick
    whose centre line is the planar polyline `poly` [M][2] at height z0.
    Mitred corners, flat end caps.  Returns triangles (vertex ids in welder)."""
    poly = np.asarray(poly, dtype=np.float64)
    ring = _rect_ring(nw, nt)
    M = len(ring)
    segs = poly[1:] - poly[:-1]
    lens = np.linalg.norm(segs, axis=1)
    dirs = segs / lens[:, None]
    nrm = np.stack([-dirs[:, 1], dirs[:, 0]], 1)
    # corner rings: perpendicular at the two ends, mitred at interior corners
    offs = [nrm[0]]
    for s in range(1, len(segs)):
        n1, n2 = nrm[s - 1], nrm[s]
        offs.append((n1 + n2) / (1.0 + n1 @ n2))
    offs.append(nrm[-1])

    def ring_at(p, off):
        P3 = np.empty((M, 3))
        P3[:, 0:2] = p[None, :] + ring[:, 0:1] * (0.5 * width) * off[None, :]
        P3[:, 2] = z0 + ring[:, 1] * 0.5 * thick
        return P3

    corner = [ring_at(poly[i], offs[i]) for i in range(len(poly))]
    stations = []
    for s in range(len(segs)):
        ns = max(1, int(round(lens[s] / ds)))
        for q in range(ns):
            f = q / ns
            # interpolating the two corner rings keeps every quad of the
            # segment between its two mitre planes (no fold-over at corners)
            stations.append((1.0 - f) * corner[s] + f * corner[s + 1])
    stations.append(corner[-1])
    rings = [welder.add_many(P3) for P3 in stations]
    rings = np.array(rings)  # [S][M]
    idx = np.concatenate([rings, rings[:, :1]], 1)  # close the ring
    tris = [_grid_tris(idx)]
    # end caps: structured grid over the cross-section, boundary shared with ring
    for end, (p, off) in ((0, (poly[0], offs[0])), (1, (poly[-1], offs[-1]))):
        g = np.empty((nw + 1, nt + 1), dtype=np.int64)
        for i in range(nw + 1):
            for j in range(nt + 1):
                u = -1 + 2 * i / nw
                v = -1 + 2 * j / nt
                q = np.array([p[0] + u * 0.5 * width * off[0], p[1] + u * 0.5 * width * off[1],
                              z0 + v * 0.5 * thick])
                g[i, j] = welder.add(q)
        tris.append(_grid_tris(g, flip=(end == 1)))
    return np.concatenate(tris)


def square_spiral(turns, outer, pitch):
    """Centre line of a square spiral: side lengths shrink by `pitch` every
    second side, starting at the outer corner."""
    a = outer / 2.0
    p = np.array([-a, -a])
    pts = [p.copy()]
    dirs = [(1, 0), (0, 1), (-1, 0), (0, -1)]
    for k in range(4 * turns):
        L = outer - (k // 2) * pitch
        p = p + L * np.array(dirs[k % 4], dtype=np.float64)
        pts.append(p.copy())
    return np.array(pts)


def coils(target_n=200_000, turns=5, width=0.1, thick=0.035, spacing=0.1, gap=0.5,
          outer=3.0, nw=8, nt=3):
    """Two identical 5-turn square planar spiral coils stacked along z with
    `gap` between their facing surfaces.  Trace width 0.1, thickness 0.035,
    spacing 0.1 (pitch 0.2).  The along-trace step is chosen so the total panel
    count is close to target_n."""
    pitch = width + spacing
    poly = square_spiral(turns, outer - width, pitch)
    length = np.linalg.norm(poly[1:] - poly[:-1], axis=1).sum()
    per_step = 2 * 2 * (nw + nt)  # triangles per station step per coil
    ds = length / max(1.0, (target_n / 2 - 2 * 2 * nw * nt) / per_step)
    W = _Welder()
    T1 = swept_trace(poly, width, thick, 0.0, nw, nt, ds, W)
    T2 = swept_trace(poly, width, thick, thick + gap, nw, nt, ds, W)
    return W.vertices(), np.concatenate([T1, T2]).astype(np.int32)


# --------------------------------------------------------------------------
# plane with holes, vias and solder balls (BGA-like package)
# --------------------------------------------------------------------------
def _square_ring_cell(cx, cy, half, rh, n_theta, nr, z, welder, flip):
    """Top or bottom face of one square cell of side 2*half with a centred hole
    of radius rh: n_theta points on the circle, the same angles projected onto
    the square, nr quad layers in between (split in two)."""
    th = 2 * np.pi * np.arange(n_theta) / n_theta
    c, s = np.cos(th), np.sin(th)
    m = np.maximum(np.abs(c), np.abs(s))
    circ = np.stack([cx + rh * c, cy + rh * s], 1)
    sq = np.stack([cx + half * c / m, cy + half * s / m], 1)
    idx = np.empty((nr + 1, n_theta + 1), dtype=np.int64)
    for k in range(nr + 1):
        f = k / nr
        P = (1 - f) * circ + f * sq
        ids = welder.add_many(np.column_stack([P, np.full(n_theta, z)]))
        idx[k, :n_theta] = ids
        idx[k, n_theta] = ids[0]
    return _grid_tris(idx, flip=flip)


def _cylinder(cx, cy, r, z0, z1, nfac, nz, welder, caps, flip=False):
    th = 2 * np.pi * np.arange(nfac) / nfac
    ring = np.stack([cx + r * np.cos(th), cy + r * np.sin(th)], 1)
    idx = np.empty((nz + 1, nfac + 1), dtype=np.int64)
    for k in range(nz + 1):
        z = z0 + (z1 - z0) * k / nz
        ids = welder.add_many(np.column_stack([ring, np.full(nfac, z)]))
        idx[k, :nfac] = ids
        idx[k, nfac] = ids[0]
    tris = [_grid_tris(idx, flip=flip)]
    if caps:
        for k, z, fl in ((0, z0, True), (nz, z1, False)):
            ctr = welder.add((cx, cy, z))
            ring_ids = idx[k, :nfac]
            fan = np.stack([np.full(nfac, ctr), ring_ids, np.roll(ring_ids, -1)], 1)
            tris.append(fan[:, [0, 2, 1]] if fl else fan)
    return np.concatenate(tris)


def _holed_plane(n_grid, pitch, hole_r, thick, z0, n_theta, nr, wall_nz, W):
    """Closed surface of a square plane of n_grid x n_grid cells of side
    `pitch`, thickness `thick`, bottom face at z0, with a circular hole of
    radius hole_r in every cell (top and bottom ring faces, hole walls and the
    outer rim).  Returns a list of triangle arrays (vertex ids in W)."""
    half = 0.5 * pitch
    L = n_grid * pitch
    x0 = -0.5 * L
    tris = []
    for i in range(n_grid):
        for j in range(n_grid):
            cx, cy = x0 + (i + 0.5) * pitch, x0 + (j + 0.5) * pitch
            tris.append(_square_ring_cell(cx, cy, half, hole_r, n_theta, nr, z0 + thick, W, flip=False))
            tris.append(_square_ring_cell(cx, cy, half, hole_r, n_theta, nr, z0, W, flip=True))
            tris.append(_cylinder(cx, cy, hole_r, z0, z0 + thick, n_theta, wall_nz, W, caps=False, flip=True))
    # outer rim: the square-boundary points of the border cells, top to bottom
    nside = n_theta // 8  # boundary points per half side of a cell
    for side in range(4):
        pts = []
        for k in range(n_grid):
            for q in range(2 * nside):
                # angles of the projected square points on one cell side
                t = -np.pi / 4 + (np.pi / 2) * q / (2 * nside)
                u = x0 + (k + 0.5) * pitch + half * np.tan(t)
                pts.append(u)
        pts.append(-x0)
        pts = np.array(pts)
        if side == 0:
            P = np.stack([np.full_like(pts, -x0), pts], 1)
        elif side == 1:
            P = np.stack([pts[::-1], np.full_like(pts, -x0)], 1)
        elif side == 2:
            P = np.stack([np.full_like(pts, x0), pts[::-1]], 1)
        else:
            P = np.stack([pts, np.full_like(pts, x0)], 1)
        idx = np.empty((wall_nz + 1, len(P)), dtype=np.int64)
        for k in range(wall_nz + 1):
            z = z0 + thick * k / wall_nz
            idx[k] = W.add_many(np.column_stack([P, np.full(len(P), z)]))
        tris.append(_grid_tris(idx, flip=True))
    return tris


def bga(n_grid=20, pitch=0.5, hole_r=0.2, thick=0.035, n_theta=64, nr=6, wall_nz=3, n_via=10, via_r=0.15,
        via_len=0.5, via_fac=16, via_nz=40, ball_r=0.2, ball_gap=0.1, ball_level=3):
    """BGA-like package: a square plane (n_grid x n_grid cells of side pitch,
    thickness thick) with a circular hole in every cell, cylindrical vias
    (16 facets, capped) through the central n_via x n_via holes without
    contact, and a solder-ball sphere ball_gap below the lower end of every via.
    Defaults: 10 x 10 plane, 400 holes of radius 0.2, 100 vias of radius 0.15
    and length 0.5, 100 balls of radius 0.2; about 1.03M triangles."""
    W = _Welder(tol=1e-10)
    half = 0.5 * pitch
    x0 = -0.5 * n_grid * pitch
    tris = _holed_plane(n_grid, pitch, hole_r, thick, 0.0, n_theta, nr, wall_nz, W)
    # vias through the central holes and balls below them
    first = (n_grid - n_via) // 2
    zmid = 0.5 * thick
    V_off = []
    for i in range(first, first + n_via):
        for j in range(first, first + n_via):
            cx, cy = x0 + (i + 0.5) * pitch, x0 + (j + 0.5) * pitch
            z0, z1 = zmid - 0.5 * via_len, zmid + 0.5 * via_len
            tris.append(_cylinder(cx, cy, via_r, z0, z1, via_fac, via_nz, W, caps=True))
            V_off.append((cx, cy, z0 - ball_gap - ball_r))
    Vs, Ts = icosphere(ball_level, radius=ball_r)
    Vbase = W.vertices()
    T = np.concatenate(tris)
    Vlist = [Vbase]
    Tlist = [T]
    nv = len(Vbase)
    for (cx, cy, cz) in V_off:
        Vlist.append(Vs + np.array([cx, cy, cz]))
        Tlist.append(Ts + nv)
        nv += len(Vs)
    return np.concatenate(Vlist), np.concatenate(Tlist).astype(np.int32)


# --------------------------------------------------------------------------
# batch of uneven meshes
# --------------------------------------------------------------------------
def batch_meshes(n_meshes=32, n_min=10_000, n_max=500_000, seed=GEOM_SEED + 4):
    """Independent meshes of uneven size for the batched matvec: N_i drawn
    log-uniformly in [n_min, n_max], each a bar, a coil pair or a plane with
    holes (seeded choice), meshed close to N_i.  Returns a list of
    (kind, V, T); the meshes are disjoint problems (each has its own P)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n_meshes):
        n = int(round(np.exp(rng.uniform(np.log(n_min), np.log(n_max)))))
        kind = ("bar", "coil", "plane")[int(rng.integers(3))]
        if kind == "bar":
            L = float(rng.uniform(5.0, 20.0))
            k = max(2, int(round(np.sqrt(n / (4.0 * (2.0 * L + 1.0))))))
            V, T = bar(k, k, max(2, int(round(k * L))), size=(1.0, 1.0, L), seed=seed + 100 + i)
        elif kind == "coil":
            small = n < 100_000
            V, T = coils(n, nw=4 if small else 8, nt=2 if small else 3)
        else:
            g = max(2, int(round(np.sqrt(n / 2016.0))))
            V, T = bga(n_grid=g, n_via=0)
        out.append((kind, V, T))
    return out


# --------------------------------------------------------------------------
# package-on-package-like stack
# --------------------------------------------------------------------------
def pop(size=12.0, n_grid=30, gap=1.0, thick=0.035, clear_r=0.15, via_r=0.1, via_fac=16, via_nz=30,
        via_over=0.1, n_theta=32, nr=3, wall_nz=2, trace_w=0.1, trace_ds=0.05, trace_nw=4, trace_nt=2):
    """Package-on-package-like stack: two square planes (size x size,
    thickness thick) `gap` apart (facing surfaces), each with a clearance hole
    of radius clear_r in every one of its n_grid x n_grid cells (pitch
    size / n_grid = 0.4); a via of radius via_r (16 facets, capped) through
    every hole pair without contact, reaching via_over past both planes; and
    two layers of parallel traces of width trace_w between the planes, in
    the channels between the via rows (along x in the lower layer, along y in
    the upper).  Defaults: 900 vias, 2 x 29 traces, about 2.1M triangles."""
    W = _Welder(tol=1e-10)
    pitch = size / n_grid
    x0 = -0.5 * size
    tris = []
    z_lo, z_hi = 0.0, thick + gap  # bottom faces of the two planes
    tris += _holed_plane(n_grid, pitch, clear_r, thick, z_lo, n_theta, nr, wall_nz, W)
    tris += _holed_plane(n_grid, pitch, clear_r, thick, z_hi, n_theta, nr, wall_nz, W)
    for i in range(n_grid):
        for j in range(n_grid):
            cx, cy = x0 + (i + 0.5) * pitch, x0 + (j + 0.5) * pitch
            tris.append(_cylinder(cx, cy, via_r, z_lo - via_over, z_hi + thick + via_over, via_fac, via_nz, W,
                                  caps=True))
    # traces in the channels between via rows, inset from the plane edge
    zt = [thick + gap / 3.0, thick + 2.0 * gap / 3.0]
    end = 0.5 * size - 0.5 * pitch
    for layer, z in enumerate(zt):
        for k in range(1, n_grid):
            c = x0 + k * pitch
            poly = [(-end, c), (end, c)] if layer == 0 else [(c, -end), (c, end)]
            tris.append(swept_trace(poly, trace_w, thick, z, trace_nw, trace_nt, trace_ds, W))
    return W.vertices(), np.concatenate(tris).astype(np.int32)
