"""GPU parity on hybrid meshes of triangles and four-sided panels (Sec. II-A,
Fig. 1: rectangles on the long faces of a bar, triangles on its caps).

The library sorts elements (the two triangles of every four-sided panel) and
sums their potentials back into the panel; the reference is the FP64 hybrid
oracle (oracle/hybrid.py: the panel entry as the sum of the triangle entries
of oracle.c, pinned by the rectangle closed forms on the CPU).  Gate as for
triangles: per complex column, relative L2 <= the FMM tolerance."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
from oracle import hybrid as H  # noqa: E402
from oracle import loops as LO  # noqa: E402
from paper_2409_12375_amd import inputs as I  # noqa: E402
from paper_2409_12375_amd import xrl  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def relerr_cols(y, ref):
    y = np.asarray(y).reshape(len(ref), -1)
    ref = np.asarray(ref).reshape(len(ref), -1)
    return np.linalg.norm(y - ref, axis=0) / np.linalg.norm(ref, axis=0)


@pytest.mark.parametrize("precision,dtype,tol", [("fp64", np.complex128, 2e-5), ("mixed", np.complex64, 5e-5),
                                                 ("fp32", np.complex64, 5e-5)])
def test_hybrid_bar_matvec_matches_oracle(precision, dtype, tol):
    V, T = I.bar(4, 4, 40, size=(1.0, 1.0, 6.0), hybrid=True)
    N = len(T)
    nq = int((T[:, 3] >= 0).sum())
    say("case: hybrid bar, %d panels (%d four-sided), %s" % (N, nq, precision))
    tree = xrl.Tree(V, T, max_leaf=32)
    ti = tree.info()
    assert ti["n_panels"] == N and ti["n_elements"] == N + nq
    plan = xrl.Plan(tree, order=8, precision=precision, max_cols=3)
    st = plan.assemble()
    pi = plan.info()
    assert pi["n_panels"] == N and pi["n_elements"] == N + nq
    assert st["n_self"] == N + nq
    x = I.densities(N, 3, dtype)
    y = plan.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    ref, _ = H.matvec(V, T, x.astype(np.complex128))
    err = relerr_cols(y, ref)
    say("  rel L2 per column", err)
    assert err.max() <= tol
    # the epilogue uses the panel area (both triangles)
    area, _ = H.panel_geometry(V, T)
    ye = plan.matvec(torch.from_numpy(x).cuda(), alpha=0.0, beta=1.0).cpu().numpy()
    assert np.abs(ye - area[:, None] * x).max() <= 1e-6 * np.abs(area[:, None] * x).max()


def test_batched_plan_of_a_hybrid_and_a_triangle_mesh():
    meshes = [I.bar(2, 2, 20, size=(1.0, 1.0, 5.0), hybrid=True), I.icosphere(3, 0.7),
              I.bar(3, 2, 15, size=(1.5, 1.0, 4.0), hybrid=True)]
    say("case: batched plan, hybrid + triangles + hybrid")
    trees = [xrl.Tree(V, T) for V, T in meshes]
    plan = xrl.Plan(trees, order=8, precision="fp64", max_cols=2)
    plan.assemble()
    Ns = [len(T) for _, T in meshes]
    x = I.densities(sum(Ns), 2)
    y = plan.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    off = 0
    for (V, T), n in zip(meshes, Ns):
        ref, _ = H.matvec(V, T, x[off:off + n])
        e = relerr_cols(y[off:off + n], ref).max()
        say("  mesh of %d panels: %.3e" % (n, e))
        assert e < 2e-5
        off += n


def test_hybrid_gmres_against_the_oracle_operator():
    V, T = I.bar(2, 2, 10, size=(1.0, 1.0, 4.0), hybrid=True)
    N = len(T)
    say("case: gmres on a hybrid bar of %d panels" % N)
    tree = xrl.Tree(V, T, max_leaf=32)
    plan = xrl.Plan(tree, order=8, precision="fp64", max_cols=2)
    plan.assemble()
    P = H.dense(V, T)
    area, _ = H.panel_geometry(V, T)
    alpha, beta = np.array([1.0, 0.5j]), np.array([0.2, 1.0 - 0.3j])
    b = I.densities(N, 2)
    x, st = plan.gmres(torch.from_numpy(b).cuda(), alpha=alpha, beta=beta, restart=50, rtol=1e-8, max_iter=400)
    assert st["status"] == 0
    x = x.cpu().numpy()
    for c in range(2):
        Aop = beta[c] * np.diag(area) + alpha[c] * P
        r = np.linalg.norm(b[:, c] - Aop @ x[:, c]) / np.linalg.norm(b[:, c])
        say("  column %d: residual against the oracle operator %.3e" % (c, r))
        assert r <= 1e-4


@pytest.mark.parametrize("precond", ["none", "diag_p", "diag_l"])
def test_hybrid_loops_match_reference(precond):
    """Loop analysis on the hybrid bar: one branch per panel side, the fan
    of every vertex, N_l = N_e - N_p + 1; the loop solve against the dense
    reference (Algorithm 1 with area centroids, eq. (8))."""
    V, T = I.bar(2, 2, 8, size=(1.0, 1.0, 4.0), hybrid=True)
    say("case: loops on a hybrid bar (%d panels), %s" % (len(T), precond))
    pairs, verts = LO.mesh_edges(T)
    L = xrl.Loops(V, T)
    info = L.info()
    assert info["n_edges"] == len(pairs)
    assert info["n_loops"] == len(pairs) - len(T) + 1
    coo = L.export(2).reshape(-1, 3)
    M = np.zeros((info["n_loops"], info["n_edges"]))
    M[coo[:, 0], coo[:, 1]] = coo[:, 2]
    gp = L.export(0).reshape(-1, 2)
    assert np.abs(LO.incidence(gp, len(T)) @ M.T).max() == 0
    A = LO.cm_maps(V, T, pairs, verts)
    P = H.dense(V, T)
    area, _ = H.panel_geometry(V, T)
    Q = LO.cycle_space(LO.incidence(pairs, len(T)))
    f = np.array([1e6, 1e9])
    alpha = 1j * 2 * np.pi * f * LO.MU0 / (4 * np.pi) * 1e-9
    beta = LO.surface_impedance(f, 5.96e7, 35e-6) * 1e-6
    tree = xrl.Tree(V, T, max_leaf=32)
    plan = xrl.Plan(tree, order=8, precision="fp64", max_cols=6)
    plan.assemble()
    # the library's branches in the reference's order
    key = {tuple(v): e for e, v in enumerate(verts.tolist())}
    perm = np.array([key[tuple(v)] for v in L.export(1).reshape(-1, 2).tolist()])
    Ve = np.random.default_rng(7).standard_normal((len(pairs), 2)) + 0j
    Ie, st = L.solve(plan, torch.from_numpy(Ve[perm]).cuda(), alpha=alpha, beta=beta, precond=precond, rtol=1e-9,
                     max_iter=2000)
    say("  gmres", st)
    assert st["status"] == 0
    Ie = Ie.cpu().numpy()
    for c in range(2):
        ref = LO.loop_solution_edges(LO.edge_impedance(P, area, A, alpha[c], beta[c]), Q, Ve[:, c])
        e = np.linalg.norm(Ie[:, c] - ref[perm]) / np.linalg.norm(ref)
        say("  column %d: rel L2 %.3e" % (c, e))
        assert e <= 1e-3
