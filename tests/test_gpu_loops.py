"""GPU tests of the loop formulation around the panel operator (Sec. II-A
Algorithm 1, Sec. II-B eq. (7), Sec. II-C eq. (8)/(9), Sec. II-D eq. (10)/(11)):
the PEEC graph and loop basis are valid (every loop conserves charge at every
panel, the loops are independent and span the cycle space: V - c + 2 g per
surface), the branch-space operator matches the dense FP64 reference, the
loop solve returns the branch currents the reference obtains without any
loop search (they do not depend on the loop basis), and the diagonal-of-P
preconditioner cuts the iteration count."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
from oracle import loops as LO  # noqa: E402
from paper_2409_12375_amd import inputs as I  # noqa: E402
from paper_2409_12375_amd import xrl  # noqa: E402

SIGMA, THICK = 5.96e7, 35e-6  # copper, 35 um
SCALE = 1e-3                  # mesh units: millimetres


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def meshes():
    return {"sphere": (I.icosphere(3, radius=1.0), 0), "torus": (I.torus(), 1),
            "bar": (I.bar(2, 2, 12, size=(1.0, 1.0, 6.0)), 0)}


def coeffs(freqs):
    """alpha = j omega mu0 / 4 pi (the factor taken out of P, Sec. II-D) and
    beta = Z_s of eq. (3), for lengths in millimetres (P scales as L^3, the
    areas as L^2: folded into the coefficients)."""
    f = np.asarray(freqs, dtype=np.float64)
    alpha = 1j * 2 * np.pi * f * LO.MU0 / (4 * np.pi) * SCALE ** 3
    beta = LO.surface_impedance(f, SIGMA, THICK) * SCALE ** 2
    return alpha, beta


def test_surface_impedance_matches_reference():
    f = np.logspace(0, 11, 23)
    z = xrl.surface_impedance(f, SIGMA, THICK)
    ref = LO.surface_impedance(f, SIGMA, THICK)
    assert np.abs(z - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("name", ["sphere", "torus", "bar"])
def test_loop_basis_is_valid(name):
    (V, T), genus = meshes()[name]
    say("case: loop basis, %s (%d panels, genus %d)" % (name, len(T), genus))
    L = xrl.Loops(V, T)
    info = L.info()
    pairs_o, verts_o = LO.mesh_edges(T)
    pairs = L.export(0).reshape(-1, 2)
    verts = L.export(1).reshape(-1, 2)
    assert info["n_edges"] == len(pairs_o)
    # the same branches (panel pair and edge), whatever the order
    key = {tuple(v): e for e, v in enumerate(verts_o.tolist())}
    perm = np.array([key[tuple(v)] for v in verts.tolist()])
    assert np.array_equal(pairs_o[perm], pairs)
    nv = len(np.unique(T))
    assert info["n_loops"] == nv - 1 + 2 * genus
    assert info["n_global_loops"] == 2 * genus
    coo = L.export(2).reshape(-1, 3)
    M = np.zeros((info["n_loops"], info["n_edges"]))
    M[coo[:, 0], coo[:, 1]] = coo[:, 2]
    D = LO.incidence(pairs, len(T))
    assert np.abs(D @ M.T).max() == 0  # charge conserved at every panel
    assert np.linalg.matrix_rank(M) == info["n_loops"]
    say("  %s" % info)


@pytest.mark.parametrize("name", ["sphere", "torus"])
def test_edge_operator_matches_reference(name):
    (V, T), _ = meshes()[name]
    say("case: branch operator, %s" % name)
    N = len(T)
    pairs, verts = LO.mesh_edges(T)
    A = LO.cm_maps(V, T, pairs, verts)
    P = O.dense(V, T)
    area = O.panel_geometry(V, T)[0]
    alpha, beta = coeffs([1e4, 1e6, 1e9])
    L = xrl.Loops(V, T)
    tree = xrl.Tree(V, T, max_leaf=32)
    plan = xrl.Plan(tree, order=8, precision="fp64", max_cols=9)
    plan.assemble()
    rng = np.random.default_rng(4)
    Ie = rng.standard_normal((len(pairs), 3)) + 1j * rng.standard_normal((len(pairs), 3))
    Ve = L.edge_matvec(plan, torch.from_numpy(Ie).cuda(), alpha=alpha, beta=beta).cpu().numpy()
    for c in range(3):
        ref = LO.edge_impedance(P, area, A, alpha[c], beta[c]) @ Ie[:, c]
        e = np.linalg.norm(Ve[:, c] - ref) / np.linalg.norm(ref)
        say("  column %d: rel L2 %.3e" % (c, e))
        assert e <= 1e-4


@pytest.mark.parametrize("name,precond", [("sphere", "none"), ("torus", "none"), ("torus", "diag_p"),
                                          ("bar", "diag_l")])
def test_loop_solve_matches_reference(name, precond):
    """Branch currents of eq. (8) from the GPU loop solve against the dense
    reference on the null space of the incidence (no loop basis)."""
    (V, T), _ = meshes()[name]
    say("case: loop solve, %s, preconditioner %s" % (name, precond))
    pairs, verts = LO.mesh_edges(T)
    A = LO.cm_maps(V, T, pairs, verts)
    P = O.dense(V, T)
    area = O.panel_geometry(V, T)[0]
    Q = LO.cycle_space(LO.incidence(pairs, len(T)))
    alpha, beta = coeffs([1e5, 1e7, 1e9])
    L = xrl.Loops(V, T)
    tree = xrl.Tree(V, T, max_leaf=32)
    plan = xrl.Plan(tree, order=8, precision="fp64", max_cols=9)
    plan.assemble()
    Ve = np.random.default_rng(5).standard_normal((len(pairs), 3)) + 0j
    Ie, st = L.solve(plan, torch.from_numpy(Ve).cuda(), alpha=alpha, beta=beta, precond=precond, rtol=1e-9,
                     max_iter=2000)
    say("  gmres", st)
    assert st["status"] == 0
    Ie = Ie.cpu().numpy()
    for c in range(3):
        ref = LO.loop_solution_edges(LO.edge_impedance(P, area, A, alpha[c], beta[c]), Q, Ve[:, c])
        e = np.linalg.norm(Ie[:, c] - ref) / np.linalg.norm(ref)
        say("  column %d: rel L2 %.3e" % (c, e))
        assert e <= 1e-3


def test_diagonal_of_p_preconditioner_cuts_iterations():
    """Sec. II-D, Table IV: the diagonal-of-P preconditioner cuts the
    iteration count (the ring conductor at 1 GHz: 59 iterations without,
    21 with it, 20 with the diagonal-of-L form measured; the paper's margin
    over diagonal-of-L, 36 against 78 on its package, does not show on this
    small ring)."""
    V, T = I.torus()
    say("case: preconditioners, torus 576, 1 GHz")
    alpha, beta = coeffs([1e9])
    L = xrl.Loops(V, T)
    tree = xrl.Tree(V, T, max_leaf=32)
    plan = xrl.Plan(tree, order=8, precision="mixed", max_cols=3)
    plan.assemble()
    Ve = torch.from_numpy(np.random.default_rng(6).standard_normal((L.info()["n_edges"], 1)) + 0j).cuda()
    its = {}
    for pc in ("none", "diag_l", "diag_p"):
        _, st = L.solve(plan, Ve, alpha=alpha, beta=beta, precond=pc, rtol=1e-6, max_iter=3000)
        assert st["status"] == 0, (pc, st)
        its[pc] = st["iterations"]
    say("  iterations", its)
    assert 2 * its["diag_p"] < its["none"]
    assert 2 * its["diag_l"] < its["none"]
