"""GPU parity of the FMM panel matvec against the FP64 CPU oracle.

The oracle (oracle/) evaluates P_kl = int_Sk int_Sl 1/|r-r'| (arXiv
2409.12375 eq. (6), second term) by direct summation; the GPU path applies P
with the FMM of Sec. II-C.  Gate: max over complex columns of the relative L2
error on the sampled rows <= 1e-4 (the FMM truncation at p = 8 and the
quadrature of the stored near field are the only differences)."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import oracle as O  # noqa: E402
from paper_2409_12375_amd import inputs as I  # noqa: E402
from paper_2409_12375_amd import xrl  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def relerr_cols(y, ref):
    y = np.asarray(y).reshape(len(ref), -1)
    ref = np.asarray(ref).reshape(len(ref), -1)
    return np.linalg.norm(y - ref, axis=0) / np.linalg.norm(ref, axis=0)


def sample_rows(N, m, seed=5):
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(N, size=min(m, N), replace=False))


def bar_mixed_sphere():
    """Adaptive test geometry: a bar with a finely meshed sphere beside it."""
    V1, T1 = I.bar(2, 2, 10, size=(1.0, 1.0, 5.0))
    V2, T2 = I.icosphere(3, radius=0.3, center=(1.6, 0.5, 2.5))
    V = np.vstack([V1, V2])
    T = np.vstack([T1, T2 + len(V1)]).astype(np.int32)
    return V, T


def test_mfma_operand_layout():
    say("case: mfma layout")
    L = xrl.lib()
    L.xrl_selftest_mfma.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    rng = np.random.default_rng(0)
    for eb, dt in ((4, np.float32), (8, np.float64)):
        A = rng.standard_normal((16, 4)).astype(dt)
        B = rng.standard_normal((4, 16)).astype(dt)
        D = np.zeros((16, 16), dtype=dt)
        assert L.xrl_selftest_mfma(eb, A.ctypes.data, B.ctypes.data, D.ctypes.data) == 0
        tol = 1e-5 if eb == 4 else 1e-13
        assert np.allclose(D, A.astype(np.float64) @ B.astype(np.float64), rtol=tol, atol=tol)
    # 16 blocks of 4x4x1 (the columns past the last full tile)
    L.xrl_selftest_mfma_4x4.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    A = rng.standard_normal((16, 4)).astype(np.float32)
    B = rng.standard_normal((16, 4)).astype(np.float32)
    D = np.zeros((16, 4, 4), dtype=np.float32)
    assert L.xrl_selftest_mfma_4x4(A.ctypes.data, B.ctypes.data, D.ctypes.data) == 0
    ref = A.astype(np.float64)[:, :, None] * B.astype(np.float64)[:, None, :]
    assert np.allclose(D, ref, rtol=1e-6, atol=1e-6)


def test_interaction_lists_cover_every_pair_exactly_once():
    say("case: list coverage, bar + sphere, max_leaf 8")
    V, T = bar_mixed_sphere()
    tree = xrl.Tree(V, T, max_leaf=8)
    assert tree.info()["depth"] >= 4
    plan = xrl.Plan(tree, order=4, precision="fp64", max_cols=1)
    N = len(T)
    rng_ = plan.export(1).reshape(-1, 2)
    rows = plan.export(3)
    src = plan.export(4)
    pairs = plan.export(5).reshape(-1, 2)
    leaf_box = plan.export(6)
    cover = np.zeros((N, N), dtype=np.int32)
    for li, b in enumerate(leaf_box):
        t0, t1 = rng_[b]
        s = src[rows[li]:rows[li + 1]]
        assert len(np.unique(s)) == len(s)
        cover[t0:t1, s] += 1
    for tb, sb in pairs:
        cover[rng_[tb][0]:rng_[tb][1], rng_[sb][0]:rng_[sb][1]] += 1
    assert cover.min() == 1 and cover.max() == 1
    info = plan.info()
    assert info["n_m2l_pairs"] > 0 and info["max_sep_ratio"] < 1.0


def _run(V, T, x, precision, order=8, max_leaf=64, engine="auto", r_near=2.0):
    tree = xrl.Tree(V, T, max_leaf=max_leaf)
    plan = xrl.Plan(tree, order=order, precision=precision, engine=engine, max_cols=x.shape[1])
    st = plan.assemble(r_near=r_near)
    xt = torch.from_numpy(x).cuda()
    y = plan.matvec(xt)
    torch.cuda.synchronize()
    return plan, y.cpu().numpy(), st


@pytest.mark.parametrize("precision,engine,dtype,tol", [
    ("fp64", "auto", np.complex128, 2e-5),
    ("mixed", "auto", np.complex64, 5e-5),
    ("fp32", "auto", np.complex64, 5e-5),
    ("mixed", "valu", np.complex64, 5e-5),
    ("mixed", "mfma_ts", np.complex64, 5e-5),
    ("fp64", "mfma_ts", np.complex128, 2e-5),
])
def test_bar_matvec_matches_oracle(precision, engine, dtype, tol):
    say("case: bar 4096, %s/%s" % (precision, engine))
    V, T = I.bar()
    N = len(T)
    x = I.densities(N, 3, dtype)
    plan, y, st = _run(V, T, x, precision, engine=engine)
    assert st["n_self"] == N
    # every unpadded near pair falls in exactly one class; the finer
    # regular rule takes the pairs below r_mid
    assert st["n_self"] + st["n_touching"] + st["n_near_singular"] + st["n_regular"] == plan.info()["n_near_pairs"]
    assert 0 < st["n_regular_fine"] < st["n_regular"]
    rows = sample_rows(N, 384)
    ref, _ = O.matvec(V, T, x.astype(np.complex128), rows=rows)
    err = relerr_cols(y[rows], ref)
    say("  rel L2 per column", err)
    assert err.max() <= tol


def test_wide_columns_target_stationary_matches_oracle_and_offset_stationary():
    """18 complex columns (36 real: three 16-column tiles, the last one
    partial) through the target-stationary translations, against the oracle
    and against the offset-stationary kernels on the same plan."""
    say("case: bar 4096, 18 columns, mixed, target- vs offset-stationary")
    V, T = I.bar()
    N = len(T)
    x = I.densities(N, 18, np.complex64)
    tree = xrl.Tree(V, T)
    ys = {}
    forms = ("mfma", "mfma_os", "refl", "lean", "p2p_scalar", "p2p_lds", "padded", "refl_padded", "l2l_ts", "m2m_ts",
             "m2m_tiles", "valu_leaf", "valu", "valu_tiles", "l2l_leaves")
    for eng in forms:
        engine = eng if eng in ("mfma_os", "valu") else ("valu" if eng == "valu_tiles" else "mfma")
        plan = xrl.Plan(tree, order=8, precision="mixed", engine=engine, max_cols=18)
        plan.assemble()
        if eng in ("padded", "refl_padded"):  # the last four columns in a padded 16-column tile
            plan.set_tuning("ts_narrow_cols", 0)
        if eng in ("refl", "refl_padded"):  # the reflected 64-operator table
            plan.set_tuning("ts_kernel", 1)
        if eng == "lean":  # two waves per SIMD, no explicit pipeline
            plan.set_tuning("ts_kernel", 2)
        if eng == "p2p_scalar":  # P2P on the vector ALU with wave-uniform scalar densities
            plan.set_tuning("p2p_form", 1)
        if eng == "p2p_lds":  # P2P on the vector ALU with the densities staged in LDS
            plan.set_tuning("p2p_form", 2)
        if eng == "l2l_ts":  # L2L target-stationary instead of source-stationary
            plan.set_tuning("l2l_form", 0)
        if eng == "m2m_ts":  # M2M one wave per target on every level
            plan.set_tuning("m2m_form", 0)
        if eng == "m2m_tiles":  # M2M one wave per row tile on every level
            plan.set_tuning("m2m_form", 1)
        if eng == "valu_tiles":  # vector-ALU translations as 6 x 4 register tiles
            plan.set_tuning("valu_form", 0)
        if eng == "l2l_leaves":  # L2L into the leaves too (L2P without the parent term)
            plan.set_tuning("leaf_l2l", 0)
        if eng == "valu_leaf":  # P2P, P2M and L2P on the vector ALU
            plan.set_tuning("leaf_form", 0)
            plan.set_tuning("p2p_form", 2)
        ys[eng] = plan.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
        plan.close()
    rows = sample_rows(N, 256)
    ref, _ = O.matvec(V, T, x.astype(np.complex128), rows=rows)
    err = relerr_cols(ys["mfma"][rows], ref)
    say("  rel L2 per column (target-stationary)", err.max())
    assert err.max() <= 5e-5
    d = np.linalg.norm(ys["mfma"] - ys["mfma_os"], axis=0) / np.linalg.norm(ys["mfma_os"], axis=0)
    say("  target- vs offset-stationary", d.max())
    assert d.max() < 1e-6
    for v in forms[2:]:
        d = np.linalg.norm(ys["mfma"] - ys[v], axis=0) / np.linalg.norm(ys[v], axis=0)
        say("  kernel form %s vs default" % v, d.max())
        assert d.max() < 1e-6


@pytest.mark.parametrize("ncomplex", [9, 10, 17])
def test_narrow_columns_past_the_last_tile(ncomplex):
    """C = 16 n + 2 or + 4 real columns: the columns past the last full tile
    on 4x4 MFMA blocks (default), against the padded tile, the
    offset-stationary kernels and the oracle."""
    say("case: bar 4096, %d columns, narrow columns on 4x4 blocks" % ncomplex)
    V, T = I.bar()
    N = len(T)
    x = I.densities(N, ncomplex, np.complex64, seed=40 + ncomplex)
    tree = xrl.Tree(V, T)
    ys = {}
    for v in ("narrow", "padded", "refl", "mfma_os"):
        plan = xrl.Plan(tree, order=8, precision="mixed", engine="mfma_os" if v == "mfma_os" else "mfma",
                        max_cols=ncomplex)
        plan.assemble()
        if v == "padded":
            plan.set_tuning("ts_narrow_cols", 0)
        if v == "refl":
            plan.set_tuning("ts_kernel", 1)
        ys[v] = plan.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
        plan.close()
    for v in ("padded", "refl", "mfma_os"):
        d = np.linalg.norm(ys["narrow"] - ys[v], axis=0) / np.linalg.norm(ys[v], axis=0)
        say("  narrow vs %s" % v, d.max())
        assert d.max() < 1e-6
    rows = sample_rows(N, 64)
    ref, _ = O.matvec(V, T, x.astype(np.complex128), rows=rows)
    err = relerr_cols(ys["narrow"][rows], ref)
    say("  rel L2 per column", err.max())
    assert err.max() <= 5e-5


@pytest.mark.parametrize("order", [6, 10])
def test_other_orders_matrix_core_forms_match_vector_forms(order):
    """Orders 6 (49 coefficients, last row on the vector ALU) and 10 (121, no
    separate row) at 18 complex columns: the matrix-core forms (target- and
    source-stationary translations with 4x4 narrow columns, MFMA P2P, P2M,
    L2P) against the offset-stationary M2L with every leaf phase on the
    vector ALU, and against the oracle within the order's truncation."""
    say("case: bar 4096, order %d, 18 columns, matrix-core vs vector forms" % order)
    V, T = I.bar()
    N = len(T)
    x = I.densities(N, 18, np.complex64, seed=60 + order)
    tree = xrl.Tree(V, T)
    ys = {}
    for v in ("mfma", "vector"):
        plan = xrl.Plan(tree, order=order, precision="mixed", engine="mfma_os" if v == "vector" else "mfma",
                        max_cols=18)
        plan.assemble()
        if v == "vector":
            plan.set_tuning("p2p_form", 2)
            plan.set_tuning("leaf_form", 0)
        ys[v] = plan.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
        plan.close()
    d = np.linalg.norm(ys["mfma"] - ys["vector"], axis=0) / np.linalg.norm(ys["vector"], axis=0)
    say("  matrix-core vs vector forms", d.max())
    assert d.max() < 1e-6
    rows = sample_rows(N, 64)
    ref, _ = O.matvec(V, T, x.astype(np.complex128), rows=rows)
    err = relerr_cols(ys["mfma"][rows], ref)
    say("  rel L2 per column", err.max())
    assert err.max() <= (3e-4 if order == 6 else 1e-5)


@pytest.mark.parametrize("precision,ncomplex", [("mixed", 18), ("fp64", 3)])
def test_leaves_of_128_panels(precision, ncomplex):
    """max_leaf = 128 (near-field blocks 128 targets wide): every P2P form,
    P2M and L2P against the vector forms and the oracle."""
    say("case: bar 4096, max_leaf 128, %s, %d columns" % (precision, ncomplex))
    V, T = I.bar()
    N = len(T)
    dt = np.complex128 if precision == "fp64" else np.complex64
    x = I.densities(N, ncomplex, dt, seed=70 + ncomplex)
    tree = xrl.Tree(V, T, max_leaf=128)
    tp = None
    ys = {}
    for v in (("mfma", "scalar", "vector") if precision == "mixed" else ("auto",)):
        plan = xrl.Plan(tree, order=8, precision=precision, engine="mfma_os" if v == "vector" else "auto",
                        max_cols=ncomplex)
        plan.assemble()
        tp = plan.export(9)
        if v == "scalar":
            plan.set_tuning("p2p_form", 1)
        if v == "vector":
            plan.set_tuning("p2p_form", 2)
            plan.set_tuning("leaf_form", 0)
        ys[v] = plan.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
        plan.close()
    # blocks wider than 64 targets, and widths that end inside a 16-target tile
    assert tp.max() > 64 and np.all(tp % 4 == 0) and np.any(tp % 16 != 0)
    first = next(iter(ys))
    for v in ys:
        if v != first:
            d = np.linalg.norm(ys[first] - ys[v], axis=0) / np.linalg.norm(ys[v], axis=0)
            say("  %s vs %s" % (first, v), d.max())
            assert d.max() < 1e-6
    rows = sample_rows(N, 64)
    ref, _ = O.matvec(V, T, x.astype(np.complex128), rows=rows)
    err = relerr_cols(ys[first][rows], ref)
    say("  rel L2 per column", err.max())
    assert err.max() <= (2e-5 if precision == "fp64" else 5e-5)


@pytest.mark.parametrize("engine", ["auto", "mfma_ts"])
def test_adaptive_tree_matvec_matches_oracle(engine):
    say("case: bar + sphere adaptive, fp64, max_leaf 16, %s" % engine)
    V, T = bar_mixed_sphere()
    N = len(T)
    x = I.densities(N, 2)
    plan, y, _ = _run(V, T, x, "fp64", max_leaf=16, engine=engine)
    ref, _ = O.matvec(V, T, x)
    err = relerr_cols(y, ref)
    say("  rel L2 per column", err)
    assert err.max() <= 2e-5


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_near_field_entries_match_oracle(precision):
    """Stored near-field entries against the oracle, by pair class: FP64
    everywhere to 1e-8; mixed precision stores FP32, with the self and
    touching entries integrated in FP64 (to FP32 rounding) and the others in
    FP32."""
    say("case: near-field entries %s" % precision)
    V, T = I.bar(2, 2, 12, size=(1.0, 1.0, 6.0))
    tree = xrl.Tree(V, T, max_leaf=16)
    plan = xrl.Plan(tree, order=4, precision=precision, max_cols=1)
    plan.assemble()
    perm = plan.export(0)
    rng_ = plan.export(1).reshape(-1, 2)
    rows = plan.export(3)
    src = plan.export(4)
    leaf_box = plan.export(6)
    tpad = plan.export(9)
    vals = np.frombuffer(plan.export(8).tobytes(), dtype=np.float64)
    rng = np.random.default_rng(2)
    off = 0
    worst = {}
    for li, b in enumerate(leaf_box):
        t0, t1 = rng_[b]
        nr = rows[li + 1] - rows[li]
        blk = vals[off:off + nr * tpad[li]].reshape(nr, tpad[li])
        off += nr * tpad[li]
        for _ in range(4):
            r = rng.integers(nr)
            j = rng.integers(t1 - t0)
            k, l = perm[t0 + j], perm[src[rows[li] + r]]
            ref = O.entry(V, T, k, l)
            shared = len(set(T[k]) & set(T[l]))
            cls = "self" if k == l else ("touch" if shared else "other")
            e = abs(blk[r, j] - ref) / abs(ref)
            worst[cls] = max(worst.get(cls, 0), e)
    say("  worst relative entry error by class", worst)
    if precision == "fp64":
        assert max(worst.values()) < 1e-8
    else:
        # FP64 results stored in FP32: within two FP32 rounding steps
        assert worst.get("self", 0) < 3e-7 and worst.get("touch", 0) < 3e-7 and worst.get("other", 0) < 1e-5


def test_linearity_determinism_and_epilogue():
    say("case: linearity / determinism / epilogue, mixed")
    V, T = I.bar(4, 4, 40, size=(1.0, 1.0, 6.0))
    N = len(T)
    tree = xrl.Tree(V, T)
    plan = xrl.Plan(tree, order=8, precision="mixed", max_cols=4)
    plan.assemble()
    a = torch.from_numpy(I.densities(N, 2, np.complex64, seed=1)).cuda()
    b = torch.from_numpy(I.densities(N, 2, np.complex64, seed=2)).cuda()
    ya = plan.matvec(a).clone()
    ya2 = plan.matvec(a).clone()
    assert torch.equal(ya, ya2)  # bitwise deterministic
    yb = plan.matvec(b).clone()
    s, t = 0.7 - 0.2j, -1.3 + 0.5j
    yab = plan.matvec(s * a + t * b)
    lin = (torch.linalg.norm(yab - (s * ya + t * yb)) / torch.linalg.norm(yab)).item()
    assert lin < 1e-5
    al = np.array([2.0 + 1.0j, -0.5j])
    be = np.array([0.3 - 0.1j, 1.5])
    ye = plan.matvec(a, alpha=al, beta=be).cpu().numpy()
    area, _, _, _ = O.panel_geometry(V, T)
    expect = ya.cpu().numpy() * al[None, :] + area[:, None] * a.cpu().numpy() * be[None, :]
    assert np.abs(ye - expect).max() <= 1e-5 * np.abs(expect).max()
    # a single column and a strided view give the same numbers
    y1 = plan.matvec(a[:, 1]).cpu().numpy()
    assert np.allclose(y1, ya[:, 1].cpu().numpy(), rtol=1e-6, atol=1e-6 * np.abs(y1).max())


def test_batched_plan_equals_separate_plans():
    say("case: batched plan of three meshes")
    meshes = [I.bar(2, 2, 20, size=(1.0, 1.0, 5.0)), I.icosphere(3, 0.7), I.bar(3, 2, 15, size=(1.5, 1.0, 4.0))]
    trees = [xrl.Tree(V, T) for V, T in meshes]
    plan = xrl.Plan(trees, order=8, precision="fp64", max_cols=2)
    plan.assemble()
    Ns = [len(T) for _, T in meshes]
    x = I.densities(sum(Ns), 2)
    y = plan.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    off = 0
    for (V, T), n in zip(meshes, Ns):
        ref, _ = O.matvec(V, T, x[off:off + n])
        assert relerr_cols(y[off:off + n], ref).max() < 2e-5
        off += n


def test_gmres_recovers_known_solution():
    say("case: gmres")
    V, T = I.bar(3, 3, 30, size=(1.0, 1.0, 5.0))
    N = len(T)
    tree = xrl.Tree(V, T)
    plan = xrl.Plan(tree, order=8, precision="fp64", max_cols=3)
    plan.assemble()
    xt = torch.from_numpy(I.densities(N, 3)).cuda()
    alpha = np.array([1.0, 1j, 0.5 + 0.5j])
    beta = np.array([0.0, 0.3, 2.0 - 1.0j])
    b = plan.matvec(xt, alpha=alpha, beta=beta).clone()
    x, st = plan.gmres(b, alpha=alpha, beta=beta, restart=30, rtol=1e-10, max_iter=300)
    say("  gmres stats", st)
    assert st["status"] == 0 and st["converged"] == 3
    err = (torch.linalg.norm(x - xt, dim=0) / torch.linalg.norm(xt, dim=0)).max().item()
    assert err < 1e-6
    # forced non-convergence is reported, not raised
    x1, st1 = plan.gmres(b, alpha=alpha, beta=beta, restart=5, rtol=1e-12, max_iter=1)
    assert st1["status"] == -5 and st1["iterations"] == 1


def test_graph_replay_matches_eager_every_time():
    """Graph mode: the captured matvec is replayed several times with eager
    work and synchronisations in between; every replay equals the eager
    result bit for bit, also with a changed epilogue and a new argument set."""
    say("case: graph replay, bar 4096, mixed, 3 columns")
    V, T = I.bar()
    N = len(T)
    x = torch.from_numpy(I.densities(N, 3, np.complex64)).cuda()
    tree = xrl.Tree(V, T)
    plan = xrl.Plan(tree, order=8, precision="mixed", max_cols=3)
    plan.assemble()
    y_eager = plan.matvec(x)
    y_ep = plan.matvec(x, alpha=[1 + 2j, 0.5, -1j], beta=0.25)
    torch.cuda.synchronize()
    plan.set_graph(True)
    y = torch.empty_like(x)
    for rep in range(4):
        plan.matvec(x, y)
        z = (x * 3).sum()  # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(y, y_eager), rep
        assert torch.isfinite(z.real)
    y.zero_()
    for rep in range(3):
        plan.matvec(x, y, alpha=[1 + 2j, 0.5, -1j], beta=0.25)
        torch.cuda.synchronize()
        assert torch.equal(y, y_ep), rep
    y2 = torch.empty_like(x)  # new argument set: recaptured
    for rep in range(2):
        plan.matvec(x, y2)
        torch.cuda.synchronize()
        assert torch.equal(y2, y_eager), rep


def test_autotune_keeps_the_fastest_form_and_the_result():
    say("case: autotune, bar 4096, mixed, 18 columns")
    V, T = I.bar()
    N = len(T)
    x = torch.from_numpy(I.densities(N, 18, np.complex64)).cuda()
    tree = xrl.Tree(V, T)
    plan = xrl.Plan(tree, order=8, precision="mixed", max_cols=18)
    plan.assemble()
    y0 = plan.matvec(x)
    r = plan.autotune(x, reps=2)
    say("  tried", r["tried"], "best", r["best"])
    assert len(r["tried"]) in (3, 4)
    assert len(r["p2p_tried"]) == 3 and r["best_p2p_form"] in (0, 1, 2)
    assert r["best"][2] == min(t[2] for t in r["tried"])
    y1 = plan.matvec(x)
    torch.cuda.synchronize()
    d = (torch.linalg.norm(y1 - y0, dim=0) / torch.linalg.norm(y0, dim=0)).max().item()
    assert d < 1e-6


def test_many_columns_several_items_per_target():
    """96 complex columns (192 real): the target-stationary translations split
    every target into several column items and P2P into several column tiles;
    against the offset-stationary kernels and against the oracle."""
    say("case: bar 4096, 96 columns, several items per target")
    V, T = I.bar()
    N = len(T)
    x = I.densities(N, 96, np.complex64, seed=31)
    tree = xrl.Tree(V, T)
    ys = {}
    for eng in ("mfma", "mfma_os"):
        plan = xrl.Plan(tree, order=8, precision="mixed", engine=eng, max_cols=96)
        plan.assemble()
        ys[eng] = plan.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
        plan.close()
    d = np.linalg.norm(ys["mfma"] - ys["mfma_os"], axis=0) / np.linalg.norm(ys["mfma_os"], axis=0)
    say("  target- vs offset-stationary", d.max())
    assert d.max() < 1e-6
    rows = sample_rows(N, 64)
    ref, _ = O.matvec(V, T, x.astype(np.complex128), rows=rows)
    err = relerr_cols(ys["mfma"][rows], ref)
    say("  rel L2 per column: max", err.max(), "median", np.median(err))
    assert err.max() <= 5e-5


def test_densities_not_aligned_to_complex_pairs():
    """x handed over the C ABI 4 bytes off an 8-byte boundary: the gather
    takes its scalar-load form and the product equals the aligned call's."""
    say("case: bar 4096, 5 columns, x at a 4-byte offset")
    V, T = I.bar()
    N = len(T)
    nc = 5
    x = I.densities(N, nc, np.complex64, seed=41)
    tree = xrl.Tree(V, T)
    plan = xrl.Plan(tree, order=8, precision="mixed", max_cols=nc)
    plan.assemble()
    xd = torch.from_numpy(x).cuda()
    y_ref = plan.matvec(xd).cpu().numpy()
    # the same values, interleaved (re, im), one float after an aligned start
    buf = torch.zeros(2 * N * nc + 1, dtype=torch.float32, device="cuda")
    buf[1:] = torch.view_as_real(xd).reshape(-1)
    y = torch.empty_like(xd)
    torch.cuda.synchronize()
    code = xrl.lib().xrl_fmm_matvec(plan.h, ctypes.c_void_p(buf.data_ptr() + 4), nc, nc, xrl.C64,
                                    ctypes.c_void_p(y.data_ptr()), nc, None, xrl._stream(None))
    torch.cuda.synchronize()
    assert code == 0, xrl.lib().xrl_last_error()
    d = np.abs(y.cpu().numpy() - y_ref).max()
    say("  max |difference| from the aligned call", d)
    assert d == 0.0
    plan.close()
