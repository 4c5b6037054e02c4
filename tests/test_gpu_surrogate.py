"""GPU tests of the learned near-singular surrogate: MFMA layout, feature
invariances, training gradients against the FP64 CPU reference network
(oracle/mlp.py), BF16 inference against the FP32 forward, what a trained
network gains over the cheap rule it corrects, and the assembly with
quadrature fall-back against the FP64 oracle."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
import oracle as O  # noqa: E402
import surrogate_train as S  # noqa: E402
from oracle import mlp as MR  # noqa: E402
from paper_2409_12375_amd import inputs as I  # noqa: E402
from paper_2409_12375_amd import xrl  # noqa: E402

WEIGHTS = os.path.join(os.path.dirname(__file__), "golden", "surrogate_mlp.npz")


def say(*a):
    print(*a, flush=True)


def test_bf16_mfma_layout():
    say("case: bf16 mfma layout")
    rng = np.random.default_rng(3)
    A = rng.standard_normal((16, 16)).astype(np.float32)
    B = rng.standard_normal((16, 16)).astype(np.float32)
    D = np.zeros((16, 16), dtype=np.float32)
    assert xrl.lib().xrl_selftest_mfma_bf16(A.ctypes.data, B.ctypes.data, D.ctypes.data) == 0

    def bf(x):  # round to nearest even, as the kernel does
        u = x.view(np.uint32).astype(np.uint64)
        u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
        return (u.astype(np.uint32) << 16).view(np.float32)

    ref = bf(A).astype(np.float64) @ bf(B).astype(np.float64)
    assert np.allclose(D, ref, rtol=1e-5, atol=1e-5)


def _pairs(n=2000, seed=4):
    V, T = I.coils(60_000, nw=6, nt=2, outer=2.6)
    ks, ls = S.near_singular_pairs(V, T, n, seed)
    return V, T, ks, ls


def test_features_invariances_and_cheap_rule():
    say("case: features")
    V, T, ks, ls = _pairs(500)
    tk = V[T[ks]].reshape(-1, 9)
    tl = V[T[ls]].reshape(-1, 9)
    f0, c0 = S.features(tk, tl)
    f0, c0 = f0.cpu().numpy(), c0.cpu().numpy()
    # vertex order of either triangle does not matter
    tk2 = V[T[ks][:, [2, 0, 1]]].reshape(-1, 9)
    tl2 = V[T[ls][:, [1, 0, 2]]].reshape(-1, 9)
    f1, c1 = S.features(tk2, tl2)
    assert np.allclose(f1.cpu().numpy(), f0, atol=2e-5)
    assert np.allclose(c1.cpu().numpy(), c0, rtol=1e-12)
    # rigid motion and scaling: same features, cheap value scales as L^3
    th = 0.7
    R = np.array([[np.cos(th), -np.sin(th), 0], [np.sin(th), np.cos(th), 0], [0, 0, 1.0]])
    R = R @ np.array([[1, 0, 0], [0, np.cos(0.3), -np.sin(0.3)], [0, np.sin(0.3), np.cos(0.3)]])
    move = lambda t: ((t.reshape(-1, 3, 3) @ R.T) * 2.5 + np.array([3.0, -1.0, 0.5])).reshape(-1, 9)
    f2, c2 = S.features(move(tk), move(tl))
    assert np.allclose(f2.cpu().numpy(), f0, atol=2e-5)
    assert np.allclose(c2.cpu().numpy(), c0 * 2.5 ** 3, rtol=1e-10)
    # the cheap value is the 3x3 conical product rule (same rule as the oracle's far rule with n = 3)
    for i in range(0, 500, 50):
        assert c0[i] == pytest.approx(O.far_pair(tk[i].reshape(3, 3), tl[i].reshape(3, 3), 3), rel=1e-12)


def test_training_gradients_match_cpu_reference():
    say("case: gradients")
    H, n = 64, 300
    rng = np.random.default_rng(5)
    w = (rng.normal(size=xrl.mlp_size(H)) * 0.2).astype(np.float32)
    X = rng.normal(size=(n, 18)).astype(np.float32)
    t = (rng.normal(size=n) * 0.5).astype(np.float32)
    lam, mu, sig, scale = 0.3, -5.0, 2.0, 1e-3
    loss, g = xrl.mlp_loss_grad(torch.from_numpy(w).cuda(), H, torch.from_numpy(X).cuda(),
                                torch.from_numpy(t).cuda(), lam, mu, sig, scale)
    (L0, L1), gref = MR.loss_and_grad(w.astype(np.float64), H, X.astype(np.float64), t.astype(np.float64), lam, mu,
                                      sig, scale)
    assert loss[0] == pytest.approx(L0, rel=1e-4)
    assert loss[1] == pytest.approx(L1, rel=1e-3)
    g = g.cpu().numpy().astype(np.float64)
    err = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    say("  gradient relative error", err)
    assert err < 1e-4


def test_bf16_inference_matches_fp32_forward():
    say("case: bf16 inference")
    H = 128
    w = torch.from_numpy(S.init_weights(H, 7)).cuda()
    V, T, ks, ls = _pairs(3000)
    f, _ = S.features(V[T[ks]].reshape(-1, 9), V[T[ls]].reshape(-1, 9))
    y32 = xrl.mlp_forward(w, H, f, bf16=False).cpu().numpy()
    y16 = xrl.mlp_forward(w, H, f, bf16=True).cpu().numpy()
    rel = np.linalg.norm(y16 - y32, axis=0) / np.linalg.norm(y32, axis=0)
    say("  bf16 vs fp32 relative difference per output", rel)
    assert rel.max() < 2e-2


@pytest.fixture(scope="module")
def small_model():
    sur, info = S.train(n_pairs=200_000, epochs=8, hidden=128, batch=512, seed=99, lr=3e-3, log=say)
    return sur, info


def test_training_converges_and_error_estimate_gates_quadrature(small_model):
    """What the trained network gains over the method without it: the share of
    near-singular pairs whose quadrature it replaces, at an accuracy its own
    error estimate guarantees on pairs it has never seen."""
    say("case: training gain")
    sur, info = small_model
    loss = info["loss"]
    say("  epoch losses", loss)
    # held-out pairs from the benchmark geometry (not in the training meshes)
    V, T = I.coils(200_000)
    ks, ls = S.near_singular_pairs(V, T, 20_000, 123)
    tk, tl = V[T[ks]].reshape(-1, 9), V[T[ls]].reshape(-1, 9)
    ref = O.pairs(V, T, ks, ls)
    f, cheap = S.features(tk, tl)
    out = xrl.mlp_forward(torch.from_numpy(sur.w).cuda(), sur.hidden, f, bf16=True).cpu().numpy()
    cheap = cheap.cpu().numpy()
    e_cheap = np.abs(cheap - ref) / ref
    e_mlp = np.abs(cheap * (1 + out[:, 0]) - ref) / ref
    acc = out[:, 1] <= sur.bound
    bad = (e_mlp[acc] > 10 * 10 ** sur.bound).mean() if acc.any() else 0.0
    say("  median rel error: cheap %.3e  corrected %.3e" % (np.median(e_cheap), np.median(e_mlp)))
    say("  accepted %.1f%% of held-out pairs; of those %.2f%% above 10x the bound (%.0e); 95th pct %.2e" % (
        100 * acc.mean(), 100 * bad, 10 ** sur.bound, np.quantile(e_mlp[acc], 0.95) if acc.any() else np.nan))
    assert loss[-1] < loss[0]
    assert np.median(e_mlp) <= 1.05 * np.median(e_cheap)  # the correction never hurts
    assert acc.mean() > 0.10                            # quadrature avoided on >10% of pairs
    assert bad < 0.02                                    # and the estimate holds on unseen pairs


def test_assembly_with_surrogate_matches_oracle(small_model):
    say("case: assembly with surrogate")
    sur, _ = small_model
    if os.path.exists(WEIGHTS):
        sur = xrl.Surrogate.load(WEIGHTS)
    V, T = I.bar(4, 4, 60, size=(1.0, 1.0, 9.0), seed=11)
    N = len(T)
    x = I.densities(N, 2, np.complex64)
    tree = xrl.Tree(V, T)
    plan = xrl.Plan(tree, order=8, precision="mixed", max_cols=2)
    st = plan.assemble(surrogate=sur, audit_every=10)
    say("  stats", {k: st[k] for k in ("n_near_singular", "n_mlp_accepted", "n_mlp_fallback",
                                         "audit_max_rel_err", "audit_rms_rel_err")})
    # the network is evaluated on the near-singular pairs of rule class 0
    # (r >= 1.5); closer pairs go to quadrature directly
    assert 0 < st["n_mlp_accepted"] + st["n_mlp_fallback"] <= st["n_near_singular"]
    y = plan.matvec(torch.from_numpy(x).cuda()).cpu().numpy()
    rows = np.sort(np.random.default_rng(1).choice(N, 300, replace=False))
    ref, _ = O.matvec(V, T, x.astype(np.complex128), rows=rows)
    err = np.linalg.norm(y[rows] - ref, axis=0) / np.linalg.norm(ref, axis=0)
    say("  rel L2 per column", err)
    assert err.max() < 1e-4
    # a bound below every prediction sends every pair to quadrature: the
    # result then equals the plain assembly bit for bit
    strict = xrl.Surrogate(sur.w, sur.hidden, sur.feat_lo, sur.feat_hi, -99.0)
    plan2 = xrl.Plan(tree, order=8, precision="mixed", max_cols=2)
    st2 = plan2.assemble(surrogate=strict)
    assert st2["n_mlp_accepted"] == 0
    plan3 = xrl.Plan(tree, order=8, precision="mixed", max_cols=2)
    plan3.assemble()
    y2 = plan2.matvec(torch.from_numpy(x).cuda())
    y3 = plan3.matvec(torch.from_numpy(x).cuda())
    assert torch.equal(y2, y3)
