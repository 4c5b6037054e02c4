"""CPU pins of the FP64 reference network used to check the GPU training
kernels: its analytic gradient equals central finite differences of the loss
(with the calibration target held fixed, as the training defines it)."""
import numpy as np

from oracle import mlp as M


def _setup(H=8, n=40, seed=0):
    rng = np.random.default_rng(seed)
    size = H * H + 22 * H + 2
    w = rng.normal(size=size) * 0.3
    X = rng.normal(size=(n, 18))
    t = rng.normal(size=n) * 0.5
    return w, X, t


def test_gradient_matches_finite_differences():
    H = 8
    w, X, t = _setup(H)
    lam, mu, sig, scale = 0.3, -5.0, 2.0, 1e-3
    (L0, L1), g = M.loss_and_grad(w, H, X, t, lam, mu, sig, scale)
    y, _ = M.forward(w, H, X)
    g_fixed = (np.log10(scale * np.abs(y[:, 0] - t) / M.rho4(X) + 1e-12) - mu) / sig
    assert abs(M.total_loss(w, H, X, t, lam, mu, sig, scale, g_fixed) - (L0 + lam * L1)) < 1e-12
    rng = np.random.default_rng(1)
    idx = rng.choice(len(w), 60, replace=False)
    h = 1e-6
    for i in idx:
        wp = w.copy()
        wm = w.copy()
        wp[i] += h
        wm[i] -= h
        fd = (M.total_loss(wp, H, X, t, lam, mu, sig, scale, g_fixed)
              - M.total_loss(wm, H, X, t, lam, mu, sig, scale, g_fixed)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])), (i, fd, g[i])


def test_pack_unpack_roundtrip_and_silu():
    H = 5
    w, _, _ = _setup(H)
    assert np.array_equal(M.pack(M.unpack(w, H)), w)
    z = np.linspace(-6, 6, 101)
    assert np.allclose(M.silu(z), z * 1 / (1 + np.exp(-z)))
    hh = 1e-6
    assert np.allclose(M.dsilu(z), (M.silu(z + hh) - M.silu(z - hh)) / (2 * hh), atol=1e-8)
