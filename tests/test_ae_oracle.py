"""Pins for the autoencoder oracle (CPU): finite differences, closed forms and
the bfloat16 rounding rule."""
import numpy as np
import pytest

from oracle import ae


def _rand_params(seed=0, scale=0.3):
    rng = np.random.default_rng(seed)
    p = {}
    for l in range(4):
        fin, fout = ae.DIMS[l], ae.DIMS[l + 1]
        p[f"W{l + 1}"] = rng.normal(0, scale, (fout, fin))
        p[f"b{l + 1}"] = rng.normal(0, 0.1, fout)
    return p


def test_finite_differences_fp64():
    """Central differences in FP64 agree with the analytic gradients."""
    rng = np.random.default_rng(1)
    p = _rand_params(1)
    X = rng.normal(0, 1, (7, 64))
    _, g = ae.loss_and_grads(p, X)
    h = 1e-4   # central differences: truncation O(h^2), roundoff O(eps*L/h)
    for k in p:
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, 6, replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = ae.loss_and_grads(p, X)
            flat[idx] = old - h
            lm, _ = ae.loss_and_grads(p, X)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * abs(an) + 1e-10, (k, idx, fd, an)


def test_constant_output_closed_form():
    """All weights zero: the output is b4, the loss is mean((b4 - x)^2) and
    dL/db4 = 2 * mean over rows of (b4 - x) / 64."""
    rng = np.random.default_rng(2)
    p = {f"W{l + 1}": np.zeros((ae.DIMS[l + 1], ae.DIMS[l])) for l in range(4)}
    p.update({f"b{l + 1}": np.zeros(ae.DIMS[l + 1]) for l in range(4)})
    c = rng.normal(0, 1, 64)
    p["b4"] = c
    X = rng.normal(0, 1, (5, 64))
    loss, g = ae.loss_and_grads(p, X)
    assert loss == pytest.approx(((c - X) ** 2).mean(), rel=1e-14)
    np.testing.assert_allclose(g["b4"], 2 * (c - X).sum(0) / (5 * 64), rtol=1e-13)
    for k in ("W1", "W2", "W3", "b1", "b2", "b3"):
        assert not g[k].any()
    np.testing.assert_allclose(g["W4"], 0.0)     # hidden activations are zero


def test_first_adam_step_is_sign_step():
    p = {"w": np.array([1.0, -2.0, 3.0])}
    g = {"w": np.array([0.5, -4.0, 1e-3])}
    m = {"w": np.zeros(3)}
    v = {"w": np.zeros(3)}
    p, m, v = ae.adam_update(p, g, m, v, 1, lr=0.01)
    np.testing.assert_allclose(p["w"], [1.0 - 0.01, -2.0 + 0.01, 3.0 - 0.01], rtol=1e-6)


def test_bf16_rounding_ties_to_even():
    one = 1.0
    vals = np.array([one, one + 2 ** -8, one + 3 * 2 ** -8, one + 2 ** -7, -(one + 2 ** -8),
                     3.140625, 1e-30], np.float64)
    r = ae.to_bf16(vals)
    assert r[0] == 1.0
    assert r[1] == 1.0                       # midpoint -> even mantissa
    assert r[2] == one + 2 ** -6             # midpoint -> even mantissa
    assert r[3] == one + 2 ** -7             # representable
    assert r[4] == -1.0
    assert r[5] == 3.140625                  # 7 mantissa bits: exact
    assert abs(r[6] - 1e-30) / 1e-30 < 2 ** -8


def test_xavier_init_bounds_and_moments():
    p = ae.init_params(123)
    for l in range(4):
        W = p[f"W{l + 1}"]
        a = np.sqrt(6.0 / (ae.DIMS[l] + ae.DIMS[l + 1]))
        assert W.shape == (ae.DIMS[l + 1], ae.DIMS[l])
        assert np.abs(W).max() <= a
        assert abs(W.mean()) < 0.05 * a
        assert abs(W.var() / (a * a / 3) - 1) < 0.1
    q = ae.init_params(123)
    assert all(np.array_equal(p[k], q[k]) for k in p)
    assert not np.array_equal(p["W1"], ae.init_params(124)["W1"])


def test_training_reduces_loss():
    """Adam on low-rank data: the loss falls well below its starting value."""
    rng = np.random.default_rng(3)
    basis = rng.normal(0, 1, (4, 64))
    X = rng.normal(0, 1, (512, 4)) @ basis
    p = ae.init_params(7)
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(v) for k, v in p.items()}
    l0, _ = ae.loss_and_grads(p, X)
    for t in range(1, 301):
        batch = X[rng.choice(512, 64, replace=False)]
        _, g = ae.loss_and_grads(p, batch)
        p, m, v = ae.adam_update(p, g, m, v, t, lr=3e-3)
    l1, _ = ae.loss_and_grads(p, X)
    assert l1 < 0.3 * l0


def test_bf16_mode_close_to_fp64():
    rng = np.random.default_rng(4)
    p = ae.init_params(5)
    X = rng.normal(0, 1, (64, 64))
    l64, g64 = ae.loss_and_grads(p, X)
    l16, g16 = ae.loss_and_grads(p, X, bf16=True)
    assert abs(l16 - l64) / l64 < 2e-2
    for k in g64:
        if k.startswith("W"):
            rel = np.linalg.norm(g16[k] - g64[k]) / np.linalg.norm(g64[k])
            assert rel < 5e-2, k


def test_fit_norm_and_scores():
    rng = np.random.default_rng(5)
    T = rng.integers(0, 1000, (6, 5, 64)).astype(np.int64)
    it = np.array([5, 5, 3, 0, 5, 1])
    mu, sd = ae.fit_norm([T], [it])
    valid = np.arange(5)[None, :] < it[:, None]
    x = T[valid].astype(np.float64)
    np.testing.assert_allclose(mu, x.mean(0), rtol=1e-6)
    np.testing.assert_allclose(sd, x.std(0), rtol=1e-6)
    p = ae.init_params(1)
    s = ae.rank_scores(p, T, it, mu, sd)
    assert s[3] == 0.0 and (s[[0, 1, 2, 4, 5]] > 0).all()
    # closed form with a network that outputs a constant c: residual score is
    # max_g |c_g - mean_i x|, error score max_g mean_i (c_g - x)^2
    z = {k: np.zeros_like(v) for k, v in p.items()}
    c = np.linspace(-1, 1, 64)
    z["b4"] = c
    X = ae.normalize(T, mu, sd).astype(np.float64)
    s0 = ae.rank_scores(z, T, it, mu, sd, kind=0)
    s1 = ae.rank_scores(z, T, it, mu, sd, kind=1)
    for r in (0, 2, 5):
        x = X[r, :it[r]]
        assert s0[r] == pytest.approx(((c - x) ** 2).mean(0).max(), rel=1e-12)
        assert s1[r] == pytest.approx(np.abs((c - x).mean(0)).max(), rel=1e-12)


def test_robust_z_textbook_cases():
    """Odd and even medians, the mean-absolute-deviation fallback and the
    all-equal case, worked by hand."""
    v = np.array([1.0, 2.0, 3.0, 4.0, 100.0])          # median 3, MAD 1
    np.testing.assert_allclose(ae.robust_z(v), (v - 3.0) / 1.4826, rtol=1e-15)
    v = np.array([4.0, 1.0, 2.0, 3.0])                  # median 2.5, MAD 1
    np.testing.assert_allclose(ae.robust_z(v), (v - 2.5) / 1.4826, rtol=1e-15)
    v = np.array([5.0, 5.0, 5.0, 9.0])                  # MAD 0, mean AD 1
    np.testing.assert_allclose(ae.robust_z(v), (v - 5.0) / 1.253314, rtol=1e-15)
    assert not ae.robust_z(np.full(7, 2.0)).any()


def test_robust_z32_textbook_cases():
    """The FP32 second stage on hand-worked samples, and agreement with the
    FP64 definition to FP32 rounding on a random one."""
    f = np.float32
    v = np.array([1, 2, 3, 4, 100], np.float32)          # median 3, MAD 1
    assert np.array_equal(ae.robust_z32(v), ((v - f(3)) / f(1.4826)).astype(np.float32))
    v = np.array([4, 1, 2, 3], np.float32)                 # median 2.5, MAD 1
    assert np.array_equal(ae.robust_z32(v), ((v - f(2.5)) / f(1.4826)).astype(np.float32))
    v = np.array([5, 5, 5, 9], np.float32)                 # MAD 0, mean AD 1
    assert np.array_equal(ae.robust_z32(v), ((v - f(5)) / f(1.253314)).astype(np.float32))
    assert not ae.robust_z32(np.full(7, 2.0, np.float32)).any()
    r = np.random.default_rng(3).normal(0, 1, 1001).astype(np.float32)
    np.testing.assert_allclose(ae.robust_z32(r), ae.robust_z(r.astype(np.float64)), rtol=1e-5,
                               atol=1e-6)


def test_residual_z_score_equals_exact_totals_scan(oracle):
    """With a network that outputs zeros, m(r,g) = -mean_i x(r,i,g), an
    increasing affine map of the rank total S(r,g) when every rank has the
    same number of iterations; the robust |z| is invariant under such maps,
    so the kind-2 score equals the C oracle's exact TOTALS robust scan."""
    rng = np.random.default_rng(11)
    R, I, G = 40, 6, 64
    T = rng.gamma(4.0, 2.5e4, (R, I, G)).astype(np.int64)
    T[3, :, 7] *= 3                                      # a slow region
    T[:, :, 9] = 1000                                    # constant region: z = 0
    T[:30, :, 10] = 500                                  # MAD 0, mean AD > 0
    it = np.full(R, I, np.int32)
    mu, sd = ae.fit_norm([T], [it])
    zero = {k: np.zeros_like(v) for k, v in ae.init_params(0).items()}
    got = ae.rank_scores(zero, T, it, mu, sd, kind=2)
    st, score, flag, nf, reg = oracle.outliers(T, it, mode=1, kind=0, tau=3.5)
    assert st == 0
    np.testing.assert_allclose(got, score, rtol=2e-5, atol=1e-6)
    # ranks without iterations take no part and score 0
    it2 = it.copy()
    it2[[0, 5]] = 0
    got2 = ae.rank_scores(zero, T, it2, mu, sd, kind=2)
    assert got2[0] == 0.0 and got2[5] == 0.0
    keep = np.ones(R, bool)
    keep[[0, 5]] = False
    sub = ae.rank_scores(zero, T[keep], it[keep], mu, sd, kind=2)
    assert np.array_equal(got2[keep], sub)


def test_gaussian_noise_moments_and_determinism():
    """The counter-based normal draws: deterministic per (key, row, feature),
    different keys give uncorrelated draws, and over 64k draws the sample
    moments are those of N(0, 1) within a few standard errors (mean, variance,
    skewness 0, kurtosis 3, P(|z| > 1.96) = 0.05)."""
    a = ae.gaussian_noise(12345, np.arange(1000))
    assert a.shape == (1000, 64)
    assert np.array_equal(a, ae.gaussian_noise(12345, np.arange(1000)))
    assert np.array_equal(a[[7, 3]], ae.gaussian_noise(12345, [7, 3]))
    z = a.reshape(-1)
    n = z.size
    assert abs(z.mean()) < 4 / np.sqrt(n)
    assert abs(z.var() - 1) < 4 * np.sqrt(2 / n)
    assert abs((z ** 3).mean()) < 4 * np.sqrt(15 / n)
    assert abs((z ** 4).mean() - 3) < 4 * np.sqrt(96 / n)
    tail = (np.abs(z) > 1.959963984540054).mean()
    assert abs(tail - 0.05) < 4 * np.sqrt(0.05 * 0.95 / n)
    b = ae.gaussian_noise(54321, np.arange(1000)).reshape(-1)
    assert abs(np.corrcoef(z, b)[0, 1]) < 4 / np.sqrt(n)
    # neighbouring features and rows are uncorrelated too
    assert abs(np.corrcoef(a[:, :-1].reshape(-1), a[:, 1:].reshape(-1))[0, 1]) < 4 / np.sqrt(n)
    assert abs(np.corrcoef(a[:-1].reshape(-1), a[1:].reshape(-1))[0, 1]) < 4 / np.sqrt(n)


def test_denoising_gradient_finite_differences():
    """With a corrupted input the gradient is still that of the loss against
    the clean rows (central differences), and it differs from the plain one."""
    rng = np.random.default_rng(4)
    p = _rand_params(4)
    X = rng.normal(0, 1, (6, 64))
    Xn = X + 0.5 * ae.gaussian_noise(99, np.arange(6))
    l0, g = ae.loss_and_grads(p, X, X_in=Xn)
    _, g_plain = ae.loss_and_grads(p, X)
    assert not np.allclose(g["W1"], g_plain["W1"])
    h = 1e-4
    for k in ("W1", "b2", "W4"):
        flat = p[k].reshape(-1)
        for idx in rng.choice(flat.size, 4, replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = ae.loss_and_grads(p, X, X_in=Xn)
            flat[idx] = old - h
            lm, _ = ae.loss_and_grads(p, X, X_in=Xn)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert abs(fd - an) <= 1e-6 * abs(an) + 1e-10, (k, idx, fd, an)
