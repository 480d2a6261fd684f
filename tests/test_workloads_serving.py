"""The serving mix's request generator (host only): seeded, Poisson arrivals
at the requested rate, and parameters within the recipe's ranges."""
import numpy as np

import workloads as W


def test_requests_are_reproducible():
    a, b = W.serving_requests(64), W.serving_requests(64)
    assert a == b
    assert W.serving_requests(64, seed=1) != a


def test_arrivals_are_poisson_at_the_rate():
    n, rate = 4000, 200.0
    r = W.serving_requests(n, rate)
    t = np.array([q["arrival"] for q in r])
    gaps = np.diff(t)
    assert t[0] == 0.0 and np.all(gaps >= 0)
    # exponential gaps: mean 1/rate, coefficient of variation 1
    assert abs(gaps.mean() * rate - 1.0) < 0.05
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.05


def test_request_parameters_in_range():
    r = W.serving_requests(512)
    kinds = {q["kind"] for q in r}
    assert kinds == {"blur", "csr"}
    for q in r:
        assert 20 <= q["k"] <= 200 and q["s"] == 2 * (q["k"] + 1)
        assert q["lam"] in (0.0, 1e-3, 1e-2)
        if q["kind"] == "blur":
            assert q["N"] in W.SERVE_BLUR_SIZES and 1.0 <= q["sigma"] <= 6.0
            assert q["r"] == W.radius_for_sigma(q["sigma"]) and q["bc"] in (0, 1)
            assert q["sketch"] == W.SKETCH_SPARSE_SIGN and q["N"] * q["N"] <= 256 * 2048
        else:
            assert q["N"] in W.SERVE_TOMO_SIZES and q["angles"] in W.SERVE_TOMO_ANGLES
            assert q["sketch"] == W.SKETCH_GAUSSIAN


def test_blur_data_matches_its_noise_level():
    q = next(q for q in W.serving_requests(512) if q["kind"] == "blur" and q["N"] == 128)
    b = W.serving_data(q)
    rng = np.random.default_rng(W.PHANTOM_SEED + q["id"])
    x = W.phantom_piecewise(q["N"], q["N"], rng)
    taps = W.gaussian_taps(q["sigma"], q["r"])
    clean = W.blur_apply_scipy(x, taps, taps, q["bc"]).ravel()
    assert abs(np.linalg.norm(b - clean) / np.linalg.norm(clean) - 0.01) < 1e-12
