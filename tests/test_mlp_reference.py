"""Pin the FP64 MLP reference (used to check the device gradients) against
central finite differences."""
import numpy as np

import mlp_reference as mr


def test_reference_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    d_in, width, L = 5, 7, 4
    n = sum(o * i + o for o, i in mr.shapes(d_in, width, L))
    p = rng.normal(0, 0.5, n)
    X = rng.normal(size=(9, d_in))
    t = rng.normal(size=9)
    loss, g = mr.loss_and_grad(p, X, t, d_in, width, L)
    h = 1e-6
    for k in rng.choice(n, 40, replace=False):
        e = np.zeros(n)
        e[k] = h
        lp, _ = mr.loss_and_grad(p + e, X, t, d_in, width, L)
        lm, _ = mr.loss_and_grad(p - e, X, t, d_in, width, L)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[k]) <= 1e-7 * max(1.0, abs(fd))
