"""Pin of the view-dependent MLP's adjoint (Eq. 5; supplement "Network
Design"): dL/dC_d, dL/dF and dL/dpsi of L = sum(g * rgb) against central
finite differences of the float64 forward."""
import numpy as np

from oracle import sh


def _loss(params, c_d, feat, d, g):
    rgb = 1.0 / (1.0 + np.exp(-(c_d + sh.mlp_view64(params, c_d, feat, d))))
    return float((g * rgb).sum())


def test_view_mlp_adjoint_matches_finite_differences():
    rng = np.random.default_rng(4)
    m = 37
    params = rng.normal(0.0, 0.3, size=5891)
    c_d = rng.random((m, 3))
    feat = rng.normal(0.0, 0.5, size=(m, 4))
    d = rng.normal(size=(m, 3))
    d[0] = 0.0                                   # zero direction: SH = 0
    g = rng.normal(size=(m, 3))
    g_cd, g_f, g_p = sh.mlp_view_backward64(params, c_d, feat, d, g)
    h = 1e-6
    for arr, grad in ((c_d, g_cd), (feat, g_f)):
        for idx in [(0, 0), (5, 1), (m - 1, 2)]:
            a0 = arr[idx]
            arr[idx] = a0 + h
            lp = _loss(params, c_d, feat, d, g)
            arr[idx] = a0 - h
            lm = _loss(params, c_d, feat, d, g)
            arr[idx] = a0
            assert abs((lp - lm) / (2 * h) - grad[idx]) < 1e-6 * (1 + abs(grad[idx]))
    # weights and biases of every layer (W0, b0, W1, b1, W2, b2 blocks)
    for j in [0, 100, 23 * 64 - 1, 23 * 64 + 5, 23 * 64 + 64 + 777, 23 * 64 + 64 + 4096 + 10,
              5891 - 3 - 1, 5891 - 1]:
        p0 = params[j]
        params[j] = p0 + h
        lp = _loss(params, c_d, feat, d, g)
        params[j] = p0 - h
        lm = _loss(params, c_d, feat, d, g)
        params[j] = p0
        assert abs((lp - lm) / (2 * h) - g_p[j]) < 1e-6 * (1 + abs(g_p[j])), j
