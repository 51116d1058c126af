"""Pins of the spherical-harmonics embedding and the view-dependent MLP:
orthonormality on the sphere by product Gauss quadrature, agreement (up to
the sign convention of each function) with scipy's complex spherical
harmonics combined into real ones, and the MLP against explicit loops."""
import numpy as np
import pytest
from scipy import special

from oracle import sh


def _sphere_quadrature(n_theta=12, n_phi=24):
    """Gauss-Legendre in cos(theta) x uniform phi: exact for polynomials of
    degree < 2 n_theta in z and trigonometric degree < n_phi in phi."""
    z, wz = np.polynomial.legendre.leggauss(n_theta)
    phi = 2 * np.pi * np.arange(n_phi) / n_phi
    Z, P = np.meshgrid(z, phi, indexing="ij")
    W = np.repeat(wz[:, None] * (2 * np.pi / n_phi), n_phi, axis=1)
    s = np.sqrt(1 - Z ** 2)
    d = np.stack([s * np.cos(P), s * np.sin(P), Z], axis=-1).reshape(-1, 3)
    return d, W.reshape(-1)


def test_sh_orthonormal_on_sphere():
    d, w = _sphere_quadrature()
    Y = sh.sh16(d)
    G = (Y * w[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def _scipy_real_sh(d):
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    theta = np.arccos(np.clip(z, -1, 1))          # polar
    phi = np.arctan2(y, x)                        # azimuth
    cols = []
    for l in range(4):
        for m in range(-l, l + 1):
            Y = special.sph_harm_y(l, abs(m), theta, phi)
            if m == 0:
                cols.append(Y.real)
            elif m > 0:
                cols.append(np.sqrt(2) * (-1) ** m * Y.real)
            else:
                cols.append(np.sqrt(2) * (-1) ** m * Y.imag)
    return np.stack(cols, axis=1)


def test_sh_matches_scipy_up_to_sign():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(500, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    ours = sh.sh16(d)
    ref = _scipy_real_sh(d)
    for k in range(16):
        s = np.sign(np.dot(ours[:, k], ref[:, k]))
        np.testing.assert_allclose(ours[:, k], s * ref[:, k], atol=1e-12)


def test_sh_normalises_and_handles_degenerate_directions():
    d = np.array([[0.0, 0.0, 2.0], [0.0, 0.0, 1.0], [0.0, 0.0, 0.0], [np.nan, 0, 1]])
    Y = sh.sh16(d)
    np.testing.assert_allclose(Y[0], Y[1], atol=1e-15)
    assert (Y[2] == 0).all() and (Y[3] == 0).all()
    # on the +z axis only the m = 0 functions are non-zero
    m0 = [0, 2, 6, 12]
    assert np.all(np.abs(np.delete(Y[1], m0)) < 1e-15)


def test_view_mlp_matches_explicit_loops():
    rng = np.random.default_rng(1)
    p = rng.normal(size=sh.N_PARAMS_VIEW)
    c_d, f, d = rng.random((5, 3)), rng.normal(size=(5, 4)), rng.normal(size=(5, 3))
    out = sh.mlp_view64(p, c_d, f, d)
    Y = sh.sh16(d)
    W0 = p[:64 * 23].reshape(64, 23)
    o = 64 * 23
    b0 = p[o:o + 64]; o += 64
    W1 = p[o:o + 4096].reshape(64, 64); o += 4096
    b1 = p[o:o + 64]; o += 64
    W2 = p[o:o + 192].reshape(3, 64); o += 192
    b2 = p[o:o + 3]
    for r in range(5):
        x = list(c_d[r]) + list(f[r]) + list(Y[r])
        h1 = [max(0.0, b0[i] + sum(W0[i][k] * x[k] for k in range(23))) for i in range(64)]
        h2 = [max(0.0, b1[i] + sum(W1[i][k] * h1[k] for k in range(64))) for i in range(64)]
        for j in range(3):
            want = b2[j] + sum(W2[j][k] * h2[k] for k in range(64))
            assert abs(out[r, j] - want) < 1e-10
