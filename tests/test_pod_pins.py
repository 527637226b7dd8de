"""Pins of the oracle POD (method of snapshots, Sec. 2.5) against facts that
do not depend on it: an SVD from another library routine, a snapshot set of
prescribed basis and spectrum, the Eckart-Young projection error, the
orthonormality of the modes, and a single snapshot."""
import numpy as np
import scipy.linalg

from oracle import pod as opod
from oracle import gram


def prescribed(n, m, s, seed, w=None):
    """Snapshots S = W^(-1/2) U diag(s) V^T with U (n x r) orthonormal and V
    (m x r) orthonormal: the W-POD of S has singular values s and modes
    W^(-1/2) U (up to sign)."""
    rng = np.random.default_rng(seed)
    r = len(s)
    U, _ = np.linalg.qr(rng.standard_normal((n, r)))
    V, _ = np.linalg.qr(rng.standard_normal((m, r)))
    S = U @ np.diag(s) @ V.T
    if w is not None:
        S = S / np.sqrt(w)[:, None]
        U = U / np.sqrt(w)[:, None]
    return S, U


def test_singular_values_match_an_svd():
    rng = np.random.default_rng(1)
    S = rng.standard_normal((700, 40)) @ np.diag(0.7 ** np.arange(40)) + 0.01 * rng.standard_normal((700, 40))
    w = rng.uniform(0.5, 2.0, 700)
    _, sigma, _ = opod(S, w=w, rtol=0.0)
    ref = scipy.linalg.svd(np.sqrt(w)[:, None] * S, compute_uv=False, lapack_driver="gesvd")
    big = ref >= 1e-4 * ref[0]
    np.testing.assert_allclose(sigma[big], ref[big], rtol=1e-10)


def test_prescribed_spectrum_and_basis():
    s = np.array([5.0, 2.0, 1.0, 0.3, 0.1, 1e-3])
    w = np.random.default_rng(3).uniform(1.0, 3.0, 500)
    S, U = prescribed(500, 30, s, 2, w)
    modes, sigma, V = opod(S, w=w, rtol=1e-6)
    assert modes.shape == (500, 6)
    np.testing.assert_allclose(sigma[:6], s, rtol=1e-9)
    assert np.all(sigma[6:] < 1e-6 * s[0])        # rank 6: the rest is rounding
    # each mode is +- the prescribed basis vector (in the W inner product)
    for i in range(6):
        c = np.sum(w * modes[:, i] * U[:, i])
        assert abs(abs(c) - 1.0) < 1e-8, (i, c)
    # W-orthonormal modes
    G = modes.T @ (w[:, None] * modes)
    np.testing.assert_allclose(G, np.eye(6), atol=1e-9)


def test_eckart_young_projection_error():
    rng = np.random.default_rng(4)
    S = rng.standard_normal((400, 25)) @ np.diag(0.5 ** np.arange(25))
    modes, sigma, _ = opod(S, rtol=0.0)
    for k in (1, 3, 8):
        Uk = modes[:, :k]
        E = S - Uk @ (Uk.T @ S)
        np.testing.assert_allclose(np.sum(E * E), np.sum(sigma[k:] ** 2), rtol=1e-8)


def test_truncation_by_relative_tolerance_and_kmax():
    s = 10.0 ** -np.arange(10)                   # 1, 0.1, ..., 1e-9
    S, _ = prescribed(300, 20, s, 5)
    for rtol, k in ((0.5, 1), (0.05, 2), (2e-5, 5), (1e-7, 7)):
        modes, sigma, _ = opod(S, rtol=rtol)
        assert modes.shape[1] == k, (rtol, modes.shape)
    modes, _, _ = opod(S, rtol=1e-7, k_max=3)
    assert modes.shape[1] == 3


def test_single_snapshot_and_duplicates():
    x = np.random.default_rng(6).standard_normal(123)
    modes, sigma, V = opod(x[:, None])
    np.testing.assert_allclose(sigma, [np.linalg.norm(x)], rtol=1e-14)
    np.testing.assert_allclose(np.abs(modes[:, 0]), np.abs(x) / np.linalg.norm(x), rtol=1e-13)
    # the same snapshot three times: one mode, singular value sqrt(3)|x|
    modes, sigma, V = opod(np.stack([x, x, x], axis=1))
    assert modes.shape[1] == 1
    np.testing.assert_allclose(sigma[0], np.sqrt(3.0) * np.linalg.norm(x), rtol=1e-13)
    assert np.all(sigma[1:] < 1e-7 * sigma[0])


def test_sign_convention_and_gram():
    rng = np.random.default_rng(7)
    S = rng.standard_normal((50, 6))
    w = rng.uniform(0.5, 1.5, 50)
    np.testing.assert_allclose(gram(S, w), (S * w[:, None]).T @ S, rtol=1e-13)
    _, _, V = opod(S, w=w, rtol=0.0)
    for i in range(V.shape[1]):
        j = int(np.argmax(np.abs(V[:, i])))
        assert V[j, i] > 0.0
