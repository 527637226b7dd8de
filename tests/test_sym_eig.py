"""Host-side eigen-decomposition of the POD (mbx_sym_eig: Householder
tridiagonalisation and implicit QR with the Wilkinson shift):
checked on the CPU against LAPACK's symmetric solver, the reconstruction
A = V diag(lam) V^T, orthonormality, repeated eigenvalues, the sign rule and
the argument checks.  No GPU is involved."""
import numpy as np
import pytest

from paper_1704_04139_amd import mbx


def sym(rng, m, spectrum=None):
    Q, _ = np.linalg.qr(rng.standard_normal((m, m)))
    lam = rng.standard_normal(m) if spectrum is None else np.asarray(spectrum, float)
    A = (Q * lam) @ Q.T
    return (A + A.T) / 2.0


@pytest.mark.parametrize("m", [1, 2, 7, 64, 131])
def test_matches_lapack_and_reconstructs(m):
    rng = np.random.default_rng(m)
    A = sym(rng, m)
    lam, V = mbx.sym_eig(A)
    ref = np.linalg.eigvalsh(A)[::-1]
    scale = np.abs(ref).max()
    np.testing.assert_allclose(lam, ref, atol=1e-13 * scale * max(m, 1) ** 0.5)
    np.testing.assert_allclose((V * lam) @ V.T, A, atol=1e-12 * scale * m)
    np.testing.assert_allclose(V.T @ V, np.eye(m), atol=1e-12 * m)
    assert np.all(np.diff(lam) <= 0.0)
    for i in range(m):
        j = int(np.argmax(np.abs(V[:, i])))
        assert V[j, i] > 0.0


def test_gram_like_spectrum_and_repeated_eigenvalues():
    rng = np.random.default_rng(9)
    s = np.concatenate([[4.0, 4.0, 4.0], 10.0 ** -np.arange(1, 12, dtype=float), np.zeros(5)])
    A = sym(rng, s.size, s)
    lam, V = mbx.sym_eig(A)
    np.testing.assert_allclose(lam, np.sort(s)[::-1], atol=1e-14 * 4.0 * s.size)
    np.testing.assert_allclose((V * lam) @ V.T, A, atol=1e-13 * 4.0 * s.size)
    # the repeated eigenvalue's eigenvectors span the same space as the input's
    P = V[:, :3] @ V[:, :3].T
    np.testing.assert_allclose(P @ A @ P, 4.0 * P, atol=1e-12)


def test_argument_checks():
    with pytest.raises(mbx.MbxError) as e:
        mbx.sym_eig(np.array([[1.0, 2.0], [2.5, 1.0]]))
    assert e.value.code == mbx.MBX_EINVAL
    with pytest.raises(mbx.MbxError) as e:
        mbx.sym_eig(np.array([[np.nan]]))
    assert e.value.code == mbx.MBX_ENAN
    big = np.eye(513)
    with pytest.raises(mbx.MbxError):
        mbx.sym_eig(big)
