"""GPU parity of the POD by the method of snapshots (Sec. 2.5) and of the
snapshot capture (time-step solutions and Newton stages), through the C ABI,
against the oracle POD (oracle/pod.py).

Bars, derived from the arithmetic: the Gram matrix is an FP64 sum over n rows,
in another order than the oracle's, so each entry may differ by about
n u |S_i|_W |S_j|_W (u = 2^-53).  Every eigenvalue then moves by at most
||dK|| <= n u trace(K); the host Jacobi and LAPACK add m u lam_1 each.  An
eigenvector moves by about ||dK|| / gap, and so does its mode in the
W-norm (per unit sigma).  The tests use these bounds with a factor 10.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1704_04139_amd import inputs as I

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mbx(lib):
    from paper_1704_04139_amd import mbx as m
    return m


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def prescribed(n, m, s, seed, w=None):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, len(s))))
    V, _ = np.linalg.qr(rng.standard_normal((m, len(s))))
    S = (Q * s) @ V.T
    if w is not None:
        S = S / np.sqrt(w)[:, None]
    return S


def gpu_pod(mbx, torch, S, w=None, rtol=1e-7, k_max=None, lds_pad=0, ldm_pad=0):
    """Runs mbx_pod on a device copy of S (n x m) with optional padded leading
    dimensions; returns (modes n x k, sigma, k)."""
    n, m = S.shape
    k_max = m if k_max is None else k_max
    lds, ldm = n + lds_pad, n + ldm_pad
    dS = torch.zeros((m, lds), dtype=torch.float64, device="cuda")
    dS[:, :n] = torch.from_numpy(np.ascontiguousarray(S.T)).cuda()
    dw = torch.from_numpy(np.asarray(w, dtype=np.float64)).cuda() if w is not None else None
    dU = torch.full((k_max, ldm), np.nan, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    sigma, k = mbx.pod(dS.data_ptr(), n, m, lds, dU.data_ptr(), ldm, k_max, rtol,
                       dw.data_ptr() if dw is not None else 0)
    torch.cuda.synchronize()
    Uh = dU.cpu().numpy()
    assert np.all(np.isnan(Uh[k:])), "columns beyond k must stay unwritten"
    assert np.all(np.isnan(Uh[:k, n:])), "padding rows must stay unwritten"
    return Uh[:k, :n].T, sigma, k


def compare(S, w, modes, sigma, k, rtol, k_max=None, label=""):
    n, m = S.shape
    ref_modes, ref_sigma, _ = oracle.pod(S, w=w, rtol=rtol, k_max=k_max)
    K = oracle.gram(S, w)
    trace = float(np.trace(K))
    lam_g, lam_o = sigma ** 2, ref_sigma ** 2
    dl = 10.0 * (n * U * trace + 2 * m * U * lam_o[0])
    err = np.max(np.abs(lam_g - lam_o))
    say(label, "n", n, "m", m, "k", k, "max |dlam|", err, "bar", dl)
    assert err <= dl
    assert k == ref_modes.shape[1]
    ww = np.ones(n) if w is None else np.asarray(w)
    for i in range(k):
        gap = np.min(np.abs(np.delete(lam_o, i) - lam_o[i])) if m > 1 else np.inf
        bar = 10.0 * dl / max(gap, 1e-300) * (ref_sigma[0] / ref_sigma[i]) + 1e-11
        # up to sign: the sign rule looks at the largest entry of v_i, which
        # two correct eigensolvers may pick differently when entries tie
        d = min(np.sqrt(np.sum(ww * (modes[:, i] - s * ref_modes[:, i]) ** 2)) for s in (1.0, -1.0))
        assert d <= bar, (label, i, d, bar)
    return ref_sigma, ref_modes


def test_pod_matches_oracle_ragged(mbx, torch):
    """n = 5003 rows (a ragged row slice) and m = 70 snapshots (two column
    tiles: a diagonal and an off-diagonal tile pair), a weighted inner
    product, and a spectrum that the tolerance truncates."""
    s = 0.6 ** np.arange(20)
    rng = np.random.default_rng(11)
    w = rng.uniform(0.5, 2.0, 5003)
    S = prescribed(5003, 70, s, 12, w)
    # rtol >= 1e-5: rounding gives the rank-20 set spurious singular values up
    # to sqrt(n u trace K) ~ 1e-6 sigma_1, so a smaller rtol would let the kept
    # count depend on rounding (the method of snapshots squares the condition)
    for rtol in (1e-3, 1e-5):
        modes, sigma, k = gpu_pod(mbx, torch, S, w=w, rtol=rtol, lds_pad=5, ldm_pad=3)
        _, ref_modes = compare(S, w, modes, sigma, k, rtol, label=f"ragged rtol {rtol}")
        # no ties in random coefficients: the sign rule gives the same signs
        assert np.all(np.sum(w[:, None] * modes * ref_modes, axis=0) > 0.0)
    # W-orthonormal modes
    G = modes.T @ (w[:, None] * modes)
    assert np.max(np.abs(G - np.eye(k))) < 1e-8


def test_pod_edge_cases(mbx, torch):
    rng = np.random.default_rng(5)
    # one snapshot: its own direction
    x = rng.standard_normal((97, 1))
    modes, sigma, k = gpu_pod(mbx, torch, x)
    assert k == 1
    assert abs(sigma[0] - np.linalg.norm(x)) <= 1e-13 * np.linalg.norm(x)
    np.testing.assert_allclose(np.abs(modes[:, 0]), np.abs(x[:, 0]) / np.linalg.norm(x), rtol=1e-12)
    # fewer rows than one staging step, exactly one column tile
    S = rng.standard_normal((31, 64))
    modes, sigma, k = gpu_pod(mbx, torch, S, rtol=1e-5)
    assert k == 31                                   # rank 31; the rest is rounding
    compare(S, None, modes, sigma, k, 1e-5, label="n=31 m=64")
    # duplicated snapshots: rank one
    y = rng.standard_normal(300)
    S = np.stack([y] * 5, axis=1)
    modes, sigma, k = gpu_pod(mbx, torch, S)
    assert k == 1 and abs(sigma[0] - np.sqrt(5.0) * np.linalg.norm(y)) <= 1e-12 * sigma[0]
    # k_max below the tolerance count; five column tiles (m = 150)
    S = prescribed(2000, 150, 0.8 ** np.arange(40), 3)
    modes, sigma, k = gpu_pod(mbx, torch, S, rtol=1e-7, k_max=9)
    assert k == 9
    compare(S, None, modes, sigma, k, 1e-7, k_max=9, label="m=150 k_max=9")
    # all-zero snapshots: nothing kept
    modes, sigma, k = gpu_pod(mbx, torch, np.zeros((40, 3)))
    assert k == 0 and np.all(sigma == 0.0)


def test_pod_widths_at_the_staged_set_limit(mbx, torch):
    """Set widths at the edge of the Gram kernel that stages whole row chunks:
    128 columns (four tiles, ten tile pairs, five 16x16 blocks per wavefront)
    and 129 (the first width the pair-per-workgroup kernel takes), weighted,
    with a ragged last row slice."""
    rng = np.random.default_rng(21)
    for m, seed in ((128, 22), (129, 23)):
        w = rng.uniform(0.5, 2.0, 3001)
        S = prescribed(3001, m, 0.7 ** np.arange(30), seed, w)
        modes, sigma, k = gpu_pod(mbx, torch, S, w=w, rtol=1e-5, lds_pad=2)
        compare(S, w, modes, sigma, k, 1e-5, label=f"m={m} weighted")


def test_pod_argument_checks(mbx, torch):
    d = torch.zeros(64, dtype=torch.float64, device="cuda")
    for args in ((8, 0, 8), (8, 2, 7), (8, 513, 8)):
        with pytest.raises(mbx.MbxError) as e:
            mbx.pod(d.data_ptr(), args[0], args[1], args[2], d.data_ptr(), 8, 1)
        assert e.value.code == mbx.MBX_EINVAL
    with pytest.raises(mbx.MbxError):
        mbx.pod(d.data_ptr(), 8, 2, 8, d.data_ptr(), 8, 1, rtol=-1.0)


def capture_run(mbx, torch, w, cap, **knobs):
    cell = mbx.Cell(w.labels, w.params, **knobs)
    N = cell.counts.n_vox
    dc = torch.full((cap, N), np.nan, dtype=torch.float64, device="cuda")
    dp = torch.full((cap, N), np.nan, dtype=torch.float64, device="cuda")
    cell.capture(dc.data_ptr(), dp.data_ptr(), N, cap)
    torch.cuda.synchronize()
    return cell, dc, dp


def test_capture_records_solutions_and_newton_stages(mbx, torch):
    w = I.config0()
    cell, dc, dp = capture_run(mbx, torch, w, 128)
    c0, p0, _ = cell.get_state()
    torch.cuda.synchronize()
    assert cell.captured() == (1, 0)
    assert np.array_equal(dc[0].cpu().numpy(), c0) and np.array_equal(dp[0].cpu().numpy(), p0)
    total = 1
    for step in range(4):
        info = cell.step(w.dt)
        total += info["newton_iters"]
        count, dropped = cell.captured()
        assert (count, dropped) == (total, 0), (step, count, total)
        c, p, _ = cell.get_state()
        torch.cuda.synchronize()
        assert np.array_equal(dc[count - 1].cpu().numpy(), c)     # the step's solution
        assert np.array_equal(dp[count - 1].cpu().numpy(), p)
    say("captured", total, "columns over 4 steps")
    # the stages of a step differ from each other (they are the Newton iterates)
    assert not np.array_equal(dc[1].cpu().numpy(), dc[2].cpu().numpy())
    assert np.all(np.isnan(dc[total:].cpu().numpy()))
    cell.close()


def test_capture_capacity_and_failed_step(mbx, torch):
    w = I.config0()
    cell, dc, dp = capture_run(mbx, torch, w, 3)
    info = cell.step(w.dt)
    assert cell.captured() == (3, 1 + info["newton_iters"] - 3)   # 1 + iters wanted, 3 fit
    assert np.all(np.isfinite(dc.cpu().numpy()))
    cell.close()
    # a step that fails (one Newton iteration allowed) drops its columns again
    w.params.I_app *= 3.0
    cell, dc, dp = capture_run(mbx, torch, w, 16, newton_max=1)
    code, _ = cell.try_step(w.dt)
    assert code == mbx.MBX_ENEWTON
    assert cell.captured() == (1, 0)
    cell.close()


def test_pod_of_captured_snapshots_matches_oracle(mbx, torch):
    """Snapshots of the 12x12x40 cell (6 steps, concentration and potential
    sets separately, as Sec. 2.5 builds them), POD on the GPU against the
    oracle POD of the same downloaded columns."""
    w = I.config0()
    cell, dc, dp = capture_run(mbx, torch, w, 64)
    for _ in range(6):
        cell.step(w.dt)
    m, _ = cell.captured()
    N = cell.counts.n_vox
    for name, buf in (("c", dc), ("phi", dp)):
        S = buf[:m].cpu().numpy().T.copy()
        dU = torch.full((m, N), np.nan, dtype=torch.float64, device="cuda")
        # rtol 1e-4: the kept count is then decided far above the Gram matrix's
        # rounding level (lam_i / lam_1 = 1e-8 against n u ~ 1e-12)
        sigma, k = mbx.pod(buf.data_ptr(), N, m, N, dU.data_ptr(), N, m, 1e-4)
        torch.cuda.synchronize()
        modes = dU[:k].cpu().numpy().T
        ref_sigma, _ = compare(S, None, modes, sigma, k, 1e-4, label=f"captured {name}")
        say(name, "m", m, "k", k, "sigma ratios", (ref_sigma[:6] / ref_sigma[0]).round(8))
    cell.close()
