"""The allocation-free POD entry point (mbx_pod_noalloc, static device
workspace) against mbx_pod (workspace from hipMalloc) through the C ABI.

Both run the same kernels on the same slicing of the rows, so sigma, the kept
count and the modes must agree bit for bit.  Two calls in a row, the second
with a smaller snapshot set, show that the shared workspace keeps no state
between calls that could leak into a result.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def snapshots(n, m, seed):
    rng = np.random.default_rng(seed)
    s = 10.0 ** -np.linspace(0.0, 9.0, m)          # a decaying spectrum, as captured states have
    Q, _ = np.linalg.qr(rng.standard_normal((n, m)))
    V, _ = np.linalg.qr(rng.standard_normal((m, m)))
    return (Q * s) @ V.T


def run_both(mbx, torch, S, w, rtol, k_max, lds_pad, ldm_pad):
    n, m = S.shape
    lds, ldm = n + lds_pad, n + ldm_pad
    dS = torch.zeros((m, lds), dtype=torch.float64, device="cuda")
    dS[:, :n] = torch.from_numpy(np.ascontiguousarray(S.T)).cuda()
    dw = torch.from_numpy(w).cuda() if w is not None else None
    out = {}
    for noalloc in (False, True):
        dU = torch.full((k_max, ldm), 7.0, dtype=torch.float64, device="cuda")
        sig, k = mbx.pod(dS.data_ptr(), n, m, lds, dU.data_ptr(), ldm, k_max, rtol,
                         w_ptr=dw.data_ptr() if dw is not None else 0,
                         stream=torch.cuda.current_stream().cuda_stream, noalloc=noalloc)
        torch.cuda.synchronize()
        out[noalloc] = (sig, k, dU.cpu().numpy())
    return out


def test_pod_noalloc_matches_pod_on_two_calls():
    import torch
    from paper_1704_04139_amd import mbx
    assert torch.cuda.is_available()
    mbx.load()
    cases = [  # (n, m, weighted, rtol, k_max, lds pad, ldm pad): each call smaller than the one before
        (40_003, 200, True, 1e-6, 64, 5, 3),
        (20_011, 128, True, 1e-6, 128, 0, 2),   # the largest workspace: 256 row slices x 10 tile pairs
        (5_003, 70, False, 1e-5, 70, 0, 1),
    ]
    for n, m, weighted, rtol, k_max, lp, mp in cases:
        say(f"[no-alloc] n={n} m={m} weighted={weighted} rtol={rtol} k_max={k_max}")
        S = snapshots(n, m, seed=n + m)
        w = np.random.default_rng(m).uniform(0.5, 2.0, n) if weighted else None
        out = run_both(mbx, torch, S, w, rtol, k_max, lp, mp)
        sig0, k0, U0 = out[False]
        sig1, k1, U1 = out[True]
        say(f"[no-alloc]   k={k0}/{k1} sigma_1={sig0[0]:.6e}")
        assert k0 == k1 and k0 > 0
        assert np.array_equal(sig0, sig1)
        # kept columns equal bit for bit, the rest left unwritten
        assert np.array_equal(U0[:k0, :n], U1[:k1, :n])
        assert np.all(U1[k1:] == 7.0) and np.all(U1[:, n:] == 7.0)


def test_pod_noalloc_rejects_more_snapshots_than_its_workspace_covers():
    import torch
    from paper_1704_04139_amd import mbx
    mbx.load()
    m = mbx.MBX_POD_MAX_SNAPSHOTS + 1 if hasattr(mbx, "MBX_POD_MAX_SNAPSHOTS") else 513
    d = torch.zeros((m, 64), dtype=torch.float64, device="cuda")
    with pytest.raises(mbx.MbxError) as e:
        mbx.pod(d.data_ptr(), 64, m, 64, d.data_ptr(), 64, 4, 1e-7, noalloc=True)
    assert e.value.code == mbx.MBX_EINVAL
