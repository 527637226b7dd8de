"""Continuous-batching server: results equal solo runs, admission honours the
memory budget, request bookkeeping is consistent.

Served parameter queries are the many-query use of the model (Sec. 1,
Sec. 2.5).  Every request's final state must equal the same cell stepped
alone to 1e-12 relative (per-cell deterministic reductions), whichever
requests shared its batches.
"""
import sys

import numpy as np
import pytest

from paper_1704_04139_amd import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mbx(lib):
    from paper_1704_04139_amd import mbx as m
    return m


def solo(mbx, w, precision, n_steps):
    c = mbx.Cell(w.labels, w.params, precision=precision)
    for _ in range(n_steps):
        c.step(w.dt)
    st = c.get_state()
    V = c.voltage()
    c.close()
    return st, V


def footprint(mbx, w, precision):
    """Device bytes of the request's cell, from the library's own face counts."""
    c = mbx.Cell(w.labels, w.params, precision=precision)
    nx, ny, nz = c.shape
    k = c.counts
    c.close()
    return mbx.footprint(nx, ny, nz, precision, k.n_an_faces, k.n_ca_faces)


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_served_equals_solo(mbx, precision):
    ws = I.config4_requests(4, scale=4)
    steps = [3, 2, 4, 3]
    say("serve", precision, [w.labels.shape for w in ws])
    srv = mbx.Server(budget_bytes=64 << 30, precision=precision, dt=ws[0].dt, keep_state=True)
    ids = []
    for k, (w, n) in enumerate(zip(ws, steps)):
        ids.append(srv.submit(w.labels, w.params, n))
    srv.drain(300.0)
    infos = [srv.poll(i) for i in ids]
    results = [srv.result(i) for i in ids]
    errors = [srv.error(i) for i in ids]
    stats = srv.stats()
    srv.close()
    say("stats", stats)
    assert stats["steps_run"] == sum(steps)
    assert stats["running"] == 0 and stats["queued"] == 0 and stats["bytes_in_use"] == 0
    assert all(srv_err == "" for srv_err in errors)
    for w, n, info, res in zip(ws, steps, infos, results):
        assert info["status"] == mbx.MBX_REQ_DONE
        assert info["steps_done"] == n
        assert 0.0 <= info["t_submit"] <= info["t_admit"] <= info["t_done"]
        ref, V = solo(mbx, w, precision, n)
        assert abs(info["V"] - V) <= 1e-12 * abs(V)
        for x, y in zip(res, ref):
            np.testing.assert_allclose(x, y, rtol=1e-12, atol=0)


def test_budget_admission(mbx):
    """With room for one request at a time, requests run strictly one after
    another in submission order; a request larger than the budget is refused."""
    w0 = I.config4_requests(1, scale=4)[0]
    ws = [w0, w0, w0]
    fp = footprint(mbx, w0, "mixed")
    say("footprint", fp)
    budget = 2 * fp - 1          # one fits, two do not
    srv = mbx.Server(budget_bytes=budget, precision="mixed", dt=ws[0].dt)
    ids = [srv.submit(w.labels, w.params, 2) for w in ws]
    srv.drain(300.0)
    infos = [srv.poll(i) for i in ids]
    big = I.config4_requests(1, base_seed=2101, scale=1)[0]
    with pytest.raises(mbx.MbxError) as e:
        srv.submit(big.labels, big.params, 1)
    assert e.value.code == mbx.MBX_EBUDGET
    # a request whose labels the library rejects fails at admission with a message
    bad = w0.labels.copy()
    bad[-1][bad[-1] == I.CATHODE] = I.PORE
    rid = srv.submit(bad, w0.params, 1)
    srv.drain(60.0)
    assert srv.poll(rid)["status"] == mbx.MBX_ELABEL
    assert "plane" in srv.error(rid)
    srv.close()
    for a, b in zip(infos, infos[1:]):
        assert b["t_admit"] >= a["t_done"]
    assert all(i["status"] == mbx.MBX_REQ_DONE and i["steps_done"] == 2 for i in infos)


def test_drain_returns_only_when_every_result_is_ready(mbx):
    """drain() polled with short time-outs: once it reports the server idle,
    every request is DONE and its result can be read (requests leave the
    running set and have their final state copied out under one count)."""
    ws = I.config4_requests(3, scale=4)
    srv = mbx.Server(budget_bytes=64 << 30, precision="mixed", dt=ws[0].dt, keep_state=True)
    ids = [srv.submit(w.labels, w.params, n) for w, n in zip(ws, (2, 1, 3))]
    polls = 0
    while True:
        polls += 1
        try:
            srv.drain(0.001)
            break
        except mbx.MbxError as e:
            assert e.code == mbx.MBX_ESTATE
            assert polls < 200000
    for rid in ids:
        assert srv.poll(rid)["status"] == mbx.MBX_REQ_DONE
        c, phi, n = srv.result(rid)
        assert np.all(np.isfinite(c)) and np.all(np.isfinite(phi))
    srv.close()
    say("drain polls", polls)
