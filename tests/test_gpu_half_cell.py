"""GPU parity for the half cell (Sec. 2.2: graphite against a Li-foil counter
electrode, label 3; Sec. 3.2: the stripping case study), through the C ABI.

  * residual and J*v against the oracle on a perturbed half-cell state;
  * the 16 x 16 x 24 copy of the paper's case (germ-grain plated Li,
    delithiation at 250 A/m^2) against the stored oracle run
    (tests/golden/half_oracle.npz, written by make_oracle_refs.py from the
    oracle alone): V every step and every field, both precisions;
  * Li balance: electrolyte + graphite + plated Li moves by I dt / F per
    step, the foil's unknowns stay put;
  * label and parameter errors.

Bars: |dV| <= 1e-6 V; relative L2 error per field <= 1e-8 (FP64), 1e-6 (mixed).
"""
import os
import sys

import numpy as np
import pytest

from oracle.cellmodel import FARADAY, Geometry, Model
from paper_1704_04139_amd import inputs as I

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
BARS = [("fp64", 1e-8), ("mixed", 1e-6)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def mbx(lib):
    from paper_1704_04139_amd import mbx as m
    return m


def small_half_cell():
    w = I.paper_half_cell(seed=4, scale=6)
    mask, n_plated, _ = I.germ_grain_plating(w.labels, w.meta["z_sep_face"], w.params.h, 4)
    return w, mask, n_plated


def perturbed(model, seed):
    rng = np.random.default_rng(seed)
    N = model.N
    u_old = model.initial_state()
    u = u_old.copy()
    u[:N] *= 1.0 + 0.03 * np.clip(rng.standard_normal(N), -1.5, 1.5)
    u[N:2 * N] += 0.01 * rng.standard_normal(N)
    u[2 * N:] = model.p["n_c"] * (1.0 + 30.0 * rng.random(model.g.F_pl))
    return u, u_old


KEYS = ("electrolyte", "anode", "cathode", "plated")


def inventory(cell):
    d = cell.inventory()
    return np.array([d[k] for k in KEYS])


def rel_l2(a, b, floor=0.0):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), floor)


def test_half_cell_residual_matches_oracle(mbx):
    w, _, _ = small_half_cell()
    say("half-cell residual", w.labels.shape)
    model = Model(Geometry(w.labels), w.params.as_dict())
    cell = mbx.Cell(w.labels, w.params)
    u, u_old = perturbed(model, 11)
    N = model.N
    dt = 1.0
    R = model.residual(u, u_old, dt)
    got = cell.residual(u[:N], u[N:2 * N], u[2 * N:], u_old[:N], u_old[2 * N:], dt)
    for g, ref in zip(got, (R[:N], R[N:2 * N], R[2 * N:])):
        np.testing.assert_allclose(g, ref, rtol=1e-9, atol=1e-11 * np.max(np.abs(ref)))
    cell.close()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("mixed", 2e-5)])
def test_half_cell_jvp_matches_oracle(mbx, prec, tol):
    import scipy.sparse as sp
    w, _, _ = small_half_cell()
    model = Model(Geometry(w.labels), w.params.as_dict())
    cell = mbx.Cell(w.labels, w.params, precision=prec)
    u, u_old = perturbed(model, 12)
    N, dt = model.N, 1.0
    J = model.jacobian(u, dt).tocsr()
    Jc = J[:2 * N, :2 * N] - J[:2 * N, 2 * N:] @ sp.diags(1.0 / J[2 * N:, 2 * N:].diagonal()) @ J[2 * N:, :2 * N]
    Du = np.concatenate([model.c_ref, np.full(N, model.RT / FARADAY)])
    Dr = np.concatenate([dt / (model.V * model.c_ref), np.full(N, 1.0 / (model.A * model.mu_ref))])
    Jh = sp.diags(Dr) @ Jc @ sp.diags(Du)
    rng = np.random.default_rng(2)
    for _ in range(2):
        v = rng.standard_normal(2 * N)
        y = cell.jvp(u[:N], u[N:2 * N], u[2 * N:], u_old[:N], u_old[2 * N:], dt, v)
        yr = Jh @ v
        scale = np.abs(Jh) @ np.abs(v)
        assert np.max(np.abs(y - yr) / np.maximum(scale, 1e-300)) < tol
    cell.close()


@pytest.mark.parametrize("prec,bar", BARS)
def test_half_cell_stripping_matches_oracle(mbx, prec, bar):
    ref = np.load(os.path.join(GOLD, "half_oracle.npz"))
    w, mask, n_plated = small_half_cell()
    assert np.array_equal(ref["labels"], w.labels) and np.array_equal(ref["plated_mask"], mask)
    say("half-cell stripping", w.labels.shape, prec, int(mask.sum()), "plated faces")
    cell = mbx.Cell(w.labels, w.params, precision=prec)
    c, p, n = cell.get_state()
    n = n.copy()
    n[mask] = n_plated
    cell.set_state(c, p, n)
    np.testing.assert_allclose(cell.get_state()[2], ref["n"][0], rtol=1e-15)
    worst = {}
    N = c.size
    pore = w.labels.ravel() == 0
    for s in range(1, len(ref["V"])):
        info = cell.step(w.dt)
        assert info["substeps"] == 1
        assert abs(info["V"] - ref["V"][s]) <= 1e-6, (s, info["V"], ref["V"][s])
        worst["V"] = max(worst.get("V", 0.0), abs(info["V"] - ref["V"][s]))
        gc, gp, gn = cell.get_state()
        e = {"c_e": rel_l2(gc[pore], ref["c"][s][pore]), "c_s": rel_l2(gc[~pore], ref["c"][s][~pore]),
             "phi": rel_l2(gp, ref["phi"][s]), "n": rel_l2(gn, ref["n"][s], floor=w.params.n_c * np.sqrt(gn.size))}
        for f, v in e.items():
            worst[f] = max(worst.get(f, 0.0), v)
            assert v <= bar, (s, f, v)
        np.testing.assert_allclose(inventory(cell), ref["inv"][s], rtol=max(bar, 1e-9))
    assert N == w.labels.size
    say("worst", prec, {k: f"{v:.2e}" for k, v in worst.items()})
    cell.close()


def test_half_cell_li_balance(mbx):
    w, mask, n_plated = small_half_cell()
    cell = mbx.Cell(w.labels, w.params, precision="fp64")
    c, p, n = cell.get_state()
    n = n.copy()
    n[mask] = n_plated
    cell.set_state(c, p, n)
    prev = inventory(cell)
    foil0 = c[w.labels.ravel() == I.FOIL].copy()
    for _ in range(3):
        cell.step(w.dt)
        inv = inventory(cell)
        moved = (inv[0] + inv[1] + inv[3]) - (prev[0] + prev[1] + prev[3])
        assert moved == pytest.approx(w.params.I_app * w.dt / FARADAY, rel=1e-9)
        assert inv[2] == prev[2]
        prev = inv
    np.testing.assert_array_equal(cell.get_state()[0][w.labels.ravel() == I.FOIL], foil0)
    cell.close()


def test_half_cell_label_and_parameter_errors(mbx):
    w, _, _ = small_half_cell()
    lab = w.labels.copy()
    lab[w.meta["z_sep_face"] + 2] = I.CATHODE          # a cathode layer inside a half cell
    with pytest.raises(mbx.MbxError) as ei:
        mbx.Cell(lab, w.params)
    assert ei.value.code == mbx.MBX_ELABEL
    lab = w.labels.copy()
    lab[lab == I.PORE] = I.FOIL                         # foil touching the graphite
    with pytest.raises(mbx.MbxError) as ei:
        mbx.Cell(lab, w.params)
    assert ei.value.code == mbx.MBX_ELABEL
    import dataclasses
    with pytest.raises(mbx.MbxError) as ei:
        mbx.Cell(w.labels, dataclasses.replace(w.params, i00_ce=0.0))
    assert ei.value.code == mbx.MBX_EINVAL
