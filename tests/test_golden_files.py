"""CPU checks of the stored oracle trajectories in tests/golden/ (written by
make_oracle_refs.py from the oracle alone): they belong to the inputs the GPU
tests rebuild, they satisfy the oracle's conservation law, and the cutoff run
is well posed."""
import os

import numpy as np
import pytest

from oracle.cellmodel import FARADAY
from paper_1704_04139_amd import inputs as I

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    path = os.path.join(GOLD, name)
    if not os.path.exists(path):
        pytest.fail(f"{name} missing: run tests/golden/make_oracle_refs.py")
    return np.load(path)


def conserved(inv, I_app, dt, rel):
    """Li inventories step to step (Sec. 2.4 conservative scheme): electrolyte
    constant, anode + plated gain I dt/F, cathode loses it."""
    q = I_app * dt / FARADAY
    d = np.diff(inv, axis=0)
    assert np.all(np.abs(d[:, 0]) <= rel * q)
    np.testing.assert_allclose(d[:, 1] + d[:, 3], q, rtol=rel)
    np.testing.assert_allclose(d[:, 2], -q, rtol=rel)


def test_c1s2_golden():
    r = load("c1s2_oracle.npz")
    w = I.config1(seed=1, scale=2)
    assert np.array_equal(r["labels"], w.labels) and r["I_app"] == w.params.I_app
    assert list(r["state_steps"]) == [1, 2, 3] and r["c"].shape == (3, w.labels.size)
    conserved(r["inv"], float(r["I_app"]), float(r["dt"]), 1e-7)


def test_c2cut_golden_is_well_posed():
    """Voltages of the crossing step and its predecessor clear the cutoff by far
    more than the 1e-6 V voltage bar, so any path that meets the bar stops at
    the same step."""
    r = load("c2cut_oracle.npz")
    w = I.config2(seed=2, scale=8)
    assert np.array_equal(r["labels"], w.labels) and r["T"] == 268.0 and r["dt"] == 2.0
    k = int(r["cutoff_step"])
    V, Vc = r["V"], float(r["V_cut"])
    assert Vc == 4.2 and V[k] >= Vc > V[k - 1] and np.all(V[1:k] < Vc)
    assert min(V[k] - Vc, Vc - V[k - 1]) > 1e-5
    assert int(r["state_steps"][-1]) == k
    conserved(r["inv"], float(r["I_app"]), float(r["dt"]), 1e-7)


def test_queries_golden():
    r = load("queries_oracle.npz")
    n = int(r["n_queries"])
    Ts, rates, pls = [], [], []
    for k in range(n):
        fam, seed = str(r["families"][k]), int(r["seeds"][k])
        w = I.sampled_query(seed, list(range(32, 97, 8)) if fam == "batched" else list(range(48, 129, 8)), scale=4)
        assert np.array_equal(r[f"q{k}_labels"], w.labels)
        assert r[f"q{k}_I_app"] == w.params.I_app and r[f"q{k}_T"] == w.params.T
        conserved(r[f"q{k}_inv"], float(r[f"q{k}_I_app"]), float(r[f"q{k}_dt"]), 1e-7)
        Ts.append(float(r[f"q{k}_T"]))
        rates.append(float(r[f"q{k}_crate"]))
        pls.append(float(r[f"q{k}_i00_pl"]) / I.CellParams().i00_pl)
    # the sample spans the sampled ranges: temperature, C-rate, plating rate constant
    assert min(Ts) < 275 and max(Ts) > 300
    assert min(rates) < 1.2 and max(rates) > 3.0
    assert min(pls) < 0.05 and max(pls) > 10


def test_c0adapt_golden():
    """The adaptive run's record: times end at t_end, steps are dt0 times powers
    of 2 (the last may be cut short), estimates within tol, Li conserved over
    the non-uniform grid."""
    r = load("c0adapt_oracle.npz")
    w = I.config0()
    assert np.array_equal(r["labels"], w.labels) and r["I_app"] == w.params.I_app
    t, dts = r["times"], r["dts"]
    assert t[0] == 0.0 and t[-1] == r["t_end"] and np.allclose(np.diff(t), dts, rtol=0, atol=1e-12)
    k = np.log2(dts[:-1] / float(r["dt0"]))
    assert np.array_equal(k, np.round(k)) and dts.min() >= r["dt_min"] and dts.max() <= r["dt_max"]
    assert np.isnan(r["ests"][0]) and np.all(r["ests"][1:] <= r["tol"])
    assert r["rejected"] > 0 and dts.max() >= 16 * dts.min()   # the controller both cut and grew the step
    q = float(r["I_app"]) * dts / FARADAY
    d = np.diff(r["inv"], axis=0)
    np.testing.assert_allclose(d[:, 2], -q, rtol=1e-7)
    np.testing.assert_allclose(d[:, 1] + d[:, 3], q, rtol=1e-7)


def test_half_golden():
    """The half-cell stripping run: its inputs, the germ-grain plated faces,
    and the half cell's Li balance (the foil is a reservoir: electrolyte +
    graphite + plated Li moves by I dt / F, the foil's inventory is fixed)."""
    r = load("half_oracle.npz")
    w = I.paper_half_cell(seed=4, scale=6)
    mask, n_plated, _ = I.germ_grain_plating(w.labels, w.meta["z_sep_face"], w.params.h, 4)
    assert np.array_equal(r["labels"], w.labels) and np.array_equal(r["plated_mask"], mask)
    assert float(r["I_app"]) == w.params.I_app < 0          # delithiation
    np.testing.assert_array_equal(r["n"][0][mask], n_plated)
    inv = r["inv"]
    q = float(r["I_app"]) * float(r["dt"]) / FARADAY
    np.testing.assert_allclose(np.diff(inv[:, 0] + inv[:, 1] + inv[:, 3]), q, rtol=1e-9)
    assert np.all(np.diff(inv[:, 2]) == 0)
    assert inv[-1, 3] < inv[0, 3]                               # plated Li is stripped first
