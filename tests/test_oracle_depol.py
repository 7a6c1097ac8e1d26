"""Pins for the depolarizing family of the 3D planar code (mixed picture):
its DEM form, the oracle's network and the GF(2) representative it uses."""

import json
import os

import numpy as np
import pytest

import synth
from oracle.exact import frontier_logprobs
from oracle.network import depol3d_network, gf2_solve
from oracle.sweep import sweep_logprob

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "depol_L3_exact.json")


def _pauli_table(dem):
    """p_{m,c} by enumerating all 4^n Paulis of the code (n = 12 at L = 2):
    the weight of (u, v) is prod_e W(u_e, v_e) with W = 1-p for I and p/3 for
    X, Y, Z; rows are keyed by (face syndrome of u, class a), columns by
    (vertex syndrome of v, class b)."""
    pr = dem.params
    n, p = pr["n_qubits"], pr["p_qubit"]
    ints = np.arange(1 << n)
    bits = (ints[:, None] >> np.arange(n)[None, :]) & 1
    logw = np.zeros((1 << n, 1 << n))
    for e in range(n):
        tab = np.log(np.array([[1 - p[e], p[e] / 3], [p[e] / 3, p[e] / 3]]))
        logw += tab[bits[:, e][:, None], bits[:, e][None, :]]
    M = np.exp(logw)
    mz = ((bits @ pr["HZ"].T.astype(np.int64)) & 1) @ (1 << np.arange(pr["HZ"].shape[0]))
    mx = ((bits @ pr["HX"].T.astype(np.int64)) & 1) @ (1 << np.arange(pr["HX"].shape[0]))
    ku = 2 * mz + ((bits @ pr["zbar"].astype(np.int64)) & 1)
    kv = 2 * mx + ((bits @ pr["xbar"].astype(np.int64)) & 1)
    cols = np.zeros((1 << n, int(kv.max()) + 1))
    cols[ints, kv] = 1.0
    rows = np.zeros((int(ku.max()) + 1, 1 << n))
    rows[ku, ints] = 1.0
    return rows @ (M @ cols)


def _lookup(table, dem, m):
    nv = dem.params["HX"].shape[0]
    mx = int((m[:nv].astype(np.int64) << np.arange(nv)).sum())
    mz = int((m[nv:].astype(np.int64) << np.arange(m.size - nv)).sum())
    return np.array([table[2 * mz + (c & 1), 2 * mx + (c >> 1)] for c in range(4)])


@pytest.fixture(scope="module")
def l2():
    rng = np.random.default_rng(11)
    dem = synth.surface3d_depolarizing(2, rng.uniform(0.05, 0.3, 12))
    return dem, _pauli_table(dem)


def test_pauli_table_normalised(l2):
    _, table = l2
    assert table.sum() == pytest.approx(1.0, abs=1e-12)


def test_dem_form_is_the_depolarizing_channel(l2):
    # three independent X, Y, Z mechanisms of rate r, r (1 - r) = p/3, against
    # the enumeration of the channel itself
    dem, table = l2
    m, _ = synth.sample_pauli(dem, 8, 21)
    for k in range(8):
        ex = frontier_logprobs(dem.H, dem.p, dem.obs, m[k])
        assert np.exp(ex) == pytest.approx(_lookup(table, dem, m[k]), rel=1e-12)


def test_sweep_exact_L2(l2):
    dem, table = l2
    m, _ = synth.sample_pauli(dem, 8, 22)
    for k in range(8):
        ref = np.log(_lookup(table, dem, m[k]))
        for c in range(4):
            lp, _, _ = sweep_logprob(depol3d_network(2, dem.params["p_qubit"], m[k], c), 64, 64, 1e-12, 1e-9)
            assert lp == pytest.approx(ref[c], abs=1e-11)


def test_sweep_exact_L3_golden():
    # exact values stored by tests/golden/make_depol_L3_exact.py (O-2 on the
    # DEM form); chi = 64 and chi_m = 256 truncate nothing on two layers of
    # rank-3 gates
    g = json.load(open(GOLDEN))
    for m, ref in zip(g["syndromes"], g["logp"]):
        for c in range(4):
            net = depol3d_network(g["L"], g["p"], np.array(m, dtype=np.uint8), c)
            lp, _, _ = sweep_logprob(net, 64, 256, eps_rel=1e-15, tau_gap=1e-12)
            assert lp == pytest.approx(ref[c], abs=1e-9)


def test_representative_is_a_gauge():
    # another representative of the same class (times vertex stabilizers)
    # relabels the generator bits of those vertices, a permutation of one
    # site's physical index between two layers: the truncated contraction is
    # unchanged
    L = 3
    dem = synth.surface3d_depolarizing(L, 0.15)
    pr = dem.params
    nv = pr["HX"].shape[0]
    m, _ = synth.sample_pauli(dem, 3, 23)
    for k in range(3):
        r = gf2_solve(pr["HZ"], m[k][nv:])
        for v in (0, 4, 13):
            r2 = r ^ pr["HX"][v]
            for c in range(4):
                lp = [sweep_logprob(depol3d_network(L, 0.15, m[k], c, rep=rr), 4, 8, 1e-12, 1e-9)[0]
                      for rr in (r, r2)]
                assert lp[1] == pytest.approx(lp[0], abs=1e-11)


def test_gf2_solve():
    rng = np.random.default_rng(5)
    for _ in range(20):
        A = (rng.random((12, 16)) < 0.3).astype(np.uint8)
        x0 = (rng.random(16) < 0.5).astype(np.uint8)
        b = (A.astype(np.int64) @ x0) & 1
        x = gf2_solve(A, b)
        assert x is not None and np.array_equal((A.astype(np.int64) @ x) & 1, b)
    A = np.array([[1, 1], [1, 1]], dtype=np.uint8)
    assert gf2_solve(A, np.array([1, 0])) is None


def test_pauli_sampler_distribution():
    # the seeded sampler draws I / X / Y / Z with 1-p, p/3, p/3, p/3 per qubit;
    # its syndromes are those of the drawn Pauli, so every face syndrome is
    # consistent (the oracle's elimination finds a representative)
    L = 3
    dem = synth.surface3d_depolarizing(L, 0.15)
    pr = dem.params
    nv = pr["HX"].shape[0]
    m, cos = synth.sample_pauli(dem, 4000, 99)
    # an X or Y on the vertical string flips a, so P(a = 1) = (1 - (1 - 4p/3)^L) / 2
    pa = np.mean(cos & 1)
    expect = 0.5 * (1 - (1 - 4 * 0.15 / 3) ** L)
    assert abs(pa - expect) < 4 * np.sqrt(expect * (1 - expect) / 4000)
    for k in range(50):
        assert gf2_solve(pr["HZ"], m[k][nv:]) is not None
