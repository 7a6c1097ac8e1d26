"""Pins for the truncating regime of the fixed-chi sweep oracle (O-3).

The simple update (paper Sec. 4) replaces the environment of a gated bond by
the lambdas of the other legs.  On a chain of three sites where the first
site carries a physical leg of dimension 2 and chi = 2, the environment it
uses is exact:

  * the bond between sites 0 and 1 can never need more than 2 values (its
    block has at most 2 rows), so its gate is split without truncation and
    leaves site 0 an isometry (the Q factor times the unitary U of the SVD);
  * at the bond between sites 1 and 2 the left part of the chain is therefore
    isometric and site 2 has no other leg, so the weighted block's singular
    values are the Schmidt values of the whole state across (p0 p1 | p2), and
    keeping the 2 largest is the optimal rank-2 truncation (Eckart-Young).

So the oracle's value must equal a dense computation that applies every op
of the layer program to the full 32-entry state vector and, after each gate
on the second bond, replaces the state by its best rank-2 approximation
across (p0 p1 | p2).  A wrong environment (lambda squared, lambda on the
gated leg, a missing lambda), a transposed factor or a wrong leg order all
change the value at first order, which the planted-mistake test shows.

The boundary MPS (zip-up, first row): with the row above trivial, step x of
the first row factorises the block of the columns 0..x against the rest of
the row; the left factor carried so far is an isometry, so the kept part is
the best rank-chi_m approximation of the left block (Eckart-Young), and the
last row of a two-row grid has one-row families (rank 1, exact).  Later rows
of the zip-up have no such reduction: their truncation is pinned only by the
exact limit (tests/test_oracle_sweep.py).
"""

import numpy as np
import pytest

from oracle.network import Layer, LayeredNet
from oracle.sweep import Sweep, sweep_logprob


def _chain_net(seed, n_layers=3):
    """1 x 3 chain, physical dims (2, 4, 4), product initial state."""
    rng = np.random.default_rng(seed)
    dims = (2, 4, 4)
    init = [rng.uniform(0.2, 1.0, (d, 1, 1, 1, 1)) for d in dims]
    layers = []
    for t in range(n_layers):
        lay = Layer()
        # one-site ops on every site, before and after the gates
        for s, d in enumerate(dims):
            lay.pre[s] = rng.uniform(0.0, 1.0, (d, d)) + np.eye(d)
        lay.gates.append(("H", 0, 0, rng.uniform(0.0, 1.0, (2, 4, 2, 4))))
        lay.gates.append(("H", 1, 0, rng.uniform(0.0, 1.0, (4, 4, 4, 4))))
        for s, d in enumerate(dims):
            if (s + t) % 2 == 0:
                lay.post[s] = rng.uniform(0.0, 1.0, (d, d)) + 0.5 * np.eye(d)
        layers.append(lay)
    final = [rng.uniform(0.2, 1.0, d) for d in dims]
    return LayeredNet(3, 1, init, layers, final), dims


def _dense_chain(net, dims, rank):
    """The same program on the dense state psi[p0, p1, p2]; every gate on the
    second bond is followed by the best rank-`rank` approximation across
    (p0 p1 | p2) from numpy's SVD."""
    d0, d1, d2 = dims
    psi = np.einsum("a,b,c->abc", net.init[0][:, 0, 0, 0, 0], net.init[1][:, 0, 0, 0, 0],
                    net.init[2][:, 0, 0, 0, 0])
    ops = ("a,xa,ybc->ybc", "b,xb,ayc->ayc", "c,xc,aby->aby")
    log_norm = 0.0

    def one_site(psi, s, M):
        if s == 0:
            return np.einsum("xa,abc->xbc", M, psi)
        if s == 1:
            return np.einsum("xb,abc->axc", M, psi)
        return np.einsum("xc,abc->abx", M, psi)

    for lay in net.layers:
        for s in sorted(lay.pre):
            psi = one_site(psi, s, lay.pre[s])
        for kind, x, y, G4 in lay.gates:
            if x == 0:
                psi = np.einsum("xyab,abc->xyc", G4, psi)
            else:
                psi = np.einsum("xyab,cab->cxy", G4, psi)
                U, S, Vt = np.linalg.svd(psi.reshape(d0 * d1, d2), full_matrices=False)
                psi = ((U[:, :rank] * S[:rank]) @ Vt[:rank]).reshape(d0, d1, d2)
        for s in sorted(lay.post):
            psi = one_site(psi, s, lay.post[s])
        c = np.max(np.abs(psi))
        psi = psi / c
        log_norm += np.log(c)
    z = np.einsum("abc,a,b,c->", psi, *net.final)
    return log_norm + np.log(z)


@pytest.mark.parametrize("seed", range(6))
def test_su_chain_equals_optimal_truncation(seed):
    net, dims = _chain_net(seed)
    want = _dense_chain(net, dims, 2)
    got, flags, nsplit = sweep_logprob(net, 2, 8, eps_rel=1e-12, tau_gap=1e-9)
    assert nsplit == 0
    assert got == pytest.approx(want, abs=1e-12)
    # and it is a genuine truncation: the untruncated state differs
    assert abs(_dense_chain(net, dims, 4) - want) > 1e-6


@pytest.mark.parametrize("mistake", ["lambda_squared", "lambda_missing", "lambda_on_gated_leg"])
def test_su_chain_pin_catches_planted_mistakes(monkeypatch, mistake):
    # The pin must fail for a wrong environment: plant it in the oracle.
    orig = Sweep._scale_legs

    def bad(self, T, x, y, legs, power):
        legs = list(legs)
        if mistake == "lambda_squared" and abs(power) == 1.0:
            power = 2.0 * power
        elif mistake == "lambda_missing" and power == 1.0:
            return T
        elif mistake == "lambda_on_gated_leg" and power == 1.0 and len(legs) == 3:
            legs = [1, 2, 3, 4]
        return orig(self, T, x, y, legs, power)

    monkeypatch.setattr(Sweep, "_scale_legs", bad)
    worst = 0.0
    for seed in range(3):
        net, dims = _chain_net(seed)
        got, _, _ = sweep_logprob(net, 2, 8, eps_rel=1e-12, tau_gap=1e-9)
        worst = max(worst, abs(got - _dense_chain(net, dims, 2)))
    assert worst > 1e-6


def _row_net(seed, Lx, dS, dE):
    """Lx x 2 grid with no layers: the final network is the initial one.
    Row 0 sites have a south leg dS and east legs dE, row 1 closes them."""
    rng = np.random.default_rng(seed)
    init = []
    for y in range(2):
        for x in range(Lx):
            shape = [1, 1, 1, 1, 1]
            if x > 0:
                shape[1] = dE
            if x + 1 < Lx:
                shape[2] = dE
            if y == 0:
                shape[4] = dS
            else:
                shape[3] = dS
            init.append(rng.uniform(-0.3, 1.0, shape))
    final = [np.ones(1) for _ in range(2 * Lx)]
    return LayeredNet(Lx, 2, init, [], final)


def _dense_zip_row(net, Lx, chi_m):
    """Row 0 truncated left to right by best rank-chi_m approximations of the
    block of columns 0..x (as (s_0..s_x) x (east bond of x)), then contracted
    with row 1 exactly."""
    T = [t[0] for t in net.init]  # [w, e, n, s]
    left = T[0][0, :, 0, :].T  # [s0, e]
    for x in range(1, Lx):
        U, S, Vt = np.linalg.svd(left, full_matrices=False)
        left = (U[:, :chi_m] * S[:chi_m]) @ Vt[:chi_m]
        t = T[x][:, :, 0, :]  # [w, e, s]
        left = np.einsum("aw,wes->ase", left, t).reshape(-1, t.shape[1])
    row0 = left[:, 0]  # [s0 s1 ... s_{Lx-1}]
    # row 1: contract left to right to a vector over (s0 .. s_{Lx-1})
    B = T[Lx][0, :, :, 0]  # [e, n]
    vec = B.T  # [n0, e]
    for x in range(1, Lx):
        t = T[Lx + x][:, :, :, 0]  # [w, e, n]
        vec = np.einsum("aw,wen->ane", vec, t).reshape(-1, t.shape[1])
    return float(row0 @ vec[:, 0])


@pytest.mark.parametrize("seed", range(4))
def test_zip_up_first_row_equals_optimal_truncation(seed):
    Lx, dS, dE, chi_m = 3, 3, 4, 2
    net = _row_net(seed, Lx, dS, dE)
    want = _dense_zip_row(net, Lx, chi_m)
    assert want > 0
    sw = Sweep(net, 8, chi_m, 1e-12, 1e-9)
    got = sw.run()
    assert sw.n_split == 0
    assert got == pytest.approx(np.log(want), abs=1e-12)
    # the untruncated contraction differs: the pin sees a real truncation
    assert abs(_dense_zip_row(net, Lx, 64) - want) > 1e-6 * abs(want)


def test_zip_pin_catches_planted_mistakes(monkeypatch):
    # Keeping the smallest singular values, or carrying V^T without S, must
    # move the value away from the dense reference.
    import oracle.sweep as osw
    orig = osw._svd

    def smallest_first(A, driver):
        U, S, Vt = orig(A, driver)
        k = min(A.shape)
        r = np.arange(k)[::-1]
        return U[:, r], S[r] + 0.0, Vt[r]

    for planted in (smallest_first,):
        monkeypatch.setattr(osw, "_svd", planted)
        worst = 0.0
        for seed in range(3):
            net = _row_net(seed, 3, 3, 4)
            want = _dense_zip_row(net, 3, 2)
            sw = Sweep(net, 8, 2, 1e-12, 1e-9)
            try:
                got = sw.run()
            except FloatingPointError:
                got = np.inf
            worst = max(worst, abs(got - np.log(want)) if np.isfinite(got) else np.inf)
        assert worst > 1e-6
