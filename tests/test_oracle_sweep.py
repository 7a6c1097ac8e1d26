"""Pins for the fixed-chi sweep oracle (O-3) and its network constructions."""

import numpy as np
import pytest

import synth
from oracle.exact import frontier_logprobs
from oracle.network import point3d_network, rotated_network
from oracle.sweep import rank_rule, sweep_logprob


def _rates(dem, seed, lo=0.02, hi=0.3):
    return dem.with_p(np.random.default_rng(seed).uniform(lo, hi, dem.n_mech))


@pytest.mark.parametrize("L,chi,chi_m", [(2, 4, 4), (3, 8, 64), (3, 64, 64)])
def test_point_sweep_exact_at_large_chi(L, chi, chi_m):
    # Two layers with a rank-2 gate per bond never need more than 2*2^2 = 8 on
    # a 3D bond, so chi = 8 truncates nothing in the sweep on the 3x3 grid; the
    # boundary MPS of the final 3x3 network needs up to 8*8 = 64.
    dem = _rates(synth.surface3d_point(L, 0.1), L)
    m, _ = synth.sample_syndromes(dem, 6, 7)
    for k in range(6):
        ex = frontier_logprobs(dem.H, dem.p, dem.obs, m[k])
        for c in range(2):
            lp, flags, _ = sweep_logprob(point3d_network(L, dem.p, m[k], c), chi, chi_m, 1e-12, 1e-9)
            assert lp == pytest.approx(ex[c], abs=1e-10)


@pytest.mark.parametrize("d,T", [(3, 1), (3, 2), (3, 3), (5, 1)])
def test_rotated_sweep_exact_at_large_chi(d, T):
    dem = _rates(synth.rotated_phenom(d, T, 0.05, 0.05), d + T)
    m, _ = synth.sample_syndromes(dem, 5, 9)
    for k in range(5):
        ex = frontier_logprobs(dem.H, dem.p, dem.obs, m[k])
        for c in range(2):
            net = rotated_network(d, T, dem.params["checks"], dem.p, m[k], c)
            lp, flags, _ = sweep_logprob(net, 512, None, 1e-12, 1e-9)
            assert lp == pytest.approx(ex[c], abs=1e-10)


def test_truncation_is_an_approximation():
    # At chi = 4 on the L = 3 point sector the sweep truncates; it stays close
    # to, but differs from, the exact value.
    dem, m, _, _ = synth.config_workload(1, n=8)
    diffs = []
    for k in range(8):
        ex = frontier_logprobs(dem.H, dem.p, dem.obs, m[k])
        for c in range(2):
            lp, _, _ = sweep_logprob(point3d_network(3, dem.p, m[k], c), 4, None, 1e-12, 1e-9)
            diffs.append(abs(lp - ex[c]))
    assert max(diffs) > 1e-6
    assert max(diffs) < 0.5


def test_svd_driver_independence():
    dem, m, _, _ = synth.config_workload(1, n=6)
    for k in range(6):
        for c in range(2):
            net = point3d_network(3, dem.p, m[k], c)
            a, fa, na = sweep_logprob(net, 4, None, 1e-12, 1e-9, svd_driver="gesdd")
            b, fb, nb = sweep_logprob(net, 4, None, 1e-12, 1e-9, svd_driver="gesvd")
            if na == 0 and nb == 0:
                assert a == pytest.approx(b, abs=1e-11)


def test_half_rate_point_sector():
    # p = 1/2 closed form survives the sweep when nothing is truncated.
    L = 3
    dem = synth.surface3d_point(L, 0.5)
    m, _ = synth.sample_syndromes(dem, 3, 2)
    rank = dem.n_det + 1
    for k in range(3):
        for c in range(2):
            lp, _, _ = sweep_logprob(point3d_network(L, dem.p, m[k], c), 64, None, 1e-12, 1e-9)
            assert lp == pytest.approx(-rank * np.log(2), abs=1e-10)


def test_rank_rule():
    S = np.array([1.0, 0.5, 0.5, 0.2, 1e-14])
    assert rank_rule(S, 10, 1e-12, 1e-9) == (4, False)  # drops the sub-eps value
    assert rank_rule(S, 2, 1e-12, 1e-9) == (1, False)  # does not split the 0.5 pair
    assert rank_rule(S, 3, 1e-12, 1e-9) == (3, False)
    # the gap is relative to the value at the cut, so small values stay separable
    S = np.array([1.0, 1e-5, 0.5e-5, 0.25e-5])
    assert rank_rule(S, 2, 1e-12, 1e-4) == (2, False)
    assert rank_rule(np.array([1.0, 1e-5, 1e-5 * (1 - 1e-6)]), 2, 1e-12, 1e-4) == (1, False)
    assert rank_rule(np.array([1.0, 1.0, 1.0]), 2, 1e-12, 1e-9) == (2, True)
    assert rank_rule(np.array([2.0]), 1, 1e-12, 1e-9) == (1, False)


def test_chi_schedule_pins():
    """chi-schedule (per-layer truncation caps): a single entry k acts as the
    constant chi = k for every layer; caps that never bind (bonds after layer
    l are at most 2 * 2^(l+1) at L = 3, and chi_m = 64 holds the boundary MPS
    of a 3-wide grid exactly) give the exact contraction."""
    from oracle.network import point3d_network
    from oracle.sweep import sweep_logprob
    from oracle.exact import frontier_logprobs
    dem = synth.surface3d_point(3, 0.1).with_p(np.random.default_rng(4).uniform(0.05, 0.25, 51))
    m, _ = synth.sample_syndromes(dem, 2, 5)
    for k in range(2):
        for c in range(2):
            net = point3d_network(3, dem.p, m[k], c)
            a = sweep_logprob(net, 16, 8, 1e-9, 1e-6, chi_layers=[3])[0]
            b = sweep_logprob(net, 3, 8, 1e-9, 1e-6)[0]
            assert a == b
            big = sweep_logprob(net, 16, 64, 1e-12, 1e-9, chi_layers=[4, 8])[0]
            ex = frontier_logprobs(dem.H, dem.p, dem.obs, m[k])[c]
            assert abs(big - ex) <= 1e-10
            # a binding cap in the first layer changes the value
            cut = sweep_logprob(net, 16, 64, 1e-12, 1e-9, chi_layers=[2, 8])[0]
            assert abs(cut - ex) > 1e-8


def test_gauge_rounds_keep_the_exact_value():
    # where chi truncates nothing, identity gates change no value
    import synth
    from oracle.exact import frontier_logprobs
    from oracle.network import rotated_network
    dem = synth.rotated_phenom(3, 2, 0.05, 0.05)
    dem = dem.with_p(np.random.default_rng(9).uniform(0.02, 0.3, dem.n_mech))
    m, _ = synth.sample_syndromes(dem, 3, 10)
    for k in range(3):
        ex = frontier_logprobs(dem.H, dem.p, dem.obs, m[k])
        for c in range(2):
            net = rotated_network(3, 2, dem.params["checks"], dem.p, m[k], c)
            lp = sweep_logprob(net, 16, 64, 1e-12, 1e-9, gauge_rounds=2)[0]
            assert abs(lp - ex[c]) <= 1e-9


def test_gauge_rounds_reach_the_schmidt_values_on_a_chain():
    # a 4-site chain (a tree): simple update with trivial gates converges to
    # the canonical form, whose bond weights are the Schmidt values of the
    # state across each bond (from a dense SVD), the largest scaled to 1
    from oracle.network import Layer, LayeredNet
    from oracle.sweep import Sweep
    rng = np.random.default_rng(12)
    init = [rng.uniform(0.2, 1, 2).reshape(2, 1, 1, 1, 1) for _ in range(4)]
    gates = [("H", x, 0, rng.uniform(0, 1, (2, 2, 2, 2))) for x in range(3)]
    net = LayeredNet(Lx=4, Ly=1, init=init, layers=[Layer(gates=gates)], final=[np.ones(2)] * 4)
    sw = Sweep(net, 64, 64, 1e-14, 1e-12)
    sw.layer(net.layers[0])
    for _ in range(8):
        sw.gauge_round()
    # the dense state: product state, then the gates in class order
    psi = np.einsum("a,b,c,d->abcd", *[t.reshape(2) for t in init])
    for (k, x, y, G) in sorted(gates, key=lambda g: g[1] % 2):
        psi = np.moveaxis(np.tensordot(G, psi, axes=([2, 3], [x, x + 1])), [0, 1], [x, x + 1])
    for x in range(3):
        S = np.linalg.svd(psi.reshape(2 ** (x + 1), -1), compute_uv=False)
        S = S[S > 1e-12 * S[0]] / S[0]
        lam = np.sort(sw.lamH[(x, 0)])[::-1]
        lam = lam[: S.size] / lam[0]
        np.testing.assert_allclose(lam, S, rtol=1e-8, atol=1e-10)
