"""Pins for the loop sector of the 3D planar code (generator picture) and for
the Walsh-Hadamard coset variant (signed networks Z_b).

Both are checked against brute-force enumeration (L = 2, 12 edges) and the
exact frontier contraction (L = 3), at bond dimensions that truncate nothing;
the p = 1/2 closed form P_L(m) = 2^-rank[H; l] pins the weights."""

import numpy as np
import pytest

import synth
from oracle.exact import brute_force_table, frontier_logprobs
from oracle.network import (loop3d_dem_parts, loop3d_network, loop3d_network_wht, point3d_network,
                            point3d_network_wht)
from oracle.sweep import sweep_logprob, sweep_signed


def height_order(L):
    """Edges by height (in-plane edges of level z at 2z, z-edges from z to
    z + 1 at 2z + 1), which keeps the open faces of the frontier to two
    levels."""
    nz, nx = L ** 3, L * (L - 1) ** 2
    keys = []
    for e in range(nz + 2 * nx):
        if e < nz:
            keys.append((2 * (e // (L * L)) + 1, e))
        elif e < nz + nx:
            keys.append((2 * ((e - nz) // (L * (L - 1)) + 1), e))
        else:
            keys.append((2 * ((e - nz - nx) // ((L - 1) * L) + 1), e))
    return [e for _, e in sorted(keys)]


def exact_tn(net):
    return sweep_logprob(net, 64, 256, 1e-12, 1e-9)[0]


def wht_logp(nets, chi, chi_m, eps=1e-12, tau=1e-9):
    """log P_L = log((1/2) sum_b (-1)^(b L) Z_b) from the signed sweeps."""
    z = []
    for net in nets:
        lz, sg, _ = sweep_signed(net, chi, chi_m, eps, tau)
        z.append(sg * np.exp(lz))
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.array([np.log(0.5 * (z[0] + (-1) ** c * z[1])) for c in range(2)])


@pytest.fixture(scope="module")
def l2():
    rng = np.random.default_rng(21)
    base = synth.surface3d_loop(2, 0.1)
    dem = base.with_p(rng.uniform(0.03, 0.3, base.n_mech))
    return dem, brute_force_table(dem.H, dem.p, dem.obs)


def test_loop_dem_shape():
    for L in (2, 3, 4):
        dem = synth.surface3d_loop(L, 0.1)
        H, string = loop3d_dem_parts(L)
        assert np.array_equal(dem.H, H) and np.array_equal(dem.obs[0], string)
        assert dem.n_mech == L ** 3 + 2 * L * (L - 1) ** 2
        assert dem.n_det == (L - 1) ** 3 + 2 * L * L * (L - 1)
        # the X membrane of the bottom dangling edges commutes with every face
        # and meets the string once; each vertex star commutes with every face
        memb = np.zeros(dem.n_mech, dtype=np.int64)
        memb[: L * L] = 1
        assert np.all((dem.H.astype(np.int64) @ memb) % 2 == 0)
        assert int(memb @ string) % 2 == 1


def test_loop_exact_vs_bruteforce(l2):
    dem, table = l2
    assert table.sum() == pytest.approx(1.0, abs=1e-12)
    H = dem.H.astype(np.int64)
    for mint in np.nonzero(table.sum(axis=1) > 0)[0][:24]:
        m = ((mint >> np.arange(dem.n_det)) & 1).astype(np.uint8)
        ex = frontier_logprobs(dem.H, dem.p, dem.obs, m)
        assert np.allclose(ex, np.log(table[mint]), atol=1e-12, rtol=0)
        tn = np.array([exact_tn(loop3d_network(2, dem.p, m, c)) for c in range(2)])
        assert np.allclose(tn, np.log(table[mint]), atol=1e-10, rtol=0)
        wh = wht_logp([loop3d_network_wht(2, dem.p, m, b) for b in range(2)], 64, 256)
        assert np.allclose(wh, np.log(table[mint]), atol=1e-10, rtol=0)
    # a syndrome outside the image (one face of a cube flipped) has no preimage
    bad = np.zeros(dem.n_det, dtype=np.uint8)
    bad[0] = 1
    assert table[int((bad.astype(np.int64) << np.arange(dem.n_det)).sum())].sum() == 0.0
    with pytest.raises(ValueError):
        loop3d_network(2, dem.p, bad, 0)


def test_loop_network_exact_L3():
    rng = np.random.default_rng(5)
    base = synth.surface3d_loop(3, 0.1)
    dem = base.with_p(rng.uniform(0.03, 0.3, base.n_mech))
    m, _ = synth.sample_syndromes(dem, 4, 11)
    for k in range(4):
        ex = frontier_logprobs(dem.H, dem.p, dem.obs, m[k], order=height_order(3))
        tn = np.array([exact_tn(loop3d_network(3, dem.p, m[k], c)) for c in range(2)])
        assert np.allclose(tn, ex, atol=1e-9, rtol=0)
        wh = wht_logp([loop3d_network_wht(3, dem.p, m[k], b) for b in range(2)], 64, 256)
        assert np.allclose(wh, ex, atol=1e-9, rtol=0)


def test_point_wht_identity_L3():
    dem = synth.surface3d_point(3, 0.1).with_p(np.random.default_rng(3).uniform(0.02, 0.3, 51))
    m, _ = synth.sample_syndromes(dem, 4, 7)
    for k in range(4):
        ex = frontier_logprobs(dem.H, dem.p, dem.obs, m[k])
        wh = wht_logp([point3d_network_wht(3, dem.p, m[k], b) for b in range(2)], 8, 64)
        assert np.allclose(wh, ex, atol=1e-10, rtol=0)
        # Z_0 is the syndrome probability: the sum over both cosets
        lz0, s0, _ = sweep_signed(point3d_network_wht(3, dem.p, m[k], 0), 8, 64, 1e-12, 1e-9)
        assert s0 == 1.0 and lz0 == pytest.approx(np.logaddexp(ex[0], ex[1]), abs=1e-10)


def test_loop_p_half_closed_form():
    """At p = 1/2 every flip pattern has weight 2^-n, so P_L(m) = 2^-rank[H; l]
    for every consistent m and both classes."""
    L = 3
    dem = synth.surface3d_loop(L, 0.5)
    m, _ = synth.sample_syndromes(dem, 2, 3)
    A = np.concatenate([dem.H, dem.obs]).astype(np.uint8)
    rank = _gf2_rank(A)
    for k in range(2):
        tn = np.array([exact_tn(loop3d_network(L, dem.p, m[k], c)) for c in range(2)])
        assert np.allclose(tn, -rank * np.log(2.0), atol=1e-10, rtol=0)


def _gf2_rank(A):
    A = A.copy() & 1
    r = 0
    for c in range(A.shape[1]):
        hits = np.nonzero(A[r:, c])[0]
        if hits.size == 0:
            continue
        k = r + hits[0]
        A[[r, k]] = A[[k, r]]
        for i in np.nonzero(A[:, c])[0]:
            if i != r:
                A[i] ^= A[r]
        r += 1
        if r == A.shape[0]:
            break
    return r


def test_coset_selection_cross_check_truncating():
    """Reading of the coset selection (parity-chain initial state instead of
    the paper's Walsh-Hadamard pair) measured at truncating chi on the small
    point-sector workload (L = 3, p = 0.15, chi = chi_m = 4): both are within
    the chi = 4 truncation error of the exact values on the most likely
    coset.  Measured on these 16 syndromes: the signed pair is the more
    accurate one here (max 5e-3 against 9e-2 nats), since the parity chain
    spends a factor 2 of the bond on the running parity."""
    dem, m, _, _ = synth.config_workload(1)
    dch, dwh = [], []
    for k in range(16):
        ex = frontier_logprobs(dem.H, dem.p, dem.obs, m[k])
        ch = np.array([sweep_logprob(point3d_network(3, dem.p, m[k], c), 4, 4, 1e-9, 1e-6)[0] for c in range(2)])
        wh = wht_logp([point3d_network_wht(3, dem.p, m[k], b) for b in range(2)], 4, 4, 1e-9, 1e-6)
        b = int(np.argmax(ex))
        dch.append(abs(ch[b] - ex[b]))
        dwh.append(abs(wh[b] - ex[b]))
    assert max(dch) < 0.2 and max(dwh) < 0.2
    assert max(dwh) < max(dch)
