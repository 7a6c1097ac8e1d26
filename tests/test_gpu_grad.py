"""GPU parity of the rate gradient (tn3d_grad_loglik and the autograd wrapper)
against the gradient oracle.

P(m) is affine in each rate, so d log P / d p_i = (P(p_i = c_i) / P - 1) /
(c_i - p_i) for any c_i != p_i; the library steps a quarter of the rate
range towards its middle.  Where chi truncates
nothing the library's gradient is the exact one (O-4, pinned to brute-force
marginals and finite differences); at truncating chi it is compared with the
same one-sided form over the oracle's fixed-chi sweep (O-3) at equal chi and
rank rule.

Tolerances follow from the per-value bound of each comparison: a log-value
error delta in P and in P(p_i = c_i) moves the term by at most
(|r| + 1) (e^(2 delta) - 1) / |c_i - p_i| with r = P(p_i = c_i) / P (taken
from the oracle: r = 1 + g (c_i - p_i)).
"""

import json
import os
import sys

import numpy as np
import pytest

import synth
from oracle.exact import frontier_logprobs
from oracle.grad import loglik_grad_exact, reduce_to_rates

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_10722_amd import tn3d
    c = tn3d.Context(0)
    yield c
    c.close()  # the gradient passes size their workspace to the free memory: release it


def syn_of(m):
    return torch.from_numpy(np.ascontiguousarray(m)).to("cuda:0")


def changed_rate(p, rate_max=1.0):
    return np.where(p <= 0.5 * rate_max, p + 0.25 * rate_max, p - 0.25 * rate_max)


def term_tol(g, p, delta, rate_max=1.0):
    """Bound on |term_gpu - term_oracle| for log-value errors <= delta."""
    c = changed_rate(p, rate_max)
    r = 1.0 + g * (c - p)
    return (np.abs(r) + 1.0) * np.expm1(2.0 * delta) / np.abs(c - p) + 1e-12


def loop_order(L):
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


def family(tn3d, ctx, which):
    """(dem, network, params, frontier order) of an untruncated case."""
    prm = tn3d.tn3d_params_default(16, 64, tn3d.PREC_FP64)
    prm.eps_rel, prm.tau_gap = 1e-12, 1e-9  # no singular value of the exact bonds is dropped
    if which == "point_L3":
        base = synth.surface3d_point(3, 0.1)
        dem = base.with_p(np.random.default_rng(41).uniform(0.02, 0.3, base.n_mech))
        return dem, tn3d.tn3d_net_surface3d_point(ctx, 3, dem.p), prm, None
    if which == "rotated_d3_T2":
        base = synth.rotated_phenom(3, 2, 0.05, 0.05)
        # rates on both sides of 1/2: both choices of c_i
        dem = base.with_p(np.random.default_rng(42).uniform(0.02, 0.8, base.n_mech))
        return dem, tn3d.tn3d_net_rotated_phenom(ctx, 3, 2, dem.p), prm, None
    if which == "loop_L3":
        base = synth.surface3d_loop(3, 0.1)
        dem = base.with_p(np.random.default_rng(43).uniform(0.03, 0.3, base.n_mech))
        return dem, tn3d.tn3d_net_surface3d_loop(ctx, 3, dem.p), prm, loop_order(3)
    if which == "dem_point_L3":
        base = synth.surface3d_point(3, 0.1)
        dem = base.with_p(np.random.default_rng(44).uniform(0.02, 0.3, base.n_mech))
        return dem, tn3d.tn3d_net_from_dem(ctx, dem.H, dem.p, dem.obs[0], dem.det_coord), prm, None
    raise ValueError(which)


@pytest.mark.parametrize("which", ["point_L3", "rotated_d3_T2", "loop_L3", "dem_point_L3"])
def test_grad_exact(ctx, which):
    """Untruncated chi, FP64: every per-item derivative against the exact
    gradient (log values within 1e-9), the batch sum, log P and its sum."""
    from paper_2310_10722_amd import tn3d
    say(f"case: gradient {which}, untruncated fp64, 6 syndromes, every mechanism")
    dem, net, prm, order = family(tn3d, ctx, which)
    m, _ = synth.sample_syndromes(dem, 6, 17)
    grad, tot, ll, flags, items = tn3d.tn3d_grad_loglik(ctx, net, syn_of(m), prm, per_item=True)
    torch.cuda.synchronize()
    grad, tot, ll, items = grad.cpu().numpy(), tot.cpu().numpy()[0], ll.cpu().numpy(), items.cpu().numpy()
    ref = [loglik_grad_exact(dem.H, dem.p, dem.obs, m[k], order=order) for k in range(6)]
    lp = np.array([r[0] for r in ref])
    g = np.array([r[1] for r in ref])
    tol = term_tol(g, dem.p[None, :], 1e-9)
    err = np.abs(items - g)
    say("  max |d term| =", err.max(), " max |d log P| =", np.abs(ll - lp).max())
    assert np.all(err <= tol)
    assert np.all(np.abs(grad - g.sum(axis=0)) <= tol.sum(axis=0))
    assert np.abs(ll - lp).max() <= 1e-9
    assert abs(tot - lp.sum()) <= 6e-9
    assert np.all((flags.cpu().numpy() & 1) == 0)


def test_grad_rate_map_autograd_and_differences(ctx):
    """Rotated d=3, 2 noisy rounds, one rate per data qubit (shared by the
    rounds) and per measurement event: the gradient over those 9 + 8 rates
    through rate_of_mech against the exact one reduced by the chain rule;
    the autograd wrapper gives the same value and gradient; central
    differences of the library's own contraction agree (h = 1e-4 p)."""
    from paper_2310_10722_amd import tn3d
    say("case: gradient rate map + autograd + differences, rotated d=3 T=2 fp64")
    d, T = 3, 2
    rng = np.random.default_rng(45)
    pq = rng.uniform(0.01, 0.1, d * d)
    qm = rng.uniform(0.01, 0.1, (T, (d * d - 1) // 2))
    dem = synth.rotated_phenom(d, T, pq, qm)
    nq, nZ = d * d, qm.shape[1]
    rate_of = np.concatenate([np.tile(np.arange(nq), T), nq + np.arange(T * nZ)]).astype(np.int32)
    r0 = np.concatenate([pq, qm.ravel()])
    assert np.allclose(r0[rate_of], dem.p)
    m, _ = synth.sample_syndromes(dem, 8, 19)
    prm = tn3d.tn3d_params_default(16, 16, tn3d.PREC_FP64)
    net = tn3d.tn3d_net_rotated_phenom(ctx, d, T, dem.p)
    syn = syn_of(m)
    grad, tot, _, _, _ = tn3d.tn3d_grad_loglik(ctx, net, syn, prm, rate_of_mech=rate_of)
    grad = grad.cpu().numpy()
    ref = [loglik_grad_exact(dem.H, dem.p, dem.obs, m[k]) for k in range(8)]
    g_mech = np.array([r[1] for r in ref])
    tol = reduce_to_rates(term_tol(g_mech, dem.p[None, :], 1e-9).sum(axis=0), rate_of, r0.size)
    want = reduce_to_rates(g_mech.sum(axis=0), rate_of, r0.size)
    say("  max |d grad| =", np.abs(grad - want).max())
    assert grad.shape == (r0.size,)
    assert np.all(np.abs(grad - want) <= tol)

    rates = torch.tensor(r0, dtype=torch.float64, requires_grad=True)

    def build(c, p):
        return tn3d.tn3d_net_rotated_phenom(c, d, T, p)

    out = tn3d.log_likelihood(ctx, build, rates, syn, prm, rate_of)
    out.backward()
    val = float(out.detach())
    assert abs(val - float(tot.cpu()[0])) <= 1e-12 * abs(val)
    np.testing.assert_allclose(rates.grad.numpy(), grad, rtol=1e-12, atol=1e-12)

    def f(r):
        n = build(ctx, r[rate_of])
        try:
            lp, _ = tn3d.tn3d_contract_cosets(ctx, n, syn, prm)
            v = lp.cpu().numpy()[:, :2]
        finally:
            n.close()
        mx = v.max(axis=1)
        return float(np.sum(mx + np.log(np.exp(v - mx[:, None]).sum(axis=1))))

    for k in (0, 4, nq, nq + 5):
        h = 1e-4 * r0[k]
        a, b = r0.copy(), r0.copy()
        a[k] += h
        b[k] -= h
        fd = (f(a) - f(b)) / (2 * h)
        say(f"  rate {k}: grad {grad[k]:.9f} central difference {fd:.9f}")
        assert abs(fd - grad[k]) <= 1e-5 * max(1.0, abs(grad[k]))


@pytest.mark.parametrize("mode", ["fp64_gram", "fp32"])
def test_grad_rotated_d7_chi16_golden(ctx, mode):
    """The gradient workload: rotated d=7, 7 noisy rounds + 1 perfect,
    per-qubit / per-measurement rates log-uniform in [0.005, 0.05], chi =
    chi_m = 16, rank rule (1e-6, 1e-2); items 0, 85, 170, 255 of its 256
    syndromes (with 60 more in FP32: 64 syndromes x 512 networks in one call)
    x 25 mechanisms against stored oracle values
    (tests/golden/make_rotated_d7_grad.py).  FP64 on the Gram route (the
    orthogonal route's one-sided Jacobi on 256-vector boundary families is
    too slow for 512 networks here): log values within 1e-6, its bound, or
    twice the oracle's spread under two SVD drivers, whichever is larger;
    FP32 1e-3 + 4 eps_32 (the decoded coset within 1e-3, a minority coset of
    weight e^-gap within 1e-3 + 4 eps_32 e^gap).  The per-rate
    gradient (49 qubit + 168 measurement rates) equals the chain-rule sum of
    the per-item derivatives."""
    from paper_2310_10722_amd import tn3d
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "rotated_d7_grad.json")))
    dem, m, _, _ = synth.config_workload(5, gold["n"])
    assert np.array_equal(m[gold["items"]], np.array(gold["syndromes"], dtype=np.uint8))
    pick = list(gold["items"])
    if mode == "fp32":
        pick += [k for k in range(gold["n"]) if k not in pick][:60]
    m = m[pick]
    say(f"case: gradient rotated d=7 T=7 chi=16 {mode}, {len(pick)} syndromes, 4 x 25 stored")
    net = tn3d.tn3d_net_rotated_phenom(ctx, 7, 7, dem.p)
    prm = tn3d.tn3d_params_default(16, 16, tn3d.PREC_FP64 if mode == "fp64_gram" else tn3d.PREC_FP32)
    prm.eps_rel, prm.tau_gap = gold["rule"]
    if mode == "fp64_gram":
        prm.flags = tn3d.OPT_GRAM_FACTOR
    nq, nZ = 49, 24
    rate_of = np.concatenate([np.tile(np.arange(nq), 7), nq + np.arange(7 * nZ)]).astype(np.int32)
    import time
    t0 = time.perf_counter()
    grad, tot, ll, flags, items = tn3d.tn3d_grad_loglik(ctx, net, syn_of(m), prm, rate_of_mech=rate_of,
                                                        per_item=True)
    torch.cuda.synchronize()
    say(f"  {len(pick)} syndromes: {time.perf_counter() - t0:.1f} s")
    grad, ll, items = grad.cpu().numpy(), ll.cpu().numpy(), items.cpu().numpy()
    idx = np.array(gold["mechanisms"])
    p = np.array(gold["p"])
    assert np.allclose(p, dem.p[idx])
    g0 = np.array(gold["grad"]["gesdd"])
    g1 = np.array(gold["grad"]["gesvd"])
    l0 = np.array(gold["loglik"]["gesdd"])
    got = items[:4][:, idx]
    if mode == "fp64_gram":
        tol = np.maximum(term_tol(g0, p[None, :], 1e-6), 2.0 * np.abs(g1 - g0)) + 1e-12
        ltol = np.maximum(1e-6, 2.0 * np.abs(np.array(gold["loglik"]["gesvd"]) - l0))
    else:
        delta = 1e-3 + 4.0 * 2.0 ** -24
        tol = term_tol(g0, p[None, :], delta)
        ltol = delta
    err = np.abs(got - g0)
    say("  max |d term| =", err.max(), " (relative to its bound:", (err / tol).max(), ")",
        " max |d log P| =", np.abs(ll[:4] - l0).max())
    assert np.all(err <= tol)
    assert np.all(np.abs(ll[:4] - l0) <= ltol)
    # chain rule over the per-item derivatives (the reduction order differs)
    want = reduce_to_rates(items.sum(axis=0), rate_of, nq + 7 * nZ)
    assert np.allclose(grad, want, rtol=1e-12, atol=1e-9)
    assert np.all(np.isfinite(grad))


def test_grad_depolarizing_equal_chi(ctx):
    """The depolarizing family (per-qubit rates in [0, 3/4], so the changed
    rate steps 3/16; four cosets): L = 3, rates drawn per qubit in
    [0.05, 0.3], chi = chi_m = 8, FP64 and the reduced rank rule, two
    syndromes, against the oracle's one-sided form over its fixed-chi sweep
    at the same chi and rule on 8 sampled qubits (log values within 1e-9)."""
    from oracle.grad import loglik_grad_one_sided
    from oracle.network import depol3d_network
    from oracle.sweep import sweep_logprob
    from paper_2310_10722_amd import tn3d
    say("case: gradient depolarizing L=3 chi=8 fp64, 2 syndromes, 8 qubits")
    base = synth.surface3d_depolarizing(3, 0.15)
    pq = np.random.default_rng(46).uniform(0.05, 0.3, base.params["p_qubit"].size)
    dem = synth.surface3d_depolarizing(3, pq)
    m, _ = synth.sample_pauli(dem, 2, 47)
    net = tn3d.tn3d_net_surface3d_depolarizing(ctx, 3, pq)
    prm = tn3d.tn3d_params_default(8, 8, tn3d.PREC_FP64)
    prm.eps_rel, prm.tau_gap = 1e-6, 1e-4
    grad, tot, ll, flags, items = tn3d.tn3d_grad_loglik(ctx, net, syn_of(m), prm, per_item=True)
    items, ll = items.cpu().numpy(), ll.cpu().numpy()
    idx = list(np.random.default_rng(48).choice(pq.size, 8, replace=False))
    for k in range(2):
        def cosets(q):
            return [sweep_logprob(depol3d_network(3, q, m[k], c), 8, 8, prm.eps_rel, prm.tau_gap)[0]
                    for c in range(4)]
        lp, g = loglik_grad_one_sided(cosets, pq, idx, rate_max=0.75)
        tol = term_tol(g, pq[idx], 1e-9, rate_max=0.75)
        err = np.abs(items[k, idx] - g)
        say(f"  syndrome {k}: max |d term| = {err.max():.3g} (relative to its bound {(err / tol).max():.3g}),"
            f" |d log P| = {abs(ll[k] - lp):.3g}")
        assert np.all(err <= tol)
        assert abs(ll[k] - lp) <= 1e-9


@pytest.mark.parametrize("family", ["loop_L4", "wht_point_L3"])
def test_grad_truncating_families_equal_chi(ctx, family):
    """The loop sector (L = 4, chi = chi_m = 8, truncating) and the
    Walsh-Hadamard form of the point sector (L = 3, chi = chi_m = 4): FP64 and
    the reduced rule, two syndromes, 6 sampled mechanisms, against the
    oracle's one-sided form over its sweep of the same networks at the same
    chi (log values within 1e-9; the Walsh-Hadamard form from the signed
    sweeps of Z_0, Z_1 combined as P_L = (Z_0 + (-1)^L Z_1) / 2)."""
    from oracle.grad import loglik_grad_one_sided
    from oracle.network import loop3d_network, point3d_network_wht
    from oracle.sweep import sweep_logprob, sweep_signed
    from paper_2310_10722_amd import tn3d
    say(f"case: gradient {family}, truncating chi, fp64, 2 syndromes, 6 mechanisms")
    prm = tn3d.tn3d_params_default(8 if family == "loop_L4" else 4, 8 if family == "loop_L4" else 4,
                                   tn3d.PREC_FP64)
    prm.eps_rel, prm.tau_gap = 1e-6, 1e-4
    if family == "loop_L4":
        base = synth.surface3d_loop(4, 0.1)
        dem = base.with_p(np.random.default_rng(51).uniform(0.03, 0.2, base.n_mech))
        net = tn3d.tn3d_net_surface3d_loop(ctx, 4, dem.p)
    else:
        base = synth.surface3d_point(3, 0.1)
        dem = base.with_p(np.random.default_rng(52).uniform(0.03, 0.2, base.n_mech))
        net = tn3d.tn3d_net_surface3d_wht(ctx, 3, tn3d.SECTOR_POINT, dem.p)
    m, _ = synth.sample_syndromes(dem, 2, 53)
    grad, tot, ll, flags, items = tn3d.tn3d_grad_loglik(ctx, net, syn_of(m), prm, per_item=True)
    items, ll = items.cpu().numpy(), ll.cpu().numpy()
    idx = list(np.random.default_rng(54).choice(dem.n_mech, 6, replace=False))
    for k in range(2):
        def cosets(q):
            if family == "loop_L4":
                return [sweep_logprob(loop3d_network(4, q, m[k], c), prm.chi, prm.chi_mps, prm.eps_rel,
                                      prm.tau_gap)[0] for c in range(2)]
            z = [sweep_signed(point3d_network_wht(3, q, m[k], b), prm.chi, prm.chi_mps, prm.eps_rel,
                              prm.tau_gap) for b in range(2)]
            v = [z[0][1] * np.exp(z[0][0]), z[1][1] * np.exp(z[1][0])]
            return [np.log((v[0] + (-1) ** L * v[1]) / 2.0) if (v[0] + (-1) ** L * v[1]) > 0 else np.nan
                    for L in range(2)]
        lp, g = loglik_grad_one_sided(cosets, dem.p, idx)
        tol = term_tol(g, dem.p[idx], 1e-9)
        err = np.abs(items[k, idx] - g)
        say(f"  syndrome {k}: max |d term| = {err.max():.3g} (relative to its bound {(err / tol).max():.3g})")
        assert np.all(err <= tol)
        assert abs(ll[k] - lp) <= 1e-9
