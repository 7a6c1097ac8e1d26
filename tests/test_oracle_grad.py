"""Pins for the gradient oracle (O-4)."""

import itertools

import numpy as np
import pytest

import synth
from oracle.exact import frontier_logprobs
from oracle.grad import (batch_loglik_grad_exact, central_difference, loglik_exact, loglik_grad_exact,
                         loglik_grad_one_sided, reduce_to_rates)
from oracle.network import rotated_network
from oracle.sweep import sweep_logprob


def _marginal_grad_brute(H, p, m):
    """(mu_i - p_i) / (p_i (1 - p_i)) with mu_i = P(x_i = 1 | m), by enumeration
    of every error pattern x in F2^n (n <= 16)."""
    H = np.asarray(H, dtype=np.int64)
    n = H.shape[1]
    X = np.array(list(itertools.product((0, 1), repeat=n)), dtype=np.int64)
    ok = np.all(((X @ H.T) & 1) == np.asarray(m, dtype=np.int64)[None, :], axis=1)
    w = np.prod(np.where(X == 1, p[None, :], 1.0 - p[None, :]), axis=1) * ok
    P = w.sum()
    mu = (w[:, None] * X).sum(axis=0) / P
    return np.log(P), (mu - p) / (p * (1.0 - p))


def test_two_mechanism_closed_form():
    # One detector seen by two mechanisms: P(1) = p1 (1 - p2) + p2 (1 - p1),
    # d log P / d p1 = (1 - 2 p2) / P(1).
    H = np.array([[1, 1]], dtype=np.uint8)
    obs = np.array([[1, 0]], dtype=np.uint8)
    p = np.array([0.13, 0.31])
    lp, g = loglik_grad_exact(H, p, obs, np.array([1], dtype=np.uint8))
    P = p[0] * (1 - p[1]) + p[1] * (1 - p[0])
    assert lp == pytest.approx(np.log(P), abs=1e-14)
    assert g[0] == pytest.approx((1 - 2 * p[1]) / P, rel=1e-13)
    assert g[1] == pytest.approx((1 - 2 * p[0]) / P, rel=1e-13)


@pytest.mark.parametrize("which", ["rep", "point2", "rot31", "surf2d"])
def test_gradient_equals_brute_force_marginals(which):
    rng = np.random.default_rng(11)
    dem = {"rep": synth.repetition_line(7, 0.1), "point2": synth.surface3d_point(2, 0.1),
           "rot31": synth.rotated_phenom(3, 1, 0.05, 0.05), "surf2d": synth.surface2d_bitflip(3, 0.1)}[which]
    if dem.n_mech > 16:
        pytest.skip("too many mechanisms to enumerate")
    dem = dem.with_p(rng.uniform(0.02, 0.4, dem.n_mech))
    m, _ = synth.sample_syndromes(dem, 4, 5)
    for k in range(4):
        lp, g = loglik_grad_exact(dem.H, dem.p, dem.obs, m[k])
        lb, gb = _marginal_grad_brute(dem.H, dem.p, m[k])
        assert lp == pytest.approx(lb, abs=1e-12)
        np.testing.assert_allclose(g, gb, rtol=1e-10, atol=1e-10)


def test_gradient_equals_central_differences_of_o2():
    dem = synth.rotated_phenom(3, 2, 0.05, 0.05)
    dem = dem.with_p(np.random.default_rng(4).uniform(0.01, 0.2, dem.n_mech))
    m, _ = synth.sample_syndromes(dem, 3, 8)
    idx = list(range(0, dem.n_mech, 3))
    for k in range(3):
        _, g = loglik_grad_exact(dem.H, dem.p, dem.obs, m[k])
        fd = central_difference(lambda q: loglik_exact(dem.H, q, dem.obs, m[k]), dem.p, idx, 1e-5)
        np.testing.assert_allclose(g[idx], fd, rtol=1e-6, atol=1e-6)


def test_batch_sum_and_rate_reduction():
    # Sum over syndromes is additive; a shared rate's derivative is the sum of
    # its mechanisms' (checked by differentiating the shared-rate function).
    d, T = 3, 2
    pq = np.array([0.02, 0.05, 0.03, 0.04, 0.01, 0.06, 0.02, 0.03, 0.05])
    qm = np.array([[0.01, 0.02, 0.03, 0.04], [0.05, 0.02, 0.01, 0.03]])
    dem = synth.rotated_phenom(d, T, pq, qm)
    m, _ = synth.sample_syndromes(dem, 3, 3)
    tot, g = batch_loglik_grad_exact(dem.H, dem.p, dem.obs, m)
    assert tot == pytest.approx(sum(loglik_exact(dem.H, dem.p, dem.obs, mm) for mm in m), abs=1e-12)
    nq, nZ = d * d, qm.shape[1]
    rate_of = np.concatenate([np.tile(np.arange(nq), T), nq + np.arange(T * nZ)])
    gr = reduce_to_rates(g, rate_of, nq + T * nZ)

    def f(r):
        q = synth.rotated_phenom(d, T, r[:nq], r[nq:].reshape(T, nZ))
        return sum(loglik_exact(q.H, q.p, q.obs, mm) for mm in m)

    r0 = np.concatenate([pq, qm.ravel()])
    fd = central_difference(f, r0, [0, 4, 8, nq, nq + 5], 1e-5)
    np.testing.assert_allclose(gr[[0, 4, 8, nq, nq + 5]], fd, rtol=1e-6, atol=1e-6)


def test_frontier_handles_certain_mechanisms():
    # p_i in {0, 1} (used by the definition) gives the restricted sums.
    dem = synth.repetition_line(5, 0.1).with_p([0.1, 0.2, 0.3, 0.25, 0.15])
    m = np.array([1, 0, 0, 1], dtype=np.uint8)
    q = dem.p.copy()
    q[2] = 1.0
    lp = frontier_logprobs(dem.H, q, dem.obs, m)
    X = np.array(list(itertools.product((0, 1), repeat=5)))
    ok = np.all(((X @ dem.H.T.astype(int)) & 1) == m, axis=1) & (X[:, 2] == 1)
    w = np.prod(np.where(X == 1, q, 1 - q), axis=1) * ok
    for L in (0, 1):
        sel = (X @ dem.obs[0].astype(int)) % 2 == L
        ref = w[sel].sum()
        assert (np.exp(lp[L]) if ref > 0 else 0.0) == pytest.approx(ref, rel=1e-12, abs=0)


def test_one_sided_form_equals_brute_force_marginals():
    # Rates on both sides of 1/2, so both choices of c_i are used; the exact
    # frontier contraction as the evaluator; enumerated posterior marginals
    # (an independent computation) as the reference.
    dem = synth.rotated_phenom(3, 1, 0.05, 0.05)
    dem = dem.with_p(np.random.default_rng(11).uniform(0.02, 0.9, dem.n_mech))
    assert dem.n_mech <= 16
    m, _ = synth.sample_syndromes(dem, 4, 12)
    for k in range(4):
        lp, g = loglik_grad_one_sided(lambda q: frontier_logprobs(dem.H, q, dem.obs, m[k]), dem.p)
        lb, gb = _marginal_grad_brute(dem.H, dem.p, m[k])
        assert lp == pytest.approx(lb, abs=1e-12)
        np.testing.assert_allclose(g, gb, rtol=1e-10, atol=1e-10)


def test_one_sided_form_rate_range():
    # The depolarizing range [0, 3/4]: the step is 3/16; a one-mechanism
    # closed form P(m=1) = p fixes the derivative 1/p at any rate.
    def cosets(q):
        return [np.log(q[0]), -np.inf]

    for p0 in (0.05, 0.5, 0.7):
        lp, g = loglik_grad_one_sided(cosets, np.array([p0]), rate_max=0.75)
        assert lp == pytest.approx(np.log(p0), abs=1e-15)
        assert g[0] == pytest.approx(1.0 / p0, rel=1e-12)


def test_one_sided_form_with_the_sweep_at_untruncated_chi():
    # With the fixed-chi sweep as the evaluator at a chi that truncates
    # nothing, the gradient is the exact one (two-sided form, O-2).
    d, T = 3, 2
    dem = synth.rotated_phenom(d, T, 0.05, 0.05)
    dem = dem.with_p(np.random.default_rng(5).uniform(0.02, 0.3, dem.n_mech))
    m, _ = synth.sample_syndromes(dem, 2, 6)
    idx = [0, 7, 13, dem.n_mech - 1]
    for k in range(2):
        def cosets(q):
            return [sweep_logprob(rotated_network(d, T, dem.params["checks"], q, m[k], c), 16, 16, 1e-12,
                                  1e-9)[0] for c in (0, 1)]
        lp, g = loglik_grad_one_sided(cosets, dem.p, idx)
        le, ge = loglik_grad_exact(dem.H, dem.p, dem.obs, m[k])
        assert lp == pytest.approx(le, abs=1e-9)
        np.testing.assert_allclose(g, ge[idx], rtol=1e-8, atol=1e-8)


def test_one_sided_form_non_positive_cosets():
    # A coset an evaluator finds non-positive (NaN) counts as zero; every
    # coset NaN at the given rates gives NaN.  One mechanism, P_0 = 1 - p,
    # P_1 reported as NaN: log P = log(1 - p), d log P / d p = -1 / (1 - p).
    lp, g = loglik_grad_one_sided(lambda q: [np.log(1.0 - q[0]), np.nan], np.array([0.2]))
    assert lp == pytest.approx(np.log(0.8), abs=1e-15)
    assert g[0] == pytest.approx(-1.0 / 0.8, rel=1e-12)
    lp, g = loglik_grad_one_sided(lambda q: [np.nan, np.nan], np.array([0.2]))
    assert np.isnan(lp) and np.isnan(g[0])
