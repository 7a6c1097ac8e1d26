"""O-4: gradients of the syndrome log-likelihood with respect to the rates.

TEST INFRASTRUCTURE ONLY (see the package header).

The quantity (paper Sec. 2.4): for a DEM (H, p, l) and a syndrome m,

    P(m) = sum_L p_{m,L} = sum over x with H x = m of prod_i p_i^{x_i} (1 - p_i)^{1 - x_i}.

P(m) is affine in each p_i separately: splitting the sum by x_i,
    P(m) = (1 - p_i) P(m | p_i = 0) + p_i P(m | p_i = 1),
where P(m | p_i = c) is the same sum with rate i set to c.  Hence

    d log P(m) / d p_i = (P(m | p_i = 1) - P(m | p_i = 0)) / P(m),

which is the plain definition used here, evaluated with the exact frontier
contraction (O-2) once per mechanism and value.  Equivalently it is
(mu_i - p_i) / (p_i (1 - p_i)) with the posterior marginal
mu_i = P(x_i = 1 | m) = p_i P(m | p_i = 1) / P(m).

Rates shared by several mechanisms (one rate per data qubit over all rounds,
one per measurement event) get the sum of their mechanisms' derivatives
(chain rule through p_i = r_{k(i)}).

Pins (tests/test_oracle_grad.py): brute-force posterior marginals on tiny
codes (the marginal form above, enumerated independently), central finite
differences of O-2, and a two-mechanism closed form.

loglik_grad_one_sided evaluates the same derivative from one changed rate
per mechanism (a quarter of the admissible range away), with any evaluator
of the coset values (pinned to brute-force marginals and to the exact form
above; with the fixed-chi sweep it is the gradient the library computes at
equal chi).

Also here: central finite differences of the fixed-chi sweep (O-3), the
derivative of the *approximate* value that a reverse pass of the sweep
computes (ranks held fixed between the two evaluations).
"""

from __future__ import annotations

import numpy as np

from .exact import default_order, frontier_logprobs


def _logsumexp(v):
    v = np.asarray(v, dtype=np.float64)
    m = np.max(v)
    if not np.isfinite(m):
        return m
    return m + np.log(np.sum(np.exp(v - m)))


def loglik_exact(H, p, obs, m, order=None):
    """log P(m) = log sum_L p_{m,L} by the exact frontier contraction."""
    return _logsumexp(frontier_logprobs(H, p, obs, m, order=order))


def loglik_grad_exact(H, p, obs, m, order=None):
    """(log P(m), d log P(m) / d p_i for every mechanism i), exactly."""
    p = np.asarray(p, dtype=np.float64)
    if order is None:
        order = default_order(H)
    lp = loglik_exact(H, p, obs, m, order)
    g = np.empty(p.size)
    for i in range(p.size):
        q = p.copy()
        q[i] = 1.0
        l1 = loglik_exact(H, q, obs, m, order)
        q[i] = 0.0
        l0 = loglik_exact(H, q, obs, m, order)
        g[i] = np.exp(l1 - lp) - np.exp(l0 - lp)
    return lp, g


def loglik_grad_one_sided(cosets_logp, p, indices=None, rate_max=1.0):
    """The same derivative from one changed rate per mechanism, for any
    evaluator cosets_logp(rates) -> log p_{m,L} over the cosets (the exact
    contraction, or the fixed-chi sweep O-3 at a given chi and rank rule).
    P is affine in p_i, so for any c_i != p_i

        d log P / d p_i = (P(p_i = c_i) / P - 1) / (c_i - p_i).

    c_i steps a quarter of the admissible range [0, rate_max] away from p_i,
    towards its middle: c_i = p_i + rate_max / 4 if p_i <= rate_max / 2, else
    p_i - rate_max / 4.  Inside the range no term of a network vanishes that
    did not vanish at p_i, and P(p_i = c_i) > 0 whenever P > 0.

    An approximate evaluator returns a value it finds non-positive as NaN;
    such a coset counts as zero (its value is below the evaluator's own
    error).  If every coset is NaN, P at the given rates is NaN (and so the
    derivatives); a changed network's P is then zero.

    Returns (log P, the derivatives for `indices`, default every mechanism)."""
    p = np.asarray(p, dtype=np.float64)
    l0 = np.asarray(cosets_logp(p), dtype=np.float64)
    lp = np.nan if np.all(np.isnan(l0)) else _logsumexp(np.where(np.isnan(l0), -np.inf, l0))
    idx = list(range(p.size)) if indices is None else list(indices)
    h = 0.25 * rate_max
    g = np.empty(len(idx))
    for k, i in enumerate(idx):
        ci = p[i] + h if p[i] <= 0.5 * rate_max else p[i] - h
        q = p.copy()
        q[i] = ci
        lq = np.asarray(cosets_logp(q), dtype=np.float64)
        lq = np.where(np.isnan(lq), -np.inf, lq)
        g[k] = np.expm1(_logsumexp(lq) - lp) / (ci - p[i])
    return lp, g


def batch_loglik_grad_exact(H, p, obs, syndromes):
    """sum_s log P(m_s) and its gradient over a batch of syndromes."""
    order = default_order(H)
    tot, g = 0.0, np.zeros(np.asarray(p).size)
    for m in syndromes:
        l, gi = loglik_grad_exact(H, p, obs, m, order)
        tot += l
        g += gi
    return tot, g


def reduce_to_rates(g_mech, rate_of_mech, n_rates):
    """Chain rule for rates shared by mechanisms: g_r = sum_{i: k(i) = r} g_i."""
    out = np.zeros(n_rates)
    np.add.at(out, np.asarray(rate_of_mech), np.asarray(g_mech))
    return out


def central_difference(fun, p, indices, rel_step=1e-5):
    """(f(p + h e_i) - f(p - h e_i)) / 2h with h = rel_step * p_i, for i in indices."""
    p = np.asarray(p, dtype=np.float64)
    out = np.empty(len(indices))
    for k, i in enumerate(indices):
        h = rel_step * p[i]
        a = p.copy()
        a[i] += h
        b = p.copy()
        b[i] -= h
        out[k] = (fun(a) - fun(b)) / (2.0 * h)
    return out
