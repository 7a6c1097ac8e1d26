"""Exact coset probabilities: brute force (O-1) and frontier contraction (O-2).

Definition (paper Sec. 2.4, the joint probability of detector outcome m and
logical value L for a DEM (H, p, l)):

    p_{m,L} = sum over x in F2^n with H x = m and l x = L of
              prod_i p_i^{x_i} (1 - p_i)^{1 - x_i},

and the optimal decision is argmax_L p_{m,L}.  For a stabilizer code with a
product Pauli distribution the same quantity is the probability of the coset
s * d(m) * l summed over stabilizers s (paper Sec. 2.3, eq. optimal_decoder);
`pauli_coset_probs` evaluates that form by enumerating Paulis.

Pins (tests/test_oracle_exact.py): the repetition-code closed form, the
normalisation sum_m sum_L p_{m,L} = 1, the p = 1/2 closed form
2^-rank[H; l], agreement of O-2 with O-1 on every syndrome of small codes,
and the [[5,1,3]] code's correction of all weight-one errors.
"""

from __future__ import annotations

import numpy as np


# ---------------------------------------------------------------------------
# O-1: brute force
# ---------------------------------------------------------------------------

def brute_force_table(H, p, obs, chunk: int = 1 << 18):
    """Table P[m_int, L_int] of p_{m,L} over all syndromes (n_det <= 22, n <= 24).

    Syndrome integer: bit i is detector i.  Observable integer: bit k is
    observable k.
    """
    H = np.asarray(H, dtype=np.int64)
    obs = np.asarray(obs, dtype=np.int64)
    p = np.asarray(p, dtype=np.float64)
    n_det, n = H.shape
    n_obs = obs.shape[0]
    if n > 24 or n_det > 22:
        raise ValueError("brute force limited to n <= 24, n_det <= 22")
    table = np.zeros((1 << n_det, 1 << n_obs), dtype=np.float64)
    logp = np.log(p)
    log1p = np.log1p(-p)
    det_w = (1 << np.arange(n_det, dtype=np.int64))
    obs_w = (1 << np.arange(n_obs, dtype=np.int64))
    total = 1 << n
    for start in range(0, total, chunk):
        ints = np.arange(start, min(total, start + chunk), dtype=np.int64)
        bits = (ints[:, None] >> np.arange(n, dtype=np.int64)[None, :]) & 1
        w = np.exp(bits @ logp + (1 - bits) @ log1p)
        mint = ((bits @ H.T) & 1) @ det_w
        lint = ((bits @ obs.T) & 1) @ obs_w
        np.add.at(table, (mint, lint), w)
    return table


def syndrome_int(m) -> int:
    m = np.asarray(m, dtype=np.int64)
    return int((m << np.arange(m.size, dtype=np.int64)).sum())


def pauli_coset_probs(stabs, logicals, probs, syndrome):
    """Coset probabilities of a stabilizer code by enumerating all 4^n Paulis.

    stabs: generator strings over {I,X,Y,Z}; logicals: the logical generators
    (x_1.., z_1..); probs: per-qubit dict {'I','X','Y','Z'} -> probability;
    syndrome: tuple of generator outcomes.  A Pauli's syndrome bit is its
    symplectic product with the generator, and its logical label is the tuple of
    symplectic products with the logical generators (paper Sec. 2.1-2.3).
    Returns {logical label tuple: probability}.
    """
    n = len(stabs[0])

    def uv(s):
        u = np.array([c in "XY" for c in s], dtype=np.int64)
        v = np.array([c in "ZY" for c in s], dtype=np.int64)
        return u, v

    S = [uv(s) for s in stabs]
    Lg = [uv(s) for s in logicals]
    out = {}
    letters = "IXYZ"
    for code in range(4 ** n):
        s = []
        c = code
        for _ in range(n):
            s.append(letters[c & 3])
            c >>= 2
        u, v = uv(s)
        syn = tuple(int((u @ sv + v @ su) & 1) for su, sv in S)
        if syn != tuple(syndrome):
            continue
        lab = tuple(int((u @ lv + v @ lu) & 1) for lu, lv in Lg)
        w = 1.0
        for q in range(n):
            w *= probs[q][s[q]]
        out[lab] = out.get(lab, 0.0) + w
    return out


# ---------------------------------------------------------------------------
# O-2: exact frontier contraction
# ---------------------------------------------------------------------------

def default_order(H, det_coord=None):
    """Mechanism order for the frontier: by the first detector each touches
    (detectors in canonical order), ties by the last."""
    H = np.asarray(H)
    n = H.shape[1]
    keys = []
    for i in range(n):
        ds = np.nonzero(H[:, i])[0]
        if ds.size == 0:
            keys.append((-1, -1, i))
        else:
            keys.append((int(ds.min()), int(ds.max()), i))
    keys.sort()
    return [k[2] for k in keys]


def frontier_logprobs(H, p, obs, m, order=None, max_open: int = 26):
    """log p_{m,L} for every L (array of length 2^n_obs), exactly.

    The sum over x is evaluated mechanism by mechanism: the state is a table
    over the parities of the currently open detectors and the observables.  A
    mechanism i multiplies the table by (1 - p_i) and adds p_i times the table
    with the parities of its detectors and observables flipped; a detector is
    opened (parity 0) when first touched and, after its last mechanism, the
    table is restricted to parity m_d.  A per-step rescaling feeds a log-scale
    accumulator.
    """
    H = np.asarray(H, dtype=np.uint8)
    obs = np.asarray(obs, dtype=np.uint8)
    p = np.asarray(p, dtype=np.float64)
    m = np.asarray(m, dtype=np.uint8)
    n_det, n = H.shape
    n_obs = obs.shape[0]
    if order is None:
        order = default_order(H)
    touched = H.any(axis=1)
    if np.any(m[~touched] != 0):
        return np.full(1 << n_obs, -np.inf)
    last = np.full(n_det, -1)
    for step, i in enumerate(order):
        for dd in np.nonzero(H[:, i])[0]:
            last[dd] = step
    # axes: observables first (fixed), then open detectors in opening order
    psi = np.zeros((2,) * n_obs)
    psi[(0,) * n_obs] = 1.0
    axis_of = {}  # detector -> axis position
    open_list = []
    logscale = 0.0
    for step, i in enumerate(order):
        dets = np.nonzero(H[:, i])[0]
        for dd in dets:
            if dd not in axis_of:
                psi = np.stack([psi, np.zeros_like(psi)], axis=-1)
                axis_of[dd] = psi.ndim - 1
                open_list.append(dd)
        if len(open_list) > max_open:
            raise ValueError("frontier too large")
        axes = [axis_of[dd] for dd in dets] + [k for k in range(n_obs) if obs[k, i]]
        if axes:
            psi = (1.0 - p[i]) * psi + p[i] * np.flip(psi, axis=tuple(axes))
        closing = [dd for dd in dets if last[dd] == step]
        for dd in sorted(closing, key=lambda q: -axis_of[q]):
            ax = axis_of.pop(dd)
            psi = np.take(psi, int(m[dd]), axis=ax)
            open_list.remove(dd)
            for q in axis_of:
                if axis_of[q] > ax:
                    axis_of[q] -= 1
        s = np.max(np.abs(psi))
        if s == 0.0:
            return np.full(1 << n_obs, -np.inf)
        psi = psi / s
        logscale += np.log(s)
    assert not open_list
    flat = np.zeros(1 << n_obs)
    for lint in range(1 << n_obs):
        idx = tuple((lint >> k) & 1 for k in range(n_obs))
        flat[lint] = psi[idx]
    with np.errstate(divide="ignore"):
        return np.log(flat) + logscale
