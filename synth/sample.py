"""Seeded error sampling: x ~ Bernoulli(p_i) independently, m = H x mod 2.

The generator is numpy's PCG64 seeded with CONFIG_SEED_BASE + workload number,
so every consumer (tests, benchmark, oracle timing) sees the same syndromes.
"""

from __future__ import annotations

import numpy as np

from .codes import surface3d_loop, Dem, rotated_phenom, surface3d_depolarizing, surface3d_point

CONFIG_SEED_BASE = 2310107220


def sample_syndromes(dem: Dem, n: int, seed: int):
    """Return (syndromes uint8 [n, n_det], observables uint8 [n, n_obs])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = (rng.random((n, dem.n_mech)) < dem.p[None, :]).astype(np.uint8)
    H = dem.H.astype(np.int64)
    m = ((x.astype(np.int64) @ H.T) & 1).astype(np.uint8)
    obs = ((x.astype(np.int64) @ dem.obs.T.astype(np.int64)) & 1).astype(np.uint8)
    return m, obs


def sample_pauli(dem: Dem, n: int, seed: int):
    """Depolarizing sampling for a code built by surface3d_depolarizing: per
    qubit, u < 1-p gives I, otherwise X, Y, Z by equal thirds of [1-p, 1).
    Returns (syndromes uint8 [n, n_det], coset int64 [n]) with coset = a + 2b."""
    pr = dem.params
    pq = pr["p_qubit"]
    rng = np.random.Generator(np.random.PCG64(seed))
    uni = rng.random((n, pq.size))
    hit = uni >= 1.0 - pq[None, :]
    kind = np.minimum(((uni - (1.0 - pq[None, :])) / (pq[None, :] / 3.0)).astype(np.int64), 2)
    xp = (hit & (kind <= 1)).astype(np.int64)   # X or Y
    zp = (hit & (kind >= 1)).astype(np.int64)   # Y or Z
    m = np.concatenate([(zp @ pr["HX"].T.astype(np.int64)) & 1,
                        (xp @ pr["HZ"].T.astype(np.int64)) & 1], axis=1).astype(np.uint8)
    a = (xp @ pr["zbar"].astype(np.int64)) & 1
    b = (zp @ pr["xbar"].astype(np.int64)) & 1
    return m, a + 2 * b


def rotated_rates(d: int, T: int, seed: int, lo: float = 0.005, hi: float = 0.05):
    """Per-qubit (d*d, shared by all rounds) and per-measurement-event (T, nZ)
    rates drawn log-uniformly in [lo, hi]."""
    nZ = (d * d - 1) // 2
    rng = np.random.Generator(np.random.PCG64(seed))
    pq = np.exp(rng.uniform(np.log(lo), np.log(hi), size=d * d))
    qm = np.exp(rng.uniform(np.log(lo), np.log(hi), size=(T, nZ)))
    return pq, qm


def config_workload(cfg: int, n: int | None = None):
    """The synthetic workloads, by number.

    1: 3D planar code L=3, point sector, i.i.d. p=0.15, 64 syndromes.
    2: rotated d=5, p=q=0.03, 5 noisy + 1 perfect round, 1024 syndromes.
    3: 3D planar code L=8, point sector, p=0.2, 256 syndromes.
    4: 3D planar code, depolarizing p=0.15, L=4 (pass n; the ragged
       L in {4, 5, 6} mix is one call per L), coset labels instead of
       observables.
    5: rotated d=7, 7 noisy + 1 perfect round, per-qubit / per-measurement
       rates log-uniform in [0.005, 0.05] (drawn first, seed + 100), 256 syndromes.
    6: 3D planar code L=8, loop sector (bit flips seen by the faces), p=0.2,
       256 syndromes; the error draws of workload 3 (same seed and edges).
    Returns (dem, syndromes, observables, seed).
    """
    seed = CONFIG_SEED_BASE + cfg
    if cfg == 1:
        dem = surface3d_point(3, 0.15)
        n = 64 if n is None else n
    elif cfg == 2:
        dem = rotated_phenom(5, 5, 0.03, 0.03)
        n = 1024 if n is None else n
    elif cfg == 3:
        dem = surface3d_point(8, 0.2)
        n = 256 if n is None else n
    elif cfg == 4:
        dem = surface3d_depolarizing(4, 0.15)
        n = 512 if n is None else n
        m, cos = sample_pauli(dem, n, seed)
        return dem, m, cos, seed
    elif cfg == 6:
        dem = surface3d_loop(8, 0.2)
        n = 256 if n is None else n
        seed = CONFIG_SEED_BASE + 3
    elif cfg == 5:
        pq, qm = rotated_rates(7, 7, seed + 100)
        dem = rotated_phenom(7, 7, pq, qm)
        dem.params["p_qubit"] = pq
        dem.params["q_meas"] = qm
        n = 256 if n is None else n
    else:
        raise ValueError(f"no workload {cfg}")
    m, obs = sample_syndromes(dem, n, seed)
    return dem, m, obs, seed
