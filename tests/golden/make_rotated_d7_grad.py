"""Writes rotated_d7_grad.json: oracle derivatives d log P(m) / d p_i of the
rotated d=7 surface code with phenomenological noise (7 noisy rounds and one
perfect one, per-qubit and per-measurement rates drawn log-uniformly in
[0.005, 0.05] from seed 2310107325), for items 0, 85, 170 and 255 of the
256 seeded syndromes of that workload (seed 2310107225) and 25
mechanisms (24 drawn from seed 2024 plus the last one), at chi = chi_m = 16
under the
reduced-precision rank rule (eps_rel 1e-6, tau_gap 1e-2; the finer FP64
default rule cuts in rounding noise on this workload).

Each P(m) is the fixed-chi FP64 sweep (O-3) and the derivative is the
one-sided form of oracle.grad.loglik_grad_one_sided, computed twice, with the
divide-and-conquer and with the QR-iteration LAPACK SVD driver: their spread
is the FP64 conditioning of the problem.  Calls only oracle/ and synth/.
About two minutes on eight cores; run from the repository root:
    python tests/golden/make_rotated_d7_grad.py
"""

import json
import os
import sys
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"  # one thread per worker process (set before numpy loads)

import numpy as np  # noqa: E402

import synth  # noqa: E402
from oracle.grad import loglik_grad_one_sided  # noqa: E402
from oracle.network import rotated_network  # noqa: E402
from oracle.sweep import sweep_logprob  # noqa: E402

D, T, CHI, CHI_M, N = 7, 7, 16, 16, 256
ITEMS = [0, 85, 170, 255]
EPS, TAU = 1e-6, 1e-2
DRIVERS = ("gesdd", "gesvd")


def mechanisms(n_mech):
    rng = np.random.default_rng(2024)
    idx = sorted(int(i) for i in rng.choice(n_mech - 1, 24, replace=False))
    return idx + [n_mech - 1]


def one(args):
    drv, k = args
    dem, m, _, _ = synth.config_workload(5, N)
    idx = mechanisms(dem.n_mech)

    def cosets(q):
        return [sweep_logprob(rotated_network(D, T, dem.params["checks"], q, m[k], c), CHI, CHI_M, EPS, TAU,
                              svd_driver=drv)[0] for c in (0, 1)]

    lp, g = loglik_grad_one_sided(cosets, dem.p, idx)
    return drv, k, float(lp), [float(x) for x in g]


def main():
    dem, m, _, seed = synth.config_workload(5, N)
    idx = mechanisms(dem.n_mech)
    jobs = [(r, k) for r in DRIVERS for k in ITEMS]
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        res = pool.map(one, jobs)
    out = {"d": D, "T": T, "chi": CHI, "chi_mps": CHI_M, "seed": seed, "n": N, "items": ITEMS,
           "mechanisms": idx, "rule": [EPS, TAU],
           "syndromes": m[ITEMS].astype(int).tolist(), "p": [float(dem.p[i]) for i in idx],
           "loglik": {r: [None] * len(ITEMS) for r in DRIVERS}, "grad": {r: [None] * len(ITEMS) for r in DRIVERS}}
    for r, k, lp, g in res:
        out["loglik"][r][ITEMS.index(k)] = lp
        out["grad"][r][ITEMS.index(k)] = g
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "rotated_d7_grad.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
