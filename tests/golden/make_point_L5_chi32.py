"""Writes point_L5_chi32.json: oracle (fixed-chi FP64 sweep) log coset
probabilities for the 3D planar code, point sector, L=5, p=0.2, at chi = 32
and chi_m = 4, for four seeded syndromes, under the default FP64 rank rule
(eps_rel 1e-9, tau_gap 1e-6) and the reduced one (1e-6, 1e-4).

At this size the layer bonds reach 32, so the GPU path takes its widest layer
classes: Grams of 64 columns, truncations of order 64, reabsorption rows of 64.
chi_m = 4 keeps the boundary-MPS families at 4 * 32 = 128 vectors or fewer.
Calls only oracle/ and synth/.  Run from the repository root:
    python tests/golden/make_point_L5_chi32.py
"""

import json
import os
import sys
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.network import point3d_network  # noqa: E402
from oracle.sweep import sweep_logprob  # noqa: E402

L, P, CHI, CHI_M, SEED, N = 5, 0.2, 32, 4, 2310107223, 4
RULES = {"fp64_default": (1e-9, 1e-6), "reduced": (1e-6, 1e-4)}


def one(args):
    k, c, rule = args
    dem = synth.surface3d_point(L, P)
    m, _ = synth.sample_syndromes(dem, N, SEED)
    eps, tau = RULES[rule]
    lp = sweep_logprob(point3d_network(L, dem.p, m[k], c), CHI, CHI_M, eps, tau)[0]
    return rule, k, c, float(lp)


def main():
    dem = synth.surface3d_point(L, P)
    m, _ = synth.sample_syndromes(dem, N, SEED)
    jobs = [(k, c, r) for r in RULES for k in range(N) for c in range(2)]
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        res = pool.map(one, jobs)
    out = {"L": L, "p": P, "chi": CHI, "chi_mps": CHI_M, "seed": SEED,
           "syndromes": m.astype(int).tolist(), "rules": {r: list(v) for r, v in RULES.items()},
           "logp": {r: [[None, None] for _ in range(N)] for r in RULES}}
    for rule, k, c, lp in res:
        out["logp"][rule][k][c] = lp
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "point_L5_chi32.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
