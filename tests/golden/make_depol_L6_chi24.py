"""Writes depol_L6_chi24.json: oracle (fixed-chi FP64 sweep) log coset
probabilities of the 3D planar code at L=6 under depolarizing noise p = 0.15
at chi = chi_m = 24 and the reduced-precision rank rule (eps_rel 1e-6,
tau_gap 1e-2), for items 0 and 3 of the 170 seeded syndromes that the
depolarizing workload draws at L=6 (seed 2310107224 + 6), all four cosets.

At this chi the gated truncations reach order 3 x 24 = 72 and the gate sides
4 x 24 = 96 columns.  Calls only oracle/ and synth/.  About a minute on eight
cores; run from the repository root:
    python tests/golden/make_depol_L6_chi24.py
"""

import json
import os
import sys
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
for _v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_v] = "1"  # one thread per worker process (set before numpy loads)

import synth  # noqa: E402
from oracle.network import depol3d_network  # noqa: E402
from oracle.sweep import sweep_logprob  # noqa: E402

L, P, CHI, SEED, N = 6, 0.15, 24, 2310107224 + 6, 170
ITEMS = [0, 3]
EPS, TAU = 1e-6, 1e-2


def draw():
    dem = synth.surface3d_depolarizing(L, P)
    m, _ = synth.sample_pauli(dem, N, SEED)
    return dem, m


def one(args):
    k, c = args
    dem, m = draw()
    lp, flags, nsplit = sweep_logprob(depol3d_network(L, dem.params["p_qubit"], m[k], c), CHI, CHI, EPS, TAU)
    return k, c, float(lp), int(flags)


def main():
    dem, m = draw()
    jobs = [(k, c) for k in ITEMS for c in range(4)]
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        res = pool.map(one, jobs)
    out = {"L": L, "p": P, "chi": CHI, "chi_mps": CHI, "seed": SEED, "n": N, "items": ITEMS, "rule": [EPS, TAU],
           "syndromes": m[ITEMS].astype(int).tolist(), "logp": [[None] * 4 for _ in ITEMS],
           "flags": [[0] * 4 for _ in ITEMS]}
    for k, c, lp, fl in res:
        out["logp"][ITEMS.index(k)][c] = lp
        out["flags"][ITEMS.index(k)][c] = fl
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "depol_L6_chi24.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
