"""Writes loop_L8_chi32.json: oracle (fixed-chi FP64 sweep) log coset
probabilities of the 3D planar code, loop sector (bit flips seen by the face
checks, generator picture), L=8, p=0.2, chi = chi_m = 32, reduced-precision rank rule
(eps_rel 1e-6, tau_gap 1e-2), for items 0, 85, 170 and 255 of the 256 seeded
syndromes of that workload (seed 2310107223, the error draws of the point
sector's workload).

At this size the layer bonds reach 32 (site tensors of 2 * 32^4 entries) and
the boundary-MPS families reach 32 * 32 = 1024 vectors.  Calls only oracle/
and synth/.  About a minute per coset on one core; run from the repository
root:
    python tests/golden/make_loop_L8_chi32.py
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
from oracle.network import loop3d_network  # noqa: E402
from oracle.sweep import sweep_logprob  # noqa: E402

L, P, CHI, CHI_M, SEED, N = 8, 0.2, 32, 32, 2310107223, 256
ITEMS = [0, 85, 170, 255]
EPS, TAU = 1e-6, 1e-2


def one(args):
    k, c = args
    dem = synth.surface3d_loop(L, P)
    m, _ = synth.sample_syndromes(dem, N, SEED)
    lp, flags, nsplit = sweep_logprob(loop3d_network(L, dem.p, m[k], c), CHI, CHI_M, EPS, TAU)
    return k, c, float(lp), int(flags), int(nsplit)


def main():
    dem = synth.surface3d_loop(L, P)
    m, _ = synth.sample_syndromes(dem, N, SEED)
    jobs = [(k, c) for k in ITEMS for c in range(2)]
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        res = pool.map(one, jobs)
    out = {"L": L, "p": P, "chi": CHI, "chi_mps": CHI_M, "seed": SEED, "n": N, "items": ITEMS,
           "rule": [EPS, TAU], "syndromes": m[ITEMS].astype(int).tolist(),
           "logp": [[None, None] for _ in ITEMS], "flags": [[0, 0] for _ in ITEMS]}
    for k, c, lp, fl, ns in res:
        out["logp"][ITEMS.index(k)][c] = lp
        out["flags"][ITEMS.index(k)][c] = fl
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "loop_L8_chi32.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
