"""Writes depol_L3_exact.json: exact log coset probabilities (O-2 frontier
contraction of the DEM form) of the 3D planar code at L=3 under depolarizing
noise p = 0.15, for three seeded syndromes and all four cosets c = a + 2b.

The DEM form draws X, Y and Z independently per qubit, each at rate r with
r (1 - r) = p/3 (that it reproduces the depolarizing channel is pinned against
Pauli enumeration at L = 2 in the tests).  The mechanisms are ordered by the
height of their qubit (z-edges between levels, in-plane edges on them), which
keeps the frontier small enough for an exact contraction in a couple of
minutes per syndrome.  Calls only oracle/ and synth/.  Run from the
repository root:
    python tests/golden/make_depol_L3_exact.py
"""

import json
import os
import sys
from multiprocessing import Pool

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle.exact import frontier_logprobs  # noqa: E402

L, P, SEED, N = 3, 0.15, 2310107224, 3


def height_order(L, n):
    """Mechanism order (X, Y, Z of each qubit together) by qubit height, then row,
    then column: the z-edge from level z sits at 2z+1, in-plane edges of level z
    at 2z."""
    nz, nx = L ** 3, L * (L - 1) ** 2
    key = []
    for e in range(n):
        if e < nz:
            key.append((2 * (e // (L * L)) + 1, (e // L) % L, e % L))
        elif e < nz + nx:
            i = e - nz
            key.append((2 * (i // ((L - 1) * L) + 1), (i // (L - 1)) % L, i % (L - 1)))
        else:
            i = e - nz - nx
            key.append((2 * (i // (L * (L - 1)) + 1), (i // L) % (L - 1), i % L))
    return sorted(range(3 * n), key=lambda i: (key[i % n], i // n))


def one(k):
    dem = synth.surface3d_depolarizing(L, P)
    m, _ = synth.sample_pauli(dem, N, SEED)
    order = height_order(L, dem.params["n_qubits"])
    return k, [float(v) for v in frontier_logprobs(dem.H, dem.p, dem.obs, m[k], order=order)]


def main():
    dem = synth.surface3d_depolarizing(L, P)
    m, cos = synth.sample_pauli(dem, N, SEED)
    with Pool(N) as pool:
        res = dict(pool.map(one, range(N)))
    out = {"L": L, "p": P, "seed": SEED, "syndromes": m.astype(int).tolist(),
           "true_coset": cos.astype(int).tolist(), "logp": [res[k] for k in range(N)]}
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "depol_L3_exact.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
