"""Seeded generic layered networks for the tests of the generic front end:
a description with syndrome-dependent ops, its flat C-ABI form, and the
oracle's LayeredNet for one syndrome and coset.  Data layout only (no part of
the contraction)."""

from __future__ import annotations

import numpy as np

from oracle.network import Layer, LayeredNet

OP_PRE, OP_GATE_H, OP_GATE_V, OP_POST = 0, 1, 2, 3


def random_description(Lx, Ly, n_layers, n_det, n_cosets, seed, d=2, d_mid=3):
    """Product initial states (positive entries); per layer a one-site op
    before the gates on three sites (the first two syndrome-dependent),
    dense positive two-site gates on every bond (about a quarter
    syndrome-dependent) and a one-site op after the gates on one site;
    positive final vectors.  Site 0 changes its physical dim: d -> d_mid by
    the first layer's op before the gates, back to d by the last layer's op
    after them."""
    rng = np.random.default_rng(seed)
    ns = Lx * Ly
    dims = [d] * ns
    init = [[rng.uniform(0.2, 1.0, d) for _ in range(ns)] for _ in range(n_cosets)]
    layers = []
    for l in range(n_layers):
        ops = []
        sites = [0] + [int(s) for s in rng.choice(np.arange(1, ns), size=2, replace=False)]
        for k, s in enumerate(sites):
            dout = d_mid if (l == 0 and s == 0) else dims[s]
            det = k % n_det if (n_det > 0 and k < 2) else -1
            M0 = rng.uniform(0.0, 1.0, (dout, dims[s]))
            M1 = rng.uniform(0.0, 1.0, (dout, dims[s])) if det >= 0 else None
            ops.append(("pre", s, det, M0, M1))
            dims[s] = dout
        for y in range(Ly):
            for x in range(Lx):
                for kind in ("H", "V"):
                    if (kind == "H" and x + 1 >= Lx) or (kind == "V" and y + 1 >= Ly):
                        continue
                    a = y * Lx + x
                    b = a + 1 if kind == "H" else a + Lx
                    det = int(rng.integers(n_det)) if (n_det > 0 and rng.uniform() < 0.25) else -1
                    shape = (dims[a], dims[b], dims[a], dims[b])
                    G0 = rng.uniform(0.0, 1.0, shape)
                    G1 = rng.uniform(0.0, 1.0, shape) if det >= 0 else None
                    ops.append((kind, x, y, det, G0, G1))
        s = 0 if l == n_layers - 1 else int(rng.integers(1, ns))
        dout = d if s == 0 else dims[s]
        ops.append(("post", s, -1, rng.uniform(0.0, 1.0, (dout, dims[s])), None))
        dims[s] = dout
        layers.append(ops)
    final = [rng.uniform(0.2, 1.0, dims[s]) for s in range(ns)]
    return {"Lx": Lx, "Ly": Ly, "n_det": n_det, "n_cosets": n_cosets, "init": init, "layers": layers,
            "final": final}


def to_abi(desc):
    """(init_dims, init_off, ops, final_off, values) for tn3d_net_from_layers."""
    values = []

    def put(a):
        off = sum(v.size for v in values)
        values.append(np.ascontiguousarray(a, dtype=np.float64).reshape(-1))
        return off

    ns = desc["Lx"] * desc["Ly"]
    init_dims = np.zeros((desc["n_cosets"], ns, 5), dtype=np.int32)
    init_off = np.zeros((desc["n_cosets"], ns), dtype=np.int64)
    for c, vecs in enumerate(desc["init"]):
        for s, v in enumerate(vecs):
            init_dims[c, s] = (v.size, 1, 1, 1, 1)
            init_off[c, s] = put(v)
    ops = []
    for l, lay in enumerate(desc["layers"]):
        for op in lay:
            if op[0] in ("pre", "post"):
                _, s, det, M0, M1 = op
                o1 = put(M1) if M1 is not None else 0
                ops.append((l, OP_PRE if op[0] == "pre" else OP_POST, s % desc["Lx"], s // desc["Lx"],
                            M0.shape[1], M0.shape[0], det, put(M0), o1))
            else:
                kind, x, y, det, G0, G1 = op
                o1 = put(G1) if G1 is not None else 0
                ops.append((l, OP_GATE_H if kind == "H" else OP_GATE_V, x, y, G0.shape[0], G0.shape[1], det,
                            put(G0), o1))
    final_off = np.array([put(f) for f in desc["final"]], dtype=np.int64)
    return init_dims, init_off, ops, final_off, np.concatenate(values)


def to_layered(desc, bits, coset):
    """The oracle's LayeredNet of one syndrome (bits) and coset: each op with
    its syndrome-selected values, one-site ops of a phase on a site composed
    in order."""
    Lx, Ly = desc["Lx"], desc["Ly"]
    init = [v.reshape(v.size, 1, 1, 1, 1).copy() for v in desc["init"][coset]]
    layers = []
    for lay in desc["layers"]:
        L = Layer()
        for op in lay:
            if op[0] in ("pre", "post"):
                _, s, det, M0, M1 = op
                M = M1 if (det >= 0 and bits[det]) else M0
                tgt = L.pre if op[0] == "pre" else L.post
                tgt[s] = M @ tgt[s] if s in tgt else M.copy()
            else:
                kind, x, y, det, G0, G1 = op
                L.gates.append((kind, x, y, G1 if (det >= 0 and bits[det]) else G0))
        layers.append(L)
    return LayeredNet(Lx=Lx, Ly=Ly, init=init, layers=layers, final=[f.copy() for f in desc["final"]])


def from_layered(net: LayeredNet):
    """A one-coset description with no syndrome-dependent ops, from an
    oracle LayeredNet (its initial tensors may carry bonds)."""
    return {"Lx": net.Lx, "Ly": net.Ly, "n_det": 0, "n_cosets": 1, "init_tensors": [net.init],
            "layers": [[("pre", s, -1, M, None) for s, M in sorted(L.pre.items())] +
                       [(k, x, y, -1, G, None) for (k, x, y, G) in L.gates] +
                       [("post", s, -1, M, None) for s, M in sorted(L.post.items())] for L in net.layers],
            "final": net.final}


def to_abi_tensors(desc):
    """to_abi for descriptions with initial tensors (p, w, e, n, s)."""
    values = []

    def put(a):
        off = sum(v.size for v in values)
        values.append(np.ascontiguousarray(a, dtype=np.float64).reshape(-1))
        return off

    ns = desc["Lx"] * desc["Ly"]
    tens = desc["init_tensors"]
    init_dims = np.zeros((len(tens), ns, 5), dtype=np.int32)
    init_off = np.zeros((len(tens), ns), dtype=np.int64)
    for c, ts in enumerate(tens):
        for s, T in enumerate(ts):
            init_dims[c, s] = T.shape
            init_off[c, s] = put(T)
    ops = []
    for l, lay in enumerate(desc["layers"]):
        for op in lay:
            if op[0] in ("pre", "post"):
                _, s, det, M0, M1 = op
                ops.append((l, OP_PRE if op[0] == "pre" else OP_POST, s % desc["Lx"], s // desc["Lx"],
                            M0.shape[1], M0.shape[0], -1, put(M0), 0))
            else:
                kind, x, y, det, G0, G1 = op
                ops.append((l, OP_GATE_H if kind == "H" else OP_GATE_V, x, y, G0.shape[0], G0.shape[1], -1,
                            put(G0), 0))
    final_off = np.array([put(f) for f in desc["final"]], dtype=np.int64)
    return init_dims, init_off, ops, final_off, np.concatenate(values)
