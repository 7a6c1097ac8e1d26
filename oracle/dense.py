"""Dense contraction of a small layered network whose initial state is a
product state (every initial bond of dimension 1): the plain definition of
the network's value, for the generic layered front end.

TEST INFRASTRUCTURE ONLY (see the package header).

The value of a layered network (paper Sec. 4: an initial boundary state, then
layers of one-site operators and two-site operators, closed by a vector on
every physical leg) is

    f^T (L_{n-1} ... L_1 L_0) psi_0,

with psi_0 the tensor product of the initial site vectors and L_l the
operator of layer l: its one-site operators before the gates, then its
two-site operators in the four bond classes (x, y)-(x+1, y) with x even, x
odd, then (x, y)-(x, y+1) with y even, y odd (two-site operators of one
class act on disjoint pairs of sites and commute), then its one-site
operators after the gates.  Here the state is kept as a dense tensor with one
axis per site (site s = y Lx + x), so only a few thousand amplitudes fit.
"""

from __future__ import annotations

import numpy as np

from .network import LayeredNet


def _apply_one(psi, M, s):
    """M (d_out x d_in) on axis s."""
    out = np.tensordot(M, psi, axes=([1], [s]))
    return np.moveaxis(out, 0, s)


def _apply_two(psi, G, a, b):
    """G[a', b', a, b] on axes a, b."""
    out = np.tensordot(G, psi, axes=([2, 3], [a, b]))
    return np.moveaxis(out, [0, 1], [a, b])


def layered_value(net: LayeredNet):
    """The network's value (float)."""
    Lx, Ly = net.Lx, net.Ly
    n = Lx * Ly
    vecs = []
    for T in net.init:
        if any(dim != 1 for dim in T.shape[1:]):
            raise ValueError("dense evaluation needs a product initial state (bond dimensions 1)")
        vecs.append(T.reshape(T.shape[0]))
    psi = vecs[0]
    for v in vecs[1:]:
        psi = np.multiply.outer(psi, v)
    psi = psi.reshape([v.size for v in vecs])
    for lay in net.layers:
        for s, M in lay.pre.items():
            psi = _apply_one(psi, M, s)
        for cls in range(4):
            for kind, x, y, G in lay.gates:
                c = (x % 2) if kind == "H" else 2 + (y % 2)
                if c != cls:
                    continue
                a = y * Lx + x
                b = a + 1 if kind == "H" else a + Lx
                psi = _apply_two(psi, G, a, b)
        for s, M in lay.post.items():
            psi = _apply_one(psi, M, s)
    for s in range(n):
        psi = np.tensordot(psi, net.final[s], axes=([0], [0]))
    return float(psi)
