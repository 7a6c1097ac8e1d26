"""Pins for the dense layered-network evaluator (oracle/dense.py)."""

import numpy as np
import pytest

from layered_inputs import random_description, to_layered
from oracle.dense import layered_value
from oracle.network import Layer, LayeredNet
from oracle.sweep import sweep_logprob


def test_closed_forms_on_a_2x2_grid():
    # product state u, one-site op M on site 0 and one gate G on (0,0)-(1,0):
    # value = sum f0[a'] f1[b'] G[a',b',a,b] (M u0)[a] u1[b] * (f2.u2) (f3.u3)
    rng = np.random.default_rng(1)
    u = [rng.uniform(0.1, 1, 2) for _ in range(4)]
    f = [rng.uniform(0.1, 1, 2) for _ in range(4)]
    M = rng.uniform(0, 1, (3, 2))
    f[0] = rng.uniform(0.1, 1, 3)
    G = rng.uniform(0, 1, (3, 2, 3, 2))
    lay = Layer(pre={0: M}, gates=[("H", 0, 0, G)])
    net = LayeredNet(Lx=2, Ly=2, init=[v.reshape(2, 1, 1, 1, 1) for v in u], layers=[lay], final=f)
    want = np.einsum("a,b,abcd,c,d->", f[0], f[1], G, M @ u[0], u[1]) * (f[2] @ u[2]) * (f[3] @ u[3])
    assert layered_value(net) == pytest.approx(want, rel=1e-14)


def test_gate_class_order():
    # two gates sharing site 1 in one layer: (0,0)-(1,0) is class "x even",
    # (1,0)-(2,0) class "x odd", so the first acts first whatever the list
    # order; swapping them in the list leaves the value unchanged, applying
    # them in the other order changes it
    rng = np.random.default_rng(2)
    u = [rng.uniform(0.1, 1, 2).reshape(2, 1, 1, 1, 1) for _ in range(6)]
    f = [rng.uniform(0.1, 1, 2) for _ in range(6)]
    G1, G2 = rng.uniform(0, 1, (2, 2, 2, 2)), rng.uniform(0, 1, (2, 2, 2, 2))
    a = layered_value(LayeredNet(3, 2, u, [Layer(gates=[("H", 0, 0, G1), ("H", 1, 0, G2)])], f))
    b = layered_value(LayeredNet(3, 2, u, [Layer(gates=[("H", 1, 0, G2), ("H", 0, 0, G1)])], f))
    assert a == b
    v = np.einsum("i,j,k->ijk", *[x.reshape(2) for x in u[:3]])
    v1 = np.einsum("abij,ijk->abk", G1, v)
    v2 = np.einsum("bcjk,ajk->abc", G2, v1)
    want = np.einsum("abc,a,b,c->", v2, *f[:3]) * np.prod([f[s] @ u[s].reshape(2) for s in range(3, 6)])
    assert a == pytest.approx(want, rel=1e-13)


@pytest.mark.parametrize("seed", [3, 4])
def test_equals_the_untruncated_sweep(seed):
    # a random 3 x 3 network (two layers, dims changing on site 0): the
    # fixed-chi sweep at a chi that truncates nothing (O-3, pinned exact on the
    # code families) gives the same value
    desc = random_description(3, 3, 2, 2, 2, seed)
    for bits in ((0, 0), (1, 0), (0, 1)):
        for c in range(2):
            net = to_layered(desc, bits, c)
            lp, _, _ = sweep_logprob(net, 64, 256, 1e-14, 1e-12)
            assert lp == pytest.approx(np.log(layered_value(net)), abs=1e-10)
