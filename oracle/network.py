"""Layered 3D tensor networks whose contraction is p_{m,L}, built per syndrome.

These are the detector-picture networks of the paper (Sec. 3.1, 3.3, 3.4) for
independent flips on CSS codes, arranged as stacks of identical layers over a
2D grid (Sec. 4: layered networks; Sec. 5.1: bond tensors on horizontal bonds
go into two-site gates, those on vertical bonds are contracted exactly between
layers).  The logical check node is replaced by a parity chain ("snake") over
the first layer's dangling legs, so each coset is one network with
non-negative entries (one positive network per coset instead of the
Walsh-Hadamard combination of Sec. 3.1.2; both give the same probabilities).

A network is described by plain Python objects:

  LayeredNet.Lx, Ly        grid; site (x, y) has index y*Lx + x
  LayeredNet.init          per site a tensor G[p, w, e, n, s] (float64)
  LayeredNet.layers        list of Layer
  LayeredNet.final         per site the vector f_s contracted with the
                           physical leg after the last layer

  Layer.pre / Layer.post   {site: matrix (d_out x d_in)} one-site ops
  Layer.gates              list of (kind, x, y, G4) with kind 'H' for the bond
                           (x,y)-(x+1,y) and 'V' for (x,y)-(x,y+1), and
                           G4[pA', pB', pA, pB] the two-site operator

Physical legs carry flip parities (of a vertical bond edge, or of the open
checks assigned to a site), so a flip mechanism between two sites is the gate
(1-p) I (x) I + p X (x) X and a detector outcome is imposed by a one-site op.
Exactness of every construction is checked against the frontier contraction
in the tests (chi large enough that nothing is truncated).
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

W_, E_, N_, S_ = 1, 2, 3, 4  # tensor axes of the four virtual legs


@dataclass
class Layer:
    pre: dict = field(default_factory=dict)
    gates: list = field(default_factory=list)
    post: dict = field(default_factory=dict)


@dataclass
class LayeredNet:
    Lx: int
    Ly: int
    init: list
    layers: list
    final: list


def xx_gate(p, dA, bitA, dB, bitB):
    """(1-p) I (x) I + p X_bitA (x) X_bitB on physical dims dA, dB."""
    G = np.zeros((dA, dB, dA, dB))
    for a in range(dA):
        for b in range(dB):
            G[a, b, a, b] += 1.0 - p
            G[a ^ (1 << bitA), b ^ (1 << bitB), a, b] += p
    return G


def flip_op(p, d, bits):
    """(1-p) I + p prod_{b in bits} X_b on a physical dim d."""
    M = (1.0 - p) * np.eye(d)
    mask = 0
    for b in bits:
        mask |= 1 << b
    for a in range(d):
        M[a ^ mask, a] += p
    return M


def snake_order(Lx, Ly):
    order = []
    for y in range(Ly):
        xs = range(Lx) if y % 2 == 0 else range(Lx - 1, -1, -1)
        order.extend((x, y) for x in xs)
    return order


def _leg_towards(a, b):
    (xa, ya), (xb, yb) = a, b
    if xb == xa + 1 and yb == ya:
        return E_
    if xb == xa - 1 and yb == ya:
        return W_
    if yb == ya + 1 and xb == xa:
        return S_
    if yb == ya - 1 and xb == xa:
        return N_
    raise ValueError("not adjacent")


def snake_state(Lx, Ly, weights, coset):
    """Parity-chain state over per-site bits: value prod_s w_s(b_s) if the
    parity of all bits equals `coset`, else 0.  weights[s] is a length-2
    vector for a site carrying a bit, or None for a site without one
    (physical dim 1).  The chain runs boustrophedon over the grid with bond
    dimension 2 carrying the running parity."""
    order = snake_order(Lx, Ly)
    tens = [None] * (Lx * Ly)
    n = len(order)
    for k, (x, y) in enumerate(order):
        w = weights[y * Lx + x]
        dp = 1 if w is None else 2
        shape = [dp, 1, 1, 1, 1]
        leg_in = _leg_towards((x, y), order[k - 1]) if k > 0 else None
        leg_out = _leg_towards((x, y), order[k + 1]) if k < n - 1 else None
        if leg_in is not None:
            shape[leg_in] = 2
        if leg_out is not None:
            shape[leg_out] = 2
        T = np.zeros(shape)
        cins = [0] if leg_in is None else [0, 1]
        for cin in cins:
            for b in range(dp):
                val = 1.0 if w is None else w[b]
                cout = cin ^ b
                if leg_out is None and cout != coset:
                    continue
                idx = [b, 0, 0, 0, 0]
                if leg_in is not None:
                    idx[leg_in] = cin
                if leg_out is not None:
                    idx[leg_out] = cout
                T[tuple(idx)] = val
        tens[y * Lx + x] = T
    return tens


# ---------------------------------------------------------------------------
# 3D planar code, point sector: sweep along z
# ---------------------------------------------------------------------------

def point3d_network(L, p, m, coset):
    """Sweep of the point-sector network of the 3D planar code along z.

    The physical leg of site (x, y) before layer z is the flip of the z-edge
    entering vertex (x, y, z) from below.  The initial state is the bottom
    layer of dangling z-edges, weighted by their flip probabilities and
    constrained to parity `coset` (the logical membrane).  Layer z applies, for
    every in-plane edge of level z, the gate (1-p) I I + p X X (a flip of that
    edge toggles the parity seen by both its vertices), then at every vertex
    X^{m} (the vertex check fixes the up-going edge's flip to the parity of
    the others xor m) followed by the up-going edge's weight diag(1-p, p).
    After the last level the top dangling edges are summed over, f = (1, 1).

    p: per-mechanism rates in the canonical numbering of the point-sector DEM.
    m: the syndrome (detector (x, y, z) -> ((z-1) L + y) L + x).
    """
    p = np.asarray(p, dtype=np.float64)
    nz = L ** 3
    nx = L * (L - 1) ** 2
    weights = []
    for y in range(L):
        for x in range(L):
            q = p[y * L + x]
            weights.append(np.array([1.0 - q, q]))
    init = snake_state(L, L, weights, coset)
    X = np.array([[0.0, 1.0], [1.0, 0.0]])
    layers = []
    for z in range(1, L):
        lay = Layer()
        for y in range(L):
            for x in range(L - 1):
                q = p[nz + ((z - 1) * L + y) * (L - 1) + x]
                lay.gates.append(("H", x, y, xx_gate(q, 2, 0, 2, 0)))
        for y in range(L - 1):
            for x in range(L):
                q = p[nz + nx + ((z - 1) * (L - 1) + y) * L + x]
                lay.gates.append(("V", x, y, xx_gate(q, 2, 0, 2, 0)))
        for y in range(L):
            for x in range(L):
                mm = int(m[((z - 1) * L + y) * L + x])
                q = p[z * L * L + y * L + x]
                Mx = X if mm else np.eye(2)
                lay.post[y * L + x] = np.diag([1.0 - q, q]) @ Mx
        layers.append(lay)
    final = [np.ones(2) for _ in range(L * L)]
    return LayeredNet(L, L, init, layers, final)


# ---------------------------------------------------------------------------
# Rotated code with phenomenological noise: sweep across data rows
# ---------------------------------------------------------------------------

def _check_column(x2):
    return 0 if x2 < 0 else (x2 - 1) // 2


def rotated_network(d, T, checks, p, m, coset):
    """Sweep of the phenomenological rotated-code network across data rows.

    The layer grid is (site column x in [0, d)) x (round y = t-1, t in
    [1, T+1]).  Z-checks of one gap row are "open" while the data rows on
    either side are being absorbed; check c with centre x2 sits at column
    (x2-1)/2 (column 0 for the left-edge checks), so the checks of one gap row
    occupy distinct columns and two consecutive gap rows share only column 0.
    The physical leg of a site lists the partial parities of the open checks
    it holds, one bit per check (older gap row in the low bit).

      initial state   the flips of data row 0, which touch gap row 0 only and
                      carry the logical: per site the distribution of the
                      parity of the flips feeding its check, chained to total
                      parity `coset`.
      layer j=1..d-1  pre: open a zero bit for every check of gap row j (if
                      j <= d-2), and apply the flips of data row j whose two
                      checks share a site; gates: the other flips of row j
                      ('H', between the two sites of its checks) and the
                      measurement flips (c, t) of gap row j-1 ('V', between
                      rounds t and t+1); post: restrict the bits of gap row
                      j-1 to the syndrome.
    p: per-mechanism rates in the canonical numbering of the DEM.
    """
    p = np.asarray(p, dtype=np.float64)
    nZ = len(checks)
    nq = d * d
    Lx, Ly = d, T + 1
    by_row = [[] for _ in range(d - 1)]
    for c, (g, cols, x2) in enumerate(checks):
        by_row[g].append(c)
    col_of = {c: _check_column(checks[c][2]) for c in range(nZ)}
    cover = {}  # (g, data column) -> check
    for c, (g, cols, x2) in enumerate(checks):
        for i in cols:
            cover[(g, i)] = c

    def pdata(i, j, t):
        return p[(t - 1) * nq + j * d + i]

    def pmeas(c, t):
        return p[T * nq + (t - 1) * nZ + c]

    # initial state: gap row 0 open at every round
    weights = [None] * (Lx * Ly)
    for c in by_row[0]:
        x = col_of[c]
        for t in range(1, T + 2):
            if t <= T:
                w = np.array([1.0, 0.0])
                for i in checks[c][1]:
                    q = pdata(i, 0, t)
                    w = np.array([w[0] * (1 - q) + w[1] * q, w[0] * q + w[1] * (1 - q)])
            else:
                w = np.array([1.0, 0.0])
            weights[(t - 1) * Lx + x] = w
    init = snake_state(Lx, Ly, weights, coset)

    layers = []
    # bits currently held per site, oldest first: list of (gap row)
    held = [[] for _ in range(Lx * Ly)]
    for c in by_row[0]:
        for t in range(1, T + 2):
            held[(t - 1) * Lx + col_of[c]].append(0)
    for j in range(1, d):
        lay = Layer()
        gclose, gopen = j - 1, (j if j <= d - 2 else None)
        if gopen is not None:
            for c in by_row[gopen]:
                for t in range(1, T + 2):
                    s = (t - 1) * Lx + col_of[c]
                    dold = 1 << len(held[s])
                    Eop = np.zeros((2 * dold, dold))
                    Eop[np.arange(dold), np.arange(dold)] = 1.0
                    lay.pre[s] = Eop
                    held[s].append(gopen)
        for t in range(1, T + 1):
            y = t - 1
            for i in range(d):
                cc = cover[(gclose, i)]
                sa = y * Lx + col_of[cc]
                ba = held[sa].index(gclose)
                q = pdata(i, j, t)
                if gopen is None:
                    M = flip_op(q, 1 << len(held[sa]), [ba])
                    lay.pre[sa] = M @ lay.pre[sa] if sa in lay.pre else M
                    continue
                co = cover[(gopen, i)]
                sb = y * Lx + col_of[co]
                bb = held[sb].index(gopen)
                if sa == sb:
                    M = flip_op(q, 1 << len(held[sa]), [ba, bb])
                    lay.pre[sa] = M @ lay.pre[sa] if sa in lay.pre else M
                    continue
                xa, xb = col_of[cc], col_of[co]
                assert abs(xa - xb) == 1
                if xa < xb:
                    G = xx_gate(q, 1 << len(held[sa]), ba, 1 << len(held[sb]), bb)
                    lay.gates.append(("H", xa, y, G))
                else:
                    G = xx_gate(q, 1 << len(held[sb]), bb, 1 << len(held[sa]), ba)
                    lay.gates.append(("H", xb, y, G))
            for c in by_row[gclose]:
                x = col_of[c]
                sa, sb = y * Lx + x, (y + 1) * Lx + x
                G = xx_gate(pmeas(c, t), 1 << len(held[sa]), held[sa].index(gclose),
                            1 << len(held[sb]), held[sb].index(gclose))
                lay.gates.append(("V", x, y, G))
        for c in by_row[gclose]:
            for t in range(1, T + 2):
                s = (t - 1) * Lx + col_of[c]
                k = held[s].index(gclose)
                dold = 1 << len(held[s])
                mm = int(m[(t - 1) * nZ + c])
                P = np.zeros((dold // 2, dold))
                for a in range(dold):
                    if (a >> k) & 1 == mm:
                        low = a & ((1 << k) - 1)
                        high = a >> (k + 1)
                        P[low | (high << k), a] = 1.0
                lay.post[s] = P
                held[s].pop(k)
        layers.append(lay)
    assert all(len(h) == 0 for h in held)
    final = [np.ones(1) for _ in range(Lx * Ly)]
    return LayeredNet(Lx, Ly, init, layers, final)


# ---------------------------------------------------------------------------
# 3D planar code, depolarizing noise: mixed picture, sweep along z
# ---------------------------------------------------------------------------

def _faces3d(L):
    """Face checks as edge lists (the canonical face order of the depolarizing
    syndrome: xy-faces by level, then xz-faces, then yz-faces, each x fastest)."""
    nz, nx = L ** 3, L * (L - 1) ** 2

    def zedge(x, y, z):
        return z * L * L + y * L + x

    def xedge(x, y, z):
        return nz + ((z - 1) * L + y) * (L - 1) + x

    def yedge(x, y, z):
        return nz + nx + ((z - 1) * (L - 1) + y) * L + x

    out = []
    for z in range(1, L):
        for y in range(L - 1):
            for x in range(L - 1):
                out.append([xedge(x, y, z), xedge(x, y + 1, z), yedge(x, y, z), yedge(x + 1, y, z)])
    for z in range(L):
        for y in range(L):
            for x in range(L - 1):
                out.append([zedge(x, y, z), zedge(x + 1, y, z)]
                           + ([xedge(x, y, z)] if z >= 1 else [])
                           + ([xedge(x, y, z + 1)] if z + 1 < L else []))
    for z in range(L):
        for y in range(L - 1):
            for x in range(L):
                out.append([zedge(x, y, z), zedge(x, y + 1, z)]
                           + ([yedge(x, y, z)] if z >= 1 else [])
                           + ([yedge(x, y, z + 1)] if z + 1 < L else []))
    return out


def gf2_solve(A, b):
    """One solution x of A x = b over F2 (Gauss-Jordan elimination), or None
    when the system is inconsistent.  Free variables are set to zero."""
    A = (np.asarray(A, dtype=np.uint8) & 1).copy()
    b = (np.asarray(b, dtype=np.uint8) & 1).copy()
    rows, cols = A.shape
    pivots = []
    r = 0
    for c in range(cols):
        hits = np.nonzero(A[r:, c])[0]
        if hits.size == 0:
            continue
        k = r + hits[0]
        A[[r, k]] = A[[k, r]]
        b[[r, k]] = b[[k, r]]
        for i in np.nonzero(A[:, c])[0]:
            if i != r:
                A[i] ^= A[r]
                b[i] ^= b[r]
        pivots.append(c)
        r += 1
        if r == rows:
            break
    if np.any(b[r:]):
        return None
    x = np.zeros(cols, dtype=np.uint8)
    for i, c in enumerate(pivots):
        x[c] = b[i]
    return x


def depol3d_network(L, p, m, coset, rep=None):
    """Depolarizing network of the 3D planar code (both sectors), coset
    c = a + 2 b, swept along z over the L x L vertex grid.

    Mixed picture.  Z parts of the errors (seen by the vertex X-checks) are
    summed in the detector picture as in point3d_network.  X parts u (seen by
    the face Z-checks) are summed in the generator picture (Sec. 3.3): every u
    with face syndrome m_Z and class a is r + sum_v g_v s_v for one fixed
    representative r of that class and a unique set of vertex stabilizers s_v
    (X on the edges at vertex v; they are independent here), so one bit g_v
    per vertex replaces the sum over u.  An edge e between vertices v, w then
    carries X part r_e + g_v + g_w, and its Pauli weight is
    W(u, v) = P(X part u, Z part v): 1-p for I, p/3 for X, Y, Z.

    Physical leg of site (x, y): (g, s) with index 2 g + s, where g is the
    generator bit of the vertex last absorbed (0 below level 1) and s the
    Z-part flip of the z-edge entering the next vertex.  Layer z:
      pre   the z-edge below vertex (x, y, z): (g, s) -> (g', s) with weight
            W(r_e + g + g', s), g' the new vertex's bit;
      gates per in-plane edge, summed over its Z part t:
            s_A ^= t, s_B ^= t, weight W(r_e + g_A + g_B, t);
      post  X^{m} on s (the vertex check fixes the up edge's Z part).
    Final: the top dangling edge, f[(g, s)] = W(r_e + g, s).  Initial state:
    g = 0, the bottom dangling edges' Z parts chained to parity b.  The class
    of u is its parity on the vertical string above (0, 0); r is a solution of
    H_Z r = m_Z, plus the bottom membrane of edges when its class differs from
    a.

    p: depolarizing rate, scalar or per qubit (edge numbering of
    surface3d_point).  m: vertex syndrome then face syndrome.  rep: a
    solution of H_Z r = m_Z to start from instead of the elimination's.
    """
    nq = L ** 3 + 2 * L * (L - 1) ** 2
    pq = np.broadcast_to(np.asarray(p, dtype=np.float64), (nq,))
    nv = L * L * (L - 1)
    m = np.asarray(m, dtype=np.uint8)
    faces = _faces3d(L)
    HZ = np.zeros((len(faces), nq), dtype=np.uint8)
    for f, es in enumerate(faces):
        HZ[f, es] = 1
    r = gf2_solve(HZ, m[nv:]) if rep is None else np.array(rep, dtype=np.uint8)
    if r is None or np.any(((HZ.astype(np.int64) @ r) & 1) != m[nv:]):
        raise ValueError("face syndrome violates a cube relation")
    a, b = coset & 1, coset >> 1
    string = [z * L * L for z in range(L)]
    if int(r[string].sum()) % 2 != a:
        r[: L * L] ^= 1

    def W(e, u, v):
        return 1.0 - pq[e] if (u == 0 and v == 0) else pq[e] / 3.0

    base = snake_state(L, L, [np.ones(2)] * (L * L), b)
    init = []
    for T in base:
        T4 = np.zeros((4,) + T.shape[1:])
        T4[0:2] = T            # g = 0
        init.append(T4)

    nz, nx = L ** 3, L * (L - 1) ** 2
    X2 = np.array([[0.0, 1.0], [1.0, 0.0]])
    layers = []
    for z in range(1, L):
        lay = Layer()
        for y in range(L):
            for x in range(L):
                e = (z - 1) * L * L + y * L + x
                O = np.zeros((4, 4))
                for g in range(2):
                    for g2 in range(2):
                        for s in range(2):
                            O[2 * g2 + s, 2 * g + s] = W(e, r[e] ^ g ^ g2, s)
                lay.pre[y * L + x] = O

        def gate(e):
            G = np.zeros((4, 4, 4, 4))
            for ga in range(2):
                for gb in range(2):
                    for sa in range(2):
                        for sb in range(2):
                            for t in range(2):
                                G[2 * ga + (sa ^ t), 2 * gb + (sb ^ t), 2 * ga + sa, 2 * gb + sb] += \
                                    W(e, r[e] ^ ga ^ gb, t)
            return G

        for y in range(L):
            for x in range(L - 1):
                lay.gates.append(("H", x, y, gate(nz + ((z - 1) * L + y) * (L - 1) + x)))
        for y in range(L - 1):
            for x in range(L):
                lay.gates.append(("V", x, y, gate(nz + nx + ((z - 1) * (L - 1) + y) * L + x)))
        for y in range(L):
            for x in range(L):
                mm = int(m[((z - 1) * L + y) * L + x])
                lay.post[y * L + x] = np.kron(np.eye(2), X2 if mm else np.eye(2))
        layers.append(lay)
    final = []
    for y in range(L):
        for x in range(L):
            e = (L - 1) * L * L + y * L + x
            final.append(np.array([W(e, r[e] ^ g, s) for g in range(2) for s in range(2)]))
    return LayeredNet(L, L, init, layers, final)


# ---------------------------------------------------------------------------
# 3D planar code, loop sector (bit flips seen by the face checks): generator
# picture, sweep along z
# ---------------------------------------------------------------------------

def loop3d_dem_parts(L):
    """(H_faces, string): the face checks of the 3D planar code as a
    faces x edges F2 matrix (canonical face order) and the indicator of the
    vertical string of z-edges above (0, 0), whose parity labels the coset of
    a bit-flip error seen by the faces."""
    nq = L ** 3 + 2 * L * (L - 1) ** 2
    faces = _faces3d(L)
    H = np.zeros((len(faces), nq), dtype=np.uint8)
    for f, es in enumerate(faces):
        H[f, es] = 1
    string = np.zeros(nq, dtype=np.uint8)
    string[[z * L * L for z in range(L)]] = 1
    return H, string


def loop3d_network(L, p, m, coset):
    """Generator-picture network of the loop sector (paper Sec. 3.2 and the
    loop-sector experiment of Sec. 5): bit flips u on the edges of the 3D
    planar code, detected by the weight-3/4 face checks (syndrome m), class =
    parity of u on the vertical string of z-edges above (0, 0).

    Every u with face syndrome m and class c is r + sum_v g_v s_v for one
    representative r of that class and exactly one set of vertex stabilizers
    s_v (X on the edges at vertex v; independent here because every vertex
    star holds dangling edges or an edge to a vertex with one), so a bit g_v
    per vertex replaces the sum over u, and every term is a product of
    non-negative edge weights W(e, u_e) = p_e^u_e (1 - p_e)^(1 - u_e) with
    u_e = r_e + g_v + g_w (one endpoint for a dangling edge).

    Physical leg of site (x, y): the generator bit g of the vertex last
    absorbed (0 before level 1).  Layer z (levels 1..L-1):
      pre   the z-edge below vertex (x, y, z): g -> g' with weight
            W(e, r_e + g + g'), g' the bit of (x, y, z);
      gates per in-plane edge of level z: diagonal, W(e, r_e + g_A + g_B).
    Final: the top dangling edge, f[g] = W(e, r_e + g).  Initial state: g = 0
    on every site (a product state).  r: a solution of H r = m from
    elimination, plus the bottom membrane of dangling edges (which meets the
    string once) when its class differs from `coset`.

    p: per-edge flip rates (edge numbering of surface3d_point), or a scalar.
    m: the face syndrome (canonical face order).
    """
    nq = L ** 3 + 2 * L * (L - 1) ** 2
    pq = np.broadcast_to(np.asarray(p, dtype=np.float64), (nq,))
    H, string = loop3d_dem_parts(L)
    m = np.asarray(m, dtype=np.uint8)
    r = gf2_solve(H, m)
    if r is None:
        raise ValueError("face syndrome violates a cube relation")
    if int(r[string == 1].sum()) % 2 != coset:
        r[: L * L] ^= 1
    return _loop3d_from_rep(L, pq, r, [np.array([1.0, 0.0])] * (L * L))


def _loop3d_from_rep(L, pq, r, init_vecs):
    def W(e, u):
        return pq[e] if u else 1.0 - pq[e]

    init = [v.reshape(2, 1, 1, 1, 1).astype(np.float64) for v in init_vecs]
    nz, nx = L ** 3, L * (L - 1) ** 2
    layers = []
    for z in range(1, L):
        lay = Layer()
        for y in range(L):
            for x in range(L):
                e = (z - 1) * L * L + y * L + x
                lay.pre[y * L + x] = np.array([[W(e, r[e] ^ g ^ g2) for g in range(2)] for g2 in range(2)])

        def gate(e):
            G = np.zeros((2, 2, 2, 2))
            for ga in range(2):
                for gb in range(2):
                    G[ga, gb, ga, gb] = W(e, r[e] ^ ga ^ gb)
            return G

        for y in range(L):
            for x in range(L - 1):
                lay.gates.append(("H", x, y, gate(nz + ((z - 1) * L + y) * (L - 1) + x)))
        for y in range(L - 1):
            for x in range(L):
                lay.gates.append(("V", x, y, gate(nz + nx + ((z - 1) * (L - 1) + y) * L + x)))
        layers.append(lay)
    final = []
    for y in range(L):
        for x in range(L):
            e = (L - 1) * L * L + y * L + x
            final.append(np.array([W(e, r[e] ^ g) for g in range(2)]))
    return LayeredNet(L, L, init, layers, final)


# ---------------------------------------------------------------------------
# Walsh-Hadamard variant (paper Sec. 3.1): signed networks Z_b with
# P_L = (1/2) sum_b (-1)^(b L) Z_b
# ---------------------------------------------------------------------------

def point3d_network_wht(L, p, m, b):
    """Z_b of the point sector: the sum over all flips x with H x = m of
    (-1)^(b * class(x)) times the weight, class = the parity of the bottom
    dangling z-edges.  The logical check node of the paper's network becomes
    the sign (-1)^(b x_e) on each bottom dangling edge, so the initial state
    is the product of the vectors (1 - q, (-1)^b q): no parity chain."""
    net = point3d_network(L, p, m, 0)
    pz = np.asarray(p, dtype=np.float64)
    init = []
    for y in range(L):
        for x in range(L):
            q = pz[y * L + x]
            init.append(np.array([1.0 - q, (-1.0) ** b * q]).reshape(2, 1, 1, 1, 1))
    return LayeredNet(net.Lx, net.Ly, init, net.layers, net.final)


def loop3d_network_wht(L, p, m, b):
    """Z_b of the loop sector: the sum over both classes a of (-1)^(a b) P_a.
    With the class-0 representative, class a adds the bottom membrane, which
    is the same as a generator bit a shared by every site below level 1; the
    initial state is that shared bit with sign (-1)^(a b): a chain of equal
    bits (bond 2) in boustrophedon order."""
    nq = L ** 3 + 2 * L * (L - 1) ** 2
    pq = np.broadcast_to(np.asarray(p, dtype=np.float64), (nq,))
    H, string = loop3d_dem_parts(L)
    r = gf2_solve(H, np.asarray(m, dtype=np.uint8))
    if r is None:
        raise ValueError("face syndrome violates a cube relation")
    if int(r[string == 1].sum()) % 2 != 0:
        r[: L * L] ^= 1
    net = _loop3d_from_rep(L, pq, r, [np.array([1.0, 0.0])] * (L * L))
    order = snake_order(L, L)
    init = [None] * (L * L)
    n = len(order)
    for k, (x, y) in enumerate(order):
        shape = [2, 1, 1, 1, 1]
        lin = _leg_towards((x, y), order[k - 1]) if k > 0 else None
        lout = _leg_towards((x, y), order[k + 1]) if k < n - 1 else None
        if lin is not None:
            shape[lin] = 2
        if lout is not None:
            shape[lout] = 2
        T = np.zeros(shape)
        for a in range(2):
            idx = [a, 0, 0, 0, 0]
            if lin is not None:
                idx[lin] = a
            if lout is not None:
                idx[lout] = a
            T[tuple(idx)] = (-1.0) ** (a * b) if k == 0 else 1.0
        init[y * L + x] = T
    return LayeredNet(net.Lx, net.Ly, init, net.layers, net.final)
