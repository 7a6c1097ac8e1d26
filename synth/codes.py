"""Detector error models (H, p, l) of the codes decoded in this repository.

A detector error model (paper, Sec. 2.4) is a triple: a parity-check matrix H
over F2 (detectors x mechanisms), a probability p_i per independent error
mechanism, and logical indicator rows l (observables x mechanisms).  For a CSS
code under independent flips of one Pauli type the decoding problem is a DEM
whose mechanisms are the qubits and whose detectors are the checks of the other
type (paper, Sec. 3.3 and Sec. 3.4).

Every builder documents its canonical numbering of detectors and mechanisms;
the C-ABI family builders use the same numbering, so a syndrome vector produced
here can be handed to either side unchanged.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Dem:
    name: str
    H: np.ndarray  # uint8 [n_det, n_mech]
    p: np.ndarray  # float64 [n_mech]
    obs: np.ndarray  # uint8 [n_obs, n_mech]
    det_coord: np.ndarray  # int64 [n_det, 3]
    params: dict = field(default_factory=dict)

    @property
    def n_det(self) -> int:
        return self.H.shape[0]

    @property
    def n_mech(self) -> int:
        return self.H.shape[1]

    @property
    def n_obs(self) -> int:
        return self.obs.shape[0]

    def with_p(self, p) -> "Dem":
        p = np.broadcast_to(np.asarray(p, dtype=np.float64), (self.n_mech,)).copy()
        return Dem(self.name, self.H, p, self.obs, self.det_coord, dict(self.params))


def _rates(p, n: int) -> np.ndarray:
    return np.broadcast_to(np.asarray(p, dtype=np.float64), (n,)).copy()


# --------------------------------------------------------------------------
# 3D planar surface code, point sector (vertex checks, i.i.d. flips)
# --------------------------------------------------------------------------

def surface3d_point(L: int, p) -> Dem:
    """Point sector of the 3D planar surface code of linear size L.

    Checks are the weight-<=6 vertex checks at (x, y, z), x, y in [0, L),
    z in [1, L): L^2 (L-1) of them.  Qubits are lattice edges: in-plane x- and
    y-edges on every vertex level and z-edges between levels, including the
    dangling z-edges below level 1 and above level L-1 (rough boundaries).
    n = L^3 + 2 L (L-1)^2.  The logical indicator is the membrane of the L^2
    bottom dangling z-edges, which meets every face stabilizer an even number of
    times and the vertical logical string once.

    Canonical numbering:
      detector (x, y, z)           -> ((z-1) L + y) L + x
      z-edge (x, y) from z to z+1  -> z L^2 + y L + x,            z in [0, L)
      x-edge (x..x+1, y) at level z -> L^3 + ((z-1) L + y)(L-1) + x
      y-edge (x, y..y+1) at level z -> L^3 + L(L-1)^2 + ((z-1)(L-1) + y) L + x
    """
    if L < 2:
        raise ValueError("L >= 2")
    n_det = L * L * (L - 1)
    nz = L ** 3
    nx = L * (L - 1) ** 2
    n = nz + 2 * nx
    H = np.zeros((n_det, n), dtype=np.uint8)

    def det(x, y, z):
        return ((z - 1) * L + y) * L + x

    for z in range(L):
        for y in range(L):
            for x in range(L):
                e = z * L * L + y * L + x
                if z >= 1:
                    H[det(x, y, z), e] = 1
                if z + 1 <= L - 1:
                    H[det(x, y, z + 1), e] = 1
    for z in range(1, L):
        for y in range(L):
            for x in range(L - 1):
                e = nz + ((z - 1) * L + y) * (L - 1) + x
                H[det(x, y, z), e] = 1
                H[det(x + 1, y, z), e] = 1
    for z in range(1, L):
        for y in range(L - 1):
            for x in range(L):
                e = nz + nx + ((z - 1) * (L - 1) + y) * L + x
                H[det(x, y, z), e] = 1
                H[det(x, y + 1, z), e] = 1
    obs = np.zeros((1, n), dtype=np.uint8)
    obs[0, : L * L] = 1
    coord = np.array([(x, y, z) for z in range(1, L) for y in range(L) for x in range(L)],
                     dtype=np.int64)
    return Dem(f"surface3d_point_L{L}", H, _rates(p, n), obs, coord, {"L": L})


# --------------------------------------------------------------------------
# 3D planar surface code, depolarizing noise (both sectors)
# --------------------------------------------------------------------------

def surface3d_faces(L: int):
    """Face (Z-type) checks of the 3D planar code of size L as edge lists, in
    canonical order (edge numbering as in surface3d_point):
      xy-face (x..x+1, y..y+1) at level z in [1, L)  -> ((z-1)(L-1) + y)(L-1) + x
      xz-face (x..x+1, y, z..z+1), z in [0, L)       -> (L-1)^3 + (z L + y)(L-1) + x
      yz-face (x, y..y+1, z..z+1), z in [0, L)       -> (L-1)^3 + L^2 (L-1) + (z (L-1) + y) L + x
    Faces between a rough boundary and level 1 (or level L-1 and the top) have
    three edges.  (L-1)^3 + 2 L^2 (L-1) faces; the six faces of a cube are
    dependent, so consistent syndromes satisfy one parity per cube.
    """
    nz = L ** 3
    nx = L * (L - 1) ** 2

    def ze(x, y, z):
        return z * L * L + y * L + x

    def xe(x, y, z):
        return nz + ((z - 1) * L + y) * (L - 1) + x

    def ye(x, y, z):
        return nz + nx + ((z - 1) * (L - 1) + y) * L + x

    faces = []
    for z in range(1, L):
        for y in range(L - 1):
            for x in range(L - 1):
                faces.append((xe(x, y, z), xe(x, y + 1, z), ye(x, y, z), ye(x + 1, y, z)))
    for z in range(L):
        for y in range(L):
            for x in range(L - 1):
                f = [ze(x, y, z), ze(x + 1, y, z)]
                if z >= 1:
                    f.append(xe(x, y, z))
                if z + 1 <= L - 1:
                    f.append(xe(x, y, z + 1))
                faces.append(tuple(f))
    for z in range(L):
        for y in range(L - 1):
            for x in range(L):
                f = [ze(x, y, z), ze(x, y + 1, z)]
                if z >= 1:
                    f.append(ye(x, y, z))
                if z + 1 <= L - 1:
                    f.append(ye(x, y, z + 1))
                faces.append(tuple(f))
    return faces


def surface3d_depolarizing(L: int, p) -> Dem:
    """3D planar surface code of size L under depolarizing noise: each qubit
    independently suffers X, Y or Z with probability p/3 each (I with 1-p).

    Both check types are decoded together.  A Pauli with X part u and Z part v
    (bit vectors over the n qubits) has syndrome (H_X v, H_Z u): the vertex
    X-checks of surface3d_point see the Z part, the face Z-checks of
    surface3d_faces see the X part.  Its logical class is c = a + 2 b with
    a = the parity of u on the vertical string of z-edges above (0, 0) (a Z
    logical) and b = the parity of v on the L^2 bottom dangling z-edges (the X
    logical membrane).

    As a DEM (paper, Sec. 2.4): three independent mechanisms per qubit, X, Y
    and Z, each of rate r with r (1 - r) = p/3, i.e. r = (1 - sqrt(1 - 4p/3)) / 2;
    the product of the three draws is the depolarizing channel.
      detector: vertex (x, y, z) as in surface3d_point, then face f -> L^2 (L-1) + f
      mechanism: X on qubit e -> e, Y -> n + e, Z -> 2 n + e
      observables: row 0 is a, row 1 is b, so the observable integer is c.
    params["p_qubit"] holds the per-qubit depolarizing rates.
    """
    if L < 2:
        raise ValueError("L >= 2")
    pt = surface3d_point(L, 0.0)
    HX = pt.H
    n = HX.shape[1]
    faces = surface3d_faces(L)
    HZ = np.zeros((len(faces), n), dtype=np.uint8)
    for f, es in enumerate(faces):
        HZ[f, list(es)] = 1
    nv = HX.shape[0]
    H = np.zeros((nv + len(faces), 3 * n), dtype=np.uint8)
    H[nv:, 0:n] = HZ          # X
    H[:nv, n:2 * n] = HX      # Y: both
    H[nv:, n:2 * n] = HZ
    H[:nv, 2 * n:] = HX       # Z
    zbar = np.zeros(n, dtype=np.uint8)
    zbar[[z * L * L for z in range(L)]] = 1
    xbar = np.zeros(n, dtype=np.uint8)
    xbar[: L * L] = 1
    obs = np.zeros((2, 3 * n), dtype=np.uint8)
    obs[0, 0:n] = zbar
    obs[0, n:2 * n] = zbar
    obs[1, n:2 * n] = xbar
    obs[1, 2 * n:] = xbar
    pq = _rates(p, n)
    r = 0.5 * (1.0 - np.sqrt(1.0 - 4.0 * pq / 3.0))
    coord = np.concatenate([pt.det_coord, np.full((len(faces), 3), -1, dtype=np.int64)])
    return Dem(f"surface3d_depolarizing_L{L}", H, np.concatenate([r, r, r]), obs, coord,
               {"L": L, "n_qubits": n, "p_qubit": pq, "HX": HX, "HZ": HZ,
                "zbar": zbar, "xbar": xbar})


def surface3d_loop(L: int, p) -> Dem:
    """Loop sector of the 3D planar code of size L: i.i.d. bit flips of rate
    p on every edge (qubit), detected by the face checks of surface3d_faces
    (loop-like syndromes).  The logical indicator is the vertical string of
    z-edges above (0, 0), which meets the X membrane of the bottom dangling
    edges once and every vertex stabilizer an even number of times.
      detector: face f (canonical face order)
      mechanism: edge e (numbering of surface3d_point)
    Consistent syndromes satisfy one parity per cube (six dependent faces).
    """
    if L < 2:
        raise ValueError("L >= 2")
    n = L ** 3 + 2 * L * (L - 1) ** 2
    faces = surface3d_faces(L)
    H = np.zeros((len(faces), n), dtype=np.uint8)
    for f, es in enumerate(faces):
        H[f, list(es)] = 1
    obs = np.zeros((1, n), dtype=np.uint8)
    obs[0, [z * L * L for z in range(L)]] = 1
    coord = np.full((len(faces), 3), -1, dtype=np.int64)
    return Dem(f"surface3d_loop_L{L}", H, _rates(p, n), obs, coord, {"L": L})


# --------------------------------------------------------------------------
# Rotated surface code, one sector, phenomenological noise
# --------------------------------------------------------------------------

def rotated_z_checks(d: int):
    """Z-checks of the rotated distance-d code as lists of data columns per gap row.

    Data qubits sit at (column i, row j), i, j in [0, d), index j*d + i.  Gap
    row g in [0, d-1) lies between data rows g and g+1.  For even g the
    weight-4 plaquettes cover column pairs (0,1), (2,3), ... and a weight-2
    check covers column d-1 on the right edge; for odd g the plaquettes cover
    (1,2), (3,4), ... and a weight-2 check covers column 0 on the left edge.
    Every gap row therefore covers every column exactly once, so each interior
    data qubit is in exactly two Z-checks and the top and bottom data rows in
    one.  Returns [(g, columns tuple, x2)] ordered by gap row, then x2, where
    x2 is twice the x-coordinate of the check centre.
    """
    if d < 3 or d % 2 == 0:
        raise ValueError("odd d >= 3")
    checks = []
    for g in range(d - 1):
        row = []
        if g % 2 == 0:
            for i in range(0, d - 1, 2):
                row.append((g, (i, i + 1), 2 * i + 1))
            row.append((g, (d - 1,), 2 * d - 1))
        else:
            row.append((g, (0,), -1))
            for i in range(1, d - 1, 2):
                row.append((g, (i, i + 1), 2 * i + 1))
        row.sort(key=lambda c: c[2])
        checks.extend(row)
    return checks


def rotated_phenom(d: int, T: int, p_data, q_meas) -> Dem:
    """Rotated distance-d surface code, X flips decoded with Z-checks, over
    T noisy measurement rounds followed by one perfect round.

    Round convention: the register starts in the code space; before each noisy
    round t = 1..T every data qubit flips independently; each noisy round's
    check outcomes flip independently; round T+1 is read out perfectly and has
    no new data flips.  Detector (c, t), t = 1..T+1, is the difference of the
    outcomes of check c in rounds t and t-1 (round 0 is noiseless and trivial).
    The logical indicator is the parity of flips on the top data row (row 0),
    on which a Z logical is supported.

    p_data: scalar, (d*d,) per qubit shared by all rounds, or (T, d*d).
    q_meas: scalar, (nZ,) per check shared by all rounds, or (T, nZ).

    Canonical numbering (nZ = (d^2-1)/2 checks ordered as rotated_z_checks):
      detector (c, t)          -> (t-1) nZ + c
      data flip (q, t)         -> (t-1) d^2 + q,           t in [1, T]
      measurement flip (c, t)  -> T d^2 + (t-1) nZ + c,    t in [1, T]
    """
    checks = rotated_z_checks(d)
    nZ = len(checks)
    nq = d * d
    n_det = nZ * (T + 1)
    n = T * nq + T * nZ
    H = np.zeros((n_det, n), dtype=np.uint8)
    qubit_checks = [[] for _ in range(nq)]
    for c, (g, cols, _) in enumerate(checks):
        for i in cols:
            qubit_checks[g * d + i].append(c)
            qubit_checks[(g + 1) * d + i].append(c)
    for t in range(1, T + 1):
        for q in range(nq):
            e = (t - 1) * nq + q
            for c in qubit_checks[q]:
                H[(t - 1) * nZ + c, e] = 1
        for c in range(nZ):
            e = T * nq + (t - 1) * nZ + c
            H[(t - 1) * nZ + c, e] = 1
            H[t * nZ + c, e] = 1
    obs = np.zeros((1, n), dtype=np.uint8)
    for t in range(1, T + 1):
        obs[0, (t - 1) * nq:(t - 1) * nq + d] = 1
    pd = np.asarray(p_data, dtype=np.float64)
    if pd.ndim == 1:
        pd = np.broadcast_to(pd, (T, nq))
    pd = np.broadcast_to(pd, (T, nq)).reshape(-1)
    qm = np.asarray(q_meas, dtype=np.float64)
    if qm.ndim == 1:
        qm = np.broadcast_to(qm, (T, nZ))
    qm = np.broadcast_to(qm, (T, nZ)).reshape(-1)
    p = np.concatenate([pd, qm]).astype(np.float64)
    coord = np.array([(checks[c][2], checks[c][0], t) for t in range(1, T + 2) for c in range(nZ)],
                     dtype=np.int64)
    return Dem(f"rotated_phenom_d{d}_T{T}", H, p, obs, coord,
               {"d": d, "T": T, "nZ": nZ, "checks": checks})


# --------------------------------------------------------------------------
# Small codes used to pin the oracle
# --------------------------------------------------------------------------

def repetition_line(n: int, p) -> Dem:
    """n bits on a line, detectors x_i xor x_{i+1}, observable x_0."""
    H = np.zeros((n - 1, n), dtype=np.uint8)
    for i in range(n - 1):
        H[i, i] = 1
        H[i, i + 1] = 1
    obs = np.zeros((1, n), dtype=np.uint8)
    obs[0, 0] = 1
    coord = np.array([(i, 0, 0) for i in range(n - 1)], dtype=np.int64)
    return Dem(f"repetition_{n}", H, _rates(p, n), obs, coord, {"n": n})


def surface2d_bitflip(d: int, p) -> Dem:
    """Unrotated planar surface code of distance d, one sector.

    Flips live on edges of a grid with d rows; each row has d horizontal edges
    whose outermost ones dangle (rough left and right boundaries), with d-1
    vertices between them, and (d-1)^2 vertical edges join the vertices of
    consecutive rows.  n = d^2 + (d-1)^2 (13 at d = 3), d (d-1) vertex checks.
    Observable: the horizontal edges of column 0.
      vertex (i, j), i in [0, d-1), j in [0, d)  -> j (d-1) + i
      horizontal edge (i, j), i in [0, d]        -> j d + i   (i in [0, d))
      vertical edge (i, j..j+1)                  -> d^2 + j (d-1) + i
    """
    nv = d * (d - 1)
    n = d * d + (d - 1) ** 2
    H = np.zeros((nv, n), dtype=np.uint8)
    for j in range(d):
        for i in range(d):
            e = j * d + i
            if i - 1 >= 0:
                H[j * (d - 1) + (i - 1), e] = 1
            if i <= d - 2:
                H[j * (d - 1) + i, e] = 1
    for j in range(d - 1):
        for i in range(d - 1):
            e = d * d + j * (d - 1) + i
            H[j * (d - 1) + i, e] = 1
            H[(j + 1) * (d - 1) + i, e] = 1
    obs = np.zeros((1, n), dtype=np.uint8)
    for j in range(d):
        obs[0, j * d] = 1
    coord = np.array([(i, j, 0) for j in range(d) for i in range(d - 1)], dtype=np.int64)
    return Dem(f"surface2d_d{d}", H, _rates(p, n), obs, coord, {"d": d})


def five_qubit_stabilizers():
    """Generators and logicals of the [[5,1,3]] code as Pauli strings (paper, Sec. 3.1).

    The paper's X logical as printed anticommutes with three of the four
    generators; XXXXX, which commutes with all of them and anticommutes with
    the printed Z logical, is used instead.
    """
    return (["XZZXI", "IXZZX", "XIXZZ", "ZXIXZ"], "XXXXX", "IZIXX")
