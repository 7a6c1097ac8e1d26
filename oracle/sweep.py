"""O-3: fixed-chi boundary sweep with simple-update truncation, FP64, LAPACK.

What it computes (paper Sec. 4): a 2D network (a PEPS whose physical legs
are the open legs towards the unabsorbed part) absorbs the layers of a
layered 3D network one at a time.  Each layer is applied as one-site ops and
two-site gates; after every gate the bond between the two sites is truncated
back to at most chi with the simple-update rule: one positive diagonal lambda
per bond stands in for the environment of the rest of the network, the two
tensors with the lambdas of their other legs absorbed are QR-factorised, the
gate is applied to the two R factors and the bond lambda, and a truncated SVD
of that block gives the new bond, its new lambda (normalised to the largest
singular value, whose log goes to a scale accumulator) and, through the Q
factors, the new tensors with the other-leg lambdas divided out again.  After
the last layer the remaining 2D network is contracted by a boundary MPS of
bond chi_m, row by row, each row absorbed with the zip-up scheme and
truncated by SVD.

Conventions fixed here (the paper leaves them to the simple-update
literature, Sec. 4):
  * gate order per layer: pre-ops, then bonds (x,y)-(x+1,y) with x even,
    x odd, then (x,y)-(x,y+1) with y even, y odd; within a class bonds are
    disjoint; then post-ops; then every site is divided by its max |entry|.
  * rank rule: keep the largest D <= min(chi, #S) with S_D > eps_rel * S_1 and
    (D = #S or S_{D+1} < (1 - tau_gap) S_D), i.e. never cut inside a cluster of
    singular values equal to relative precision tau_gap; if none, D =
    min(chi, #S) and the result is flagged (a degenerate cluster was split).
  * final stage: contract f_s into the physical leg, put sqrt(lambda) on both
    ends of every bond, boundary MPS from row 0 down, zip-up left to right,
    every new MPS site divided by its max |entry|.
Pins: with chi at or above the exact bond dimensions the sweep equals the
frontier contraction (tests); the result does not depend on the LAPACK SVD
driver beyond rounding (tests).
"""

from __future__ import annotations

import numpy as np

from .network import E_, N_, S_, W_, Layer, LayeredNet

FLAG_TRUNC_CLUSTER = 1 << 1
FLAG_NUMERIC = 1 << 0


def rank_rule(S, chi, eps_rel, tau_gap):
    """Returns (D, split_cluster)."""
    n = len(S)
    top = min(chi, n)
    if n == 0 or S[0] <= 0.0:
        return 0, True
    s1 = S[0]
    for D in range(top, 0, -1):
        if S[D - 1] <= eps_rel * s1:
            continue
        if D == n or S[D] < (1.0 - tau_gap) * S[D - 1]:
            return D, False
    return top, True


def _svd(A, driver):
    if driver == "gesdd":
        return np.linalg.svd(A, full_matrices=False)
    import scipy.linalg as sl
    return sl.svd(A, full_matrices=False, lapack_driver=driver)


class Sweep:
    def __init__(self, net: LayeredNet, chi, chi_m, eps_rel=1e-9, tau_gap=1e-6,
                 svd_driver="gesdd", chi_layers=None, gauge_rounds=0):
        self.net = net
        # rounds of identity gates on every bond before each layer after the
        # first (simple update with trivial gates: the bond environments move
        # towards the Vidal gauge before the layer's truncations)
        self.gauge_rounds = gauge_rounds
        self.Lx, self.Ly = net.Lx, net.Ly
        self.chi, self.chi_m = chi, chi_m
        # chi-schedule: the gates of layer l keep at most
        # chi_layers[min(l, len - 1)] values (None: chi for every layer)
        self.chi_layers = list(chi_layers) if chi_layers else None
        self.chi_cur = chi
        self.eps, self.tau = eps_rel, tau_gap
        self.driver = svd_driver
        self.G = [t.copy() for t in net.init]
        self.lamH = {}
        self.lamV = {}
        for y in range(self.Ly):
            for x in range(self.Lx):
                if x + 1 < self.Lx:
                    D = self.G[y * self.Lx + x].shape[E_]
                    self.lamH[(x, y)] = np.ones(D)
                if y + 1 < self.Ly:
                    D = self.G[y * self.Lx + x].shape[S_]
                    self.lamV[(x, y)] = np.ones(D)
        self.logscale = 0.0
        self.flags = 0
        self.n_split = 0
        self.signed = False  # allow a negative contraction value (signed networks)
        self.sign = 1.0

    # lambda of the bond on `leg` of site (x, y), or None at the grid edge
    def _lam(self, x, y, leg):
        if leg == W_:
            return self.lamH.get((x - 1, y))
        if leg == E_:
            return self.lamH.get((x, y))
        if leg == N_:
            return self.lamV.get((x, y - 1))
        return self.lamV.get((x, y))

    def _scale_legs(self, T, x, y, legs, power):
        for leg in legs:
            lam = self._lam(x, y, leg)
            if lam is None:
                continue
            shape = [1] * 5
            shape[leg] = lam.size
            T = T * (lam.reshape(shape) ** power)
        return T

    def one_site(self, s, M):
        self.G[s] = np.tensordot(M, self.G[s], axes=([1], [0]))

    def gate(self, kind, x, y, G4):
        Lx = self.Lx
        if kind == "H":
            (xa, ya), (xb, yb), la, lb = (x, y), (x + 1, y), E_, W_
            lam = self.lamH[(x, y)]
        else:
            (xa, ya), (xb, yb), la, lb = (x, y), (x, y + 1), S_, N_
            lam = self.lamV[(x, y)]
        sa, sb = ya * Lx + xa, yb * Lx + xb
        A, B = self.G[sa], self.G[sb]
        othA = [l for l in (W_, E_, N_, S_) if l != la]
        othB = [l for l in (W_, E_, N_, S_) if l != lb]
        MA = self._scale_legs(A, xa, ya, othA, 1.0)
        MB = self._scale_legs(B, xb, yb, othB, 1.0)
        # matrices (other legs) x (p, bond)
        permA = othA + [0, la]
        permB = othB + [0, lb]
        MA_t = np.transpose(MA, permA)
        MB_t = np.transpose(MB, permB)
        oshapeA, oshapeB = MA_t.shape[:3], MB_t.shape[:3]
        dA, D = MA_t.shape[3], MA_t.shape[4]
        dB = MB_t.shape[3]
        QA, RA = np.linalg.qr(MA_t.reshape(-1, dA * D))
        QB, RB = np.linalg.qr(MB_t.reshape(-1, dB * D))
        rA, rB = RA.shape[0], RB.shape[0]
        RA3 = RA.reshape(rA, dA, D)
        RB3 = RB.reshape(rB, dB, D)
        theta = np.einsum("abpq,ipx,x,jqx->iajb", G4, RA3, lam, RB3).reshape(rA * dA, rB * dB)
        U, S, Vt = _svd(theta, self.driver)
        Dn, split = rank_rule(S, self.chi_cur, self.eps, self.tau)
        if split:
            self.flags |= FLAG_TRUNC_CLUSTER
            self.n_split += 1
        if Dn == 0:
            self.flags |= FLAG_NUMERIC
            raise FloatingPointError("zero block in gate")
        s1 = S[0]
        self.logscale += np.log(s1)
        lam_new = S[:Dn] / s1
        newA = (QA @ U[:, :Dn].reshape(rA, dA * Dn)).reshape(*oshapeA, dA, Dn)
        newB = (QB @ Vt[:Dn, :].T.reshape(rB, dB * Dn)).reshape(*oshapeB, dB, Dn)
        newA = np.transpose(newA, np.argsort(permA))
        newB = np.transpose(newB, np.argsort(permB))
        if kind == "H":
            self.lamH[(x, y)] = lam_new
        else:
            self.lamV[(x, y)] = lam_new
        newA = self._scale_legs(newA, xa, ya, othA, -1.0)
        newB = self._scale_legs(newB, xb, yb, othB, -1.0)
        self.G[sa], self.G[sb] = newA, newB

    def rescale(self):
        for s in range(len(self.G)):
            c = np.max(np.abs(self.G[s]))
            if c == 0.0:
                self.flags |= FLAG_NUMERIC
                raise FloatingPointError("zero site tensor")
            self.G[s] = self.G[s] / c
            self.logscale += np.log(c)

    def layer(self, lay):
        for s in sorted(lay.pre):
            self.one_site(s, lay.pre[s])
        for cls in (("H", 0), ("H", 1), ("V", 0), ("V", 1)):
            for (kind, x, y, G4) in lay.gates:
                if kind != cls[0]:
                    continue
                par = x if kind == "H" else y
                if par % 2 != cls[1]:
                    continue
                self.gate(kind, x, y, G4)
        for s in sorted(lay.post):
            self.one_site(s, lay.post[s])
        self.rescale()

    def final_tensors(self):
        """T[w, e, n, s] per site: f contracted, sqrt(lambda) on each bond."""
        Ts = []
        for y in range(self.Ly):
            for x in range(self.Lx):
                s = y * self.Lx + x
                T = np.tensordot(self.net.final[s], self.G[s], axes=([0], [0]))
                T = self._scale_legs(T[None], x, y, (W_, E_, N_, S_), 0.5)[0]
                Ts.append(T)
        return Ts

    def boundary_mps(self, Ts):
        """Zip-up boundary MPS; returns log of the contraction value."""
        Lx, Ly = self.Lx, self.Ly
        # MPS site: [a (left), s (down-going physical), a' (right)]
        mps = [np.ones((1, 1, 1)) for _ in range(Lx)]
        logscale = 0.0
        for y in range(Ly):
            K = np.ones((1, 1, 1))  # [nu, a, omega]
            new = []
            for x in range(Lx):
                T = Ts[y * Lx + x]  # [w, e, n, s]
                M = mps[x]
                L4 = np.einsum("naw,asb->nwsb", K, M)
                theta = np.einsum("nwsb,weso->nobe", L4, T)  # [nu, s', a', omega']
                nn, so, bb, ee = theta.shape
                if x < Lx - 1:
                    mat = theta.reshape(nn * so, bb * ee)
                    U, S, Vt = _svd(mat, self.driver)
                    Dn, split = rank_rule(S, self.chi_m, self.eps, self.tau)
                    if split:
                        self.flags |= FLAG_TRUNC_CLUSTER
                        self.n_split += 1
                    if Dn == 0:
                        raise FloatingPointError("zero block in boundary MPS")
                    site = U[:, :Dn].reshape(nn, so, Dn)
                    K = (S[:Dn, None] * Vt[:Dn]).reshape(Dn, bb, ee)
                else:
                    site = theta.reshape(nn, so, bb * ee)
                c = np.max(np.abs(site))
                if c == 0.0:
                    raise FloatingPointError("zero boundary site")
                new.append(site / c)
                logscale += np.log(c)
            mps = new
        v = np.ones((1,))
        for x in range(Lx):
            v = v @ mps[x][:, 0, :]
        z = float(v[0])
        if self.signed and z < 0.0:
            self.sign = -1.0
            z = -z
        if not z > 0.0:
            self.flags |= FLAG_NUMERIC
            return np.nan
        return logscale + np.log(z)

    def gauge_round(self):
        """Identity gates on every bond, the four classes in the layer order,
        each truncated at the current cap (that of the layer before), then the
        per-site rescale of a layer."""
        Lx, Ly = self.Lx, self.Ly
        gates = []
        for y in range(Ly):
            for x in range(Lx):
                s = y * Lx + x
                dA = self.G[s].shape[0]
                if x + 1 < Lx:
                    dB = self.G[s + 1].shape[0]
                    gates.append(("H", x, y, np.einsum("ac,bd->abcd", np.eye(dA), np.eye(dB))))
                if y + 1 < Ly:
                    dB = self.G[s + Lx].shape[0]
                    gates.append(("V", x, y, np.einsum("ac,bd->abcd", np.eye(dA), np.eye(dB))))
        self.layer(Layer(gates=gates))

    def run(self):
        for li, lay in enumerate(self.net.layers):
            if li > 0:
                for _ in range(self.gauge_rounds):
                    self.gauge_round()
            if self.chi_layers:
                self.chi_cur = min(self.chi, self.chi_layers[min(li, len(self.chi_layers) - 1)])
            self.layer(lay)
        Ts = self.final_tensors()
        return self.logscale + self.boundary_mps(Ts)


def sweep_logprob(net: LayeredNet, chi, chi_m=None, eps_rel=1e-9, tau_gap=1e-6,
                  svd_driver="gesdd", chi_layers=None, gauge_rounds=0):
    """log of the approximate contraction value of one network; returns
    (logp, flags, n_cluster_splits).  The rank rule defaults to the FP64 rule
    (eps_rel 1e-9, tau_gap 1e-6); a strict rule (1e-12, 1e-9) is passed
    explicitly where the exact limit is compared."""
    sw = Sweep(net, chi, chi if chi_m is None else chi_m, eps_rel, tau_gap, svd_driver, chi_layers,
               gauge_rounds)
    try:
        lp = sw.run()
    except FloatingPointError:
        return np.nan, sw.flags | FLAG_NUMERIC, sw.n_split
    return lp, sw.flags, sw.n_split


def sweep_signed(net: LayeredNet, chi, chi_m=None, eps_rel=1e-9, tau_gap=1e-6, svd_driver="gesdd"):
    """The same sweep for a network whose value may be negative (the signed
    Walsh-Hadamard networks of Sec. 3.1): returns (log |Z|, sign of Z, flags).
    Site rescaling divides by positive maxima and the truncations keep
    positive singular values, so the sign of Z is the sign of the final
    boundary-MPS contraction."""
    sw = Sweep(net, chi, chi if chi_m is None else chi_m, eps_rel, tau_gap, svd_driver)
    sw.signed = True
    try:
        lp = sw.run()
    except FloatingPointError:
        return np.nan, 0.0, sw.flags | FLAG_NUMERIC
    return lp, sw.sign, sw.flags
