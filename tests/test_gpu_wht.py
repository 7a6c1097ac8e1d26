"""GPU parity for the Walsh-Hadamard coset selection (paper Sec. 3.1): two
signed networks Z_0, Z_1 per syndrome, log p_{m,L} = log((Z_0 +
(-1)^L Z_1) / 2), against the oracle's signed sweeps of the same networks at
equal chi, chi_m and rank rule, and against the exact contraction where chi
truncates nothing.

Bounds: Z_0 and Z_1 agree with the oracle to the FP64 parity bound (about
1e-9 relative); the minority coset is their difference, P_min = (Z_0 -
|Z_1|)/2, so its log carries that error times (P_0 + P_1)/P_min = 1 + e^gap.
"""

import sys

import numpy as np
import pytest

import synth
from oracle.exact import frontier_logprobs
from oracle.network import loop3d_network_wht, point3d_network, point3d_network_wht
from oracle.sweep import sweep_logprob, sweep_signed

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_10722_amd import tn3d
    return tn3d.Context(0)


def gpu_logp(ctx, net, m, prm):
    from paper_2310_10722_amd import tn3d
    syn = torch.from_numpy(np.ascontiguousarray(m)).to("cuda:0")
    logp, flags = tn3d.tn3d_contract_cosets(ctx, net, syn, prm)
    torch.cuda.synchronize()
    return logp.cpu().numpy()[:, :2], flags.cpu().numpy()


def oracle_wht(build, m, prm):
    out = []
    for k in range(m.shape[0]):
        z = []
        for b in range(2):
            lz, sg, _ = sweep_signed(build(m[k], b), prm.chi, prm.chi_mps, prm.eps_rel, prm.tau_gap)
            z.append(sg * np.exp(lz))
        with np.errstate(invalid="ignore", divide="ignore"):
            out.append([np.log(0.5 * (z[0] + (-1) ** c * z[1])) for c in range(2)])
    return np.array(out)


def height_order(L):
    nz, nx = L ** 3, L * (L - 1) ** 2
    keys = []
    for e in range(nz + 2 * nx):
        if e < nz:
            keys.append((2 * (e // (L * L)) + 1, e))
        elif e < nz + nx:
            keys.append((2 * ((e - nz) // (L * (L - 1)) + 1), e))
        else:
            keys.append((2 * ((e - nz - nx) // ((L - 1) * L) + 1), e))
    return [e for _, e in sorted(keys)]


def check_fp64(got, ref):
    """Where a truncated |Z_1| exceeds Z_0 the minority coset's value is not
    positive (NaN with NUMERIC, reading C14) on both sides alike; the other
    values are compared."""
    assert np.array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref).any(axis=1)
    say("  items with a non-positive coset value (both sides):", int((~ok).sum()))
    g, r = got[ok], ref[ok]
    err = np.abs(g - r)
    maj = np.argmax(r, axis=1)
    rows = np.arange(len(maj))
    gap = np.abs(r[:, 0] - r[:, 1])
    say("  decoded coset", err[rows, maj].max(), " other", err[rows, 1 - maj].max(), " gap max", gap.max())
    assert err[rows, maj].max() <= 1e-9
    assert np.all(err[rows, 1 - maj] <= 1e-9 * (1.0 + np.exp(gap)))
    bad = np.nonzero(~ok)[0]
    if bad.size:
        # the finite coset of such an item still agrees
        fin = np.isfinite(ref[bad])
        assert np.max(np.abs(got[bad][fin] - ref[bad][fin])) <= 1e-9


@pytest.mark.parametrize("sector", ["point", "loop"])
def test_wht_exact_chi(ctx, sector):
    from paper_2310_10722_amd import tn3d
    say(f"case: Walsh-Hadamard {sector} L=3 untruncated chi=8 chi_m=64 fp64 vs exact")
    base = synth.surface3d_point(3, 0.1) if sector == "point" else synth.surface3d_loop(3, 0.1)
    dem = base.with_p(np.random.default_rng(9).uniform(0.03, 0.3, base.n_mech))
    m, _ = synth.sample_syndromes(dem, 6, 19)
    net = tn3d.tn3d_net_surface3d_wht(ctx, 3, tn3d.SECTOR_POINT if sector == "point" else tn3d.SECTOR_LOOP, dem.p)
    prm = tn3d.tn3d_params_default(8, 64, tn3d.PREC_FP64)
    prm.eps_rel, prm.tau_gap = 1e-12, 1e-9  # the strict rule: no singular value of the exact bonds is dropped
    got, flags = gpu_logp(ctx, net, m, prm)
    order = None if sector == "point" else height_order(3)
    ex = np.array([frontier_logprobs(dem.H, dem.p, dem.obs, m[k], order=order) for k in range(6)])
    check_fp64(got, ex)
    assert np.all(flags == 0)


def test_wht_point_L3_chi4(ctx):
    """The small point-sector workload (L = 3, p = 0.15, chi = chi_m = 4, 64
    syndromes) in the Walsh-Hadamard form, against the oracle's signed sweeps
    (FP64); and the measured accuracy of both coset selections against the
    exact values on the decoded coset."""
    from paper_2310_10722_amd import tn3d
    say("case: Walsh-Hadamard point sector L=3 p=0.15 chi=4 fp64, 64 syndromes")
    dem, m, _, _ = synth.config_workload(1)
    net = tn3d.tn3d_net_surface3d_wht(ctx, 3, tn3d.SECTOR_POINT, dem.p)
    prm = tn3d.tn3d_params_default(4, 4, tn3d.PREC_FP64)
    got, _ = gpu_logp(ctx, net, m, prm)
    ref = oracle_wht(lambda mm, b: point3d_network_wht(3, dem.p, mm, b), m, prm)
    check_fp64(got, ref)
    chain = tn3d.tn3d_net_surface3d_point(ctx, 3, dem.p)
    gch, _ = gpu_logp(ctx, chain, m, prm)
    ex = np.array([frontier_logprobs(dem.H, dem.p, dem.obs, m[k]) for k in range(m.shape[0])])
    b = np.argmax(ex, axis=1)
    rows = np.arange(len(b))
    e_w, e_c = np.abs(got[rows, b] - ex[rows, b]), np.abs(gch[rows, b] - ex[rows, b])
    say(f"  vs exact, decoded coset: Walsh-Hadamard max {e_w.max():.2e} median {np.median(e_w):.2e}; "
        f"parity chain max {e_c.max():.2e} median {np.median(e_c):.2e}")
    assert e_w.max() < 0.2 and e_c.max() < 0.2


def test_wht_loop_L4_chi8(ctx):
    from paper_2310_10722_amd import tn3d
    say("case: Walsh-Hadamard loop sector L=4 p=0.15 chi=8 fp64, 8 syndromes")
    dem = synth.surface3d_loop(4, 0.15)
    m, _ = synth.sample_syndromes(dem, 8, 23)
    net = tn3d.tn3d_net_surface3d_wht(ctx, 4, tn3d.SECTOR_LOOP, dem.p)
    prm = tn3d.tn3d_params_default(8, 8, tn3d.PREC_FP64)
    got, _ = gpu_logp(ctx, net, m, prm)
    ref = oracle_wht(lambda mm, b: loop3d_network_wht(4, dem.p, mm, b), m, prm)
    check_fp64(got, ref)


def test_wht_fp32_decoded_coset(ctx):
    """FP32 site tensors: the decoded coset within 1e-3 of the FP64 oracle
    (the minority coset is a difference of nearly equal FP32 values and is
    not compared)."""
    from paper_2310_10722_amd import tn3d
    say("case: Walsh-Hadamard point sector L=3 chi=4 fp32 (reduced rule), 32 syndromes")
    dem, m, _, _ = synth.config_workload(1, n=32)
    net = tn3d.tn3d_net_surface3d_wht(ctx, 3, tn3d.SECTOR_POINT, dem.p)
    prm = tn3d.tn3d_params_default(4, 4, tn3d.PREC_FP32)
    prm.eps_rel, prm.tau_gap = 1e-6, 1e-4
    got, _ = gpu_logp(ctx, net, m, prm)
    ref = oracle_wht(lambda mm, b: point3d_network_wht(3, dem.p, mm, b), m, prm)
    maj = np.argmax(ref, axis=1)
    rows = np.arange(len(maj))
    err = np.abs(got[rows, maj] - ref[rows, maj])
    say("  decoded coset max |d log p| =", err.max())
    assert err.max() <= 1e-3
