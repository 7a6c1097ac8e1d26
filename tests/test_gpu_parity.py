"""GPU parity: the HIP sweep (through the C-ABI) against the CPU oracle.

Tolerances: FP64 path |d log p| <= 1e-9 against the fixed-chi oracle at the
same chi / chi_m / rank rule, for every rule (the FP64 route factors every
truncation orthogonally: Householder QR of the gate sides, one-sided Jacobi
on the boundary-MPS families); the FP64 Gram route (TN3D_OPT_GRAM_FACTOR)
<= 1e-6; FP32 path |d log p| <= 1e-3 against the same oracle; untruncated chi
against the exact frontier contraction <= 1e-9.
"""

import sys

import numpy as np
import pytest

import synth
from oracle.exact import frontier_logprobs
from oracle.network import point3d_network, rotated_network
from oracle.sweep import sweep_logprob

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
    return logp.cpu().numpy(), flags.cpu().numpy()


def oracle_point(dem, L, m, prm):
    return np.array([[sweep_logprob(point3d_network(L, dem.p, m[k], c), prm.chi, prm.chi_mps, prm.eps_rel,
                                    prm.tau_gap)[0] for c in range(2)] for k in range(m.shape[0])])


def oracle_rot(dem, m, prm, driver="gesdd"):
    d, T = dem.params["d"], dem.params["T"]
    return np.array([[sweep_logprob(rotated_network(d, T, dem.params["checks"], dem.p, m[k], c), prm.chi,
                                    prm.chi_mps, prm.eps_rel, prm.tau_gap, svd_driver=driver)[0] for c in range(2)]
                     for k in range(m.shape[0])])


def test_point_L3_fp64_chi4_full_workload(ctx):
    from paper_2310_10722_amd import tn3d
    say("case: point sector L=3 p=0.15 chi=4 fp64, 64 syndromes")
    dem, m, _, _ = synth.config_workload(1)
    net = tn3d.tn3d_net_surface3d_point(ctx, 3, dem.p)
    prm = tn3d.tn3d_params_default(4, 4, tn3d.PREC_FP64)
    got, flags = gpu_logp(ctx, net, m, prm)
    ref = oracle_point(dem, 3, m, prm)
    assert np.all(np.isfinite(got[:, :2]))
    assert np.all(np.isneginf(got[:, 2:]))
    err = np.max(np.abs(got[:, :2] - ref))
    say("  max |d log p| =", err)
    assert err <= 1e-9


def test_point_L3_exact_chi(ctx):
    from paper_2310_10722_amd import tn3d
    say("case: point sector L=3 untruncated chi=8 chi_m=64 fp64 vs exact")
    dem = synth.surface3d_point(3, 0.1).with_p(np.random.default_rng(3).uniform(0.02, 0.3, 51))
    m, _ = synth.sample_syndromes(dem, 6, 7)
    net = tn3d.tn3d_net_surface3d_point(ctx, 3, dem.p)
    prm = tn3d.tn3d_params_default(8, 64, tn3d.PREC_FP64)
    got, _ = gpu_logp(ctx, net, m, prm)
    ex = np.array([frontier_logprobs(dem.H, dem.p, dem.obs, m[k]) for k in range(6)])
    err = np.max(np.abs(got[:, :2] - ex))
    say("  max |d log p| =", err)
    assert err <= 1e-9


@pytest.mark.parametrize("d,T", [(3, 1), (3, 2), (5, 1)])
def test_rotated_exact_chi(ctx, d, T):
    from paper_2310_10722_amd import tn3d
    say(f"case: rotated d={d} T={T} untruncated fp64 vs exact")
    dem = synth.rotated_phenom(d, T, 0.05, 0.05)
    dem = dem.with_p(np.random.default_rng(d + T).uniform(0.02, 0.3, dem.n_mech))
    m, _ = synth.sample_syndromes(dem, 5, 9)
    net = tn3d.tn3d_net_rotated_phenom(ctx, d, T, dem.p)
    prm = tn3d.tn3d_params_default(16, 16, tn3d.PREC_FP64)  # nothing is truncated at these sizes
    got, _ = gpu_logp(ctx, net, m, prm)
    ex = np.array([frontier_logprobs(dem.H, dem.p, dem.obs, m[k]) for k in range(5)])
    err = np.max(np.abs(got[:, :2] - ex))
    say("  max |d log p| =", err)
    assert err <= 1e-9


def test_rotated_d5_fp64_chi16(ctx):
    from paper_2310_10722_amd import tn3d
    say("case: rotated d=5 T=5 chi=16 fp64, 12 syndromes")
    dem, m, _, _ = synth.config_workload(2, n=12)
    net = tn3d.tn3d_net_rotated_phenom(ctx, 5, 5, dem.p)
    prm = tn3d.tn3d_params_default(16, 16, tn3d.PREC_FP64)
    got, _ = gpu_logp(ctx, net, m, prm)
    ref = oracle_rot(dem, m, prm)
    err = np.max(np.abs(got[:, :2] - ref))
    say("  max |d log p| =", err)
    assert err <= 1e-9


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_rotated_d5_fp32_chi16(ctx, prec):
    from paper_2310_10722_amd import tn3d
    say(f"case: rotated d=5 T=5 chi=16 {prec}, 32 syndromes")
    dem, m, _, _ = synth.config_workload(2, n=32)
    net = tn3d.tn3d_net_rotated_phenom(ctx, 5, 5, dem.p)
    prm = tn3d.tn3d_params_default(16, 16, tn3d.PREC_FP32 if prec == "fp32" else tn3d.PREC_BF16)
    got, _ = gpu_logp(ctx, net, m, prm)
    ref = oracle_rot(dem, m, prm)
    err = np.abs(got[:, :2] - ref)
    say("  max |d log p| =", err.max(), " median", np.median(err))
    assert err.max() <= 1e-3


@pytest.mark.parametrize("prec", ["fp64", "fp64_gram", "fp32"])
def test_rotated_d5_boundary_chi32_gram_route(ctx, prec):
    """chi_m = 32 with the reduced-precision rule (eps_rel 1e-6, tau_gap 1e-4),
    so FP32 (and FP64 with the Gram option) takes the Gram route in the
    boundary MPS: the interior steps reach Gram orders 96 to 128 (measured on
    the oracle for this workload) and take the 512-thread decomposition, the
    first and last rows and the first column stay on the one-wavefront solver
    (Jacobi up to order 16, tridiagonal above).  FP64 without the option
    decomposes the families by one-sided Jacobi.  Bounds: 1e-9 in FP64,
    1e-6 on the FP64 Gram route, 1e-3 in FP32."""
    from paper_2310_10722_amd import tn3d
    say(f"case: rotated d=5 T=5 chi=16 chi_m=32 {prec}, rule 1e-6/1e-4, 6 syndromes")
    dem, m, _, _ = synth.config_workload(2, n=6)
    net = tn3d.tn3d_net_rotated_phenom(ctx, 5, 5, dem.p)
    prm = tn3d.tn3d_params_default(16, 32, tn3d.PREC_FP32 if prec == "fp32" else tn3d.PREC_FP64)
    prm.eps_rel, prm.tau_gap = 1e-6, 1e-4
    if prec == "fp64_gram":
        prm.flags = tn3d.OPT_GRAM_FACTOR
    got, flags = gpu_logp(ctx, net, m, prm)
    ref = oracle_rot(dem, m, prm)
    err = np.abs(got[:, :2] - ref)
    say("  max |d log p| =", err.max(), " flags", np.unique(flags))
    assert np.all(flags & 8 == 0)  # every decomposition converged
    assert err.max() <= {"fp64": 1e-9, "fp64_gram": 1e-6, "fp32": 1e-3}[prec]


@pytest.mark.parametrize("mode", ["fp64_default", "fp64_reduced", "fp32_reduced", "bf16_reduced"])
def test_point_L5_chi32_golden(ctx, mode):
    """3D planar code, point sector, L=5, p=0.2, chi = 32, chi_m = 4: the
    layer bonds reach 32, so the widest layer classes run (Grams of 64
    columns, truncations of order 64, reabsorption rows of 64); chi_m = 4 keeps
    the boundary-MPS families at 128 vectors or fewer (one-sided Jacobi on the
    FP64 default rule, the 512-thread Gram decomposition above 64 on the
    reduced one).  Against stored oracle values
    (tests/golden/make_point_L5_chi32.py, which calls only the oracle).  Bounds
    as for the other workloads: 1e-9 (FP64, either rule), 1e-3 (FP32)."""
    import json
    import os
    from paper_2310_10722_amd import tn3d
    say(f"case: point sector L=5 p=0.2 chi=32 chi_m=4 {mode}, 4 stored syndromes")
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "point_L5_chi32.json")))
    rule = "fp64_default" if mode == "fp64_default" else "reduced"
    m = np.array(gold["syndromes"], dtype=np.uint8)
    ref = np.array(gold["logp"][rule])
    dem = synth.surface3d_point(gold["L"], gold["p"])
    net = tn3d.tn3d_net_surface3d_point(ctx, gold["L"], dem.p)
    prec = {"fp32_reduced": tn3d.PREC_FP32, "bf16_reduced": tn3d.PREC_BF16}.get(mode, tn3d.PREC_FP64)
    prm = tn3d.tn3d_params_default(gold["chi"], gold["chi_mps"], prec)
    prm.eps_rel, prm.tau_gap = gold["rules"][rule]
    got, _ = gpu_logp(ctx, net, m, prm)
    err = np.abs(got[:, :2] - ref)
    say("  max |d log p| =", err.max())
    assert err.max() <= {"fp64_default": 1e-9, "fp64_reduced": 1e-9, "fp32_reduced": 1e-3, "bf16_reduced": 1e-3}[mode]


@pytest.mark.parametrize("mode", ["fp64", "fp32"])
def test_rotated_d7_nonuniform_rates(ctx, mode):
    """Rotated d=7, 7 noisy + 1 perfect rounds, one rate per data qubit and
    per measurement drawn log-uniform in [0.005, 0.05] (the forward pass of
    the gradient workload): a 7 x 8 grid, 511 mechanisms with unequal rates,
    chi = chi_m = 16, 8 syndromes against the oracle, with the reduced rank
    rule (eps_rel 1e-6, tau_gap 1e-4).  The finer FP64 default rule is not
    compared on this workload: there the cut follows rounding noise in tiny
    singular values, and the oracle's own values miss the exact ones by up to
    1.5 nats, while the reduced rule stays within the chi = 16 truncation
    error (at most 0.15 nats on the items checked against the exact
    contraction).  FP64: every coset within 1e-9 of the oracle or within
    twice the oracle's own spread under two LAPACK SVD drivers (divide and
    conquer, QR iteration), whichever is larger: on this workload the FP64
    rounding of the problem itself reaches 8e-8 on minority cosets.  FP32: the
    decoded (majority) coset within 1e-3 and the same decision; the minority
    coset, a component e^-gap of the swept state (gap = 4 to 17 nats here),
    is read from site tensors rounded at about 4 eps_32 of the state, so its
    error is at most 1e-3 + 4 eps_32 e^gap (measured up to 1.2 eps_32 e^gap,
    0.13 nats at gap 15)."""
    from paper_2310_10722_amd import tn3d
    say(f"case: rotated d=7 T=7 non-uniform rates chi=16 {mode}, rule 1e-6/1e-4, 8 syndromes")
    dem, m, _, _ = synth.config_workload(5, n=8)
    net = tn3d.tn3d_net_rotated_phenom(ctx, 7, 7, dem.p)
    prm = tn3d.tn3d_params_default(16, 16, tn3d.PREC_FP64 if mode == "fp64" else tn3d.PREC_FP32)
    prm.eps_rel, prm.tau_gap = 1e-6, 1e-4
    got, flags = gpu_logp(ctx, net, m, prm)
    ref = oracle_rot(dem, m, prm)
    assert np.all(np.isfinite(ref)) and np.all(np.isfinite(got[:, :2]))
    err = np.abs(got[:, :2] - ref)
    say("  max |d log p| =", err.max())
    if mode == "fp64":
        spread = np.abs(oracle_rot(dem, m, prm, driver="gesvd") - ref)
        say("  oracle driver spread", spread.max())
        assert np.all(err <= np.maximum(1e-9, 2.0 * spread))
    else:
        maj = np.argmax(ref, axis=1)
        rows = np.arange(len(maj))
        say("  majority", err[rows, maj].max(), " minority", err[rows, 1 - maj].max())
        assert err[rows, maj].max() <= 1e-3
        assert np.all(np.argmax(got[:, :2], axis=1) == maj)
        gap = np.abs(ref[:, 0] - ref[:, 1])
        assert np.all(err[rows, 1 - maj] <= 1e-3 + 4.0 * 2.0 ** -24 * np.exp(gap))


def test_decode_and_ragged_batch(ctx):
    from paper_2310_10722_amd import tn3d
    say("case: ragged batch L=2 / L=3 decode fp64")
    d2 = synth.surface3d_point(2, 0.15)
    d3 = synth.surface3d_point(3, 0.15)
    m2, _ = synth.sample_syndromes(d2, 5, 1)
    m3, _ = synth.sample_syndromes(d3, 5, 2)
    n2 = tn3d.tn3d_net_surface3d_point(ctx, 2, d2.p)
    n3 = tn3d.tn3d_net_surface3d_point(ctx, 3, d3.p)
    width = max(d2.n_det, d3.n_det)
    syn = np.zeros((10, width), dtype=np.uint8)
    nets = []
    for i in range(10):
        if i % 2 == 0:
            syn[i, :d2.n_det] = m2[i // 2]
            nets.append(n2)
        else:
            syn[i, :d3.n_det] = m3[i // 2]
            nets.append(n3)
    prm = tn3d.tn3d_params_default(4, 4, tn3d.PREC_FP64)
    coset, lr, logp, flags = tn3d.tn3d_decode(ctx, nets, torch.from_numpy(syn).cuda(), prm)
    torch.cuda.synchronize()
    logp = logp.cpu().numpy()
    for i in range(10):
        L, dem, m = (2, d2, m2[i // 2]) if i % 2 == 0 else (3, d3, m3[i // 2])
        ref = oracle_point(dem, L, m[None], prm)[0]
        assert np.max(np.abs(logp[i, :2] - ref)) <= 1e-9
        best = int(np.argmax(ref))
        assert int(coset[i]) == best or abs(ref[0] - ref[1]) <= 2e-9
        assert float(lr[i]) == pytest.approx(abs(ref[0] - ref[1]), abs=1e-8)


def test_deterministic_and_empty(ctx):
    from paper_2310_10722_amd import tn3d
    say("case: determinism and empty batch")
    dem, m, _, _ = synth.config_workload(2, n=8)
    net = tn3d.tn3d_net_rotated_phenom(ctx, 5, 5, dem.p)
    prm = tn3d.tn3d_params_default(16, 16, tn3d.PREC_FP32)
    a, _ = gpu_logp(ctx, net, m, prm)
    b, _ = gpu_logp(ctx, net, m, prm)
    assert np.array_equal(a, b)
    e, f = gpu_logp(ctx, net, m[:0], prm)
    assert e.shape == (0, 4)


def test_near_tie_fp64_resweep(ctx):
    """FP32 decode with a wide near-tie band: exactly the items whose FP32
    log-ratio falls inside it are contracted again in FP64 (same chi and rank
    rule, Gram route) and then agree with the oracle to 1e-6; the others keep
    the FP32 result (1e-3)."""
    from paper_2310_10722_amd import tn3d
    say("case: near-tie re-sweep, point sector L=3 p=0.15 chi=4 fp32, band 0.5")
    dem, m, _, _ = synth.config_workload(1)
    net = tn3d.tn3d_net_surface3d_point(ctx, 3, dem.p)
    syn = torch.from_numpy(np.ascontiguousarray(m)).cuda()
    p32 = tn3d.tn3d_params_default(4, 4, tn3d.PREC_FP32)
    p32.near_tie = 0.0
    _, lr32, _, _ = tn3d.tn3d_decode(ctx, net, syn, p32)
    p32.near_tie = 0.5
    coset, lr, logp, flags = tn3d.tn3d_decode(ctx, net, syn, p32)
    torch.cuda.synchronize()
    lr32, lr, logp, flags, coset = (t.cpu().numpy() for t in (lr32, lr, logp, flags, coset))
    band = lr32 < 0.5
    resw = (flags & tn3d.FLAG_RESWEPT) != 0
    say("  re-swept", int(resw.sum()), "of", len(resw))
    assert band.sum() > 0 and np.array_equal(resw, band)
    ref64 = oracle_point(dem, 3, m[band], p32)
    assert np.max(np.abs(logp[band, :2] - ref64)) <= 1e-6
    ref32 = oracle_point(dem, 3, m[~band], p32)
    assert np.max(np.abs(logp[~band, :2] - ref32)) <= 1e-3
    ref = np.empty((len(m), 2))
    ref[band], ref[~band] = ref64, ref32
    best = np.argmax(ref, axis=1)
    agree = (coset == best) | (np.abs(ref[:, 0] - ref[:, 1]) <= 2e-3)
    assert agree.all()
    assert np.allclose(lr, np.abs(logp[:, 0] - logp[:, 1]))


def test_rotated_d5_full_batch_sampled(ctx):
    """The full 1024-syndrome batch of the rotated d=5 workload in one decode
    call (the launch configuration of the benchmark), checked item by item
    against the FP32-rule oracle on a sample spread over the batch."""
    from paper_2310_10722_amd import tn3d
    say("case: rotated d=5 T=5 chi=16 fp32, full batch of 1024, 24 sampled items")
    dem, m, _, _ = synth.config_workload(2)
    assert m.shape[0] == 1024
    net = tn3d.tn3d_net_rotated_phenom(ctx, 5, 5, dem.p)
    prm = tn3d.tn3d_params_default(16, 16, tn3d.PREC_FP32)
    coset, lr, logp, flags = tn3d.tn3d_decode(ctx, net, torch.from_numpy(m).cuda(), prm)
    torch.cuda.synchronize()
    coset, logp, flags = coset.cpu().numpy(), logp.cpu().numpy(), flags.cpu().numpy()
    assert np.all(np.isfinite(logp[:, :2]).all(axis=1) | ((flags & tn3d.FLAG_NUMERIC) != 0))
    idx = np.linspace(0, 1023, 24).astype(int)
    ref = oracle_rot(dem, m[idx], prm)
    err = np.abs(logp[idx, :2] - ref)
    say("  max |d log p| =", err.max())
    assert err.max() <= 1e-3
    best = np.argmax(ref, axis=1)
    assert np.all((coset[idx] == best) | (np.abs(ref[:, 0] - ref[:, 1]) <= 2e-3))


def test_rotated_d5_full_batch_headline_fp64(ctx):
    """The benchmark's timed configuration: the full 1024-syndrome batch,
    FP64 site tensors, rank rule eps_rel 1e-6 / tau_gap 1e-4, one decode call
    with graph replay.  Sampled items against the oracle at the same chi and
    rule, bound 1e-9."""
    from paper_2310_10722_amd import tn3d
    say("case: rotated d=5 T=5 chi=16 fp64, rule 1e-6/1e-4, full batch of 1024, 24 sampled items")
    dem, m, _, _ = synth.config_workload(2)
    net = tn3d.tn3d_net_rotated_phenom(ctx, 5, 5, dem.p)
    prm = tn3d.tn3d_params_default(16, 16, tn3d.PREC_FP64)
    prm.eps_rel, prm.tau_gap = 1e-6, 1e-4
    syn = torch.from_numpy(m).cuda()
    for _ in range(2):  # the second call replays the captured sequence
        coset, lr, logp, flags = tn3d.tn3d_decode(ctx, net, syn, prm)
    torch.cuda.synchronize()
    coset, logp, flags = coset.cpu().numpy(), logp.cpu().numpy(), flags.cpu().numpy()
    assert np.all(np.isfinite(logp[:, :2]).all(axis=1) | ((flags & tn3d.FLAG_NUMERIC) != 0))
    idx = np.linspace(0, 1023, 24).astype(int)
    ref = oracle_rot(dem, m[idx], prm)
    fin = np.isfinite(ref).all(axis=1)
    err = np.abs(logp[idx, :2] - ref)[fin]
    say("  max |d log p| =", err.max())
    assert err.max() <= 1e-9
    best = np.argmax(ref[fin], axis=1)
    assert np.all((coset[idx][fin] == best) | (np.abs(ref[fin, 0] - ref[fin, 1]) <= 2e-9))


def test_unsupported_width_is_refused(ctx):
    """A gated site wider than the kernels hold (physical dim x chi > 96: 4 x
    32 on the rotated code's widest sites) is refused with
    TN3D_E_UNSUPPORTED before any launch."""
    from paper_2310_10722_amd import tn3d
    dem, m, _, _ = synth.config_workload(2, n=2)
    net = tn3d.tn3d_net_rotated_phenom(ctx, 5, 5, dem.p)
    prm = tn3d.tn3d_params_default(32, 32, tn3d.PREC_FP32)
    with pytest.raises(tn3d.Tn3dError, match="UNSUPPORTED"):
        gpu_logp(ctx, net, m, prm)


def test_graph_cache_separates_factorisation_routes(ctx):
    """The FP64 Gram route and the FP64 orthogonal route use different
    workspace layouts: calls that alternate between them on one context (same
    network, batch, chi and rank rule) each replay their own captured
    sequence and equal the eager launches bit for bit."""
    from paper_2310_10722_amd import tn3d
    say("case: graph cache, FP64 Gram route and orthogonal route alternating, rotated d=5 chi=16")
    dem, m, _, _ = synth.config_workload(2, n=12)
    net = tn3d.tn3d_net_rotated_phenom(ctx, 5, 5, dem.p)
    eager = tn3d.Context(0)
    eager.set_graphs(False)
    net_e = tn3d.tn3d_net_rotated_phenom(eager, 5, 5, dem.p)
    prm = {}
    for route in ("gram", "orth"):
        prm[route] = tn3d.tn3d_params_default(16, 16, tn3d.PREC_FP64)
        prm[route].eps_rel, prm[route].tau_gap = 1e-6, 1e-4
        prm[route].flags = tn3d.OPT_GRAM_FACTOR if route == "gram" else 0
    ref = {r: gpu_logp(eager, net_e, m, prm[r]) for r in prm}
    for route in ("gram", "orth", "gram", "orth"):
        got, got_f = gpu_logp(ctx, net, m, prm[route])
        assert np.array_equal(got, ref[route][0]) and np.array_equal(got_f, ref[route][1]), route
    assert np.max(np.abs(ref["gram"][0][:, :2] - ref["orth"][0][:, :2])) <= 1e-6


def test_graph_replay_matches_eager(ctx):
    """Captured launch sequences: the first call of a shape captures, later
    calls replay.  Every replay, with other device work and synchronisations
    in between, equals the eager launches bit for bit; a new batch size
    captures a new graph; timing mode (stamp kernels in the sequence)
    replays too."""
    from paper_2310_10722_amd import tn3d
    say("case: graph replay vs eager, rotated d=5 chi=16 fp32")
    dem, m, _, _ = synth.config_workload(2, n=40)
    net = tn3d.tn3d_net_rotated_phenom(ctx, 5, 5, dem.p)
    prm = tn3d.tn3d_params_default(16, 16, tn3d.PREC_FP32)
    eager = tn3d.Context(0)
    eager.set_graphs(False)
    net_e = tn3d.tn3d_net_rotated_phenom(eager, 5, 5, dem.p)
    assert eager.graphs_cached() == 0
    for n in (40, 17):
        ref, ref_f = gpu_logp(eager, net_e, m[:n], prm)
        for rep in range(3):
            got, got_f = gpu_logp(ctx, net, m[:n], prm)
            x = torch.randn(256, 256, device="cuda:0")
            (x @ x).sum().item()
            torch.cuda.synchronize()
            assert np.array_equal(got, ref) and np.array_equal(got_f, ref_f), (n, rep)
            assert ctx.graphs_cached() >= 1
    ctx.set_timing(1)  # stamps are captured with the sequence: a new graph, same results
    n0 = ctx.graphs_cached()
    launches = []
    for rep in range(2):
        got, _ = gpu_logp(ctx, net, m[:17], prm)
        assert np.array_equal(got, gpu_logp(eager, net_e, m[:17], prm)[0])
        t = ctx.last_timing()  # sums since set_timing: both calls by the second round
        assert t[0] > 0 and t[1] > 0 and 0 < t[2] < t[0] and t[3] > 0 and t[4] > 0
        assert 0 < t[5] < t[1] and t[6] > 0 and t[7] > 0  # the Gram route's eigen-decompositions
        launches.append(t[3])
    assert launches[1] == 2 * launches[0]
    assert ctx.graphs_cached() == n0 + 1
    ctx.set_timing(1)  # restarts the sums
    assert all(v == 0 for v in ctx.last_timing())
    ctx.set_timing(0)


@pytest.mark.parametrize("mode", ["bf16", "fp32", "fp64_gram"])
def test_point_L8_chi32_full_batch_golden(ctx, mode):
    """The 3D planar code at L=8, p=0.2, chi = chi_m = 32 (layer bonds of 32,
    site tensors of 2 * 32^4 entries, boundary-MPS families of up to 1024
    vectors on the subspace-iteration solver): the whole 256-syndrome batch in
    one call, items 0, 85, 170, 255 against stored oracle values
    (tests/golden/make_point_L8_chi32.py, reduced rule).  Bounds 1e-3 (FP32),
    1e-6 (FP64 Gram route)."""
    import json
    import os
    from paper_2310_10722_amd import tn3d
    say(f"case: point sector L=8 p=0.2 chi=chi_m=32 {mode}, 256 syndromes, 4 stored")
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "point_L8_chi32.json")))
    dem, m, _, _ = synth.config_workload(3)
    assert m.shape[0] == gold["n"]
    assert np.array_equal(m[gold["items"]], np.array(gold["syndromes"], dtype=np.uint8))
    net = tn3d.tn3d_net_surface3d_point(ctx, 8, dem.p)
    prec = {"bf16": tn3d.PREC_BF16, "fp32": tn3d.PREC_FP32, "fp64_gram": tn3d.PREC_FP64}[mode]
    prm = tn3d.tn3d_params_default(32, 32, prec)
    prm.eps_rel, prm.tau_gap = gold["rule"]
    if mode == "fp64_gram":
        prm.flags = tn3d.OPT_GRAM_FACTOR
    got, flags = gpu_logp(ctx, net, m, prm)
    assert np.all(np.isfinite(got[:, :2]))
    err = np.abs(got[gold["items"], :2] - np.array(gold["logp"]))
    say("  max |d log p| =", err.max(), " flags", np.bincount(flags, minlength=1).tolist()[:16])
    assert err.max() <= (1e-6 if mode == "fp64_gram" else 1e-3)


def test_workspace_chunks_bit_equal(ctx):
    """A workspace cap that splits the batch into several chunks gives the
    same bits as one chunk (each chunk replays its own captured sequence)."""
    from paper_2310_10722_amd import tn3d
    say("case: point sector L=3 chi=4 fp64, 20 syndromes, capped workspace (several chunks) vs one chunk")
    dem, m, _, _ = synth.config_workload(1, n=20)
    net = tn3d.tn3d_net_surface3d_point(ctx, 3, dem.p)
    prm = tn3d.tn3d_params_default(4, 4, tn3d.PREC_FP64)
    one, f1 = gpu_logp(ctx, net, m, prm)
    small = tn3d.tn3d_params_default(4, 4, tn3d.PREC_FP64)
    small.workspace_bytes = 1
    with pytest.raises(tn3d.Tn3dError) as ei:
        gpu_logp(ctx, net, m, small)
    need = int(str(ei.value).split("needs ")[1].split(" ")[0])
    small.workspace_bytes = 3 * need
    got, f2 = gpu_logp(ctx, net, m, small)
    say("  one item needs", need, "bytes; cap", 3 * need)
    assert np.array_equal(got, one) and np.array_equal(f1, f2)


def test_chi_one(ctx):
    """chi = chi_m = 1 (every bond truncated to one value).  On the loop
    sector with unequal rates the cuts are never degenerate: against the
    oracle at the same chi, FP64, 1e-9.  On the point sector the parity chain
    makes the two singular values of some bonds equal, so a cut at 1 splits a
    degenerate pair and the kept vector is implementation-defined (reading
    C10): both sides flag TRUNC_CLUSTER on every such item and return finite
    values, which are not compared."""
    from oracle.network import loop3d_network
    from paper_2310_10722_amd import tn3d
    say("case: loop sector L=3 chi=1 fp64 (no degenerate cut), point sector L=3 chi=1 (degenerate cuts flagged)")
    base = synth.surface3d_loop(3, 0.1)
    dem = base.with_p(np.random.default_rng(3).uniform(0.02, 0.3, base.n_mech))
    m, _ = synth.sample_syndromes(dem, 6, 7)
    net = tn3d.tn3d_net_surface3d_loop(ctx, 3, dem.p)
    prm = tn3d.tn3d_params_default(1, 1, tn3d.PREC_FP64)
    got, flags = gpu_logp(ctx, net, m, prm)
    ref = np.array([[sweep_logprob(loop3d_network(3, dem.p, m[k], c), 1, 1, prm.eps_rel, prm.tau_gap)[0]
                     for c in range(2)] for k in range(6)])
    say("  loop sector max |d log p| =", np.max(np.abs(got[:, :2] - ref)))
    assert np.max(np.abs(got[:, :2] - ref)) <= 1e-9
    assert np.all(flags == 0)
    dem2, m2, _, _ = synth.config_workload(1, n=8)
    net2 = tn3d.tn3d_net_surface3d_point(ctx, 3, dem2.p)
    got2, flags2 = gpu_logp(ctx, net2, m2, prm)
    oflags = np.array([sweep_logprob(point3d_network(3, dem2.p, m2[k], c), 1, 1, prm.eps_rel, prm.tau_gap)[1]
                       for k in range(8) for c in range(2)]).reshape(8, 2)
    split = (oflags & 2).any(axis=1)
    say("  point sector: items with a degenerate cut", int(split.sum()), "of 8")
    assert np.all(flags2[split] & 2)
    assert np.all(np.isfinite(got2[:, :2]))


def test_rates_zero_and_one(ctx):
    """Mechanisms with rate exactly 0 or 1 (certain flips and impossible
    ones): untruncated chi against the exact contraction, FP64."""
    from paper_2310_10722_amd import tn3d
    say("case: point sector L=3 with rates 0 and 1, untruncated chi, fp64 vs exact")
    dem = synth.surface3d_point(3, 0.1)
    p = dem.p.copy()
    idx = np.random.default_rng(1).choice(len(p), 10, replace=False)
    p[idx[:5]] = 0.0
    p[idx[5:]] = 1.0
    dem = dem.with_p(p)
    m, _ = synth.sample_syndromes(dem, 6, 3)
    net = tn3d.tn3d_net_surface3d_point(ctx, 3, dem.p)
    prm = tn3d.tn3d_params_default(8, 64, tn3d.PREC_FP64)
    got, _ = gpu_logp(ctx, net, m, prm)
    ex = np.array([frontier_logprobs(dem.H, dem.p, dem.obs, m[k]) for k in range(6)])
    say("  max |d log p| vs exact =", np.max(np.abs(got[:, :2] - ex)))
    assert np.max(np.abs(got[:, :2] - ex)) <= 1e-9


def test_rate_half_closed_form(ctx):
    """p = 1/2 on every mechanism: every flip pattern has weight 2^-n, so
    P_L(m) = 2^-rank[H; l] for every consistent syndrome and both cosets
    (rank 19 at L = 3)."""
    from paper_2310_10722_amd import tn3d
    say("case: point sector L=3 p=1/2 closed form, fp64")
    dem = synth.surface3d_point(3, 0.5)
    m, _ = synth.sample_syndromes(dem, 4, 3)
    net = tn3d.tn3d_net_surface3d_point(ctx, 3, dem.p)
    prm = tn3d.tn3d_params_default(8, 64, tn3d.PREC_FP64)
    got, _ = gpu_logp(ctx, net, m, prm)
    assert np.max(np.abs(got[:, :2] + 19.0 * np.log(2.0))) <= 1e-9


def test_invalid_rates_rejected(ctx):
    from paper_2310_10722_amd import tn3d
    say("case: invalid rates rejected by the builders")
    n = synth.surface3d_point(3, 0.1).n_mech
    for bad in (-0.1, 1.5, np.nan):
        with pytest.raises(tn3d.Tn3dError):
            tn3d.tn3d_net_surface3d_point(ctx, 3, np.full(n, bad))
    with pytest.raises(ValueError):
        tn3d.tn3d_net_surface3d_point(ctx, 3, np.full(n - 1, 0.1))
    with pytest.raises(tn3d.Tn3dError):
        tn3d.tn3d_net_rotated_phenom(ctx, 5, 5, np.full(185, 2.0))


def test_chi_schedule(ctx):
    """Per-layer truncation caps (chi-schedule) against the oracle running the
    same schedule: 3D planar L = 4 (three layers) at chi = 8 with caps 4, 6, 8
    and 3, 8, FP64 (1e-9); the constant chi in between (each schedule is its
    own captured launch sequence)."""
    from paper_2310_10722_amd import tn3d
    say("case: point sector L=4 p=0.1 chi=8 fp64 with chi-schedules [4,6,8], [3,8] and constant 8")
    dem = synth.surface3d_point(4, 0.1)
    m, _ = synth.sample_syndromes(dem, 6, 29)
    net = tn3d.tn3d_net_surface3d_point(ctx, 4, dem.p)
    for sched in ([4, 6, 8], [], [3, 8]):
        prm = tn3d.tn3d_params_default(8, 8, tn3d.PREC_FP64)
        prm.set_chi_schedule(sched)
        got, _ = gpu_logp(ctx, net, m, prm)
        ref = np.array([[sweep_logprob(point3d_network(4, dem.p, m[k], c), 8, 8, prm.eps_rel, prm.tau_gap,
                                       chi_layers=sched or None)[0] for c in range(2)] for k in range(6)])
        err = np.max(np.abs(got[:, :2] - ref))
        say(f"  schedule {sched}: max |d log p| = {err}")
        assert err <= 1e-9
    bad = tn3d.tn3d_params_default(8, 8, tn3d.PREC_FP64)
    bad.set_chi_schedule([4, 9])
    with pytest.raises(tn3d.Tn3dError):
        gpu_logp(ctx, net, m, bad)


def test_autotune_keeps_results(ctx):
    """The autotuner times the launch-shape candidates on the rotated d = 5
    workload (256 syndromes, chi = 16, FP64 and FP32) and caches the fastest;
    contractions afterwards use it and stay within the precision's rounding
    of the default shape (1e-9 FP64, 1e-4 FP32 on the decoded coset), with the
    same decisions."""
    from paper_2310_10722_amd import tn3d
    dem, m, _, _ = synth.config_workload(2, n=256)
    net = tn3d.tn3d_net_rotated_phenom(ctx, 5, 5, dem.p)
    for prec, tol in ((tn3d.PREC_FP64, 1e-9), (tn3d.PREC_FP32, 1e-4)):
        say(f"case: autotune rotated d=5 chi=16 precision {prec}, 256 syndromes")
        prm = tn3d.tn3d_params_default(16, 16, prec)
        prm.eps_rel, prm.tau_gap = 1e-6, 1e-4
        before, _ = gpu_logp(ctx, net, m, prm)
        syn = torch.from_numpy(np.ascontiguousarray(m)).to("cuda:0")
        res = tn3d.tn3d_autotune(ctx, net, syn, prm)
        say(f"  chosen candidate {int(res[0])} (team {int(res[1])}, mid {int(res[2])}, narrow {int(res[3])}): "
            f"{res[4]:.3f} ms against {res[5]:.3f} ms for the default shape")
        after, _ = gpu_logp(ctx, net, m, prm)
        b = np.argmax(before[:, :2], axis=1)
        rows = np.arange(len(b))
        assert np.array_equal(np.argmax(after[:, :2], axis=1), b)
        assert np.max(np.abs(after[rows, b] - before[rows, b])) <= tol
        assert res[4] <= res[5]


def test_context_closed_before_its_network():
    """A context destroyed while one of its networks is alive detaches the
    network (its device arrays freed then); destroying the network afterwards
    only frees the handle.  The binding closes a context's networks first."""
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2310_10722_amd import tn3d
    say("case: context destroyed before its network (library order and binding order)")
    dem = synth.surface3d_point(3, 0.1)
    c2 = tn3d.Context(0)
    n2 = tn3d.tn3d_net_surface3d_point(c2, 3, dem.p)
    c2.lib.tn3d_ctx_destroy(c2.h)  # the raw C order: context first
    c2.h = None
    n2.close()
    c3 = tn3d.Context(0)
    n3 = tn3d.tn3d_net_surface3d_point(c3, 3, dem.p)
    c3.close()  # the binding closes n3 first
    assert n3.h is None
