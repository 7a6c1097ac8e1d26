"""GPU parity of the gauge rounds (tn3d_net_with_gauge_rounds: rounds of
identity gates on every bond before each layer after the first) against the
oracle's sweep with the same rounds, at equal chi and rank rule, and in the
exact limit; the gradient of a network with gauge rounds."""

import sys

import numpy as np
import pytest

import synth
from oracle.exact import frontier_logprobs
from oracle.grad import loglik_grad_exact
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


def gpu_logp(tn3d, ctx, net, m, prm):
    syn = torch.from_numpy(np.ascontiguousarray(m)).to("cuda:0")
    lp, fl = tn3d.tn3d_contract_cosets(ctx, net, syn, prm)
    torch.cuda.synchronize()
    return lp.cpu().numpy()[:, :2], fl.cpu().numpy()


@pytest.mark.parametrize("rounds", [1, 2])
def test_gauge_rounds_rotated_d5_equal_chi(ctx, rounds):
    """Rotated d = 5, 5 + 1 rounds, chi = chi_m = 6 (truncating), FP64 and the
    reduced rule: 8 syndromes against the oracle with the same gauge rounds,
    every coset within 1e-9 or twice the oracle's spread under two SVD
    drivers."""
    from paper_2310_10722_amd import tn3d
    say(f"case: gauge rounds {rounds}, rotated d=5 chi=6 fp64, 8 syndromes")
    dem, m, _, _ = synth.config_workload(2, n=8)
    base = tn3d.tn3d_net_rotated_phenom(ctx, 5, 5, dem.p)
    net = tn3d.tn3d_net_with_gauge_rounds(ctx, base, rounds)
    assert net.shape == base.shape
    prm = tn3d.tn3d_params_default(6, 6, tn3d.PREC_FP64)
    prm.eps_rel, prm.tau_gap = 1e-6, 1e-4
    got, _ = gpu_logp(tn3d, ctx, net, m, prm)
    plain, _ = gpu_logp(tn3d, ctx, base, m, prm)

    def ref(drv):
        return np.array([[sweep_logprob(rotated_network(5, 5, dem.params["checks"], dem.p, m[k], c), 6, 6,
                                        prm.eps_rel, prm.tau_gap, svd_driver=drv, gauge_rounds=rounds)[0]
                          for c in range(2)] for k in range(8)])
    r0 = ref("gesdd")
    spread = np.abs(ref("gesvd") - r0)
    err = np.abs(got - r0)
    say("  max |d log p| =", err.max(), " driver spread", spread.max(),
        " change by the rounds", np.abs(got - plain).max())
    assert np.all(err <= np.maximum(1e-9, 2.0 * spread))
    assert np.abs(got - plain).max() > 1e-9  # the rounds change the truncated value


def test_gauge_rounds_point_L4_and_exact_limit(ctx):
    """Point sector L = 4, chi = 4, two rounds, against the oracle (1e-9); the
    rotated d = 3 network untruncated with two rounds against the exact
    contraction (1e-9)."""
    from paper_2310_10722_amd import tn3d
    say("case: gauge rounds 2, point L=4 chi=4 and rotated d=3 exact")
    dem = synth.surface3d_point(4, 0.1)
    m, _ = synth.sample_syndromes(dem, 4, 23)
    net = tn3d.tn3d_net_with_gauge_rounds(ctx, tn3d.tn3d_net_surface3d_point(ctx, 4, dem.p), 2)
    prm = tn3d.tn3d_params_default(4, 4, tn3d.PREC_FP64)
    prm.eps_rel, prm.tau_gap = 1e-6, 1e-4
    got, _ = gpu_logp(tn3d, ctx, net, m, prm)
    ref = np.array([[sweep_logprob(point3d_network(4, dem.p, m[k], c), 4, 4, prm.eps_rel, prm.tau_gap,
                                   gauge_rounds=2)[0] for c in range(2)] for k in range(4)])
    say("  point L=4: max |d log p| =", np.abs(got - ref).max())
    assert np.abs(got - ref).max() <= 1e-9
    d3 = synth.rotated_phenom(3, 2, 0.05, 0.05)
    d3 = d3.with_p(np.random.default_rng(24).uniform(0.02, 0.3, d3.n_mech))
    m3, _ = synth.sample_syndromes(d3, 4, 25)
    n3 = tn3d.tn3d_net_with_gauge_rounds(ctx, tn3d.tn3d_net_rotated_phenom(ctx, 3, 2, d3.p), 2)
    prm = tn3d.tn3d_params_default(16, 16, tn3d.PREC_FP64)
    prm.eps_rel, prm.tau_gap = 1e-12, 1e-9
    got, _ = gpu_logp(tn3d, ctx, n3, m3, prm)
    ex = np.array([frontier_logprobs(d3.H, d3.p, d3.obs, m3[k]) for k in range(4)])
    say("  rotated d=3 exact limit: max |d log p| =", np.abs(got - ex).max())
    assert np.abs(got - ex).max() <= 1e-9
    # the gradient of a network with rounds rebuilds its changed networks with them
    grad, _, _, _, _ = tn3d.tn3d_grad_loglik(ctx, n3, torch.from_numpy(m3).to("cuda:0"), prm)
    want = sum(loglik_grad_exact(d3.H, d3.p, d3.obs, m3[k])[1] for k in range(4))
    say("  gradient with rounds: max |d grad| =", np.abs(grad.cpu().numpy() - want).max())
    assert np.allclose(grad.cpu().numpy(), want, rtol=1e-7, atol=1e-7)


def test_gauge_rounds_invalid(ctx):
    from paper_2310_10722_amd import tn3d
    dem = synth.surface3d_point(3, 0.1)
    base = tn3d.tn3d_net_surface3d_point(ctx, 3, dem.p)
    for r in (-1, 17):
        with pytest.raises(tn3d.Tn3dError, match="INVALID"):
            tn3d.tn3d_net_with_gauge_rounds(ctx, base, r)


def test_gauge_rounds_with_chi_schedule(ctx):
    """A chi-schedule counts the network's layers, not the gauge rounds; a
    round keeps the cap of the layer before it: rotated d = 5, schedule
    (4, 6, 8, 8, 6), one round, FP64, against the oracle with the same
    schedule and rounds (1e-9 or twice the driver spread)."""
    from paper_2310_10722_amd import tn3d
    say("case: gauge rounds 1 with chi-schedule (4, 6, 8, 8, 6), rotated d=5 fp64, 6 syndromes")
    dem, m, _, _ = synth.config_workload(2, n=6)
    net = tn3d.tn3d_net_with_gauge_rounds(ctx, tn3d.tn3d_net_rotated_phenom(ctx, 5, 5, dem.p), 1)
    sched = [4, 6, 8, 8, 6]
    prm = tn3d.tn3d_params_default(8, 8, tn3d.PREC_FP64)
    prm.eps_rel, prm.tau_gap = 1e-6, 1e-4
    prm.set_chi_schedule(sched)
    got, _ = gpu_logp(tn3d, ctx, net, m, prm)

    def ref(drv):
        return np.array([[sweep_logprob(rotated_network(5, 5, dem.params["checks"], dem.p, m[k], c), 8, 8,
                                        prm.eps_rel, prm.tau_gap, svd_driver=drv, chi_layers=sched,
                                        gauge_rounds=1)[0] for c in range(2)] for k in range(6)])
    r0 = ref("gesdd")
    spread = np.abs(ref("gesvd") - r0)
    err = np.abs(got - r0)
    say("  max |d log p| =", err.max(), " driver spread", spread.max())
    assert np.all(err <= np.maximum(1e-9, 2.0 * spread))
