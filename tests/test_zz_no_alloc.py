"""The allocation-free entry point (tn3d_contract_cosets_noalloc) against
tn3d_contract_cosets, through the C-ABI: two calls in a row (the second with
a smaller batch, on the same static scratch), bit-identical results (the same
kernels on the same items); an item larger than the scratch is refused."""

import sys

import numpy as np
import pytest

import synth

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


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_matches_contract_cosets(ctx, prec):
    from paper_2310_10722_amd import tn3d
    say(f"case: noalloc vs contract_cosets, rotated d=5 T=5 chi=16 {prec}, 48 then 11 syndromes")
    dem, m, _, _ = synth.config_workload(2, n=48)
    net = tn3d.tn3d_net_rotated_phenom(ctx, 5, 5, dem.p)
    prm = tn3d.tn3d_params_default(16, 16, tn3d.PREC_FP64 if prec == "fp64" else tn3d.PREC_FP32)
    for n in (48, 11):
        syn = torch.from_numpy(np.ascontiguousarray(m[:n])).cuda()
        ref, ref_f = tn3d.tn3d_contract_cosets(ctx, net, syn, prm)
        got, got_f = tn3d.tn3d_contract_cosets_noalloc(ctx, net, syn, prm)
        torch.cuda.synchronize()
        ref, ref_f, got, got_f = (t.cpu().numpy() for t in (ref, ref_f, got, got_f))
        say(f"  n={n}: max |d log p| = {np.nanmax(np.abs(got[:, :2] - ref[:, :2]))}")
        assert np.array_equal(np.isnan(got), np.isnan(ref))
        fin = np.isfinite(ref)
        assert np.all(np.abs(got[fin] - ref[fin]) <= 1e-9)
        assert np.array_equal(got[fin], ref[fin]) and np.array_equal(got_f, ref_f)


def test_noalloc_depolarizing_then_point(ctx):
    """Different networks one after the other on the same scratch (the
    second call must not see the first one's contents)."""
    from paper_2310_10722_amd import tn3d
    say("case: noalloc depolarizing L=3 then point L=3, fp64")
    dd = synth.surface3d_depolarizing(3, 0.15)
    md, _ = synth.sample_pauli(dd, 6, 5)
    nd = tn3d.tn3d_net_surface3d_depolarizing(ctx, 3, dd.params["p_qubit"])
    dp, mp_, _, _ = synth.config_workload(1, n=9)
    npn = tn3d.tn3d_net_surface3d_point(ctx, 3, dp.p)
    prm = tn3d.tn3d_params_default(4, 4, tn3d.PREC_FP64)
    for net, m in ((nd, md), (npn, mp_[:5])):
        syn = torch.from_numpy(np.ascontiguousarray(m)).cuda()
        got, _ = tn3d.tn3d_contract_cosets_noalloc(ctx, net, syn, prm)
        ref, _ = tn3d.tn3d_contract_cosets(ctx, net, syn, prm)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy())


def test_noalloc_refuses_items_beyond_the_scratch(ctx):
    """The 3D planar code at L=8, chi = 32 in FP64 needs about a gigabyte per
    item: beyond the static scratch, refused with TN3D_E_OOM before any launch."""
    from paper_2310_10722_amd import tn3d
    dem, m, _, _ = synth.config_workload(3, n=1)
    net = tn3d.tn3d_net_surface3d_point(ctx, 8, dem.p)
    prm = tn3d.tn3d_params_default(32, 32, tn3d.PREC_FP64)
    with pytest.raises(tn3d.Tn3dError, match="OOM.*static scratch"):
        tn3d.tn3d_contract_cosets_noalloc(ctx, net, torch.from_numpy(m).cuda(), prm)
