"""GPU parity for the generic DEM front end (tn3d_net_from_dem): graph-like
detector error models on a grid, swept along the detector coordinate t, at
bond dimensions that truncate nothing, against the exact frontier
contraction of the same DEM (O-2)."""

import sys

import numpy as np
import pytest

import synth
from oracle.exact import frontier_logprobs

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


def exact_params(tn3d):
    prm = tn3d.tn3d_params_default(16, 64, tn3d.PREC_FP64)
    prm.eps_rel, prm.tau_gap = 1e-12, 1e-9
    return prm


def test_dem_point_sector_exact(ctx):
    """The point-sector DEM of the 3D planar code at L = 3 (its detector
    coordinates give the layers) with rates drawn per mechanism."""
    from paper_2310_10722_amd import tn3d
    say("case: DEM front end, 3D planar point sector L=3, untruncated, fp64 vs exact")
    base = synth.surface3d_point(3, 0.1)
    dem = base.with_p(np.random.default_rng(31).uniform(0.02, 0.3, base.n_mech))
    m, _ = synth.sample_syndromes(dem, 8, 37)
    net = tn3d.tn3d_net_from_dem(ctx, dem.H, dem.p, dem.obs[0], dem.det_coord)
    got, flags = gpu_logp(ctx, net, m, exact_params(tn3d))
    ex = np.array([frontier_logprobs(dem.H, dem.p, dem.obs, m[k]) for k in range(8)])
    say("  max |d log p| vs exact =", np.max(np.abs(got - ex)))
    assert np.max(np.abs(got - ex)) <= 1e-9
    assert np.all(flags == 0)


def test_dem_with_parallel_and_boundary_mechanisms(ctx):
    """The same code with extra mechanisms the family builders never make:
    a second mechanism on a third of the in-plane edges and time-like edges
    (parallel), and boundary flips on a third of the detectors; the front end
    merges them exactly."""
    from paper_2310_10722_amd import tn3d
    say("case: DEM front end, point sector L=3 with parallel and extra boundary mechanisms, fp64 vs exact")
    base = synth.surface3d_point(3, 0.1)
    rng = np.random.default_rng(41)
    H = base.H.copy()
    L = 3
    nz = L ** 3
    extra = []
    for e in range(L * L, base.n_mech):
        if rng.random() < 1 / 3 and H[:, e].sum() == 2:
            extra.append(H[:, e].copy())
    for d in range(base.n_det):
        if rng.random() < 1 / 3:
            col = np.zeros(base.n_det, dtype=np.uint8)
            col[d] = 1
            extra.append(col)
    H2 = np.concatenate([H, np.array(extra, dtype=np.uint8).T], axis=1)
    n2 = H2.shape[1]
    p2 = rng.uniform(0.02, 0.3, n2)
    obs2 = np.zeros((1, n2), dtype=np.uint8)
    obs2[0, : base.n_mech] = base.obs[0]
    dem = synth.Dem("point_L3_extra", H2, p2, obs2, base.det_coord)
    m, _ = synth.sample_syndromes(dem, 8, 43)
    net = tn3d.tn3d_net_from_dem(ctx, dem.H, dem.p, dem.obs[0], dem.det_coord)
    got, _ = gpu_logp(ctx, net, m, exact_params(tn3d))
    ex = np.array([frontier_logprobs(dem.H, dem.p, dem.obs, m[k]) for k in range(8)])
    say(f"  {len(extra)} extra mechanisms; max |d log p| vs exact =", np.max(np.abs(got - ex)))
    assert np.max(np.abs(got - ex)) <= 1e-9
    assert nz > 0


def test_dem_unsupported_models(ctx):
    from paper_2310_10722_amd import tn3d
    say("case: DEM front end refuses models outside its class")
    base = synth.surface3d_point(3, 0.1)
    # a mechanism joining detectors two layers apart
    col = np.zeros((base.n_det, 1), dtype=np.uint8)
    col[0, 0] = 1
    col[base.n_det - 1, 0] = 1
    H = np.concatenate([base.H, col], axis=1)
    p = np.concatenate([base.p, [0.1]])
    obs = np.concatenate([base.obs[0], [0]])
    with pytest.raises(tn3d.Tn3dError, match="UNSUPPORTED"):
        tn3d.tn3d_net_from_dem(ctx, H, p, obs, base.det_coord)
    # an observable on an in-plane mechanism
    obs = base.obs[0].copy()
    obs[-1] = 1
    with pytest.raises(tn3d.Tn3dError, match="UNSUPPORTED"):
        tn3d.tn3d_net_from_dem(ctx, base.H, base.p, obs, base.det_coord)
    # two detectors on one grid point
    co = base.det_coord.copy()
    co[1] = co[0]
    with pytest.raises(tn3d.Tn3dError):
        tn3d.tn3d_net_from_dem(ctx, base.H, base.p, base.obs[0], co)
