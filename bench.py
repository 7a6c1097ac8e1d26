"""Benchmark: syndromes decoded per second at fixed chi on one MI355X.

Headline workload (--config 3, the default): the 3D planar surface code at
L = 8, point sector, i.i.d. flips p = 0.2; 256 seeded syndromes (both cosets
each: 512 sweeps of an 8 x 8 grid through 7 layers); chi = chi_mps = 32; the
BF16 precision mode (FP32 site tensors; the reabsorption and boundary-MPS
contraction on BF16 matrix cores with FP32 accumulation, the Grams on FP64
matrix cores; truncations and log accumulators in FP64), rank rule eps_rel
1e-6 / tau_gap 1e-2 (the reduced-precision rule).  A step is one tn3d_decode
call over the whole batch with the syndromes already resident in HBM,
replaying the captured launch sequences:
the BF16 contraction of every (syndrome, coset), the decision, and the FP64
re-sweep (Gram route, same chi and rule) of every item whose BF16 log-ratio
lies inside the library's near-tie band (4e-3).  At p = 0.2 the point sector
is far above its threshold, the two cosets of every syndrome are equal to
within FP64 rounding, and the whole batch is re-swept.  The timed steps run
with the kernels' device-side execution windows and work counters on (the
roofline comes from those same steps).

The JSON line also reports
  roofline            the dominant kernel of the step, from the device
                      windows and the algorithmic work the kernels count;
  roofline_streaming  the layer-absorption Gram + reabsorption kernels
                      against HBM (algorithmic bytes: each site tensor read by
                      its Gram, read and written by its reabsorption);
  bf16_pass_only      the same decode without the re-sweep (one step), with
                      the roofline of the boundary-MPS contraction k_zip_a;
  fp64_gram_route     the same batch in FP64 (Gram route), one step;
  one_syndrome_per_call  one syndrome per call (the unbatched path);
  cpu_baseline        the CPU oracle (fixed-chi FP64 sweep, same chi, chi_mps
                      and rule) on 8 syndromes x 2 cosets, one sweep per worker;
  accuracy            |log p_GPU - log p_oracle| per coset over those 8 items
                      and the 4 stored ones (tests/golden/point_L8_chi32.json),
                      and the decision agreement (tie band 2e-3).

Other workloads: --config 6 (the same L = 8 code and error draws in the loop
sector, bit flips seen by the faces, below its threshold at p = 0.2),
--config 2 (rotated d=5, phenomenological, chi = 16 or --chi, FP64, optionally
with --gauge-rounds rounds of identity gates before each layer), --config 4
(depolarizing, ragged L in {4, 5, 6}), --config 5 (the gradient of the
syndrome log-likelihood with respect to 217 rates, rotated d=7, chi = 16).
"""

from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "syndromes decoded/sec at fixed chi + coset log-prob error vs FP64 oracle"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6     # MI355X FP64 vector and FP64 matrix (dense) peak
BF16_PEAK_TFS = 2500.0   # MI355X dense BF16 matrix peak
CPU_WORKERS = 16         # the host CPU share of one GPU on the benchmark machines
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2310_10722_amd", "csrc", f) for f in ("linalg.h", "sweep.hip")]


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(profile, sweeps_per_launch):
    """HBM bytes per launch from a committed counter summary (FETCH_SIZE x
    its copy-calibrated scale + WRITE_SIZE, per sweep the launch covers)
    times the sweeps per launch, or None when the summary is missing or was
    taken on other kernel sources."""
    try:
        with open(os.path.join(ROOT, "profiles", profile)) as fh:
            text = fh.read()
    except OSError:
        return None
    rec = {}
    for line in text.splitlines():
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            rec[k.strip()] = v.strip().strip("`")
    if rec.get("kernel source sha256") != kernel_source_hash():
        return None
    try:
        return float(rec["traffic bytes per sweep and launch"]) * sweeps_per_launch
    except (KeyError, ValueError):
        return None


def say(*a):
    """Progress on stderr (the JSON line is the only stdout output)."""
    print("bench:", *a, file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def _oracle_one(args):
    fam, prm_fam, p, m, c, chi, chi_m, eps, tau = args[:9]
    rounds = args[9] if len(args) > 9 else 0
    from oracle.network import point3d_network, rotated_network
    from oracle.sweep import sweep_logprob
    if fam == "rotated":
        net = rotated_network(prm_fam["d"], prm_fam["T"], prm_fam["checks"], p, m, c)
    elif fam == "loop":
        from oracle.network import loop3d_network
        net = loop3d_network(prm_fam["L"], p, m, c)
    elif fam == "depol":
        from oracle.network import depol3d_network
        net = depol3d_network(prm_fam["L"], p, m, c)
    else:
        net = point3d_network(prm_fam["L"], p, m, c)
    return sweep_logprob(net, chi, chi_m, eps, tau, gauge_rounds=rounds)[0]


def cpu_oracle(fam, prm_fam, p, ms, prm, workers, gauge_rounds=0):
    """The oracle on every (syndrome, coset) of ms, one sweep per task, on a
    pool of `workers` single-threaded processes; returns (logp [n, 2], wall s)."""
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    jobs = [(fam, prm_fam, p, ms[i], c, prm.chi, prm.chi_mps, prm.eps_rel, prm.tau_gap, gauge_rounds)
            for i in range(len(ms)) for c in range(2)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        pool.map(int, range(workers))  # start-up outside the clock
        t0 = time.perf_counter()
        res = pool.map(_oracle_one, jobs, chunksize=1)
        dt = time.perf_counter() - t0
    import numpy as np
    return np.array(res).reshape(len(ms), 2), dt


def accuracy(np, got, ref, coset=None):
    err = np.abs(got - ref)
    fin = np.isfinite(err)
    out = {"n_items": int(ref.shape[0]), "max_abs_dlogp": float(err[fin].max()) if fin.any() else None,
           "p999_abs_dlogp": float(np.quantile(err[fin], 0.999)) if fin.any() else None,
           "cosets_within_1e-3": float(np.mean(err <= 1e-3)),
           "not_finite": [int(i) for i in np.nonzero(~fin.all(axis=1))[0]]}
    if coset is not None:
        best = np.argmax(ref, axis=1)
        out["decision_agreement"] = float(np.mean((coset == best) | (np.abs(ref[:, 0] - ref[:, 1]) <= 2e-3)))
        out["oracle_median_abs_log_ratio"] = float(np.median(np.abs(ref[:, 0] - ref[:, 1])))
    return out


def autotune_entry(tn3d, ctx, nets, syn, prm, what):
    """Runs the library's autotuner on (nets, syn) for these parameters (the
    choice is cached in the context and used by the timed steps after it)."""
    r = tn3d.tn3d_autotune(ctx, nets, syn, prm)
    return {"tuned_on": what, "choice": {"index": int(r[0]), "team8": int(r[1]), "mid": int(r[2]),
                                        "narrow_reabsorb": int(r[3])},
            "tuned_ms": r[4], "default_ms": r[5], "speedup": r[5] / r[4] if r[4] > 0 else None}


def roof_entry(name, bound, work, ms, launches, peak, unit, traffic=None):
    if not ms or ms <= 0 or not launches:
        return None
    per_launch = work / launches
    t = ms / launches
    achieved = per_launch / (t * 1e-3) / (1e12 if unit == "TFLOP/s" else 1e9)
    out = {"bound": bound, "kernel": name, "achieved": achieved, "peak": peak, "unit": unit,
           "frac": achieved / peak, ("algorithmic_flops_per_launch" if unit == "TFLOP/s" else
                                     "algorithmic_bytes_per_launch"): per_launch,
           "avg_launch_ms": t, "traffic": traffic}
    return out


def bench_point_L8(a, tn3d, np, torch):
    import synth
    loop = a.config == 6
    sector = "loop" if loop else "point"
    dem, m, _, _ = synth.config_workload(6 if loop else 3)
    B = m.shape[0]
    L, chi = 8, 32
    a.precision = a.precision or "bf16"
    if a.precision == "fp64":
        raise SystemExit("the L = 8 workloads run in bf16 or fp32 (the FP64 Gram route is reported beside them)")
    prec = {"bf16": tn3d.PREC_BF16, "fp32": tn3d.PREC_FP32}[a.precision]
    ctx = tn3d.Context(0)
    net = (tn3d.tn3d_net_surface3d_loop if loop else tn3d.tn3d_net_surface3d_point)(ctx, L, dem.p)
    prm = tn3d.tn3d_params_default(chi, chi, prec)  # the reduced-precision rule: eps_rel 1e-6, tau_gap 1e-2
    # the library default near-tie band: every item whose BF16 log-ratio is
    # below it is contracted again in FP64 (Gram route) inside the same call
    syn = torch.from_numpy(m).to("cuda:0")
    tune = None
    if not a.no_autotune:
        say("autotune on 32 syndromes")
        tune = autotune_entry(tn3d, ctx, net, syn[:32], prm, "syndromes 0..31 (the choice holds for the network "
                                                             "and parameters)")
    ctx.set_timing(1)  # device windows and work counters inside the captured sequence
    for i in range(a.warmup):
        tn3d.tn3d_decode(ctx, net, syn, prm)
        torch.cuda.synchronize()
        say(f"warmup step {i + 1}/{a.warmup} done")
    ctx.set_timing(1)  # the sums restart: they cover the timed steps only
    results = None
    t0 = time.perf_counter()
    for i in range(a.steps):
        results = tn3d.tn3d_decode(ctx, net, syn, prm)
        if a.steps > 1:
            torch.cuda.synchronize()
            say(f"timed step {i + 1}/{a.steps} done")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    say(f"{a.steps} timed steps: {dt:.2f} s")
    t = ctx.last_timing()
    (lay_ms, fin_ms, hot_ms, hot_launch, hot_bytes, eig_ms, eig_launch, eig_flops, za_ms, za_flops, za_launch,
     sub_ms, sub_flops, sub_launch, sub_sweeps) = t
    coset, lr, logp, flags = [x.cpu().numpy() for x in results]
    rf_eig = roof_entry("k_zip_bsub (boundary-MPS leading eigenpairs of families above 64 vectors: subspace "
                        "iteration with Rayleigh-Ritz on the FP64 matrix cores; BF16 pass and FP64 re-sweep)", "mfma",
                        sub_flops, sub_ms, sub_launch, FP64_PEAK_TFS, "TFLOP/s",
                        recorded_traffic("pmc_k_zip_bsub_point_L8_chi32_bf16.md",
                                         sub_sweeps / sub_launch if sub_launch else 0.0))
    if rf_eig:
        rf_eig["sweeps_per_launch"] = sub_sweeps / sub_launch
    stream = roof_entry("k_gram2 + k_reabsorb2 + k_reabsorb (site-tensor streaming; BF16 pass and FP64 re-sweep)",
                        "hbm", hot_bytes, hot_ms, hot_launch, HBM_PEAK_GBS, "GB/s", None)
    out = {"metric": METRIC, "value": a.steps * B / dt, "unit": "syndromes/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": dt * 1e3 / a.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "bf16" if prec == tn3d.PREC_BF16 else "f32",
           "data": "synthetic (seeded Bernoulli flips of every qubit, p = 0.2)",
           "config": {"workload": f"3D planar surface code L=8, {sector} sector, i.i.d. flips p=0.2, 8x8 grid x 7 layers, "
                                  "chi=32, chi_mps=32, 256 syndromes x 2 cosets, rank rule eps_rel 1e-6 / tau_gap "
                                  "1e-2, FP64 re-sweep of near ties", "global_batch": B, "chi": chi, "chi_mps": chi,
                      "precision": a.precision, "near_tie": prm.near_tie},
           "launch": "captured launch sequences replayed (HIP graph), device execution windows on",
           "items_reswept_fp64": int(np.sum(flags & 16 != 0)),
           "phases_ms_per_step": {"layer_absorption": lay_ms / a.steps, "boundary_mps": fin_ms / a.steps,
                                  "gram_plus_reabsorb": hot_ms / a.steps,
                                  "boundary_decomposition_small": eig_ms / a.steps,
                                  "boundary_decomposition_subspace": sub_ms / a.steps,
                                  "boundary_contraction": za_ms / a.steps},
           "roofline": rf_eig, "roofline_streaming": stream, "autotune": tune,
           "flags": {"numeric": int(np.sum(flags & 1 != 0)), "trunc_cluster": int(np.sum(flags & 2 != 0)),
                     "near_tie": int(np.sum(flags & 4 != 0)), "no_converge": int(np.sum(flags & 8 != 0))}}
    # the BF16 pass alone (no re-sweep), one instrumented step
    p0 = tn3d.tn3d_params_default(chi, chi, prec)
    p0.near_tie = 0.0
    ctx.set_timing(1)
    b0 = time.perf_counter()
    r0 = tn3d.tn3d_decode(ctx, net, syn, p0)
    torch.cuda.synchronize()
    b1 = time.perf_counter()
    t0s = ctx.last_timing()
    ctx.set_timing(0)
    say(f"BF16 pass alone: {b1 - b0:.2f} s")
    za_peak = BF16_PEAK_TFS / 6.0 if prec == tn3d.PREC_BF16 else FP64_PEAK_TFS
    rf_za = roof_entry("k_zip_a (boundary-MPS contraction Theta on the BF16 matrix cores, six BF16 products per "
                       "FP32-accurate product, and its Gram on the FP64 ones)", "mfma", t0s[9], t0s[8], t0s[10],
                       za_peak, "TFLOP/s", None)
    if rf_za:
        rf_za["peak_note"] = ("BF16 dense peak / 6 (each FP32-accurate product takes six BF16 products); the Gram "
                              "part runs on the FP64 matrix cores at 78.6")
    lp0 = r0[2].cpu().numpy()
    out["bf16_pass_only"] = {"value": B / (b1 - b0), "ms_per_step": (b1 - b0) * 1e3,
                             "note": "the same decode with near_tie = 0 (no FP64 re-sweep), one instrumented step",
                             "roofline_k_zip_a": rf_za,
                             "roofline_k_zip_bsub": roof_entry("k_zip_bsub", "mfma", t0s[12], t0s[11], t0s[13],
                                                               FP64_PEAK_TFS, "TFLOP/s", None)}
    if not a.headline_only:
        # FP64 (Gram route), one step
        p64 = tn3d.tn3d_params_default(chi, chi, tn3d.PREC_FP64)
        p64.eps_rel, p64.tau_gap = prm.eps_rel, prm.tau_gap
        p64.flags = tn3d.OPT_GRAM_FACTOR
        tn3d.tn3d_decode(ctx, net, syn, p64)
        torch.cuda.synchronize()
        f0 = time.perf_counter()
        r64 = tn3d.tn3d_decode(ctx, net, syn, p64)
        torch.cuda.synchronize()
        f1 = time.perf_counter()
        lp64 = r64[2].cpu().numpy()
        say(f"fp64 Gram-route decode: {f1 - f0:.2f} s")
        out["fp64_gram_route"] = {"value": B / (f1 - f0), "ms_per_step": (f1 - f0) * 1e3,
                                  "median_abs_log_ratio": float(np.median(r64[1].cpu().numpy()))}
        # one syndrome per call
        n1 = 4
        tn3d.tn3d_decode(ctx, net, syn[:1], prm)
        torch.cuda.synchronize()
        o0 = time.perf_counter()
        for i in range(n1):
            tn3d.tn3d_decode(ctx, net, syn[i:i + 1], prm)
        torch.cuda.synchronize()
        o1 = time.perf_counter()
        out["one_syndrome_per_call"] = {"value": n1 / (o1 - o0), "unit": "syndromes/s", "calls": n1}
        # accuracy against the stored oracle values
    if not a.headline_only and not loop:
        gold = json.load(open(os.path.join(ROOT, "tests", "golden", "point_L8_chi32.json")))
        ref_g = np.array(gold["logp"])
        it = gold["items"]
        out["accuracy_stored"] = accuracy(np, logp[it, :2], ref_g, coset[it])
        out["accuracy_stored"]["vs"] = "oracle values stored by tests/golden/make_point_L8_chi32.py (items 0, 85, " \
                                       "170, 255)"
        out["accuracy_stored"]["bf16_pass_max_abs_dlogp"] = float(np.max(np.abs(lp0[it, :2] - ref_g)))
        out["accuracy_stored"]["fp64_gram_route_max_abs_dlogp"] = float(np.max(np.abs(lp64[it, :2] - ref_g)))
    if not a.no_cpu:
        n = 8
        say(f"cpu baseline: {2 * n} oracle sweeps on {CPU_WORKERS} workers")
        ref, cdt = cpu_oracle(sector, {"L": L}, dem.p, m[:n], prm, CPU_WORKERS)
        say(f"cpu baseline: {cdt:.1f} s")
        out["cpu_baseline"] = {"value": n / cdt, "unit": "syndromes/s", "cores": CPU_WORKERS, "kind": "oracle",
                               "cpu_model": cpu_model(),
                               "sample": f"syndromes 0..{n - 1} of the 256, both cosets: {2 * n} fixed-chi FP64 "
                                         f"sweeps (numpy/LAPACK), one per single-threaded worker, same chi, chi_mps "
                                         f"and rank rule; wall time of the pool"}
        out["accuracy"] = accuracy(np, logp[:n, :2], ref, coset[:n])
        out["accuracy"]["vs"] = "CPU oracle (fixed-chi FP64 sweep), the cpu_baseline sample"
        out["accuracy"]["bf16_pass_max_abs_dlogp"] = float(np.max(np.abs(lp0[:n, :2] - ref)))
    print(json.dumps(out))


def bench_rotated_d5(a, tn3d, np, torch):
    """Rotated d=5, phenomenological p=q=0.03, 5 noisy + 1 perfect rounds,
    chi = chi_mps = 16, 1024 syndromes, FP64 (orthogonal factorisations),
    rank rule 1e-6 / 1e-4."""
    import synth
    dem, m, _, _ = synth.config_workload(2)
    B = m.shape[0]
    ctx = tn3d.Context(0)
    net = tn3d.tn3d_net_rotated_phenom(ctx, 5, 5, dem.p)
    if a.gauge_rounds > 0:
        net = tn3d.tn3d_net_with_gauge_rounds(ctx, net, a.gauge_rounds)
    prm = tn3d.tn3d_params_default(a.chi if a.chi_given else 16, a.chi if a.chi_given else 16, tn3d.PREC_FP64)
    prm.eps_rel, prm.tau_gap = 1e-6, 1e-4
    if a.gram_route:
        prm.flags = tn3d.OPT_GRAM_FACTOR
    syn = torch.from_numpy(m).to("cuda:0")
    tune = None if a.no_autotune else autotune_entry(tn3d, ctx, net, syn, prm, "the whole batch")
    for _ in range(a.warmup):
        tn3d.tn3d_decode(ctx, net, syn, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        res = tn3d.tn3d_decode(ctx, net, syn, prm)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    coset, lr, logp, flags = [x.cpu().numpy() for x in res]
    out = {"metric": METRIC, "value": a.steps * B / dt, "unit": "syndromes/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": dt * 1e3 / a.steps, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64", "data": "synthetic (seeded Bernoulli error samples of the code's DEM)",
           "config": {"workload": "rotated d=5 surface code, phenomenological p=q=0.03, 5 noisy + 1 perfect rounds, "
                                  f"5x6 grid x 4 layers, chi={prm.chi}, chi_mps={prm.chi_mps}, 1024 syndromes x 2 "
                                  f"cosets, gauge rounds {a.gauge_rounds}, FP64 "
                                  f"{'Gram' if a.gram_route else 'orthogonal'} route", "global_batch": B},
           "roofline": None, "autotune": tune}
    if not a.no_cpu:
        n = min(a.cpu_sample, B)
        ref, cdt = cpu_oracle("rotated", dict(dem.params), dem.p, m[:n], prm, CPU_WORKERS, a.gauge_rounds)
        out["cpu_baseline"] = {"value": n / cdt, "unit": "syndromes/s", "cores": CPU_WORKERS, "kind": "oracle",
                               "cpu_model": cpu_model(), "sample": f"first {n} syndromes, both cosets"}
        out["accuracy"] = accuracy(np, logp[:n, :2], ref, coset[:n])
    print(json.dumps(out))


def _oracle_grad_cosets(args):
    d, T, checks, q, m, chi, chi_m, eps, tau = args
    from oracle.network import rotated_network
    from oracle.sweep import sweep_logprob
    return [sweep_logprob(rotated_network(d, T, checks, q, m, c), chi, chi_m, eps, tau)[0] for c in (0, 1)]


def bench_rotated_d7_grad(a, tn3d, np, torch):
    """The gradient workload: rotated d=7, 7 noisy + 1 perfect rounds,
    per-qubit / per-measurement rates log-uniform in [0.005, 0.05], 256
    syndromes, chi = chi_mps = 16, FP32 site tensors, rank rule 1e-6 / 1e-2.
    A step is one tn3d_grad_loglik call: d/dr of sum_s log P(m_s) over the
    49 + 168 rate parameters (the network at the rates and at each of the 511
    single-rate changes, 256 x 512 x 2 sweeps, and the reduction)."""
    import synth
    dem, m, _, _ = synth.config_workload(5)
    B = m.shape[0]
    d, T, nq, nZ = 7, 7, 49, 24
    rate_of = np.concatenate([np.tile(np.arange(nq), T), nq + np.arange(T * nZ)]).astype(np.int32)
    a.precision = a.precision or "fp32"
    prec = {"bf16": tn3d.PREC_BF16, "fp32": tn3d.PREC_FP32, "fp64": tn3d.PREC_FP64}[a.precision]
    ctx = tn3d.Context(0)
    net = tn3d.tn3d_net_rotated_phenom(ctx, d, T, dem.p)
    prm = tn3d.tn3d_params_default(16, 16, prec)
    prm.eps_rel, prm.tau_gap = 1e-6, 1e-2
    syn = torch.from_numpy(m).to("cuda:0")
    # the forward pass alone, for the ratio
    for _ in range(2):
        tn3d.tn3d_contract_cosets(ctx, net, syn, prm)
    torch.cuda.synchronize()
    f0 = time.perf_counter()
    for _ in range(3):
        tn3d.tn3d_contract_cosets(ctx, net, syn, prm)
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - f0) * 1e3 / 3
    for i in range(a.warmup):
        tn3d.tn3d_grad_loglik(ctx, net, syn, prm, rate_of_mech=rate_of)
        torch.cuda.synchronize()
        say(f"warmup step {i + 1}/{a.warmup} done")
    ctx.set_timing(1)
    res = None
    t0 = time.perf_counter()
    for i in range(a.steps):
        res = tn3d.tn3d_grad_loglik(ctx, net, syn, prm, rate_of_mech=rate_of, per_item=(i == a.steps - 1))
        torch.cuda.synchronize()
        say(f"timed step {i + 1}/{a.steps} done")
    dt = time.perf_counter() - t0
    t = ctx.last_timing()
    ctx.set_timing(0)
    (lay_ms, fin_ms, hot_ms, hot_launch, hot_bytes, eig_ms, eig_launch, eig_flops, za_ms, za_flops, za_launch,
     sub_ms, sub_flops, sub_launch, _) = t
    grad, tot, ll, flags, items = res
    grad, ll, flags, items = grad.cpu().numpy(), ll.cpu().numpy(), flags.cpu().numpy(), items.cpu().numpy()
    rf_eig = roof_entry("k_zip_beig (boundary-MPS decompositions of families up to 64 vectors, one wavefront each)",
                        "alu", eig_flops, eig_ms, eig_launch, FP64_PEAK_TFS, "TFLOP/s", None)
    stream = roof_entry("k_gram2 + k_reabsorb2 + k_reabsorb (site-tensor streaming)", "hbm", hot_bytes, hot_ms,
                        hot_launch, HBM_PEAK_GBS, "GB/s", None)
    rf_sub = roof_entry("k_zip_bsub (boundary-MPS leading eigenpairs of families above 64 vectors: subspace "
                        "iteration on the FP64 matrix cores)", "mfma", sub_flops, sub_ms, sub_launch, FP64_PEAK_TFS,
                        "TFLOP/s", None)
    rf_za = roof_entry("k_zip_a (boundary-MPS contraction Theta and its Gram, FP64 matrix cores)", "mfma", za_flops,
                       za_ms, za_launch, FP64_PEAK_TFS, "TFLOP/s", None)
    cands = [(eig_ms, rf_eig), (hot_ms, stream), (sub_ms, rf_sub), (za_ms, rf_za)]
    dom = max((c for c in cands if c[1] is not None), key=lambda c: c[0], default=(0, None))[1]
    out = {"metric": "syndrome log-likelihood gradients/sec at fixed chi (d/dr sum_s log P(m_s), 217 rates)",
           "value": a.steps * B / dt, "unit": "syndromes/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
           "ms_per_step": dt * 1e3 / a.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"bf16": "bf16", "fp32": "f32", "fp64": "f64"}[a.precision],
           "data": "synthetic (seeded Bernoulli error samples of the code's DEM)",
           "config": {"workload": "rotated d=7 surface code, phenomenological noise, 7 noisy + 1 perfect rounds, "
                                  "per-qubit / per-measurement rates log-uniform in [0.005, 0.05], 7x8 grid x 7 "
                                  "layers, chi=16, chi_mps=16, 256 syndromes, gradient over 49 + 168 rates "
                                  "(511 mechanisms)", "global_batch": B, "precision": a.precision},
           "forward_only_ms": fwd_ms, "gradient_over_forward": (dt * 1e3 / a.steps) / fwd_ms,
           "phases_ms_per_step": {"layer_absorption": lay_ms / a.steps, "boundary_mps": fin_ms / a.steps,
                                  "gram_plus_reabsorb": hot_ms / a.steps,
                                  "boundary_decomposition_small": eig_ms / a.steps,
                                  "boundary_decomposition_subspace": sub_ms / a.steps,
                                  "boundary_contraction": za_ms / a.steps},
           "roofline": dom, "roofline_streaming": stream, "roofline_k_zip_beig": rf_eig,
           "roofline_k_zip_bsub": rf_sub, "roofline_k_zip_a": rf_za,
           "loglik_sum": float(tot.cpu()[0]), "grad_abs_max": float(np.abs(grad).max()),
           "flags": {"numeric": int(np.sum(flags & 1 != 0)), "trunc_cluster": int(np.sum(flags & 2 != 0)),
                     "no_converge": int(np.sum(flags & 8 != 0))}}
    if not a.no_cpu:
        # the oracle's one-sided gradient of one syndrome over every mechanism
        from oracle.grad import loglik_grad_one_sided
        k = 0
        jobs = [(d, T, dem.params["checks"], dem.p, m[k], prm.chi, prm.chi_mps, prm.eps_rel, prm.tau_gap)]
        for i in range(dem.n_mech):
            q = dem.p.copy()
            q[i] = dem.p[i] + 0.25 if dem.p[i] <= 0.5 else dem.p[i] - 0.25  # the oracle's changed rate
            jobs.append((d, T, dem.params["checks"], q, m[k], prm.chi, prm.chi_mps, prm.eps_rel, prm.tau_gap))
        for v in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            os.environ[v] = "1"
        say(f"cpu baseline: {2 * len(jobs)} oracle sweeps on {CPU_WORKERS} workers")
        mpc = mp.get_context("spawn")
        with mpc.Pool(CPU_WORKERS) as pool:
            pool.map(int, range(CPU_WORKERS))
            c0 = time.perf_counter()
            vals = pool.map(_oracle_grad_cosets, jobs, chunksize=1)
            cdt = time.perf_counter() - c0
        say(f"cpu baseline: {cdt:.1f} s")
        table = {-1: vals[0]}
        table.update({i: vals[i + 1] for i in range(dem.n_mech)})

        def cosets(q):
            ch = np.nonzero(q != dem.p)[0]
            return table[int(ch[0]) if ch.size else -1]

        lp, g = loglik_grad_one_sided(cosets, dem.p)
        c = np.where(dem.p <= 0.5, dem.p + 0.25, dem.p - 0.25)
        bound = (np.abs(1.0 + g * (c - dem.p)) + 1.0) * np.expm1(2.0 * (1e-3 + 4.0 * 2.0 ** -24)) / np.abs(c - dem.p)
        err = np.abs(items[k] - g)
        out["cpu_baseline"] = {"value": 1.0 / cdt, "unit": "syndromes/s", "cores": CPU_WORKERS, "kind": "oracle",
                               "cpu_model": cpu_model(),
                               "sample": f"syndrome 0: its gradient over all {dem.n_mech} mechanisms, "
                                         f"{2 * len(jobs)} fixed-chi FP64 sweeps (the network at the rates and at "
                                         f"each single-rate change), one per single-threaded worker"}
        out["accuracy"] = {"vs": "CPU oracle one-sided gradient (fixed-chi FP64 sweeps), syndrome 0",
                           "max_abs_dterm": float(err.max()), "max_err_over_bound": float((err / bound).max()),
                           "abs_dloglik": float(abs(ll[k] - lp))}
    print(json.dumps(out))


def bench_depolarizing(a, tn3d, np, torch):
    """3D planar code under depolarizing noise p = 0.15, 512 syndromes with
    L = 4, 5, 6 (171 / 171 / 170, shuffled by the seed) decoded in one ragged
    call, four cosets each, reduced rank rule, chi = chi_mps = --chi (24 by
    default: gate sides of 4 x 24 = 96 columns), FP32 site tensors by default
    (--precision; FP64 takes the Gram route there)."""
    import synth
    seed = synth.CONFIG_SEED_BASE + 4
    ctx = tn3d.Context(0)
    pr_name = a.precision or "fp32"
    prec = {"bf16": tn3d.PREC_BF16, "fp32": tn3d.PREC_FP32, "fp64": tn3d.PREC_FP64}[pr_name]
    prm = tn3d.tn3d_params_default(a.chi, a.chi, prec)
    prm.eps_rel, prm.tau_gap = 1e-6, 1e-2  # the reduced-precision rule, in every precision here
    if prec == tn3d.PREC_FP64 and 4 * a.chi > 64:
        prm.flags = tn3d.OPT_GRAM_FACTOR
    parts = []
    for L, n in ((4, 171), (5, 171), (6, 170)):
        dem = synth.surface3d_depolarizing(L, 0.15)
        m, _ = synth.sample_pauli(dem, n, seed + L)
        parts.append((L, dem, m, tn3d.tn3d_net_surface3d_depolarizing(ctx, L, dem.params["p_qubit"])))
    width = max(p[2].shape[1] for p in parts)
    rows, nets, src = [], [], []
    for L, dem, m, net in parts:
        for k in range(m.shape[0]):
            r = np.zeros(width, dtype=np.uint8)
            r[: m.shape[1]] = m[k]
            rows.append(r)
            nets.append(net)
            src.append((L, k))
    perm = np.random.Generator(np.random.PCG64(seed)).permutation(len(rows))
    syn = torch.from_numpy(np.stack([rows[i] for i in perm])).to("cuda:0")
    nets = [nets[i] for i in perm]
    B = len(nets)
    tune = None if a.no_autotune else autotune_entry(tn3d, ctx, nets, syn, prm, "the whole batch")
    for _ in range(a.warmup):
        tn3d.tn3d_decode(ctx, nets, syn, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        res = tn3d.tn3d_decode(ctx, nets, syn, prm)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    flags = res[3].cpu().numpy()
    logp = res[2].cpu().numpy()
    out = {"metric": METRIC, "value": a.steps * B / dt, "unit": "syndromes/s", "n_gpus": 1,
           "steps": a.steps, "warmup": a.warmup, "ms_per_step": dt / a.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": {"bf16": "bf16", "fp32": "f32", "fp64": "f64"}[pr_name],
           "data": "synthetic (seeded depolarizing errors)",
           "config": {"workload": f"3D planar code, depolarizing p=0.15, ragged L in (4, 5, 6) x "
                                  f"(171, 171, 170), chi={a.chi}, chi_mps={a.chi}, 512 syndromes x 4 "
                                  f"cosets, rank rule eps_rel 1e-6 / tau_gap 1e-2", "global_batch": B, "precision": pr_name},
           "roofline": None, "autotune": tune,
           "flags": {"numeric": int(np.sum(flags & 1 != 0)), "inconsistent": int(np.sum(flags & 32 != 0))}}
    if not a.no_cpu:
        # the FP64 oracle on the first item of each L in the batch, all four
        # cosets, one sweep per single-threaded worker
        for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
            os.environ[k] = "1"
        inv = np.argsort(perm)
        jobs, rows_at = [], []
        for L, dem, m, _ in parts:
            rows_at.append(int(inv[[i for i, (LL, k) in enumerate(src) if LL == L and k == 0][0]]))
            jobs += [("depol", {"L": L}, dem.params["p_qubit"], m[0], c, a.chi, a.chi, prm.eps_rel, prm.tau_gap)
                     for c in range(4)]
        t_or = time.perf_counter()
        with mp.get_context("spawn").Pool(min(CPU_WORKERS, len(jobs))) as pool:
            res_or = np.array(pool.map(_oracle_one, jobs, chunksize=1)).reshape(len(parts), 4)
        errs = []
        for q, j in enumerate(rows_at):
            b = int(np.argmax(res_or[q]))
            errs.append(abs(logp[j, b] - res_or[q, b]))
        out["accuracy"] = {"n_items": len(parts), "decoded_coset_max_abs_dlogp": float(max(errs)),
                           "vs": "CPU oracle (fixed-chi FP64 sweep), item 0 of each L, four cosets",
                           "oracle_seconds": time.perf_counter() - t_or}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 3 for the L = 8 and gradient workloads; 5 otherwise)")
    ap.add_argument("--warmup", type=int, default=None,
                    help="untimed steps (default 1 for the L = 8 and gradient workloads; 2 otherwise)")
    ap.add_argument("--config", type=int, default=3,
                    help="3: 3D planar L=8 point sector, chi 32 (the headline); 6: the same in the loop sector; "
                         "2: rotated d=5; 4: depolarizing, ragged L in {4, 5, 6}; 5: the rate gradient, rotated d=7")
    ap.add_argument("--precision", default=None, choices=("bf16", "fp32", "fp64"),
                    help="--config 3 and 6 (default bf16), --config 4 and 5 (default fp32)")
    ap.add_argument("--chi", type=int, default=None, help="chi = chi_mps for --config 4 (default 24) and 2 (16)")
    ap.add_argument("--gram-route", action="store_true",
                    help="--config 2: FP64 through Grams (TN3D_OPT_GRAM_FACTOR) instead of orthogonal factorisations")
    ap.add_argument("--gauge-rounds", type=int, default=0,
                    help="--config 2: rounds of identity gates on every bond before each layer")
    ap.add_argument("--cpu-sample", type=int, default=256)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="time the default launch shapes")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the timed steps (no other-precision, re-sweep or one-syndrome runs): the short run "
                         "a profiler traces")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-sized device buffer once (the calibration run for the HBM byte "
                         "counters of a profiler) and exit")
    a = ap.parse_args()
    a.chi_given = a.chi is not None
    if a.chi is None:
        a.chi = 24
    big = a.config in (3, 5, 6)
    if a.steps is None:
        a.steps = 3 if big else 5
    if a.warmup is None:
        a.warmup = 1 if big else 2
    if a.copy_probe > 0:
        import torch
        n = a.copy_probe * (1 << 20) // 4
        x = torch.ones(n, dtype=torch.float32, device="cuda:0")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": n * 4, "copy_probe_bytes_written": n * 4}))
        return
    if a.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the batch would shard by syndrome with no exchange during a sweep).", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2310_10722_amd import tn3d

    if a.config in (3, 6):
        return bench_point_L8(a, tn3d, np, torch)
    if a.config == 2:
        return bench_rotated_d5(a, tn3d, np, torch)
    if a.config == 4:
        return bench_depolarizing(a, tn3d, np, torch)
    if a.config == 5:
        return bench_rotated_d7_grad(a, tn3d, np, torch)
    raise SystemExit(f"no benchmark workload {a.config}")


if __name__ == "__main__":
    main()
