"""Throughput of the well-balanced WCSPH hot path on one MI355X.

Workload (default): 3D sloshing tank 1.0 x 0.5 x 0.56 m, water depth 0.28 m,
dx = 0.002 m -> 17,500,000 fluid + 2,047,296 wall dummies, horizontal tank
forcing (A = 5 mm, period 1.2x the first natural period), delta-SPH,
shifting, TIC and free-surface detection on.  A step is one full SSP-RK2 step:
two right-hand sides, each with wall mirror, fused pair pass, free-surface
detection and stage update, plus the device-side dt reduction; the first
sorts the particles into cells (hash, counting sort, reorder) and keeps its
candidate lists, the second runs from them (cells of 1.01 h leave room for
the lists' skin; --keep-cell 0 sorts and searches at both right-hand sides).

Prints one compact JSON line on stdout (a few KB: metric, value = pair
evaluations per second of the FP64 path, ms/step, the dominant kernel's
roofline, the CPU oracle baseline, one summary per path -- mixed, learned,
single precision -- and per side measurement); the full record (histories,
probe traces, per-kernel times) goes to the file given by --detail.  Progress
goes to stderr.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms/step & pair evals/s at 17.5M particles, FP64 vs mixed+learned; spurious |u|"
PEAK_FP64_TFLOPS = 78.6   # MI355X FP64 vector: 256 CU x 64 lanes x 2 (FMA) x 2.4 GHz
PEAK_FP32_TFLOPS = 157.3  # MI355X FP32 vector (packed); non-packed issue equals the FP64 figure
# Algorithmic floating-point operations of the pair pass, counted from the body:
# per in-range ordered pair (3D body of Eq. sph with delta-SPH and shifting),
# and per candidate distance test (difference vector and squared norm).
FLOP_PER_PAIR_3D = 95
FLOP_PER_TEST_3D = 8
# sources of the profiled pair kernels (the committed counter summaries hold
# their hash; the traffic is reported only while it matches)
_F64_SRC = ["paper_2608_22269_amd/csrc/pair.hip", "paper_2608_22269_amd/csrc/common.h",
            "paper_2608_22269_amd/csrc/coop.h", "paper_2608_22269_amd/csrc/pair_common.h"]
_MIXED_SRC = ["paper_2608_22269_amd/csrc/mixed.hip", "paper_2608_22269_amd/csrc/common.h",
              "paper_2608_22269_amd/csrc/coop.h", "paper_2608_22269_amd/csrc/pair_common.h",
              "paper_2608_22269_amd/csrc/mixed.h"]
PAIR_SOURCES = {"pair_f64": _F64_SRC, "pair_kept_f64": _F64_SRC, "pair_mixed": _MIXED_SRC, "pair_kept_mixed": _MIXED_SRC}


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def source_sha(paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profile_summary(kernel_key):
    """The committed counter summary of a kernel if it was taken on the
    current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"{kernel_key}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("source_sha") != source_sha(d.get("sources", [])):
        return None
    return d


def load_classifier():
    path = os.path.join(ROOT, "paper_2608_22269_amd", "data", "fs_classifier.npz")
    with np.load(path) as z:
        return {k: z[k] for k in ("params", "mean", "std", "margin")}


def misclassification(sim, case, clf):
    """Free-surface flags of the learned detector against the exact scan-region
    criterion on the same state: one right-hand side with the trained margin,
    one with an infinite margin (every candidate decided by the exact test)."""
    f = case["kind"] == 0
    sim.eval_rates()
    fs_l = sim.field("fs")[f]
    st = sim.stats()
    sim.set_classifier(clf["params"], clf["mean"], clf["std"], float("inf"))
    sim.eval_rates()
    fs_e = sim.field("fs")[f]
    sim.set_classifier(clf["params"], clf["mean"], clf["std"], float(clf["margin"]))
    wrong = int((fs_l != fs_e).sum())
    cand = max(float(st["n_cand"]), 1.0)
    return {"fluid": int(f.sum()), "candidates": int(st["n_cand"]), "decided_by_mlp": int(st["n_mlp"]),
            "fallback_exact": int(st["n_scan"]), "misclassified": wrong,
            "rate_of_fluid": wrong / max(int(f.sum()), 1), "rate_of_candidates": wrong / cand,
            "fs_exact": int(fs_e.sum()), "fs_learned": int(fs_l.sum())}


def run_path(case, label, steps, warmup, clf=None, after=None):
    import torch
    from paper_2608_22269_amd import Simulation

    log(f"{label}: init ({case['meta']['n_fluid']} fluid + {case['meta']['n_dummy']} dummies)")
    t0 = time.time()
    sim = Simulation(case)
    if clf is not None:
        sim.set_classifier(clf["params"], clf["mean"], clf["std"], float(clf["margin"]))
    torch.cuda.synchronize()
    log(f"{label}: init done in {time.time() - t0:.1f} s; warmup {warmup} steps")
    sim.step(warmup)
    sim.sync()
    sim.profile(True)
    sim.profile_read()
    stream = sim.stream
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    sim.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_total = e0.elapsed_time(e1)
    sim.sync()
    prof = sim.profile_read()
    st = sim.stats()
    sim.profile(False)
    kept = st["n_kept"] > 0
    # pairs and candidate tests of the last searching pass and of the last
    # pass from kept lists
    pairs_rhs = st["pairs_search"]
    tests_rhs = st["tests_search"]
    ms_step = ms_total / steps
    pair_evals_per_step = (st["pairs_search"] + st["pairs_kept"]) if kept else 2.0 * pairs_rhs
    pair = prof["pair"]
    pair_ms = pair["ms"] / max(pair["launches"], 1)
    flops = pairs_rhs * FLOP_PER_PAIR_3D + tests_rhs * FLOP_PER_TEST_3D
    achieved = flops / (pair_ms * 1e-3) / 1e12 if pair_ms > 0 else None
    out = {
        "ms_per_step": ms_step,
        "pair_evals_per_s": pair_evals_per_step / (ms_step * 1e-3),
        "pairs_per_rhs": pairs_rhs,
        "candidate_tests_per_rhs": tests_rhs,
        "pair_pass_ms": pair_ms,
        "pair_pass_tflops": achieved,
        "rhs_from_kept_lists": st["n_kept"],
        "rhs_sorted": st["n_rebuilt"],
        "searching_passes_per_step": pair["launches"] / steps,
        "kernel_ms_per_step": {k: v["ms"] / steps for k, v in prof.items()},
        "t_end": st["t"],
        "umax_end": st["umax"],
        "fs_count": st["n_fs"],
        "fs_candidates": st["n_cand"],
    }
    if kept:
        kp = prof["pair_kept"]
        kept_ms = kp["ms"] / max(kp["launches"], 1)
        kflops = st["pairs_kept"] * FLOP_PER_PAIR_3D + st["tests_kept"] * FLOP_PER_TEST_3D
        out["kept_pass"] = {"ms": kept_ms, "pairs": st["pairs_kept"], "kept_candidates_tested": st["tests_kept"],
                            "tflops": kflops / (kept_ms * 1e-3) / 1e12, "launches_per_step": kp["launches"] / steps}
    if clf is not None:
        out["fs_decided_by_mlp"] = st["n_mlp"]
        out["fs_fallback_exact"] = st["n_scan"]
    log(f"{label}: {ms_step:.2f} ms/step, {out['pair_evals_per_s']:.3e} pair-evals/s, "
        f"searching pair pass {pair_ms:.2f} ms x {pair['launches'] / steps:.2f} per step")
    if clf is not None:
        out["misclassification"] = misclassification(sim, case, clf)
        log(f"{label}: free-surface misclassification {out['misclassification']}")
    if after is not None:
        after(sim, out)
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return out


def cpu_baseline(dx):
    """The CPU oracle on a bounded sample of the same workload: a 0.2 x 0.1 m
    column of the sloshing tank at the same dx, depth and physics (one
    right-hand side), timed on the host cores."""
    import oracle
    import workloads as wl

    sample = wl.slosh3d(dx=dx, tank=(0.2, 0.1, 0.56), depth=0.28)
    nthreads = oracle.num_threads()
    log(f"cpu baseline: {sample['meta']['n_fluid']} fluid sample, {nthreads} threads")
    t0 = time.perf_counter()
    r = oracle.eval_rates(sample)
    el = time.perf_counter() - t0
    f = sample["kind"] == 0
    pairs = float(r["nnb"][f].sum())
    # one host core (the paper's CPU reference is a single core), on a
    # narrower column
    small = wl.slosh3d(dx=dx, tank=(0.05, 0.1, 0.56), depth=0.28)
    oracle.set_num_threads(1)
    try:
        t1 = time.perf_counter()
        r1 = oracle.eval_rates(small)
        el1 = time.perf_counter() - t1
    finally:
        oracle.set_num_threads(nthreads)
    pairs1 = float(r1["nnb"][small["kind"] == 0].sum())
    return {
        "value": pairs / el, "unit": "pair-evals/s", "cores": int(nthreads), "kind": "oracle",
        "sample": (f"one right-hand side of a 0.2 x 0.1 x 0.56 m column of the sloshing tank at dx={dx} "
                   f"({sample['meta']['n_fluid']} fluid + {sample['meta']['n_dummy']} dummies, "
                   f"{pairs:.3e} ordered pairs) in {el:.2f} s"),
        "sample_short": (f"1 RHS of a 0.2x0.1x0.56 m column of the tank, {sample['meta']['n_fluid']} fluid, "
                         f"{el:.1f} s"),
        "single_core": {"value": pairs1 / el1, "unit": "pair-evals/s", "cores": 1,
                        "sample": (f"one right-hand side of a 0.05 x 0.1 x 0.56 m column ({small['meta']['n_fluid']} "
                                   f"fluid, {pairs1:.3e} ordered pairs) in {el1:.2f} s")},
    }


def spurious_velocity(precision, steps):
    """Hydrostatic 2D tank (5,000 fluid, the scheme without stabilisers):
    fluid max |U| every 50 steps up to `steps`."""
    import workloads as wl
    from paper_2608_22269_amd import Simulation
    case = wl.tank2d(precision=precision)
    f = case["kind"] == 0
    sim = Simulation(case)
    out = {}
    for k in range(50, steps + 1, 50):
        sim.step(50)
        out[str(k)] = float(np.abs(sim.field("u")[f]).max())
    sim.close()
    log(f"tank2d {precision}: max |U| {out}")
    return out


def mlp_inference(n, reps=5):
    """BF16 MFMA inference of the trained classifier over n rows of 16 FP32
    features (seeded normal values scaled like the training data), as one
    call on 17.5M particles would run it; HBM bytes 16 x 4 in + 4 out per
    row, 2 x (16 x 64 + 64 x 64 + 64) FLOP per row."""
    import torch
    from paper_2608_22269_amd import learn
    clf = load_classifier()
    g = torch.Generator(device="cuda").manual_seed(5)
    X = torch.randn(n, 16, device="cuda", generator=g) * torch.as_tensor(clf["std"], device="cuda") \
        + torch.as_tensor(clf["mean"], device="cuda")
    s = torch.cuda.current_stream()
    learn.infer_bf16(clf["params"], clf["mean"], clf["std"], X)  # warm-up
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        learn.infer_bf16(clf["params"], clf["mean"], clf["std"], X)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    nbytes = n * (16 * 4 + 4)
    flop = n * 2 * (16 * 64 + 64 * 64 + 64)
    del X
    return {"rows": n, "ms_per_call": ms, "rows_per_s": n / (ms * 1e-3),
            "hbm_gb_s": nbytes / (ms * 1e-3) / 1e9, "hbm_frac": nbytes / (ms * 1e-3) / 8e12,
            "tflops": flop / (ms * 1e-3) / 1e12, "bf16_mfma_frac": flop / (ms * 1e-3) / 2.5e15,
            "note": "includes the per-call upload of the weights and the normalisation (5,345 floats)"}


def state_of(sim, case):
    """A case dict holding the simulation's current fluid state (and a free
    body's state; its dummies stay in their reference pose)."""
    c = dict(case)
    c["x"], c["u"], c["phi"], c["mass"] = sim.field("x"), sim.field("u"), sim.field("phi"), sim.field("mass")
    d = case["kind"] != 0
    c["u"][d] = case["u"][d]
    c["phi"][d] = case["phi"][d]
    if case.get("body") is not None:
        b = case["kind"] == 2
        c["x"][b] = case["x"][b]
        st = sim.body_state()
        c["body"] = {k: [float(v) for v in st[k]] for k in ("c", "q", "v", "w")}
    c["t"] = sim.stats()["t"]
    return c


def dambreak_detection(spin, steps):
    """Exact vs learned free-surface detection on a dam break the classifier
    never saw (its training used the 3.22 x 1 x 1 m tank with a 1.2 x 1 x
    0.55 m column and a 2.0 x 0.6 x 1.0 m tank with a 0.5 x 0.6 x 0.6 m
    column, both at dx = 0.01): a 2.4 x 0.7 x 0.9 m tank, a 0.7 x 0.7 x
    0.45 m column, dx = 0.008 (mixed precision), after `spin` steps of the
    collapse: step time, detection time per step and misclassification on
    the same state."""
    import workloads as wl
    from paper_2608_22269_amd import Simulation
    clf = load_classifier()
    case = wl.dambreak3d(dx=0.008, tank=(2.4, 0.7, 0.9), column=(0.7, 0.7, 0.45), precision="mixed")
    case = wl.with_params(case, cell_size=case["params"]["h"])
    sim = Simulation(case)
    sim.step(spin)
    state = state_of(sim, case)
    sim.close()
    out = {"workload": (f"3D dam break (held out) tank 2.4x0.7x0.9, column 0.7x0.7x0.45, dx=0.008, "
                        f"{case['meta']['n_fluid']} fluid, after {spin} steps (t = {state['t']:.3f} s)")}
    out.update(detection_from_state(state, steps, "dam break", clf))
    return out


def detection_from_state(state, steps, label, clf):
    """Step time and detection time with exact and learned detection from one
    state, and the learned detector's misclassification on it."""
    import torch
    import workloads as wl
    from paper_2608_22269_amd import Simulation
    out = {}
    for mode in ("exact", "learned"):
        s2 = Simulation(wl.with_params(state, fs_mode=mode))
        if mode == "learned":
            s2.set_classifier(clf["params"], clf["mean"], clf["std"], float(clf["margin"]))
        s2.step(2)
        s2.sync()
        s2.profile(True)
        s2.profile_read()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s2.stream)
        s2.step(steps)
        e1.record(s2.stream)
        torch.cuda.synchronize()
        prof = s2.profile_read()
        st = s2.stats()
        s2.profile(False)
        r = {"ms_per_step": e0.elapsed_time(e1) / steps, "fs_detect_ms_per_step": prof["fs_detect"]["ms"] / steps,
             "pair_ms_per_step": prof["pair"]["ms"] / steps, "candidates": st["n_cand"], "fluid": st["n_fluid"]}
        if mode == "learned":
            r["misclassification"] = misclassification(s2, state, clf)
        s2.close()
        out[mode] = r
        log(f"{label} {mode}: {r}")
    return out


def cylinder_detection(dx, spin, steps):
    """The learned detector on the cylinder water entry (a splash crown and
    cavity no training snapshot holds; FP64, the free body): `spin` steps
    with exact detection from the release, then exact against learned
    detection from that state."""
    import workloads as wl
    from paper_2608_22269_amd import Simulation
    clf = load_classifier()
    case = wl.cylinder_entry(3, dx=dx)
    case = wl.with_params(case, cell_size=case["params"]["h"])
    sim = Simulation(case)
    sim.step(spin)
    state = state_of(sim, case)
    sim.close()
    out = {"workload": (f"cylinder entry dx={dx}, {case['meta']['n_fluid']} fluid, after {spin} steps "
                        f"(t = {state['t'] * 1e3:.2f} ms, body centre {state['body']['c'][2]:.4f} m, "
                        f"v_z {state['body']['v'][2]:.3f} m/s)")}
    out.update(detection_from_state(state, steps, "cylinder entry", clf))
    return out


def sloshing_after_spinup(dx, keep_cell, spin, steps, warmup):
    """The sloshing tank's forced flow itself as the timed state: `spin` steps
    from the hydrostatic start under the tank-frame forcing (FP64, lists kept
    across steps with cells of 1.03 h, the fastest exact configuration), then
    the headline configuration (cells of keep_cell h, one sort per step) and
    mixed + learned timed from that state, with the learned detector's
    misclassification on it."""
    import workloads as wl
    from paper_2608_22269_amd import Simulation
    clf = load_classifier()
    case = wl.slosh3d(dx=dx)
    h = case["params"]["h"]
    spin_case = wl.with_params(case, cell_size=1.03 * h, keep_lists=True, keep_across_steps=True)
    sim = Simulation(spin_case)
    done = 0
    while done < spin:
        k = min(1000, spin - done)
        sim.step(k)
        done += k
        st = sim.stats()
        log(f"spin-up: {done} steps, t = {st['t']:.4f} s, max |U| {st['umax']:.4f} m/s")
    state = state_of(sim, case)
    sim.close()
    state = wl.with_params(state, cell_size=keep_cell * h, keep_lists=True)
    out = {"workload": (f"sloshing tank dx={dx} after {spin} forced steps from rest (t = {state['t']:.4f} s, "
                        f"T_f = {2 * math.pi / case['params']['forcing_omega']:.4f} s)")}
    out["fp64"] = run_path(state, "fp64 after spin-up", steps, warmup)
    out["mixed_learned"] = run_path(wl.with_params(state, precision="mixed", fs_mode="learned"),
                                    "mixed_learned after spin-up", steps, warmup, clf=clf)
    return out


def slosh_surface_detection(dx, steps):
    """The learned detector on the full-size sloshing tank with a moved
    surface, a state no training snapshot holds: the first mode's shape
    (2 cm, cos(pi x/L)) released from rest, after `steps` steps of the mixed
    path with the classifier; misclassification against the exact criterion
    on that state."""
    import workloads as wl
    from paper_2608_22269_amd import Simulation
    clf = load_classifier()
    case = wl.slosh3d(dx=dx, surface_amp=0.02, precision="mixed", fs_mode="learned")
    h = case["params"]["h"]
    case = wl.with_params(case, cell_size=1.01 * h, keep_lists=True)
    sim = Simulation(case)
    sim.set_classifier(clf["params"], clf["mean"], clf["std"], float(clf["margin"]))
    sim.step(steps)
    m = misclassification(sim, case, clf)
    st = sim.stats()
    sim.close()
    m["workload"] = (f"3D sloshing tank dx={dx}, surface 0.28 + 0.02 cos(pi x/L) released from rest, "
                     f"{case['meta']['n_fluid']} fluid, after {steps} steps (t = {st['t']:.4f} s, "
                     f"max |U| {st['umax']:.3f} m/s)")
    log(f"slosh surface detection: {m}")
    return m


def dambreak_probes(seconds, every=100):
    """Pressure at probes on the downstream wall of the 3D dam break (x = 3.22
    m, y = 0.5 m; z = 0.025, 0.1, 0.2, 0.4 m) from t = 0 to `seconds`, FP64
    and mixed (all stabilisers, exact detection, cells of 1.01 h, second
    stages from kept lists; the front reaches the wall near 0.55 s, and after
    0.7 s particles pass through the wall layers): Shepard
    interpolation of p = C0^2 (rho - rho0) over the fluid within 2h of each
    probe, every `every` steps; the mixed series is interpolated to the FP64
    times.  Reports the maximum and RMS difference per probe against the
    FP64 series' largest pressure there."""
    import workloads as wl
    from paper_2608_22269_amd import Simulation
    from paper_2608_22269_amd._lib import SphError
    case = wl.dambreak3d(dx=0.01)
    h = case["params"]["h"]
    case = wl.with_params(case, cell_size=1.01 * h, keep_lists=True)
    f = case["kind"] == 0
    probes = np.array([[3.22, 0.5, z] for z in (0.025, 0.1, 0.2, 0.4)])
    alpha = 21.0 / (16.0 * np.pi * h ** 3)

    def probe_p(sim):
        x = sim.field("x")[f]
        p = sim.field("p")[f]
        V = sim.field("mass")[f] / sim.field("rho")[f]
        out = []
        for q in probes:
            d = np.sqrt(((x - q) ** 2).sum(1)) / h
            sel = d < 2.0
            w = alpha * (1.0 - 0.5 * d[sel]) ** 4 * (2.0 * d[sel] + 1.0) * V[sel]
            out.append(float((w * p[sel]).sum() / w.sum()) if w.sum() > 0 else 0.0)
        return out

    series, stops = {}, {}
    t0 = time.time()
    for prec in ("fp64", "mixed"):
        sim = Simulation(wl.with_params(case, precision=prec))
        ts, ps = [], []
        try:
            while True:
                sim.step(every)
                t, p = sim.stats()["t"], probe_p(sim)
                ts.append(t)
                ps.append(p)
                if t >= seconds:
                    break
        except SphError as e:  # a device error ends the series (reported)
            stops[prec] = str(e)
        series[prec] = (np.array(ts), np.array(ps))
        sim.close()
        log(f"dam break probes {prec}: {len(ts)} records to t = {ts[-1]:.3f} s {stops.get(prec, '')}")
    t64, p64 = series["fp64"]
    tm, pm = series["mixed"]
    keep = t64 <= tm[-1]
    pmi = np.stack([np.interp(t64[keep], tm, pm[:, k]) for k in range(len(probes))], axis=1)
    diff = pmi - p64[keep]
    scale = np.maximum(np.abs(p64).max(axis=0), 1e-30)
    # the same over moving averages of 5 records (500 steps): impact spikes
    # are not reproducible pointwise between the two paths
    ker = np.ones(5) / 5.0
    sm = lambda a: np.stack([np.convolve(a[:, k], ker, mode="valid") for k in range(a.shape[1])], axis=1)
    dsm = sm(pmi) - sm(p64[keep])
    return {
        "workload": (f"3D dam break dx=0.01, {int(f.sum())} fluid, R = 1.01 h, t = 0..{t64[-1]:.3f} s, "
                     f"every {every} steps"),
        "probes_xyz": probes.tolist(), "t": t64.tolist(), "p_fp64": p64.tolist(), "p_mixed": pm.tolist(),
        "t_mixed": tm.tolist(), "max_abs_p_fp64": scale.tolist(),
        "max_diff_over_max_p": (np.abs(diff).max(axis=0) / scale).tolist(),
        "rms_diff_over_max_p": (np.sqrt((diff ** 2).mean(axis=0)) / scale).tolist(),
        "rms_diff_of_5_record_means_over_max_p": (np.sqrt((dsm ** 2).mean(axis=0)) / scale).tolist(),
        "stopped": stops, "seconds": time.time() - t0,
    }


def hydrostatic_l2(steps, every, c0=30.0, h_factor=1.5):
    """The paper's hydrostatic cases (Sec. 4) with the paper's constants (C0 =
    30 m/s, h = 1.5 dx): a 1 x 1 m container with 1 m of water over a
    rectangular, triangular or Gaussian bottom bump 0.5 m high and 0.4 m wide
    (Gaussian: sigma = 0.1 m), dx = 0.01, the scheme without stabilisers,
    FP64: the paper's L2 velocity error sqrt(sum |U|^2 V / sum V) over the
    fluid every `every` steps.  A run stops at the first record with max |U|
    above 1 m/s (the free-surface mode's blow-up) or on a device error."""
    import workloads as wl
    from paper_2608_22269_amd import Simulation
    from paper_2608_22269_amd._lib import SphError
    out = {"_constants": {"c0": c0, "h_over_dx": h_factor, "dx": 0.01}}
    for shape in ("rect", "tri", "gauss"):
        case = wl.bump2d(shape, dx=0.01, width=1.0, depth=1.0, amp=0.5, bump_width=0.4, sigma=0.1, c0=c0,
                         h_factor=h_factor)
        f = case["kind"] == 0
        sim = Simulation(case)
        hist, err = [], None
        try:
            for k in range(0, steps, every):
                sim.step(every)
                u = sim.field("u")[f]
                V = sim.field("mass")[f] / sim.field("rho")[f]
                u2 = (u * u).sum(1)
                hist.append([k + every, sim.stats()["t"], float(np.sqrt((u2 * V).sum() / V.sum())),
                             float(np.sqrt(u2.max()))])
                if hist[-1][3] > 1.0:
                    err = "stopped: max |U| above 1 m/s"
                    break
        except SphError as e:
            err = str(e)
        sim.close()
        out[shape] = {"n_fluid": int(f.sum()), "step_t_l2_maxu": hist, "error": err}
        log(f"hydrostatic {shape}: first {hist[0] if hist else None}, last {hist[-1] if hist else None} {err or ''}")
    return out


def bump_history(steps, every):
    """2D water layer 2.0 x 0.5 m over a Gaussian bump (amplitude 0.1 m, sigma
    0.1 m), dx = 0.002 (243.7k fluid), hydrostatic start: fluid max |U| every
    `every` steps on the FP64 and the mixed path, with the printed scheme
    (no stabilisers) and with the tensile-instability switch on.  A run that
    blows up (the free-surface mode) stops at the first record above 1 m/s or
    on a device error, and reports it."""
    import workloads as wl
    from paper_2608_22269_amd import Simulation
    from paper_2608_22269_amd._lib import SphError
    out = {}
    for label, kw in (("literal", {}), ("tic", {"tic": True, "cont_uncorr": True})):
        for prec in ("fp64", "mixed"):
            case = wl.bump2d(precision=prec, **kw)
            f = case["kind"] == 0
            sim = Simulation(case)
            hist, err = [], None
            t0 = time.time()
            try:
                for k in range(0, steps, every):
                    sim.step(every)
                    u = sim.field("u")[f]
                    hist.append([k + every, float(np.sqrt((u * u).sum(1)).max())])
                    if hist[-1][1] > 1.0:  # the blow-up: later steps only clump particles
                        err = "stopped: max |U| above 1 m/s"
                        break
            except SphError as e:
                err = str(e)
            out[f"{label}/{prec}"] = {"max_u": hist, "error": err, "seconds": time.time() - t0,
                                      "n_fluid": int(f.sum())}
            log(f"bump2d {label}/{prec}: {hist[-1] if hist else None} {err or ''}")
            sim.close()
    return out


def moving_body(dx, steps, warmup):
    """3D tank with a box body cutting the free surface and moving along the
    paper's ditching velocity history (5 m/s along x): FP64 and mixed, and
    FP64 with the same body at rest (the difference is the cost of moving
    and re-sorting the dummies at every right-hand side)."""
    import workloads as wl
    case = wl.ditch3d(dx=dx)
    h = case["params"]["h"]
    case = wl.with_params(case, cell_size=h)
    at_rest = dict(case)
    at_rest["params"] = {k: v for k, v in case["params"].items() if not k.startswith("body_")}
    res = {"workload": case["meta"]["desc"], "n_fluid": case["meta"]["n_fluid"],
           "n_dummy": case["meta"]["n_dummy"], "n_body": case["meta"]["n_body"], "cell_size_over_h": 1.0}
    res["fp64"] = run_path(case, "ditch3d moving body (fp64)", steps, warmup)
    res["fp64_body_at_rest"] = run_path(at_rest, "ditch3d body at rest (fp64)", steps, warmup)
    res["mixed"] = run_path(wl.with_params(case, precision="mixed"), "ditch3d moving body (mixed)", steps, warmup)
    res["motion_cost_ms_per_step"] = res["fp64"]["ms_per_step"] - res["fp64_body_at_rest"]["ms_per_step"]
    return res


def cylinder_entry_run(dx, cell, steps, warmup):
    """The paper's cylinder water entry at its size (Sec. 4; dx = D/20 =
    0.0025: 15.36M fluid + 2.37M dummies): a free solid cylinder (D = 0.05 m,
    L = 0.2 m, density 1370) entering the water at 6.22 m/s, FP64 and mixed,
    its force, torque and state at every right-hand side.  The
    paper's figure for the same case (1000 steps in 270.31 s, FP32, one
    RTX 3090) is context, not a target of the same precision."""
    import workloads as wl
    case = wl.cylinder_entry(3, dx=dx)
    h = case["params"]["h"]
    case = wl.with_params(case, cell_size=cell * h)
    body0 = {k: list(map(float, v)) for k, v in case["body"].items()}

    def after(sim, out):
        st = sim.body_state()
        out["body_end"] = {k: [float(a) for a in v] for k, v in st.items()}

    res = {"workload": case["meta"]["desc"], "n_fluid": case["meta"]["n_fluid"],
           "n_dummy": case["meta"]["n_dummy"], "n_body": case["meta"]["n_body"], "cell_size_over_h": cell,
           "body_start": body0, "paper_ms_per_step": 270.31, "paper_particles": 17.53e6,
           "paper_note": "1000 steps in 270.31 s on one RTX 3090, FP32 (Sec. 5, efficiency table)"}
    res["fp64"] = run_path(case, "cylinder entry (fp64, free body)", steps, warmup, after=after)
    res["mixed"] = run_path(wl.with_params(case, precision="mixed"), "cylinder entry (mixed, free body)", steps,
                            warmup, after=after)
    res["fp32"] = run_path(wl.with_params(case, precision="fp32"), "cylinder entry (single precision, free body)",
                           steps, warmup, after=after)
    res["particles"] = res["n_fluid"] + res["n_dummy"]
    res["particle_steps_per_s"] = res["particles"] / (res["fp64"]["ms_per_step"] * 1e-3)
    return res


def dambreak_obstacle_run(dx, keep_cell, cell, steps, warmup):
    """The paper's 3D dam break against an obstacle at its size (Sec. 4:
    the obstacle 30 spacings wide, dx = 0.161/30; 4.34M fluid + 2.49M
    dummies with 3 wall layers), FP64 and mixed from the column at rest, in
    the headline's configuration (kept lists in cells of keep_cell h; cells
    of cell h and both right-hand sides searching when keep_cell is 0).  The
    paper's figure (1000 steps in 79.40 s, FP32, one RTX 3090, 7.59M
    particles with its dummies) is context, not a target of the same
    precision."""
    import workloads as wl
    case = wl.dambreak_obstacle3d(dx=dx)
    h = case["params"]["h"]
    case = (wl.with_params(case, cell_size=keep_cell * h, keep_lists=True) if keep_cell > 0
            else wl.with_params(case, cell_size=cell * h))
    res = {"workload": case["meta"]["desc"], "n_fluid": case["meta"]["n_fluid"],
           "n_dummy": case["meta"]["n_dummy"], "n_obstacle": case["meta"]["n_obstacle"],
           "cell_size_over_h": keep_cell if keep_cell > 0 else cell,
           "paper_ms_per_step": 79.40, "paper_particles": 7.59e6,
           "paper_note": "1000 steps in 79.40 s on one RTX 3090, FP32 (Sec. 5, efficiency table)"}
    res["fp64"] = run_path(case, "dam break + obstacle (fp64)", steps, warmup)
    res["mixed"] = run_path(wl.with_params(case, precision="mixed"), "dam break + obstacle (mixed)", steps, warmup)
    res["fp32"] = run_path(wl.with_params(case, precision="fp32"), "dam break + obstacle (single precision)", steps,
                           warmup)
    res["particles"] = res["n_fluid"] + res["n_dummy"]
    return res


def _sig(v, n=4):
    """v rounded to n significant digits (non-floats pass through; non-finite
    floats become strings so that the line stays strict JSON)."""
    if isinstance(v, float):
        if not math.isfinite(v):
            return str(v)
        return float(f"{v:.{n}g}")
    return v


def _short(s, n=90):
    return s if not isinstance(s, str) or len(s) <= n else s[:n - 3] + "..."


def _roof_summary(r, full=True):
    if r is None:
        return None
    out = {k: _sig(r.get(k)) for k in ("bound", "achieved", "peak", "unit", "frac", "traffic")}
    out["kernel"] = r["kernel"] if full else r["kernel"].split(" ")[0]
    out["launch_ms"] = _sig(r["pair_pass_ms"])
    out["pairs_per_launch"] = _sig(r["pairs_per_launch"])
    out["candidate_tests_per_launch"] = _sig(r["tests_per_launch"])
    if full:
        out["flop_per_pair"] = FLOP_PER_PAIR_3D
        out["tflops_with_tests"] = _sig(r["tflops_with_tests"])
    if "valu_issue" in r:
        out["valu_issue_frac"] = _sig(r["valu_issue"]["frac"], 3)
    if "ta_busy" in r:
        out["ta_busy_frac"] = _sig(r["ta_busy"]["frac"], 3)
    return out


def _path_summary(r):
    out = {"ms_per_step": _sig(r["ms_per_step"]), "pair_evals_per_s": _sig(r["pair_evals_per_s"]),
           "pair_pass_ms": _sig(r["pair_pass_ms"])}
    if "kept_pass" in r:
        out["kept_pass_ms"] = _sig(r["kept_pass"]["ms"])
    kms = r.get("kernel_ms_per_step", {})
    if "fs_detect" in kms:
        out["fs_detect_ms"] = _sig(kms["fs_detect"], 3)
    if "misclassification" in r:
        m = r["misclassification"]
        out["fs_candidates"] = m["candidates"]
        out["decided_by_mlp"] = m["decided_by_mlp"]
        out["misclassified"] = m["misclassified"]
        out["misclassified_frac"] = _sig(m["rate_of_candidates"], 3)
    return out


def compact_line(d):
    """The one JSON line bench.py prints: the headline with its roofline and
    CPU baseline, then one short summary per path and per side measurement.
    The full record (histories, probe traces, per-kernel times) goes to the
    detail file named in the line."""
    head = d["paths"]["fp64"]
    line = {
        "metric": METRIC, "value": _sig(head["pair_evals_per_s"]), "unit": "pair-evals/s", "n_gpus": 1,
        "steps": d["steps"], "warmup": d["warmup"], "ms_per_step": _sig(head["ms_per_step"]),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": d["data"], "config": d["config"], "roofline": _roof_summary(d["roofline"]),
    }
    if d.get("cpu_baseline"):
        c = d["cpu_baseline"]
        line["cpu_baseline"] = {"value": _sig(c["value"]), "unit": c["unit"], "cores": c["cores"], "kind": c["kind"],
                                "sample": c["sample_short"], "cpu_model": c["cpu_model"],
                                "single_core_value": _sig(c["single_core"]["value"])}
    line["paths"] = {k: _path_summary(v) for k, v in d["paths"].items()}
    p = d["paths"]
    ratios = {}
    for k in ("mixed", "mixed_learned", "fp32"):
        if k in p:
            ratios[f"{k}_over_fp64"] = _sig(p["fp64"]["ms_per_step"] / p[k]["ms_per_step"], 3)
    if "mixed" in p and "mixed_learned" in p:
        ratios["mixed_learned_over_mixed"] = _sig(p["mixed"]["ms_per_step"] / p["mixed_learned"]["ms_per_step"], 3)
    line["step_rate_ratios"] = ratios
    if d.get("at_rest"):
        line["at_rest_ms_per_step"] = {k: _sig(v["ms_per_step"]) for k, v in d["at_rest"].items()}
    if d.get("roofline_kept"):
        line["roofline_kept_pass"] = _roof_summary(d["roofline_kept"], full=False)
    if d.get("spurious_u_tank2d"):
        line["spurious_u_tank2d_max"] = {k: {s: _sig(u, 2) for s, u in v.items() if s in ("100", "200")}
                                         for k, v in d["spurious_u_tank2d"].items()}
    if d.get("hydrostatic_l2_paper_cases"):
        hs = {}
        for shape, r in d["hydrostatic_l2_paper_cases"].items():
            if shape.startswith("_"):
                continue
            hist = r["step_t_l2_maxu"]
            below = [s for s, _, l2, _ in hist if l2 <= 1e-12]
            at = {int(s): _sig(l2, 2) for s, _, l2, _ in hist if int(s) in (100, 200)}
            hs[shape] = {"l2_at": at, "last_step_below_1e-12": max(below) if below else 0}
        hs["constants"] = d["hydrostatic_l2_paper_cases"].get("_constants")
        line["hydrostatic_paper_cases"] = hs
    if d.get("spurious_u_bump2d"):
        line["bump2d_last_step_max_u"] = {k: [v["max_u"][-1][0], _sig(v["max_u"][-1][1], 2)] if v["max_u"] else None
                                          for k, v in d["spurious_u_bump2d"].items()}
    if d.get("keep_across_steps"):
        k = d["keep_across_steps"]
        line["keep_across_steps_ms_per_step"] = {n: _sig(k[n]["ms_per_step"]) for n in
                                                 ("from_rest", "moving", "moving_within_step") if n in k}
    if d.get("moving_body"):
        b = d["moving_body"]
        line["moving_body"] = {"n_fluid": b["n_fluid"], "fp64_ms_per_step": _sig(b["fp64"]["ms_per_step"]),
                               "mixed_ms_per_step": _sig(b["mixed"]["ms_per_step"]),
                               "motion_cost_ms_per_step": _sig(b["motion_cost_ms_per_step"], 3)}
    if d.get("cylinder_entry"):
        c = d["cylinder_entry"]
        line["cylinder_entry"] = {"n": c["particles"], "fp64_ms": _sig(c["fp64"]["ms_per_step"]),
                                  "mixed_ms": _sig(c["mixed"]["ms_per_step"]) if "mixed" in c else None,
                                  "fp32_ms": _sig(c["fp32"]["ms_per_step"]) if "fp32" in c else None,
                                  "paper_ms_fp32_3090": c["paper_ms_per_step"],
                                  "vz_end": _sig(c["fp64"].get("body_end", {}).get("v", [0, 0, 0])[2], 4)}
    if d.get("dambreak_obstacle"):
        c = d["dambreak_obstacle"]
        line["dambreak_obstacle"] = {"n": c["particles"], "fp64_ms": _sig(c["fp64"]["ms_per_step"]),
                                     "mixed_ms": _sig(c["mixed"]["ms_per_step"]),
                                     "fp32_ms": _sig(c["fp32"]["ms_per_step"]) if "fp32" in c else None,
                                     "paper_ms_fp32_3090": c["paper_ms_per_step"]}
    if d.get("mlp_inference_17_5M"):
        m = d["mlp_inference_17_5M"]
        line["mlp_inference"] = {"rows": m["rows"], "ms_per_call": _sig(m["ms_per_call"]),
                                 "hbm_frac": _sig(m["hbm_frac"], 3)}
    if d.get("slosh_after_spinup"):
        r = d["slosh_after_spinup"]
        line["slosh_after_spinup_ms"] = {"fp64": _sig(r["fp64"]["ms_per_step"]),
                                         "mixed_learned": _sig(r["mixed_learned"]["ms_per_step"]),
                                         "wrong": r["mixed_learned"]["misclassification"]["misclassified"]}
    if d.get("cylinder_detection"):
        r = d["cylinder_detection"]
        m = r["learned"]["misclassification"]
        line["cylinder_heldout_detection"] = {"cand": m["candidates"], "wrong": m["misclassified"],
                                              "ms": [_sig(r["exact"]["ms_per_step"]), _sig(r["learned"]["ms_per_step"])]}
    if d.get("dambreak_detection"):
        r = d["dambreak_detection"]
        ln = r["learned"]
        line["dambreak_heldout_detection"] = {
            "exact_ms_per_step": _sig(r["exact"]["ms_per_step"]), "learned_ms_per_step": _sig(ln["ms_per_step"]),
            "candidates": ln["misclassification"]["candidates"],
            "misclassified": ln["misclassification"]["misclassified"]}
    if d.get("slosh_surface_detection"):
        m = d["slosh_surface_detection"]
        line["slosh_moved_surface_detection"] = {"candidates": m["candidates"], "misclassified": m["misclassified"],
                                                 "fallback_exact": m["fallback_exact"]}
    if d.get("dambreak_wall_pressure"):
        r = d["dambreak_wall_pressure"]
        line["dambreak_wall_pressure"] = {"t_end": _sig(r["t"][-1], 3) if r["t"] else None,
                                          "rms_diff_over_max_p": [_sig(v, 2) for v in r["rms_diff_over_max_p"]],
                                          "stopped": {k: _short(v, 60) for k, v in r["stopped"].items()}}
    line["detail"] = d.get("detail_path")
    return line


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dx", type=float, default=0.002)
    ap.add_argument("--cell", type=float, default=1.0,
                    help="background cell size in units of h (the paper's R = 2h is 2.0; R = h visits fewer "
                         "candidates for the same neighbour sets)")
    ap.add_argument("--keep-cell", type=float, default=1.01,
                    help="cell size in units of h when the first stage's candidate lists serve the second (room "
                         "for a skin of (2 x keep-cell - 2) h); 0: no kept lists, cells of --cell h")
    ap.add_argument("--state", choices=("moving", "rest"), default="moving",
                    help="state the paths are timed on: 'moving' = the lattice jittered by N(0, (0.05 dx)^2) "
                         "with seeded velocities N(0, 0.05^2) m/s per component (irregular neighbour lists, "
                         "particles moving through the lists' skin); 'rest' = the hydrostatic lattice")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-at-rest", action="store_true", help="skip the FP64 and learned runs at rest")
    ap.add_argument("--no-across-steps", action="store_true",
                    help="skip the runs with the candidate lists kept across steps")
    ap.add_argument("--across-cell", type=float, default=1.03,
                    help="cell size in units of h of the runs with the lists kept across steps (more room: longer "
                         "lived lists, slightly more candidates)")
    ap.add_argument("--paths", default="fp64,mixed,mixed_learned,fp32",
                    help="fp64: FP64 path, exact detection; mixed: mixed precision, exact detection; "
                         "mixed_learned: mixed precision with the trained classifier and exact fallback; "
                         "fp32: the single-precision form")
    ap.add_argument("--spinup-steps", type=int, default=0,
                    help="forced steps of the sloshing tank before a second timing of fp64 and mixed + learned "
                         "from that state (16760 reach T_f/4 at dx = 0.002; 0: skip; several minutes)")
    ap.add_argument("--spinup-timed", type=int, default=200, help="timed steps after the spin-up (50 warm-up)")
    ap.add_argument("--cylinder-detect-spin", type=int, default=1000,
                    help="steps of the cylinder entry before exact and learned detection are compared on its state "
                         "(0: skip)")
    ap.add_argument("--dambreak-spin", type=int, default=5000,
                    help="steps of the held-out 3D dam break before the exact / learned detection comparison "
                         "(0: skip)")
    ap.add_argument("--surface-steps", type=int, default=200,
                    help="steps of the full-size tank with a moved (cosine) surface before the learned "
                         "detector's misclassification is taken (0: skip)")
    ap.add_argument("--probe-seconds", type=float, default=0.7,
                    help="simulated seconds of the 3D dam-break wall-pressure comparison, FP64 vs mixed (0: skip)")
    ap.add_argument("--hydro-steps", type=int, default=1000,
                    help="steps of the paper's three hydrostatic cases (L2 velocity error; 0: skip)")
    ap.add_argument("--tank-steps", type=int, default=200,
                    help="steps of the 2D hydrostatic tank's spurious-velocity check (0: skip)")
    ap.add_argument("--bump-steps", type=int, default=10000,
                    help="steps of the 2D Gaussian-bump spurious-velocity history (0: skip)")
    ap.add_argument("--body-dx", type=float, default=0.005,
                    help="particle spacing of the 3D moving-body run (3.82M fluid at 0.005; 0: skip)")
    ap.add_argument("--cylinder-dx", type=float, default=0.0025,
                    help="particle spacing of the cylinder water entry (the paper's D/20: 17.7M particles; 0: skip)")
    ap.add_argument("--obstacle-dx", type=float, default=0.161 / 30,
                    help="particle spacing of the dam break against an obstacle (the paper's 0.161/30: "
                         "6.84M particles; 0: skip)")
    ap.add_argument("--mlp", action=argparse.BooleanOptionalAction, default=True,
                    help="standalone BF16 MLP inference over as many rows as the tank has fluid particles")
    ap.add_argument("--calib", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--detail", default="bench_detail.json",
                    help="file that receives the full record (histories, traces, per-kernel times)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (slab decomposition is designed, "
              "not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    log(f"device {torch.cuda.get_device_name(0)}")
    log("generating workload")
    case = wl.slosh3d(dx=args.dx)
    h = case["params"]["h"]
    case = wl.with_params(case, cell_size=args.cell * h)
    if args.calib:
        src_t = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst_t = torch.empty_like(src_t)
        dst_t.copy_(src_t)
        torch.cuda.synchronize()
        log("calibration copy: 1 GiB read + 1 GiB written")
        del src_t, dst_t
    # every path keeps the first stage's candidate lists for the second (cells
    # of keep_cell h, room for the skin) unless --keep-cell 0
    rest_case = case if args.keep_cell <= 0 else wl.with_params(case, cell_size=args.keep_cell * h, keep_lists=True)
    run_case = rest_case
    if args.state == "moving":
        run_case = wl.random_velocity(wl.jitter(rest_case, 0.05, seed=11), 0.05, seed=12)
    state_desc = ("lattice jittered 0.05 dx, velocities 0.05 m/s rms per axis (seeded)"
                  if args.state == "moving" else "hydrostatic lattice at rest")
    d = {"steps": args.steps, "warmup": args.warmup, "paths": {}}
    clf = load_classifier()
    for path in args.paths.split(","):
        if path == "fp64":
            d["paths"]["fp64"] = run_path(run_case, "fp64", args.steps, args.warmup)
        elif path == "mixed":
            d["paths"]["mixed"] = run_path(wl.with_params(run_case, precision="mixed"), "mixed", args.steps,
                                           args.warmup)
        elif path == "fp32":
            d["paths"]["fp32"] = run_path(wl.with_params(run_case, precision="fp32"), "fp32", args.steps, args.warmup)
        elif path == "mixed_learned":
            d["paths"]["mixed_learned"] = run_path(wl.with_params(run_case, precision="mixed", fs_mode="learned"),
                                                   "mixed_learned", args.steps, args.warmup, clf=clf)
        else:
            raise SystemExit(f"unknown path {path}")
    head = d["paths"]["fp64"]
    if args.state == "moving" and not args.no_at_rest:
        d["at_rest"] = {"fp64": run_path(rest_case, "fp64 at rest", args.steps, args.warmup),
                        "mixed_learned": run_path(wl.with_params(rest_case, precision="mixed", fs_mode="learned"),
                                                  "mixed_learned at rest", args.steps, args.warmup, clf=clf)}

    def roofline(res, key, kernel, kept=False):
        src = PAIR_SOURCES[key]
        prof = profile_summary(f"{key}_slosh3d")
        if kept:  # the second stage's pass from the kept lists
            k = res["kept_pass"]
            ms, pairs, tests = k["ms"], k["pairs"], k["kept_candidates_tested"]
        else:
            ms, pairs, tests = res["pair_pass_ms"], res["pairs_per_rhs"], res["candidate_tests_per_rhs"]
        # the method's work only: FLOP of the in-range pairs; the candidate
        # distance tests of the search are reported beside it
        achieved = pairs * FLOP_PER_PAIR_3D / (ms * 1e-3) / 1e12
        out = {
            "bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": prof["hbm_bytes_per_launch"] if prof else None,
            "kernel": kernel, "pair_pass_ms": ms, "pairs_per_launch": pairs, "tests_per_launch": tests,
            "tflops_with_tests": (pairs * FLOP_PER_PAIR_3D + tests * FLOP_PER_TEST_3D) / (ms * 1e-3) / 1e12,
            "source_sha": source_sha(src),
        }
        if prof and "valu_issue_frac" in prof:
            # VALU instruction issue (counted by the SQ)
            out["valu_issue"] = {"frac": prof["valu_issue_frac"], "lane_instr_per_s": prof["valu_lane_instr_per_s"],
                                 "peak": prof["valu_issue_peak"], "from": f"profiles/{key}_slosh3d_pmc.json"}
        if prof and "ta_busy_frac" in prof:
            # the texture addresser (vector memory address unit): the record gathers
            out["ta_busy"] = {"frac": prof["ta_busy_frac"], "from": f"profiles/{key}_slosh3d_pmc.json"}
        return out

    d["roofline"] = roofline(head, "pair_f64", "k_pair_f64<3,true,true> (first-stage search + pair pass)")
    d["data"] = f"synthetic: seeded lattice tank, tank-frame forcing; timed state: {state_desc}"
    d["config"] = {"workload": (f"3D sloshing tank 1.0x0.5x0.56 m, depth 0.28 m, dx={args.dx}: "
                                f"{case['meta']['n_fluid']} fluid + {case['meta']['n_dummy']} dummies"),
                   "path": "fp64", "fs_mode": "exact", "state": args.state,
                   "cell_size_over_h": args.keep_cell if args.keep_cell > 0 else args.cell,
                   "second_stage": "kept candidate lists" if args.keep_cell > 0 else "rebuild and search",
                   "parallelism": "single GPU"}
    if "kept_pass" in head:
        d["roofline_kept"] = roofline(head, "pair_kept_f64", "k_pair_kept_f64<3,true> (second stage, kept "
                                      "lists)", kept=True)
    if "mixed" in d["paths"]:
        # non-packed FP32 issues at the FP64 rate on this chip: same peak
        d["roofline_mixed"] = roofline(d["paths"]["mixed"], "pair_mixed",
                                       "k_pair_mixed<3,true,true,false> (first-stage pass, FP32 body + FP64 sums)")
        if "kept_pass" in d["paths"]["mixed"]:
            d["roofline_kept_mixed"] = roofline(d["paths"]["mixed"], "pair_kept_mixed",
                                                "k_pair_kept_mixed<3,true,false> (second stage from the kept "
                                                "lists)", kept=True)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(args.dx)
        cb["cpu_model"] = cpu_model()
        d["cpu_baseline"] = cb
    if args.keep_cell > 0 and not args.no_across_steps:
        # the lists kept across steps as well (SPH_F_KEEP_ACROSS_STEPS): from
        # the lattice near rest (one build serves many steps) and from a
        # moving state (seeded random velocities, |U| up to about 0.3 m/s),
        # where the bound on the particles' moves runs out sooner
        xs = wl.with_params(case, cell_size=args.across_cell * h, keep_lists=True, keep_across_steps=True)
        moving = wl.random_velocity(xs, 0.05, 21)
        d["keep_across_steps"] = {
            "cell_size_over_h": args.across_cell,
            "from_rest": run_path(xs, "fp64 across steps (near rest)", args.steps, args.warmup),
            "moving": run_path(moving, "fp64 across steps (moving, |U| <= ~0.3 m/s)", args.steps, args.warmup),
            "moving_within_step": run_path(wl.with_params(moving, keep_across_steps=False),
                                           "fp64 within steps (moving)", args.steps, args.warmup),
        }
    if args.body_dx > 0:
        d["moving_body"] = moving_body(args.body_dx, args.steps, args.warmup)
    if args.cylinder_dx > 0:
        d["cylinder_entry"] = cylinder_entry_run(args.cylinder_dx, args.cell, args.steps, args.warmup)
    if args.obstacle_dx > 0:
        d["dambreak_obstacle"] = dambreak_obstacle_run(args.obstacle_dx, args.keep_cell, args.cell, args.steps,
                                                       args.warmup)
    if args.mlp:
        d["mlp_inference_17_5M"] = mlp_inference(case["meta"]["n_fluid"])
    if args.dambreak_spin > 0:
        d["dambreak_detection"] = dambreak_detection(args.dambreak_spin, 20)
    if args.spinup_steps > 0:
        d["slosh_after_spinup"] = sloshing_after_spinup(args.dx, args.keep_cell, args.spinup_steps,
                                                        args.spinup_timed, 50)
    if args.cylinder_detect_spin > 0 and args.cylinder_dx > 0:
        d["cylinder_detection"] = cylinder_detection(args.cylinder_dx, args.cylinder_detect_spin, 20)
    if args.surface_steps > 0:
        d["slosh_surface_detection"] = slosh_surface_detection(args.dx, args.surface_steps)
    if args.probe_seconds > 0:
        d["dambreak_wall_pressure"] = dambreak_probes(args.probe_seconds)
    if args.tank_steps > 0:
        d["spurious_u_tank2d"] = {k: spurious_velocity(k, args.tank_steps) for k in ("fp64", "mixed", "fp32")}
    if args.bump_steps > 0:
        d["spurious_u_bump2d"] = bump_history(args.bump_steps, 500)
    if args.hydro_steps > 0:
        d["hydrostatic_l2_paper_cases"] = hydrostatic_l2(args.hydro_steps, 50)
    d["detail_path"] = args.detail
    try:
        os.makedirs(os.path.dirname(os.path.abspath(args.detail)), exist_ok=True)
        with open(args.detail, "w") as f:
            json.dump(d, f)
    except OSError as e:
        log(f"detail file not written: {e}")
        d["detail_path"] = None
    print(json.dumps(compact_line(d), separators=(",", ":")), flush=True)


if __name__ == "__main__":
    main()
