"""The bench's stdout line: one compact JSON object with the headline, the
roofline of the dominant kernel and the CPU baseline, however long the side
measurements' histories are (they go to the detail file).  CPU only: the line
is built from stub results."""
import json

import bench


def _path(ms, learned=False):
    r = {"ms_per_step": ms, "pair_evals_per_s": 2.79e9 / (ms * 1e-3), "pair_pass_ms": 0.55 * ms,
         "pairs_per_rhs": 1.395e9, "candidate_tests_per_rhs": 3.28e9,
         "kept_pass": {"ms": 0.3 * ms, "pairs": 1.395e9, "kept_candidates_tested": 1.40e9},
         "kernel_ms_per_step": {"pair": 15.6, "mirror": 0.5, "rebuild": 1.1, "fs_detect": 0.45, "stage": 1.8,
                                "pair_kept": 8.3}}
    if learned:
        r["misclassification"] = {"fluid": 17500000, "candidates": 131072, "decided_by_mlp": 130000,
                                  "fallback_exact": 1072, "misclassified": 3, "rate_of_fluid": 1.7e-7,
                                  "rate_of_candidates": 2.3e-5, "fs_exact": 125000, "fs_learned": 125002}
    return r


def _roof(ms):
    return {"bound": "alu", "achieved": 8.5, "peak": 78.6, "unit": "TFLOP/s", "frac": 0.108, "traffic": 1.68e10,
            "kernel": "k_pair_f64<3,true,true> (first-stage search + pair pass)",
            "pair_pass_ms": ms, "pairs_per_launch": 1.395e9, "tests_per_launch": 3.28e9, "tflops_with_tests": 10.2,
            "source_sha": "0123456789abcdef", "valu_issue": {"frac": 0.54}, "ta_busy": {"frac": 0.68}}


def stub_detail():
    long_hist = [[k, 1e-17 * 1.1 ** (k / 50)] for k in range(0, 10000, 50)]
    paper = {s: {"n_fluid": 9000, "step_t_l2_maxu": [[k, k * 1e-4, 1e-17 * 1.3 ** (k / 10), 1e-16 * 1.3 ** (k / 10)]
                                                       for k in range(50, 1001, 50)], "error": None}
             for s in ("rect", "tri", "gauss")}
    paper["_constants"] = {"c0": 30.0, "h_over_dx": 1.5, "dx": 0.01}
    return {
        "steps": 20, "warmup": 5,
        "paths": {"fp64": _path(27.9), "mixed": _path(25.4), "mixed_learned": _path(25.9, True), "fp32": _path(24.5)},
        "at_rest": {"fp64": _path(27.0), "mixed_learned": _path(25.0, True)},
        "roofline": _roof(15.6), "roofline_kept": _roof(8.3), "roofline_mixed": _roof(13.4),
        "data": "synthetic: seeded lattice tank, tank-frame forcing; timed state: lattice jittered by 0.05 dx, "
                "velocities 0.05 m/s rms per component (seeded)",
        "config": {"workload": "3D sloshing tank 1.0x0.5x0.56 m, depth 0.28 m, dx=0.002: 17500000 fluid + 2047296 "
                               "dummies", "path": "fp64", "fs_mode": "exact", "state": "moving",
                   "cell_size_over_h": 1.01, "second_stage": "kept candidate lists", "parallelism": "single GPU"},
        "cpu_baseline": {"value": 3.7e7, "unit": "pair-evals/s", "cores": 16, "kind": "oracle",
                         "sample": "x" * 400, "sample_short": "1 RHS of a 0.2x0.1x0.56 m column of the tank, 700000 "
                                                             "fluid, 12.3 s",
                         "cpu_model": "AMD EPYC 9575F 64-Core Processor", "single_core": {"value": 1.26e7}},
        "keep_across_steps": {"from_rest": _path(19.5), "moving": _path(22.1), "moving_within_step": _path(28.8)},
        "moving_body": {"n_fluid": 3820800, "fp64": _path(8.0), "mixed": _path(6.8), "motion_cost_ms_per_step": 0.24},
        "mlp_inference_17_5M": {"rows": 17500000, "ms_per_call": 1.52, "hbm_frac": 0.098},
        "cylinder_detection": {"exact": {"ms_per_step": 29.5}, "learned": {"ms_per_step": 29.2, "misclassification": {
            "candidates": 93000, "misclassified": 12}}},
        "cylinder_entry": {"particles": 17728988, "paper_ms_per_step": 270.31,
                           "fp64": dict(_path(31.5), body_end={"v": [1e-17, -2e-17, -6.2134567]}),
                           "mixed": _path(29.5), "fp32": _path(27.1)},
        "dambreak_obstacle": {"particles": 6837984, "paper_ms_per_step": 79.40, "fp64": _path(11.3),
                              "mixed": _path(10.4), "fp32": _path(9.9)},
        "dambreak_detection": {"exact": {"ms_per_step": 2.13}, "learned": {"ms_per_step": 2.08,
                                                                          "misclassification": {"candidates": 21683,
                                                                                                "misclassified": 15}}},
        "slosh_surface_detection": {"candidates": 412000, "misclassified": 17, "fallback_exact": 9000},
        "dambreak_wall_pressure": {"t": [k * 0.01 for k in range(70)], "p_fp64": [[1.0] * 4] * 70,
                                   "rms_diff_over_max_p": [0.1, 0.2, 0.26, 0.15], "stopped": {}},
        "spurious_u_tank2d": {p: {str(k): 1e-14 * 1.5 ** (k / 50) for k in range(50, 201, 50)}
                              for p in ("fp64", "mixed", "fp32")},
        "spurious_u_bump2d": {f"{a}/{b}": {"max_u": long_hist, "error": None} for a in ("literal", "tic")
                              for b in ("fp64", "mixed")},
        "hydrostatic_l2_paper_cases": paper,
        "detail_path": "bench_detail.json",
    }


def test_line_is_compact_and_complete():
    line = bench.compact_line(stub_detail())
    text = json.dumps(line, separators=(",", ":"))  # as bench.py prints it
    assert len(text) < 3900, len(text)  # a reader that keeps only the tail of stdout still holds all of it
    back = json.loads(text)
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better", "scaling",
              "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in back, k
    assert "workload" in back["config"]
    for k in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert k in back["roofline"], k
    assert abs(back["roofline"]["frac"] - back["roofline"]["achieved"] / back["roofline"]["peak"]) < 1e-2
    for k in ("value", "unit", "cores", "kind", "sample"):
        assert k in back["cpu_baseline"], k
    assert back["cpu_baseline"]["kind"] == "oracle"
    r = back["step_rate_ratios"]
    assert {"mixed_over_fp64", "mixed_learned_over_fp64", "mixed_learned_over_mixed", "fp32_over_fp64"} <= set(r)
    assert back["paths"]["mixed_learned"]["misclassified"] == 3
    assert back["value"] == bench._sig(2.79e9 / 27.9e-3)


def test_line_without_side_measurements():
    d = stub_detail()
    for k in ("at_rest", "keep_across_steps", "moving_body", "cylinder_entry", "cylinder_detection", "dambreak_obstacle",
              "mlp_inference_17_5M", "dambreak_detection",
              "slosh_surface_detection",
              "dambreak_wall_pressure", "spurious_u_tank2d", "spurious_u_bump2d", "hydrostatic_l2_paper_cases",
              "cpu_baseline", "roofline_kept"):
        d.pop(k)
    d["paths"] = {"fp64": d["paths"]["fp64"]}
    line = json.loads(json.dumps(bench.compact_line(d)))
    assert line["value"] > 0 and "roofline" in line and "cpu_baseline" not in line


def test_nonfinite_values_stay_strict_json():
    assert bench._sig(float("inf")) == "inf"
    json.loads(json.dumps(bench._sig(float("nan"))))
