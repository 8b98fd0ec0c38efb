#!/usr/bin/env python
"""Benchmark: one full forward + backward pass of the SBR radar simulator per
step on one MI355X, on a seeded synthetic scene.

Step = BVH build, trace (ray launch, traversal, multi-bounce), FP64 path
refinement + IF synthesis (Eq. 8), radar cube (Eq. 16's T), CA-CFAR points,
IF-loss gradient, backward (synthesis adjoint, Eqs. 11-12, and geometry
adjoint to the vertices, Eq. 13).  Inputs are resident in device memory before
the timed region.

Prints one JSON line.  `--gpus N` with N > 1 exits: the library runs on one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak
PEAK_HBM_GBS = 8000.0
# LDS bandwidth from the unit counts: 256 CUs x 128 B per clock x 2.4 GHz
PEAK_LDS_GBS = 256 * 128 * 2.4
# the spreading of the non-uniform FFT synthesis: 7 taps, each one 64-bit LDS
# atomic add of the packed (re, im) pair, per (path, antenna, chirp)
LDS_BYTES_PER_PAC = 7 * 8
# the tap kernel of the non-uniform FFT adjoint: 7 float4 row reads from LDS
# per (path, antenna, chirp)
LDS_READ_BYTES_PER_PAC = 7 * 16
FLOP_PER_PATH_SAMPLE = {"synth": 8.0, "synth_adj": 20.0}
# lane operations per second of the FP32 vector units: 256 CUs x 4 SIMDs x 32
# lanes x 2.4 GHz (one VALU instruction per lane per clock; an FMA counts once)
PEAK_VALU_LANE_OPS = 256 * 4 * 32 * 2.4e9
# algorithmic VALU operations of the trace: a slab test of a node box, a
# watertight ray-triangle test
OPS_PER_NODE_TEST, OPS_PER_TRI_TEST = 14, 27


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic__k_nu_spread__clutter_50k_fwd_bwd.md")
KERNEL_SOURCES = {
    "k_nu_spread": ["synth.hip", "sbr_internal.h", "sbr_device.h", "nu_weights.h"],
    "k_synth_adj_nu": ["backward.hip", "sbr_internal.h", "sbr_device.h", "nu_weights.h"],
    "k_synth_adj": ["backward.hip", "sbr_internal.h", "sbr_device.h"],
    "k_synth_mfma": ["synth.hip", "sbr_internal.h", "sbr_device.h"],
    "k_synth": ["synth.hip", "sbr_internal.h", "sbr_device.h"],
}


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed rocprofv3 counter runs (FETCH_SIZE
    + WRITE_SIZE, calibrated against a plain copy), or None when the kernel's
    sources changed since the counters were taken or the workload differs."""
    import hashlib
    if workload != "clutter_50k" or not os.path.exists(TRAFFIC_FILE):
        return None
    kv = {}
    for line in open(TRAFFIC_FILE):
        if line.startswith(kernel + ".") and "=" in line:
            k, v = line.split("=", 1)
            kv[k.strip().split(".", 1)[1]] = v.strip()
    src = b"".join(open(os.path.join(ROOT, "paper_2311_13182_amd", "csrc", f), "rb").read()
                   for f in KERNEL_SOURCES[kernel])
    if kv.get("source_sha1") != hashlib.sha1(src).hexdigest():
        return None
    return float(kv["traffic_bytes"])


LDS_RATE_FILE = os.path.join(ROOT, "profiles", "lds_rate__probe_512x1024.md")


def measured_lds_atomic_peak():
    """LDS bandwidth of 64-bit atomic adds at conflict-free addresses, in GB/s at
    2.4 GHz on 256 CUs (the basis of the nominal LDS peak): the rate the
    committed LDS probe summary gives for "ds_add_u64 linear", in lanes per clock
    per CU times 8 bytes; None when the summary is missing."""
    import re
    if not os.path.exists(LDS_RATE_FILE):
        return None
    for line in open(LDS_RATE_FILE):
        if line.startswith("ds_add_u64 linear"):
            m = re.search(r"([0-9.]+) lanes/clk/CU", line)
            if m:
                return float(m.group(1)) * 8 * 256 * 2.4
    return None


def make_workload(name: str):
    from paper_2311_13182_amd import scenes as S
    if name == "clutter_50k":
        return S.clutter_scene()
    if name == "icosphere_20k":
        return S.icosphere_scene()
    if name == "imaging_400":
        return S.imaging_scene()
    raise SystemExit(f"unknown workload {name}")


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline(scene, queries_full: int, budget_rows: int = 8, chirp_stride: int = 16):
    """The FP64 oracle (trace + paths + synthesis + synthesis adjoint) on a
    bounded sample: every `budget_rows`-th ray row and column, every
    `chirp_stride`-th chirp; scaled linearly to the full workload.  Also its
    brute-force ray-triangle tests/s and FP64 path-samples/s (Eq. 8 terms)."""
    import numpy as np
    from oracle import pyoracle as orc
    g = scene.grid
    sub = np.arange(budget_rows // 2, g.nx, budget_rows)
    rows = np.arange(budget_rows // 2, g.ny, budget_rows)
    rays = (rows[:, None] * g.nx + sub[None, :]).reshape(-1).astype(np.int32)
    Cs = max(1, scene.chirp.n_chirps // chirp_stride)
    sc_s = scene.with_chirp(n_chirps=Cs)
    t0 = time.perf_counter()
    tr = orc.trace(scene, rays=rays)
    t1 = time.perf_counter()
    p = orc.paths(sc_s, tr["tri"], tr["flags"], rays=rays)
    cube = orc.synth(sc_s, p)
    t2 = time.perf_counter()
    G = np.random.default_rng(0).normal(size=cube.shape) + 1j * np.random.default_rng(1).normal(size=cube.shape)
    orc.synth_adjoint(sc_s, p, G)
    t3 = time.perf_counter()
    fr = g.n_rays / len(rays)
    fc = scene.chirp.n_chirps / Cs
    est = (t1 - t0) * fr + (t3 - t1) * fr * fc
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    Vs, Ss = scene.radar.n_virtual, scene.chirp.n_samples
    return {
        "value": queries_full / est,
        "unit": "ray-bounces/s",
        "cores": threads,
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "tests_per_s": tr["queries"] * scene.nf / (t1 - t0),
        "fp64_path_samples_per_s": len(p["amp"]) * Vs * Cs * Ss / (t2 - t1),
        "sample": (f"{len(rays)} of {g.n_rays} rays (every {budget_rows}th row/col), {Cs} of "
                   f"{scene.chirp.n_chirps} chirps, {len(p['amp'])} paths; measured {t3 - t0:.1f} s "
                   f"(trace {t1 - t0:.1f} s, synth {t2 - t1:.1f} s, adjoint {t3 - t2:.1f} s); "
                   f"full fwd+bwd time extrapolated linearly in rays and chirps: {est:.0f} s"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="clutter_50k", choices=["clutter_50k", "icosphere_20k", "imaging_400"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true", help="skip the request-latency measurement")
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run one plain 256 MiB device copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the library runs on one GPU only (the ray-sharded multi-GPU split is a design "
              "note, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2311_13182_amd import _lib
    from paper_2311_13182_amd import scenes as S
    from paper_2311_13182_amd.sbr import Simulator, sbr_profile, sbr_profile_read

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    _lib.load()
    dev = torch.device("cuda:0")
    scene = make_workload(args.workload)
    g, ch, rd = scene.grid, scene.chirp, scene.radar
    V, C, Sn = rd.n_virtual, ch.n_chirps, ch.n_samples

    # target IF cube of the same scene with 2 mm vertex jitter (untimed)
    tsim = Simulator(S.jitter(scene, 2e-3, 33), dev)
    target = tsim.forward().clone()
    del tsim
    torch.cuda.empty_cache()

    sim = Simulator(scene, dev)
    cube = torch.empty((V, C, Sn, 2), dtype=torch.float32, device=dev)
    grad = torch.empty_like(cube)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    gv = torch.empty((sim.mesh.nv, 3), dtype=torch.float32, device=dev)

    def step():
        sim.build()
        sim.trace()
        sim.synth(cube)
        X = sim.radar_cube(cube)
        sim.cfar(X, max_points=4096)
        sim.loss_grad(cube, target, grad, loss)
        gv.zero_()
        # the backward pass takes the path records of this step's synthesis
        # from the scratch (same mesh, hits and radar) instead of recomputing them
        sim.backward(grad, gv, reuse_paths=True)

    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    # path and query counts of this scene (counted on the device)
    sim.build()
    sim.counters.zero_()
    sim.trace(count=True)
    sim.synth(cube)
    torch.cuda.synchronize()
    n_paths = sim.n_paths()
    cnt = sim.counters.cpu().numpy()
    queries, node_tests, tri_tests = int(cnt[0]), int(cnt[1]), int(cnt[2])
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sbr_profile(2)
    sbr_profile(1)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev[0].record()
    for i in range(args.steps):
        step()
        ev[i + 1].record()
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    e0, e1 = ev[0], ev[-1]
    per_step = np.array([ev[i].elapsed_time(ev[i + 1]) for i in range(args.steps)])
    sbr_profile(0)
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / args.steps
    k_ms = {}
    for name, kid in (("synth", _lib.PROF_SYNTH), ("synth_adj", _lib.PROF_SYNTH_ADJ), ("trace", _lib.PROF_TRACE),
                      ("nu_spread", _lib.PROF_NU_SPREAD), ("nu_taps", _lib.PROF_NU_TAPS)):
        tot, n = sbr_profile_read(kid)
        k_ms[name] = tot / max(n, 1)
    ps = float(n_paths) * V * C * Sn          # path-samples per launch
    pac = float(n_paths) * V * C              # (path, antenna, chirp) per launch
    nufft = 16 <= Sn <= 1024                  # both sums run as non-uniform FFTs
    if nufft:
        # the spreading kernel of the synthesis, bound by its 64-bit LDS atomics:
        # their operand bytes against the LDS bandwidth of the unit counts
        achieved = LDS_BYTES_PER_PAC * pac / (k_ms["nu_spread"] * 1e-3) / 1e9
        roof = {"bound": "lds", "kernel": "k_nu_spread", "achieved": round(achieved, 1), "peak": PEAK_LDS_GBS,
                "unit": "GB/s", "frac": round(achieved / PEAK_LDS_GBS, 4),
                "traffic": measured_traffic("k_nu_spread", args.workload)}
        # beside it, the rate 64-bit LDS atomic adds reach at all (the LDS probe,
        # conflict-free addresses)
        ceil = measured_lds_atomic_peak()
        roof["atomic_ceiling"] = None if ceil is None else {
            "peak": round(ceil, 1), "frac": round(achieved / ceil, 4),
            "source": "LDS probe, ds_add_u64 at conflict-free addresses"}
    else:
        dominant = max(("synth", "synth_adj"), key=lambda k: k_ms[k])
        achieved = FLOP_PER_PATH_SAMPLE[dominant] * ps / (k_ms[dominant] * 1e-3) / 1e12
        # the synthesis runs on the matrix cores for runs of 256 samples, else on the VALU
        synth_kernel = "k_synth_mfma" if Sn % 256 == 0 else "k_synth"
        kern = "k_synth_adj" if dominant == "synth_adj" else synth_kernel
        roof = {"bound": "alu", "kernel": kern, "achieved": round(achieved, 3), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": measured_traffic(kern, args.workload)}
    out = {
        "metric": "ray-bounces/s fwd+bwd",
        "value": queries / (ms_step * 1e-3),
        "unit": "ray-bounces/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_p10_p50_p90": [round(float(np.percentile(per_step, q)), 3) for q in (10, 50, 90)],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}_fwd_bwd", "triangles": scene.nf, "rays": g.n_rays,
                   "max_bounces": g.max_bounces, "virtual_antennas": V, "chirps": C, "samples": Sn,
                   "parallelism": "single-gpu"},
        "ray_bounces_per_step": queries,
        "paths": n_paths,
        "if_path_samples_per_s": ps / (ms_step * 1e-3),
        "if_output_samples_per_s": V * C * Sn / (ms_step * 1e-3),
        "kernel_ms": {k: round(v, 4) for k, v in k_ms.items()},
        # both sums of the path-sample work run as non-uniform FFTs for 16 <= S <= 1024:
        # times per stage and the rates of the direct sums they replace (which a
        # direct evaluation could reach at most at the FP32 peak)
        "synth": {"form": "nufft" if nufft else "direct", "ms": round(k_ms["synth"], 4),
                  "spread_ms": round(k_ms["nu_spread"], 4) if nufft else None,
                  "direct_sum_equivalent_tflops": round(FLOP_PER_PATH_SAMPLE["synth"] * ps /
                                                        (k_ms["synth"] * 1e-3) / 1e12, 2)},
        "adjoint": {"form": "nufft" if nufft else "direct", "ms": round(k_ms["synth_adj"], 4),
                    "taps_ms": round(k_ms["nu_taps"], 4) if nufft else None,
                    "path_antenna_chirps_per_s": pac / (k_ms["synth_adj"] * 1e-3),
                    # the tap kernel's row reads from LDS (7 float4 per (path, antenna,
                    # chirp)) against the LDS bandwidth of the unit counts
                    "taps_lds_read_gbs": round(LDS_READ_BYTES_PER_PAC * pac / (k_ms["nu_taps"] * 1e-3) / 1e9, 1)
                    if nufft else None,
                    "taps_lds_frac": round(LDS_READ_BYTES_PER_PAC * pac / (k_ms["nu_taps"] * 1e-3) / 1e9 /
                                           PEAK_LDS_GBS, 4) if nufft else None,
                    "direct_sum_equivalent_tflops": round(FLOP_PER_PATH_SAMPLE["synth_adj"] * ps /
                                                          (k_ms["synth_adj"] * 1e-3) / 1e12, 2)},
        "trace": {"ray_bounces_per_s": queries / (k_ms["trace"] * 1e-3), "node_tests": node_tests,
                  "tri_tests": tri_tests,
                  "alg_valu_ops_per_s": (OPS_PER_NODE_TEST * node_tests + OPS_PER_TRI_TEST * tri_tests) /
                  (k_ms["trace"] * 1e-3),
                  "frac_of_valu_peak": round((OPS_PER_NODE_TEST * node_tests + OPS_PER_TRI_TEST * tri_tests) /
                                             (k_ms["trace"] * 1e-3) / PEAK_VALU_LANE_OPS, 4)},
        "wall_ms_per_step": (w1 - w0) * 1e3 / args.steps,
        "roofline": roof,
    }
    if not args.no_serving:
        # request latency of the serving loop on the mixed request stream
        # (meshes of 1k-200k triangles, 256^2-2048^2 rays, 2-4 bounces, 4-12
        # antennas x 32-128 chirps, 30 % with backward), Poisson arrivals at
        # 1.25x the measured one-at-a-time service rate
        del sim, cube, grad, gv, target
        torch.cuda.empty_cache()
        from paper_2311_13182_amd.serve import serving_benchmark
        sv = serving_benchmark(n=args.serving_requests, phases=(("main", 1.25), ("low", 0.5)), quiet=True)
        m = sv["main"]
        out["serving"] = {"requests": args.serving_requests, "collect_workers": sv["collect_workers"],
                          "qps": round(m["qps"], 2),
                          "throughput_rps": round(m["server"]["throughput_rps"], 2),
                          "p50_latency_ms": round(m["server"]["p50_latency_ms"], 1),
                          "p99_latency_ms": round(m["server"]["p99_latency_ms"], 1),
                          "sequential_throughput_rps": round(m["sequential"]["throughput_rps"], 2),
                          "sequential_p50_latency_ms": round(m["sequential"]["p50_latency_ms"], 1),
                          "sequential_p99_latency_ms": round(m["sequential"]["p99_latency_ms"], 1),
                          "mean_batch": round(m["server"]["mean_batch"], 3)}
        lo = sv["low"]
        out["serving"]["low_load"] = {"qps": round(lo["qps"], 2),
                                      "p50_latency_ms": round(lo["server"]["p50_latency_ms"], 1),
                                      "p99_latency_ms": round(lo["server"]["p99_latency_ms"], 1),
                                      "sequential_p50_latency_ms": round(lo["sequential"]["p50_latency_ms"], 1),
                                      "sequential_p99_latency_ms": round(lo["sequential"]["p99_latency_ms"], 1),
                                      "mean_batch": round(lo["server"]["mean_batch"], 3)}
        bu = sv["burst"]
        out["serving"]["burst"] = {"requests": bu["requests"],
                                   "throughput_rps": round(bu["server"]["throughput_rps"], 2),
                                   "sequential_throughput_rps": round(bu["sequential"]["throughput_rps"], 2),
                                   "mean_batch": round(bu["server"]["mean_batch"], 3),
                                   "max_batch": bu["server"]["max_batch"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scene, queries)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
