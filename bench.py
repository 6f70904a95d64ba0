"""Benchmark: fused state-vector evolution of the 30-qubit grid random circuit.

Workload: 5x6 grid random circuit, depth 20, 845 gates (600 single-qubit
sqrt(X)/sqrt(Y)/sqrt(W), 245 fSim(pi/2, pi/6)), complex64 state of 2^30
amplitudes (8 GiB), seed 1.  One step = reset to |0..0>, fuse the gates
(greedy fusion, blocks of at most max_k qubits) and apply every block, then
the FP64 norm: the whole path from gate list to reduced result.  Inputs are
resident on the device before the timed region.  Default arithmetic: tiled
passes of 4-qubit blocks as split FP16 MFMA products (FP32's per-amplitude
error; `--precision` selects split BF16, BF16 with a three-part state, or
FP32).

Reported next to the fused throughput: the plain per-gate complex64 run, the
fidelity error and amplitude max-abs error of both against a complex128 GPU
run of the same circuit (first 2^20 amplitudes for the max-abs), the roofline
of the dominant kernel (HIP-event timed inside the timed region), and the CPU
oracle timed on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--max-k K]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
MFMA_FP32_PEAK_TFLOPS = 157.3
FAMILY_NAMES = {1: "reg", 2: "generic", 3: "mfma_f32", 4: "split_bf16", 5: "split_fp16", 9: "tile",
                10: "tile_bf16", 11: "tile_fp16", 12: "tile_bf16x3"}
KERNEL_SOURCES = {1: "apply.hip", 2: "apply.hip", 3: "mfma.hip", 4: "mfma.hip", 5: "mfma.hip", 9: "tile.hip",
                  10: "tile.hip", 11: "tile.hip", 12: "tile.hip"}
TILE_FAMILIES = (9, 10, 11, 12)
PRECISIONS = {"fp32": 0, "bf16": 1, "fp16": 2, "bf16x3": 4}  # SV_PREC_* codes
DEFAULT_PRECISION = {"circuit": "fp16", "gradient": "fp32", "trajectories": "fp16", "density": "bf16x3",
                     "jumps": "fp32"}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_hash(fam: int) -> str:
    p = os.path.join(ROOT, "paper_2111_06868_amd", "csrc", KERNEL_SOURCES[fam])
    return hashlib.sha256(open(p, "rb").read()).hexdigest()[:16]


def read_traffic(fam: int, k: int, n: int):
    """HBM bytes per launch from a committed rocprofv3 counter summary, or
    None when there is none or the kernel source changed since."""
    tag = FAMILY_NAMES[fam] if k == 0 else "%s_k%d" % (FAMILY_NAMES[fam], k)
    name = os.path.join(ROOT, "profiles", "traffic_%s_%dq.md" % (tag, n))
    if not os.path.exists(name):
        return None
    kv = {}
    for ln in open(name):
        if ":" in ln and ln.startswith("- "):
            key, _, val = ln[2:].partition(":")
            kv[key.strip()] = val.strip().strip("`")
    if kv.get("kernel_source_sha256_16") != source_hash(fam):
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    """The host CPU's model name (as lscpu prints it), from /proc/cpuinfo."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.lower().startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, gates, budget_s=20.0):
    """The oracle (complex128, gate at a time, OpenMP over amplitude groups)
    on the full-size state for the circuit's first gates."""
    import numpy as np
    from oracle import ref
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    psi = np.zeros(1 << n, dtype=np.complex128)
    psi[0] = 1.0
    ops = [(ref.matrix_of(g), g.qubits) for g in gates]
    done = 0
    t0 = time.perf_counter()
    while done < len(ops):
        ref.run_matrices(psi, ops[done:done + 1])
        done += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    del psi
    return {"value": done / dt, "unit": "gates/s", "cores": threads, "kind": "oracle",
            "sample": "first %d of %d gates on the full %d-qubit complex128 state" % (done, len(ops), n)}


def cpu_baseline_one_thread(config, budget_s):
    """cpu_baseline in a child process limited to one OpenMP thread."""
    import subprocess
    env = dict(os.environ, OMP_NUM_THREADS="1")
    code = ("import json, sys; sys.path.insert(0, %r); import bench; from workloads import circuits as wc; "
            "n, g = wc.config_circuit(%d); print(json.dumps(bench.cpu_baseline(n, g, %r)))" % (ROOT, config, budget_s))
    r = subprocess.run([sys.executable, "-c", code], env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                       text=True, timeout=budget_s + 300)
    if r.returncode != 0:
        log("one-thread oracle failed: %s" % r.stderr[-500:])
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def small_circuit_lines(prec, steps=20):
    """The 14-qubit grid circuit (225 gates, a 128 KiB state that a compute
    unit's LDS could hold): microseconds per gate on the GPU, fused (tiled
    rule, k <= 4, in the headline's arithmetic `prec`) and per gate, and for
    the CPU oracle (all threads)."""
    import numpy as np
    import torch
    import paper_2111_06868_amd as sv
    from oracle import ref
    from workloads import circuits as wc
    n, gates = wc.config_circuit(0)
    ga = sv.GateArray([(g.name, g.qubits, g.params) for g in gates])
    st = sv.State(n, "c64")
    out = {}
    for name, kw in (("fused", dict(max_k=4, rule=sv.RULE_TILED, precision=prec)),
                     ("per_gate", dict(rule=sv.RULE_NONE))):
        st.set_basis(0).run(ga, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            st.set_basis(0).run(ga, **kw)
        torch.cuda.synchronize()
        out["gpu_%s_us_per_gate" % name] = round(1e6 * (time.perf_counter() - t0) / steps / len(gates), 3)
    want = ref.simulate(n, gates, "0")
    out["gpu_fused_fidelity_err"] = ref.fidelity_error(want, st.set_basis(0).run(
        ga, max_k=4, rule=sv.RULE_TILED, precision=prec).read())
    t0 = time.perf_counter()
    reps = 0
    while reps < 3 or time.perf_counter() - t0 < 1.0:
        ref.simulate(n, gates, "0")
        reps += 1
    out["cpu_oracle_us_per_gate"] = round(1e6 * (time.perf_counter() - t0) / reps / len(gates), 3)
    out["workload"] = "grid random circuit 2x7 depth 12 seed 0, 14 qubits, 225 gates"
    return out


def plan_tiles(blocks, n, tile_bits=14, page_bits=18):
    """The launches of a plan's tile passes and lone blocks: for each, the
    blocks' qubits, the union of their positions and the HBM layout of one
    tile (the union plus the lowest free positions, tile_bits in all: runs of
    2^run contiguous amplitudes, spread over 2^pages pages of 2^page_bits
    amplitudes)."""
    groups = []
    for b in blocks:
        if b.tile_pass >= 0 and groups and groups[-1][0] == b.tile_pass:
            groups[-1][1].append(b.qubits)
        else:
            groups.append((b.tile_pass, [b.qubits]))
    out = []
    for tp, qs in groups:
        union = sorted(set(q for b in qs for q in b))
        tile = set(union)
        for p in range(n):
            if len(tile) >= tile_bits:
                break
            tile.add(p)
        run = 0
        while run in tile:
            run += 1
        out.append({"tile_pass": tp, "blocks": qs, "union": union, "tile": sorted(tile), "run": run,
                    "pages": sum(1 for p in tile if p >= page_bits)})
    return out


def copy_ceiling(st, tiles, max_blocks, reps=3):
    """Streaming read + write passes (sv_stream_probe) over the state at the
    layouts of the plan's tile-pass launches, and at whole 128 KiB runs and
    the 128-byte runs of the top ten positions: the achievable time of a pass
    with each layout."""
    n = st.n
    cache = {}

    def probe(tile):
        key = tuple(tile)
        if key not in cache:
            cache[key] = st.stream_probe(key, reps=reps)
        return cache[key]

    contiguous = probe(range(14))
    top = probe(list(range(4)) + list(range(n - 10, n)))
    launches = []
    for t in tiles:
        if t["tile_pass"] >= 0 or len(t["union"]) <= 4:
            count = -(-len(t["blocks"]) // max_blocks)
            launches += [probe(t["tile"])] * count
    pass_bytes = 16.0 * (1 << n)
    out = {"contiguous_ms": round(contiguous, 4), "contiguous_GBps": round(pass_bytes / contiguous / 1e6, 1),
           "top10_128B_runs_ms": round(top, 4), "top10_128B_runs_GBps": round(pass_bytes / top / 1e6, 1)}
    if launches:
        mean = sum(launches) / len(launches)
        out.update({"plan_layouts_ms_per_launch": round(mean, 4),
                    "plan_layouts_GBps": round(pass_bytes / mean / 1e6, 1), "plan_launches": len(launches)})
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--max-k", type=int, default=4)
    ap.add_argument("--rule", default="tiled", choices=["paper", "enhanced", "tiled", "auto"])
    ap.add_argument("--precision", default=None, choices=["fp32", "bf16", "fp16", "bf16x3"],
                    help="tile-pass arithmetic; default: fp16 for the circuits (FP32's per-amplitude "
                         "error, unitary gates) and the trajectory batch (per-tile scales), bf16x3 for "
                         "the density matrix (trace-preserving to about 1e-6), fp32 for the gradient "
                         "and the sampled jumps")
    ap.add_argument("--config", type=int, default=1, choices=[1, 2])
    ap.add_argument("--workload", default="circuit", choices=["circuit", "gradient", "trajectories", "density", "jumps"],
                    help="circuit: the grid random circuit (default); gradient: 20-qubit ansatz "
                         "energy + adjoint gradient; trajectories: 512 noisy trajectories; density: "
                         "exact density matrix of a noisy 15-qubit grid circuit (a 30-qubit state); jumps: "
                         "amplitude damping sampled on a 26-qubit state")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-reference", action="store_true")
    ap.add_argument("--no-per-gate", action="store_true")
    ap.add_argument("--autotune", action="store_true", help="tune launch shapes first, fuse with max_k=-1")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--lightcone", action="store_true",
                    help="trajectories: keep only the light cone of qubit 0 (the paper's pop) and run each "
                         "trajectory on the cone's qubits")
    ap.add_argument("--plan", action="store_true",
                    help="print the fused plan's tile passes (blocks, union, HBM layout) and exit; no GPU needed")
    args = ap.parse_args()
    if args.precision is None:
        args.precision = DEFAULT_PRECISION[args.workload]
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the state-vector path here is built and measured "
              "on a single MI355X (--gpus %d is not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2111_06868_amd as sv
    from workloads import circuits as wc

    if args.plan:
        return print_plan(args)
    torch.cuda.set_device(0)
    if args.workload == "gradient":
        return bench_gradient(args)
    if args.workload == "trajectories":
        return bench_trajectories(args)
    if args.workload == "density":
        return bench_density(args)
    if args.workload == "jumps":
        return bench_jumps(args)
    n, gates = wc.config_circuit(args.config)
    bound = [(g.name, g.qubits, g.params) for g in gates]
    ga = sv.GateArray(bound)
    rule = {"enhanced": sv.RULE_ENHANCED, "paper": sv.RULE_PAPER, "tiled": sv.RULE_TILED,
            "auto": sv.RULE_AUTO}[args.rule]
    prec = PRECISIONS[args.precision]
    G = len(gates)
    pass_bytes = 16.0 * (1 << n)

    max_k = args.max_k
    if args.autotune:
        scratch = sv.State(n, "c64")
        cost = sv.autotune(scratch, prec)
        del scratch
        log("autotuned cost table (ms per block, k=1..6): %s" % ", ".join("%.3f" % c for c in cost[1:]))
        max_k = -1
    plan = sv.fuse(ga, n, max_k, rule, precision=prec)  # the plan the runs below form
    if max_k == -1 or rule == sv.RULE_AUTO:
        # the plan records what was chosen; the timed steps fuse with that choice
        max_k = plan.max_k
        args.max_k = max_k
        rule = plan.rule
        args.rule = {sv.RULE_ENHANCED: "enhanced", sv.RULE_PAPER: "paper", sv.RULE_TILED: "tiled"}[rule]
    blocks = plan.blocks(False)
    n_passes = len(blocks)  # tiled: several blocks share one pass (counted from the launches below)
    kh = {}
    for b in blocks:
        kh[len(b.qubits)] = kh.get(len(b.qubits), 0) + 1
    log("n=%d gates=%d fused blocks=%d k-histogram=%s" % (n, G, n_passes, kh))

    st = sv.State(n, "c64")
    stream = st.stream

    def step():
        # |0..0> and the circuit in one call: the first tile pass produces the
        # basis state itself instead of reading a filled state
        st.run(ga, max_k=args.max_k, rule=rule, precision=prec, basis=0)
        return st.norm2()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # throughput: K steps as the job runs (no per-launch events)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        nrm = step()
        log("step %d done, norm-1 = %.2e" % (i, nrm - 1))
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    ms_step = 1e3 * t_total / args.steps
    # kernel durations: K more steps with a HIP event pair around every launch
    # on the library's stream, kept out of the throughput run
    sv.stats_reset()
    sv.stats_enable(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for i in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_step_events = 1e3 * (time.perf_counter() - t1) / args.steps
    sv.stats_enable(False)
    log("timed steps: %.2f ms without launch events, %.2f ms with" % (ms_step, ms_step_events))

    # dominant kernel in the timed region.  Block kernels are instantiated
    # per block size k; a tile-pass kernel takes its block count at run time,
    # so its launches are one kernel whatever the count (k = 0 below).
    per_class, tile_blocks = {}, {}
    for fam in FAMILY_NAMES:
        for k in range(1, 17 if fam in TILE_FAMILIES else 7):
            cnt, ms = sv.stats_query(FAMILY_NAMES[fam], k)
            if not cnt:
                continue
            key = (fam, 0) if fam in TILE_FAMILIES else (fam, k)
            c0, m0 = per_class.get(key, (0, 0.0))
            per_class[key] = (c0 + cnt, m0 + ms)
            if fam in TILE_FAMILIES:
                tile_blocks[fam] = tile_blocks.get(fam, 0) + cnt * k
    (dfam, dk), (dcnt, dms) = max(per_class.items(), key=lambda kv: kv[1][1])
    avg_ms = dms / dcnt
    # algorithmic bytes per launch, averaged over the family's launches: a run
    # whose first tile pass produces |0..0> itself (FP32 and split-FP16 tile
    # passes, sv_run_circuit_basis) reads nothing in that pass, 8 B per amplitude
    alg_bytes = float(pass_bytes)
    starts_in_tile = (rule == sv.RULE_TILED and args.precision in ("fp32", "fp16") and blocks
                      and blocks[0].tile_pass >= 0 and dfam in (9, 11))
    if starts_in_tile:
        alg_bytes = pass_bytes * (1.0 - 0.5 * args.steps / dcnt)
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    kernel_ms_total = sum(ms for _, ms in per_class.values()) / args.steps
    state_passes = sum(cnt for cnt, _ in per_class.values()) // args.steps
    traffic = read_traffic(dfam, dk, n)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": FAMILY_NAMES[dfam] if dk == 0 else "%s k=%d" % (FAMILY_NAMES[dfam], dk),
                "avg_launch_ms": round(avg_ms, 4),
                "launches_per_step": dcnt // args.steps,
                "algorithmic_bytes_per_launch": round(alg_bytes)}
    if dfam in TILE_FAMILIES:
        blocks_per_launch = tile_blocks[dfam] / dcnt
        roofline["blocks_per_launch"] = round(blocks_per_launch, 3)
        # 8 * 16 flop per amplitude per 4-qubit block; split BF16 runs four products, FP16 three,
        # BF16X3 six
        flops = {10: 4, 11: 3, 12: 6}.get(dfam, 1) * 8.0 * 16 * (1 << n) * blocks_per_launch
        roofline["mfma_tflops"] = round(flops / (avg_ms * 1e-3) / 1e12, 2)
        if dfam == 9:
            roofline["mfma_frac"] = round(roofline["mfma_tflops"] / MFMA_FP32_PEAK_TFLOPS, 4)
    if dfam in (3, 4, 5):
        flops = 8.0 * (1 << dk) * (1 << n) * {4: 4, 5: 3}.get(dfam, 1)
        roofline["mfma_tflops"] = round(flops / (avg_ms * 1e-3) / 1e12, 2)
        if dfam == 3:
            roofline["mfma_frac"] = round(roofline["mfma_tflops"] / MFMA_FP32_PEAK_TFLOPS, 4)
    log("timed %.1f ms/step; dominant %s avg %.3f ms -> %.0f GB/s" % (ms_step, roofline["kernel"], avg_ms, achieved))
    fused_state = st

    # the achievable copy at the same layouts (the state is left unchanged);
    # the plan was formed for this precision, so each of its passes is one launch
    tiles = plan_tiles(blocks, n) if rule == sv.RULE_TILED else []
    max_blocks = max([len(t["blocks"]) for t in tiles] + [1])
    ceiling = copy_ceiling(st, tiles, max_blocks)
    roofline["copy_ceiling"] = ceiling
    if dfam in TILE_FAMILIES and "plan_layouts_GBps" in ceiling:
        roofline["frac_of_copy_ceiling"] = round(achieved / ceiling["plan_layouts_GBps"], 4)
    log("copy ceiling: %s" % ceiling)
    # host planning (fusion and block matrices), which each step repeats before its launches
    t1 = time.perf_counter()
    for _ in range(5):
        sv.fuse(ga, n, args.max_k, rule, precision=prec)
    host_plan_ms = 1e3 * (time.perf_counter() - t1) / 5

    extra = {}
    pg = None
    if not args.no_per_gate:
        # plain per-gate complex64 run (same circuit), one timed run
        pg = sv.State(n, "c64")
        pg.run(ga, rule=sv.RULE_NONE)  # warm
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pg.set_basis(0)
        pg.run(ga, rule=sv.RULE_NONE)
        pg.norm2()
        torch.cuda.synchronize()
        t_pg = time.perf_counter() - t1
        extra["per_gate_gates_per_s"] = round(G / t_pg, 2)
        extra["per_gate_ms"] = round(1e3 * t_pg, 2)
        extra["fused_speedup_vs_per_gate"] = round(t_pg * 1e3 / ms_step, 3)
        log("per-gate: %.1f ms" % (1e3 * t_pg))

    if not args.no_reference:
        refst = sv.State(n, "c128")
        refst.run(ga, rule=sv.RULE_NONE)
        nr = refst.norm2()
        fe_fused = sv.fidelity_error(refst, fused_state)
        first = 1 << 20
        a = refst.read(0, first)
        extra["fidelity_err_fused"] = fe_fused
        # unnormalised: 1 - |<ref|psi>|^2 with ||ref|| = 1, which norm drift does not cancel
        extra["fidelity_err_raw_fused"] = 1.0 - abs(refst.inner(fused_state)) ** 2
        extra["max_abs_first_2^20_fused"] = float(np.max(np.abs(fused_state.read(0, first) - a)))
        fe_pg = None
        if pg is not None:
            fe_pg = sv.fidelity_error(refst, pg)
            extra["fidelity_err_per_gate"] = fe_pg
            extra["max_abs_first_2^20_per_gate"] = float(np.max(np.abs(pg.read(0, first) - a)))
        extra["norm_minus_1_fused"] = fused_state.norm2() - 1.0
        extra["norm_minus_1_c128"] = nr - 1.0
        log("fidelity err fused %.2e per-gate %s" % (fe_fused, fe_pg))
        del refst
    del pg

    # plain device copy for the achievable-bandwidth context
    x = torch.empty(1 << 29, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(10):
        y.copy_(x)
    ev1.record()
    torch.cuda.synchronize()
    extra["copy_kernel_GBps"] = round(10 * 2 * x.numel() * 4 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9, 1)
    del x, y

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(n, gates, args.cpu_budget)
        cpu["cpu_model"] = cpu_model()
        one = cpu_baseline_one_thread(args.config, args.cpu_budget / 2)
        if one is not None:
            cpu["one_thread"] = {"value": one["value"], "unit": one["unit"], "sample": one["sample"]}
        log("14-qubit circuit lines ...")
        extra["small_circuit"] = small_circuit_lines(prec)

    out = {
        "metric": "gates/s + effective HBM GB/s at 30q; fused vs per-gate at <=1e-5 fidelity err",
        "value": round(G / (ms_step * 1e-3), 2),
        "unit": "gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "ms_per_step_with_launch_events": round(ms_step_events, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "bf16": "bf16 split (3-part matrix, hi+lo state), f32 accumulate",
                  "fp16": "f16 split (2-part matrix, hi+lo state, per-tile scale), f32 accumulate",
                  "bf16x3": "bf16 split (3-part matrix, 3-part state), f32 accumulate"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "grid random circuit %s, %d qubits, %d gates, complex64, fused k<=%d (%s rule, %s)"
                   % ({1: "5x6 depth 20 seed 1", 2: "4x8 depth 14 seed 2"}[args.config], n, G, args.max_k,
                      args.rule, args.precision),
                   "qubits": n, "gates": G, "max_k": args.max_k, "blocks": n_passes,
                   "block_sizes": {str(k): v for k, v in sorted(kh.items())}},
        "state_passes": state_passes,
        "effective_GBps": round((state_passes * pass_bytes - (pass_bytes / 2 if starts_in_tile else 0))
                                / (ms_step * 1e-3) / 1e9, 1),
        "kernel_ms_per_step": round(kernel_ms_total, 3),
        "host_fusion_ms_per_step": round(host_plan_ms, 3),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)


def print_plan(args, tile_bits=14, page_bits=18):
    """Tile passes of the circuit's plan: for each pass its blocks, the union
    of their positions and the HBM layout of one tile (the union plus the
    lowest free positions, tile_bits in all: runs of 2^r contiguous
    amplitudes, spread over 2^h pages of 2^page_bits amplitudes)."""
    import paper_2111_06868_amd as sv
    from workloads import circuits as wc

    n, gates = wc.config_circuit(args.config)
    ga = sv.GateArray([(g.name, g.qubits, g.params) for g in gates])
    rule = {"enhanced": sv.RULE_ENHANCED, "paper": sv.RULE_PAPER, "tiled": sv.RULE_TILED,
            "auto": sv.RULE_AUTO}[args.rule]
    prec = PRECISIONS[args.precision]
    blocks = sv.fuse(ga, n, args.max_k, rule, precision=prec).blocks(False)
    tiles = plan_tiles(blocks, n, tile_bits, page_bits)
    print("n=%d gates=%d blocks=%d passes=%d" % (n, len(gates), len(blocks), len(tiles)))
    for i, t in enumerate(tiles):
        if t["tile_pass"] < 0 and len(t["union"]) > 4:
            print("%3d dense k=%d on %s" % (i, len(t["union"]), t["union"]))
            continue
        # a lone block of k <= 4 (tile_pass < 0) may run as a one-block tile pass
        print("%3d %s s=%d union=%s run=2^%d pages=2^%d blocks=%s"
              % (i, "tile" if t["tile_pass"] >= 0 else "single", len(t["blocks"]), t["union"], t["run"],
                 t["pages"], " ".join(",".join(map(str, b)) for b in t["blocks"])))


def _timed_steps(args, step):
    import torch
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        log("step %d done" % i)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / args.steps


def bench_gradient(args):
    """20-qubit hardware-efficient ansatz (12 layers, 480 angles): one step =
    forward circuit, <H> (39 Pauli terms) and the adjoint gradient."""
    import numpy as np
    import paper_2111_06868_amd as sv
    from workloads import circuits as wc
    n = 20
    gates, thetas = wc.ansatz_circuit(n, 12, seed=3)
    H = sv.pauli_sum(wc.ansatz_observable(n))
    ga = sv.GateArray([(g.name, g.qubits, g.params, g.param_index) for g in gates])
    psi, scratch = sv.State(n, "c64"), sv.State(n, "c64")
    prec = PRECISIONS[args.precision]
    # launch shapes and block costs for 20-qubit states (sizes the fusion of
    # the forward circuit and of the adjoint's dagger blocks)
    sv.autotune(scratch, prec)
    out = {}

    def step():
        psi.set_basis(0)
        psi.run(ga, max_k=-1, rule=sv.RULE_AUTO, precision=prec)
        out["E"] = psi.expectation(H)
        out["g"] = sv.backward(psi, scratch, ga, H, len(thetas), precision=prec)

    t = _timed_steps(args, step)
    print(json.dumps({"metric": "energy + adjoint gradient evaluations/s (20-qubit ansatz, 480 parameters)",
                      "value": round(1.0 / t, 3), "unit": "evals/s", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "ms_per_step": round(1e3 * t, 3), "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None,
                      "dtype": {"fp32": "f32", "bf16": "f32 state; bf16 hi+lo split products",
                                "fp16": "f32 state; f16 hi+lo split products",
                                "bf16x3": "f32 state; bf16 three-part split products"}[args.precision],
                      "data": "synthetic",
                      "config": {"workload": "20-qubit ansatz, 12 layers RY/RZ + CZ ladder, 708 gates, 480 angles"},
                      "energy": out["E"], "grad_norm": float(np.linalg.norm(out["g"]))}), flush=True)


def bench_trajectories(args):
    """512 noisy trajectories (n in 10..22, depth 8..24, p = 1e-3): one step =
    one replay of the captured batch graph and the <Z_0> readback."""
    import numpy as np
    import paper_2111_06868_amd as sv
    from workloads import circuits as wc
    trajs = wc.trajectory_batch()
    # tile passes of the trajectories with >= 14 qubits, by --precision (default split FP16)
    prec = PRECISIONS[args.precision]
    circuits = [(t.n, [(g.name, g.qubits, g.params) for g in t.gates]) for t in trajs]
    if args.lightcone:
        circuits = [lightcone_circuit(n_, gs) for n_, gs in circuits]
    b = sv.Batch(circuits, max_k=-1, precision=prec)
    out = {}

    def step():
        out["z"] = b.run(use_graph=True)

    t = _timed_steps(args, step)
    amps = sum(1 << n_ for n_, _ in circuits)
    print(json.dumps({"metric": "noisy trajectories/s (512 trajectories, 10..22 qubits)",
                      "value": round(len(trajs) / t, 2), "unit": "trajectories/s", "n_gpus": 1,
                      "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(1e3 * t, 3),
                      "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
                      "dtype": {"fp32": "f32", "bf16": "f32; bf16 hi+lo split tile passes (n >= 14)",
                                "fp16": "f32; f16 hi+lo split tile passes (n >= 14)",
                                "bf16x3": "f32; bf16 three-part split tile passes (n >= 14)"}[args.precision],
                      "data": "synthetic",
                      "config": {"workload": "512 ladder random circuits, n~U{10..22}, depth~U{8..24}, "
                                             "2q depolarizing p=1e-3 sampled per trajectory"
                                             + ("; light cone of qubit 0 only" if args.lightcone else ""),
                                 "gates": sum(len(gs) for _, gs in circuits), "amplitudes": amps},
                      "mean_z0": float(np.mean(out["z"]))}), flush=True)


def lightcone_circuit(n, gates, pinned=0):
    """The gates in the light cone of qubit `pinned` (sv.lightcone), moved onto
    the qubits they touch (sv.compact_qubits; the pinned qubit 0 stays
    position 0)."""
    import paper_2111_06868_amd as sv
    keep = sv.lightcone(gates, n, (pinned,))
    n_used, moved, _ = sv.compact_qubits([gates[i] for i in keep], n, (pinned,))
    return n_used, moved


def bench_density(args):
    """Exact density matrix of the 3x5 grid circuit (depth 20) with the
    two-qubit depolarizing channel (p = 1e-3) after every fSim: rho of 15
    qubits is a 30-qubit complex64 state (8 GiB).  One step = reset to
    |0..0><0..0|, rewrite and fuse the super circuit, apply it (tiled rule),
    and read Tr(rho Z_0)."""
    import numpy as np
    import torch
    import paper_2111_06868_amd as sv
    from workloads import circuits as wc
    if args.precision == "fp16":
        print("bench.py: density matrices do not run split FP16 tile passes (super operators may raise "
              "the 2-norm they rely on); use --precision bf16 or fp32", file=sys.stderr)
        sys.exit(2)
    n = 15
    gates, channels = wc.noisy_grid_circuit(3, 5, 20, seed=7, p=1e-3)
    ga = sv.GateArray([(g.name, g.qubits, g.params) for g in gates])
    ops = [sv.depolarizing(q, p, after=a) for a, q, p in channels]
    prec = PRECISIONS[args.precision]
    rho = sv.DensityMatrix(n, "c64")
    Z0 = sv.pauli_sum([(1.0, ((0, "Z"),))])
    out = {}

    def step():
        rho.set_basis(0)
        rho.run(ga, ops, max_k=4, rule=sv.RULE_TILED, precision=prec)
        out["z0"] = rho.expectation(Z0)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    sv.stats_reset()
    sv.stats_enable(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        log("step %d done" % i)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / args.steps
    sv.stats_enable(False)
    fam = {sv.PREC_SPLIT_BF16: 10, sv.PREC_SPLIT_BF16X3: 12}.get(prec, 9)
    cnt = ms = 0
    for k in range(1, 17):
        c, m = sv.stats_query(FAMILY_NAMES[fam], k)
        cnt, ms = cnt + c, ms + m
    avg_ms = ms / max(cnt, 1)
    achieved = 16.0 * (1 << (2 * n)) / (avg_ms * 1e-3) / 1e9
    # complex128 reference run (not timed): Tr(rho Z_0), trace and the first 2^20 entries
    ref_rho = sv.DensityMatrix(n, "c128").run(ga, ops, max_k=4, rule=sv.RULE_ENHANCED, precision=sv.PREC_FP64)
    z0_ref = ref_rho.expectation(Z0)
    head = 1 << 20
    max_abs = float(np.abs(rho.state.read(0, head).astype(np.complex128) - ref_rho.state.read(0, head)).max())
    trace = rho.trace()
    del ref_rho
    n_ops = len(gates) + len(channels)
    print(json.dumps({"metric": "noisy super-circuit operations/s (15-qubit density matrix, exact)",
                      "value": round(n_ops / t, 2), "unit": "operations/s", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "ms_per_step": round(1e3 * t, 3), "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None,
                      "dtype": {"fp32": "f32", "bf16": "f32; bf16 hi+lo split tile passes",
                                "bf16x3": "f32; bf16 three-part split tile passes"}[args.precision],
                      "data": "synthetic",
                      "config": {"workload": "3x5 grid random circuit, depth 20, 2q depolarizing p=1e-3 after "
                                             "every fSim; rho as a 30-qubit complex64 state",
                                 "gates": len(gates), "channels": len(channels)},
                      "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                                   "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                                   "kernel": FAMILY_NAMES[fam], "avg_launch_ms": round(avg_ms, 4),
                                   "launches_per_step": cnt // args.steps},
                      "z0": out["z0"], "z0_c128": z0_ref, "trace": trace,
                      "max_abs_first_2^20_vs_c128": max_abs}), flush=True)


def bench_jumps(args):
    """Amplitude damping (gamma = 0.01) sampled on a pure 26-qubit state: the
    2x13 grid circuit of depth 10 with the channel on every qubit after each
    cycle's fSims.  One step = one trajectory: fused gate runs
    between channels, and per channel one FP64 pass for the outcome weights,
    the draw and the application of K_i / sqrt(p_i)."""
    import numpy as np
    import paper_2111_06868_amd as sv
    from workloads import circuits as wc
    n = 26
    gates = wc.grid_rqc(2, 13, 10, seed=5)
    ends = [i + 1 for i, g in enumerate(gates)
            if g.name == "FSIM" and (i + 1 == len(gates) or gates[i + 1].name != "FSIM")]
    ops = [sv.amplitude_damping(q, 0.01, after=a) for a in ends for q in range(n)]
    ga = sv.GateArray([(g.name, g.qubits, g.params) for g in gates])
    st = sv.State(n, "c64")
    rng = np.random.default_rng(6)
    out = {}

    def step():
        st.set_basis(0)
        out["jumps"] = int(np.count_nonzero(st.run_trajectory(ga, ops, rng.random(len(ops)), max_k=4,
                                                              rule=sv.RULE_TILED)))

    for _ in range(args.warmup):
        step()
    sv.stats_reset()
    sv.stats_enable(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        step()
        log("step %d done (%d jumps)" % (i, out["jumps"]))
    t = (time.perf_counter() - t0) / args.steps
    sv.stats_enable(False)
    cnt, ms = sv.stats_query("reduce", 6)
    avg_ms = ms / max(cnt, 1)
    achieved = 8.0 * (1 << n) / (avg_ms * 1e-3) / 1e9
    print(json.dumps({"metric": "sampled Kraus channels/s (amplitude damping on a 26-qubit state)",
                      "value": round(len(ops) / t, 2), "unit": "channels/s", "n_gpus": 1, "steps": args.steps,
                      "warmup": args.warmup, "ms_per_step": round(1e3 * t, 3), "higher_is_better": True,
                      "scaling": "weak", "vs_baseline": None, "dtype": "f32 state, f64 weights",
                      "data": "synthetic",
                      "config": {"workload": "2x13 grid random circuit, depth 10, amplitude damping gamma=0.01 on "
                                             "every qubit after each cycle, one trajectory per step",
                                 "gates": len(gates), "channels": len(ops)},
                      "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                                   "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": None,
                                   "kernel": "k_kraus_probs", "avg_launch_ms": round(avg_ms, 4),
                                   "launches_per_step": cnt // max(args.steps, 1)},
                      "jumps_last_step": out["jumps"]}), flush=True)


if __name__ == "__main__":
    main()
