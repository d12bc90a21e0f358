#!/usr/bin/env python3
"""Benchmark of the split-step SSA hot path on one MI355X.

By default one step = one complete run of the batched ensemble: 64 parameter
sets (32 SIR, 32 SISe) x 64 replicates = 4,096 runs of 100..20,000 nodes each
(13.9 million nodes) over 365 days in one launch replayed from a captured HIP
graph at the autotuned launch shape (SSA to every day boundary, post-time
steps, weekly per-run sums), inputs resident in device memory.  The largest
single-GPU configuration; --workload sir-events times one run of the SIR
model with scheduled events on 10,000 nodes (exit/enter events per node,
external transfers between nodes, U recorded every day).  Prints one JSON
line:

  value            node-days per second over the timed steps (wall clock,
                   bracketed by device synchronisation)
  transitions_per_s executed transitions per second
  roofline         the SSA kernel against the VALU peak (see OPS_PER_STEP)
  hbm_roofline     transitions/s against the bytes-per-transition HBM bound
  cpu_baseline     the CPU oracle (OpenMP) on the same workload

  python bench.py [--gpus 1] [--steps 20] [--warmup 3]
  python bench.py --workload sir-events|sise-events|sir-plain|mlp
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SSA node-days/sec + transitions/sec on 1 MI355X; surrogate speedup at fixed error"

# VALU lane-operations of one SSA step: the 172 VALU instructions of the
# compiled draw loop of the SISe lane-queue kernel (18 32x32->64 products, 56
# integer and logic, 53 FP64, 45 selects, compares and moves), each counted
# once -- a lower bound on their issue cost, so the peak step rate below is an
# upper bound.
OPS_PER_STEP = 172
# 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz: one full-rate VALU op per lane-cycle
# (equals the published 78.6 TFLOP/s fp64 vector peak counted as FMA = 2).
VALU_PEAK_OPS = 256 * 4 * 16 * 2.4e9


SOLVER = "ssm"  # the solver of the timed runs and of the CPU baseline (--solver)
SSA_SOURCES = ("device_types.h", "device_math.h", "internal.h", "models.h", "runtime.cpp", "ssa_kernels.hip",
               "generated.cpp")


def _progress(*a):
    """A progress line on stderr (the result line alone goes to stdout)."""
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    """sha256 over the sources that decide the SSA kernels' code and data
    layout (the network's file is left out: it does not touch them)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1605_01421_amd", "csrc")
    for name in SSA_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources (FETCH_SIZE + WRITE_SIZE, copy-calibrated)."""
    return measured_traffic_at(kernel, workload)[0]


def measured_traffic_at(kernel: str, workload: str):
    """(HBM bytes per launch, the launch shape the counters were taken at),
    or (None, None) when there is no summary for the current sources."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.txt")
    if not os.path.exists(path):
        return None, None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_hash():
        return None, None
    try:
        return float(vals["hbm_bytes_per_launch"]), vals.get("launch_shape")
    except (KeyError, ValueError):
        return None, None


MODEL_NAMES = {0: "SIR", 1: "SIS", 2: "SISe", 3: "birth-death", 4: "immigration-death", 5: "SISe_sp"}
HBM_PEAK = 8.0e12  # bytes/s, MI355X HBM3E (published)


def algorithmic_bytes(spec, record_sums: bool) -> float:
    """HBM bytes one run (or batch) must move at least: node data read once
    (state, continuous state, local data and three 4-byte identities), node-
    local event records (16 B) read once, each external transfer's two
    per-node items and records (2 x 32 B), and the records written: per node
    and record 4 B per compartment and 8 B per continuous variable, or, for a
    batch recorded as sums, 8 B per run, record and compartment; for a
    spatially coupled model each stored neighbour's index and weight once."""
    runs = spec if isinstance(spec, list) else [(spec, 1)]
    total = 0.0
    for sp, reps in runs:
        nn, nc = sp.Nn, sp.Nc
        nv = int(np.asarray(sp.v0).reshape(nn, -1).shape[1]) if nn else 0
        nld = int(np.asarray(sp.ldata).reshape(nn, -1).shape[1]) if nn else 0
        ev = np.asarray(sp.events["event"])
        n_e2 = int((ev == 3).sum())
        n_e1 = int(ev.size) - n_e2
        ntspan = int(np.asarray(sp.tspan).size)
        per_run = nn * (4 * nc + 8 * (nv + nld) + 12) + 16 * n_e1 + 64 * n_e2
        per_run += 8 * ntspan * nc if record_sums else ntspan * nn * (4 * nc + 8 * nv)
        if getattr(sp, "neighbours", None) is not None:
            # the coupled post-time step: each neighbour's index and weight
            # read once (4 B + 8 B); the daily posts stay in the caches
            per_run += 12 * len(sp.neighbours["idx"])
        total += reps * per_run
    return float(total)


def build_workload(name):
    """(model argument, description) of a named workload: one run (a spec) or
    a batch ([(spec, replicates)])."""
    from paper_1605_01421_amd import workloads as W
    if name == "sir-events":
        spec = W.sir_with_events()
    elif name == "sir-plain":
        spec = W.plain_sir()
    elif name == "sise-events":
        spec = W.sise_with_events()
    elif name == "sise-sp":
        spec = W.sise_sp_with_events()
    elif name == "vaccination":
        spec = W.vaccination_example(infected=16)
    elif name == "ensemble":
        sets = W.ensemble_sets(seed=3, n_sets=64, replicates=64)
        nodes = sum(s.spec.Nn for s in sets) * 64
        desc = {"workload": "ensemble-64x64-365d", "runs": 64 * 64, "parameter_sets": 64, "replicates": 64,
                "nodes": nodes, "days": 365, "scheduled_events": 0, "model": "SIR (32 sets) + SISe (32 sets)",
                "record": "weekly sums per run"}
        return [(s.spec, 64) for s in sets], desc
    else:
        raise SystemExit(f"unknown workload {name}")
    model = ("generated: " + "; ".join(spec.mparse["transitions"])) if spec.mparse else MODEL_NAMES[int(spec.model)]
    desc = {"workload": spec.name, "nodes": spec.Nn, "days": spec.n_days,
            "scheduled_events": int(len(spec.events["time"])), "model": model, "record": "U every day"}
    return spec, desc


def cpu_baseline_batch(batch, seed, seconds, gpu_sums):
    """The oracle on a sample of a batch's runs: one replicate of each
    parameter set in a seeded shuffled order of the sets, then another
    replicate of each, and so on (run r uses stream r), until the time budget
    is spent; the weekly sums of every sampled run are checked against the
    GPU's."""
    import oracle
    threads = min(16, os.cpu_count() or 1)
    flat = [spec for spec, reps in batch for _ in range(reps)]
    starts = np.cumsum([0] + [reps for _, reps in batch])[:-1]
    order = np.random.default_rng(7).permutation(len(batch))
    sample = [int(starts[s] + (s + j) % batch[s][1]) for j in range(max(r for _, r in batch)) for s in order
              if j < batch[s][1]]
    runs, node_days, t_total, parity = 0, 0, 0.0, True
    for r in sample:
        if t_total >= seconds:
            break
        t0 = time.perf_counter()
        out = oracle.run(flat[r], seed, r, nthreads=threads, solver=SOLVER)
        t_total += time.perf_counter() - t0
        sums = out["U"].astype("int64").sum(axis=1)
        parity = parity and out["status"] == 0 and bool((gpu_sums[r, :, :sums.shape[1]] == sums).all())
        node_days += out["node_days"]
        runs += 1
    return {"value": node_days / t_total, "unit": "node-days/s", "cores": threads, "kind": "oracle",
            "sample": f"{runs} of the batch's {len(flat)} runs (replicates of all {len(batch)} parameter sets in "
                      f"turn, seed {seed}), {node_days} node-days in {t_total:.1f} s of CPU time",
            "sums_match_gpu": parity}


def cpu_baseline(spec, seed, seconds, gpu_counters):
    """Time the oracle (as it stands) on the same workload on the host cores."""
    import oracle
    threads = min(16, os.cpu_count() or 1)
    runs = 0
    node_days = 0
    t_total = 0.0
    parity = None
    while t_total < seconds and runs < 2000:
        t0 = time.perf_counter()
        r = oracle.run(spec, seed + runs, 0, nthreads=threads, solver=SOLVER)
        t_total += time.perf_counter() - t0
        if runs == 0:
            parity = (r["transitions"], r["events"]) == (gpu_counters["transitions"], gpu_counters["events"])
        node_days += r["node_days"]
        runs += 1
    return {"value": node_days / t_total, "unit": "node-days/s", "cores": threads, "kind": "oracle",
            "sample": f"{runs} full runs of the same workload (seeds {seed}..{seed + runs - 1}), "
                      f"{t_total:.1f} s of CPU time", "counters_match_gpu": parity}


MLP_DIMS = (8, 256, 256, 256, 256, 156)
BF16_PEAK = 2.5e15  # dense bf16 matrix-core FLOP/s of the MI355X (published)


def bench_mlp(args):
    """The surrogate network on the matrix cores: K training steps (forward,
    backward and AdamW at batch 4096) and K inference passes at batch 65536,
    each timed with HIP events on the launch stream."""
    import numpy as np
    import torch
    from paper_1605_01421_amd import siminf
    from paper_1605_01421_amd import workloads as W
    torch.cuda.set_device(0)
    fwd_flops = 2 * sum(a * b for a, b in zip(MLP_DIMS[:-1], MLP_DIMS[1:]))
    # backward: the weight gradient of every layer and the input gradient of
    # every layer but the first
    bwd_flops = 2 * fwd_flops - 2 * MLP_DIMS[0] * MLP_DIMS[1]
    rng = np.random.default_rng(0)
    Bt, Bi = 4096, 65536
    net = siminf.MLP(MLP_DIMS, Bi)
    net.set_params(W.mlp_init(MLP_DIMS, 1))
    Xt = torch.from_numpy(rng.normal(size=(Bt, 8)).astype(np.float32)).cuda()
    Tt = torch.from_numpy(rng.normal(size=(Bt, 156)).astype(np.float32)).cuda()
    Xi = torch.from_numpy(rng.normal(size=(Bi, 8)).astype(np.float32)).cuda()
    Yi = torch.empty((Bi, 156), dtype=torch.float32, device="cuda")
    for _ in range(args.warmup):
        net.backward(Xt, Tt, want_loss=False)
        net.adamw(1e-4)
        net.forward(Xi, Yi)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    for _ in range(args.steps):
        net.backward(Xt, Tt, want_loss=False)
        net.adamw(1e-4)
    ev[1].record()
    ev[2].record()
    for _ in range(args.steps):
        net.forward(Xi, Yi)
    ev[3].record()
    torch.cuda.synchronize()
    t_train = ev[0].elapsed_time(ev[1]) / 1e3 / args.steps
    t_inf = ev[2].elapsed_time(ev[3]) / 1e3 / args.steps
    inf_achieved = fwd_flops * Bi / t_inf
    out = {
        "metric": "surrogate MLP training samples/s (batch 4096, forward + backward + AdamW)",
        "value": Bt / t_train, "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_train * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16", "data": "synthetic",
        "config": {"workload": "surrogate-mlp", "dims": list(MLP_DIMS), "train_batch": Bt, "infer_batch": Bi},
        "train_tflops": (fwd_flops + bwd_flops) * Bt / t_train / 1e12,
        "inference_samples_per_s": Bi / t_inf, "inference_ms": t_inf * 1e3,
        "roofline": {"bound": "mfma", "achieved": inf_achieved / 1e12, "peak": BF16_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": inf_achieved / BF16_PEAK, "traffic": None,
                     "kernel": "forward pass at batch 65536 (five bf16 GEMMs with fused epilogues)",
                     "flops_per_sample": fwd_flops},
    }
    net.close()
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ensemble",
                    help="ensemble (default: 64 sets x 64 replicates), sir-events, sise-events, sise-sp, vaccination "
                         "(a model given as transition strings), sir-plain, mlp")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--order", type=int, default=0)
    ap.add_argument("--lanes", type=int, default=0, help="lanes per node: 0 auto, 1, 64")
    ap.add_argument("--wide", type=int, default=0, help="with --lanes 64: wavefront-wide nodes")
    ap.add_argument("--pipeline", type=int, default=0, help="0 auto, 1 on, 2 off")
    ap.add_argument("--pack", type=int, default=0, help="nodes per one-lane-per-node wavefront: 0 auto, 4, 8, 16, 32, 64")
    ap.add_argument("--group", type=int, default=0,
                    help="nodes after the wide ones on a group of 8 lanes: 0 none/tuned, -1 all, N")
    ap.add_argument("--lane-queue", type=int, default=0,
                    help="runs without transfers: 1 every lane advances its own node, 2 lanes in lockstep, 0 auto")
    ap.add_argument("--chunk", type=int, default=0, help="lane queue: nodes per chunk (0 auto)")
    ap.add_argument("--batch", type=int, default=0, help="lane queue: lanes per day-end batch (0 auto)")
    ap.add_argument("--graph", type=int, default=-1,
                    help="replay the run from a captured HIP graph: 1 on, 0 off, -1 on for batches without transfers")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner (launch shape from heuristics)")
    ap.add_argument("--solver", default="ssm", choices=["ssm", "aem"],
                    help="ssm: the split-step direct method (default); aem: the all events method")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="after the timed steps, copy a 256 MiB device buffer once (known-size reference "
                         "kernel for hardware byte counters)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    args = ap.parse_args()
    global SOLVER
    SOLVER = args.solver
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the simulation of one run "
              "is not sharded across GPUs", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1605_01421_amd import siminf

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "mlp":
        bench_mlp(args)
        return
    torch.cuda.set_device(0)
    spec, desc = build_workload(args.workload)
    _progress("workload built:", desc["workload"])
    batch = isinstance(spec, list)
    graph = args.graph if args.graph >= 0 else int(batch)
    model = siminf.Model(spec, record=siminf.RECORD_SUMS if batch else siminf.RECORD_FULL, block=args.block,
                         order=args.order, lanes=args.lanes, wide=args.wide, pipeline=args.pipeline,
                         pack=args.pack, graph=graph, group=args.group, lane_queue=args.lane_queue,
                         chunk=args.chunk, batch=args.batch, solver=args.solver)
    seed0 = 20240000
    tuned_ms = None
    if not args.no_tune:
        # one plain run first: long runs are tuned on one repeat per shape,
        # short ones on the mean over four seeds (a shape that is fast on
        # most seeds but slow on some, e.g. with the heaviest nodes on one
        # lane, is not taken)
        model.run(seed0 - 2000)
        assert model.wait() == 0, model.error_info()
        probe_ms = model.timing()["kernel_ms"]
        repeats = 1 if probe_ms > 500 else 2 if probe_ms > 100 else 4
        if probe_ms > 500:
            os.environ["SIMINF_AUTOTUNE_LOG"] = "1"  # a line per shape: long tunes keep printing
        _progress(f"autotuning ({probe_ms:.1f} ms per run, {repeats} repeat(s) per shape)")
        tuned_ms = model.autotune(seed=seed0 - 1000, repeats=repeats)
        _progress("autotuned:", model.launch_info(), f"{tuned_ms:.3f} ms")
    for w in range(args.warmup):
        model.run(seed0 - 1 - w)
        assert model.wait() == 0, model.error_info()
    torch.cuda.synchronize()
    _progress(f"warm-up done; timing {args.steps} steps")

    kernel_ms, node_days, transitions, draws, events = [], 0, 0, 0, 0
    first_counters = None
    t0 = time.perf_counter()
    for k in range(args.steps):
        model.run(seed0 + k)
        rc = model.wait()
        if rc != 0:
            raise SystemExit(f"run failed: {model.error_info()}")
        c = model.counters()
        if first_counters is None:
            first_counters = c
        kernel_ms.append(model.timing()["kernel_ms"])
        node_days += c["node_days"]
        transitions += c["transitions"]
        draws += c["draws"]
        events += c["events"]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    if args.calibrate_copy:
        src = torch.empty(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()

    mean_kernel_s = sum(kernel_ms) / len(kernel_ms) / 1e3
    draws_per_launch = draws / args.steps
    achieved = draws_per_launch * OPS_PER_STEP / mean_kernel_s
    info = model.launch_info()
    kernel_name = ["free_kernel", "sync_kernel", "flow_kernel", "lane_kernel"][info["mode"]]
    if args.solver == "aem":
        kernel_name += "_aem"  # the all events method's instantiation
    traffic_bytes, traffic_launch = measured_traffic_at(kernel_name, desc["workload"])
    out = {
        "metric": METRIC,
        "value": node_days / wall,
        "unit": "node-days/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": dict(desc, seed=seed0, block=info["block"], blocks=info["blocks"],
                       kernel=["free-running", "grid-barrier", "dataflow", "lane-queue"][info["mode"]],
                       chunk=info["chunk"], batch=info["batch"],
                       wide_nodes=info["wide"], pipeline=info["pipeline"], pack=info["pack"],
                       group_nodes=info["group"], graph=graph, solver=args.solver),
        "transitions_per_s": transitions / wall,
        "events_per_step": events / args.steps,
        "kernel_ms_mean": mean_kernel_s * 1e3,
        "autotune_best_ms": tuned_ms,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_PEAK_OPS / 1e12,
                     "unit": "TOP/s", "frac": achieved / VALU_PEAK_OPS,
                     "traffic": traffic_bytes,
                     # the counters' launch shape: the autotuner may pick another one from run to run
                     "traffic_launch": traffic_launch,
                     "kernel": kernel_name,
                     "ssa_steps_per_launch": draws_per_launch, "ops_per_step": OPS_PER_STEP},
    }
    alg = algorithmic_bytes(spec, batch)
    per_tr = alg / max(transitions / args.steps, 1.0)
    traffic = out["roofline"]["traffic"]
    out["hbm_roofline"] = {
        "algorithmic_bytes_per_launch": alg, "bytes_per_transition": per_tr,
        "transitions_per_s_at_peak": HBM_PEAK / per_tr,
        "frac": (transitions / wall) / (HBM_PEAK / per_tr),
        "measured_gb_per_s": traffic / mean_kernel_s / 1e9 if traffic else None,
        "peak_gb_per_s": HBM_PEAK / 1e9}
    if not args.no_cpu:
        _progress(f"GPU timing done ({mean_kernel_s * 1e3:.3f} ms per run); CPU oracle baseline")
        if batch:
            out["cpu_baseline"] = cpu_baseline_batch(spec, seed0 + args.steps - 1, args.cpu_seconds, model.sums())
        else:
            out["cpu_baseline"] = cpu_baseline(spec, seed0, args.cpu_seconds, first_counters)
    model.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
