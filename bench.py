"""Throughput of the PTHR hot path on one MI355X.

One step = one elementary Monte Carlo step (EMCS) of the whole batch: the
Metropolis sweeps of every PT clone (10) and reservoir clone (240), the
Houdayer step on every replica pair below T = 1, the PT and reservoir
exchanges, and the observables.  Default workload: L=16, 1024 samples of
Gaussian couplings, 4 replica groups x 36 temperatures on [0.2, 1.6], 4
reservoir clones per group, FP32 form.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload l16_fp32]
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2605_25872_amd import inputs  # noqa: E402

METRIC = "spin-flip attempts/ns + Houdayer moves/s, batched 3D EA L=16, one MI355X"
# MI355X: 256 compute units x 4 SIMDs at 2.4 GHz.  gfx950 issues a wave64
# VALU instruction in 2 cycles (32 lane-operations per SIMD per cycle, the
# FP32 vector rate of 157.3 TFLOP/s) for 32-bit floating-point add, mul and
# fma and integer add, sub, logic and right shifts, and in 4 cycles (16 per
# cycle, the FP64 vector rate of 78.6 TFLOP/s) for FP64 arithmetic and the
# other 32-bit instructions the sweep needs: widening multiplies, three-input
# logic, conversions, compares, rounding, ldexp, bit-field ops and left
# shifts (measured per instruction kind: profiles/gfx950_valu_issue_rates.md).
FAST_OPS_PER_S = 256 * 4 * 32 * 2.4e9
HALF_OPS_PER_S = 256 * 4 * 16 * 2.4e9
# EMCS needed to equilibrate one L=16 sample (paper, App. A.2 table).
T_EQ_EMCS = {12: 2 ** 17, 14: 6.4e6, 16: 3.84e7, 18: 3.48e7}

# Algorithmic VALU operations of one attempt, counted from the method's steps
# (one lane-operation per step, the exponential included for every attempt as
# the branch-free form evaluates it), split by issue class ("fast": 2-cycle,
# "half": 4-cycle instructions).
#   Metropolis FP32 (36): half = 1/4 of a Philox4x32-10 block (10 rounds x
#   (2 widening multiplies + 2 three-way XORs)) 10, float(w) 1, ldexp 1,
#   flip bit 1; fast = local field (6 sign insertions + 5 adds) 11,
#   t = -(beta log2 e) dE 1, k = rint(t) by the float adder (add and
#   subtract 1.5 2^23, integer k from the sum's bits) 3, f = t - k 1, 6 Horner
#   steps (degree-6 polynomial of 2^f), test (2^t 2^32 - float(w)) 1.
#   Metropolis FP64 (57): half = 1/2 block 20, 5 adds of the local field,
#   -beta dE 1, k (multiply, rint) 2, 2 Cody-Waite steps, r to float 1, k to
#   int 1, d = u 2^-k in float (two converts of the 53 random bits, ldexp) 3,
#   compares (dE <= 0, x >= -708, d against the two float bounds) 4, flip bit
#   1; fast = 6 sign insertions, the random bits' shift and multiply-add 2,
#   f = r log2 e 1, 6 Horner steps of the float 2^f, the two bounds 2.  The
#   FP64 polynomial that decides tests within 2^-20 of the bound (about one
#   in 10^6) is not counted.
#   Heat bath FP32 (41): fast = field 11, t 1, f 1, 6 Horner steps,
#   u = float(w) 2^-32 1, the fused multiply-add 1; half = Philox 10,
#   float(w) 1, rint 1, 2^k (convert + ldexp) 2, a zeroed below the cut and
#   the threshold a or 1 (a compare and a select each) 4, the final compare
#   1, flip bit 1.
#   Heat bath FP64 (63): half = 1/2 block 20, two converts of the 53-bit
#   uniform 2, the field's 5 adds, -beta |dE| 1, the FP64 exponential (2 for
#   k, 2 Cody-Waite steps, 14 Horner steps, scale 1) 19, a zeroed below the
#   cut and the threshold a or 1 (a compare and two selects each) 6, the
#   fused multiply-add 1, the final compare 1, flip bit 1; fast = 6 sign
#   insertions, 1 shift of the uniform.
OPS_BY_CLASS = {
    ("metropolis", "fp32"): {"fast": 11 + 1 + 3 + 1 + 6 + 1, "half": 10 + 1 + 1 + 1},
    ("metropolis", "fp64"): {"fast": 6 + 2 + 1 + 6 + 2, "half": 20 + 5 + 1 + 2 + 2 + 1 + 1 + 3 + 4 + 1},
    ("heatbath", "fp32"): {"fast": 11 + 1 + 1 + 6 + 1 + 1, "half": 10 + 1 + 1 + 2 + 2 + 2 + 1 + 1},
    ("heatbath", "fp64"): {"fast": 6 + 1, "half": 20 + 2 + 5 + 1 + 19 + 6 + 1 + 1 + 1},
}


def valu_peak(update: str, precision: str) -> tuple[float, int]:
    """Issue-limited rate of algorithmic operations (lane-operations per s)
    for the attempt's mix of 2- and 4-cycle instructions, and the operations
    per attempt."""
    c = OPS_BY_CLASS[(update, precision)]
    n = c["fast"] + c["half"]
    return n / (c["fast"] / FAST_OPS_PER_S + c["half"] / HALF_OPS_PER_S), n


# HBM bytes per sweep launch of the L=16 FP32 workload, from rocprofv3 counter
# runs (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, the factors that make a 256 MiB
# device copy read and write 256 MiB), valid for the kernel sources whose
# SHA-256 is recorded here; any other source reports null.
SWEEP_TRAFFIC = {
    "workload": "l16_fp32",
    "sources_sha256": "a6018820b7b04cb522803854d02c34a6925ba69ba1af38cf77d0f0e47cf09753",
    "fetch_kib": 75035.92,
    "write_kib": 98304.0,
}
# Utilisation of the Houdayer kernel in the same counter runs (L=16 FP32, all-
# cluster moves): VALU issue = SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x kernel
# cycles); LDS pipe busy = (2 cycles per LDS wave instruction + bank-conflict
# cycles) / (256 CUs x kernel cycles), a lower bound.  Neither is saturated:
# the kernel waits on the latency of dependent union-find steps.
HOUDAYER_COUNTERS = {
    "workload": "l16_fp32",
    "sources_sha256": SWEEP_TRAFFIC["sources_sha256"],
    "valu_issue": 0.641,
    "lds_pipe_busy": 0.345,
}
KERNEL_SOURCES = ("paper_2605_25872_amd/csrc/pthr_kernels.hip", "paper_2605_25872_amd/csrc/pthr_internal.h")


def kernel_sources_sha256() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def sweep_traffic_bytes(workload: str):
    """Counter-measured HBM bytes per sweep launch, or None if the kernel
    sources changed since the counters were taken (or another workload)."""
    if workload != SWEEP_TRAFFIC["workload"] or kernel_sources_sha256() != SWEEP_TRAFFIC["sources_sha256"]:
        return None
    return 1024.0 * (2.0 * SWEEP_TRAFFIC["fetch_kib"] + 1.0 * SWEEP_TRAFFIC["write_kib"])


def houdayer_utilisation(workload: str, mode: str):
    """Counter-measured VALU and LDS utilisation of the Houdayer kernel, or
    None if the kernel sources changed since the counters were taken (or
    another workload or Houdayer mode)."""
    c = HOUDAYER_COUNTERS
    if workload != c["workload"] or mode != "acu" or kernel_sources_sha256() != c["sources_sha256"]:
        return None
    return {"bound": "lds latency", "valu_issue": c["valu_issue"], "lds_pipe_busy": c["lds_pipe_busy"]}


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def attempts_per_emcs(w) -> float:
    npt = w.n_replicas * w.n_temps
    ner = w.n_replicas * w.n_reservoir
    return float(w.V * (w.sweeps_per_emcs * npt + w.er_sweeps_per_emcs * ner)) * w.n_samples


def moves_per_emcs(w, T) -> int:
    k_acu = int(np.sum(T < w.t_acu))
    return w.n_samples * (w.n_replicas // 2) * k_acu


def cpu_baseline(w, n_samples: int, mode: str, update: str = "metropolis") -> dict:
    """The CPU oracle on a bounded sample of the same workload (all host cores)."""
    import oracle

    T = w.temperatures()
    prec = oracle.FP64 if w.precision == "fp64" else oracle.FP32
    o = oracle.Oracle(w.L, n_samples, w.n_replicas, w.n_temps, w.n_reservoir, w.sweeps_per_emcs,
                      w.er_sweeps_per_emcs, prec, oracle.SINGLE_NEG if mode == "single" else oracle.ACU,
                      w.t_acu, w.seed,
                      local_update={"heatbath": oracle.HEAT_BATH, "micsa": oracle.MICSA}.get(update, oracle.METROPOLIS))
    o.init(w.couplings(n_samples), T)
    t0 = time.perf_counter()
    o.run(1)
    dt = time.perf_counter() - t0
    sub = inputs.Workload(**{**w.__dict__, "n_samples": n_samples})
    att = attempts_per_emcs(sub)
    return {"value": att / (dt * 1e9), "unit": "spin-flip attempts/ns", "cores": oracle_threads(),
            "kind": "oracle", "seconds": dt,
            "houdayer_moves_per_s": moves_per_emcs(sub, T) / dt,
            "sample": f"{n_samples} of {w.n_samples} samples, 1 EMCS, {w.precision} oracle"}


def precision_check(args) -> dict:
    """FP32 form against the FP64 form (bit-identical to the FP64 oracle) on
    the L=12 workload's shape (4 x 28 temperatures on [0.2, 1.6], 4 reservoir
    clones): per-temperature energy per spin paired on couplings and seed,
    and the P(q) distance against the spread between independent FP64 runs
    (analysis.precision_statement states the criteria)."""
    from paper_2605_25872_amd import analysis

    w = inputs.WORKLOADS[args.precision_workload]
    res = analysis.compare_precisions(w, args.samples, args.emcs,
                                      list(range(1, args.seeds + 1)), progress=log)
    return {"mode": "fp32_vs_fp64", "workload_name": w.name, **res}


def reservoir_decorrelation(args) -> dict:
    """C(tau) = (1/V) sum_i sigma_i(t) sigma_i(t + tau) of reservoir clones
    swept at T_max from an equilibrated start (paper Sec. 3, ER paragraph:
    the 960-sweep residence is calibrated by C(960) < 1e-3 at the paper's
    T_max), at the workload's T_max and at the paper's T_max = 2, on the GPU:
    per tau the mean over samples of each sample's average over its 8
    reservoir clones and its sites, with its standard error."""
    import torch
    from paper_2605_25872_amd import pthr

    w = inputs.WORKLOADS[args.workload if args.workload != "mixed" else "l16_fp32"]
    S = min(args.samples, w.n_samples)
    taus = [60, 120, 240, 480, 720, 960, 1440, 1920]
    out = {"mode": "reservoir_decorrelation", "L": w.L, "samples": S, "precision": w.precision,
           "reservoir_clones_per_sample": 8, "warmup_sweeps": 960, "taus": taus, "C": {}}
    for t_max in sorted({w.t_max, 2.0}):
        g = pthr.Pthr(w.L, S, 2, 2, 4, 0, 240, w.precision, "acu", 0.0, 5)
        g.init_samples(w.couplings(S), np.array([t_max - 0.1, t_max]))
        for _ in range(4):
            g.sweep(0, 240)
            g.pt_swap(False)  # closes the EMCS without a reservoir exchange
        er = slice(4, 12)
        s0 = g.read_spins()[:, er].astype(np.int8)
        done, m, rows = 0, 0, []
        for tau in taus:
            while done < tau:
                n = min(tau - done, 240 - m)
                g.sweep(0, n)
                done += n
                m += n
                if m == 240:
                    g.pt_swap(False)
                    m = 0
            cs = (s0.astype(np.int32) * g.read_spins()[:, er]).mean(axis=(1, 2))
            rows.append([float(cs.mean()), float(cs.std(ddof=1) / np.sqrt(S))])
            log(f"T_max={t_max}: C({tau}) = {rows[-1][0]:.5f} +- {rows[-1][1]:.5f}")
        torch.cuda.synchronize()
        g.check()
        out["C"][str(t_max)] = rows
    return out


def bench_mixed(args) -> dict:
    """Five lattice sizes (L = 8, 10, 12, 14, 16; FP32) advanced together: one
    graph launch per EMCS with a branch per size, against the same contexts
    run one after the other."""
    import torch
    from paper_2605_25872_amd import pthr

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    members = []
    batch = [dataclasses.replace(w, n_reservoir=0, t_acu=0.0) if args.mode == "plain" else w
             for w in inputs.MIXED_BATCH]
    for w in batch:
        g = pthr.Pthr(w.L, w.n_samples, w.n_replicas, w.n_temps, w.n_reservoir, w.sweeps_per_emcs,
                      w.er_sweeps_per_emcs, w.precision, "single" if args.mode == "single" else "acu", w.t_acu,
                      w.seed)
        g.init_samples(w.couplings(), w.temperatures())
        if not args.no_autotune:  # the mixed batch is defined with per-size autotuned schedules
            # each candidate timed over >= ~1.5e10 attempts, so that small lattices are not timed on one EMCS
            best = g.autotune(max(1, math.ceil(1.5e10 / attempts_per_emcs(w))))
            log(f"autotune L={w.L}: {best:.2f} ms/EMCS, {g.schedule().threads_per_sample} work-items, "
                f"clone split {g.schedule().clone_split}, sample split {g.schedule().sample_split}, "
                f"early-out below T = {g.schedule().exp_early_out / 1000:g}")
        members.append(g)
    # each size's own sample split, for the run of one size after the other
    alone_split = [g.schedule().sample_split for g in members]
    if not args.split_group_samples:
        # the sizes run side by side and fill the GPU together: splitting a
        # size's samples over several workgroups (which pays when it runs
        # alone, as the autotuner times it) only repeats per-word work here
        for g in members:
            g.set_schedule(sample_split=1)
    group_split = [g.schedule().sample_split for g in members]
    group = pthr.Group(members)
    obs = [g.new_obs() for g in members]
    # one graph launch runs `window` EMCS of every size as parallel branches
    # (each size's chain advances without waiting for the others in between)
    window = max(1, min(16, args.steps))
    group.run(max(args.warmup, window), obs, graph_window=window)  # captures the group graph
    torch.cuda.synchronize()
    log("mixed batch: warm-up done")
    t0 = time.perf_counter()
    group.run(args.steps, obs, graph_window=window)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # the same contexts one after the other, each with its own graph of the
    # same window and the sample split it takes alone
    for g, o, split in zip(members, obs, alone_split):
        g.set_schedule(graph_window=window, sample_split=split)
        g.run(window, o)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for g, o in zip(members, obs):
        g.run(args.steps, o)
    torch.cuda.synchronize()
    sequential = time.perf_counter() - t1
    for g in members:
        g.check()
    att = sum(attempts_per_emcs(w) for w in batch)
    moves = sum(moves_per_emcs(w, w.temperatures()) for w in batch)
    value = att * args.steps / (elapsed * 1e9)
    log(f"mixed batch: {value:.1f} attempts/ns together, "
        f"{att * args.steps / (sequential * 1e9):.1f} one size after the other")
    return {
        "metric": METRIC.replace("L=16", "L=8..16 mixed"),
        "value": value,
        "unit": "spin-flip attempts/ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "mixed_l8_to_l16", "graph_window": window,
                   "members": [{"L": w.L, "samples": w.n_samples, "temperatures": w.n_temps,
                                "threads_per_sample": g.schedule().threads_per_sample,
                                "exp_early_out_below_T": g.schedule().exp_early_out / 1000,
                                "clone_split": g.schedule().clone_split,
                                "sample_split_in_group": gs, "sample_split_alone": als}
                               for w, g, gs, als in zip(batch, members, group_split, alone_split)],
                   "replicas": 4, "reservoir_clones": 4, "houdayer": args.mode},
        "attempts_per_emcs": att,
        "houdayer_moves_per_s": moves * args.steps / elapsed,
        "one_size_after_the_other": {"value": att * args.steps / (sequential * 1e9),
                                     "ms_per_step": sequential / args.steps * 1e3},
    }


def oracle_threads() -> int:
    import oracle
    return int(oracle._lib().oracle_num_threads())


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="l16_fp32", choices=sorted(inputs.WORKLOADS) + ["mixed"],
                    help="'mixed': L = 8..16 side by side, one graph launch per EMCS")
    ap.add_argument("--mode", default="acu", choices=["acu", "single", "plain"],
                    help="Houdayer all-cluster (paper), single cluster, or plain PT (no Houdayer, no reservoir)")
    ap.add_argument("--update", default="metropolis", choices=["metropolis", "heatbath", "micsa"],
                    help="local update of the PT clones: Metropolis (paper), heat bath, or MicSA (PTHR*)")
    ap.add_argument("--cpu-samples", type=int, default=192)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--compare-fp64-samples", type=int, default=16,
                    help="samples for the unbatched FP64 one-sample-per-launch comparison (0 = skip)")
    ap.add_argument("--shard-samples", type=int, default=128,
                    help="also time one GPU's share of the batch sharded over 8 GPUs (0 = skip)")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--overlap-reservoir", action="store_true",
                    help="reservoir sweeps on a second stream beside the Houdayer step (plain launches)")
    ap.add_argument("--plain-launches", action="store_true", help="time pthr_run as plain launches, no graph")
    ap.add_argument("--no-autotune", action="store_true", help="mixed batch: keep the default schedules")
    ap.add_argument("--split-group-samples", action="store_true",
                    help="mixed batch: keep the sample split the schedules pick for each size alone")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy a MIB-MiB device buffer 3 times (HBM counter calibration)")
    ap.add_argument("--reservoir-decorrelation", action="store_true",
                    help="only measure C(tau) of reservoir clones at T_max (the workload's and 2.0)")
    ap.add_argument("--fp32-vs-fp64", action="store_true",
                    help="only compare the FP32 form with the FP64 form statistically")
    ap.add_argument("--precision-workload", default="l12_fp64", choices=sorted(inputs.WORKLOADS),
                    help="--fp32-vs-fp64: the workload whose shape both forms run")
    ap.add_argument("--samples", type=int, default=512)
    ap.add_argument("--emcs", type=int, default=2048)
    ap.add_argument("--seeds", type=int, default=4, help="--fp32-vs-fp64: independent runs per form")
    args = ap.parse_args()

    if args.reservoir_decorrelation:
        print(json.dumps(reservoir_decorrelation(args)), flush=True)
        return 0
    if args.fp32_vs_fp64:
        print(json.dumps(precision_check(args)), flush=True)
        return 0

    if args.copy_calibration:
        import torch
        n = args.copy_calibration << 20
        src = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_per_copy": n, "copies": 3}), flush=True)
        return 0

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: samples are independent, a multi-GPU run "
              "shards them with no exchange between GPUs; use --gpus 1", file=sys.stderr)
        return 2

    if args.workload == "mixed":
        print(json.dumps(bench_mixed(args)), flush=True)
        return 0

    import torch
    from paper_2605_25872_amd import pthr

    w = inputs.WORKLOADS[args.workload]
    if args.mode == "plain":
        # plain PT: the EMCS without the Houdayer step and the reservoir (paper Sec. 4)
        w = dataclasses.replace(w, n_reservoir=0, t_acu=0.0)
    lib_mode = "single" if args.mode == "single" else "acu"
    T = w.temperatures()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log(f"workload {w.name}: L={w.L} S={w.n_samples} NR={w.n_replicas} NT={w.n_temps} "
        f"NER={w.n_reservoir} {w.precision} {args.mode}")
    g = pthr.Pthr(w.L, w.n_samples, w.n_replicas, w.n_temps, w.n_reservoir, w.sweeps_per_emcs,
                  w.er_sweeps_per_emcs, w.precision, lib_mode, w.t_acu, w.seed, local_update=args.update)
    g.init_samples(w.couplings(), T)
    obs = g.new_obs()
    if args.autotune:
        # time each candidate over >= ~1.5e10 attempts so that small lattices are not timed on one EMCS
        best = g.autotune(max(1, math.ceil(1.5e10 / attempts_per_emcs(w))))
        sch = g.schedule()
        log(f"autotune: {best:.2f} ms/EMCS with {sch.threads_per_sample} work-items per sample, "
            f"clone split {sch.clone_split}, sample split {sch.sample_split}, "
            f"exp early-out below T = {sch.exp_early_out / 1000:g}, reservoir overlap {sch.overlap_reservoir}")
    if args.overlap_reservoir:
        g.set_schedule(overlap_reservoir=1)
    stream = torch.cuda.current_stream(dev)
    n_er = w.er_sweeps_per_emcs if w.n_reservoir else 0
    att = attempts_per_emcs(w)
    moves = moves_per_emcs(w, T)

    # Timed region: the persistent form the L=16 workload names, K EMCS as
    # replays of a captured graph of the phase kernels (pthr_run), with the
    # observables accumulated every EMCS.  The warm-up captures the graph.
    # (the reservoir overlap runs as plain launches)
    window = 0 if args.overlap_reservoir or args.plain_launches else max(1, min(args.steps, 32))
    g.set_schedule(graph_window=window)
    g.run(max(args.warmup, window), obs)
    torch.cuda.synchronize()
    log(f"warm-up done ({max(args.warmup, window)} EMCS, graph of {window} EMCS captured)")
    t0 = time.perf_counter()
    g.run(args.steps, obs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    g.check()
    ms_per_step = elapsed / args.steps * 1e3
    value = att * args.steps / (elapsed * 1e9)
    log(f"timed {args.steps} EMCS ({'graph replays' if window else 'plain launches'}) in {elapsed:.3f} s: "
        f"{value:.1f} attempts/ns")

    # Kernel breakdown: the same EMCS as eager per-phase launches on the same
    # stream, HIP events around the sweep and Houdayer kernels (the sweep's
    # roofline is taken from these launches: the same kernel, launch shape and
    # data as in the graph).
    micsa = args.update == "micsa"

    def step(ev):
        if micsa:
            # PTHR*: MicSA on the PT clones (micsa_kernel), then Metropolis on
            # the reservoir clones (sweep_kernel); the two classes are independent
            ev[4].record(stream)
            g.sweep(w.sweeps_per_emcs, 0)
            ev[0].record(stream)
            g.sweep(0, n_er)
        else:
            ev[0].record(stream)
            g.sweep(w.sweeps_per_emcs, n_er)
        ev[1].record(stream)
        g.houdayer()
        ev[2].record(stream)
        g.pt_swap(True)
        g.measure(obs)
        ev[3].record(stream)

    evs = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(5)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for ev in evs:
        step(ev)
    torch.cuda.synchronize()
    eager_elapsed = time.perf_counter() - t1
    g.check()
    sweep_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
    micsa_ms = float(np.mean([e[4].elapsed_time(e[0]) for e in evs])) if micsa else None
    houdayer_ms = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
    pt_measure_ms = float(np.mean([e[2].elapsed_time(e[3]) for e in evs]))
    log(f"eager per-phase EMCS: {att * args.steps / (eager_elapsed * 1e9):.1f} attempts/ns; "
        f"sweep kernel {sweep_ms:.2f} ms, Houdayer {houdayer_ms:.3f} ms, PT + observables {pt_measure_ms:.3f} ms")

    # the roofline of the Metropolis sweep kernel: all attempts, or with MicSA
    # the reservoir clones' (the PT clones' MicSA kernel is reported beside it)
    rule = "metropolis" if micsa else args.update
    peak_ops, ops_per_attempt = valu_peak(rule, w.precision)
    pt_att = float(w.V * w.sweeps_per_emcs * w.n_replicas * w.n_temps) * w.n_samples
    sweep_att = att - pt_att if micsa else att
    ops = ops_per_attempt * sweep_att
    achieved = ops / (sweep_ms * 1e-3)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "spin-flip attempts/ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if w.precision == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "L": w.L, "samples": w.n_samples, "replicas": w.n_replicas,
                   "temperatures": w.n_temps, "t_range": [w.t_min, w.t_max],
                   "reservoir_clones": w.n_reservoir, "sweeps_per_emcs": w.sweeps_per_emcs,
                   "reservoir_sweeps_per_emcs": w.er_sweeps_per_emcs, "houdayer": args.mode,
                   "local_update": args.update,
                   "threads_per_sample": g.schedule().threads_per_sample,
                   "exp_early_out_below_T": g.schedule().exp_early_out / 1000,
                   "clone_split": g.schedule().clone_split,
                   "sample_split": g.schedule().sample_split,
                   "overlap_reservoir": g.schedule().overlap_reservoir,
                   "timed_form": (f"pthr_run replaying a captured graph of {window} EMCS, observables every EMCS"
                                  if window else "pthr_run as plain launches, observables every EMCS")},
        "houdayer_moves_per_s": moves * args.steps / elapsed,
        "eager_per_phase": {"value": att * args.steps / (eager_elapsed * 1e9),
                            "ms_per_step": eager_elapsed / args.steps * 1e3,
                            "sweep_ms": sweep_ms, "houdayer_ms": houdayer_ms,
                            "pt_and_observables_ms": pt_measure_ms},
        "houdayer_kernel": {"ms_per_launch": houdayer_ms,
                            "moves_per_s": moves / (houdayer_ms * 1e-3) if moves else None,
                            "utilisation": houdayer_utilisation(w.name, args.mode)},
        "attempts_per_emcs": att,
        "wall_time_per_equilibrated_sample_s":
            (elapsed / args.steps) / w.n_samples * T_EQ_EMCS.get(w.L, float("nan")),
        "roofline": {"bound": "alu", "kernel": "sweep_kernel", "achieved": achieved / 1e12,
                     "peak": peak_ops / 1e12, "unit": "TOP/s", "frac": achieved / peak_ops,
                     "traffic": sweep_traffic_bytes(w.name) if args.update == "metropolis" else None,
                     "traffic_unit": "HBM bytes per launch",
                     "ops_per_attempt": ops_per_attempt,
                     "ops_by_issue_class": OPS_BY_CLASS[(rule, w.precision)],
                     "attempts_per_launch": sweep_att,
                     "sweep_ms_per_launch": sweep_ms},
    }
    if micsa:
        out["micsa_kernel"] = {"ms_per_launch": micsa_ms, "attempts_per_launch": pt_att,
                               "attempts_per_ns": pt_att / (micsa_ms * 1e6)}
        log(f"micsa kernel {micsa_ms:.2f} ms per launch: {pt_att / (micsa_ms * 1e6):.1f} attempts/ns")

    if args.shard_samples > 0 and args.shard_samples < w.n_samples:
        # One GPU's share of the batch sharded over 8 GPUs (samples are
        # independent): the first S/8 samples, same form and timing as above.
        n = args.shard_samples
        sub = inputs.Workload(**{**w.__dict__, "n_samples": n})
        h = pthr.Pthr(w.L, n, w.n_replicas, w.n_temps, w.n_reservoir, w.sweeps_per_emcs,
                      w.er_sweeps_per_emcs, w.precision, lib_mode, w.t_acu, w.seed, local_update=args.update)
        h.init_samples(sub.couplings(), T)
        if args.autotune:
            h.autotune(max(1, math.ceil(1.5e10 / attempts_per_emcs(sub))))
        h.set_schedule(graph_window=window)
        hobs = h.new_obs()
        h.run(max(args.warmup, window), hobs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        h.run(args.steps, hobs)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        h.check()
        sch = h.schedule()
        out["per_gpu_shard"] = {
            "samples": n, "value": attempts_per_emcs(sub) * args.steps / (dt * 1e9),
            "unit": "spin-flip attempts/ns", "ms_per_step": dt / args.steps * 1e3,
            "threads_per_sample": sch.threads_per_sample, "clone_split": sch.clone_split,
            "sample_split": sch.sample_split}
        log(f"per-GPU shard of {n} samples: {out['per_gpu_shard']['value']:.1f} attempts/ns")
        del h

    if args.compare_fp64_samples > 0:
        n = min(args.compare_fp64_samples, w.n_samples)
        sub = inputs.Workload(**{**w.__dict__, "n_samples": n, "precision": "fp64"})
        h = pthr.Pthr(w.L, n, w.n_replicas, w.n_temps, w.n_reservoir, w.sweeps_per_emcs,
                      w.er_sweeps_per_emcs, "fp64", lib_mode, w.t_acu, w.seed, local_update=args.update)
        h.init_samples(sub.couplings(), T)
        h.set_schedule(samples_per_launch=1)
        hobs = h.new_obs()
        h.run(1, hobs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        h.run(1, hobs)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t1
        out["fp64_one_sample_per_launch"] = {
            "value": attempts_per_emcs(sub) / (dt * 1e9), "unit": "spin-flip attempts/ns",
            "samples": n, "emcs": 1,
            "houdayer_moves_per_s": moves_per_emcs(sub, T) / dt}
        out["speedup_vs_fp64_one_sample_per_launch"] = value / out["fp64_one_sample_per_launch"]["value"]
        log(f"fp64 one-sample-per-launch: {out['fp64_one_sample_per_launch']['value']:.2f} attempts/ns")

    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on {args.cpu_samples} samples x 1 EMCS")
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_samples, args.mode, args.update)
        log(f"cpu baseline: {out['cpu_baseline']['value']:.4f} attempts/ns "
            f"on {out['cpu_baseline']['cores']} threads")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
