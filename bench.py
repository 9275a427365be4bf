"""Throughput of the matrix-element hot path on one MI355X.

One step = one pass of the whole hot path over one batch of synthetic
events: RAMBO phase space (Philox4x32-10 counters, flat, no cuts) written to
device memory, then |M|^2 summed over the good helicities and all colours.
The default workload is g g -> t t~ g g at sqrt(s) = 1500 GeV, 524288
events per batch, FP64 (the paper's standalone double-precision
configuration with a grid of 524288 events).

Prints one JSON line.  `value` is events per second over the timed steps;
`roofline` is measured live with HIP events around every matrix-element
launch on the stream it runs on; `cpu_baseline` times the oracle on a
bounded sample of the same events on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (pdg key, events per batch, sqrt(s) GeV)
    "gg_ttgg": ("gg_ttgg", 524288, 1500.0),
    "gg_ttggg": ("gg_ttggg", 65536, 1500.0),
    "gg_ttg": ("gg_ttg", 65536, 1500.0),
    "gg_tt": ("gg_tt", 524288, 1500.0),
    "ee_mumu": ("ee_mumu", 16384, 500.0),
}
SEED = 230318244
FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 78.6   # the same lanes without packed FP32 instructions
# HBM traffic of the dominant kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE
# runs (KiB per dispatch), valid only for the kernels identified by
# kernel_hash; each counter is scaled by what it reads for a plain
# device-to-device copy of known size (FETCH_SIZE reports half the bytes
# read on this GPU, WRITE_SIZE all of them).
TRAFFIC = {
    ("gg_ttgg", "fp64"): {"kernel_hash": 928121246631932704, "fetch_kib": 51787.6, "write_kib": 4096.0,
                     "fetch_scale": 2.0, "write_scale": 1.0},
}
# The paper's standalone CUDA throughput on one V100 for this workload
# (g g -> t t~ g g, double, grid 524288): 4.21E5 MEs/s.
PAPER_MES = {("gg_ttgg", 0): 4.21e5, ("gg_ttgg", 1): 8.77e5}


def cpu_baseline(name: str, n_events: int, mom_host, me_gpu=None, result=None, seconds: float = 12.0):
    """Oracle MEs/s on the host cores, on the leading events of the batch.
    The oracle's values on that sample also give the error of the GPU
    result `me_gpu` (stored in result["vs_oracle"])."""
    import numpy as np

    import oracle

    P = oracle.Process(oracle.PROCESSES[name])
    threads = max(1, min(16, os.cpu_count() or 1))
    # size the sample from a short probe so that it takes about `seconds`
    probe = mom_host[: 2 * threads]
    t0 = time.perf_counter()
    P.me(probe, nthreads=threads)
    per_event = (time.perf_counter() - t0) / len(probe)
    n = int(min(len(mom_host), max(len(probe), seconds / max(per_event, 1e-9))))
    t0 = time.perf_counter()
    ref = P.me(mom_host[:n], nthreads=threads)
    wall = time.perf_counter() - t0
    if me_gpu is not None and result is not None:
        rel = np.abs(me_gpu[:n] - ref) / np.abs(ref)
        result["vs_oracle"] = {"events": n, "rel_err_median": float(np.median(rel)),
                               "rel_err_p99": float(np.quantile(rel, 0.99)), "rel_err_max": float(rel.max()),
                               "batch_mean_rel": float(abs(me_gpu[:n].sum() / ref.sum() - 1.0))}
    return {"value": n / wall, "unit": "MEs/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} of the {n_events} benchmark events, all helicities, FP64, "
                      f"{threads} threads, {wall:.1f} s wall"}


def serve_bench(n_requests: int, rho: float, slots: int, seed: int = 7) -> dict:
    """Serving mix: requests for g g -> t t~ (+0..3 g), log-uniform batch
    sizes 1024..524288 events, FP64 or mixed precision with equal odds,
    Poisson arrivals at rho times the capacity measured by running the same
    requests one at a time.  Returns latency percentiles and throughput."""
    import numpy as np
    import torch

    import paper_2303_18244_amd as M

    rng = np.random.default_rng(seed)
    names = ["gg_tt", "gg_ttg", "gg_ttgg", "gg_ttggg"]
    procs = {n: M.Process(M.PROCESSES[n]) for n in names}
    plan = []
    for k in range(n_requests):
        name = names[rng.integers(len(names))]
        n = int(np.exp(rng.uniform(np.log(1024), np.log(524288))))
        prec = M.FP64 if rng.random() < 0.5 else M.MIXED
        plan.append((name, n, prec))
    moms = []
    for k, (name, n, prec) in enumerate(plan):
        mom, _ = procs[name].rambo(1500.0, SEED, k << 20, n)  # request k: events of its own counter range
        moms.append(mom)
    outs = [torch.empty(n, dtype=torch.float64, device="cuda") for _, n, _ in plan]
    torch.cuda.synchronize()
    # capacity: the same requests back to back, one at a time
    alone_ms = []
    for (name, n, prec), mom, out in zip(plan, moms, outs):
        t0 = time.perf_counter()
        procs[name].matrix_element(mom, precision=prec, out=out)
        torch.cuda.synchronize()
        alone_ms.append((time.perf_counter() - t0) * 1e3)
    mean_service = float(np.mean(alone_ms)) * 1e-3
    rate = rho / mean_service
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    S = M.Server(n_slots=slots, hbm_budget_bytes=48 << 30)
    t0 = time.perf_counter()
    due = t0
    ids = []
    for (name, n, prec), mom, out, gap in zip(plan, moms, outs, gaps):
        due += gap
        while time.perf_counter() < due:
            time.sleep(min(0.001, max(0.0, due - time.perf_counter())))
        ids.append(S.submit(procs[name], mom, precision=prec, out=out))
    for i in ids:
        S.wait(i)
    wall = time.perf_counter() - t0
    st = S.stats()
    S.close()
    events = sum(n for _, n, _ in plan)
    return {"metric": "serving mix: latency p50/p99 and MEs/s", "value": events / st["wall_s"],
            "unit": "MEs/s", "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"], "mean_ms": st["mean_ms"],
            "max_ms": st["max_ms"], "requests": n_requests, "events": events, "offered_load": rho,
            "slots": slots, "max_concurrent": st["max_concurrent"],
            "alone_p50_ms": float(np.median(alone_ms)), "alone_p99_ms": float(np.quantile(alone_ms, 0.99)),
            "alone_mes_per_s": events / (sum(alone_ms) * 1e-3), "wall_s": wall,
            "config": {"workload": "serving mix gg->tt+0..3g, sizes log-uniform 1024..524288, FP64/mixed 50/50",
                       "arrivals": f"Poisson, rate {rate:.2f}/s", "seed": seed},
            "data": "synthetic (RAMBO flat phase space)"}


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="gg_ttgg", choices=list(WORKLOADS))
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32", "mixed", "fp64_fp32colour"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serve", type=int, default=0, metavar="N",
                    help="instead of the benchmark, run the serving mix with N requests")
    ap.add_argument("--rho", type=float, default=0.8)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="instead of the benchmark, time a plain device-to-device copy of this many bytes "
                         "(the reference kernel for scaling the FETCH_SIZE / WRITE_SIZE counters)")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported (events are independent, "
              f"so N GPUs would each run this batch on their own share).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if a.serve:
        print(json.dumps(serve_bench(a.serve, a.rho, a.slots)), flush=True)
        return 0

    if a.copy_bytes:
        n = a.copy_bytes // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            dst.copy_(src)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / a.steps
        print(json.dumps({"copy_bytes": n * 8, "ms_per_copy": dt * 1e3, "GB_per_s": 2 * n * 8 / dt * 1e-9}))
        return 0

    import paper_2303_18244_amd as M

    key, nevt, sqrt_s = WORKLOADS[a.workload]
    prec = {"fp64": M.FP64, "fp32": M.FP32, "mixed": M.MIXED, "fp64_fp32colour": M.FP64_FP32COLOUR}[a.precision]
    P = M.Process(M.PROCESSES[key])
    info = P.info
    dev = torch.device("cuda", 0)
    mom = torch.empty((P.n_ext, 4, nevt), dtype=torch.float64, device=dev)
    wgt = torch.empty(nevt, dtype=torch.float64, device=dev)
    me = torch.empty(nevt, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    def step(i, ev=None):
        P.rambo(sqrt_s, SEED, i * nevt, nevt, mom=mom, wgt=wgt)
        if ev is not None:
            ev[0].record(stream)
        P.matrix_element(mom, precision=prec, out=me)
        if ev is not None:
            ev[1].record(stream)

    for i in range(a.warmup):
        step(i)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(a.steps)]
    t0 = time.perf_counter()
    for i in range(a.steps):
        step(a.warmup + i, evs[i])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    me_ms = sum(e0.elapsed_time(e1) for e0, e1 in evs) / a.steps
    ms_per_step = wall * 1e3 / a.steps
    value = nevt / (ms_per_step * 1e-3)
    ngood = info["n_good_hel"]
    flops = (info["flops_per_hel"] * ngood + info["flops_per_event"]) * nevt
    achieved = flops / (me_ms * 1e-3) * 1e-12
    peak = FP64_VALU_PEAK_TFLOPS if prec in (M.FP64, M.FP64_FP32COLOUR) else FP32_VALU_PEAK_TFLOPS
    tr = TRAFFIC.get((key, a.precision))
    traffic = None
    if tr is not None and tr["kernel_hash"] == info["kernel_hash"]:
        traffic = (tr["fetch_kib"] * tr["fetch_scale"] + tr["write_kib"] * tr["write_scale"]) * 1024.0
    assert bool(torch.isfinite(me).all()), "non-finite matrix element"

    result = {
        "metric": "MEs/s (tree-level |M|^2 summed over helicities and colours, RAMBO + ME per batch)",
        "value": value,
        "unit": "MEs/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": (value / PAPER_MES[(key, prec)]) if (key, prec) in PAPER_MES else None,
        "dtype": {M.FP64: "f64", M.FP32: "f32", M.MIXED: "f32+f16", M.FP64_FP32COLOUR: "f64+f32"}[prec],
        "data": "synthetic (RAMBO flat phase space, Philox seed 230318244)",
        "config": {"workload": key, "events_per_batch": nevt, "sqrt_s_gev": sqrt_s,
                   "precision": a.precision, "good_helicities": ngood, "diagrams": info["n_diagrams"],
                   "colour_flows": info["n_colour"], "kernel_hash": str(info["kernel_hash"])},
        "me_only": {"ms_per_launch": me_ms, "mes_per_s": nevt / (me_ms * 1e-3)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "kernel": f"me_kernel<{'double' if prec == M.FP64 else 'float'}> ({key}, {a.precision})",
                     "flops_per_launch": flops},
    }
    if info["n_colour"] > 24 or prec != M.FP64:
        result["roofline"]["kernel"] = (f"every kernel of one mgme_matrix_element call ({key}, {a.precision}): "
                                        "diagram kernels, colour sum and helicity sum, timed together")
    if prec != M.FP64:
        # accuracy and speed against plain FP64 on the same GPU and the same events
        me64 = torch.empty_like(me)
        P.matrix_element(mom, precision=M.FP64, out=me64)
        torch.cuda.synchronize()
        e64 = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
        for e0, e1 in e64:
            e0.record(stream)
            P.matrix_element(mom, precision=M.FP64, out=me64)
            e1.record(stream)
        torch.cuda.synchronize()
        ms64 = sum(e0.elapsed_time(e1) for e0, e1 in e64) / len(e64)
        rel = ((me - me64).abs() / me64.abs()).cpu().numpy()
        result["vs_fp64_same_gpu"] = {
            "fp64_me_ms_per_launch": ms64, "speedup_me_only": ms64 / me_ms,
            "rel_err_median": float(np.median(rel)), "rel_err_p99": float(np.quantile(rel, 0.99)),
            "rel_err_max": float(rel.max()),
            "batch_mean_rel": float(abs(me.sum().item() / me64.sum().item() - 1.0)), "events": nevt}
    if not a.no_cpu_baseline:
        host = mom.cpu().numpy().transpose(2, 0, 1)
        host = np.ascontiguousarray(host[:65536])
        result["cpu_baseline"] = cpu_baseline(key, nevt, host, me.cpu().numpy(), result)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
