"""Throughput benchmark of the jump-SDE proton dose path on one MI355X.

One step = one pass of the whole hot path over the 150 MeV water workload
(1e7 histories, 1 % energy spread, 3 mm lateral spread, water 200 x 200 x 300
mm at 1 mm voxels): tally reset, the persistent transport launch (source
sampling, Euler-Maruyama stepping with jumps, int64 fixed-point scoring) and
the FP64 dose conversion.  Inputs (tables, packed phantom, spot table) are
resident in HBM before the timed region.

Prints one JSON line.  ``--gpus`` above 1 is refused: this build measures one
GPU (the multi-GPU reduction is a design note only).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "proton histories/s @150 MeV water; time-to-gamma≥95% denoised vs plain"
# MI355X issue capacity for non-packed 32-bit VALU work: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz, in lane-operations per second.
VALU_PEAK = 256 * 4 * 16 * 2.4e9
# VALU instruction slots of one straight-line Euler-Maruyama step of the
# transport kernel (no jump, refill or end-of-range), counted from the gfx950
# ISA of the step body with quarter-rate instructions weighted by 4; see the
# design notes.  Used as the algorithmic work per step.
STEP_SLOTS = 262


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--histories", type=int, default=10_000_000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target duration of the oracle CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", type=str, default="", help="JSON launch overrides")
    return ap.parse_args()


def cpu_baseline(wl, target_s: float) -> dict:
    """The FP64 oracle, as it stands, on a bounded prefix of the same histories."""
    import oracle
    import workloads
    nuc = workloads.nuclear_for_phantom(wl.phantom, wl.params.lattice())
    threads = oracle.n_threads_default()
    n = 2000
    t0 = time.perf_counter()
    oracle.transport(wl.phantom, wl.spots, wl.params, nuc, seed=wl.seed, h_begin=0, h_end=n,
                     n_threads=threads)
    dt = time.perf_counter() - t0
    n2 = int(min(wl.n_histories, max(n, n * target_s / max(dt, 1e-3))))
    t0 = time.perf_counter()
    oracle.transport(wl.phantom, wl.spots, wl.params, nuc, seed=wl.seed, h_begin=0, h_end=n2,
                     n_threads=threads)
    dt2 = time.perf_counter() - t0
    return {"value": n2 / dt2, "unit": "histories/s", "cores": threads, "kind": "oracle",
            "sample": f"histories 0..{n2} of the same workload (FP64, {threads} threads, "
                      f"{dt2:.1f} s)"}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {a.gpus} is not supported by this build "
              "(the multi-GPU path is a design note: shard histories, all-reduce the int64 tally)",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2511_03115_amd import sde
    import workloads
    from workloads import configs

    wl = configs.water150(n=a.histories)
    launch = json.loads(a.launch) if a.launch else None
    print(f"[bench] workload {wl.name} n={wl.n_histories} shape={wl.phantom.shape}", flush=True)
    stream = torch.cuda.Stream()
    sde.set_stream(stream)
    sde.init_materials(wl.phantom.materials, wl.params,
                       workloads.nuclear_for_phantom(wl.phantom, wl.params.lattice()))
    dph = sde.DevicePhantom.from_host(wl.phantom)
    plan = sde.Plan(wl.spots, dph, wl.seed, launch=launch)
    dose = torch.zeros(wl.phantom.material_id.shape, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    for i in range(a.warmup):
        plan.execute(dose)
        stream.synchronize()
        print(f"[bench] warmup {i} kernel {plan.kernel_ms():.1f} ms", flush=True)

    kern = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        plan.execute(dose)
        kern.append(plan.kernel_ms())      # waits for this step's transport kernel
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ledger, scale = plan.results()
    steps_per_launch = int(ledger[sde.LEDGER_STEPS])
    n = wl.n_histories
    ms_step = wall / a.steps * 1e3
    kms = float(np.mean(kern))
    achieved = STEP_SLOTS * steps_per_launch / (kms * 1e-3)
    print(f"[bench] step {ms_step:.2f} ms, kernel {kms:.2f} ms, steps/launch {steps_per_launch}, "
          f"jumps {int(ledger[sde.LEDGER_JUMPS])}", flush=True)
    out = {
        "metric": METRIC, "value": n / (ms_step * 1e-3), "unit": "histories/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "water150: 150 MeV proton pencil beam, 1% Gaussian energy "
                               "spread, 3 mm Gaussian lateral spread, 1e7 histories, water "
                               "200x200x300 mm at 1 mm voxels, FP32 stepping, int64 tally",
                   "histories": n, "seed": wl.seed, "launch": launch or "default"},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK,
                     "unit": "lane-op/s", "frac": achieved / VALU_PEAK, "traffic": None,
                     "kernel": "k_transport", "kernel_ms": kms,
                     "work_per_unit": f"{STEP_SLOTS} VALU slots per step",
                     "units_per_launch": steps_per_launch},
    }
    if not a.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, a.cpu_seconds)
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
