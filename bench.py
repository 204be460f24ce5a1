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
# MI355X issue capacity for full-rate 32-bit VALU work: 256 CUs x 4 SIMDs x
# 16 lanes x 2.4 GHz, in lane-operations per second.
VALU_PEAK = 256 * 4 * 16 * 2.4e9
# Algorithmic work of one Euler-Maruyama step in full-rate VALU issue slots:
# the straight path of a step (voxel and table lookup, one Philox4x32-10
# block, Bethe loss, straggling, jump test, midpoint deposit, move,
# Lynch-Dahl width and the spherical Brownian motion turn at small t,
# renormalisation), counted operation by operation: 244 full-rate
# operations, 18 transcendentals (log, rcp, rsq, sqrt, sin, cos), weighted 2
# (gfx950's transcendental unit issues 8 lanes per SIMD per clock), and the
# Philox round's 20 32x32->64 products, weighted 1 (v_mad_u64_u32 issues at
# the full rate).  The microbenchmarks below measure both weights.  The
# breakdown is in the design notes.
STEP_FULL, STEP_TRANS, STEP_MUL64 = 244, 18, 20
TRANS_WEIGHT, MUL64_WEIGHT = 2, 1
STEP_SLOTS = STEP_FULL + TRANS_WEIGHT * STEP_TRANS + MUL64_WEIGHT * STEP_MUL64   # 300
# global int64 atomics per launch of the water workload (rocprofv3
# TCC_ATOMIC_sum of the committed counter summary), for the atomic roof
ATOMICS_FILE = os.path.join(ROOT, "profiles", "k_transport_water150_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_2511_03115_amd", "csrc", "sde_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_transport_water150_traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--histories", type=int, default=10_000_000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target duration of the oracle CPU-baseline sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plan", action="store_true",
                    help="skip the batched-plan leg (1000 spots, hipGraph replay)")
    ap.add_argument("--launch", type=str, default="auto",
                    help="'auto' (autotuner), 'default', or a JSON launch configuration")
    ap.add_argument("--no-gamma", action="store_true",
                    help="skip the time-to-gamma leg (plain SDE vs denoised, plan at 2 mm)")
    ap.add_argument("--no-hetero", action="store_true",
                    help="skip the heterogeneous-phantom leg (slab and insert, 100/150 MeV)")
    ap.add_argument("--no-roofs", action="store_true",
                    help="skip the microbenchmarks of the transport's ingredients")
    ap.add_argument("--no-geodesic", action="store_true",
                    help="skip the leg timing the geodesic Gaussian small-angle step")
    return ap.parse_args()


def cpu_baseline(wl, target_s: float) -> dict:
    """The FP64 oracle, as it stands, on a bounded prefix of the same histories."""
    import oracle
    import workloads
    nuc = workloads.nuclear_for_phantom(wl.phantom, wl.params.lattice())
    threads = oracle.n_threads_default()
    # calibrate on two sizes so the fixed set-up cost (tables, per-thread
    # tallies) is not mistaken for per-history work
    times = []
    for n in (2000, 20000):
        t0 = time.perf_counter()
        oracle.transport(wl.phantom, wl.spots, wl.params, nuc, seed=wl.seed, h_begin=0,
                         h_end=n, n_threads=threads)
        times.append(time.perf_counter() - t0)
    per_h = max((times[1] - times[0]) / 18000.0, 1e-7)
    fixed = max(times[0] - 2000 * per_h, 0.0)
    n2 = int(min(wl.n_histories, max(20000, (target_s - fixed) / per_h)))
    # the first n2 histories as a workload of their own (same Philox words,
    # weights per n2), so the GPU can run exactly the same sample
    spots2 = workloads.with_histories(wl.spots, n2)
    t0 = time.perf_counter()
    r2 = oracle.transport(wl.phantom, spots2, wl.params, nuc, seed=wl.seed, n_threads=threads)
    dt2 = time.perf_counter() - t0
    # one thread, as the paper times its own implementation: a smaller prefix
    n1 = int(min(n2, max(1000, 3.0 / (per_h * threads))))
    t0 = time.perf_counter()
    oracle.transport(wl.phantom, wl.spots, wl.params, nuc, seed=wl.seed, h_begin=0, h_end=n1,
                     n_threads=1)
    dt1 = time.perf_counter() - t0
    return {"value": n2 / dt2, "unit": "histories/s", "cores": threads, "kind": "oracle",
            "sample": f"histories 0..{n2} of the same workload (FP64, {threads} threads, "
                      f"{dt2:.1f} s)",
            "value_1thread": n1 / dt1,
            "sample_1thread": f"histories 0..{n1} (FP64, 1 thread, {dt1:.1f} s)",
            "cpu": cpu_model(),
            "parity": oracle_parity(wl, spots2, n2, oracle.dose(r2.edep, wl.phantom))}


def oracle_parity(wl, spots, n, d_ref) -> dict:
    """The GPU path on the oracle's sample (the same n histories): per-voxel
    difference over the maximum, gamma 1 %/0.5 mm (local, 1 % threshold) and
    the R80 difference, the workloads' parity measures."""
    import numpy as np
    import torch
    import oracle
    import workloads
    from paper_2511_03115_amd import sde
    sde.init_materials(wl.phantom.materials, wl.params,
                       workloads.nuclear_for_phantom(wl.phantom, wl.params.lattice()))
    dph = sde.DevicePhantom.from_host(wl.phantom)
    dose = torch.zeros(wl.phantom.material_id.shape, dtype=torch.float64, device="cuda")
    sde.transport(spots, dph, wl.seed, dose_out=dose)
    torch.cuda.synchronize()
    d = dose.cpu().numpy()
    g, _, _ = sde.gamma(torch.from_numpy(np.ascontiguousarray(d_ref)).cuda(), dose,
                        wl.phantom.voxel_cm, 0.01, 0.05, 0.01, 10, True)
    dz = wl.phantom.voxel_cm[2]
    return {"histories": int(n), "max_rel_diff": float(np.abs(d - d_ref).max() / d_ref.max()),
            "gamma_1pct_05mm": float(g),
            "dr80_mm": float(abs(oracle.range_rx(d_ref, dz) - oracle.range_rx(d, dz)) * 10)}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def measured_traffic(launch, histories):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, if it was taken on the current kernel source, launch and size."""
    import hashlib
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if t.get("kernel_sha256") != src or t.get("histories") != histories or \
            t.get("launch") != launch:
        return None
    return t.get("bytes_per_launch")


def measured_atomics(launch, histories):
    """Global int64 atomics per launch (rocprofv3 TCC_ATOMIC_sum) from the
    committed counter summary, if taken on the current kernel source, launch
    and size."""
    import hashlib
    try:
        t = json.load(open(ATOMICS_FILE))
    except (OSError, ValueError):
        return None
    src = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if t.get("kernel_sha256") != src or t.get("histories") != histories or \
            t.get("launch") != launch:
        return None
    return t.get("tcc_atomic_per_launch")


def plan_leg(steps: int, stream) -> dict:
    """The batched plan: 1000 spots (70-230 MeV, lognormal weights, 1e3-1e5
    histories each) on a 256x256x200 random-density phantom at 2 mm, one
    persistent launch per execution, replayed from a hipGraph."""
    import numpy as np
    import torch
    import workloads
    from workloads import configs
    from paper_2511_03115_amd import autotune, sde
    wl = configs.plan()
    print(f"[bench] plan n={wl.n_histories} spots={len(wl.spots)}", flush=True)
    sde.init_materials(wl.phantom.materials, wl.params,
                       workloads.nuclear_for_phantom(wl.phantom, wl.params.lattice()))
    dph = sde.DevicePhantom.from_host(wl.phantom)
    launch = autotune.tune(wl.spots, dph, wl.seed)
    plan = sde.Plan(wl.spots, dph, wl.seed, launch=launch)
    dose = torch.zeros(wl.phantom.material_id.shape, dtype=torch.float64, device="cuda")
    plan.execute(dose, use_graph=True)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    times = []
    for _ in range(max(1, steps)):
        ev0.record(stream)           # the library's stream
        plan.execute(dose, use_graph=True)
        ev1.record(stream)
        ev1.synchronize()
        times.append(ev0.elapsed_time(ev1))
    led, _ = plan.results()
    plan.close()
    ms = float(np.mean(times))
    print(f"[bench] plan {ms:.2f} ms per execution", flush=True)
    return {"workload": "plan: 1000 spots 70-230 MeV, lognormal weights, 1e3-1e5 histories "
                        "per spot, 256x256x200 at 2 mm, random density + bone/lung ellipsoids",
            "histories": int(wl.n_histories), "ms_per_execution": ms,
            "histories_per_s": wl.n_histories / (ms * 1e-3), "hipgraph": True,
            "steps_per_execution": int(led[sde.LEDGER_STEPS]), "launch": launch}


WEIGHTS = os.path.join(ROOT, "paper_2511_03115_amd", "weights", "denoiser_plan2mm.npz")
BF16_PEAK = 2.5e15       # MI355X dense bf16 matrix-core peak, FLOP/s
GAMMA_LADDER = [1000 * 2 ** k for k in range(9)]        # histories per spot
GAMMA_REFERENCE = 2_000_000                              # histories per spot


def gamma_leg() -> dict:
    """Wall time to a dose with gamma >= 95 % (local 2 %/0.5 mm, 1 % threshold)
    against a 2e6-histories-per-spot reference, on the batched plan (1000
    spots, 2 mm): plain SDE on a doubling ladder of histories per spot vs
    the denoised 1e3-per-spot run with the plain fallback."""
    from dataclasses import replace
    import numpy as np
    import workloads
    from workloads import configs
    from paper_2511_03115_amd import denoiser, judge, sde
    wl = configs.plan_uniform(1000)
    sde.init_materials(wl.phantom.materials, wl.params,
                       workloads.nuclear_for_phantom(wl.phantom, wl.params.lattice()))
    dph = sde.DevicePhantom.from_host(wl.phantom)
    dn = denoiser.Denoiser(WEIGHTS, wl.phantom.material_id.shape)
    log = lambda m: print(m, flush=True)
    from paper_2511_03115_amd import autotune
    launch = autotune.tune(wl.spots, dph, wl.seed)     # the same launch for every run
    res = judge.time_to_gamma(lambda n: [replace(sp, n_histories=n) for sp in wl.spots], dph,
                              wl.seed, GAMMA_LADDER, GAMMA_REFERENCE, denoise=dn,
                              name="plan", launch=launch, log=log)
    dn.close()
    out = res.as_dict()
    # the denoiser's forward pass against the dense bf16 matrix-core peak
    m = 1 << (denoiser.LEVELS - 1)
    padded = [-(-n // m) * m for n in wl.phantom.material_id.shape]
    # FLOPs of the sums the network has: the first conv over its 2 used input
    # channels (the nominal count, with all 16, is given beside it)
    flops = denoiser.forward_flops(padded, used_in=2)
    nominal = denoiser.forward_flops(padded)
    nvox = int(np.prod(padded))
    t_dn = [r.denoise_gpu_s for r in res.rungs if r.denoise_gpu_s]
    w_dn = [r.denoise_s for r in res.rungs if r.denoise_s]
    if t_dn:
        # the whole pass between HIP events on the library stream (the
        # denoiser's kernels and the gaps between them), as the transport's
        # kernel time is taken; the host-inclusive wall time beside it
        t = sum(t_dn) / len(t_dn)
        out["denoiser_roofline"] = {
            "bound": "mfma", "achieved": flops / t, "peak": BF16_PEAK, "unit": "FLOP/s",
            "frac": flops / t / BF16_PEAK, "traffic": None,
            "kernel": "denoiser forward (14 bf16 MFMA convs + layout kernels, whole pass)",
            "ms": t * 1e3, "wall_ms": sum(w_dn) / len(w_dn) * 1e3,
            "work_per_unit": f"{flops // nvox} FLOP per voxel",
            "units_per_launch": nvox, "frac_nominal_16_input_channels": nominal / t / BF16_PEAK}
    out["workload"] = ("plan: 1000 spots 70-230 MeV, lognormal weights, equal histories per "
                       "spot, 256x256x200 at 2 mm, random density + bone/lung ellipsoids")
    out["launch"] = launch
    out["gamma"] = {"dd": judge.DD, "dta_cm": judge.DTA_CM, "threshold": judge.THRESH,
                    "local": True, "target": judge.TARGET}
    return out


def hetero_leg(steps: int) -> list:
    """Throughput on the heterogeneous phantoms: water/bone/lung slabs, the
    lateral bone insert and the CT-like head (bone shell, air cavity), 200
    mm cubes at 1 mm, 1e7 histories at 100 and 150 MeV (the same beam model
    as the water workload); and a spread-out Bragg peak plan in water."""
    import numpy as np
    import workloads
    from workloads import configs
    from paper_2511_03115_amd import autotune, sde
    out = []
    make = {"slab": configs.slab, "insert": configs.insert, "ct": configs.ct_like}
    for kind in ("slab", "insert", "ct"):
        for E in (100.0, 150.0):
            wl = make[kind](E)
            sde.init_materials(wl.phantom.materials, wl.params,
                               workloads.nuclear_for_phantom(wl.phantom, wl.params.lattice()))
            dph = sde.DevicePhantom.from_host(wl.phantom)
            launch = autotune.tune(wl.spots, dph, wl.seed)
            plan = sde.Plan(wl.spots, dph, wl.seed, launch=launch)
            plan.execute(None)
            ms = []
            for _ in range(max(1, steps)):
                plan.execute(None)
                ms.append(plan.kernel_ms())
            led, _ = plan.results()
            plan.close()
            k = float(np.mean(ms))
            print(f"[bench] {wl.name}: {k:.2f} ms per launch", flush=True)
            out.append({"workload": f"{kind} {E:.0f} MeV, 1e7 histories, 200 mm cube at 1 mm",
                        "kernel_ms": k, "histories_per_s": wl.n_histories / (k * 1e-3),
                        "steps_per_launch": int(led[sde.LEDGER_STEPS]),
                        "jumps_per_launch": int(led[sde.LEDGER_JUMPS]), "launch": launch})
    # a spread-out Bragg peak plan: 11 layers (87-117 MeV) x 25 spots, 5.5e6 histories
    wl = configs.sobp(n=5_500_000)
    sde.init_materials(wl.phantom.materials, wl.params,
                       workloads.nuclear_for_phantom(wl.phantom, wl.params.lattice()))
    dph = sde.DevicePhantom.from_host(wl.phantom)
    launch = autotune.tune(wl.spots, dph, wl.seed)
    plan = sde.Plan(wl.spots, dph, wl.seed, launch=launch)
    plan.execute(None)
    ms = []
    for _ in range(max(1, steps)):
        plan.execute(None)
        ms.append(plan.kernel_ms())
    led, _ = plan.results()
    plan.close()
    k = float(np.mean(ms))
    print(f"[bench] sobp: {k:.2f} ms per launch", flush=True)
    out.append({"workload": "sobp: 11 layers (6-10 cm peaks, 87-117 MeV) x 5x5 spots, 5.5e6 "
                            "histories shared like the layer weights, water 80x80x150 mm at 1 mm",
                "kernel_ms": k, "histories_per_s": wl.n_histories / (k * 1e-3),
                "steps_per_launch": int(led[sde.LEDGER_STEPS]),
                "jumps_per_launch": int(led[sde.LEDGER_JUMPS]), "launch": launch})
    return out


def geodesic_leg(wl, launch, steps: int, kms_method: float) -> dict:
    """The water workload with the small-angle diffusion drawn by the
    geodesic Gaussian step instead of the spherical Brownian motion law (the
    switch SBM off), same launch, timed per launch like the main leg."""
    from dataclasses import replace
    import numpy as np
    import workloads
    from paper_2511_03115_amd import sde
    params = replace(wl.params, flags=sde.ALL & ~sde.SBM)
    sde.init_materials(wl.phantom.materials, params,
                       workloads.nuclear_for_phantom(wl.phantom, params.lattice()))
    dph = sde.DevicePhantom.from_host(wl.phantom)
    plan = sde.Plan(wl.spots, dph, wl.seed, launch=launch)
    plan.execute(None)
    ms = []
    for _ in range(max(1, steps)):
        plan.execute(None)
        ms.append(plan.kernel_ms())
    led, _ = plan.results()
    plan.close()
    k = float(np.mean(ms))
    print(f"[bench] water150 with the geodesic Gaussian step: {k:.2f} ms per launch", flush=True)
    return {"workload": "water150 (the main workload), small-angle diffusion by the geodesic "
                        "Gaussian step", "flags": int(params.flags), "kernel_ms": k,
            "histories_per_s": wl.n_histories / (k * 1e-3),
            "steps_per_launch": int(led[sde.LEDGER_STEPS]),
            "time_vs_method": k / kms_method}


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
    print(f"[bench] workload {wl.name} n={wl.n_histories} shape={wl.phantom.shape}", flush=True)
    stream = torch.cuda.Stream()
    sde.set_stream(stream)
    sde.init_materials(wl.phantom.materials, wl.params,
                       workloads.nuclear_for_phantom(wl.phantom, wl.params.lattice()))
    dph = sde.DevicePhantom.from_host(wl.phantom)
    if a.launch == "auto":
        from paper_2511_03115_amd import autotune
        launch = autotune.tune(wl.spots, dph, wl.seed, verbose=True)
    elif a.launch == "default":
        launch = None
    else:
        launch = json.loads(a.launch)
    print(f"[bench] launch {json.dumps(launch)}", flush=True)
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
                     "unit": "lane-op/s", "frac": achieved / VALU_PEAK,
                     "traffic": measured_traffic(launch, n),
                     "kernel": "k_transport", "kernel_ms": kms,
                     "work_per_unit": f"{STEP_SLOTS} VALU slots per step",
                     "units_per_launch": steps_per_launch},
    }
    plan.close()
    if not a.no_roofs:
        # the transport's ingredients timed alone: the measured FMA issue
        # rate beside the derived peak, the quarter-rate weights and the
        # atomic and HBM ceilings
        print("[bench] microbenchmarks (VALU, atomics, HBM)", flush=True)
        from paper_2511_03115_amd import roofs
        n_cu = torch.cuda.get_device_properties(0).multi_processor_count
        out["roofs"] = roofs.measure_roofs(n_cu)
        pm = out["roofs"]["fma_lane_ops_s"]
        out["roofline"]["peak_measured"] = pm
        out["roofline"]["frac_measured"] = achieved / pm
        out["roofline"]["weights_measured"] = {
            "transcendental": min(out["roofs"][f"{k}_slots"] for k in roofs.TRANS_NAMES),
            "mul64": out["roofs"]["mul64_slots"]}
        # the second roof: the tally's global int64 atomics against the
        # measured random-address atomic rate
        atom = measured_atomics(launch, n)
        if atom:
            rate = atom / (kms * 1e-3)
            top = out["roofs"]["global_atomic64_random_2MiB_per_s"]
            out["roofline"]["atomics"] = {"per_launch": atom, "achieved": rate, "peak_measured": top,
                                          "frac": rate / top, "unit": "atomic/s"}
    if not a.no_geodesic:
        out["geodesic_step"] = geodesic_leg(wl, launch, min(a.steps, 3), kms)
    if not a.no_plan:
        out["plan"] = plan_leg(a.steps, stream)
    if not a.no_hetero:
        out["heterogeneous"] = hetero_leg(min(a.steps, 3))
    if not a.no_gamma:
        print("[bench] time to gamma >= 95% (plain vs denoised)", flush=True)
        sde.set_stream(None)
        out["time_to_gamma"] = gamma_leg()
    if not a.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", flush=True)
        out["cpu_baseline"] = cpu_baseline(wl, a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
