"""Train the dose denoiser on SDE-generated pairs, on the GPU.

    python -m paper_2511_03115_amd.train_denoiser --targets 192 --steps 6000 \
        --out paper_2511_03115_amd/weights/denoiser.npz

Pairs (``--source patches``): training patches
``workloads.configs.denoiser_patch(i)`` (64 x 64 x 128 voxels of 2 mm,
random density field with bone and lung inclusions, 1-64 plan-like spots of
70-230 MeV); for each, one high-history target (``--n-target`` histories)
and ``--inputs-per-target`` low-history inputs with histories drawn from
``--n-in``.  Patches 0 .. targets-1 train, the next ``--val-targets``
validate.

Pairs (``--source plans``): whole 1000-spot plans
``workloads.configs.plan_variant(k)`` for k = 1 .. plans (k = 0, the
evaluation plan, is never used), each run at ``--plan-high`` histories per
spot and at every ``--plan-low`` count, trained on random 128 x 64 x 64
crops; the next ``--val-plans`` variants validate.

Prints one line per logging interval.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--targets", type=int, default=192)
    ap.add_argument("--val-targets", type=int, default=16)
    ap.add_argument("--inputs-per-target", type=int, default=4)
    ap.add_argument("--n-target", type=float, default=1e8)
    ap.add_argument("--n-in", type=str, default="30000,100000,300000")
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--eps", type=float, default=0.02)
    ap.add_argument("--thr", type=float, default=0.01)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", type=str, required=True, help="parameters-only checkpoint")
    ap.add_argument("--full-checkpoint", type=str, default=None,
                    help="checkpoint with Adam state, written during training")
    ap.add_argument("--resume", type=str, default=None)
    ap.add_argument("--source", choices=("patches", "plans"), default="patches")
    ap.add_argument("--plans", type=int, default=12)
    ap.add_argument("--val-plans", type=int, default=1)
    ap.add_argument("--plan-low", type=str, default="1000,2000,4000,8000,16000,32000,64000")
    ap.add_argument("--plan-high", type=int, default=500_000)
    a = ap.parse_args(argv)

    import numpy as np
    import torch
    from paper_2511_03115_amd import denoiser, nn

    log = lambda m: print(m, flush=True)
    n_in = [int(float(x)) for x in a.n_in.split(",")]
    t0 = time.time()
    if a.source == "patches":
        train = denoiser.generate_pairs(range(a.targets), a.inputs_per_target, n_in,
                                        int(a.n_target), a.eps, a.thr, log=log)
        val = denoiser.generate_pairs(range(a.targets, a.targets + a.val_targets), 1, n_in,
                                      int(a.n_target), a.eps, a.thr, log=log)
        D, H, W = train.lo.shape[1:]
    else:
        lows = [int(float(x)) for x in a.plan_low.split(",")]
        train = denoiser.generate_plan_pairs(range(1, a.plans + 1), lows, a.plan_high,
                                             eps=a.eps, thr=a.thr, log=log)
        val = denoiser.generate_plan_pairs(range(a.plans + 1, a.plans + 1 + a.val_plans), lows,
                                           a.plan_high, eps=a.eps, thr=a.thr, log=log)
        D, H, W = train.crop
    log(f"[pairs] done in {time.time() - t0:.1f} s: {train.lo.shape[0]} train, "
        f"{val.lo.shape[0]} val inputs")
    net = nn.Net(denoiser.LEVELS, denoiser.C0, denoiser.CIN, denoiser.ALPHA, max_batch=a.batch,
                 max_dims=(D, H, W), train=True)
    if a.resume:
        ck = denoiser.load_checkpoint(a.resume)
        net.set_params(ck["params"])
        if "adam_m" in ck:
            net.set_adam_state(ck["adam_m"], ck["adam_v"], int(ck["adam_step"][0]))
    else:
        net.set_params(denoiser.init_params(a.seed))
    zero = nn.Net(denoiser.LEVELS, denoiser.C0, denoiser.CIN, denoiser.ALPHA, max_batch=a.batch,
                  max_dims=(D, H, W), train=True)          # zero parameters: no network
    base = denoiser.evaluate(zero, val, a.batch)
    zero.close()
    log(f"[train] validation loss without the network {base:.4e}")
    t1 = time.time()
    curve = denoiser.train(net, train, a.steps, a.batch, a.lr, seed=a.seed, log=log, val=val,
                           checkpoint=a.full_checkpoint)
    final = denoiser.evaluate(net, val, a.batch)
    e_in, e_out = denoiser.relative_errors(net, val, a.thr)
    log(f"[train] {a.steps} steps in {time.time() - t1:.1f} s; validation loss {final:.4e} "
        f"(no network {base:.4e}); rms relative error above {a.thr}: input {e_in:.4f}, "
        f"denoised {e_out:.4f}")
    meta = {"source": a.source, "steps": a.steps, "eps": a.eps, "batch": a.batch}
    if a.source == "patches":
        meta.update({"targets": a.targets, "inputs_per_target": a.inputs_per_target,
                     "n_target": int(a.n_target), "n_in": n_in})
    else:
        meta.update({"plans": a.plans, "plan_low": a.plan_low, "plan_high": a.plan_high})
    meta.update({
            "thr": a.thr, "lr": a.lr, "val_loss": final, "val_loss_no_net": base,
            "val_rel_err_input": e_in, "val_rel_err_denoised": e_out,
            "curve": curve[-20:]})
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    denoiser.save_checkpoint(a.out, net, meta, adam=False)
    log(json.dumps({k: v for k, v in meta.items() if k != "curve"}))
    net.close()


if __name__ == "__main__":
    main()
