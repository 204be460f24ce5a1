"""Wall-time probe of the denoiser on one GPU, for profiling runs.

  python3 -m paper_2511_03115_amd.denoiser_timing denoise   # plan grid, 256x256x200 padded
  python3 -m paper_2511_03115_amd.denoiser_timing train     # one training step, 4 x 128x64x64

`denoise` runs the shipped network on a synthetic dose map of the plan
grid's size (gamma-distributed values, unit density); `train` runs
loss_grad + adam_step of the shipped architecture on random crops.  Each
prints the median and minimum wall time over 10 calls after 3 warm-up
calls.  Inputs are seeded; nothing here is used by the library itself.
"""

import argparse
import os
import time

import numpy as np


def _time(fn, reps=10, warmup=3):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t)
    return float(np.median(ts)), float(min(ts))


def denoise():
    import torch
    from . import denoiser
    weights = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights",
                           "denoiser_plan2mm.npz")
    shape = (200, 256, 256)
    d = denoiser.Denoiser(weights, shape)
    rng = np.random.default_rng(0)
    dose = torch.from_numpy(rng.gamma(2.0, 1.0, size=shape)).cuda()
    rho = torch.ones(shape, dtype=torch.float32, device="cuda")
    out = torch.empty_like(dose)
    med, mn = _time(lambda: d(dose, rho, out))
    print(f"denoise {shape}: median {med * 1e3:.3f} ms min {mn * 1e3:.3f} ms "
          f"checksum {float(out.double().sum()):.6e}", flush=True)
    d.close()


def train():
    import torch
    from . import denoiser, nn
    B, D, H, W = 4, 128, 64, 64
    net = nn.Net(denoiser.LEVELS, denoiser.C0, denoiser.CIN, denoiser.ALPHA, max_batch=B,
                 max_dims=(D, H, W), train=True)
    net.set_params(denoiser.init_params(5, levels=denoiser.LEVELS))
    rng = np.random.default_rng(0)
    dose = torch.from_numpy(rng.gamma(2.0, 1.0, (B, D, H, W)).astype(np.float32)).cuda()
    rho = torch.ones((B, D, H, W), dtype=torch.float32, device="cuda")
    tgt = torch.from_numpy(rng.gamma(2.0, 1.0, (B, D, H, W)).astype(np.float32)).cuda()

    def step():
        net.loss_grad(dose, rho, tgt)
        net.adam_step(1e-4)

    med, mn = _time(step)
    print(f"train step {(B, D, H, W)}: median {med * 1e3:.3f} ms min {mn * 1e3:.3f} ms",
          flush=True)
    net.close()


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["denoise", "train"])
    a = ap.parse_args()
    denoise() if a.what == "denoise" else train()
