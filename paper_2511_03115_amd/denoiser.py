"""The learned part: a 3D convolutional denoiser trained on pairs that the
SDE transport itself generates, its checkpoints and its inference.

The network, its loss, its gradients and its Adam update run in the HIP
kernels behind ``include/sde_nn.h`` (``nn.Net``); this module orders the
calls.  Training pairs are (low-history, high-history) dose grids of the
same beam on the same phantom, computed by ``sde.transport`` with
independent seeds, normalised by the low map's maximum on the device
(``Net.prepare_pair``), and kept resident in HBM for the whole run.
"""

from __future__ import annotations

import json
import math
import os
import time
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import nn, sde

LEVELS, C0, CIN, ALPHA = 4, 16, 16, 0.01
WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")


def param_layout(levels: int = LEVELS, c0: int = C0, cin: int = CIN) -> List[Tuple[str, tuple]]:
    """Names and shapes of the parameter vector, in the order of include/sde_nn.h."""
    c = [c0 << l for l in range(levels)]
    out: List[Tuple[str, tuple]] = []
    for l in range(levels):
        ci = cin if l == 0 else c[l - 1]
        out += [(f"enc{l}a.w", (c[l], 27, ci)), (f"enc{l}a.b", (c[l],)),
                (f"enc{l}b.w", (c[l], 27, c[l])), (f"enc{l}b.b", (c[l],))]
    for l in range(levels - 2, -1, -1):
        out += [(f"dec{l}a.w", (c[l], 27, c[l] + c[l + 1])), (f"dec{l}a.b", (c[l],)),
                (f"dec{l}b.w", (c[l], 27, c[l])), (f"dec{l}b.b", (c[l],))]
    out += [("head.w", (c0,)), ("head.b", (1,))]
    return out


def init_params(seed: int = 0, levels: int = LEVELS, c0: int = C0, cin: int = CIN,
                alpha: float = ALPHA) -> np.ndarray:
    """He initialisation for LeakyReLU convs, zero biases and a zero head: the
    untrained network returns its input dose unchanged."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shp in param_layout(levels, c0, cin):
        if name.endswith(".w") and len(shp) == 3:
            fan_in = 27 * (2 if name == "enc0a.w" else shp[2])   # real input channels
            std = math.sqrt(2.0 / ((1.0 + alpha * alpha) * fan_in))
            parts.append(rng.normal(0.0, std, size=shp))
        else:
            parts.append(np.zeros(shp))
    return np.concatenate([p.ravel() for p in parts]).astype(np.float32)


# ---------------------------------------------------------------------------
# checkpoints
# ---------------------------------------------------------------------------

def save_checkpoint(path: str, net: nn.Net, meta: Optional[dict] = None, adam: bool = True):
    """FP32 master parameters (+ Adam moments and step when ``adam``) and the
    configuration, as a numpy .npz file (no pickled objects)."""
    cfg = {"levels": net.levels, "base_channels": net.c0, "in_channels": net.cin,
           "alpha": net.alpha}
    cfg.update(meta or {})
    arrays = {"params": net.get_params(), "config": np.array(json.dumps(cfg))}
    if adam:
        m, v, step = net.get_adam_state()
        arrays.update(adam_m=m, adam_v=v, adam_step=np.array([step], np.int64))
    tmp = path + ".tmp.npz"
    np.savez(tmp, **arrays)
    os.replace(tmp, path)


def load_checkpoint(path: str) -> Dict[str, object]:
    with np.load(path, allow_pickle=False) as z:
        out = {k: z[k] for k in z.files}
    out["config"] = json.loads(str(out["config"]))
    return out


# ---------------------------------------------------------------------------
# inference
# ---------------------------------------------------------------------------

class Denoiser:
    """Inference on whole dose grids with a trained checkpoint."""

    def __init__(self, checkpoint: str, grid_zyx: Sequence[int]):
        ck = load_checkpoint(checkpoint)
        cfg = ck["config"]
        m = 1 << (cfg["levels"] - 1)
        dims = tuple(int(math.ceil(n / m) * m) for n in grid_zyx)
        self.net = nn.Net(cfg["levels"], cfg["base_channels"], cfg["in_channels"], cfg["alpha"],
                          max_batch=1, max_dims=dims, train=False)
        self.net.set_params(ck["params"])
        self.config = cfg

    def __call__(self, dose, rho, out=None):
        """dose: float64 (nz, ny, nx) device tensor; rho float32 or None."""
        import torch
        if out is None:
            out = torch.empty_like(dose)
        self.net.denoise(dose, rho, out)
        return out

    def close(self):
        self.net.close()


# ---------------------------------------------------------------------------
# training data
# ---------------------------------------------------------------------------

@dataclass
class PairSet:
    """Normalised pairs resident on the device: row k holds one low-history
    input and its target (rows of one patch share the high-history run)."""
    lo: object            # float32 (n_in, D, H, W)
    hi: object            # float32 (n_in, D, H, W), each input's target / the input's max
    wt: object            # float32 (n_in, D, H, W) loss weights
    rho: object           # float32 (n_in, D, H, W) density
    n_in: np.ndarray      # histories of each input


def generate_pairs(indices: Sequence[int], inputs_per_target: int = 4,
                   n_in_choices: Sequence[int] = (30_000, 100_000, 300_000),
                   n_target: int = 100_000_000, eps: float = 0.02, thr: float = 0.01,
                   launch=None, log=print) -> PairSet:
    """Runs the transport for each training patch (``workloads.configs.
    denoiser_patch``): one high-history target and ``inputs_per_target``
    low-history inputs with independent seeds, normalised on the device."""
    import torch
    import workloads
    from workloads import configs
    first = configs.denoiser_patch(int(indices[0]), 1)
    sde.init_materials(first.phantom.materials, first.params,
                       workloads.nuclear_for_phantom(first.phantom, first.params.lattice()))
    nz, ny, nx = first.phantom.material_id.shape
    n = len(indices) * inputs_per_target
    f32 = dict(dtype=torch.float32, device="cuda")
    lo = torch.empty((n, nz, ny, nx), **f32)
    hi = torch.empty((n, nz, ny, nx), **f32)
    wt = torch.empty((n, nz, ny, nx), **f32)
    rho = torch.empty((n, nz, ny, nx), **f32)
    nin = np.zeros(n, np.int64)
    prep = nn.Net(1, 16, 16, 0.01, 1, (1, 1, 1), train=False)   # scratch for the maxima
    dose_hi = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
    dose_lo = torch.empty_like(dose_hi)
    rng = np.random.default_rng(int(indices[0]) * 7 + 1)
    t0 = time.time()
    k = 0
    for j, i in enumerate(indices):
        wl = configs.denoiser_patch(int(i), n_target)
        dph = sde.DevicePhantom.from_host(wl.phantom)
        sde.transport(wl.spots, dph, wl.seed, dose_out=dose_hi, launch=launch)
        for r in range(inputs_per_target):
            n_in = int(rng.choice(n_in_choices))
            spots = workloads.with_histories(wl.spots, n_in)
            sde.transport(spots, dph, wl.seed + 1_000_003 * (r + 1), dose_out=dose_lo,
                          launch=launch)
            prep.prepare_pair(dose_lo, dose_hi, lo[k], hi[k], wt[k], eps=eps, thr=thr)
            rho[k].copy_(dph.density)
            nin[k] = n_in
            k += 1
        if (j + 1) % 8 == 0 or j + 1 == len(indices):
            torch.cuda.synchronize()
            log(f"[pairs] {j + 1}/{len(indices)} targets, {time.time() - t0:.1f} s")
    torch.cuda.synchronize()
    prep.close()
    return PairSet(lo, hi, wt, rho, nin)


# ---------------------------------------------------------------------------
# training
# ---------------------------------------------------------------------------

def cosine_lr(step: int, total: int, lr_max: float, lr_min: float, warmup: int) -> float:
    if step < warmup:
        return lr_max * (step + 1) / warmup
    t = (step - warmup) / max(1, total - warmup)
    return lr_min + 0.5 * (lr_max - lr_min) * (1.0 + math.cos(math.pi * min(1.0, t)))


def evaluate(net: nn.Net, ps: PairSet, batch: int) -> float:
    """Mean weighted loss of the network on a pair set (a network with zero
    parameters gives the loss of the input itself, i.e. of no network)."""
    losses = []
    for s in range(0, ps.lo.shape[0], batch):
        e = min(s + batch, ps.lo.shape[0])
        losses.append(net.loss_grad(ps.lo[s:e], ps.rho[s:e], ps.hi[s:e], ps.wt[s:e]) * (e - s))
    return float(np.sum(losses) / ps.lo.shape[0])


def relative_errors(net: nn.Net, ps: PairSet, thr: float = 0.01) -> Tuple[float, float]:
    """Root-mean-square relative error against the target, over voxels with
    target >= thr, of the inputs and of the network's outputs (a metric of
    the evaluation, computed with torch on the device)."""
    import torch
    e_in, e_out = [], []
    out = torch.empty_like(ps.lo[:1])
    for k in range(ps.lo.shape[0]):
        net.forward(ps.lo[k:k + 1], ps.rho[k:k + 1], out)
        h = ps.hi[k:k + 1]
        m = h >= thr
        e_in.append(torch.sqrt((((ps.lo[k:k + 1] - h) / h)[m] ** 2).mean()).item())
        e_out.append(torch.sqrt((((out - h) / h)[m] ** 2).mean()).item())
    return float(np.mean(e_in)), float(np.mean(e_out))


def train(net: nn.Net, ps: PairSet, steps: int, batch: int = 4, lr_max: float = 3e-4,
          lr_min: float = 1e-5, warmup: int = 200, seed: int = 0, log=print,
          log_every: int = 50, val: Optional[PairSet] = None, checkpoint: Optional[str] = None,
          checkpoint_every: int = 500) -> List[Tuple[int, float]]:
    """Adam on random mini-batches of the resident pairs; returns the loss curve."""
    import torch
    rng = np.random.default_rng(seed)
    n = ps.lo.shape[0]
    curve = []
    t0 = time.time()
    run = []
    for it in range(steps):
        idx = torch.from_numpy(rng.choice(n, size=batch, replace=False)).cuda()
        loss = net.loss_grad(ps.lo.index_select(0, idx), ps.rho.index_select(0, idx),
                             ps.hi.index_select(0, idx), ps.wt.index_select(0, idx))
        net.adam_step(cosine_lr(it, steps, lr_max, lr_min, warmup))
        run.append(loss)
        if (it + 1) % log_every == 0 or it + 1 == steps:
            m = float(np.mean(run))
            run = []
            curve.append((it + 1, m))
            msg = f"[train] step {it + 1}/{steps} loss {m:.4e} ({time.time() - t0:.1f} s)"
            if val is not None and ((it + 1) % (log_every * 10) == 0 or it + 1 == steps):
                msg += f" val {evaluate(net, val, batch):.4e}"
            log(msg)
        if checkpoint and ((it + 1) % checkpoint_every == 0 or it + 1 == steps):
            save_checkpoint(checkpoint, net, {"step": it + 1})
    return curve
