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


def forward_flops(dims_zyx: Sequence[int], batch: int = 1, levels: int = LEVELS, c0: int = C0,
                  cin: int = CIN, used_in: Optional[int] = None) -> int:
    """Algorithmic FLOPs of one forward pass: 2 * 27 * Ci * Co per output
    voxel of every conv, at each level's resolution (D, H, W as the network
    sees them, i.e. already padded to multiples of 2^(levels-1)).  With
    used_in, the first conv counts only that many input channels (the input
    has 2 used channels, the other cin - 2 are zero and drop out of its
    sums)."""
    nv0 = batch * int(np.prod(dims_zyx))
    total = 0
    for name, shp in param_layout(levels, c0, cin):
        if name.endswith(".w") and len(shp) == 3:
            lvl = int(name[3])
            ci = used_in if (used_in is not None and name == "enc0a.w") else shp[2]
            total += 2 * 27 * shp[0] * ci * (nv0 >> (3 * lvl))
    return total


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

    def sample(self, rng, batch: int):
        """A random mini-batch (lo, rho, hi, wt) of whole pairs."""
        import torch
        idx = torch.from_numpy(rng.choice(self.lo.shape[0], size=batch, replace=False)).cuda()
        return tuple(t.index_select(0, idx) for t in (self.lo, self.rho, self.hi, self.wt))

    def batches(self, batch: int):
        """The whole set in order, as (lo, rho, hi, wt) mini-batches."""
        for s in range(0, self.lo.shape[0], batch):
            e = min(s + batch, self.lo.shape[0])
            yield self.lo[s:e], self.rho[s:e], self.hi[s:e], self.wt[s:e]


@dataclass
class PlanPairs:
    """Normalised pairs on whole plan grids (N, nz, ny, nx) resident on the
    device, sampled as random crops of ``crop`` = (D, H, W) voxels that
    overlap the field (``lo_zyx``..``hi_zyx`` bounds the crops' origins)."""
    lo: object
    hi: object
    wt: object
    rho: object
    n_in: np.ndarray
    crop: Tuple[int, int, int]
    lo_zyx: Tuple[int, int, int]
    hi_zyx: Tuple[int, int, int]

    def _crop(self, k: int, z: int, y: int, x: int):
        D, H, W = self.crop
        sl = (k, slice(z, z + D), slice(y, y + H), slice(x, x + W))
        return [t[sl] for t in (self.lo, self.rho, self.hi, self.wt)]

    def sample(self, rng, batch: int):
        import torch
        parts = [[], [], [], []]
        for _ in range(batch):
            k = int(rng.integers(0, self.lo.shape[0]))
            z, y, x = (int(rng.integers(a, b + 1)) for a, b in zip(self.lo_zyx, self.hi_zyx))
            for p, t in zip(parts, self._crop(k, z, y, x)):
                p.append(t)
        return tuple(torch.stack(p).contiguous() for p in parts)

    def batches(self, batch: int, per_map: int = 4, seed: int = 12345):
        """Fixed crops (``per_map`` per map, seeded) for validation."""
        rng = np.random.default_rng(seed)
        crops = []
        for k in range(self.lo.shape[0]):
            for _ in range(per_map):
                crops.append((k,) + tuple(int(rng.integers(a, b + 1))
                                          for a, b in zip(self.lo_zyx, self.hi_zyx)))
        import torch
        for s in range(0, len(crops), batch):
            parts = [[], [], [], []]
            for c in crops[s:s + batch]:
                for p, t in zip(parts, self._crop(*c)):
                    p.append(t)
            yield tuple(torch.stack(p).contiguous() for p in parts)


def generate_plan_pairs(variants: Sequence[int], n_low: Sequence[int], n_high: int,
                        crop=(128, 64, 64), eps: float = 0.02, thr: float = 0.01, launch=None,
                        log=print) -> PlanPairs:
    """For each plan variant k (``workloads.configs.plan_variant``): one run
    at ``n_high`` histories per spot and one at each of ``n_low`` per spot
    (independent seeds), each low map normalised with its high map."""
    import torch
    import workloads
    from dataclasses import replace
    from workloads import configs
    t0 = time.time()
    wl0 = configs.plan_variant(int(variants[0]), 1)
    sde.init_materials(wl0.phantom.materials, wl0.params,
                       workloads.nuclear_for_phantom(wl0.phantom, wl0.params.lattice()))
    nz, ny, nx = wl0.phantom.material_id.shape
    n = len(variants) * len(n_low)
    f32 = dict(dtype=torch.float32, device="cuda")
    lo, hi, wt, rho = (torch.empty((n, nz, ny, nx), **f32) for _ in range(4))
    nin = np.zeros(n, np.int64)
    prep = nn.Net(1, 16, 16, 0.01, 1, (1, 1, 1), train=False)
    d_hi = torch.empty((nz, ny, nx), dtype=torch.float64, device="cuda")
    d_lo = torch.empty_like(d_hi)
    k = 0
    for j, v in enumerate(variants):
        wl = configs.plan_variant(int(v), int(n_high))
        dph = sde.DevicePhantom.from_host(wl.phantom)
        sde.transport(wl.spots, dph, wl.seed, dose_out=d_hi, launch=launch)
        for r, nl in enumerate(n_low):
            spots = [replace(sp, n_histories=int(nl)) for sp in wl.spots]
            sde.transport(spots, dph, wl.seed + 7_000_003 * (r + 1), dose_out=d_lo, launch=launch)
            prep.prepare_pair(d_lo, d_hi, lo[k], hi[k], wt[k], eps=eps, thr=thr)
            rho[k].copy_(dph.density)
            nin[k] = int(nl)
            k += 1
        torch.cuda.synchronize()
        log(f"[pairs] plan variant {v}: {j + 1}/{len(variants)} ({time.time() - t0:.1f} s)")
    prep.close()
    D, H, W = crop
    # crop origins: depth from the entrance, laterally over the spot raster
    cy, cx = ny // 2, nx // 2
    lo_zyx = (0, max(0, cy - 24 - H // 2), max(0, cx - 24 - W // 2))
    hi_zyx = (nz - D, min(ny - H, cy + 24 - H // 2), min(nx - W, cx + 24 - W // 2))
    return PlanPairs(lo, hi, wt, rho, nin, (D, H, W), lo_zyx, hi_zyx)


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


def evaluate(net: nn.Net, ps, batch: int) -> float:
    """Mean weighted loss of the network on a pair set's fixed batches (a
    network with zero parameters gives the loss of the input itself, i.e.
    of no network)."""
    tot, n = 0.0, 0
    for lo, rho, hi, wt in ps.batches(batch):
        tot += net.loss_grad(lo, rho, hi, wt) * lo.shape[0]
        n += lo.shape[0]
    return tot / max(n, 1)


def relative_errors(net: nn.Net, ps, thr: float = 0.01) -> Tuple[float, float]:
    """Root-mean-square relative error against the target, over voxels with
    target >= thr, of the inputs and of the network's outputs (a metric of
    the evaluation, computed with torch on the device)."""
    import torch
    e_in, e_out = [], []
    for lo, rho, hi, _ in ps.batches(1):
        out = torch.empty_like(lo)
        net.forward(lo, rho, out)
        m = hi >= thr
        e_in.append(torch.sqrt((((lo - hi) / hi)[m] ** 2).mean()).item())
        e_out.append(torch.sqrt((((out - hi) / hi)[m] ** 2).mean()).item())
    return float(np.mean(e_in)), float(np.mean(e_out))


def train(net: nn.Net, ps, steps: int, batch: int = 4, lr_max: float = 3e-4,
          lr_min: float = 1e-5, warmup: int = 200, seed: int = 0, log=print,
          log_every: int = 50, val=None, checkpoint: Optional[str] = None,
          checkpoint_every: int = 500) -> List[Tuple[int, float]]:
    """Adam on random mini-batches of the resident pairs (``ps.sample``);
    returns the loss curve."""
    rng = np.random.default_rng(seed)
    curve = []
    t0 = time.time()
    run = []
    for it in range(steps):
        loss = net.loss_grad(*ps.sample(rng, batch))
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
