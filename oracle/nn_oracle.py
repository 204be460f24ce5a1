"""FP64 CPU oracle of the dose denoiser (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module; the product path never does.  It shares no
code with the HIP library.

The denoiser is the learned part built beside the transport: a fully
convolutional 3D encoder-decoder (U-Net shape) that maps a low-history dose
map (plus the density map) to the high-history one.  The paper has no
network; its definition here is this module's, written in the plainest form:
every layer is its mathematical definition, every gradient is the chain rule
applied to that definition, in float64 numpy.

Layout and conventions (shared with the HIP side only through this text):

* volumes are channels-last arrays ``(B, D, H, W, C)``; D is z, H is y, W is x;
* a 3x3x3 convolution (zero padding 1, stride 1) has weights ``w[co, t, ci]``
  with tap ``t = 9 (dz+1) + 3 (dy+1) + (dx+1)`` reading the input at
  ``(z+dz, y+dy, x+dx)`` (a cross-correlation), and a bias ``b[co]``;
* activation: LeakyReLU with slope ``alpha`` below zero;
* down: 2x2x2 average pooling; up: nearest-neighbour x2 replication;
* decoder input at level l: channel concatenation ``[skip_l, up(lower)]``;
* head: 1x1x1 convolution to one channel plus the input dose (residual);
* loss: weighted mean squared error ``mean(m (out - tgt)^2)``;
* optimiser: Adam (Kingma and Ba, 2015) with bias correction.

Storage precision.  With ``bf16_storage=True`` the network rounds, to the
nearest bf16 value (ties to even), exactly the quantities that a bf16
implementation stores: the conv weights, the network input's conv channels,
every activation after LeakyReLU, every pooled tensor, and the activation
gradient that enters the weight- and input-gradient products.  Everything
else (sums, the residual, the head, the loss, the gradients themselves)
stays float64.  With ``False`` (the default) nothing is rounded.

Parameter order (``param_shapes``): for each level l = 0..L-1 the encoder
convs ``enc{l}a``, ``enc{l}b``; then for l = L-2..0 the decoder convs
``dec{l}a``, ``dec{l}b``; each conv as (weight, bias); then the head weight
``(c0,)`` and bias ``(1,)``.  Channels at level l are ``c0 * 2**l``.
"""

from __future__ import annotations

from typing import Dict, List, Tuple

import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


# ---------------------------------------------------------------------------
# layers
# ---------------------------------------------------------------------------

def bf16(a: np.ndarray) -> np.ndarray:
    """Nearest bf16 value (ties to even) of each element, as float64: the
    float32 bit pattern with its low 16 bits rounded away."""
    bits = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (bits >> np.uint64(16)) & np.uint64(1)
    bits = ((bits + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3d(x: np.ndarray, w: np.ndarray, b: np.ndarray | None) -> np.ndarray:
    """y[b, z, y, x, co] = b[co] + sum_t sum_ci x[b, z+dz, y+dy, x+dx, ci] w[co, t, ci],
    with x taken as zero outside the volume."""
    B, D, H, W, Ci = x.shape
    Co = w.shape[0]
    assert w.shape == (Co, 27, Ci)
    xp = np.zeros((B, D + 2, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1, 1:-1, :] = x
    y = np.zeros((B, D, H, W, Co))
    for t, (dz, dy, dx) in enumerate(TAPS):
        sl = xp[:, 1 + dz:1 + dz + D, 1 + dy:1 + dy + H, 1 + dx:1 + dx + W, :]
        y += sl @ w[:, t, :].T
    if b is not None:
        y += b
    return y


def conv3d_backward(dy: np.ndarray, x: np.ndarray, w: np.ndarray, need_dx: bool = True):
    """Gradients of ``conv3d`` by the chain rule on its definition:
    dx[v + off(t), ci] += dy[v, co] w[co, t, ci];  dw[co, t, ci] = sum_v dy[v, co] x[v + off(t), ci];
    db[co] = sum_v dy[v, co]."""
    B, D, H, W, Ci = x.shape
    Co = w.shape[0]
    xp = np.zeros((B, D + 2, H + 2, W + 2, Ci))
    xp[:, 1:-1, 1:-1, 1:-1, :] = x
    dxp = np.zeros_like(xp) if need_dx else None
    dw = np.zeros_like(w)
    dyf = dy.reshape(-1, Co)
    for t, (dz, dy_, dx) in enumerate(TAPS):
        zs, ys, xs = slice(1 + dz, 1 + dz + D), slice(1 + dy_, 1 + dy_ + H), slice(1 + dx, 1 + dx + W)
        sl = xp[:, zs, ys, xs, :].reshape(-1, Ci)
        dw[:, t, :] = dyf.T @ sl
        if need_dx:
            dxp[:, zs, ys, xs, :] += dy @ w[:, t, :]
    db = dyf.sum(axis=0)
    dxo = dxp[:, 1:-1, 1:-1, 1:-1, :] if need_dx else None
    return dxo, dw, db


def lrelu(z: np.ndarray, alpha: float) -> np.ndarray:
    return np.where(z > 0, z, alpha * z)


def lrelu_backward(dy: np.ndarray, z: np.ndarray, alpha: float) -> np.ndarray:
    return np.where(z > 0, dy, alpha * dy)


def pool2(x: np.ndarray) -> np.ndarray:
    """2x2x2 average: y[b, z, y, x] = mean over the eight children (2z+i, 2y+j, 2x+k)."""
    B, D, H, W, C = x.shape
    return x.reshape(B, D // 2, 2, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4, 6))


def pool2_backward(dy: np.ndarray) -> np.ndarray:
    return up2(dy) / 8.0


def up2(x: np.ndarray) -> np.ndarray:
    """Nearest x2: y[b, z, y, x] = x[b, z // 2, y // 2, x // 2]."""
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def up2_backward(dy: np.ndarray) -> np.ndarray:
    B, D, H, W, C = dy.shape
    return dy.reshape(B, D // 2, 2, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4, 6))


def mse(out: np.ndarray, tgt: np.ndarray, m: np.ndarray | None = None):
    """Loss mean(m (out - tgt)^2) and its gradient with respect to out."""
    if m is None:
        m = np.ones_like(out)
    d = out - tgt
    n = out.size
    return float((m * d * d).sum() / n), 2.0 * m * d / n


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, 2015, Algorithm 1); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------

def channels(levels: int, c0: int) -> List[int]:
    return [c0 << l for l in range(levels)]


def param_shapes(levels: int, c0: int, cin: int) -> List[Tuple[str, tuple]]:
    c = channels(levels, c0)
    out = []

    def conv(name, ci, co):
        out.append((name + ".w", (co, 27, ci)))
        out.append((name + ".b", (co,)))

    for l in range(levels):
        conv(f"enc{l}a", cin if l == 0 else c[l - 1], c[l])
        conv(f"enc{l}b", c[l], c[l])
    for l in range(levels - 2, -1, -1):
        conv(f"dec{l}a", c[l] + c[l + 1], c[l])
        conv(f"dec{l}b", c[l], c[l])
    out.append(("head.w", (c0,)))
    out.append(("head.b", (1,)))
    return out


def unflatten(flat: np.ndarray, levels: int, c0: int, cin: int) -> Dict[str, np.ndarray]:
    p, o = {}, 0
    for name, shp in param_shapes(levels, c0, cin):
        n = int(np.prod(shp))
        p[name] = np.asarray(flat[o:o + n], dtype=np.float64).reshape(shp)
        o += n
    assert o == flat.size
    return p


def flatten(p: Dict[str, np.ndarray], levels: int, c0: int, cin: int) -> np.ndarray:
    return np.concatenate([p[name].reshape(-1) for name, _ in param_shapes(levels, c0, cin)])


class UNet:
    """The denoiser in FP64.  ``x`` is (B, D, H, W, cin) with the normalised
    dose in channel 0; the output (B, D, H, W) is x[..., 0] plus the head."""

    def __init__(self, params: Dict[str, np.ndarray], levels: int, c0: int, cin: int,
                 alpha: float = 0.01, bf16_storage: bool = False):
        self.L, self.c0, self.cin, self.alpha = levels, c0, cin, alpha
        self.r = bf16 if bf16_storage else (lambda a: a)
        self.p = {k: (self.r(v) if k.endswith(".w") and np.ndim(v) == 3 else v)
                  for k, v in params.items()}

    def _conv(self, name, x, cache):
        z = conv3d(x, self.p[name + ".w"], self.p[name + ".b"])
        cache[name] = (x, z)
        return self.r(lrelu(z, self.alpha))

    def forward(self, x: np.ndarray):
        cache: Dict[str, tuple] = {}
        skips = []
        h = self.r(x)
        for l in range(self.L):
            if l > 0:
                h = self.r(pool2(h))
            h = self._conv(f"enc{l}a", h, cache)
            h = self._conv(f"enc{l}b", h, cache)
            skips.append(h)
        for l in range(self.L - 2, -1, -1):
            h = np.concatenate([skips[l], up2(h)], axis=-1)
            h = self._conv(f"dec{l}a", h, cache)
            h = self._conv(f"dec{l}b", h, cache)
        cache["head"] = h
        out = x[..., 0] + h @ self.p["head.w"] + self.p["head.b"][0]
        return out, cache

    def _conv_back(self, name, dy, cache, grads, need_dx=True):
        x, z = cache[name]
        dz = self.r(lrelu_backward(dy, z, self.alpha))
        dx, dw, db = conv3d_backward(dz, x, self.p[name + ".w"], need_dx)
        grads[name + ".w"] = dw
        grads[name + ".b"] = db
        return dx

    def backward(self, dout: np.ndarray, cache) -> Dict[str, np.ndarray]:
        """Gradients of the loss with respect to every parameter, given dL/dout."""
        grads: Dict[str, np.ndarray] = {}
        h = cache["head"]
        grads["head.w"] = (h * dout[..., None]).reshape(-1, h.shape[-1]).sum(axis=0)
        grads["head.b"] = np.array([dout.sum()])
        dh = dout[..., None] * self.p["head.w"]
        c = channels(self.L, self.c0)
        dskip = [None] * self.L
        for l in range(0, self.L - 1):
            dh = self._conv_back(f"dec{l}b", dh, cache, grads)
            dcat = self._conv_back(f"dec{l}a", dh, cache, grads)
            dskip[l] = dcat[..., :c[l]]
            dh = up2_backward(dcat[..., c[l]:])
        for l in range(self.L - 1, -1, -1):
            if dskip[l] is not None:
                dh = dh + dskip[l]
            dh = self._conv_back(f"enc{l}b", dh, cache, grads)
            dh = self._conv_back(f"enc{l}a", dh, cache, grads, need_dx=l > 0)
            if l > 0:
                dh = pool2_backward(dh)
        return grads

    def loss_and_grads(self, x, tgt, m=None):
        out, cache = self.forward(x)
        loss, dout = mse(out, tgt, m)
        return loss, self.backward(dout, cache), out
