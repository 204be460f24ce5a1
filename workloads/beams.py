"""Pencil-beam spots and treatment-plan style spot lists.

A spot is a Gaussian pencil beam travelling along +z from the phantom's
entrance face: nominal energy E (MeV) with relative Gaussian spread sigmaE,
lateral centre (x, y) in cm with Gaussian spread sigma_xy, a weight (the
number of protons the spot stands for) and the number of simulated
histories.  Each simulated history carries weight/n_histories.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List

import numpy as np


@dataclass(frozen=True)
class Spot:
    E_MeV: float
    sigmaE_rel: float = 0.0
    x_cm: float = 0.0
    y_cm: float = 0.0
    sigma_xy_cm: float = 0.0
    weight: float = 1.0
    n_histories: int = 0


def single_spot(E_MeV: float, n: int, sigmaE_rel: float = 0.0, sigma_xy_cm: float = 0.0,
                x_cm: float = 0.0, y_cm: float = 0.0, weight: float | None = None) -> List[Spot]:
    """One spot; by default its weight equals its history count (dose of n protons)."""
    return [Spot(E_MeV, sigmaE_rel, x_cm, y_cm, sigma_xy_cm,
                 float(n) if weight is None else float(weight), int(n))]


def plan_spots(n_spots: int = 1000, pitch_cm: float = 0.5, e_lo: float = 70.0,
               e_hi: float = 230.0, w_sigma: float = 0.5, logn_lo: float = 3.0,
               logn_hi: float = 5.0, sigmaE_rel: float = 0.01, sigma_xy_cm: float = 0.3,
               seed: int = 102, n_scale: float = 1.0) -> List[Spot]:
    """Raster of spots on a square lateral grid, centred on the axis.

    Energies U(e_lo, e_hi), weights LogNormal(0, w_sigma), histories
    round(10**U(logn_lo, logn_hi)) (times ``n_scale``, at least 1), all from
    one seeded generator.  Positions fill a ceil(sqrt(n))^2 raster row by row.
    """
    rng = np.random.default_rng(seed)
    side = int(np.ceil(np.sqrt(n_spots)))
    E = rng.uniform(e_lo, e_hi, n_spots)
    w = rng.lognormal(0.0, w_sigma, n_spots)
    n = np.rint(10.0 ** rng.uniform(logn_lo, logn_hi, n_spots))
    n = np.maximum(1, np.rint(n * n_scale)).astype(np.int64)
    spots = []
    for k in range(n_spots):
        iy, ix = divmod(k, side)
        x = (ix - (side - 1) / 2.0) * pitch_cm
        y = (iy - (side - 1) / 2.0) * pitch_cm
        spots.append(Spot(float(E[k]), sigmaE_rel, float(x), float(y), sigma_xy_cm,
                          float(w[k]), int(n[k])))
    return spots


def with_histories(spots: List[Spot], total: int) -> List[Spot]:
    """The same spots (energies, positions, weights) with ``total`` histories
    shared in proportion to the weights (at least one each).  The expected
    dose does not change: each history carries weight/n_histories."""
    w = np.array([s.weight for s in spots], dtype=np.float64)
    n = np.maximum(1, np.rint(total * w / w.sum())).astype(np.int64)
    return [Spot(s.E_MeV, s.sigmaE_rel, s.x_cm, s.y_cm, s.sigma_xy_cm, s.weight, int(k))
            for s, k in zip(spots, n)]


def patch_spots(seed: int, n_max: int = 64, pitch_cm: float = 0.5, half_cm: float = 4.0,
                e_lo: float = 70.0, e_hi: float = 230.0, w_sigma: float = 0.5,
                sigmaE_rel: float = 0.01, sigma_xy_cm: float = 0.3) -> List[Spot]:
    """Spots for one denoiser training patch, drawn like the batched plan's:
    between 1 and ``n_max`` distinct positions of a ``pitch_cm`` lateral grid
    within +-``half_cm`` of the axis, energies U(e_lo, e_hi), weights
    LogNormal(0, w_sigma); history counts are set by ``with_histories``."""
    rng = np.random.default_rng(seed)
    side = int(2 * half_cm / pitch_cm) + 1
    k = int(rng.integers(1, n_max + 1))
    cells = rng.choice(side * side, size=k, replace=False)
    E = rng.uniform(e_lo, e_hi, k)
    w = rng.lognormal(0.0, w_sigma, k)
    out = []
    for j in range(k):
        iy, ix = divmod(int(cells[j]), side)
        out.append(Spot(float(E[j]), sigmaE_rel, -half_cm + ix * pitch_cm, -half_cm + iy * pitch_cm,
                        sigma_xy_cm, float(w[j]), 1))
    return out


def sobp_weights(n_layers: int, p: float = 1.77) -> np.ndarray:
    """Relative weights of the Bragg peaks of a spread-out Bragg peak, from
    the shallowest (index 0) to the deepest (index n_layers - 1).

    With ranges R = alpha E^p (Bragg-Kleeman), a flat dose over the modulated
    depths needs a continuous weight density proportional to (R0 - r)^(-1/p)
    in the peak range r (Bortfeld and Schlegel 1996).  Peak k at the
    normalised position x_k = k / n (n = n_layers - 1) takes that density's
    integral over [x_k - 1/(2n), x_k + 1/(2n)] clipped to [0, 1] (the
    discrete form of Jette and Chen 2011); the weights sum to 1.
    """
    n = n_layers - 1
    if n < 1:
        return np.ones(1)
    q = 1.0 - 1.0 / p
    lo = np.clip((np.arange(n_layers) - 0.5) / n, 0.0, 1.0)
    hi = np.clip((np.arange(n_layers) + 0.5) / n, 0.0, 1.0)
    w = (1.0 - lo) ** q - (1.0 - hi) ** q
    return w / w.sum()


def sobp_spots(r0_cm: float = 10.0, mod_cm: float = 4.0, n_layers: int = 11,
               grid: int = 5, pitch_cm: float = 0.5, n_total: int = 550_000,
               sigmaE_rel: float = 0.01, sigma_xy_cm: float = 0.3,
               alpha: float = 0.0022, p: float = 1.77) -> List[Spot]:
    """A spread-out Bragg peak in water: n_layers energy layers whose peaks
    span ranges [r0 - mod, r0] evenly, each a grid x grid raster of spots
    (pitch ``pitch_cm``, centred on the axis).  Layer energies from the
    ranges by Bragg-Kleeman, E = (R / alpha)^(1/p) (water, R in cm); each
    spot's weight is its layer's ``sobp_weights`` share split evenly over the
    raster, and its history count the same share of ``n_total``, so that
    every history carries (about) the same weight.
    """
    w = sobp_weights(n_layers, p)
    ranges = r0_cm - mod_cm + mod_cm * np.arange(n_layers) / max(n_layers - 1, 1)
    energies = (ranges / alpha) ** (1.0 / p)
    c = (np.arange(grid) - 0.5 * (grid - 1)) * pitch_cm
    spots: List[Spot] = []
    for k in range(n_layers):
        for y in c:
            for x in c:
                share = float(w[k]) / (grid * grid)
                spots.append(Spot(float(energies[k]), sigmaE_rel, float(x), float(y), sigma_xy_cm,
                                  share, max(1, int(round(share * n_total)))))
    return spots

