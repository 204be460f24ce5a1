"""Named workloads with their sizes and seeds.

* ``water100_small``: 100 MeV monoenergetic point beam, 1e4 histories, water
  40 x 40 x 150 mm at 1 mm voxels, seed 0 (small parity case).
* ``water150``: 150 MeV, 1 % Gaussian energy spread, 3 mm Gaussian lateral
  spread, 1e7 histories, water 200 x 200 x 300 mm at 1 mm, seed 1 (the
  throughput workload).
* ``slab``/``insert``: 100 or 150 MeV with the water150 beam model,
  200 x 200 x 200 mm at 1 mm.
* ``plan``: 1000 spots, 70-230 MeV, lognormal weights, 1e3-1e5 histories per
  spot, 256 x 256 x 200 voxels of 2 mm with a random density field;
  ``plan_uniform``: the same spots with one history count for every spot;
  ``plan_variant``: the family of such plans with other seeds.
* ``denoiser_patch``: training patches of the denoiser, 64 x 64 x 128 voxels
  of 2 mm with a random density field and inclusions and 1-64 spots, all
  drawn like the plan's (index i seeds everything).

Physics parameters are the paper's run settings (section 2.2, "Test cases",
and section 2.1): step 0.5 mm, Lynch-Dahl path length 0.05 cm, F = 0.98,
absorption energy 0.05 MeV, Rutherford cut 0.02 rad, backscatter cut 0.04 rad.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np

from .beams import Spot, single_spot, plan_spots, patch_spots, sobp_spots, with_histories
from .nuclear import EnergyLattice
from .phantoms import Phantom, ct_like_phantom, grf_phantom, insert_phantom, slab_phantom, water_box

# physics switches (bit values shared by both implementations' interfaces)
F_LOSS = 1
F_STRAGGLE = 2
F_MCS = 4
F_ELASTIC = 8
F_INELASTIC = 16
F_END_OF_RANGE = 32
F_SBM = 64
F_ALL = 127
F_FP64 = 128   # not a physics switch: the GPU path steps in double precision
F_ECUT = 256   # variant: large-angle elastic cut 2.5 sigma(E) instead of theta_cut_rad


@dataclass(frozen=True)
class PhysicsParams:
    step_cm: float = 0.05
    ld_z_cm: float = 0.05
    e_min_MeV: float = 0.05
    e_max_MeV: float = 260.0
    ld_F: float = 0.98
    theta_cut_rad: float = 0.02
    backscatter_cut_rad: float = 0.04
    n_energy: int = 1024
    flags: int = F_ALL
    max_steps: int = 65536

    def lattice(self) -> EnergyLattice:
        return EnergyLattice(self.n_energy, self.e_min_MeV, self.e_max_MeV)


@dataclass
class Workload:
    name: str
    phantom: Phantom
    spots: List[Spot]
    seed: int
    params: PhysicsParams = field(default_factory=PhysicsParams)

    @property
    def n_histories(self) -> int:
        return int(sum(s.n_histories for s in self.spots))


def water100_small(n: int = 10_000, seed: int = 0) -> Workload:
    return Workload("water100_small", water_box(40, 40, 150, 0.1),
                    single_spot(100.0, n), seed)


def water150(n: int = 10_000_000, seed: int = 1) -> Workload:
    return Workload("water150", water_box(200, 200, 300, 0.1),
                    single_spot(150.0, n, sigmaE_rel=0.01, sigma_xy_cm=0.3), seed)


def slab(E: float = 150.0, n: int = 10_000_000, seed: int = 2, size: int = 200,
         depth: int = 200) -> Workload:
    return Workload(f"slab{int(E)}", slab_phantom(size, 0.1, nz=depth),
                    single_spot(E, n, sigmaE_rel=0.01, sigma_xy_cm=0.3), seed)


def insert(E: float = 150.0, n: int = 10_000_000, seed: int = 4, size: int = 200,
           depth: int = 200) -> Workload:
    return Workload(f"insert{int(E)}", insert_phantom(size, 0.1, nz=depth),
                    single_spot(E, n, sigmaE_rel=0.01, sigma_xy_cm=0.3), seed)


def ct_like(E: float = 150.0, n: int = 10_000_000, seed: int = 7, size: int = 200,
            depth: int = 200) -> Workload:
    return Workload(f"ct{int(E)}", ct_like_phantom(size, 0.1, nz=depth),
                    single_spot(E, n, sigmaE_rel=0.01, sigma_xy_cm=0.3), seed)


def sobp(n: int = 550_000, seed: int = 8, size: int = 80, depth: int = 150) -> Workload:
    """Spread-out Bragg peak plan in water: 11 energy layers with peaks from 6
    to 10 cm (about 87-117 MeV), each a 5 x 5 raster at 5 mm, n histories in
    all shared like the weights, 1 mm voxels."""
    return Workload("sobp", water_box(size, size, depth, 0.1),
                    sobp_spots(10.0, 4.0, 11, 5, 0.5, n), seed)


def plan(n_spots: int = 1000, n_scale: float = 1.0, seed: int = 6,
         shape=(256, 256, 200)) -> Workload:
    nx, ny, nz = shape
    return Workload("plan", grf_phantom(nx, ny, nz, 0.2),
                    plan_spots(n_spots, n_scale=n_scale), seed)


def plan_uniform(n_per_spot: int, n_spots: int = 1000, seed: int = 6,
                 shape=(256, 256, 200)) -> Workload:
    """The batched plan with ``n_per_spot`` histories in every spot (same
    energies, positions and weights as ``plan``)."""
    nx, ny, nz = shape
    e = float(np.log10(n_per_spot))
    return Workload(f"plan_{n_per_spot}", grf_phantom(nx, ny, nz, 0.2),
                    plan_spots(n_spots, logn_lo=e, logn_hi=e), seed)


def plan_variant(k: int, n_per_spot: int, n_spots: int = 1000,
                 shape=(256, 256, 200)) -> Workload:
    """Plan k of a family drawn like ``plan`` (k = 0 is ``plan_uniform``
    itself): density field seed 100 + 1000k, inclusions 101 + 1000k, spots
    102 + 1000k, transport seed 6 + 1000k; ``n_per_spot`` histories in every
    spot."""
    nx, ny, nz = shape
    e = float(np.log10(n_per_spot))
    return Workload(f"plan_variant{k}_{n_per_spot}",
                    grf_phantom(nx, ny, nz, 0.2, seed_field=100 + 1000 * k,
                                seed_incl=101 + 1000 * k),
                    plan_spots(n_spots, logn_lo=e, logn_hi=e, seed=102 + 1000 * k), 6 + 1000 * k)


def denoiser_patch(i: int, n_histories: int = 100_000, shape=(64, 64, 128)) -> Workload:
    """Training patch i: a 2 mm random-density phantom (correlation 1 cm,
    0-3 bone and 0-2 lung ellipsoids) and 1-64 plan-like spots sharing
    ``n_histories`` histories.  Seeds: field 1000+i, inclusions 5000+i,
    spots 9000+i, transport 20000+i."""
    nx, ny, nz = shape
    rng = np.random.default_rng(13000 + i)
    ph = grf_phantom(nx, ny, nz, 0.2, n_bone=int(rng.integers(0, 4)),
                     n_lung=int(rng.integers(0, 3)), seed_field=1000 + i, seed_incl=5000 + i)
    spots = with_histories(patch_spots(9000 + i, half_cm=min(4.0, 0.2 * nx / 2 - 1.0)), n_histories)
    return Workload(f"denoiser_patch{i}", ph, spots, 20000 + i)
