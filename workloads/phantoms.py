"""Voxel phantoms: per-voxel material index (uint8) and density (float32).

Layout: C-contiguous arrays of shape (nz, ny, nx), x fastest.  The grid's
low corner is ``origin`` (cm); the beam enters through the z = origin_z face
travelling along +z.  The lateral centre of every phantom below is x = y = 0.

Geometries follow the paper's test cases (section 2.2, "Test cases"): a water
box, a longitudinal slab stack and a lateral bone insert, plus a
planning-style random phantom (smooth density field with bone and lung
ellipsoids).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

from .materials import Material, air, bone, lung, water


@dataclass
class Phantom:
    shape: Tuple[int, int, int]          # (nx, ny, nz)
    voxel_cm: Tuple[float, float, float]  # (dx, dy, dz)
    origin_cm: Tuple[float, float, float]
    material_id: np.ndarray              # uint8 (nz, ny, nx)
    density: np.ndarray                  # float32 (nz, ny, nx), g/cm3
    materials: List[Material] = field(default_factory=list)

    @property
    def nvox(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz

    def voxel_volume_cm3(self) -> float:
        dx, dy, dz = self.voxel_cm
        return dx * dy * dz

    def centers(self, axis: int) -> np.ndarray:
        n = self.shape[axis]
        return self.origin_cm[axis] + (np.arange(n) + 0.5) * self.voxel_cm[axis]


def _box(nx: int, ny: int, nz: int, d_cm: float, mats: List[Material]) -> Phantom:
    origin = (-0.5 * nx * d_cm, -0.5 * ny * d_cm, 0.0)
    mid = np.zeros((nz, ny, nx), dtype=np.uint8)
    rho = np.full((nz, ny, nx), mats[0].rho_nominal, dtype=np.float32)
    return Phantom((nx, ny, nz), (d_cm, d_cm, d_cm), origin, mid, rho, list(mats))


def water_box(nx: int, ny: int, nz: int, d_cm: float = 0.1) -> Phantom:
    """Homogeneous water (rho = 1.0, I = 75 eV)."""
    return _box(nx, ny, nz, d_cm, [water()])


def slab_phantom(n: int = 200, d_cm: float = 0.1,
                 layers_cm=((0.0, 2.0, 0), (2.0, 4.0, 1), (4.0, 7.0, 2)),
                 nz: int | None = None) -> Phantom:
    """Longitudinal slabs: water 0-2 cm, bone 2-4 cm, lung 4-7 cm, water beyond.

    Layer bounds are (z_lo, z_hi, material index) with materials
    [water, bone, lung]; voxels whose centre lies in a layer take it.
    """
    ph = _box(n, n, nz or n, d_cm, [water(), bone(), lung()])
    zc = ph.centers(2)
    for lo, hi, m in layers_cm:
        sel = (zc >= lo) & (zc < hi)
        ph.material_id[sel] = m
        ph.density[sel] = ph.materials[m].rho_nominal
    return ph


def insert_phantom(n: int = 200, d_cm: float = 0.1, z_lo: float = 3.0,
                   z_hi: float = 5.0, nz: int | None = None) -> Phantom:
    """Water with a bone block for y >= 0 and z_lo <= z < z_hi (cm).

    The interface y = 0 is parallel to the beam and contains the beam axis.
    """
    ph = _box(n, n, nz or n, d_cm, [water(), bone()])
    zc, yc = ph.centers(2), ph.centers(1)
    sel = ((zc >= z_lo) & (zc < z_hi))[:, None, None] & (yc >= 0.0)[None, :, None]
    sel = np.broadcast_to(sel, ph.material_id.shape)
    ph.material_id[sel] = 1
    ph.density[sel] = ph.materials[1].rho_nominal
    return ph


def ct_like_phantom(n: int = 200, d_cm: float = 0.1, nz: int | None = None) -> Phantom:
    """A CT-like head geometry with sharp density contrasts, the setting the
    paper names for its next step (voxelised materials, air cavities).

    Materials [water (soft tissue, 1.0), bone (1.85), air (0.001205)].  With
    L the lateral half-width and the beam along +z on the axis: soft tissue
    everywhere (the beam enters tissue, as in the paper's phantoms), with an
    ellipsoid of lateral semi-axes 0.8 L (x) and 0.9 L (y) and depth
    semi-axis 9 cm centred at z = 10 cm whose outer 0.6 cm is bone (a skull
    shell); inside it an air cavity (a sinus: semi-axes 0.15 L, 0.12 L,
    2 cm) centred at (0.05 L, 0, 4.5 cm) lies on the beam path, and a bone
    block (side 0.1 L) at (-0.12 L, 0.08 L, 7 cm) sits beside it.  Voxel
    centres decide membership.
    """
    ph = _box(n, n, nz or n, d_cm, [water(), bone(), air()])
    L = 0.5 * n * d_cm
    xc, yc, zc = ph.centers(0), ph.centers(1), ph.centers(2)
    Z, Y, X = np.meshgrid(zc, yc, xc, indexing="ij")

    def ell(cx, cy, cz, ax, ay, az):
        return ((X - cx) / ax) ** 2 + ((Y - cy) / ay) ** 2 + ((Z - cz) / az) ** 2 <= 1.0

    mid = np.zeros(ph.material_id.shape, dtype=np.uint8)             # soft tissue
    head = ell(0.0, 0.0, 10.0, 0.8 * L, 0.9 * L, 9.0)
    brain = ell(0.0, 0.0, 10.0, 0.8 * L - 0.6, 0.9 * L - 0.6, 9.0 - 0.6)
    mid[head] = 1                                                     # bone shell
    mid[brain] = 0                                                    # soft tissue
    mid[ell(0.05 * L, 0.0, 4.5, 0.15 * L, 0.12 * L, 2.0)] = 2         # sinus
    h = 0.05 * L
    block = ((np.abs(X + 0.12 * L) <= h) & (np.abs(Y - 0.08 * L) <= h) &
             (np.abs(Z - 7.0) <= h))
    mid[block] = 1
    ph.material_id[...] = mid
    ph.density[...] = np.array([m.rho_nominal for m in ph.materials],
                               dtype=np.float32)[mid]
    return ph


def grf_phantom(nx: int = 256, ny: int = 256, nz: int = 200, d_cm: float = 0.2,
                corr_cm: float = 1.0, n_bone: int = 20, n_lung: int = 10,
                seed_field: int = 100, seed_incl: int = 101) -> Phantom:
    """Water-material Gaussian random density field in [0.9, 1.1] with ellipsoids.

    White noise (seed ``seed_field``) is smoothed with a Gaussian filter of
    width ``corr_cm`` and min-max scaled to [0.9, 1.1].  Then ``n_bone`` bone
    (1.85) and ``n_lung`` lung (0.26) ellipsoids with semi-axes U(0.5, 3) cm,
    random orientation and centres uniform in the box are painted in order
    (seed ``seed_incl``).
    """
    from scipy.ndimage import gaussian_filter

    ph = _box(nx, ny, nz, d_cm, [water(), bone(), lung()])
    rng = np.random.default_rng(seed_field)
    noise = rng.standard_normal((nz, ny, nx))
    sm = gaussian_filter(noise, sigma=corr_cm / d_cm, mode="wrap")
    lo, hi = sm.min(), sm.max()
    ph.density[...] = (0.9 + 0.2 * (sm - lo) / (hi - lo)).astype(np.float32)
    del noise, sm

    rng = np.random.default_rng(seed_incl)
    xc, yc, zc = ph.centers(0), ph.centers(1), ph.centers(2)
    ext = np.array([nx * d_cm, ny * d_cm, nz * d_cm])
    low = np.array(ph.origin_cm)
    kinds = [1] * n_bone + [2] * n_lung
    for m in kinds:
        c = low + rng.uniform(0.0, 1.0, 3) * ext
        semi = rng.uniform(0.5, 3.0, 3)
        q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        # bounding box of the ellipsoid, in voxel indices
        r = semi.max()
        ix = np.nonzero(np.abs(xc - c[0]) <= r)[0]
        iy = np.nonzero(np.abs(yc - c[1]) <= r)[0]
        iz = np.nonzero(np.abs(zc - c[2]) <= r)[0]
        if len(ix) == 0 or len(iy) == 0 or len(iz) == 0:
            continue
        Z, Y, X = np.meshgrid(zc[iz], yc[iy], xc[ix], indexing="ij")
        P = np.stack([X - c[0], Y - c[1], Z - c[2]], axis=-1) @ q
        inside = ((P / semi) ** 2).sum(-1) <= 1.0
        sub_m = ph.material_id[iz[0]:iz[-1] + 1, iy[0]:iy[-1] + 1, ix[0]:ix[-1] + 1]
        sub_r = ph.density[iz[0]:iz[-1] + 1, iy[0]:iy[-1] + 1, ix[0]:ix[-1] + 1]
        sub_m[inside] = m
        sub_r[inside] = ph.materials[m].rho_nominal
    return ph
