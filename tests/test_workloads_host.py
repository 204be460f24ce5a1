"""Host checks of the synthetic workloads (no GPU)."""

import numpy as np

from workloads import configs, materials


def test_air_composition_and_density():
    a = materials.air()
    assert abs(sum(a.w) - 1.0) < 1e-12
    assert a.Z == (6, 7, 8, 18) and abs(a.rho_nominal - 0.001205) < 1e-12
    # Z/A of dry air, 0.49919 (from the mass fractions and atomic weights)
    zoa = sum(w * z / A for z, A, w in zip(a.Z, a.A, a.w))
    assert abs(zoa - 0.49919) < 2e-4


def test_ct_like_phantom_geometry():
    """Along the beam axis: tissue, the bone shell, tissue, the air cavity,
    tissue, the far shell, tissue; the bone block lies off the axis; every
    density is its material's."""
    ph = configs.ct_like(100.0, n=10, size=80).phantom
    mats = [m.name for m in ph.materials]
    assert mats == ["water", "bone", "air"]
    rho = np.array([m.rho_nominal for m in ph.materials], dtype=np.float32)
    assert np.array_equal(ph.density, rho[ph.material_id])
    nx, ny, nz = ph.shape
    axis = ph.material_id[:, ny // 2, nx // 2]
    runs = [int(axis[0])]
    for m in axis[1:]:
        if m != runs[-1]:
            runs.append(int(m))
    assert runs == [0, 1, 0, 2, 0, 1, 0], runs
    zc = ph.centers(2)
    # the cavity (centre z = 4.5 cm, depth semi-axis 2 cm, centred 0.05 L off
    # the axis): a chord of 2 sqrt(1 - (0.15 / 0.6)^2) 2 cm = 3.87 cm at the
    # voxel column x = 0.05 cm
    cavity = zc[(axis == 2) & (zc > 1.5) & (zc < 9.0)]
    assert cavity.min() >= 2.5 and cavity.max() <= 6.5
    assert abs((cavity.max() - cavity.min() + 0.1) - 3.87) <= 0.1
    assert (ph.material_id == 1).sum() > 0 and (ph.material_id == 0).sum() > 0
