"""The gamma-index kernel (section 2.2.3) through the C ABI against the
oracle's double-precision evaluation of the definition: pass counts equal,
exactly, on grids that exercise every path of the kernel (the pass at the
zero offset, the range bound and the early end of the search, the full
search when the distance to agreement exceeds a voxel, the grid faces) and
on maps built to put many voxels exactly on the pass boundary."""

import numpy as np
import pytest

import oracle
from gpu_common import log

pytestmark = pytest.mark.gpu


def _both(ref, ev, d, dd=0.02, dta=0.05, thr=0.01, interp=10, local=True):
    import torch
    from paper_2511_03115_amd import sde
    _, ne0, np0 = oracle.gamma_pass_rate(ref, ev, d, dd, dta, thr, interp, local)
    _, ne1, np1 = sde.gamma(torch.from_numpy(np.ascontiguousarray(ref)).cuda(),
                            torch.from_numpy(np.ascontiguousarray(ev)).cuda(), d, dd, dta, thr,
                            interp, local)
    return (ne0, np0), (ne1, np1)


def _smooth_field(shape, rng, blobs=6):
    z, y, x = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    f = np.zeros(shape)
    for _ in range(blobs):
        c = [rng.uniform(0, n) for n in shape]
        s = rng.uniform(2, 8)
        f += rng.uniform(0.3, 1.0) * np.exp(-((z - c[0]) ** 2 + (y - c[1]) ** 2 +
                                              (x - c[2]) ** 2) / (2 * s * s))
    return f


@pytest.mark.parametrize("local", [True, False])
@pytest.mark.parametrize("d,dta,interp", [
    ((0.1, 0.12, 0.09), 0.05, 10),   # bound on (dta below a voxel)
    ((0.2, 0.2, 0.2), 0.05, 10),     # the plan's 2 mm voxels
    ((0.1, 0.1, 0.1), 0.2, 5),       # dta above a voxel: full search, no bound
    ((0.1, 0.1, 0.1), 0.05, 16),
])
def test_gamma_counts_equal_random(local, d, dta, interp):
    rng = np.random.default_rng(7)
    ref = rng.uniform(0.1, 1.0, (14, 13, 12))
    ev = ref * rng.uniform(0.97, 1.03, ref.shape)
    a, b = _both(ref, ev, d, 0.02, dta, 0.01, interp, local)
    log(f"gamma random local={local} d={d} dta={dta} interp={interp}: oracle {a} gpu {b}")
    assert a == b


@pytest.mark.parametrize("local", [True, False])
def test_gamma_counts_equal_noisy_dose(local):
    """A smooth dose with 1-8 % relative noise on 64 x 48 x 40 voxels of
    2 mm (most voxels pass at the zero offset, many need the search)."""
    rng = np.random.default_rng(3)
    ref = _smooth_field((40, 48, 64), rng)
    for noise in (0.01, 0.03, 0.08):
        ev = ref * (1 + noise * rng.standard_normal(ref.shape))
        ev = np.maximum(ev, 0.0)
        a, b = _both(ref, ev, (0.2, 0.2, 0.2), local=local)
        log(f"gamma noisy local={local} noise={noise}: oracle {a} gpu {b} "
            f"({a[1] / max(a[0], 1):.4f})")
        assert a == b


def test_gamma_ties_on_the_boundary():
    """The evaluated map is the reference scaled by exactly 1 + dd (and by
    1 - dd), so that at the zero offset the test sits on 1 up to rounding:
    both sides must round it the same way."""
    rng = np.random.default_rng(11)
    ref = _smooth_field((16, 18, 20), rng)
    for f in (1.02, 0.98, 1.01, 1.0200000000000002):
        a, b = _both(ref, ref * f, (0.1, 0.1, 0.1))
        log(f"gamma ties f={f}: oracle {a} gpu {b}")
        assert a == b
    # constant maps: every zero-offset test is a tie
    c = np.full((8, 9, 10), 0.7)
    for f in (1.02, 0.98):
        a, b = _both(c, c * f, (0.1, 0.1, 0.1))
        assert a == b


@pytest.mark.parametrize("shape", [(1, 1, 1), (1, 1, 7), (1, 5, 6), (3, 1, 4), (2, 2, 2)])
def test_gamma_degenerate_grids(shape):
    """Single voxels, lines and planes: trilinear evaluation on an axis of
    one node, and offsets leaving the grid on every side."""
    rng = np.random.default_rng(sum(shape))
    ref = rng.uniform(0.2, 1.0, shape)
    ev = ref * rng.uniform(0.95, 1.05, shape)
    for local in (True, False):
        a, b = _both(ref, ev, (0.1, 0.1, 0.1), local=local)
        assert a == b, (shape, local, a, b)


def test_gamma_threshold_and_empty():
    """Nothing above the threshold evaluates nothing; an all-zero reference
    evaluates nothing."""
    ref = np.zeros((4, 4, 4))
    a, b = _both(ref, ref + 1.0, (0.1, 0.1, 0.1))
    assert a == b == (0, 0)
    ref[1, 2, 3] = 1.0
    a, b = _both(ref, ref, (0.1, 0.1, 0.1), thr=0.5)
    assert a == b == (1, 1)
