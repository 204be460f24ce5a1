"""sde_gamma_noalloc (no device allocation, fixed scratch) against sde_gamma
and the oracle, through the C ABI: two calls in a row, the second on a
smaller grid, counts equal; and a grid whose search list overflows the
scratch list (voxels searched in the first pass), counts still equal."""

import numpy as np
import pytest

import oracle
from gpu_common import log

pytestmark = pytest.mark.gpu


def _field(shape, rng):
    z, y, x = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    f = np.zeros(shape)
    for _ in range(5):
        c = [rng.uniform(0, n) for n in shape]
        s = rng.uniform(3, 9)
        f += np.exp(-((z - c[0]) ** 2 + (y - c[1]) ** 2 + (x - c[2]) ** 2) / (2 * s * s))
    return f


def test_gamma_noalloc_matches_gamma_two_calls():
    import torch
    from paper_2511_03115_amd import sde
    rng = np.random.default_rng(21)
    for shape, d in (((48, 40, 36), (0.2, 0.2, 0.2)), ((12, 10, 9), (0.1, 0.12, 0.09))):
        ref = _field(shape, rng)
        ev = np.maximum(ref * (1 + 0.05 * rng.standard_normal(shape)), 0.0)
        r, e = torch.from_numpy(ref).cuda(), torch.from_numpy(ev).cuda()
        for local in (True, False):
            a = sde.gamma(r, e, d, local=local)
            b = sde.gamma_noalloc(r, e, d, local=local)
            _, ne0, np0 = oracle.gamma_pass_rate(ref, ev, d, local=local)
            log(f"noalloc {shape} local={local}: gamma {a[1:]} noalloc {b[1:]} oracle {(ne0, np0)}")
            assert a[1:] == b[1:] == (ne0, np0)


def test_gamma_noalloc_list_overflow():
    """More than 2^20 voxels failing at the zero offset: the overflow is
    searched in the first pass, with the same counts as sde_gamma."""
    import torch
    from paper_2511_03115_amd import sde
    rng = np.random.default_rng(5)
    shape = (64, 160, 160)                      # 1.6e6 voxels, most failing at o = 0
    ref = rng.uniform(0.5, 1.0, shape)
    ev = ref * rng.uniform(0.9, 1.1, shape)
    r, e = torch.from_numpy(ref).cuda(), torch.from_numpy(ev).cuda()
    a = sde.gamma(r, e, (0.2, 0.2, 0.2))
    b = sde.gamma_noalloc(r, e, (0.2, 0.2, 0.2))
    hard = int(np.sum(np.abs(ev - ref) > 0.02 * ref))   # failing at the zero offset
    log(f"noalloc overflow: gamma {a[1:]} noalloc {b[1:]}, {hard} voxels to search")
    assert a[1:] == b[1:]
    assert hard > (1 << 20) + 1000                       # the list overflowed
