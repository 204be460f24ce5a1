"""The lane guard through the C ABI: a history whose direction the host
poisons with a NaN (the launch's nan_history test hook) is ended by the guard
after its first step (whose deposit, made off the box, counts as escaped),
with its energy in the bad-lane ledger slot, so the energy
balance still closes; the other histories run exactly as without the hook;
and sound runs leave the slot at zero.  The condition is forced from the
host: nothing faults, every lane exits normally."""

import numpy as np
import pytest

import oracle
from workloads import configs
from gpu_common import log, nuclear_for

pytestmark = pytest.mark.gpu

FP64 = 128


def _plan(wl, flags, launch):
    import torch
    from dataclasses import replace
    from paper_2511_03115_amd import sde
    params = replace(wl.params, flags=flags)
    sde.init_materials(wl.phantom.materials, params, nuclear_for(wl.phantom, params))
    dph = sde.DevicePhantom.from_host(wl.phantom)
    plan = sde.Plan(wl.spots, dph, wl.seed, launch=launch)
    rec = torch.zeros((plan.n_histories, 12), dtype=torch.float32, device="cuda")
    plan.set_records(rec)
    dose = torch.zeros(wl.phantom.material_id.shape, dtype=torch.float64, device="cuda")
    plan.execute(dose)
    tal = torch.zeros(wl.phantom.material_id.shape, dtype=torch.int64, device="cuda")
    ledger, scale = plan.results(tal)
    out = rec.cpu().numpy(), tal.cpu().numpy(), ledger.astype(np.int64), scale
    plan.close()
    return out


@pytest.mark.parametrize("flags", [oracle.ALL, oracle.ALL | FP64])
def test_guard_ends_a_poisoned_history(flags):
    from paper_2511_03115_amd import sde
    n, bad_h = 3000, 1234
    wl = configs.water100_small(n=n)
    log(f"case lane guard flags={flags} poisoned history {bad_h}")
    rec0, tal0, led0, _ = _plan(wl, flags, None)
    rec1, tal1, led1, _ = _plan(wl, flags, {"nan_history": bad_h + 1})
    log(f"ledger clean {led0.tolist()}")
    log(f"ledger guard {led1.tolist()}")
    DEP, ESC, NUC, E0, TR, B = (sde.LEDGER_DEPOSITED, sde.LEDGER_ESCAPED, sde.LEDGER_NUCLEAR,
                                sde.LEDGER_INITIAL, sde.LEDGER_TRUNCATED, sde.LEDGER_BAD_LANES)
    assert led0[B] == 0 and led1[B] > 0
    assert led1[sde.LEDGER_HISTORIES] == n and led1[E0] == led0[E0]
    # the poisoned history ends after its first step with code 6; no other
    # history ends so
    assert rec1[bad_h, 3] == 6 and rec1[bad_h, 1] == 1
    others = np.arange(n) != bad_h
    assert (rec0[:, 3] != 6).all() and (rec1[others, 3] != 6).all()
    # every other history runs identically
    assert np.array_equal(rec0[others], rec1[others])
    # the slot holds what that history carried in the clean run
    moved = sum(int(led0[k]) - int(led1[k]) for k in (DEP, ESC, NUC, TR))
    assert abs(int(led1[B]) - moved) <= 1e-9 * int(led0[E0]) + 1024, (int(led1[B]), moved)
    # the energy balance closes with the slot, in both runs
    for led in (led0, led1):
        lhs = sum(int(led[k]) for k in (DEP, ESC, NUC, TR, B))
        assert abs(lhs - int(led[E0])) <= 1e-9 * int(led[E0]) + 1024
    # the tallies differ by exactly what that history deposited
    assert int(tal0.sum()) - int(tal1.sum()) == int(led0[DEP]) - int(led1[DEP])
