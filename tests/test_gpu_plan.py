"""Batched plans: many spots of different energies, weights and history
counts in one persistent launch, replayed from a hipGraph."""

import numpy as np
import pytest

import oracle
import workloads
from workloads import configs
from gpu_common import log, parity_metrics

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def plan_workload():
    return configs.plan(n_spots=1000, n_scale=0.05)


def _device(wl):
    from paper_2511_03115_amd import sde
    sde.init_materials(wl.phantom.materials, wl.params,
                       workloads.nuclear_for_phantom(wl.phantom, wl.params.lattice()))
    return sde.DevicePhantom.from_host(wl.phantom)


def test_plan_parity_subset(plan_workload):
    """100 of the spots against the oracle on the full random phantom."""
    import torch
    from dataclasses import replace
    from paper_2511_03115_amd import sde
    wl = plan_workload
    spots = [replace(s, n_histories=max(1, s.n_histories * 2)) for s in wl.spots[450:550]]
    n = sum(s.n_histories for s in spots)
    log(f"case plan subset spots={len(spots)} n={n}")
    dph = _device(wl)
    dose = torch.zeros(wl.phantom.material_id.shape, dtype=torch.float64, device="cuda")
    res = sde.transport(spots, dph, wl.seed, dose_out=dose)
    assert res.ledger[sde.LEDGER_HISTORIES] == n
    d_gpu = dose.cpu().numpy()
    r = oracle.transport(wl.phantom, spots, wl.params,
                         workloads.nuclear_for_phantom(wl.phantom, wl.params.lattice()),
                         seed=wl.seed)
    d_ref = oracle.dose(r.edep, wl.phantom)
    m = parity_metrics(d_ref, d_gpu, wl.phantom)
    log(f"metrics {m}")
    assert m["gamma_1pct_05mm"] >= 0.99, m
    assert m["dr80_mm"] <= 0.1, m
    # weighted energy balance agrees with the oracle's to FP32 accuracy
    assert abs(res.ledger[sde.LEDGER_DEPOSITED] / res.scale - r.ledger[oracle.L_DEP]) <= \
        1e-4 * r.ledger[oracle.L_E0]


def test_plan_graph_replay(plan_workload):
    """The 1000-spot plan replayed from a hipGraph equals plain launches, replay after replay."""
    import torch
    from paper_2511_03115_amd import sde
    wl = plan_workload
    dph = _device(wl)
    log(f"case plan graph n={wl.n_histories} spots={len(wl.spots)}")
    plan = sde.Plan(wl.spots, dph, wl.seed)
    shape = wl.phantom.material_id.shape
    dose = torch.zeros(shape, dtype=torch.float64, device="cuda")
    tal = torch.zeros(shape, dtype=torch.int64, device="cuda")
    plan.execute(dose, use_graph=False)
    led0, _ = plan.results(tal)
    ref_tal, ref_dose = tal.clone(), dose.clone()
    assert led0[sde.LEDGER_HISTORIES] == wl.n_histories
    for i in range(3):
        dose.zero_()
        plan.execute(dose, use_graph=True)
        _ = float(dose.sum())            # eager work between replays
        led, _ = plan.results(tal)
        log(f"replay {i} ledger ok {np.array_equal(led, led0)}")
        assert np.array_equal(led, led0)
        assert torch.equal(tal, ref_tal)
        assert torch.equal(dose, ref_dose)
    plan.close()
