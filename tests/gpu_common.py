"""Shared helpers of the GPU tests: run a workload through libsde and the oracle."""

from __future__ import annotations

import sys
from dataclasses import replace

import numpy as np

import oracle
import workloads


def log(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def nuclear_for(phantom, params):
    return workloads.nuclear_for_phantom(phantom, params.lattice())


def run_gpu(wl, flags=None, launch=None, n=None, tally=True):
    """(dose numpy (nz,ny,nx), tally numpy int64, ledger, scale) from libsde."""
    import torch
    from paper_2511_03115_amd import sde
    params = wl.params if flags is None else replace(wl.params, flags=flags)
    nuc = nuclear_for(wl.phantom, params)
    sde.init_materials(wl.phantom.materials, params, nuc)
    dph = sde.DevicePhantom.from_host(wl.phantom)
    nz_ny_nx = wl.phantom.material_id.shape
    dose = torch.zeros(nz_ny_nx, dtype=torch.float64, device="cuda")
    tal = torch.zeros(nz_ny_nx, dtype=torch.int64, device="cuda") if tally else None
    res = sde.transport(wl.spots, dph, wl.seed, dose_out=dose, tally_out=tal,
                        n_histories=n or 0, launch=launch)
    torch.cuda.synchronize()
    return (dose.cpu().numpy(), tal.cpu().numpy() if tally else None, res.ledger, res.scale)


def run_oracle(wl, flags=None, n=None, energy=False):
    """(dose, ledger) from the oracle; with energy=True (energy, ledger), the
    deposited energy per voxel in MeV (weighted like the tally)."""
    params = wl.params if flags is None else replace(wl.params, flags=flags)
    nuc = nuclear_for(wl.phantom, params)
    spots = wl.spots
    if n:
        spots = [replace(spots[0], n_histories=n)]
    r = oracle.transport(wl.phantom, spots, params, nuc, seed=wl.seed)
    return (r.edep if energy else oracle.dose(r.edep, wl.phantom)), r.ledger


def parity_metrics(d_ref, d_gpu, phantom):
    mx = d_ref.max()
    dmax = np.abs(d_gpu - d_ref).max() / mx
    g, ne, npass = oracle.gamma_pass_rate(d_ref, d_gpu, phantom.voxel_cm, dd=0.01, dta_cm=0.05,
                                          thresh=0.01, interp=10, local=True)
    dz = phantom.voxel_cm[2]
    r_ref = oracle.range_rx(d_ref, dz, 0.8)
    r_gpu = oracle.range_rx(d_gpu, dz, 0.8)
    return dict(max_rel_diff=float(dmax), gamma_1pct_05mm=float(g), gamma_n=ne,
                r80_ref_cm=r_ref, r80_gpu_cm=r_gpu, dr80_mm=abs(r_ref - r_gpu) * 10)


def run_gpu_records(wl, flags=None):
    """(records numpy (n, 12), dose numpy) from a plan with per-history records."""
    import torch
    from paper_2511_03115_amd import sde
    params = wl.params if flags is None else replace(wl.params, flags=flags)
    sde.init_materials(wl.phantom.materials, params, nuclear_for(wl.phantom, params))
    dph = sde.DevicePhantom.from_host(wl.phantom)
    plan = sde.Plan(wl.spots, dph, wl.seed)
    rec = torch.zeros((plan.n_histories, 12), dtype=torch.float32, device="cuda")
    plan.set_records(rec)
    dose = torch.zeros(wl.phantom.material_id.shape, dtype=torch.float64, device="cuda")
    plan.execute(dose)
    out = rec.cpu().numpy().astype(np.float64), dose.cpu().numpy()
    plan.close()
    return out


def history_agreement(g, o):
    """Fractions of histories whose discrete path (steps, jump count, first and
    last jump step, end event) is identical, and, among those, the end-position
    and end-energy differences."""
    oj = o[:, oracle.R_NEL] + o[:, oracle.R_NNE]
    same = ((g[:, 1] == o[:, oracle.R_STEPS]) & (g[:, 2] == oj) & (g[:, 3] == o[:, oracle.R_END])
            & (g[:, 8] == o[:, oracle.R_J1]) & (g[:, 9] == o[:, oracle.R_J2]))
    pos = np.sqrt(((g[:, 4:7] - o[:, [oracle.R_X, oracle.R_Y, oracle.R_Z]]) ** 2).sum(1))
    dE = np.abs(g[:, 7] - o[:, oracle.R_EEND])
    return dict(same_frac=float(same.mean()), pos_p99=float(np.percentile(pos[same], 99)),
                pos_close_frac=float((pos[same] < 1e-3).mean()),
                dE_p99=float(np.percentile(dE[same], 99)),
                e0_equal=float(np.mean(np.abs(g[:, 0] - o[:, oracle.R_E0]) <= 1e-5 * o[:, oracle.R_E0])))
