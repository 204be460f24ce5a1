"""The plain SDE as judge and fallback of the denoiser, and the wall time to
a dose whose gamma pass rate reaches 95 %.

Gamma (section 2.2): local dose difference 2 %, distance to agreement
0.5 mm, voxels below 1 % of the reference maximum excluded, search at
DTA/10 with trilinear interpolation of the evaluated map (``sde.gamma``,
a HIP kernel).  The reference is a high-history SDE run of the same plan
with an independent seed; its cost is reported on its own.

* plain: the smallest history count on a doubling ladder whose map passes;
  its time is that one run's time (plain SDE needs no judge).
* denoised, configured protocol (the headline): one run at the lowest rung,
  denoised and judged against the reference; if the denoised map passes,
  its time is run + inference + judge; otherwise the map is rerun plain
  (fallback) at the plain ladder's passing rung, and that run's time is
  added.
* denoised ladder (the rung is selected with the reference, so it is not a
  protocol a user could run blind): every rung up to the plain passing one
  is also denoised and judged; the smallest rung whose denoised map passes
  gives run + inference + judge; if none does, the plain run is the
  fallback.
Both also report the cumulative time of walking the ladder up to the
passing rung (every run, and for the denoised ladder every inference and
judge), for plain and denoised alike.
All times are GPU wall times (stream-synchronised), with tables, phantom and
plan set up beforehand; set-up times are reported beside them.
"""

from __future__ import annotations

import time
from dataclasses import asdict, dataclass, field
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

from . import sde

DD, DTA_CM, THRESH, INTERP, TARGET = 0.02, 0.05, 0.01, 10, 0.95


def gamma_pass(ref, ev, voxel_cm, dd: float = DD, dta_cm: float = DTA_CM,
               thresh: float = THRESH, local: bool = True) -> float:
    frac, _, _ = sde.gamma(ref, ev, voxel_cm, dd, dta_cm, thresh, INTERP, local)
    return float(frac)


def _timed(fn) -> float:
    import torch
    torch.cuda.synchronize()
    t = time.perf_counter()
    fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t


def _timed_gpu(fn, stream) -> Tuple[float, float]:
    """(wall seconds, GPU seconds between HIP events recorded on ``stream``
    around fn's launches)."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t, e0.elapsed_time(e1) * 1e-3


@dataclass
class Rung:
    n_per_spot: int
    histories: int
    setup_s: float
    run_s: float
    gamma_plain: float
    denoise_s: Optional[float] = None
    gamma_denoised: Optional[float] = None
    judge_s: Optional[float] = None       # the gamma evaluation of the denoised map
    denoise_gpu_s: Optional[float] = None   # the denoise between HIP events on its stream


@dataclass
class TimeToGamma:
    workload: str
    reference_histories: int
    reference_s: float
    rungs: List[Rung] = field(default_factory=list)
    plain_n_per_spot: Optional[int] = None
    plain_s: Optional[float] = None
    plain_cumulative_s: Optional[float] = None
    first_rung_denoised_s: Optional[float] = None
    first_rung_passed: Optional[bool] = None
    denoised_n_per_spot: Optional[int] = None
    denoised_s: Optional[float] = None
    denoised_cumulative_s: Optional[float] = None
    fallback: Optional[bool] = None

    def as_dict(self) -> dict:
        d = asdict(self)
        # headline: the configured protocol (first rung, judged, with fallback)
        d["speedup_first_rung"] = (self.plain_s / self.first_rung_denoised_s
                                   if self.plain_s and self.first_rung_denoised_s else None)
        # the ladder's rung is selected with the reference: reported beside it
        d["speedup_ladder_selected"] = (self.plain_s / self.denoised_s
                                        if self.plain_s and self.denoised_s else None)
        d["judge_included"] = True
        return d


def decide(res: TimeToGamma) -> TimeToGamma:
    """Fill the plain, denoised-ladder and first-rung results of ``res`` from
    its rungs (each with its run time, plain gamma and, where denoised, the
    inference time and denoised gamma), by the rules in the module text."""
    res.plain_n_per_spot = res.plain_s = res.plain_cumulative_s = None
    res.denoised_n_per_spot = res.denoised_s = res.denoised_cumulative_s = None
    res.first_rung_denoised_s = res.first_rung_passed = res.fallback = None
    cum_plain = cum_den = 0.0
    any_denoised = any(r.gamma_denoised is not None for r in res.rungs)
    for k, r in enumerate(res.rungs):
        cum_plain += r.run_s
        if r.gamma_denoised is not None and res.denoised_s is None:
            judged = r.run_s + r.denoise_s + (r.judge_s or 0.0)
            cum_den += judged
            if r.gamma_denoised >= TARGET:
                res.denoised_n_per_spot = r.n_per_spot
                res.denoised_s = judged
                res.denoised_cumulative_s = cum_den
            if k == 0:
                res.first_rung_passed = r.gamma_denoised >= TARGET
                res.first_rung_denoised_s = judged
        if r.gamma_plain >= TARGET and res.plain_s is None:
            res.plain_n_per_spot, res.plain_s = r.n_per_spot, r.run_s
            res.plain_cumulative_s = cum_plain
    if any_denoised:
        if res.first_rung_passed is False and res.first_rung_denoised_s is not None:
            res.first_rung_denoised_s = (res.first_rung_denoised_s + res.plain_s
                                         if res.plain_s is not None else None)
        res.fallback = res.denoised_s is None
        if res.fallback and res.plain_s is not None:
            res.denoised_n_per_spot = res.plain_n_per_spot
            res.denoised_s = res.plain_s
            res.denoised_cumulative_s = cum_den + res.plain_s
    return res


def time_to_gamma(spots_for: Callable[[int], list], phantom, seed: int, ladder: Sequence[int],
                  n_reference: int, denoise=None, name: str = "", launch=None,
                  log=print) -> TimeToGamma:
    """``spots_for(n)``: the plan's spots with n histories per spot;
    ``phantom``: a sde.DevicePhantom (materials already initialised);
    ``denoise(dose, rho, out)``: the trained network (or None).  Walks the
    ladder until the plain map passes, denoising every rung until a
    denoised map passes, then applies ``decide``."""
    import torch
    shape = tuple(phantom.material_id.shape)
    vcm = tuple(phantom.voxel_cm)
    ref = torch.zeros(shape, dtype=torch.float64, device="cuda")
    plan = sde.Plan(spots_for(n_reference), phantom, seed + 999_983, launch=launch)
    t_ref = _timed(lambda: plan.execute(ref))
    n_ref_total = plan.n_histories
    plan.close()
    log(f"[judge] {name} reference {n_ref_total} histories in {t_ref:.2f} s")
    res = TimeToGamma(name, n_ref_total, t_ref)
    dose = torch.zeros(shape, dtype=torch.float64, device="cuda")
    den = torch.zeros_like(dose)
    denoised_passed = False
    for k, n in enumerate(ladder):
        t0 = time.perf_counter()
        plan = sde.Plan(spots_for(n), phantom, seed + k, launch=launch)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        t_run = _timed(lambda: plan.execute(dose))
        rung = Rung(n, plan.n_histories, t_setup, t_run, gamma_pass(ref, dose, vcm))
        plan.close()
        if denoise is not None and not denoised_passed:
            rung.denoise_s, rung.denoise_gpu_s = _timed_gpu(
                lambda: denoise(dose, phantom.density, den), sde.library_stream())
            g = []
            rung.judge_s = _timed(lambda: g.append(gamma_pass(ref, den, vcm)))
            rung.gamma_denoised = g[0]
            denoised_passed = rung.gamma_denoised >= TARGET
        res.rungs.append(rung)
        log(f"[judge] {name} {n}/spot: {rung.histories} histories {t_run * 1e3:.1f} ms, "
            f"gamma plain {rung.gamma_plain:.4f}"
            + (f", denoised {rung.gamma_denoised:.4f} (+{rung.denoise_s * 1e3:.1f} ms, "
               f"judge {rung.judge_s * 1e3:.1f} ms)"
               if rung.gamma_denoised is not None else ""))
        if rung.gamma_plain >= TARGET:
            break
    return decide(res)
