"""The double-precision instance of the transport and the random numbers,
through the C ABI, against the FP64 oracle.

The water parity workload is stated in FP64 at 1e4 histories (100 MeV point
beam, 40 x 40 x 150 mm water, seed 0).  Stepping in double precision, with the
Lynch-Dahl width and the elastic rate from their formulas, the GPU follows
the oracle history by history, so the bar (per-voxel |dose difference| <=
1e-3 of the maximum, gamma >= 99 % at 1 %/0.5 mm, |dR80| <= 0.1 mm) holds at
the stated size and below it.  The FP32 production instance at the same size
is reported with the histories whose discrete path differs, by index.
"""

import numpy as np
import pytest

import oracle
from workloads import configs
from gpu_common import (history_agreement, log, nuclear_for, parity_metrics, run_gpu,
                        run_gpu_records, run_oracle)

pytestmark = pytest.mark.gpu

FP64 = 128


def _bar(m):
    assert m["max_rel_diff"] <= 1e-3, m
    assert m["gamma_1pct_05mm"] >= 0.99, m
    assert m["dr80_mm"] <= 0.1, m


def test_philox_words_match_oracle():
    """The transport's Philox4x32-10 words (its own device function, through
    sde_philox_words) equal the oracle's bit for bit on 1e6 counters: random
    (h, n, b), the source block n = 2^32 - 1, and the extreme h and seeds."""
    import torch
    from paper_2511_03115_amd import sde
    rng = np.random.default_rng(12)
    m = 1_000_000
    h = rng.integers(0, 2 ** 63, m, dtype=np.int64).astype(np.uint64) * np.uint64(2) + \
        rng.integers(0, 2, m).astype(np.uint64)
    n = rng.integers(0, 2 ** 32, m, dtype=np.uint64).astype(np.uint32)
    b = rng.integers(0, 3, m).astype(np.uint32)
    h[:8] = [0, 1, 2 ** 32 - 1, 2 ** 32, 2 ** 64 - 1, 12345, 2 ** 63, 7]
    n[:8] = [0, 2 ** 32 - 1, 1, 0, 2 ** 32 - 1, 2 ** 32 - 1, 5, 0]
    n[8:1000] = 2 ** 32 - 1
    for seed in (0, 1, 6, 2 ** 64 - 1, 0x9E3779B97F4A7C15):
        dh = torch.from_numpy(h.view(np.int64)).cuda()
        dn = torch.from_numpy(n.view(np.int32)).cuda()
        db = torch.from_numpy(b.view(np.int32)).cuda()
        got = sde.philox_words(seed, dh, dn, db).cpu().numpy().view(np.uint32)
        want = oracle.rng_blocks(seed, h, n, b)
        bad = int(np.sum(np.any(got != want, axis=1)))
        log(f"philox seed={seed}: {bad} of {m} blocks differ")
        assert bad == 0


def test_parity_water100_fp64_stated_size():
    """The water parity workload as stated: FP64, 1e4 histories, seed 0, the
    method; all three bars, the ledger balanced, and history by history the
    same discrete path as the oracle."""
    wl = configs.water100_small(n=10_000)
    flags = oracle.ALL | FP64
    log(f"case water100_small fp64 seed={wl.seed} n={wl.n_histories}")
    d_gpu, tal, led, scale = run_gpu(wl, flags=flags)
    d_ref, led_ref = run_oracle(wl, flags=oracle.ALL)
    m = parity_metrics(d_ref, d_gpu, wl.phantom)
    log(f"metrics {m}")
    assert led[6] == wl.n_histories
    bal = led[0] + led[1] + led[2] + led[4] - led[3]
    assert abs(bal) <= 2 * led[5] + 1e-6 * led[3], (bal, led)
    assert abs(led[0] / scale - led_ref[oracle.L_DEP]) <= 1e-6 * led_ref[oracle.L_E0]
    assert int(tal.sum()) == int(led[0])
    _bar(m)
    g, _ = run_gpu_records(wl, flags=flags)
    r = oracle.transport(wl.phantom, wl.spots, wl.params, nuclear_for(wl.phantom, wl.params),
                         seed=wl.seed, records=True, tally=False, flags=oracle.ALL)
    a = history_agreement(g, r.records)
    log(f"agreement {a}")
    assert a["e0_equal"] == 1.0
    assert a["same_frac"] >= 0.9999
    assert a["pos_p99"] < 5e-6   # float32 records of both end points


@pytest.mark.parametrize("flags", [
    oracle.LOSS | oracle.STRAGGLE | oracle.EOR,
    oracle.LOSS | oracle.MCS | oracle.SBM | oracle.EOR,
    oracle.LOSS | oracle.ELASTIC | oracle.INELASTIC | oracle.EOR,
    oracle.LOSS | oracle.STRAGGLE | oracle.MCS | oracle.SBM,
    oracle.ALL & ~oracle.SBM,
])
def test_parity_fp64_subsets_small(flags):
    """Physics subsets in double precision at 3e3 histories, a third of the
    stated size: the bar holds without the extra histories single precision
    needs."""
    wl = configs.water100_small(n=3_000)
    log(f"case fp64 subset flags={flags}")
    d_gpu, _, _, _ = run_gpu(wl, flags=flags | FP64)
    d_ref, _ = run_oracle(wl, flags=flags)
    m = parity_metrics(d_ref, d_gpu, wl.phantom)
    log(f"metrics {m}")
    _bar(m)


def test_fp32_at_stated_size_reported():
    """The single-precision method at the stated 1e4 histories: gamma and R80
    meet the bar; the per-voxel difference is reported together with the
    histories (by index) whose discrete path differs from the oracle's, which
    carry it.  At most 10 such histories."""
    wl = configs.water100_small(n=10_000)
    log(f"case water100_small fp32 seed={wl.seed} n={wl.n_histories}")
    d_gpu, _, _, _ = run_gpu(wl)
    d_ref, _ = run_oracle(wl)
    m = parity_metrics(d_ref, d_gpu, wl.phantom)
    log(f"metrics {m}")
    g, _ = run_gpu_records(wl)
    r = oracle.transport(wl.phantom, wl.spots, wl.params, nuclear_for(wl.phantom, wl.params),
                         seed=wl.seed, records=True, tally=False)
    o = r.records
    oj = o[:, oracle.R_NEL] + o[:, oracle.R_NNE]
    diff = np.nonzero((g[:, 1] != o[:, oracle.R_STEPS]) | (g[:, 2] != oj) |
                      (g[:, 3] != o[:, oracle.R_END]) | (g[:, 8] != o[:, oracle.R_J1]) |
                      (g[:, 9] != o[:, oracle.R_J2]))[0]
    for k in diff:
        log(f"flip h={k}: gpu steps={g[k, 1]:.0f} jumps={g[k, 2]:.0f} end={g[k, 3]:.0f} "
            f"j1={g[k, 8]:.0f} j2={g[k, 9]:.0f} | oracle steps={o[k, oracle.R_STEPS]:.0f} "
            f"jumps={oj[k]:.0f} end={o[k, oracle.R_END]:.0f} j1={o[k, oracle.R_J1]:.0f} "
            f"j2={o[k, oracle.R_J2]:.0f}")
    log(f"fp32 at 1e4: max_rel_diff={m['max_rel_diff']:.3e} with {len(diff)} histories on "
        f"another discrete path")
    assert m["gamma_1pct_05mm"] >= 0.99 and m["dr80_mm"] <= 0.1, m
    assert len(diff) <= 10


ECUT = 256


@pytest.mark.parametrize("flags,n", [
    (oracle.LOSS | oracle.ELASTIC | oracle.EOR | ECUT, 10_000),
    (oracle.ALL | ECUT, 30_000),
    (oracle.ALL | ECUT | FP64, 10_000),
])
def test_parity_energy_dependent_cut(flags, n):
    """The large-angle elastic cut at 2.5 sigma(E) (section 2.1.4) instead of
    0.02 rad: the general single-precision instance and the FP64 instance
    against the oracle with the same switch, all three bars."""
    wl = configs.water100_small(n=n)
    log(f"case ecut flags={flags} n={n}")
    d_gpu, tal, led, scale = run_gpu(wl, flags=flags)
    d_ref, led_ref = run_oracle(wl, flags=flags & ~FP64)
    m = parity_metrics(d_ref, d_gpu, wl.phantom)
    log(f"metrics {m} jumps gpu {led[7]} oracle {led_ref[oracle.L_JUMPS]:.0f}")
    assert abs(led[7] - led_ref[oracle.L_JUMPS]) <= 0.01 * led_ref[oracle.L_JUMPS] + 10
    _bar(m)


@pytest.mark.parametrize("E", [100.0, 150.0])
def test_energy_dependent_cut_effect(E):
    """What the energy-dependent cut changes, on the GPU (1e6 histories of
    the water beam model on the 40 x 40 x 150 mm (100 MeV) or
    40 x 40 x 200 mm (150 MeV) box): large-angle jumps per history (several
    times more), the IDD's largest relative change before the peak and the
    R80 shift, logged; the R80 moves by less than 0.5 mm.  Measured: 2.28 ->
    4.58 jumps per history at 100 MeV and 2.45 -> 9.06 at 150 MeV (the rate
    with the cut is ~0.6 per cm at every energy, the fixed cut's falls as
    1/E^2)."""
    from dataclasses import replace
    from workloads.phantoms import water_box
    from workloads.beams import single_spot
    n = 1_000_000
    wl = configs.Workload(f"water{int(E)}_cut", water_box(40, 40, 150 if E < 120 else 200, 0.1),
                          single_spot(E, n, sigmaE_rel=0.01, sigma_xy_cm=0.3), 17)
    out = {}
    for name, flags in (("fixed", oracle.ALL), ("ecut", oracle.ALL | ECUT)):
        d, _, led, _ = run_gpu(wl, flags=flags)
        out[name] = (d, led[7] / led[6])
    idd0, idd1 = oracle.idd(out["fixed"][0]), oracle.idd(out["ecut"][0])
    ipk = int(np.argmax(idd0))
    rel = np.abs(idd1[:ipk] - idd0[:ipk]) / idd0[:ipk]
    r0 = oracle.range_rx(out["fixed"][0], 0.1, 0.8)
    r1 = oracle.range_rx(out["ecut"][0], 0.1, 0.8)
    log(f"cut effect E={E}: jumps/history fixed {out['fixed'][1]:.3f} ecut {out['ecut'][1]:.3f}; "
        f"IDD max rel change before the peak {rel.max():.4f} (mean {rel.mean():.4f}); "
        f"R80 {r0:.4f} -> {r1:.4f} cm")
    assert out["ecut"][1] > 1.5 * out["fixed"][1]
    assert abs(r1 - r0) < 0.05
