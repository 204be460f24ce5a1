"""The judge's decisions (plain, denoised ladder, first rung with plain
fallback) from given rung results: host logic, no GPU."""

import os

import pytest

_LIB = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2511_03115_amd", "libsde.so")
if not os.path.exists(_LIB):            # the package's binding loads the library on import
    from paper_2511_03115_amd import build
    build.build()

from paper_2511_03115_amd.judge import Rung, TimeToGamma, decide  # noqa: E402


def _res(rows, judge=0.0):
    r = TimeToGamma("t", 0, 0.0)
    for n, run, gp, dn, gd in rows:
        r.rungs.append(Rung(n, n * 1000, 0.0, run, gp, dn, gd,
                            judge if gd is not None else None))
    return decide(r)


def test_denoised_ladder_beats_plain():
    r = _res([(1, 1.0, 0.5, 0.5, 0.80), (2, 2.0, 0.7, 0.5, 0.96), (4, 4.0, 0.93, None, None),
              (8, 8.0, 0.97, None, None)])
    assert r.plain_n_per_spot == 8 and r.plain_s == 8.0 and r.plain_cumulative_s == 15.0
    assert r.denoised_n_per_spot == 2 and r.denoised_s == 2.5
    assert r.denoised_cumulative_s == 1.5 + 2.5
    assert r.first_rung_passed is False and r.first_rung_denoised_s == 1.5 + 8.0
    assert r.fallback is False
    d = r.as_dict()
    assert d["speedup_ladder_selected"] == pytest.approx(8.0 / 2.5)
    assert d["speedup_first_rung"] == pytest.approx(8.0 / 9.5)


def test_judge_time_counts_in_the_denoised_times():
    """Every denoised rung's gamma evaluation is part of its time (the plain
    SDE judges each denoised map); plain runs carry none."""
    r = _res([(1, 1.0, 0.5, 0.5, 0.80), (2, 2.0, 0.7, 0.5, 0.96), (4, 4.0, 0.93, None, None),
              (8, 8.0, 0.97, None, None)], judge=0.25)
    assert r.plain_s == 8.0
    assert r.denoised_s == pytest.approx(2.0 + 0.5 + 0.25)
    assert r.denoised_cumulative_s == pytest.approx(1.75 + 2.75)
    assert r.first_rung_denoised_s == pytest.approx(1.75 + 8.0)
    assert r.as_dict()["judge_included"] is True


def test_first_rung_passes():
    r = _res([(1, 1.0, 0.6, 0.5, 0.955), (2, 2.0, 0.96, None, None)])
    assert r.first_rung_passed is True and r.first_rung_denoised_s == 1.5
    assert r.denoised_n_per_spot == 1 and r.fallback is False
    assert r.plain_n_per_spot == 2


def test_fallback_when_no_denoised_map_passes():
    r = _res([(1, 1.0, 0.5, 0.5, 0.9), (2, 2.0, 0.8, 0.5, 0.94), (4, 4.0, 0.96, 0.5, 0.949)])
    assert r.fallback is True
    assert r.denoised_n_per_spot == 4 and r.denoised_s == 4.0        # the plain run
    assert r.denoised_cumulative_s == 1.5 + 2.5 + 4.5 + 4.0
    assert r.first_rung_denoised_s == 1.5 + 4.0


def test_plain_never_passes():
    r = _res([(1, 1.0, 0.5, None, None), (2, 2.0, 0.8, None, None)])
    assert r.plain_s is None and r.denoised_s is None and r.fallback is None
    assert r.as_dict()["speedup_ladder_selected"] is None


def test_threshold_is_inclusive():
    r = _res([(1, 1.0, 0.95, 0.1, 0.95)])
    assert r.plain_n_per_spot == 1 and r.denoised_n_per_spot == 1 and r.first_rung_passed
