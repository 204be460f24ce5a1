"""Pins of the oracle's energy-dependent large-angle elastic cut.

Section 2.1.4 places the boundary between the Lynch-Dahl diffusion and the
large-angle elastic jumps at 2.5 sigma(E) and fixes it at 0.02 rad for the
runs; with the ECUT switch the oracle takes 2.5 sigma(E) itself, sigma the
Lynch-Dahl width of the medium at its density over the width's path z.
These tests check the cut against the width (pinned elsewhere against
Highland's formula), the rate against scipy quadrature of the CM cross
sections up to that cut, the samplers' inverse CDFs at those cuts, and the
jump count of whole tracks against the sum of the per-step probabilities.
"""

import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import workloads
from workloads.configs import PhysicsParams
from workloads.phantoms import Phantom

MP = 938.27208816
ECUT = oracle.ECUT


def _dcs_h(eta):
    def f(mu):   # Mott, units of (eta/k)^2
        L = math.log((1 + mu) / (1 - mu))
        return 2 / (1 - mu * mu) * ((1 + mu * mu) / (1 - mu * mu) - 0.5 * math.cos(eta * L))
    return f


def _quad(f, lo, hi):
    pts = [x for x in (-0.99, 0.0, 0.99, 0.9999) if lo < x < hi]
    edges = [lo, *pts, hi]
    return sum(integrate.quad(f, a, b, limit=400, epsrel=1e-12)[0] for a, b in zip(edges, edges[1:]))


def test_cut_is_two_and_a_half_lynch_dahl_widths(water, params):
    """The cut is 2.5 sigma(E) at the medium's density over the path z; the
    fixed cut without the switch."""
    for E in (5.0, 30.0, 150.0):
        for rho in (1.0, 0.26, 1.85):
            s = oracle.ld_sigma(water, rho, E, params.ld_z_cm, params.ld_F)
            assert oracle.elastic_cut(water, params, rho, E, flags=oracle.ELASTIC | ECUT) == \
                pytest.approx(2.5 * s, rel=1e-14)
            assert oracle.elastic_cut(water, params, rho, E, flags=oracle.ELASTIC) == 0.02


@pytest.mark.parametrize("E", [12.0, 70.0, 150.0])
def test_ecut_rate_vs_quadrature(water, params, E):
    """Total elastic rate of water with the cut 2.5 sigma(E): sum over H
    (Mott, from -cos 0.04) and O (Rutherford, from -1) of
    2 pi n_i int dcs dmu 1e-24 up to cos(2.5 sigma), by scipy quad."""
    tc = 2.5 * oracle.ld_sigma(water, 1.0, E, params.ld_z_cm, params.ld_F)
    tot = oracle.channel_total_rate(water, params, 1.0, E, flags=oracle.ELASTIC | ECUT)
    ref = 0.0
    for Z, A, w in zip(water.Z, water.A, water.w):
        nd = 6.02214076e23 * w / A
        e2k2 = (Z * 1.439964548 * (1 + A) / (2 * A * E)) ** 2 * 0.01
        if Z == 1:
            f = _dcs_h(7.2973525693e-3 * math.sqrt(MP / (2 * E)))
            lo = -math.cos(0.04)
        else:
            f = lambda mu: 1.0 / (1 - mu) ** 2
            lo = -1.0
        ref += 2 * math.pi * nd * e2k2 * _quad(f, lo, math.cos(tc)) * 1e-24
    assert abs(tot / ref - 1) < 1e-7, (E, tot, ref)
    # the cut narrows with energy: the rate is ~30x the fixed cut's at 150 MeV
    if E == 150.0:
        fixed = oracle.channel_total_rate(water, params, 1.0, E, flags=oracle.ELASTIC)
        assert 20 < tot / fixed < 40


@pytest.mark.parametrize("E", [12.0, 70.0, 150.0])
def test_ecut_samplers_invert_their_cdf(water, params, E):
    """At the cut 2.5 sigma(E): the Rutherford 1 - mu and the hydrogen mu
    drawn for U have CDF U (scipy quadrature of the cross sections)."""
    tc = 2.5 * oracle.ld_sigma(water, 1.0, E, params.ld_z_cm, params.ld_F)
    hi = math.cos(tc)
    f = lambda mu: 1.0 / (1 - mu) ** 2
    tot = _quad(f, -1.0, hi)
    for U in (0.02, 0.4, 0.9, 0.999):
        mu = 1 - oracle.lib().or_rutherford_one_minus_mu(U, tc)
        assert abs(_quad(f, -1.0, mu) / tot - U) < 1e-7
    g = _dcs_h(7.2973525693e-3 * math.sqrt(MP / (2 * E)))
    lo = -math.cos(0.04)
    tot = _quad(g, lo, hi)
    for U in (0.05, 0.5, 0.95):
        mu = oracle.lib().or_mott_sample_mu(E, U, tc, 0.04)
        assert abs(_quad(g, lo, mu) / tot - U) < 1e-7


def test_ecut_limits_at_low_energy(water, params):
    """Where 2.5 sigma(E) reaches pi (a few hundred keV in water), the
    Rutherford interval [-1, cos(cut)] is empty and hydrogen's closes at
    pi - 0.04: the elastic rate falls to zero instead of turning negative."""
    E = 0.06
    assert oracle.elastic_cut(water, params, 1.0, E, flags=ECUT) > math.pi
    assert oracle.channel_total_rate(water, params, 1.0, E, flags=oracle.ELASTIC | ECUT) == 0.0
    for E in (0.2, 1.0, 3.0):
        assert oracle.channel_total_rate(water, params, 1.0, E, flags=oracle.ELASTIC | ECUT) > 0.0


def _slab(thick_cm, mat, half_width_cm=50.0):
    mid = np.zeros((1, 1, 1), dtype=np.uint8)
    rho = np.full((1, 1, 1), mat.rho_nominal, dtype=np.float32)
    return Phantom((1, 1, 1), (2 * half_width_cm, 2 * half_width_cm, thick_cm),
                   (-half_width_cm, -half_width_cm, 0.0), mid, rho, [mat])


def test_ecut_jump_count_of_tracks(water):
    """Loss and elastic jumps with the cut 2.5 sigma(E), 40 steps from
    150 MeV (the energies are deterministic, elastic jumps keep them): the
    mean number of jumps is sum_k (1 - exp(-Delta rate(E_k))) within four
    standard errors of the Poisson-binomial law."""
    E0, nst, n = 150.0, 40, 200_000
    D = 0.05
    p = PhysicsParams(max_steps=nst)
    flags = oracle.LOSS | oracle.ELASTIC | ECUT
    E, pk = E0, []
    for _ in range(nst):
        rate = oracle.channel_total_rate(water, p, 1.0, E, flags=flags)
        pk.append(-math.expm1(-D * rate))
        E = E - oracle.stopping_mass(water, E) * D
    pk = np.array(pk)
    r = oracle.transport(_slab(5.0, water), workloads.single_spot(E0, n), p, None, seed=33,
                         flags=flags, tally=False, records=True)
    rec = r.records
    assert np.mean(rec[:, oracle.R_END] == oracle.END_MAXSTEPS) > 0.999
    k = rec[:, oracle.R_NEL]
    mean, var = pk.sum(), (pk * (1 - pk)).sum()
    assert abs(k.mean() - mean) < 4 * math.sqrt(var / n), (k.mean(), mean)
    assert mean > 1.0     # ~3 % per step at 150 MeV: the switch is on


def test_ecut_sampled_angles_respect_the_cut(water):
    """One step with loss and elastic jumps only (no small-angle diffusion):
    every jumped history leaves at a lab angle at least the CM -> lab image
    of the cut for the lighter target (hydrogen), and most jumps lie below
    what the fixed 0.02 rad cut allows (the drawn CM angles use the
    energy-dependent cut, not only the rate)."""
    E0, n = 150.0, 200_000
    p = PhysicsParams(max_steps=1)
    flags = oracle.LOSS | oracle.ELASTIC | ECUT
    r = oracle.transport(_slab(5.0, water), workloads.single_spot(E0, n), p, None, seed=5,
                         flags=flags, tally=False, records=True)
    rec = r.records
    jumped = rec[:, oracle.R_NEL] > 0
    assert jumped.sum() > 3000
    th = np.arccos(np.clip(rec[jumped, oracle.R_OZ], -1, 1))
    tc = oracle.elastic_cut(water, p, 1.0, E0, flags=flags)
    cm2lab = oracle.lib().or_cm_to_lab
    lo = min(cm2lab(E0, A, math.cos(tc), math.sin(tc), 0.0) for A in water.A)
    fixed_lo = min(cm2lab(E0, A, math.cos(0.02), math.sin(0.02), 0.0) for A in water.A)
    assert th.min() >= lo * (1 - 1e-6), (th.min(), lo)
    assert np.mean(th < fixed_lo) > 0.5, (np.mean(th < fixed_lo), fixed_lo)
