"""Pins of the oracle's elastic nuclear arithmetic (section 2.1.4).

The ENDF/JEFF values are not in the container, so the data are synthetic
(``workloads.synthetic_elastic_nuclear``: smooth shapes, seeded); what is
pinned is the arithmetic that consumes them:

* the uniform cubic B-spline of P_NI(mu, E) and of a_l(E), b_l(E) against
  scipy's BSpline, and the integral of P_NI against BSpline.integrate;
* sigma_NI P_NI linear in the lattice coordinate between lattice energies;
* the hydrogen nuclear term Eq. (hydrogen_not_ruther): even in mu (as the
  paper notes), its isotropic b_0 limit, and its antiderivative by
  Appendix A.2's recursion against scipy quadrature of the literal formula;
* the summed cross sections' samplers (Eq. (large_elastic_cdf)) against
  quadrature, and the rates against quadrature.

The physical values of the synthetic tables are parity unpinned.
"""

import math

import numpy as np
import pytest
from scipy import integrate
from scipy.interpolate import BSpline

import oracle
import workloads
from workloads.nuclear import (EnergyLattice, placeholder_nuclear_tables,
                               synthetic_elastic_nuclear, with_elastic_nuclear)

MP = 938.27208816


@pytest.fixture(scope="module")
def tables(water):
    lat = EnergyLattice(n=64)
    nt = placeholder_nuclear_tables(water.Z, water.A, lat)
    el = synthetic_elastic_nuclear(water.Z, water.A, lat, n_mu=24, n_l=8, seed=3)
    return with_elastic_nuclear(nt, el)


@pytest.fixture(scope="module")
def view(tables):
    return oracle.NuclearView(tables)


def _uniform_bspline(c, m, x0, h):
    knots = x0 + (np.arange(len(c) + 4) - 3.0) * h
    return BSpline(knots, np.asarray(c, dtype=np.float64), 3, extrapolate=False)


def test_bspline_is_scipys():
    """The uniform cubic B-spline (knots x0 + (j - 3) h) equals scipy's
    BSpline on its interval, at random coefficients."""
    rng = np.random.default_rng(1)
    for m, x0, h in ((5, -1.0, 0.4), (21, -1.0, 2 / 21), (63, 0.0, 1.0)):
        c = rng.standard_normal(m + 3)
        sp = _uniform_bspline(c, m, x0, h)
        for x in np.linspace(x0, x0 + m * h, 37):
            assert abs(oracle.bspline3(c, m, x0, h, x) - sp(x)) < 1e-12 * (1 + abs(sp(x)))


def test_p_ni_integral_is_bspline_integral(tables, view):
    """int_{-1}^{x} P_NI(mu, E_i) dmu equals scipy's BSpline.integrate, and
    the synthetic P_NI integrates to 1 over [-1, 1]."""
    el = tables.elastic
    m = el.ni_p.shape[-1] - 3
    for i in (0, 17, 40, 63):
        sp = _uniform_bspline(el.ni_p[0, i], m, -1.0, 2.0 / m)
        for x in (-1.0, -0.73, 0.0, 0.41, 0.9998, 1.0):
            want = sp.integrate(-1.0, x) if x > -1.0 else 0.0
            assert abs(view.p_ni_integral(0, i, x) - want) < 1e-12
        assert abs(view.p_ni_integral(0, i, 1.0) - 1.0) < 1e-12
    # and P_NI >= 0 (a density)
    mu = np.linspace(-1, 1, 401)
    assert min(_uniform_bspline(el.ni_p[0, i], m, -1.0, 2.0 / m)(mu).min()
               for i in range(0, 64, 7)) > 0.0


def test_ni_term_linear_in_the_lattice_coordinate(tables, view):
    """sigma_NI P_NI at E between lattice energies is the linear blend, in the
    lattice coordinate, of its values at the two neighbours (density and
    integral)."""
    el, lat = tables.elastic, tables.lattice
    m = el.ni_p.shape[-1] - 3
    Es = lat.energies()
    for E in (0.31, 7.7, 64.0, 151.3, 259.0):
        t = (math.log(E) - math.log(lat.e_lo)) / (math.log(lat.e_hi) - math.log(lat.e_lo)) * (lat.n - 1)
        i = min(int(t), lat.n - 2)
        f = t - i
        for mu in (-0.5, 0.2, 0.97):
            s = [_uniform_bspline(el.ni_p[0, k], m, -1.0, 2.0 / m) for k in (i, i + 1)]
            want = (1 - f) * el.ni_sigma[0, i] * s[0](mu) + f * el.ni_sigma[0, i + 1] * s[1](mu)
            assert abs(view.ni_density(0, E, mu) - want) < 1e-12 * abs(want)
            want_i = ((1 - f) * el.ni_sigma[0, i] * s[0].integrate(-1, mu) +
                      f * el.ni_sigma[0, i + 1] * s[1].integrate(-1, mu))
            assert abs(view.ni_integral(0, E, mu) - want_i) < 1e-12 * abs(want_i)


def test_hydrogen_term_is_even_and_isotropic_limit(tables, view):
    """sigma_N^c(mu) = sigma_N^c(-mu) (the paper uses this evenness in
    Appendix A.2); with only b_0 it is b_0 / 2 (the l = 0 term)."""
    for E in (5.0, 60.0, 200.0):
        for mu in (0.1, 0.5, 0.93, 0.999):
            a, b = view.h_nuclear_density(E, mu), view.h_nuclear_density(E, -mu)
            assert abs(a - b) < 1e-12 * max(abs(a), 1e-12), (E, mu, a, b)
    el = tables.elastic
    iso = workloads.nuclear.ElasticNuclear(
        ni_Z=el.ni_Z, ni_sigma=el.ni_sigma, ni_p=el.ni_p, h_are=np.zeros((1, el.h_b.shape[1])),
        h_aim=np.zeros((1, el.h_b.shape[1])), h_b=np.full((1, el.h_b.shape[1]), 0.02))
    v = oracle.NuclearView(with_elastic_nuclear(tables, iso))
    for mu in (-0.8, 0.0, 0.6):
        assert abs(v.h_nuclear_density(80.0, mu) - 0.01) < 1e-15


@pytest.mark.parametrize("E", [3.0, 45.0, 150.0, 230.0])
def test_hydrogen_antiderivative_recursion_vs_quadrature(view, E):
    """Appendix A.2: the antiderivative of sigma_N^c built from the recursive
    antiderivatives of (1 +- mu)^-1 cos/sin(eta ln((1 +- mu)/2)) and repeated
    integration by parts equals scipy's quadrature of the literal Eq.
    (hydrogen_not_ruther) on intervals across [-cos 0.04, cos 0.02]."""
    f = lambda mu: view.h_nuclear_density(E, mu)
    pts = [-math.cos(0.04), -0.9, -0.3, 0.0, 0.5, 0.95, 0.999, math.cos(0.02)]
    for a, b in zip(pts, pts[1:]):
        want = integrate.quad(f, a, b, limit=400, epsabs=0, epsrel=1e-12)[0]
        got = view.h_nuclear_antiderivative(E, b) - view.h_nuclear_antiderivative(E, a)
        assert abs(got - want) < 1e-9 * max(abs(want), 1e-6), (E, a, b, got, want)


def _mott_barn(E, A):
    eta = 7.2973525693e-3 * math.sqrt(MP / (2 * E))
    e2k2 = (1.439964548 * (1 + A) / (2 * A * E)) ** 2 * 0.01

    def f(mu):
        L = math.log((1 + mu) / (1 - mu))
        return e2k2 * 2 / (1 - mu * mu) * ((1 + mu * mu) / (1 - mu * mu) - 0.5 * math.cos(eta * L))
    return f


def _quad(f, lo, hi):
    pts = [x for x in (-0.99, 0.0, 0.99, 0.9999) if lo < x < hi]
    edges = [lo, *pts, hi]
    return sum(integrate.quad(f, a, b, limit=400, epsrel=1e-12)[0] for a, b in zip(edges, edges[1:]))


@pytest.mark.parametrize("E", [20.0, 150.0])
def test_summed_samplers_invert_their_cdf(water, view, E):
    """The CM cosine drawn for U from the summed cross sections (hydrogen:
    Mott + sigma_N on [-cos 0.04, cos 0.02]; oxygen: Rutherford +
    sigma_NI P_NI on [-1, cos 0.02]) has CDF U by scipy quadrature, and the
    summed densities are positive."""
    A_h, A_o = water.A[0], water.A[1]
    lo, hi = -math.cos(0.04), math.cos(0.02)
    fh = lambda mu: _mott_barn(E, A_h)(mu) + view.h_nuclear_density(E, mu)
    assert min(fh(x) for x in np.linspace(lo, hi, 301)) > 0
    tot = _quad(fh, lo, hi)
    assert abs(view.elastic_cum_barn(1, A_h, E, lo, hi) / tot - 1) < 1e-9
    for U in (0.03, 0.5, 0.97):
        mu = view.elastic_sample_mu(1, A_h, E, U)
        assert abs(_quad(fh, lo, mu) / tot - U) < 1e-8
    e2k2 = (8 * 1.439964548 * (1 + A_o) / (2 * A_o * E)) ** 2 * 0.01
    fo = lambda mu: e2k2 / (1 - mu) ** 2 + view.ni_density(0, E, mu)
    tot = _quad(fo, -1.0, hi)
    for U in (0.03, 0.5, 0.97):
        mu = view.elastic_sample_mu(8, A_o, E, U)
        assert abs(_quad(fo, -1.0, mu) / tot - U) < 1e-8


@pytest.mark.parametrize("E", [30.0, 120.0])
def test_rates_include_the_nuclear_terms(water, params, tables, view, E):
    """The elastic rate with the nuclear data is the Coulomb rate plus
    2 pi n_i 1e-24 times each element's nuclear integral (quadrature)."""
    base = oracle.channel_total_rate(water, params, 1.0, E, flags=oracle.ELASTIC)
    tot = oracle.channel_total_rate(water, params, 1.0, E, tables, flags=oracle.ELASTIC)
    lo, hi = -math.cos(0.04), math.cos(0.02)
    add = 0.0
    for Z, A, w in zip(water.Z, water.A, water.w):
        nd = 6.02214076e23 * w / A
        if Z == 1:
            x = _quad(lambda mu: view.h_nuclear_density(E, mu), lo, hi)
        else:
            x = _quad(lambda mu: view.ni_density(0, E, mu), -1.0, hi)
        add += 2 * math.pi * nd * x * 1e-24
    assert abs((tot - base) / add - 1) < 1e-8, (E, tot - base, add)
    assert add > 0.02 * base      # the synthetic nuclear terms matter


def test_transport_with_elastic_nuclear_data_conserves_energy(tables):
    """Whole tracks with the nuclear elastic terms: per-history energy
    balance to 1e-12, and more elastic jumps than without them."""
    wl = workloads.configs.water100_small(n=2000)
    from dataclasses import replace
    p = replace(wl.params, n_energy=tables.lattice.n)
    plain = placeholder_nuclear_tables(wl.phantom.materials[0].Z, wl.phantom.materials[0].A,
                                       tables.lattice)
    r0 = oracle.transport(wl.phantom, wl.spots, p, plain, seed=4, records=True, tally=False)
    r1 = oracle.transport(wl.phantom, wl.spots, p, tables, seed=4, records=True, tally=False)
    rec = r1.records
    bal = (rec[:, oracle.R_DEP] + rec[:, oracle.R_ESC] + rec[:, oracle.R_NUC] +
           rec[:, oracle.R_TRUNC] - rec[:, oracle.R_E0])
    assert np.abs(bal).max() <= 1e-12 * rec[:, oracle.R_E0].max()
    assert rec[:, oracle.R_NEL].sum() > r0.records[:, oracle.R_NEL].sum()
