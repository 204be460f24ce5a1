"""Pins of the oracle's source sampler and inelastic branch.

The source and the inelastic draw consume the same Philox words on both
sides, so a mistake shared by the oracle's reading of them would pass every
GPU parity test.  These tests check them against what fixes them instead:
the spot's Gaussian moments (section 2.2.2 beam as the workloads state it),
exactness of linear interpolation on tables that are linear in the lattice
coordinate, the closed-form loss-fraction law the placeholder tables are
written from, the Kalbach-Mann distribution function, and an explicit
Lorentz boost of the CM momentum four-vector (Appendix A.1).
"""

import math

import numpy as np
import pytest
from scipy import stats

import oracle
from workloads.beams import Spot
from workloads.nuclear import EnergyLattice, NuclearTables, placeholder_nuclear_tables

MP = 938.27208816
AMU = 931.49410242


# --------------------------------------------------------------------------
# Source (Gaussian pencil beam on the entrance face)
# --------------------------------------------------------------------------

def test_source_moments_and_normality():
    """2e5 histories of a spot E = 150 MeV, sigma_E = 1 %, centre (0.7, -0.4)
    cm, sigma_xy = 0.3 cm: means and variances of E0, x0, y0 within 4
    standard errors, the three uncorrelated, each standardised coordinate
    normal by Kolmogorov-Smirnov, and z0 the entrance face.  Using sigma as
    a variance, a wrong centre, a shared normal for x and y, or the energy
    spread applied absolutely fails one of these."""
    sp = Spot(150.0, 0.01, 0.7, -0.4, 0.3, 1.0, 200_000)
    n = sp.n_histories
    s = oracle.source(sp, -1.25, seed=3, h0=12345, n=n)
    E, x, y, z = s[:, 0], s[:, 1], s[:, 2], s[:, 3]
    assert np.all(z == -1.25)
    for v, mu, sd in ((E, 150.0, 1.5), (x, 0.7, 0.3), (y, -0.4, 0.3)):
        assert abs(v.mean() - mu) < 4 * sd / math.sqrt(n), (v.mean(), mu)
        var_se = sd * sd * math.sqrt(2.0 / (n - 1))
        assert abs(v.var(ddof=1) - sd * sd) < 4 * var_se, (v.var(ddof=1), sd * sd)
        assert stats.kstest((v - mu) / sd, "norm").pvalue > 1e-3
    c = np.corrcoef(np.vstack([E, x, y]))
    assert np.all(np.abs(c[np.triu_indices(3, 1)]) < 4 / math.sqrt(n)), c


def test_source_point_beam_is_exact():
    """A point monoenergetic spot starts every history at its nominal energy
    and centre."""
    sp = Spot(100.0, 0.0, 0.25, -0.5, 0.0, 1.0, 1000)
    s = oracle.source(sp, 0.0, seed=0, h0=0, n=1000)
    assert np.all(s[:, 0] == 100.0) and np.all(s[:, 1] == 0.25) and np.all(s[:, 2] == -0.5)


def test_source_independent_histories():
    """Consecutive histories of one spot are independent draws: the lag-1
    correlation of E0 is within 4/sqrt(n) of zero, and the history index, not
    the position in the batch, keys the draw."""
    sp = Spot(120.0, 0.02, 0.0, 0.0, 0.5, 1.0, 50_000)
    s = oracle.source(sp, 0.0, seed=9, h0=0, n=50_000)
    r = np.corrcoef(s[:-1, 0], s[1:, 0])[0, 1]
    assert abs(r) < 4 / math.sqrt(50_000)
    tail = oracle.source(sp, 0.0, seed=9, h0=49_990, n=10)
    assert np.array_equal(tail, s[-10:])


# --------------------------------------------------------------------------
# Inelastic branch: lattice position, rate and (E, u) tables
# --------------------------------------------------------------------------

def _lattice_coord(lat, E):
    """Position of E on the lattice uniform in ln E, clamped to its ends."""
    t = (math.log(E) - math.log(lat.e_lo)) / (math.log(lat.e_hi) - math.log(lat.e_lo)) * (lat.n - 1)
    return min(max(t, 0.0), lat.n - 1.0)


def _bilinear_tables(lat, n_u):
    """Two elements with every table bilinear in (lattice index i, u index j),
    c0 + c1 i + c2 j + c3 i j, different coefficients per element and table,
    so that bilinear interpolation is exact and any transposition of i and j
    (n_e != n_u) or of the three tables shows."""
    i = np.arange(lat.n)[:, None].astype(np.float64)
    j = np.arange(n_u)[None, :].astype(np.float64)
    coef = {}
    tabs = {}
    for name, base in (("u", 0.01), ("r", 0.2), ("a", 1.0)):
        arr = np.zeros((2, lat.n, n_u))
        for t in range(2):
            c = (base * (t + 1), 3e-3 * (t + 2), 7e-3 / (t + 1), -2e-5 * (t + 1))
            coef[(name, t)] = c
            arr[t] = c[0] + c[1] * i + c[2] * j + c[3] * i * j
        tabs[name] = arr
    sig = np.vstack([0.3 + 0.01 * np.arange(lat.n), 2.0 - 0.015 * np.arange(lat.n)])
    nt = NuclearTables(lattice=lat, n_u=n_u, Z=np.array([6, 8], dtype=np.int32),
                       A=np.array([12.011, 15.999]), sigma=sig, u_icdf=tabs["u"],
                       kalbach_r=tabs["r"], kalbach_a=tabs["a"])
    return nt, coef


def test_inelastic_tables_exact_on_bilinear_data():
    """sigma(E) linear in the lattice coordinate and every (E, u) table
    bilinear in (lattice coordinate, u index): the oracle's interpolation
    reproduces them to rounding at random (E, x), including the clamped ends."""
    lat = EnergyLattice(n=37, e_lo=0.05, e_hi=260.0)
    n_u = 9
    nt, coef = _bilinear_tables(lat, n_u)
    view = oracle.NuclearView(nt)
    rng = np.random.default_rng(5)
    Es = np.concatenate([np.exp(rng.uniform(math.log(0.05), math.log(260.0), 200)),
                         [0.05, 260.0, 0.01, 400.0]])
    for E in Es:
        tau = _lattice_coord(lat, E)
        for t in range(2):
            want = (0.3 + 0.01 * tau) if t == 0 else (2.0 - 0.015 * tau)
            assert abs(view.sigma_barn(t, E) - want) < 1e-12 * max(1.0, abs(want))
        for x in (0.0, 1.0, -0.5, 1.5, *rng.uniform(0, 1, 5)):
            xi = min(max(x, 0.0), 1.0) * (n_u - 1)
            for name in ("u", "r", "a"):
                for t in range(2):
                    c = coef[(name, t)]
                    want = c[0] + c[1] * tau + c[2] * xi + c[3] * tau * xi
                    got = view.table(t, name, E, x)
                    assert abs(got - want) < 1e-11, (name, t, E, x, got, want)


def test_lattice_position_at_nodes():
    """At the lattice energies E_i = exp(ln e_lo + i d) the position is i
    (the last node is the top of the last interval)."""
    lat = EnergyLattice(n=101, e_lo=0.05, e_hi=260.0)
    nt, _ = _bilinear_tables(lat, 5)
    view = oracle.NuclearView(nt)
    for i, E in enumerate(lat.energies()):
        k, f = view.lattice_pos(E)
        assert 0 <= k <= lat.n - 2 and 0.0 <= f <= 1.0
        assert abs(k + f - i) < 1e-9, (i, k, f)


def _oxygen_tables(n_u=33, n=1024):
    return placeholder_nuclear_tables([1, 8], [1.008, 15.999], EnergyLattice(n=n), n_u=n_u)


def test_placeholder_kalbach_lookup():
    """Kalbach r and a looked up at lattice energies and u nodes are the
    placeholder's defining values r = 0.1 + 0.5 (1 - u),
    a = 0.5 + 2 (1 - u) + E/200; r, linear in u and constant in E, is exact
    everywhere; hydrogen has no table."""
    nt = _oxygen_tables()
    assert list(nt.Z) == [8]
    view = oracle.NuclearView(nt)
    Es = nt.lattice.energies()
    for i in (0, 17, 512, 900, 1023):
        for j in (0, 5, 16, 31, 32):
            u = j / 32.0
            assert abs(view.table(0, "r", Es[i], u) - (0.1 + 0.5 * (1 - u))) < 1e-12
            want_a = 0.5 + 2.0 * (1 - u) + Es[i] / 200.0
            assert abs(view.table(0, "a", Es[i], u) - want_a) < 1e-9 * want_a
    rng = np.random.default_rng(2)
    for E, u in zip(np.exp(rng.uniform(math.log(0.05), math.log(260), 50)), rng.uniform(0, 1, 50)):
        assert abs(view.table(0, "r", E, u) - (0.1 + 0.5 * (1 - u))) < 1e-12


def _trunc_exp_cdf(u, E, u_min=0.02):
    """The placeholder's loss-fraction law: exponential of scale
    0.15 + 0.15 E/250 truncated to [u_min, 1]."""
    lam = 0.15 + 0.15 * E / 250.0
    return (1.0 - np.exp(-(u - u_min) / lam)) / (1.0 - math.exp(-(1.0 - u_min) / lam))


@pytest.mark.parametrize("i", [700, 950])
def test_loss_fraction_law(i):
    """Loss fractions drawn through the inverse-CDF table (1025 u nodes) at a
    lattice energy follow the closed-form truncated exponential the table is
    written from (Kolmogorov-Smirnov, 1e5 draws; the table's own
    interpolation moves the law by < 2e-4).  Drawing with 1 - U or from the
    wrong table fails."""
    nt = _oxygen_tables(n_u=1025)
    view = oracle.NuclearView(nt)
    E = float(nt.lattice.energies()[i])
    U = np.random.default_rng(i).uniform(0, 1, 100_000)
    u = np.array([view.table(0, "u", E, x) for x in U])
    assert u.min() >= 0.02 and u.max() <= 1.0
    ks = stats.kstest(u, lambda v: _trunc_exp_cdf(v, E))
    assert ks.statistic < 1.63 / math.sqrt(len(U)) + 2e-4, ks


def test_inelastic_draw_composes_loss_and_kalbach():
    """The whole inelastic draw at a lattice energy: u from the loss table at
    U1, then the CM cosine from the Kalbach-Mann law with r(E, u) and
    a(E, u): the Kalbach distribution function of the drawn cosine, with r
    and a from the placeholder's definition at the drawn u, is U3 (swapping r
    and a, or looking them up at U1 instead of u, fails)."""
    nt = _oxygen_tables(n_u=1025)
    view = oracle.NuclearView(nt)
    E = float(nt.lattice.energies()[900])
    rng = np.random.default_rng(7)
    for U1, U3 in rng.uniform(0, 1, (300, 2)):
        u, mu = view.draw(0, E, U1, U3)
        assert abs(u - view.table(0, "u", E, U1)) < 1e-15
        r = 0.1 + 0.5 * (1 - u)
        a = 0.5 + 2.0 * (1 - u) + E / 200.0
        F = (math.sinh(a * mu) + math.sinh(a) + r * (math.cosh(a * mu) - math.cosh(a))) / (
            2 * math.sinh(a))
        assert abs(F - U3) < 1e-9, (U1, U3, u, mu, F)


# --------------------------------------------------------------------------
# CM -> lab with an energy loss (Appendix A.1)
# --------------------------------------------------------------------------

def _boost_theta_lab(K, A, th_cm, u_loss):
    """Lab polar angle of the outgoing proton by an explicit Lorentz boost of
    its CM four-momentum: incident kinetic energy K on a target of A amu at
    rest, outgoing lab energy E_1L - u_loss K; its CM speed from the
    collinear velocity transform of that lab speed, its CM momentum at
    th_cm, boosted along z by the CM velocity p_1L/(E_1L + m2)."""
    m1, m2 = MP, A * AMU
    E1 = K + m1
    p1 = math.sqrt(E1 * E1 - m1 * m1)
    beta = p1 / (E1 + m2)
    gam = 1.0 / math.sqrt(1.0 - beta * beta)
    E1p = E1 - u_loss * K
    v_lab = math.sqrt(E1p * E1p - m1 * m1) / E1p
    v_cm = (v_lab - beta) / (1.0 - beta * v_lab)
    g_cm = 1.0 / math.sqrt(1.0 - v_cm * v_cm)
    p4 = np.array([m1 * g_cm, m1 * g_cm * v_cm * math.sin(th_cm), 0.0,
                   m1 * g_cm * v_cm * math.cos(th_cm)])
    L = np.array([[gam, 0, 0, gam * beta], [0, 1, 0, 0], [0, 0, 1, 0],
                  [gam * beta, 0, 0, gam]])
    q = L @ p4
    return math.atan2(q[1], q[3])


@pytest.mark.parametrize("K,A", [(150.0, 15.999), (60.0, 12.011), (220.0, 40.078)])
def test_cm_to_lab_with_loss_is_a_lorentz_boost(K, A):
    """Eq. (cm_to_lab) with E* = u E_n > 0 equals the explicit boost of the
    CM momentum four-vector (outgoing CM speed positive: losses up to 0.6),
    and the loss matters (it moves theta_L by more than 1e-3 rad at
    u = 0.3)."""
    cm2lab = oracle.lib().or_cm_to_lab
    for u_loss in (0.05, 0.3, 0.6):
        for th in (0.01, 0.4, 1.3, 2.2, 3.0):
            got = cm2lab(K, A, math.cos(th), math.sin(th), u_loss)
            want = _boost_theta_lab(K, A, th, u_loss)
            assert abs(got - want) < 1e-12, (u_loss, th, got, want)
    th = 1.3
    assert abs(cm2lab(K, A, math.cos(th), math.sin(th), 0.3) -
               cm2lab(K, A, math.cos(th), math.sin(th), 0.0)) > 1e-3


def test_inelastic_rate_adds_to_elastic(water, params):
    """With the inelastic switch the total jump rate gains
    N_A rho w_O / A_O sigma_O(E) 1e-24 per cm, sigma_O linear in the lattice
    coordinate between the placeholder's nodes (computed here from the
    placeholder's closed form at the two nodes); hydrogen adds nothing."""
    nt = placeholder_nuclear_tables(water.Z, water.A, EnergyLattice())
    lat = nt.lattice
    el = oracle.ELASTIC
    for E in (12.0, 55.5, 150.0, 231.7):
        r_el = oracle.channel_total_rate(water, params, 1.0, E, nt, flags=el)
        r_all = oracle.channel_total_rate(water, params, 1.0, E, nt, flags=el | oracle.INELASTIC)
        tau = _lattice_coord(lat, E)
        i = min(int(math.floor(tau)), lat.n - 2)
        f = tau - i
        Ei, Ej = lat.energies()[i], lat.energies()[i + 1]
        geo = math.pi * 1.2 ** 2 * 15.999 ** (2 / 3) * 1e-2
        s = lambda e: geo * (1 - 10.0 / e) if e > 10.0 else 0.0
        sig = (1 - f) * s(Ei) + f * s(Ej)
        k = list(water.Z).index(8)
        want = 6.02214076e23 * water.w[k] / water.A[k] * sig * 1e-24
        assert abs((r_all - r_el) - want) < 1e-10 * want, (E, r_all - r_el, want)
