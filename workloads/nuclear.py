"""Placeholder nuclear inelastic tables.

The paper takes the inelastic proton-nucleus data (rate sigma_ne(E), the
outgoing-energy distribution pi_ne(E; du), and the Kalbach-Mann parameters
r(E, u) and a(E, u)) from the ENDF/B-VIII.1 and JEFF-4.0 libraries
(section 2.1, "Parameterisation for inelastic proton-nucleus interactions").
Those libraries are not available here, so this module writes smooth,
documented placeholder tables of the same shape.  Every physics statement
that depends on them is a statement about the placeholder, not about nature.

Table layout (shared definition of the input, consumed by both the oracle
and the HIP path):

* energy lattice: ``n_e`` points uniform in ln E over [e_lo, e_hi];
* ``sigma[t, i]``: total inelastic cross section of element t at E_i, barn;
  values between lattice points are linear in the lattice coordinate;
* ``u_icdf[t, i, j]``: inverse CDF of the energy-loss fraction u at
  U_j = j/(n_u-1); a sample is the bilinear interpolation at (E, U);
* ``kalbach_r[t, i, j]``, ``kalbach_a[t, i, j]``: r and a at (E_i, u_j) with
  u_j = j/(n_u-1); bilinear interpolation at (E, u).

Hydrogen has no inelastic channel below the pion threshold, so it gets no
table.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Sequence

import numpy as np

# nuclear radius parameter of the geometric placeholder cross section, fm
_R0_FM = 1.2
# placeholder reaction threshold, MeV
_E_THRESH = 10.0


@dataclass(frozen=True)
class EnergyLattice:
    n: int = 1024
    e_lo: float = 0.05
    e_hi: float = 260.0

    def energies(self) -> np.ndarray:
        return np.exp(np.linspace(np.log(self.e_lo), np.log(self.e_hi), self.n))


@dataclass
class ElasticNuclear:
    """Elastic nuclear data of section 2.1.4 in the layout both sides read.

    * ``ni_Z``, ``ni_sigma[t, i]`` (barn) and ``ni_p[t, i, j]``: for elements
      other than hydrogen, sigma_NI(E_i) and the cubic B-spline coefficients
      of P_NI(mu, E_i) on uniform knots over mu in [-1, 1] (knot j at
      -1 + (j - 3) h, h = 2 / (n_mu - 3));
    * ``h_are[l, k]``, ``h_aim[l, k]``, ``h_b[l, k]`` (barn): for hydrogen,
      l = 0..n_l-1, the cubic B-spline coefficients in the lattice
      coordinate of Re a_l(E), Im a_l(E) and b_l(E) (n_e + 2 per l).
    """
    ni_Z: np.ndarray
    ni_sigma: np.ndarray
    ni_p: np.ndarray
    h_are: np.ndarray
    h_aim: np.ndarray
    h_b: np.ndarray


@dataclass
class NuclearTables:
    lattice: EnergyLattice
    n_u: int
    Z: np.ndarray          # int32 [n_tab]
    A: np.ndarray          # float64 [n_tab], g/mol (for reference only)
    sigma: np.ndarray      # float64 [n_tab, n_e] barn
    u_icdf: np.ndarray     # float64 [n_tab, n_e, n_u]
    kalbach_r: np.ndarray  # float64 [n_tab, n_e, n_u]
    kalbach_a: np.ndarray  # float64 [n_tab, n_e, n_u]
    elastic: "ElasticNuclear | None" = None


def placeholder_nuclear_tables(elements: Sequence[int], atomic_weights: Sequence[float],
                               lattice: EnergyLattice = EnergyLattice(),
                               n_u: int = 33) -> NuclearTables:
    """Write placeholder inelastic tables for every element with Z > 1.

    sigma(E) = pi r0^2 A^(2/3) (1 - E_th/E) above E_th = 10 MeV (geometric
    size with a threshold factor).  The energy-loss fraction u follows a
    truncated exponential on [0.02, 1] with an E-dependent scale
    lam(E) = 0.15 + 0.15 E/250 MeV.  Kalbach r = 0.1 + 0.5 (1 - u),
    a = 0.5 + 2 (1 - u) + E/200 MeV (more forward for small losses).
    """
    E = lattice.energies()
    zs, As = [], []
    for z, a in zip(elements, atomic_weights):
        if int(z) > 1 and int(z) not in zs:
            zs.append(int(z))
            As.append(float(a))
    n_t = len(zs)
    sigma = np.zeros((n_t, lattice.n))
    u_icdf = np.zeros((n_t, lattice.n, n_u))
    kr = np.zeros((n_t, lattice.n, n_u))
    ka = np.zeros((n_t, lattice.n, n_u))
    U = np.linspace(0.0, 1.0, n_u)
    u_min = 0.02
    for t, a in enumerate(As):
        geo_b = np.pi * _R0_FM ** 2 * a ** (2.0 / 3.0) * 1e-2   # fm^2 -> barn
        sigma[t] = np.where(E > _E_THRESH, geo_b * (1.0 - _E_THRESH / E), 0.0)
        lam = 0.15 + 0.15 * E / 250.0
        span = 1.0 - np.exp(-(1.0 - u_min) / lam)
        u_icdf[t] = u_min - lam[:, None] * np.log1p(-U[None, :] * span[:, None])
        u_icdf[t, :, -1] = 1.0
        kr[t] = 0.1 + 0.5 * (1.0 - U)[None, :] + 0.0 * E[:, None]
        ka[t] = 0.5 + 2.0 * (1.0 - U)[None, :] + E[:, None] / 200.0
    return NuclearTables(lattice=lattice, n_u=n_u, Z=np.array(zs, dtype=np.int32),
                         A=np.array(As), sigma=sigma, u_icdf=u_icdf,
                         kalbach_r=kr, kalbach_a=ka)


def nuclear_for_phantom(phantom, lattice: EnergyLattice) -> NuclearTables:
    """Placeholder tables for every element of a phantom's materials."""
    zs = [z for m in phantom.materials for z in m.Z]
    As = [a for m in phantom.materials for a in m.A]
    return placeholder_nuclear_tables(zs, As, lattice)


def synthetic_elastic_nuclear(elements: Sequence[int], atomic_weights: Sequence[float],
                              lattice: EnergyLattice = EnergyLattice(), n_mu: int = 24,
                              n_l: int = 8, seed: int = 0) -> ElasticNuclear:
    """Synthetic elastic nuclear data of the ENDF shapes (no library values):
    every element heavier than hydrogen gets sigma_NI(E) = 0.3 A^(2/3)
    (1 - exp(-E / 20 MeV)) barn and a P_NI(mu, E) that rises towards forward
    angles, exp(k (mu - 1)) with k = 1 + E / 40 MeV, normalised to integrate
    to 1 over [-1, 1] (its B-spline coefficients are those values at the
    knots' Greville points, a smooth shape, not an interpolation);
    hydrogen gets seeded smooth amplitudes: b_0(E) around 0.012 barn with
    higher b_l falling as 0.1^l, and complex a_l of modulus <= 5e-4 barn,
    small enough that the summed hydrogen cross section stays positive (the
    tests check it)."""
    rng = np.random.default_rng(seed)
    m = n_mu - 3
    h = 2.0 / m
    greville = -1.0 + (np.arange(n_mu) - 1.0) * h      # centres of the basis functions
    E = lattice.energies()
    zs, As = [], []
    for z, a in zip(elements, atomic_weights):
        if int(z) > 1 and int(z) not in zs:
            zs.append(int(z))
            As.append(float(a))
    ni_sigma = np.zeros((len(zs), lattice.n))
    ni_p = np.zeros((len(zs), lattice.n, n_mu))
    for t, a in enumerate(As):
        ni_sigma[t] = 0.3 * a ** (2.0 / 3.0) * (1.0 - np.exp(-E / 20.0))
        k = 1.0 + E / 40.0
        c = np.exp(k[:, None] * (np.clip(greville, -1.0, 1.0)[None, :] - 1.0))
        # normalise each energy's spline to unit integral: the integral of a
        # uniform cubic spline is h times the sum of its coefficients, less
        # the parts of the three boundary basis functions outside [-1, 1]
        w = np.ones(n_mu)
        w[0] = w[-1] = 1.0 / 24.0
        w[1] = w[-2] = 0.5
        w[2] = w[-3] = 23.0 / 24.0
        ni_p[t] = c / (h * (c * w[None, :]).sum(axis=1))[:, None]
    n_c = lattice.n + 2
    tt = np.arange(n_c) - 1.0                          # lattice coordinate of coefficient k
    x = tt / max(lattice.n - 1, 1)
    h_b = np.zeros((n_l, n_c))
    h_are = np.zeros((n_l, n_c))
    h_aim = np.zeros((n_l, n_c))
    for l in range(n_l):
        ph = rng.uniform(0, 2 * np.pi, 3)
        h_b[l] = 0.012 * 0.1 ** l * (1.0 + 0.2 * np.sin(np.pi * x * (l + 2) + ph[0]))
        amp = 5e-4 / (l + 1)
        h_are[l] = amp * np.cos(np.pi * x * 1.5 + ph[1])
        h_aim[l] = amp * np.sin(np.pi * x * 2.5 + ph[2])
    return ElasticNuclear(ni_Z=np.array(zs, dtype=np.int32), ni_sigma=ni_sigma, ni_p=ni_p,
                          h_are=h_are, h_aim=h_aim, h_b=h_b)


def with_elastic_nuclear(nt: NuclearTables, el: ElasticNuclear) -> NuclearTables:
    """The same inelastic tables with elastic nuclear data attached."""
    return NuclearTables(lattice=nt.lattice, n_u=nt.n_u, Z=nt.Z, A=nt.A, sigma=nt.sigma,
                         u_icdf=nt.u_icdf, kalbach_r=nt.kalbach_r, kalbach_a=nt.kalbach_a,
                         elastic=el)
