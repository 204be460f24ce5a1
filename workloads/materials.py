"""Material descriptors: element list, mass fractions and mean excitation energy.

The paper parameterises a medium by its chemical composition and its mean
excitation energy I (section 2.1, "Parameterisation for inelastic Coulomb
scattering", Bragg additivity).  The compositions it used (a Geant4 bone
material and an ICRP-110 lung) are not given in the paper, so the stand-ins
below are built from stoichiometry only:

* water: exact H2O;
* bone: a 50/50 mass mixture of water and hydroxyapatite Ca10(PO4)6(OH)2,
  a synthetic stand-in (elements H, O, P, Ca), not a database record;
* lung: H2O composition at lung density;
* air: dry air near sea level by mass (N 0.755267, O 0.231781,
  Ar 0.012827, C 0.000124), 0.001205 g/cm3, I = 85.7 eV (the usual
  dosimetry values), for the cavities of the CT-like phantom.

Densities and I values are the ones the workloads fix (water 1.0 g/cm3 and
75 eV, bone 1.85 g/cm3 and 92 eV, lung 0.26 g/cm3 and 75 eV).  Atomic weights
are IUPAC standard atomic weights (abridged, g/mol).
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Dict, List, Tuple

# Z -> (symbol, standard atomic weight in g/mol)
ELEMENTS: Dict[int, Tuple[str, float]] = {
    1: ("H", 1.008),
    6: ("C", 12.011),
    7: ("N", 14.007),
    8: ("O", 15.999),
    15: ("P", 30.974),
    18: ("Ar", 39.948),
    20: ("Ca", 40.078),
}


@dataclass(frozen=True)
class Material:
    name: str
    Z: Tuple[int, ...]
    A: Tuple[float, ...]       # g/mol
    w: Tuple[float, ...]       # mass fractions, sum to 1
    I_eV: float                # mean excitation energy
    rho_nominal: float         # g/cm3 used by the phantoms

    def as_dict(self) -> dict:
        return dict(name=self.name, Z=list(self.Z), A=list(self.A), w=list(self.w),
                    I_eV=self.I_eV, rho_nominal=self.rho_nominal)


def _fractions(atoms: Dict[int, float]) -> Dict[int, float]:
    """Mass fractions of a formula given as {Z: atom count}."""
    mass = {z: n * ELEMENTS[z][1] for z, n in atoms.items()}
    tot = sum(mass.values())
    return {z: m / tot for z, m in mass.items()}


def _mix(parts: List[Tuple[float, Dict[int, float]]]) -> Dict[int, float]:
    """Mass-weighted mixture of fraction dictionaries."""
    out: Dict[int, float] = {}
    for frac, comp in parts:
        for z, w in comp.items():
            out[z] = out.get(z, 0.0) + frac * w
    return out


def material(name: str, fractions: Dict[int, float], I_eV: float, rho: float) -> Material:
    zs = tuple(sorted(fractions))
    tot = sum(fractions.values())
    return Material(name=name, Z=zs, A=tuple(ELEMENTS[z][1] for z in zs),
                    w=tuple(fractions[z] / tot for z in zs), I_eV=float(I_eV),
                    rho_nominal=float(rho))


_H2O = _fractions({1: 2, 8: 1})
_HAP = _fractions({20: 10, 15: 6, 8: 26, 1: 2})   # Ca10(PO4)6(OH)2


def water() -> Material:
    return material("water", _H2O, 75.0, 1.0)


def bone() -> Material:
    return material("bone", _mix([(0.5, _H2O), (0.5, _HAP)]), 92.0, 1.85)


def lung() -> Material:
    return material("lung", _H2O, 75.0, 0.26)


def air() -> Material:
    return material("air", {7: 0.755267, 8: 0.231781, 18: 0.012827, 6: 0.000124}, 85.7,
                    0.001205)
