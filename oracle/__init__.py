"""FP64 CPU oracle for the jump-SDE proton dose path (test infrastructure).

This package is the parity reference and nothing else: only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import it.  The product path never calls it.  It shares no code with the
HIP library; both consume the seeded inputs of ``workloads``.

* ``sde_oracle.c``: the transport (Eq. (VSDE) with the jump law Eq. (Npi)),
  the physics functionals of section 2.1, dose-to-medium, and the gamma
  index of section 2.2, all in FP64.
* this module: the ctypes binding and the analysis of section 2.2 in numpy
  (integrated depth dose, R80/R90, D99-normalised differences).
* ``nn_oracle``: the dose denoiser (layers, network, loss, Adam) in float64
  numpy, the reference for the learned part's kernels.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sde_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

MAX_ELEM = 16
MAX_MAT = 16

# physics switches
LOSS, STRAGGLE, MCS, ELASTIC, INELASTIC, EOR = 1, 2, 4, 8, 16, 32
SBM = 64   # small-angle diffusion by the spherical Brownian motion law (else geodesic step)
ALL = 127  # the method
ECUT = 256  # variant: large-angle elastic cut 2.5 sigma(E) instead of the fixed 0.02 rad
PHYSICS = ALL | ECUT   # every bit the oracle reads

# ledger slots and record fields (mirror the enums of sde_oracle.c)
L_DEP, L_ESC, L_NUC, L_E0, L_TRUNC, L_STEPS, L_HIST, L_JUMPS = range(8)
(R_E0, R_DEP, R_ESC, R_NUC, R_TRUNC, R_STEPS, R_NEL, R_NNE, R_END,
 R_X, R_Y, R_Z, R_OX, R_OY, R_OZ, R_EEND, R_J1, R_J2) = range(18)
R_N = 18
END_EOR, END_EXIT, END_EMIN, END_MAXSTEPS, END_SOURCE = 1, 2, 3, 4, 5


def build(force: bool = False) -> str:
    """Compile sde_oracle.c with gcc into liboracle.so next to it.  With
    ORACLE_SANITIZE_LIB set, compile an AddressSanitizer + UndefinedBehavior-
    Sanitizer build to that path instead (the process must preload libasan)."""
    san = os.environ.get("ORACLE_SANITIZE_LIB")
    if san:
        if force or not os.path.exists(san) or os.path.getmtime(san) < os.path.getmtime(_SRC):
            subprocess.check_call(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
                                   "-fsanitize=address,undefined",
                                   "-fno-sanitize-recover=undefined", "-shared", "-fPIC",
                                   "-std=gnu11", "-o", san, _SRC, "-lm"])
        return san
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=gnu11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Material(C.Structure):
    _fields_ = [("n_elem", C.c_int), ("Z", C.c_int * MAX_ELEM), ("A", C.c_double * MAX_ELEM),
                ("w", C.c_double * MAX_ELEM), ("I_eV", C.c_double)]


class Params(C.Structure):
    _fields_ = [("step_cm", C.c_double), ("ld_z_cm", C.c_double), ("e_min", C.c_double),
                ("e_max", C.c_double), ("ld_F", C.c_double), ("theta_cut", C.c_double),
                ("theta_bs", C.c_double), ("max_steps", C.c_longlong), ("flags", C.c_uint),
                ("pad", C.c_int)]


class Nuclear(C.Structure):
    _fields_ = [("n_tab", C.c_int), ("n_e", C.c_int), ("n_u", C.c_int), ("pad", C.c_int),
                ("e_lo", C.c_double), ("e_hi", C.c_double), ("Z", C.POINTER(C.c_int)),
                ("sigma", C.POINTER(C.c_double)), ("u_icdf", C.POINTER(C.c_double)),
                ("kr", C.POINTER(C.c_double)), ("ka", C.POINTER(C.c_double)),
                ("n_ni", C.c_int), ("n_mu", C.c_int), ("ni_Z", C.POINTER(C.c_int)),
                ("ni_sigma", C.POINTER(C.c_double)), ("ni_p", C.POINTER(C.c_double)),
                ("n_l", C.c_int), ("pad2", C.c_int), ("h_are", C.POINTER(C.c_double)),
                ("h_aim", C.POINTER(C.c_double)), ("h_b", C.POINTER(C.c_double))]


class PhantomS(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("pad", C.c_int),
                ("d", C.c_double * 3), ("origin", C.c_double * 3),
                ("mat", C.POINTER(C.c_ubyte)), ("rho", C.POINTER(C.c_float))]


class SpotS(C.Structure):
    _fields_ = [("E", C.c_double), ("sigmaE", C.c_double), ("x", C.c_double), ("y", C.c_double),
                ("sigma_xy", C.c_double), ("weight", C.c_double), ("n", C.c_ulonglong)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build()
        L = C.CDLL(path)
        d, P = C.c_double, C.POINTER
        for name in ("or_stopping_mass", "or_straggle_mass"):
            getattr(L, name).argtypes = [P(Material), d]
            getattr(L, name).restype = d
        L.or_csda_range_g.argtypes = [P(Material), d, d]
        L.or_csda_range_g.restype = d
        L.or_ld_sigma.argtypes = [P(Material), d, d, d, d]
        L.or_ld_sigma.restype = d
        L.or_rutherford_integral_barn.argtypes = [d, d, d, d]
        L.or_rutherford_integral_barn.restype = d
        L.or_mott_integral_barn.argtypes = [d, d, d, d]
        L.or_mott_integral_barn.restype = d
        L.or_mott_G.argtypes = [d, d]
        L.or_mott_G.restype = d
        L.or_mott_eta.argtypes = [d]
        L.or_mott_eta.restype = d
        L.or_eta2_over_k2_fm2.argtypes = [d, d, d]
        L.or_eta2_over_k2_fm2.restype = d
        L.or_rutherford_one_minus_mu.argtypes = [d, d]
        L.or_rutherford_one_minus_mu.restype = d
        L.or_mott_sample_mu.argtypes = [d, d, d, d]
        L.or_mott_sample_mu.restype = d
        L.or_kalbach_mu.argtypes = [d, d, d]
        L.or_kalbach_mu.restype = d
        L.or_cm_to_lab.argtypes = [d, d, d, d, d]
        L.or_cm_to_lab.restype = d
        L.or_turn.argtypes = [P(d), d, d, d]
        L.or_turn.restype = None
        for f in ("or_sbm_lineage_mean", "or_sbm_lineage_var"):
            getattr(L, f).argtypes = [d]
            getattr(L, f).restype = d
        L.or_sbm_upper_tail.argtypes = [d, d]
        L.or_sbm_upper_tail.restype = d
        L.or_sbm_t_switch.argtypes = []
        L.or_sbm_t_switch.restype = d
        L.or_sbm_polar_n.argtypes = [C.c_size_t, d, P(d), P(d), P(d), P(d)]
        L.or_sbm_polar_n.restype = None
        L.or_bspline3.argtypes = [P(d), C.c_int, d, d, d]
        L.or_bspline3.restype = d
        for f in ("or_p_ni_integral",):
            getattr(L, f).argtypes = [P(Nuclear), C.c_int, C.c_int, d]
            getattr(L, f).restype = d
        for f in ("or_ni_density", "or_ni_integral"):
            getattr(L, f).argtypes = [P(Nuclear), C.c_int, d, d]
            getattr(L, f).restype = d
        for f in ("or_h_nuclear_density", "or_h_nuclear_antiderivative"):
            getattr(L, f).argtypes = [P(Nuclear), d, d]
            getattr(L, f).restype = d
        L.or_elastic_sample_mu.argtypes = [P(Nuclear), C.c_int, d, d, d, d, d]
        L.or_elastic_sample_mu.restype = d
        L.or_elastic_cum_barn.argtypes = [P(Nuclear), C.c_int, d, d, d, d]
        L.or_elastic_cum_barn.restype = d
        L.or_elastic_cut.argtypes = [P(Material), P(Params), d, d]
        L.or_elastic_cut.restype = d
        L.or_channel_total_rate.argtypes = [P(Material), P(Nuclear), P(Params), d, d]
        L.or_channel_total_rate.restype = d
        L.or_rng_block.argtypes = [C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32,
                                   P(C.c_uint32)]
        L.or_rng_block.restype = None
        L.or_rng_blocks.argtypes = [C.c_uint64, C.c_size_t, P(C.c_uint64), P(C.c_uint32),
                                    P(C.c_uint32), P(C.c_uint32)]
        L.or_rng_blocks.restype = None
        L.or_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.or_philox4x32_10.restype = None
        L.or_philox4x64_10.argtypes = [P(C.c_uint64), P(C.c_uint64), P(C.c_uint64)]
        L.or_philox4x64_10.restype = None
        L.or_source_n.argtypes = [P(SpotS), d, C.c_uint64, C.c_uint64, C.c_size_t, P(d)]
        L.or_source_n.restype = None
        L.or_lattice_pos.argtypes = [P(Nuclear), d, P(C.c_int), P(d)]
        L.or_lattice_pos.restype = None
        L.or_inelastic_sigma_barn.argtypes = [P(Nuclear), C.c_int, d]
        L.or_inelastic_sigma_barn.restype = d
        L.or_table_eu.argtypes = [P(Nuclear), C.c_int, C.c_int, d, d]
        L.or_table_eu.restype = d
        L.or_inelastic_draw.argtypes = [P(Nuclear), C.c_int, d, d, d, P(d), P(d)]
        L.or_inelastic_draw.restype = None
        L.or_transport.argtypes = [P(Material), C.c_int, P(Params), P(Nuclear), P(PhantomS),
                                   P(SpotS), C.c_int, C.c_uint64, C.c_uint64, C.c_uint64,
                                   C.c_int, P(d), P(d), P(d)]
        L.or_transport.restype = C.c_int
        L.or_dose.argtypes = [P(d), P(C.c_float), C.c_size_t, d, P(d)]
        L.or_dose.restype = None
        L.or_gamma.argtypes = [P(d), P(d), C.c_int, C.c_int, C.c_int, P(d), d, d, d, C.c_int,
                               C.c_int, C.c_int, P(C.c_longlong), P(C.c_longlong)]
        L.or_gamma.restype = d
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


def n_threads_default() -> int:
    """Host threads for the oracle: the affinity set, at most 16 (the CPU share
    of one GPU on the target machines), or SDE_ORACLE_THREADS."""
    env = os.environ.get("SDE_ORACLE_THREADS")
    if env:
        return max(1, int(env))
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def material_struct(m) -> Material:
    s = Material()
    s.n_elem = len(m.Z)
    for i, (z, a, w) in enumerate(zip(m.Z, m.A, m.w)):
        s.Z[i], s.A[i], s.w[i] = int(z), float(a), float(w)
    s.I_eV = float(m.I_eV)
    return s


def params_struct(p, flags: Optional[int] = None) -> Params:
    """From a workloads PhysicsParams (its flag bits are the same as here)."""
    s = Params()
    s.step_cm, s.ld_z_cm = p.step_cm, p.ld_z_cm
    s.e_min, s.e_max = p.e_min_MeV, p.e_max_MeV
    s.ld_F, s.theta_cut, s.theta_bs = p.ld_F, p.theta_cut_rad, p.backscatter_cut_rad
    s.max_steps = int(p.max_steps)
    # the oracle always steps in double precision: only the physics switches count
    s.flags = int(p.flags if flags is None else flags) & PHYSICS
    return s


@dataclass
class _Keep:
    arrays: list


def nuclear_struct(nt) -> tuple:
    """Returns (struct, keep-alive list) for workloads NuclearTables or None."""
    if nt is None:
        return None, []
    Z = np.ascontiguousarray(nt.Z, dtype=np.int32)
    sg = np.ascontiguousarray(nt.sigma, dtype=np.float64)
    ui = np.ascontiguousarray(nt.u_icdf, dtype=np.float64)
    kr = np.ascontiguousarray(nt.kalbach_r, dtype=np.float64)
    ka = np.ascontiguousarray(nt.kalbach_a, dtype=np.float64)
    s = Nuclear()
    s.n_tab, s.n_e, s.n_u = len(Z), nt.lattice.n, nt.n_u
    s.e_lo, s.e_hi = nt.lattice.e_lo, nt.lattice.e_hi
    s.Z, s.sigma, s.u_icdf = _ptr(Z, C.c_int), _ptr(sg, C.c_double), _ptr(ui, C.c_double)
    s.kr, s.ka = _ptr(kr, C.c_double), _ptr(ka, C.c_double)
    keep = [Z, sg, ui, kr, ka]
    el = getattr(nt, "elastic", None)
    if el is not None:
        nZ = np.ascontiguousarray(el.ni_Z, dtype=np.int32)
        ns = np.ascontiguousarray(el.ni_sigma, dtype=np.float64)
        npp = np.ascontiguousarray(el.ni_p, dtype=np.float64)
        ha = np.ascontiguousarray(el.h_are, dtype=np.float64)
        hi = np.ascontiguousarray(el.h_aim, dtype=np.float64)
        hb = np.ascontiguousarray(el.h_b, dtype=np.float64)
        s.n_ni, s.n_mu = len(nZ), int(npp.shape[-1]) if npp.size else 0
        s.ni_Z, s.ni_sigma, s.ni_p = _ptr(nZ, C.c_int), _ptr(ns, C.c_double), _ptr(npp, C.c_double)
        s.n_l = int(ha.shape[0])
        s.h_are, s.h_aim, s.h_b = _ptr(ha, C.c_double), _ptr(hi, C.c_double), _ptr(hb, C.c_double)
        keep += [nZ, ns, npp, ha, hi, hb]
    return s, keep


def phantom_struct(ph) -> tuple:
    mat = np.ascontiguousarray(ph.material_id, dtype=np.uint8)
    rho = np.ascontiguousarray(ph.density, dtype=np.float32)
    s = PhantomS()
    s.nx, s.ny, s.nz = ph.shape
    for k in range(3):
        s.d[k] = ph.voxel_cm[k]
        s.origin[k] = ph.origin_cm[k]
    s.mat, s.rho = _ptr(mat, C.c_ubyte), _ptr(rho, C.c_float)
    return s, [mat, rho]


def spots_struct(spots) -> C.Array:
    arr = (SpotS * len(spots))()
    for i, sp in enumerate(spots):
        arr[i].E, arr[i].sigmaE = sp.E_MeV, sp.sigmaE_rel
        arr[i].x, arr[i].y, arr[i].sigma_xy = sp.x_cm, sp.y_cm, sp.sigma_xy_cm
        arr[i].weight, arr[i].n = sp.weight, int(sp.n_histories)
    return arr


@dataclass
class TransportResult:
    edep: Optional[np.ndarray]      # (nz, ny, nx) weighted MeV
    ledger: np.ndarray              # [8]
    records: Optional[np.ndarray]   # (n, 18)


def transport(phantom, spots, params, nuclear=None, seed: int = 0, h_begin: int = 0,
              h_end: Optional[int] = None, n_threads: Optional[int] = None,
              flags: Optional[int] = None, tally: bool = True,
              records: bool = False) -> TransportResult:
    """Run histories [h_begin, h_end) (default: all) through the FP64 oracle."""
    L = lib()
    mats = (Material * len(phantom.materials))()
    for i, m in enumerate(phantom.materials):
        mats[i] = material_struct(m)
    ps = params_struct(params, flags)
    ns, keep_n = nuclear_struct(nuclear)
    phs, keep_p = phantom_struct(phantom)
    sps = spots_struct(spots)
    total = int(sum(s.n_histories for s in spots))
    h_end = total if h_end is None else int(h_end)
    nz_ny_nx = phantom.material_id.shape
    edep = np.zeros(nz_ny_nx, dtype=np.float64) if tally else None
    ledger = np.zeros(8, dtype=np.float64)
    rec = np.zeros((h_end - h_begin, R_N), dtype=np.float64) if records else None
    nt = n_threads_default() if n_threads is None else int(n_threads)
    rc = L.or_transport(mats, len(phantom.materials), C.byref(ps),
                        C.byref(ns) if ns is not None else None, C.byref(phs), sps, len(spots),
                        C.c_uint64(seed), C.c_uint64(h_begin), C.c_uint64(h_end), nt,
                        _ptr(edep, C.c_double) if edep is not None else None,
                        _ptr(ledger, C.c_double),
                        _ptr(rec, C.c_double) if rec is not None else None)
    del keep_n, keep_p
    if rc != 0:
        raise ValueError("oracle transport rejected its input")
    return TransportResult(edep, ledger, rec)


def dose(edep: np.ndarray, phantom) -> np.ndarray:
    """Dose to medium in Gy from weighted MeV per voxel."""
    rho = np.ascontiguousarray(phantom.density, dtype=np.float32)
    e = np.ascontiguousarray(edep, dtype=np.float64)
    out = np.zeros_like(e)
    lib().or_dose(_ptr(e, C.c_double), _ptr(rho, C.c_float), e.size,
                  phantom.voxel_volume_cm3(), _ptr(out, C.c_double))
    return out


def gamma_pass_rate(ref: np.ndarray, ev: np.ndarray, voxel_cm: Sequence[float],
                    dd: float = 0.02, dta_cm: float = 0.05, thresh: float = 0.01,
                    interp: int = 10, local: bool = True,
                    n_threads: Optional[int] = None) -> tuple:
    """Gamma pass fraction of ``ev`` against ``ref`` (arrays (nz, ny, nx))."""
    r = np.ascontiguousarray(ref, dtype=np.float64)
    e = np.ascontiguousarray(ev, dtype=np.float64)
    assert r.shape == e.shape
    nz, ny, nx = r.shape
    d = np.array(voxel_cm, dtype=np.float64)
    ne, npass = C.c_longlong(0), C.c_longlong(0)
    nt = n_threads_default() if n_threads is None else int(n_threads)
    frac = lib().or_gamma(_ptr(r, C.c_double), _ptr(e, C.c_double), nx, ny, nz,
                          _ptr(d, C.c_double), dd, dta_cm, thresh, int(interp), int(local), nt,
                          C.byref(ne), C.byref(npass))
    return frac, int(ne.value), int(npass.value)


# ---------------------------------------------------------------------------
# Physics functionals, exposed for the pins
# ---------------------------------------------------------------------------

def stopping_mass(m, E: float) -> float:
    s = material_struct(m)
    return lib().or_stopping_mass(C.byref(s), float(E))


def straggle_mass(m, E: float) -> float:
    s = material_struct(m)
    return lib().or_straggle_mass(C.byref(s), float(E))


def csda_range_g(m, E: float, e_min: float = 0.05) -> float:
    s = material_struct(m)
    return lib().or_csda_range_g(C.byref(s), float(e_min), float(E))


def ld_sigma(m, rho: float, E: float, z: float = 0.05, F: float = 0.98) -> float:
    s = material_struct(m)
    return lib().or_ld_sigma(C.byref(s), float(rho), float(E), float(z), float(F))


def sbm_lineage_mean(t: float) -> float:
    return lib().or_sbm_lineage_mean(float(t))


def sbm_lineage_var(t: float) -> float:
    return lib().or_sbm_lineage_var(float(t))


def sbm_upper_tail(t: float, c: float) -> float:
    """P(cos(angle) > c) of spherical Brownian motion on S^2 at time t."""
    return lib().or_sbm_upper_tail(float(t), float(c))


def sbm_t_switch() -> float:
    return lib().or_sbm_t_switch()


def sbm_polar(t: float, z: np.ndarray, u: np.ndarray):
    """(cos, sin) of the polar angle of the spherical Brownian motion step at
    time t for normal deviates z and uniforms u (arrays of one length)."""
    z = np.ascontiguousarray(z, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    assert z.shape == u.shape
    ct = np.empty_like(z)
    st = np.empty_like(z)
    d = C.c_double
    lib().or_sbm_polar_n(z.size, float(t), _ptr(z, d), _ptr(u, d), _ptr(ct, d), _ptr(st, d))
    return ct, st


def philox4x32(ctr: Sequence[int], key: Sequence[int]) -> List[int]:
    c = (C.c_uint32 * 4)(*ctr)
    k = (C.c_uint32 * 2)(*key)
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return list(o)


def philox4x64(ctr: Sequence[int], key: Sequence[int]) -> List[int]:
    c = (C.c_uint64 * 4)(*ctr)
    k = (C.c_uint64 * 2)(*key)
    o = (C.c_uint64 * 4)()
    lib().or_philox4x64_10(c, k, o)
    return list(o)


def rng_block(seed: int, h: int, n: int, b: int) -> List[int]:
    o = (C.c_uint32 * 4)()
    lib().or_rng_block(C.c_uint64(seed), C.c_uint64(h), C.c_uint32(n), C.c_uint32(b), o)
    return list(o)


def source(spot, z0_cm: float, seed: int, h0: int, n: int) -> np.ndarray:
    """Source (E, x, y, z) of histories [h0, h0 + n) of one spot, (n, 4)."""
    out = np.zeros((int(n), 4), dtype=np.float64)
    sp = spots_struct([spot])
    lib().or_source_n(sp, float(z0_cm), C.c_uint64(seed), C.c_uint64(h0), int(n),
                      _ptr(out, C.c_double))
    return out


class NuclearView:
    """The oracle's view of a workloads NuclearTables, for the inelastic pins."""

    def __init__(self, nt):
        self.s, self._keep = nuclear_struct(nt)

    def lattice_pos(self, E: float):
        i, f = C.c_int(0), C.c_double(0.0)
        lib().or_lattice_pos(C.byref(self.s), float(E), C.byref(i), C.byref(f))
        return i.value, f.value

    def sigma_barn(self, t: int, E: float) -> float:
        return lib().or_inelastic_sigma_barn(C.byref(self.s), int(t), float(E))

    def table(self, t: int, which: str, E: float, x: float) -> float:
        k = {"u": 0, "r": 1, "a": 2}[which]
        return lib().or_table_eu(C.byref(self.s), int(t), k, float(E), float(x))

    def p_ni_integral(self, t: int, i: int, x: float) -> float:
        return lib().or_p_ni_integral(C.byref(self.s), int(t), int(i), float(x))

    def ni_density(self, t: int, E: float, mu: float) -> float:
        return lib().or_ni_density(C.byref(self.s), int(t), float(E), float(mu))

    def ni_integral(self, t: int, E: float, x: float) -> float:
        return lib().or_ni_integral(C.byref(self.s), int(t), float(E), float(x))

    def h_nuclear_density(self, E: float, mu: float) -> float:
        return lib().or_h_nuclear_density(C.byref(self.s), float(E), float(mu))

    def h_nuclear_antiderivative(self, E: float, mu: float) -> float:
        return lib().or_h_nuclear_antiderivative(C.byref(self.s), float(E), float(mu))

    def elastic_sample_mu(self, Z: int, A: float, E: float, U: float, tc: float = 0.02,
                          tb: float = 0.04) -> float:
        return lib().or_elastic_sample_mu(C.byref(self.s), int(Z), float(A), float(E),
                                          float(U), float(tc), float(tb))

    def elastic_cum_barn(self, Z: int, A: float, E: float, lo: float, x: float) -> float:
        return lib().or_elastic_cum_barn(C.byref(self.s), int(Z), float(A), float(E),
                                         float(lo), float(x))

    def draw(self, t: int, E: float, U1: float, U3: float):
        u, c = C.c_double(0.0), C.c_double(0.0)
        lib().or_inelastic_draw(C.byref(self.s), int(t), float(E), float(U1), float(U3),
                                C.byref(u), C.byref(c))
        return u.value, c.value


def rng_blocks(seed: int, h: np.ndarray, n: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Philox4x32-10 blocks (count, 4) uint32 for counters (h, n, b)."""
    h = np.ascontiguousarray(h, dtype=np.uint64)
    n = np.ascontiguousarray(n, dtype=np.uint32)
    b = np.ascontiguousarray(b, dtype=np.uint32)
    out = np.zeros((h.size, 4), dtype=np.uint32)
    lib().or_rng_blocks(C.c_uint64(seed), h.size, _ptr(h, C.c_uint64), _ptr(n, C.c_uint32),
                        _ptr(b, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def elastic_cut(m, params, rho: float, E: float, flags=None) -> float:
    """The large-angle elastic cut (CM, rad) at E in medium m of density rho."""
    s = material_struct(m)
    ps = params_struct(params, flags)
    return lib().or_elastic_cut(C.byref(s), C.byref(ps), float(rho), float(E))


def bspline3(c: np.ndarray, m: int, x0: float, h: float, x: float) -> float:
    c = np.ascontiguousarray(c, dtype=np.float64)
    return lib().or_bspline3(_ptr(c, C.c_double), int(m), float(x0), float(h), float(x))


def channel_total_rate(m, params, rho: float, E: float, nuclear=None, flags=None) -> float:
    s = material_struct(m)
    ps = params_struct(params, flags)
    ns, keep = nuclear_struct(nuclear)
    r = lib().or_channel_total_rate(C.byref(s), C.byref(ns) if ns is not None else None,
                                    C.byref(ps), float(rho), float(E))
    del keep
    return r


# ---------------------------------------------------------------------------
# Analysis of section 2.2 ("Comparison metrics")
# ---------------------------------------------------------------------------

def idd(dose_zyx: np.ndarray) -> np.ndarray:
    """Integrated depth dose: sum over each depth slice."""
    return dose_zyx.sum(axis=(1, 2))


def range_rx(dose_zyx: np.ndarray, dz_cm: float, frac: float = 0.8, z0_cm: float = 0.0) -> float:
    """Depth (cm) where the IDD falls to ``frac`` of its maximum on the distal
    side, linear between voxel-centre depths."""
    c = idd(dose_zyx)
    i = int(np.argmax(c))
    lvl = frac * c[i]
    z = z0_cm + (np.arange(len(c)) + 0.5) * dz_cm
    for k in range(i + 1, len(c)):
        if c[k] < lvl:
            t = (c[k - 1] - lvl) / (c[k - 1] - c[k])
            return float(z[k - 1] + t * (z[k] - z[k - 1]))
    return float(z[-1])


def d99_difference(ref: np.ndarray, ev: np.ndarray, roi_frac: float = 0.01) -> np.ndarray:
    """Voxel difference (ev - ref) normalised to the 99th percentile of the
    reference inside the ROI (voxels >= roi_frac max(ref)); NaN outside."""
    roi = ref >= roi_frac * ref.max()
    d99 = np.percentile(ref[roi], 99.0)
    out = np.full(ref.shape, np.nan)
    out[roi] = (ev[roi] - ref[roi]) / d99
    return out
