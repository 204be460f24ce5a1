"""ctypes binding of libsde (include/sde.h): argument marshalling only.

Every step of the transport, the tally, the dose conversion and the gamma
index runs in the HIP library.  torch provides device memory and streams.
If libsde.so is missing the import of this module fails: there is no CPU
fallback.
"""

from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsde.so")

OK, E_INVALID, E_HIP, E_RANGE, E_OVERFLOW, E_STATE, E_NOMEM = 0, -1, -2, -3, -4, -5, -6
LOSS, STRAGGLE, MCS, ELASTIC, INELASTIC, END_OF_RANGE = 1, 2, 4, 8, 16, 32
SBM = 64   # small-angle diffusion by the spherical Brownian motion law (else geodesic step)
ALL = 127  # the method
FP64 = 128  # step in double precision (not a physics switch)
ECUT = 256  # variant: large-angle elastic cut 2.5 sigma(E) instead of the fixed cut
(LEDGER_DEPOSITED, LEDGER_ESCAPED, LEDGER_NUCLEAR, LEDGER_INITIAL, LEDGER_TRUNCATED,
 LEDGER_STEPS, LEDGER_HISTORIES, LEDGER_JUMPS, LEDGER_BAD_LANES) = range(9)
LEDGER_N = 9
EXPORTS = ("sde_init_materials", "sde_set_stream", "sde_transport", "sde_transport_ex",
           "sde_plan_create", "sde_plan_execute", "sde_plan_results", "sde_plan_destroy",
           "sde_plan_kernel_ms", "sde_plan_set_records", "sde_gamma", "sde_launch_limits",
           "sde_sbm_polar", "sde_philox_words", "sde_gamma_noalloc", "sde_free",
           "sde_last_error")


class SdeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libsde error {code}: {msg}")
        self.code = code


class MaterialDesc(C.Structure):
    _fields_ = [("n_elem", C.c_int), ("Z", C.POINTER(C.c_int)), ("A", C.POINTER(C.c_double)),
                ("w", C.POINTER(C.c_double)), ("I_eV", C.c_double)]


class PhysicsParams(C.Structure):
    _fields_ = [("step_cm", C.c_double), ("ld_z_cm", C.c_double), ("e_min_MeV", C.c_double),
                ("e_max_MeV", C.c_double), ("ld_F", C.c_double), ("theta_cut_rad", C.c_double),
                ("backscatter_cut_rad", C.c_double), ("n_energy", C.c_int), ("flags", C.c_uint),
                ("max_steps", C.c_int64)]


class NuclearTables(C.Structure):
    _fields_ = [("n_tab", C.c_int), ("n_u", C.c_int), ("Z", C.POINTER(C.c_int)),
                ("sigma_barn", C.POINTER(C.c_double)), ("u_icdf", C.POINTER(C.c_double)),
                ("kalbach_r", C.POINTER(C.c_double)), ("kalbach_a", C.POINTER(C.c_double)),
                ("n_ni", C.c_int), ("n_mu", C.c_int), ("ni_Z", C.POINTER(C.c_int)),
                ("ni_sigma_barn", C.POINTER(C.c_double)), ("ni_p", C.POINTER(C.c_double)),
                ("n_l", C.c_int), ("h_a_re", C.POINTER(C.c_double)),
                ("h_a_im", C.POINTER(C.c_double)), ("h_b", C.POINTER(C.c_double))]


class SpotS(C.Structure):
    _fields_ = [("E_MeV", C.c_double), ("sigmaE_rel", C.c_double), ("x_cm", C.c_double),
                ("y_cm", C.c_double), ("sigma_xy_cm", C.c_double), ("weight", C.c_double),
                ("n_histories", C.c_uint64)]


class Beam(C.Structure):
    _fields_ = [("n_spots", C.c_int), ("spots", C.POINTER(SpotS))]


class PhantomS(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int), ("dx_cm", C.c_double),
                ("dy_cm", C.c_double), ("dz_cm", C.c_double), ("origin_cm", C.c_double * 3),
                ("material_id", C.c_void_p), ("density", C.c_void_p)]


class Launch(C.Structure):
    _fields_ = [("block", C.c_int), ("grid", C.c_int), ("refill", C.c_int),
                ("jump_batch", C.c_int), ("tally_replicas", C.c_int), ("claim_chunk", C.c_int),
                ("tile_nx", C.c_int), ("tile_ny", C.c_int), ("tile_nz", C.c_int),
                ("tile_x0", C.c_int), ("tile_y0", C.c_int), ("tile_z0", C.c_int),
                ("nan_history", C.c_uint64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    # torch ships its own HIP runtime under the same soname; loading torch
    # first makes libsde bind to that one, so the process has a single HIP
    # runtime (loading libsde first would bring a second one, and torch's
    # would then find no device)
    import torch  # noqa: F401
    L = C.CDLL(LIB_PATH)
    P, V = C.POINTER, C.c_void_p
    L.sde_init_materials.argtypes = [P(MaterialDesc), C.c_int, P(PhysicsParams), P(NuclearTables)]
    L.sde_set_stream.argtypes = [V]
    L.sde_transport.argtypes = [P(Beam), P(PhantomS), C.c_uint64, C.c_uint64, V]
    L.sde_transport_ex.argtypes = [P(Beam), P(PhantomS), C.c_uint64, C.c_uint64, V, V,
                                   P(C.c_int64), P(C.c_double), P(Launch)]
    L.sde_plan_create.argtypes = [P(Beam), P(PhantomS), C.c_uint64, C.c_uint64, P(Launch), P(V)]
    L.sde_plan_execute.argtypes = [V, V, C.c_int]
    L.sde_plan_results.argtypes = [V, V, P(C.c_int64), P(C.c_double)]
    L.sde_plan_destroy.argtypes = [V]
    L.sde_plan_kernel_ms.argtypes = [V, P(C.c_float)]
    L.sde_plan_set_records.argtypes = [V, V]
    L.sde_gamma.argtypes = [V, V, C.c_int, C.c_int, C.c_int, C.c_double, C.c_double, C.c_double,
                            C.c_double, C.c_double, C.c_double, C.c_int, C.c_int, P(C.c_int64)]
    L.sde_launch_limits.argtypes = [P(C.c_int), P(C.c_int), P(C.c_int)]
    L.sde_sbm_polar.argtypes = [V, V, V, C.c_int64, V, V]
    L.sde_gamma_noalloc.argtypes = L.sde_gamma.argtypes
    L.sde_philox_words.argtypes = [C.c_uint64, V, V, V, C.c_int64, V]
    L.sde_free.argtypes = []
    L.sde_free.restype = None
    L.sde_last_error.argtypes = []
    L.sde_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("sde_free", "sde_last_error"):
            getattr(L, name).restype = C.c_int
    return L


lib = _load()


def _check(rc: int):
    if rc != OK:
        raise SdeError(rc, lib.sde_last_error().decode())


def _dptr(t) -> int:
    """Device pointer of a contiguous torch CUDA tensor."""
    if not t.is_cuda:
        raise ValueError("expected a device (cuda) tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


_keep = []


def init_materials(materials: Sequence, params, nuclear=None) -> None:
    """Build and upload the per-material tables.

    materials: workloads Material objects; params: workloads PhysicsParams;
    nuclear: workloads NuclearTables on params' lattice, or None.
    """
    keep = []
    arr = (MaterialDesc * len(materials))()
    for i, m in enumerate(materials):
        Z = np.ascontiguousarray(m.Z, dtype=np.int32)
        A = np.ascontiguousarray(m.A, dtype=np.float64)
        w = np.ascontiguousarray(m.w, dtype=np.float64)
        keep += [Z, A, w]
        arr[i].n_elem = len(Z)
        arr[i].Z = Z.ctypes.data_as(C.POINTER(C.c_int))
        arr[i].A = A.ctypes.data_as(C.POINTER(C.c_double))
        arr[i].w = w.ctypes.data_as(C.POINTER(C.c_double))
        arr[i].I_eV = float(m.I_eV)
    pp = PhysicsParams(params.step_cm, params.ld_z_cm, params.e_min_MeV, params.e_max_MeV,
                       params.ld_F, params.theta_cut_rad, params.backscatter_cut_rad,
                       int(params.n_energy), int(params.flags), int(params.max_steps))
    nt = None
    if nuclear is not None and len(nuclear.Z) > 0:
        if nuclear.lattice.n != params.n_energy:
            raise ValueError("nuclear tables must use the physics energy lattice")
        Z = np.ascontiguousarray(nuclear.Z, dtype=np.int32)
        sg = np.ascontiguousarray(nuclear.sigma, dtype=np.float64)
        ui = np.ascontiguousarray(nuclear.u_icdf, dtype=np.float64)
        kr = np.ascontiguousarray(nuclear.kalbach_r, dtype=np.float64)
        ka = np.ascontiguousarray(nuclear.kalbach_a, dtype=np.float64)
        keep += [Z, sg, ui, kr, ka]
        d = C.POINTER(C.c_double)
        nt = NuclearTables(len(Z), int(nuclear.n_u), Z.ctypes.data_as(C.POINTER(C.c_int)),
                           sg.ctypes.data_as(d), ui.ctypes.data_as(d), kr.ctypes.data_as(d),
                           ka.ctypes.data_as(d))
        el = getattr(nuclear, "elastic", None)
        if el is not None:
            nZ = np.ascontiguousarray(el.ni_Z, dtype=np.int32)
            ns = np.ascontiguousarray(el.ni_sigma, dtype=np.float64)
            npp = np.ascontiguousarray(el.ni_p, dtype=np.float64)
            ha = np.ascontiguousarray(el.h_are, dtype=np.float64)
            hi = np.ascontiguousarray(el.h_aim, dtype=np.float64)
            hb = np.ascontiguousarray(el.h_b, dtype=np.float64)
            keep += [nZ, ns, npp, ha, hi, hb]
            nt.n_ni, nt.n_mu = len(nZ), int(npp.shape[-1]) if len(nZ) else 0
            nt.ni_Z = nZ.ctypes.data_as(C.POINTER(C.c_int))
            nt.ni_sigma_barn, nt.ni_p = ns.ctypes.data_as(d), npp.ctypes.data_as(d)
            nt.n_l = int(ha.shape[0])
            nt.h_a_re, nt.h_a_im, nt.h_b = ha.ctypes.data_as(d), hi.ctypes.data_as(d), \
                hb.ctypes.data_as(d)
    _check(lib.sde_init_materials(arr, len(materials), C.byref(pp),
                                  C.byref(nt) if nt is not None else None))


_STREAM = None   # what set_stream was given


def set_stream(stream=None) -> None:
    """Use a torch.cuda.Stream (or its raw handle); None = the null stream."""
    global _STREAM
    if stream is None:
        h = None
    elif isinstance(stream, int):
        h = stream
    else:
        h = stream.cuda_stream
    _check(lib.sde_set_stream(C.c_void_p(h)))
    _STREAM = stream


def library_stream():
    """The torch stream the library's work runs on (for events around it)."""
    import torch
    if _STREAM is None:
        return torch.cuda.default_stream()
    if isinstance(_STREAM, int):
        return torch.cuda.ExternalStream(_STREAM)
    return _STREAM


def beam_struct(spots) -> tuple:
    arr = (SpotS * len(spots))()
    for i, s in enumerate(spots):
        arr[i] = SpotS(s.E_MeV, s.sigmaE_rel, s.x_cm, s.y_cm, s.sigma_xy_cm, s.weight,
                       int(s.n_histories))
    return Beam(len(spots), C.cast(arr, C.POINTER(SpotS))), arr


@dataclass
class DevicePhantom:
    """A phantom whose voxel arrays live in device memory (torch tensors)."""
    shape: tuple                # (nx, ny, nz)
    voxel_cm: tuple
    origin_cm: tuple
    material_id: object         # torch uint8 (nz, ny, nx) on cuda
    density: object             # torch float32 (nz, ny, nx) on cuda

    @staticmethod
    def from_host(ph, device="cuda"):
        import torch
        return DevicePhantom(tuple(ph.shape), tuple(ph.voxel_cm), tuple(ph.origin_cm),
                             torch.from_numpy(np.ascontiguousarray(ph.material_id)).to(device),
                             torch.from_numpy(np.ascontiguousarray(ph.density)).to(device))

    def struct(self) -> PhantomS:
        nx, ny, nz = self.shape
        o = (C.c_double * 3)(*self.origin_cm)
        return PhantomS(nx, ny, nz, self.voxel_cm[0], self.voxel_cm[1], self.voxel_cm[2], o,
                        _dptr(self.material_id), _dptr(self.density))


def launch_struct(launch: Optional[dict]):
    if not launch:
        return None
    L = Launch()
    for k, v in launch.items():
        setattr(L, k, int(v))
    return L


@dataclass
class TransportResult:
    ledger: np.ndarray      # int64 [LEDGER_N]
    scale: float


def transport(spots, phantom: DevicePhantom, seed: int, dose_out=None, tally_out=None,
              n_histories: int = 0, launch: Optional[dict] = None) -> TransportResult:
    """Run sde_transport_ex.  dose_out: float64 (nz,ny,nx) cuda tensor or None;
    tally_out: int64 (nz,ny,nx) cuda tensor or None."""
    beam, keep = beam_struct(spots)
    ph = phantom.struct()
    ledger = np.zeros(LEDGER_N, dtype=np.int64)
    scale = C.c_double(0.0)
    L = launch_struct(launch)
    rc = lib.sde_transport_ex(C.byref(beam), C.byref(ph), C.c_uint64(n_histories),
                              C.c_uint64(seed),
                              C.c_void_p(_dptr(dose_out) if dose_out is not None else None),
                              C.c_void_p(_dptr(tally_out) if tally_out is not None else None),
                              ledger.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(scale),
                              C.byref(L) if L is not None else None)
    del keep
    _check(rc)
    return TransportResult(ledger, scale.value)


class Plan:
    """A prepared beam + phantom + seed; execute() runs one persistent launch
    (optionally replayed from a hipGraph)."""

    def __init__(self, spots, phantom: DevicePhantom, seed: int, n_histories: int = 0,
                 launch: Optional[dict] = None):
        beam, keep = beam_struct(spots)
        ph = phantom.struct()
        L = launch_struct(launch)
        h = C.c_void_p()
        _check(lib.sde_plan_create(C.byref(beam), C.byref(ph), C.c_uint64(n_histories),
                                   C.c_uint64(seed), C.byref(L) if L is not None else None,
                                   C.byref(h)))
        del keep
        self._h = h
        self.phantom = phantom
        self.n_histories = (int(n_histories) if n_histories and len(spots) == 1
                            else int(sum(sp.n_histories for sp in spots)))

    def execute(self, dose_out=None, use_graph: bool = False) -> None:
        _check(lib.sde_plan_execute(self._h, C.c_void_p(_dptr(dose_out) if dose_out is not None
                                                        else None), int(use_graph)))

    def results(self, tally_out=None):
        """(ledger int64[LEDGER_N], scale); copies the tally into tally_out (cuda int64
        (nz,ny,nx)) when given.  Synchronises the stream."""
        ledger = np.zeros(LEDGER_N, dtype=np.int64)
        sc = C.c_double()
        _check(lib.sde_plan_results(self._h, C.c_void_p(_dptr(tally_out) if tally_out is not None
                                                        else None),
                                    ledger.ctypes.data_as(C.POINTER(C.c_int64)), C.byref(sc)))
        return ledger, sc.value

    def set_records(self, rec) -> None:
        """Per-history records into rec (cuda float32 (n, 12)) from the next execution."""
        if rec is not None and (rec.dtype.itemsize != 4 or rec.numel() < 12 * self.n_histories):
            raise ValueError("records need a float32 buffer of n_histories x 12")
        _check(lib.sde_plan_set_records(self._h, C.c_void_p(_dptr(rec) if rec is not None
                                                            else None)))
        self._rec = rec

    def kernel_ms(self) -> float:
        """Event-timed duration of the transport kernel of the last plain execution."""
        ms = C.c_float()
        _check(lib.sde_plan_kernel_ms(self._h, C.byref(ms)))
        return float(ms.value)

    def close(self) -> None:
        if self._h:
            _check(lib.sde_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sbm_polar(t, u, z):
    """(cos, sin) of the small-angle step's polar angle as the transport draws
    it with SBM, for float32 device tensors t, u, z of one length."""
    import torch
    n = t.numel()
    assert u.numel() == n and z.numel() == n
    for a in (t, u, z):
        assert a.dtype == torch.float32 and a.is_cuda and a.is_contiguous()
    c = torch.empty_like(t)
    s = torch.empty_like(t)
    _check(lib.sde_sbm_polar(C.c_void_p(_dptr(t)), C.c_void_p(_dptr(u)), C.c_void_p(_dptr(z)),
                             int(n), C.c_void_p(_dptr(c)), C.c_void_p(_dptr(s))))
    return c, s


def philox_words(seed: int, h, n, b):
    """Philox4x32-10 blocks (count, 4) uint32 -> int32 tensor as the transport
    draws them, for device tensors h (int64), n, b (int32) of one length."""
    import torch
    count = h.numel()
    assert n.numel() == count and b.numel() == count
    assert h.dtype == torch.int64 and n.dtype == torch.int32 and b.dtype == torch.int32
    for a in (h, n, b):
        assert a.is_cuda and a.is_contiguous()
    out = torch.empty((count, 4), dtype=torch.int32, device=h.device)
    _check(lib.sde_philox_words(C.c_uint64(seed), C.c_void_p(_dptr(h)), C.c_void_p(_dptr(n)),
                                C.c_void_p(_dptr(b)), int(count), C.c_void_p(_dptr(out))))
    return out


def gamma(ref, ev, voxel_cm, dd: float = 0.02, dta_cm: float = 0.05, thresh: float = 0.01,
          interp: int = 10, local: bool = True):
    """(pass fraction, n evaluated, n passed) of cuda float64 (nz,ny,nx) tensors."""
    if ref.shape != ev.shape or ref.dtype != ev.dtype:
        raise ValueError("ref and ev must have the same shape and dtype")
    nz, ny, nx = ref.shape
    cnt = np.zeros(2, dtype=np.int64)
    _check(lib.sde_gamma(C.c_void_p(_dptr(ref)), C.c_void_p(_dptr(ev)), nx, ny, nz,
                         voxel_cm[0], voxel_cm[1], voxel_cm[2], dd, dta_cm, thresh, int(interp),
                         int(local), cnt.ctypes.data_as(C.POINTER(C.c_int64))))
    ne, npass = int(cnt[0]), int(cnt[1])
    return (npass / ne if ne else 1.0), ne, npass


def gamma_noalloc(ref, ev, voxel_cm, dd: float = 0.02, dta_cm: float = 0.05,
                  thresh: float = 0.01, interp: int = 10, local: bool = True):
    """As ``gamma``, through the entry point that allocates no device memory."""
    if ref.shape != ev.shape or ref.dtype != ev.dtype:
        raise ValueError("ref and ev must have the same shape and dtype")
    nz, ny, nx = ref.shape
    cnt = np.zeros(2, dtype=np.int64)
    _check(lib.sde_gamma_noalloc(C.c_void_p(_dptr(ref)), C.c_void_p(_dptr(ev)), nx, ny, nz,
                                 voxel_cm[0], voxel_cm[1], voxel_cm[2], dd, dta_cm, thresh,
                                 int(interp), int(local),
                                 cnt.ctypes.data_as(C.POINTER(C.c_int64))))
    ne, npass = int(cnt[0]), int(cnt[1])
    return (npass / ne if ne else 1.0), ne, npass


def launch_limits():
    """(compute units, LDS bytes per workgroup, LDS bytes used by the tables)."""
    a, b, c = C.c_int(), C.c_int(), C.c_int()
    _check(lib.sde_launch_limits(C.byref(a), C.byref(b), C.byref(c)))
    return a.value, b.value, c.value


def free() -> None:
    lib.sde_free()
