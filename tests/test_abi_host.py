"""The C-ABI library without a GPU: it loads, exports every declared entry
point, and rejects bad input before any device work."""

import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("sde.h", "sde_nn.h", "sde_roofs.h")]
LIB = os.path.join(ROOT, "paper_2511_03115_amd", "libsde.so")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2511_03115_amd import build
        build.build()
    import torch  # noqa: F401  (one HIP runtime per process: torch's, loaded first)
    lib = C.CDLL(LIB)
    lib.sde_last_error.restype = C.c_char_p
    return lib


def declared_functions():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"^\s*(?:int|void|const char\*)\s+(sde_\w+)\s*\(", src, re.M))
    return sorted(names)


def test_header_declares_entry_points():
    names = declared_functions()
    for must in ("sde_init_materials", "sde_transport", "sde_free", "sde_set_stream",
                 "sde_transport_ex", "sde_plan_create", "sde_gamma", "sde_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    for n in declared_functions():
        assert hasattr(lib, n)


def test_binding_names_match_header():
    import importlib
    sde = importlib.import_module("paper_2511_03115_amd.sde")
    nn = importlib.import_module("paper_2511_03115_amd.nn")
    roofs = importlib.import_module("paper_2511_03115_amd.roofs")
    assert not set(sde.EXPORTS) & set(nn.EXPORTS)
    assert not (set(sde.EXPORTS) | set(nn.EXPORTS)) & set(roofs.EXPORTS)
    assert set(sde.EXPORTS) | set(nn.EXPORTS) | set(roofs.EXPORTS) == set(declared_functions())


def test_host_validation_without_gpu(lib):
    from paper_2511_03115_amd import sde
    # transport before tables: state error, no device call
    beam = sde.Beam(0, None)
    assert lib.sde_transport(C.byref(beam), None, C.c_uint64(0), C.c_uint64(0), None) in (
        sde.E_STATE, sde.E_INVALID)
    # invalid materials and parameters are rejected by the host table build
    pp = sde.PhysicsParams(0.05, 0.05, 0.05, 260.0, 0.98, 0.02, 0.04, 1024, 63, 65536)
    assert lib.sde_init_materials(None, 0, C.byref(pp), None) == sde.E_INVALID
    bad = sde.PhysicsParams(-1.0, 0.05, 0.05, 260.0, 0.98, 0.02, 0.04, 1024, 63, 65536)
    Z = (C.c_int * 1)(1)
    A = (C.c_double * 1)(1.008)
    w = (C.c_double * 1)(1.0)
    m = sde.MaterialDesc(1, C.cast(Z, C.POINTER(C.c_int)), C.cast(A, C.POINTER(C.c_double)),
                         C.cast(w, C.POINTER(C.c_double)), 19.2)
    lib.sde_init_materials.argtypes = [C.POINTER(sde.MaterialDesc), C.c_int,
                                       C.POINTER(sde.PhysicsParams), C.c_void_p]
    assert lib.sde_init_materials(C.byref(m), 1, C.byref(bad), None) == sde.E_INVALID
    lib.sde_last_error.restype = C.c_char_p
    assert b"invalid physics parameters" in lib.sde_last_error()
    # the sampler's test entry point checks its arguments before any device call
    lib.sde_sbm_polar.argtypes = [C.c_void_p] * 3 + [C.c_int64] + [C.c_void_p] * 2
    assert lib.sde_sbm_polar(None, None, None, 5, None, None) == sde.E_INVALID
    assert lib.sde_sbm_polar(None, None, None, -1, None, None) == sde.E_INVALID
    assert lib.sde_sbm_polar(None, None, None, 0, None, None) == sde.OK
    # bits other than the physics switches, SDE_FP64 and SDE_ECUT
    unk = sde.PhysicsParams(0.05, 0.05, 0.05, 260.0, 0.98, 0.02, 0.04, 1024, 63 | 512, 65536)
    assert lib.sde_init_materials(C.byref(m), 1, C.byref(unk), None) == sde.E_INVALID
    assert b"unknown physics switch" in lib.sde_last_error()
    # the random-number test entry point checks its arguments before any device call
    lib.sde_philox_words.argtypes = [C.c_uint64] + [C.c_void_p] * 3 + [C.c_int64, C.c_void_p]
    V = C.c_void_p
    assert lib.sde_philox_words(0, None, None, None, 4, None) == sde.E_INVALID
    assert lib.sde_philox_words(0, None, None, None, -1, None) == sde.E_INVALID
    assert lib.sde_philox_words(0, None, None, None, 0, None) == sde.OK
    # a misaligned output (the fake addresses are never dereferenced)
    assert lib.sde_philox_words(0, V(0x10000), V(0x10000), V(0x10000), 4, V(0x10008)) == \
        sde.E_INVALID
    assert b"misaligned" in lib.sde_last_error()
    # a medium whose Bethe stopping power is negative at e_min (I far too large)
    m.I_eV = 5000.0
    assert lib.sde_init_materials(C.byref(m), 1, C.byref(pp), None) == sde.E_INVALID
    assert b"stopping power" in lib.sde_last_error()
    # gamma argument checks
    cnt = (C.c_int64 * 2)()
    assert lib.sde_gamma(None, None, 1, 1, 1, C.c_double(0.1), C.c_double(0.1),
                         C.c_double(0.1), C.c_double(0.02), C.c_double(0.05), C.c_double(0.01),
                         10, 1, cnt) == sde.E_INVALID


def test_nn_config_validation_without_gpu(lib):
    from paper_2511_03115_amd import nn
    h = C.c_void_p()

    def create(**kw):
        base = dict(levels=4, base_channels=16, in_channels=16, leaky_alpha=0.01, max_batch=1,
                    max_d=64, max_h=64, max_w=64, train=0, adam_beta1=0.9, adam_beta2=0.999,
                    adam_eps=1e-8, store_concat=0)
        base.update(kw)
        cfg = nn.Config(*[base[f] for f, _ in nn.Config._fields_])
        return lib.sde_nn_create(C.byref(cfg), C.byref(h))

    from paper_2511_03115_amd import sde
    assert create(levels=0) == sde.E_INVALID
    assert create(base_channels=24) == sde.E_INVALID
    assert create(in_channels=2) == sde.E_INVALID
    assert create(leaky_alpha=0.0) == sde.E_INVALID
    assert create(max_d=60) == sde.E_INVALID          # not a multiple of 2^(L-1)
    assert create(levels=5) == sde.E_INVALID          # 256 channels: outside the tile set
    assert b"tile set" in lib.sde_last_error()
    n = C.c_size_t()
    assert lib.sde_nn_conv3d_workspace(1, 4, 4, 4, 8, 16, C.byref(n)) == sde.E_INVALID
    assert lib.sde_nn_conv3d_workspace(2, 4, 4, 4, 32, 64, C.byref(n)) == sde.OK
    assert n.value >= 27 * 32 * 64 * 4


def test_nn_layer_alignment_is_checked_without_gpu(lib):
    """The layer entry points read bf16 operands 16 bytes at a time: a
    misaligned pointer is refused before any device call (the fake addresses
    below are never dereferenced)."""
    from paper_2511_03115_amd import sde
    V, F, Z = C.c_void_p, C.c_float, C.c_size_t
    ok, bad = V(0x10000), V(0x10002)
    assert lib.sde_nn_conv3d_fwd(bad, ok, None, 1, 2, 2, 2, 16, 16, F(0.01), 1, ok, None) == \
        sde.E_INVALID
    assert b"aligned" in lib.sde_last_error()
    assert lib.sde_nn_conv3d_fwd(ok, ok, None, 1, 2, 2, 2, 16, 16, F(0.01), 1, bad, None) == \
        sde.E_INVALID
    assert lib.sde_nn_conv3d_dgrad(ok, bad, 1, 2, 2, 2, 16, 16, ok, ok, Z(1 << 20)) == \
        sde.E_INVALID
    assert lib.sde_nn_conv3d_wgrad(ok, ok, 1, 2, 2, 2, 16, 16, ok, None, bad, Z(1 << 20)) == \
        sde.E_INVALID


def test_microbench_arguments_are_checked_without_gpu(lib):
    """The microbenchmark entry point refuses bad shapes, kinds, variants and
    buffers before any device call."""
    from paper_2511_03115_amd import roofs, sde
    u, m = C.c_double(), C.c_double()
    mb = lib.sde_microbench
    mb.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_size_t, C.c_int, C.c_int, C.c_int64,
                   C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]

    def call(kind, variant, buf=None, nbytes=0, grid=8, block=64, iters=4, reps=1):
        return mb(kind, variant, buf, nbytes, grid, block, iters, reps, C.byref(u), C.byref(m))
    assert call(roofs.FMA, 0, block=96) == sde.E_INVALID
    assert call(roofs.FMA, 0, grid=0) == sde.E_INVALID
    assert call(roofs.FMA, 0, reps=0) == sde.E_INVALID
    assert call(roofs.FMA, 0, iters=0) == sde.E_INVALID
    assert call(roofs.FMA, 5) == sde.E_INVALID
    assert call(roofs.TRANS, 6) == sde.E_INVALID
    assert call(roofs.MIX, 3) == sde.E_INVALID
    assert call(roofs.LATOMIC, 1) == sde.E_INVALID
    assert call(9, 0) == sde.E_INVALID
    assert b"unknown" in lib.sde_last_error()
    assert call(roofs.GATOMIC, 2) == sde.E_INVALID                     # no buffer
    assert call(roofs.HBM, 0, C.c_void_p(0x10000), 4096) == sde.E_INVALID   # < 1 MiB
    assert call(roofs.HBM, 0, C.c_void_p(0x10008), 1 << 20) == sde.E_INVALID  # misaligned
    assert mb(0, 0, None, 0, 8, 64, 4, 1, None, None) == sde.E_INVALID
