"""ctypes binding of the microbenchmark C ABI (include/sde_roofs.h):
argument marshalling only, plus the table of measurements the benchmark
reports.  The kernels run in ``libsde.so``; torch supplies the buffers."""

from __future__ import annotations

import ctypes as C

from .sde import _check, lib

EXPORTS = ("sde_microbench",)

FMA, TRANS, MIX, MUL64, GATOMIC, LATOMIC, HBM = range(7)
INT = 1        # variant of FMA: integer shift-add chains
TRANS_NAMES = ("exp2", "log2", "rcp", "sqrt", "rsq", "sin")

lib.sde_microbench.argtypes = [C.c_int, C.c_int, C.c_void_p, C.c_size_t, C.c_int, C.c_int,
                               C.c_int64, C.c_int, C.POINTER(C.c_double),
                               C.POINTER(C.c_double)]
lib.sde_microbench.restype = C.c_int


def microbench(kind: int, variant: int = 0, buf=None, grid: int = 2048, block: int = 256,
               iters: int = 4096, reps: int = 3):
    """Run one microbenchmark; returns (units per launch, ms per launch).
    ``buf``: a CUDA tensor (atomic and HBM kinds) or None."""
    units, ms = C.c_double(), C.c_double()
    ptr = C.c_void_p(buf.data_ptr()) if buf is not None else None
    nbytes = buf.numel() * buf.element_size() if buf is not None else 0
    _check(lib.sde_microbench(kind, variant, ptr, nbytes, grid, block, iters, reps,
                              C.byref(units), C.byref(ms)))
    return units.value, ms.value


def measure_roofs(n_cu: int, hbm_bytes: int = 4 << 30, atomic_bytes: int = 1 << 30) -> dict:
    """The transport kernel's ingredients timed alone on cuda:0: rates per
    second (lane-operations, atomics, bytes) and costs in FMA issue slots."""
    import torch
    grid = 8 * n_cu
    out = {}
    # bring the clocks to their loaded state first (about 0.2 s of FMAs)
    microbench(FMA, grid=grid, iters=65536, reps=20)
    u, ms = microbench(FMA, grid=grid, iters=32768)
    fma = u / (ms * 1e-3)
    out["fma_lane_ops_s"] = fma
    for v, name in ((1, "lshl_add"), (2, "mul_f32"), (3, "add_f32"), (4, "xor")):
        u, ms = microbench(FMA, v, grid=grid, iters=32768)
        out[f"{name}_lane_ops_s"] = u / (ms * 1e-3)
        out[f"{name}_slots"] = fma / out[f"{name}_lane_ops_s"]
    # each transcendental alone: its cost in FMA issue slots
    for v, name in enumerate(TRANS_NAMES):
        u, ms = microbench(TRANS, v, grid=grid, iters=2048)
        out[f"{name}_lane_ops_s"] = u / (ms * 1e-3)
        out[f"{name}_slots"] = fma / out[f"{name}_lane_ops_s"]
    # a square root beside K FMAs: FMA slots per (1 square root + K FMAs),
    # measured, and what issuing them one after the other would take
    for k in (1, 2, 4, 8):
        u, ms = microbench(MIX, k, grid=grid, iters=4096)
        groups = u / (1 + k)
        out[f"mix_sqrt_plus_{k}fma_slots"] = (ms * 1e-3) * fma / groups
        out[f"mix_sqrt_plus_{k}fma_serial_slots"] = out["sqrt_slots"] + k
    # 32 x 32 -> 64 multiply-adds
    u, ms = microbench(MUL64, grid=grid, iters=8192)
    out["mul64_per_s"] = u / (ms * 1e-3)
    out["mul64_slots"] = fma / out["mul64_per_s"]
    # int64 atomics: one address; one per wave; random over a footprint that
    # stays in each XCD's L2 (2 MiB) and over one that does not
    abuf = torch.zeros(atomic_bytes // 8, dtype=torch.int64, device="cuda")
    for v, name, b in ((0, "same", abuf), (1, "wave", abuf), (2, "random_2MiB", abuf[: 1 << 18]),
                       (2, f"random_{atomic_bytes >> 20}MiB", abuf)):
        iters = 16 if v == 0 else 256
        u, ms = microbench(GATOMIC, v, b, grid=grid, iters=iters)
        out[f"global_atomic64_{name}_per_s"] = u / (ms * 1e-3)
    del abuf
    for v, name in ((0, "same"), (2, "random")):
        u, ms = microbench(LATOMIC, v, grid=grid, iters=1024 if v == 2 else 256)
        out[f"lds_atomic64_{name}_per_s"] = u / (ms * 1e-3)
    hbuf = torch.empty(hbm_bytes // 4, dtype=torch.float32, device="cuda")
    hbuf.fill_(1.0)
    for v, name in ((0, "read"), (1, "write"), (2, "copy")):
        u, ms = microbench(HBM, v, hbuf, grid=grid * 4, block=256)
        out[f"hbm_{name}_bytes_s"] = u / (ms * 1e-3)
    del hbuf
    torch.cuda.synchronize()
    return out
