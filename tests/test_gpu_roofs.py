"""The microbenchmarks of the transport's ingredients (VALU issue, int64
atomics, HBM stream) through the C ABI: their work counts are exact (the
atomics add up, the stream writes and copies what it says) and no measured
rate exceeds the chip's published or derived ceiling."""

import numpy as np
import pytest

from gpu_common import log

pytestmark = pytest.mark.gpu

VALU_PEAK = 256 * 4 * 16 * 2.4e9      # non-packed 32-bit lane-operations/s
HBM_PEAK = 8.0e12                     # bytes/s


def test_atomic_counts_are_exact():
    import torch
    from paper_2511_03115_amd import roofs
    buf = torch.zeros(1 << 16, dtype=torch.int64, device="cuda")
    grid, block, iters, reps = 64, 256, 8, 2
    for variant in (0, 1, 2):
        buf.zero_()
        u, ms = roofs.microbench(roofs.GATOMIC, variant, buf, grid=grid, block=block,
                                 iters=iters, reps=reps)
        torch.cuda.synchronize()
        total = int(buf.sum().item())
        log(f"global atomics variant {variant}: units {u:.0f} ms {ms:.4f} sum {total}")
        assert u == grid * block * iters
        assert total == u * (1 + reps)
        if variant == 0:
            assert int(buf[0].item()) == total
        if variant == 1:   # one word per wave, 32 words apart
            nz = torch.nonzero(buf).flatten().cpu().numpy()
            assert len(nz) == grid * block // 64 and np.all(nz % 32 == 0)


def test_stream_writes_and_copies():
    import torch
    from paper_2511_03115_amd import roofs
    n = (1 << 22)                      # 16 MiB of float32
    buf = torch.zeros(n, dtype=torch.float32, device="cuda")
    u, ms = roofs.microbench(roofs.HBM, 1, buf, grid=512, block=256, reps=1)
    assert u == n * 4
    want = torch.tensor([1.0, 2.0, 3.0, 4.0], device="cuda").repeat(n // 4)
    assert torch.equal(buf, want)
    buf[: n // 2] = torch.arange(n // 2, dtype=torch.float32, device="cuda")
    u, ms = roofs.microbench(roofs.HBM, 2, buf, grid=512, block=256, reps=1)
    assert u == n * 4                  # read half + write half
    assert torch.equal(buf[n // 2:], buf[: n // 2])


def test_measured_rates_stay_under_the_ceilings():
    import torch
    from paper_2511_03115_amd import roofs
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    r = roofs.measure_roofs(n_cu, hbm_bytes=2 << 30, atomic_bytes=256 << 20)
    for k, v in r.items():
        log(f"{k} {v:.4g}")
    assert 0.5 * VALU_PEAK < r["fma_lane_ops_s"] <= 1.02 * VALU_PEAK
    for name in roofs.TRANS_NAMES:
        assert r[f"{name}_slots"] >= 0.98
    assert r["hbm_read_bytes_s"] <= 1.02 * HBM_PEAK
    assert r["hbm_copy_bytes_s"] <= 1.02 * HBM_PEAK
    assert r["global_atomic64_random_2MiB_per_s"] > 0 and r["lds_atomic64_random_per_s"] > 0
    assert r["lshl_add_slots"] > 0.3 and r["mul64_slots"] > 0.3
