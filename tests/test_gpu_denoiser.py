"""The trained denoiser against the method without it, and checkpoints.

Gain: on held-out training-style patches (never seen in training: patch
indices 1000+), a 1e5-history map is compared with a 1e8-history
reference of the same beam (independent seeds) before and after the
network.  The network must lower the RMS relative error above 1 % of the
maximum and raise the gamma pass rate (local 2 %/0.5 mm, 1 % threshold).
"""

import os

import numpy as np
import pytest

from gpu_common import log

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2511_03115_amd", "weights", "denoiser_plan2mm.npz")


def _rel_err(d, ref, thr=0.01):
    m = ref >= thr * ref.max()          # masked before dividing: no zero denominators
    return float(np.sqrt((((d[m] - ref[m]) / ref[m]) ** 2).mean()))


def test_trained_network_gains_over_no_network():
    import torch
    import workloads
    from paper_2511_03115_amd import denoiser, judge, sde
    from workloads import configs
    assert os.path.exists(WEIGHTS), "trained weights are part of the package"
    first = configs.denoiser_patch(1000, 1)
    sde.init_materials(first.phantom.materials, first.params,
                       workloads.nuclear_for_phantom(first.phantom, first.params.lattice()))
    shape = first.phantom.material_id.shape
    dn = denoiser.Denoiser(WEIGHTS, shape)
    plain_e, den_e, plain_g, den_g = [], [], [], []
    for i in range(1000, 1004):
        wl = configs.denoiser_patch(i, 100_000_000)
        dph = sde.DevicePhantom.from_host(wl.phantom)
        ref = torch.zeros(shape, dtype=torch.float64, device="cuda")
        low = torch.zeros_like(ref)
        sde.transport(wl.spots, dph, wl.seed, dose_out=ref)
        sde.transport(workloads.with_histories(wl.spots, 100_000), dph, wl.seed + 77, dose_out=low)
        den = dn(low, dph.density)
        r, l, d = ref.cpu().numpy(), low.cpu().numpy(), den.cpu().numpy()
        vcm = wl.phantom.voxel_cm
        plain_e.append(_rel_err(l, r))
        den_e.append(_rel_err(d, r))
        plain_g.append(judge.gamma_pass(ref, low, vcm))
        den_g.append(judge.gamma_pass(ref, den, vcm))
        log(f"patch {i}: rel err plain {plain_e[-1]:.4f} denoised {den_e[-1]:.4f}; "
            f"gamma plain {plain_g[-1]:.4f} denoised {den_g[-1]:.4f}")
    dn.close()
    assert np.mean(den_e) < 0.8 * np.mean(plain_e)
    assert np.mean(den_g) > np.mean(plain_g)


def test_checkpoint_resume_is_exact(tmp_path):
    """Training 2k steps equals training k, saving, loading into a fresh
    network and training k more (bit for bit)."""
    import torch
    from paper_2511_03115_amd import denoiser, nn
    rng = np.random.default_rng(3)
    B, D, H, W = 2, 16, 16, 16
    dose = torch.from_numpy(rng.uniform(0, 1, (B, D, H, W)).astype(np.float32)).cuda()
    tgt = torch.from_numpy(rng.uniform(0, 1, (B, D, H, W)).astype(np.float32)).cuda()

    def steps(net, k):
        for _ in range(k):
            net.loss_grad(dose, None, tgt)
            net.adam_step(1e-3)

    a = nn.Net(3, 16, 16, 0.01, B, (D, H, W), train=True)
    a.set_params(denoiser.init_params(5, levels=3))
    steps(a, 6)
    b = nn.Net(3, 16, 16, 0.01, B, (D, H, W), train=True)
    b.set_params(denoiser.init_params(5, levels=3))
    steps(b, 3)
    path = str(tmp_path / "ck.npz")
    denoiser.save_checkpoint(path, b, {"note": "test"})
    b.close()
    ck = denoiser.load_checkpoint(path)
    assert ck["config"]["levels"] == 3 and ck["config"]["note"] == "test"
    c = nn.Net(3, 16, 16, 0.01, B, (D, H, W), train=True)
    c.set_params(ck["params"])
    c.set_adam_state(ck["adam_m"], ck["adam_v"], int(ck["adam_step"][0]))
    steps(c, 3)
    assert np.array_equal(a.get_params(), c.get_params())
    a.close()
    c.close()
