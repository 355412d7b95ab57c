"""What the trained network gains over the method without it (Sec. 5,
"Comparison against previous work": the network against shading with one
sample per pixel).  The paper-size decoder is trained on the GPU by the
library's own kernels (generated batches, 256-sample analytic targets,
Adam; about 20 s) and its BF16 shading of the 1080p workload is compared
with one jittered analytic sample per pixel, both against the oracle's
256-sample footprint filter on the seeded 1 % of the frame the benchmark
uses: over all of those pixels, not a band of footprints."""
import math
import sys

import numpy as np
import pytest

import fabric_inputs as fi
from tests.helpers import require_gpu

pytestmark = pytest.mark.gpu

STEPS = 48_000
BATCH = 1 << 16


def rmse(a, b):
    return float(np.sqrt(np.mean((np.asarray(a, np.float64) - b) ** 2)))


def test_trained_network_beats_one_analytic_sample(orc):
    torch = require_gpu()
    import paper_2406_17782_amd as pkg
    wl = fi.WORKLOADS["fabric8_1080p"]
    mats = wl.materials()
    g = wl.gbuffer()
    fab = pkg.Fabric(0, seed=4600)
    try:
        fab.encode(mats)
        params = fi.init_paper_params(5, bias_scale=0.0)
        z = fi.random_latents(len(mats), 6, scale=0.1, dim=64)
        pkg.fabric_paper_prepare(fab.ctx, torch.from_numpy(params).cuda(),
                                 torch.from_numpy(z).cuda())
        d = pkg.DeviceGBuffer.from_host(g)
        out = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
        idx = fi.subset_indices(g.n, 0.01, 99)
        _, o_rgb, _, _ = orc.filter_gbuffer(mats, g.subset(idx), 256, 4242, same_sample=True,
                                            pixel_index=idx)
        pkg.fabric_paper_shade(fab.ctx, d, out, "bf16")
        untrained = rmse(out.cpu().numpy()[:, idx], o_rgb)
        for s in range(STEPS):
            lr = 1e-2 * 0.5 * (1.0 + math.cos(math.pi * s / STEPS))
            last = s == STEPS - 1
            loss = pkg.fabric_paper_train_step(fab.ctx, None, None,
                                               dict(batch=BATCH, gt_samples=256,
                                                    seed=3_000_000 + s, lr=lr),
                                               want_loss=last or s % 12_000 == 0)
            if loss is not None:
                print(f"step {s}: loss {loss:.5f}", flush=True, file=sys.stderr)
        pkg.fabric_paper_shade(fab.ctx, d, out, "bf16")
        net = rmse(out.cpu().numpy()[:, idx], o_rgb)
        one = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
        pkg.fabric_gt_filtered(fab.ctx, d, 1, 777, one, None)
        one_spp = rmse(one.cpu().numpy()[:, idx], o_rgb)
        print(f"RMSE over {idx.size} pixels: trained network (BF16) {net:.4f}, one analytic "
              f"sample {one_spp:.4f}, untrained network {untrained:.4f}")
        assert net < one_spp < untrained
    finally:
        fab.close()
