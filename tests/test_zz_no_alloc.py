"""fabric_shade_gbuffer_noalloc (hybrid shading with its fallback queue in
the library's fixed device array) against fabric_shade_gbuffer, through the
C ABI: bitwise the same output on two calls in a row, the second with a
smaller frame, and the size limit."""
import ctypes

import numpy as np
import pytest

import fabric_inputs as fi
from tests.helpers import require_gpu

pytestmark = pytest.mark.gpu


def test_noalloc_matches_shade_gbuffer_twice():
    torch = require_gpu()
    import paper_2406_17782_amd as pkg
    from paper_2406_17782_amd import _abi

    wl = fi.WORKLOADS["hybrid_1080p"]
    mats = wl.materials()
    fab = pkg.Fabric(0, seed=wl.seed())
    try:
        fab.encode(mats)
        big = pkg.DeviceGBuffer.from_host(wl.gbuffer())
        small_h = fi.make_gbuffer(333, 211, 8, seed=wl.seed() + 91, out_of_range_frac=0.3)
        small = pkg.DeviceGBuffer.from_host(small_h)
        # (frame, precision, fallback samples, seed): the large frame through the
        # 32-pixel tiles and the wave-per-pixel queue, the small (ragged) one
        # through the 16-pixel fp32 tiles and the lane-per-pixel queue.
        cases = [(big, "bf16", 256, 5), (small, "fp32", 16, 6)]
        refs = []
        for g, prec, n_s, seed in cases:
            ref = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
            pkg.fabric_shade_gbuffer(fab.ctx, g, pkg.PREC[prec], n_s, seed, ref)
            refs.append(ref)
        outs = []
        for g, prec, n_s, seed in cases:      # two calls in a row, then one sync
            out = torch.full((3, g.n), float("nan"), dtype=torch.float32, device="cuda")
            pkg.fabric_shade_gbuffer_noalloc(fab.ctx, g, pkg.PREC[prec], n_s, seed, out)
            outs.append(out)
        torch.cuda.synchronize()
        for (g, prec, n_s, _), ref, out in zip(cases, refs, outs):
            r, o = ref.cpu().numpy(), out.cpu().numpy()
            print(f"{prec} n={g.n} fallback={n_s}: max |diff| {np.abs(r - o).max():.3g}")
            assert np.array_equal(r, o), (prec, g.n)
        # The small frame's fallback pixels really went through the queue.
        oor = (small_h.radius > 1.0) | (small_h.wo_z < 0.05)
        assert oor.mean() > 0.2
        assert fab.error_count() == 0

        # Beyond the fixed array's frame size: E_RANGE before any device work.
        gs = small.c_struct()
        gs.n = _abi.FABRIC_NOALLOC_MAX_PIXELS + 1
        st = _abi.lib().fabric_shade_gbuffer_noalloc(fab.ctx, ctypes.byref(gs), pkg.FABRIC_BF16,
                                                     16, ctypes.c_uint64(1), outs[1].data_ptr(),
                                                     None)
        assert st == _abi.FABRIC_E_RANGE
    finally:
        fab.close()
