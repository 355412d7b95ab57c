"""GPU tests of the inter-yarn visibility V of Eq. (3)-(4) in the analytic
filter, through the C ABI, against the FP64 oracle with the same samples
and the same float32 march: several fabrics with tall yarns and a ragged
pixel count, the 1080p workload on a sampled subset, flat fabrics (equal to
V = 1 bit for bit), the switch, the hybrid fallback and generated training
targets."""
import numpy as np
import pytest

import fabric_inputs as fi
from tests.helpers import assert_filter_parity_vis, require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def pkg(torch):
    import paper_2406_17782_amd as pkg
    return pkg


@pytest.fixture()
def fab(pkg):
    f = pkg.Fabric(0, seed=41)
    yield f
    f.close()


def tall(mats, seed):
    rng = np.random.default_rng(seed)
    for m in mats:
        m.beta[:] = rng.uniform(0.8, 2.0, 2).astype(np.float32)
    return mats


def test_filter_visibility_matches_oracle(fab, pkg, orc, torch):
    mats = tall(fi.materials_for(8, 170), 171)
    g = fi.make_gbuffer(64, 65, 8, seed=172)
    g.fabric_id[:] = np.random.default_rng(173).integers(0, 8, g.n).astype(np.uint16)
    fab.encode(mats)
    d = pkg.DeviceGBuffer.from_host(g)
    _, c0 = fab.gt_filtered(d, 256, 174)
    fab.set_visibility(True)
    _, c1 = fab.gt_filtered(d, 256, 174)
    c0, c1 = c0.cpu().numpy(), c1.cpu().numpy()
    o_comp, _, flagged, _ = orc.filter_gbuffer(mats, g, 256, 174, same_sample=True, visibility=True)
    print(assert_filter_parity_vis(c1, o_comp, flagged, 256))
    changed = np.abs(c1 - c0).max(axis=0) > 1e-3 * np.abs(c0).max(axis=0)
    print("pixels changed by visibility", changed.mean())
    assert changed.mean() > 0.05
    fab.set_visibility(False)
    _, c2 = fab.gt_filtered(d, 256, 174)
    assert np.array_equal(c2.cpu().numpy(), c0)


def test_filter_visibility_below_64_samples(fab, pkg, orc, torch):
    """The lane-per-pixel filter with V, 16 samples, against the oracle."""
    mats = fi.materials_for(8, 180)
    g = fi.make_gbuffer(45, 29, 8, seed=181)
    g.fabric_id[:] = np.random.default_rng(182).integers(0, 8, g.n).astype(np.uint16)
    fab.encode(mats)
    fab.set_visibility(True)
    _, comp = fab.gt_filtered(pkg.DeviceGBuffer.from_host(g), 16, 183)
    o_comp, _, flagged, _ = orc.filter_gbuffer(mats, g, 16, 183, same_sample=True, visibility=True)
    print(assert_filter_parity_vis(comp.cpu().numpy(), o_comp, flagged, 16))


def test_flat_fabrics_unchanged(fab, pkg, torch):
    mats = fi.materials_for(8, 175)
    for m in mats:
        m.beta[:] = 0.0
    g = fi.make_gbuffer(40, 33, 8, seed=176)
    fab.encode(mats)
    d = pkg.DeviceGBuffer.from_host(g)
    r0, c0 = fab.gt_filtered(d, 64, 177)
    fab.set_visibility(True)
    r1, c1 = fab.gt_filtered(d, 64, 177)
    assert np.array_equal(c0.cpu().numpy(), c1.cpu().numpy())
    assert np.array_equal(r0.cpu().numpy(), r1.cpu().numpy())


def test_visibility_1080p_sampled(fab, pkg, orc, torch):
    wl = fi.WORKLOADS["fabric8_1080p"]
    mats, g = wl.materials(), wl.gbuffer()
    fab.encode(mats)
    fab.set_visibility(True)
    d = pkg.DeviceGBuffer.from_host(g)
    _, comp = fab.gt_filtered(d, 256, 178)
    idx = fi.subset_indices(g.n, 0.002, 179)
    o_comp, _, flagged, _ = orc.filter_gbuffer(mats, g.subset(idx), 256, 178, same_sample=True,
                                               pixel_index=idx, visibility=True)
    print(assert_filter_parity_vis(comp.cpu().numpy()[:, idx], o_comp, flagged, 256))


def test_hybrid_fallback_uses_visibility(fab, pkg, torch):
    mats = tall(fi.materials_for(8, 180), 181)
    g = fi.make_gbuffer(64, 48, 8, seed=182, out_of_range_frac=0.3)
    fab.encode(mats)
    fab.set_visibility(True)
    d = pkg.DeviceGBuffer.from_host(g)
    rgb_f, _ = fab.gt_filtered(d, 64, 183)
    hyb = fab.shade(d, "bf16", fallback_samples=64, seed=183).cpu().numpy()
    oor = (g.radius > np.float32(1.0)) | (g.wo_z < np.float32(0.05))
    assert oor.any()
    assert np.array_equal(hyb[:, oor], rgb_f.cpu().numpy()[:, oor])


def test_generated_targets_use_visibility(fab, pkg, torch):
    """A step's generated targets are the filter's components with V: the
    loss and gradient equal those of the same batch with those targets."""
    mats = tall(fi.materials_for(8, 184), 185)
    fab.set_params(fi.init_params(186, bias_scale=0.05))
    fab.encode(mats)
    fab.set_visibility(True)
    n = 4096
    batch = pkg.DeviceGBuffer.empty(n)
    pkg.fabric_make_batch(fab.ctx, 187, n, 1e-3, 0.5, batch)
    _, comp = fab.gt_filtered(batch, 64, 187 ^ 1, rgb=False)
    cfg = dict(prec=pkg.FABRIC_FP32, gt_samples=64, seed=187, batch=n)
    l_gen, g_gen = fab.loss_grad(None, None, **cfg)
    l_tgt, g_tgt = fab.loss_grad(batch, comp, **cfg)
    assert l_gen == l_tgt
    assert np.array_equal(g_gen.cpu().numpy(), g_tgt.cpu().numpy())
    fab.set_visibility(False)
    l_off, _ = fab.loss_grad(None, None, **cfg)
    assert l_off != l_gen
