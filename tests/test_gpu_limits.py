"""GPU tests at the boundary's limits, against the FP64 oracle: the largest
fabric table (every fabric's constants and c_f staged in LDS), the largest
footprint sample count, and one-pixel / sub-tile frames."""
import numpy as np
import pytest

import fabric_inputs as fi
from tests.helpers import assert_filter_parity, rel_norm_err, require_gpu
from tests.test_gpu_fp8 import FP8_BOUND

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
    f = pkg.Fabric(0, seed=23)
    yield f
    f.close()


def test_max_fabrics_shading(fab, pkg, orc, torch):
    """FABRIC_MAX_FABRICS (256) fabrics, every pixel on a seeded random one:
    fp32 / bf16 / fp8 shading against the oracle's decoder, and the filter."""
    n_fab = pkg.FABRIC_MAX_FABRICS
    mats = fi.materials_for(n_fab, 120, max_random_side=16)
    g = fi.make_gbuffer(96, 67, n_fab, seed=121)
    g.fabric_id[:] = np.random.default_rng(122).integers(0, n_fab, g.n).astype(np.uint16)
    params = fi.init_params(123, bias_scale=0.05)
    fab.set_params(params)
    fab.encode(mats)
    d = pkg.DeviceGBuffer.from_host(g)
    z = orc.encoder(params[fi.N_DECODER_PARAMS:].astype(np.float64), mats)
    _, orgb = orc.decoder_gbuffer(params[: fi.N_DECODER_PARAMS], z, mats, g)
    errs = {p: rel_norm_err(fab.shade(d, p).cpu().numpy(), orgb) for p in ("fp32", "bf16", "fp8")}
    print("256 fabrics", errs)
    assert errs["fp32"] < 1e-5 and errs["bf16"] < 6e-2 and errs["fp8"] < FP8_BOUND
    idx = fi.subset_indices(g.n, 0.1, 124)
    _, comp = fab.gt_filtered(d, 64, 125)
    o_comp, _, flagged, _ = orc.filter_gbuffer(mats, g.subset(idx), 64, 125, same_sample=True,
                                               pixel_index=idx)
    print(assert_filter_parity(comp.cpu().numpy()[:, idx], o_comp, flagged, 64))


def test_max_samples_filter(fab, pkg, orc, torch):
    """FABRIC_MAX_SAMPLES (128^2) footprint samples per pixel on a few pixels
    with large footprints, same samples as the oracle; one more sample is
    rejected."""
    mats = fi.materials_for(4, 130)
    g = fi.make_gbuffer(5, 3, 4, seed=131)
    g.radius[:] = np.linspace(0.3, 4.0, g.n).astype(np.float32)
    fab.encode(mats)
    d = pkg.DeviceGBuffer.from_host(g)
    n_s = pkg.FABRIC_MAX_SAMPLES
    _, comp = fab.gt_filtered(d, n_s, 132)
    o_comp, _, flagged, _ = orc.filter_gbuffer(mats, g, n_s, 132, same_sample=True)
    print(assert_filter_parity(comp.cpu().numpy(), o_comp, flagged, n_s))
    with pytest.raises(pkg.FabricError):
        fab.gt_filtered(d, 129 * 129, 132)


@pytest.mark.parametrize("n", [1, 2, 31, 33])
def test_tiny_frames(fab, pkg, orc, torch, n):
    """Frames smaller than one 32-pixel tile or one tile plus a pixel: every
    precision's shading and the filter against the oracle."""
    mats = fi.materials_for(3, 140)
    g = fi.make_gbuffer(n, 1, 3, seed=141 + n)
    params = fi.init_params(142, bias_scale=0.05)
    fab.set_params(params)
    fab.encode(mats)
    d = pkg.DeviceGBuffer.from_host(g)
    z = orc.encoder(params[fi.N_DECODER_PARAMS:].astype(np.float64), mats)
    _, orgb = orc.decoder_gbuffer(params[: fi.N_DECODER_PARAMS], z, mats, g)
    for prec, bound in (("fp32", 1e-5), ("bf16", 6e-2), ("fp16", 8e-3), ("fp8", FP8_BOUND)):
        rgb = fab.shade(d, prec).cpu().numpy()
        assert rgb.shape == (3, n)
        assert rel_norm_err(rgb, orgb) < bound, prec
    _, comp = fab.gt_filtered(d, 16, 143)
    o_comp, _, flagged, _ = orc.filter_gbuffer(mats, g, 16, 143, same_sample=True)
    assert_filter_parity(comp.cpu().numpy(), o_comp, flagged, 16)
