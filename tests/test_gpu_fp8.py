"""GPU tests of the FP8-E4M3 shading decoder (per-layer power-of-two scales,
FP32 accumulation) against the FP64 oracle, through the C ABI.

E4M3 keeps 3 mantissa bits: unit roundoff u = 2^-4, i.e. a uniform relative
rounding error of rms u / sqrt(3) = 3.6 % per operand.  A layer rounds both
its weights and its input, so its output carries about sqrt(2) x 3.6 % = 5 %
relative error (rms over the outputs); four chained layers add up to about
sqrt(4) x 5 % = 10 %.  The tests allow 25 % norm-wise (2.5x margin)."""
import numpy as np
import pytest

import fabric_inputs as fi
from tests.helpers import rel_norm_err, require_gpu

pytestmark = pytest.mark.gpu

FP8_BOUND = 0.25


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def pkg(torch):
    import paper_2406_17782_amd as pkg
    return pkg


def _fab(pkg):
    return pkg.Fabric(0, seed=17)


def _case(n_fab=8, w=64, h=65, seed=70):
    mats = fi.materials_for(n_fab, seed)
    g = fi.make_gbuffer(w, h, n_fab, seed=seed + 1)
    g.fabric_id[:] = np.random.default_rng(seed).integers(0, n_fab, g.n).astype(np.uint16)
    params = fi.init_params(seed + 2, bias_scale=0.05)
    return mats, g, params


def test_fp8_shade_error_vs_oracle(pkg, orc, torch):
    """8 fabrics, 64 x 65 pixels (ragged last tile): fp8 shading against the
    oracle's FP64 decoder and composition, beside bf16."""
    mats, g, params = _case()
    fab = _fab(pkg)
    try:
        fab.set_params(params)
        fab.encode(mats)
        d = pkg.DeviceGBuffer.from_host(g)
        z = orc.encoder(params[fi.N_DECODER_PARAMS:].astype(np.float64), mats)
        _, orgb = orc.decoder_gbuffer(params[: fi.N_DECODER_PARAMS], z, mats, g)
        e8 = rel_norm_err(fab.shade(d, "fp8").cpu().numpy(), orgb)
        e16 = rel_norm_err(fab.shade(d, "bf16").cpu().numpy(), orgb)
        print("fp8 shade rel err", e8, "bf16", e16)
        assert np.isfinite(e8) and e8 < FP8_BOUND
    finally:
        fab.close()


def test_fp8_scales_do_not_depend_on_the_frame(pkg, torch):
    """The scales come from the parameters and encoded fabrics only: shading
    a subset of the pixels reproduces them bitwise."""
    mats, g, params = _case(seed=80)
    fab = _fab(pkg)
    try:
        fab.set_params(params)
        fab.encode(mats)
        full = fab.shade(pkg.DeviceGBuffer.from_host(g), "fp8").cpu().numpy()
        idx = np.arange(3, g.n, 7)
        part = fab.shade(pkg.DeviceGBuffer.from_host(g.subset(idx)), "fp8").cpu().numpy()
        assert np.array_equal(part, full[:, idx])
    finally:
        fab.close()


def test_fp8_recalibrates_after_encode_and_parameter_change(pkg, torch):
    """A context that re-encodes (or takes new parameters) after an fp8 frame
    shades exactly like a fresh context set up with the final state."""
    mats_a, g, params = _case(seed=90)
    mats_b = fi.materials_for(8, 91)
    params2 = fi.init_params(93, bias_scale=0.05)
    d = pkg.DeviceGBuffer.from_host(g)
    f1, f2 = _fab(pkg), _fab(pkg)
    try:
        f1.set_params(params)
        f1.encode(mats_a)
        f1.shade(d, "fp8")
        f1.encode(mats_b)
        r1 = f1.shade(d, "fp8").cpu().numpy()
        f2.set_params(params)
        f2.encode(mats_b)
        r2 = f2.shade(d, "fp8").cpu().numpy()
        assert np.array_equal(r1, r2)
        f1.set_params(params2)
        f1.encode(mats_b)
        f2.set_params(params2)
        f2.encode(mats_b)
        assert np.array_equal(f1.shade(d, "fp8").cpu().numpy(), f2.shade(d, "fp8").cpu().numpy())
        assert not np.array_equal(r1, f1.shade(d, "fp8").cpu().numpy())
    finally:
        f1.close()
        f2.close()


def test_fp8_faults_and_hybrid_routing(pkg, torch):
    mats = fi.materials_for(8, 100)
    g = fi.make_gbuffer(96, 40, 8, seed=101, out_of_range_frac=0.2)
    g.wo_z[3] = -0.2
    g.radius[5] = 0.0
    g.u[7] = np.nan
    g.fabric_id[9] = 8
    fab = _fab(pkg)
    try:
        fab.set_params(fi.init_params(102, bias_scale=0.05))
        fab.encode(mats)
        d = pkg.DeviceGBuffer.from_host(g)
        fab.error_count(reset=True)
        neural = fab.shade(d, "fp8").cpu().numpy()
        assert np.all(neural[:, [3, 5, 7, 9]] == 0.0)
        assert fab.error_count(reset=True) == 4
        hybrid = fab.shade(d, "fp8", fallback_samples=64, seed=9).cpu().numpy()
        analytic = fab.gt_filtered(d, 64, 9)[0].cpu().numpy()
        bad = np.zeros(g.n, bool)
        bad[[3, 5, 7, 9]] = True
        oor = ((g.radius > 1.0) | (g.wo_z < 0.05)) & ~bad
        assert 0.1 < oor.mean() < 0.3
        assert np.array_equal(hybrid[:, ~oor], neural[:, ~oor])
        assert np.array_equal(hybrid[:, oor], analytic[:, oor])
        empty = fi.make_gbuffer(0, 0, 1, seed=1)
        assert fab.shade(pkg.DeviceGBuffer.from_host(empty), "fp8").shape == (3, 0)
    finally:
        fab.close()


def test_fp8_raw_decoder_forward_is_rejected(pkg, torch):
    """The raw decoder forward (training and autograd) exists in fp32 and
    bf16 only; fp8 is a shading precision."""
    mats, g, params = _case(n_fab=2, w=8, h=8, seed=110)
    fab = _fab(pkg)
    try:
        fab.encode(mats)
        dp = torch.from_numpy(params[: fi.N_DECODER_PARAMS]).cuda()
        dl = torch.from_numpy(fi.random_latents(2, 111)).cuda()
        y = torch.empty((4, g.n), device="cuda")
        with pytest.raises(pkg.FabricError):
            pkg.fabric_decoder_forward(fab.ctx, pkg.DeviceGBuffer.from_host(g),
                                       pkg.FABRIC_FP8_E4M3, dp, dl, y)
    finally:
        fab.close()
