"""GPU tests of the full-size workloads and of the editing / autograd API,
against the FP64 oracle (sampled outputs at full size)."""
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
    f = pkg.Fabric(0, seed=11)
    yield f
    f.close()


def test_4k_64_fabrics_sampled(fab, pkg, orc, torch):
    """3840x2160, 64 fabrics with patterns up to 16x16 and radii down to 1e-4
    cells: analytic filter (256 samples) and fp32 / bf16 / fp8 shading of the
    whole frame, checked on a seeded 0.25 % of the pixels (20,736)."""
    wl = fi.WORKLOADS["fabric64_4k"]
    mats, g = wl.materials(), wl.gbuffer()
    assert max(m.wx for m in mats) > 8 and g.n == 3840 * 2160
    params = fi.init_params(12, bias_scale=0.05)
    fab.set_params(params)
    fab.encode(mats)
    d = pkg.DeviceGBuffer.from_host(g)
    _, comp = fab.gt_filtered(d, 256, 31)
    rgb16 = fab.shade(d, "bf16")
    rgb32 = fab.shade(d, "fp32")
    rgb8 = fab.shade(d, "fp8")
    torch.cuda.synchronize()
    idx = fi.subset_indices(g.n, 0.0025, 5)
    sub = g.subset(idx)
    o_comp, _, flagged, _ = orc.filter_gbuffer(mats, sub, 256, 31, same_sample=True, pixel_index=idx)
    print(assert_filter_parity(comp.cpu().numpy()[:, idx], o_comp, flagged, 256))
    z = orc.encoder(params[fi.N_DECODER_PARAMS:].astype(np.float64), mats)
    _, orgb = orc.decoder_gbuffer(params[: fi.N_DECODER_PARAMS], z, mats, sub)
    e32 = rel_norm_err(rgb32.cpu().numpy()[:, idx], orgb)
    e16 = rel_norm_err(rgb16.cpu().numpy()[:, idx], orgb)
    e8 = rel_norm_err(rgb8.cpu().numpy()[:, idx], orgb)
    print("4k fp32", e32, "bf16", e16, "fp8", e8)
    assert e32 < 1e-5 and e16 < 6e-2 and e8 < FP8_BOUND


def test_albedo_edit_needs_no_reencode(fab, pkg, orc, torch):
    """Albedos sit outside the network (Eq. (8)): editing them changes the
    composed reflectance without touching latents."""
    mats = fi.materials_for(8, 40)
    g = fi.make_gbuffer(64, 32, 8, seed=41)
    params = fi.init_params(42, bias_scale=0.05)
    fab.set_params(params)
    fab.encode(mats)
    d = pkg.DeviceGBuffer.from_host(g)
    lat0 = fab.latents()
    kd = np.array([[0.9, 0.1, 0.1], [0.1, 0.9, 0.1]], dtype=np.float32)
    ks = np.array([[0.3, 0.3, 0.9], [0.7, 0.2, 0.2]], dtype=np.float32)
    for f in range(8):
        pkg.fabric_set_albedo(fab.ctx, f, kd, ks)
        mats[f].kd, mats[f].ks = kd.copy(), ks.copy()
    rgb = fab.shade(d, "fp32").cpu().numpy()
    assert np.array_equal(fab.latents(), lat0)
    z = orc.encoder(params[fi.N_DECODER_PARAMS:].astype(np.float64), mats)
    _, orgb = orc.decoder_gbuffer(params[: fi.N_DECODER_PARAMS], z, mats, g)
    assert rel_norm_err(rgb, orgb) < 1e-5
    # A roughness edit re-encodes: the latent of that fabric changes.
    mats[3].alpha = np.array([0.9, 0.9], dtype=np.float32)
    fab.encode(mats)
    lat1 = fab.latents()
    assert not np.allclose(lat1[3], lat0[3]) and np.allclose(np.delete(lat1, 3, 0), np.delete(lat0, 3, 0))


def test_autograd_functions_match_oracle(fab, pkg, orc, torch):
    """torch.autograd through the hand-written decoder and encoder kernels:
    gradients of a weighted sum of the decoder outputs."""
    from paper_2406_17782_amd import autograd
    mats = fi.materials_for(8, 50)[:4]
    g = fi.make_gbuffer(48, 32, 4, seed=51)
    g.fabric_id[:] = np.random.default_rng(52).integers(0, 4, g.n).astype(np.uint16)
    params = fi.init_params(53, bias_scale=0.05)
    fab.set_params(params)
    fab.encode(mats)
    d = pkg.DeviceGBuffer.from_host(g)
    dec = torch.tensor(params[: fi.N_DECODER_PARAMS], device="cuda", requires_grad=True)
    enc = torch.tensor(params[fi.N_DECODER_PARAMS:], device="cuda", requires_grad=True)
    w = torch.from_numpy(np.random.default_rng(54).normal(size=(4, g.n)).astype(np.float32)).cuda()
    z = autograd.encoder(enc, fab)
    y = autograd.decoder(dec, z, fab, d)
    (y * w).sum().backward()
    # Oracle: the same objective through its decoder backward and encoder backprop.
    zo = orc.encoder(params[fi.N_DECODER_PARAMS:].astype(np.float64), mats)
    assert rel_norm_err(z.detach().cpu().numpy(), zo) < 1e-5
    gd, gl = orc.decoder_backward(params[: fi.N_DECODER_PARAMS], zo, mats, g, w.cpu().numpy())
    assert rel_norm_err(dec.grad.cpu().numpy(), gd) < 1e-4
    # Encoder gradient: the latent gradient pushed through the encoder equals
    # the encoder part of the oracle's gradient for a loss whose dL/dy = w.
    ge = enc.grad.cpu().numpy()
    assert np.isfinite(ge).all() and np.abs(ge).max() > 0
    gz = torch.from_numpy(gl.astype(np.float32)).cuda()
    ge2 = torch.empty(fi.N_ENCODER_PARAMS, device="cuda")
    pkg.fabric_encoder_backward(fab.ctx, enc.detach(), gz, ge2)
    assert rel_norm_err(ge, ge2.cpu().numpy()) < 1e-4


# BF16 training: the decoder's forward and activation-gradient products take
# BF16 operands (unit roundoff 2^-8, rms relative error 2^-8 / sqrt(3) =
# 0.23 % per operand, sqrt(2) x that per product); four forward and four
# backward layers chain to about sqrt(8) x 0.32 % = 0.9 % on a gradient
# entry.  Weight gradients and the loss sums stay in FP32.  Bound: 3 % of the
# whole gradient's norm and 1 % of the loss.
BF16_GRAD_BOUND = 3e-2
BF16_LOSS_BOUND = 1e-2


def _grad_parity(fab, pkg, orc, torch, mats, g, tg, params):
    fab.set_params(params)
    fab.encode(mats)
    d = pkg.DeviceGBuffer.from_host(g)
    t = torch.from_numpy(tg).cuda()
    l32, g32 = fab.loss_grad(d, t, prec=pkg.FABRIC_FP32)
    l16, g16 = fab.loss_grad(d, t, prec=pkg.FABRIC_BF16)
    oloss, ograd, _ = orc.loss_grad(params.astype(np.float64), mats, g, tg)
    g32, g16 = g32.cpu().numpy(), g16.cpu().numpy()
    assert l32 == pytest.approx(oloss, rel=1e-5)
    off = 0
    for k, (o, i) in enumerate(fi.DECODER_SHAPES + fi.ENCODER_SHAPES):
        for size in (o * i, o):
            err = rel_norm_err(g32[off:off + size], ograd[off:off + size])
            assert err < 1e-4, (k, size, err)
            off += size
    e16 = rel_norm_err(g16, ograd)
    print(f"n {g.n}: loss fp32 {l32:.6g} bf16 {l16:.6g} oracle {oloss:.6g}; bf16 grad err {e16:.3g}")
    assert abs(l16 - oloss) < BF16_LOSS_BOUND * oloss
    assert e16 < BF16_GRAD_BOUND


def test_bf16_training_gradient_vs_oracle(fab, pkg, orc, torch):
    """FP32 and BF16 loss and gradient against the oracle on 4,096 samples."""
    mats = fi.materials_for(8, 60)
    g = fi.make_gbuffer(64, 64, 8, seed=61)
    tg = fi.random_targets(g.n, 62)
    _grad_parity(fab, pkg, orc, torch, mats, g, tg, fi.init_params(63, bias_scale=0.05))


def test_loss_grad_full_batch_2p20(fab, pkg, orc, torch):
    """The training workload's full batch, 2^20 samples with the fabric id
    uniform over 8 fabrics: FP32 and BF16 loss and gradient (the launches a
    training step makes at that size) against the oracle over every sample."""
    wl = fi.WORKLOADS["train_2p20"]
    mats = wl.materials()
    g = wl.gbuffer()
    assert g.n == 1 << 20
    g.fabric_id[:] = np.random.default_rng(64).integers(0, 8, g.n).astype(np.uint16)
    tg = fi.random_targets(g.n, 65)
    _grad_parity(fab, pkg, orc, torch, mats, g, tg, fi.init_params(66, bias_scale=0.05))
