"""GPU parity of the HIP path against the FP64 oracle, through the C ABI.

Footprint filter: same samples (SplitMix64 jitter, concentric map) on both
sides, the oracle rounding the sample position to float32 before
classification; every pixel with no sample near a classification edge agrees
to 1e-4 of its largest component, and a pixel with k of its N samples near
an edge to 1e-4 + k / N.
Decoder FP32: norm-wise 1e-5 (elementwise 1e-4); BF16 / FP16: bounds derived
from the operand unit roundoff (see the tests).  Gradients: 1e-4 norm-wise per
tensor against the oracle's FP64 backprop.
"""
import math

import numpy as np
import pytest

import fabric_inputs as fi
from tests.helpers import assert_filter_parity, rel_norm_err, require_gpu

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
    f = pkg.Fabric(0, seed=7)
    yield f
    f.close()


def dev(pkg, g):
    return pkg.DeviceGBuffer.from_host(g)


def params_for(seed, bias=0.05):
    return fi.init_params(seed, bias_scale=bias)


# ---------------------------------------------------------------------------
# Footprint filter
# ---------------------------------------------------------------------------

def test_gt_filter_plain128_all_pixels(fab, pkg, orc, torch):
    """Plain weave, 128 x 128, 64 samples: every pixel against the oracle."""
    wl = fi.WORKLOADS["plain128"]
    mats, g = wl.materials(), wl.gbuffer()
    fab.encode(mats)
    seed = 1234
    rgb, comp = fab.gt_filtered(dev(pkg, g), 64, seed)
    torch.cuda.synchronize()
    o_comp, o_rgb, flagged, fault = orc.filter_gbuffer(mats, g, 64, seed, same_sample=True)
    assert fault.sum() == 0
    print(assert_filter_parity(comp.cpu().numpy(), o_comp, flagged, 64))
    assert_filter_parity(rgb.cpu().numpy(), o_rgb, flagged, 64)
    assert fab.error_count() == 0


def test_gt_filter_eight_fabrics_ragged(fab, pkg, orc, torch):
    """8 weaves, per-pixel fabric ids, 256 samples, n not a multiple of 4 waves."""
    mats = fi.materials_for(8, 2000)
    g = fi.make_gbuffer(77, 53, 8, seed=2001)
    g.fabric_id[:] = np.random.default_rng(5).integers(0, 8, g.n).astype(np.uint16)
    fab.encode(mats)
    rgb, comp = fab.gt_filtered(dev(pkg, g), 256, 99)
    torch.cuda.synchronize()
    o_comp, o_rgb, flagged, _ = orc.filter_gbuffer(mats, g, 256, 99, same_sample=True)
    print(assert_filter_parity(comp.cpu().numpy(), o_comp, flagged, 256))
    assert_filter_parity(rgb.cpu().numpy(), o_rgb, flagged, 256)


def test_gt_filter_1080p_sampled(fab, pkg, orc, torch):
    """The 1080p, 8-fabric workload at 256 samples as the benchmark launches it;
    a seeded 0.2 % of the pixels checked against the oracle one by one."""
    wl = fi.WORKLOADS["fabric8_1080p"]
    mats, g = wl.materials(), wl.gbuffer()
    fab.encode(mats)
    rgb, comp = fab.gt_filtered(dev(pkg, g), 256, 4242)
    torch.cuda.synchronize()
    idx = fi.subset_indices(g.n, 0.002, 77)
    sub = g.subset(idx)
    o_comp, o_rgb, flagged, _ = orc.filter_gbuffer(mats, sub, 256, 4242, same_sample=True,
                                                   pixel_index=idx)
    gc = comp.cpu().numpy()[:, idx]
    print(assert_filter_parity(gc, o_comp, flagged, 256))


def test_gt_filter_deterministic_and_seeded(fab, pkg, torch):
    mats = fi.materials_for(8, 3000)
    g = fi.make_gbuffer(64, 32, 8, seed=3001)
    fab.encode(mats)
    d = dev(pkg, g)
    a = fab.gt_filtered(d, 256, 5)[1].cpu().numpy()
    b = fab.gt_filtered(d, 256, 5)[1].cpu().numpy()
    assert np.array_equal(a, b)
    c = fab.gt_filtered(d, 256, 6)[1].cpu().numpy()
    assert not np.array_equal(a, c)


@pytest.mark.parametrize("n_samples", [1, 4, 16, 49])
def test_gt_filter_below_64_samples(fab, pkg, orc, torch, n_samples):
    """Below 64 samples a lane owns a pixel and takes its samples in order:
    8 weaves, per-pixel fabric ids, n not a multiple of the 256-pixel
    workgroup; every pixel against the oracle with the same samples."""
    mats = fi.materials_for(8, 2100)
    g = fi.make_gbuffer(61, 37, 8, seed=2101)
    g.fabric_id[:] = np.random.default_rng(2102).integers(0, 8, g.n).astype(np.uint16)
    fab.encode(mats)
    rgb, comp = fab.gt_filtered(dev(pkg, g), n_samples, 321)
    torch.cuda.synchronize()
    o_comp, o_rgb, flagged, _ = orc.filter_gbuffer(mats, g, n_samples, 321, same_sample=True)
    print(assert_filter_parity(comp.cpu().numpy(), o_comp, flagged, n_samples))
    assert_filter_parity(rgb.cpu().numpy(), o_rgb, flagged, n_samples)
    assert fab.error_count() == 0


def test_gt_filter_1080p_16_samples_sampled(fab, pkg, orc, torch):
    """The 1080p frame at 16 samples (one lane per pixel, as the equal-time
    comparison launches it); a seeded 0.2 % of the pixels against the oracle."""
    wl = fi.WORKLOADS["fabric8_1080p"]
    mats, g = wl.materials(), wl.gbuffer()
    fab.encode(mats)
    _, comp = fab.gt_filtered(dev(pkg, g), 16, 778)
    torch.cuda.synchronize()
    idx = fi.subset_indices(g.n, 0.002, 78)
    o_comp, _, flagged, _ = orc.filter_gbuffer(mats, g.subset(idx), 16, 778, same_sample=True,
                                               pixel_index=idx)
    print(assert_filter_parity(comp.cpu().numpy()[:, idx], o_comp, flagged, 16))


# ---------------------------------------------------------------------------
# Decoder forward
# ---------------------------------------------------------------------------

def _decoder_case(n_fab=8, w=64, h=65, seed=10):
    mats = fi.materials_for(n_fab, seed)
    g = fi.make_gbuffer(w, h, n_fab, seed=seed + 1)
    g.fabric_id[:] = np.random.default_rng(seed).integers(0, n_fab, g.n).astype(np.uint16)
    params = params_for(seed + 2)
    lat = fi.random_latents(n_fab, seed + 3)
    return mats, g, params, lat


def test_decoder_forward_fp32_matches_oracle(fab, pkg, orc, torch):
    mats, g, params, lat = _decoder_case()
    fab.encode(mats)
    dp = torch.from_numpy(params[: fi.N_DECODER_PARAMS]).cuda()
    dl = torch.from_numpy(lat).cuda()
    y = torch.empty((4, g.n), device="cuda")
    pkg.fabric_decoder_forward(fab.ctx, dev(pkg, g), pkg.FABRIC_FP32, dp, dl, y)
    torch.cuda.synchronize()
    oy, _ = orc.decoder_gbuffer(params[: fi.N_DECODER_PARAMS], lat, mats, g)
    gy = y.cpu().numpy()
    err = rel_norm_err(gy, oy)
    print("fp32 decoder rel err", err)
    assert err < 1e-5
    scale = np.abs(oy).max()
    assert np.abs(gy - oy).max() < 1e-4 * scale


@pytest.mark.parametrize("prec,bound", [("bf16", 3e-2), ("fp16", 4e-3)])
def test_decoder_forward_low_precision_error(fab, pkg, orc, torch, prec, bound):
    """Operand rounding to bf16 (unit roundoff 2^-8) or fp16 (2^-11) in four
    chained layers: the norm-wise error stays within ~4 roundoffs of FP64 per
    layer chain on these inputs; the bound leaves a 2x margin (per-pixel
    bounds: tests/test_gpu_precision.py)."""
    mats, g, params, lat = _decoder_case(seed=20)
    fab.encode(mats)
    dp = torch.from_numpy(params[: fi.N_DECODER_PARAMS]).cuda()
    dl = torch.from_numpy(lat).cuda()
    oy, _ = orc.decoder_gbuffer(params[: fi.N_DECODER_PARAMS], lat, mats, g)
    if prec == "bf16":
        y = torch.empty((4, g.n), device="cuda")
        pkg.fabric_decoder_forward(fab.ctx, dev(pkg, g), pkg.FABRIC_BF16, dp, dl, y)
        gy = y.cpu().numpy()
        err = rel_norm_err(gy, oy)
        print(prec, "decoder rel err", err)
        assert err < bound
    # Composed shading at this precision vs the oracle composition.
    fab.set_params(params)
    fab.encode(mats)
    z = orc.encoder(params[fi.N_DECODER_PARAMS:].astype(np.float64), mats)
    _, orgb = orc.decoder_gbuffer(params[: fi.N_DECODER_PARAMS], z, mats, g)
    rgb = fab.shade(dev(pkg, g), prec).cpu().numpy()
    err = rel_norm_err(rgb, orgb)
    print(prec, "shade rel err", err)
    assert err < 2 * bound


def test_shade_fp32_matches_oracle_with_encoded_latents(fab, pkg, orc, torch):
    mats, g, params, _ = _decoder_case(seed=30)
    fab.set_params(params)
    fab.encode(mats)
    z = orc.encoder(params[fi.N_DECODER_PARAMS:].astype(np.float64), mats)
    assert rel_norm_err(fab.latents(), z) < 1e-5
    _, orgb = orc.decoder_gbuffer(params[: fi.N_DECODER_PARAMS], z, mats, g)
    rgb = fab.shade(dev(pkg, g), "fp32").cpu().numpy()
    err = rel_norm_err(rgb, orgb)
    print("fp32 shade rel err", err)
    assert err < 1e-5


def test_faults_empty_and_state(fab, pkg, orc, torch):
    mats, g, params, _ = _decoder_case(n_fab=2, w=16, h=4, seed=40)
    with pytest.raises(pkg.FabricError) as e:
        fab.shade(dev(pkg, g), "fp32")
    assert e.value.status == 6          # E_STATE: nothing encoded yet
    fab.set_params(params)
    fab.encode(mats)
    g.wo_z[3] = -0.2
    g.radius[5] = 0.0
    g.u[7] = np.inf
    g.fabric_id[9] = 2
    fab.error_count(reset=True)
    rgb = fab.shade(dev(pkg, g), "bf16").cpu().numpy()
    assert np.all(rgb[:, [3, 5, 7, 9]] == 0.0)
    assert fab.error_count(reset=True) == 4
    _, comp = fab.gt_filtered(dev(pkg, g), 16, 1)
    assert np.all(comp.cpu().numpy()[:, [3, 5, 7, 9]] == 0.0)
    assert fab.error_count(reset=True) == 4
    empty = fi.make_gbuffer(0, 0, 1, seed=1)
    assert fab.shade(dev(pkg, empty), "bf16").shape == (3, 0)
    with pytest.raises(pkg.FabricError):
        fab.gt_filtered(dev(pkg, g), 15, 1)            # not a perfect square


def test_hybrid_routing_matches_both_paths(fab, pkg, torch):
    mats = fi.materials_for(8, 50)
    g = fi.make_gbuffer(96, 40, 8, seed=51, out_of_range_frac=0.2)
    fab.set_params(params_for(52))
    fab.encode(mats)
    d = dev(pkg, g)
    neural = fab.shade(d, "bf16").cpu().numpy()
    hybrid = fab.shade(d, "bf16", fallback_samples=64, seed=9).cpu().numpy()
    analytic = fab.gt_filtered(d, 64, 9)[0].cpu().numpy()
    oor = (g.radius > 1.0) | (g.wo_z < 0.05)
    assert 0.1 < oor.mean() < 0.3
    assert np.array_equal(hybrid[:, ~oor], neural[:, ~oor])
    assert np.array_equal(hybrid[:, oor], analytic[:, oor])
    # Below 64 samples both the queue and the plain filter take a lane per pixel.
    hybrid9 = fab.shade(d, "bf16", fallback_samples=9, seed=9).cpu().numpy()
    analytic9 = fab.gt_filtered(d, 9, 9)[0].cpu().numpy()
    assert np.array_equal(hybrid9[:, ~oor], neural[:, ~oor])
    assert np.array_equal(hybrid9[:, oor], analytic9[:, oor])


# ---------------------------------------------------------------------------
# Gradients and training
# ---------------------------------------------------------------------------

def test_decoder_backward_matches_oracle(fab, pkg, orc, torch):
    mats, g, params, lat = _decoder_case(n_fab=4, w=64, h=33, seed=60)
    fab.encode(mats)
    dy = np.random.default_rng(61).normal(size=(4, g.n)).astype(np.float32)
    dp = torch.from_numpy(params[: fi.N_DECODER_PARAMS]).cuda()
    dl = torch.from_numpy(lat).cuda()
    gp = torch.empty(fi.N_DECODER_PARAMS, device="cuda")
    gl = torch.empty((4, 32), device="cuda")
    pkg.fabric_decoder_backward(fab.ctx, dev(pkg, g), dp, dl, torch.from_numpy(dy).cuda(), gp, gl)
    torch.cuda.synchronize()
    ogp, ogl = orc.decoder_backward(params[: fi.N_DECODER_PARAMS], lat, mats, g, dy)
    gp = gp.cpu().numpy()
    off = 0
    for k, (o, i) in enumerate(fi.DECODER_SHAPES):
        for name, size in ((f"W{k + 1}", o * i), (f"b{k + 1}", o)):
            err = rel_norm_err(gp[off:off + size], ogp[off:off + size])
            print(name, err)
            assert err < 1e-4, name
            off += size
    assert rel_norm_err(gl.cpu().numpy(), ogl) < 1e-4


def test_loss_grad_matches_oracle(fab, pkg, orc, torch):
    """Loss of Eq. (9)-(11) and the full encoder + decoder gradient (FP32)."""
    mats = fi.materials_for(8, 70)
    g = fi.make_gbuffer(64, 64, 8, seed=71)
    g.fabric_id[:] = np.random.default_rng(72).integers(0, 8, g.n).astype(np.uint16)
    tg = fi.random_targets(g.n, 73)
    params = params_for(74)
    fab.set_params(params)
    fab.encode(mats)
    grad = torch.empty(fi.N_PARAMS, device="cuda")
    loss = pkg.fabric_loss_grad(fab.ctx, dev(pkg, g), torch.from_numpy(tg).cuda(),
                                {"prec": pkg.FABRIC_FP32}, grad)
    oloss, ograd, _ = orc.loss_grad(params, mats, g, tg)
    assert loss == pytest.approx(oloss, rel=1e-5)
    gg = grad.cpu().numpy()
    off = 0
    for k, (o, i) in enumerate(fi.DECODER_SHAPES + fi.ENCODER_SHAPES):
        for size in (o * i, o):
            err = rel_norm_err(gg[off:off + size], ograd[off:off + size])
            assert err < 1e-4, (k, size, err)
            off += size


def test_loss_grad_bf16_matches_oracle(fab, pkg, orc, torch):
    """The training step's own precision (Sec. 5.2 config: BF16 operands on
    the matrix cores, FP32 accumulation): loss and the full encoder +
    decoder gradient against the oracle's FP64 backward on a ragged batch.
    Bars from BF16's unit roundoff 2^-8: a rounded product errs by at most
    2u with zero mean, so a layer's output picks up a relative norm error
    of about u sqrt(2/3) ~ 3.2e-3; four forward and three transposed layers
    stacked in quadrature give ~8.5e-3 on a delta, and a weight gradient
    carries both of its factors' errors: 4e-2 per tensor, 2e-2 on the whole
    gradient, 1e-2 on the loss (the forward's output error, doubled by the
    square).  The encoder's tensors inherit the latents' gradient error."""
    mats = fi.materials_for(8, 75)
    g = fi.make_gbuffer(67, 61, 8, seed=76)          # 4,087 samples: a ragged last tile
    g.fabric_id[:] = np.random.default_rng(77).integers(0, 8, g.n).astype(np.uint16)
    g.wo_z[11] = -0.2                                # a faulted sample contributes nothing
    tg = fi.random_targets(g.n, 78)
    params = params_for(79)
    fab.set_params(params)
    fab.encode(mats)
    grad = torch.empty(fi.N_PARAMS, device="cuda")
    loss = pkg.fabric_loss_grad(fab.ctx, dev(pkg, g), torch.from_numpy(tg).cuda(),
                                {"prec": pkg.FABRIC_BF16}, grad)
    oloss, ograd, _ = orc.loss_grad(params, mats, g, tg)
    gg = grad.cpu().numpy()
    errs, off = [], 0
    for o, i in fi.DECODER_SHAPES + fi.ENCODER_SHAPES:
        for size in (o * i, o):
            errs.append(rel_norm_err(gg[off:off + size], ograd[off:off + size]))
            off += size
    whole = rel_norm_err(gg, ograd)
    print("bf16 loss", loss, oloss, "whole", "%.2e" % whole, "per tensor",
          ["%.2e" % e for e in errs])
    assert loss == pytest.approx(oloss, rel=1e-2)
    assert whole < 2e-2
    assert max(errs) < 4e-2


@pytest.mark.parametrize("n_fab", [16, 20, 70])
def test_loss_grad_many_fabrics(pkg, orc, torch, n_fab):
    """Training gradients with more fabrics: 16 (the most whose dL/dc_f tiles
    the fused BF16 launch holds), 20 (BF16 through the blocked planes in
    HBM) and 70 (two one-hot jobs); FP32 at 1e-4 per tensor, BF16 at the
    bars of test_loss_grad_bf16_matches_oracle."""
    mats = fi.materials_for(n_fab, 700 + n_fab)
    g = fi.make_gbuffer(50, 41, n_fab, seed=701)
    g.fabric_id[:] = np.random.default_rng(702).integers(0, n_fab, g.n).astype(np.uint16)
    tg = fi.random_targets(g.n, 703)
    params = params_for(704)
    f = pkg.Fabric(0, seed=705)
    try:
        f.set_params(params)
        f.encode(mats)
        oloss, ograd, _ = orc.loss_grad(params, mats, g, tg)
        for prec, tensor_bar, whole_bar, loss_rel in ((pkg.FABRIC_FP32, 1e-4, 1e-4, 1e-5),
                                                      (pkg.FABRIC_BF16, 4e-2, 2e-2, 1e-2)):
            grad = torch.empty(fi.N_PARAMS, device="cuda")
            loss = pkg.fabric_loss_grad(f.ctx, dev(pkg, g), torch.from_numpy(tg).cuda(),
                                        {"prec": prec}, grad)
            gg = grad.cpu().numpy()
            errs, off = [], 0
            for o, i in fi.DECODER_SHAPES + fi.ENCODER_SHAPES:
                for size in (o * i, o):
                    errs.append(rel_norm_err(gg[off:off + size], ograd[off:off + size]))
                    off += size
            print(n_fab, "fabrics, prec", prec, "loss", loss, oloss, "worst tensor %.2e" % max(errs))
            assert loss == pytest.approx(oloss, rel=loss_rel)
            assert max(errs) < tensor_bar
            assert rel_norm_err(gg, ograd) < whole_bar
    finally:
        f.close()


def test_make_batch_matches_oracle_recipe(fab, pkg, orc, torch):
    fab.encode(fi.materials_for(8, 80))
    n = 100_003
    out = pkg.DeviceGBuffer.empty(n)
    pkg.fabric_make_batch(fab.ctx, 31337, n, 1e-3, 0.5, out)
    torch.cuda.synchronize()
    ref = orc.batch_gen(31337, n, 8, 1e-3, 0.5)
    assert np.array_equal(out.fabric_id.view(torch.int16).cpu().numpy().view(np.uint16), ref.fabric_id)
    assert np.array_equal(out.u.cpu().numpy(), ref.u)
    assert np.array_equal(out.v.cpu().numpy(), ref.v)
    for f in ("radius", "wi_x", "wi_y", "wi_z", "wo_x", "wo_y", "wo_z"):
        a = getattr(out, f).cpu().numpy().astype(np.float64)
        b = getattr(ref, f).astype(np.float64)
        assert np.abs(a - b).max() <= 4e-7 * max(1.0, np.abs(b).max()), f


def test_adam_step_matches_oracle(fab, pkg, orc, torch):
    mats = fi.materials_for(8, 90)
    g = fi.make_gbuffer(32, 32, 8, seed=91)
    tg = fi.random_targets(g.n, 92)
    params = params_for(93)
    fab.set_params(params)
    fab.encode(mats)
    theta = params.copy()
    m = np.zeros(fi.N_PARAMS)
    v = np.zeros(fi.N_PARAMS)
    dg, dt = dev(pkg, g), torch.from_numpy(tg).cuda()
    for t in (1, 2):
        _, ograd, _ = orc.loss_grad(theta.astype(np.float64), mats, g, tg)
        orc.adam_step(theta, ograd, m, v, t, 1e-3)
        fab.train_step(dg, dt, prec=pkg.FABRIC_FP32, lr=1e-3)
        got = fab.params()
        solid = np.abs(ograd) > 1e-5
        assert np.abs(got[solid] - theta[solid]).max() < 2e-6 * t
        assert np.abs(got - theta).max() <= 2.1e-3 * t


def test_checkpoint_roundtrip_and_resume(fab, pkg, torch):
    mats = fi.materials_for(8, 100)
    fab.encode(mats)
    cfg = dict(batch=4096, gt_samples=16, prec=pkg.FABRIC_BF16, lr=2e-3)
    for s in range(3):
        fab.train_step(seed=s, **cfg)
    blob = pkg.fabric_save(fab.ctx)
    for s in range(3, 5):
        fab.train_step(seed=s, **cfg)
    ref = fab.params()
    other = pkg.Fabric(0, seed=1)
    other.encode(mats)
    pkg.fabric_load(other.ctx, blob)
    for s in range(3, 5):
        other.train_step(seed=s, **cfg)
    assert np.array_equal(other.params(), ref)
    other.close()


def test_training_reduces_loss(fab, pkg, torch):
    mats = fi.materials_for(8, 110)
    fab.encode(mats)
    losses = [fab.train_step(seed=s, batch=1 << 14, gt_samples=64, prec=pkg.FABRIC_BF16, lr=3e-3)
              for s in range(60)]
    assert all(math.isfinite(l) for l in losses)
    assert np.mean(losses[-10:]) < 0.7 * np.mean(losses[:5])
    with pytest.raises(pkg.FabricError):
        fab.shade(dev(pkg, fi.make_gbuffer(4, 4, 8, seed=1)), "bf16")   # stale latents
    fab.encode(mats)
    fab.shade(dev(pkg, fi.make_gbuffer(4, 4, 8, seed=1)), "bf16")
