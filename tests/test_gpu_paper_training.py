"""GPU parity of the paper-size decoder's training (Sec. 4.2 "Decoder", loss
of Eq. (9)-(11), per-fabric latents trained as parameters) through the C
ABI: the FP32 loss and gradient against the oracle's FP64 backward on a
ragged batch with transmission and faulted samples (norm-wise per tensor
1e-4, as for the config decoder); two Adam steps against the oracle's;
training on generated batches lowers the loss and the shading image follows
the trained masters; the same without the one-blob footprint encoding
(the encoding's ablation) and without the spatial fusion stage (the
fusion's ablation); call errors."""
import numpy as np
import pytest

import fabric_inputs as fi
from tests.helpers import rel_norm_err, require_gpu

pytestmark = pytest.mark.gpu

N = fi.N_PAPER_DECODER_PARAMS


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def pkg(torch):
    import paper_2406_17782_amd as pkg
    return pkg


@pytest.fixture()
def fab(pkg):
    f = pkg.Fabric(0, seed=71)
    yield f
    f.close()


def prepare(fab, pkg, torch, mats, seed):
    fab.encode(mats)
    params = fi.init_paper_params(seed, bias_scale=0.05)
    z = fi.random_latents(len(mats), seed + 1, dim=64)
    pkg.fabric_paper_prepare(fab.ctx, torch.from_numpy(params).cuda(), torch.from_numpy(z).cuda())
    return params, z


def batch(n_fab, w, h, seed):
    g = fi.make_gbuffer(w, h, n_fab, seed=seed, btdf_frac=0.3)
    g.fabric_id[:] = np.random.default_rng(seed + 1).integers(0, n_fab, g.n).astype(np.uint16)
    return g


def per_tensor_errors(got, ref, n_fab):
    errs, off = [], 0
    for o, i in fi.PAPER_DECODER_SHAPES:
        for size in (o * i, o):
            errs.append(rel_norm_err(got[off:off + size], ref[off:off + size]))
            off += size
    errs.append(rel_norm_err(got[off:off + n_fab * 64], ref[off:off + n_fab * 64]))
    return errs


def test_paper_loss_grad_matches_oracle(fab, pkg, orc, torch):
    mats = fi.materials_for(5, 300)
    g = batch(5, 61, 53, 301)            # 3,233 samples: ragged in every split
    g.wo_z[5] = -0.3                     # faulted samples contribute nothing
    g.radius[9] = 0.0
    tg = fi.random_targets(g.n, 302)
    params, z = prepare(fab, pkg, torch, mats, 303)
    grad = torch.empty(N + 5 * 64, device="cuda")
    loss = pkg.fabric_paper_loss_grad(fab.ctx, pkg.DeviceGBuffer.from_host(g),
                                      torch.from_numpy(tg).cuda(), {}, grad)
    oloss, ograd, odlat = orc.paper_loss_grad(params, z, mats, g, tg)
    assert loss == pytest.approx(oloss, rel=1e-5)
    errs = per_tensor_errors(grad.cpu().numpy(), np.concatenate([ograd, odlat.ravel()]), 5)
    print("paper gradient errors", ["%.2e" % e for e in errs])
    assert max(errs) < 1e-4


def test_paper_loss_grad_full_batch_2p16(fab, pkg, orc, torch):
    """The batch the benchmark trains the paper-size network on: 2^16
    samples of the 1080p workload's 8 fabrics (the training workload's
    recipe, cut to 2^16), at the launch size of a training step, against the
    oracle over every sample."""
    wl = fi.WORKLOADS["train_2p20"]
    mats = wl.materials()
    g = wl.gbuffer().subset(np.arange(1 << 16))
    g.fabric_id[:] = np.random.default_rng(74).integers(0, 8, g.n).astype(np.uint16)
    tg = fi.random_targets(g.n, 75)
    params, z = prepare(fab, pkg, torch, mats, 76)
    grad = torch.empty(N + 8 * 64, device="cuda")
    loss = pkg.fabric_paper_loss_grad(fab.ctx, pkg.DeviceGBuffer.from_host(g),
                                      torch.from_numpy(tg).cuda(), {}, grad)
    oloss, ograd, odlat = orc.paper_loss_grad(params, z, mats, g, tg)
    assert loss == pytest.approx(oloss, rel=1e-5)
    errs = per_tensor_errors(grad.cpu().numpy(), np.concatenate([ograd, odlat.ravel()]), 8)
    print("paper gradient errors at 2^16", ["%.2e" % e for e in errs])
    assert max(errs) < 1e-4


def test_paper_adam_steps_match_oracle(fab, pkg, orc, torch):
    mats = fi.materials_for(3, 310)
    g = batch(3, 40, 31, 311)
    tg = fi.random_targets(g.n, 312)
    params, z = prepare(fab, pkg, torch, mats, 313)
    theta = np.concatenate([params, z.ravel()]).astype(np.float32)
    m = np.zeros(theta.size)
    v = np.zeros(theta.size)
    dg, dt = pkg.DeviceGBuffer.from_host(g), torch.from_numpy(tg).cuda()
    for t in (1, 2):
        _, og, odl = orc.paper_loss_grad(theta[:N].astype(np.float64),
                                         theta[N:].reshape(3, 64).astype(np.float64), mats, g, tg)
        full = np.concatenate([og, odl.ravel()])
        orc.adam_step(theta, full, m, v, t, 1e-3)
        pkg.fabric_paper_train_step(fab.ctx, dg, dt, {"lr": 1e-3})
        gp, gz = pkg.fabric_paper_get_params(fab.ctx, 3)
        got = np.concatenate([gp, gz.ravel()])
        solid = np.abs(full) > 1e-5
        assert np.abs(got[solid] - theta[solid]).max() < 2e-6 * t
        assert np.abs(got - theta).max() <= 2.1e-3 * t


def test_paper_training_lowers_loss_and_shades(fab, pkg, orc, torch):
    mats = fi.materials_for(8, 320)
    prepare(fab, pkg, torch, mats, 321)
    cfg = dict(batch=1 << 13, gt_samples=16, lr=3e-3)
    first = pkg.fabric_paper_train_step(fab.ctx, None, None, dict(cfg, seed=1))
    for s in range(2, 80):
        pkg.fabric_paper_train_step(fab.ctx, None, None, dict(cfg, seed=s), want_loss=False)
    last = np.mean([pkg.fabric_paper_train_step(fab.ctx, None, None, dict(cfg, seed=100 + s))
                    for s in range(5)])
    print("paper training loss", first, last)
    assert last < 0.5 * first
    # The shading image is re-packed from the trained masters.
    gp, gz = pkg.fabric_paper_get_params(fab.ctx, 8)
    g = batch(8, 48, 40, 322)
    out = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
    pkg.fabric_paper_shade(fab.ctx, pkg.DeviceGBuffer.from_host(g), out, "fp16")
    _, orgb = orc.paper_decoder_gbuffer(gp, gz, mats, g)
    err = rel_norm_err(out.cpu().numpy(), orgb)
    print("trained paper decoder fp16 vs oracle", err)
    assert err < 2e-2


def test_unencoded_footprint_shading_and_gradient(fab, pkg, orc, torch):
    """The footprint encoding's ablation: shading (FP16) and the loss
    gradient without the one-blob encoding against the oracle's, and the
    switch back to the encoding."""
    mats = fi.materials_for(4, 340)
    g = batch(4, 45, 37, 341)
    tg = fi.random_targets(g.n, 342)
    params, z = prepare(fab, pkg, torch, mats, 343)
    d = pkg.DeviceGBuffer.from_host(g)
    out = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
    pkg.fabric_paper_set_footprint_encoding(fab.ctx, False)
    pkg.fabric_paper_shade(fab.ctx, d, out, "fp16")
    _, o_raw = orc.paper_decoder_gbuffer(params, z, mats, g, raw=True)
    _, o_blob = orc.paper_decoder_gbuffer(params, z, mats, g)
    err_raw = rel_norm_err(out.cpu().numpy(), o_raw)
    print("unencoded fp16 vs oracle", err_raw, "encodings differ by", rel_norm_err(o_raw, o_blob))
    assert err_raw < 2e-2 and rel_norm_err(o_raw, o_blob) > 0.1
    grad = torch.empty(N + 4 * 64, device="cuda")
    loss = pkg.fabric_paper_loss_grad(fab.ctx, d, torch.from_numpy(tg).cuda(), {}, grad)
    oloss, ograd, odlat = orc.paper_loss_grad(params, z, mats, g, tg, raw=True)
    assert loss == pytest.approx(oloss, rel=1e-5)
    assert max(per_tensor_errors(grad.cpu().numpy(), np.concatenate([ograd, odlat.ravel()]), 4)) < 1e-4
    pkg.fabric_paper_set_footprint_encoding(fab.ctx, True)
    pkg.fabric_paper_shade(fab.ctx, d, out, "fp16")
    assert rel_norm_err(out.cpu().numpy(), o_blob) < 2e-2
    c = pkg._abi.lib().fabric_paper_set_footprint_encoding(fab.ctx, 2)
    assert c == 1                                     # E_INVAL


def test_unfused_shading_and_gradient(fab, pkg, orc, torch):
    """The spatial-fusion ablation: shading (FP16) and the loss gradient of
    the network whose angular inputs enter the first layer, against the
    oracle's, and the switch back to the paper's wiring."""
    mats = fi.materials_for(4, 350)
    g = batch(4, 45, 37, 351)
    tg = fi.random_targets(g.n, 352)
    params, z = prepare(fab, pkg, torch, mats, 353)
    d = pkg.DeviceGBuffer.from_host(g)
    out = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
    pkg.fabric_paper_set_spatial_fusion(fab.ctx, False)
    pkg.fabric_paper_shade(fab.ctx, d, out, "fp16")
    _, o_nf = orc.paper_decoder_gbuffer(params, z, mats, g, fused=False)
    _, o_f = orc.paper_decoder_gbuffer(params, z, mats, g)
    err = rel_norm_err(out.cpu().numpy(), o_nf)
    print("unfused fp16 vs oracle", err, "wirings differ by", rel_norm_err(o_nf, o_f))
    assert err < 2e-2 and rel_norm_err(o_nf, o_f) > 0.1
    grad = torch.empty(N + 4 * 64, device="cuda")
    loss = pkg.fabric_paper_loss_grad(fab.ctx, d, torch.from_numpy(tg).cuda(), {}, grad)
    oloss, ograd, odlat = orc.paper_loss_grad(params, z, mats, g, tg, fused=False)
    assert loss == pytest.approx(oloss, rel=1e-5)
    errs = per_tensor_errors(grad.cpu().numpy(), np.concatenate([ograd, odlat.ravel()]), 4)
    print("unfused gradient errors", ["%.2e" % e for e in errs])
    assert max(errs) < 1e-4
    pkg.fabric_paper_set_spatial_fusion(fab.ctx, True)
    pkg.fabric_paper_shade(fab.ctx, d, out, "fp16")
    assert rel_norm_err(out.cpu().numpy(), o_f) < 2e-2
    assert pkg._abi.lib().fabric_paper_set_spatial_fusion(fab.ctx, 2, None) == 1     # E_INVAL


def test_paper_training_deterministic_and_follows_visibility(fab, pkg, torch):
    """Fixed-order reductions: the same steps from the same masters give
    bitwise the same parameters; generated targets follow the context's
    visibility setting (a different loss with V, the same again without)."""
    mats = fi.materials_for(4, 360)
    cfg = dict(batch=4096, gt_samples=16, lr=1e-3)
    runs = []
    for _ in range(2):
        prepare(fab, pkg, torch, mats, 361)
        for s in range(3):
            pkg.fabric_paper_train_step(fab.ctx, None, None, dict(cfg, seed=10 + s), want_loss=False)
        runs.append(pkg.fabric_paper_get_params(fab.ctx, 4))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
    grad = torch.empty(N + 4 * 64, device="cuda")
    l0 = pkg.fabric_paper_loss_grad(fab.ctx, None, None, dict(cfg, seed=20), grad)
    fab.set_visibility(True)
    l1 = pkg.fabric_paper_loss_grad(fab.ctx, None, None, dict(cfg, seed=20), grad)
    fab.set_visibility(False)
    l2 = pkg.fabric_paper_loss_grad(fab.ctx, None, None, dict(cfg, seed=20), grad)
    print("paper loss without / with visibility", l0, l1)
    assert l1 != l0 and l2 == l0


def test_paper_training_errors(fab, pkg, torch):
    mats = fi.materials_for(2, 330)
    fab.encode(mats)
    with pytest.raises(pkg.FabricError) as e:
        pkg.fabric_paper_train_step(fab.ctx, None, None, dict(batch=256, gt_samples=4))
    assert e.value.status == 6                        # E_STATE: no prepare yet
    prepare(fab, pkg, torch, mats, 331)
    for prec in (pkg.FABRIC_FP16, pkg.FABRIC_FP8_E4M3):
        c = pkg._train_cfg(dict(batch=256, gt_samples=4, prec=prec))
        st = pkg._abi.lib().fabric_paper_train_step(fab.ctx, None, None, pkg.ctypes.byref(c), None, None)
        assert st == 1                                # E_INVAL: FP32 or BF16 only
    pkg.fabric_paper_train_step(fab.ctx, None, None, dict(batch=256, gt_samples=4))
    fab.encode(mats)
    with pytest.raises(pkg.FabricError) as e:
        pkg.fabric_paper_train_step(fab.ctx, None, None, dict(batch=256, gt_samples=4))
    assert e.value.status == 6                        # E_STATE: table re-encoded
    many = fi.materials_for(65, 332)
    prepare(fab, pkg, torch, many, 333)
    with pytest.raises(pkg.FabricError) as e:
        pkg.fabric_paper_train_step(fab.ctx, None, None, dict(batch=256, gt_samples=4))
    assert e.value.status == 2                        # E_RANGE: more than 64 fabrics
