"""GPU parity of the paper-size decoder's training with BF16 operands on the
matrix cores (Sec. 4.2 "Decoder", loss of Eq. (9)-(11)) through the C ABI,
against the oracle's FP64 loss and backward.

The bars follow from the arithmetic.  Every layer rounds its two operands
(weights, activations or gradients) to BF16, whose unit roundoff is
u = 2^-8, and accumulates in FP32.  A rounded product carries a relative
error of at most 2u with zero mean, so a layer's output vector picks up a
relative norm error of about u sqrt(2/3) ~ 3.2e-3 when its terms do not
cancel.  Six forward and six transposed layers stacked in quadrature give
about sqrt(12) x 3.2e-3 ~ 1.1e-2 on a delta plane, and a weight gradient
(activation times delta, summed over the batch) carries both sides' error;
the per-tensor bar is 4e-2, about three times that estimate, and the
whole-gradient bar 2e-2.  The loss is a sum of squared residuals whose
output error is the forward's, ~ sqrt(6) x 3.2e-3 relative on the
network's output: the loss bar is 1e-2 relative.  Faulted samples
contribute exactly nothing, as in FP32."""
import numpy as np
import pytest

import fabric_inputs as fi
from tests.helpers import rel_norm_err, require_gpu

pytestmark = pytest.mark.gpu

N = fi.N_PAPER_DECODER_PARAMS
TENSOR_BAR = 4e-2
WHOLE_BAR = 2e-2
LOSS_BAR = 1e-2


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def pkg(torch):
    import paper_2406_17782_amd as pkg
    return pkg


@pytest.fixture()
def fab(pkg):
    f = pkg.Fabric(0, seed=72)
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


def check(pkg, fab, torch, orc, params, z, mats, g, tg, label, **variant):
    n_fab = len(mats)
    grad = torch.empty(N + n_fab * 64, device="cuda")
    loss = pkg.fabric_paper_loss_grad(fab.ctx, pkg.DeviceGBuffer.from_host(g),
                                      torch.from_numpy(tg).cuda(), {"prec": pkg.FABRIC_BF16}, grad)
    oloss, ograd, odlat = orc.paper_loss_grad(params, z, mats, g, tg, **variant)
    got = grad.cpu().numpy()
    ref = np.concatenate([ograd, odlat.ravel()])
    errs = per_tensor_errors(got, ref, n_fab)
    whole = rel_norm_err(got, ref)
    print(label, "loss", loss, oloss, "whole", "%.2e" % whole, "per tensor",
          ["%.2e" % e for e in errs])
    assert loss == pytest.approx(oloss, rel=LOSS_BAR)
    assert whole < WHOLE_BAR
    assert max(errs) < TENSOR_BAR
    return loss, got


def test_bf16_loss_grad_matches_oracle(fab, pkg, orc, torch):
    mats = fi.materials_for(5, 300)
    g = batch(5, 61, 53, 301)            # 3,233 samples: a ragged last wave and block
    g.wo_z[5] = -0.3                     # faulted samples contribute nothing
    g.radius[9] = 0.0
    tg = fi.random_targets(g.n, 302)
    params, z = prepare(fab, pkg, torch, mats, 303)
    check(pkg, fab, torch, orc, params, z, mats, g, tg, "bf16 3233")


def test_bf16_faulted_samples_change_nothing(fab, pkg, torch):
    """Faulted samples contribute nothing, whatever their fields and
    targets: two batches that differ only there (different faults, NaN
    targets in one) give bitwise the same loss and gradient."""
    mats = fi.materials_for(3, 305)
    a = batch(3, 33, 9, 306)             # 297 samples
    a.wo_z[[4, 100, 250]] = -0.5
    b = a.subset(np.arange(a.n))
    b.radius[4] = 0.0
    b.u[100] = np.nan
    b.wi_x[250] = 7.0
    ta = fi.random_targets(a.n, 307)
    tb = ta.copy()
    tb[:, [4, 100, 250]] = np.nan
    prepare(fab, pkg, torch, mats, 308)
    cfg = {"prec": pkg.FABRIC_BF16}
    out = []
    for g, tg in ((a, ta), (b, tb)):
        grad = torch.empty(N + 3 * 64, device="cuda")
        loss = pkg.fabric_paper_loss_grad(fab.ctx, pkg.DeviceGBuffer.from_host(g),
                                          torch.from_numpy(tg).cuda(), cfg, grad)
        out.append((loss, grad.cpu().numpy()))
    assert np.isfinite(out[0][0]) and out[0][0] == out[1][0]
    assert np.array_equal(out[0][1], out[1][1])


def test_bf16_loss_grad_full_batch_2p16(fab, pkg, orc, torch):
    """The benchmark's training batch: 2^16 samples of the 1080p workload's
    8 fabrics, against the oracle over every sample."""
    wl = fi.WORKLOADS["train_2p20"]
    mats = wl.materials()
    g = wl.gbuffer().subset(np.arange(1 << 16))
    g.fabric_id[:] = np.random.default_rng(74).integers(0, 8, g.n).astype(np.uint16)
    tg = fi.random_targets(g.n, 75)
    params, z = prepare(fab, pkg, torch, mats, 76)
    check(pkg, fab, torch, orc, params, z, mats, g, tg, "bf16 2^16")


@pytest.mark.parametrize("variant", ["raw", "unfused"])
def test_bf16_ablations(fab, pkg, orc, torch, variant):
    """Without the one-blob footprint encoding, and without the spatial
    fusion stage: the same bars."""
    mats = fi.materials_for(4, 340)
    g = batch(4, 45, 37, 341)
    tg = fi.random_targets(g.n, 342)
    params, z = prepare(fab, pkg, torch, mats, 343)
    if variant == "raw":
        pkg.fabric_paper_set_footprint_encoding(fab.ctx, False)
        check(pkg, fab, torch, orc, params, z, mats, g, tg, "bf16 raw", raw=True)
    else:
        pkg.fabric_paper_set_spatial_fusion(fab.ctx, False)
        check(pkg, fab, torch, orc, params, z, mats, g, tg, "bf16 unfused", fused=False)


def test_bf16_training_lowers_loss_and_tracks_fp32(fab, pkg, orc, torch):
    """BF16 training on generated batches lowers the loss as FP32 training
    does, and the trained decoder's BF16 shading matches the oracle's
    forward of its masters at the BF16 shading bound."""
    mats = fi.materials_for(8, 320)
    cfg = dict(batch=1 << 13, gt_samples=16, lr=3e-3)
    finals = {}
    for prec in (pkg.FABRIC_FP32, pkg.FABRIC_BF16):
        prepare(fab, pkg, torch, mats, 321)
        c = dict(cfg, prec=prec)
        first = pkg.fabric_paper_train_step(fab.ctx, None, None, dict(c, seed=1))
        for s in range(2, 80):
            pkg.fabric_paper_train_step(fab.ctx, None, None, dict(c, seed=s), want_loss=False)
        grad = torch.empty(N + 8 * 64, device="cuda")
        # the same held-out batches, each measured in FP32
        last = np.mean([pkg.fabric_paper_loss_grad(fab.ctx, None, None,
                                                   dict(cfg, seed=100 + s, prec=pkg.FABRIC_FP32), grad)
                        for s in range(5)])
        print("paper training loss, prec", prec, first, last)
        assert last < 0.5 * first
        finals[prec] = last
    # BF16 training ends within 10 % of FP32 training's held-out loss
    assert finals[pkg.FABRIC_BF16] < 1.1 * finals[pkg.FABRIC_FP32]
    gp, gz = pkg.fabric_paper_get_params(fab.ctx, 8)
    g = batch(8, 48, 40, 322)
    out = torch.empty((3, g.n), dtype=torch.float32, device="cuda")
    pkg.fabric_paper_shade(fab.ctx, pkg.DeviceGBuffer.from_host(g), out, "bf16")
    _, orgb = orc.paper_decoder_gbuffer(gp, gz, mats, g)
    err = rel_norm_err(out.cpu().numpy(), orgb)
    print("bf16-trained paper decoder bf16 vs oracle", err)
    # the BF16 shading bound of the paper-size decoder's own parity tests
    # (operand roundoff over seven layers and the specular decoding's e^y)
    assert err < 6e-2


def test_bf16_training_deterministic(fab, pkg, torch):
    mats = fi.materials_for(4, 360)
    cfg = dict(batch=4096, gt_samples=16, lr=1e-3, prec=pkg.FABRIC_BF16)
    runs = []
    for _ in range(2):
        prepare(fab, pkg, torch, mats, 361)
        for s in range(3):
            pkg.fabric_paper_train_step(fab.ctx, None, None, dict(cfg, seed=10 + s), want_loss=False)
        runs.append(pkg.fabric_paper_get_params(fab.ctx, 4))
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][1], runs[1][1])
