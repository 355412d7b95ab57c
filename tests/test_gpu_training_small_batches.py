"""BF16 training on batches too small to fill the kernels' blocks: the loss
and gradient of 1, 5, 37, 64, 65 and 200 samples (a lone sample, a part of
one 32-sample group, a group and a half, exactly one 64-sample region of
the BF16 planes, one sample past it, a ragged few regions) against the
oracle's FP64 backward, for the config-size network and the paper-size
network: the weight-gradient kernels' tails (groups cut short, blocks with
no samples) and the planes' last region read no stale values.  Bars: the
loss within the error that its outputs' BF16 error allows: with y of
relative error eps, |dloss| <= 2 sqrt(loss E) + E, E = mean over samples of
sum_c lambda_c (eps |y_c|)^2 (Cauchy-Schwarz on the residual times the
output error), eps = 3e-2, three times the ~6.4e-3 / 8.5e-3 that BF16
operands give over four / seven layers (u sqrt(2/3) per layer in
quadrature); a relative loss bar does not hold for a single sample, whose
residual may be far smaller than its output.  The gradient, a mean of
per-sample gradients g_s, errs by at most 4e-2 (the per-tensor bar of the
full-batch tests, whose derivation from BF16 roundoff through the chained
layers assumes no averaging over samples) times the mean of |g_s|: over a
few samples with random targets the g_s largely cancel, so the error is
bounded against their sizes, not against the norm of their mean (the
oracle gives each g_s as the gradient of a one-sample batch).  Each batch
follows a larger one, so the scratch holds another batch's values."""
import numpy as np
import pytest

import fabric_inputs as fi
from tests.helpers import rel_norm_err, require_gpu

pytestmark = pytest.mark.gpu

SIZES = (1, 5, 37, 64, 65, 200)
GRAD_BAR = 4e-2
EPS_Y = 3e-2
LAMBDA = np.array([0.1, 0.1, 0.4, 0.4])      # lambda_C, lambda_S of Eq. (11)


def loss_bound(y, oloss):
    """The largest loss error that outputs y [4][n] of relative error EPS_Y allow."""
    e = float(np.mean(np.sum(LAMBDA[:, None] * (EPS_Y * y) ** 2, axis=0)))
    return 2.0 * np.sqrt(oloss * e) + e


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def pkg(torch):
    import paper_2406_17782_amd as pkg
    return pkg


def small_batch(n_fab, n, seed):
    g = fi.make_gbuffer(n, 1, n_fab, seed=seed, btdf_frac=0.3)
    g.fabric_id[:] = np.random.default_rng(seed + 1).integers(0, n_fab, g.n).astype(np.uint16)
    return g, fi.random_targets(g.n, seed + 2)


@pytest.mark.parametrize("n", SIZES)
def test_config_network_bf16_small_batch(pkg, orc, torch, n):
    mats = fi.materials_for(4, 600)
    fab = pkg.Fabric(0, seed=601)
    try:
        params = fi.init_params(602, bias_scale=0.05)
        fab.set_params(params)
        fab.encode(mats)
        g, tg = small_batch(4, n, 603 + n)
        grad = torch.empty(fi.N_PARAMS, device="cuda")
        big, tb = small_batch(4, 3000, 604)
        pkg.fabric_loss_grad(fab.ctx, pkg.DeviceGBuffer.from_host(big), torch.from_numpy(tb).cuda(),
                             {"prec": pkg.FABRIC_BF16}, grad)
        loss = pkg.fabric_loss_grad(fab.ctx, pkg.DeviceGBuffer.from_host(g), torch.from_numpy(tg).cuda(),
                                    {"prec": pkg.FABRIC_BF16}, grad)
        oloss, ograd, _ = orc.loss_grad(params, mats, g, tg)
        dec, enc = params[:fi.N_DECODER_PARAMS], params[fi.N_DECODER_PARAMS:]
        y, _ = orc.decoder_gbuffer(dec, orc.encoder(enc, mats), mats, g)
        scale = np.mean([np.linalg.norm(orc.loss_grad(params, mats, g.subset([i]), tg[:, [i]])[1])
                         for i in range(n)])
        err = float(np.linalg.norm(grad.cpu().numpy() - ograd)) / scale
        bound = loss_bound(y, oloss)
        print(f"config n={n}: loss {loss:.6g} oracle {oloss:.6g} (bound {bound:.3g}); grad err "
              f"{err:.3g} of the mean per-sample gradient, {rel_norm_err(grad.cpu().numpy(), ograd):.3g} "
              "of the batch gradient")
        assert abs(loss - oloss) <= bound
        assert err < GRAD_BAR
    finally:
        fab.close()


@pytest.mark.parametrize("n", SIZES)
def test_paper_network_bf16_small_batch(pkg, orc, torch, n):
    mats = fi.materials_for(3, 610)
    fab = pkg.Fabric(0, seed=611)
    try:
        fab.encode(mats)
        params = fi.init_paper_params(612, bias_scale=0.05)
        z = fi.random_latents(3, 613, dim=64)
        pkg.fabric_paper_prepare(fab.ctx, torch.from_numpy(params).cuda(), torch.from_numpy(z).cuda())
        g, tg = small_batch(3, n, 614 + n)
        grad = torch.empty(fi.N_PAPER_DECODER_PARAMS + 3 * 64, device="cuda")
        big, tb = small_batch(3, 3000, 615)
        cfg = {"prec": pkg.FABRIC_BF16}
        pkg.fabric_paper_loss_grad(fab.ctx, pkg.DeviceGBuffer.from_host(big), torch.from_numpy(tb).cuda(),
                                   cfg, grad)
        loss = pkg.fabric_paper_loss_grad(fab.ctx, pkg.DeviceGBuffer.from_host(g),
                                          torch.from_numpy(tg).cuda(), cfg, grad)
        oloss, ograd, odlat = orc.paper_loss_grad(params, z, mats, g, tg)
        y, _ = orc.paper_decoder_gbuffer(params, z, mats, g)
        ref = np.concatenate([ograd, odlat.ravel()])

        def one(i):
            _, gi, di = orc.paper_loss_grad(params, z, mats, g.subset([i]), tg[:, [i]])
            return np.linalg.norm(np.concatenate([gi, di.ravel()]))
        scale = np.mean([one(i) for i in range(n)])
        err = float(np.linalg.norm(grad.cpu().numpy() - ref)) / scale
        bound = loss_bound(y, oloss)
        print(f"paper n={n}: loss {loss:.6g} oracle {oloss:.6g} (bound {bound:.3g}); grad err "
              f"{err:.3g} of the mean per-sample gradient, {rel_norm_err(grad.cpu().numpy(), ref):.3g} "
              "of the batch gradient")
        assert abs(loss - oloss) <= bound
        assert err < GRAD_BAR
    finally:
        fab.close()
