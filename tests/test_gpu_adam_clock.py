"""Adam's step count lives on the device with its moments: a step whose loss
is not finite (NaN targets) changes neither the parameters nor the count,
also when no loss is read back, so the steps around it land exactly where
the same steps without it do (bitwise), for the config-size network and the
paper-size network; the count survives a checkpoint round trip."""
import numpy as np
import pytest

import fabric_inputs as fi
from tests.helpers import require_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    return require_gpu()


@pytest.fixture(scope="module")
def pkg(torch):
    import paper_2406_17782_amd as pkg
    return pkg


def batch(pkg, torch, n_fab, seed):
    g = fi.make_gbuffer(40, 24, n_fab, seed=seed)
    g.fabric_id[:] = np.random.default_rng(seed + 1).integers(0, n_fab, g.n).astype(np.uint16)
    tg = fi.random_targets(g.n, seed + 2)
    bad = tg.copy()
    bad[0, 3] = np.nan
    return (pkg.DeviceGBuffer.from_host(g), torch.from_numpy(tg).cuda(),
            torch.from_numpy(bad).cuda())


def test_config_network_skipped_step_is_not_counted(pkg, torch):
    mats = fi.materials_for(3, 500)
    d, tg, bad = batch(pkg, torch, 3, 501)
    cfg = dict(lr=1e-3, prec=pkg.FABRIC_FP32)
    runs = []
    for with_bad in (False, True):
        fab = pkg.Fabric(0, seed=502)
        try:
            fab.encode(mats)
            pkg.fabric_train_step(fab.ctx, d, tg, cfg, want_loss=False)
            if with_bad:
                # no loss read back: the host cannot know the step was skipped
                pkg.fabric_train_step(fab.ctx, d, bad, cfg, want_loss=False)
                with pytest.raises(pkg.FabricError) as e:
                    pkg.fabric_train_step(fab.ctx, d, bad, cfg)
                assert e.value.status == 5                   # E_NONFINITE
            pkg.fabric_train_step(fab.ctx, d, tg, cfg, want_loss=False)
            runs.append(fab.params())
            if with_bad:
                # the checkpoint carries the count: two steps
                blob = pkg.fabric_save(fab.ctx)
                other = pkg.Fabric(0, seed=9)
                try:
                    pkg.fabric_load(other.ctx, blob)
                    other.encode(mats)
                    fab.encode(mats)
                    pkg.fabric_train_step(fab.ctx, d, tg, cfg, want_loss=False)
                    pkg.fabric_train_step(other.ctx, d, tg, cfg, want_loss=False)
                    assert np.array_equal(fab.params(), other.params())
                finally:
                    other.close()
        finally:
            fab.close()
    assert np.array_equal(runs[0], runs[1])


def test_paper_network_skipped_step_is_not_counted(pkg, torch):
    mats = fi.materials_for(3, 510)
    d, tg, bad = batch(pkg, torch, 3, 511)
    params = torch.from_numpy(fi.init_paper_params(512, bias_scale=0.05)).cuda()
    z = torch.from_numpy(fi.random_latents(3, 513, dim=64)).cuda()
    runs = []
    for with_bad in (False, True):
        fab = pkg.Fabric(0, seed=514)
        try:
            fab.encode(mats)
            pkg.fabric_paper_prepare(fab.ctx, params, z)
            pkg.fabric_paper_train_step(fab.ctx, d, tg, {"lr": 1e-3}, want_loss=False)
            if with_bad:
                pkg.fabric_paper_train_step(fab.ctx, d, bad, {"lr": 1e-3}, want_loss=False)
            pkg.fabric_paper_train_step(fab.ctx, d, tg, {"lr": 1e-3}, want_loss=False)
            gp, gz = pkg.fabric_paper_get_params(fab.ctx, 3)
            runs.append(np.concatenate([gp, gz.ravel()]))
        finally:
            fab.close()
    assert np.array_equal(runs[0], runs[1])
