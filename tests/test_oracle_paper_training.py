"""Pins of the oracle's loss gradient for the paper-size decoder (Sec. 4.2
"Decoder", loss of Eq. (9)-(11)) with per-fabric latents as parameters:
central differences of the oracle's own loss in FP64 for entries of every
layer, bias and latent; the loss against the forward outputs; faulted
samples contribute nothing; latents of fabrics absent from the batch get no
gradient."""
import dataclasses

import numpy as np
import pytest

import fabric_inputs as fi
import oracle as orc

SH = fi.PAPER_DECODER_SHAPES


def case(n=24, n_fab=3, seed=5, btdf_frac=0.3):
    mats = fi.materials_for(n_fab, seed)
    g = fi.make_gbuffer(n, 1, n_fab, seed=seed + 1, btdf_frac=btdf_frac)
    g.fabric_id[:] = np.random.default_rng(seed).integers(0, n_fab, g.n).astype(np.uint16)
    # FP64 copies, so that a perturbation of 1e-6 is not rounded away.
    P = fi.init_paper_params(seed + 2, bias_scale=0.1).astype(np.float64)
    Z = fi.random_latents(n_fab, seed + 3, dim=64).astype(np.float64)
    rng = np.random.default_rng(seed + 4)
    T = np.abs(rng.normal(0.0, 0.3, (4, g.n))).astype(np.float32)
    return mats, g, P, Z, T


def layer_offsets():
    out, off = [], 0
    for o, i in SH:
        out.append((off, o, i))
        off += o * i + o
    return out


@pytest.mark.parametrize("raw,fused", [(False, True), (True, True), (False, False)])
def test_gradient_matches_central_differences(raw, fused):
    mats, g, P, Z, T = case()
    kw = dict(raw=raw, fused=fused)
    loss, grad, dlat = orc.paper_loss_grad(P, Z, mats, g, T, **kw)
    assert np.isfinite(loss) and loss > 0
    rng = np.random.default_rng(11)
    idx = []
    for off, o, i in layer_offsets():
        idx += list(off + rng.integers(0, o * i, 6))           # weights
        idx += list(off + o * i + rng.integers(0, o, 2))        # biases
    a1 = layer_offsets()[2][0]
    idx += [a1 + 5 * 69 + 64, a1 + 17 * 69 + 66, a1 + 40 * 69 + 68]   # A1's angular columns
    h = 1e-6
    for k in idx:
        Pp, Pm = P.copy(), P.copy()
        Pp[k] += h
        Pm[k] -= h
        fd = (orc.paper_loss_grad(Pp, Z, mats, g, T, **kw)[0] -
              orc.paper_loss_grad(Pm, Z, mats, g, T, **kw)[0]) / (2 * h)
        assert abs(fd - grad[k]) <= 1e-6 * max(1.0, abs(grad).max()), (k, fd, grad[k])
    for f, j in [(0, 0), (1, 17), (2, 63), (1, 40)]:
        Zp, Zm = Z.copy(), Z.copy()
        Zp[f, j] += h
        Zm[f, j] -= h
        fd = (orc.paper_loss_grad(P, Zp, mats, g, T, **kw)[0] -
              orc.paper_loss_grad(P, Zm, mats, g, T, **kw)[0]) / (2 * h)
        assert abs(fd - dlat[f, j]) <= 1e-6 * max(1.0, abs(dlat).max()), (f, j, fd, dlat[f, j])


def test_loss_against_forward_outputs():
    mats, g, P, Z, T = case(n=40, btdf_frac=0.5)
    loss, _, _ = orc.paper_loss_grad(P, Z, mats, g, T)
    y, _ = orc.paper_decoder_gbuffer(P, Z, mats, g)
    k = np.where(g.wi_z < 0, 1000.0, 100.0)
    T = T.astype(np.float64)
    ref = (0.1 * ((y[:2] - T[:2]) ** 2).sum() + 0.4 * ((y[2:] - np.log(k * T[2:] + 1.0)) ** 2).sum()) / g.n
    assert abs(loss - ref) <= 1e-12 * ref


def test_faulted_samples_and_absent_fabrics():
    mats, g, P, Z, T = case(n=30, n_fab=4)
    g.fabric_id[:] = np.where(g.fabric_id == 3, 0, g.fabric_id).astype(np.uint16)   # fabric 3 absent
    loss, grad, dlat = orc.paper_loss_grad(P, Z, mats, g, T)
    assert np.all(dlat[3] == 0.0) and np.abs(dlat[:3]).max() > 0
    # A faulted sample (wo below the surface) changes nothing but the 1/n.
    g2 = fi.GBuffer(**{f.name: np.concatenate([getattr(g, f.name), getattr(g, f.name)[:1]])
                       for f in dataclasses.fields(fi.GBuffer)})
    g2.wo_z[-1] = -0.5
    T2 = np.concatenate([T, T[:, :1]], axis=1)
    loss2, grad2, _ = orc.paper_loss_grad(P, Z, mats, g2, T2)
    assert abs(loss2 * (g.n + 1) - loss * g.n) <= 1e-12 * loss * g.n
    np.testing.assert_allclose(grad2 * (g.n + 1), grad * g.n, rtol=1e-10, atol=1e-14)


def test_raw_footprint_inputs():
    """Without the encoding (the ablation of Sec. 5 "Encoding of
    footprint") the inputs are p_u = (u mod W_x) / W_x, p_v likewise and
    tau = clamp((log2 r + 14) / 16, 0, 1), in the channels of their first
    one-blob bin; every other channel is 0."""
    for (u, v, r, wx, wy), (pu, pv, tau) in [((2.5, -1.25, 0.25, 4, 3), (0.625, 1.75 / 3, 0.75)),
                                             ((7.0, 3.0, 2.0 ** -20, 2, 3), (0.5, 0.0, 0.0)),
                                             ((0.0, 0.5, 8.0, 5, 1), (0.0, 0.5, 1.0))]:
        f = orc.paper_features(u, v, r, wx, wy, raw=True)
        assert f[0] == pytest.approx(pu, abs=1e-15) and f[8] == pytest.approx(pv, abs=1e-15)
        assert f[16] == pytest.approx(tau, abs=1e-15)
        assert np.count_nonzero(np.delete(f, [0, 8, 16])) == 0
    # The network sees exactly these inputs: with weights that pass F1's
    # neuron 0 (reading channel 16) through F2, A1, the residual skip, A4
    # and A5 unchanged, the first output is tau.
    mats, g, P, Z, _ = case(n=6, n_fab=1)
    P = np.zeros_like(P)
    (f1, _, i1), (f2, _, i2), (a1, _, ia1), _, _, (a4, _, i4), (a5, _, _) = layer_offsets()
    P[f1 + 64 + 16] = 1.0                 # WF1[0][z(64) + channel 16]
    P[f2] = P[a1] = P[a4] = P[a5] = 1.0   # WF2[0][0], WA1[0][0], WA4[0][0], WA5[0][0]
    y, _ = orc.paper_decoder_gbuffer(P, Z, mats, g, raw=True)
    tau = np.clip((np.log2(g.radius.astype(np.float64)) + 14.0) / 16.0, 0.0, 1.0)
    np.testing.assert_allclose(y[0], tau, rtol=0, atol=1e-15)


def test_angular_inputs_enter_first_layer_without_fusion():
    """Without the spatial fusion stage (the ablation of Sec. 5 "Spatial
    fusion") wi and wo enter the first layer through A1's angular columns
    and A1 sees zeros in their place.  With WA1[0][wi.z] = 1, F2[0][0] = -1
    and pass-through weights elsewhere, the paper's network outputs wi.z
    (A1 adds it after the spatial feature, which is 0), the unfused one
    outputs -1e-8 wi.z (wi.z passes the first layer, is negated by F2 and
    then takes four leaky slopes)."""
    mats, g, P, Z, _ = case(n=8, n_fab=1, btdf_frac=0.0)
    P = np.zeros_like(P)
    (f1, _, _), (f2, _, _), (a1, _, _), _, _, (a4, _, _), (a5, _, _) = layer_offsets()
    P[a1 + 64 + 2] = 1.0                  # WA1[0][wi.z]
    P[f2] = -1.0                          # WF2[0][0]
    P[a1] = P[a4] = P[a5] = 1.0           # WA1[0][0], WA4[0][0], WA5[0][0]
    wz = g.wi_z.astype(np.float64)
    y_f, _ = orc.paper_decoder_gbuffer(P, Z, mats, g)
    y_n, _ = orc.paper_decoder_gbuffer(P, Z, mats, g, fused=False)
    np.testing.assert_allclose(y_f[0], wz, rtol=1e-15, atol=0)
    np.testing.assert_allclose(y_n[0], -1e-8 * wz, rtol=1e-12, atol=0)
