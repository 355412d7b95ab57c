"""Pins of the oracle's encoder for the paper-size network (Sec. 4.2
"Encoder": a residual block of two fully connected layers of 128 before the
latent of 64; inputs: the one-hot weave grid and the 12 yarn scalars, as the
config-size encoder takes them): its wiring through hand-built weights, a
numpy float64 chain, the latent-32 case equal to the config encoder, and
the backward pass against central differences of the paper-size decoder's
loss with the encoder's latents."""
import math

import numpy as np
import pytest

import fabric_inputs as fi
import oracle as orc

LAT = 64


def slices(shapes, off=0):
    out = {}
    for k, (o, i) in enumerate(shapes):
        out[f"E{k + 1}"] = slice(off, off + o * i)
        off += o * i
        out[f"c{k + 1}"] = slice(off, off + o)
        off += o
    return out


def test_counts():
    assert orc.encoder_param_count(64) == fi.N_PAPER_ENCODER_PARAMS == 108480
    assert orc.encoder_param_count(32) == fi.N_ENCODER_PARAMS


def test_wiring_with_hand_built_weights():
    """e1 picks a cell and a scalar; the residual branch adds before the last
    ReLU; outputs 32..63 are wired (the rows beyond the config latent)."""
    sl = slices(fi.PAPER_ENCODER_SHAPES)
    Q = np.zeros(fi.N_PAPER_ENCODER_PARAMS)
    E1 = np.zeros((128, 524)); E1[0, 0] = 1.0; E1[1, 513] = 1.0    # cell (0,0) warp; weft roughness
    c1 = np.zeros(128); c1[2] = 0.75
    c3 = np.zeros(128); c3[2] = -0.5                                # relu(0.75 - 0.5)
    E2 = np.zeros((128, 128)); E3 = np.zeros((128, 128))
    E2[3, 0] = 2.0; E3[3, 3] = 3.0                                  # 3 relu(2 e1[0])
    E4 = np.zeros((64, 128)); c4 = np.zeros(64)
    E4[63, 0] = 1.0; E4[40, 1] = -2.0; E4[32, 2] = 1.0; E4[33, 3] = 1.0
    c4[50] = 0.125
    for name, arr in (("E1", E1), ("c1", c1), ("E2", E2), ("E3", E3), ("c3", c3), ("E4", E4),
                      ("c4", c4)):
        Q[sl[name]] = arr.ravel()
    m = fi.uniform_material(fi.pattern_plain(), alpha=0.55)      # weft roughness scales to 0.5
    z = orc.encoder(Q, [m], lat=LAT)[0]
    want = np.zeros(64)
    want[[63, 40, 32, 33, 50]] = [1.0, -1.0, 0.25, 6.0, 0.125]
    assert z == pytest.approx(want, abs=1e-7)     # the scalar is float32 0.55


def test_against_numpy_chain():
    Q = fi.init_paper_encoder_params(71, bias_scale=0.1).astype(np.float64)
    mats = fi.materials_for(8, 72)
    z = orc.encoder(Q, mats, lat=LAT)
    sl = slices(fi.PAPER_ENCODER_SHAPES)
    W = {k: Q[v] for k, v in sl.items()}
    for f, m in enumerate(mats):
        x = orc.encoder_input(m)
        e1 = np.maximum(W["E1"].reshape(128, 524) @ x + W["c1"], 0)
        r2 = np.maximum(W["E2"].reshape(128, 128) @ e1 + W["c2"], 0)
        e2 = np.maximum(e1 + W["E3"].reshape(128, 128) @ r2 + W["c3"], 0)
        ref = W["E4"].reshape(64, 128) @ e2 + W["c4"]
        np.testing.assert_allclose(z[f], ref, rtol=1e-12, atol=1e-12)


def test_latent_32_is_the_config_encoder():
    params = fi.init_params(73, bias_scale=0.1).astype(np.float64)
    Q = params[fi.N_DECODER_PARAMS:]
    mats = fi.materials_for(4, 74)
    np.testing.assert_array_equal(orc.encoder(Q, mats, lat=32), orc.encoder(Q, mats))


@pytest.mark.slow
def test_backward_matches_central_differences():
    """d loss / d encoder parameter, the paper-size decoder's loss with the
    encoder's latents: the oracle's backward (decoder backward to the
    latents, then through the encoder) against central differences."""
    mats = fi.materials_for(3, 75)
    g = fi.make_gbuffer(6, 4, 3, seed=76)
    g.fabric_id[:] = np.arange(g.n) % 3
    tg = fi.random_targets(g.n, 77)
    P = fi.init_paper_params(78, bias_scale=0.05).astype(np.float64)
    Q = fi.init_paper_encoder_params(79, bias_scale=0.05).astype(np.float64)

    def loss_of(q):
        return orc.paper_loss_grad(P, orc.encoder(q, mats, lat=LAT), mats, g, tg)[0]

    _, _, dlat = orc.paper_loss_grad(P, orc.encoder(Q, mats, lat=LAT), mats, g, tg)
    grad = orc.encoder_backward(Q, mats, dlat, lat=LAT)
    sl = slices(fi.PAPER_ENCODER_SHAPES)
    picked = 0
    for name, s_ in sl.items():
        idx = np.arange(s_.start, s_.stop)
        for e in idx[np.argsort(-np.abs(grad[idx]))[:3]]:
            h = 1e-6
            qp, qm = Q.copy(), Q.copy()
            qp[e] += h
            qm[e] -= h
            fd = (loss_of(qp) - loss_of(qm)) / (2 * h)
            assert abs(fd - grad[e]) <= 1e-6 * max(1.0, np.abs(grad).max()), (name, e, fd, grad[e])
            picked += 1
    assert picked == 24
