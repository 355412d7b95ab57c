"""torch.autograd.Function wrappers of the hand-written decoder and encoder
kernels (forward and backward both run in libfabric.so)."""
from __future__ import annotations

import torch

from . import (FABRIC_FP32, FABRIC_N_DECODER_PARAMS, DeviceGBuffer, fabric_decoder_backward,
               fabric_decoder_forward, fabric_encoder_backward, fabric_encoder_forward)


class DecoderFunction(torch.autograd.Function):
    """y4 [4, n] = decoder(dec_params [13572], latents [F, 32]; G-buffer).

    The G-buffer and the context are non-differentiable arguments; gradients
    flow to the decoder parameters and the per-fabric latents."""

    @staticmethod
    def forward(ctx, dec_params, latents, fab, gbuf: DeviceGBuffer, prec: int = FABRIC_FP32):
        dec_params = dec_params.contiguous()
        latents = latents.contiguous()
        y4 = torch.empty((4, gbuf.n), dtype=torch.float32, device=dec_params.device)
        fabric_decoder_forward(fab.ctx, gbuf, prec, dec_params, latents, y4)
        ctx.save_for_backward(dec_params, latents)
        ctx.fab = fab
        ctx.gbuf = gbuf
        return y4

    @staticmethod
    def backward(ctx, grad_y4):
        dec_params, latents = ctx.saved_tensors
        gp = torch.empty(FABRIC_N_DECODER_PARAMS, dtype=torch.float32, device=dec_params.device)
        gl = torch.empty_like(latents)
        fabric_decoder_backward(ctx.fab.ctx, ctx.gbuf, dec_params, latents, grad_y4.contiguous(), gp, gl)
        return gp, gl, None, None, None


class EncoderFunction(torch.autograd.Function):
    """latents [F, 32] = encoder(enc_params [104352]) over the encoded fabric table."""

    @staticmethod
    def forward(ctx, enc_params, fab):
        enc_params = enc_params.contiguous()
        z = torch.empty((fab.n_mats, 32), dtype=torch.float32, device=enc_params.device)
        fabric_encoder_forward(fab.ctx, enc_params, z)
        ctx.save_for_backward(enc_params)
        ctx.fab = fab
        return z

    @staticmethod
    def backward(ctx, grad_z):
        (enc_params,) = ctx.saved_tensors
        g = torch.empty_like(enc_params)
        fabric_encoder_backward(ctx.fab.ctx, enc_params, grad_z.contiguous(), g)
        return g, None


def decoder(dec_params, latents, fab, gbuf, prec: int = FABRIC_FP32):
    return DecoderFunction.apply(dec_params, latents, fab, gbuf, prec)


def encoder(enc_params, fab):
    return EncoderFunction.apply(enc_params, fab)
