"""MI355X (gfx950) woven-fabric shading: neural decoder and footprint-filtered
analytic model behind the C ABI of include/fabric.h.

Every step of the shading, filtering and training path runs in the HIP
library ``libfabric.so``; this package only marshals arguments.  PyTorch
supplies device memory and streams.  The functions named ``fabric_*`` mirror
the C entry points one to one; :class:`Fabric` bundles them around a context.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Sequence

import numpy as np

from . import _abi
from ._abi import (FABRIC_BF16, FABRIC_FP8_E4M3, FABRIC_FP16, FABRIC_FP32, FABRIC_LATENT,
                   FABRIC_MAX_FABRICS, FABRIC_MAX_SAMPLES, FABRIC_N_DECODER_PARAMS,
                   FABRIC_N_ENCODER_PARAMS, FABRIC_N_PAPER_DECODER_PARAMS,
                   FABRIC_N_PAPER_ENCODER_PARAMS, FABRIC_N_PARAMS,
                   FABRIC_PAPER_LATENT, PREC, FabricError, check)

__all__ = [
    "Fabric", "DeviceGBuffer", "FabricError", "PREC", "FABRIC_FP32", "FABRIC_BF16", "FABRIC_FP16",
    "FABRIC_FP8_E4M3", "FABRIC_N_PARAMS", "FABRIC_N_DECODER_PARAMS", "FABRIC_N_ENCODER_PARAMS",
    "FABRIC_MAX_FABRICS", "FABRIC_MAX_SAMPLES", "FABRIC_LATENT",
    "fabric_create", "fabric_destroy", "fabric_encode", "fabric_set_albedo", "fabric_lerp_latents",
    "fabric_set_visibility", "fabric_paper_prepare", "fabric_paper_shade", "fabric_paper_forward",
    "fabric_paper_prepare_encoder", "fabric_paper_encode", "fabric_paper_get_encoder",
    "FABRIC_N_PAPER_ENCODER_PARAMS",
    "fabric_paper_train_step", "fabric_paper_loss_grad", "fabric_paper_get_params",
    "fabric_paper_set_footprint_encoding", "fabric_paper_set_spatial_fusion", "FABRIC_PAPER_LATENT", "FABRIC_N_PAPER_DECODER_PARAMS",
    "fabric_shade_gbuffer", "fabric_shade_gbuffer_noalloc", "fabric_gt_filtered",
    "fabric_decoder_forward", "fabric_decoder_backward", "fabric_encoder_forward", "fabric_encoder_backward",
    "fabric_make_batch", "fabric_loss_grad", "fabric_train_step", "fabric_get_params", "fabric_set_params",
    "fabric_get_latents", "fabric_save", "fabric_load", "fabric_error_count",
]

GBUF_FIELDS = ("u", "v", "radius", "wi_x", "wi_y", "wi_z", "wo_x", "wo_y", "wo_z")


def _torch():
    import torch
    return torch


def _stream(stream) -> Optional[int]:
    """A HIP stream handle: torch's current stream for None, a torch stream's
    handle, or an integer handle as given."""
    if stream is None:
        torch = _torch()
        return torch.cuda.current_stream().cuda_stream
    return int(getattr(stream, "cuda_stream", stream))


def _dptr(t) -> int:
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return t.data_ptr()


@dataclasses.dataclass
class DeviceGBuffer:
    """A G-buffer as device tensors (structure of arrays)."""
    fabric_id: "object"   # torch.uint16 [n]
    u: "object"
    v: "object"
    radius: "object"
    wi_x: "object"
    wi_y: "object"
    wi_z: "object"
    wo_x: "object"
    wo_y: "object"
    wo_z: "object"

    @property
    def n(self) -> int:
        return int(self.u.shape[0])

    @classmethod
    def from_host(cls, g, device="cuda") -> "DeviceGBuffer":
        """Copy a host G-buffer (numpy arrays with the same field names)."""
        torch = _torch()
        fid = torch.from_numpy(np.ascontiguousarray(g.fabric_id, dtype=np.uint16).view(np.int16))
        fid = fid.to(device).view(torch.uint16)
        kw = {f: torch.from_numpy(np.ascontiguousarray(getattr(g, f), dtype=np.float32)).to(device)
              for f in GBUF_FIELDS}
        return cls(fabric_id=fid, **kw)

    @classmethod
    def empty(cls, n: int, device="cuda") -> "DeviceGBuffer":
        torch = _torch()
        kw = {f: torch.empty(n, dtype=torch.float32, device=device) for f in GBUF_FIELDS}
        return cls(fabric_id=torch.empty(n, dtype=torch.uint16, device=device), **kw)

    def subset(self, idx) -> "DeviceGBuffer":
        return DeviceGBuffer(**{f.name: getattr(self, f.name)[idx].contiguous()
                                for f in dataclasses.fields(self)})

    def c_struct(self, cls=_abi.fabric_gbuffer):
        return cls(self.n, _dptr(self.fabric_id), *[_dptr(getattr(self, f)) for f in GBUF_FIELDS])


def _material_struct(m) -> _abi.fabric_material:
    s = _abi.fabric_material()
    pat = np.ascontiguousarray(m.pattern, dtype=np.uint8)
    s.wy, s.wx = int(pat.shape[0]), int(pat.shape[1])
    flat = pat.reshape(-1)
    ctypes.memmove(ctypes.addressof(s.pattern), flat.ctypes.data, flat.size)
    for name in ("alpha", "beta", "twist", "incl", "gap", "wblend"):
        vals = np.asarray(getattr(m, name), dtype=np.float32)
        getattr(s, name)[0] = float(vals[0])
        getattr(s, name)[1] = float(vals[1])
    for y in range(2):
        for c in range(3):
            s.kd[y][c] = float(m.kd[y][c])
            s.ks[y][c] = float(m.ks[y][c])
    return s


# ---------------------------------------------------------------------------
# One function per C entry point (argument marshalling only)
# ---------------------------------------------------------------------------

def fabric_create(device: int = 0, seed: int = 0) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    check(_abi.lib().fabric_create(ctypes.byref(ctx), device, ctypes.c_uint64(seed)), "fabric_create")
    return ctx


def fabric_destroy(ctx) -> None:
    _abi.lib().fabric_destroy(ctx)


def fabric_encode(ctx, materials: Sequence, stream=None) -> None:
    arr = (_abi.fabric_material * max(1, len(materials)))(*[_material_struct(m) for m in materials])
    check(_abi.lib().fabric_encode(ctx, arr, len(materials), _stream(stream)), "fabric_encode")


def fabric_set_albedo(ctx, fabric: int, kd, ks, stream=None) -> None:
    kd = np.ascontiguousarray(kd, dtype=np.float32).reshape(2, 3)
    ks = np.ascontiguousarray(ks, dtype=np.float32).reshape(2, 3)
    check(_abi.lib().fabric_set_albedo(ctx, fabric, kd.ctypes.data, ks.ctypes.data, _stream(stream)),
          "fabric_set_albedo")


def fabric_paper_prepare(ctx, params, latents, stream=None) -> None:
    check(_abi.lib().fabric_paper_prepare(ctx, _dptr(params), _dptr(latents), _stream(stream)),
          "fabric_paper_prepare")


def fabric_paper_prepare_encoder(ctx, params, enc_params, stream=None) -> None:
    check(_abi.lib().fabric_paper_prepare_encoder(ctx, _dptr(params), _dptr(enc_params),
                                                  _stream(stream)), "fabric_paper_prepare_encoder")


def fabric_paper_encode(ctx, stream=None) -> None:
    check(_abi.lib().fabric_paper_encode(ctx, _stream(stream)), "fabric_paper_encode")


def fabric_paper_get_encoder(ctx) -> np.ndarray:
    out = np.zeros(FABRIC_N_PAPER_ENCODER_PARAMS, dtype=np.float32)
    check(_abi.lib().fabric_paper_get_encoder(ctx, out.ctypes.data), "fabric_paper_get_encoder")
    return out


def fabric_paper_shade(ctx, g: DeviceGBuffer, out_rgb, prec: str = "bf16", stream=None) -> None:
    gs = g.c_struct()
    check(_abi.lib().fabric_paper_shade(ctx, ctypes.byref(gs), PREC[prec], _dptr(out_rgb),
                                        _stream(stream)), "fabric_paper_shade")


def fabric_paper_forward(ctx, g: DeviceGBuffer, y4, stream=None) -> None:
    gs = g.c_struct()
    check(_abi.lib().fabric_paper_forward(ctx, ctypes.byref(gs), _dptr(y4), _stream(stream)),
          "fabric_paper_forward")


def fabric_set_visibility(ctx, enable: bool) -> None:
    check(_abi.lib().fabric_set_visibility(ctx, int(bool(enable))), "fabric_set_visibility")


def fabric_lerp_latents(ctx, dst, a, b, t, stream=None) -> None:
    dst = np.ascontiguousarray(dst, dtype=np.int32).reshape(-1)
    a = np.ascontiguousarray(a, dtype=np.int32).reshape(-1)
    b = np.ascontiguousarray(b, dtype=np.int32).reshape(-1)
    t = np.ascontiguousarray(t, dtype=np.float32).reshape(-1)
    if not (dst.size == a.size == b.size == t.size):
        raise ValueError("dst, a, b and t need one entry per blend")
    check(_abi.lib().fabric_lerp_latents(ctx, dst.ctypes.data, a.ctypes.data, b.ctypes.data,
                                         t.ctypes.data, int(dst.size), _stream(stream)),
          "fabric_lerp_latents")


def fabric_shade_gbuffer(ctx, g: DeviceGBuffer, prec: int, fallback_samples: int, seed: int,
                         out_rgb, stream=None) -> None:
    gs = g.c_struct()
    check(_abi.lib().fabric_shade_gbuffer(ctx, ctypes.byref(gs), prec, fallback_samples,
                                          ctypes.c_uint64(seed), _dptr(out_rgb), _stream(stream)),
          "fabric_shade_gbuffer")


def fabric_shade_gbuffer_noalloc(ctx, g: DeviceGBuffer, prec: int, fallback_samples: int,
                                 seed: int, out_rgb, stream=None) -> None:
    gs = g.c_struct()
    check(_abi.lib().fabric_shade_gbuffer_noalloc(ctx, ctypes.byref(gs), prec, fallback_samples,
                                                  ctypes.c_uint64(seed), _dptr(out_rgb),
                                                  _stream(stream)),
          "fabric_shade_gbuffer_noalloc")


def fabric_gt_filtered(ctx, g: DeviceGBuffer, n_samples: int, seed: int, out_rgb=None,
                       out_comp=None, stream=None) -> None:
    gs = g.c_struct()
    check(_abi.lib().fabric_gt_filtered(ctx, ctypes.byref(gs), n_samples, ctypes.c_uint64(seed),
                                        _dptr(out_rgb), _dptr(out_comp), _stream(stream)),
          "fabric_gt_filtered")


def fabric_decoder_forward(ctx, g: DeviceGBuffer, prec: int, dec_params, latents, y4,
                           stream=None) -> None:
    gs = g.c_struct()
    check(_abi.lib().fabric_decoder_forward(ctx, ctypes.byref(gs), prec, _dptr(dec_params),
                                            _dptr(latents), _dptr(y4), _stream(stream)),
          "fabric_decoder_forward")


def fabric_decoder_backward(ctx, g: DeviceGBuffer, dec_params, latents, grad_y4, grad_params,
                            grad_latents, stream=None) -> None:
    gs = g.c_struct()
    check(_abi.lib().fabric_decoder_backward(ctx, ctypes.byref(gs), _dptr(dec_params), _dptr(latents),
                                             _dptr(grad_y4), _dptr(grad_params),
                                             _dptr(grad_latents), _stream(stream)),
          "fabric_decoder_backward")


def fabric_encoder_forward(ctx, enc_params, latents, stream=None) -> None:
    check(_abi.lib().fabric_encoder_forward(ctx, _dptr(enc_params), _dptr(latents), _stream(stream)),
          "fabric_encoder_forward")


def fabric_encoder_backward(ctx, enc_params, grad_latents, grad_enc_params, stream=None) -> None:
    check(_abi.lib().fabric_encoder_backward(ctx, _dptr(enc_params), _dptr(grad_latents),
                                             _dptr(grad_enc_params), _stream(stream)),
          "fabric_encoder_backward")


def fabric_make_batch(ctx, seed: int, n: int, r_lo: float, r_hi: float, out: DeviceGBuffer,
                      btdf_frac: float = 0.0, stream=None) -> None:
    os_ = out.c_struct(_abi.fabric_gbuffer_out)
    check(_abi.lib().fabric_make_batch(ctx, ctypes.c_uint64(seed), n, r_lo, r_hi, btdf_frac,
                                       ctypes.byref(os_), _stream(stream)), "fabric_make_batch")


def _train_cfg(cfg: dict) -> _abi.fabric_train_cfg:
    return _abi.fabric_train_cfg(
        int(cfg.get("batch", 1 << 20)), int(cfg.get("gt_samples", 256)), int(cfg.get("prec", FABRIC_BF16)),
        int(cfg.get("seed", 0)), float(cfg.get("lr", 1e-3)), float(cfg.get("beta1", 0.9)),
        float(cfg.get("beta2", 0.999)), float(cfg.get("eps", 1e-8)), float(cfg.get("r_lo", 1e-3)),
        float(cfg.get("r_hi", 0.5)), float(cfg.get("btdf_frac", 0.0)))


def fabric_loss_grad(ctx, batch: Optional[DeviceGBuffer], targets, cfg: dict, grad,
                     want_loss: bool = True, stream=None) -> Optional[float]:
    c = _train_cfg(cfg)
    loss = ctypes.c_float(0.0)
    gs = batch.c_struct() if batch is not None else None
    st = _abi.lib().fabric_loss_grad(ctx, ctypes.byref(gs) if gs is not None else None, _dptr(targets),
                                     ctypes.byref(c), _dptr(grad),
                                     ctypes.byref(loss) if want_loss else None, _stream(stream))
    check(st, "fabric_loss_grad")
    return float(loss.value) if want_loss else None


def fabric_train_step(ctx, batch: Optional[DeviceGBuffer], targets, cfg: dict, want_loss: bool = True,
                      stream=None) -> Optional[float]:
    c = _train_cfg(cfg)
    loss = ctypes.c_float(0.0)
    gs = batch.c_struct() if batch is not None else None
    st = _abi.lib().fabric_train_step(ctx, ctypes.byref(gs) if gs is not None else None, _dptr(targets),
                                      ctypes.byref(c), ctypes.byref(loss) if want_loss else None,
                                      _stream(stream))
    check(st, "fabric_train_step")
    return float(loss.value) if want_loss else None


def fabric_paper_loss_grad(ctx, batch: Optional[DeviceGBuffer], targets, cfg: dict, grad,
                           want_loss: bool = True, stream=None) -> Optional[float]:
    c = _train_cfg(dict({"prec": FABRIC_FP32}, **cfg))
    loss = ctypes.c_float(0.0)
    gs = batch.c_struct() if batch is not None else None
    st = _abi.lib().fabric_paper_loss_grad(ctx, ctypes.byref(gs) if gs is not None else None,
                                           _dptr(targets), ctypes.byref(c), _dptr(grad),
                                           ctypes.byref(loss) if want_loss else None, _stream(stream))
    check(st, "fabric_paper_loss_grad")
    return float(loss.value) if want_loss else None


def fabric_paper_train_step(ctx, batch: Optional[DeviceGBuffer], targets, cfg: dict,
                            want_loss: bool = True, stream=None) -> Optional[float]:
    c = _train_cfg(dict({"prec": FABRIC_FP32}, **cfg))
    loss = ctypes.c_float(0.0)
    gs = batch.c_struct() if batch is not None else None
    st = _abi.lib().fabric_paper_train_step(ctx, ctypes.byref(gs) if gs is not None else None,
                                            _dptr(targets), ctypes.byref(c),
                                            ctypes.byref(loss) if want_loss else None, _stream(stream))
    check(st, "fabric_paper_train_step")
    return float(loss.value) if want_loss else None


def fabric_paper_set_footprint_encoding(ctx, one_blob: bool) -> None:
    check(_abi.lib().fabric_paper_set_footprint_encoding(ctx, 1 if one_blob else 0),
          "fabric_paper_set_footprint_encoding")


def fabric_paper_set_spatial_fusion(ctx, fused: bool, stream=None) -> None:
    check(_abi.lib().fabric_paper_set_spatial_fusion(ctx, 1 if fused else 0, _stream(stream)),
          "fabric_paper_set_spatial_fusion")


def fabric_paper_get_params(ctx, n_mats: int):
    params = np.zeros(FABRIC_N_PAPER_DECODER_PARAMS, dtype=np.float32)
    latents = np.zeros((n_mats, FABRIC_PAPER_LATENT), dtype=np.float32)
    check(_abi.lib().fabric_paper_get_params(ctx, params.ctypes.data, latents.ctypes.data),
          "fabric_paper_get_params")
    return params, latents


def fabric_get_params(ctx) -> np.ndarray:
    out = np.zeros(FABRIC_N_PARAMS, dtype=np.float32)
    check(_abi.lib().fabric_get_params(ctx, out.ctypes.data, out.size), "fabric_get_params")
    return out


def fabric_set_params(ctx, params) -> None:
    p = np.ascontiguousarray(params, dtype=np.float32)
    check(_abi.lib().fabric_set_params(ctx, p.ctypes.data, p.size), "fabric_set_params")


def fabric_get_latents(ctx, n_mats: int) -> np.ndarray:
    out = np.zeros((n_mats, FABRIC_LATENT), dtype=np.float32)
    check(_abi.lib().fabric_get_latents(ctx, out.ctypes.data, n_mats), "fabric_get_latents")
    return out


def fabric_save(ctx) -> bytes:
    size = ctypes.c_size_t(0)
    check(_abi.lib().fabric_save(ctx, None, ctypes.byref(size)), "fabric_save")
    buf = ctypes.create_string_buffer(size.value)
    check(_abi.lib().fabric_save(ctx, buf, ctypes.byref(size)), "fabric_save")
    return buf.raw[: size.value]


def fabric_load(ctx, blob: bytes) -> None:
    buf = ctypes.create_string_buffer(blob, len(blob))
    check(_abi.lib().fabric_load(ctx, buf, len(blob)), "fabric_load")


def fabric_error_count(ctx, reset: bool = False) -> int:
    return int(_abi.lib().fabric_error_count(ctx, 1 if reset else 0))


# ---------------------------------------------------------------------------
# Convenience wrapper
# ---------------------------------------------------------------------------

class Fabric:
    """A library context plus the fabrics it has encoded."""

    def __init__(self, device: int = 0, seed: int = 0):
        _abi.lib()
        self.device = device
        self.ctx = fabric_create(device, seed)
        self.n_mats = 0

    def close(self) -> None:
        if self.ctx is not None:
            fabric_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def encode(self, materials: Sequence) -> None:
        fabric_encode(self.ctx, materials)
        self.n_mats = len(materials)

    def shade(self, g: DeviceGBuffer, prec: str = "bf16", fallback_samples: int = 0, seed: int = 0,
              out=None):
        torch = _torch()
        if out is None:
            out = torch.empty((3, g.n), dtype=torch.float32, device=g.u.device)
        fabric_shade_gbuffer(self.ctx, g, PREC[prec], fallback_samples, seed, out)
        return out

    def gt_filtered(self, g: DeviceGBuffer, n_samples: int, seed: int, rgb: bool = True,
                    comp: bool = True):
        torch = _torch()
        o_rgb = torch.empty((3, g.n), dtype=torch.float32, device=g.u.device) if rgb else None
        o_comp = torch.empty((4, g.n), dtype=torch.float32, device=g.u.device) if comp else None
        fabric_gt_filtered(self.ctx, g, n_samples, seed, o_rgb, o_comp)
        return o_rgb, o_comp

    def params(self) -> np.ndarray:
        return fabric_get_params(self.ctx)

    def set_params(self, p) -> None:
        fabric_set_params(self.ctx, p)

    def latents(self) -> np.ndarray:
        return fabric_get_latents(self.ctx, self.n_mats)

    def set_visibility(self, enable: bool) -> None:
        """Inter-yarn visibility V in the analytic filter (targets, ground
        truth, fallback); off by default."""
        fabric_set_visibility(self.ctx, enable)

    def lerp_latents(self, dst, a, b, t, stream=None) -> None:
        """z[dst[k]] = (1 - t[k]) z[a[k]] + t[k] z[b[k]] on the device (latent
        interpolation / extrapolation between encoded fabrics)."""
        fabric_lerp_latents(self.ctx, dst, a, b, t, stream)

    def train_step(self, gbuf: Optional[DeviceGBuffer] = None, targets=None, want_loss: bool = True,
                   **cfg) -> Optional[float]:
        """One optimiser step on `gbuf` (or on cfg["batch"] generated samples)."""
        return fabric_train_step(self.ctx, gbuf, targets, cfg, want_loss=want_loss)

    def loss_grad(self, gbuf: Optional[DeviceGBuffer] = None, targets=None, **cfg):
        torch = _torch()
        grad = torch.empty(FABRIC_N_PARAMS, dtype=torch.float32, device="cuda")
        loss = fabric_loss_grad(self.ctx, gbuf, targets, cfg, grad)
        return loss, grad

    def error_count(self, reset: bool = False) -> int:
        return fabric_error_count(self.ctx, reset)
