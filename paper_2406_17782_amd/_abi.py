"""ctypes declarations of include/fabric.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfabric.so")

FABRIC_OK = 0
FABRIC_E_INVAL = 1
FABRIC_E_RANGE = 2
FABRIC_E_NOMEM = 3
FABRIC_E_DEVICE = 4
FABRIC_E_NONFINITE = 5
FABRIC_E_STATE = 6

FABRIC_FP32 = 0
FABRIC_BF16 = 1
FABRIC_FP16 = 2
FABRIC_FP8_E4M3 = 3

FABRIC_MAX_FABRICS = 256
FABRIC_MAX_SAMPLES = 16384
FABRIC_NOALLOC_MAX_PIXELS = 4194304
FABRIC_LATENT = 32
FABRIC_N_DECODER_PARAMS = 13572
FABRIC_PAPER_LATENT = 64
FABRIC_N_PAPER_DECODER_PARAMS = 27076
FABRIC_N_PAPER_ENCODER_PARAMS = 108480
FABRIC_N_ENCODER_PARAMS = 104352
FABRIC_N_PARAMS = FABRIC_N_DECODER_PARAMS + FABRIC_N_ENCODER_PARAMS

PREC = {"fp32": FABRIC_FP32, "bf16": FABRIC_BF16, "fp16": FABRIC_FP16, "fp8": FABRIC_FP8_E4M3}

_F2 = ctypes.c_float * 2


class fabric_material(ctypes.Structure):
    _fields_ = [("wx", ctypes.c_uint8), ("wy", ctypes.c_uint8),
                ("pattern", ctypes.c_uint8 * 256),
                ("alpha", _F2), ("beta", _F2), ("twist", _F2), ("incl", _F2), ("gap", _F2),
                ("wblend", _F2), ("kd", (ctypes.c_float * 3) * 2), ("ks", (ctypes.c_float * 3) * 2)]


_GB_FIELDS = [("n", ctypes.c_int64), ("fabric_id", ctypes.c_void_p)] + [
    (f, ctypes.c_void_p) for f in
    ("u", "v", "radius", "wi_x", "wi_y", "wi_z", "wo_x", "wo_y", "wo_z")]


class fabric_gbuffer(ctypes.Structure):
    _fields_ = _GB_FIELDS


class fabric_gbuffer_out(ctypes.Structure):
    _fields_ = _GB_FIELDS


class fabric_train_cfg(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int64), ("gt_samples", ctypes.c_int32),
                ("prec", ctypes.c_int32), ("seed", ctypes.c_uint64), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("r_lo", ctypes.c_float), ("r_hi", ctypes.c_float), ("btdf_frac", ctypes.c_float)]


EXPORTS = [
    "fabric_create", "fabric_destroy", "fabric_status_str", "fabric_encode", "fabric_set_albedo",
    "fabric_lerp_latents", "fabric_set_visibility", "fabric_paper_prepare", "fabric_paper_shade",
    "fabric_paper_forward", "fabric_paper_prepare_encoder", "fabric_paper_encode",
    "fabric_paper_get_encoder",
    "fabric_paper_train_step", "fabric_paper_loss_grad", "fabric_paper_get_params",
    "fabric_paper_set_footprint_encoding", "fabric_paper_set_spatial_fusion",
    "fabric_shade_gbuffer", "fabric_shade_gbuffer_noalloc", "fabric_gt_filtered",
    "fabric_decoder_forward", "fabric_decoder_backward", "fabric_encoder_forward", "fabric_encoder_backward",
    "fabric_make_batch", "fabric_loss_grad", "fabric_train_step", "fabric_get_params", "fabric_set_params",
    "fabric_get_latents", "fabric_save", "fabric_load", "fabric_error_count",
]

_P = ctypes.c_void_p
_S = ctypes.c_int  # fabric_status


def _declare(L):
    L.fabric_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_uint64]
    L.fabric_create.restype = _S
    L.fabric_destroy.argtypes = [_P]
    L.fabric_destroy.restype = None
    L.fabric_status_str.argtypes = [_S]
    L.fabric_status_str.restype = ctypes.c_char_p
    L.fabric_encode.argtypes = [_P, ctypes.POINTER(fabric_material), ctypes.c_int32, _P]
    L.fabric_encode.restype = _S
    L.fabric_set_albedo.argtypes = [_P, ctypes.c_int32, _P, _P, _P]
    L.fabric_set_albedo.restype = _S
    L.fabric_lerp_latents.argtypes = [_P, _P, _P, _P, _P, ctypes.c_int32, _P]
    L.fabric_lerp_latents.restype = _S
    L.fabric_set_visibility.argtypes = [_P, ctypes.c_int32]
    L.fabric_set_visibility.restype = _S
    L.fabric_paper_prepare.argtypes = [_P, _P, _P, _P]
    L.fabric_paper_prepare.restype = _S
    L.fabric_paper_prepare_encoder.argtypes = [_P, _P, _P, _P]
    L.fabric_paper_prepare_encoder.restype = _S
    L.fabric_paper_encode.argtypes = [_P, _P]
    L.fabric_paper_encode.restype = _S
    L.fabric_paper_get_encoder.argtypes = [_P, _P]
    L.fabric_paper_get_encoder.restype = _S
    L.fabric_paper_shade.argtypes = [_P, ctypes.POINTER(fabric_gbuffer), ctypes.c_int, _P, _P]
    L.fabric_paper_shade.restype = _S
    L.fabric_paper_forward.argtypes = [_P, ctypes.POINTER(fabric_gbuffer), _P, _P]
    L.fabric_paper_forward.restype = _S
    L.fabric_paper_train_step.argtypes = [_P, ctypes.POINTER(fabric_gbuffer), _P,
                                          ctypes.POINTER(fabric_train_cfg), ctypes.POINTER(ctypes.c_float), _P]
    L.fabric_paper_train_step.restype = _S
    L.fabric_paper_loss_grad.argtypes = [_P, ctypes.POINTER(fabric_gbuffer), _P,
                                         ctypes.POINTER(fabric_train_cfg), _P, ctypes.POINTER(ctypes.c_float), _P]
    L.fabric_paper_loss_grad.restype = _S
    L.fabric_paper_set_footprint_encoding.argtypes = [_P, ctypes.c_int32]
    L.fabric_paper_set_footprint_encoding.restype = _S
    L.fabric_paper_set_spatial_fusion.argtypes = [_P, ctypes.c_int32, _P]
    L.fabric_paper_set_spatial_fusion.restype = _S
    L.fabric_paper_get_params.argtypes = [_P, _P, _P]
    L.fabric_paper_get_params.restype = _S
    L.fabric_shade_gbuffer.argtypes = [_P, ctypes.POINTER(fabric_gbuffer), ctypes.c_int,
                                       ctypes.c_int32, ctypes.c_uint64, _P, _P]
    L.fabric_shade_gbuffer.restype = _S
    L.fabric_shade_gbuffer_noalloc.argtypes = L.fabric_shade_gbuffer.argtypes
    L.fabric_shade_gbuffer_noalloc.restype = _S
    L.fabric_gt_filtered.argtypes = [_P, ctypes.POINTER(fabric_gbuffer), ctypes.c_int32,
                                     ctypes.c_uint64, _P, _P, _P]
    L.fabric_gt_filtered.restype = _S
    L.fabric_decoder_forward.argtypes = [_P, ctypes.POINTER(fabric_gbuffer), ctypes.c_int, _P, _P,
                                         _P, _P]
    L.fabric_decoder_forward.restype = _S
    L.fabric_decoder_backward.argtypes = [_P, ctypes.POINTER(fabric_gbuffer), _P, _P, _P, _P, _P, _P]
    L.fabric_decoder_backward.restype = _S
    L.fabric_encoder_forward.argtypes = [_P, _P, _P, _P]
    L.fabric_encoder_forward.restype = _S
    L.fabric_encoder_backward.argtypes = [_P, _P, _P, _P, _P]
    L.fabric_encoder_backward.restype = _S
    L.fabric_make_batch.argtypes = [_P, ctypes.c_uint64, ctypes.c_int64, ctypes.c_float,
                                    ctypes.c_float, ctypes.c_float,
                                    ctypes.POINTER(fabric_gbuffer_out), _P]
    L.fabric_make_batch.restype = _S
    L.fabric_loss_grad.argtypes = [_P, ctypes.POINTER(fabric_gbuffer), _P,
                                   ctypes.POINTER(fabric_train_cfg), _P, ctypes.POINTER(ctypes.c_float), _P]
    L.fabric_loss_grad.restype = _S
    L.fabric_train_step.argtypes = [_P, ctypes.POINTER(fabric_gbuffer), _P,
                                    ctypes.POINTER(fabric_train_cfg), ctypes.POINTER(ctypes.c_float), _P]
    L.fabric_train_step.restype = _S
    L.fabric_get_params.argtypes = [_P, _P, ctypes.c_size_t]
    L.fabric_get_params.restype = _S
    L.fabric_set_params.argtypes = [_P, _P, ctypes.c_size_t]
    L.fabric_set_params.restype = _S
    L.fabric_get_latents.argtypes = [_P, _P, ctypes.c_int32]
    L.fabric_get_latents.restype = _S
    L.fabric_save.argtypes = [_P, _P, ctypes.POINTER(ctypes.c_size_t)]
    L.fabric_save.restype = _S
    L.fabric_load.argtypes = [_P, _P, ctypes.c_size_t]
    L.fabric_load.restype = _S
    L.fabric_error_count.argtypes = [_P, ctypes.c_int]
    L.fabric_error_count.restype = ctypes.c_int64


_lib = None


def lib():
    """The loaded HIP library.  Raises ImportError if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                "(python -m paper_2406_17782_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        _declare(L)
        _lib = L
    return _lib


class FabricError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        name = lib().fabric_status_str(status).decode() if _lib is not None else str(status)
        super().__init__(f"{where}: {name} (status {status})")


def check(status: int, where: str) -> None:
    if status != FABRIC_OK:
        raise FabricError(status, where)
