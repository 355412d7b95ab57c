"""Shared helpers of the GPU tests: device set-up and tolerance checks."""
import numpy as np
import pytest


def require_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs an MI355X GPU")
    return torch


def rel_norm_err(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def filter_mismatch(gpu_comp, orc_comp, flagged, rel=1e-4, abs_floor=1e-9):
    """Per-pixel error of the footprint filter, relative to the pixel's largest
    component.  Returns (bad mask, per-pixel error)."""
    g = np.asarray(gpu_comp, dtype=np.float64)
    o = np.asarray(orc_comp, dtype=np.float64)
    scale = np.abs(o).max(axis=0)
    err = np.abs(g - o).max(axis=0) / np.maximum(scale, abs_floor)
    bad = np.abs(g - o).max(axis=0) > rel * scale + abs_floor
    return bad, err


def assert_filter_parity(gpu_comp, orc_comp, flagged, rel=1e-4, max_bad=1e-3, unflagged_cap=2e-3):
    """At least 1 - `max_bad` of the pixels agree within `rel` of their
    largest component.  The rest are pixels whose samples sit within 1e-5
    cells of a classification edge (flagged: FP32 and FP64 may put a sample
    in different yarns), or pixels where the FP32 integrand is sensitive
    (a sharp specular lobe amplifies the few-ulp error of the hardware
    transcendentals); an unflagged pixel never deviates by more than
    `unflagged_cap`."""
    bad, err = filter_mismatch(gpu_comp, orc_comp, flagged, rel)
    flagged = np.asarray(flagged) > 0
    n = bad.size
    unflagged_bad = bad & ~flagged
    max_unflagged = float(err[~flagged].max()) if (~flagged).any() else 0.0
    msg = (f"pixels {n}, bad {int(bad.sum())}, unflagged bad {int(unflagged_bad.sum())}, "
           f"flagged {int(flagged.sum())}, max err unflagged {max_unflagged:.3g}")
    assert max_unflagged <= unflagged_cap, msg
    assert bad.sum() <= max(1, max_bad * n), msg
    return msg


def assert_filter_parity_vis(gpu_comp, orc_comp, flagged, rel=1e-4, max_bad=1e-3,
                             flagged_cap=5e-2):
    """Footprint filter with visibility, same samples.  Unflagged pixels as
    assert_filter_parity.  A flagged pixel holds a sample within 4e-6 cells
    of a texel boundary (or 1e-5 of a classification edge): float32 sample
    positions rounded in another order may start its ray in the neighbouring
    texel, which changes that sample's V; such pixels stay within
    `flagged_cap` of their largest component."""
    bad, err = filter_mismatch(gpu_comp, orc_comp, flagged, rel)
    flagged = np.asarray(flagged) > 0
    n = bad.size
    unflagged_bad = bad & ~flagged
    max_flagged = float(err[flagged].max()) if flagged.any() else 0.0
    msg = (f"pixels {n}, bad {int(bad.sum())}, unflagged bad {int(unflagged_bad.sum())}, "
           f"flagged {int(flagged.sum())}, max err flagged {max_flagged:.3g}")
    assert unflagged_bad.sum() <= max(1, max_bad * n), msg
    assert max_flagged <= flagged_cap, msg
    return msg
