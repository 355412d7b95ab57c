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


def assert_filter_parity(gpu_comp, orc_comp, flagged, n_samples, rel=1e-4, abs_floor=1e-9):
    """The same-sample bar of the footprint filter.  Every pixel none of whose
    samples the oracle flags agrees within `rel` of its largest component.  A
    flagged sample lies within 1e-5 cells of a classification edge (with
    visibility, also within 4e-6 cells of a texel boundary), where float32
    and float64 may classify it differently; a pixel with k flagged samples of
    N may deviate by at most rel + k / N, one sample's share of the estimate
    per flagged sample.  Differences below `abs_floor` are ignored (pixels
    whose components are all near zero)."""
    bad, err = filter_mismatch(gpu_comp, orc_comp, flagged, rel, abs_floor)
    k = np.asarray(flagged)
    fl = k > 0
    allowed = rel + k / float(n_samples)
    dev = np.abs(np.asarray(gpu_comp, np.float64) - np.asarray(orc_comp, np.float64)).max(axis=0)
    over = dev > allowed * np.abs(np.asarray(orc_comp, np.float64)).max(axis=0) + abs_floor
    unflagged_bad = bad & ~fl
    sig = dev > abs_floor
    max_unflagged = float(err[~fl & sig].max()) if (~fl & sig).any() else 0.0
    max_ratio = float((err[fl & sig] / allowed[fl & sig]).max()) if (fl & sig).any() else 0.0
    msg = (f"pixels {bad.size}, unflagged beyond {rel:g}: {int(unflagged_bad.sum())} "
           f"(max err {max_unflagged:.3g}); flagged {int(fl.sum())}, beyond their allowance: "
           f"{int((over & fl).sum())} (max err / allowance {max_ratio:.3g})")
    assert not unflagged_bad.any(), msg
    assert not over.any(), msg
    return msg


# The same bar with the visibility flags of the oracle.
assert_filter_parity_vis = assert_filter_parity
