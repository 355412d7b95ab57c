"""The C ABI library loads, exports every entry point include/fabric.h
declares, and its struct layouts agree with the Python binding (no GPU)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fabric.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fabric_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2406_17782_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _abi.lib()


def test_library_exports_every_declared_entry_point(lib):
    from paper_2406_17782_amd import _abi
    decl = declared_functions()
    assert len(decl) >= 20
    for name in decl:
        assert hasattr(lib, name), name
    assert sorted(_abi.EXPORTS) == decl


def test_status_strings(lib):
    from paper_2406_17782_amd import _abi
    assert lib.fabric_status_str(0) == b"ok"
    assert lib.fabric_status_str(6) == b"invalid call order"
    assert lib.fabric_status_str(99) == b"unknown status"


def test_null_arguments_are_rejected_without_a_device(lib):
    # Validation happens before any device work, so these run on the CPU.
    assert lib.fabric_create(None, 0, 0) == 1
    assert lib.fabric_encode(None, None, 1, None) == 1
    assert lib.fabric_shade_gbuffer(None, None, 0, 0, 0, None, None) == 1
    assert lib.fabric_shade_gbuffer_noalloc(None, None, 0, 0, 0, None, None) == 1
    assert lib.fabric_gt_filtered(None, None, 64, 0, None, None, None) == 1
    assert lib.fabric_train_step(None, None, None, None, None, None) == 1
    assert lib.fabric_error_count(None, 0) == -1
    # The later entry points validate the same way.
    assert lib.fabric_set_visibility(None, 1) == 1
    assert lib.fabric_lerp_latents(None, None, None, None, None, 0, None) == 1
    assert lib.fabric_paper_prepare(None, None, None, None) == 1
    assert lib.fabric_paper_shade(None, None, 1, None, None) == 1
    assert lib.fabric_paper_forward(None, None, None, None) == 1
    assert lib.fabric_paper_train_step(None, None, None, None, None, None) == 1
    assert lib.fabric_paper_loss_grad(None, None, None, None, None, None, None) == 1
    assert lib.fabric_paper_set_footprint_encoding(None, 1) == 1
    assert lib.fabric_paper_set_spatial_fusion(None, 1, None) == 1
    assert lib.fabric_paper_get_params(None, None, None) == 1
    assert lib.fabric_paper_prepare_encoder(None, None, None, None) == 1
    assert lib.fabric_paper_encode(None, None) == 1
    assert lib.fabric_paper_get_encoder(None, None) == 1
    lib.fabric_destroy(None)


def test_struct_layouts_match_the_header(tmp_path):
    from paper_2406_17782_amd import _abi
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "fabric.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(fabric_material), offsetof(fabric_material, alpha),
         offsetof(fabric_material, kd), offsetof(fabric_material, ks));
  printf("%zu %zu\n", sizeof(fabric_gbuffer), offsetof(fabric_gbuffer, wo_z));
  printf("%zu %zu %zu %zu\n", sizeof(fabric_train_cfg), offsetof(fabric_train_cfg, seed),
         offsetof(fabric_train_cfg, lr), offsetof(fabric_train_cfg, r_hi));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    M, G, C = _abi.fabric_material, _abi.fabric_gbuffer, _abi.fabric_train_cfg
    expect = [ctypes.sizeof(M), M.alpha.offset, M.kd.offset, M.ks.offset,
              ctypes.sizeof(G), G.wo_z.offset,
              ctypes.sizeof(C), C.seed.offset, C.lr.offset, C.r_hi.offset]
    assert [int(x) for x in out] == expect


def test_product_path_does_not_touch_the_oracle():
    """The HIP package never imports or loads the oracle."""
    pkg = os.path.join(ROOT, "paper_2406_17782_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), f


def test_binding_constants_match_header():
    """The Python binding's limits and sizes are the header's #defines."""
    import re
    from paper_2406_17782_amd import _abi
    text = open(os.path.join(ROOT, "include", "fabric.h")).read()
    defs = dict(re.findall(r"#define (FABRIC_\w+) (\d+)\s", text))
    for name in ("FABRIC_MAX_FABRICS", "FABRIC_MAX_SAMPLES", "FABRIC_LATENT",
                 "FABRIC_N_DECODER_PARAMS", "FABRIC_N_ENCODER_PARAMS", "FABRIC_PAPER_LATENT",
                 "FABRIC_N_PAPER_DECODER_PARAMS", "FABRIC_N_PAPER_ENCODER_PARAMS",
                 "FABRIC_NOALLOC_MAX_PIXELS"):
        assert getattr(_abi, name) == int(defs[name]), name


def test_stream_arguments_accept_handles_and_stream_objects():
    """The binding passes a HIP stream handle: an integer as given, or the
    handle of a stream object (torch's `cuda_stream`)."""
    import paper_2406_17782_amd as pkg

    class FakeStream:
        cuda_stream = 0x1234

    assert pkg._stream(0x5678) == 0x5678
    assert pkg._stream(FakeStream()) == 0x1234
