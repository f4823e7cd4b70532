"""Host-side checks of the C ABI (no GPU needed): the built library loads and
exports every function include/cf.h declares, and the binding's structures and
model blob match the header's layout."""
import ctypes
import os
import re

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cf.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cf_[a-z0-9_]+)\s*\(", src)))


def _lib():
    from paper_2104_04547_amd import cfabi
    if not os.path.exists(cfabi.LIB_PATH):
        from paper_2104_04547_amd import build
        build.build()
    return cfabi, cfabi.load()


def test_library_exports_every_declared_function():
    cfabi, lib = _lib()
    names = _declared()
    assert len(names) >= 13
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(cfabi.EXPORTS) == names


def test_struct_layouts_match_header():
    from paper_2104_04547_amd import cfabi
    # cf_model_desc: 3 + 8*5 + 8 + 7 four-byte fields
    assert ctypes.sizeof(cfabi.cf_model_desc) == 4 * (3 + 40 + 8 + 7)
    assert ctypes.sizeof(cfabi.cf_pose_batch) == 8 + 5 * 8
    assert ctypes.sizeof(cfabi.cf_csr) == 24


@pytest.mark.parametrize("arch_name", ["tiny", "full", "full_mid", "full_late", "paper"])
def test_model_blob_size_and_order(arch_name):
    from paper_2104_04547_amd import cfabi
    arch = synth.ARCHS[arch_name]
    w = synth.make_weights(arch)
    blob = cfabi.pack_model(arch, w)
    assert len(blob) == ctypes.sizeof(cfabi.cf_model_desc) + 4 * synth.n_params(arch)
    assert sorted(cfabi.blob_param_order(arch)) == sorted(w.keys())
    # the generator draws the tensors in the blob's order
    assert cfabi.blob_param_order(arch) == [n for n, _, _ in synth.model.param_shapes(arch)]
    d = cfabi.cf_model_desc.from_buffer_copy(blob[:ctypes.sizeof(cfabi.cf_model_desc)])
    assert d.magic == cfabi.CF_MODEL_MAGIC and d.n_conv == len(arch.conv) and d.H == arch.H
    first = np.frombuffer(blob, dtype="<f4", count=8, offset=ctypes.sizeof(cfabi.cf_model_desc))
    np.testing.assert_array_equal(first, w["conv0.w"].reshape(-1)[:8])
    # the head's parameters close the blob, in the header's documented order
    last = arch.head_outputs[-1]
    np.testing.assert_array_equal(np.frombuffer(blob[-4:], dtype="<f4"), w[last + ".b"])
    assert d.head == cfabi.HEAD_KINDS[arch.head] and d.fusion_layers == arch.n_fusion


def test_last_error_is_callable_without_device():
    cfabi, lib = _lib()
    assert isinstance(cfabi.cf_last_error(), str)


def test_create_rejects_bad_blob_before_touching_a_device():
    # a corrupt header is rejected on the host (invalid argument), not by a kernel
    cfabi, lib = _lib()
    out = ctypes.c_void_p()
    junk = ctypes.create_string_buffer(b"\0" * 300, 300)
    rc = lib.cf_create(ctypes.cast(junk, ctypes.c_void_p), 300, 0, 0, ctypes.byref(out))
    assert rc in (cfabi.CF_ERR_INVALID_ARG, cfabi.CF_ERR_HIP)
    assert not out.value
