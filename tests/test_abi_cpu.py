"""CPU-only checks of the C-ABI library: it loads, exports every declared symbol,
and validates arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

import paper_2608_21227_amd as svdv

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    text = open(os.path.join(ROOT, "include", "svdv.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(?:int64_t|int|const char\*)\s+(\w+)\s*\(", text)))


def test_header_and_binding_agree():
    assert _header_functions() == sorted(svdv.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = svdv.lib()
    for name in _header_functions():
        assert hasattr(lib, name), name


def test_status_strings():
    lib = svdv.lib()
    assert lib.svdv_status_string(0) == b"SVDV_OK"
    assert lib.svdv_status_string(-2) == b"SVDV_ERR_UNSUPPORTED"


def test_argument_validation_happens_before_any_gpu_call():
    lib = svdv.lib()
    cfg = svdv.Config()
    dummy = ctypes.c_void_p(0x1000)
    # negative size, lda too small, bad dtype, NULL A with nonzero size
    assert lib.svd_values_ex(dummy, -1, 4, 4, 0, dummy, None, ctypes.byref(cfg._c())) == -1
    assert lib.svd_values_ex(dummy, 8, 4, 4, 0, dummy, None, ctypes.byref(cfg._c())) == -1
    assert lib.svd_values_ex(dummy, 4, 4, 4, 7, dummy, None, ctypes.byref(cfg._c())) == -1
    assert lib.svd_values_ex(None, 4, 4, 4, 0, dummy, None, ctypes.byref(cfg._c())) == -1
    assert b"lda" in lib.svdv_last_error() or b"NULL" in lib.svdv_last_error()
    # empty matrices succeed and touch nothing
    assert lib.svd_values_ex(None, 0, 5, 1, 0, None, None, None) == 0
    assert lib.svd_values_ex(None, 5, 0, 5, 1, None, None, None) == 0
    # unsupported configurations are reported as such (the tuner's skip signal)
    bad = svdv.Config(tile=48)
    assert lib.svd_values_ex(dummy, 4, 4, 4, 0, dummy, None, ctypes.byref(bad._c())) == -2
    assert lib.svdv_stage_bidiag(dummy, 10, 24, 25, dummy, dummy, None, None) == -2
    assert lib.svdv_apply_qt(dummy, 4, dummy, 4, dummy, 4, 4, 4, 4, 0, 5, None, None) == -1


def test_config_space_validity_rules():
    # float64 tile 128 is not built; oversized register tiles are rejected
    assert not svdv.check_config(256, 256, "float64", svdv.Config(tile=128))
    assert svdv.check_config(256, 256, "float32", svdv.Config(tile=128, threads=256, inner_block=1, sweep_width=2))
    assert not svdv.check_config(256, 256, "float32", svdv.Config(tile=128, threads=1024, inner_block=8))
    assert svdv.check_config(256, 256, "float64", svdv.Config(tile=16, threads=64, inner_block=2, sweep_width=8))
    assert not svdv.check_config(256, 256, "float32", svdv.Config(tile=128, sweep_width=8))
    d = svdv.default_config(4096, 4096, "float32")
    assert svdv.check_config(4096, 4096, "float32", d)


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    import importlib
    monkeypatch.setattr(svdv, "LIB_PATH", str(tmp_path / "nope.so"))
    monkeypatch.setattr(svdv, "_lib", None)
    with pytest.raises(RuntimeError):
        svdv.lib()


def test_reduced_precision_config_rules():
    ok = svdv.Config(tile=16, threads=1024, inner_block=1, sweep_width=4, update_precision=2)
    assert svdv.check_config(512, 512, "float32", ok)
    assert svdv.check_config(512, 512, "float32", svdv.Config(16, 1024, 1, 4, 3))
    assert not svdv.check_config(512, 512, "float64", ok)  # float32 input only
    assert not svdv.check_config(512, 512, "float32", svdv.Config(16, 1024, 1, 4, 1))  # no such precision
    assert not svdv.check_config(512, 512, "float32", svdv.Config(16, 256, 2, 4, 2))  # streaming-only configuration


def test_binding_rejects_host_tensors_before_the_library():
    """The binding checks its tensors before any pointer reaches the library (which
    cannot tell a host pointer from a device one): host tensors raise at once."""
    torch = pytest.importorskip("torch")
    a = torch.zeros((4, 4))
    d, e = torch.zeros(4, dtype=torch.float64), torch.zeros(3, dtype=torch.float64)
    for call in (lambda: svdv.svd_values(a), lambda: svdv.stage_band(a),
                 lambda: svdv.stage_bidiag(torch.zeros((4, 17), dtype=torch.float64), 16),
                 lambda: svdv.stage_values(d, e), lambda: svdv.svd_values_batched([a]),
                 lambda: svdv.apply_qt(a, a, a), lambda: svdv.mlp_forward(torch.zeros(svdv.MLP_NPARAM), a)):
        with pytest.raises(ValueError, match="on a GPU"):
            call()
    with pytest.raises(TypeError, match="out_dtype"):
        svdv.stage_values(d, e, out_dtype=torch.int32)
