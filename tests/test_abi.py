"""Host-side checks of the C ABI: the library loads, exports every entry point
that include/geninv.h declares, and rejects bad arguments before touching a
device.  No compute call is made, so these run without a GPU."""
import ctypes
import os
import re

import pytest

from paper_0804_4809_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "geninv.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(geninv_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libgeninv.so not built")
    return _lib.load()


def test_header_declares_expected_entry_points():
    names = _declared()
    for must in ("geninv_dgeninv", "geninv_dlstsq", "geninv_dgram", "geninv_dfrchol", "geninv_dspdinv",
                 "geninv_dchain", "geninv_create", "geninv_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(_lib.exported_names()) == _declared()


def test_version_and_strerror(lib):
    assert lib.geninv_version() >= 100
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.geninv_strerror(code)
    assert lib.geninv_strerror(123) == b"unknown status"


def test_null_context_is_einval(lib):
    assert lib.geninv_dgeninv(None, 3, 3, None, 3, 0.0, None, 3, None, None) == -1
    assert lib.geninv_dlstsq(None, 3, 3, 1, None, 3, None, 3, 0.0, None, 3, None) == -1
    assert lib.geninv_dgram(None, 3, 3, None, 3, None, 3, 0) == -1
    assert lib.geninv_dfrchol(None, 3, None, 3, 0.0, None, 3, None, None, None, None) == -1
    assert lib.geninv_dspdinv(None, 3, None, 3, None, 3) == -1
    assert lib.geninv_dchain(None, 3, 3, 2, None, 3, None, 2, None, 3, None, 3) == -1
    assert lib.geninv_dgemm(None, 0, 0, 2, 2, 2, 1.0, None, 2, None, 2, 0.0, None, 2) == -1
    assert lib.geninv_set_stream(None, None) == -1
    assert lib.geninv_sync_status(None) == -1
    assert lib.geninv_lstsq_batched(None, 0, None, None, 4, None, None, None, None, 0.0, None, None, None,
                                    None) == -1
    assert lib.geninv_set_workspace_limit(None, 0) == -1
    assert lib.geninv_set_debug(None, 0) == -1
    assert lib.geninv_debug_poison(None) == -1
    assert lib.geninv_batch_plan_graph_fallbacks(None) == -1
    assert lib.geninv_batch_plan_autotune(None, 1, None, None, None, None, None) == -1
    assert lib.geninv_batch_plan_config(None, 0, 256) == -1
    assert lib.geninv_batch_plan_get_config(None, None, None) == -1
    assert lib.geninv_dlstsq_noalloc(None, 3, 3, 1, None, 3, None, 3, 0.0, None, 3, None) == -1
    assert lib.geninv_destroy(None) == 0


def test_create_rejects_null_handle_and_bad_device(lib):
    assert lib.geninv_create(None, 0, None) == -1
    h = ctypes.c_void_p()
    assert lib.geninv_create(ctypes.byref(h), -1, None) in (-1, -3)


def test_workspace_query(lib):
    FP64, BF16, INT8 = 0, 1, 2
    assert lib.geninv_workspace_bytes(0, 5, 0, FP64, 0, 0, 0) == 0
    small = lib.geninv_workspace_bytes(200, 50, 3, FP64, 0, 0, 0)
    big = lib.geninv_workspace_bytes(8192, 2048, 8, FP64, 0, 0, 0)
    assert 0 < small < big
    # four n x n float64 slots dominate
    assert big >= 4 * 2048 * 2048 * 8
    # transposed problems factor the smaller dimension
    assert lib.geninv_workspace_bytes(50, 200, 0, FP64, 0, 0, 0) == lib.geninv_workspace_bytes(200, 50, 0, FP64,
                                                                                                0, 0, 0)
    # the mixed forms add their operand planes: 4 bfloat16 slices of G (8 bytes
    # per element), or 16 int8 residues (16 bytes per element)
    m, n = 32768, 4096
    base = lib.geninv_workspace_bytes(m, n, 0, FP64, 0, 0, 0)
    bf = lib.geninv_workspace_bytes(m, n, 0, BF16, 4, 4, 0)
    i8 = lib.geninv_workspace_bytes(m, n, 0, INT8, 16, 16, 0)
    assert bf >= base + 2 * 4 * m * n
    assert i8 >= base + 16 * m * n
    # the Newton-Schulz steps work in the float64 slots
    assert lib.geninv_workspace_bytes(m, n, 0, INT8, 16, 16, 2) == i8
    # invalid digits or precision
    assert lib.geninv_workspace_bytes(m, n, 0, BF16, 5, 4, 0) == 0
    assert lib.geninv_workspace_bytes(m, n, 0, INT8, 17, 16, 0) == 0
    assert lib.geninv_workspace_bytes(m, n, 0, 7, 4, 4, 0) == 0


def test_python_api_refuses_cpu_tensors():
    torch = pytest.importorskip("torch")
    from paper_0804_4809_amd import api
    with pytest.raises(ValueError, match="GPU"):
        api.geninv(torch.zeros((4, 3), dtype=torch.float64))
    with pytest.raises(ValueError, match="GPU"):
        api.lstsq(torch.zeros((4, 3), dtype=torch.float64), torch.zeros((4, 1), dtype=torch.float64))


def test_batched_python_api_checks_shapes_before_touching_a_device():
    pytest.importorskip("torch")
    import numpy as np
    from paper_0804_4809_amd import api
    G = np.zeros((6, 3), np.float32)
    with pytest.raises(ValueError, match="differ in length"):
        api.lstsq_batched([G, G], [np.zeros((6, 2), np.float32)])
    with pytest.raises(ValueError, match="same number of columns"):
        api.lstsq_batched([G, G], [np.zeros((6, 2), np.float32), np.zeros((6, 3), np.float32)])
