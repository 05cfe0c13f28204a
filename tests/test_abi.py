"""The C-ABI library loads and exports every entry point its header declares (no GPU needed),
and the Python binding refuses to run without the built library (no CPU fallback)."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "logdet_cheb.h")


def _declared() -> list:
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ld_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def built_lib():
    import paper_1503_06394_amd as pkg

    if not os.path.exists(pkg.LIB_PATH):
        from paper_1503_06394_amd.build import build

        build()
    return ctypes.CDLL(pkg.LIB_PATH)


def test_header_declares_the_boundary():
    names = _declared()
    for expected in ("ld_logdet_cheb", "ld_logabsdet_cheb", "ld_logdet_cheb_grad", "ld_logdet_cheb_batched",
                     "ld_gershgorin", "ld_probes", "ld_transpose", "ld_workspace_bytes", "ld_last_error"):
        assert expected in names


def test_library_exports_every_declared_symbol(built_lib):
    for name in _declared():
        assert hasattr(built_lib, name), name


def test_version_and_error_string_without_gpu(built_lib):
    built_lib.ld_version.restype = ctypes.c_char_p
    assert b"gfx950" in built_lib.ld_version()
    built_lib.ld_last_error.restype = ctypes.c_char_p
    assert isinstance(built_lib.ld_last_error(), bytes)


def test_argument_validation_happens_before_any_device_work(built_lib):
    """Invalid arguments are rejected on the host (no HIP call is made for them)."""
    import paper_1503_06394_amd as pkg

    L = pkg.lib()
    c = pkg._CSR(4, 5, 0, None, None, None, 1, 0, 0.0)  # not square
    r = pkg._Result()
    assert L.ld_logdet_cheb(ctypes.byref(c), 0.1, 1.0, 3, 2, 0, None, None, ctypes.byref(r)) == -1
    assert b"square" in L.ld_last_error()
    c = pkg._CSR(0, 0, 0, None, None, None, 1, 0, 0.0)
    assert L.ld_logdet_cheb(ctypes.byref(c), 1.0, 0.5, 3, 2, 0, None, None, ctypes.byref(r)) == -1  # a >= b
    assert L.ld_logdet_cheb(ctypes.byref(c), 0.1, 1.0, -1, 2, 0, None, None, ctypes.byref(r)) == -1  # n < 0
    assert L.ld_logdet_cheb(ctypes.byref(c), 0.1, 1.0, 3, 0, 0, None, None, ctypes.byref(r)) == -1  # M < 1
    c = pkg._CSR(0, 0, 0, None, None, None, 7, 0, 0.0)
    assert L.ld_logdet_cheb(ctypes.byref(c), 0.1, 1.0, 3, 2, 0, None, None, ctypes.byref(r)) == -2  # dtype
    assert L.ld_logdet_cheb_batched(0, None, None, None, None, 4, 0, None, None, None) == -1
    assert L.ld_logdet_cheb_grad(None, 0.1, 1.0, 3, 2, 0, 1.0, None, 0, None, None, ctypes.byref(r)) == -1


def test_workspace_size_is_positive_and_grows_with_degree(built_lib):
    import paper_1503_06394_amd as pkg

    L = pkg.lib()
    c = pkg._CSR(1000, 1000, 5000, None, None, None, 1, 0, 0.0)
    w1 = L.ld_workspace_bytes(ctypes.byref(c), 10, 32, 0, 0)
    w2 = L.ld_workspace_bytes(ctypes.byref(c), 100, 32, 0, 0)
    wg = L.ld_workspace_bytes(ctypes.byref(c), 100, 32, 2, 0)
    assert 0 < w1 < w2 < wg
    assert w1 >= 2 * 1000 * 32 * 4


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    import paper_1503_06394_amd as pkg

    monkeypatch.setattr(pkg, "_lib", None)
    monkeypatch.setattr(pkg, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(pkg.LogdetChebError):
        pkg.lib()


def test_product_package_does_not_import_the_oracle():
    src_dir = os.path.join(ROOT, "paper_1503_06394_amd")
    for dirpath, _, files in os.walk(src_dir):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text and "ldo_" not in text, f


def test_noalloc_refusals_happen_on_the_host(built_lib):
    """ld_logdet_cheb_noalloc refuses a caller workspace (LD_EINVAL) and a problem beyond its fixed
    scratch array (LD_EWORKSPACE) before any HIP call; the array pointers here are never read."""
    import paper_1503_06394_amd as pkg

    L = pkg.lib()
    r = pkg._Result()
    fake = 0x1000
    big = pkg._CSR(1_000_000, 1_000_000, 5_000_000, fake, fake, fake, 1, 0, 0.0)
    assert L.ld_logdet_cheb_noalloc(ctypes.byref(big), 0.5, 2.0, 10, 64, 0, None, None, ctypes.byref(r)) == -3
    assert b"scratch" in L.ld_last_error()
    o = pkg._Opts()
    o.workspace = fake
    o.workspace_bytes = 1 << 20
    small = pkg._CSR(100, 100, 100, fake, fake, fake, 1, 0, 0.0)
    assert L.ld_logdet_cheb_noalloc(ctypes.byref(small), 0.5, 2.0, 10, 8, 0, ctypes.byref(o), None,
                                    ctypes.byref(r)) == -1
    assert b"workspace" in L.ld_last_error()
