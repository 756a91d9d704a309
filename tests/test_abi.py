"""The C-ABI library loads and exports every symbol include/qs.h declares
(no compute calls: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    src = open(os.path.join(ROOT, "include", "qs.h")).read()
    return sorted(set(re.findall(r"^\s*(?:qs_status|const char\*)\s+(qs_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    syms = header_symbols()
    for name in ("qs_alloc", "qs_apply_layer", "qs_expect", "qs_adjoint_grad", "qs_plan_create",
                 "qs_apply_gates", "qs_batch_run", "qs_infidelity"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    from paper_2609_19147_amd import _lib
    lib = _lib.lib()
    missing = [s for s in header_symbols() if not hasattr(lib, s)]
    assert not missing, missing
    assert sorted(_lib.EXPORTED) == header_symbols()


def test_version_and_error_message():
    from paper_2609_19147_amd import _lib
    lib = _lib.lib()
    assert b"gfx950" in lib.qs_version()
    h = ctypes.c_void_p()
    rc = lib.qs_plan_create(0, None, 0, 0, None, ctypes.byref(h))
    assert rc == _lib.QS_EINVAL
    assert b"qubit count" in lib.qs_last_error()


def test_null_arguments_are_rejected_without_a_device():
    from paper_2609_19147_amd import _lib
    lib = _lib.lib()
    assert lib.qs_norm2(None, None) == _lib.QS_EINVAL
    assert lib.qs_apply_layer(None, None, 0, 0) == _lib.QS_EINVAL
    assert lib.qs_alloc(40, 0, None, None, 0, None, ctypes.byref(ctypes.c_void_p())) == _lib.QS_EINVAL
    assert lib.qs_alloc(4, 7, None, None, 0, None, ctypes.byref(ctypes.c_void_p())) == _lib.QS_EINVAL


def test_extension_missing_fails_loudly(monkeypatch, tmp_path):
    from paper_2609_19147_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "nope.so"))
    with pytest.raises(ImportError):
        _lib.lib()


def test_max_bytes_cap_refuses_before_any_device_call():
    # a fresh process with QS_MAX_BYTES set: a state above the cap fails with
    # QS_ENOMEM and names the cap, with no device present
    import subprocess
    import sys
    code = (
        "import ctypes\n"
        "from paper_2609_19147_amd import _lib\n"
        "lib = _lib.lib()\n"
        "h = ctypes.c_void_p()\n"
        "rc = lib.qs_alloc(20, _lib.QS_C64, None, None, 0, None, ctypes.byref(h))\n"
        "held, cap = ctypes.c_size_t(), ctypes.c_size_t()\n"
        "assert lib.qs_memory_info(ctypes.byref(held), ctypes.byref(cap)) == 0\n"
        "print(rc, cap.value, held.value, lib.qs_last_error().decode())\n"
    )
    env = dict(os.environ, QS_MAX_BYTES="4096")
    out = subprocess.run([sys.executable, "-c", code], env=env, cwd=ROOT, capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr[-2000:]
    rc, cap, held, msg = out.stdout.strip().split(" ", 3)
    from paper_2609_19147_amd import _lib
    assert int(rc) == _lib.QS_ENOMEM
    assert int(cap) == 4096 and int(held) == 0
    assert "QS_MAX_BYTES" in msg
