"""Host-side contracts of the package and the benchmark (no GPU needed): the
library loader fails loudly when the HIP library is missing (there is no CPU
fallback), the benchmark refuses more than one GPU with a message, and every
signature the binding declares names an exported symbol."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_loader_fails_loudly_without_the_library(tmp_path):
    from paper_2203_11875_amd import _abi
    with pytest.raises(ImportError, match="missing"):
        _abi.load(str(tmp_path / "librhipm.so"))


def test_bench_refuses_several_gpus():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, cwd=ROOT, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout.strip() == ""


def test_every_bound_signature_is_exported():
    from paper_2203_11875_amd import _abi
    lib = _abi.load()
    assert len(_abi.SIGNATURES) > 40
    for name in _abi.SIGNATURES:
        assert hasattr(lib, name), name


def test_noalloc_solve_rejects_bad_arguments_before_any_device_work():
    """rh_cholesky_solve_noalloc checks its arguments on the host: orders past
    its static workspace (1024), a negative shift or a missing status word
    return RH_ERR_ARG without touching the device (the pointers are never
    dereferenced)."""
    import ctypes as C
    from paper_2203_11875_amd import _abi
    lib = _abi.load()
    f = lib.rh_cholesky_solve_noalloc
    dummy = C.c_void_p(0x1000)
    assert f(dummy, 1025, 1025, 0.0, dummy, dummy, dummy, None) == _abi.RH_ERR_ARG
    assert f(dummy, 8, 8, -1.0, dummy, dummy, dummy, None) == _abi.RH_ERR_ARG
    assert f(dummy, 8, 8, 0.0, dummy, dummy, None, None) == _abi.RH_ERR_ARG
    assert f(dummy, 4, 8, 0.0, dummy, dummy, dummy, None) == _abi.RH_ERR_ARG   # ldk < n
