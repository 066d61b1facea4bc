"""Host-side behaviour that needs no GPU: the benchmark's one-GPU contract, and the library's
entry points failing cleanly (a status, no crash) where no device exists."""
import ctypes
import os
import subprocess
import sys

import pytest

from paper_2011_02107_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no benchmark line


def _no_gpu():
    import torch

    return not torch.cuda.is_available()


@pytest.mark.skipif(not _no_gpu(), reason="checks the behaviour on a machine without a GPU")
def test_create_without_a_device_returns_invalid():
    lib = binding.load_library()
    h = ctypes.c_void_p()
    st = lib.dacp_create(0, None, ctypes.byref(h))
    assert st == -1  # DACP_E_INVALID: no such device
    assert not h.value


def test_null_arguments_are_rejected_without_a_device():
    lib = binding.load_library()
    assert lib.dacp_create(0, None, None) == -1
    assert lib.dacp_last_error(None).decode() == "null context"
    lib.dacp_destroy(None)  # a no-op
