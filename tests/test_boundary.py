"""CPU checks of the C-ABI boundary: the library loads, exports every symbol that
include/fpca.h declares, and rejects bad arguments synchronously (no GPU needed:
these paths return before any device work)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fpca.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fpca_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_abi():
    syms = declared_symbols()
    for s in ("fpca_bin", "fpca_smooth_mean", "fpca_smooth_cov", "fpca_eig_randomized", "fpca_create",
              "fpca_destroy", "fpca_set_stream", "fpca_sync", "fpca_last_error"):
        assert s in syms


def test_library_exports_every_declared_symbol():
    import paper_1510_04439_amd as F
    lib = F.load_library()
    for s in declared_symbols():
        assert hasattr(lib, s), s
    assert sorted(F.EXPORTED_SYMBOLS) == sorted(declared_symbols())


def test_null_handle_and_bad_arguments_rejected():
    import paper_1510_04439_amd as F
    from paper_1510_04439_amd._binding import _GridC
    lib = F.load_library()
    g = _GridC()
    g.d = 2
    g.M[0], g.M[1], g.M[2] = 8, 8, 1
    rc = lib.fpca_bin(None, ctypes.byref(g), 0, 0, 1, 1, 1, None, None, None, None, 0, None, None, None,
                      None, None)
    assert rc == F.FPCA_ERR_INVALID_ARG
    assert b"handle" in lib.fpca_last_error()
    bw = (ctypes.c_double * 2)(0.1, 0.1)
    assert lib.fpca_smooth_mean(None, ctypes.byref(g), 1, None, None, 0, bw, None, None) == F.FPCA_ERR_INVALID_ARG
    ev = (ctypes.c_double * 2)()
    assert lib.fpca_eig_randomized(None, 1, 1, ctypes.byref(g), None, None, 2, 2, 1, 7, ev, None, None) \
        == F.FPCA_ERR_INVALID_ARG


def test_create_without_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import paper_1510_04439_amd as F
    with pytest.raises(F.FpcaError) as e:
        F.Handle(0)
    assert e.value.code in (F.FPCA_ERR_DEVICE, F.FPCA_ERR_INVALID_ARG)


def test_noise_pace_reconstruct_reject_null_handle():
    import paper_1510_04439_amd as F
    from paper_1510_04439_amd._binding import _GridC
    lib = F.load_library()
    g = _GridC()
    g.d = 1
    g.M[0], g.M[1], g.M[2] = 9, 1, 1
    s2 = ctypes.c_double()
    cnt = ctypes.c_int64()
    assert lib.fpca_noise_variance(None, ctypes.byref(g), 1, None, None, None, None, ctypes.byref(s2),
                                   ctypes.byref(cnt)) == F.FPCA_ERR_INVALID_ARG
    ev = (ctypes.c_double * 2)(1.0, 0.5)
    assert lib.fpca_pace_scores(None, ctypes.byref(g), 1, 1, 2, None, None, None, None, None, 2, ev, 0.1,
                                None) == F.FPCA_ERR_INVALID_ARG
    assert lib.fpca_reconstruct(None, 1, 9, 2, 2, None, None, None, None) == F.FPCA_ERR_INVALID_ARG
    assert b"handle" in lib.fpca_last_error()


def test_bench_refuses_more_than_one_gpu():
    import json
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]
