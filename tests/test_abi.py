"""The C-ABI library loads and exports every function its header declares (no GPU)."""
import ctypes
import os
import re
import types

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"^\s*(?:[\w\s\*]+?)\b(knnj_\w+)\s*\(", txt, flags=re.M))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("knnj_build_index", "knnj_join", "knnj_join_bf", "knnj_index_free", "knnj_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1011_2807_amd import knnj
    lib = ctypes.CDLL(knnj.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_loads():
    import paper_1011_2807_amd as kj
    lib = kj.load_library()
    assert lib.knnj_last_error() == b""


def test_binding_rejects_bad_arrays_before_any_call():
    """Arrays the kernels would read or write out of bounds are refused on the
    host: wrong dtype, non-contiguous, host memory, or too few elements."""
    import pytest
    import torch
    import paper_1011_2807_amd as kj
    from paper_1011_2807_amd import knnj
    ok = torch.zeros(6, dtype=torch.int32)
    with pytest.raises(TypeError):
        knnj._require(ok.to(torch.int64), "x", torch.int32, 6)
    with pytest.raises(TypeError):
        knnj._require(torch.zeros(12, dtype=torch.int32)[::2], "x", torch.int32, 6)
    with pytest.raises(ValueError):          # host tensor: not on the HIP device
        knnj._require(ok, "x", torch.int32, 6)
    with pytest.raises(ValueError):
        kj.knn_join(types.SimpleNamespace(dtype=knnj.KNNJ_U8, _h=None), kj.DeviceCSR(torch.zeros(2, dtype=torch.int64), torch.zeros(1, dtype=torch.int32),
                                       torch.ones(1, dtype=torch.uint8), 4), 2,
                    out=(ok, ok, ok))
    with pytest.raises(TypeError):
        kj.DeviceCSR(torch.zeros(2, dtype=torch.int64), torch.zeros(1, dtype=torch.int32),
                     torch.ones(1, dtype=torch.int16), 4)._c()
    assert knnj._require(None, "x", torch.int32, 6) is None


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU; asking for more ends with a message (before any
    device work)."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_host_csr_checks_without_a_device():
    """HostCSR (the blocked join's S) keeps host arrays as they are and refuses
    wrong dtypes or mismatched sizes before any library call."""
    import numpy as np
    import pytest
    import synth
    from paper_1011_2807_amd import knnj
    m = synth.draw(3, 20, 50, (1, 10))
    h = knnj.HostCSR(m, pin=False)
    assert h.n_rows == 20 and h.n_dims == 50 and int(h.indices.numel()) == m.nnz
    c = h._c()
    assert c.n_rows == 20 and c.nnz == m.nnz and c.dtype == knnj.KNNJ_U8
    bad = synth.CSR(m.indptr.astype(np.int32), m.indices, m.values, 50)
    with pytest.raises(TypeError):
        knnj.HostCSR(bad, pin=False)
    short = synth.CSR(m.indptr, m.indices, m.values[:-1], 50)
    with pytest.raises(ValueError):
        knnj.HostCSR(short, pin=False)


def test_autotune_cache_key_names_the_candidate_set():
    """A cached tuning result is reused only for the same candidates (any order)."""
    from paper_1011_2807_amd import autotune
    a = autotune.candidates_key((2048, 4096), (0, 128), (0, 4), (2, 4))
    assert a == autotune.candidates_key((4096, 2048), (128, 0), (4, 0), (4, 2))
    assert a != autotune.candidates_key((2048,), (0, 128), (0, 4), (2, 4))
    assert a != autotune.candidates_key((2048, 4096), (0, 128), (0, 4, 8), (2, 4))
