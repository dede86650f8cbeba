"""The C ABI library loads and exports every entry point its header declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tlmpm.h")
LIB = os.path.join(ROOT, "paper_2609_27342_amd", "libtlmpm.so")


def declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(tlmpm_[a-z_]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("tlmpm_create_scene", "tlmpm_assign_labels", "tlmpm_step", "tlmpm_read_state"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    for n in declared():
        assert hasattr(L, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_footprint_and_validation_without_gpu():
    from paper_2609_27342_amd import tlmpm, workloads as W
    s = W.small()
    nb = tlmpm.footprint(s)
    assert nb > s["X"].shape[0] * 100
    bad = dict(s, params=dict(s["params"], max_cuts=99))
    with pytest.raises(tlmpm.TlmpmError) as e:
        tlmpm.footprint(bad)
    assert e.value.code == tlmpm.E_INVALID


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_quadratic_stencil_validation_without_gpu():
    """The 27-node stencil needs half a cell of grid around every particle; other
    stencil values are refused."""
    from paper_2609_27342_amd import tlmpm, workloads as W
    s = W.small()
    q = dict(s, params=dict(s["params"], stencil=1))
    assert tlmpm.footprint(q) > tlmpm.footprint(s)
    X = s["X"].copy()
    X[0, 0] = s["params"]["origin"][0] + 0.3 * s["params"]["dx"]
    with pytest.raises(tlmpm.TlmpmError) as e:
        tlmpm.footprint(dict(q, X=X))
    assert e.value.code == tlmpm.E_INVALID
    tlmpm.footprint(dict(s, X=X))  # the trilinear stencil accepts it
    with pytest.raises(tlmpm.TlmpmError):
        tlmpm.footprint(dict(s, params=dict(s["params"], stencil=2)))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_batch_validation_without_gpu():
    """Empty or null member lists are refused before any device call."""
    L = ctypes.CDLL(LIB)
    nb = ctypes.c_size_t()
    assert L.tlmpm_batch_footprint(None, 0, ctypes.byref(nb)) == 1
    arr = (ctypes.c_void_p * 2)(None, None)
    assert L.tlmpm_batch_footprint(arr, 2, ctypes.byref(nb)) == 1
    out = ctypes.c_void_p()
    assert L.tlmpm_batch_create(None, 0, None, ctypes.c_size_t(0), None, ctypes.byref(out)) == 1
    assert L.tlmpm_batch_step(None, None, None, 1, None) == 1


def test_tuning_round_trip_and_validation_without_gpu():
    from paper_2609_27342_amd import tlmpm
    d = tlmpm.get_tuning()
    assert d == {"pair_div": 128, "pair_cap": 4096, "split_lo": 512, "split_hi": 4096, "split_div": 4,
                 "split_cap": 256, "one_stream_bricks": 2048, "pair_skip": 1}
    try:
        tlmpm.set_tuning(pair_div=64, split_cap=0)
        assert tlmpm.get_tuning() == dict(d, pair_div=64, split_cap=0)
        for bad in (dict(pair_div=0), dict(pair_cap=0), dict(split_lo=5000), dict(split_div=0), dict(split_cap=-1),
                    dict(one_stream_bricks=-1), dict(pair_skip=2)):
            with pytest.raises(tlmpm.TlmpmError):
                tlmpm.set_tuning(**bad)
        assert tlmpm.get_tuning() == dict(d, pair_div=64, split_cap=0)  # a refused setting changes nothing
        with pytest.raises(ValueError):
            tlmpm.set_tuning(lanes=4)
    finally:
        tlmpm.set_tuning(None)
    assert tlmpm.get_tuning() == d
