"""The C ABI library loads, exports every function include/passjoin.h declares, and rejects
invalid host inputs before any device work (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1111_7171_amd as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "passjoin.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pj_[a-z_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = _declared()
    for need in ("pj_self_join", "pj_join", "pj_build_index", "pj_query", "pj_pairs_free",
                 "pj_index_free", "pj_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol():
    lib = P.load()
    for name in _declared():
        assert hasattr(lib, name), name
        assert isinstance(getattr(lib, name), C._CFuncPtr)


def test_version_string():
    assert P.pj_version().startswith("passjoin")


def _err(fn, *a, **k):
    with pytest.raises(P.PassJoinError) as ei:
        fn(*a, **k)
    return ei.value.code


def test_invalid_inputs_rejected_on_host():
    ok = (np.frombuffer(b"abcabc", np.uint8), np.array([0, 3, 6], np.int32))
    assert _err(P.pj_self_join, ok, -1) == P.PJ_EINVAL
    assert _err(P.pj_self_join, ok, 64) == P.PJ_EINVAL
    assert _err(P.pj_self_join, (ok[0], np.array([1, 3, 6], np.int32)), 1) == P.PJ_EINVAL
    assert _err(P.pj_self_join, (ok[0], np.array([0, 4, 3], np.int32)), 1) == P.PJ_EINVAL
    long = np.zeros(2048, np.uint8)
    assert _err(P.pj_self_join, (long, np.array([0, 2048], np.int32)), 1) == P.PJ_ERANGE
    assert _err(P.pj_join, ok, (ok[0], np.array([0, 5, 3], np.int32)), 1) == P.PJ_EINVAL
    assert "offsets" in P.pj_last_error()
    # streamed self-join: positive window, host strings
    assert _err(P.pj_self_join_streamed, ok, 1, 0) == P.PJ_EINVAL
    assert _err(P.pj_self_join_streamed, ok, 64, 100) == P.PJ_EINVAL
    assert _err(P.pj_self_join_streamed, (ok[0], np.array([0, 4, 3], np.int32)), 1, 100) \
        == P.PJ_EINVAL
    # an empty set has no length window: no device work, no pairs
    got = P.pj_self_join_streamed((np.zeros(0, np.uint8), np.zeros(1, np.int32)), 2, 100)
    assert got.shape == (0, 2)
    assert P.pj_last_stats()["pairs"] == 0
    # substring-selection method outside PJ_SELECT_*
    assert _err(P.pj_self_join, ok, 1, selection=4) == P.PJ_EINVAL
    assert _err(P.pj_join, ok, ok, 1, selection=-1) == P.PJ_EINVAL
    assert "selection" in P.pj_last_error()


def test_null_arguments_rejected():
    lib = P.load()
    assert lib.pj_self_join(None, 1, None, None) == P.PJ_EINVAL
    raw = P.PjPairs()
    assert lib.pj_self_join(None, 1, None, C.byref(raw)) == P.PJ_EINVAL
    assert raw.count == 0 and not raw.a
    h = C.c_void_p()
    s = P.PjStrings(0, None, None)
    assert lib.pj_build_index(C.byref(s), 3, 2, None, C.byref(h)) == P.PJ_EINVAL
    assert not h.value
    assert lib.pj_query(None, C.byref(s), None, None, C.byref(raw)) == P.PJ_EINVAL
    assert lib.pj_index_info(None, None, None, None, None) == P.PJ_EINVAL
    lib.pj_index_free(None)
    lib.pj_pairs_free(None)
    lib.pj_pairs_free(C.byref(raw))


def test_tune_rejects_invalid_arguments_on_host():
    lib = P.load()
    ok = (np.frombuffer(b"abcabc", np.uint8), np.array([0, 3, 6], np.int32))
    assert _err(P.pj_tune, ok, -1) == P.PJ_EINVAL
    assert _err(P.pj_tune, ok, 64) == P.PJ_EINVAL
    assert _err(P.pj_tune, (ok[0], np.array([0, 4, 3], np.int32)), 1) == P.PJ_EINVAL
    s = P.PjStrings(0, None, None)
    assert lib.pj_tune(C.byref(s), 1, None, None) == P.PJ_EINVAL
    o = P.PjOptions()
    o.inputs_on_device = 1
    r = P.PjTuneResult()
    assert lib.pj_tune(C.byref(s), 1, C.byref(o), C.byref(r)) == P.PJ_EINVAL
    assert "host" in P.pj_last_error()


def test_device_flag_with_host_pointers_rejected():
    """inputs_on_device = 1 with host arrays: the library checks every pointer before a kernel
    reads it, so host memory (or, without a GPU, any pointer) is refused, never dereferenced."""
    lib = P.load()
    chars = np.frombuffer(b"abcabc", np.uint8).copy()
    offs = np.array([0, 3, 6], np.int32)
    s = P.PjStrings(2, chars.ctypes.data, offs.ctypes.data)
    o = P.PjOptions()
    o.inputs_on_device = 1
    raw = P.PjPairs()
    rc = lib.pj_self_join(C.byref(s), 1, C.byref(o), C.byref(raw))
    assert rc in (P.PJ_EINVAL, P.PJ_EDEVICE) and raw.count == 0 and not raw.a
    rc = lib.pj_join(C.byref(s), C.byref(s), 1, C.byref(o), C.byref(raw))
    assert rc in (P.PJ_EINVAL, P.PJ_EDEVICE) and raw.count == 0


def test_binding_rejects_mixed_host_and_device_arrays():
    """The binding refuses a set whose two arrays are not both device tensors (checked before
    any library call; torch CPU tensors stand in for a mismatched pair here)."""
    import torch

    class FakeDev:
        """A CPU tensor claiming to be on a device: the check must not trust one array alone."""
        __module__ = "torch"

        def __init__(self, t):
            self.t = t
            self.is_cuda = True

    chars = torch.from_numpy(np.frombuffer(b"abcabc", np.uint8).copy())
    offs = torch.tensor([0, 3, 6], dtype=torch.int32)
    assert _err(P.pj_self_join, (chars, FakeDev(offs)), 1) == P.PJ_EINVAL


def test_plan_rejects_host_strings_and_null_arguments():
    """pj_self_join_plan takes device strings only (refused before any device work) and checks
    its pointer arguments; pj_plan_run and pj_plan_free accept no plan / a null plan."""
    lib = P.load()
    chars = np.frombuffer(b"abcabc", np.uint8).copy()
    offs = np.array([0, 3, 6], np.int32)
    s = P.PjStrings(2, chars.ctypes.data, offs.ctypes.data)
    h = C.c_void_p()
    assert lib.pj_self_join_plan(C.byref(s), 1, None, C.byref(h)) == P.PJ_EINVAL
    assert not h.value
    o = P.PjOptions()
    assert lib.pj_self_join_plan(C.byref(s), 1, C.byref(o), C.byref(h)) == P.PJ_EINVAL
    assert "device" in P.pj_last_error() and not h.value
    assert lib.pj_self_join_plan(C.byref(s), 1, C.byref(o), None) == P.PJ_EINVAL
    assert lib.pj_self_join_plan(None, 1, C.byref(o), C.byref(h)) == P.PJ_EINVAL
    raw = P.PjPairs()
    assert lib.pj_plan_run(None, C.byref(raw)) == P.PJ_EINVAL and raw.count == 0
    lib.pj_plan_free(None)
    with pytest.raises(P.PassJoinError):
        P.Plan((chars, offs), 1)
