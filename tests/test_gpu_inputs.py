"""Device inputs that must be refused with PJ_EINVAL before any kernel reads them: a host chars
array beside device offsets, a chars allocation shorter than offsets[n], NULL bytes with
offsets[n] > 0, host memory passed as device memory.  Each case is a host-side check (the
binding's or the library's), so no kernel ever runs on a bad pointer."""
import ctypes as C

import numpy as np
import pytest

import paper_1111_7171_amd as P

pytestmark = pytest.mark.gpu


def _err(fn, *a, **k):
    with pytest.raises(P.PassJoinError) as ei:
        fn(*a, **k)
    return ei.value.code


def test_bad_device_inputs_rejected():
    import torch
    offs_d = torch.tensor([0, 3, 6], dtype=torch.int32, device="cuda")
    chars_h = torch.from_numpy(np.frombuffer(b"abcabc", np.uint8).copy())
    # host chars beside device offsets (binding)
    assert _err(P.pj_self_join, (chars_h, offs_d), 1) == P.PJ_EINVAL
    # NULL, host and too-short pointers (library checks; lengths within PJ_LEN_MAX)
    lib = P.load()
    big_offs = torch.tensor([0, 2000], dtype=torch.int32, device="cuda")
    tiny = torch.empty(2, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    huge_offs = torch.tensor([0, 2047, 4094], dtype=torch.int32, device="cuda")
    o = P.PjOptions()
    o.inputs_on_device = 1
    o.hip_stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    raw = P.PjPairs()
    s = P.PjStrings(1, None, big_offs.data_ptr())                   # NULL bytes, offsets[1] > 0
    assert lib.pj_self_join(C.byref(s), 1, C.byref(o), C.byref(raw)) == P.PJ_EINVAL
    assert "null bytes" in P.pj_last_error()
    host_bytes = np.zeros(16, np.uint8)
    s = P.PjStrings(1, host_bytes.ctypes.data, big_offs.data_ptr())  # host bytes as device
    assert lib.pj_self_join(C.byref(s), 1, C.byref(o), C.byref(raw)) == P.PJ_EINVAL
    host_offs = np.array([0, 2], np.int32)
    s = P.PjStrings(1, tiny.data_ptr(), host_offs.ctypes.data)       # host offsets as device
    assert lib.pj_self_join(C.byref(s), 1, C.byref(o), C.byref(raw)) == P.PJ_EINVAL
    # a dedicated allocation (hipMalloc through the library's own runtime) of 64 bytes against
    # offsets[n] = 4094
    hip_malloc = lib.hipMalloc
    hip_malloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
    hip_free = lib.hipFree
    hip_free.argtypes = [C.c_void_p]
    p = C.c_void_p()
    assert hip_malloc(C.byref(p), 64) == 0
    try:
        s = P.PjStrings(2, p.value, huge_offs.data_ptr())
        assert lib.pj_self_join(C.byref(s), 1, C.byref(o), C.byref(raw)) == P.PJ_EINVAL
        assert "exceeds" in P.pj_last_error()
    finally:
        hip_free(p)
    assert raw.count == 0 and not raw.a
    # a valid call still works afterwards
    chars_d = torch.tensor(list(b"abcabd"), dtype=torch.uint8, device="cuda")
    got = P.pj_self_join((chars_d, offs_d), 1)
    assert got.tolist() == [[0, 1]]
