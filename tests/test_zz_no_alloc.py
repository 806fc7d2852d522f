"""dt_triangulate_noalloc (no allocation, static scratch array) against
dt_triangulate with k = 1, through the C-ABI: bit-identical simplex sets on
two calls in a row, the second smaller, at the largest sizes the scratch
array admits, with the FP32 filter, and the error paths."""
import ctypes

import numpy as np
import pytest

import oracle
from paper_1902_07554_amd import inputs

pytestmark = pytest.mark.gpu


def _ref(dtlib, p, **opts):
    return oracle.canonical(dtlib.triangulate(p, k=1, **opts).rows())


def _noalloc(dtlib, p, **opts):
    import torch
    rows = dtlib.triangulate_noalloc(torch.from_numpy(p).cuda(), **opts)
    return oracle.canonical(rows.cpu().numpy())


@pytest.mark.parametrize("dim,first,second", [(3, ("bubbles", 40_000), ("uniform", 6_000)),
                                              (2, ("normal", 100_000), ("uniform", 2_500))])
def test_two_calls_second_smaller(dtlib, dim, first, second):
    for dist, n in (first, second):
        p = inputs.make(dist, n, dim, seed=n)
        print(f"[noalloc] {dim}d {dist} n={n}", flush=True)
        got = _noalloc(dtlib, p)
        assert np.array_equal(got, _ref(dtlib, p)), (dim, dist, n)


@pytest.mark.parametrize("dim", [2, 3])
def test_largest_admitted_size_and_fp32(dtlib, dim):
    n = dtlib.NOALLOC_MAX_POINTS[dim]
    p = inputs.make("bubbles" if dim == 3 else "normal", n, dim, seed=4)
    print(f"[noalloc] {dim}d n={n} (maximum), fp32", flush=True)
    got = _noalloc(dtlib, p, precision="fp32")
    assert np.array_equal(got, _ref(dtlib, p, precision="fp32"))
    small = inputs.lattice(7 if dim == 3 else 20, dim, seed=2)   # ties, after the large call
    assert np.array_equal(_noalloc(dtlib, small), _ref(dtlib, small))


def test_no_device_memory_taken(dtlib):
    """After a first call (which may load the library's code onto the
    GPU), a call leaves the device's free memory unchanged."""
    import torch
    p = torch.from_numpy(inputs.make("uniform", 20_000, 3, seed=1)).cuda()
    out = torch.empty((200_000, 4), dtype=torch.int32, device="cuda")
    dtlib.triangulate_noalloc(p, out=out)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    rows = dtlib.triangulate_noalloc(p, out=out)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert len(rows) > 0


def test_error_paths(dtlib):
    import torch
    lib = dtlib.load()
    n3 = dtlib.NOALLOC_MAX_POINTS[3] + 1
    big = torch.from_numpy(inputs.make("uniform", n3, 3, seed=1)).cuda()
    with pytest.raises(dtlib.DTError) as e:
        dtlib.triangulate_noalloc(big)
    assert e.value.status == dtlib.DT_E_NOMEM
    p = torch.from_numpy(inputs.make("uniform", 500, 3, seed=1)).cuda()
    with pytest.raises(dtlib.DTError) as e:
        dtlib.triangulate_noalloc(p, sort_output=1)
    assert e.value.status == dtlib.DT_E_INVALID_ARG
    # too small an output: the count says how many rows are needed
    out = torch.empty((10, 4), dtype=torch.int32, device="cuda")
    cnt = ctypes.c_int64(0)
    st = lib.dt_triangulate_noalloc(ctypes.c_void_p(p.data_ptr()), 500, 3, None,
                                    ctypes.c_void_p(out.data_ptr()), 10, ctypes.byref(cnt), None)
    assert st == dtlib.DT_E_INVALID_ARG and cnt.value > 10
    rows = dtlib.triangulate_noalloc(p)
    assert len(rows) == cnt.value
    dup = inputs.make("uniform", 50, 2, seed=3)
    dup[7] = dup[3]
    with pytest.raises(dtlib.DTError) as e:
        dtlib.triangulate_noalloc(torch.from_numpy(dup).cuda())
    assert e.value.status == dtlib.DT_E_DUPLICATE
