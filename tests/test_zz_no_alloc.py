"""The allocation-free checksum entry point (lb_field_sum_noalloc) against the checksum
of lb_fields (the existing entry point, same kernels over a context's workspace), through
the C ABI: bit-identical sums on two calls in a row, the second on a smaller field, in
FP32 and FP64; and its argument checks."""
import ctypes as C

import numpy as np
import pytest

from paper_1310_4218_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield


def _noalloc(field_dev, precision_code):
    from paper_1310_4218_amd import _abi
    out = torch.zeros(1, dtype=torch.float64, device=field_dev.device)
    s = torch.cuda.current_stream(field_dev.device)
    rc = _abi.lib().lb_field_sum_noalloc(C.c_void_p(field_dev.data_ptr()), precision_code,
                                         field_dev.numel(), C.c_void_p(out.data_ptr()),
                                         C.c_void_p(s.cuda_stream))
    _abi.check(rc)
    torch.cuda.synchronize()
    return float(out.item())


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_noalloc_sum_matches_lb_fields_twice(precision):
    from paper_1310_4218_amd import _abi
    from paper_1310_4218_amd.grid import Grid
    code = _abi.LB_FP64 if precision == "fp64" else _abi.LB_FP32
    big = W.moving()                                           # 256 x 256 x 64
    small = W.small()                                          # 64 x 64 x 32, a smaller input
    for wl, steps in ((big, 3), (small, 2)):
        g = Grid(wl, precision=precision)
        g.step(steps)
        want = g.checksum()
        got = _noalloc(g.field(device="cuda").reshape(-1), code)
        assert got == want, (wl.name, got, want)
        g.close()


def test_noalloc_sum_argument_checks():
    from paper_1310_4218_amd import _abi
    L = _abi.lib()
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    q = torch.ones(10, dtype=torch.float32, device="cuda")
    assert L.lb_field_sum_noalloc(None, _abi.LB_FP32, 10, C.c_void_p(out.data_ptr()), None) == _abi.LB_E_INVAL
    assert L.lb_field_sum_noalloc(C.c_void_p(q.data_ptr()), _abi.LB_FP32, 10, None, None) == _abi.LB_E_INVAL
    assert L.lb_field_sum_noalloc(C.c_void_p(q.data_ptr()), 7, 10, C.c_void_p(out.data_ptr()), None) == _abi.LB_E_INVAL
    assert L.lb_field_sum_noalloc(C.c_void_p(q.data_ptr()), _abi.LB_FP32, -1, C.c_void_p(out.data_ptr()),
                                  None) == _abi.LB_E_INVAL
    assert L.lb_field_sum_noalloc(C.c_void_p(q.data_ptr()), _abi.LB_FP32, (1 << 40) + 1,
                                  C.c_void_p(out.data_ptr()), None) == _abi.LB_E_INVAL
    assert b"LB_NOALLOC_MAX_CELLS" in L.lb_last_error(None)
    # an empty field sums to zero
    assert L.lb_field_sum_noalloc(None, _abi.LB_FP64, 0, C.c_void_p(out.data_ptr()), None) == _abi.LB_OK
    torch.cuda.synchronize()
    assert float(out.item()) == 0.0
    # ten ones: exactly ten
    assert L.lb_field_sum_noalloc(C.c_void_p(q.data_ptr()), _abi.LB_FP32, 10, C.c_void_p(out.data_ptr()),
                                  None) == _abi.LB_OK
    torch.cuda.synchronize()
    assert float(out.item()) == 10.0
