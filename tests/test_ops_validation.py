"""Host-side validation in the torch wrappers: bad operands are refused with
ValueError before any pointer reaches the C ABI (no kernel is launched).

The wrappers are exercised without a device plan: the checks run before the
plan handle is used, so a plan object with only its sizes set suffices."""
import pytest
import torch

from paper_2103_06393_amd import ops


def _bare_plan(m=5, rows=24):
    P = object.__new__(ops.TuckerPlan)
    P.handle, P.m, P.rows, P._ws = 0, m, rows, {}
    return P


@pytest.mark.parametrize("x", [
    torch.zeros(5, dtype=torch.complex64),            # host memory
    torch.zeros(5, dtype=torch.complex128),           # wrong dtype
    torch.zeros(5, dtype=torch.float32),
    torch.zeros(4, dtype=torch.complex64),            # wrong length
    torch.zeros(5, 0, dtype=torch.complex64),
    torch.zeros(2, 5, 3, dtype=torch.complex64),
])
def test_matvec_refuses_bad_operands(x):
    with pytest.raises(ValueError):
        _bare_plan().matvec(x)


@pytest.mark.parametrize("y", [
    torch.zeros(24, dtype=torch.complex64),
    torch.zeros(24, dtype=torch.float32),
    torch.zeros(23, dtype=torch.complex64),
])
def test_rmatvec_refuses_bad_operands(y):
    with pytest.raises(ValueError):
        _bare_plan().rmatvec(y)


def test_out_buffer_shape_and_layout():
    dev = torch.device("cpu")
    ok = torch.zeros(3, 24, dtype=torch.complex64)
    assert ops._check_out(ok, 3, 24, dev).shape == (3, 24)
    colmajor = torch.zeros(3, 24, dtype=torch.complex64).t()
    assert ops._check_out(colmajor, 3, 24, dev).data_ptr() == colmajor.data_ptr()
    for bad in (torch.zeros(3, 23, dtype=torch.complex64),          # too small
                torch.zeros(24, 3, dtype=torch.complex64),          # row-major (rows, p)
                torch.zeros(3, 24, dtype=torch.complex128),
                torch.zeros(6, 24, dtype=torch.complex64)[::2]):   # strided
        with pytest.raises(ValueError):
            ops._check_out(bad, 3, 24, dev)
