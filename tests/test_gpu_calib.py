"""The reference kernels for the traffic counters (bh_calib_copy) move the
bytes they claim: the vector copy reproduces its source, the scalar read
sums every 64-byte block once."""

import ctypes

import numpy as np
import pytest

from gpu_util import cuda_device, say

pytestmark = pytest.mark.gpu


def test_calib_kernels():
    import torch
    from paper_2509_01180_amd._lib import (BH_CALIB_COPY_VECTOR, BH_CALIB_READ_GROUPS,
                                           BH_CALIB_READ_SCALAR, BhError, check, lib)
    dev = cuda_device()
    say("calibration kernels")
    n = (3 << 20) + 16                    # doubles: not a multiple of the groups
    src = torch.arange(n, dtype=torch.float64, device=dev)
    dst = torch.zeros_like(src)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    check(lib().bh_calib_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                              n * 8, BH_CALIB_COPY_VECTOR, st), "bh_calib_copy")
    torch.cuda.synchronize()
    assert torch.equal(dst, src)
    sums = torch.zeros(BH_CALIB_READ_GROUPS, dtype=torch.float64, device=dev)
    check(lib().bh_calib_copy(ctypes.c_void_p(sums.data_ptr()), ctypes.c_void_p(src.data_ptr()),
                              n * 8, BH_CALIB_READ_SCALAR, st), "bh_calib_copy")
    torch.cuda.synchronize()
    assert float(sums.sum()) == float(n) * (n - 1) / 2     # exact: integers below 2^53
    with pytest.raises(BhError):
        check(lib().bh_calib_copy(ctypes.c_void_p(dst.data_ptr()),
                                  ctypes.c_void_p(src.data_ptr()), 40, BH_CALIB_READ_SCALAR, st),
              "bh_calib_copy")
    with pytest.raises(BhError):
        check(lib().bh_calib_copy(ctypes.c_void_p(dst.data_ptr()),
                                  ctypes.c_void_p(src.data_ptr()), 64, 7, st), "bh_calib_copy")
