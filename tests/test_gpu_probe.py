"""The bandwidth probe's triad against numpy (s = 2 makes the fused and the
separately rounded forms identical)."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n", [1, 2, 7, 4096, 100003])
def test_stream_triad(cuda, n):
    import torch

    from paper_1107_0538_amd import capi

    rng = np.random.default_rng(n)
    a, b = rng.uniform(-1, 1, n), rng.uniform(-1, 1, n)
    A, B = torch.as_tensor(a, device=cuda), torch.as_tensor(b, device=cuda)
    C = torch.empty_like(A)
    st = torch.cuda.current_stream()
    assert capi.load().jpcg_stream_triad(A.data_ptr(), B.data_ptr(), C.data_ptr(), 2.0, n, 0,
                                         ctypes.c_void_p(st.cuda_stream)) == 0
    assert np.array_equal(C.cpu().numpy(), a + 2.0 * b)
    # Misaligned pointers are refused before any launch.
    assert capi.load().jpcg_stream_triad(A.data_ptr() + 8, B.data_ptr(), C.data_ptr(), 2.0, max(n - 1, 0), 0,
                                         ctypes.c_void_p(st.cuda_stream)) == -1
