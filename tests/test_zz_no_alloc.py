"""The no-allocation Gram product, dense_gram_noalloc, called through the C ABI.

It shares dense_gram's kernels and chunking, so its result must be bitwise
dense_gram's.  The fixed scratch keeps the previous call's partials, so two
calls run back to back, the second on a smaller input; a request at the
scratch's exact capacity works and one chunk more is refused with
CG_ESCRATCH before any work is enqueued.
"""
import ctypes

import numpy as np
import pytest

from paper_1107_0538_amd import capi

pytestmark = pytest.mark.gpu


def _gram(name, A, B, C, stream):
    fn = getattr(capi.load(), name)
    return fn(A.data_ptr(), A.shape[0], A.shape[1], A.stride(0), B.data_ptr(), B.shape[1], B.stride(0),
              C.data_ptr(), ctypes.c_void_p(stream.cuda_stream))


def _both(A, B, stream):
    import torch

    C0 = torch.full((A.shape[1], B.shape[1]), float("nan"), dtype=torch.float64, device=A.device)
    C1 = C0.clone()
    assert _gram("dense_gram", A, B, C0, stream) == 0
    assert _gram("dense_gram_noalloc", A, B, C1, stream) == 0
    stream.synchronize()
    return C0.cpu().numpy(), C1.cpu().numpy()


def test_noalloc_gram_matches_dense_gram_on_consecutive_calls(cuda):
    import torch

    stream = torch.cuda.current_stream()
    rng = np.random.default_rng(7)
    # First call: 35 chunks of partials of 100 x 37; second: 3 chunks of 64 x 64.
    for n, ka, kb in [(70001, 100, 37), (5000, 64, 64)]:
        A = torch.as_tensor(rng.standard_normal((n, ka)), device=cuda)
        B = torch.as_tensor(rng.standard_normal((n, kb)), device=cuda)
        ref, got = _both(A, B, stream)
        assert np.array_equal(got, ref), (n, ka, kb)
        exact = A.cpu().numpy().T @ B.cpu().numpy()
        assert np.linalg.norm(got - exact) <= 1e-13 * np.linalg.norm(exact)


def test_noalloc_gram_strided_views(cuda):
    import torch

    stream = torch.cuda.current_stream()
    S = torch.as_tensor(np.random.default_rng(8).standard_normal((3000, 90)), device=cuda)
    ref, got = _both(S[:, :40], S[:, 50:], stream)
    assert np.array_equal(got, ref)


def test_noalloc_gram_capacity_limit(cuda):
    import torch

    stream = torch.cuda.current_stream()
    cap, chunk = capi.GRAM_SCRATCH_DOUBLES, capi.GRAM_CHUNK
    k = 64
    n_max = chunk * (cap // (k * k))  # exactly fills the scratch
    A = torch.empty((n_max + 1, k), dtype=torch.float64, device=cuda)
    A.uniform_(-1.0, 1.0, generator=torch.Generator(device=cuda).manual_seed(9))
    ref, got = _both(A[:n_max], A[:n_max], stream)
    assert np.array_equal(got, ref)
    C = torch.zeros((k, k), dtype=torch.float64, device=cuda)
    assert _gram("dense_gram_noalloc", A, A, C, stream) == capi.CG_ESCRATCH  # one chunk more
    stream.synchronize()
    assert not C.any()
    # The refusal left the scratch usable: a small call afterwards is still exact.
    ref, got = _both(A[:4097, :3], A[:4097, 5:9], stream)
    assert np.array_equal(got, ref)
