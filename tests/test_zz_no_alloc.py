"""The no-allocation resampling entry point against mls2mc_resample, through
the C ABI: bit-identical ancestors on two calls in a row, the second with a
smaller input (the shared static scratch keeps the first call's contents),
and a clear error beyond its size limit."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import paper_1709_09763_amd as P
from tests import inputs
from tests.gpu_util import case, device, host, to_dev

pytestmark = pytest.mark.gpu


def _vp(t):
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _both(L, ctx, N, seed, zero_frac):
    w = inputs.weights(seed, N, spread=4.0, zero_frac=zero_frac)
    if w.max() == 0:
        w[0] = 1.0
    u = inputs.uniforms53(seed + 1, N)
    wd, ud = to_dev(w), to_dev(u)
    a_ref = torch.full((N,), -7, dtype=torch.int32, device="cuda:0")
    a_new = torch.full((N,), -7, dtype=torch.int32, device="cuda:0")
    assert L.mls2mc_resample(ctx.h, N, _vp(wd), _vp(ud), _vp(a_ref), _stream()) == 0
    assert L.mls2mc_resample_noalloc(N, _vp(wd), _vp(ud), _vp(a_new), _stream()) == 0, P.mls2mc_last_error()
    return host(a_ref), host(a_new), w, u


@pytest.mark.parametrize("sizes", [(1 << 20, 4099), (100003, 1000), (8192, 1)])
def test_resample_noalloc_equals_resample(sizes):
    device()
    L = P.lib()
    ctx = P.Context(3, 3, 4, 1.0, 0.3, 2, 0.1)
    for k, N in enumerate(sizes):
        case(f"resample_noalloc call {k + 1}: N={N}")
        a_ref, a_new, w, u = _both(L, ctx, N, 500 + 7 * k + N % 97, 0.2 if k == 0 else 0.0)
        np.testing.assert_array_equal(a_new, a_ref)
        assert a_new.min() >= 0 and a_new.max() < N
        if N <= 100003:
            np.testing.assert_array_equal(a_new, oracle.resample(w, u))


def test_resample_noalloc_rejects_oversize_and_bad_input():
    device()
    L = P.lib()
    N = (1 << 20) + 1
    w = torch.ones(N, dtype=torch.float64, device="cuda:0")
    a = torch.empty(N, dtype=torch.int32, device="cuda:0")
    assert L.mls2mc_resample_noalloc(N, _vp(w), _vp(w), _vp(a), _stream()) == 1
    assert "2^20" in P.mls2mc_last_error()
    assert L.mls2mc_resample_noalloc(0, _vp(w), _vp(w), _vp(a), _stream()) == 1
    assert L.mls2mc_resample_noalloc(8, None, _vp(w), _vp(a), _stream()) == 1
    # invalid weights: every ancestor is -1, as with mls2mc_resample
    z = torch.zeros(16, dtype=torch.float64, device="cuda:0")
    a16 = torch.empty(16, dtype=torch.int32, device="cuda:0")
    assert L.mls2mc_resample_noalloc(16, _vp(z), _vp(z), _vp(a16), _stream()) == 0
    assert (host(a16) == -1).all()
