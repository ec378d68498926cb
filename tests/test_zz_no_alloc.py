"""The allocation-free correlation spectrum (qhfpe_spectrum_corr_noalloc)
against qhfpe_spectrum_corr with a caller-provided workspace, through the
C-ABI: two calls in a row, the second with a smaller input (the fixed
scratch keeps the first call's contents), and the size limit."""

import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_1706_09590_amd import qhfpe  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def corr(r3, w1, w3, dt1, dt3, noalloc):
    L = qhfpe.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    n1, n3 = r3.shape[0], r3.shape[1]
    out = torch.full((w3.numel(), w1.numel()), float("nan"), dtype=torch.float64, device="cuda")
    if noalloc:
        rc = L.qhfpe_spectrum_corr_noalloc(_p(r3), n1, n3, dt1, dt3, _p(w1), w1.numel(), _p(w3), w3.numel(),
                                           _p(out), s)
    else:
        work = torch.empty((n1, w3.numel(), 2), dtype=torch.float64, device="cuda")
        rc = L.qhfpe_spectrum_corr(_p(r3), n1, n3, dt1, dt3, _p(w1), w1.numel(), _p(w3), w3.numel(), _p(work),
                                   _p(out), s)
    qhfpe._check(rc)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def case(n1, n3, nw1, nw3, seed):
    g = torch.Generator().manual_seed(seed)
    r3 = torch.randn((n1, n3, 2), generator=g, dtype=torch.float64).cuda()
    w1 = torch.linspace(0.0, 12.0, nw1, dtype=torch.float64).cuda()
    w3 = torch.linspace(0.5, 15.0, nw3, dtype=torch.float64).cuda()
    return r3, w1, w3


def test_noalloc_matches_the_workspace_entry_point_on_two_calls():
    # the 2D spectrum's own size (64 coherence times, 401 detection
    # frequencies), then a smaller one: the second call reads only what it wrote
    for (n1, n3, nw1, nw3, seed) in [(64, 4001, 401, 401, 1), (5, 33, 7, 11, 2)]:
        say(f"noalloc corr n1={n1} n3={n3} nw1={nw1} nw3={nw3}")
        r3, w1, w3 = case(n1, n3, nw1, nw3, seed)
        ref = corr(r3, w1, w3, 0.05, 0.005, noalloc=False)
        got = corr(r3, w1, w3, 0.05, 0.005, noalloc=True)
        assert np.all(np.isfinite(got))
        # same kernels, same order: identical up to rounding (here bit for bit)
        assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
        assert np.array_equal(got, ref)


def test_noalloc_rejects_sizes_beyond_its_scratch():
    r3, w1, w3 = case(200, 8, 3, 400, 3)  # n1 * n_w3 = 80000 > 65536
    L = qhfpe.lib()
    out = torch.empty((w3.numel(), w1.numel()), dtype=torch.float64, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = L.qhfpe_spectrum_corr_noalloc(_p(r3), 200, 8, 0.1, 0.1, _p(w1), w1.numel(), _p(w3), w3.numel(), _p(out), s)
    assert rc == qhfpe.EINVAL
    assert b"scratch" in L.qhfpe_last_error()
    # at the limit it runs
    r3, w1, w3 = case(128, 8, 3, 512, 4)  # 65536
    ref = corr(r3, w1, w3, 0.1, 0.1, noalloc=False)
    got = corr(r3, w1, w3, 0.1, 0.1, noalloc=True)
    assert np.array_equal(got, ref)
