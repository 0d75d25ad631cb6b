"""The allocation-free batched line solve (tridiag_solve_batched_noalloc) through
the C ABI against the allocating entry point (tridiag_solve_batched) on the same
inputs: two calls in a row on the partition path (which uses the library's fixed
scratch), the second with a smaller input, plus the on-chip path and the size
limit.  The two entry points share their kernels, so the results are bitwise
equal; both also meet the oracle's bar (the line-solve tolerance, 1e-5 relative
L2 in FP32, 1e-13 in FP64)."""
import ctypes

import numpy as np
import pytest

from tests.conftest import rel_l2

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {torch.float32: 1e-5, torch.float64: 1e-13}


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2006_10142_amd import _lib
    return _lib


def systems(n, batch, ss, es, dtype, seed):
    size = (batch - 1) * ss + (n - 1) * es + 1
    g = torch.Generator(device="cuda").manual_seed(seed)
    a = torch.rand(size, device="cuda", generator=g, dtype=dtype) - 0.5
    c = torch.rand(size, device="cuda", generator=g, dtype=dtype) - 0.5
    b = a.abs() + c.abs() + 0.5
    d = torch.rand(size, device="cuda", generator=g, dtype=dtype)
    return a, b, c, d


def call(lib, name, dtype, n, batch, a, b, c, d, ss, es):
    code = lib.ADI_F32 if dtype == torch.float32 else lib.ADI_F64
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    fn = getattr(lib.load(), name)
    return fn(code, n, batch, a.data_ptr(), b.data_ptr(), c.data_ptr(), d.data_ptr(), ss, es, stream)


def solve_both(lib, dtype, n, batch, ss, es, seed):
    a, b, c, d0 = systems(n, batch, ss, es, dtype, seed)
    d_ref, d_na = d0.clone(), d0.clone()
    assert call(lib, "tridiag_solve_batched", dtype, n, batch, a, b, c, d_ref, ss, es) == lib.ADI_OK
    assert call(lib, "tridiag_solve_batched_noalloc", dtype, n, batch, a, b, c, d_na, ss, es) == lib.ADI_OK
    torch.cuda.synchronize()
    return (a, b, c, d0), d_ref, d_na


def residual(a, b, c, d, x, n, batch, ss, es):
    """relative residual of all systems (FP64 on the host)"""
    A, B, C, D, X = (t.double().cpu().numpy() for t in (a, b, c, d, x))
    idx = np.arange(batch)[:, None] * ss + np.arange(n)[None, :] * es
    a_, b_, c_, d_, x_ = (v[idx] for v in (A, B, C, D, X))
    r = b_ * x_ - d_
    r[:, 1:] += a_[:, 1:] * x_[:, :-1]
    r[:, :-1] += c_[:, :-1] * x_[:, 1:]
    return float(np.linalg.norm(r) / np.linalg.norm(d_))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_noalloc_matches_allocating_entry_point(lib, oracle_lib, dtype):
    # partition path (interleaved systems): a large call, then a smaller one that reuses
    # the fixed scratch with stale contents from the first
    for (n, batch, seed) in ((2000, 3000, 1), (301, 77, 2)):
        ss, es = 1, batch
        print(f"noalloc interleaved {dtype} n={n} batch={batch}", flush=True)
        (a, b, c, d0), d_ref, d_na = solve_both(lib, dtype, n, batch, ss, es, seed)
        assert torch.equal(d_ref, d_na)
        assert residual(a, b, c, d0, d_na, n, batch, ss, es) <= TOL[dtype]
        # a few systems against the oracle
        cols = [0, batch // 2, batch - 1]
        sub = [t.view(n, batch)[:, cols].double().t().contiguous().cpu().numpy().ravel() for t in (a, b, c, d0)]
        ref = oracle_lib.tridiag_batched(*sub, n, len(cols), n, 1)
        got = d_na.view(n, batch)[:, cols].double().t().contiguous().cpu().numpy().ravel()
        assert rel_l2(got, ref) <= TOL[dtype]


def test_noalloc_on_chip_path_and_limit(lib):
    # contiguous systems take the on-chip kernels (no scratch at all)
    print("noalloc contiguous", flush=True)
    (a, b, c, d0), d_ref, d_na = solve_both(lib, torch.float32, 1000, 64, 1000, 1, 3)
    assert torch.equal(d_ref, d_na)
    # a layout whose workspace exceeds the fixed scratch is refused before any work
    n, batch = 8192, 16384                         # 6 * 256 * 16384 * 4 B = 96 MiB
    a = torch.ones(n * batch, device="cuda")
    d = torch.zeros(n * batch, device="cuda")
    before = d.clone()
    st = call(lib, "tridiag_solve_batched_noalloc", torch.float32, n, batch, a, a + 2, a, d, 1, batch)
    assert st == lib.ADI_EINVAL
    assert b"no-allocation scratch" in lib.load().adi_last_error()
    torch.cuda.synchronize()
    assert torch.equal(d, before)
