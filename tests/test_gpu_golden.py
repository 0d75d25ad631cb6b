"""The HIP path against the stored reference values in tests/golden (written by
the oracle; the oracle is not run here): the C1 standing wave in FP64, the C3
recipe at 96^2 in FP64 and with FP32 inputs (final level at sampled nodes and
all receiver traces), and the stored tridiagonal solves."""
import numpy as np
import pytest

from tests.conftest import rel_l2
from tests.golden import cases, store

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def adw():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2006_10142_amd as m
    m._lib.load()
    return m


@pytest.mark.parametrize("name", sorted(cases.CASES))
def test_gpu_matches_stored_run(adw, name):
    from tests.test_gpu_parity import gpu_run
    p, nodes = cases.CASES[name]()
    offs, vals, recs, traces = store.load(name)
    assert np.array_equal(offs, nodes)
    print(f"golden {name}", flush=True)
    _, got, tr = gpu_run(adw, p, rec=traces is not None)
    assert rel_l2(got.ravel()[offs], vals) <= TOL[p.dtype]
    if traces is not None:
        assert np.array_equal(recs, p.rec_idx)
        assert rel_l2(tr, traces) <= TOL[p.dtype]


def test_gpu_matches_stored_tridiagonal_solutions(adw):
    for rows in store.load_tridiag():
        a, b, c, d, x = (np.ascontiguousarray(v) for v in rows.T)
        n = x.size
        A, B, C, D = (torch.from_numpy(v).cuda() for v in (a, b, c, d))
        adw.tridiag_solve_batched(A, B, C, D, n, 1, n, 1)
        torch.cuda.synchronize()
        assert rel_l2(D.cpu().numpy(), x) <= 1e-13
