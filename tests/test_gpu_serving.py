"""Serving (continuous batching): results alone and in the mix, admission by
HBM budget, latency statistics.

Each served request computes exactly what tm_solve computes for the same
inputs (same kernels, launch shapes and fixed-order reductions, whatever
else runs beside it), so a request solved alone through tm_solve and the same
request solved while others share the GPU must agree to the last bit; the
test asserts the iteration count exactly and E_G and the eigenvalues to
1e-12 relative, well inside the 1e-10 accuracy target.
"""

import numpy as np
import pytest

from tests.gpu_common import ctx_or_skip, host, print_case
from workloads import StencilSpec, make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return ctx_or_skip()


@pytest.fixture(scope="module")
def tm():
    import paper_1108_4509_amd as tm
    return tm


def _problems():
    out = []
    for i, (side, m, wells) in enumerate([(12, 8, 2), (16, 16, 3), (14, 12, 2), (20, 24, 4),
                                          (16, 27, 0), (18, 20, 3)]):
        out.append(make_problem(f"s{i}", StencilSpec(3, (side,) * 3, 2, "periodic", 0.5), m=m,
                                seed=100 + i, n_wells=wells))
    return out


def test_alone_vs_mix(ctx, tm):
    probs = _problems()
    opts = tm.opts(precision="mixed")
    alone = []
    for p in probs:
        print_case(test="serving_alone", name=p.name, N=p.N, m=p.m)
        H = tm.matrix_from_problem(ctx, p)
        r, C, w, _ = tm.solve(ctx, H, p.m, 1e-8, tm.to_block(p.C0()), opts, want_vectors=False)
        alone.append((r, host(w)))
    srv = tm.Server(max_slots=4, hbm_budget=4 << 30)
    try:
        print_case(test="serving_mix", requests=len(probs))
        ids = [srv.submit(*p.csr(), p.m, 1e-8, p.C0(), tm.opts(precision="mixed")) for p in probs]
        mixed = [srv.wait(i, timeout=120.0) for i in ids]
        st = srv.stats()
    finally:
        srv.close()
    for p, (ra, wa), got in zip(probs, alone, mixed):
        assert got is not None, f"{p.name} did not finish"
        rm, wm = got
        assert rm["status"] == 0 and ra["converged"] == 1
        assert rm["iterations"] == ra["iterations"]
        assert abs(rm["E_G"] - ra["E_G"]) <= 1e-12 * abs(ra["E_G"])
        assert np.max(np.abs(wm - wa)) <= 1e-12 * np.max(np.abs(wa))
        assert rm["max_residual"] <= 1e-8
    assert st["completed"] == len(probs) and st["failed"] == 0
    assert 0 < st["p50_latency_s"] <= st["p99_latency_s"] <= st["max_latency_s"]
    assert st["hbm_peak"] <= st["hbm_budget"]


def test_admission_by_hbm_budget(ctx, tm):
    """A budget that holds one large request at a time still serves every
    request (they wait their turn); one larger than the budget is rejected."""
    probs = _problems()[:4]
    o = tm.opts(precision="mixed")
    need = [tm.solve_footprint(p.N, len(p.csr()[1]), p.m, o) for p in probs]
    budget = int(1.2 * max(need))
    srv = tm.Server(max_slots=4, hbm_budget=budget)
    try:
        print_case(test="serving_admission", budget=budget)
        ids = [srv.submit(*p.csr(), p.m, 1e-8, p.C0(), tm.opts(precision="mixed")) for p in probs]
        big = make_problem("big", StencilSpec(3, (40, 40, 40), 2, "periodic", 0.5), m=64, seed=7,
                           n_wells=0)
        with pytest.raises(tm.TraceminError) as e:
            srv.submit(*big.csr(), big.m, 1e-8, big.C0(), tm.opts(precision="mixed"))
        assert e.value.status == tm._abi.TM_ENOMEM
        res = [srv.wait(i, timeout=120.0) for i in ids]
        st = srv.stats()
    finally:
        srv.close()
    assert all(r is not None and r[0]["status"] == 0 for r in res)
    assert st["completed"] == len(probs) and st["rejected"] == 1
    assert st["hbm_peak"] <= budget
