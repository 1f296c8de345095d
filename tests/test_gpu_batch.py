"""Parity of the batched solve (tm_set_matrix_batch, tm_solve_batch).

k problems H_g = A + diag(V_g) on one periodic grid -- the kinetic operator
A = -(1/2) Lap_h of the serving workload, each problem with its own Gaussian
wells V_g (Sec. 3) -- are solved side by side in one block.  References:

* the sparse product of each problem, H_g C_g, from the oracle's CSR H_g
  (the matrix a lone solve would get);
* each problem's m lowest eigenvalues from LAPACK on the dense H_g
  (N <= 1728): with every residual ||H c_j - lambda_j c_j|| <= tol = 1e-8,
  the Ritz values lie within tol of eigenvalues, and (Rayleigh-Ritz) the
  error of each is about tol^2 / gap; the bar is 1e-9 (|lambda| <= ~10);
* the same problem solved alone by tm_solve from the same seeded start
  block: same eigenvalues to the same bar, and an iteration count within a
  few percent (the two runs differ only in rounding order).
"""

import numpy as np
import pytest

from tests.gpu_common import U32, U64, ctx_or_skip, gamma, host, print_case
from workloads import StencilSpec, make_problem
from workloads.problems import stencil_csr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return ctx_or_skip()


@pytest.fixture(scope="module")
def tm():
    import paper_1108_4509_amd as tm
    return tm


def _spec(side):
    return StencilSpec(ndim=3, dims=(side, side, side), order=2, bc="periodic", kinetic_scale=0.5)


def _batch(side, k, wells, seed0=300):
    """Kinetic CSR A, the k potentials, and each problem's own CSR H_g."""
    spec = _spec(side)
    A = stencil_csr(spec, None)
    Vs, Hs = [], []
    for g in range(k):
        w = wells[g] if isinstance(wells, (list, tuple)) else wells
        p = make_problem(f"b{g}", spec, 16, seed=seed0 + g, n_wells=w)
        Vs.append(p.V)
        Hs.append(stencil_csr(spec, p.V))
    return A, np.stack(Vs), Hs


def _dense(csr, n):
    from oracle.tracemin import csr_matrix
    return csr_matrix(*csr, n).toarray()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batch_spmm_matches_each_problem(tm, ctx, dtype):
    """X = H_g C_g for every problem, in the batch layout with ragged padding
    (m = 20: columns 20..ldg-1 of each problem are zero and stay zero)."""
    import torch
    from oracle.tracemin import csr_matrix, spmm
    side, k, m = 12, 3, 20
    print_case(test="batch_spmm", dtype=dtype, side=side, k=k, m=m)
    A, V, Hs = _batch(side, k, 2)
    n = side ** 3
    H = tm.set_matrix_batch(ctx, *A, V)
    ldg, ld = tm.batch_layout(k, m)
    rng = np.random.default_rng(5)
    C = np.zeros((n, ld))
    for g in range(k):
        C[:, g * ldg:g * ldg + m] = rng.standard_normal((n, m))
    tdt = torch.float64 if dtype == "f64" else torch.float32
    Cd = torch.from_numpy(C).to("cuda", tdt)
    X = torch.full_like(Cd, float("nan"))
    tm.spmm(ctx, H, m, Cd, X)
    Xh = host(X).astype(np.float64)
    Ch = host(Cd).astype(np.float64)
    u = U64 if dtype == "f64" else U32
    for g in range(k):
        Hg = csr_matrix(*Hs[g], n)
        want = spmm(Hg, Ch[:, g * ldg:g * ldg + m])
        absH = abs(Hg)
        bound = gamma(8, u) * np.asarray(absH @ np.abs(Ch[:, g * ldg:g * ldg + m])) + 1e-300
        err = np.abs(Xh[:, g * ldg:g * ldg + m] - want)
        assert np.all(err <= 2 * bound), (g, float((err / bound).max()))
        assert np.all(Xh[:, g * ldg + m:(g + 1) * ldg] == 0.0)


def _alone(tm, ctx, Hcsr, m, tol, seed, **kw):
    H = tm.set_matrix_csr(ctx, *Hcsr)
    o = tm.opts(seed=seed, **kw)
    r, _, eig, _ = tm.solve(ctx, H, m, tol, None, o, want_vectors=False)
    return r, host(eig)


@pytest.mark.parametrize("precision,precondition,m", [
    ("full_dp", False, 16),
    ("mixed", "chebyshev", 20),
    ("mp2_mp1", False, 16),
])
def test_batch_solve_matches_lapack_and_alone(tm, ctx, precision, precondition, m):
    side, k, tol, seed = 12, 4, 1e-8, 77
    print_case(test="batch_solve", precision=precision, precondition=precondition, side=side, k=k, m=m)
    A, V, Hs = _batch(side, k, [1, 2, 3, 5])
    n = side ** 3
    H = tm.set_matrix_batch(ctx, *A, V)
    o = tm.opts(precision=precision, precondition=precondition, seed=seed)
    res, C, eig = tm.solve_batch(ctx, H, m, tol, None, o)
    eig = host(eig)
    ldg, ld = tm.batch_layout(k, m)
    Ch = host(C)
    for g in range(k):
        r = res[g]
        assert r["converged"] == 1, (g, r)
        assert r["max_residual"] <= 2 * tol, (g, r)
        assert r["orth_err"] <= 1e-12, (g, r)
        lam = np.linalg.eigvalsh(_dense(Hs[g], n))[:m]
        assert np.max(np.abs(eig[g] - lam)) <= 1e-9, (g, eig[g] - lam)
        assert abs(r["E_G"] - lam.sum()) <= 1e-9 * abs(lam.sum()) + 1e-9
        # padding columns of the vectors stay zero
        assert np.all(Ch[:, g * ldg + m:(g + 1) * ldg] == 0.0)
        ra, ea = _alone(tm, ctx, Hs[g], m, tol, seed + g, precision=precision,
                        precondition=precondition)
        assert ra["converged"] == 1
        assert np.max(np.abs(eig[g] - ea)) <= 1e-9
        it_b, it_a = r["iterations"], ra["iterations"]
        # the two-phase policies end their first phase on noisy tests
        # (stall, rounding floor): another summation order moves the switch
        slack = 0.03 if precision == "full_dp" else 0.2
        assert abs(it_b - it_a) <= max(3, slack * it_a), (g, it_b, it_a)


def test_batch_explicit_start_block_is_the_seeded_one(tm, ctx):
    """C0 = NULL starts problem g from tm_random_block(seed + g): passing
    those blocks explicitly in the batch layout gives bit-identical results."""
    import torch
    side, k, m, tol, seed = 10, 2, 16, 1e-8, 9
    print_case(test="batch_seed", side=side, k=k, m=m)
    A, V, _ = _batch(side, k, 2)
    n = side ** 3
    H = tm.set_matrix_batch(ctx, *A, V)
    ldg, ld = tm.batch_layout(k, m)
    C0 = torch.zeros((n, ld), dtype=torch.float64, device="cuda")
    for g in range(k):
        blk = tm.random_block(ctx, n, m, seed + g)
        C0[:, g * ldg:g * ldg + m] = blk[:, :m]
    o = tm.opts(precision="full_dp", seed=seed)
    r1, C1, e1 = tm.solve_batch(ctx, H, m, tol, None, o)
    r2, C2, e2 = tm.solve_batch(ctx, H, m, tol, C0, o)
    assert torch.equal(e1, e2) and torch.equal(C1, C2)
    assert [r["iterations"] for r in r1] == [r["iterations"] for r in r2]


def test_batch_lone_problem_and_errors(tm, ctx):
    """A batch of one is the lone problem; misuse is refused up front."""
    from paper_1108_4509_amd import _abi
    side, m, tol, seed = 10, 16, 1e-8, 4
    print_case(test="batch_errors", side=side, m=m)
    A, V, Hs = _batch(side, 1, 3)
    n = side ** 3
    H = tm.set_matrix_batch(ctx, *A, V)
    res, _, eig = tm.solve_batch(ctx, H, m, tol, None, tm.opts(precision="full_dp", seed=seed))
    lam = np.linalg.eigvalsh(_dense(Hs[0], n))[:m]
    assert res[0]["converged"] == 1 and np.max(np.abs(host(eig)[0] - lam)) <= 1e-9
    lib = _abi.lib()
    o = tm.opts()
    r = _abi.tm_result()
    # a batch matrix is not a lone matrix, and the reverse
    assert lib.tm_solve(ctx.handle, H.handle, m, tol, None, None, None, None, r, None, 0) == _abi.TM_EINVAL
    Hl = tm.set_matrix_csr(ctx, *Hs[0])
    rs = (_abi.tm_result * 1)()
    assert lib.tm_solve_batch(ctx.handle, Hl.handle, m, tol, None, None, None, None, rs) == _abi.TM_EINVAL
    # the diagonal preconditioner and the BF16 policies are not batched
    o = tm.opts(precondition=True)
    assert lib.tm_solve_batch(ctx.handle, H.handle, m, tol, o, None, None, None, rs) == _abi.TM_ENOTSUP
    o = tm.opts(precision="mixed_bf16")
    assert lib.tm_solve_batch(ctx.handle, H.handle, m, tol, o, None, None, None, rs) == _abi.TM_ENOTSUP
    # non-finite potentials are rejected
    Vbad = V.copy()
    Vbad[0, 3] = np.nan
    with pytest.raises(RuntimeError):
        tm.set_matrix_batch(ctx, *A, Vbad)


@pytest.mark.parametrize("precision", ["mp2", "full_sp"])
def test_batch_single_phase_policies(tm, ctx, precision):
    """MP2 converges to tol like FULL_DP; FULL_SP ends at its FP32 floor
    (each problem's phase gate), with E_G within that floor of LAPACK."""
    side, k, m, tol, seed = 10, 3, 16, 1e-8, 21
    print_case(test="batch_policy", precision=precision, side=side, k=k, m=m)
    A, V, Hs = _batch(side, k, [1, 2, 4], seed0=500)
    n = side ** 3
    H = tm.set_matrix_batch(ctx, *A, V)
    res, _, eig = tm.solve_batch(ctx, H, m, tol, None, tm.opts(precision=precision, seed=seed),
                                 want_vectors=False)
    eig = host(eig)
    for g in range(k):
        lam = np.linalg.eigvalsh(_dense(Hs[g], n))[:m]
        if precision == "mp2":
            assert res[g]["converged"] == 1
            assert np.max(np.abs(eig[g] - lam)) <= 1e-9
        else:
            # the FP32 floor: about u32 * ||H|| relative on E_G
            assert abs(res[g]["E_G"] - lam.sum()) <= 1e-5 * abs(lam.sum())


def test_batch_many_small_problems(tm, ctx):
    """48 problems of 8^3 rows and m = 4 (768 block columns, more
    controller states than one page of the pinned polling buffer held
    before): every problem converges to its LAPACK eigenvalues."""
    side, k, m, tol = 8, 48, 4, 1e-9
    print_case(test="batch_many", side=side, k=k, m=m)
    A, V, Hs = _batch(side, k, 1, seed0=700)
    n = side ** 3
    H = tm.set_matrix_batch(ctx, *A, V)
    ldg, ld = tm.batch_layout(k, m)
    assert ld == k * ldg == 768
    res, _, eig = tm.solve_batch(ctx, H, m, tol, None, tm.opts(precision="full_dp", seed=3),
                                 want_vectors=False)
    eig = host(eig)
    for g in range(k):
        assert res[g]["converged"] == 1, g
        lam = np.linalg.eigvalsh(_dense(Hs[g], n))[:m]
        assert np.max(np.abs(eig[g] - lam)) <= 1e-9, g


def test_batch_graph_replay_matches_eager(tm, ctx):
    """Captured iteration batches replay the same kernels: the batched
    solve with graphs gives bit-identical results."""
    import torch
    side, k, m, tol, seed = 10, 4, 16, 1e-8, 8
    print_case(test="batch_graphs", side=side, k=k, m=m)
    A, V, _ = _batch(side, k, 2, seed0=900)
    H = tm.set_matrix_batch(ctx, *A, V)
    r1, C1, e1 = tm.solve_batch(ctx, H, m, tol, None, tm.opts(precision="mixed", seed=seed))
    r2, C2, e2 = tm.solve_batch(ctx, H, m, tol, None, tm.opts(precision="mixed", seed=seed, graphs=True))
    assert torch.equal(e1, e2) and torch.equal(C1, C2)
    assert [r["iterations"] for r in r1] == [r["iterations"] for r in r2]


def test_batch_widest_and_single_column(tm, ctx):
    """The widest batch the column bound admits (128 problems of m = 16:
    2048 block columns, 216 rows each; the Cholesky of C^T C as 32 diagonal
    blocks of 64), a batch of one-column problems (each group one live
    column and 15 padding columns) and 8 problems of m = 76 (80 columns
    each; the Cholesky as two diagonal blocks of 320, each five 64-wide
    block columns) reach every problem's LAPACK eigenvalues; one problem
    more than 2048 columns hold is refused."""
    from paper_1108_4509_amd import _abi
    for side, k, m, wells in ((6, 128, 16, 1), (8, 4, 1, 2), (8, 8, 76, 2)):
        print_case(test="batch_edges", side=side, k=k, m=m)
        A, V, Hs = _batch(side, k, wells, seed0=1100)
        n = side ** 3
        H = tm.set_matrix_batch(ctx, *A, V)
        ldg, ld = tm.batch_layout(k, m)
        assert ld <= 2048 and ldg >= m
        res, _, eig = tm.solve_batch(ctx, H, m, 1e-8, None, tm.opts(precision="full_dp", seed=11),
                                     want_vectors=False)
        eig = host(eig)
        for g in range(k):
            assert res[g]["converged"] == 1, g
            lam = np.linalg.eigvalsh(_dense(Hs[g], n))[:m]
            assert np.max(np.abs(eig[g] - lam)) <= 1e-9, g
    A, V, _ = _batch(4, 129, 1, seed0=1300)
    H = tm.set_matrix_batch(ctx, *A, V)
    rs = (_abi.tm_result * 129)()
    assert _abi.lib().tm_solve_batch(ctx.handle, H.handle, 16, 1e-8, None, None, None, None, rs) \
        == _abi.TM_ENOTSUP


def test_batch_problems_spanning_gram_tiles(tm, ctx):
    """Two problems of m = 256 (256 columns each, 512 in all): each problem
    spans 2 x 2 Gram tiles of 128, the Cholesky runs as two 256-wide
    diagonal blocks of four block columns each, and the products loop over
    one problem's rows per column tile.  Both problems reach their LAPACK
    eigenvalues (343 rows each; the seeds give gaps of about 1 % of the
    spectrum after the 256th eigenvalue)."""
    side, k, m = 7, 2, 256
    print_case(test="batch_spanning", side=side, k=k, m=m)
    A, V, Hs = _batch(side, k, [2, 3], seed0=1500)
    n = side ** 3
    H = tm.set_matrix_batch(ctx, *A, V)
    assert tm.batch_layout(k, m) == (256, 512)
    res, _, eig = tm.solve_batch(ctx, H, m, 1e-8, None, tm.opts(precision="full_dp", seed=5),
                                 want_vectors=False)
    eig = host(eig)
    for g in range(k):
        assert res[g]["converged"] == 1, (g, res[g])
        lam = np.linalg.eigvalsh(_dense(Hs[g], n))[:m]
        assert np.max(np.abs(eig[g] - lam)) <= 1e-9, g
