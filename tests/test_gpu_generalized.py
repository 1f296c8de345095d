"""tm_solve_generalized (H x = lambda S x, S symmetric positive definite;
Sec. 2.1) against the FP64 CPU oracle and closed forms.

Workloads: Q1 finite elements on uniform grids, whose nonorthogonal basis
gives a 27-point (3-D) or 9-point (2-D) mass matrix S; their generalized
spectrum is known in closed form (1-D: mu = 6 (1 - cos t) / (2 + cos t),
summed over the axes).  Tolerances as for the standard solver:
|Delta E_G| / |E_G| <= 1e-10 and residuals ||H c_j - lambda_j S c_j|| <= 1e-8.
"""

import numpy as np
import pytest

from tests.gpu_common import ctx_or_skip, host, print_case
from workloads import StencilSpec, fem_problem, make_problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return ctx_or_skip()


@pytest.fixture(scope="module")
def tm():
    import paper_1108_4509_amd as tm
    return tm


@pytest.fixture(scope="module")
def orc():
    from oracle import build
    build.build()
    import oracle
    return oracle


def fem_spectrum(n, ndim, bc, scale=0.5):
    th = 2 * np.pi * np.arange(n) / n if bc == "periodic" else np.arange(1, n + 1) * np.pi / (n + 1)
    mu = 6.0 * (1.0 - np.cos(th)) / (2.0 + np.cos(th))
    tot = mu
    for _ in range(ndim - 1):
        tot = (tot[..., None] + mu).reshape(-1)
    return np.sort(scale * tot)


def _gsolve(tm, ctx, p, tol=1e-8, hist=0, **kw):
    H = tm.set_matrix_csr(ctx, *p.csr_H(), check_symmetry=True)
    S = tm.set_matrix_csr(ctx, *p.csr_S(), check_symmetry=True)
    o = tm.opts(precision="full_dp", history=hist > 0, **kw)
    return tm.solve(ctx, H, p.m, tol, tm.to_block(p.C0()), o, history_len=hist, S=S)


@pytest.mark.parametrize("case", ["3d_periodic", "2d_dirichlet"])
def test_fem_closed_form(ctx, tm, case):
    if case == "3d_periodic":
        n, ndim, bc, scale = 12, 3, "periodic", 0.5
        lam = fem_spectrum(n, ndim, bc, scale)
        m = 7
    else:
        n, ndim, bc, scale = 40, 2, "dirichlet", 1.0
        lam = fem_spectrum(n, ndim, bc, scale)
        m = next(k for k in range(40, 90) if lam[k] - lam[k - 1] > 1e-3)
    p = fem_problem("fem", ndim, n, m, bc, seed=7, kinetic_scale=scale)
    print_case(test="gen_fem_closed_form", case=case, N=p.N, m=m)
    r, C, w, _ = _gsolve(tm, ctx, p)
    assert r["converged"] == 1
    ref = lam[:m].sum()
    assert abs(r["E_G"] - ref) <= 1e-10 * max(1.0, abs(ref))
    assert np.max(np.abs(host(w) - lam[:m])) < 1e-9
    assert r["max_residual"] <= 1e-8 and r["orth_err"] < 1e-12
    # C^T S C = I on the host, with the oracle's own S
    import scipy.sparse as sp
    rowptr, col, val = p.csr_S()
    S = sp.csr_matrix((val, col, rowptr), shape=(p.N, p.N))
    Ch = host(C, m)
    assert np.max(np.abs(Ch.T @ (S @ Ch) - np.eye(m))) < 1e-12


def test_wells_against_oracle(ctx, tm, orc):
    """FEM with Gaussian wells (no closed form): E_G, the Ritz values and the
    first energies of the iteration against the oracle's generalized solve."""
    p = fem_problem("fw", 3, 12, 20, "periodic", seed=5, n_wells=6)
    print_case(test="gen_wells", N=p.N, m=p.m)
    H = orc.csr_matrix(*p.csr_H(), p.N)
    S = orc.csr_matrix(*p.csr_S(), p.N)
    ref = orc.solve(H, p.C0(), orc.OracleOptions(tol=1e-10, k_rot=50), S=S)
    r, C, w, hist = _gsolve(tm, ctx, p, hist=800)
    assert r["converged"] == 1
    assert abs(r["E_G"] - ref.E_G) <= 1e-10 * abs(ref.E_G)
    assert np.max(np.abs(host(w) - ref.eigenvalues)) <= 1e-9
    Eo = np.array(ref.energies)
    k = 30
    assert np.max(np.abs(hist[:k, 0] - Eo[:k]) / np.abs(Eo[:k])) < 1e-9
    assert abs(r["iterations"] - ref.iterations) <= 0.25 * ref.iterations + 10


def test_identity_and_diagonal_metric(ctx, tm, orc):
    """S = I (as CSR) reproduces the standard solver; a diagonal S given as a
    stencil (kinetic scale 0, V = the diagonal) matches the oracle with the
    same S as CSR."""
    import scipy.sparse as sp
    p = make_problem("w10", StencilSpec(3, (10, 10, 10), 2, "periodic", 0.5), m=12, seed=3,
                     n_wells=4)
    print_case(test="gen_identity_diag")
    H = tm.matrix_from_problem(ctx, p)
    C0 = tm.to_block(p.C0())
    r0, _, _, _ = tm.solve(ctx, H, p.m, 1e-8, C0)
    ones = np.ones(p.N)
    I = tm.set_matrix_csr(ctx, np.arange(p.N + 1, dtype=np.int64), np.arange(p.N, dtype=np.int32), ones)
    r1, _, _, _ = tm.solve(ctx, H, p.m, 1e-8, C0, S=I)
    assert abs(r1["E_G"] - r0["E_G"]) <= 1e-12 * abs(r0["E_G"])
    d = 1.0 + 0.5 * np.random.default_rng(1).random(p.N)
    Sd = tm.set_matrix_stencil(ctx, 3, (10, 10, 10), 2, True, 0.0, d)
    r2, _, w2, _ = tm.solve(ctx, H, p.m, 1e-8, C0, S=Sd)
    Ho = orc.csr_matrix(*p.csr(), p.N)
    ref = orc.solve(Ho, p.C0(), orc.OracleOptions(tol=1e-10, k_rot=50), S=sp.diags(d, 0, format="csr"))
    assert r2["converged"] == 1
    assert abs(r2["E_G"] - ref.E_G) <= 1e-10 * abs(ref.E_G)
    assert np.max(np.abs(host(w2) - ref.eigenvalues)) <= 1e-9


def test_generalized_errors(ctx, tm):
    p = fem_problem("fe", 3, 6, 4, "periodic", seed=1)
    H = tm.set_matrix_csr(ctx, *p.csr_H())
    S = tm.set_matrix_csr(ctx, *p.csr_S())
    C0 = tm.to_block(p.C0())
    with pytest.raises(tm.TraceminError) as ei:
        tm.solve(ctx, H, p.m, 1e-8, C0, tm.opts(precision="mixed"), S=S)
    assert ei.value.status == tm.TM_ENOTSUP
    q = fem_problem("fe2", 3, 7, 4, "periodic", seed=1)
    S2 = tm.set_matrix_csr(ctx, *q.csr_S())
    with pytest.raises(tm.TraceminError) as ei:
        tm.solve(ctx, H, p.m, 1e-8, C0, S=S2)
    assert ei.value.status == tm.TM_EINVAL
