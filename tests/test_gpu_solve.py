"""End-to-end parity of tm_solve with the FP64 CPU oracle.

Tolerances: |Delta E_G| / |E_G| <= 1e-10 against the oracle and against
closed forms, and max_j ||H c_j - lambda_j c_j|| <= tol (1e-8) -- the accuracy
targets of the solver.  In FULL_DP the GPU and the oracle run the same
iteration from the same C_0, so their energy trajectories are also compared
step by step while the iterates are still far from converged (where rounding
has not yet been amplified by the CG recurrences).
"""

import json
import math
import os

import numpy as np
import pytest

from tests.gpu_common import ctx_or_skip, host, print_case
from workloads import StencilSpec, config_problem, make_problem

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


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


def periodic_spectrum(n, order=2):
    th = 2 * np.pi * np.arange(n) / n
    f = (1 - np.cos(th)) if order == 2 else (1 - np.cos(th)) * (7 - np.cos(th)) / 6
    return np.sort((f[:, None, None] + f[None, :, None] + f[None, None, :]).reshape(-1))


def eq16_spectrum(n):
    s = 4.0 * np.sin(np.arange(1, n + 1) * np.pi / (2 * (n + 1))) ** 2
    return np.sort((s[:, None] + s[None, :]).reshape(-1))


def _solve(tm, ctx, prob, precision="full_dp", tol=1e-8, stencil=False, hist=0, **kw):
    H = tm.matrix_from_problem(ctx, prob, stencil=stencil)
    C0 = tm.to_block(prob.C0())
    o = tm.opts(precision=precision, history=hist > 0, **kw)
    return tm.solve(ctx, H, prob.m, tol, C0, o, history_len=hist)


@pytest.fixture(scope="module")
def c1_oracle(orc):
    p = config_problem("c1")
    return orc.solve(orc.csr_matrix(*p.csr(), p.N), p.C0(),
                     orc.OracleOptions(tol=1e-8, k_rot=50))


@pytest.mark.parametrize("stencil", [False, True], ids=["csr", "stencil"])
def test_c1_full_dp(ctx, tm, c1_oracle, stencil):
    p = config_problem("c1")
    print_case(test="c1_full_dp", stencil=stencil)
    r, C, w, hist = _solve(tm, ctx, p, stencil=stencil, hist=400)
    exact = 54 * (1 - math.cos(math.pi / 8))
    assert r["converged"] == 1 and r["status"] == 0
    assert abs(r["E_G"] - exact) <= 1e-10 * exact
    assert abs(r["E_G"] - c1_oracle.E_G) <= 1e-10 * exact
    assert r["max_residual"] <= 1e-8
    assert r["orth_err"] < 1e-13
    assert np.max(np.abs(host(w) - periodic_spectrum(16)[:27])) < 1e-9
    # same iteration, step by step, while rounding has not been amplified
    Eo = np.array(c1_oracle.energies)
    k = 40
    assert np.max(np.abs(hist[:k, 0] - Eo[:k]) / np.abs(Eo[:k])) < 1e-9
    # and a comparable iteration count
    assert abs(r["iterations"] - c1_oracle.iterations) <= 0.25 * c1_oracle.iterations + 10


def test_c1_rotation_transport(ctx, tm, orc):
    """With P and G_prev carried through each rotation (k_rot = 5) the GPU
    iteration follows the oracle's: the energies agree while rounding has not
    been amplified, the rotation at i = 5 leaves the energy curve of the
    unrotated oracle run intact to the line-step weights, and E_G is exact."""
    p = config_problem("c1")
    print_case(test="c1_transport", k_rot=5)
    Ho = orc.csr_matrix(*p.csr(), p.N)
    ref = orc.solve(Ho, p.C0(), orc.OracleOptions(tol=1e-8, k_rot=5, transport=True))
    r, C, w, hist = _solve(tm, ctx, p, hist=400, k_rot=5, transport=True)
    exact = 54 * (1 - math.cos(math.pi / 8))
    assert r["converged"] == 1 and r["restarts"] == 1
    assert abs(r["E_G"] - exact) <= 1e-10 * exact
    Eo = np.array(ref.energies)
    k = 30
    assert np.max(np.abs(hist[:k, 0] - Eo[:k]) / np.abs(Eo[:k])) < 1e-9
    assert abs(r["iterations"] - ref.iterations) <= 0.25 * ref.iterations + 10


def test_c1_vectors_and_residual_definition(ctx, tm, orc):
    """The returned C: orthonormal, and max_j ||H c_j - C (C^T H c_j)|| <= 1e-8."""
    p = config_problem("c1")
    r, C, w, _ = _solve(tm, ctx, p)
    Ch = host(C, p.m)
    H = orc.csr_matrix(*p.csr(), p.N)
    X = orc.spmm(H, Ch)
    R = X - Ch @ (Ch.T @ X)
    assert np.max(np.linalg.norm(R, axis=0)) <= 1e-8
    assert np.max(np.abs(Ch.T @ Ch - np.eye(p.m))) < 1e-13
    assert np.all(host(C)[:, p.m:] == 0)


@pytest.fixture(scope="module")
def wells_problem():
    return make_problem("w12", StencilSpec(3, (12, 12, 12), 2, "periodic", 0.5), m=20, seed=5,
                        n_wells=6)


@pytest.fixture(scope="module")
def wells_oracle(orc, wells_problem):
    p = wells_problem
    return orc.solve(orc.csr_matrix(*p.csr(), p.N), p.C0(),
                     orc.OracleOptions(tol=1e-10, k_rot=50))


@pytest.mark.parametrize("precision", ["full_dp", "mixed", "mp2", "mixed_bf16", "mp1", "mp2_mp1"])
def test_wells_precisions(ctx, tm, wells_problem, wells_oracle, precision):
    print_case(test="wells", precision=precision)
    r, C, w, _ = _solve(tm, ctx, wells_problem, precision=precision)
    ref = wells_oracle.E_G
    assert r["converged"] == 1
    assert abs(r["E_G"] - ref) <= 1e-10 * abs(ref)
    assert r["max_residual"] <= 1e-8
    assert np.max(np.abs(host(w) - wells_oracle.eigenvalues)) <= 1e-9


def test_wells_full_bf16_floor(ctx, tm, wells_problem, wells_oracle):
    """The two-term BF16 bulk phase alone stalls at its rounding floor: it
    reports ENOCONV and an E_G error between the FP32 floor and plain BF16."""
    print_case(test="wells_full_bf16")
    r, C, w, _ = _solve(tm, ctx, wells_problem, precision="full_bf16", tol=1e-12)
    ref = wells_oracle.E_G
    err = abs(r["E_G"] - ref) / abs(ref)
    print(f"full_bf16 E_G relative error {err:.3e}, iterations {r['iterations']}")
    assert r["converged"] == 0
    assert err < 1e-3


def test_wells_brute_force_and_full_sp(ctx, tm, orc):
    """Brute-force dense Jacobi pins E_G; full SP reaches only FP32 accuracy."""
    p = make_problem("bf", StencilSpec(3, (8, 8, 8), 2, "periodic", 0.5), m=12, seed=9,
                     n_wells=4)
    E_bf, wall, gap = orc.brute_force_lowest(p.dense(), p.m)
    r, _, _, _ = _solve(tm, ctx, p)
    assert abs(r["E_G"] - E_bf) <= 1e-10 * abs(E_bf)
    r_sp, _, _, _ = _solve(tm, ctx, p, precision="full_sp")
    err = abs(r_sp["E_G"] - E_bf) / abs(E_bf)
    assert err < 1e-5          # FP32-level, and it reports itself as such:
    assert r_sp["converged"] == 0 and r_sp["status"] == tm.TM_ENOCONV


def test_paper_matrix_eq16(ctx, tm):
    """2-D Dirichlet Laplacian (Eq. 14-15), stencil and CSR, vs Eq. 16."""
    n = 40
    lam = eq16_spectrum(n)
    m = next(k for k in range(40, 80) if lam[k] - lam[k - 1] > 1e-3)
    p = make_problem("d40", StencilSpec(2, (n, n), 2, "dirichlet", 1.0), m=m, seed=3)
    for stencil in (False, True):
        for precision in ("full_dp", "mixed"):
            print_case(test="eq16", stencil=stencil, precision=precision)
            r, _, w, _ = _solve(tm, ctx, p, precision=precision, stencil=stencil)
            assert abs(r["E_G"] - lam[:m].sum()) <= 1e-10 * lam[:m].sum()
            assert np.max(np.abs(host(w) - lam[:m])) < 1e-9


def test_preconditioned(ctx, tm, wells_problem, wells_oracle):
    r, _, _, _ = _solve(tm, ctx, wells_problem, precondition=True)
    assert r["converged"] == 1
    assert abs(r["E_G"] - wells_oracle.E_G) <= 1e-10 * abs(wells_oracle.E_G)


def test_preconditioned_trajectory(ctx, tm, orc, wells_problem):
    """Eq. 18 with the diagonal M (varying with the wells here, so not a
    scalar): the GPU's preconditioned iteration -- M formed on the device, G'
    = M G in the direction update, the M-weighted Polak-Ribiere traces fused
    into the gradient epilogue -- follows the oracle's energies step by step
    while rounding has not been amplified, and ends at the same E_G."""
    p = wells_problem
    print_case(test="preconditioned_trajectory")
    ref = orc.solve(orc.csr_matrix(*p.csr(), p.N), p.C0(),
                    orc.OracleOptions(tol=1e-10, k_rot=50, precondition=True))
    M = orc.jacobi_preconditioner(orc.csr_matrix(*p.csr(), p.N))
    assert M.max() / M.min() > 1.3
    r, _, w, hist = _solve(tm, ctx, p, hist=600, precondition=True)
    Eo = np.array(ref.energies)
    k = 40
    assert np.max(np.abs(hist[:k, 0] - Eo[:k]) / np.abs(Eo[:k])) < 1e-9
    assert r["converged"] == 1
    assert abs(r["E_G"] - ref.E_G) <= 1e-10 * abs(ref.E_G)
    assert abs(r["iterations"] - ref.iterations) <= 0.25 * ref.iterations + 10


def test_seeded_start_block(ctx, tm, orc, wells_problem):
    """tm_solve with no start block draws the seeded one (tm_random_block):
    the same result as passing that block, and the oracle's E_G from it."""
    import torch
    p = wells_problem
    print_case(test="seeded_start")
    H = tm.matrix_from_problem(ctx, p)
    C0 = tm.random_block(ctx, p.N, p.m, 2024)
    r1, C1, w1, _ = tm.solve(ctx, H, p.m, 1e-8, None, tm.opts(seed=2024))
    r2, C2, w2, _ = tm.solve(ctx, H, p.m, 1e-8, C0, tm.opts())
    assert r1["E_G"] == r2["E_G"] and r1["iterations"] == r2["iterations"]
    assert torch.equal(C1, C2)
    ref = orc.solve(orc.csr_matrix(*p.csr(), p.N), host(C0, p.m), orc.OracleOptions(tol=1e-10))
    assert abs(r1["E_G"] - ref.E_G) <= 1e-10 * abs(ref.E_G)
    r3, _, _, _ = tm.solve(ctx, H, p.m, 1e-8, None, tm.opts(seed=2025))
    assert abs(r3["E_G"] - ref.E_G) <= 1e-10 * abs(ref.E_G)


def test_phase_accounting(ctx, tm, wells_problem):
    """Per-phase iterations and seconds add up to the totals."""
    for precision, two in (("mixed", True), ("mp2_mp1", True), ("full_dp", False)):
        print_case(test="phase_accounting", precision=precision)
        r, _, _, _ = _solve(tm, ctx, wells_problem, precision=precision)
        assert r["converged"] == 1
        assert r["iters_sp"] + r["iters_phase2"] == r["iterations"]
        assert (r["iters_phase2"] > 0) == two and r["iters_sp"] > 0
        ph = r["seconds_phase"]
        assert min(ph) >= 0 and abs(sum(ph) - r["seconds"]) <= 1e-3 + 0.01 * r["seconds"]


def test_csr_flags(ctx, tm, wells_problem):
    """TM_CHECK_SYMMETRY rejects a matrix that is not symmetric and accepts
    the stencil matrices; TM_DEVICE_PTRS takes device arrays and gives the
    same matrix (the same solve, bit for bit) as the host arrays."""
    import torch
    p = wells_problem
    rowptr, col, val = p.csr()
    Hh = tm.set_matrix_csr(ctx, rowptr, col, val, check_symmetry=True)
    Hd = tm.set_matrix_csr(ctx, torch.from_numpy(rowptr).cuda(), torch.from_numpy(col).cuda(),
                           torch.from_numpy(val).cuda(), check_symmetry=True)
    C0 = tm.to_block(p.C0())
    ra, Ca, _, _ = tm.solve(ctx, Hh, p.m, 1e-8, C0)
    rb, Cb, _, _ = tm.solve(ctx, Hd, p.m, 1e-8, C0)
    assert ra["E_G"] == rb["E_G"] and torch.equal(Ca, Cb)
    bad = val.copy()
    k = next(i for i in range(int(rowptr[5]), int(rowptr[6])) if col[i] != 5)   # off-diagonal, row 5
    bad[k] += 1e-3
    with pytest.raises(tm.TraceminError) as ei:
        tm.set_matrix_csr(ctx, rowptr, col, bad, check_symmetry=True)
    assert ei.value.status == tm.TM_EINVAL and "symmetric" in str(ei.value)
    tm.set_matrix_csr(ctx, rowptr, col, bad)    # unchecked: accepted as given
    with pytest.raises(tm.TraceminError):
        tm.set_matrix_csr(ctx, torch.from_numpy(rowptr).cuda(), torch.from_numpy(col).cuda(),
                          torch.from_numpy(bad).cuda(), check_symmetry=True)


@pytest.mark.parametrize("precision", ["full_dp", "mp1", "mp2", "mixed"])
def test_table1_row1(ctx, tm, precision):
    """Table 1's first row (the 2-D Dirichlet H_N of Eq. 14-15, N = 96^2,
    m = 220) in stencil mode under each policy: E_G against the closed form
    of Eq. 16 to 1e-10 and the printed E_G = 35.25."""
    n, m = 96, 220
    lam = eq16_spectrum(n)
    p = config_problem("t1_96_220")
    print_case(test="table1_row1", precision=precision)
    r, _, w, _ = _solve(tm, ctx, p, precision=precision, stencil=True)
    assert r["converged"] == 1
    assert abs(r["E_G"] - lam[:m].sum()) <= 1e-10 * lam[:m].sum()
    assert round(r["E_G"], 2) == 35.25
    assert np.max(np.abs(host(w) - lam[:m])) < 1e-9


def test_table1_widest_row(ctx, tm):
    """Table 1's last row, N = 192^2 and m = 1519 (ld = 1536), MIXED in
    stencil mode and FULL_DP on the CSR path: E_G = 395.6 against Eq. 16 to
    1e-10."""
    n, m = 192, 1519
    lam = eq16_spectrum(n)
    p = config_problem("t1_192_1519")
    for precision, stencil in (("mixed", True), ("full_dp", False)):
        print_case(test="table1_widest", precision=precision, stencil=stencil)
        r, _, w, _ = _solve(tm, ctx, p, precision=precision, stencil=stencil)
        assert r["converged"] == 1
        assert abs(r["E_G"] - lam[:m].sum()) <= 1e-10 * lam[:m].sum()
        assert round(r["E_G"], 1) == 395.6
        assert np.max(np.abs(host(w) - lam[:m])) < 1e-9


def test_13_point_closed_shell(ctx, tm):
    p = make_problem("o4", StencilSpec(3, (10, 10, 10), 4, "periodic", 0.5), m=7, seed=12)
    lam = periodic_spectrum(10, 4)
    for stencil in (False, True):
        r, _, w, _ = _solve(tm, ctx, p, stencil=stencil, tol=1e-9)
        assert np.max(np.abs(host(w) - lam[:7])) < 1e-10


def test_edge_cases(ctx, tm, orc):
    import torch
    # m = 1: lowest eigenvalue of the periodic Laplacian is 0
    p = make_problem("m1", StencilSpec(3, (8, 8, 8), 2, "periodic", 0.5), m=1, seed=4)
    r, _, w, _ = _solve(tm, ctx, p)
    assert abs(r["E_G"]) < 1e-12 and r["converged"] == 1
    # m = N: the whole space; E_G = trace(H)
    p = make_problem("full", StencilSpec(3, (4, 4, 2), 2, "periodic", 0.5), m=32, seed=4,
                     n_wells=0)
    r, _, _, _ = _solve(tm, ctx, p)
    assert abs(r["E_G"] - np.trace(p.dense())) < 1e-11
    # max_iter reached: TM_ENOCONV, result still filled
    p = config_problem("c1")
    r, _, _, _ = _solve(tm, ctx, p, max_iter=3)
    assert r["status"] == tm.TM_ENOCONV and r["converged"] == 0 and r["iterations"] == 3
    assert r["E_G"] > 4.110505244390517
    # rank-deficient start block: duplicated columns -> Cholesky breakdown
    C0 = p.C0().copy()
    C0[:, 5] = C0[:, 4]
    H = tm.matrix_from_problem(ctx, p)
    with pytest.raises(tm.TraceminError) as ei:
        tm.solve(ctx, H, p.m, 1e-8, tm.to_block(C0))
    assert ei.value.status == tm.TM_ENOTSPD
    # invalid arguments are rejected before any device work
    with pytest.raises(tm.TraceminError) as ei:
        tm.solve(ctx, H, 0, 1e-8, tm.to_block(C0))
    assert ei.value.status == tm.TM_EINVAL
    with pytest.raises(tm.TraceminError):
        tm.solve(ctx, H, p.m, -1.0, tm.to_block(C0))
    # empty matrix
    with pytest.raises(tm.TraceminError):
        tm.set_matrix_csr(ctx, np.zeros(1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    # out-of-range column index
    with pytest.raises(tm.TraceminError):
        tm.set_matrix_csr(ctx, np.array([0, 1], np.int64), np.array([3], np.int32),
                          np.array([1.0]))
    del torch


def _golden(name):
    path = os.path.join(HERE, "golden", f"oracle_{name}_s0.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated")
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("precision,precondition", [("mixed", "chebyshev"), ("full_dp", "chebyshev"),
                                                     ("mixed", False)])
def test_c2_full_size(ctx, tm, precision, precondition):
    """48^3 7-point + 64 wells, m = 256, in the benchmark's configuration
    (MIXED and FULL_DP with the degree-2 polynomial M) and without M."""
    g = _golden("c2")
    p = config_problem("c2")
    print_case(test="c2_full", precision=precision, precondition=precondition)
    r, C, w, _ = _solve(tm, ctx, p, precision=precision, precondition=precondition)
    assert r["converged"] == 1
    assert abs(r["E_G"] - g["E_G"]) <= 1e-10 * abs(g["E_G"])
    assert r["max_residual"] <= 1e-8
    assert np.max(np.abs(host(w) - np.array(g["eigenvalues"]))) <= 1e-8


@pytest.mark.slow
def test_c3_full_size_certified(ctx, tm, orc):
    """64^3 13-point + 200 wells, m = 512, MIXED, as timed by the benchmark's
    C3 line.  Pinned against the oracle's stored solve of the same input
    (tests/golden/oracle_c3_s0.json, written by make_golden.py from oracle/
    only): |dE_G| / |E_G| <= 1e-10 and the Ritz values to 1e-8.  Certified in
    FP64 on the host from the returned Ritz pairs as well: every
    ||H c_j - lambda_j c_j|| <= 1e-8, C^T C = I to 1e-12, E_G = tr(C^T H C).
    The certification alone shows that C spans an invariant subspace, not
    that it is the lowest one; the stored oracle value is what pins E_G (the
    test skips that comparison, and says so, while the file is absent)."""
    p = config_problem("c3")
    print_case(test="c3_full", N=p.N, m=p.m)
    r, C, w, _ = _solve(tm, ctx, p, precision="mixed", precondition="chebyshev")
    assert r["converged"] == 1 and r["max_residual"] <= 1e-8
    Ch = host(C, p.m)
    wh = host(w)
    del C
    H = orc.csr_matrix(*p.csr(), p.N)
    X = orc.spmm(H, Ch)
    res = np.linalg.norm(X - Ch * wh[None, :], axis=0)
    assert np.max(res) <= 1e-8
    S = Ch.T @ Ch
    assert np.max(np.abs(S - np.eye(p.m))) <= 1e-12
    E_rq = float(np.einsum("ij,ij->", Ch, X))
    assert abs(E_rq - r["E_G"]) <= 1e-12 * abs(r["E_G"])
    print(f"c3: E_G {r['E_G']:.15f} iterations {r['iterations']} max residual {np.max(res):.2e}")
    path = os.path.join(HERE, "golden", "oracle_c3_s0.json")
    if not os.path.exists(path):
        pytest.skip("certified; E_G unpinned until tests/golden/oracle_c3_s0.json exists")
    with open(path) as f:
        g = json.load(f)
    assert g["converged"] and g["N"] == p.N and g["m"] == p.m
    assert abs(r["E_G"] - g["E_G"]) <= 1e-10 * abs(g["E_G"])
    assert np.max(np.abs(wh - np.array(g["eigenvalues"]))) <= 1e-8


@pytest.mark.parametrize("precision", ["full_dp", "mixed"])
def test_graph_replay_matches_eager(ctx, tm, wells_problem, precision):
    """Batches of k_check iterations replayed from captured HIP graphs run
    the same kernels on the same buffers as the eager launches: every
    quantity must agree bit for bit.  A solve replays its graphs many times,
    with eager rotation batches, polls and (MIXED) a phase switch to new
    buffers in between."""
    print_case(test="graphs", precision=precision)
    ra, Ca, wa, ha = _solve(tm, ctx, wells_problem, precision=precision, hist=3000, graphs=False)
    rg, Cg, wg, hg = _solve(tm, ctx, wells_problem, precision=precision, hist=3000, graphs=True)
    assert ra["iterations"] > 3 * 10
    assert rg["iterations"] == ra["iterations"] and rg["iters_sp"] == ra["iters_sp"]
    assert rg["E_G"] == ra["E_G"]
    assert np.array_equal(host(wg), host(wa))
    assert np.array_equal(host(Cg), host(Ca))
    k = ra["iterations"]
    assert np.array_equal(hg[:k], ha[:k])


@pytest.mark.parametrize("degree", [2, 3])
def test_chebyshev_trajectory(ctx, tm, orc, wells_problem, degree):
    """The polynomial preconditioner (Eq. 18 with M = p(H - sigma I), the
    Chebyshev iteration on the Gershgorin interval) in FULL_DP follows the
    oracle's preconditioned iteration step by step and ends at the same E_G,
    in fewer iterations than the unpreconditioned solve; CSR and stencil
    agree (the same Gershgorin interval).  Degree 2 runs as one SpMM with the
    expanded linear polynomial a G + b H G; degree 3 through the recurrence."""
    p = wells_problem
    print_case(test="chebyshev_trajectory", degree=degree)
    ref = orc.solve(orc.csr_matrix(*p.csr(), p.N), p.C0(),
                    orc.OracleOptions(tol=1e-10, k_rot=50, chebyshev=degree))
    plain, _, _, _ = _solve(tm, ctx, p)
    for stencil in (False, True):
        r, _, w, hist = _solve(tm, ctx, p, hist=600, precondition="chebyshev", cheb_degree=degree,
                               stencil=stencil)
        Eo = np.array(ref.energies)
        k = 40
        assert np.max(np.abs(hist[:k, 0] - Eo[:k]) / np.abs(Eo[:k])) < 1e-9
        assert r["converged"] == 1
        assert abs(r["E_G"] - ref.E_G) <= 1e-10 * abs(ref.E_G)
        assert np.max(np.abs(host(w) - ref.eigenvalues)) <= 1e-9
        assert r["iterations"] < 0.8 * plain["iterations"]
        assert abs(r["iterations"] - ref.iterations) <= 0.25 * ref.iterations + 10


@pytest.mark.parametrize("precision", ["mixed", "mp2", "mp1"])
def test_chebyshev_single_precision(ctx, tm, wells_problem, wells_oracle, precision):
    """M applied in FP32 (the precision of G in these policies, Sec. 4): the
    result keeps full FP64 accuracy."""
    print_case(test="chebyshev_sp", precision=precision)
    r, _, w, _ = _solve(tm, ctx, wells_problem, precision=precision, precondition="chebyshev")
    assert r["converged"] == 1
    assert abs(r["E_G"] - wells_oracle.E_G) <= 1e-10 * abs(wells_oracle.E_G)
    assert np.max(np.abs(host(w) - wells_oracle.eigenvalues)) <= 1e-9
