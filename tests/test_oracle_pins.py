"""Pins of the FP64 CPU oracle against facts fixed by the paper and by mathematics.

Nothing here compares the oracle with itself: each check is a closed form
(Eq. 16 of the paper, the Fourier spectra of periodic stencils, the 1-D
Dirichlet Laplacian), a value printed in the paper (Table 1), an invariant of
the method (Sec. 2.1: C^T C = I, E invariant under C -> CU, Ky Fan bound), a
finite-difference derivative, brute force on tiny inputs, or a library routine
the oracle does not use (numpy's eigvalsh / qr) as an outside witness.
"""

import json
import math
import os

import numpy as np
import pytest

from workloads import StencilSpec, config_problem, make_problem
from workloads.problems import stencil_csr

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- closed forms

def eq16_spectrum(n):
    """Eq. 16: lambda_pq = 4 (sin^2(p pi / 2(n+1)) + sin^2(q pi / 2(n+1)))."""
    p = np.arange(1, n + 1)
    s = 4.0 * np.sin(p * np.pi / (2 * (n + 1))) ** 2
    return np.sort((s[:, None] + s[None, :]).reshape(-1))


def periodic_spectrum(n, order, ndim=3):
    """Fourier spectrum of -(1/2) Lap_h on an n^ndim periodic grid."""
    th = 2 * np.pi * np.arange(n) / n
    if order == 2:
        f = 1.0 - np.cos(th)
    else:
        f = (1.0 - np.cos(th)) * (7.0 - np.cos(th)) / 6.0
    total = f
    for _ in range(ndim - 1):
        total = (total[..., None] + f).reshape(-1)
    return np.sort(total)


def _H(oracle_mod, problem):
    return oracle_mod.csr_matrix(*problem.csr(), problem.N)


# ------------------------------------------------------------------ eigensolver

def test_jacobi_1d_dirichlet_closed_form(oracle_mod):
    n = 40
    A = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    w, V, _ = oracle_mod.jacobi_eigh(A)
    k = np.arange(1, n + 1)
    exact = np.sort(2 - 2 * np.cos(k * np.pi / (n + 1)))
    assert np.max(np.abs(w - exact)) < 1e-13
    assert np.max(np.abs(A @ V - V * w)) < 1e-13
    assert np.max(np.abs(V.T @ V - np.eye(n))) < 1e-13


def test_jacobi_random_symmetric(oracle_mod):
    rng = np.random.default_rng(5)
    for n in (1, 2, 7, 64, 150):
        B = rng.standard_normal((n, n))
        A = B + B.T
        w, V, _ = oracle_mod.jacobi_eigh(A)
        assert np.all(np.diff(w) >= 0)
        scale = np.linalg.norm(A)
        assert np.max(np.abs(A @ V - V * w)) < 1e-13 * scale
        assert np.max(np.abs(V.T @ V - np.eye(n))) < 1e-13
        assert abs(np.sum(w) - np.trace(A)) < 1e-12 * scale
        # outside witness: LAPACK via numpy (not used by the oracle)
        assert np.max(np.abs(w - np.linalg.eigvalsh(A))) < 1e-12 * scale


def test_jacobi_two_by_two_and_diagonal(oracle_mod):
    a, b, d = 1.0, 2.0, -3.0
    w, _, _ = oracle_mod.jacobi_eigh(np.array([[a, b], [b, d]]))
    mid, rad = (a + d) / 2, math.hypot((a - d) / 2, b)
    assert np.allclose(w, [mid - rad, mid + rad], atol=1e-15, rtol=0)
    D = np.diag([3.0, -1.0, 2.0])
    w, V, sweeps = oracle_mod.jacobi_eigh(D)
    assert np.array_equal(w, [-1.0, 2.0, 3.0]) and sweeps == 0
    assert np.array_equal(np.abs(V), np.abs(np.eye(3)[:, [1, 2, 0]]))


# ---------------------------------------------------------- orthonormalization

def test_cholesky_recovers_known_factor(oracle_mod):
    rng = np.random.default_rng(1)
    m = 30
    R = 0.3 * np.triu(rng.standard_normal((m, m)), 1)
    R[np.diag_indices(m)] = rng.uniform(1.0, 3.0, m)   # well conditioned
    S = R.T @ R
    Rc = oracle_mod.cholesky_upper(S)
    assert np.max(np.abs(Rc - R)) < 1e-13
    with pytest.raises(ArithmeticError):
        oracle_mod.cholesky_upper(np.array([[1.0, 2.0], [2.0, 1.0]]))


def test_upper_inverse_closed_form(oracle_mod):
    m, beta = 12, 0.7
    R = np.eye(m) - beta * np.eye(m, k=1)
    W = oracle_mod.upper_triangular_inverse(R)
    i, j = np.indices((m, m))
    exact = np.where(j >= i, beta ** (j - i), 0.0)
    assert np.max(np.abs(W - exact)) < 1e-14


def test_orthonormalize_is_cholesky_qr(oracle_mod):
    rng = np.random.default_rng(2)
    C = rng.standard_normal((500, 20))
    Q = oracle_mod.orthonormalize(C)
    assert np.max(np.abs(Q.T @ Q - np.eye(20))) < 1e-13
    # same as Householder QR with a positive-diagonal R (outside witness)
    Qh, Rh = np.linalg.qr(C)
    Qh = Qh * np.sign(np.diag(Rh))[None, :]
    assert np.max(np.abs(Q - Qh)) < 1e-12
    # C = Q T with T upper triangular, positive diagonal (Fig. 4 convention)
    T = Q.T @ C
    assert np.max(np.abs(np.tril(T, -1))) < 1e-12
    assert np.all(np.diag(T) > 0)


# --------------------------------------------------------- energy and gradient

@pytest.fixture(scope="module")
def small_well_problem():
    return make_problem("w6", StencilSpec(3, (6, 6, 6), 2, "periodic", 0.5),
                        m=10, seed=3, n_wells=3)


def test_alg1_equals_alg2(oracle_mod, small_well_problem):
    p = small_well_problem
    H = _H(oracle_mod, p)
    C = oracle_mod.orthonormalize(p.C0())
    E1, G1, _, _ = oracle_mod.energy_gradient_alg1(H, C)
    E2, G2, _, _, _ = oracle_mod.energy_gradient_alg2(H, C)
    assert abs(E1 - E2) < 1e-13 * abs(E1)
    assert np.linalg.norm(G1 - G2) < 1e-13 * np.linalg.norm(G1)


def test_gradient_is_directional_derivative(oracle_mod, small_well_problem):
    """-tr(P^T G) is the slope of E(orthonormalize(C + eps P)) at eps = 0."""
    p = small_well_problem
    H = _H(oracle_mod, p)
    C = oracle_mod.orthonormalize(p.C0())
    E0, G, _, _ = oracle_mod.energy_gradient_alg1(H, C)
    P = np.random.default_rng(9).standard_normal(C.shape)
    eps = 1e-5

    def E_at(e):
        return oracle_mod.energy_gradient_alg1(H, oracle_mod.orthonormalize(C + e * P))[0]

    fd = (E_at(eps) - E_at(-eps)) / (2 * eps)
    assert abs(fd - (-np.sum(P * G))) < 1e-6 * abs(fd)


def test_unitary_invariance_and_tangency(oracle_mod, small_well_problem):
    p = small_well_problem
    H = _H(oracle_mod, p)
    C = oracle_mod.orthonormalize(p.C0())
    E, G, _, _ = oracle_mod.energy_gradient_alg1(H, C)
    Q, _ = np.linalg.qr(np.random.default_rng(4).standard_normal((p.m, p.m)))
    E2, G2, _, _ = oracle_mod.energy_gradient_alg1(H, C @ Q)
    assert abs(E - E2) < 1e-13 * abs(E)
    assert np.linalg.norm(G @ Q - G2) < 1e-12 * np.linalg.norm(G)
    assert np.max(np.abs(C.T @ G)) < 1e-12 * np.linalg.norm(G)


# ---------------------------------------------------------------- full solves

def test_c1_closed_form_shell():
    """16^3 periodic 7-point, m = 27: E_G = 54 (1 - cos(pi/8)) in closed form."""
    lam = periodic_spectrum(16, 2)
    assert abs(np.sum(lam[:27]) - 54 * (1 - math.cos(math.pi / 8))) < 1e-12
    assert lam[27] - lam[26] > 0.06


def test_solve_c1_matches_closed_form(oracle_mod):
    p = config_problem("c1")
    r = oracle_mod.solve(_H(oracle_mod, p), p.C0(),
                         oracle_mod.OracleOptions(tol=1e-9, k_rot=50))
    exact = periodic_spectrum(16, 2)[:27]
    assert r.converged
    assert abs(r.E_G - 54 * (1 - math.cos(math.pi / 8))) < 1e-12 * r.E_G
    assert np.max(np.abs(r.eigenvalues - exact)) < 1e-12
    assert r.max_residual <= 1e-9
    assert r.orth_err < 1e-13
    # Ky Fan: every iterate's trace is an upper bound of E_G
    assert min(r.energies) >= r.E_G - 1e-12
    # preconditioned run reaches the same answer (Eq. 18 changes only the path)
    rp = oracle_mod.solve(_H(oracle_mod, p), p.C0(),
                          oracle_mod.OracleOptions(tol=1e-9, k_rot=50, precondition=True))
    assert abs(rp.E_G - r.E_G) < 1e-12 * r.E_G


def test_solve_13_point_closed_shell(oracle_mod):
    """8^3 periodic 13-point, m = 7 (k = 0 plus the six +-1 modes)."""
    p = make_problem("o4", StencilSpec(3, (8, 8, 8), 4, "periodic", 0.5), m=7, seed=11)
    lam = periodic_spectrum(8, 4)
    r = oracle_mod.solve(_H(oracle_mod, p), p.C0(),
                         oracle_mod.OracleOptions(tol=1e-10, k_rot=50))
    assert r.converged
    assert np.max(np.abs(r.eigenvalues - lam[:7])) < 1e-12


def test_solve_2d_dirichlet_eq16_small(oracle_mod):
    """The paper's H_N (Eq. 14-15) at n = 24; E_G from the closed form Eq. 16."""
    n = 24
    lam = eq16_spectrum(n)
    m = next(k for k in range(30, 60) if lam[k] - lam[k - 1] > 1e-3)
    p = make_problem("d24", StencilSpec(2, (n, n), 2, "dirichlet", 1.0), m=m, seed=7)
    r = oracle_mod.solve(_H(oracle_mod, p), p.C0(),
                         oracle_mod.OracleOptions(tol=1e-9, k_rot=50))
    assert r.converged
    assert abs(r.E_G - lam[:m].sum()) < 1e-11 * lam[:m].sum()


def test_table1_first_row(oracle_mod):
    """Table 1, N = 96^2, m = 220: printed E_G = 35.25 and gap 6.2e-3."""
    with open(os.path.join(HERE, "golden", "table1.json")) as f:
        row = json.load(f)["rows"][0]
    lam = eq16_spectrum(row["n"])
    m = row["m"]
    assert round(float(lam[:m].sum()), 2) == row["E_G"]
    assert abs((lam[m] - lam[m - 1]) - row["gap"]) < 0.05e-3
    p = config_problem("t1_96_220")
    r = oracle_mod.solve(_H(oracle_mod, p), p.C0(),
                         oracle_mod.OracleOptions(tol=1e-7, k_rot=50))
    assert r.converged
    assert abs(r.E_G - lam[:m].sum()) < 1e-10 * lam[:m].sum()
    assert round(r.E_G, 2) == row["E_G"]


def test_wells_brute_force(oracle_mod):
    """Tiny grids with wells: iterative E_G equals brute-force dense Jacobi."""
    for n, m, K, seed in ((4, 5, 2, 21), (6, 12, 3, 22)):
        p = make_problem("bf", StencilSpec(3, (n, n, n), 2, "periodic", 0.5),
                         m=m, seed=seed, n_wells=K)
        Hd = p.dense()
        assert np.array_equal(Hd, Hd.T)
        E_bf, w, gap = oracle_mod.brute_force_lowest(Hd, m)
        assert gap > 1e-3
        assert np.max(np.abs(w - np.linalg.eigvalsh(Hd))) < 1e-12   # witness
        r = oracle_mod.solve(_H(oracle_mod, p), p.C0(),
                             oracle_mod.OracleOptions(tol=1e-10, k_rot=50))
        assert r.converged
        assert abs(r.E_G - E_bf) < 1e-12 * abs(E_bf)
        assert np.max(np.abs(r.eigenvalues - w[:m])) < 1e-11


def test_potential_shift_and_scaling(oracle_mod):
    """V -> V + v shifts E_G by m v; H -> a H scales E_G by a."""
    p = make_problem("s", StencilSpec(3, (6, 6, 6), 2, "periodic", 0.5),
                     m=7, seed=31, n_wells=2)
    H = _H(oracle_mod, p)
    base = oracle_mod.solve(H, p.C0(), oracle_mod.OracleOptions(tol=1e-10, k_rot=50))
    v = 0.375
    shifted = oracle_mod.csr_matrix(*stencil_csr(p.spec, p.V + v), p.N)
    r1 = oracle_mod.solve(shifted, p.C0(), oracle_mod.OracleOptions(tol=1e-10, k_rot=50))
    assert abs(r1.E_G - (base.E_G + p.m * v)) < 1e-12 * abs(base.E_G)
    r2 = oracle_mod.solve(2.5 * H, p.C0(), oracle_mod.OracleOptions(tol=1e-10, k_rot=50))
    assert abs(r2.E_G - 2.5 * base.E_G) < 1e-12 * abs(base.E_G)


def test_single_vector_rayleigh_minimum(oracle_mod):
    """m = 1: the minimum of the Rayleigh quotient is lambda_1 (periodic: 0)."""
    p = make_problem("m1", StencilSpec(3, (8, 8, 8), 2, "periodic", 0.5), m=1, seed=41)
    r = oracle_mod.solve(_H(oracle_mod, p), p.C0(),
                         oracle_mod.OracleOptions(tol=1e-10))
    assert r.converged
    assert abs(r.E_G) < 1e-15 + 1e-12
    c = r.C[:, 0]
    assert np.max(np.abs(np.abs(c) - 1 / math.sqrt(p.N))) < 1e-9


def test_rotation_transport_leaves_cg_intact(oracle_mod):
    """A subspace rotation C <- C U changes neither E nor the subspace
    (Sec. 2.1), and the gradient maps as G -> G U, so the Polak-Ribiere gamma
    (Eq. 8) computed after carrying P and G_prev through the same U equals the
    gamma of the unrotated run to rounding; the step along the carried
    direction differs only through the per-column curvature weights of the
    line step (about 1 % here).  A transposed U or a block left uncarried moves
    gamma by ~20 % or the step by ~80 %."""
    from workloads import config_problem
    p = config_problem("c1")
    H = oracle_mod.csr_matrix(*p.csr(), p.N)
    base = oracle_mod.solve(H, p.C0(), oracle_mod.OracleOptions(tol=1e-8, k_rot=0, max_iter=8))
    rot = oracle_mod.solve(H, p.C0(), oracle_mod.OracleOptions(tol=1e-8, k_rot=5, transport=True,
                                                               max_iter=8))
    assert np.allclose(rot.energies[:6], base.energies[:6], rtol=1e-13, atol=0)
    assert abs(rot.gammas[5] - base.gammas[5]) <= 1e-12 * abs(base.gammas[5])
    assert abs(rot.alphas[5] - base.alphas[5]) <= 0.05 * base.alphas[5]
    assert rot.restarts == 1          # only i = 0
    full = oracle_mod.solve(H, p.C0(), oracle_mod.OracleOptions(tol=1e-8, k_rot=5, transport=True))
    exact = 54 * (1 - math.cos(math.pi / 8))
    assert full.converged and abs(full.E_G - exact) <= 1e-12 * exact


# ------------------------------------------------ line step and preconditioner

def _ritz_basis_and_tangent(oracle_mod, p, seed):
    """An orthonormal C whose m x m H = C^T H C is diagonal (a Ritz basis,
    rotated with numpy's eigh as an outside witness) and a random direction P
    projected onto the orthogonal complement of span(C)."""
    H = _H(oracle_mod, p)
    C = oracle_mod.orthonormalize(p.C0())
    A = C.T @ (H @ C)
    _, U = np.linalg.eigh(0.5 * (A + A.T))
    C = C @ U
    P = np.random.default_rng(seed).standard_normal(C.shape)
    P -= C @ (C.T @ P)
    P /= np.linalg.norm(P, axis=0)[None, :]
    return H, C, P


def _omega(H, C, P, a):
    """E at the orthonormalized C + a P without orthonormalizing: the energy
    depends on the span only (Sec. 2.1), so with S = B^T B for B = C + a P it
    is tr(S^{-1} B^T H B) (numpy's solve, not the oracle's Cholesky)."""
    B = C + a * P
    return float(np.trace(np.linalg.solve(B.T @ B, B.T @ (H @ B))))


def test_line_step_curvature_is_second_derivative(oracle_mod, small_well_problem):
    """The line step's curvature 2 sum_j (p_j.Hp_j - A_jj p_j.p_j) is the
    second derivative of E along P at a Ritz basis with P orthogonal to C,
    the case where the second-order model is exact; central differences at
    three step sizes converge to it at the O(eps^2) rate.  Its slope
    tr(P^T G) is -dE/da (the gradient pin above), and the step is the
    minimizer of the model: the differences of E at alpha * (1 +- 0.01)
    match the model's parabola."""
    H, C, P = _ritz_basis_and_tangent(oracle_mod, small_well_problem, 17)
    E0, G, X, A = oracle_mod.energy_gradient_alg1(H, C)
    assert np.max(np.abs(A - np.diag(np.diag(A)))) < 1e-13 * np.max(np.abs(A))
    Y = oracle_mod.spmm(H, P)
    alpha, info = oracle_mod.line_step(P, Y, G, np.diag(A).copy())
    curv = info["curv"]
    assert abs(curv) > 1.0
    om0 = _omega(H, C, P, 0.0)
    assert abs(om0 - E0) < 1e-13 * abs(E0)
    errs = []
    for eps in (4e-3, 2e-3, 1e-3):
        fd2 = (_omega(H, C, P, eps) - 2 * om0 + _omega(H, C, P, -eps)) / eps ** 2
        errs.append(abs(fd2 - curv) / abs(curv))
    assert errs[-1] < 1e-5
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0   # O(eps^2)
    # a factor or sign slip in either term is far outside that agreement
    pp = np.einsum("ij,ij->j", P, P)
    py = np.einsum("ij,ij->j", P, Y)
    for wrong in (np.sum(py - np.diag(A) * pp), 2 * np.sum(py + np.diag(A) * pp),
                  2 * np.sum(py)):
        assert abs(wrong - curv) > 1e-2 * abs(curv)
    # the step: the minimizer pg / curv of the parabola E0 - pg a + curv a^2 / 2
    # when the curvature is positive, capped at 1 / max_j ||p_j||
    assert abs(info["pg"] - float(np.sum(P * G))) < 1e-14 * abs(info["pg"])
    cap = 1.0 / np.sqrt(pp.max())
    assert alpha == pytest.approx(min(info["pg"] / curv, cap) if curv > 0 else cap, rel=1e-15)


def test_preconditioner_scalar_multiple_reproduces_plain_cg(oracle_mod):
    """Eq. 18 with a scalar M = c I (a matrix with a constant diagonal,
    here the V = 0 periodic Laplacian, diagonal 3, so M = I / 3): G' = M G
    scales every direction by c, the M-weighted Polak-Ribiere gamma is
    unchanged, the step alpha grows by 1 / c and the iterates are those of
    the unpreconditioned CG."""
    p = config_problem("c1")
    H = _H(oracle_mod, p)
    M = oracle_mod.jacobi_preconditioner(H)
    assert np.all(M == 1.0 / 3.0)
    opts = dict(tol=1e-14, k_rot=0, max_iter=15)
    base = oracle_mod.solve(H, p.C0(), oracle_mod.OracleOptions(**opts))
    pre = oracle_mod.solve(H, p.C0(), oracle_mod.OracleOptions(precondition=True, **opts))
    assert np.allclose(pre.energies, base.energies, rtol=1e-13, atol=0)
    g0, g1 = np.array(base.gammas), np.array(pre.gammas)
    assert g0[0] == 0 and g1[0] == 0 and np.all(g0[1:] != 0)
    # equal up to rounding amplified by the recurrences over 15 iterations
    assert np.max(np.abs(g1 - g0)) <= 1e-10 * np.max(np.abs(g0))
    ratio = np.array(pre.alphas) / np.array(base.alphas)
    assert np.max(np.abs(ratio - 3.0)) < 1e-10


# ------------------------------------------------ generalized H x = lambda S x

def fem_spectrum(n, ndim, bc, scale=0.5):
    """Generalized eigenvalues of Q1 finite elements on a uniform grid: in 1-D
    K u = mu M u with u_j = sin(j theta) or exp(i j theta) gives
    mu = 6 (1 - cos theta) / (2 + cos theta); tensor products add them."""
    if bc == "periodic":
        th = 2 * np.pi * np.arange(n) / n
    else:
        th = np.arange(1, n + 1) * np.pi / (n + 1)
    mu = 6.0 * (1.0 - np.cos(th)) / (2.0 + np.cos(th))
    tot = mu
    for _ in range(ndim - 1):
        tot = (tot[..., None] + mu).reshape(-1)
    return np.sort(scale * tot)


def _gen_mats(oracle_mod, p):
    H = oracle_mod.csr_matrix(*p.csr_H(), p.N)
    S = oracle_mod.csr_matrix(*p.csr_S(), p.N)
    return H, S


def test_generalized_fem_closed_form(oracle_mod):
    """Q1 finite elements, 3-D periodic 8^3, m = 7 (the constant mode and the
    six +-1 modes): E_G and the Ritz values against the closed form; C is
    S-orthonormal and every residual ||H c_j - lambda_j S c_j|| is small."""
    from workloads import fem_problem
    p = fem_problem("f8", 3, 8, 7, "periodic", seed=3)
    H, S = _gen_mats(oracle_mod, p)
    lam = fem_spectrum(8, 3, "periodic")
    assert lam[7] - lam[6] > 0.1
    r = oracle_mod.solve(H, p.C0(), oracle_mod.OracleOptions(tol=1e-10, k_rot=50), S=S)
    assert r.converged
    assert abs(r.E_G - lam[:7].sum()) < 1e-12 * max(1.0, lam[:7].sum())
    assert np.max(np.abs(r.eigenvalues - lam[:7])) < 1e-11
    assert r.orth_err < 1e-13 and r.max_residual < 1e-9
    C = r.C
    assert np.max(np.abs(C.T @ (S @ C) - np.eye(7))) < 1e-13


def test_generalized_2d_dirichlet_closed_form(oracle_mod):
    from workloads import fem_problem
    n = 14
    lam = fem_spectrum(n, 2, "dirichlet", scale=1.0)
    m = next(k for k in range(10, 40) if lam[k] - lam[k - 1] > 1e-2)
    p = fem_problem("f2d", 2, n, m, "dirichlet", seed=4, kinetic_scale=1.0)
    H, S = _gen_mats(oracle_mod, p)
    r = oracle_mod.solve(H, p.C0(), oracle_mod.OracleOptions(tol=1e-10, k_rot=50), S=S)
    assert r.converged
    assert abs(r.E_G - lam[:m].sum()) < 1e-12 * lam[:m].sum()


def test_generalized_reduces_to_standard(oracle_mod):
    """S = I gives the standard iteration (same energies, same E_G); S = c I
    divides every eigenvalue by c."""
    import scipy.sparse as sp
    p = make_problem("s", StencilSpec(3, (6, 6, 6), 2, "periodic", 0.5), m=7, seed=31, n_wells=2)
    H = _H(oracle_mod, p)
    o = oracle_mod.OracleOptions(tol=1e-10, k_rot=50)
    base = oracle_mod.solve(H, p.C0(), o)
    I = sp.identity(p.N, format="csr")
    same = oracle_mod.solve(H, p.C0(), o, S=I)
    k = min(len(base.energies), len(same.energies), 40)
    assert np.allclose(same.energies[:k], base.energies[:k], rtol=1e-12, atol=0)
    assert abs(same.E_G - base.E_G) < 1e-12 * abs(base.E_G)
    c = 2.5
    scaled = oracle_mod.solve(H, p.C0(), o, S=c * I)
    assert abs(scaled.E_G - base.E_G / c) < 1e-12 * abs(base.E_G)


def test_generalized_brute_force_with_wells(oracle_mod):
    """Tiny FEM grid with wells: iterative E_G equals the brute-force
    Cholesky reduction plus dense Jacobi, with scipy's generalized eigh (not
    used by the oracle) as an outside witness."""
    import scipy.linalg as sl
    from workloads import fem_problem
    p = fem_problem("fw", 3, 6, 9, "periodic", seed=23, n_wells=3)
    Hd, Sd = p.dense()
    E_bf, w, gap = oracle_mod.brute_force_generalized(Hd, Sd, p.m)
    assert gap > 1e-3
    assert np.max(np.abs(w - sl.eigh(Hd, Sd, eigvals_only=True))) < 1e-11
    H, S = _gen_mats(oracle_mod, p)
    r = oracle_mod.solve(H, p.C0(), oracle_mod.OracleOptions(tol=1e-10, k_rot=50), S=S)
    assert r.converged
    assert abs(r.E_G - E_bf) < 1e-12 * abs(E_bf)
    assert np.max(np.abs(r.eigenvalues - w[:p.m])) < 1e-11


def _omega_gen(H, S, C, P, a):
    B = C + a * P
    return float(np.trace(np.linalg.solve(B.T @ (S @ B), B.T @ (H @ B))))


def test_generalized_gradient_and_curvature(oracle_mod):
    """-tr(P^T G) is the slope of E along P under the S constraint, and at an
    S-orthonormal Ritz basis with P S-orthogonal to C the line step's
    curvature 2 sum_j (p_j.H p_j - A_jj p_j.S p_j) is the second derivative
    (central differences, O(eps^2))."""
    import scipy.linalg as sl
    from workloads import fem_problem
    p = fem_problem("fg", 3, 6, 6, "periodic", seed=5, n_wells=2)
    H, S = _gen_mats(oracle_mod, p)
    C = oracle_mod.orthonormalize_generalized(S, p.C0())
    A = C.T @ (H @ C)
    _, U = sl.eigh(0.5 * (A + A.T))
    C = C @ U
    E0, G, X, A, Z = oracle_mod.energy_gradient_generalized(H, S, C)
    assert np.max(np.abs(A - np.diag(np.diag(A)))) < 1e-12 * np.max(np.abs(A))
    assert np.max(np.abs(C.T @ G)) < 1e-12 * np.linalg.norm(G)
    P = np.random.default_rng(8).standard_normal(C.shape)
    eps = 1e-5
    fd = (_omega_gen(H, S, C, P, eps) - _omega_gen(H, S, C, P, -eps)) / (2 * eps)
    assert abs(fd - (-np.sum(P * G))) < 1e-6 * abs(fd)
    P -= C @ (Z.T @ P)                       # S-orthogonal to C
    P /= np.sqrt(np.einsum("ij,ij->j", P, S @ P))[None, :]
    assert np.max(np.abs(Z.T @ P)) < 1e-12
    Y, SP = H @ P, S @ P
    _, info = oracle_mod.line_step(P, Y, G, np.diag(A).copy(), SP)
    curv = info["curv"]
    om0 = _omega_gen(H, S, C, P, 0.0)
    errs = []
    for e in (4e-3, 2e-3, 1e-3):
        fd2 = (_omega_gen(H, S, C, P, e) - 2 * om0 + _omega_gen(H, S, C, P, -e)) / e ** 2
        errs.append(abs(fd2 - curv) / abs(curv))
    assert errs[-1] < 1e-5 and errs[0] / errs[1] > 3.0


# ------------------------------------- polynomial (non-diagonal) preconditioner

def test_chebyshev_preconditioner_closed_form(oracle_mod):
    """On an eigenvector v of H (a Fourier mode of the periodic Laplacian,
    eigenvalue lam) the Chebyshev-iteration preconditioner acts as p(lam) v
    with p(x) = (1 - T_s((theta - (x - sigma)) / delta) / T_s(theta / delta))
    / (x - sigma), T_s the Chebyshev polynomial (cos(s arccos t) inside
    [-1, 1], cosh(s arccosh t) above); p > 0 on the spectrum, so M is
    symmetric positive definite, and the Gershgorin interval contains the
    spectrum."""
    n = 10
    p = make_problem("k", StencilSpec(3, (n, n, n), 2, "periodic", 0.5), m=1, seed=1)
    H = _H(oracle_mod, p)
    lo, hi = oracle_mod.gershgorin_bounds(H)
    assert lo == pytest.approx(0.0, abs=1e-15) and hi == pytest.approx(6.0, abs=1e-15)
    x, y, z = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    for deg in (1, 2, 4, 7):
        M = oracle_mod.chebyshev_preconditioner(H, degree=deg, shift=0.02)
        a, b = M.interval
        theta, delta = 0.5 * (a + b), 0.5 * (b - a)

        def T(s, t):
            t = np.asarray(t, dtype=float)
            return np.where(np.abs(t) <= 1, np.cos(s * np.arccos(np.clip(t, -1, 1))),
                            np.cosh(s * np.arccosh(np.maximum(np.abs(t), 1.0))) * np.sign(t) ** s)

        for k in ((0, 0, 0), (1, 0, 0), (2, 3, 1), (5, 5, 5)):
            th = 2 * np.pi * np.array(k) / n
            lam = float(np.sum(1 - np.cos(th)))
            v = np.cos(th[0] * z + th[1] * y + th[2] * x).reshape(-1, 1)   # x fastest
            assert np.allclose(H @ v, lam * v, atol=1e-12)
            xs = lam - M.sigma
            want = (1.0 - T(deg, (theta - xs) / delta) / T(deg, theta / delta)) / xs
            got = M(v)
            assert np.max(np.abs(got - want * v)) < 1e-12 * max(1.0, abs(want))
            assert want > 0


def test_chebyshev_preconditioner_spd_and_solve(oracle_mod):
    """M = p(H) formed densely on a tiny wells problem is symmetric with
    positive eigenvalues, and the preconditioned solve reaches the closed-form
    C1 energy in far fewer iterations than plain CG."""
    p = make_problem("w5", StencilSpec(3, (5, 5, 5), 2, "periodic", 0.5), m=4, seed=2, n_wells=2)
    H = _H(oracle_mod, p)
    M = oracle_mod.chebyshev_preconditioner(H, degree=4)
    Md = M(np.eye(p.N))
    assert np.max(np.abs(Md - Md.T)) < 1e-13 * np.max(np.abs(Md))
    assert np.linalg.eigvalsh(0.5 * (Md + Md.T)).min() > 0
    q = config_problem("c1")
    Hq = _H(oracle_mod, q)
    plain = oracle_mod.solve(Hq, q.C0(), oracle_mod.OracleOptions(tol=1e-9, k_rot=50))
    pre = oracle_mod.solve(Hq, q.C0(), oracle_mod.OracleOptions(tol=1e-9, k_rot=50, chebyshev=4))
    exact = 54 * (1 - math.cos(math.pi / 8))
    assert pre.converged and abs(pre.E_G - exact) < 1e-12 * exact
    assert pre.iterations < 0.5 * plain.iterations
