"""Plain FP64 trace-minimization eigensolver (CPU oracle, test infrastructure).

Follows Tsuchida & Choe, "Iterative diagonalization of symmetric matrices in
mixed precision":

* E(C) = trace(C^T H C) minimized subject to C^T C = I (Sec. 2.1, Eq. 4-7);
  at the minimum E equals E_G, the sum of the m lowest eigenvalues (Eq. 2).
* Nonlinear conjugate gradients (Fig. 1) with the Polak-Ribiere gamma (Eq. 8).
* Energy and gradient (Fig. 2): Algorithm-1 is the plain form used here;
  Algorithm-2 is provided to check that the two agree.
* Cholesky orthonormalization (Fig. 4), read as Cholesky-QR: S = C^T C = R^T R
  with R upper triangular (R = L^T), and C_out = C_in R^{-1}.  Taken
  literally, C_in L^{-1} with S = L L^T does not give orthonormal columns; the
  only product of C_in with a triangular factor of S that does is C_in L^{-T}.
* Optional diagonal preconditioner G' = M G (Sec. 4, Eq. 18).
* Explicit eigenpairs from diagonalizing the m x m H once HC = CH (Eq. 9),
  also used as the occasional subspace rotation (Sec. 3, MP2 discussion).

Everything is FP64.  Library primitives used as single steps: the sparse
product H C (scipy CSR times dense) and dense matrix products (numpy).  The
Cholesky factorization, the triangular inverse and the eigensolver are written
out (the eigensolver in plain C, ``jacobi.c``).

Readings where the paper is silent (listed with their reasons in the design
notes of the repository):
* line minimization (Sec. 2.1 cites it without detail): second-order model of
  E along P, see ``line_step``;
* convergence test: rho = ||X - C A||_F = ||G||_F / 2 <= tol;
* CG restarts (gamma = 0): at i = 0, after a subspace rotation (unless the
  rotation also carries P and G_prev into the new basis, ``transport``), when
  E rose by more than ``rise_tol * |E|``, and when P is not a descent direction.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import List, Optional, Tuple

import numpy as np
import scipy.sparse

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _jacobi_lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "_tmo_jacobi.so")
        if not os.path.exists(path):
            from . import build as _build
            _build.build()
        lib = ctypes.CDLL(path)
        lib.tmo_jacobi_eigh.restype = ctypes.c_int
        lib.tmo_jacobi_eigh.argtypes = [
            ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
            ctypes.c_double, ctypes.c_int]
        _LIB = lib
    return _LIB


# --------------------------------------------------------------------------
# Building blocks
# --------------------------------------------------------------------------

def csr_matrix(rowptr, col, val, n: int):
    """The sparse symmetric H (Sec. 2.1) as a scipy CSR matrix in FP64."""
    return scipy.sparse.csr_matrix(
        (np.asarray(val, dtype=np.float64), np.asarray(col), np.asarray(rowptr)),
        shape=(n, n))


def spmm(H, C: np.ndarray) -> np.ndarray:
    """X = H C (Fig. 2, step (1) of both algorithms)."""
    return np.asarray(H @ C)


def energy_gradient_alg1(H, C: np.ndarray):
    """Fig. 2, Algorithm-1: X = HC, A = C^T X, E = tr A, G = -2 (X - C A).

    A is symmetric in exact arithmetic; it is symmetrized before use.
    Returns (E, G, X, A).
    """
    X = spmm(H, C)
    A = C.T @ X
    A = 0.5 * (A + A.T)
    E = float(np.trace(A))
    G = -2.0 * (X - C @ A)
    return E, G, X, A


def energy_gradient_alg2(H, C: np.ndarray, zero_diag: bool = True):
    """Fig. 2, Algorithm-2 (mathematically equal to Algorithm-1).

    X = HC; H_D = diag(C^T X); E = tr H_D; X' = X - C H_D; H' = C^T X';
    G = -2 (X' - C H').  diag(H') is zero in exact arithmetic and is set to
    zero explicitly (Sec. 2.2, MP2).  Returns (E, G, X, h, Hp) with h the
    diagonal of H_D.
    """
    X = spmm(H, C)
    h = np.einsum("ij,ij->j", C, X)
    E = float(np.sum(h))
    Xp = X - C * h[None, :]
    Hp = C.T @ Xp
    if zero_diag:
        np.fill_diagonal(Hp, 0.0)
    G = -2.0 * (Xp - C @ Hp)
    return E, G, X, h, Hp


class NotPositiveDefinite(ArithmeticError):
    pass


def cholesky_upper(S: np.ndarray) -> np.ndarray:
    """Textbook Cholesky S = R^T R, R upper triangular (Fig. 4, step (2)).

    Row j of R: r_jj = sqrt(s_jj - sum_k<j r_kj^2) and
    r_jl = (s_jl - sum_k<j r_kj r_kl) / r_jj for l > j.  No pivoting; a pivot
    that is not positive raises NotPositiveDefinite.
    """
    m = S.shape[0]
    R = np.zeros_like(S, dtype=np.float64)
    for j in range(m):
        d = S[j, j] - R[:j, j] @ R[:j, j]
        if not d > 0.0:
            raise NotPositiveDefinite(f"pivot {j} is {d}")
        R[j, j] = np.sqrt(d)
        R[j, j + 1:] = (S[j, j + 1:] - R[:j, j] @ R[:j, j + 1:]) / R[j, j]
    return R


def upper_triangular_inverse(R: np.ndarray) -> np.ndarray:
    """W = R^{-1} for upper-triangular R (Fig. 4, step (3)).

    Back substitution on R W = I, one row of W at a time from the bottom:
    w_i = (e_i - sum_{k>i} r_ik w_k) / r_ii.
    """
    m = R.shape[0]
    W = np.zeros_like(R, dtype=np.float64)
    for i in range(m - 1, -1, -1):
        rhs = -(R[i, i + 1:] @ W[i + 1:, :])
        rhs[i] += 1.0
        W[i, :] = rhs / R[i, i]
    return W


def orthonormalize(C: np.ndarray) -> np.ndarray:
    """Fig. 4 as Cholesky-QR: S = C^T C = R^T R, C_out = C R^{-1}."""
    S = C.T @ C
    R = cholesky_upper(S)
    W = upper_triangular_inverse(R)
    return C @ W


def jacobi_eigh(A: np.ndarray, tol: float = 1e-15, max_sweeps: int = 100):
    """Eigenvalues (ascending) and eigenvectors of a symmetric matrix.

    Cyclic Jacobi, in plain C (``jacobi.c``).  Returns (w, V, sweeps).
    """
    A = np.ascontiguousarray(A, dtype=np.float64).copy()
    n = A.shape[0]
    w = np.zeros(n)
    V = np.zeros((n, n))
    sweeps = _jacobi_lib().tmo_jacobi_eigh(
        n, A.ctypes.data, w.ctypes.data, V.ctypes.data, tol, max_sweeps)
    if sweeps < 0:
        raise ArithmeticError("Jacobi eigensolver did not converge")
    return w, V, sweeps


def ritz_rotation(H, C: np.ndarray):
    """The m x m H = C^T H C (symmetrized) and its eigendecomposition:
    returns (U, w), w ascending, so that (C U)^T H (C U) = diag(w)."""
    X = spmm(H, C)
    A = C.T @ X
    A = 0.5 * (A + A.T)
    w, U, _ = jacobi_eigh(A)
    return U, w


def rayleigh_ritz(H, C: np.ndarray):
    """Diagonalize the m x m H = C^T H C and rotate C into its eigenbasis.

    Eq. 9: at convergence HC = CH, so the eigenvalues of the m x m matrix are
    eigenvalues of H.  Returns (C U, w) with w ascending.
    """
    U, w = ritz_rotation(H, C)
    return C @ U, w


# ------------------------------------------------ generalized H x = lambda S x

def energy_gradient_generalized(H, S, C: np.ndarray):
    """Energy and gradient for H x = lambda S x with S symmetric positive
    definite (Sec. 2.1: the extension to a nonorthogonal basis).  E(C) =
    tr(C^T H C) is minimized subject to C^T S C = I; its span-invariant form
    tr((C^T S C)^{-1} C^T H C) has, at C^T S C = I, the gradient
    2 (H C - S C A) with A = C^T H C.  Algorithm-1 with the metric S:
    X = HC, Z = SC, A = C^T X (symmetrized), E = tr A, G = -2 (X - Z A).
    Returns (E, G, X, A, Z)."""
    X = spmm(H, C)
    Z = spmm(S, C)
    A = C.T @ X
    A = 0.5 * (A + A.T)
    E = float(np.trace(A))
    G = -2.0 * (X - Z @ A)
    return E, G, X, A, Z


def orthonormalize_generalized(S, C: np.ndarray) -> np.ndarray:
    """Fig. 4 in the S inner product: C^T S C = R^T R, C_out = C R^{-1}, so
    that C_out^T S C_out = I."""
    Sg = C.T @ spmm(S, C)
    R = cholesky_upper(0.5 * (Sg + Sg.T))
    return C @ upper_triangular_inverse(R)


def brute_force_generalized(H_dense: np.ndarray, S_dense: np.ndarray, m: int):
    """Brute force for tiny N: S = R^T R (the oracle's Cholesky), the standard
    problem R^{-T} H R^{-1} y = lambda y by cyclic Jacobi.  Returns (E_G,
    eigenvalues ascending, gap)."""
    R = cholesky_upper(np.asarray(S_dense, dtype=np.float64))
    W = upper_triangular_inverse(R)
    Ht = W.T @ np.asarray(H_dense, dtype=np.float64) @ W
    w, _, _ = jacobi_eigh(0.5 * (Ht + Ht.T))
    gap = float(w[m] - w[m - 1]) if m < len(w) else float("nan")
    return float(np.sum(w[:m])), w, gap


def jacobi_preconditioner(H) -> np.ndarray:
    """Diagonal preconditioner M (Eq. 18): M_ii = 1 / (H_ii - sigma).

    sigma = min(0, min_i H_ii - 1/2) keeps M symmetric positive definite.
    M approximates the inverse Hessian only through the diagonal of H; this
    particular choice is a reading (the paper fixes M only as diagonal and SPD).
    """
    d = np.asarray(H.diagonal(), dtype=np.float64)
    sigma = min(0.0, float(d.min()) - 0.5)
    return 1.0 / (d - sigma)


def gershgorin_bounds(H) -> Tuple[float, float]:
    """[lo, hi] containing the spectrum of the symmetric H (Gershgorin discs:
    H_ii -+ sum_{j != i} |H_ij|)."""
    H = H.tocsr()
    d = np.asarray(H.diagonal(), dtype=np.float64)
    off = np.asarray(abs(H).sum(axis=1)).ravel() - np.abs(d)
    return float(np.min(d - off)), float(np.max(d + off))


def chebyshev_preconditioner(H, degree: int = 4, shift: float = 0.02):
    """A non-diagonal preconditioner for Eq. 18 (Sec. 4: more elaborate
    preconditioners than a diagonal, evaluated in single precision): M =
    p(H - sigma I), the result of ``degree`` steps of the Chebyshev iteration
    (Chebyshev acceleration for a symmetric positive definite system) for
    (H - sigma I) z = g from z = 0, on the interval [a, b] = [lo - sigma,
    hi - sigma] given by the Gershgorin bounds, with sigma = lo - shift *
    (hi - lo) below the spectrum.  Its residual polynomial is r(x) =
    T_s((theta - x) / delta) / T_s(theta / delta), theta = (a + b) / 2,
    delta = (b - a) / 2, |r| < 1 on [a, b], so p(x) = (1 - r(x)) / x > 0
    there and M is symmetric positive definite.  Returns apply(G) -> M G
    (FP64 here; the GPU applies it in FP32)."""
    lo, hi = gershgorin_bounds(H)
    sigma = lo - shift * (hi - lo)
    a, b = lo - sigma, hi - sigma
    theta, delta = 0.5 * (a + b), 0.5 * (b - a)
    s1 = theta / delta

    def apply(G: np.ndarray) -> np.ndarray:
        r = G.copy()
        d = r / theta
        z = d.copy()
        rho = 1.0 / s1
        for _ in range(degree - 1):
            r = r - (spmm(H, d) - sigma * d)
            rho_new = 1.0 / (2.0 * s1 - rho)
            d = (rho_new * rho) * d + (2.0 * rho_new / delta) * r
            z = z + d
            rho = rho_new
        return z

    apply.interval = (a, b)
    apply.sigma = sigma
    apply.degree = degree
    return apply


def line_step(P: np.ndarray, Y: np.ndarray, G: np.ndarray,
              a_diag: np.ndarray, SP: Optional[np.ndarray] = None) -> Tuple[float, dict]:
    """Step length alpha along P (Fig. 1, the line minimization).

    The paper cites a line minimization without giving one.  Reading: minimize
    a second-order model of the orthonormality-invariant energy
    Omega(a) = tr[((C+aP)^T (C+aP))^{-1} (C+aP)^T H (C+aP)].  Its slope at
    a = 0 is -tr(P^T G) exactly; its curvature is taken as
    2 sum_j (p_j^T H p_j - A_jj p_j^T p_j), exact when P is orthogonal to C
    and A = C^T H C is diagonal.  alpha = tr(P^T G) / curvature, capped at
    1 / max_j ||p_j|| (no column turns by more than 45 degrees); the cap is
    also the step when the curvature is not positive.

    Generalized problem (SP = S P given): the constraint is C^T S C = I, so
    the norms above become S-norms, p_j^T S p_j (exact when C^T S P = 0).
    """
    pg = float(np.sum(P * G))
    pp = np.einsum("ij,ij->j", P, P if SP is None else SP)
    py = np.einsum("ij,ij->j", P, Y)
    curv = 2.0 * float(np.sum(py - a_diag * pp))
    cap = 1.0 / np.sqrt(float(pp.max())) if pp.max() > 0 else 0.0
    if curv > 0.0:
        alpha = min(pg / curv, cap)
    else:
        alpha = cap
    return alpha, dict(pg=pg, curv=curv, cap=cap)


# --------------------------------------------------------------------------
# Driver
# --------------------------------------------------------------------------

@dataclasses.dataclass
class OracleOptions:
    tol: float = 1e-10          # stop when ||X - C A||_F <= tol
    max_iter: int = 20000
    k_rot: int = 0              # subspace rotation every k_rot iterations (0: never)
    precondition: bool = False  # diagonal M of Eq. 18
    chebyshev: int = 0          # > 0: the polynomial M of that degree (chebyshev_preconditioner)
    cheb_shift: float = 0.02
    rise_tol: float = 1e-13     # restart CG when E rises by more than this * |E|
    transport: bool = True      # at a rotation C <- C U, also P <- P U, G_prev <- G_prev U


@dataclasses.dataclass
class OracleResult:
    E_G: float
    eigenvalues: np.ndarray
    C: np.ndarray
    iterations: int
    converged: bool
    energies: List[float]
    residual_norms: List[float]
    alphas: List[float]
    gammas: List[float]
    restarts: int
    max_residual: float
    frob_residual: float
    orth_err: float


def solve(H, C0: np.ndarray, opts: Optional[OracleOptions] = None,
          callback=None, S=None) -> OracleResult:
    """Trace minimization by nonlinear CG (Fig. 1), all in FP64.

    for i = 0, 1, ...:  E_i, G_i = -grad E(C_i) (Fig. 2); stop if converged;
    P_i = Z_i + gamma_i P_{i-1} with Z = M G (Eq. 18, Z = G without M) and the
    Polak-Ribiere gamma of Eq. 8 (M-weighted when preconditioned); alpha_i
    from ``line_step``; C_{i+1} = orthonormalize(C_i + alpha_i P_i) (Fig. 4).
    With S (sparse, symmetric positive definite) the problem is
    H x = lambda S x: the energy, gradient, orthonormalization and line step
    take the S inner product (``energy_gradient_generalized``).
    """
    o = opts or OracleOptions()
    M = jacobi_preconditioner(H) if o.precondition else None
    Mpoly = chebyshev_preconditioner(H, o.chebyshev, o.cheb_shift) if o.chebyshev > 0 else None
    gen = S is not None

    def orth(B):
        return orthonormalize_generalized(S, B) if gen else orthonormalize(B)

    def energy_grad(B):
        if gen:
            E, G, X, A, _ = energy_gradient_generalized(H, S, B)
            return E, G, X, A
        return energy_gradient_alg1(H, B)

    C = orth(np.asarray(C0, dtype=np.float64))
    energies, rhos, alphas, gammas = [], [], [], []
    G_prev = Z_prev = P_prev = None
    E_prev = None
    restart = True
    restarts = 0
    converged = False
    it = 0
    for it in range(o.max_iter):
        if o.k_rot > 0 and it > 0 and it % o.k_rot == 0:
            U, _ = ritz_rotation(H, C)
            C = C @ U
            if o.transport and P_prev is not None:
                # E(C U) = E(C) and G(C U) = G(C) U (Sec. 2.1): expressed in
                # the rotated basis the previous direction and gradient are
                # P U and G U, and the Polak-Ribiere traces are unchanged
                P_prev, G_prev, Z_prev = P_prev @ U, G_prev @ U, Z_prev @ U
            else:
                restart = True
        E, G, X, A = energy_grad(C)
        rho = 0.5 * float(np.linalg.norm(G))
        energies.append(E)
        rhos.append(rho)
        if callback is not None:
            callback(it, E, rho)
        if rho <= o.tol:
            converged = True
            break
        if E_prev is not None and E > E_prev + o.rise_tol * abs(E_prev):
            restart = True
        if Mpoly is not None:
            Z = Mpoly(G)
        else:
            Z = G * M[:, None] if M is not None else G
        if restart:
            gamma = 0.0
        else:
            gamma = float(np.sum((G - G_prev) * Z)) / float(np.sum(G_prev * Z_prev))
        P = Z + gamma * P_prev if gamma != 0.0 else Z.copy()
        if float(np.sum(P * G)) <= 0.0:
            P = Z.copy()
            gamma = 0.0
        if gamma == 0.0:
            restarts += 1
        Y = spmm(H, P)
        alpha, _ = line_step(P, Y, G, np.diag(A).copy(), spmm(S, P) if gen else None)
        alphas.append(alpha)
        gammas.append(gamma)
        C = orth(C + alpha * P)
        G_prev, Z_prev, P_prev, E_prev = G, Z, P, E
        restart = False
    iterations = it + 1 if not converged else it
    C, w = rayleigh_ritz(H, C)
    X = spmm(H, C)
    Zc = spmm(S, C) if gen else C
    R = X - Zc * w[None, :]
    col_res = np.sqrt(np.einsum("ij,ij->j", R, R))
    Sg = C.T @ Zc
    orth = float(np.max(np.abs(Sg - np.eye(Sg.shape[0]))))
    return OracleResult(
        E_G=float(np.sum(w)), eigenvalues=w, C=C, iterations=iterations,
        converged=converged, energies=energies, residual_norms=rhos,
        alphas=alphas, gammas=gammas, restarts=restarts,
        max_residual=float(col_res.max()),
        frob_residual=float(np.sqrt(np.sum(col_res ** 2))), orth_err=orth)


def brute_force_lowest(H_dense: np.ndarray, m: int):
    """Brute force for tiny N: all eigenvalues of the dense H by cyclic Jacobi.

    Returns (E_G, eigenvalues ascending, gap lambda_{m+1} - lambda_m) per
    Eq. 2 and Eq. 3.
    """
    w, _, _ = jacobi_eigh(np.asarray(H_dense, dtype=np.float64))
    gap = float(w[m] - w[m - 1]) if m < len(w) else float("nan")
    return float(np.sum(w[:m])), w, gap
