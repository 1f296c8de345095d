"""Parity of each kernel of the iteration against the FP64 CPU oracle.

Every comparison is element by element on seeded inputs, with a tolerance
derived a priori from the arithmetic: a k-term FP64 (FP32) sum of products
carries at most gamma_k(u) * sum |a_i b_i| rounding error (Higham), and both
sides round, so the tests allow twice that.  Sizes span several tiles and a
ragged tail (N not a multiple of the row tiles, ld > m, partial 64-column
tiles).  Full-size cases check sampled outputs that the oracle computes one by
one.
"""

import numpy as np
import pytest

from tests.gpu_common import U32, U64, ctx_or_skip, gamma, host, print_case, rand_block
from workloads import StencilSpec, config_problem, make_problem

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


def _problems():
    return [
        ("c1", config_problem("c1")),
        ("w12", make_problem("w12", StencilSpec(3, (12, 12, 12), 2, "periodic", 0.5), m=76,
                             seed=5, n_wells=6)),
        ("o4", make_problem("o4", StencilSpec(3, (10, 11, 9), 4, "periodic", 0.5), m=40,
                            seed=6)),
        ("d2", make_problem("d2", StencilSpec(2, (37, 29), 2, "dirichlet", 1.0), m=33, seed=7)),
        ("o4d", make_problem("o4d", StencilSpec(3, (7, 6, 5), 4, "dirichlet", 0.5), m=5, seed=8)),
    ]


@pytest.mark.parametrize("name,prob", _problems(), ids=[p[0] for p in _problems()])
@pytest.mark.parametrize("stencil", [False, True], ids=["csr", "stencil"])
def test_spmm_f64(ctx, tm, orc, name, prob, stencil):
    import torch
    print_case(test="spmm_f64", problem=name, stencil=stencil, N=prob.N, m=prob.m)
    H = orc.csr_matrix(*prob.csr(), prob.N)
    Hd = tm.matrix_from_problem(ctx, prob, stencil=stencil)
    C = rand_block(np.random.default_rng(1), prob.N, prob.m)
    Cd = tm.to_block(C)
    Xd = torch.full_like(Cd, np.nan)
    tm.spmm(ctx, Hd, prob.m, Cd, Xd)
    X = orc.spmm(H, C)
    absHC = abs(H) @ np.abs(C)
    nnz_row = int(np.max(np.diff(prob.csr()[0])))
    tol = 2 * gamma(nnz_row + 1, U64) * absHC
    got = host(Xd)
    assert np.all(np.abs(got[:, :prob.m] - X) <= tol + 1e-300)
    assert np.all(got[:, prob.m:] == 0)          # padded columns stay zero


@pytest.mark.parametrize("stencil", [False, True], ids=["csr", "stencil"])
def test_spmm_f32(ctx, tm, orc, stencil):
    import torch
    prob = _problems()[1][1]
    print_case(test="spmm_f32", stencil=stencil)
    H = orc.csr_matrix(*prob.csr(), prob.N)
    Hd = tm.matrix_from_problem(ctx, prob, stencil=stencil)
    C = rand_block(np.random.default_rng(2), prob.N, prob.m).astype(np.float32)
    Cd = tm.to_block(C, dtype=torch.float32)
    Xd = torch.empty_like(Cd)
    tm.spmm(ctx, Hd, prob.m, Cd, Xd)
    # the FP32 kernel multiplies by FP32-rounded matrix values
    X = orc.spmm(H, C.astype(np.float64))
    absHC = abs(H) @ np.abs(C.astype(np.float64))
    tol = 2 * gamma(9, U32) * absHC
    assert np.all(np.abs(host(Xd, prob.m) - X) <= tol)


def _irregular_csr(rng, n, long_every, empty_every):
    """A general sparse matrix: mostly 1-9 entries per row, every long_every-th
    row 100-199 entries, every empty_every-th row and the last three rows
    empty (rows of one workgroup then exceed the staged-metadata capacity when
    long rows are frequent, and empty rows sit at block ends)."""
    rowptr = [0]
    cols, vals = [], []
    for r in range(n):
        if r % empty_every == 5 or r >= n - 3:
            k = 0
        elif r % long_every == 3:
            k = int(rng.integers(100, 200))
        else:
            k = int(rng.integers(1, 10))
        c = np.sort(rng.choice(n, size=k, replace=False))
        cols.append(c)
        vals.append(rng.standard_normal(k))
        rowptr.append(rowptr[-1] + k)
    return (np.array(rowptr, dtype=np.int64), np.concatenate(cols).astype(np.int32),
            np.concatenate(vals))


@pytest.mark.parametrize("long_every", [23, 5], ids=["staged", "unstaged"])
@pytest.mark.parametrize("m", [64, 96, 256])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_spmm_irregular_csr(ctx, tm, orc, long_every, m, dt):
    """General CSR rows (empty, short and long) through every SpMM path:
    column chunks with LDS-staged row data, chunks reading the row data from
    memory when a workgroup's rows hold too many entries, and the whole-row
    kernels for widths that are not a multiple of a chunk."""
    import torch
    n = 3001
    print_case(test="spmm_irregular", long_every=long_every, m=m, dt=dt)
    rng = np.random.default_rng(long_every * 1000 + m)
    rowptr, col, val = _irregular_csr(rng, n, long_every, 17)
    Hd = tm.set_matrix_csr(ctx, rowptr, col, val)
    H = orc.csr_matrix(rowptr, col, val, n)
    C = rand_block(np.random.default_rng(3), n, m)
    tdt, u = (torch.float64, U64) if dt == "f64" else (torch.float32, U32)
    if dt == "f32":
        C = C.astype(np.float32).astype(np.float64)
    Cd = tm.to_block(C, dtype=tdt)
    Xd = torch.full_like(Cd, np.nan)
    tm.spmm(ctx, Hd, m, Cd, Xd)
    X = orc.spmm(H, C)
    nnz_row = int(np.max(np.diff(rowptr)))
    absH = abs(H)
    if dt == "f32":
        # the FP32 kernel multiplies by FP32-rounded matrix values
        absHC = absH @ np.abs(C)
        tol = 2 * gamma(nnz_row + 2, u) * absHC
    else:
        tol = 2 * gamma(nnz_row + 1, u) * (absH @ np.abs(C))
    got = host(Xd)
    assert np.all(np.abs(got[:, :m] - X) <= tol + 1e-300)
    assert np.all(got[n - 3:, :m] == 0)          # empty rows give zero rows
    assert np.all(got[:, m:] == 0)               # padded columns stay zero


@pytest.mark.parametrize("n,m", [(5000, 27), (3001, 76), (4099, 130), (2050, 256), (1500, 512),
                                 (700, 1)])
@pytest.mark.parametrize("shift", [False, True], ids=["plain", "shift"])
def test_gram_bf16x3(ctx, tm, n, m, shift):
    """Two-term BF16 operands on BF16 matrix cores: each operand is carried to
    2^-16 relative and the dropped lo*lo product is 2^-16 of |a||b|, so
    |err| <= 4 * 2^-16 * S + gamma_{3K}(u32) * S with S = |A|^T |B'| and K the
    rows one workgroup accumulates in FP32 (<= n / 8).  A BF16-only product
    (a dropped cross term) is off by up to 2^-8 S and fails this."""
    import torch
    print_case(test="gram_bf16x3", n=n, m=m, shift=shift)
    rng = np.random.default_rng(n + m)
    A = rand_block(rng, n, m).astype(np.float32)
    B = rand_block(rng, n, m).astype(np.float32)
    h = rng.standard_normal(m) if shift else None
    Ad = tm.to_block(A, dtype=torch.float32)
    Bd = tm.to_block(B, dtype=torch.float32)
    hd = torch.tensor(h, device=Ad.device) if shift else None
    got = host(tm.gram(ctx, m, Ad, Bd, h=hd, bf16x3=True))
    A64, B64 = A.astype(np.float64), B.astype(np.float64)
    Bp = B64 - A64 * h[None, :] if shift else B64
    ref = A64.T @ Bp
    S = np.abs(A64).T @ np.abs(Bp)
    tol = (4 * 2.0 ** -16 + gamma(3 * ((n + 7) // 8), U32)) * S
    assert np.all(np.abs(got - ref) <= tol)


@pytest.mark.parametrize("n,m", [(5000, 27), (3001, 76), (4099, 130), (2050, 256), (1500, 512),
                                 (700, 1), (64, 64), (1100, 1024), (1600, 1519)])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_gram(ctx, tm, n, m, dt):
    import torch
    print_case(test="gram", n=n, m=m, dt=dt)
    rng = np.random.default_rng(n + m)
    A = rand_block(rng, n, m)
    B = rand_block(rng, n, m)
    h = rng.standard_normal(m)
    tdt, u = (torch.float64, U64) if dt == "f64" else (torch.float32, U32)
    if dt == "f32":
        A, B = A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
    Ad, Bd = tm.to_block(A, dtype=tdt), tm.to_block(B, dtype=tdt)
    hd = torch.from_numpy(h).cuda()
    # plain product
    got = host(tm.gram(ctx, m, Ad, Bd))
    ref = A.T @ B
    tol = 2 * gamma(n, u) * (np.abs(A).T @ np.abs(B))
    assert np.all(np.abs(got - ref) <= tol)
    # symmetric product (upper tiles only, mirrored)
    got = host(tm.gram(ctx, m, Ad, Ad))
    ref = A.T @ A
    tol = 2 * gamma(n, u) * (np.abs(A).T @ np.abs(A))
    assert np.all(np.abs(got - ref) <= tol)
    # shifted product A^T (B - A diag(h)) (Fig. 2, steps (5)-(6)); the shift is
    # formed in FP64 and rounded once to the matrix-core precision
    got = host(tm.gram(ctx, m, Ad, Bd, h=hd))
    Bs = B - A * h[None, :]
    ref = A.T @ Bs
    tol = 2 * gamma(n + 2, u) * (np.abs(A).T @ (np.abs(B) + np.abs(A) * np.abs(h)[None, :]))
    assert np.all(np.abs(got - ref) <= tol)


@pytest.mark.parametrize("n,m", [(5000, 27), (3001, 76), (2050, 256), (1100, 512), (1030, 1024),
                                 (1600, 1519)])
@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_rotate(ctx, tm, n, m, dt):
    import torch
    print_case(test="rotate", n=n, m=m, dt=dt)
    rng = np.random.default_rng(3 * n + m)
    A = rand_block(rng, n, m)
    W = rng.standard_normal((m, m))
    tdt, u = (torch.float64, U64) if dt == "f64" else (torch.float32, U32)
    if dt == "f32":
        A = A.astype(np.float32).astype(np.float64)
        W = W.astype(np.float32).astype(np.float64)
    Ad = tm.to_block(A, dtype=tdt)
    out = tm.rotate(ctx, m, Ad, torch.from_numpy(W).cuda())
    ref = A @ W
    tol = 2 * gamma(m, u) * (np.abs(A) @ np.abs(W))
    got = host(out)
    assert np.all(np.abs(got[:, :m] - ref) <= tol)
    assert np.all(got[:, m:] == 0)


@pytest.mark.parametrize("name,prob", _problems()[:3], ids=[p[0] for p in _problems()[:3]])
def test_energy_grad_alg2_full_dp(ctx, tm, orc, name, prob):
    print_case(test="energy_grad_dp", problem=name)
    H = orc.csr_matrix(*prob.csr(), prob.N)
    Hd = tm.matrix_from_problem(ctx, prob)
    C = orc.orthonormalize(prob.C0())
    E, G, X, h, Hp = tm.energy_grad(ctx, Hd, prob.m, tm.to_block(C))
    E_o, G_o, X_o, h_o, Hp_o = orc.energy_gradient_alg2(H, C)
    n, m = C.shape
    # scales: |X| <= |H||C|; every quantity is a sum of at most n products
    absX = abs(H) @ np.abs(C)
    g = gamma(n + 16, U64)
    assert abs(E - E_o) <= 4 * g * np.sum(np.abs(C) * absX)
    assert np.all(np.abs(host(h) - h_o) <= 4 * g * np.sum(np.abs(C) * absX, axis=0))
    absXp = absX + np.abs(C) * np.abs(h_o)[None, :]
    mirror = _mirror_term(C, h_o)
    assert np.all(np.abs(host(Hp) - Hp_o) <= 4 * g * (np.abs(C).T @ absXp) + mirror)
    absG = 2 * (absXp + np.abs(C) @ np.abs(Hp_o))
    bound = 8 * g * (absG + 2 * np.abs(C) @ (np.abs(C).T @ absXp)) + 2 * np.abs(C) @ mirror
    assert np.all(np.abs(host(G, m) - G_o) <= bound)
    assert np.all(np.abs(host(X, m) - X_o) <= 2 * gamma(14, U64) * absX)


def _mirror_term(C, h):
    """H' is formed from its upper block tiles and mirrored, which is exact
    only when C^T C = I: entry (i, j) then differs from c_i . x'_j by
    (c_i . c_j)(h_j - h_i).  Bound of that term for the given (FP64) C, with
    the rounding of the check's own C^T C added."""
    n = C.shape[0]
    O = np.abs(C.T @ C - np.eye(C.shape[1])) + gamma(n, U64) * (np.abs(C).T @ np.abs(C))
    return 2 * O * np.abs(h[:, None] - h[None, :])


def test_energy_grad_mp2(ctx, tm, orc):
    """MP2 (Sec. 2.2): steps (6)-(7) on FP32 matrix cores.  X' = X - C H_D is
    formed in FP64 (the cancellation happens there) and rounded once to FP32
    for step (7), so the error of G is bounded by FP32 rounding of H', of
    C H' and of X' (u32 relative to each), not of X or C H_D."""
    prob = _problems()[1][1]
    print_case(test="energy_grad_mp2")
    H = orc.csr_matrix(*prob.csr(), prob.N)
    Hd = tm.matrix_from_problem(ctx, prob)
    C = orc.orthonormalize(prob.C0())
    E, G, X, h, Hp = tm.energy_grad(ctx, Hd, prob.m, tm.to_block(C), precision="mp2")
    E_o, G_o, X_o, h_o, Hp_o = orc.energy_gradient_alg2(H, C)
    n, m = C.shape
    absX = abs(H) @ np.abs(C)
    assert abs(E - E_o) <= 4 * gamma(n + 16, U64) * np.sum(np.abs(C) * absX)  # DP energy
    absXp = absX + np.abs(C) * np.abs(h_o)[None, :]
    mirror = _mirror_term(C, h_o)
    assert np.all(np.abs(host(Hp) - Hp_o) <= 4 * gamma(n + 4, U32) * (np.abs(C).T @ absXp) + mirror)
    Xp_o = X_o - C * h_o[None, :]
    bound = 8 * gamma(n + m + 4, U32) * (np.abs(C) @ (np.abs(C).T @ absXp)) \
        + 4 * U32 * np.abs(Xp_o) + 8 * gamma(n + 16, U64) * absXp + 2 * np.abs(C) @ mirror
    assert np.all(np.abs(host(G, m) - G_o) <= bound)


def test_energy_grad_mp2_wide(ctx, tm, orc):
    """MP2 gradient at a 256-wide block (m = 250, the width whose H' and R'
    are kept in LDS by the gradient and triangular products) with a ragged
    last row strip (n = 45 x 47 = 2115 = 132 x 16 + 3); same bounds as the
    MP2 case above."""
    prob = make_problem("d250", StencilSpec(2, (45, 47), 2, "dirichlet", 1.0), m=250, seed=9)
    print_case(test="energy_grad_mp2_wide", n=prob.N, m=prob.m)
    H = orc.csr_matrix(*prob.csr(), prob.N)
    Hd = tm.matrix_from_problem(ctx, prob)
    C = orc.orthonormalize(prob.C0())
    E, G, X, h, Hp = tm.energy_grad(ctx, Hd, prob.m, tm.to_block(C), precision="mp2")
    E_o, G_o, X_o, h_o, Hp_o = orc.energy_gradient_alg2(H, C)
    n, m = C.shape
    absX = abs(H) @ np.abs(C)
    absXp = absX + np.abs(C) * np.abs(h_o)[None, :]
    mirror = _mirror_term(C, h_o)
    assert np.all(np.abs(host(Hp) - Hp_o) <= 4 * gamma(n + 4, U32) * (np.abs(C).T @ absXp) + mirror)
    Xp_o = X_o - C * h_o[None, :]
    bound = 8 * gamma(n + m + 4, U32) * (np.abs(C) @ (np.abs(C).T @ absXp)) \
        + 4 * U32 * np.abs(Xp_o) + 8 * gamma(n + 16, U64) * absXp + 2 * np.abs(C) @ mirror
    got = host(G)
    assert np.all(np.abs(got[:, :m] - G_o) <= bound)
    assert np.all(got[:, m:] == 0)


@pytest.mark.parametrize("m", [1000, 1519])
@pytest.mark.parametrize("precision", ["full_dp", "mp1", "mp2"])
def test_energy_grad_wide(ctx, tm, orc, m, precision):
    """Algorithm-2 at 1024- and 1536-wide blocks (Table 1's m = 1064 and 1519
    need ld = 1088 and 1536) on a small 2-D Dirichlet matrix, under each
    policy; bounds as in the cases above.  MP1 (i) forms G in FP64 and
    rounds it to FP32 once (u32 |G| more)."""
    n1 = 48 if m == 1000 else 41
    prob = make_problem("dw", StencilSpec(2, (n1, 45), 2, "dirichlet", 1.0), m=m, seed=13)
    print_case(test="energy_grad_wide", n=prob.N, m=m, precision=precision)
    H = orc.csr_matrix(*prob.csr(), prob.N)
    Hd = tm.matrix_from_problem(ctx, prob)
    C = orc.orthonormalize(prob.C0())
    E, G, X, h, Hp = tm.energy_grad(ctx, Hd, m, tm.to_block(C), precision=precision)
    E_o, G_o, X_o, h_o, Hp_o = orc.energy_gradient_alg2(H, C)
    n = C.shape[0]
    absX = abs(H) @ np.abs(C)
    g = gamma(n + 16, U64)
    assert abs(E - E_o) <= 4 * g * np.sum(np.abs(C) * absX)
    absXp = absX + np.abs(C) * np.abs(h_o)[None, :]
    mirror = _mirror_term(C, h_o)
    got = host(G)
    if precision == "mp2":
        assert np.all(np.abs(host(Hp) - Hp_o) <= 4 * gamma(n + 4, U32) * (np.abs(C).T @ absXp) + mirror)
        Xp_o = X_o - C * h_o[None, :]
        bound = 8 * gamma(n + m + 4, U32) * (np.abs(C) @ (np.abs(C).T @ absXp)) \
            + 4 * U32 * np.abs(Xp_o) + 8 * g * absXp + 2 * np.abs(C) @ mirror
    else:
        assert np.all(np.abs(host(Hp) - Hp_o) <= 4 * g * (np.abs(C).T @ absXp) + mirror)
        absG = 2 * (absXp + np.abs(C) @ np.abs(Hp_o))
        bound = 8 * g * (absG + 2 * np.abs(C) @ (np.abs(C).T @ absXp)) + 2 * np.abs(C) @ mirror
        if precision == "mp1":
            bound = bound + 2 * U32 * np.abs(G_o)
    assert np.all(np.abs(got[:, :m] - G_o) <= bound)
    assert np.all(got[:, m:] == 0)


def test_random_block(ctx, tm):
    """tm_random_block against Philox4x32-10 + Box-Muller written out in numpy
    from their published definitions: same counters, so the same normals to
    the rounding of log, sqrt, sin and cos; zero padding; a ragged shape."""
    from tests.philox_ref import random_block
    for n, m, seed in ((1000, 27, 0), (333, 256, 2**40 + 77)):
        print_case(test="random_block", n=n, m=m, seed=seed)
        got = host(tm.random_block(ctx, n, m, seed))
        ref = random_block(n, m, seed)
        assert np.max(np.abs(got[:, :m] - ref)) <= 64 * U64 * (1.0 + np.abs(ref).max())
        assert np.all(got[:, m:] == 0)


@pytest.mark.parametrize("n,m", [(4096, 27), (3001, 76), (2050, 256)])
@pytest.mark.parametrize("precision", ["full_dp", "mp2"])
def test_orthonormalize(ctx, tm, orc, n, m, precision):
    print_case(test="orthonormalize", n=n, m=m, precision=precision)
    rng = np.random.default_rng(n * 7 + m)
    # near-orthonormal input, as inside the iteration (C + alpha P), plus a
    # random one, as at the start (Fig. 1, C_0)
    Q = orc.orthonormalize(rng.standard_normal((n, m)))
    for C in (Q + 1e-3 * rng.standard_normal((n, m)), rng.standard_normal((n, m))):
        Cd = tm.to_block(C)
        tm.orthonormalize(ctx, m, Cd, precision=precision)
        got = host(Cd, m)
        ref = orc.orthonormalize(C)
        S = got.T @ got
        if precision == "full_dp":
            assert np.max(np.abs(S - np.eye(m))) < 64 * m * U64 * 10
            assert np.max(np.abs(got - ref)) < 1e-12 * max(1.0, np.linalg.cond(C))
        else:
            # MP1 (ii): C R' in FP32; error ~ u32 * |R'|, which is small only
            # when C is already close to orthonormal (Eq. 11-13)
            Rp = np.abs(np.triu(orc.upper_triangular_inverse(orc.cholesky_upper(C.T @ C)), 1))
            bound = 4 * gamma(m, U32) * (np.abs(C) @ Rp) + 1e-13
            assert np.all(np.abs(got - ref) <= bound)


@pytest.mark.parametrize("m", [1, 2, 5, 16, 17, 33, 65, 100, 130, 256, 300, 520, 1000, 1024,
                               1519, 2048])
def test_cholesky_inverse(ctx, tm, orc, m):
    import torch
    print_case(test="cholesky_inverse", m=m)
    rng = np.random.default_rng(m)
    B = rng.standard_normal((3 * m + 5, m))
    S = B.T @ B
    R_inv = host(tm.cholesky_inverse(ctx, torch.from_numpy(S).cuda()))
    R = orc.cholesky_upper(S)
    ref = orc.upper_triangular_inverse(R)
    cond = np.linalg.cond(R)
    assert np.all(np.tril(R_inv, -1) == 0)
    assert np.max(np.abs(R_inv - ref)) <= 64 * m * U64 * cond * np.max(np.abs(ref))
    # the defining property: R^-T S R^-1 = I
    assert np.max(np.abs(R_inv.T @ S @ R_inv - np.eye(m))) < 64 * m * U64 * cond


def test_cholesky_not_spd(ctx, tm):
    import torch
    S = np.eye(20)
    S[7, 7] = -1.0
    with pytest.raises(tm.TraceminError) as ei:
        tm.cholesky_inverse(ctx, torch.from_numpy(S).cuda())
    assert ei.value.status == tm.TM_ENOTSPD


@pytest.mark.parametrize("m,bad", [(200, 150), (150, 120), (64, 63)])
def test_cholesky_breakdown_later_block(ctx, tm, m, bad):
    """A breakdown past the first 64-wide block (or at the last pivot of one)
    is reported after the earlier blocks have been factored: S = B^T B with
    column `bad` of B equal to column 30 is singular at pivot `bad`."""
    import torch
    print_case(test="cholesky_breakdown", m=m, bad=bad)
    rng = np.random.default_rng(m)
    B = rng.standard_normal((3 * m, m))
    B[:, bad] = B[:, 30]
    S = B.T @ B
    with pytest.raises(tm.TraceminError) as ei:
        tm.cholesky_inverse(ctx, torch.from_numpy(S).cuda())
    assert ei.value.status == tm.TM_ENOTSPD
    # the reported pivot is the first one that broke down (1-based)
    assert f"(pivot {bad + 1})" in str(ei.value), str(ei.value)
    # the same matrix without the dependence factors
    B[:, bad] = rng.standard_normal(3 * m)
    R_inv = host(tm.cholesky_inverse(ctx, torch.from_numpy(B.T @ B).cuda()))
    assert np.all(np.isfinite(R_inv))


@pytest.mark.parametrize("m", [1, 2, 3, 27, 64, 101, 256, 600, 1024])
def test_sym_eig(ctx, tm, orc, m):
    import torch
    print_case(test="sym_eig", m=m)
    rng = np.random.default_rng(100 + m)
    B = rng.standard_normal((m, m))
    A = B + B.T
    w, U = tm.sym_eig(ctx, torch.from_numpy(A).cuda())
    w, U = host(w), host(U)
    w_o, _, _ = orc.jacobi_eigh(A)
    scale = np.linalg.norm(A)
    assert np.max(np.abs(w - w_o)) <= 64 * m * U64 * scale
    assert np.max(np.abs(A @ U - U * w[None, :])) <= 64 * m * U64 * scale
    assert np.max(np.abs(U.T @ U - np.eye(m))) <= 64 * m * U64


@pytest.mark.parametrize("m", [1519, 2048])
def test_sym_eig_wide(ctx, tm, m):
    """Widths past the oracle's reach in test time (Table 1's m = 1519 and the
    limit 2048): the 1-D Dirichlet Laplacian with a diagonal ramp has no
    degenerate eigenvalues; eigenvalues against numpy's LAPACK as an outside
    witness, residuals and orthogonality at any size, and the trace."""
    import torch
    print_case(test="sym_eig_wide", m=m)
    A = 2 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1) + np.diag(np.linspace(0.0, 1.0, m))
    w, U = tm.sym_eig(ctx, torch.from_numpy(A).cuda())
    w, U = host(w), host(U)
    scale = np.linalg.norm(A)
    assert np.max(np.abs(w - np.linalg.eigvalsh(A))) <= 64 * m * U64 * scale
    assert np.max(np.abs(A @ U - U * w[None, :])) <= 64 * m * U64 * scale
    assert np.max(np.abs(U.T @ U - np.eye(m))) <= 64 * m * U64
    # the sum of m eigenvalues, each within the bound above, with independent
    # rounding: about sqrt(m) times one eigenvalue's bound
    assert abs(np.sum(w) - np.trace(A)) <= 64 * m * U64 * scale * np.sqrt(m)


def test_sym_eig_closed_form(ctx, tm):
    """1-D Dirichlet Laplacian: eigenvalues 2 - 2 cos(k pi / (n + 1))."""
    import torch
    n = 50
    A = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    w, _ = tm.sym_eig(ctx, torch.from_numpy(A).cuda())
    exact = np.sort(2 - 2 * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))
    # Jacobi is backward stable: |dw| <= c n u ||A||_F with a modest c
    assert np.max(np.abs(host(w) - exact)) <= 64 * n * U64 * np.linalg.norm(A)


# ------------------------------------------------------- full-size sampling

@pytest.fixture(scope="module")
def c2():
    return config_problem("c2")


@pytest.mark.parametrize("stencil", [False, True], ids=["csr", "stencil"])
def test_c2_spmm_sampled(ctx, tm, orc, c2, stencil):
    import torch
    print_case(test="c2_spmm_sampled", stencil=stencil)
    H = orc.csr_matrix(*c2.csr(), c2.N)
    Hd = tm.matrix_from_problem(ctx, c2, stencil=stencil)
    C = c2.C0()
    for dt, u in ((torch.float64, U64), (torch.float32, U32)):
        Cd = tm.to_block(C, dtype=dt)
        Xd = torch.empty_like(Cd)
        tm.spmm(ctx, Hd, c2.m, Cd, Xd)
        rows = np.random.default_rng(0).choice(c2.N, 2000, replace=False)
        Cr = host(Cd, c2.m).astype(np.float64)
        ref = np.asarray(H[rows] @ Cr)
        absref = np.asarray(abs(H)[rows] @ np.abs(Cr))
        assert np.all(np.abs(host(Xd[rows], c2.m) - ref) <= 2 * gamma(8, u) * absref)


def test_c2_gram_sampled(ctx, tm, c2):
    import torch
    print_case(test="c2_gram_sampled")
    C = c2.C0()
    rng = np.random.default_rng(1)
    X = rng.standard_normal(C.shape)
    for dt, u in ((torch.float64, U64), (torch.float32, U32)):
        Cd, Xd = tm.to_block(C, dtype=dt), tm.to_block(X, dtype=dt)
        G = host(tm.gram(ctx, c2.m, Cd, Xd))
        Ch, Xh = host(Cd, c2.m).astype(np.float64), host(Xd, c2.m).astype(np.float64)
        for i, j in rng.integers(0, c2.m, size=(64, 2)):
            ref = float(Ch[:, i] @ Xh[:, j])
            bound = 2 * gamma(c2.N, u) * float(np.abs(Ch[:, i]) @ np.abs(Xh[:, j]))
            assert abs(G[i, j] - ref) <= bound


def test_c4_full_size_sampled(ctx, tm, orc):
    """The 100^3 workload at full size (N = 10^6, m = 1024, FP32 blocks, the
    shapes and launch configurations its solve uses): sampled rows of H C and
    sampled entries of S = C^T C (upper tiles, mirrored) and of the shifted
    Gram C^T (B - C diag h), each against the oracle's own sum over the
    FP32-rounded operands.  The second operand B is the start block with its
    rows rolled (a seeded permutation of the same synthetic input)."""
    import torch
    p = config_problem("c4")
    print_case(test="c4_full_size_sampled", N=p.N, m=p.m)
    m, n = p.m, p.N
    C = p.C0()
    rng = np.random.default_rng(44)
    h = rng.standard_normal(m)
    Cd = tm.to_block(C, dtype=torch.float32)
    B = np.roll(C, 12345, axis=0)
    Bd = tm.to_block(B, dtype=torch.float32)
    f32 = lambda a: a.astype(np.float32).astype(np.float64)
    # H C on sampled rows
    H = orc.csr_matrix(*p.csr(), n)
    Hd = tm.matrix_from_problem(ctx, p)
    Xd = torch.full_like(Cd, np.nan)
    tm.spmm(ctx, Hd, m, Cd, Xd)
    rows = rng.choice(n, 1000, replace=False)
    nnz_row = int(np.max(np.diff(p.csr()[0])))
    cols_needed = np.unique(H[rows].indices)
    Cr = f32(C[cols_needed])
    Hsub = H[rows][:, cols_needed]
    ref = np.asarray(Hsub @ Cr)
    absref = np.asarray(abs(Hsub) @ np.abs(Cr))
    got = Xd[torch.from_numpy(rows).cuda()].cpu().numpy().astype(np.float64)
    assert np.all(np.abs(got - ref) <= 2 * gamma(nnz_row + 1, U32) * absref)
    del Xd
    # S = C^T C and H' = C^T (B - C diag h) on sampled entries
    S = host(tm.gram(ctx, m, Cd, Cd))
    Hp = host(tm.gram(ctx, m, Cd, Bd, h=torch.from_numpy(h).cuda()))
    pairs = rng.integers(0, m, size=(48, 2))
    pairs[:8, 1] = pairs[:8, 0]           # diagonal entries
    pairs[8:16, 1] = pairs[8:16, 0] + 1   # next to the diagonal (the mirror seam)
    pairs = np.clip(pairs, 0, m - 1)
    for i, j in pairs:
        ci, cj, bj = f32(C[:, i]), f32(C[:, j]), f32(B[:, j])
        ref = float(ci @ cj)
        assert abs(S[i, j] - ref) <= 2 * gamma(n, U32) * float(np.abs(ci) @ np.abs(cj))
        if i // 64 != j // 64:
            assert S[i, j] == S[j, i]   # mirrored across 64-column blocks
        bs = bj - cj * h[j]
        ref = float(ci @ bs)
        bound = 2 * gamma(n + 2, U32) * float(np.abs(ci) @ (np.abs(bj) + np.abs(cj) * abs(h[j])))
        assert abs(Hp[i, j] - ref) <= bound


# Large blocks (65536+ rows, 128 to 1024 columns): ragged row counts, both
# stencil orders, one to eight vectors per lane in the wave-per-row kernels,
# and the fused column dots.
_LARGE_CASES = [
    ("7pt_m128", StencilSpec(3, (42, 42, 42), 2, "periodic", 0.5), 128, 3),
    ("7pt_m512", StencilSpec(3, (41, 43, 40), 2, "periodic", 0.5), 512, 0),
    ("13pt_m256", StencilSpec(3, (41, 41, 41), 4, "periodic", 0.5), 256, 4),
    ("7pt_m1024", StencilSpec(3, (42, 40, 40), 2, "dirichlet", 0.5), 1000, 0),
]


@pytest.mark.parametrize("case", _LARGE_CASES, ids=[c[0] for c in _LARGE_CASES])
@pytest.mark.parametrize("stencil", [False, True], ids=["csr", "stencil"])
def test_spmm_large_blocks(ctx, tm, orc, case, stencil):
    import torch
    name, spec, m, wells = case
    prob = make_problem(name, spec, m=m, seed=11, n_wells=wells)
    print_case(test="spmm_large", case=name, stencil=stencil, N=prob.N, m=m)
    H = orc.csr_matrix(*prob.csr(), prob.N)
    Hd = tm.matrix_from_problem(ctx, prob, stencil=stencil)
    C = rand_block(np.random.default_rng(3), prob.N, m)
    rows = np.random.default_rng(4).choice(prob.N, 1500, replace=False)
    nnz_row = int(np.max(np.diff(prob.csr()[0])))
    for dt, u in ((torch.float64, U64), (torch.float32, U32)):
        Cd = tm.to_block(C, dtype=dt)
        Xd = torch.full_like(Cd, np.nan)
        tm.spmm(ctx, Hd, m, Cd, Xd)
        Cr = host(Cd, m).astype(np.float64)
        ref = np.asarray(H[rows] @ Cr)
        absref = np.asarray(abs(H)[rows] @ np.abs(Cr))
        got = host(Xd[rows])
        assert np.all(np.abs(got[:, :m] - ref) <= 2 * gamma(nnz_row + 1, u) * absref)
        assert np.all(got[:, m:] == 0)
    # the fused h_j = c_j . (H c_j) of Algorithm-2, step (2), FP64
    Q = orc.orthonormalize(C)
    E, G, X, h, Hp = tm.energy_grad(ctx, Hd, m, tm.to_block(Q))
    Xo = orc.spmm(H, Q)
    h_o = np.einsum("ij,ij->j", Q, Xo)
    bound = 4 * gamma(prob.N + nnz_row, U64) * np.einsum("ij,ij->j", np.abs(Q), abs(H) @ np.abs(Q))
    assert np.all(np.abs(host(h) - h_o) <= bound)
