"""Test Hamiltonians and start blocks for the trace-minimization eigensolver.

Two families of sparse symmetric H are generated:

* The paper's benchmark matrix (Sec. 3, Eq. 14-15): the 2-D discrete
  Laplacian on an n x n grid with Dirichlet boundaries, i.e. block-tridiagonal
  with D_n = tridiag(-1, 4, -1) on the diagonal and -I_n off the diagonal.
* Three-dimensional periodic finite-difference Hamiltonians
  H = -(1/2) Lap_h + V with grid spacing 1, using either the second-order
  7-point stencil or the fourth-order 13-point stencil, and a potential V made
  of Gaussian wells.  These are the workloads the GPU path is sized for; they
  are not in the paper, which only states that H is real, symmetric and sparse
  with O(N) nonzeros (Sec. 2.1).

The kinetic operator is written as ``kinetic_scale * (-Lap_h)``, where the
one-dimensional stencil of -Lap_h is (-1, 2, -1) for order 2 and
(1, -16, 30, -16, 1)/12 for order 4.  With ``kinetic_scale = 1`` and 2-D
Dirichlet boundaries this is exactly Eq. 14-15; with ``kinetic_scale = 1/2`` it
is -(1/2) Lap_h.

Everything random is drawn from ``numpy.random.default_rng(seed)`` in a fixed
order: well centres (K x 3, uniform on [0, n) for x, y, z), well depths
(K, uniform on [-2, -0.5]), then the start block C_0 (N x m, standard normal,
row-major).  Both the oracle and the GPU path receive the arrays produced here,
so neither side owns a random number generator.
"""

from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Tuple

import numpy as np

# Per-axis coefficients of -Lap_h, as (offset, coefficient) pairs.
_NEG_LAPLACIAN_1D = {
    2: ((0, 2.0), (1, -1.0), (-1, -1.0)),
    4: ((0, 30.0 / 12.0), (1, -16.0 / 12.0), (-1, -16.0 / 12.0),
        (2, 1.0 / 12.0), (-2, 1.0 / 12.0)),
}

WELL_WIDTH = 1.5           # Gaussian standard deviation, in grid units
WELL_DEPTH = (-2.0, -0.5)  # uniform depth range


@dataclasses.dataclass(frozen=True)
class StencilSpec:
    """Matrix-free description of H = kinetic_scale * (-Lap_h) + V.

    ``dims`` lists the grid extent fastest axis first (x, y[, z]); the row
    index of grid point (x, y, z) is ``(z * ny + y) * nx + x``.
    """

    ndim: int
    dims: Tuple[int, ...]
    order: int = 2
    bc: str = "periodic"          # "periodic" or "dirichlet"
    kinetic_scale: float = 0.5

    @property
    def n(self) -> int:
        return int(np.prod(self.dims))

    def axis_coefficients(self) -> Tuple[Tuple[int, float], ...]:
        """(offset, coefficient) pairs of the 1-D kinetic stencil."""
        return tuple((o, self.kinetic_scale * c)
                     for o, c in _NEG_LAPLACIAN_1D[self.order])

    def diagonal_kinetic(self) -> float:
        """Kinetic part of every diagonal element."""
        return self.ndim * self.kinetic_scale * _NEG_LAPLACIAN_1D[self.order][0][1]


def _stencil_triplets(spec: StencilSpec) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(row, col, val) triplets of the kinetic operator, duplicates not merged."""
    dims = spec.dims
    n = spec.n
    idx = np.arange(n, dtype=np.int64)
    coords = []
    rem = idx.copy()
    for d in dims:
        coords.append(rem % d)
        rem //= d
    strides = [1]
    for d in dims[:-1]:
        strides.append(strides[-1] * d)
    rows, cols, vals = [], [], []
    # diagonal once
    rows.append(idx)
    cols.append(idx)
    vals.append(np.full(n, spec.diagonal_kinetic()))
    for axis in range(spec.ndim):
        for off, coef in spec.axis_coefficients():
            if off == 0:
                continue
            c = coords[axis] + off
            if spec.bc == "periodic":
                c = c % dims[axis]
                keep = np.ones(n, dtype=bool)
            elif spec.bc == "dirichlet":
                keep = (c >= 0) & (c < dims[axis])
            else:
                raise ValueError(f"unknown boundary condition {spec.bc!r}")
            nb = idx + (c - coords[axis]) * strides[axis]
            rows.append(idx[keep])
            cols.append(nb[keep])
            vals.append(np.full(int(keep.sum()), coef))
    return np.concatenate(rows), np.concatenate(cols), np.concatenate(vals)


def stencil_csr(spec: StencilSpec, V: Optional[np.ndarray] = None):
    """CSR arrays (rowptr int64, col int32, val float64) of the stencil plus V.

    Entries that land on the same column (small periodic grids, where +2 and -2
    wrap onto one point) are summed; columns are sorted within each row.
    """
    n = spec.n
    r, c, v = _stencil_triplets(spec)
    if V is not None:
        V = np.asarray(V, dtype=np.float64).reshape(-1)
        if V.shape[0] != n:
            raise ValueError("V has the wrong length")
        r = np.concatenate([r, np.arange(n, dtype=np.int64)])
        c = np.concatenate([c, np.arange(n, dtype=np.int64)])
        v = np.concatenate([v, V])
    key = r * n + c
    order = np.argsort(key, kind="stable")
    key = key[order]
    v = v[order]
    uniq, start = np.unique(key, return_index=True)
    vals = np.add.reduceat(v, start)
    rows = uniq // n
    cols = (uniq % n).astype(np.int32)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, cols, vals.astype(np.float64)


def laplacian_2d_dirichlet_csr(n: int):
    """The paper's H_N of Eq. 14-15 (N = n^2) as CSR arrays."""
    spec = StencilSpec(ndim=2, dims=(n, n), order=2, bc="dirichlet",
                       kinetic_scale=1.0)
    return stencil_csr(spec)


def periodic_fd_csr(n: int, order: int = 2, V: Optional[np.ndarray] = None):
    """-(1/2) Lap_h + V on an n^3 periodic grid as CSR arrays."""
    spec = StencilSpec(ndim=3, dims=(n, n, n), order=order, bc="periodic",
                       kinetic_scale=0.5)
    return stencil_csr(spec, V)


def _well_centres_depths(rng: np.random.Generator, n: int, K: int):
    centres = rng.uniform(0.0, float(n), size=(K, 3))
    depths = rng.uniform(WELL_DEPTH[0], WELL_DEPTH[1], size=K)
    return centres, depths


def gaussian_wells(n: int, K: int, rng: np.random.Generator,
                   width: float = WELL_WIDTH) -> np.ndarray:
    """Sum of K Gaussian wells on an n^3 periodic grid, flattened x-fastest.

    V(r) = sum_k d_k exp(-|r - R_k|^2 / (2 w^2)) with the minimum-image
    distance on the torus, R_k uniform in [0, n)^3 and d_k uniform in
    [-2, -0.5].  The Gaussian factorizes over axes, which is how it is
    evaluated.
    """
    centres, depths = _well_centres_depths(rng, n, K)
    grid = np.arange(n, dtype=np.float64)
    V = np.zeros((n, n, n), dtype=np.float64)   # indexed [z, y, x]
    inv2w2 = 1.0 / (2.0 * width * width)
    for k in range(K):
        f = []
        for axis in range(3):
            d = np.abs(grid - centres[k, axis]) % n
            d = np.minimum(d, n - d)
            f.append(np.exp(-d * d * inv2w2))
        ex, ey, ez = f
        V += depths[k] * (ez[:, None, None] * ey[None, :, None] * ex[None, None, :])
    return V.reshape(-1)


def start_block(rng: np.random.Generator, N: int, m: int) -> np.ndarray:
    """Random start block C_0 (N x m, row-major, standard normal entries)."""
    return rng.standard_normal((N, m))


@dataclasses.dataclass
class Problem:
    """One eigenproblem: H (stencil + V, and CSR on request), m and C_0."""

    name: str
    spec: StencilSpec
    m: int
    seed: int
    n_wells: int = 0
    V: Optional[np.ndarray] = None
    _C0: Optional[np.ndarray] = dataclasses.field(default=None, repr=False)
    _csr: Optional[tuple] = dataclasses.field(default=None, repr=False)
    _rng_state: Optional[dict] = dataclasses.field(default=None, repr=False)

    @property
    def N(self) -> int:
        return self.spec.n

    def csr(self):
        if self._csr is None:
            self._csr = stencil_csr(self.spec, self.V)
        return self._csr

    def C0(self) -> np.ndarray:
        if self._C0 is None:
            rng = np.random.default_rng()
            rng.bit_generator.state = self._rng_state
            self._C0 = start_block(rng, self.N, self.m)
        return self._C0

    def V_or_zero(self) -> np.ndarray:
        return self.V if self.V is not None else np.zeros(self.N)

    def dense(self) -> np.ndarray:
        """Dense H (small problems only)."""
        if self.N > 4096:
            raise ValueError("dense H only for N <= 4096")
        rowptr, col, val = self.csr()
        H = np.zeros((self.N, self.N))
        for r in range(self.N):
            H[r, col[rowptr[r]:rowptr[r + 1]]] += val[rowptr[r]:rowptr[r + 1]]
        return H


def make_problem(name: str, spec: StencilSpec, m: int, seed: int = 0,
                 n_wells: int = 0) -> Problem:
    """Draw the wells (if any) and fix the RNG state that C_0 is drawn from."""
    rng = np.random.default_rng(seed)
    V = None
    if n_wells > 0:
        if spec.ndim != 3 or len(set(spec.dims)) != 1:
            raise ValueError("wells are defined on cubic 3-D grids")
        V = gaussian_wells(spec.dims[0], n_wells, rng)
    p = Problem(name=name, spec=spec, m=m, seed=seed, n_wells=n_wells, V=V)
    p._rng_state = rng.bit_generator.state
    return p


def _cube(n: int, order: int = 2) -> StencilSpec:
    return StencilSpec(ndim=3, dims=(n, n, n), order=order, bc="periodic",
                       kinetic_scale=0.5)


def _square_dirichlet(n: int) -> StencilSpec:
    return StencilSpec(ndim=2, dims=(n, n), order=2, bc="dirichlet",
                       kinetic_scale=1.0)


# name -> (spec factory, m, wells)
CONFIGS: Dict[str, tuple] = {
    # 16^3 periodic 7-point, V = 0, m = 27 (closed shell 1 + 6 + 12 + 8)
    "c1": (lambda: _cube(16), 27, 0),
    # 48^3 periodic 7-point + 64 wells, m = 256
    "c2": (lambda: _cube(48), 256, 64),
    # 64^3 periodic 13-point (4th order) + 200 wells, m = 512
    "c3": (lambda: _cube(64, order=4), 512, 200),
    # 100^3 periodic 7-point + 800 wells, m = 1024
    "c4": (lambda: _cube(100), 1024, 800),
    # The paper's Table 1 rows (2-D Dirichlet Laplacian, Eq. 14-15)
    "t1_96_220": (lambda: _square_dirichlet(96), 220, 0),
    "t1_192_220": (lambda: _square_dirichlet(192), 220, 0),
    "t1_192_534": (lambda: _square_dirichlet(192), 534, 0),
    "t1_192_1064": (lambda: _square_dirichlet(192), 1064, 0),
    "t1_192_1519": (lambda: _square_dirichlet(192), 1519, 0),
}


# ------------------------------------------------------------ H x = lambda S x
# Linear finite elements on a uniform grid (spacing 1): the basis functions are
# not orthogonal, so the discretized problem is the generalized one the paper
# names for nonorthogonal bases (Sec. 2.1).  In 1-D the stiffness and mass
# matrices are K = tridiag(-1, 2, -1) and M = tridiag(1, 4, 1) / 6; on a
# tensor-product (Q1) grid H = kinetic_scale * sum_d M x .. x K_d x .. x M
# (+ diag(V)) and S = M x M (x M), both 9-point (2-D) or 27-point (3-D).

def _fem_1d(n: int, bc: str):
    import scipy.sparse as sp
    if bc == "periodic":
        if n < 3:
            raise ValueError("periodic FEM needs n >= 3")
        K = sp.diags([2.0] * n, 0, format="lil")
        M = sp.diags([4.0 / 6.0] * n, 0, format="lil")
        for i in range(n):
            for j in ((i - 1) % n, (i + 1) % n):
                K[i, j] = K[i, j] - 1.0
                M[i, j] = M[i, j] + 1.0 / 6.0
        return K.tocsr(), M.tocsr()
    if bc != "dirichlet":
        raise ValueError(f"unknown boundary condition {bc!r}")
    K = sp.diags([[-1.0] * (n - 1), [2.0] * n, [-1.0] * (n - 1)], [-1, 0, 1], format="csr")
    M = sp.diags([[1.0 / 6.0] * (n - 1), [4.0 / 6.0] * n, [1.0 / 6.0] * (n - 1)], [-1, 0, 1],
                 format="csr")
    return K, M


def _csr_arrays(A):
    A = A.tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return (A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data.astype(np.float64))


@dataclasses.dataclass
class GenProblem:
    """H x = lambda S x from Q1 finite elements: CSR arrays of H and S, m, C_0."""

    name: str
    ndim: int
    n: int
    bc: str
    m: int
    seed: int
    kinetic_scale: float = 0.5
    n_wells: int = 0
    V: Optional[np.ndarray] = None
    _mats: Optional[tuple] = dataclasses.field(default=None, repr=False)
    _C0: Optional[np.ndarray] = dataclasses.field(default=None, repr=False)
    _rng_state: Optional[dict] = dataclasses.field(default=None, repr=False)

    @property
    def N(self) -> int:
        return self.n ** self.ndim

    def _build(self):
        import scipy.sparse as sp
        if self._mats is None:
            K, M = _fem_1d(self.n, self.bc)
            H = None
            for d in range(self.ndim):
                term = None
                for a in range(self.ndim):
                    f = K if a == d else M
                    term = f if term is None else sp.kron(f, term, format="csr")
                H = term if H is None else H + term
            H = self.kinetic_scale * H
            if self.V is not None:
                H = H + sp.diags(self.V, 0, format="csr")
            S = M
            for _ in range(self.ndim - 1):
                S = sp.kron(M, S, format="csr")
            self._mats = (_csr_arrays(H), _csr_arrays(S))
        return self._mats

    def csr_H(self):
        return self._build()[0]

    def csr_S(self):
        return self._build()[1]

    def C0(self) -> np.ndarray:
        if self._C0 is None:
            rng = np.random.default_rng()
            rng.bit_generator.state = self._rng_state
            self._C0 = start_block(rng, self.N, self.m)
        return self._C0

    def dense(self):
        if self.N > 4096:
            raise ValueError("dense matrices only for N <= 4096")
        out = []
        for (rowptr, col, val) in self._build():
            A = np.zeros((self.N, self.N))
            for r in range(self.N):
                A[r, col[rowptr[r]:rowptr[r + 1]]] += val[rowptr[r]:rowptr[r + 1]]
            out.append(A)
        return tuple(out)


def fem_problem(name: str, ndim: int, n: int, m: int, bc: str = "periodic", seed: int = 0,
                n_wells: int = 0, kinetic_scale: float = 0.5) -> GenProblem:
    """Q1 finite-element H x = lambda S x on an n^ndim grid; wells (3-D cubic
    grids) as in ``make_problem``, added to H's diagonal (lumped mass: the
    rows of S sum to one)."""
    rng = np.random.default_rng(seed)
    V = None
    if n_wells > 0:
        if ndim != 3:
            raise ValueError("wells are defined on cubic 3-D grids")
        V = gaussian_wells(n, n_wells, rng)
    p = GenProblem(name=name, ndim=ndim, n=n, bc=bc, m=m, seed=seed,
                   kinetic_scale=kinetic_scale, n_wells=n_wells, V=V)
    p._rng_state = rng.bit_generator.state
    return p


def config_problem(name: str, seed: int = 0) -> Problem:
    spec_fn, m, wells = CONFIGS[name]
    return make_problem(name, spec_fn(), m, seed=seed, n_wells=wells)


def serving_stream(n_requests: int = 200, mean_interarrival_s: float = 0.05,
                   seed: int = 0) -> List[dict]:
    """Arrival schedule of the serving workload.

    Inter-arrival times are exponential with the given mean, grid sides are
    uniform on {16, 24, 32, 40, 48}, the well count is max(1, round(64 N / 48^3))
    and m = clamp(round(256 N / 48^3), 16, 256).  Request i draws its own wells
    and start block from seed 1000 + i.
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(mean_interarrival_s, size=n_requests)
    sides = rng.choice(np.array([16, 24, 32, 40, 48]), size=n_requests)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    ref = 48 ** 3
    for i in range(n_requests):
        n = int(sides[i])
        N = n ** 3
        wells = max(1, int(round(64 * N / ref)))
        m = min(256, max(16, int(round(256 * N / ref))))
        out.append(dict(index=i, arrival_s=float(t[i]), side=n, N=N, m=m,
                        wells=wells, seed=1000 + i))
    return out


def serving_problem(req: dict) -> Problem:
    return make_problem(f"req{req['index']}", _cube(req["side"]), req["m"],
                        seed=req["seed"], n_wells=req["wells"])


__all__ = [
    "StencilSpec", "Problem", "stencil_csr", "laplacian_2d_dirichlet_csr",
    "periodic_fd_csr", "gaussian_wells", "start_block", "make_problem",
    "config_problem", "serving_stream", "serving_problem", "CONFIGS", "GenProblem",
    "fem_problem",
]
