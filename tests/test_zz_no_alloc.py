"""The allocation-free Gram entry point (tm_gram_noalloc) against tm_gram.

Both compute A^T (B - A diag(h)) (or A^T B, or the symmetric A^T A) on the
same kernels; the allocation-free one keeps its split-K partials in the
library's fixed device array, with the row splits capped to fit it, so the
two may differ in summation order only: each is within the a-priori bound
2 gamma_n(u) |A|^T |B| of the exact product, so they are within twice that of
each other.  Two calls in a row, the second smaller, check that nothing of
the first call's partials survives into the second.
"""

import numpy as np
import pytest

from tests.gpu_common import U32, U64, ctx_or_skip, gamma, host, print_case, rand_block

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return ctx_or_skip()


@pytest.fixture(scope="module")
def tm():
    import paper_1108_4509_amd as tm
    return tm


def _check(tm, ctx, n, m, dt, seed):
    import torch
    rng = np.random.default_rng(seed)
    A = rand_block(rng, n, m)
    B = rand_block(rng, n, m)
    h = rng.standard_normal(m)
    tdt, u = (torch.float64, U64) if dt == "f64" else (torch.float32, U32)
    if dt != "f64":
        A, B = A.astype(np.float32).astype(np.float64), B.astype(np.float32).astype(np.float64)
    Ad, Bd = tm.to_block(A, dtype=tdt), tm.to_block(B, dtype=tdt)
    hd = torch.from_numpy(h).cuda()
    cases = [("plain", Ad, Bd, None, A.T @ B, np.abs(A).T @ np.abs(B)),
             ("sym", Ad, Ad, None, A.T @ A, np.abs(A).T @ np.abs(A)),
             ("shift", Ad, Bd, hd, A.T @ (B - A * h[None, :]),
              np.abs(A).T @ (np.abs(B) + np.abs(A) * np.abs(h)[None, :]))]
    for name, a, b, hh, ref, mag in cases:
        print_case(test="gram_noalloc", n=n, m=m, dt=dt, case=name)
        bf = dt == "bf16x3"
        want = host(tm.gram(ctx, m, a, b, h=hh, bf16x3=bf))
        out = torch.full((m, m), np.nan, dtype=torch.float64, device="cuda")
        tm.gram_noalloc(ctx, m, a, b, h=hh, out=out, bf16x3=bf)
        torch.cuda.synchronize()
        got = host(out)
        # two-term BF16 operands: 2^-16 per operand and the dropped lo*lo term,
        # plus FP32 accumulation over at most all n rows in one workgroup
        bound = (2 * gamma(n + 2, u) if not bf else 4 * 2.0 ** -16 + gamma(3 * n, U32)) * mag
        assert np.all(np.abs(got - ref) <= bound)
        assert np.all(np.abs(got - want) <= 2 * bound)


@pytest.mark.parametrize("dt", ["f64", "f32", "bf16x3"])
def test_gram_noalloc_two_calls(ctx, tm, dt):
    # a large call (many row splits; capped by the 32 MiB array at m = 1024),
    # then a smaller one on the same array
    _check(tm, ctx, 9000, 1024 if dt == "f64" else 300, dt, 1)
    _check(tm, ctx, 700, 40, dt, 2)


def test_gram_noalloc_rejects_oversize(ctx, tm):
    import torch
    n, m = 2100, 2048
    A = torch.zeros((n, tm.leading_dim(m)), dtype=torch.float32, device="cuda")
    out = torch.empty((m, m), dtype=torch.float64, device="cuda")
    with pytest.raises(tm.TraceminError) as ei:
        tm.gram_noalloc(ctx, m, A, A, out=out)
    assert ei.value.status == -2 and "scratch" in str(ei.value)
