"""Helpers shared by the GPU parity tests (imported only by tests)."""

import numpy as np

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def ctx_or_skip():
    import pytest
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1108_4509_amd as tm
    return tm.Context(0)


def gamma(k, u):
    """Higham's gamma_k = k u / (1 - k u): bound of a k-term dot product."""
    return k * u / (1.0 - k * u)


def host(t, m=None):
    a = t.detach().cpu().numpy()
    return a[:, :m] if (m is not None and a.ndim == 2) else a


def rand_block(rng, n, m, scale=1.0):
    return scale * rng.standard_normal((n, m))


def print_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)
