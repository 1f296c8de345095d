"""Host-only checks of the C ABI: the library builds, loads and exports every
function that include/tracemin.h declares, with no GPU compute calls."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tracemin.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(tm_[a-z_0-9]+)\s*\(", text))
    return sorted(n for n in names if not n.endswith("_fn"))


@pytest.fixture(scope="module")
def lib():
    from paper_1108_4509_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_1108_4509_amd import build
        build.build()
    return _abi.lib()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("tm_create", "tm_destroy", "tm_set_matrix_csr", "tm_set_matrix_stencil",
                     "tm_free_matrix", "tm_solve", "tm_spmm", "tm_gram", "tm_rotate",
                     "tm_energy_grad", "tm_orthonormalize", "tm_cholesky_inverse",
                     "tm_sym_eig", "tm_status_string", "tm_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    from paper_1108_4509_amd import _abi
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in _abi.SIGNATURES, f"{name} missing from the Python binding"


def test_pure_host_entry_points(lib):
    from paper_1108_4509_amd import _abi
    assert lib.tm_status_string(0) == b"ok"
    assert lib.tm_status_string(_abi.TM_ENOTSPD) == b"C^T C not positive definite"
    assert [lib.tm_leading_dim(m) for m in (1, 27, 32, 33, 256, 1000)] == [32, 32, 32, 64, 256, 1024]
    o = _abi.tm_opts()
    lib.tm_opts_default(ctypes.byref(o))
    assert o.precision == _abi.TM_FULL_DP and o.k_rot == 50 and o.max_iter > 0
    assert lib.tm_matrix_rows(None) == -1


def test_struct_layouts_match_header(lib):
    """The ctypes mirrors have the sizes the C compiler gives the structs."""
    from paper_1108_4509_amd import _abi
    assert ctypes.sizeof(_abi.tm_opts) == 8 * 4 + 3 * 8 + 8 + 2 * 4 + 8 + 2 * 8
    assert ctypes.sizeof(_abi.tm_result) == 6 * 8 + 3 * 8 + 6 * 4
    assert ctypes.sizeof(_abi.tm_stencil) == 6 * 4 + 8 + 8


def test_null_arguments_rejected_without_device(lib):
    from paper_1108_4509_amd import _abi
    out = ctypes.c_void_p()
    assert lib.tm_create(0, None, None, None) == _abi.TM_EINVAL
    assert lib.tm_solve(None, None, 1, 1e-8, None, None, None, None, None, None, 0) == _abi.TM_EINVAL
    assert lib.tm_set_matrix_csr(None, 1, None, None, None, 0, ctypes.byref(out)) == _abi.TM_EINVAL
    assert lib.tm_random_block(None, 4, 2, 0, None) == _abi.TM_EINVAL
    assert b"null" in lib.tm_last_error()


def test_serving_structs_and_footprint(lib):
    """Serving structs match the header; the admission bound grows with n and
    m, covers the blocks of the chosen precision, and malformed calls are
    rejected without touching a device."""
    from paper_1108_4509_amd import _abi
    assert ctypes.sizeof(_abi.tm_server_opts) == 4 + 4 + 8 + 4 + 4
    assert ctypes.sizeof(_abi.tm_request) == 8 * 4 + 4 + 4 + 8 * 3
    assert ctypes.sizeof(_abi.tm_server_stats) == 6 * 8 + 6 * 8 + 2 * 8 + 4 * 8 + 8

    def fp(n, nnz, m, precision):
        o = _abi.tm_opts()
        lib.tm_opts_default(ctypes.byref(o))
        o.precision = precision
        out = ctypes.c_uint64()
        assert lib.tm_solve_footprint(n, nnz, m, ctypes.byref(o), ctypes.byref(out)) == 0
        return out.value

    n, m = 110592, 256
    ld = 256
    for prec, blocks in ((_abi.TM_FULL_DP, 7 * 8), (_abi.TM_MP2, 3 * 8 + 4 * 4),
                         (_abi.TM_MIXED, 3 * 4 + 3 * 8 + 4 * 4)):
        b = fp(n, 7 * n, m, prec)
        assert b >= (blocks + 8) * n * ld          # blocks plus the start block
        assert b <= (blocks + 8) * n * ld + (256 << 20)
    assert fp(n, 7 * n, m, _abi.TM_MIXED) < fp(2 * n, 14 * n, m, _abi.TM_MIXED)
    assert fp(n, 7 * n, 128, _abi.TM_MIXED) < fp(n, 7 * n, m, _abi.TM_MIXED)
    out = ctypes.c_uint64()
    assert lib.tm_solve_footprint(10, 30, 11, None, ctypes.byref(out)) == _abi.TM_EINVAL
    bad = _abi.tm_server_opts(device=0, max_slots=0, hbm_budget=1 << 30)
    h = ctypes.c_void_p()
    assert lib.tm_server_create(ctypes.byref(bad), ctypes.byref(h)) == _abi.TM_EINVAL
    # batching options: up to 256 requests, 64..2048 block columns (0: default)
    for mb, mc in ((-1, 0), (257, 0), (8, 32), (8, 4096)):
        bad = _abi.tm_server_opts(device=0, max_slots=2, hbm_budget=1 << 30, max_batch=mb,
                                  max_batch_cols=mc)
        assert lib.tm_server_create(ctypes.byref(bad), ctypes.byref(h)) == _abi.TM_EINVAL
    assert lib.tm_server_submit(None, None, None) == _abi.TM_EINVAL
    assert lib.tm_server_poll(None, 1, None, None) == _abi.TM_EINVAL


def test_philox_reference_known_answers():
    """The numpy Philox4x32-10 used to check tm_random_block reproduces the
    known-answer vectors published with the generator (Random123 kat_vectors:
    zero counter and key; all-ones; the digits of pi)."""
    import numpy as np
    from tests.philox_ref import philox4x32_10
    cases = [((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
             ((0xffffffff,) * 4, (0xffffffff, 0xffffffff),
              (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
             ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
              (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1))]
    for ctr, key, want in cases:
        got = philox4x32_10(np.array([ctr], dtype=np.uint64), key)[0]
        assert [int(x) for x in got] == list(want)


def test_random_block_reference_is_standard_normal():
    import numpy as np
    from tests.philox_ref import random_block
    z = random_block(2000, 50, 12345)
    assert abs(z.mean()) < 0.01 and abs(z.std() - 1.0) < 0.01
    assert np.array_equal(random_block(3, 5, 7), random_block(30, 5, 7)[:3])
    assert not np.array_equal(random_block(3, 5, 7), random_block(3, 5, 8))


def test_batch_layout(lib):
    """Each problem's columns: m rounded up to 16, then widened until the
    batch spans a multiple of 64 columns (the FP32 width of the
    column-chunked SpMM); bad sizes are refused without a device."""
    import ctypes as ct
    from paper_1108_4509_amd import _abi

    def lay(k, m):
        ldg, ld = ct.c_int32(), ct.c_int32()
        assert lib.tm_batch_layout(k, m, ct.byref(ldg), ct.byref(ld)) == 0
        return ldg.value, ld.value

    assert lay(4, 16) == (16, 64)
    assert lay(8, 16) == (16, 128)
    assert lay(2, 20) == (32, 64)
    assert lay(3, 20) == (64, 192)
    assert lay(1, 16) == (64, 64)
    assert lay(4, 76) == (80, 320)
    for k in range(1, 20):
        for m in (1, 15, 16, 17, 33, 100):
            ldg, ld = lay(k, m)
            assert ldg >= m and ldg % 16 == 0 and (k * ldg) % 64 == 0 and ld == k * ldg
    x = ct.c_int32()
    assert lib.tm_batch_layout(0, 16, ct.byref(x), ct.byref(x)) == _abi.TM_EINVAL
    assert lib.tm_batch_layout(257, 16, ct.byref(x), ct.byref(x)) == _abi.TM_EINVAL
    assert lib.tm_set_matrix_batch(None, 4, None, None, None, 1, None, 0, ct.byref(ct.c_void_p())) \
        == _abi.TM_EINVAL
