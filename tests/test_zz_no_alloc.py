"""qf_expect_noalloc (partial sums in the library's static device array, no
allocation) against qf_expect (stream-ordered workspace) through the C ABI:
two calls in a row, the second on a smaller state, plus the size limit."""
import ctypes

import numpy as np
import pytest

import qf_inputs as qi
from oracle import measure
from tests.gpu_helpers import rounded, to_dev, to_np

pytestmark = pytest.mark.gpu


def test_expect_noalloc_matches_expect_twice():
    import torch

    import paper_2409_17716_amd as qf
    cases = [(3, 12, 3, "c64", qi.zsum_terms(12)),   # 3 registers of 3^12: 390 partial sums
             (5, 4, 2, "c128", qi.z0_terms())]        # then a smaller one
    for D, n, batch, dt, terms in cases:
        print(f"[noalloc] D={D} n={n} batch={batch} {dt}", flush=True)
        psi = qi.random_state(D, n, 31 + D, batch=batch).reshape(-1)
        t = to_dev(psi, dt)
        ref = qf.qf_expect(t, n, D, terms)
        out = torch.full((2 * batch,), float("nan"), dtype=torch.float64, device="cuda")
        qf.qf_expect_noalloc(t, n, D, terms, out)
        a, b = to_np(out), to_np(ref)
        assert np.array_equal(a, b), (a, b)  # same kernels, same summation order
        for r, reg in enumerate(rounded(psi, dt).reshape(batch, -1)):
            want = measure.expect_diag(reg, D, n, terms)
            assert abs(complex(a[2 * r], a[2 * r + 1]) - want) <= 1e-12


def test_expect_noalloc_size_limit():
    """States whose partial sums exceed the scratch array are refused before
    any launch (the state pointer is never touched)."""
    import paper_2409_17716_amd as qf
    big = qf.qf_state(0x1000, 31, 2, 1, qf.QF_C64)  # 2^31 amplitudes: 524288 partial sums > 262144
    qs = (ctypes.c_int32 * 1)(0)
    td = (ctypes.c_double * 4)(1, 0, -1, 0)
    out = (ctypes.c_double * 2)()
    st = qf.lib.qf_expect_noalloc(ctypes.byref(big), 1, qs, td, out, None)
    assert st == qf.QF_ERANGE
    assert b"scratch" in qf.lib.qf_last_error()
