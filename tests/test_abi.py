"""The C ABI library: loads, exports every entry point include/logdet.h
declares, and its host-only paths (constants, argument checks) behave.
No GPU compute happens here."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2405_03474_amd as L
from paper_2405_03474_amd import _binding as B
from oracle import rational

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "logdet.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(B.EXPORTED)


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(B.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.parametrize("k", [1, 3, 5])
def test_library_constants_match_oracle(k):
    b, a, c = L.rational_coeffs(k)
    ob, oa, oc = rational.partial_fraction(k)
    assert b == pytest.approx(ob, rel=1e-15)
    np.testing.assert_allclose(a, oa, rtol=2e-15)
    np.testing.assert_allclose(c, oc, rtol=2e-15)


def test_library_constants_reject_even_or_out_of_range_orders():
    for k in (0, 2, 4, 6, 7):
        with pytest.raises(L.LogdetError) as ei:
            L.rational_coeffs(k) if k > 0 else B._check(B.load().ld_rational_coeffs(
                0, ctypes.byref(ctypes.c_double()), (ctypes.c_double * 1)(), (ctypes.c_double * 1)()))
        assert ei.value.status == B.LD_EINVAL


def test_null_context_is_rejected_before_any_work():
    lib = B.load()
    op = B.Operator(X=None, n=10, d=3, kind=0, lengthscale=1.0, variance=1.0, noise=0.1,
                    precision=0, M_stored=None)
    res = B.Result()
    st = lib.logdet_estimate(None, ctypes.byref(op), None, 3, 4, 0, 1e-6, 10, ctypes.byref(res), None)
    assert st == B.LD_EINVAL
    assert b"context" in lib.ld_last_error()
    assert lib.kernel_matmat(None, ctypes.byref(op), None, 1, None) == B.LD_EINVAL


def _sizing_operator(n=5000, d=3, precision=0):
    # X is never dereferenced by the sizing query: any non-null address
    return B.Operator(X=ctypes.c_void_p(4096), n=n, d=d, kind=1, lengthscale=0.2, variance=1.0,
                      noise=1e-3, precision=precision, M_stored=None)


def test_workspace_bytes_host_logic():
    lib = B.load()
    op = _sizing_operator()
    base = lib.ld_workspace_bytes(ctypes.byref(op), 32, 100, 10, 3)
    assert base > 0
    # grows with the probe block and the rank; covers every order alike
    assert lib.ld_workspace_bytes(ctypes.byref(op), 64, 100, 10, 3) > base
    assert lib.ld_workspace_bytes(ctypes.byref(op), 32, 400, 10, 3) > base
    assert lib.ld_workspace_bytes(ctypes.byref(op), 32, 100, 10, 5) == base
    # at least the probe block and the five CG vectors of n x s
    assert base >= 6 * 5000 * 32 * 8
    for bad in ((0, 100, 10, 3), (32, 0, 10, 3), (32, 100, -1, 3), (32, 4995, 10, 3),
                (32, 100, 10, 2)):
        assert lib.ld_workspace_bytes(ctypes.byref(op), *bad) == 0
        assert lib.ld_last_error()
    bad_op = _sizing_operator(d=0)
    assert lib.ld_workspace_bytes(ctypes.byref(bad_op), 32, 100, 10, 3) == 0


def test_set_workspace_argument_checks():
    lib = B.load()
    assert lib.ld_set_workspace(None, None, 0) == B.LD_EINVAL
    assert b"context" in lib.ld_last_error()
