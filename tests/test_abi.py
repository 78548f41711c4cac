"""The C-ABI library on the CPU: it loads, exports every function that
include/hps.h declares (and the Python binding declares exactly those), and
its host-side logic (argument checks, error reporting, the memory plan) works
without touching a GPU.  No compute call is made here."""
import ctypes
import os
import re

import pytest

from paper_2112_02211_amd import hps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hps.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)          # drop comments
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\**\s*(hps_[a-z0-9_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(hps.LIB_PATH):
        from paper_2112_02211_amd import build
        build.build()
    return hps.lib()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("hps_setup", "hps_apply", "hps_precond", "hps_op_left", "hps_gmres", "hps_free",
                 "hps_setup_bytes", "hps_last_error"):
        assert must in names
    assert len(names) >= 19


def test_every_declared_symbol_is_exported(L):
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_exactly_the_header():
    assert sorted(hps.SIGNATURES) == declared_functions()


def _err(L):
    return L.hps_last_error().decode()


def test_null_arguments_are_rejected_without_a_device(L):
    z = ctypes.c_void_p(0)
    assert L.hps_apply(None, z, z, 1) == hps.HPS_ERR_ARG and "hps_apply" in _err(L)
    assert L.hps_precond(None, z, z, 1) == hps.HPS_ERR_ARG
    assert L.hps_op_left(None, z, z, 1) == hps.HPS_ERR_ARG and "hps_op_left" in _err(L)
    assert L.hps_precond_prec(None, z, z, 1, 1) == hps.HPS_ERR_ARG
    assert L.hps_assemble_rhs(None, z, z, z, 1) == hps.HPS_ERR_ARG
    assert L.hps_set_timing(None, 1) == hps.HPS_ERR_ARG
    assert L.hps_num_unknowns(None) == -1
    assert L.hps_device_bytes(None) < 0
    assert L.hps_trim(None) == hps.HPS_ERR_ARG
    assert L.hps_solve_bytes(None, 30, 1, None) < 0
    assert L.hps_iti_build(None) == hps.HPS_ERR_ARG
    assert L.hps_iti_apply(None, z, z, 1) == hps.HPS_ERR_ARG and "hps_iti_apply" in _err(L)
    assert L.hps_iti_rhs(None, z, z, z, 1) == hps.HPS_ERR_ARG
    assert L.hps_iti_recover(None, z, z, z, z, 1) == hps.HPS_ERR_ARG
    L.hps_free(None)   # a no-op


def _setup(L, p=8, q=None, n=(2, 2, 2), kappa=10.0, eta=10.0, lo=(0, 0, 0), hi=(1, 1, 1), opts=None):
    d = hps._Domain((ctypes.c_double * 3)(*lo), (ctypes.c_double * 3)(*hi))
    ne = (ctypes.c_int * 3)(*n)
    out = ctypes.c_void_p()
    rc = L.hps_setup(ctypes.byref(d), kappa, eta, None, p, p - 2 if q is None else q, ne,
                     None if opts is None else ctypes.byref(opts), ctypes.byref(out))
    return rc, out


def test_setup_argument_checks_run_before_any_device_call(L):
    assert _setup(L, p=3)[0] == hps.HPS_ERR_UNSUPPORTED
    assert _setup(L, p=17)[0] == hps.HPS_ERR_UNSUPPORTED
    assert _setup(L, p=8, q=5)[0] == hps.HPS_ERR_UNSUPPORTED and "q must equal" in _err(L)
    assert _setup(L, n=(2, 0, 2))[0] == hps.HPS_ERR_ARG
    assert _setup(L, kappa=-1.0)[0] == hps.HPS_ERR_ARG
    assert _setup(L, hi=(1, 1, 0))[0] == hps.HPS_ERR_ARG
    assert _setup(L, n=(2, 2, 2), hi=(1, 1, 2))[0] == hps.HPS_ERR_ARG and "cubes" in _err(L)
    for bad in (-0.1, float("nan"), float("inf")):
        rc, out = _setup(L, opts=hps._Opts(1, None, 0, bad))
        assert rc == hps.HPS_ERR_ARG and "lambda_bucket" in _err(L) and not out.value
    assert L.hps_num_blocks(None) == -1


@pytest.mark.parametrize("p,n,precs,cplx", [(10, (8, 8, 8), 1, 0), (10, (8, 8, 8), 7, 0),
                                            (12, (16, 16, 16), 7, 1), (4, (1, 2, 3), 2, 0)])
def test_setup_bytes_is_the_documented_plan(L, p, n, precs, cplx):
    n1 = p - 2
    ni, nb, nl = n1 ** 3, 6 * n1 ** 2, n[0] * n[1] * n[2]
    tab = 2 * p * p + 2 * n1 * n1 + n1 + p + ni       # D, D2, V, W, E, nodes, E_Delta
    want = 8 * tab + 4 * 6 * nl + nl * ni * (16 if cplx else 8) + 16 * nl
    for bit, cw, el in ((1, 1, 16), (2, 2, 8), (4, 4, 4)):
        if precs & bit:
            want += nl * ((nb + cw - 1) // cw * cw) * nb * el
    tr = ctypes.c_int64()
    got = L.hps_setup_bytes(p, (ctypes.c_int * 3)(*n), precs, cplx, ctypes.byref(tr))
    assert got == want
    assert tr.value > 16 * nb * nb     # at least one Schur block in flight
    # FP64 blocks of the 8^3, p = 10 workload: 512 x 384^2 x 16 B
    if (p, n, precs) == (10, (8, 8, 8), 1):
        assert got - (want - nl * nb * nb * 16) == 1_207_959_552


@pytest.mark.parametrize("p,precs", [(10, 8), (16, 8), (8, 8 | 4)])
def test_setup_bytes_separable_form(L, p, precs):
    # separable J^-1: one table of 2 n1^2 + n1 + 4 complex entries, no FP64 blocks;
    # nothing transient unless reduced-precision blocks are built too
    n = (4, 3, 2)
    n1 = p - 2
    ni, nb, nl = n1 ** 3, 6 * n1 ** 2, 24
    tab = 2 * p * p + 2 * n1 * n1 + n1 + p + ni
    want = 8 * tab + 4 * 6 * nl + nl * ni * 8 + 16 * nl + 16 * (2 * n1 * n1 + n1 + 4)
    if precs & 4:
        want += nl * ((nb + 3) // 4 * 4) * nb * 4
    tr = ctypes.c_int64()
    assert L.hps_setup_bytes(p, (ctypes.c_int * 3)(*n), precs, 0, ctypes.byref(tr)) == want
    assert (tr.value > 0) == bool(precs & 4)


def test_setup_rejects_separable_with_fp64_blocks_or_buckets(L):
    rc, out = _setup(L, opts=hps._Opts(1 | 8, None, 0, 0.0))
    assert rc == hps.HPS_ERR_ARG and "SEPARABLE" in _err(L) and not out.value
    rc, out = _setup(L, opts=hps._Opts(8, None, 0, 1e-2))
    assert rc == hps.HPS_ERR_ARG and "separable" in _err(L) and not out.value
    rc, out = _setup(L, opts=hps._Opts(16, None, 0, 0.0))
    assert rc == hps.HPS_ERR_ARG and not out.value


def test_setup_bytes_rejects_bad_sizes(L):
    assert L.hps_setup_bytes(3, (ctypes.c_int * 3)(1, 1, 1), 1, 0, None) < 0
    assert L.hps_setup_bytes(8, (ctypes.c_int * 3)(1, 0, 1), 1, 0, None) < 0


def test_autotune_table_round_trip(L, tmp_path):
    # the process-wide table of block-GEMM tile shapes: set / get / rule / save / load
    hps.autotune_set(10, "fp32", 20, 4)
    assert hps.autotune_get(10, "fp32", 20) == 4
    assert hps.autotune_get(10, "fp32", 21) == 1      # rule: the 32-column panel
    assert hps.autotune_get(10, "bf16", 5) == 2       # rule: the 16-column panel
    assert hps.autotune_get(10, "fp64", 64) == 0      # rule: the 64-column panel
    path = tmp_path / "shapes.txt"
    hps.autotune_save(str(path))
    assert "gemm 10 2 20 4" in path.read_text()
    hps.autotune_set(10, "fp32", 20, -1)
    assert hps.autotune_get(10, "fp32", 20) == 1
    hps.autotune_load(str(path))
    assert hps.autotune_get(10, "fp32", 20) == 4
    bad = tmp_path / "bad.txt"
    bad.write_text("gemm 10 2 20 9 0.1\n")            # shape out of range
    with pytest.raises(hps.HPSError):
        hps.autotune_load(str(bad))
    assert hps.autotune_get(10, "fp32", 20) == 4      # unchanged
    with pytest.raises(hps.HPSError):
        hps.autotune_set(10, "fp32", 20, 6)
    hps.autotune_set(10, "fp32", 20, -1)


def test_iti_bytes_is_the_documented_plan(L):
    # R (n_b x n_b) and A_ii^-1 (n_i x n_i) complex per leaf, plus F_bi and A_ib (real, shared)
    for p, n in ((10, (8, 8, 8)), (6, (2, 3, 1))):
        n1 = p - 2
        ni, nb, nl = n1 ** 3, 6 * n1 ** 2, n[0] * n[1] * n[2]
        assert hps.iti_bytes(n, p) == 16 * nl * (nb * nb + ni * ni) + 16 * ni * nb
    assert hps.iti_bytes((8, 8, 8), 10) == 512 * 16 * (384 ** 2 + 512 ** 2) + 16 * 512 * 384
    with pytest.raises(hps.HPSError):
        hps.iti_bytes((8, 0, 8), 10)


def test_group_setup_argument_checks(L):
    d = hps._Domain((ctypes.c_double * 3)(0, 0, 0), (ctypes.c_double * 3)(1, 1, 1))
    ne = (ctypes.c_int * 3)(2, 2, 2)
    out = ctypes.c_void_p()
    k = (ctypes.c_double * 3)(10.0, 12.0, 14.0)
    for nop in (0, 65):
        assert L.hps_setup_group(ctypes.byref(d), nop, k, k, None, 8, 6, ne, None, ctypes.byref(out)) == hps.HPS_ERR_ARG
    assert L.hps_setup_group(ctypes.byref(d), 3, None, k, None, 8, 6, ne, None, ctypes.byref(out)) == hps.HPS_ERR_ARG
    bad = (ctypes.c_double * 3)(10.0, -1.0, 14.0)
    assert L.hps_setup_group(ctypes.byref(d), 3, bad, k, None, 8, 6, ne, None, ctypes.byref(out)) == hps.HPS_ERR_ARG
    opts = hps._Opts(1, None, 0, 0.01)
    assert L.hps_setup_group(ctypes.byref(d), 3, k, k, None, 8, 6, ne, ctypes.byref(opts),
                             ctypes.byref(out)) == hps.HPS_ERR_UNSUPPORTED and "groups" in _err(L)
    assert not out.value
    assert L.hps_num_operators(None) == -1
