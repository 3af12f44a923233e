"""CPU tests of the native library's host side (no GPU needed):
  * libstokes.so loads and exports every entry point that include/stokes.h declares;
  * the closed-form saddle sparsity pattern of the library equals the oracle's
    element-overlap pattern (integer work, bit-exact);
  * the triangular-solve schedules, executed by a CPU emulator of the kernel's
    three-wave protocol, reproduce a direct triangular solve, keep every LDS slot
    read on the value of the expected row, and never deadlock.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from oracle.oracle import Oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1309_5048_amd", "csrc")


@pytest.fixture(scope="session")
def hostcheck(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("hc") / "libhostcheck.so")
    cmd = ["hipcc", "-O2", "-std=c++17", "-fPIC", "-shared", "-x", "hip", "--offload-arch=gfx950",
           "-I" + CSRC, os.path.join(ROOT, "tests", "native", "trsv_schedule_check.cpp"),
           os.path.join(CSRC, "host_setup.cpp"), "-o", out]
    subprocess.check_call(cmd)
    L = ctypes.CDLL(out)
    L.hc_pattern.argtypes = [ctypes.c_int] * 3 + [ctypes.c_void_p] * 6
    L.hc_schedule_check.argtypes = [ctypes.c_int] * 6 + [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int]
    L.hc_row_split.argtypes = [ctypes.c_int] * 5 + [ctypes.c_void_p] * 2
    return L


def test_library_exports_every_declared_symbol():
    from paper_1309_5048_amd import build as B
    if not os.path.exists(B.LIB):
        B.build()
    header = open(os.path.join(ROOT, "include", "stokes.h")).read()
    declared = sorted(set(re.findall(r"\b(stokes_[a-z_]+)\s*\(", header)))
    assert len(declared) >= 18
    lib = ctypes.CDLL(B.LIB)
    for name in declared:
        assert hasattr(lib, name), name
    from paper_1309_5048_amd import _native
    assert sorted(_native.EXPORTS) == declared


def _hc_pattern(L, N, kp, dim):
    nu, np_, nnz = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    L.hc_pattern(N, kp, dim, ctypes.byref(nu), ctypes.byref(np_), ctypes.byref(nnz), None, None, None)
    n = nu.value + np_.value
    rp = np.zeros(n + 1, np.int64)
    col = np.zeros(nnz.value, np.int32)
    aend = np.zeros(nu.value, np.int64)
    L.hc_pattern(N, kp, dim, ctypes.byref(nu), ctypes.byref(np_), ctypes.byref(nnz), rp.ctypes.data,
                 col.ctypes.data, aend.ctypes.data)
    return nu.value, np_.value, rp, col, aend


@pytest.mark.parametrize("N,kp,dim", [(5, 1, 2), (6, 2, 2), (4, 3, 2), (3, 1, 3), (3, 2, 3)])
def test_saddle_pattern_equals_oracle(hostcheck, N, kp, dim):
    n_u, n_p, rp, col, aend = _hc_pattern(hostcheck, N, kp, dim)
    o = Oracle(N, kp, dim, pattern_only=True)
    assert (n_u, n_p) == (o.n_u, o.n_p)
    K = o.saddle().tocsr()
    K.sort_indices()
    assert np.array_equal(rp, K.indptr.astype(np.int64))
    assert np.array_equal(col, K.indices.astype(np.int32))
    # the A part of each velocity row ends where the B^T columns start
    for i in range(0, n_u, max(1, n_u // 50)):
        row = col[rp[i]:rp[i + 1]]
        assert aend[i] - rp[i] == np.count_nonzero(row < n_u)


@pytest.mark.parametrize("N,kp,dim,strip", [(16, 1, 2, 8), (16, 1, 2, 1), (12, 2, 2, 4), (20, 3, 2, 8),
                                             (6, 1, 3, 2), (8, 1, 3, 1), (4, 1, 3, 4), (64, 2, 2, 8)])
def test_trsv_schedule_emulation(hostcheck, N, kp, dim, strip):
    st = np.zeros(16)
    msg = ctypes.create_string_buffer(256)
    rc = hostcheck.hc_schedule_check(N, kp, dim, strip, 7, 0, st.ctypes.data, msg, 256)
    assert rc == 0, msg.value.decode()
    assert st[7] < 1e-12 and st[8] < 1e-10, st[7:9]
    assert st[0] == st[1]  # forward and backward DAGs have the same depth


@pytest.mark.parametrize("N,kp,dim,strip,helpers", [(16, 1, 2, 8, 2), (16, 1, 2, 1, 1), (12, 2, 2, 4, 2),
                                                     (20, 3, 2, 8, 3), (64, 2, 2, 8, 2), (5, 2, 2, 8, 2),
                                                     (1, 1, 2, 8, 2), (6, 1, 3, 2, 2), (8, 1, 3, 1, 1),
                                                     (4, 1, 3, 4, 3), (1, 1, 3, 2, 2)])
def test_trsv_schedule_emulation_coupled(hostcheck, N, kp, dim, strip, helpers):
    """Schedules whose rows take their dependencies on earlier velocity components as one
    coupling value per source component, computed by helper groups: the emulated solves
    reproduce the direct ones, every LDS read holds its expected row, and no wait deadlocks.
    A dependency path passes through at most one coupling row per component boundary, so
    the level count grows by at most dim - 1."""
    st = np.zeros(16)
    msg = ctypes.create_string_buffer(256)
    rc = hostcheck.hc_schedule_check(N, kp, dim, strip, 7, helpers, st.ctypes.data, msg, 256)
    assert rc == 0, msg.value.decode()
    assert st[7] < 1e-12 and st[8] < 1e-10, st[7:9]
    st0 = np.zeros(16)
    assert hostcheck.hc_schedule_check(N, kp, dim, strip, 7, 0, st0.ctypes.data, msg, 256) == 0
    assert st0[0] <= st[0] <= st0[0] + dim - 1 and st0[1] <= st[1] <= st0[1] + dim - 1
    assert st[2] > st0[2] and st[13] > 0


@pytest.mark.slow
def test_trsv_schedule_headline_sizes(hostcheck):
    """N=256, k'=2 (1,295 levels) with the default strip; the 3D N=32, k'=1 case (341 levels)."""
    for N, kp, dim, strip, lev in ((256, 2, 2, 8, 1295), (32, 1, 3, 2, 341)):
        st = np.zeros(16)
        msg = ctypes.create_string_buffer(256)
        rc = hostcheck.hc_schedule_check(N, kp, dim, strip, 3, 0, st.ctypes.data, msg, 256)
        assert rc == 0, msg.value.decode()
        assert int(st[0]) == lev
        assert st[7] < 1e-12 and st[8] < 1e-10
    st = np.zeros(16)
    msg = ctypes.create_string_buffer(256)
    rc = hostcheck.hc_schedule_check(256, 2, 2, 8, 3, 2, st.ctypes.data, msg, 256)
    assert rc == 0, msg.value.decode()
    assert st[7] < 1e-12 and st[8] < 1e-10


@pytest.mark.parametrize("N,kp,dim", [(1, 1, 2), (3, 2, 2), (16, 1, 2), (64, 2, 2), (256, 2, 2), (6, 1, 3), (16, 3, 3)])
def test_row_split(hostcheck, N, kp, dim):
    """The row ranges of the SpMV kernels cover every row once, in order, within the block
    limits, and balance the work (entries + 16 per row) to within one row of the mean."""
    nu, np_, rp, col, aend = _hc_pattern(hostcheck, N, kp, dim)
    for which, nrows in ((0, nu + np_), (1, nu)):
        for cus in (1, 256):
            nb = ctypes.c_int()
            assert hostcheck.hc_row_split(N, kp, dim, which, cus, ctypes.byref(nb), None) == 0
            nb = nb.value
            assert 1 <= nb <= min(4096, 8 * cus) and (nb <= 8 or nb % 8 == 0)
            split = np.zeros(nb + 1, np.int32)
            hostcheck.hc_row_split(N, kp, dim, which, cus, ctypes.byref(ctypes.c_int()), split.ctypes.data)
            assert split[0] == 0 and split[-1] == nrows and np.all(np.diff(split) >= 0)
            end = rp[1:nrows + 1] if which == 0 else aend
            cost = (end - rp[:nrows]) + 16
            work = np.add.reduceat(np.append(cost, 0), split[:-1])[:nb] * (np.diff(split) > 0)
            assert work.max() <= cost.sum() / nb + 2 * cost.max()
