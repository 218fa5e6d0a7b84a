"""The C interface on the CPU: the library loads, exports every symbol that
include/ctp.h declares, and its host-side argument checks behave as the
header documents.  No call here reaches the GPU."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ctp.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ctp_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1305_2353_amd import ctp
    if not os.path.exists(ctp.LIB_PATH):
        pytest.skip("libctp.so not built")
    return ctp.load()


def test_header_declares_the_binding_names():
    from paper_1305_2353_amd import ctp
    assert _declared() == sorted(ctp.EXPORTED)


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_default_opts(lib):
    from paper_1305_2353_amd import ctp
    o = ctp.CtpOpts()
    lib.ctp_default_opts(ctypes.byref(o))
    assert (o.method, o.u, o.small, o.prec, o.tile) == (ctp.CTP_RELAXED, 0.01, 1e-20, 0, -1)
    assert "gfx950" in ctp.ctp_version()


def test_workspace_size_and_argument_checks(lib):
    from paper_1305_2353_amd import ctp
    o = ctp.ctp_default_opts("strict")
    sz = ctypes.c_size_t()
    assert lib.ctp_workspace_size(100, 10, ctypes.byref(o), ctypes.byref(sz)) == 0
    assert sz.value >= 10 * 10 * 8 + 90 * 4
    assert lib.ctp_workspace_size(5, 10, ctypes.byref(o), ctypes.byref(sz)) == -1
    assert lib.ctp_workspace_size(10, -1, ctypes.byref(o), ctypes.byref(sz)) == -2
    bad = ctp.ctp_default_opts("relaxed", u=0.7)
    assert lib.ctp_workspace_size(10, 5, ctypes.byref(bad), ctypes.byref(sz)) == -3
    bad = ctp.ctp_default_opts("relaxed", u=0.0)
    assert lib.ctp_workspace_size(10, 5, ctypes.byref(bad), ctypes.byref(sz)) == -3
    # factor: invalid arguments are rejected on the host before any launch
    nul = ctypes.c_void_p(0)
    assert lib.ctp_factor_supernode(5, 10, nul, 5, ctypes.byref(o), nul, nul, nul, nul, nul, nul, 0, nul) == -1
    assert lib.ctp_factor_supernode(20, 10, nul, 20, ctypes.byref(o), nul, nul, nul, nul, nul, nul, 0, nul) == -3
    fake = ctypes.c_void_p(4096)
    assert lib.ctp_factor_supernode(20, 10, fake, 19, ctypes.byref(o), fake, fake, fake, fake, fake, fake,
                                    1 << 20, nul) == -4
    assert lib.ctp_factor_supernode(20, 10, fake, 20, ctypes.byref(o), fake, fake, fake, fake, fake, fake,
                                    0, nul) == -12
    assert lib.ctp_schur(20, 10, fake, 20, fake, fake, fake, 5, 6, fake, 6, ctypes.byref(o), None, 0, nul) == -9
    assert lib.ctp_schur(20, 10, fake, 20, fake, fake, fake, 0, 6, fake, 5, ctypes.byref(o), None, 0, nul) == -11
    assert lib.ctp_schur(20, 10, fake, 20, fake, fake, fake, 0, 6, fake, 6, ctypes.byref(o), fake, 16, nul) == -14
    assert lib.ctp_solve_supernode(600, 513, fake, 600, fake, fake, fake, fake, ctypes.byref(o), fake,
                                   1 << 30, nul) == -2
    assert lib.ctp_solve_supernode(600, 50, fake, 600, fake, fake, fake, fake, ctypes.byref(o), fake,
                                   16, nul) == -11
    assert lib.ctp_compress(20, 10, fake, 20, 0, fake, 10, fake, fake, fake, 1 << 20, nul) == -5
    # dense driver: host-side argument checks
    dsz = ctypes.c_size_t(0)
    assert lib.ctp_dense_workspace_size(100, 0, ctypes.byref(o), 4, ctypes.byref(dsz)) == -2
    assert lib.ctp_dense_workspace_size(100, 513, ctypes.byref(o), 4, ctypes.byref(dsz)) == -2
    assert lib.ctp_dense_workspace_size(100, 32, ctypes.byref(o), 17, ctypes.byref(dsz)) == -4
    assert lib.ctp_dense_workspace_size(100, 32, ctypes.byref(o), 4, ctypes.byref(dsz)) == 0
    small = dsz.value
    lowp = ctp.ctp_default_opts("relaxed", prec="fp32")
    assert lib.ctp_dense_workspace_size(100, 32, ctypes.byref(lowp), 4, ctypes.byref(dsz)) == 0
    assert dsz.value > small          # the FP32 trailing matrix and operand rows
    bad_prec = ctp.ctp_default_opts("relaxed", prec=3)
    assert lib.ctp_dense_workspace_size(100, 32, ctypes.byref(bad_prec), 4, ctypes.byref(dsz)) == -3
    np_ = ctypes.c_int(0)
    assert lib.ctp_ldlt_dense(100, 32, fake, 99, ctypes.byref(o), fake, fake, fake, fake, ctypes.byref(np_),
                              fake, 1 << 30, nul) == -4
    assert lib.ctp_ldlt_dense(100, 32, fake, 100, ctypes.byref(o), fake, fake, fake, fake, ctypes.byref(np_),
                              fake, 16, nul) == -12
    assert lib.ctp_ldlt_solve(100, 17, fake, 100, fake, fake, fake, fake, 100, ctypes.byref(o), 32, fake,
                              1 << 30, nul) == -2
    assert lib.ctp_ldlt_solve(100, 2, fake, 100, fake, fake, fake, fake, 100, ctypes.byref(o), 32, fake,
                              16, nul) == -13
    # batches of dense systems: host-side argument checks
    bsz = ctypes.c_size_t(0)
    assert lib.ctp_dense_batched_workspace_size(-1, 100, 32, ctypes.byref(o), ctypes.byref(bsz)) == -1
    assert lib.ctp_dense_batched_workspace_size(4, 100, 0, ctypes.byref(o), ctypes.byref(bsz)) == -3
    assert lib.ctp_dense_batched_workspace_size(4, 100, 32, ctypes.byref(lowp), ctypes.byref(bsz)) == -4
    tpp = ctp.ctp_default_opts("tpp")
    assert lib.ctp_dense_batched_workspace_size(4, 100, 32, ctypes.byref(tpp), ctypes.byref(bsz)) == -4
    assert lib.ctp_dense_batched_workspace_size(4, 100, 32, ctypes.byref(o), ctypes.byref(bsz)) == 0
    assert bsz.value > 0
    assert lib.ctp_ldlt_dense_batched(4, 100, 32, fake, 100, 9999, ctypes.byref(o), fake, fake, fake, fake, None,
                                      fake, 1 << 40, nul) == -6
    assert lib.ctp_ldlt_dense_batched(4, 100, 32, fake, 100, 10000, ctypes.byref(lowp), fake, fake, fake, fake,
                                      None, fake, 1 << 40, nul) == -7
    assert lib.ctp_ldlt_dense_batched(4, 100, 32, fake, 100, 10000, ctypes.byref(o), fake, fake, fake, fake, None,
                                      fake, 16, nul) == -14
    assert lib.ctp_ldlt_solve_batched(4, 100, 17, fake, 100, 10000, fake, fake, fake, fake, 100, 1700,
                                      ctypes.byref(o), 32, fake, 1 << 40, nul) == -3
    assert lib.ctp_ldlt_solve_batched(4, 100, 2, fake, 100, 10000, fake, fake, fake, fake, 100, 199,
                                      ctypes.byref(o), 32, fake, 1 << 40, nul) == -12
    assert lib.ctp_ldlt_solve_batched(4, 100, 2, fake, 100, 10000, fake, fake, fake, fake, 100, 200,
                                      ctypes.byref(o), 32, fake, 16, nul) == -16
    assert lib.ctp_ldlt_adjoint_batched(4, 100, 2, fake, 100, 10000, fake, fake, fake, fake, 100, 200, fake, 100,
                                        200, fake, 100, 9999, ctypes.byref(o), 32, fake, 1 << 40, nul) == -16


def test_fused_and_batched_argument_checks(lib):
    from paper_1305_2353_amd import ctp
    o = ctp.ctp_default_opts("relaxed")
    nul = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(4096)
    # fused Factor + Solve + Form: S leading dimension below n - p, workspace too small
    assert lib.ctp_supernode(100, 10, fake, 100, ctypes.byref(o), fake, fake, fake, fake, fake, fake, 89,
                             fake, 1 << 30, nul) == -12
    assert lib.ctp_supernode(100, 10, fake, 100, ctypes.byref(o), fake, fake, fake, fake, fake, fake, 90,
                             fake, 16, nul) == -13
    # batched tasks: count, info, method and workspace checks
    info = ctp.CtpBatchInfo()
    info.count = 2
    info.work_bytes = 1 << 20
    tpp = ctp.ctp_default_opts("tpp")
    args = (fake, ctypes.byref(info), fake)
    assert lib.ctp_factor_supernode_batched(-1, *args, fake, fake, fake, fake, fake, ctypes.byref(o), fake,
                                            1 << 20, nul) == -1
    assert lib.ctp_factor_supernode_batched(3, *args, fake, fake, fake, fake, fake, ctypes.byref(o), fake,
                                            1 << 20, nul) == -3
    assert lib.ctp_factor_supernode_batched(2, *args, fake, fake, fake, fake, fake, ctypes.byref(tpp), fake,
                                            1 << 20, nul) == -11
    assert lib.ctp_solve_supernode_batched(2, *args, fake, fake, fake, fake, ctypes.byref(o), fake, 16,
                                           nul) == -12
    assert lib.ctp_schur_batched(2, *args, fake, fake, fake, nul, ctypes.byref(o), fake, 1 << 20, nul) == -5
    assert lib.ctp_schur_batched(0, *args, fake, fake, fake, fake, ctypes.byref(o), fake, 1 << 20, nul) == -3


def test_noalloc_rejects_panels_beyond_its_scratch(lib):
    # checked on the host before the device is touched
    from paper_1305_2353_amd import ctp
    o = ctp.ctp_default_opts("relaxed")
    fake = ctypes.c_void_p(4096)
    sz = ctypes.c_size_t()
    assert lib.ctp_workspace_size(20000, 512, ctypes.byref(o), ctypes.byref(sz)) == 0
    assert sz.value > ctp.CTP_NOALLOC_SCRATCH_BYTES
    assert lib.ctp_supernode_noalloc(20000, 512, fake, 20000, ctypes.byref(o), fake, fake, fake, fake, fake,
                                     None, 1, None) == ctp.CTP_ERR_SCRATCH_TOO_SMALL
    assert lib.ctp_supernode_noalloc(5, 10, fake, 5, ctypes.byref(o), fake, fake, fake, fake, fake, None, 1,
                                     None) == -1


def test_scatter_argument_checks_and_plan(lib):
    from paper_1305_2353_amd import ctp
    nul = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(4096)
    # ctp_extend_add: shapes and leading dimensions checked on the host
    assert lib.ctp_extend_add(10, 11, fake, 10, fake, 1, fake, fake, fake, 20, 5, fake, 20, fake, 15, None,
                              nul) == -2
    assert lib.ctp_extend_add(10, 4, fake, 9, fake, 6, fake, fake, fake, 20, 5, fake, 20, fake, 15, None,
                              nul) == -4
    assert lib.ctp_extend_add(10, 4, fake, 10, fake, 5, fake, fake, fake, 20, 5, fake, 20, fake, 15, None,
                              nul) == -6
    assert lib.ctp_extend_add(10, 4, fake, 10, fake, 6, fake, fake, fake, 20, 21, fake, 20, fake, 15, None,
                              nul) == -11
    assert lib.ctp_extend_add(10, 4, fake, 10, fake, 6, fake, fake, fake, 20, 5, fake, 19, fake, 15, None,
                              nul) == -13
    assert lib.ctp_extend_add(10, 4, fake, 10, fake, 6, fake, fake, fake, 20, 5, fake, 20, nul, 15, None,
                              nul) == -14
    assert lib.ctp_extend_add(10, 4, fake, 10, fake, 6, fake, fake, fake, 20, 5, fake, 20, fake, 14, None,
                              nul) == -15
    # the plan numbers 64 x 64 tiles of each child's lower triangle in order
    tasks = (ctp.CtpScatterTask * 3)()
    for t, (n, p) in zip(tasks, [(64, 10), (65, 65), (200, 30)]):
        t.n, t.p, t.lda, t.lds = n, p, n, max(n - p, 1)
        t.np, t.pp, t.ldf, t.ld22 = 300, 100, 300, 200
        t.s_off = 0 if n > p else -1
        t.f22_off = 0
    assert ctp.ctp_scatter_plan(tasks) == 1 + 3 + 10
    assert [t.tile_off for t in tasks] == [0, 1, 4]
    tasks[2].lds = 169            # below n - p
    with pytest.raises(ctp.CtpError, match="-102"):
        ctp.ctp_scatter_plan(tasks)
    tasks[2].lds = 170
    tasks[1].f22_off = -1         # the parent has a trailing block
    with pytest.raises(ctp.CtpError, match="-101"):
        ctp.ctp_scatter_plan(tasks)
