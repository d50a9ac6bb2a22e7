"""C-ABI checks that need no GPU: the library loads, exports every entry point
declared in include/qf.h, and rejects bad arguments before touching HIP."""
import ctypes
import os
import re

import numpy as np
import pytest

import qf_inputs as qi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qf.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qf_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def qf():
    import paper_2409_17716_amd as qf
    return qf


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["qf_state_init", "qf_apply_1q", "qf_apply_ctrl", "qf_apply_diag", "qf_apply_fused", "qf_probs",
              "qf_expect", "qf_adjoint_grad"]:
        assert n in names


def test_library_exports_every_declared_symbol(qf):
    for name in _declared():
        assert hasattr(qf.lib, name), name


def test_version(qf):
    assert qf.lib.qf_version() >= 100


def _fake_state(qf, n=3, dim=3, batch=1, dtype=0):
    return qf.qf_state(0x1000, n, dim, batch, dtype)


def test_validation_errors_before_any_hip_call(qf):
    lib = qf.lib
    U = np.eye(3, dtype=np.complex128).view(np.float64)
    pU = U.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    s = _fake_state(qf)
    assert lib.qf_apply_1q(ctypes.byref(s), 3, pU, None) == qf.QF_EINVAL
    assert b"outside" in lib.qf_last_error()
    assert lib.qf_apply_1q(ctypes.byref(s), -1, pU, None) == qf.QF_EINVAL
    assert lib.qf_apply_1q(None, 0, pU, None) == qf.QF_EINVAL
    assert lib.qf_apply_1q(ctypes.byref(s), 0, None, None) == qf.QF_EINVAL
    bad = np.array(U)
    bad[0] = np.nan
    assert lib.qf_apply_1q(ctypes.byref(s), 0, bad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                           None) == qf.QF_EINVAL
    s_null = qf.qf_state(0, 3, 3, 1, 0)
    assert lib.qf_apply_1q(ctypes.byref(s_null), 0, pU, None) == qf.QF_EINVAL
    s_dt = qf.qf_state(0x1000, 3, 3, 1, 7)
    assert lib.qf_apply_1q(ctypes.byref(s_dt), 0, pU, None) == qf.QF_EDTYPE
    s_dim = qf.qf_state(0x1000, 3, 17, 1, 0)
    assert lib.qf_apply_1q(ctypes.byref(s_dim), 0, pU, None) == qf.QF_ERANGE
    s_big = qf.qf_state(0x1000, 21, 3, 1, 0)  # 3^21 > 2^32
    assert lib.qf_apply_1q(ctypes.byref(s_big), 0, pU, None) == qf.QF_ERANGE
    s_bat = qf.qf_state(0x1000, 20, 3, 2, 0)  # 2 * 3^20 > 2^32
    assert lib.qf_apply_1q(ctypes.byref(s_bat), 0, pU, None) == qf.QF_ERANGE
    sh = (ctypes.c_int32 * 3)(0, 1, 2)
    assert lib.qf_apply_ctrl(ctypes.byref(s), 1, 1, sh, None) == qf.QF_EINVAL
    assert lib.qf_apply_ctrl(ctypes.byref(s), 5, 1, sh, None) == qf.QF_EINVAL
    assert lib.qf_apply_ctrl(ctypes.byref(s), 0, 1, None, None) == qf.QF_EINVAL
    qs = (ctypes.c_int32 * 2)(1, 1)
    ph = (ctypes.c_double * 18)()
    assert lib.qf_apply_diag(ctypes.byref(s), 2, qs, ph, None) == qf.QF_EINVAL
    assert lib.qf_apply_fused(ctypes.byref(s), 2, 2, ctypes.c_void_p(0x2000), None) == qf.QF_EINVAL
    s10 = qf.qf_state(0x1000, 4, 10, 1, 0)
    assert lib.qf_apply_fused(ctypes.byref(s10), 4, 0, ctypes.c_void_p(0x2000), None) == qf.QF_ERANGE
    assert lib.qf_probs(ctypes.byref(s), 0, None, None, None) == qf.QF_EINVAL
    mq = (ctypes.c_int32 * 2)(0, 0)
    assert lib.qf_probs(ctypes.byref(s), 2, mq, ctypes.c_void_p(0x3000), None) == qf.QF_EINVAL
    tq = (ctypes.c_int32 * 1)(4)
    td = (ctypes.c_double * 6)()
    out = (ctypes.c_double * 2)()
    assert lib.qf_expect(ctypes.byref(s), 1, tq, td, out, None) == qf.QF_EINVAL
    dg = (ctypes.c_int32 * 3)(0, 3, 0)
    assert lib.qf_state_init(ctypes.byref(s), dg, None) == qf.QF_EINVAL


def test_plan_validation_and_schedule(qf):
    # plans without custom matrices allocate nothing on the device
    c = qi.config2(n=6, layers=2)
    p = qf.plan_for(c, fuse=1)
    assert p.num_stages == len(c.ops)
    for bad in ([("rx", 0, 1, 1, 0)], [("rz", 0, 0, 0)], [("csum", 1, 1)], [("h", 9)], [("rx", 0, 0, 1, 5)]):
        with pytest.raises(qf.QfError):
            qf.Plan(3, 4, bad, 1)


def test_tile_search(qf):
    """Stage planning on the host: the swap-improved tile choice never costs
    passes (the plan keeps whichever choice has fewer), and it saves passes on
    the D=10, n=8 ansatz, whose greedy tiles leave entangling gates behind."""
    for c in (qi.config2(), qi.config3(), qi.config5(), qi.config2(n=8, layers=3)):
        greedy = qf.plan_for(c, tile_search=1)
        auto = qf.plan_for(c)
        full = qf.plan_for(c, tile_search=2)
        assert auto.num_stages <= greedy.num_stages
        assert full.num_stages <= greedy.num_stages
        assert auto.num_adjoint_stages <= greedy.num_adjoint_stages
    c5 = qi.config5()
    assert qf.plan_for(c5).num_stages < qf.plan_for(c5, tile_search=1).num_stages
    with pytest.raises(qf.QfError):
        qf.plan_for(c5, tile_search=3)


def test_fastdiv_host(tmp_path):
    """The library's division by invariant divisors (Granlund & Montgomery)
    matches plain division for divisors up to 2^32 - 1 (registers of more than
    2^31 amplitudes need the s = 32 case) on edge and random numerators."""
    import shutil
    import subprocess
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "fastdiv_check")
    src = os.path.join(ROOT, "tests", "fastdiv_check.cpp")
    r = subprocess.run([hipcc, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950", src, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout
    assert "OK" in r.stdout


def test_forced_allocation_failure_returns_enomem():
    """QF_TEST_FAIL_ALLOC=1 makes every library allocation fail with QF_ENOMEM
    before any HIP call: a plan with a custom dense gate allocates its matrix
    at creation, so creation reports QF_ENOMEM and leaves no plan behind."""
    import subprocess
    import sys
    code = (
        "import numpy as np, paper_2409_17716_amd as qf\n"
        "try:\n"
        "    qf.Plan(3, 2, [('u', 0, 2, np.eye(9))], 0)\n"
        "    print('NO ERROR')\n"
        "except qf.QfError as e:\n"
        "    print('STATUS', e.status, str(e))\n")
    env = dict(os.environ, QF_TEST_FAIL_ALLOC="1", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, cwd=ROOT)
    assert "STATUS -4" in r.stdout, r.stdout + r.stderr
    assert "QF_TEST_FAIL_ALLOC" in r.stdout


def test_adjoint_flag_validation(qf):
    """Unknown adjoint flags are refused synchronously (no HIP call)."""
    c = qi.config2(n=3, layers=1)
    p = qf.plan_for(c, fuse=1)
    s = _fake_state(qf)
    lam = qf.qf_state(0x2000, 3, 3, 1, 0)
    th = np.zeros(c.nparams)
    g = np.zeros(c.nparams)
    qs = (ctypes.c_int32 * 1)(0)
    td = (ctypes.c_double * 6)()
    PD = ctypes.POINTER(ctypes.c_double)
    st = qf.lib.qf_adjoint_grad(p._h, ctypes.byref(s), ctypes.byref(lam), th.ctypes.data_as(PD), 1, qs, td,
                                g.ctypes.data_as(PD), 4, None)
    assert st == qf.QF_EINVAL
    assert b"flags" in qf.lib.qf_last_error()


def test_single_qudit_plans(qf):
    """n = 1 registers: every schedule plans (the tile is the whole register)."""
    c = qi.Circuit(5, 1, [("h", 0), ("rx", 0, 0, 3, 0), ("clock", 0, 2), ("ry", 0, 1, 4, 1), ("x", 0, 3)],
                   np.array([0.3, -1.1]))
    for fuse in (0, 1, 2, 3):
        p = qf.plan_for(c, fuse=fuse)
        assert p.num_stages >= 1
    qf.qf_shutdown()
    qf.qf_shutdown()


def test_crot_validation(qf):
    """qf_apply_crot rejects bad kinds, qudits and levels synchronously."""
    s = _fake_state(qf)  # D = 3, n = 3
    f = qf.lib.qf_apply_crot
    assert f(ctypes.byref(s), qf.QF_OP_RX, 0, 1, 0, 1, 0.5, None) == qf.QF_EINVAL
    assert f(ctypes.byref(s), qf.QF_OP_CRX, 1, 1, 0, 1, 0.5, None) == qf.QF_EINVAL
    assert f(ctypes.byref(s), qf.QF_OP_CRX, 0, 3, 0, 1, 0.5, None) == qf.QF_EINVAL
    assert f(ctypes.byref(s), qf.QF_OP_CRY, 0, 1, 1, 1, 0.5, None) == qf.QF_EINVAL
    assert f(ctypes.byref(s), qf.QF_OP_CRY, 0, 1, 0, 3, 0.5, None) == qf.QF_EINVAL
    assert f(ctypes.byref(s), qf.QF_OP_CRZ, 0, 1, 0, 0, 0.5, None) == qf.QF_EINVAL
    assert f(ctypes.byref(s), qf.QF_OP_CRZ, 0, 1, 1, 0, float("nan"), None) == qf.QF_EINVAL
    with pytest.raises(qf.QfError):
        qf.Plan(3, 3, [("crx", 0, 0, 0, 1, 0)], 1)
    p = qf.Plan(3, 3, [("cry", 0, 2, 0, 2, 0), ("h", 1), ("crz", 2, 1, 2, 1)], 2)
    assert p.num_stages >= 2


def test_swap_mcx_rot_validation(qf):
    s = _fake_state(qf)  # D = 3, n = 3
    assert qf.lib.qf_apply_swap(ctypes.byref(s), 1, 1, None) == qf.QF_EINVAL
    assert qf.lib.qf_apply_swap(ctypes.byref(s), 0, 3, None) == qf.QF_EINVAL
    c2 = (ctypes.c_int32 * 2)(0, 0)
    assert qf.lib.qf_apply_mcx(ctypes.byref(s), 2, c2, 2, None) == qf.QF_EINVAL
    c1 = (ctypes.c_int32 * 1)(2)
    assert qf.lib.qf_apply_mcx(ctypes.byref(s), 1, c1, 2, None) == qf.QF_EINVAL
    assert qf.lib.qf_apply_mcx(ctypes.byref(s), 0, c1, 1, None) == qf.QF_EINVAL
    assert qf.lib.qf_apply_rot(ctypes.byref(s), qf.QF_OP_CRX, 0, 0, 1, 0.1, None) == qf.QF_EINVAL
    assert qf.lib.qf_apply_rot(ctypes.byref(s), qf.QF_OP_RX, 0, 1, 1, 0.1, None) == qf.QF_EINVAL
    assert qf.lib.qf_apply_rot(ctypes.byref(s), qf.QF_OP_RZ, 0, 3, 0, 0.1, None) == qf.QF_EINVAL
    for bad in ([("swap", 1, 1)], [("mcx", (0, 0), 2)], [("mcx", (2,), 2)], [("mcx", tuple(range(9)), 2)]):
        with pytest.raises(qf.QfError):
            qf.Plan(3, 3, bad, 0)
    p = qf.Plan(3, 4, [("swap", 0, 3), ("mcx", (0, 1, 2), 3), ("h", 2)], 0)
    assert p.num_stages >= 2


def test_sample_validation(qf):
    f = qf.lib.qf_sample
    s = _fake_state(qf)  # D = 3, n = 3
    u, cnt, smp = ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000), ctypes.c_void_p(0x4000)
    assert f(ctypes.byref(s), 0, None, 10, u, None, None, None) == qf.QF_EINVAL  # counts NULL
    assert f(ctypes.byref(s), 0, None, -1, u, cnt, None, None) == qf.QF_EINVAL
    assert f(ctypes.byref(s), 0, None, 10, None, cnt, None, None) == qf.QF_EINVAL  # u NULL
    q = (ctypes.c_int32 * 2)(1, 1)
    assert f(ctypes.byref(s), 0, q, 10, u, cnt, None, None) == qf.QF_EINVAL
    assert f(ctypes.byref(s), 2, q, 10, u, cnt, None, None) == qf.QF_EINVAL  # listed twice
    q3 = (ctypes.c_int32 * 1)(3)
    assert f(ctypes.byref(s), 1, q3, 10, u, cnt, None, None) == qf.QF_EINVAL
    assert f(ctypes.byref(s), 4, q, 10, u, cnt, None, None) == qf.QF_EINVAL  # m > n
    big = qf.qf_state(0x1000, 20, 3, 1, 0)  # 3^20 outcomes > 2^31: no int32 samples
    assert f(ctypes.byref(big), 0, None, 10, u, cnt, smp, None) == qf.QF_ERANGE
    two = qf.qf_state(0x1000, 3, 3, 2, 0)
    assert f(ctypes.byref(two), 0, None, 1 << 31, u, cnt, None, None) == qf.QF_ERANGE  # batch * shots


def test_mixed_dimension_validation(qf):
    lib = qf.lib
    d3 = (ctypes.c_int32 * 3)(2, 3, 4)
    s = qf.qf_state(0x1000, 3, 0, 1, 0, d3)
    bad_dim = qf.qf_state(0x1000, 3, 3, 1, 0, d3)  # dim must be 0 with dims
    U = np.eye(4, dtype=np.complex128).view(np.float64)
    pU = U.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert lib.qf_apply_1q(ctypes.byref(bad_dim), 0, pU, None) == qf.QF_EINVAL
    d_bad = (ctypes.c_int32 * 3)(2, 17, 4)
    assert lib.qf_apply_1q(ctypes.byref(qf.qf_state(0x1000, 3, 0, 1, 0, d_bad)), 0, pU, None) == qf.QF_ERANGE
    assert lib.qf_apply_swap(ctypes.byref(s), 0, 2, None) == qf.QF_EINVAL  # dimensions 2 and 4
    f = lib.qf_apply_crot
    assert f(ctypes.byref(s), qf.QF_OP_CRX, 2, 0, 0, 2, 0.5, None) == qf.QF_EINVAL  # level 2 of a qubit target
    assert f(ctypes.byref(s), qf.QF_OP_CRZ, 0, 1, 3, 0, 0.5, None) == qf.QF_EINVAL  # j = 3 on a qutrit
    assert lib.qf_apply_rot(ctypes.byref(s), qf.QF_OP_RY, 1, 1, 3, 0.5, None) == qf.QF_EINVAL
    dg = (ctypes.c_int32 * 3)(1, 2, 4)  # digit 4 on the d = 4 qudit
    assert lib.qf_state_init(ctypes.byref(s), dg, None) == qf.QF_EINVAL
    # plans: mixed registers run the per-gate schedules
    ops = [("h", 0), ("rx", 2, 1, 3, 0), ("csum", 0, 2), ("crz", 2, 1, 2, 1), ("cz", 1, 0)]
    p = qf.Plan([2, 3, 4], 3, ops, 2)
    assert p.num_stages == 5
    for kw in ({"fuse": 3}, {"ckpt_every": 2}):
        with pytest.raises(qf.QfError) as e:
            qf.Plan([2, 3, 4], 3, ops, 2, **kw)
        assert e.value.status == qf.QF_EUNSUPPORTED
    for bad in ([("rx", 0, 0, 2, 0)], [("rz", 1, 3, 0)], [("swap", 0, 1)], [("crx", 0, 1, 1, 3, 0)]):
        with pytest.raises(qf.QfError):
            qf.Plan([2, 3, 4], 3, bad, 1)
    assert qf.Plan([3, 3, 3], 3, [("h", 0), ("csum", 0, 1)], 0).num_stages >= 1  # equal dims: uniform plan
    th = np.zeros(2)
    o = qf.qf_plan_opts()
    assert lib.qf_plan_autotune(p._h, ctypes.byref(s), th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 0,
                                ctypes.byref(o), None) == qf.QF_EUNSUPPORTED
    u = qf.Plan(3, 3, [("h", 0), ("rx", 1, 0, 1, 0)], 1)
    su = qf.qf_state(0x1000, 3, 3, 1, 0)
    assert lib.qf_plan_autotune(u._h, ctypes.byref(su), th.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 4,
                                ctypes.byref(o), None) == qf.QF_EINVAL  # unknown flag
