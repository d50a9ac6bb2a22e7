"""Python binding of libqf.so, the MI355X (gfx950) qudit state-vector library.

Every function named ``qf_*`` here marshals arguments for the C entry point of
the same name in ``include/qf.h``; all computation runs in the HIP kernels of
that library.  PyTorch supplies device memory and the current HIP stream.  If
the shared library is missing, importing this package raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libqf.so")

QF_OK, QF_EINVAL, QF_EDTYPE, QF_ERANGE, QF_ENOMEM, QF_EHIP, QF_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
QF_C64, QF_C128 = 0, 1
QF_SEED = 1  # adjoint flag: lam holds torch's gradient of the output state
QF_TUNE_ADJOINT = 1  # autotuner flag: time forward + adjoint gradient
QF_TUNE_BOUND = 2  # autotuner flag: device-parameter schedules only, timed bound
(QF_OP_H, QF_OP_X, QF_OP_CLOCK, QF_OP_RX, QF_OP_RY, QF_OP_RZ, QF_OP_CSUM, QF_OP_CSHIFT, QF_OP_CZ,
 QF_OP_U, QF_OP_CRX, QF_OP_CRY, QF_OP_CRZ, QF_OP_SWAP, QF_OP_MCX) = range(15)


class QfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"qf status {status}: {msg}")
        self.status = status


class qf_state(ctypes.Structure):
    _fields_ = [("amps", ctypes.c_void_p), ("n", ctypes.c_int32), ("dim", ctypes.c_int32),
                ("batch", ctypes.c_int64), ("dtype", ctypes.c_int32), ("dims", ctypes.POINTER(ctypes.c_int32))]


class qf_op(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("q0", ctypes.c_int32), ("q1", ctypes.c_int32),
                ("j", ctypes.c_int32), ("k", ctypes.c_int32), ("param", ctypes.c_int32),
                ("shifts", ctypes.c_int32 * 16), ("mat", ctypes.POINTER(ctypes.c_double))]


class qf_plan_opts(ctypes.Structure):
    _fields_ = [("fuse", ctypes.c_int32), ("tile_digits", ctypes.c_int32), ("low_digits", ctypes.c_int32),
                ("ckpt_every", ctypes.c_int32), ("adj_tile_digits", ctypes.c_int32), ("stage_kernel", ctypes.c_int32),
                ("group_digits", ctypes.c_int32), ("pipe_wgs", ctypes.c_int32), ("tile_order", ctypes.c_int32),
                ("tile_search", ctypes.c_int32)]


class qf_kernel_stat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("bytes", ctypes.c_double)]


_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_PI32 = ctypes.POINTER(ctypes.c_int32)
_PD = ctypes.POINTER(ctypes.c_double)
_PS = ctypes.POINTER(qf_state)

_SIGS = {
    "qf_state_init": [_PS, _PI32, _P],
    "qf_apply_1q": [_PS, _I32, _PD, _P],
    "qf_apply_ctrl": [_PS, _I32, _I32, _PI32, _P],
    "qf_apply_diag": [_PS, _I32, _PI32, _PD, _P],
    "qf_apply_fused": [_PS, _I32, _I32, _P, _P],
    "qf_apply_crot": [_PS, _I32, _I32, _I32, _I32, _I32, ctypes.c_double, _P],
    "qf_apply_rot": [_PS, _I32, _I32, _I32, _I32, ctypes.c_double, _P],
    "qf_apply_swap": [_PS, _I32, _I32, _P],
    "qf_apply_mcx": [_PS, _I32, _PI32, _I32, _P],
    "qf_probs": [_PS, _I32, _PI32, _P, _P],
    "qf_sample": [_PS, _I32, _PI32, ctypes.c_int64, _P, _P, _P, _P],
    "qf_expect": [_PS, _I32, _PI32, _PD, _PD, _P],
    "qf_expect_noalloc": [_PS, _I32, _PI32, _PD, _PD, _P],
    "qf_plan_create": [_I32, _I32, _I32, ctypes.POINTER(qf_op), _I32, _I32, ctypes.POINTER(qf_plan_opts),
                       ctypes.POINTER(ctypes.c_void_p)],
    "qf_plan_create_dims": [_PI32, _I32, _I32, ctypes.POINTER(qf_op), _I32, _I32, ctypes.POINTER(qf_plan_opts),
                            ctypes.POINTER(ctypes.c_void_p)],
    "qf_plan_forward": [_P, _PS, _PD, _P],
    "qf_adjoint_grad": [_P, _PS, _PS, _PD, _I32, _PI32, _PD, _PD, ctypes.c_uint32, _P],
    "qf_plan_set_profiling": [_P, _I32],
    "qf_plan_autotune": [_P, _PS, _PD, ctypes.c_uint32, ctypes.POINTER(qf_plan_opts), _P],
    "qf_plan_bind": [_P, ctypes.c_int64],
    "qf_plan_forward_dev": [_P, _PS, _P, ctypes.c_int64, _P],
    "qf_adjoint_grad_dev": [_P, _PS, _PS, _P, ctypes.c_int64, _I32, _PI32, _PD, _P, _P, ctypes.c_uint32, _P],
    "qf_plan_read_profile": [_P, ctypes.POINTER(qf_kernel_stat), _I32, _PI32],
}


def _load() -> ctypes.CDLL:
    # torch links its own libamdhip64 (soname libamdhip64.so.7).  Loading torch
    # first lets libqf.so bind to that same HIP runtime by soname; loading
    # libqf.so first would put a second HIP runtime in the process.
    import torch  # noqa: F401
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2409_17716_amd/build.py` "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int32
    lib.qf_last_error.restype = ctypes.c_char_p
    lib.qf_last_error.argtypes = []
    lib.qf_version.restype = ctypes.c_int32
    for name in ("qf_plan_num_stages", "qf_plan_num_adjoint_stages"):
        getattr(lib, name).restype = ctypes.c_int32
        getattr(lib, name).argtypes = [_P]
    lib.qf_plan_destroy.restype = None
    lib.qf_plan_destroy.argtypes = [_P]
    lib.qf_shutdown.restype = None
    lib.qf_shutdown.argtypes = []
    return lib


lib = _load()


def _check(st: int) -> None:
    if st != QF_OK:
        raise QfError(st, lib.qf_last_error().decode())


def _torch():
    import torch
    return torch


def _stream(stream=None) -> int:
    if stream is not None:
        return int(stream)
    return int(_torch().cuda.current_stream().cuda_stream)


def _i32(a) -> ctypes.Array:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return a, a.ctypes.data_as(_PI32)


def _c128(a) -> tuple:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128)).view(np.float64)
    return a, a.ctypes.data_as(_PD)


def _size(n: int, dim) -> int:
    """Amplitudes of one register: dim^n, or the product of a list of per-qudit dimensions."""
    if isinstance(dim, (int, np.integer)):
        return int(dim) ** n
    if len(dim) != n:
        raise QfError(QF_EINVAL, f"{len(dim)} dimensions for {n} qudits")
    return int(np.prod([int(d) for d in dim]))


def _dim_of(dim, q: int) -> int:
    return int(dim) if isinstance(dim, (int, np.integer)) else int(dim[q])


def state_of(t, n: int, dim, batch: Optional[int] = None) -> qf_state:
    """qf_state describing a torch complex64/complex128 CUDA tensor of batch
    registers; dim is the common dimension or a list of per-qudit dimensions."""
    torch = _torch()
    if not t.is_cuda:
        raise QfError(QF_EINVAL, "state tensor must live on the GPU")
    if not t.is_contiguous():
        raise QfError(QF_EINVAL, "state tensor must be contiguous")
    if t.dtype == torch.complex64:
        dt = QF_C64
    elif t.dtype == torch.complex128:
        dt = QF_C128
    else:
        raise QfError(QF_EDTYPE, f"unsupported dtype {t.dtype}")
    N = _size(n, dim)
    b = t.numel() // N if batch is None else batch
    if b * N != t.numel():
        raise QfError(QF_EINVAL, f"tensor of {t.numel()} elements is not batch * {N} amplitudes")
    if isinstance(dim, (int, np.integer)):
        return qf_state(t.data_ptr(), n, int(dim), b, dt)
    arr, p = _i32(dim)
    s = qf_state(t.data_ptr(), n, 0, b, dt, p)
    s._dims_keep = arr  # the array the dims pointer refers to
    return s


# ---------------------------------------------------------------------------
# Per-gate entry points (same names as the C ABI).
# ---------------------------------------------------------------------------

def qf_state_init(t, n: int, dim: int, digits=None, stream=None) -> None:
    s = state_of(t, n, dim)
    if digits is None:
        _check(lib.qf_state_init(ctypes.byref(s), None, _stream(stream)))
    else:
        arr, p = _i32(np.broadcast_to(np.asarray(digits), (s.batch, n)).reshape(-1))
        _check(lib.qf_state_init(ctypes.byref(s), p, _stream(stream)))


def qf_apply_1q(t, n: int, dim: int, q: int, U, stream=None) -> None:
    s = state_of(t, n, dim)
    arr, p = _c128(U)
    _check(lib.qf_apply_1q(ctypes.byref(s), q, p, _stream(stream)))


def qf_apply_ctrl(t, n: int, dim: int, ctrl: int, tgt: int, shift, stream=None) -> None:
    s = state_of(t, n, dim)
    arr, p = _i32(shift)
    _check(lib.qf_apply_ctrl(ctypes.byref(s), ctrl, tgt, p, _stream(stream)))


def qf_apply_diag(t, n: int, dim: int, qudits: Sequence[int], phases, stream=None) -> None:
    s = state_of(t, n, dim)
    qa, qp = _i32(qudits)
    pa, pp = _c128(phases)
    _check(lib.qf_apply_diag(ctypes.byref(s), len(qudits), qp, pp, _stream(stream)))


def qf_apply_crot(t, n: int, dim: int, kind: str, ctrl: int, tgt: int, j: int, k: int, theta: float,
                  stream=None) -> None:
    """Controlled rotation sum_m |m><m|_ctrl (x) R(m theta)_tgt; kind "crx", "cry" or "crz"
    (crz uses level j, k is ignored)."""
    s = state_of(t, n, dim)
    _check(lib.qf_apply_crot(ctypes.byref(s), _KIND[kind], ctrl, tgt, j, k, float(theta), _stream(stream)))


def qf_apply_rot(t, n: int, dim: int, kind: str, q: int, j: int, k: int, theta: float, stream=None) -> None:
    """One rotation ("rx", "ry" on levels j < k, or "rz" with level j) as a slab sweep."""
    s = state_of(t, n, dim)
    _check(lib.qf_apply_rot(ctypes.byref(s), _KIND[kind], q, j, k, float(theta), _stream(stream)))


def qf_apply_swap(t, n: int, dim: int, a: int, b: int, stream=None) -> None:
    s = state_of(t, n, dim)
    _check(lib.qf_apply_swap(ctypes.byref(s), a, b, _stream(stream)))


def qf_apply_mcx(t, n: int, dim: int, ctrls: Sequence[int], tgt: int, stream=None) -> None:
    """x_tgt -> x_tgt + prod of the control digits mod dim."""
    s = state_of(t, n, dim)
    ca, cp = _i32(ctrls)
    _check(lib.qf_apply_mcx(ctypes.byref(s), len(ctrls), cp, tgt, _stream(stream)))


def qf_apply_fused(t, n: int, dim: int, q0: int, k: int, B, stream=None) -> None:
    """B: device tensor (K x K) in the state's precision."""
    s = state_of(t, n, dim)
    if not B.is_cuda or B.dtype != t.dtype or not B.is_contiguous():
        raise QfError(QF_EINVAL, "B must be a contiguous device tensor of the state's dtype")
    _check(lib.qf_apply_fused(ctypes.byref(s), k, q0, ctypes.c_void_p(B.data_ptr()), _stream(stream)))


def qf_probs(t, n: int, dim: int, qudits: Optional[Sequence[int]] = None, out=None, stream=None):
    torch = _torch()
    s = state_of(t, n, dim)
    rdt = torch.float32 if t.dtype == torch.complex64 else torch.float64
    m = 0 if qudits is None else len(qudits)
    size = s.batch * (_size(n, dim) if m == 0 else int(np.prod([_dim_of(dim, q) for q in qudits])))
    if out is None:
        out = torch.empty(size, dtype=rdt, device=t.device)
    if qudits is None:
        _check(lib.qf_probs(ctypes.byref(s), 0, None, ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    else:
        qa, qp = _i32(qudits)
        _check(lib.qf_probs(ctypes.byref(s), m, qp, ctypes.c_void_p(out.data_ptr()), _stream(stream)))
    return out


def qf_sample(t, n: int, dim: int, shots: int, u, qudits: Optional[Sequence[int]] = None, samples: bool = False,
              stream=None):
    """Histogram of shots draws per register (of the listed qudits' marginal,
    or of the full register), drawn by the caller's uniforms u (a float64
    device tensor of batch * shots values in [0, 1)).  Returns the int64 counts
    (batch * outcomes) and, with samples=True, the int32 outcome of every draw."""
    torch = _torch()
    s = state_of(t, n, dim)
    m = 0 if qudits is None else len(qudits)
    outcomes = _size(n, dim) if m == 0 else int(np.prod([_dim_of(dim, q) for q in qudits]))
    if shots > 0 and (u is None or not u.is_cuda or u.dtype != torch.float64 or not u.is_contiguous()
                      or u.numel() != s.batch * shots):
        raise QfError(QF_EINVAL, "u must be a contiguous float64 device tensor of batch * shots values")
    counts = torch.empty(s.batch * outcomes, dtype=torch.int64, device=t.device)
    draws = torch.empty(s.batch * shots, dtype=torch.int32, device=t.device) if samples else None
    qa, qp = _i32(qudits) if qudits is not None else (None, None)
    _check(lib.qf_sample(ctypes.byref(s), m, qp, int(shots), ctypes.c_void_p(u.data_ptr() if shots > 0 else 0),
                         ctypes.c_void_p(counts.data_ptr()),
                         ctypes.c_void_p(draws.data_ptr() if samples and shots > 0 else 0), _stream(stream)))
    return (counts, draws) if samples else counts


def _terms_arrays(dim, terms) -> tuple:
    """terms: list of (qudit, "z") or (qudit, table of d_q complex values)."""
    qs = [int(q) for q, _ in terms]
    tabs = []
    for q, d in terms:
        dq = _dim_of(dim, int(q))
        if isinstance(d, str):
            if d != "z":
                raise QfError(QF_EINVAL, f"unknown term {d}")
            tabs.append(np.exp(2j * np.pi / dq) ** np.arange(dq))
        else:
            tabs.append(np.asarray(d, dtype=np.complex128))
    return qs, np.concatenate(tabs)


def qf_expect(t, n: int, dim: int, terms, out=None, stream=None):
    torch = _torch()
    s = state_of(t, n, dim)
    qs, tab = _terms_arrays(dim, terms)
    qa, qp = _i32(qs)
    ta, tp = _c128(tab)
    if out is None:
        out = torch.empty(2 * s.batch, dtype=torch.float64, device=t.device)
    _check(lib.qf_expect(ctypes.byref(s), len(qs), qp, tp,
                         ctypes.cast(ctypes.c_void_p(out.data_ptr()), _PD), _stream(stream)))
    return out


def qf_expect_noalloc(t, n: int, dim: int, terms, out, stream=None):
    """qf_expect into a caller-allocated out (2 * batch doubles on the device),
    with the library's static scratch array: no allocation."""
    s = state_of(t, n, dim)
    qs, tab = _terms_arrays(dim, terms)
    qa, qp = _i32(qs)
    ta, tp = _c128(tab)
    _check(lib.qf_expect_noalloc(ctypes.byref(s), len(qs), qp, tp,
                                 ctypes.cast(ctypes.c_void_p(out.data_ptr()), _PD), _stream(stream)))
    return out


# ---------------------------------------------------------------------------
# Plans.
# ---------------------------------------------------------------------------

_KIND = {"h": QF_OP_H, "x": QF_OP_X, "clock": QF_OP_CLOCK, "clockp": QF_OP_CLOCK, "rx": QF_OP_RX, "ry": QF_OP_RY,
         "rz": QF_OP_RZ, "csum": QF_OP_CSUM, "cshift": QF_OP_CSHIFT, "cz": QF_OP_CZ, "u": QF_OP_U,
         "crx": QF_OP_CRX, "cry": QF_OP_CRY, "crz": QF_OP_CRZ, "swap": QF_OP_SWAP, "mcx": QF_OP_MCX}


def ops_to_c(ops: Sequence[tuple]):
    """Translate gate descriptors (see qf_inputs) into a qf_op array; returns the
    array and the host matrices it points to (kept alive by the caller)."""
    arr = (qf_op * max(1, len(ops)))()
    keep = []
    for i, op in enumerate(ops):
        kind = op[0]
        o = arr[i]
        o.kind = _KIND[kind]
        o.param = -1
        if kind == "h":
            o.q0 = op[1]
        elif kind in ("x", "clock"):
            o.q0, o.j = op[1], int(op[2])
        elif kind == "clockp":  # clock gate whose exponent is theta[op[2]]
            o.q0, o.param = op[1], int(op[2])
        elif kind in ("rx", "ry"):
            o.q0, o.j, o.k, o.param = op[1], op[2], op[3], op[4]
        elif kind == "rz":
            o.q0, o.j, o.param = op[1], op[2], op[3]
        elif kind in ("csum", "cz"):
            o.q0, o.q1 = op[1], op[2]
        elif kind == "cshift":
            o.q0, o.q1 = op[1], op[2]
            for c, v in enumerate(op[3]):
                o.shifts[c] = int(v)
        elif kind in ("crx", "cry"):
            o.q0, o.q1, o.j, o.k, o.param = op[1], op[2], op[3], op[4], op[5]
        elif kind == "crz":
            o.q0, o.q1, o.j, o.param = op[1], op[2], op[3], op[4]
        elif kind == "swap":
            o.q0, o.q1 = op[1], op[2]
        elif kind == "mcx":
            ctrls = list(op[1])
            if not 1 <= len(ctrls) <= 8:
                raise QfError(QF_EINVAL, "mcx takes 1..8 controls")
            o.q1, o.j = op[2], len(ctrls)
            for i, c in enumerate(ctrls):
                o.shifts[i] = int(c)
        elif kind == "u":
            o.q0, o.q1 = op[1], op[2]
            m, p = _c128(op[3])
            keep.append(m)
            o.mat = p
        else:
            raise QfError(QF_EINVAL, f"unknown gate kind {kind}")
    return arr, keep


class Plan:
    """A compiled circuit (qf_plan_create) for registers of n qudits of dimension
    dim, or of per-qudit dimensions when dim is a list (qf_plan_create_dims)."""

    def __init__(self, dim, n: int, ops: Sequence[tuple], nparams: int, dtype: str = "c64",
                 fuse: int = 0, tile_digits: int = 0, low_digits: int = 0, ckpt_every: int = 0,
                 adj_tile_digits: int = 0, stage_kernel: int = 0, group_digits: int = 0, pipe_wgs: int = 0,
                 tile_order: int = 0, tile_search: int = 0):
        self.dim, self.n, self.nparams = dim, n, nparams
        self.dtype = QF_C64 if dtype == "c64" else QF_C128
        arr, keep = ops_to_c(ops)
        opts = qf_plan_opts(fuse, tile_digits, low_digits, ckpt_every, adj_tile_digits, stage_kernel, group_digits,
                            pipe_wgs, tile_order, tile_search)
        h = ctypes.c_void_p()
        if isinstance(dim, (int, np.integer)):
            _check(lib.qf_plan_create(int(dim), n, self.dtype, arr, len(ops), nparams, ctypes.byref(opts),
                                      ctypes.byref(h)))
        else:
            self.dim = [int(d) for d in dim]
            da, dp = _i32(self.dim)
            _check(lib.qf_plan_create_dims(dp, n, self.dtype, arr, len(ops), nparams, ctypes.byref(opts),
                                           ctypes.byref(h)))
        self._h = h

    @property
    def num_stages(self) -> int:
        return lib.qf_plan_num_stages(self._h)

    @property
    def num_adjoint_stages(self) -> int:
        return lib.qf_plan_num_adjoint_stages(self._h)

    def autotune(self, t, theta, adjoint: bool = False, bound: bool = False, stream=None) -> dict:
        """qf_plan_autotune on state t (overwritten); returns the chosen options.
        adjoint: time forward + adjoint gradient; bound: only device-parameter
        schedules, timed bound to t's batch (the plan is left unbound)."""
        s = state_of(t, self.n, self.dim)
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
        o = qf_plan_opts()
        flags = (QF_TUNE_ADJOINT if adjoint else 0) | (QF_TUNE_BOUND if bound else 0)
        _check(lib.qf_plan_autotune(self._h, ctypes.byref(s), th.ctypes.data_as(_PD), flags, ctypes.byref(o),
                                    _stream(stream)))
        self.bound = 0
        return {f: getattr(o, f) for f, _ in qf_plan_opts._fields_}

    # ---- device-parameter mode (graph-capturable) ----
    def bind(self, batch: int) -> None:
        _check(lib.qf_plan_bind(self._h, int(batch)))
        self.bound = int(batch)

    def forward_dev(self, t, theta_dev, theta_stride: int, stream=None) -> None:
        s = state_of(t, self.n, self.dim)
        _check(lib.qf_plan_forward_dev(self._h, ctypes.byref(s), ctypes.c_void_p(theta_dev.data_ptr()),
                                       int(theta_stride), _stream(stream)))

    def adjoint_grad_dev(self, psi, lam, theta_dev, theta_stride: int, terms, grad_dev, loss_dev=None,
                         stream=None, seed: bool = False) -> None:
        """qf_adjoint_grad_dev.  seed=True: lam holds torch's gradient of the
        final state (QF_SEED) and terms is ignored."""
        s = state_of(psi, self.n, self.dim)
        sl = state_of(lam, self.n, self.dim)
        if seed:
            self._keep = ((None, None), (None, None))
            nt = 0
        else:
            qs, tab = _terms_arrays(self.dim, terms)
            self._keep = (_i32(qs), _c128(tab))
            nt = len(qs)
        (qa, qp), (ta, tp) = self._keep
        _check(lib.qf_adjoint_grad_dev(self._h, ctypes.byref(s), ctypes.byref(sl),
                                       ctypes.c_void_p(theta_dev.data_ptr()), int(theta_stride), nt, qp, tp,
                                       ctypes.c_void_p(grad_dev.data_ptr()),
                                       ctypes.c_void_p(loss_dev.data_ptr()) if loss_dev is not None else None,
                                       QF_SEED if seed else 0, _stream(stream)))

    def set_profiling(self, enable: bool) -> None:
        _check(lib.qf_plan_set_profiling(self._h, 1 if enable else 0))

    def read_profile(self) -> dict:
        """{family: (launches, total_ms, bytes)} of the launches recorded since
        profiling was enabled or last read (waits for their events)."""
        arr = (qf_kernel_stat * 16)()
        cnt = ctypes.c_int32()
        _check(lib.qf_plan_read_profile(self._h, arr, 16, ctypes.byref(cnt)))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms, arr[i].bytes) for i in range(cnt.value)}

    def forward(self, t, theta, stream=None) -> None:
        s = state_of(t, self.n, self.dim)
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
        _check(lib.qf_plan_forward(self._h, ctypes.byref(s), th.ctypes.data_as(_PD), _stream(stream)))

    def adjoint_grad(self, psi, lam, theta, terms, stream=None, seed: bool = False) -> np.ndarray:
        """qf_adjoint_grad (synchronises).  seed=True: lam holds torch's gradient
        of the final state (QF_SEED) and terms is ignored."""
        s = state_of(psi, self.n, self.dim)
        sl = state_of(lam, self.n, self.dim)
        th = np.ascontiguousarray(np.asarray(theta, dtype=np.float64))
        if seed:
            qa = qp = ta = tp = None
            nt = 0
        else:
            qs, tab = _terms_arrays(self.dim, terms)
            qa, qp = _i32(qs)
            ta, tp = _c128(tab)
            nt = len(qs)
        g = np.zeros(s.batch * self.nparams, dtype=np.float64)
        _check(lib.qf_adjoint_grad(self._h, ctypes.byref(s), ctypes.byref(sl), th.ctypes.data_as(_PD), nt,
                                   qp, tp, g.ctypes.data_as(_PD), QF_SEED if seed else 0, _stream(stream)))
        return g.reshape(s.batch, self.nparams) if s.batch > 1 else g

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and lib is not None:
            lib.qf_plan_destroy(h)
            self._h = None


def plan_for(circuit, dtype: str = "c64", **kw) -> Plan:
    """Plan of a circuit description (uniform: .dim; mixed: .dims)."""
    dim = list(circuit.dims) if hasattr(circuit, "dims") else circuit.dim
    return Plan(dim, circuit.n, circuit.ops, circuit.nparams, dtype, **kw)


def qf_shutdown() -> None:
    """Release library-wide state (the autotuner cache)."""
    lib.qf_shutdown()


def new_state(n: int, dim, dtype: str = "c64", batch: int = 1, device="cuda"):
    torch = _torch()
    dt = torch.complex64 if dtype == "c64" else torch.complex128
    return torch.empty(batch * _size(n, dim), dtype=dt, device=device)
