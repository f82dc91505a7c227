"""Python binding of libqoc (ctypes; argument marshalling only).

Every step of the cost and gradient runs in the HIP kernels of
``libqoc.so``; this module converts arrays to the C-ABI layout declared in
``include/qoc.h`` and raises :class:`QocError` on any non-zero status.
There is no fallback: if the shared library is missing or fails to load,
``load()`` raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqoc.so")

QOC_FP64, QOC_FP32, QOC_BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": QOC_FP64, "fp32": QOC_FP32, "bf16x3": QOC_BF16X3}
QOC_FID_COHERENT, QOC_FID_INCOHERENT = 0, 1
QOC_WARN_DRIFT, QOC_WARN_TAYLOR, QOC_WARN_PRECISION, QOC_WARN_UNITARITY = 1, 2, 4, 8
QOC_WARN_NO_PAIR = 16
QOC_GRAD_EXACT, QOC_GRAD_FIRST_ORDER = 0, 1
QOC_PROP_MATRIX, QOC_PROP_ACTION = 0, 1
QOC_FORM_HORNER, QOC_FORM_BATCHED, QOC_FORM_ACTION = 0, 1, 2
PROPAGATIONS = {"matrix": QOC_PROP_MATRIX, "action": QOC_PROP_ACTION}
QOC_BF3_TAYLOR, QOC_BF3_SQUARING, QOC_BF3_BLOCKPROD, QOC_BF3_ADJOINT = 1, 2, 4, 8
QOC_BF3_ALL = 15
PHASES = ["norm", "assemble", "taylor", "blockprod", "fwd_blocks", "fwd_replay", "cost",
          "bwd_blocks", "bwd_pairs", "adjoint"]
STATUS = {0: "QOC_OK", -1: "QOC_ERR_ARG", -2: "QOC_ERR_SHAPE", -3: "QOC_ERR_NOT_HERMITIAN",
          -4: "QOC_ERR_NONFINITE", -5: "QOC_ERR_NOMEM", -6: "QOC_ERR_DEVICE",
          -7: "QOC_ERR_UNSUPPORTED"}
EXPORTS = ["qoc_create", "qoc_forward", "qoc_cost_grad", "qoc_cost_grad_device",
           "qoc_cost_grad_device_noalloc",
           "qoc_cost_grad_batched", "qoc_get_info", "qoc_profile_enable",
           "qoc_profile_read", "qoc_taylor_select", "qoc_set_taylor", "qoc_set_sweep",
           "qoc_set_bf16x3", "qoc_set_unitarity_check", "qoc_set_structure", "qoc_set_gradient",
           "qoc_adam_step", "qoc_select_pair", "qoc_pair_for", "qoc_destroy",
           "qoc_status_string",
           "qoc_last_error", "qoc_version"]

_dp = C.POINTER(C.c_double)


class Desc(C.Structure):
    _fields_ = [("d", C.c_int), ("M", C.c_int), ("N", C.c_int), ("S", C.c_int),
                ("dt", C.c_double), ("H0", _dp), ("Hk", _dp), ("psi0", _dp), ("psiT", _dp),
                ("penalty_w", _dp), ("alpha_fid", C.c_double), ("alpha_amp", C.c_double),
                ("alpha_var", C.c_double), ("alpha_pen", C.c_double), ("fid_mode", C.c_int),
                ("precision", C.c_int), ("checkpoint_every", C.c_int),
                ("taylor_tol", C.c_double), ("taylor_p", C.c_int), ("taylor_n", C.c_int),
                ("drift_warn", C.c_double), ("device", C.c_int), ("n_forbidden", C.c_int),
                ("forbidden", _dp), ("alpha_time", C.c_double), ("pad_multiple", C.c_int),
                ("segment_steps", C.c_int), ("propagation", C.c_int)]


class Info(C.Structure):
    _fields_ = [("p", C.c_int), ("n", C.c_int), ("theta_max", C.c_double),
                ("norm_drift", C.c_double), ("block_len", C.c_int), ("n_blocks", C.c_int),
                ("d_pad", C.c_int), ("flags", C.c_int), ("device_bytes", C.c_size_t),
                ("bf16x3_classes", C.c_int), ("unitarity_drift", C.c_double),
                ("structured", C.c_int), ("segments", C.c_int), ("propagation", C.c_int)]


class QocError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libqoc.so (raises if it is missing: there is no CPU fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing; build it with "
                          "`python -m paper_1612_04929_amd.build`")
    # One HIP runtime per process.  PyTorch-ROCm ships its own HIP and HSA
    # runtimes (under sonames of their own) and places them in the global
    # symbol scope when it is imported; loading torch first makes the
    # library bind to that runtime, so device pointers and stream handles
    # from torch are the library's own.  Loaded the other way round, the
    # process would hold two runtimes and torch's would fail to start.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.qoc_create.argtypes = [C.POINTER(Desc), C.POINTER(vp)]
    lib.qoc_forward.argtypes = [vp, _dp, _dp, _dp, _dp, C.POINTER(C.c_int)]
    lib.qoc_cost_grad.argtypes = [vp, _dp, _dp, _dp, _dp, _dp, C.POINTER(C.c_int)]
    lib.qoc_cost_grad_device.argtypes = [vp, vp, vp, vp, vp]
    lib.qoc_cost_grad_device_noalloc.argtypes = [vp, vp, vp, vp, vp]
    lib.qoc_cost_grad_batched.argtypes = [C.c_int, C.POINTER(vp), C.POINTER(vp),
                                          C.POINTER(vp), C.POINTER(vp), vp]
    lib.qoc_get_info.argtypes = [vp, C.POINTER(Info)]
    lib.qoc_profile_enable.argtypes = [vp, C.c_int]
    lib.qoc_profile_read.argtypes = [vp, _dp, C.POINTER(C.c_longlong), C.c_int]
    lib.qoc_taylor_select.argtypes = [C.c_double, C.c_double, C.POINTER(C.c_int),
                                      C.POINTER(C.c_int)]
    lib.qoc_select_pair.argtypes = [C.c_double, C.c_double, C.c_int, C.POINTER(C.c_int),
                                    C.POINTER(C.c_int)]
    lib.qoc_pair_for.argtypes = [vp, C.c_double, C.POINTER(C.c_int), C.POINTER(C.c_int)]
    lib.qoc_set_taylor.argtypes = [vp, C.c_int, C.c_int]
    lib.qoc_set_sweep.argtypes = [vp, C.c_int, C.c_int]
    lib.qoc_set_bf16x3.argtypes = [vp, C.c_int]
    lib.qoc_set_unitarity_check.argtypes = [vp, C.c_int]
    lib.qoc_set_structure.argtypes = [vp, C.c_int]
    lib.qoc_set_gradient.argtypes = [vp, C.c_int]
    lib.qoc_adam_step.argtypes = [C.c_long, vp, vp, vp, vp, vp, C.c_double, C.c_double,
                                  C.c_double, C.c_double, vp]
    lib.qoc_destroy.argtypes = [vp]
    lib.qoc_destroy.restype = None
    for f in ["qoc_status_string", "qoc_last_error", "qoc_version"]:
        getattr(lib, f).restype = C.c_char_p
    lib.qoc_status_string.argtypes = [C.c_int]
    for f in ["qoc_create", "qoc_forward", "qoc_cost_grad", "qoc_cost_grad_device",
              "qoc_cost_grad_device_noalloc",
              "qoc_cost_grad_batched", "qoc_get_info", "qoc_profile_enable",
              "qoc_profile_read", "qoc_taylor_select", "qoc_set_taylor", "qoc_set_sweep",
              "qoc_set_bf16x3", "qoc_set_unitarity_check", "qoc_set_structure",
              "qoc_set_gradient", "qoc_adam_step", "qoc_select_pair", "qoc_pair_for"]:
        getattr(lib, f).restype = C.c_int
    _lib = lib
    return lib


def _check(st):
    if st != 0:
        raise QocError(st, load().qoc_last_error().decode())


def _cplx(a, shape):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.complex128).reshape(shape))
    return a, a.view(np.float64).ctypes.data_as(_dp)


def taylor_select(theta: float, tol: float):
    p, n = C.c_int(), C.c_int()
    _check(load().qoc_taylor_select(float(theta), float(tol), C.byref(p), C.byref(n)))
    return p.value, n.value


def select_pair(theta: float, tol: float, form: int = 0):
    """(p, n) by the rule of an evaluation form (QOC_FORM_HORNER, _BATCHED,
    _ACTION)."""
    p, n = C.c_int(), C.c_int()
    _check(load().qoc_select_pair(float(theta), float(tol), int(form), C.byref(p), C.byref(n)))
    return p.value, n.value


def version() -> str:
    return load().qoc_version().decode()


class Problem:
    """A handle on one optimal-control problem resident on the GPU.

    ``prob`` is any object with the attributes d, M, N, S, dt, H0 (d x d),
    Hk (M x d x d), psi0 / psiT (S x d, row s = state s), w (d or None),
    alpha_fid / alpha_pen / alpha_amp / alpha_var and fid_mode.
    """

    def __init__(self, prob, precision="fp32", checkpoint_every=0, taylor_tol=0.0,
                 taylor_pn=None, drift_warn=0.0, device=0, structure=-1, pad_multiple=0,
                 segment_steps=0, propagation="matrix"):
        lib = load()
        self.d, self.M, self.N, self.S = int(prob.d), int(prob.M), int(prob.N), int(prob.S)
        keep = []
        H0, pH0 = _cplx(prob.H0, (self.d, self.d))
        Hk, pHk = _cplx(prob.Hk if self.M else np.zeros((1, self.d, self.d)),
                        (max(self.M, 1), self.d, self.d))
        p0, pp0 = _cplx(prob.psi0, (self.S, self.d))
        pT, ppT = _cplx(prob.psiT, (self.S, self.d))
        keep += [H0, Hk, p0, pT]
        pw = None
        if getattr(prob, "w", None) is not None:
            w = np.ascontiguousarray(np.asarray(prob.w, dtype=np.float64).reshape(self.d))
            keep.append(w)
            pw = w.ctypes.data_as(_dp)
        forb = getattr(prob, "forbidden", None)
        nf, pf = 0, None
        if forb is not None and len(forb):
            fa, pf = _cplx(forb, (len(forb), self.d))
            keep.append(fa)
            nf = len(forb)
        mode = getattr(prob, "fid_mode", "coherent")
        fid = {"coherent": 0, "incoherent": 1}.get(mode, mode)
        tp, tn = (0, 0) if taylor_pn is None else (int(taylor_pn[0]), int(taylor_pn[1]))
        desc = Desc(self.d, self.M, self.N, self.S, float(prob.dt), pH0,
                    pHk if self.M else None, pp0, ppT, pw, float(prob.alpha_fid),
                    float(prob.alpha_amp), float(prob.alpha_var), float(prob.alpha_pen),
                    int(fid), PRECISIONS.get(precision, precision), int(checkpoint_every),
                    float(taylor_tol), tp, tn, float(drift_warn), int(device), nf, pf,
                    float(getattr(prob, "alpha_time", 0.0)), int(pad_multiple),
                    int(segment_steps), PROPAGATIONS.get(propagation, propagation))
        self._h = C.c_void_p()
        _check(lib.qoc_create(C.byref(desc), C.byref(self._h)))
        self.precision = precision
        if structure != -1:
            self.set_structure(structure)

    # -- host-array calls -------------------------------------------------
    def _u(self, u):
        u = np.ascontiguousarray(np.asarray(u, dtype=np.float64).reshape(self.M, self.N))
        return u, u.ctypes.data_as(_dp)

    def forward(self, u):
        u, pu = self._u(u)
        cf = C.c_double()
        c = np.zeros(self.N)
        psiN = np.zeros((self.S, self.d), dtype=np.complex128)
        flags = C.c_int()
        _check(load().qoc_forward(self._h, pu, C.byref(cf), c.ctypes.data_as(_dp),
                                  psiN.view(np.float64).ctypes.data_as(_dp), C.byref(flags)))
        return {**self.info(), **dict(C_fid=cf.value, c=c, psiN=psiN, flags=flags.value)}

    def cost_grad(self, u):
        u, pu = self._u(u)
        cc, cf = C.c_double(), C.c_double()
        c = np.zeros(self.N)
        g = np.zeros((max(self.M, 1), self.N))
        flags = C.c_int()
        _check(load().qoc_cost_grad(self._h, pu, C.byref(cc), C.byref(cf),
                                    c.ctypes.data_as(_dp), g.ctypes.data_as(_dp),
                                    C.byref(flags)))
        return {**self.info(), **dict(C=cc.value, C_fid=cf.value, c=c, grad=g[: self.M],
                                      flags=flags.value)}

    # -- device-pointer call (e.g. torch tensors) ---------------------------
    def cost_grad_device(self, u_ptr: int, out_ptr: int, grad_ptr: int, stream: int = 0):
        _check(load().qoc_cost_grad_device(self._h, C.c_void_p(u_ptr), C.c_void_p(out_ptr),
                                           C.c_void_p(grad_ptr), C.c_void_p(stream)))

    def cost_grad_device_noalloc(self, u_ptr: int, out_ptr: int, grad_ptr: int,
                                 stream: int = 0):
        """qoc_cost_grad_device without device allocation (static scratch)."""
        _check(load().qoc_cost_grad_device_noalloc(self._h, C.c_void_p(u_ptr),
                                                   C.c_void_p(out_ptr), C.c_void_p(grad_ptr),
                                                   C.c_void_p(stream)))

    def pair_for(self, theta: float):
        """The (p, n) this handle would choose per call at theta_max = theta."""
        p, n = C.c_int(), C.c_int()
        _check(load().qoc_pair_for(self._h, float(theta), C.byref(p), C.byref(n)))
        return p.value, n.value

    def set_taylor(self, p: int, n: int = 0):
        """Fix (p, n) for later calls (p = 0: choose per call)."""
        _check(load().qoc_set_taylor(self._h, int(p), int(n)))

    def set_sweep(self, which: int, variant: int):
        """Sweep kernel variant (which: 0..3 or -1 for all; variant 0 auto,
        1 per-block workgroups, 2 per-step launches, 3 four-wavefront LDS
        workgroups for padded d <= 64)."""
        _check(load().qoc_set_sweep(self._h, int(which), int(variant)))

    def set_bf16x3(self, classes: int):
        """Product classes (QOC_BF3_* mask) run as bf16x3 split products by
        a bf16x3 handle; -1 restores the automatic choice."""
        _check(load().qoc_set_bf16x3(self._h, int(classes)))

    def check_last(self):
        """Raise QocError if the last device-pointer call ran with a clamped
        (p, n) (QOC_WARN_NO_PAIR: no pair met the tolerance within the
        path's capacity, or theta_max was not finite).  Synchronises."""
        inf = self.info()
        if inf["flags"] & QOC_WARN_NO_PAIR:
            raise QocError(-7, f"no (p, n) met the tolerance at theta_max = {inf['theta_max']}; "
                               "the last call's results are not accurate")
        return inf

    def set_gradient(self, mode: int):
        """QOC_GRAD_EXACT (default) or QOC_GRAD_FIRST_ORDER (the paper's eq. 7)."""
        _check(load().qoc_set_gradient(self._h, int(mode)))

    def set_structure(self, mode: int):
        """Structured (sparse) norm and gradient contraction: -1 automatic,
        0 dense, 1 structured."""
        _check(load().qoc_set_structure(self._h, int(mode)))

    def set_unitarity_check(self, stride: int):
        """FP64 check of max |(U^H U - I)_{rc}| on every stride-th step (0: off)."""
        _check(load().qoc_set_unitarity_check(self._h, int(stride)))

    def info(self):
        inf = Info()
        _check(load().qoc_get_info(self._h, C.byref(inf)))
        return dict(p=inf.p, n=inf.n, theta_max=inf.theta_max, norm_drift=inf.norm_drift,
                    block_len=inf.block_len, n_blocks=inf.n_blocks, d_pad=inf.d_pad,
                    flags=inf.flags, device_bytes=inf.device_bytes,
                    bf16x3_classes=inf.bf16x3_classes, unitarity_drift=inf.unitarity_drift,
                    structured=inf.structured, segments=inf.segments,
                    propagation=inf.propagation)

    def profile_enable(self, on=True):
        _check(load().qoc_profile_enable(self._h, 1 if on else 0))

    def profile_read(self, reset=False):
        ms = (C.c_double * len(PHASES))()
        calls = (C.c_longlong * len(PHASES))()
        _check(load().qoc_profile_read(self._h, ms, calls, 1 if reset else 0))
        return {ph: (ms[i], calls[i]) for i, ph in enumerate(PHASES)}

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().qoc_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def adam_step(n: int, u_ptr: int, grad_ptr: int, m_ptr: int, v_ptr: int, t_ptr: int,
              lr: float, betas=(0.9, 0.999), eps: float = 1e-8, stream: int = 0):
    """One Adam step over n FP64 device amplitudes (qoc_adam_step)."""
    _check(load().qoc_adam_step(int(n), C.c_void_p(u_ptr), C.c_void_p(grad_ptr),
                                C.c_void_p(m_ptr), C.c_void_p(v_ptr), C.c_void_p(t_ptr),
                                float(lr), float(betas[0]), float(betas[1]), float(eps),
                                C.c_void_p(stream)))


def cost_grad_batched(problems, u_ptrs, out_ptrs, grad_ptrs, stream: int = 0):
    """One call over several handles (device pointers, one stream)."""
    B = len(problems)
    arr = lambda xs: (C.c_void_p * max(B, 1))(*[C.c_void_p(int(x)) for x in xs])
    hs = (C.c_void_p * max(B, 1))(*[p._h for p in problems])
    _check(load().qoc_cost_grad_batched(B, hs, arr(u_ptrs), arr(out_ptrs), arr(grad_ptrs),
                                        C.c_void_p(stream)))
