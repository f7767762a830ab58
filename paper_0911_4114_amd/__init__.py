"""Python binding of the MI355X Fourier-basis Helmholtz FMM library (include/ffmm.h).

Argument marshalling only: every step of the matvec runs in the HIP kernels of _ffmm.so. PyTorch
provides device memory and the current stream. The library must be built in-tree first
(``python paper_0911_4114_amd/build.py`` or ``__graft_entry__.build()``); without it every call
raises.
"""
import atexit
import ctypes
import os
import weakref

import numpy as np
import torch  # imported first so that the library binds to the HIP runtime torch has loaded

__all__ = ["Plan", "FfmmError", "select_level_params", "library_path", "load_library", "Allocator",
           "FP64", "FP32", "STAGE_NEAR", "STAGE_FAR", "STAGE_ALL", "MAX_LEVELS", "apply"]

FP64, FP32 = 0, 1
STAGE_NEAR, STAGE_FAR, STAGE_ALL = 1, 2, 3
MAX_LEVELS = 22

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "_ffmm.so")
_lib = None


def library_path():
    return _LIB_PATH


class FfmmError(RuntimeError):
    """A failed library call: ``status`` is the ffmm_status code."""

    def __init__(self, status, message):
        super().__init__("ffmm status %d: %s" % (status, message))
        self.status = status
        self.message = message


class Options(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_leaf_points", ctypes.c_int32), ("depth", ctypes.c_int32),
                ("alpha", ctypes.c_double), ("eps_safety", ctypes.c_double),
                ("max_rhs", ctypes.c_int32), ("reduce_depth", ctypes.c_int32),
                ("ell_override", ctypes.c_int32 * MAX_LEVELS), ("method", ctypes.c_int32),
                ("best_effort", ctypes.c_int32), ("fast_near_phase", ctypes.c_int32),
                ("quarter_nphi", ctypes.c_int32)]


_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class Allocator(ctypes.Structure):
    """ffmm_allocator: device-memory hooks of a plan."""
    _fields_ = [("ctx", ctypes.c_void_p), ("alloc", _ALLOC_FN), ("free", _FREE_FN)]


def _torch_alloc(ctx, nbytes, stream):
    # ctx carries the device index; NULL on failure (the library reports out of memory)
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), device=int(ctx or 0),
                                                  stream=int(stream or 0))
    except Exception:
        return None


def _torch_free(ctx, ptr, stream):
    try:
        torch.cuda.caching_allocator_delete(int(ptr))
    except Exception:
        pass


# kept for the life of the module: the library calls these while plans exist
_TORCH_ALLOC = _ALLOC_FN(_torch_alloc)
_TORCH_FREE = _FREE_FN(_torch_free)
# live plans, closed before the interpreter tears torch down (their memory returns through the
# hooks above)
_LIVE = weakref.WeakSet()


@atexit.register
def _close_live_plans():
    for pl in list(_LIVE):
        try:
            pl.close()
        except Exception:
            pass


class PlanInfo(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("n_points", ctypes.c_int64), ("kappa", ctypes.c_double),
                ("eps", ctypes.c_double), ("root_lo", ctypes.c_double * 3),
                ("root_side", ctypes.c_double), ("ell", ctypes.c_int32 * MAX_LEVELS),
                ("ntheta", ctypes.c_int32 * MAX_LEVELS), ("nphi_max", ctypes.c_int32 * MAX_LEVELS),
                ("K", ctypes.c_int64 * MAX_LEVELS), ("n_boxes", ctypes.c_int64 * MAX_LEVELS),
                ("n_ilist", ctypes.c_int64 * MAX_LEVELS),
                ("predicted_err", ctypes.c_double * MAX_LEVELS),
                ("n_near_pairs", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("max_rhs", ctypes.c_int32), ("method", ctypes.c_int32),
                ("max_leaf_count", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_int32), ("near_stream", ctypes.c_int32),
                ("p2p_blocks_per_cu", ctypes.c_int32), ("m2l_rhs_block", ctypes.c_int32),
                ("rs_slab", ctypes.c_int32 * 4), ("m2l_by_parent", ctypes.c_int32),
                ("m2l_chunk", ctypes.c_int32)]


TUNING_FIELDS = ("near_stream", "p2p_blocks_per_cu", "m2l_rhs_block", "rs_slab", "m2l_by_parent",
                 "m2l_chunk")

_P = ctypes.c_void_p
_SIGS = {
    "ffmm_options_default": [ctypes.POINTER(Options)],
    "ffmm_plan_create": [_P, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                         ctypes.POINTER(Options), ctypes.POINTER(Allocator), _P, ctypes.POINTER(_P)],
    "ffmm_position_gradient": [_P, _P, _P, _P, ctypes.c_int32, _P],
    "ffmm_matvec": [_P, _P, _P, ctypes.c_int32, _P],
    "ffmm_matvec_static": [_P, _P, _P, ctypes.c_int32, _P],
    "ffmm_plan_set_m2l_levels": [_P, ctypes.c_uint32],
    "ffmm_matvec_stages": [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P],
    "ffmm_adjoint": [_P, _P, _P, ctypes.c_int32, _P],
    "ffmm_field_gradient": [_P, _P, _P, ctypes.c_int32, _P],
    "ffmm_plan_info_get": [_P, ctypes.POINTER(PlanInfo)],
    "ffmm_plan_destroy": [_P],
    "ffmm_select_level_params": [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_int32, ctypes.c_int32, _P, _P, _P, ctypes.c_int32, _P],
    "ffmm_plan_get_perm": [_P, _P],
    "ffmm_plan_get_level": [_P, ctypes.c_int32] + [_P] * 9,
    "ffmm_plan_get_nphi": [_P, ctypes.c_int32, _P],
    "ffmm_plan_get_transfer": [_P, ctypes.c_int32, ctypes.c_int32, _P],
    "ffmm_plan_get_signature": [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P],
    "ffmm_profile_enable": [_P, ctypes.c_int32],
    "ffmm_tuning_default": [ctypes.POINTER(Tuning)],
    "ffmm_plan_set_tuning": [_P, ctypes.POINTER(Tuning)],
    "ffmm_plan_get_tuning": [_P, ctypes.POINTER(Tuning)],
    "ffmm_plan_autotune": [_P, _P, _P, ctypes.c_int32, _P, ctypes.POINTER(Tuning)],
    "ffmm_profile_read": [_P, _P, _P],
}

PROF_STAGES = ["gather", "p2m", "m2m", "m2l", "l2l", "l2p", "p2p", "scatter", "leaf_m2l"]


def load_library():
    """Load _ffmm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError("the HIP library %s is not built; run "
                              "python paper_0911_4114_amd/build.py" % _LIB_PATH)
        lib = ctypes.CDLL(_LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        lib.ffmm_last_error_message.restype = ctypes.c_char_p
        lib.ffmm_last_error_message.argtypes = []
        lib.ffmm_status_string.restype = ctypes.c_char_p
        lib.ffmm_status_string.argtypes = [ctypes.c_int]
        _lib = lib
    return _lib


def _check(status):
    if status != 0:
        msg = load_library().ffmm_last_error_message().decode()
        raise FfmmError(status, msg)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def select_level_params(ka, alpha, eps, precision=FP64, ell=0):
    """Host-side parameter choice of one level in box units (no GPU needed).
    Returns (ell, ntheta, nphi list, predicted error)."""
    lib = load_library()
    e = ctypes.c_int32()
    nt = ctypes.c_int32()
    cap = 8192
    nphi = (ctypes.c_int32 * cap)()
    pred = ctypes.c_double()
    _check(lib.ffmm_select_level_params(float(ka), float(alpha), float(eps), int(precision),
                                        int(ell), ctypes.byref(e), ctypes.byref(nt), nphi, cap,
                                        ctypes.byref(pred)))
    return e.value, nt.value, list(nphi[: nt.value // 2 + 1]), pred.value


def _prec_code(precision):
    if precision in ("fp64", FP64, torch.complex128):
        return FP64
    if precision in ("fp32", FP32, torch.complex64):
        return FP32
    raise ValueError("precision must be 'fp64' or 'fp32'")


class Plan:
    """A plan for phi = A q with A_ij = e^{i kappa |x_i - x_j|}/|x_i - x_j| (i != j).

    points: CUDA float64 tensor [N, 3]. precision 'fp64' (complex128 I/O) or 'fp32' (complex64).
    allocator: 'torch' (default: the plan's device memory comes from torch's caching allocator
    through the library's allocator hooks) or None (the library's own hipMalloc).
    best_effort: build the plan even where eps is out of reach (low-frequency breakdown) instead
    of raising FfmmError with status -5. fast_near_phase: FP32 near-field phase form (see
    ffmm_options). quarter_nphi: common phi length from which the resample's row steps run on
    quarter ranges (None: the library's default).
    """

    def __init__(self, points, kappa, eps, precision="fp64", depth=None, max_leaf=64,
                 alpha=None, eps_safety=None, max_rhs=1, reduce_depth=True, ell_override=None,
                 method="fmm", best_effort=False, fast_near_phase=False, quarter_nphi=None,
                 allocator="torch"):
        lib = load_library()
        if not (isinstance(points, torch.Tensor) and points.is_cuda):
            raise TypeError("points must be a CUDA tensor")
        if points.dtype != torch.float64 or points.dim() != 2 or points.shape[1] != 3:
            raise TypeError("points must be float64 of shape [N, 3]")
        pts = points.contiguous()
        o = Options()
        _check(lib.ffmm_options_default(ctypes.byref(o)))
        o.precision = _prec_code(precision)
        o.max_leaf_points = int(max_leaf)
        o.depth = 0 if depth is None else int(depth)
        if alpha is not None:
            o.alpha = float(alpha)
        if eps_safety is not None:
            o.eps_safety = float(eps_safety)
        o.max_rhs = int(max_rhs)
        o.method = {"fmm": 0, "direct": 1, "auto": 2}[method]
        o.reduce_depth = 1 if reduce_depth else 0
        for l, v in (ell_override or {}).items():
            o.ell_override[int(l)] = int(v)
        o.best_effort = 1 if best_effort else 0
        o.fast_near_phase = 1 if fast_near_phase else 0
        o.quarter_nphi = 0 if quarter_nphi is None else int(quarter_nphi)
        if allocator == "torch":
            al = Allocator(ctypes.c_void_p(pts.device.index or 0), _TORCH_ALLOC, _TORCH_FREE)
            alp = ctypes.byref(al)
        elif allocator is None:
            alp = None
        else:
            raise ValueError("allocator must be 'torch' or None")
        h = ctypes.c_void_p()
        _check(lib.ffmm_plan_create(ctypes.c_void_p(pts.data_ptr()), pts.shape[0], float(kappa),
                                    float(eps), ctypes.byref(o), alp, _stream(), ctypes.byref(h)))
        self._h = h
        _LIVE.add(self)
        self.n = pts.shape[0]
        self.precision = o.precision
        self.cdtype = torch.complex128 if o.precision == FP64 else torch.complex64
        self.max_rhs = o.max_rhs
        self.device = pts.device

    # ---- products ---------------------------------------------------------------------
    def _prep(self, q):
        if not (isinstance(q, torch.Tensor) and q.is_cuda):
            raise TypeError("input must be a CUDA tensor")
        if q.dtype != self.cdtype:
            raise TypeError("input dtype must be %s for this plan" % self.cdtype)
        squeeze = q.dim() == 1
        q2 = q.reshape(1, -1) if squeeze else q
        if q2.dim() != 2 or q2.shape[1] != self.n:
            raise ValueError("input must have shape [N] or [nrhs, N]")
        return q2.contiguous(), squeeze

    def _call(self, fn, q, width=1, stages=None, out=None):
        q2, squeeze = self._prep(q)
        nrhs = q2.shape[0]
        shape = (nrhs, self.n) if width == 1 else (nrhs, self.n, width)
        if out is None:
            out = torch.empty(shape, dtype=self.cdtype, device=q2.device)
        elif (out.dtype != self.cdtype or out.device != q2.device or not out.is_contiguous()
              or out.numel() != nrhs * self.n * width):
            raise ValueError("out must be a contiguous %s tensor of %d elements on %s"
                             % (self.cdtype, nrhs * self.n * width, q2.device))
        else:
            out = out.view(shape)
        args = [self._h, ctypes.c_void_p(q2.data_ptr()), ctypes.c_void_p(out.data_ptr()), nrhs]
        if stages is not None:
            args.append(int(stages))
        _check(fn(*args, _stream()))
        return out[0] if squeeze else out

    def matvec(self, q):
        """phi = A q; q [N] or [nrhs, N] in the caller's order."""
        return self._call(load_library().ffmm_matvec, q)

    def matvec_static(self, q, out=None):
        """phi = A q through ffmm_matvec_static: the library allocates nothing during the call (its
        per-call workspaces live in one fixed device array of the library); pass ``out`` (a
        contiguous tensor of the result's size) to avoid the output allocation here as well."""
        return self._call(load_library().ffmm_matvec_static, q, out=out)

    def matvec_stages(self, q, stages):
        """Only the selected parts: STAGE_NEAR (P2P), STAGE_FAR (the FMM far field) or both."""
        return self._call(load_library().ffmm_matvec_stages, q, stages=stages)

    def adjoint(self, g):
        """A^H g = conj(A conj(g))."""
        return self._call(load_library().ffmm_adjoint, g)

    def field_gradient(self, q):
        """F_i(q) = sum_{j != i} G'(R_ij)(x_i - x_j)/R_ij q_j; shape [..., N, 3]."""
        return self._call(load_library().ffmm_field_gradient, q, width=3)

    def position_gradient(self, q, g):
        """dL/dx [N, 3] float64 for phi = A(x) q and G = dL/dRe(phi) + i dL/dIm(phi) (q and g of
        equal shape [N] or [nrhs, N]); computed by the library (ffmm_position_gradient)."""
        q2, _ = self._prep(q)
        g2, _ = self._prep(g)
        if q2.shape != g2.shape:
            raise ValueError("q and g must have the same shape")
        out = torch.empty((self.n, 3), dtype=torch.float64, device=q2.device)
        _check(load_library().ffmm_position_gradient(self._h, ctypes.c_void_p(q2.data_ptr()),
                                                     ctypes.c_void_p(g2.data_ptr()),
                                                     ctypes.c_void_p(out.data_ptr()), q2.shape[0],
                                                     _stream()))
        return out

    # ---- inspection ---------------------------------------------------------------------
    def info(self):
        pi = PlanInfo()
        _check(load_library().ffmm_plan_info_get(self._h, ctypes.byref(pi)))
        d = pi.depth
        return {
            "depth": d, "precision": pi.precision, "n_points": pi.n_points, "kappa": pi.kappa,
            "eps": pi.eps, "root_lo": list(pi.root_lo), "root_side": pi.root_side,
            "ell": list(pi.ell[: d + 1]), "ntheta": list(pi.ntheta[: d + 1]),
            "nphi_max": list(pi.nphi_max[: d + 1]), "K": list(pi.K[: d + 1]),
            "n_boxes": list(pi.n_boxes[: d + 1]), "n_ilist": list(pi.n_ilist[: d + 1]),
            "predicted_err": list(pi.predicted_err[: d + 1]), "n_near_pairs": pi.n_near_pairs,
            "device_bytes": pi.device_bytes, "max_rhs": pi.max_rhs,
            "method": ("fmm", "direct")[pi.method], "max_leaf_points": pi.max_leaf_count,
        }

    def perm(self):
        out = np.empty(self.n, dtype=np.int64)
        _check(load_library().ffmm_plan_get_perm(self._h, out.ctypes.data))
        return out

    def level(self, l):
        info = self.info()
        nb = info["n_boxes"][l]
        keys = np.empty(nb, np.uint64)
        parent = np.empty(nb, np.int32)
        out = {"keys": keys}
        args = [keys.ctypes.data, parent.ctypes.data if l >= 1 else None]
        if l >= 1:
            out["parent"] = parent
        if l == info["depth"]:
            start = np.empty(nb, np.int32)
            count = np.empty(nb, np.int32)
            nb_ptr = np.empty(nb + 1, np.int32)
            nb_src = np.empty(27 * nb, np.int32)
            out.update(start=start, count=count, nb_ptr=nb_ptr, nb_src=nb_src)
            args += [start.ctypes.data, count.ctypes.data]
        else:
            args += [None, None]
        if l >= 2:
            nil = info["n_ilist"][l]
            il_ptr = np.empty(nb + 1, np.int32)
            il_src = np.empty(max(nil, 1), np.int32)
            il_code = np.empty(max(nil, 1), np.int32)
            out.update(il_ptr=il_ptr, il_src=il_src[:nil], il_code=il_code[:nil])
            args += [il_ptr.ctypes.data, il_src.ctypes.data, il_code.ctypes.data]
        else:
            args += [None, None, None]
        if l == info["depth"]:
            args += [out["nb_ptr"].ctypes.data, out["nb_src"].ctypes.data]
        else:
            args += [None, None]
        _check(load_library().ffmm_plan_get_level(self._h, l, *args))
        if l == info["depth"]:
            out["nb_src"] = out["nb_src"][: out["nb_ptr"][-1]]
        return out

    def set_m2l_levels(self, levels=None):
        """Error studies: run the transfer pass only at the given levels (None: all levels)."""
        mask = 0xffffffff if levels is None else sum(1 << int(l) for l in levels)
        _check(load_library().ffmm_plan_set_m2l_levels(self._h, mask))

    def nphi(self, l):
        info = self.info()
        out = np.empty(info["ntheta"][l] // 2 + 1, np.int32)
        _check(load_library().ffmm_plan_get_nphi(self._h, l, out.ctypes.data))
        return out

    def transfer(self, l, code):
        K = self.info()["K"][l]
        out = np.empty(K, np.complex128)
        _check(load_library().ffmm_plan_get_transfer(self._h, l, code, out.ctypes.data))
        return out

    def signature(self, kind, l, rhs=0):
        info = self.info()
        out = np.empty(info["n_boxes"][l] * info["K"][l], np.complex128)
        _check(load_library().ffmm_plan_get_signature(self._h, kind, l, rhs, out.ctypes.data))
        return out.reshape(info["n_boxes"][l], info["K"][l])

    # ---- launch configuration -------------------------------------------------------------
    @staticmethod
    def _tuning_dict(t):
        return {"near_stream": t.near_stream, "p2p_blocks_per_cu": t.p2p_blocks_per_cu,
                "m2l_rhs_block": t.m2l_rhs_block, "rs_slab": list(t.rs_slab),
                "m2l_by_parent": t.m2l_by_parent, "m2l_chunk": t.m2l_chunk}

    def tuning(self):
        """The plan's launch configuration (see ffmm_tuning)."""
        t = Tuning()
        _check(load_library().ffmm_plan_get_tuning(self._h, ctypes.byref(t)))
        return self._tuning_dict(t)

    def set_tuning(self, **fields):
        """Change fields of the launch configuration (unknown names raise)."""
        t = Tuning()
        _check(load_library().ffmm_plan_get_tuning(self._h, ctypes.byref(t)))
        for k, v in fields.items():
            if k not in TUNING_FIELDS:
                raise KeyError(k)
            if k == "rs_slab":
                t.rs_slab = (ctypes.c_int32 * 4)(*v)
            else:
                setattr(t, k, int(v))
        _check(load_library().ffmm_plan_set_tuning(self._h, ctypes.byref(t)))

    def autotune(self, q):
        """Time candidate launch configurations on the right-hand sides q (the plan keeps the
        fastest) and return it."""
        q2, _ = self._prep(q)
        out = torch.empty((q2.shape[0], self.n), dtype=self.cdtype, device=q2.device)
        t = Tuning()
        _check(load_library().ffmm_plan_autotune(self._h, ctypes.c_void_p(q2.data_ptr()),
                                                 ctypes.c_void_p(out.data_ptr()), q2.shape[0],
                                                 _stream(), ctypes.byref(t)))
        return self._tuning_dict(t)

    def profile(self, on=True):
        """Record per-stage HIP event times on later calls (see profile_read)."""
        _check(load_library().ffmm_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        """{stage: (milliseconds, launches)} accumulated since the last read."""
        ms = (ctypes.c_double * len(PROF_STAGES))()
        calls = (ctypes.c_int64 * len(PROF_STAGES))()
        _check(load_library().ffmm_profile_read(self._h, ms, calls))
        return {name: (ms[i], calls[i]) for i, name in enumerate(PROF_STAGES)}

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.ffmm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _Apply(torch.autograd.Function):
    """phi = A(x) q with gradients for q and the positions x (see ``apply``)."""

    @staticmethod
    def forward(ctx, points, q, plan):
        ctx.plan = plan
        ctx.save_for_backward(q)
        return plan.matvec(q)

    @staticmethod
    def backward(ctx, grad):
        (q,) = ctx.saved_tensors
        plan = ctx.plan
        grad = grad.contiguous()
        gq = plan.adjoint(grad) if ctx.needs_input_grad[1] else None
        gx = plan.position_gradient(q, grad) if ctx.needs_input_grad[0] else None
        return gx, gq, None


def apply(plan, points, q):
    """Differentiable phi = A q. Backward (C-ABI adjoint and position-gradient calls):
    dL/dq = conj(A conj(G)) and dL/dx_i = Re[conj(G_i) F_i(q) + q_i F_i(conj G)], with
    G = dL/dRe(phi) + i dL/dIm(phi) (torch's convention). ``points`` must be the tensor the plan
    was built from; the tree stays fixed. Any max_rhs works (the library groups the field
    gradients of q and conj(G) by what the plan's workspaces hold)."""
    return _Apply.apply(points, q, plan)
