"""ctypes binding of libglr (argument marshalling only).

The names follow the C ABI (``include/glr.h``): ``forward``, ``adjoint``,
``fft2d``, ``data_step``, ``detect_keys``, ``match_topk``,
``lowrank_aggregate``, ``prior_step``, ``reconstruct``, ``read_stats``.
Tensors must be contiguous CUDA (HIP) tensors of the documented dtype; the
calls are enqueued on ``torch.cuda.current_stream()``.
"""
import ctypes
import os

import numpy as np

CACTI, MRI, MSFA = 0, 1, 2
SOLVER_GAP, SOLVER_ADMM, SOLVER_GAP_ACC = 0, 1, 2
PREC = {"fp32": 0, "bf16": 1}
STATUS_NAMES = {0: "GLR_OK", 1: "GLR_ERR_INVALID_ARG", 2: "GLR_ERR_SHAPE",
                3: "GLR_ERR_ALIGNMENT", 4: "GLR_ERR_UNSUPPORTED",
                5: "GLR_ERR_WORKSPACE_TOO_SMALL", 6: "GLR_ERR_HIP"}
_MODALITY = {"cacti": CACTI, "mri": MRI, "msfa": MSFA}
EXEMPLARS = {"corner": 0, "uniform": 1, "corner_uniform": 2}
SEARCH = {"global": 0, "window": 1}
SCORE = {"l2": 0, "edge": 1}
AGG_WEIGHTS = {"uniform": 0, "rank": 1}
LOWRANK = {"stacked": 0, "complex": 1}
STATIC_SCRATCH_BYTES = 64 << 20          # GLR_STATIC_SCRATCH_BYTES

_c_i32 = ctypes.c_int32
_vp = ctypes.c_void_p


class Problem(ctypes.Structure):
    _fields_ = [("modality", _c_i32), ("H", _c_i32), ("W", _c_i32), ("C", _c_i32),
                ("mask", _vp)]


class Params(ctypes.Structure):
    _fields_ = [("patch", _c_i32), ("n_keys", _c_i32), ("k", _c_i32), ("iters", _c_i32),
                ("solver", _c_i32), ("rho", ctypes.c_float),
                ("sigma", ctypes.POINTER(ctypes.c_float)),
                ("wnnm_c", ctypes.c_float), ("wnnm_eps", ctypes.c_float),
                ("precision", _c_i32), ("dist_chunk_mb", _c_i32), ("timing", _c_i32),
                ("surrogate", _c_i32), ("surrogate_frac", ctypes.c_float),
                ("judge_stride", _c_i32), ("judge_delta_max", ctypes.c_float),
                ("cnn_packed", _vp), ("exemplars", _c_i32), ("uniform_step", _c_i32),
                ("search", _c_i32), ("window", _c_i32), ("score", _c_i32),
                ("agg_weights", _c_i32), ("wnnm_iters", _c_i32),
                ("wnnm_delta", ctypes.c_float), ("wnnm_lambda", ctypes.c_float),
                ("lowrank", _c_i32)]


class Stats(ctypes.Structure):
    _fields_ = [("prior_steps", ctypes.c_int64), ("margin_sum", ctypes.c_int64),
                ("margin_max", _c_i32), ("overflow_keys", _c_i32),
                ("jacobi_sweeps_max", _c_i32), ("keys_selected", _c_i32),
                ("ms_detect", ctypes.c_float), ("ms_match", ctypes.c_float),
                ("ms_topk", ctypes.c_float), ("ms_select", ctypes.c_float),
                ("ms_lowrank", ctypes.c_float), ("ms_aggregate", ctypes.c_float),
                ("ms_data", ctypes.c_float), ("ms_norms", ctypes.c_float),
                ("match_launches", ctypes.c_int64), ("jacobi_sweeps_sum", ctypes.c_int64),
                ("rematch_keys", ctypes.c_int64), ("surrogate_steps", ctypes.c_int64),
                ("fallback_steps", ctypes.c_int64), ("judge_delta_last", ctypes.c_float),
                ("ms_cnn", ctypes.c_float), ("ms_judge", ctypes.c_float),
                ("regather_keys", ctypes.c_int64), ("ms_rematch", ctypes.c_float),
                ("rematch_launches", ctypes.c_int64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class GlrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_LIB = None


def library_path():
    return os.path.join(os.path.dirname(os.path.abspath(__file__)), "libglr.so")


def lib():
    """Load libglr.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(path)
    st = _c_i32
    sig = {
        "glr_version": (_c_i32, []),
        "glr_status_string": (ctypes.c_char_p, [st]),
        "glr_last_error_message": (ctypes.c_char_p, []),
        "glr_params_default": (None, [ctypes.POINTER(Params)]),
        "glr_plan_create": (st, [ctypes.POINTER(_vp), ctypes.POINTER(Problem),
                                 ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]),
        "glr_plan_destroy": (st, [_vp]),
        "glr_workspace_size": (st, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
        "glr_plan_keys": (st, [_vp, ctypes.POINTER(_c_i32)]),
        "glr_forward": (st, [_vp, _vp, _vp, _vp, _vp]),
        "glr_adjoint": (st, [_vp, _vp, _vp, _vp, _vp]),
        "glr_fft2d": (st, [_vp, _vp, _vp, _c_i32, _vp, _vp]),
        "glr_data_step": (st, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
        "glr_detect_keys": (st, [_vp, _vp, _vp, _vp, _vp]),
        "glr_match_topk": (st, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
        "glr_lowrank_aggregate": (st, [_vp, _vp, _vp, ctypes.c_float, _vp, _vp, _vp, _vp]),
        "glr_prior_step": (st, [_vp, _vp, ctypes.c_float, _vp, _vp, _vp]),
        "glr_prior_step_static": (st, [_vp, _vp, ctypes.c_float, _vp, _vp]),
        "glr_state_bytes": (st, [_vp, ctypes.POINTER(ctypes.c_size_t)]),
        "glr_reconstruct": (st, [_vp, _vp, _vp, _c_i32, _c_i32, _vp, _vp, _vp]),
        "glr_pre_prior": (st, [_vp, _vp, _vp, _vp, _vp, _vp]),
        "glr_read_stats": (st, [_vp, ctypes.POINTER(Stats), _c_i32]),
        "glr_cnn_param_count": (_c_i32, []),
        "glr_cnn_packed_bytes": (ctypes.c_size_t, []),
        "glr_cnn_workspace_size": (st, [_c_i32, _c_i32, _c_i32, _c_i32,
                                        ctypes.POINTER(ctypes.c_size_t)]),
        "glr_cnn_pack": (st, [_vp, _vp, _vp]),
        "glr_cnn_forward": (st, [_vp, _vp, _vp, _vp, _c_i32, _c_i32, _c_i32, _vp, _vp]),
        "glr_cnn_loss_grad": (st, [_vp, _vp, _vp, _vp, _c_i32, _c_i32, _c_i32, _vp, _vp, _vp,
                                   _vp, _vp]),
        "glr_cnn_adam": (st, [_vp, _vp, _vp, _vp, _c_i32, ctypes.c_float, _vp, _vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _LIB = L
    return L


def _check(status):
    if status != 0:
        msg = lib().glr_last_error_message().decode(errors="replace")
        raise GlrError(status, msg)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Plan:
    """One problem shape: modality, image size, patch size, keys, K, solver."""

    def __init__(self, modality, H, W, C, patch, n_keys, k, iters=0, sigma=None, mask=None,
                 rho=1.0, wnnm_c=None, wnnm_eps=None, precision="fp32", dist_chunk_mb=16384,
                 timing=False, device="cuda", allocate=True, cnn=None, surrogate_frac=0.6,
                 judge_stride=8, judge_delta_max=0.02, exemplars="corner", uniform_step=4,
                 search="global", window=20, gap_acc=False, score="l2",
                 agg_weights="uniform", wnnm_iters=1, wnnm_delta=None, wnnm_lambda=None,
                 lowrank="stacked"):
        import torch
        L = lib()
        self.modality = _MODALITY[modality] if isinstance(modality, str) else int(modality)
        self.H, self.W, self.C = int(H), int(W), int(C)
        self.patch, self.n_keys, self.k, self.iters = int(patch), int(n_keys), int(k), int(iters)
        self.device = device
        self.mask = mask
        if mask is not None:
            assert mask.dtype == torch.uint8 and mask.is_contiguous()
        prob = Problem(self.modality, self.H, self.W, self.C, _ptr(mask))
        par = Params()
        L.glr_params_default(ctypes.byref(par))
        par.patch, par.n_keys, par.k, par.iters = self.patch, self.n_keys, self.k, self.iters
        par.solver = SOLVER_ADMM if self.modality == MRI else (
            SOLVER_GAP_ACC if gap_acc else SOLVER_GAP)
        par.rho = float(rho)
        if wnnm_c is not None:
            par.wnnm_c = float(wnnm_c)
        if wnnm_eps is not None:
            par.wnnm_eps = float(wnnm_eps)
        par.precision = PREC[precision]
        par.dist_chunk_mb = int(dist_chunk_mb)
        par.timing = 1 if timing else 0
        par.exemplars = EXEMPLARS[exemplars]
        par.uniform_step = int(uniform_step)
        par.search = SEARCH[search]
        par.window = int(window)
        par.score = SCORE[score]
        par.agg_weights = AGG_WEIGHTS[agg_weights]
        par.wnnm_iters = int(wnnm_iters)
        if wnnm_delta is not None:
            par.wnnm_delta = float(wnnm_delta)
        if wnnm_lambda is not None:
            par.wnnm_lambda = float(wnnm_lambda)
        par.lowrank = LOWRANK[lowrank]
        self.cnn = cnn                      # keeps the packed weights alive
        if cnn is not None:
            par.surrogate = 1
            par.surrogate_frac = float(surrogate_frac)
            par.judge_stride = int(judge_stride)
            par.judge_delta_max = float(judge_delta_max)
            par.cnn_packed = _vp(cnn.packed.data_ptr())
        self._sigma = np.ascontiguousarray(
            np.asarray(sigma if sigma is not None else [], dtype=np.float32))
        if self.iters > 0:
            if self._sigma.shape[0] != self.iters:
                raise ValueError("sigma must have one value per iteration")
            par.sigma = self._sigma.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        h = _vp()
        wsb = ctypes.c_size_t()
        _check(L.glr_plan_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(par),
                                 ctypes.byref(wsb)))
        self._h = h
        nk = _c_i32()
        _check(L.glr_plan_keys(h, ctypes.byref(nk)))
        self.n_keys = int(nk.value)          # exemplar keys per prior step (N)
        self.workspace_bytes = int(wsb.value)
        self.ws = None
        if allocate:
            self.ws = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=device)

    # ------------------------------------------------------------ helpers
    @classmethod
    def for_workload(cls, wl, mask=None, **kw):
        """A plan with the shapes and method parameters of a ``synth`` workload."""
        import synth
        args = dict(iters=wl.iters, sigma=synth.sigma_schedule(wl), mask=mask,
                    precision=wl.precision, exemplars=wl.exemplars,
                    uniform_step=wl.uniform_step, search=wl.search, window=wl.window,
                    gap_acc=wl.gap_acc, score=wl.score, agg_weights=wl.agg_weights,
                    wnnm_iters=wl.wnnm_iters, wnnm_delta=wl.wnnm_delta,
                    wnnm_lambda=wl.wnnm_lambda, lowrank=wl.lowrank)
        args.update(kw)
        return cls(wl.modality, wl.H, wl.W, wl.C, wl.patch, wl.n_keys, wl.k, **args)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _LIB is not None:
            _LIB.glr_plan_destroy(h)
            self._h = None

    @property
    def real_channels(self):
        return 2 if self.modality == MRI else self.C

    @property
    def n_cand(self):
        return (self.H - self.patch + 1) * (self.W - self.patch + 1)

    def _stream(self):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)

    def _image(self, x, name="x"):
        import torch
        if self.modality == MRI:
            exp, shape = torch.complex64, (self.H, self.W)
        else:
            exp, shape = torch.float32, (self.C, self.H, self.W)
        if not (x.is_cuda and x.dtype == exp and tuple(x.shape) == shape and x.is_contiguous()):
            raise ValueError(f"{name}: need contiguous {exp} {shape} on the GPU")
        return x

    def _meas(self, y):
        import torch
        exp = torch.complex64 if self.modality == MRI else torch.float32
        if not (y.is_cuda and y.dtype == exp and tuple(y.shape) == (self.H, self.W)
                and y.is_contiguous()):
            raise ValueError(f"y: need contiguous {exp} {(self.H, self.W)} on the GPU")
        return y

    def _empty_image(self):
        import torch
        if self.modality == MRI:
            return torch.empty((self.H, self.W), dtype=torch.complex64, device=self.device)
        return torch.empty((self.C, self.H, self.W), dtype=torch.float32, device=self.device)

    # ------------------------------------------------------------ operators
    def forward(self, x, y=None):
        import torch
        self._image(x)
        if y is None:
            y = torch.empty((self.H, self.W), device=self.device,
                            dtype=torch.complex64 if self.modality == MRI else torch.float32)
        _check(lib().glr_forward(self._h, _ptr(x), _ptr(y), _ptr(self.ws), self._stream()))
        return y

    def adjoint(self, y, x=None):
        self._meas(y)
        x = self._empty_image() if x is None else x
        _check(lib().glr_adjoint(self._h, _ptr(y), _ptr(x), _ptr(self.ws), self._stream()))
        return x

    def fft2d(self, x, inverse=False, out=None):
        import torch
        out = torch.empty_like(x) if out is None else out
        _check(lib().glr_fft2d(self._h, _ptr(x), _ptr(out), 1 if inverse else 0,
                               _ptr(self.ws), self._stream()))
        return out

    def data_step(self, y, x=None, z=None, u=None, out=None):
        self._meas(y)
        out = self._empty_image() if out is None else out
        _check(lib().glr_data_step(self._h, _ptr(y), _ptr(x), _ptr(z), _ptr(u), _ptr(out),
                                   _ptr(self.ws), self._stream()))
        return out

    # ------------------------------------------------------------ prior step
    def detect_keys(self, x, keys=None):
        import torch
        self._image(x)
        keys = torch.empty(self.n_keys, dtype=torch.int32, device=self.device) if keys is None else keys
        _check(lib().glr_detect_keys(self._h, _ptr(x), _ptr(keys), _ptr(self.ws), self._stream()))
        return keys

    def match_topk(self, x, keys):
        import torch
        self._image(x)
        if not (keys.dtype == torch.int32 and keys.is_cuda and keys.numel() == self.n_keys):
            raise ValueError("keys: need int32 [n_keys] on the GPU")
        idx = torch.empty((self.n_keys, self.k), dtype=torch.int32, device=self.device)
        dist = torch.empty((self.n_keys, self.k), dtype=torch.float32, device=self.device)
        _check(lib().glr_match_topk(self._h, _ptr(x), _ptr(keys), _ptr(idx), _ptr(dist),
                                    _ptr(self.ws), self._stream()))
        return idx, dist

    def lowrank_aggregate(self, x, idx, sigma, want_sv=False):
        import torch
        self._image(x)
        out = self._empty_image()
        sv = torch.empty((self.n_keys, self.k), dtype=torch.float32, device=self.device) if want_sv else None
        _check(lib().glr_lowrank_aggregate(self._h, _ptr(x), _ptr(idx), float(sigma), _ptr(out),
                                           _ptr(sv), _ptr(self.ws), self._stream()))
        return (out, sv) if want_sv else out

    def prior_step(self, x, sigma, out=None):
        self._image(x)
        out = self._empty_image() if out is None else out
        _check(lib().glr_prior_step(self._h, _ptr(x), float(sigma), _ptr(out), _ptr(self.ws),
                                    self._stream()))
        return out

    def prior_step_static(self, x, sigma, out=None):
        """The prior step on the library's static per-GPU scratch (no workspace
        argument; the plan's workspace must fit in STATIC_SCRATCH_BYTES)."""
        self._image(x)
        out = self._empty_image() if out is None else out
        _check(lib().glr_prior_step_static(self._h, _ptr(x), float(sigma), _ptr(out),
                                           self._stream()))
        return out

    # ------------------------------------------------------------ loop
    def state_bytes(self):
        b = ctypes.c_size_t()
        _check(lib().glr_state_bytes(self._h, ctypes.byref(b)))
        return int(b.value)

    def new_state(self):
        import torch
        return torch.zeros(self.state_bytes(), dtype=torch.uint8, device=self.device)

    def reconstruct(self, y, t_begin=0, t_end=None, state=None, out=None):
        self._meas(y)
        t_end = self.iters if t_end is None else t_end
        state = self.new_state() if state is None else state
        out = self._empty_image() if out is None else out
        _check(lib().glr_reconstruct(self._h, _ptr(y), _ptr(state), int(t_begin), int(t_end),
                                     _ptr(out), _ptr(self.ws), self._stream()))
        return out, state

    def pre_prior(self, y, state, out=None):
        """The image the next iteration's prior step receives, from ``state``."""
        self._meas(y)
        out = self._empty_image() if out is None else out
        _check(lib().glr_pre_prior(self._h, _ptr(y), _ptr(state), _ptr(out), _ptr(self.ws),
                                   self._stream()))
        return out

    def read_stats(self, reset=False):
        s = Stats()
        _check(lib().glr_read_stats(self._h, ctypes.byref(s), 1 if reset else 0))
        return s.as_dict()


class Cnn:
    """The residual CNN surrogate: parameters (flat FP32), Adam moments and the
    packed BF16 weights live in device tensors owned here; every call runs the
    library's kernels on torch's current stream."""

    def __init__(self, params, device="cuda"):
        import torch
        self.device = torch.device(device)
        n = int(lib().glr_cnn_param_count())
        p = torch.as_tensor(params, dtype=torch.float32).to(self.device).contiguous()
        if p.numel() != n:
            raise ValueError(f"need {n} parameters, got {p.numel()}")
        self.params = p
        self.m = torch.zeros_like(p)
        self.v = torch.zeros_like(p)
        self.grad = torch.zeros_like(p)
        self.step = 0
        self.packed = torch.empty(int(lib().glr_cnn_packed_bytes()), dtype=torch.uint8,
                                  device=self.device)
        self._ws = {}
        self.repack()

    @staticmethod
    def param_count():
        return int(lib().glr_cnn_param_count())

    def _stream(self):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _workspace(self, B, h, w, train):
        import torch
        key = (B, h, w, train)
        if key not in self._ws:
            b = ctypes.c_size_t()
            _check(lib().glr_cnn_workspace_size(B, h, w, train, ctypes.byref(b)))
            self._ws = {key: torch.empty(int(b.value), dtype=torch.uint8, device=self.device)}
        return self._ws[key]

    def repack(self):
        _check(lib().glr_cnn_pack(_ptr(self.params), _ptr(self.packed), self._stream()))

    def _shape(self, x, sigma):
        import torch
        if x.dim() != 3 or x.dtype != torch.float32 or not x.is_contiguous():
            raise ValueError("x: contiguous float32 [B][h][w]")
        sig = torch.as_tensor(sigma, dtype=torch.float32, device=self.device).reshape(-1)
        if sig.numel() == 1:
            sig = sig.expand(x.shape[0])
        return x.shape[0], x.shape[1], x.shape[2], sig.contiguous()

    def forward(self, x, sigma, out=None):
        import torch
        B, h, w, sig = self._shape(x, sigma)
        out = torch.empty_like(x) if out is None else out
        ws = self._workspace(B, h, w, 0)
        _check(lib().glr_cnn_forward(_ptr(self.packed), _ptr(x), _ptr(sig), _ptr(out), B, h, w,
                                     _ptr(ws), self._stream()))
        return out

    def loss_grad(self, x, sigma, target):
        """Loss (device scalar), gradient (self.grad) and the estimate."""
        import torch
        B, h, w, sig = self._shape(x, sigma)
        out = torch.empty_like(x)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        ws = self._workspace(B, h, w, 1)
        _check(lib().glr_cnn_loss_grad(_ptr(self.packed), _ptr(x), _ptr(sig), _ptr(target),
                                       B, h, w, _ptr(loss), _ptr(self.grad), _ptr(out),
                                       _ptr(ws), self._stream()))
        return loss, self.grad, out

    def adam(self, lr):
        self.step += 1
        _check(lib().glr_cnn_adam(_ptr(self.params), _ptr(self.m), _ptr(self.v),
                                  _ptr(self.grad), self.step, float(lr), _ptr(self.packed),
                                  self._stream()))

    def train_step(self, x, sigma, target, lr):
        loss, _, _ = self.loss_grad(x, sigma, target)
        self.adam(lr)
        return loss
