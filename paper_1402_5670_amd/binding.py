"""ctypes binding of libshearlet's C ABI (include/shearlet.h).

Argument marshalling only: every step of the transform runs in the HIP
library.  PyTorch provides device memory and the current stream; the
library fails loudly (ImportError / RuntimeError) when it is missing or a
call fails.  There is no CPU fallback.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# SL_LIB may name an alternative build of the same library (same ABI)
LIB_PATH = os.environ.get("SL_LIB") or os.path.join(_PKG, "libshearlet.so")

SL_F32, SL_F16, SL_BF16 = 0, 1, 2
_DTYPES = {"f32": SL_F32, "f16": SL_F16, "bf16": SL_BF16}
_ERRORS = {-1: "SL_EINVAL", -2: "SL_ENOMEM", -3: "SL_EUNSUPPORTED", -4: "SL_EILLCOND",
           -5: "SL_EHIP"}


class ShearletError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("dims", ctypes.c_int64 * 3),
        ("n_scales", ctypes.c_int),
        ("shear_levels", ctypes.POINTER(ctypes.c_int)),
        ("qmf", ctypes.POINTER(ctypes.c_double)),
        ("qmf_len", ctypes.c_int),
        ("dir_filter", ctypes.POINTER(ctypes.c_double)),
        ("dir_rows", ctypes.c_int),
        ("dir_cols", ctypes.c_int),
        ("full_system", ctypes.c_int),
        ("coeff_dtype", ctypes.c_int),
    ]


class ShrinkageModel(ctypes.Structure):
    _fields_ = [("params_dev", ctypes.c_void_p), ("packed_dev", ctypes.c_void_p)]


class Subband(ctypes.Structure):
    _fields_ = [("cone", ctypes.c_int), ("j", ctypes.c_int), ("k1", ctypes.c_int),
                ("k2", ctypes.c_int), ("l2norm", ctypes.c_double), ("l1norm", ctypes.c_double)]


_lib = None

_SIGS = {
    "sl_abi_version": ([], ctypes.c_int),
    "sl_last_error": ([], ctypes.c_char_p),
    "sl_config_num_subbands": ([ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "sl_build_filters_host": ([ctypes.POINTER(Config), ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p], ctypes.c_int),
    "sl_build_system": ([ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "sl_free_system": ([ctypes.c_void_p], None),
    "sl_system_num_subbands": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "sl_system_subband": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(Subband)], ctypes.c_int),
    "sl_workspace_size": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
                          ctypes.c_int),
    "sl_forward": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
                   ctypes.c_int),
    "sl_inverse": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                    ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "sl_denoise": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p],
                   ctypes.c_int),
    "sl_denoise_workspace_size": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                   ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "sl_get_filters": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "sl_denoise_fused_noalloc": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p],
                                 ctypes.c_int),
    "sl_get_dual_weight": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "sl_denoise_fused": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                          ctypes.c_void_p], ctypes.c_int),
    "sl_inpaint_workspace_size": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)],
                                  ctypes.c_int),
    "sl_inpaint": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                    ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                    ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t,
                    ctypes.c_void_p], ctypes.c_int),
    "sl_build_wavelet_system": ([ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_void_p)],
                                ctypes.c_int),
    "sl_build_wavelet_filters_host": ([ctypes.POINTER(Config), ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p], ctypes.c_int),
    "sl_decompose_workspace_size": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "sl_decompose": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                      ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                      ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "sl_inverse_adjoint": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                            ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "sl_cnn_packed_bytes": ([ctypes.c_int], ctypes.c_size_t),
    "sl_cnn_pack": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p],
                    ctypes.c_int),
    "sl_cnn_workspace_size": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                               ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "sl_cnn_apply": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "sl_cnn_backward": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                         ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                         ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "sl_cnn_adam": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                     ctypes.c_int, ctypes.c_float, ctypes.c_int, ctypes.c_void_p], ctypes.c_int),
    "sl_sq_error_grad": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_float,
                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "sl_render_cartoons": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                            ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_void_p,
                            ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "sl_system_set_chunk_bytes": ([ctypes.c_void_p, ctypes.c_size_t], ctypes.c_int),
    "sl_system_chunk_bytes": ([ctypes.c_void_p], ctypes.c_size_t),
    "sl_system_set_block_shape": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "sl_system_set_xcd": ([ctypes.c_void_p, ctypes.c_int, ctypes.c_int], ctypes.c_int),
    "sl_system_set_line_plan": ([ctypes.c_void_p, ctypes.c_int], ctypes.c_int),
    "sl_system_line_plan": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "sl_system_xcd_active": ([ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int)],
                             ctypes.c_int),
    "sl_system_block_shape": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                               ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "sl_multi_create": ([ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                         ctypes.POINTER(ctypes.c_void_p)], ctypes.c_int),
    "sl_multi_free": ([ctypes.c_void_p], None),
    "sl_multi_workspace_size": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "sl_multi_run": ([ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 6 +
                     [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p], ctypes.c_int),
    "sl_multi_autotune": ([ctypes.c_void_p] + [ctypes.c_void_p] * 4 +
                          [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_char_p, ctypes.c_void_p],
                          ctypes.c_int),
    "sl_multi_graph_build": ([ctypes.c_void_p, ctypes.c_int] + [ctypes.c_void_p] * 6 +
                             [ctypes.c_void_p, ctypes.c_size_t], ctypes.c_int),
    "sl_multi_graph_launch": ([ctypes.c_void_p, ctypes.c_void_p], ctypes.c_int),
    "sl_multi_set_schedule": ([ctypes.c_void_p, ctypes.c_int], ctypes.c_int),
    "sl_multi_schedule": ([ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "sl_timing_enable": ([ctypes.c_int], ctypes.c_int),
    "sl_timing_reset": ([], ctypes.c_int),
    "sl_timing_num_passes": ([], ctypes.c_int),
    "sl_timing_pass_name": ([ctypes.c_int], ctypes.c_char_p),
    "sl_timing_query": ([ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                         ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
}


def lib():
    """Load libshearlet.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run python -m paper_1402_5670_amd.build")
        h = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(h, name)
            fn.argtypes = args
            fn.restype = res
        _lib = h
    return _lib


def exported_symbols():
    return list(_SIGS)


def timing_enable(on=True):
    check(lib().sl_timing_enable(int(bool(on))))


def timing_reset():
    check(lib().sl_timing_reset())


def timing_report():
    """{pass name: (total ms, launches)} for the launches since the last reset."""
    out = {}
    for p in range(lib().sl_timing_num_passes()):
        ms, n = ctypes.c_double(), ctypes.c_int()
        check(lib().sl_timing_query(p, ctypes.byref(ms), ctypes.byref(n)))
        if n.value:
            out[lib().sl_timing_pass_name(p).decode()] = (ms.value, n.value)
    return out


def check(rc):
    if rc != 0:
        raise ShearletError(rc, lib().sl_last_error().decode())


class _Cfg:
    """Keeps the ctypes arrays referenced by a Config alive."""

    def __init__(self, dims, n_scales, shear_levels, full_system=False, dtype="f32", qmf=None,
                 dir_filter=None):
        self.levels = (ctypes.c_int * len(shear_levels))(*[int(v) for v in shear_levels])
        c = Config()
        c.ndim = len(dims)
        for i, d in enumerate(dims):
            c.dims[i] = int(d)
        c.n_scales = int(n_scales)
        c.shear_levels = self.levels
        if qmf is not None:
            self.qmf = np.ascontiguousarray(qmf, dtype=np.float64)
            c.qmf = self.qmf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            c.qmf_len = len(self.qmf)
        if dir_filter is not None:
            self.dirf = np.ascontiguousarray(dir_filter, dtype=np.float64)
            c.dir_filter = self.dirf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            c.dir_rows, c.dir_cols = self.dirf.shape
        c.full_system = int(bool(full_system))
        c.coeff_dtype = _DTYPES[dtype] if isinstance(dtype, str) else int(dtype)
        self.c = c


def num_subbands(dims, n_scales, shear_levels, full_system=False):
    cfg = _Cfg(dims, n_scales, shear_levels, full_system)
    R = ctypes.c_int()
    check(lib().sl_config_num_subbands(ctypes.byref(cfg.c), ctypes.byref(R)))
    return R.value


def build_filters_host(dims, n_scales, shear_levels, full_system=False, qmf=None,
                       dir_filter=None):
    """Host FP64 closed-form filters: (filters [R, *dims], Psi_hat, subbands)."""
    cfg = _Cfg(dims, n_scales, shear_levels, full_system, "f32", qmf, dir_filter)
    R = ctypes.c_int()
    check(lib().sl_config_num_subbands(ctypes.byref(cfg.c), ctypes.byref(R)))
    filt = np.zeros((R.value, *dims), dtype=np.float64)
    dual = np.zeros(dims, dtype=np.float64)
    subs = (Subband * R.value)()
    check(lib().sl_build_filters_host(ctypes.byref(cfg.c), filt.ctypes.data, dual.ctypes.data,
                                      ctypes.cast(subs, ctypes.c_void_p)))
    return filt, dual, [(s.cone, s.j, s.k1, s.k2, s.l2norm, s.l1norm) for s in subs]


def build_wavelet_filters_host(dims, n_scales, qmf=None):
    """Host FP64 wavelet bank: (filters [3J+1, *dims], Psi_hat, subbands)."""
    cfg = _Cfg(dims, n_scales, [0] * int(n_scales), False, "f32", qmf, None)
    R = 3 * int(n_scales) + 1
    filt = np.zeros((R, *dims), dtype=np.float64)
    dual = np.zeros(dims, dtype=np.float64)
    subs = (Subband * R)()
    check(lib().sl_build_wavelet_filters_host(ctypes.byref(cfg.c), filt.ctypes.data,
                                              dual.ctypes.data, ctypes.cast(subs, ctypes.c_void_p)))
    return filt, dual, [(s.cone, s.j, s.k1, s.k2, s.l2norm, s.l1norm) for s in subs]


def _ptr(t):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class System:
    """A shearlet system resident on the current HIP device."""

    def __init__(self, dims, n_scales, shear_levels=None, full_system=False, dtype="f32",
                 qmf=None, dir_filter=None, wavelet=False):
        """wavelet=True builds the undecimated separable wavelet bank
        (sl_build_wavelet_system) instead; shear_levels do not apply."""
        self.dims = tuple(int(d) for d in dims)
        self.n_scales = int(n_scales)
        if shear_levels is None:
            if not wavelet:
                raise ValueError("shear_levels is required for a shearlet system")
            shear_levels = [0] * self.n_scales
        self.shear_levels = tuple(int(v) for v in shear_levels)
        self.dtype = dtype
        self.wavelet = bool(wavelet)
        self._cfg = _Cfg(dims, n_scales, shear_levels, full_system, dtype, qmf, dir_filter)
        h = ctypes.c_void_p()
        build = lib().sl_build_wavelet_system if wavelet else lib().sl_build_system
        check(build(ctypes.byref(self._cfg.c), ctypes.byref(h)))
        self._h = h
        R = ctypes.c_int()
        check(lib().sl_system_num_subbands(h, ctypes.byref(R)))
        self.R = R.value
        self.subbands = []
        for i in range(self.R):
            s = Subband()
            check(lib().sl_system_subband(h, i, ctypes.byref(s)))
            self.subbands.append((s.cone, s.j, s.k1, s.k2, s.l2norm, s.l1norm))
        self._ws = {}

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.sl_free_system(h)
            self._h = None

    @property
    def l2norms(self):
        return np.array([s[4] for s in self.subbands])

    @property
    def torch_coeff_dtype(self):
        import torch
        return {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}[self.dtype]

    def workspace_bytes(self, batch):
        n = ctypes.c_size_t()
        check(lib().sl_workspace_size(self._h, int(batch), ctypes.byref(n)))
        return n.value

    def workspace(self, batch, device):
        import torch
        n = self.workspace_bytes(batch)
        ws = self._ws.get(str(device))
        if ws is None or ws.numel() < n:
            ws = torch.empty(n, dtype=torch.uint8, device=device)
            self._ws[str(device)] = ws
        return ws

    def alloc_coeffs(self, batch, device):
        import torch
        c = torch.empty((batch, self.R, *self.dims), dtype=self.torch_coeff_dtype, device=device)
        s = torch.empty((batch, self.R), dtype=torch.float32, device=device)
        return c, s

    def _check_x(self, x):
        import torch
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32
                and x.is_contiguous() and tuple(x.shape[1:]) == self.dims):
            raise ValueError(f"expected a contiguous float32 CUDA tensor [B, {self.dims}]")

    def forward(self, x, coeffs=None, scales=None, workspace=None):
        self._check_x(x)
        B = x.shape[0]
        if coeffs is None:
            coeffs, scales = self.alloc_coeffs(B, x.device)
        ws = workspace if workspace is not None else self.workspace(B, x.device)
        check(lib().sl_forward(self._h, _ptr(x), B, _ptr(coeffs), _ptr(scales), _ptr(ws),
                               ws.numel(), _stream()))
        return coeffs, scales

    def inverse(self, coeffs, scales=None, sigma=None, K=None, out=None, workspace=None):
        import torch
        B = coeffs.shape[0]
        if out is None:
            out = torch.empty((B, *self.dims), dtype=torch.float32, device=coeffs.device)
        ws = workspace if workspace is not None else self.workspace(B, coeffs.device)
        Kh = None
        if sigma is not None:
            Kh = (ctypes.c_float * len(K))(*[float(k) for k in K])
        check(lib().sl_inverse(self._h, _ptr(coeffs), _ptr(scales), B, _ptr(sigma),
                               ctypes.cast(Kh, ctypes.c_void_p) if Kh is not None else None,
                               _ptr(out), _ptr(ws), ws.numel(), _stream()))
        return out

    def inverse_adjoint(self, r, coeffs=None, workspace=None):
        """Adjoint of the inverse: forward transform with the dual filters."""
        import torch
        B = r.shape[0]
        if coeffs is None:
            coeffs = torch.empty((B, self.R, *self.dims), dtype=torch.float32, device=r.device)
        ws = workspace if workspace is not None else self.workspace(B, r.device)
        check(lib().sl_inverse_adjoint(self._h, _ptr(r), B, _ptr(coeffs), _ptr(ws), ws.numel(),
                                       _stream()))
        return coeffs

    def get_filters(self):
        """FP64 filter bank [R, *dims] of the built system (host)."""
        f = np.empty((self.R, *self.dims), dtype=np.float64)
        check(lib().sl_get_filters(self._h, f.ctypes.data))
        return f

    def get_dual_weight(self):
        """FP64 dual-frame weight Psi_hat [*dims] of the built system (host)."""
        d = np.empty(self.dims, dtype=np.float64)
        check(lib().sl_get_dual_weight(self._h, d.ctypes.data))
        return d

    def denoise_workspace_bytes(self, batch, with_model):
        n = ctypes.c_size_t()
        check(lib().sl_denoise_workspace_size(self._h, int(batch), int(bool(with_model)),
                                              ctypes.byref(n)))
        return n.value

    def denoise(self, x, sigma, K=None, coeffs=None, scales=None, out=None, workspace=None,
                model=None):
        """T^-1 S T x with S the hard threshold (model None) or the learned
        shrinkage of a Shrinkage network."""
        import torch
        self._check_x(x)
        B = x.shape[0]
        if coeffs is None:
            coeffs, scales = self.alloc_coeffs(B, x.device)
        if out is None:
            out = torch.empty_like(x)
        if model is None:
            ws = workspace if workspace is not None else self.workspace(B, x.device)
            Kh = (ctypes.c_float * len(K))(*[float(k) for k in K])
            mp = None
        else:
            if workspace is None:
                workspace = torch.empty(self.denoise_workspace_bytes(B, True), dtype=torch.uint8,
                                        device=x.device)
            ws = workspace
            Kh = None
            m = ShrinkageModel(_ptr(model.params), _ptr(model.packed))
            mp = ctypes.byref(m)
        check(lib().sl_denoise(self._h, _ptr(x), B, _ptr(sigma),
                               ctypes.cast(Kh, ctypes.c_void_p) if Kh is not None else None,
                               mp, _ptr(coeffs), _ptr(scales), _ptr(out), _ptr(ws), ws.numel(),
                               _stream()))
        return out

    def denoise_fused_noalloc(self, x, sigma, K, out=None):
        """sl_denoise_fused on the library's static scratch array (no workspace)."""
        import torch
        self._check_x(x)
        B = x.shape[0]
        if out is None:
            out = torch.empty_like(x)
        Kh = (ctypes.c_float * len(K))(*[float(k) for k in K])
        check(lib().sl_denoise_fused_noalloc(self._h, _ptr(x), B, _ptr(sigma),
                                             ctypes.cast(Kh, ctypes.c_void_p), _ptr(out),
                                             _stream()))
        return out

    def denoise_fused(self, x, sigma, K, out=None, workspace=None):
        """Hard-threshold denoising without materialised coefficients (float32)."""
        import torch
        self._check_x(x)
        B = x.shape[0]
        if out is None:
            out = torch.empty_like(x)
        ws = workspace if workspace is not None else self.workspace(B, x.device)
        Kh = (ctypes.c_float * len(K))(*[float(k) for k in K])
        check(lib().sl_denoise_fused(self._h, _ptr(x), B, _ptr(sigma),
                                     ctypes.cast(Kh, ctypes.c_void_p), _ptr(out), _ptr(ws),
                                     ws.numel(), _stream()))
        return out

    def decompose_workspace_bytes(self, other, batch):
        n = ctypes.c_size_t()
        check(lib().sl_decompose_workspace_size(self._h, other._h, int(batch), ctypes.byref(n)))
        return n.value

    def decompose(self, other, f, delta_init, delta_min, iterations, t_begin=0, t_end=None,
                  f0=None, f1=None, use_graph=False, workspace=None):
        """Iterations t_begin..t_end-1 of image decomposition (sl_decompose)
        with this system as T0 and `other` as T1.  Returns (f0, f1), updated
        in place when given."""
        import torch
        self._check_x(f)
        B = f.shape[0]
        f0 = torch.empty_like(f) if f0 is None else f0
        f1 = torch.empty_like(f) if f1 is None else f1
        self._check_x(f0)
        self._check_x(f1)
        if workspace is None:
            n = self.decompose_workspace_bytes(other, B)
            key = ("decompose", id(other), str(f.device))
            workspace = self._ws.get(key)
            if workspace is None or workspace.numel() < n:
                workspace = torch.empty(n, dtype=torch.uint8, device=f.device)
                self._ws[key] = workspace
        t_end = iterations if t_end is None else t_end
        check(lib().sl_decompose(self._h, other._h, _ptr(f), B, _ptr(delta_init),
                                 float(delta_min), int(iterations), int(t_begin), int(t_end),
                                 _ptr(f0), _ptr(f1), 1 if use_graph else 0, _ptr(workspace),
                                 workspace.numel(), _stream()))
        return f0, f1

    def set_line_plan(self, values_factor):
        """Values per thread of the 1024-point line FFTs: 1 (default) or 2."""
        check(lib().sl_system_set_line_plan(self._h, int(values_factor)))

    def line_plan(self):
        v = ctypes.c_int()
        check(lib().sl_system_line_plan(self._h, ctypes.byref(v)))
        return v.value

    def set_xcd(self, enable=True, spin_limit=0):
        """Turn the XCD-cooperative 2D passes on or off (off by default;
        spin_limit: polls before a wait gives up, 0 = default)."""
        check(lib().sl_system_set_xcd(self._h, int(bool(enable)), int(spin_limit)))

    def xcd_active(self, batch):
        a = ctypes.c_int()
        check(lib().sl_system_xcd_active(self._h, int(batch), ctypes.byref(a)))
        return bool(a.value)

    def set_block_shape(self, inv_images=0, split_pairs=1):
        """Schedule choice of the 2D column passes (sl_system_set_block_shape)."""
        check(lib().sl_system_set_block_shape(self._h, int(inv_images), int(split_pairs)))
        self._ws = {}

    def inpaint_workspace_bytes(self, batch):
        n = ctypes.c_size_t()
        check(lib().sl_inpaint_workspace_size(self._h, int(batch), ctypes.byref(n)))
        return n.value

    def inpaint(self, f_masked, mask, delta_init, delta_min, iterations, t_begin=0, t_end=None,
                f=None, use_graph=False, workspace=None):
        """Iterations t_begin..t_end-1 of inpainting by iterative hard
        thresholding (sl_inpaint).  mask: uint8 [B, dims], nonzero = known;
        delta_init: float32 [B] on the device; f: the estimate after t_begin
        iterations (updated in place and returned)."""
        import torch
        self._check_x(f_masked)
        B = f_masked.shape[0]
        if not (mask.dtype == torch.uint8 and mask.is_cuda and mask.is_contiguous()
                and mask.shape == f_masked.shape):
            raise ValueError("mask must be a contiguous uint8 CUDA tensor shaped like f_masked")
        if f is None:
            f = torch.empty_like(f_masked)
        self._check_x(f)
        if workspace is None:
            n = self.inpaint_workspace_bytes(B)
            workspace = self._ws.get(("inpaint", str(f.device)))
            if workspace is None or workspace.numel() < n:
                workspace = torch.empty(n, dtype=torch.uint8, device=f.device)
                self._ws[("inpaint", str(f.device))] = workspace
        t_end = iterations if t_end is None else t_end
        check(lib().sl_inpaint(self._h, _ptr(f_masked), _ptr(mask), B, _ptr(delta_init),
                               float(delta_min), int(iterations), int(t_begin), int(t_end),
                               _ptr(f), 1 if use_graph else 0, _ptr(workspace),
                               workspace.numel(), _stream()))
        return f


CNN_PARAMS = 10145
SQERR_SCRATCH = 1025


class Shrinkage:
    """Per-scale learned shrinkage network bound to a 2D system.

    params holds the FP32 master copy [J, CNN_PARAMS]; the matrix-core
    kernels read the bfloat16 operand pack rebuilt by pack()."""

    def __init__(self, system, params):
        import torch
        self.sys = system
        self.J = system.n_scales
        self.params = params.contiguous()
        assert self.params.shape == (self.J, CNN_PARAMS) and self.params.dtype == torch.float32
        n = lib().sl_cnn_packed_bytes(self.J)
        self.packed = torch.empty(n, dtype=torch.uint8, device=params.device)
        self._ws = {}
        self.pack()

    def pack(self):
        check(lib().sl_cnn_pack(_ptr(self.params), self.J, _ptr(self.packed), _stream()))

    def _workspace(self, B, training, device):
        import torch
        n = ctypes.c_size_t()
        check(lib().sl_cnn_workspace_size(self.sys._h, int(B), int(training), ctypes.byref(n)))
        key = (int(training), str(device))
        ws = self._ws.get(key)
        if ws is None or ws.numel() < n.value:
            ws = torch.empty(n.value, dtype=torch.uint8, device=device)
            self._ws[key] = ws
        return ws

    def apply(self, coeffs, sigma, out=None, gains=None):
        import torch
        B = coeffs.shape[0]
        if out is None:
            out = torch.empty_like(coeffs)
        ws = self._workspace(B, False, coeffs.device)
        check(lib().sl_cnn_apply(self.sys._h, _ptr(self.params), _ptr(self.packed), _ptr(coeffs),
                                 _ptr(sigma), B, _ptr(out), _ptr(gains), _ptr(ws), ws.numel(),
                                 _stream()))
        return out

    def backward(self, coeffs, sigma, dcoeffs, grads=None):
        import torch
        B = coeffs.shape[0]
        if grads is None:
            grads = torch.empty_like(self.params)
        ws = self._workspace(B, True, coeffs.device)
        check(lib().sl_cnn_backward(self.sys._h, _ptr(self.params), _ptr(self.packed),
                                    _ptr(coeffs), _ptr(sigma), B, _ptr(dcoeffs), _ptr(grads),
                                    _ptr(ws), ws.numel(), _stream()))
        return grads


def adam_step(params, grads, m, v, lr, step):
    check(lib().sl_cnn_adam(_ptr(params), _ptr(grads), _ptr(m), _ptr(v), params.numel(),
                            float(lr), int(step), _stream()))


def sq_error_grad(a, b, scale, out, scratch):
    """out = scale (a - b); scratch[0] = sum (a - b)^2 (scratch >= SQERR_SCRATCH floats)."""
    check(lib().sl_sq_error_grad(_ptr(a), _ptr(b), a.numel(), float(scale), _ptr(out),
                                 _ptr(scratch), _stream()))
    return out


def render_cartoons(shapes, H, W, sigma, noise_seed, clean, noisy=None):
    """Rasterise packed shape tables ([n, 1 + 16 * 24] float32 on the device)."""
    n = shapes.shape[0]
    max_shapes = (shapes.shape[1] - 1) // 24
    check(lib().sl_render_cartoons(_ptr(shapes), n, H, W, max_shapes, _ptr(sigma),
                                   int(noise_seed) & 0xFFFFFFFFFFFFFFFF, _ptr(clean), _ptr(noisy),
                                   _stream()))
    return clean, noisy


def _ptr_array(tensors):
    arr = (ctypes.c_void_p * len(tensors))(*[0 if t is None else t.data_ptr() for t in tensors])
    return arr


class Multi:
    """Uneven batch: one system per size class, images of a class contiguous."""

    def __init__(self, systems, counts):
        self.systems = list(systems)
        self.counts = [int(c) for c in counts]
        h = ctypes.c_void_p()
        sysarr = (ctypes.c_void_p * len(systems))(*[s._h.value for s in systems])
        cnt = (ctypes.c_int * len(counts))(*self.counts)
        check(lib().sl_multi_create(sysarr, cnt, len(systems), ctypes.byref(h)))
        self._h = h
        self._keep = []

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.sl_multi_free(h)
            self._h = None

    def workspace_bytes(self):
        n = ctypes.c_size_t()
        check(lib().sl_multi_workspace_size(self._h, ctypes.byref(n)))
        return n.value

    def _args(self, xs, coeffs, scales, sigmas, K, outs):
        arrs = [_ptr_array(xs), _ptr_array(coeffs),
                _ptr_array(scales) if scales is not None else None,
                _ptr_array(sigmas) if sigmas is not None else None,
                (ctypes.c_float * len(K))(*[float(k) for k in K]) if K is not None else None,
                _ptr_array(outs) if outs is not None else None]
        self._keep.append(arrs)
        return [ctypes.cast(a, ctypes.c_void_p) if a is not None else None for a in arrs]

    def run(self, what, xs, coeffs, scales=None, sigmas=None, K=None, outs=None, workspace=None):
        a = self._args(xs, coeffs, scales, sigmas, K, outs)
        check(lib().sl_multi_run(self._h, int(what), *a, _ptr(workspace), workspace.numel(),
                                 _stream()))

    def autotune(self, xs, coeffs, scales, outs, workspace, cache_path=None):
        a = self._args(xs, coeffs, scales, None, None, outs)
        check(lib().sl_multi_autotune(self._h, a[0], a[1], a[2], a[5], _ptr(workspace),
                                      workspace.numel(),
                                      cache_path.encode() if cache_path else None, _stream()))

    def graph_build(self, what, xs, coeffs, scales=None, sigmas=None, K=None, outs=None,
                    workspace=None):
        a = self._args(xs, coeffs, scales, sigmas, K, outs)
        check(lib().sl_multi_graph_build(self._h, int(what), *a, _ptr(workspace),
                                         workspace.numel()))

    def set_schedule(self, per_class):
        check(lib().sl_multi_set_schedule(self._h, int(bool(per_class))))

    def multi_class_rows(self):
        v = ctypes.c_int()
        check(lib().sl_multi_schedule(self._h, ctypes.byref(v)))
        return bool(v.value)

    def graph_launch(self):
        check(lib().sl_multi_graph_launch(self._h, _stream()))
