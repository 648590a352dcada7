"""Python face of libhrt.so: plans, forward/adjoint on torch device tensors,
and an autograd Function.  PyTorch supplies device memory and streams; the
transform itself runs only in the library's HIP kernels."""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib


def describe(desc) -> dict:
    """Host-only geometry and sizes of a plan (no GPU needed)."""
    lib = _lib.load()
    info = _lib.HrtInfo()
    _lib.check(lib.hrt_plan_describe(C.byref(_lib.make_desc(desc)), C.byref(info)),
               "hrt_plan_describe")
    return info.as_dict()


def _stream_handle(stream) -> C.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Plan:
    """A log-polar hyperbolic Radon transform plan on the current device."""

    def __init__(self, desc, device=None):
        self.desc = desc
        self._lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device()
                                   if device is None else torch.device(device).index)
        handle = C.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self._lib.hrt_plan_create(C.byref(_lib.make_desc(desc)),
                                                 C.byref(handle)), "hrt_plan_create")
        self._h = handle
        info = _lib.HrtInfo()
        _lib.check(self._lib.hrt_query(self._h, C.byref(info)), "hrt_query")
        self.info = info.as_dict()
        self.data_shape = (int(desc.nx), int(desc.nt))
        self.radon_shape = (int(desc.nq), int(desc.ntau))

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.hrt_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check_in(self, x: torch.Tensor, shape, name: str) -> None:
        if not isinstance(x, torch.Tensor) or x.device != self.device:
            raise ValueError(f"{name} must be a tensor on {self.device}")
        if x.dtype != torch.float32 or not x.is_contiguous():
            raise ValueError(f"{name} must be contiguous float32")
        if tuple(x.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(x.shape)}, expected {shape}")

    def _call(self, fn, x, out, in_shape, out_shape, stream, where):
        self._check_in(x, in_shape, "input")
        if out is None:
            out = torch.empty(out_shape, dtype=torch.float32, device=self.device)
        else:
            self._check_in(out, out_shape, "out")
        _lib.check(fn(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
                      _stream_handle(stream)), where)
        return out

    def forward(self, f: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        """g = R_h f: f (nx, nt) -> g (nq, ntau)."""
        return self._call(self._lib.hrt_forward, f, out, self.data_shape,
                          self.radon_shape, stream, "hrt_forward")

    def adjoint(self, g: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        """f = R_h^T g: g (nq, ntau) -> f (nx, nt)."""
        return self._call(self._lib.hrt_adjoint, g, out, self.radon_shape,
                          self.data_shape, stream, "hrt_adjoint")

    def direct_forward(self, f: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        """Direct summation over hyperbolas (float32 GPU reference method)."""
        return self._call(self._lib.hrt_direct_forward, f, out, self.data_shape,
                          self.radon_shape, stream, "hrt_direct_forward")

    def direct_adjoint(self, g: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        return self._call(self._lib.hrt_direct_adjoint, g, out, self.radon_shape,
                          self.data_shape, stream, "hrt_direct_adjoint")

    # kernels in the order of the library's profile slots
    STAGES = ("fwd_spread", "fwd_rowfft", "fwd_colfft", "fwd_rowifft", "fwd_gather",
              "adj_spread", "adj_rowfft", "adj_colfft", "adj_rowifft", "adj_gather")

    def profile_begin(self, max_records: int) -> None:
        """Start per-kernel HIP-event timing of forward/adjoint launches."""
        _lib.check(self._lib.hrt_profile_begin(self._h, int(max_records)),
                   "hrt_profile_begin")

    def profile_end(self) -> dict:
        """{stage: (summed ms, launches)} since profile_begin."""
        ms = (C.c_double * len(self.STAGES))()
        cnt = (C.c_int64 * len(self.STAGES))()
        _lib.check(self._lib.hrt_profile_end(self._h, ms, cnt), "hrt_profile_end")
        return {name: (ms[i], cnt[i]) for i, name in enumerate(self.STAGES)}

    def kernel(self) -> np.ndarray:
        """The plan's kernel multiplier K[k1][k2] (complex64, k1 < k1_kept,
        0 <= k2 < k2_kept)."""
        k1, k2 = self.info["k1_kept"], self.info["k2_kept"]
        out = np.empty((k1, k2, 2), dtype=np.float32)
        _lib.check(self._lib.hrt_plan_kernel(self._h, C.c_void_p(out.ctypes.data)),
                   "hrt_plan_kernel")
        return out[..., 0] + 1j * out[..., 1]


class HRTFunction(torch.autograd.Function):
    """g = R_h f with backward grad_f = R_h^T grad_g (R_h is linear)."""

    @staticmethod
    def forward(ctx, f, plan):
        ctx.plan = plan
        return plan.forward(f.contiguous())

    @staticmethod
    def backward(ctx, grad_g):
        return ctx.plan.adjoint(grad_g.contiguous()), None


def hrt_forward(f: torch.Tensor, plan: Plan) -> torch.Tensor:
    return HRTFunction.apply(f, plan)
