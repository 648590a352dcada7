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

    def __init__(self, desc, device=None, flags: int = 0, tuned: bool = False):
        """flags: HRT_TUNE_* kernel variants; tuned=True takes them from the
        autotuner's cache (paper_1604_07651_amd.autotune) when it has them."""
        if tuned:
            from . import autotune
            flags = autotune.tuned_flags(desc)
        self.desc = desc
        self.flags = int(flags)
        self._lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device()
                                   if device is None else torch.device(device).index)
        handle = C.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self._lib.hrt_plan_create(C.byref(_lib.make_desc(desc, self.flags)),
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

    def forward_noalloc(self, f: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
        """hrt_forward_noalloc: g = R_h f with the library's static per-device
        workspace instead of the plan's (the caller provides `out`)."""
        return self._call(self._lib.hrt_forward_noalloc, f, out, self.data_shape,
                          self.radon_shape, stream, "hrt_forward_noalloc")

    def adjoint(self, g: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        """f = R_h^T g: g (nq, ntau) -> f (nx, nt)."""
        return self._call(self._lib.hrt_adjoint, g, out, self.radon_shape,
                          self.data_shape, stream, "hrt_adjoint")

    def normal(self, f: torch.Tensor, g=None, out=None, stream=None):
        """g = R_h f and R_h^T g in one call (hrt_normal): f (nx, nt) -> (g (nq, ntau),
        R_h^T g (nx, nt)); out may be f itself."""
        self._check_in(f, self.data_shape, "input")
        if g is None:
            g = torch.empty(self.radon_shape, dtype=torch.float32, device=self.device)
        else:
            self._check_in(g, self.radon_shape, "g")
        if out is None:
            out = torch.empty(self.data_shape, dtype=torch.float32, device=self.device)
        else:
            self._check_in(out, self.data_shape, "out")
        _lib.check(self._lib.hrt_normal(self._h, C.c_void_p(f.data_ptr()),
                                        C.c_void_p(g.data_ptr()), C.c_void_p(out.data_ptr()),
                                        _stream_handle(stream)), "hrt_normal")
        return g, out

    def direct_forward(self, f: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        """Direct summation over hyperbolas (float32 GPU reference method)."""
        return self._call(self._lib.hrt_direct_forward, f, out, self.data_shape,
                          self.radon_shape, stream, "hrt_direct_forward")

    def direct_adjoint(self, g: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        return self._call(self._lib.hrt_direct_adjoint, g, out, self.radon_shape,
                          self.data_shape, stream, "hrt_direct_adjoint")

    # kernels in the order of the library's profile slots
    STAGES = ("fwd_absmax", "fwd_spread", "fwd_rowfft", "fwd_colfft", "fwd_rowifft",
              "fwd_gather", "adj_absmax", "adj_spread", "adj_rowfft", "adj_colfft",
              "adj_rowifft", "adj_gather")

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


    # --- soft-thresholding iterations (Section 3, eqs. iters / itersmd) ---

    def _work(self, work):
        if work is None:
            work = (torch.empty(self.data_shape, device=self.device),
                    torch.empty(self.radon_shape, device=self.device))
        self._check_in(work[0], self.data_shape, "work_data")
        self._check_in(work[1], self.radon_shape, "work_radon")
        return work

    def _ista_args(self, f, mask, g):
        self._check_in(f, self.data_shape, "f")
        self._check_in(g, self.radon_shape, "g")
        if mask is not None:
            self._check_in(mask, self.data_shape, "mask")
        return C.c_void_p(mask.data_ptr()) if mask is not None else None

    def ista_iterate(self, f, g, iters: int, c2: float, mu: float, mask=None, work=None,
                     stream=None) -> torch.Tensor:
        """`iters` steps of g <- S_{c2 mu}(g + c2 R(f - mask R^T g)), in place on g."""
        m = self._ista_args(f, mask, g)
        wd, wr = self._work(work)
        _lib.check(self._lib.hrt_ista_iterate(
            self._h, C.c_void_p(f.data_ptr()), m, C.c_void_p(g.data_ptr()),
            C.c_void_p(wd.data_ptr()), C.c_void_p(wr.data_ptr()), int(iters), float(c2),
            float(mu), _stream_handle(stream)), "hrt_ista_iterate")
        return g

    def ista_graph(self, f, g, iters: int, c2: float, mu: float, mask=None, work=None):
        """The same iterations captured in a HIP graph; returns an IstaGraph
        whose launch() replays them on the bound arrays."""
        m = self._ista_args(f, mask, g)
        wd, wr = self._work(work)
        handle = C.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self._lib.hrt_ista_graph_create(
                self._h, C.c_void_p(f.data_ptr()), m, C.c_void_p(g.data_ptr()),
                C.c_void_p(wd.data_ptr()), C.c_void_p(wr.data_ptr()), int(iters), float(c2),
                float(mu), C.byref(handle)), "hrt_ista_graph_create")
        return IstaGraph(self._lib, handle, (f, mask, g, wd, wr))

    def opnorm2(self, iters: int = 30, seed: int = 0, stream=None) -> float:
        """||R||^2 by float64 power iteration on R^T R."""
        wd = torch.empty(self.data_shape, device=self.device)
        wd2 = torch.empty(self.data_shape, device=self.device)
        wr = torch.empty(self.radon_shape, device=self.device)
        out = C.c_double()
        _lib.check(self._lib.hrt_opnorm2(self._h, int(iters), C.c_uint64(seed),
                                         C.c_void_p(wd.data_ptr()), C.c_void_p(wd2.data_ptr()),
                                         C.c_void_p(wr.data_ptr()), C.byref(out),
                                         _stream_handle(stream)), "hrt_opnorm2")
        return out.value


    def demultiple(self, f, g, qb0: float, qb_slope: float = 0.0, out=None, work=None,
                   stream=None) -> torch.Tensor:
        """Primaries f - R^T (g where q > qb0 + qb_slope tau) (Section 6)."""
        self._check_in(f, self.data_shape, "f")
        self._check_in(g, self.radon_shape, "g")
        if out is None:
            out = torch.empty(self.data_shape, device=self.device)
        self._check_in(out, self.data_shape, "out")
        wr = torch.empty(self.radon_shape, device=self.device) if work is None else work
        self._check_in(wr, self.radon_shape, "work")
        _lib.check(self._lib.hrt_demultiple(self._h, C.c_void_p(f.data_ptr()),
                                            C.c_void_p(g.data_ptr()), float(qb0),
                                            float(qb_slope), C.c_void_p(out.data_ptr()),
                                            C.c_void_p(wr.data_ptr()), _stream_handle(stream)),
                   "hrt_demultiple")
        return out


class IstaGraph:
    """An executable HIP graph of soft-thresholding iterations (keeps the
    arrays it was captured on alive)."""

    def __init__(self, lib, handle, arrays):
        self._lib, self._h, self._arrays = lib, handle, arrays

    def launch(self, stream=None) -> None:
        _lib.check(self._lib.hrt_graph_launch(self._h, _stream_handle(stream)),
                   "hrt_graph_launch")

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.hrt_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ista(plan: Plan, f: torch.Tensor, mask=None, iters: int = 100, mu: float = 0.0,
         c2=None, graph: bool = True, g0=None) -> torch.Tensor:
    """Sparse Radon panel g of a gather f with missing traces (mask = 1 where
    recorded) by `iters` soft-thresholding iterations of eq. itersmd; the
    step c2 defaults to 0.99 / ||R||^2 (float64 power iteration).  Returns g;
    the interpolated gather is plan.adjoint(g)."""
    if c2 is None:
        c2 = 0.99 / plan.opnorm2()
    g = torch.zeros(plan.radon_shape, device=plan.device) if g0 is None else g0.clone()
    if graph:
        gr = plan.ista_graph(f, g, iters, c2, mu, mask)
        gr.launch()
        torch.cuda.current_stream().synchronize()
        gr.close()
    else:
        plan.ista_iterate(f, g, iters, c2, mu, mask)
    return g


class Batch:
    """Uneven batch of gathers transformed by one launch per kernel; arrays
    are packed 1-D float32 tensors (see offsets)."""

    def __init__(self, descs, device=None, flags=0, tuned: bool = False):
        """flags: HRT_TUNE_* kernel variants, one int for every gather or
        one per gather; tuned=True takes each gather's from the autotuner's
        cache (its default where the cache has no entry)."""
        self._lib = _lib.load()
        self.descs = list(descs)
        n = len(self.descs)
        self.device = torch.device("cuda", torch.cuda.current_device()
                                   if device is None else torch.device(device).index)
        if tuned:
            from . import autotune
            with torch.cuda.device(self.device):
                flags = [autotune.tuned_flags(d) for d in self.descs]
        self.flags = [int(flags)] * n if isinstance(flags, int) else [int(x) for x in flags]
        if len(self.flags) != n:
            raise ValueError("one flags value per gather")
        arr = (_lib.HrtDesc * n)(*[_lib.make_desc(d, fl) for d, fl in zip(self.descs, self.flags)])
        handle = C.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self._lib.hrt_batch_create(arr, n, C.byref(handle)), "hrt_batch_create")
        self._h = handle
        d_off = (C.c_int64 * (n + 1))()
        r_off = (C.c_int64 * (n + 1))()
        _lib.check(self._lib.hrt_batch_offsets(self._h, d_off, r_off), "hrt_batch_offsets")
        self.data_off = list(d_off)
        self.radon_off = list(r_off)

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.hrt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _call(self, fn, x, out, n_in, n_out, stream, where):
        if x.dtype != torch.float32 or not x.is_contiguous() or x.numel() != n_in \
                or x.device != self.device:
            raise ValueError(f"input must be a contiguous float32 tensor of {n_in} "
                             f"elements on {self.device}")
        if out is None:
            out = torch.empty(n_out, dtype=torch.float32, device=self.device)
        elif out.dtype != torch.float32 or not out.is_contiguous() or out.numel() != n_out:
            raise ValueError(f"out must be a contiguous float32 tensor of {n_out} elements")
        _lib.check(fn(self._h, C.c_void_p(x.data_ptr()), C.c_void_p(out.data_ptr()),
                      _stream_handle(stream)), where)
        return out

    def forward(self, f_packed, out=None, stream=None):
        return self._call(self._lib.hrt_batch_forward, f_packed, out, self.data_off[-1],
                          self.radon_off[-1], stream, "hrt_batch_forward")

    def adjoint(self, g_packed, out=None, stream=None):
        return self._call(self._lib.hrt_batch_adjoint, g_packed, out, self.radon_off[-1],
                          self.data_off[-1], stream, "hrt_batch_adjoint")

    def pack_data(self, fs):
        return torch.cat([torch.as_tensor(f, dtype=torch.float32, device=self.device).reshape(-1)
                          for f in fs])

    def pack_radon(self, gs):
        return self.pack_data(gs)

    def unpack_data(self, packed):
        return [packed[self.data_off[i]:self.data_off[i + 1]].view(d.nx, d.nt)
                for i, d in enumerate(self.descs)]

    def unpack_radon(self, packed):
        return [packed[self.radon_off[i]:self.radon_off[i + 1]].view(d.nq, d.ntau)
                for i, d in enumerate(self.descs)]

    def _ista_args(self, f, mask, g, c2, mu, work):
        n = len(self.descs)

        def flat(x, size, name):
            if (not isinstance(x, torch.Tensor) or x.device != self.device
                    or x.dtype != torch.float32 or not x.is_contiguous() or x.numel() != size):
                raise ValueError(f"{name} must be a contiguous float32 tensor of {size} "
                                 f"elements on {self.device}")
            return C.c_void_p(x.data_ptr())

        nd, nr = self.data_off[-1], self.radon_off[-1]
        if work is None:
            work = (torch.empty(nd, device=self.device), torch.empty(nr, device=self.device))
        ptrs = (flat(f, nd, "f"), flat(mask, nd, "mask") if mask is not None else None,
                flat(g, nr, "g"), flat(work[0], nd, "work_data"), flat(work[1], nr, "work_radon"))
        c2v = np.broadcast_to(np.asarray(c2, dtype=np.float32), (n,)).copy()
        muv = np.broadcast_to(np.asarray(mu, dtype=np.float32), (n,)).copy()
        as_c = lambda a: a.ctypes.data_as(C.POINTER(C.c_float))  # noqa: E731
        return ptrs, (c2v, muv), as_c, work

    def opnorm2(self, i: int, iters: int = 30, seed: int = 0, stream=None) -> float:
        """||R_i||^2 of gather i by float64 power iteration (for its step
        c2_i < 1 / ||R_i||^2)."""
        d = self.descs[i]
        h = C.c_void_p()
        _lib.check(self._lib.hrt_batch_plan(self._h, int(i), C.byref(h)), "hrt_batch_plan")
        wd = torch.empty((d.nx, d.nt), device=self.device)
        wd2 = torch.empty((d.nx, d.nt), device=self.device)
        wr = torch.empty((d.nq, d.ntau), device=self.device)
        out = C.c_double()
        _lib.check(self._lib.hrt_opnorm2(h, int(iters), C.c_uint64(seed),
                                         C.c_void_p(wd.data_ptr()), C.c_void_p(wd2.data_ptr()),
                                         C.c_void_p(wr.data_ptr()), C.byref(out),
                                         _stream_handle(stream)), "hrt_opnorm2")
        return out.value

    def ista_iterate(self, f, g, iters: int, c2, mu, mask=None, work=None, stream=None):
        """`iters` soft-thresholding steps for every gather at once (packed
        arrays, in place on g); c2 and mu: one value or one per gather."""
        ptrs, (c2v, muv), as_c, _ = self._ista_args(f, mask, g, c2, mu, work)
        _lib.check(self._lib.hrt_batch_ista_iterate(self._h, *ptrs, int(iters), as_c(c2v),
                                                    as_c(muv), _stream_handle(stream)),
                   "hrt_batch_ista_iterate")
        return g

    def ista_graph(self, f, g, iters: int, c2, mu, mask=None, work=None):
        """The same iterations captured in one HIP graph (IstaGraph)."""
        ptrs, (c2v, muv), as_c, work = self._ista_args(f, mask, g, c2, mu, work)
        handle = C.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self._lib.hrt_batch_ista_graph_create(self._h, *ptrs, int(iters),
                                                             as_c(c2v), as_c(muv),
                                                             C.byref(handle)),
                       "hrt_batch_ista_graph_create")
        return IstaGraph(self._lib, handle, (f, mask, g) + tuple(work))


def split_edges(desc, n_t: int = 2, n_q: int = 2, first: float = 0.375):
    """Band edges for Split: time bands cut at the fractions first^(n_t-1),
    ..., first^2, first of the time samples (the early bands the shortest:
    they are where the Radon samples crowd on the lattice), slowness rows cut
    into n_q equal bands."""
    nt, nq = int(desc.nt), int(desc.nq)
    cuts = sorted({int(round(nt * first ** k)) for k in range(1, n_t)})
    t_edges = [0] + [c for c in cuts if 0 < c < nt] + [nt]
    q_edges = [nq * i // n_q for i in range(n_q + 1)]
    if len(set(q_edges)) != len(q_edges):
        raise ValueError("more slowness bands than slowness rows")
    return t_edges, q_edges


def _edges(edges):
    e = [int(v) for v in edges]
    return len(e) - 1, (C.c_int32 * len(e))(*e)


def describe_part(desc, t_edges, q_edges, part: int) -> dict:
    """Host-only: part `part`'s grid (keys of the description), its bands
    (j_lo, j_hi, l_lo, l_hi) and its plan summary (no GPU needed)."""
    lib = _lib.load()
    n_t, te = _edges(t_edges)
    n_q, qe = _edges(q_edges)
    sub = _lib.HrtDesc()
    win = (C.c_int32 * 4)()
    info = _lib.HrtInfo()
    _lib.check(lib.hrt_split_describe(C.byref(_lib.make_desc(desc)), n_t, te, n_q, qe,
                                      int(part), C.byref(sub), win, C.byref(info)),
               "hrt_split_describe")
    out = {name: getattr(sub, name) for name, _ in sub._fields_}
    out.update(j_lo=win[0], j_hi=win[1], l_lo=win[2], l_hi=win[3], info=info.as_dict())
    return out


class Split(Plan):
    """The transform cut into time and slowness bands (Section 4, eq.
    tsplit; Section 5): one plan per part, each rescaled to its own grid, the
    parts' results added into the whole arrays.  Same array shapes as Plan."""

    def __init__(self, desc, t_edges, q_edges, device=None, flags: int = 0):
        self.desc = desc
        self.flags = int(flags)
        self._lib = _lib.load()
        self.device = torch.device("cuda", torch.cuda.current_device()
                                   if device is None else torch.device(device).index)
        self.t_edges = [int(v) for v in t_edges]
        self.q_edges = [int(v) for v in q_edges]
        n_t, te = _edges(self.t_edges)
        n_q, qe = _edges(self.q_edges)
        handle = C.c_void_p()
        with torch.cuda.device(self.device):
            _lib.check(self._lib.hrt_split_create(C.byref(_lib.make_desc(desc, self.flags)),
                                                  n_t, te, n_q, qe, C.byref(handle)),
                       "hrt_split_create")
        self._h = handle
        self.n_parts = n_t * n_q
        self.parts = []
        for p in range(self.n_parts):
            info = _lib.HrtInfo()
            _lib.check(self._lib.hrt_split_query(self._h, p, C.byref(info)), "hrt_split_query")
            self.parts.append(info.as_dict())
        self.info = self.parts[-1]
        self.data_shape = (int(desc.nx), int(desc.nt))
        self.radon_shape = (int(desc.nq), int(desc.ntau))

    def close(self) -> None:
        if getattr(self, "_h", None):
            self._lib.hrt_split_destroy(self._h)
            self._h = None

    def forward(self, f: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        """g = sum over parts of the parts' forwards: f (nx, nt) -> g (nq, ntau)."""
        return self._call(self._lib.hrt_split_forward, f, out, self.data_shape,
                          self.radon_shape, stream, "hrt_split_forward")

    def adjoint(self, g: torch.Tensor, out=None, stream=None) -> torch.Tensor:
        """The exact transpose of forward: g (nq, ntau) -> f (nx, nt)."""
        return self._call(self._lib.hrt_split_adjoint, g, out, self.radon_shape,
                          self.data_shape, stream, "hrt_split_adjoint")

    def _unsupported(self, *a, **k):
        raise NotImplementedError("not available on a split; use a Plan")

    direct_forward = direct_adjoint = profile_begin = profile_end = kernel = _unsupported
    ista_iterate = ista_graph = opnorm2 = demultiple = _unsupported


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
