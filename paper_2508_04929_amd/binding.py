"""ctypes binding of libcryosplat (argument marshalling only).

Every computation runs in the HIP library; this module checks tensor
placement, dtype and contiguity, packs the C structs declared in
``include/cryosplat.h`` and passes device pointers plus the current torch
stream.  It raises if the shared library is missing: there is no fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import threading
from typing import Optional

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcryosplat.so")

CS_SUM, CS_MEAN = 0, 1
_SCALE_ACT = {"exp": 0, "softplus": 1}
_AMP_ACT = {"identity": 0, "softplus": 1}


class CsGaussians(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("amps", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("scale_act", ctypes.c_int32),
                ("amp_act", ctypes.c_int32)]


class CsViews(ctypes.Structure):
    _fields_ = [("rot", ctypes.c_void_p), ("shift", ctypes.c_void_p), ("b", ctypes.c_int64),
                ("d", ctypes.c_int32), ("pixel", ctypes.c_float)]


class CsCtf(ctypes.Structure):
    _fields_ = [("defocus_u", ctypes.c_void_p), ("defocus_v", ctypes.c_void_p),
                ("astig", ctypes.c_void_p), ("phase", ctypes.c_void_p),
                ("voltage_kv", ctypes.c_double), ("cs_mm", ctypes.c_double),
                ("amp_contrast", ctypes.c_double), ("bfactor", ctypes.c_double)]


class CsGrads(ctypes.Structure):
    _fields_ = [("means", ctypes.c_void_p), ("log_scales", ctypes.c_void_p),
                ("quats", ctypes.c_void_p), ("amps", ctypes.c_void_p)]


class CsOptions(ctypes.Structure):
    _fields_ = [("q_cut", ctypes.c_float), ("tile", ctypes.c_int32), ("halo", ctypes.c_int32),
                ("budget", ctypes.c_int32), ("graph", ctypes.c_int32)]


class CsProblem(ctypes.Structure):
    _fields_ = [("g", CsGaussians), ("v", CsViews), ("ctf", ctypes.POINTER(CsCtf)),
                ("opt", CsOptions), ("observed", ctypes.c_void_p), ("reduction", ctypes.c_int32),
                ("loss", ctypes.c_void_p), ("grads", CsGrads), ("images_out", ctypes.c_void_p)]


#: Entry points declared in include/cryosplat.h.
EXPORTS = ("cs_create", "cs_destroy", "cs_last_error", "cs_render", "cs_render_backward",
           "cs_loss_and_grad", "cs_loss_and_grad_multi", "cs_autotune", "cs_adam_step",
           "cs_pair_count", "cs_set_timing", "cs_stage_time")


class CryoSplatError(RuntimeError):
    pass


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """dlopen libcryosplat.so and declare its signatures (no GPU needed)."""
    if not os.path.exists(path):
        raise CryoSplatError(
            f"{path} is missing: build it with paper_2508_04929_amd.build.build() "
            "(the renderer has no CPU fallback)")
    lib = ctypes.CDLL(path)
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    P = ctypes.POINTER
    lib.cs_create.argtypes = [ctypes.c_int, P(vp)]
    lib.cs_create.restype = ctypes.c_int
    lib.cs_destroy.argtypes = [vp]
    lib.cs_destroy.restype = None
    lib.cs_last_error.argtypes = [vp]
    lib.cs_last_error.restype = ctypes.c_char_p
    lib.cs_render.argtypes = [vp, P(CsGaussians), P(CsViews), P(CsCtf), P(CsOptions), vp, vp]
    lib.cs_render.restype = ctypes.c_int
    lib.cs_render_backward.argtypes = [vp, P(CsGaussians), P(CsViews), P(CsCtf), P(CsOptions), vp,
                                       P(CsGrads), vp]
    lib.cs_render_backward.restype = ctypes.c_int
    lib.cs_loss_and_grad.argtypes = [vp, P(CsGaussians), P(CsViews), P(CsCtf), P(CsOptions), vp,
                                     i32, vp, P(CsGrads), vp, vp]
    lib.cs_loss_and_grad.restype = ctypes.c_int
    lib.cs_loss_and_grad_multi.argtypes = [vp, P(CsProblem), i32, i32, vp]
    lib.cs_loss_and_grad_multi.restype = ctypes.c_int
    lib.cs_autotune.argtypes = [vp, P(CsProblem), i32, i32, vp]
    lib.cs_autotune.restype = ctypes.c_int
    lib.cs_adam_step.argtypes = [vp, vp, vp, vp, vp, i64, i64, f32, f32, f32, f32, vp]
    lib.cs_adam_step.restype = ctypes.c_int
    lib.cs_pair_count.argtypes = [vp, P(CsGaussians), P(CsViews), P(CsOptions), vp, vp]
    lib.cs_pair_count.restype = ctypes.c_int
    lib.cs_set_timing.argtypes = [vp, ctypes.c_int]
    lib.cs_set_timing.restype = ctypes.c_int
    lib.cs_stage_time.argtypes = [vp, ctypes.c_char_p, P(ctypes.c_double), P(i64)]
    lib.cs_stage_time.restype = ctypes.c_int
    return lib


@dataclasses.dataclass
class Ctf:
    """Per-image CTF parameters as device tensors [B] plus microscope scalars."""
    defocus_u: torch.Tensor
    defocus_v: torch.Tensor
    astig: Optional[torch.Tensor] = None
    phase: Optional[torch.Tensor] = None
    voltage_kv: float = 300.0
    cs_mm: float = 2.7
    amp_contrast: float = 0.1
    bfactor: float = 0.0


@dataclasses.dataclass
class Options:
    q_cut: float = 0.0   # <= 0: library default 2 ln 1e6
    tile: int = 0
    halo: int = 0
    budget: int = 0
    graph: int = 0       # 1: capture/replay the call as a HIP graph


@dataclasses.dataclass
class Problem:
    """One independent problem of a batched call (device tensors).

    ``loss`` [B+1] and the gradient tensors are outputs; they are allocated
    by :meth:`Library.make_problem` and reused across calls so that a
    captured graph stays valid.
    """
    means: torch.Tensor
    log_scales: torch.Tensor
    quats: torch.Tensor
    amps: torch.Tensor
    rot: torch.Tensor
    shift: Optional[torch.Tensor]
    D: int
    pixel: float
    observed: torch.Tensor
    ctf: Optional[Ctf] = None
    options: Optional[Options] = None
    reduction: str = "sum"
    loss: Optional[torch.Tensor] = None
    grads: Optional[dict] = None
    images_out: Optional[torch.Tensor] = None
    scale_act: str = "exp"
    amp_act: str = "identity"


def _ptr(t: Optional[torch.Tensor], name: str, device, shape=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t.data_ptr()


class Library:
    """One libcryosplat context per device, created lazily."""

    def __init__(self, lib: ctypes.CDLL):
        self.lib = lib
        self._ctx = {}
        self._lock = threading.Lock()

    def ctx(self, device: torch.device):
        idx = device.index if device.index is not None else torch.cuda.current_device()
        with self._lock:
            if idx not in self._ctx:
                h = ctypes.c_void_p()
                rc = self.lib.cs_create(idx, ctypes.byref(h))
                if rc != 0:
                    raise CryoSplatError(f"cs_create({idx}) failed with status {rc}")
                self._ctx[idx] = h
            return self._ctx[idx]

    def _check(self, ctx, rc, what):
        if rc != 0:
            msg = self.lib.cs_last_error(ctx).decode(errors="replace")
            raise CryoSplatError(f"{what} failed ({rc}): {msg}")

    # -- struct packing -------------------------------------------------
    @staticmethod
    def _pack(means, log_scales, quats, amps, rot, shift, D, pixel, ctf, options,
              scale_act, amp_act):
        dev = rot.device
        n = means.shape[0]
        b = rot.shape[0]
        g = CsGaussians(_ptr(means, "means", dev, (n, 3)), _ptr(log_scales, "log_scales", dev, (n, 3)),
                        _ptr(quats, "quats", dev, (n, 4)), _ptr(amps, "amps", dev, (n,)), n,
                        _SCALE_ACT[scale_act], _AMP_ACT[amp_act])
        v = CsViews(_ptr(rot, "rot", dev, (b, 3, 3)), _ptr(shift, "shift", dev, (b, 2)), b, int(D),
                    float(pixel))
        c = None
        if ctf is not None:
            c = CsCtf(_ptr(ctf.defocus_u, "defocus_u", dev, (b,)), _ptr(ctf.defocus_v, "defocus_v", dev, (b,)),
                      _ptr(ctf.astig, "astig", dev, (b,)), _ptr(ctf.phase, "phase", dev, (b,)),
                      float(ctf.voltage_kv), float(ctf.cs_mm), float(ctf.amp_contrast),
                      float(ctf.bfactor))
        o = None
        if options is not None:
            o = CsOptions(float(options.q_cut), int(options.tile), int(options.halo),
                          int(options.budget), int(options.graph))
        return dev, n, b, g, v, c, o

    @staticmethod
    def _ref(s):
        return ctypes.byref(s) if s is not None else None

    # -- entry points ----------------------------------------------------
    def render(self, means, log_scales, quats, amps, rot, shift, D, pixel, ctf=None,
               options=None, scale_act="exp", amp_act="identity", out=None):
        dev, n, b, g, v, c, o = self._pack(means, log_scales, quats, amps, rot, shift, D, pixel,
                                           ctf, options, scale_act, amp_act)
        if out is None:
            out = torch.empty((b, D, D), device=dev, dtype=torch.float32)
        _ptr(out, "images", dev, (b, D, D))
        ctx = self.ctx(dev)
        rc = self.lib.cs_render(ctx, ctypes.byref(g), ctypes.byref(v), self._ref(c), self._ref(o),
                                out.data_ptr(), torch.cuda.current_stream(dev).cuda_stream)
        self._check(ctx, rc, "cs_render")
        return out

    def _grads(self, dev, n, want=True):
        z = lambda *s: torch.empty(s, device=dev, dtype=torch.float32)
        gr = {"means": z(n, 3), "log_scales": z(n, 3), "quats": z(n, 4), "amps": z(n)}
        cg = CsGrads(gr["means"].data_ptr(), gr["log_scales"].data_ptr(), gr["quats"].data_ptr(),
                     gr["amps"].data_ptr())
        return gr, cg

    def render_backward(self, means, log_scales, quats, amps, rot, shift, D, pixel, d_images,
                        ctf=None, options=None, scale_act="exp", amp_act="identity"):
        dev, n, b, g, v, c, o = self._pack(means, log_scales, quats, amps, rot, shift, D, pixel,
                                           ctf, options, scale_act, amp_act)
        _ptr(d_images, "d_images", dev, (b, D, D))
        gr, cg = self._grads(dev, n)
        ctx = self.ctx(dev)
        rc = self.lib.cs_render_backward(ctx, ctypes.byref(g), ctypes.byref(v), self._ref(c),
                                         self._ref(o), d_images.data_ptr(), ctypes.byref(cg),
                                         torch.cuda.current_stream(dev).cuda_stream)
        self._check(ctx, rc, "cs_render_backward")
        return gr

    def loss_and_grad(self, means, log_scales, quats, amps, rot, shift, D, pixel, observed,
                      ctf=None, options=None, reduction="sum", want_grads=True,
                      want_images=False, scale_act="exp", amp_act="identity", grads=None,
                      loss=None):
        dev, n, b, g, v, c, o = self._pack(means, log_scales, quats, amps, rot, shift, D, pixel,
                                           ctf, options, scale_act, amp_act)
        _ptr(observed, "observed", dev, (b, D, D))
        if loss is None:
            loss = torch.empty(b + 1, device=dev, dtype=torch.float32)
        _ptr(loss, "loss", dev, (b + 1,))
        cg = None
        if want_grads:
            if grads is None:
                grads, cg = self._grads(dev, n)
            else:
                cg = CsGrads(*(_ptr(grads[k], k, dev) for k in ("means", "log_scales", "quats", "amps")))
        images = torch.empty((b, D, D), device=dev, dtype=torch.float32) if want_images else None
        ctx = self.ctx(dev)
        rc = self.lib.cs_loss_and_grad(
            ctx, ctypes.byref(g), ctypes.byref(v), self._ref(c), self._ref(o), observed.data_ptr(),
            CS_MEAN if reduction == "mean" else CS_SUM, loss.data_ptr(), self._ref(cg),
            images.data_ptr() if images is not None else None,
            torch.cuda.current_stream(dev).cuda_stream)
        self._check(ctx, rc, "cs_loss_and_grad")
        return loss, (grads if want_grads else None), images

    # -- batched problems -------------------------------------------------
    def make_problem(self, means, log_scales, quats, amps, rot, shift, D, pixel, observed,
                     ctf=None, options=None, reduction="sum", want_grads=True, want_images=False,
                     scale_act="exp", amp_act="identity") -> Problem:
        dev = rot.device
        n, b = means.shape[0], rot.shape[0]
        z = lambda *s: torch.zeros(s, device=dev, dtype=torch.float32)
        grads = ({"means": z(n, 3), "log_scales": z(n, 3), "quats": z(n, 4), "amps": z(n)}
                 if want_grads else None)
        return Problem(means, log_scales, quats, amps, rot, shift, D, pixel, observed, ctf,
                       options or Options(), reduction, z(b + 1), grads,
                       z(b, D, D) if want_images else None, scale_act, amp_act)

    def _problem_struct(self, pr: Problem):
        dev, n, b, g, v, c, o = self._pack(pr.means, pr.log_scales, pr.quats, pr.amps, pr.rot,
                                           pr.shift, pr.D, pr.pixel, pr.ctf,
                                           pr.options or Options(), pr.scale_act, pr.amp_act)
        _ptr(pr.observed, "observed", dev, (b, pr.D, pr.D))
        _ptr(pr.loss, "loss", dev, (b + 1,))
        cg = CsGrads()
        if pr.grads is not None:
            cg = CsGrads(*(_ptr(pr.grads[k], k, dev) for k in ("means", "log_scales", "quats", "amps")))
        io = _ptr(pr.images_out, "images_out", dev, (b, pr.D, pr.D)) if pr.images_out is not None else None
        s = CsProblem(g, v, ctypes.pointer(c) if c is not None else None, o, pr.observed.data_ptr(),
                      CS_MEAN if pr.reduction == "mean" else CS_SUM, pr.loss.data_ptr(), cg, io)
        return dev, s, c

    def _problem_array(self, problems):
        structs, keep, dev = [], [], None
        for pr in problems:
            dev, s, c = self._problem_struct(pr)
            structs.append(s)
            keep.append(c)
        arr = (CsProblem * len(structs))(*structs)
        return dev, arr, keep

    def loss_and_grad_multi(self, problems, use_graph=True):
        """All problems' losses and gradients in one batched call (writes pr.loss / pr.grads)."""
        dev, arr, keep = self._problem_array(problems)
        ctx = self.ctx(dev)
        rc = self.lib.cs_loss_and_grad_multi(ctx, arr, len(problems), 1 if use_graph else 0,
                                             torch.cuda.current_stream(dev).cuda_stream)
        self._check(ctx, rc, "cs_loss_and_grad_multi")
        del keep
        return problems

    def autotune(self, problems, reps=2):
        """Choose tile/halo/budget per problem (writes pr.options)."""
        dev, arr, keep = self._problem_array(problems)
        ctx = self.ctx(dev)
        rc = self.lib.cs_autotune(ctx, arr, len(problems), int(reps),
                                  torch.cuda.current_stream(dev).cuda_stream)
        self._check(ctx, rc, "cs_autotune")
        for pr, s in zip(problems, arr):
            base = pr.options or Options()
            pr.options = Options(q_cut=base.q_cut, tile=s.opt.tile, halo=s.opt.halo,
                                 budget=s.opt.budget, graph=base.graph)
        del keep
        return problems

    def adam_step(self, params, grads, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        dev = params.device
        for t, nm in ((params, "params"), (grads, "grads"), (m, "m"), (v, "v")):
            _ptr(t, nm, dev, tuple(params.shape))
        ctx = self.ctx(dev)
        rc = self.lib.cs_adam_step(ctx, params.data_ptr(), grads.data_ptr(), m.data_ptr(),
                                   v.data_ptr(), params.numel(), int(step), float(lr), float(b1),
                                   float(b2), float(eps), torch.cuda.current_stream(dev).cuda_stream)
        self._check(ctx, rc, "cs_adam_step")

    def pair_count(self, means, log_scales, quats, amps, rot, shift, D, pixel, options=None,
                   scale_act="exp"):
        dev, n, b, g, v, c, o = self._pack(means, log_scales, quats, amps, rot, shift, D, pixel,
                                           None, options, scale_act, "identity")
        out = torch.empty(b, device=dev, dtype=torch.int64)
        ctx = self.ctx(dev)
        rc = self.lib.cs_pair_count(ctx, ctypes.byref(g), ctypes.byref(v), self._ref(o),
                                    out.data_ptr(), torch.cuda.current_stream(dev).cuda_stream)
        self._check(ctx, rc, "cs_pair_count")
        return out


    def set_timing(self, device, enable: bool):
        ctx = self.ctx(torch.device(device))
        self._check(ctx, self.lib.cs_set_timing(ctx, 1 if enable else 0), "cs_set_timing")

    def stage_time(self, device, name: str):
        """(total milliseconds, launches) of one library stage since timing was enabled."""
        ctx = self.ctx(torch.device(device))
        ms, n = ctypes.c_double(), ctypes.c_int64()
        self._check(ctx, self.lib.cs_stage_time(ctx, name.encode(), ctypes.byref(ms), ctypes.byref(n)),
                    "cs_stage_time")
        return ms.value, n.value


#: Kernel stages the library may launch (names reported by stage_time).
STAGES = ("k_build", "k_bin_count", "k_bin_blockscan", "k_scan", "k_bin_scatter", "k_ctf_table", "k_splat_fwd", "k_canvas_reduce",
          "k_big_fwd", "k_fft_rows_fwd", "k_fft_cols_ctf", "k_fft_rows_inv_loss", "k_fft_rows_inv",
          "k_residual", "k_loss_reduce", "k_loss_total", "k_splat_bwd", "k_big_bwd", "k_chain", "k_adam",
          "k_fill", "k_pair_count")

_LIB: Optional[Library] = None


def library() -> Library:
    """The process-wide binding (loads libcryosplat.so on first use)."""
    global _LIB
    if _LIB is None:
        _LIB = Library(load_library())
    return _LIB
