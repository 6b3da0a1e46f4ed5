"""Torch-facing helpers over the C ABI: device tensors in, device tensors out.

Every computation runs in libjso's HIP kernels; torch only allocates device
memory and supplies the stream (the context is bound to torch's current
stream before each call).
"""
from __future__ import annotations

from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L


class Context:
    """One jso context on a GPU, bound to torch's current stream."""

    def __init__(self, device: int = 0):
        if not torch.cuda.is_available():
            raise L.JsoError("no GPU visible: the jso library needs a HIP device")
        self.device = device
        torch.cuda.set_device(device)
        self.ctx = L.jso_create(device, 0)

    def bind(self):
        L.check(L.jso_set_stream(self.ctx, torch.cuda.current_stream(self.device).cuda_stream),
                self.ctx, "jso_set_stream")
        return self.ctx

    def synchronize(self):
        L.check(L.jso_synchronize(self.ctx), self.ctx, "jso_synchronize")

    def close(self):
        if self.ctx is not None:
            L.jso_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dptr(t: Optional[torch.Tensor]) -> int:
    if t is None:
        return 0
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


class Problem:
    """One inverse-rendering problem (a loaded scene with its optimiser state)."""

    def __init__(self, spec, context: Optional[Context] = None, device: int = 0):
        self.context = context or Context(device)
        self.spec = spec
        c = self.context.bind()
        self.sid = L.jso_load_scene(c, spec)
        self.n_params, self.width, self.height = L.jso_scene_info(c, self.sid)
        self.dev = torch.device("cuda", self.context.device)

    @property
    def ctx(self):
        return self.context.bind()

    # -- parameters / target ------------------------------------------------
    def set_params(self, p) -> None:
        if isinstance(p, torch.Tensor) and p.is_cuda:
            p = p.float().contiguous()
            L.check(L.jso_set_params(self.ctx, self.sid, p.data_ptr(), L.JSO_MEM_DEVICE,
                                     self.n_params), self.context.ctx, "jso_set_params")
        else:
            L.check(L.jso_set_params(self.ctx, self.sid, np.asarray(p, np.float32)),
                    self.context.ctx, "jso_set_params")

    def get_params(self) -> np.ndarray:
        return L.jso_get_params(self.ctx, self.sid)

    def get_params_prev(self) -> np.ndarray:
        return L.jso_get_params_prev(self.ctx, self.sid)

    def set_target(self, img) -> None:
        if isinstance(img, torch.Tensor) and img.is_cuda:
            img = img.float().contiguous()
            L.check(L.jso_set_target(self.ctx, self.sid, img.data_ptr(), L.JSO_MEM_DEVICE,
                                     img.numel()), self.context.ctx, "jso_set_target")
        else:
            L.check(L.jso_set_target(self.ctx, self.sid, np.asarray(img, np.float32)),
                    self.context.ctx, "jso_set_target")

    # -- rendering ----------------------------------------------------------
    def params_tensor(self, p) -> torch.Tensor:
        if isinstance(p, torch.Tensor):
            return p.to(self.dev, torch.float32).contiguous()
        return torch.as_tensor(np.asarray(p, np.float32), device=self.dev).contiguous()

    def render(self, params, seed: int, iteration: int, tag: int, spp: int, flags: int = 0,
               crop=None, mask: Optional[torch.Tensor] = None,
               out: Optional[torch.Tensor] = None) -> torch.Tensor:
        p = self.params_tensor(params)
        img = out if out is not None else torch.zeros(self.height, self.width, 3, device=self.dev)
        o = L.render_opts(flags, crop, _dptr(mask))
        L.check(L.jso_render(self.ctx, self.sid, p.data_ptr(), seed, iteration, tag, spp, o,
                             img.data_ptr()), self.context.ctx, "jso_render")
        return img

    def render_bwd(self, params, dimg: torch.Tensor, seed: int, iteration: int, tag: int,
                   spp: int, flags: int = 0, crop=None, mask: Optional[torch.Tensor] = None,
                   out: Optional[torch.Tensor] = None) -> torch.Tensor:
        p = self.params_tensor(params)
        d = dimg.to(self.dev, torch.float32).contiguous()
        g = out if out is not None else torch.zeros(self.n_params, device=self.dev)
        o = L.render_opts(flags, crop, _dptr(mask))
        L.check(L.jso_render_bwd(self.ctx, self.sid, p.data_ptr(), seed, iteration, tag, spp,
                                 d.data_ptr(), o, g.data_ptr()), self.context.ctx,
                "jso_render_bwd")
        return g

    def estimate_gradients(self, seed: int, iteration: int, spp_prop: int = 2, spp_fd: int = 1,
                           flags: int = 0, crop=None, mask: Optional[torch.Tensor] = None,
                           with_fd: bool = True, want_img: bool = False,
                           loss: int = L.JSO_LOSS_L2, fd_mode: int = L.JSO_FD_REPLAY):
        F = torch.zeros(self.n_params, device=self.dev)
        dF = torch.zeros(self.n_params, device=self.dev) if with_fd else None
        img = torch.zeros(self.height, self.width, 3, device=self.dev) if want_img else None
        o = L.render_opts(flags, crop, _dptr(mask), loss, fd_mode)
        rc, loss = L.jso_estimate_gradients(self.ctx, self.sid, seed, iteration, spp_prop,
                                            spp_fd, o, F.data_ptr(), _dptr(dF), _dptr(img),
                                            want_loss=True)
        L.check(rc, self.context.ctx, "jso_estimate_gradients")
        return dict(F=F, dF=dF, img=img, loss=loss)

    # -- optimisation -------------------------------------------------------
    def precondition(self, g: torch.Tensor, lam: float) -> torch.Tensor:
        """(I + lam L)^-1 g per channel on the texel grid, in place (g: device
        float32 tensor of n_params)."""
        assert g.is_cuda and g.dtype == torch.float32 and g.is_contiguous()
        assert g.numel() == self.n_params
        L.check(L.jso_precondition(self.ctx, self.sid, g.data_ptr(), lam), self.context.ctx,
                "jso_precondition")
        return g

    def meta_step(self, F: torch.Tensor, dF: torch.Tensor, eta: float, beta_F: float = 0.99,
                  beta_D: float = 0.9) -> None:
        L.check(L.jso_meta_step(self.ctx, self.sid, _dptr(F.contiguous()),
                                _dptr(dF.contiguous()), eta, beta_F, beta_D),
                self.context.ctx, "jso_meta_step")

    def adam_step(self, g: torch.Tensor, eta: float, beta1=0.9, beta2=0.999, eps=1e-8) -> None:
        L.check(L.jso_adam_step(self.ctx, self.sid, _dptr(g.contiguous()), eta, beta1, beta2,
                                eps), self.context.ctx, "jso_adam_step")

    def grad_step(self, opts, want_stats: bool = False):
        rc, stats = L.jso_grad_step(self.ctx, [self.sid], opts, want_stats)
        L.check(rc, self.context.ctx, "jso_grad_step")
        return stats[0] if want_stats else None

    def get_state(self) -> dict:
        return L.jso_get_state(self.ctx, self.sid)

    def set_state(self, st: dict) -> None:
        L.check(L.jso_set_state(self.ctx, self.sid, st), self.context.ctx, "jso_set_state")


def grad_step_many(problems: Sequence[Problem], opts, want_stats: bool = False):
    """One iteration for several problems sharing a context."""
    ctxs = {id(p.context) for p in problems}
    if len(ctxs) != 1:
        raise ValueError("problems must share one Context")
    rc, stats = L.jso_grad_step(problems[0].ctx, [p.sid for p in problems], opts, want_stats)
    L.check(rc, problems[0].context.ctx, "jso_grad_step")
    return stats


class Batch:
    """Problems of one context optimised together: one launch per kernel per
    iteration for all of them, replayed from a captured HIP graph when
    use_graph is set.  max_iters[k] = 0 means no limit for problem k."""

    def __init__(self, problems: Sequence[Problem], opts, max_iters=None,
                 use_graph: bool = True):
        ctxs = {id(p.context) for p in problems}
        if len(ctxs) != 1:
            raise ValueError("problems must share one Context")
        self.context = problems[0].context
        self.problems = list(problems)
        self.batch = L.jso_batch_create(self.context.bind(), [p.sid for p in problems], opts,
                                        max_iters, use_graph)

    def step(self, iterations: int = 1) -> None:
        L.jso_batch_step(self.context.bind(), self.batch, iterations)

    def active(self) -> int:
        return L.jso_batch_active(self.context.bind(), self.batch)

    def autotune(self, iterations: int = 3):
        """Pick the fastest tile shape for this batch; returns (shape, ms per shape)."""
        return L.jso_batch_autotune(self.context.bind(), self.batch, iterations)

    def close(self) -> None:
        if self.batch:
            L.jso_batch_destroy(self.batch)
            self.batch = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
