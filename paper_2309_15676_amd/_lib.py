"""ctypes binding of libjso.so (include/jso.h): argument marshalling only.

Every function here has the name of the C entry point it calls and returns
its status code; `check()` turns a failure into JsoError with the library's
message.  Device pointers are plain integers (e.g. torch ``data_ptr()``).
The library must have been built (``python -m paper_2309_15676_amd.build``);
loading fails loudly otherwise -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libjso.so")

JSO_OK, JSO_E_INVALID, JSO_E_OOM, JSO_E_HIP, JSO_E_STATE, JSO_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
JSO_MEM_HOST, JSO_MEM_DEVICE = 0, 1
JSO_MAT_PARAM = -1
JSO_TAG_TARGET, JSO_TAG_PRIMAL_PROP, JSO_TAG_ADJ_PROP = 1, 2, 3
JSO_TAG_PRIMAL_FD, JSO_TAG_ADJ_FD = 4, 5
JSO_TAG_ADAM_PRIMAL, JSO_TAG_ADAM_ADJ, JSO_TAG_EVAL = 6, 7, 8
JSO_F_NO_NEE, JSO_F_LAMBERT_ONLY, JSO_F_PARAM_INDEP, JSO_F_PIXEL_CENTER = 1, 2, 4, 8
JSO_OPT_META, JSO_OPT_ADAM = 0, 1
JSO_TAG_VAR_PRIMAL_PROP, JSO_TAG_VAR_ADJ_PROP, JSO_TAG_VAR_PRIMAL_FD, JSO_TAG_VAR_ADJ_FD = 9, 10, 11, 12
JSO_LOSS_L2, JSO_LOSS_RELATIVE = 0, 1
JSO_F_DETERMINISTIC = 16
JSO_F_NO_HIT_RECORDS = 32
JSO_ABLATE_CENTRED, JSO_ABLATE_NO_CLIP, JSO_ABLATE_UNCORRELATED = 1, 2, 4
JSO_FD_REPLAY, JSO_FD_SHARED = 0, 1
JSO_MAX_SPHERES, JSO_MAX_FIXED_MATS, JSO_MAX_TRIS = 32, 8, 4194304
JSO_LAYOUT_TEXTURE, JSO_LAYOUT_VERTEX, JSO_LAYOUT_VOLUME = 0, 1, 2
JSO_MAX_VIEWS, JSO_MAX_VOL_RES = 16, 512

EXPORTED = [
    "jso_create", "jso_destroy", "jso_last_error", "jso_set_stream", "jso_synchronize",
    "jso_set_debug", "jso_stream_key", "jso_philox", "jso_load_scene", "jso_free_scene",
    "jso_scene_info", "jso_set_params", "jso_get_params", "jso_get_params_prev",
    "jso_set_target", "jso_render", "jso_render_bwd", "jso_estimate_gradients",
    "jso_meta_step", "jso_adam_step", "jso_grad_step", "jso_get_state", "jso_set_state",
    "jso_set_timing", "jso_get_kernel_time", "jso_set_work_counting", "jso_get_work",
    "jso_batch_create", "jso_batch_step", "jso_batch_active", "jso_batch_destroy",
    "jso_batch_autotune", "jso_set_launch_config", "jso_precondition", "jso_render_bwd_noalloc",
    "jso_ub_copy", "jso_ub_atomics", "jso_ub_launch",
]
JSO_UB_RANDOM, JSO_UB_LINES, JSO_UB_16, JSO_UB_SAME, JSO_UB_ROWS = 0, 1, 2, 3, 4
JSO_NOALLOC_SCRATCH_BYTES = 128 << 20
JSO_NOALLOC_MAX_PIXELS = JSO_NOALLOC_SCRATCH_BYTES // 24
JSO_TILE_16x16, JSO_TILE_16x8, JSO_TILE_8x8, JSO_TILE_SHAPES = 0, 1, 2, 3
JSO_LAUNCH_CONFIGS = 15
PERSIST_PER_CU = (0, 1, 2, 4, 8)


def config_name(c: int) -> str:
    """Tile shape and grid of launch configuration c."""
    tile = ("16x16", "16x8", "8x8")[c % JSO_TILE_SHAPES]
    p = PERSIST_PER_CU[c // JSO_TILE_SHAPES]
    return tile + (" persistent x%d" % p if p else "")
JSO_K_FORWARD, JSO_K_ADJOINT, JSO_K_META, JSO_K_ADAM, JSO_K_FINALIZE = 0, 1, 2, 3, 4
JSO_K_PRECOND = 5
JSO_K_COUNT = 6


class JsoError(RuntimeError):
    pass


class jso_scene_desc(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int), ("height", ctypes.c_int),
        ("cam_eye", ctypes.c_float * 3), ("cam_target", ctypes.c_float * 3),
        ("cam_up", ctypes.c_float * 3), ("vfov_deg", ctypes.c_float),
        ("plane_enabled", ctypes.c_int), ("plane_mat", ctypes.c_int),
        ("plane_extent", ctypes.c_float * 4),
        ("n_spheres", ctypes.c_int), ("spheres", ctypes.POINTER(ctypes.c_float)),
        ("sphere_mat", ctypes.POINTER(ctypes.c_int)),
        ("light_enabled", ctypes.c_int), ("light_center", ctypes.c_float * 3),
        ("light_side", ctypes.c_float), ("light_Le", ctypes.c_float * 3),
        ("env", ctypes.c_float * 3),
        ("depth", ctypes.c_int), ("rr_start", ctypes.c_int), ("rr_q", ctypes.c_float),
        ("tex_w", ctypes.c_int), ("tex_h", ctypes.c_int), ("ch_mask", ctypes.c_int),
        ("fixed_default", ctypes.c_float * 5),
        ("n_fixed", ctypes.c_int), ("fixed_mats", ctypes.POINTER(ctypes.c_float)),
        ("n_verts", ctypes.c_int), ("n_tris", ctypes.c_int),
        ("verts", ctypes.POINTER(ctypes.c_float)), ("tris", ctypes.POINTER(ctypes.c_int)),
        ("mesh_mat", ctypes.c_int), ("param_layout", ctypes.c_int),
        ("vol_res", ctypes.c_int), ("vol_views", ctypes.c_int),
        ("vol_box", ctypes.c_float * 4), ("vol_sigma", ctypes.c_float),
    ]


class jso_render_opts(ctypes.Structure):
    _fields_ = [("flags", ctypes.c_uint32), ("crop", ctypes.c_int * 4),
                ("pixel_mask", ctypes.c_void_p), ("loss", ctypes.c_int),
                ("fd_mode", ctypes.c_int)]


class jso_step_opts(ctypes.Structure):
    _fields_ = [
        ("optimizer", ctypes.c_int), ("eta", ctypes.c_float), ("beta_F", ctypes.c_float),
        ("beta_D", ctypes.c_float), ("spp_prop", ctypes.c_int), ("spp_fd", ctypes.c_int),
        ("adam_beta1", ctypes.c_float), ("adam_beta2", ctypes.c_float),
        ("adam_eps", ctypes.c_float), ("adam_spp", ctypes.c_int), ("seed", ctypes.c_uint64),
        ("flags", ctypes.c_uint32), ("precond_lambda", ctypes.c_float),
        ("loss", ctypes.c_int), ("ablate", ctypes.c_uint32), ("fd_mode", ctypes.c_int),
    ]


class jso_step_stats(ctypes.Structure):
    _fields_ = [("loss", ctypes.c_double), ("step_norm2", ctypes.c_double),
                ("iteration", ctypes.c_uint32)]


class jso_state(ctypes.Structure):
    _fields_ = [
        ("params", ctypes.c_void_p), ("params_prev", ctypes.c_void_p),
        ("mean", ctypes.c_void_p), ("var", ctypes.c_void_p), ("alpha_prev", ctypes.c_void_p),
        ("m2_F", ctypes.c_void_p), ("m2_D", ctypes.c_void_p),
        ("adam_m", ctypes.c_void_p), ("adam_v", ctypes.c_void_p),
        ("iteration", ctypes.c_uint32), ("count_F", ctypes.c_uint32),
        ("count_D", ctypes.c_uint32), ("adam_t", ctypes.c_uint32),
        ("step_norm2", ctypes.c_double),
    ]


_lib: Optional[ctypes.CDLL] = None


def load() -> ctypes.CDLL:
    """Load libjso.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise JsoError("libjso.so not found at %s: build it with "
                       "`python -m paper_2309_15676_amd.build`" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P, I, U32, U64, SZ, D = (ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_uint64,
                             ctypes.c_size_t, ctypes.c_double)
    F = ctypes.c_float
    sig = {
        "jso_create": (I, [ctypes.POINTER(P), I, P]),
        "jso_destroy": (I, [P]),
        "jso_last_error": (ctypes.c_char_p, [P]),
        "jso_set_stream": (I, [P, P]),
        "jso_synchronize": (I, [P]),
        "jso_set_debug": (I, [P, U32]),
        "jso_stream_key": (U64, [U64, U32, U32]),
        "jso_philox": (I, [P, U64, P, SZ, P]),
        "jso_load_scene": (I, [P, P, ctypes.POINTER(I)]),
        "jso_free_scene": (I, [P, I]),
        "jso_scene_info": (I, [P, I, ctypes.POINTER(SZ), ctypes.POINTER(I), ctypes.POINTER(I)]),
        "jso_set_params": (I, [P, I, P, SZ, I]),
        "jso_get_params": (I, [P, I, P, SZ, I]),
        "jso_get_params_prev": (I, [P, I, P, SZ, I]),
        "jso_set_target": (I, [P, I, P, SZ, I]),
        "jso_render": (I, [P, I, P, U64, U32, U32, I, P, P]),
        "jso_render_bwd": (I, [P, I, P, U64, U32, U32, I, P, P, P]),
        "jso_render_bwd_noalloc": (I, [P, I, P, U64, U32, U32, I, P, P, P]),
        "jso_ub_copy": (I, [P, P, P, SZ, I, ctypes.POINTER(D)]),
        "jso_ub_atomics": (I, [P, P, SZ, I, SZ, I, ctypes.POINTER(D)]),
        "jso_ub_launch": (I, [P, P, I, I, I, ctypes.POINTER(D)]),
        "jso_estimate_gradients": (I, [P, I, U64, U32, I, I, P, P, P, P, P]),
        "jso_meta_step": (I, [P, I, P, P, F, F, F]),
        "jso_adam_step": (I, [P, I, P, F, F, F, F]),
        "jso_grad_step": (I, [P, P, I, P, P]),
        "jso_get_state": (I, [P, I, P]),
        "jso_set_state": (I, [P, I, P]),
        "jso_set_timing": (I, [P, I]),
        "jso_get_kernel_time": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(U64), I]),
        "jso_set_work_counting": (I, [P, I]),
        "jso_get_work": (I, [P, ctypes.POINTER(U64), I]),
        "jso_batch_create": (I, [P, ctypes.POINTER(I), I, ctypes.c_void_p,
                                 ctypes.POINTER(ctypes.c_uint32), I, ctypes.POINTER(P)]),
        "jso_batch_step": (I, [P, I]),
        "jso_batch_active": (I, [P, ctypes.POINTER(I)]),
        "jso_batch_destroy": (I, [P]),
        "jso_batch_autotune": (I, [P, I, ctypes.POINTER(I), ctypes.POINTER(D)]),
        "jso_set_launch_config": (I, [P, I]),
        "jso_precondition": (I, [P, I, P, F]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(rc: int, ctx=None, what: str = "") -> None:
    if rc != JSO_OK:
        msg = load().jso_last_error(ctx).decode() if ctx else ""
        raise JsoError("%s failed (%d): %s" % (what or "jso call", rc, msg))


# ---------------------------------------------------------------------------
# same-named wrappers
# ---------------------------------------------------------------------------
def jso_create(device: int = 0, stream: int = 0):
    ctx = ctypes.c_void_p()
    rc = load().jso_create(ctypes.byref(ctx), device, stream or None)
    check(rc, None, "jso_create")
    return ctx


def jso_destroy(ctx) -> int:
    return load().jso_destroy(ctx)


def jso_last_error(ctx) -> str:
    return load().jso_last_error(ctx).decode()


def jso_set_stream(ctx, stream: int) -> int:
    return load().jso_set_stream(ctx, stream or None)


def jso_synchronize(ctx) -> int:
    return load().jso_synchronize(ctx)


def jso_set_debug(ctx, flags: int) -> int:
    return load().jso_set_debug(ctx, flags)


def jso_stream_key(seed: int, iteration: int, tag: int) -> int:
    return int(load().jso_stream_key(seed, iteration, tag))


def jso_philox(ctx, key: int, ctr_ptr: int, n: int, out_ptr: int) -> int:
    return load().jso_philox(ctx, key, ctr_ptr, n, out_ptr)


class SceneDesc:
    """Marshals a SceneSpec-like object into a jso_scene_desc (keeps arrays alive)."""

    def __init__(self, spec):
        self.spheres = np.ascontiguousarray(np.asarray(spec.spheres, np.float32).reshape(-1, 4))
        self.sphere_mat = np.ascontiguousarray(np.asarray(spec.sphere_mat, np.int32).reshape(-1))
        self.fixed = np.ascontiguousarray(np.asarray(spec.fixed_mats, np.float32).reshape(-1, 5))
        self.verts = np.ascontiguousarray(
            np.asarray(getattr(spec, "verts", np.zeros((0, 3))), np.float32).reshape(-1, 3))
        self.tris = np.ascontiguousarray(
            np.asarray(getattr(spec, "tris", np.zeros((0, 3))), np.int32).reshape(-1, 3))
        d = jso_scene_desc()
        d.width, d.height = spec.width, spec.height
        d.cam_eye[:] = spec.cam_eye
        d.cam_target[:] = spec.cam_target
        d.cam_up[:] = spec.cam_up
        d.vfov_deg = spec.vfov_deg
        d.plane_enabled = int(spec.plane_enabled)
        d.plane_mat = int(spec.plane_mat)
        d.plane_extent[:] = spec.plane_extent
        d.n_spheres = self.spheres.shape[0]
        d.spheres = self.spheres.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        d.sphere_mat = self.sphere_mat.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        d.light_enabled = int(spec.light_enabled)
        d.light_center[:] = spec.light_center
        d.light_side = spec.light_side
        d.light_Le[:] = spec.light_Le
        d.env[:] = spec.env
        d.depth, d.rr_start, d.rr_q = spec.depth, spec.rr_start, spec.rr_q
        d.tex_w, d.tex_h, d.ch_mask = spec.tex_w, spec.tex_h, spec.ch_mask
        d.fixed_default[:] = spec.fixed_default
        d.n_fixed = self.fixed.shape[0]
        d.fixed_mats = self.fixed.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        d.n_verts, d.n_tris = self.verts.shape[0], self.tris.shape[0]
        d.verts = self.verts.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
        d.tris = self.tris.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        d.mesh_mat = int(getattr(spec, "mesh_mat", JSO_MAT_PARAM))
        d.param_layout = int(getattr(spec, "param_layout", JSO_LAYOUT_TEXTURE))
        d.vol_res = int(getattr(spec, "vol_res", 0))
        d.vol_views = int(getattr(spec, "vol_views", 1))
        d.vol_box[:] = tuple(getattr(spec, "vol_box", (0.0, 0.0, 0.0, 1.0)))
        d.vol_sigma = float(getattr(spec, "vol_sigma", 0.0))
        self.desc = d


def jso_load_scene(ctx, spec) -> int:
    sd = SceneDesc(spec)
    sid = ctypes.c_int(-1)
    check(load().jso_load_scene(ctx, ctypes.byref(sd.desc), ctypes.byref(sid)), ctx,
          "jso_load_scene")
    return sid.value


def jso_free_scene(ctx, sid: int) -> int:
    return load().jso_free_scene(ctx, sid)


def jso_scene_info(ctx, sid: int):
    n, w, h = ctypes.c_size_t(), ctypes.c_int(), ctypes.c_int()
    check(load().jso_scene_info(ctx, sid, ctypes.byref(n), ctypes.byref(w), ctypes.byref(h)),
          ctx, "jso_scene_info")
    return n.value, w.value, h.value


def _host_f32(a):
    return np.ascontiguousarray(np.asarray(a, np.float32).reshape(-1))


def jso_set_params(ctx, sid: int, p, mem: int = JSO_MEM_HOST, n: Optional[int] = None) -> int:
    if mem == JSO_MEM_HOST:
        a = _host_f32(p)
        return load().jso_set_params(ctx, sid, a.ctypes.data, a.size, mem)
    return load().jso_set_params(ctx, sid, p, n, mem)


def jso_get_params(ctx, sid: int, out=None, mem: int = JSO_MEM_HOST, n: Optional[int] = None):
    if mem == JSO_MEM_HOST:
        P = jso_scene_info(ctx, sid)[0]
        out = np.zeros(P, np.float32) if out is None else out
        check(load().jso_get_params(ctx, sid, out.ctypes.data, out.size, mem), ctx,
              "jso_get_params")
        return out
    return load().jso_get_params(ctx, sid, out, n, mem)


def jso_get_params_prev(ctx, sid: int):
    P = jso_scene_info(ctx, sid)[0]
    out = np.zeros(P, np.float32)
    check(load().jso_get_params_prev(ctx, sid, out.ctypes.data, out.size, JSO_MEM_HOST), ctx,
          "jso_get_params_prev")
    return out


def jso_set_target(ctx, sid: int, img, mem: int = JSO_MEM_HOST, n: Optional[int] = None) -> int:
    if mem == JSO_MEM_HOST:
        a = _host_f32(img)
        return load().jso_set_target(ctx, sid, a.ctypes.data, a.size, mem)
    return load().jso_set_target(ctx, sid, img, n, mem)


def render_opts(flags: int = 0, crop=None, mask_ptr: int = 0, loss: int = JSO_LOSS_L2,
                fd_mode: int = JSO_FD_REPLAY):
    o = jso_render_opts()
    o.flags = flags
    o.crop[:] = tuple(crop) if crop is not None else (0, 0, 0, 0)
    o.pixel_mask = mask_ptr or None
    o.loss = loss
    o.fd_mode = fd_mode
    return o


def jso_render(ctx, sid, params_ptr, seed, iteration, tag, spp, opts, img_ptr) -> int:
    return load().jso_render(ctx, sid, params_ptr, seed, iteration, tag, spp,
                             ctypes.byref(opts) if opts is not None else None, img_ptr)


def jso_render_bwd(ctx, sid, params_ptr, seed, iteration, tag, spp, dimg_ptr, opts,
                   dparams_ptr) -> int:
    return load().jso_render_bwd(ctx, sid, params_ptr, seed, iteration, tag, spp, dimg_ptr,
                                 ctypes.byref(opts) if opts is not None else None, dparams_ptr)


def jso_ub_copy(ctx, dst_ptr, src_ptr, nbytes, reps) -> float:
    """Mean ms per copy of nbytes (device to device) over reps runs."""
    ms = ctypes.c_double(0.0)
    check(load().jso_ub_copy(ctx, dst_ptr, src_ptr, nbytes, reps, ctypes.byref(ms)), ctx,
          "jso_ub_copy")
    return ms.value


def jso_ub_launch(ctx, counter_ptr, n_kernels, use_graph, reps) -> float:
    """Mean ms per chain of n_kernels dependent one-block launches, issued one
    by one or replayed from a captured graph."""
    ms = ctypes.c_double(0.0)
    check(load().jso_ub_launch(ctx, counter_ptr, n_kernels, 1 if use_graph else 0, reps,
                               ctypes.byref(ms)), ctx, "jso_ub_launch")
    return ms.value


def jso_ub_atomics(ctx, buf_ptr, n_buf, pattern, n_ops, reps) -> float:
    """Mean ms per launch of n_ops no-return FP32 atomic adds (pattern JSO_UB_*)."""
    ms = ctypes.c_double(0.0)
    check(load().jso_ub_atomics(ctx, buf_ptr, n_buf, pattern, n_ops, reps, ctypes.byref(ms)),
          ctx, "jso_ub_atomics")
    return ms.value


def jso_render_bwd_noalloc(ctx, sid, params_ptr, seed, iteration, tag, spp, dimg_ptr, opts,
                           dparams_ptr) -> int:
    return load().jso_render_bwd_noalloc(ctx, sid, params_ptr, seed, iteration, tag, spp,
                                         dimg_ptr, ctypes.byref(opts) if opts is not None
                                         else None, dparams_ptr)


def jso_estimate_gradients(ctx, sid, seed, iteration, spp_prop, spp_fd, opts, F_ptr, dF_ptr,
                           img_ptr=0, want_loss=False):
    loss = ctypes.c_double(0.0)
    rc = load().jso_estimate_gradients(ctx, sid, seed, iteration, spp_prop, spp_fd,
                                       ctypes.byref(opts) if opts is not None else None,
                                       F_ptr, dF_ptr or None, img_ptr or None,
                                       ctypes.byref(loss) if want_loss else None)
    return rc, loss.value


def jso_meta_step(ctx, sid, F_ptr, dF_ptr, eta, beta_F, beta_D) -> int:
    return load().jso_meta_step(ctx, sid, F_ptr, dF_ptr, eta, beta_F, beta_D)


def jso_adam_step(ctx, sid, g_ptr, eta, beta1=0.9, beta2=0.999, eps=1e-8) -> int:
    return load().jso_adam_step(ctx, sid, g_ptr, eta, beta1, beta2, eps)


def step_opts(optimizer=JSO_OPT_META, eta=1e-3, beta_F=0.99, beta_D=0.9, spp_prop=2, spp_fd=1,
              adam_beta1=0.9, adam_beta2=0.999, adam_eps=1e-8, adam_spp=64, seed=0, flags=0,
              precond_lambda=0.0, loss=JSO_LOSS_L2, ablate=0, fd_mode=JSO_FD_REPLAY):
    o = jso_step_opts()
    o.optimizer, o.eta, o.beta_F, o.beta_D = optimizer, eta, beta_F, beta_D
    o.spp_prop, o.spp_fd = spp_prop, spp_fd
    o.adam_beta1, o.adam_beta2, o.adam_eps, o.adam_spp = adam_beta1, adam_beta2, adam_eps, adam_spp
    o.seed, o.flags, o.precond_lambda = seed, flags, precond_lambda
    o.loss, o.ablate, o.fd_mode = loss, ablate, fd_mode
    return o


def jso_precondition(ctx, sid: int, g_ptr: int, lam: float) -> int:
    return load().jso_precondition(ctx, sid, g_ptr, lam)


def jso_grad_step(ctx, sids, opts, want_stats=False):
    ids = (ctypes.c_int * len(sids))(*sids)
    stats = (jso_step_stats * len(sids))() if want_stats else None
    rc = load().jso_grad_step(ctx, ids, len(sids), ctypes.byref(opts), stats)
    return rc, (list(stats) if want_stats else None)


def jso_get_state(ctx, sid):
    P = jso_scene_info(ctx, sid)[0]
    bufs = dict(params=np.zeros(P, np.float32), params_prev=np.zeros(P, np.float32),
                mean=np.zeros(P), var=np.zeros(P), alpha_prev=np.zeros(P), m2_F=np.zeros(P),
                m2_D=np.zeros(P), adam_m=np.zeros(P, np.float32), adam_v=np.zeros(P, np.float32))
    st = jso_state()
    for k, v in bufs.items():
        setattr(st, k, v.ctypes.data)
    check(load().jso_get_state(ctx, sid, ctypes.byref(st)), ctx, "jso_get_state")
    bufs.update(iteration=st.iteration, count_F=st.count_F, count_D=st.count_D,
                adam_t=st.adam_t, step_norm2=st.step_norm2)
    return bufs


def jso_set_state(ctx, sid, state: dict) -> int:
    st = jso_state()
    keep = {}
    for k in ("params", "params_prev", "adam_m", "adam_v"):
        keep[k] = np.ascontiguousarray(np.asarray(state[k], np.float32))
        setattr(st, k, keep[k].ctypes.data)
    for k in ("mean", "var", "alpha_prev", "m2_F", "m2_D"):
        keep[k] = np.ascontiguousarray(np.asarray(state[k], np.float64))
        setattr(st, k, keep[k].ctypes.data)
    st.iteration, st.count_F = state["iteration"], state["count_F"]
    st.count_D, st.adam_t, st.step_norm2 = state["count_D"], state["adam_t"], state["step_norm2"]
    return load().jso_set_state(ctx, sid, ctypes.byref(st))


def jso_set_timing(ctx, enable: bool) -> int:
    return load().jso_set_timing(ctx, 1 if enable else 0)


def jso_get_kernel_time(ctx, kernel: int, reset: bool = False):
    """(total ms, launches) of one kernel class since timing was enabled/reset."""
    ms, n = ctypes.c_double(0.0), ctypes.c_uint64(0)
    check(load().jso_get_kernel_time(ctx, kernel, ctypes.byref(ms), ctypes.byref(n),
                                     1 if reset else 0), ctx, "jso_get_kernel_time")
    return ms.value, n.value


def jso_set_work_counting(ctx, enable: bool) -> int:
    return load().jso_set_work_counting(ctx, 1 if enable else 0)


def jso_batch_create(ctx, sids, opts, max_iters=None, use_graph: bool = True):
    """A batch of problems stepped together; returns the batch handle."""
    n = len(sids)
    ids = (ctypes.c_int * n)(*sids)
    mi = None if max_iters is None else (ctypes.c_uint32 * n)(*[int(m) for m in max_iters])
    out = ctypes.c_void_p()
    check(load().jso_batch_create(ctx, ids, n, ctypes.byref(opts), mi, 1 if use_graph else 0,
                                  ctypes.byref(out)), ctx, "jso_batch_create")
    return out


def jso_batch_step(ctx, batch, iterations: int = 1) -> None:
    check(load().jso_batch_step(batch, iterations), ctx, "jso_batch_step")


def jso_batch_active(ctx, batch) -> int:
    out = ctypes.c_int(0)
    check(load().jso_batch_active(batch, ctypes.byref(out)), ctx, "jso_batch_active")
    return out.value


def jso_batch_autotune(ctx, batch, iterations: int = 3):
    """Returns (best launch configuration, [ms per iteration of each])."""
    best = ctypes.c_int(0)
    ms = (ctypes.c_double * JSO_LAUNCH_CONFIGS)()
    check(load().jso_batch_autotune(batch, iterations, ctypes.byref(best), ms), ctx,
          "jso_batch_autotune")
    return best.value, list(ms)


def jso_set_launch_config(ctx, config: int) -> None:
    check(load().jso_set_launch_config(ctx, config), ctx, "jso_set_launch_config")


def jso_batch_destroy(batch) -> int:
    return load().jso_batch_destroy(batch)


def jso_get_work(ctx, reset: bool = False):
    """(replayed paths, their vertices, forward-traced paths, their vertices)
    since counting was enabled/reset."""
    out = (ctypes.c_uint64 * 4)()
    check(load().jso_get_work(ctx, out, 1 if reset else 0), ctx, "jso_get_work")
    return tuple(int(v) for v in out)
