"""FP64 CPU oracle for the joint sampling-and-optimisation hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It is
written from the paper (Bálint et al., SIGGRAPH Asia 2023) independently of
the GPU library and shares no code with it.

Contents
  liboracle.so (oracle.cpp):  Philox4x32-10 / SplitMix64, FP64 path tracer,
      proportional gradient sample <F_i> (Eq. 2) with a tape-based adjoint.
  meta.py:  Moment2 variance EMAs (Eq. 9, 13-14), the meta-estimator
      (Eq. 7-8, 15, 17), its stabilised step (Eq. 21) and plain Adam
      (Eq. 18-20), plus the exponential-rate toy of Figure 2.

``gradient_pair`` below assembles <F_i> and the finite-difference sample
<dF_i> = g(pi_i) - g(pi_{i-1}) of Eq. 5 (same random numbers at both
parameter vectors).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

# random-stream tags (which estimator a path belongs to)
TAG_TARGET, TAG_PRIMAL_PROP, TAG_ADJ_PROP = 1, 2, 3
TAG_PRIMAL_FD, TAG_ADJ_FD = 4, 5
TAG_ADAM_PRIMAL, TAG_ADAM_ADJ, TAG_EVAL = 6, 7, 8

NO_NEE, LAMBERT_ONLY, PARAM_INDEP, PIXEL_CENTER = 1, 2, 4, 8


def build(force: bool = False) -> str:
    """Compile liboracle.so with g++ (plain C++17, -O2)."""
    src = os.path.join(_HERE, "oracle.cpp")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < max(
            os.path.getmtime(src), os.path.getmtime(os.path.join(_HERE, "oracle.h"))):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-pthread",
                               src, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Scene(ctypes.Structure):
    _fields_ = [
        ("width", ctypes.c_int), ("height", ctypes.c_int),
        ("cam_eye", ctypes.c_double * 3), ("cam_target", ctypes.c_double * 3),
        ("cam_up", ctypes.c_double * 3), ("vfov_deg", ctypes.c_double),
        ("plane_enabled", ctypes.c_int), ("plane_mat", ctypes.c_int),
        ("plane_extent", ctypes.c_double * 4),
        ("n_spheres", ctypes.c_int), ("spheres", ctypes.POINTER(ctypes.c_double)),
        ("sphere_mat", ctypes.POINTER(ctypes.c_int)),
        ("light_enabled", ctypes.c_int), ("light_center", ctypes.c_double * 3),
        ("light_side", ctypes.c_double), ("light_Le", ctypes.c_double * 3),
        ("env", ctypes.c_double * 3),
        ("depth", ctypes.c_int), ("rr_start", ctypes.c_int), ("rr_q", ctypes.c_double),
        ("tex_w", ctypes.c_int), ("tex_h", ctypes.c_int), ("ch_mask", ctypes.c_int),
        ("fixed_default", ctypes.c_double * 5),
        ("n_fixed", ctypes.c_int), ("fixed_mats", ctypes.POINTER(ctypes.c_double)),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        d, u32, u64, i = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        L.orc_splitmix64.restype = u64
        L.orc_splitmix64.argtypes = [u64]
        L.orc_stream_key.restype = u64
        L.orc_stream_key.argtypes = [u64, u32, u32]
        L.orc_philox4x32_10.argtypes = [d, d, d]
        L.orc_bsdf.argtypes = [d, d, d, d, i, d]
        L.orc_bsdf_many.argtypes = [i, d, d, d, d, i, d]
        L.orc_render.argtypes = [d, d, u64, u32, u32, i, i, d, d, d, i]
        L.orc_render.restype = i
        L.orc_grad.argtypes = [d, d, u64, u32, u32, u32, i, d, i, d, d, d, d, d, d, i]
        L.orc_grad.restype = i
        L.orc_render_bwd.argtypes = [d, d, u64, u32, u32, i, d, i, d, d, d, d, d, i]
        L.orc_render_bwd.restype = i
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class _Marshalled:
    """Keeps the numpy arrays a _Scene points into alive."""

    def __init__(self, spec):
        self.spheres = np.ascontiguousarray(np.asarray(spec.spheres, np.float64).reshape(-1, 4))
        self.sphere_mat = np.ascontiguousarray(np.asarray(spec.sphere_mat, np.int32).reshape(-1))
        self.fixed = np.ascontiguousarray(np.asarray(spec.fixed_mats, np.float64).reshape(-1, 5))
        if len(getattr(spec, "tris", ())) > 0:
            raise NotImplementedError("oracle: triangle meshes are not supported")
        s = _Scene()
        s.width, s.height = spec.width, spec.height
        s.cam_eye[:] = spec.cam_eye
        s.cam_target[:] = spec.cam_target
        s.cam_up[:] = spec.cam_up
        s.vfov_deg = spec.vfov_deg
        s.plane_enabled = int(spec.plane_enabled)
        s.plane_mat = int(spec.plane_mat)
        s.plane_extent[:] = spec.plane_extent
        s.n_spheres = self.spheres.shape[0]
        s.spheres = self.spheres.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s.sphere_mat = self.sphere_mat.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        s.light_enabled = int(spec.light_enabled)
        s.light_center[:] = spec.light_center
        s.light_side = spec.light_side
        s.light_Le[:] = spec.light_Le
        s.env[:] = spec.env
        s.depth, s.rr_start = spec.depth, spec.rr_start
        # the survival probability is defined as a float32 value on both sides
        s.rr_q = float(np.float32(spec.rr_q))
        s.tex_w, s.tex_h, s.ch_mask = spec.tex_w, spec.tex_h, spec.ch_mask
        s.fixed_default[:] = spec.fixed_default
        s.n_fixed = self.fixed.shape[0]
        s.fixed_mats = self.fixed.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self.s = s

    def ptr(self):
        return ctypes.cast(ctypes.pointer(self.s), ctypes.c_void_p)


def _nthreads(n: Optional[int]) -> int:
    return int(n or os.environ.get("ORACLE_THREADS", 0) or os.cpu_count() or 1)


def _crop_arr(crop):
    return None if crop is None else np.asarray(crop, np.int32)


# ----------------------------------------------------------------------------
# random numbers
# ----------------------------------------------------------------------------
def splitmix64(x: int) -> int:
    return int(lib().orc_splitmix64(x))


def stream_key(seed: int, iteration: int, tag: int) -> int:
    return int(lib().orc_stream_key(seed, iteration, tag))


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> Tuple[int, int, int, int]:
    c = np.asarray(ctr, np.uint32)
    k = np.asarray(key, np.uint32)
    o = np.zeros(4, np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(o))
    return tuple(int(v) for v in o)


def bsdf(mat, n, wo, wi, flags: int = 0) -> np.ndarray:
    out = np.zeros(13)
    args = [np.ascontiguousarray(np.asarray(v, np.float64)) for v in (mat, n, wo, wi)]
    lib().orc_bsdf(*[_ptr(a) for a in args], flags, _ptr(out))
    return out


def bsdf_many(mat, n, wo, wi, flags: int = 0) -> np.ndarray:
    """bsdf() for many directions wi (count, 3) -> (count, 13)."""
    wi = np.ascontiguousarray(np.asarray(wi, np.float64).reshape(-1, 3))
    out = np.zeros((wi.shape[0], 13))
    args = [np.ascontiguousarray(np.asarray(v, np.float64)) for v in (mat, n, wo)]
    lib().orc_bsdf_many(wi.shape[0], *[_ptr(a) for a in args], _ptr(wi), flags, _ptr(out))
    return out


# ----------------------------------------------------------------------------
# rendering and gradient samples
# ----------------------------------------------------------------------------
def render(spec, params, seed: int, iteration: int, tag: int, spp: int, flags: int = 0,
           crop=None, nthreads: Optional[int] = None):
    """Primal image (H, W, 3) and per-pixel decision margins (H, W)."""
    m = _Marshalled(spec)
    p = np.ascontiguousarray(np.asarray(params, np.float64))
    img = np.zeros((spec.height, spec.width, 3))
    mg = np.full((spec.height, spec.width), np.inf)
    c = _crop_arr(crop)
    rc = lib().orc_render(m.ptr(), _ptr(p), seed, iteration, tag, spp, flags, _ptr(c),
                          _ptr(img), _ptr(mg), _nthreads(nthreads))
    if rc:
        raise ValueError("orc_render failed")
    return img, mg


def grad(spec, params, target, seed: int, iteration: int, tag_primal: int, tag_adj: int,
         spp: int, flags: int = 0, crop=None, mask=None, nthreads: Optional[int] = None):
    """One gradient sample of the L2 loss: returns (grad, gabs, img, margin)."""
    m = _Marshalled(spec)
    p = np.ascontiguousarray(np.asarray(params, np.float64))
    t = np.ascontiguousarray(np.asarray(target, np.float64).reshape(spec.height, spec.width, 3))
    g = np.zeros(spec.n_params)
    ga = np.zeros(spec.n_params)
    img = np.zeros((spec.height, spec.width, 3))
    mg = np.full((spec.height, spec.width), np.inf)
    mk = None if mask is None else np.ascontiguousarray(np.asarray(mask, np.uint8))
    c = _crop_arr(crop)
    rc = lib().orc_grad(m.ptr(), _ptr(p), seed, iteration, tag_primal, tag_adj, spp, _ptr(t),
                        flags, _ptr(c), _ptr(mk), _ptr(g), _ptr(ga), _ptr(img), _ptr(mg),
                        _nthreads(nthreads))
    if rc:
        raise ValueError("orc_grad failed")
    return g, ga, img, mg


def render_bwd(spec, params, dimg, seed: int, iteration: int, tag: int, spp: int,
               flags: int = 0, crop=None, mask=None, nthreads: Optional[int] = None):
    """Fixed-adjoint backward pass: (grad, gabs, margin)."""
    m = _Marshalled(spec)
    p = np.ascontiguousarray(np.asarray(params, np.float64))
    d = np.ascontiguousarray(np.asarray(dimg, np.float64).reshape(spec.height, spec.width, 3))
    g = np.zeros(spec.n_params)
    ga = np.zeros(spec.n_params)
    mg = np.full((spec.height, spec.width), np.inf)
    mk = None if mask is None else np.ascontiguousarray(np.asarray(mask, np.uint8))
    c = _crop_arr(crop)
    rc = lib().orc_render_bwd(m.ptr(), _ptr(p), seed, iteration, tag, spp, _ptr(d), flags,
                              _ptr(c), _ptr(mk), _ptr(g), _ptr(ga), _ptr(mg), _nthreads(nthreads))
    if rc:
        raise ValueError("orc_render_bwd failed")
    return g, ga, mg


def gradient_pair(spec, params, params_prev, target, seed: int, iteration: int,
                  spp_prop: int = 2, spp_fd: int = 1, flags: int = 0, crop=None, mask=None,
                  nthreads: Optional[int] = None):
    """<F_i> (Eq. 2) and <dF_i> (Eq. 5) for one iteration.

    <F_i>: spp_prop primal + spp_prop adjoint paths at pi_i (own streams).
    <dF_i>: the same spp_fd primal/adjoint streams evaluated at pi_i and at
    pi_{i-1}, differenced; zero at i = 0 or when no previous parameters exist.
    Returns dict with F, dF, F_abs, dF_abs (FP64), I (prop primal) and margin.
    """
    F, Fa, I, mg = grad(spec, params, target, seed, iteration, TAG_PRIMAL_PROP, TAG_ADJ_PROP,
                        spp_prop, flags, crop, mask, nthreads)
    dF = np.zeros_like(F)
    dFa = np.zeros_like(F)
    if iteration >= 1 and params_prev is not None:
        g1, a1, _, m1 = grad(spec, params, target, seed, iteration, TAG_PRIMAL_FD, TAG_ADJ_FD,
                             spp_fd, flags, crop, mask, nthreads)
        g0, a0, _, m0 = grad(spec, params_prev, target, seed, iteration, TAG_PRIMAL_FD,
                             TAG_ADJ_FD, spp_fd, flags, crop, mask, nthreads)
        dF = g1 - g0
        dFa = a1 + a0
        mg = np.minimum(mg, np.minimum(m1, m0))
    return dict(F=F, dF=dF, F_abs=Fa, dF_abs=dFa, I=I, margin=mg)
