"""FP64 CPU oracle for the joint sampling-and-optimisation hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path never does.  It is
written from the paper (Bálint et al., SIGGRAPH Asia 2023) independently of
the GPU library and shares no code with it.

Contents
  liboracle.so (oracle.cpp):  Philox4x32-10 / SplitMix64, FP64 path tracer,
      proportional gradient sample <F_i> (Eq. 2) with a tape-based adjoint,
      the shared-path variant of Eq. 5 (paths drawn at other parameters) and
      an emission-absorption voxel volume.
  meta.py:  Moment2 variance EMAs (Eq. 9, 13-14), the meta-estimator
      (Eq. 7-8, 15, 17), its stabilised step (Eq. 21) and plain Adam
      (Eq. 18-20), plus the exponential-rate toy of Figure 2.

``gradient_pair`` below assembles <F_i> and the finite-difference sample
<dF_i> = g(pi_i) - g(pi_{i-1}) of Eq. 5 (same random numbers at both
parameter vectors).
"""
from __future__ import annotations

import ctypes
import math
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

NO_NEE, LAMBERT_ONLY, PARAM_INDEP, PIXEL_CENTER, RELATIVE_LOSS = 1, 2, 4, 8, 16


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
        ("n_verts", ctypes.c_int), ("n_tris", ctypes.c_int),
        ("verts", ctypes.POINTER(ctypes.c_double)), ("tris", ctypes.POINTER(ctypes.c_int)),
        ("mesh_mat", ctypes.c_int), ("param_layout", ctypes.c_int),
        ("vol_res", ctypes.c_int), ("vol_views", ctypes.c_int),
        ("vol_box", ctypes.c_double * 4), ("vol_sigma", ctypes.c_double),
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
        L.orc_set_jitter_offset.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_reset_stats.argtypes = []
        L.orc_get_stats.argtypes = [d]
        L.orc_bsdf.argtypes = [d, d, d, d, i, d]
        L.orc_bsdf_many.argtypes = [i, d, d, d, d, i, d]
        L.orc_render.argtypes = [d, d, u64, u32, u32, i, i, d, d, d, i]
        L.orc_render.restype = i
        L.orc_grad.argtypes = [d, d, u64, u32, u32, u32, i, d, i, d, d, d, d, d, d, d, i]
        L.orc_grad.restype = i
        L.orc_render_bwd.argtypes = [d, d, u64, u32, u32, i, d, i, d, d, d, d, d, d, i]
        L.orc_render_bwd.restype = i
        L.orc_render_sampled.argtypes = [d, d, d, u64, u32, u32, i, i, d, d, d, i]
        L.orc_render_sampled.restype = i
        L.orc_grad_sampled.argtypes = [d, d, d, u64, u32, u32, u32, i, d, i, d, d, d, d, d, d, d,
                                       i]
        L.orc_grad_sampled.restype = i
        L.orc_render_bwd_sampled.argtypes = [d, d, d, u64, u32, u32, i, d, i, d, d, d, d, d, d, i]
        L.orc_render_bwd_sampled.restype = i
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(v):
    """Scene constants are defined as float32 values (the inputs both sides see)."""
    return np.asarray(v, np.float32).astype(np.float64)


class _Marshalled:
    """Keeps the numpy arrays a _Scene points into alive."""

    def __init__(self, spec):
        self.spheres = np.ascontiguousarray(_f32(spec.spheres).reshape(-1, 4))
        self.sphere_mat = np.ascontiguousarray(np.asarray(spec.sphere_mat, np.int32).reshape(-1))
        self.fixed = np.ascontiguousarray(_f32(spec.fixed_mats).reshape(-1, 5))
        self.verts = np.ascontiguousarray(_f32(spec.verts).reshape(-1, 3))
        self.tris = np.ascontiguousarray(np.asarray(spec.tris, np.int32).reshape(-1, 3))
        s = _Scene()
        s.width, s.height = spec.width, spec.height
        s.cam_eye[:] = _f32(spec.cam_eye)
        s.cam_target[:] = _f32(spec.cam_target)
        s.cam_up[:] = _f32(spec.cam_up)
        s.vfov_deg = float(_f32(spec.vfov_deg))
        s.plane_enabled = int(spec.plane_enabled)
        s.plane_mat = int(spec.plane_mat)
        s.plane_extent[:] = _f32(spec.plane_extent)
        s.n_spheres = self.spheres.shape[0]
        s.spheres = self.spheres.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s.sphere_mat = self.sphere_mat.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        s.light_enabled = int(spec.light_enabled)
        s.light_center[:] = _f32(spec.light_center)
        s.light_side = float(_f32(spec.light_side))
        s.light_Le[:] = _f32(spec.light_Le)
        s.env[:] = _f32(spec.env)
        s.depth, s.rr_start = spec.depth, spec.rr_start
        # the survival probability is defined as a float32 value on both sides
        s.rr_q = float(np.float32(spec.rr_q))
        s.tex_w, s.tex_h, s.ch_mask = spec.tex_w, spec.tex_h, spec.ch_mask
        s.fixed_default[:] = _f32(spec.fixed_default)
        s.n_fixed = self.fixed.shape[0]
        s.fixed_mats = self.fixed.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s.n_verts, s.n_tris = self.verts.shape[0], self.tris.shape[0]
        s.verts = self.verts.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        s.tris = self.tris.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        s.mesh_mat = int(spec.mesh_mat)
        s.param_layout = int(getattr(spec, "param_layout", 0))
        s.vol_res = int(getattr(spec, "vol_res", 0))
        s.vol_views = int(getattr(spec, "vol_views", 1))
        s.vol_box[:] = _f32(getattr(spec, "vol_box", (0.0, 0.0, 0.0, 1.0)))
        s.vol_sigma = float(_f32(getattr(spec, "vol_sigma", 0.0)))
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


def reset_stats() -> None:
    lib().orc_reset_stats()


def get_stats() -> dict:
    """Paths traced, their surface vertices and parameterised-material vertices."""
    out = np.zeros(3, np.uint64)
    lib().orc_get_stats(_ptr(out))
    return dict(paths=int(out[0]), vertices=int(out[1]), param_vertices=int(out[2]))


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
def _sample_arr(spec, sample_params):
    if sample_params is None:
        return None
    sp = np.ascontiguousarray(np.asarray(sample_params, np.float64))
    if sp.size != spec.n_params:
        raise ValueError("sample_params has %d entries, the scene %d" % (sp.size, spec.n_params))
    return sp


def render(spec, params, seed: int, iteration: int, tag: int, spp: int, flags: int = 0,
           crop=None, nthreads: Optional[int] = None, sample_params=None):
    """Primal image (H, W, 3) and per-pixel decision margins (H, W).

    sample_params (optional): draw the paths at these parameters and weight
    them by f(x; params) / p(x; sample_params) (every BSDF density taken at
    sample_params): the previous-parameter half of Eq. 5's finite-difference
    sample when params = pi_{i-1} and sample_params = pi_i."""
    m = _Marshalled(spec)
    p = np.ascontiguousarray(np.asarray(params, np.float64))
    sp = _sample_arr(spec, sample_params)
    img = np.zeros((spec.height, spec.width, 3))
    mg = np.full((spec.height, spec.width), np.inf)
    c = _crop_arr(crop)
    rc = lib().orc_render_sampled(m.ptr(), _ptr(p), _ptr(sp), seed, iteration, tag, spp, flags,
                                  _ptr(c), _ptr(img), _ptr(mg), _nthreads(nthreads))
    if rc:
        raise ValueError("orc_render failed")
    return img, mg


def grad(spec, params, target, seed: int, iteration: int, tag_primal: int, tag_adj: int,
         spp: int, flags: int = 0, crop=None, mask=None, nthreads: Optional[int] = None,
         sample_params=None):
    """One gradient sample of the L2 loss: returns (grad, gabs, img, margin, adj_img)
    with img the primal image and adj_img the mean radiance of the adjoint paths.
    sample_params: as in render(), for the primal and the adjoint paths."""
    m = _Marshalled(spec)
    p = np.ascontiguousarray(np.asarray(params, np.float64))
    sp = _sample_arr(spec, sample_params)
    t = np.ascontiguousarray(np.asarray(target, np.float64).reshape(spec.height, spec.width, 3))
    g = np.zeros(spec.n_params)
    ga = np.zeros(spec.n_params)
    img = np.zeros((spec.height, spec.width, 3))
    aimg = np.zeros((spec.height, spec.width, 3))
    mg = np.full((spec.height, spec.width), np.inf)
    mk = None if mask is None else np.ascontiguousarray(np.asarray(mask, np.uint8))
    c = _crop_arr(crop)
    rc = lib().orc_grad_sampled(m.ptr(), _ptr(p), _ptr(sp), seed, iteration, tag_primal,
                                tag_adj, spp, _ptr(t), flags, _ptr(c), _ptr(mk), _ptr(g),
                                _ptr(ga), _ptr(img), _ptr(mg), _ptr(aimg), _nthreads(nthreads))
    if rc:
        raise ValueError("orc_grad failed")
    return g, ga, img, mg, aimg


def render_bwd(spec, params, dimg, seed: int, iteration: int, tag: int, spp: int,
               flags: int = 0, crop=None, mask=None, nthreads: Optional[int] = None,
               sample_params=None):
    """Fixed-adjoint backward pass: (grad, gabs, margin, adj_img).
    sample_params: as in render()."""
    m = _Marshalled(spec)
    p = np.ascontiguousarray(np.asarray(params, np.float64))
    sp = _sample_arr(spec, sample_params)
    d = np.ascontiguousarray(np.asarray(dimg, np.float64).reshape(spec.height, spec.width, 3))
    g = np.zeros(spec.n_params)
    ga = np.zeros(spec.n_params)
    mg = np.full((spec.height, spec.width), np.inf)
    aimg = np.zeros((spec.height, spec.width, 3))
    mk = None if mask is None else np.ascontiguousarray(np.asarray(mask, np.uint8))
    c = _crop_arr(crop)
    rc = lib().orc_render_bwd_sampled(m.ptr(), _ptr(p), _ptr(sp), seed, iteration, tag, spp,
                                      _ptr(d), flags, _ptr(c), _ptr(mk), _ptr(g), _ptr(ga),
                                      _ptr(mg), _ptr(aimg), _nthreads(nthreads))
    if rc:
        raise ValueError("orc_render_bwd failed")
    return g, ga, mg, aimg


def rounding_sensitivity(spec, fn, radians: float = 1e-6):
    """Run fn() and, with the same random numbers, again with every primary ray
    turned by `radians` in +-x and +-y; return (fn(), max |deviation|).

    1e-6 rad is about 16 single-precision epsilons: the deviation measures how
    strongly each pixel's (or parameter's) paths amplify rounding of that size
    -- near-specular GGX peaks and grazing directions amplify it most -- and
    serves as the per-element floor of an FP32 vs FP64 comparison.
    fn returns an array, a tuple of arrays (None entries are skipped) or a
    dict of arrays; the deviation has the same structure."""
    px = radians / (2.0 * math.tan(math.radians(float(np.float32(spec.vfov_deg))) / 2) /
                    spec.height)
    base = fn()

    def dev(a, b):
        if isinstance(a, dict):
            return {k: dev(a[k], b[k]) for k in a if isinstance(a[k], np.ndarray)}
        if isinstance(a, tuple):
            return tuple(dev(x, y) for x, y in zip(a, b))
        if a is None:
            return None
        a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
        with np.errstate(invalid="ignore"):
            d = np.abs(a - b)
        return np.where(np.isfinite(d), d, 0.0)  # (unbounded margins compare as 0)

    def worse(w, d):
        if isinstance(d, dict):
            return {k: worse(w[k], d[k]) for k in d}
        if isinstance(d, tuple):
            return tuple(worse(x, y) for x, y in zip(w, d))
        return None if d is None else np.maximum(w, d)

    worst = None
    try:
        for dx, dy in ((px, 0.0), (-px, 0.0), (0.0, px), (0.0, -px)):
            lib().orc_set_jitter_offset(dx, dy)
            d = dev(fn(), base)
            worst = d if worst is None else worse(worst, d)
    finally:
        lib().orc_set_jitter_offset(0.0, 0.0)
    return base, worst


def gradient_pair(spec, params, params_prev, target, seed: int, iteration: int,
                  spp_prop: int = 2, spp_fd: int = 1, flags: int = 0, crop=None, mask=None,
                  nthreads: Optional[int] = None, fd_shared: bool = False):
    """<F_i> (Eq. 2) and <dF_i> (Eq. 5) for one iteration.

    <F_i>: spp_prop primal + spp_prop adjoint paths at pi_i (own streams).
    <dF_i>: the same spp_fd primal/adjoint streams evaluated at pi_i and at
    pi_{i-1}, differenced; zero at i = 0 or when no previous parameters exist.
    By default each half draws its paths at its own parameters from the same
    random numbers (primary-sample-space replay); fd_shared: the pi_{i-1} half
    takes the paths drawn at pi_i, weighted by f(x; pi_{i-1}) / p(x; pi_i) --
    Eq. 5 as written: one path, the integrand at both parameter vectors.
    Returns dict with F, dF, F_abs, dF_abs (FP64), I (prop primal image), margin,
    and the per-pixel radiance of every stream: A (prop adjoint paths),
    I_fd1 / I_fd0 (FD primal at pi_i / pi_{i-1}), A_fd1 / A_fd0 (FD adjoint).
    """
    F, Fa, I, mg, A = grad(spec, params, target, seed, iteration, TAG_PRIMAL_PROP,
                           TAG_ADJ_PROP, spp_prop, flags, crop, mask, nthreads)
    out = dict(F=F, F_abs=Fa, I=I, A=A)
    dF = np.zeros_like(F)
    dFa = np.zeros_like(F)
    if iteration >= 1 and params_prev is not None:
        g1, a1, i1, m1, A1 = grad(spec, params, target, seed, iteration, TAG_PRIMAL_FD,
                                  TAG_ADJ_FD, spp_fd, flags, crop, mask, nthreads)
        g0, a0, i0, m0, A0 = grad(spec, params_prev, target, seed, iteration, TAG_PRIMAL_FD,
                                  TAG_ADJ_FD, spp_fd, flags, crop, mask, nthreads,
                                  sample_params=params if fd_shared else None)
        dF = g1 - g0
        dFa = a1 + a0
        mg = np.minimum(mg, np.minimum(m1, m0))
        out.update(I_fd1=i1, I_fd0=i0, A_fd1=A1, A_fd0=A0)
    out.update(dF=dF, dF_abs=dFa, margin=mg)
    return out


STREAM_IMAGES = ("I", "A", "I_fd1", "I_fd0", "A_fd1", "A_fd0")


def ill_conditioned(result: dict, floor: dict, rel: float = 1e-2) -> np.ndarray:
    """Pixels (H, W) where some stream's radiance moves by more than `rel` of
    its scale when the primary rays turn by the rounding_sensitivity angle:
    chaotic paths (curved geometry + textured roughness + specular sampling
    amplify single-precision rounding into a different path), for which an
    FP32 vs FP64 comparison of individual samples is not meaningful."""
    bad = None
    for k in STREAM_IMAGES:
        if k not in result:
            continue
        img = result[k]
        traced = np.abs(img).max(-1) > 0  # pixels outside a crop / mask stay zero
        mean = np.abs(img[traced]).mean() if traced.any() else 0.0
        scale = np.maximum(np.abs(img), 1e-3 * mean + 1e-300)
        b = (floor[k] / scale).max(-1) > rel
        bad = b if bad is None else (bad | b)
    return bad
