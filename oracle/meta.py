"""FP64 oracle of the meta-estimator and the optimisers (numpy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Follows the paper's Sections 4 (variance estimation) and 5 (optimisation)
and the supplement's pseudocode, in the paper's order and notation:

  Var[F_i]      zero-centred second moment of <F_i>, bias-corrected EMA with
                coefficient beta_F                                  (Eq. 9)
  Var[dF_i]_D   same EMA (beta_D) of <dF_i> / ||dpi_i||_2           (Eq. 13)
  Var[dF_i]     = Var[dF_i]_D * ||dpi_i||_2^2                       (Eq. 14)
  alpha_i       = Var[F_i] / (Var[F_i] + Var[F_{i-1}]_M + Var[dF_i])  (Eq. 8)
                clipped by 1 / (2 - alpha_{i-1})                    (Eq. 17)
  <F_i>_M       = alpha_i (<F_{i-1}>_M + <dF_i>) + (1 - alpha_i) <F_i>  (Eq. 7)
  Var[F_i]_M    = alpha_i^2 (Var[F_{i-1}]_M + Var[dF_i])
                  + (1 - alpha_i)^2 Var[F_i]                        (Eq. 15)
  dpi_{i+1}     = -eta <F_i>_M / (sqrt(Var[F_i]_M) + eps)          (Eq. 21)

Readings where the paper is silent or ambiguous:
  * ||dpi_i||_2 is the Euclidean norm over all parameters of one problem of
    the step actually applied (after projection), pi_i - pi_{i-1}.
  * At i = 0, and whenever ||dpi_i|| = 0, there is no finite-difference
    sample: <dF_i> = 0, the Var_D EMA does not step, Var[dF_i] = 0.
  * The EMAs are the bias-corrected form of the supplement's Moment2
    (after its first step the moment equals x^2 exactly).
  * alpha_{-1} = -inf, so alpha_0 = 0 and <F_0>_M = <F_0> (matches Eq. 7's
    initialisation).
  * Parameters are stored as float32; pi_{i+1} = clip(f32(pi_i + dpi), lo, hi).
"""
from __future__ import annotations

import math
from typing import Optional

import numpy as np

ALPHA_EPS = 1e-30   # guards the inverse-variance ratio
STEP_EPS = 1e-8     # epsilon of the stabilised step


class Moment2:
    """Zero-centred second moment, exponential moving average with start-up
    bias correction: after `count` steps the weights of the samples sum to 1.

    centred=True is the ablation of the Experiments section ("Zero-centred
    EMAs"): the same weights also average x, and the variance is the second
    moment minus the squared mean (floored at 0)."""

    def __init__(self, shape, decay: float, centred: bool = False):
        self.decay = float(decay)
        self.count = 0
        self.centred = centred
        self.m2 = np.zeros(shape, np.float64)
        self.m1 = np.zeros(shape, np.float64)

    def step(self, x: np.ndarray) -> None:
        self.count += 1
        w = 1.0 - self.decay
        w_sum = 1.0 - self.decay ** self.count
        x = np.asarray(x, np.float64)
        self.m2 = self.m2 + (w / w_sum) * (x ** 2 - self.m2)
        self.m1 = self.m1 + (w / w_sum) * (x - self.m1)

    @property
    def var(self) -> np.ndarray:
        if not self.centred:
            return self.m2
        return np.maximum(self.m2 - self.m1 ** 2, 0.0)


class Meta:
    """Recurrent meta-estimator <F_i>_M with its variance, and the step of Eq. 21."""

    def __init__(self, shape, eta: float, clip: bool = True):
        self.eta = float(eta)
        self.clip = clip  # False: the "Alpha clipping" ablation of the Experiments section
        self.mean = np.zeros(shape, np.float64)
        self.var = np.zeros(shape, np.float64)
        self.alpha_prev = np.full(shape, -np.inf)
        self.alpha = np.zeros(shape, np.float64)

    def step(self, F, dF, var_F, var_dF) -> np.ndarray:
        # carry the previous meta-estimate to this iteration (Eq. 6 update)
        self.mean = self.mean + dF
        self.var = self.var + var_dF
        # inverse-variance weight (Eq. 8), clipped (Eq. 17)
        alpha = var_F / (var_F + self.var + ALPHA_EPS)
        if self.clip:
            alpha = np.minimum(alpha, 1.0 / (2.0 - self.alpha_prev))
        else:
            # the ablation drops Eq. 17 only; Eq. 7's initialisation
            # <F_0>_M = <F_0> (alpha_0 = 0) stays
            alpha = np.where(np.isneginf(self.alpha_prev), 0.0, alpha)
        self.alpha_prev = alpha
        self.alpha = alpha
        # combine (Eq. 7) and propagate the variance (Eq. 15)
        self.mean = alpha * self.mean + (1.0 - alpha) * F
        self.var = alpha ** 2 * self.var + (1.0 - alpha) ** 2 * var_F
        # stabilised step (Eq. 21)
        return -self.eta * self.mean / (np.sqrt(self.var) + STEP_EPS)


class MetaOptimizer:
    """One problem's optimisation loop state (supplement: optimisation loop).

    Ablations of the Experiments section: centred (non-zero-centred variance
    EMAs), clip=False (no alpha clipping); and, in step(), separate samples
    F_var / dF_var for the variance EMAs ("Sample reuse": uncorrelated
    variance samples instead of the ones the estimate is made of)."""

    def __init__(self, params, lo, hi, eta: float = 1e-3, beta_F: float = 0.99,
                 beta_D: float = 0.9, centred: bool = False, clip: bool = True):
        self.params = np.asarray(params, np.float32).copy()
        self.params_prev = self.params.copy()
        self.lo = np.asarray(lo, np.float32)
        self.hi = np.asarray(hi, np.float32)
        n = self.params.shape
        self.var_F = Moment2(n, beta_F, centred)
        self.var_D = Moment2(n, beta_D, centred)
        self.meta = Meta(n, eta, clip)
        self.iteration = 0
        self.step_norm2 = 0.0   # ||pi_i - pi_{i-1}||^2 of the step that produced pi_i

    def step(self, F, dF, F_var=None, dF_var=None) -> np.ndarray:
        F = np.asarray(F, np.float64)
        n2 = self.step_norm2
        self.var_F.step(F if F_var is None else F_var)
        if self.iteration >= 1 and n2 > 0.0:
            dF = np.asarray(dF, np.float64)
            xd = dF if dF_var is None else np.asarray(dF_var, np.float64)
            self.var_D.step(xd / math.sqrt(n2))
            var_dF = self.var_D.var * n2
        else:
            dF = np.zeros_like(F)
            var_dF = np.zeros_like(F)
        d = self.meta.step(F, dF, self.var_F.var, var_dF)
        new = np.clip((self.params.astype(np.float64) + d).astype(np.float32), self.lo, self.hi)
        diff = new.astype(np.float64) - self.params.astype(np.float64)
        self.step_norm2 = float(np.sum(diff * diff))
        self.params_prev = self.params
        self.params = new
        self.iteration += 1
        return new


class Adam:
    """Adam (Kingma & Ba) with bias-corrected first and second moments (Eq. 18-20)."""

    def __init__(self, params, lo, hi, eta: float, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8):
        self.params = np.asarray(params, np.float32).copy()
        self.lo = np.asarray(lo, np.float32)
        self.hi = np.asarray(hi, np.float32)
        self.eta, self.b1, self.b2, self.eps = float(eta), float(beta1), float(beta2), float(eps)
        self.m = np.zeros(self.params.shape)
        self.v = np.zeros(self.params.shape)
        self.t = 0

    def step(self, g) -> np.ndarray:
        g = np.asarray(g, np.float64)
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        d = -self.eta * mh / (np.sqrt(vh) + self.eps)
        self.params = np.clip((self.params.astype(np.float64) + d).astype(np.float32),
                              self.lo, self.hi)
        return self.params


# ----------------------------------------------------------------------------
# Figure 2 toy: fit the rate of an exponential distribution so that its mean
# is 2.0 (ground-truth rate 0.5), 32 samples per iteration.
# ----------------------------------------------------------------------------
def toy_samples(lam: float, u: np.ndarray) -> np.ndarray:
    """Inverse-CDF samples of Exp(lam): x = -ln(1 - u) / lam (dx/dlam = -x/lam)."""
    return -np.log1p(-u) / lam


def toy_grad(lam: float, u: np.ndarray, target: float = 2.0) -> float:
    """Gradient of the decorrelated L2 loss (xbar_A - t)(xbar_B - t) w.r.t. lam,
    the 32 samples split in two halves A, B so the product is an unbiased
    estimate of (E[x] - t)^2."""
    half = len(u) // 2
    xa, xb = toy_samples(lam, u[:half]), toy_samples(lam, u[half:])
    ma, mb = xa.mean(), xb.mean()
    dma, dmb = -ma / lam, -mb / lam
    return dma * (mb - target) + (ma - target) * dmb


def toy_run(method: str, iters: int, seed: int, lam0: float = 1.0, eta: float = 0.02,
            beta_F: float = 0.99, beta_D: float = 0.9, n: int = 32):
    """Optimise the toy with 'meta' (one proportional + one finite-difference
    sample per iteration, same sample count n each) or 'adam'.  Returns the
    rate trajectory."""
    g = np.random.Generator(np.random.PCG64(seed))
    lo, hi = np.array([1e-2], np.float32), np.array([10.0], np.float32)
    traj = []
    if method == "adam":
        opt = Adam(np.array([lam0], np.float32), lo, hi, eta)
        for _ in range(iters):
            gr = toy_grad(float(opt.params[0]), g.random(n))
            opt.step(np.array([gr]))
            traj.append(float(opt.params[0]))
        return np.array(traj)
    opt = MetaOptimizer(np.array([lam0], np.float32), lo, hi, eta, beta_F, beta_D)
    for i in range(iters):
        lam = float(opt.params[0])
        F = toy_grad(lam, g.random(n))
        u = g.random(n)  # one set of random numbers used at both rates
        dF = toy_grad(lam, u) - toy_grad(float(opt.params_prev[0]), u) if i >= 1 else 0.0
        opt.step(np.array([F]), np.array([dF]))
        traj.append(float(opt.params[0]))
    return np.array(traj)
