"""FP64 oracle of the meta-estimator and the optimisers (numpy).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Written from the equations of Sections 3-5 of the paper, one function per
equation, in the order the method applies them within an iteration i:

  Var[F_i]         Eq. 9: a zero-centred exponential moving average of
                   <F_i>^2 with coefficient beta_F
  Var[dF_i]_D      Eq. 13: the same kind of average, coefficient beta_D, of
                   (<dF_i> / ||dpi_i||_2)^2
  Var[dF_i]        Eq. 14: Var[dF_i]_D ||dpi_i||_2^2
  carry            Eq. 6: <F_{i-1}>_M + <dF_i> is an unbiased estimate of
                   F_i; for independent samples its variance is
                   Var[F_{i-1}]_M + Var[dF_i]
  alpha_i          Eq. 8 (inverse-variance weight), bounded by Eq. 17
  <F_i>_M          Eq. 7, with Var[F_i]_M from Eq. 15
  dpi_{i+1}        Eq. 21, the stabilised step

Readings where the paper is silent or ambiguous:
  * Start-up bias of the averages: Eq. 9 and Eq. 13 start from zero, so
    after n samples their weights sum to 1 - beta^n.  The average used is the
    raw one divided by that total weight (the correction Eq. 19 applies to
    Adam's second moment); after one sample it equals x^2 exactly.  The
    average of <dF> counts its own samples (it starts at i = 1).
  * ||dpi_i||_2 is the Euclidean norm, over all parameters of one problem,
    of the step actually applied (after projection), pi_i - pi_{i-1}.
  * At i = 0, and whenever ||dpi_i|| = 0, there is no finite-difference
    sample: <dF_i> = 0, the Var_D average takes no sample, Var[dF_i] = 0.
  * alpha_0 = 0 (Eq. 7 initialises <F_0>_M = <F_0>); Eq. 17 bounds alpha_i
    from i = 1 on.
  * Eq. 8 is 0/0 for a parameter whose three variances are all zero (no
    path has touched it yet); alpha_i = 0 there.
  * epsilon of Eq. 21 is 1e-8, Adam's published default (Kingma & Ba).
  * Parameters are stored as float32; pi_{i+1} = clip(f32(pi_i + dpi), lo, hi).
"""
from __future__ import annotations

import math

import numpy as np

STEP_EPS = 1e-8  # epsilon of Eq. 21


class DecayedMoment:
    """Zero-centred exponential moving average of x^2 (Eq. 9, Eq. 13),
    start-up corrected by its total weight 1 - beta^n.

    centred=True is the "Zero-centred EMAs" ablation of the Experiments
    section: the same weights also average x, and the variance estimate is
    the second moment minus the squared mean, floored at 0."""

    def __init__(self, shape, beta: float, centred: bool = False):
        self.beta = float(beta)
        self.centred = centred
        self.n = 0                                   # samples taken so far
        self.raw_sq = np.zeros(shape, np.float64)    # Eq. 9 as written, from 0
        self.raw_x = np.zeros(shape, np.float64)     # centred ablation only

    def push(self, x) -> None:
        x = np.asarray(x, np.float64)
        b = self.beta
        self.raw_sq = b * self.raw_sq + (1.0 - b) * (x * x)
        if self.centred:
            self.raw_x = b * self.raw_x + (1.0 - b) * x
        self.n += 1

    def _weight(self) -> float:
        return 1.0 - self.beta ** self.n

    @property
    def second_moment(self) -> np.ndarray:
        if self.n == 0:
            return np.zeros_like(self.raw_sq)
        return self.raw_sq / self._weight()

    @property
    def estimate(self) -> np.ndarray:
        """The variance approximation the method uses."""
        m2 = self.second_moment
        if not self.centred:
            return m2
        m1 = self.raw_x / self._weight() if self.n else np.zeros_like(m2)
        return np.maximum(m2 - m1 * m1, 0.0)


def inverse_variance_weight(var_F, var_carried) -> np.ndarray:
    """Eq. 8: alpha = Var[F_i] / (Var[F_i] + Var[F_{i-1}]_M + Var[dF_i]),
    where var_carried = Var[F_{i-1}]_M + Var[dF_i]; 0 where all vanish."""
    var_F = np.asarray(var_F, np.float64)
    total = var_F + var_carried
    out = np.zeros_like(total)
    np.divide(var_F, total, out=out, where=total > 0.0)
    return out


def clip_by_previous(alpha, alpha_before) -> np.ndarray:
    """Eq. 17: alpha_i <= 1 / (2 - alpha_{i-1})."""
    return np.minimum(alpha, 1.0 / (2.0 - alpha_before))


class MetaEstimate:
    """The recurrent meta-estimate <F_i>_M (Eq. 7) and its variance
    Var[F_i]_M (Eq. 15), one value per parameter.

    clip=False is the "Alpha clipping" ablation of the Experiments section:
    Eq. 17 is dropped, Eq. 7's initialisation alpha_0 = 0 stays."""

    def __init__(self, shape, clip: bool = True):
        self.clip = clip
        self.i = 0                                        # estimates formed so far
        self.F_M = np.zeros(shape, np.float64)            # <F_{i}>_M
        self.V_M = np.zeros(shape, np.float64)            # Var[F_{i}]_M
        self.alpha_last = np.full(shape, -np.inf)         # alpha of the last update

    def update(self, F, dF, var_F, var_dF) -> None:
        F = np.asarray(F, np.float64)
        var_F = np.asarray(var_F, np.float64)
        # Eq. 6: the previous estimate moved to pi_i by the finite difference
        carried = self.F_M + dF
        var_carried = self.V_M + var_dF
        if self.i == 0:
            alpha = np.zeros_like(F)                      # <F_0>_M = <F_0>
        else:
            alpha = inverse_variance_weight(var_F, var_carried)
            if self.clip:
                alpha = clip_by_previous(alpha, self.alpha_last)
        self.F_M = alpha * carried + (1.0 - alpha) * F                       # Eq. 7
        self.V_M = alpha ** 2 * var_carried + (1.0 - alpha) ** 2 * var_F     # Eq. 15
        self.alpha_last = alpha
        self.i += 1


def stabilised_step(eta: float, F_M, V_M) -> np.ndarray:
    """Eq. 21: dpi_{i+1} = -eta <F_i>_M / (sqrt(Var[F_i]_M) + eps)."""
    return -eta * F_M / (np.sqrt(V_M) + STEP_EPS)


def project(params_f32, step, lo, hi) -> np.ndarray:
    """Apply a step to float32 parameters and clamp them to their domain."""
    moved = (np.asarray(params_f32, np.float32).astype(np.float64) + step).astype(np.float32)
    return np.clip(moved, lo, hi)


class MetaOptimizer:
    """One problem's optimisation loop (Sections 4-5): the two variance
    averages, the meta-estimate and the stabilised, projected step.

    Ablations of the Experiments section: centred (non-zero-centred variance
    averages), clip=False (no alpha clipping); and, in step(), separate
    samples F_var / dF_var that feed only the variance averages ("Sample
    reuse": uncorrelated variance samples)."""

    def __init__(self, params, lo, hi, eta: float = 1e-3, beta_F: float = 0.99,
                 beta_D: float = 0.9, centred: bool = False, clip: bool = True):
        self.params = np.asarray(params, np.float32).copy()
        self.params_prev = self.params.copy()
        self.lo = np.asarray(lo, np.float32)
        self.hi = np.asarray(hi, np.float32)
        self.eta = float(eta)
        shape = self.params.shape
        self.var_F = DecayedMoment(shape, beta_F, centred)   # Eq. 9
        self.var_D = DecayedMoment(shape, beta_D, centred)   # Eq. 13
        self.meta = MetaEstimate(shape, clip)
        self.iteration = 0
        self.step_norm2 = 0.0   # ||pi_i - pi_{i-1}||^2 of the step that produced pi_i

    def step(self, F, dF, F_var=None, dF_var=None) -> np.ndarray:
        F = np.asarray(F, np.float64)
        self.var_F.push(F if F_var is None else F_var)
        sq = self.step_norm2
        have_fd = self.iteration >= 1 and sq > 0.0
        if have_fd:
            dF = np.asarray(dF, np.float64)
            norm = math.sqrt(sq)
            self.var_D.push((dF if dF_var is None else np.asarray(dF_var, np.float64)) / norm)
            var_dF = self.var_D.estimate * sq                                # Eq. 14
        else:
            dF = np.zeros_like(F)
            var_dF = np.zeros_like(F)
        self.meta.update(F, dF, self.var_F.estimate, var_dF)
        new = project(self.params, stabilised_step(self.eta, self.meta.F_M, self.meta.V_M),
                      self.lo, self.hi)
        applied = new.astype(np.float64) - self.params.astype(np.float64)
        self.step_norm2 = float(np.dot(applied.ravel(), applied.ravel()))
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
        self.params = project(self.params, -self.eta * mh / (np.sqrt(vh) + self.eps),
                              self.lo, self.hi)
        return self.params


# ----------------------------------------------------------------------------
# Figure 2 toy: fit the rate of an exponential distribution so that its mean
# is 2.0 (ground-truth rate 0.5), 32 samples per iteration.
# ----------------------------------------------------------------------------
def toy_samples(lam: float, u: np.ndarray) -> np.ndarray:
    """Inverse-CDF samples of Exp(lam): x = -ln(1 - u) / lam (dx/dlam = -x/lam)."""
    return -np.log1p(-u) / lam


def toy_grad(lam, u: np.ndarray, target: float = 2.0):
    """Gradient of the decorrelated L2 loss (xbar_A - t)(xbar_B - t) w.r.t. lam,
    the samples along the last axis of u split in two halves A, B so the
    product is an unbiased estimate of (E[x] - t)^2.  lam may be an array of
    independent runs (one row of u each)."""
    half = u.shape[-1] // 2
    lam = np.asarray(lam, np.float64)
    lam_c = lam[..., None] if lam.ndim else lam
    ma = toy_samples(lam_c, u[..., :half]).mean(axis=-1)
    mb = toy_samples(lam_c, u[..., half:]).mean(axis=-1)
    dma, dmb = -ma / lam, -mb / lam
    return dma * (mb - target) + (ma - target) * dmb


def toy_true_grad(lam: float, target: float = 2.0) -> float:
    """d/dlam of (E[x] - t)^2 with E[x] = 1 / lam."""
    return 2.0 * (1.0 / lam - target) * (-1.0 / (lam * lam))


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


def toy_track(schedule, runs: int, seed: int, beta_F: float = 0.99, beta_D: float = 0.9,
              beta1: float = 0.9, beta2: float = 0.999, n: int = 32):
    """Estimate the toy's gradient along a fixed rate schedule in `runs`
    independent runs (no optimiser feedback: the protocol of the
    Experiments' "Variance reduction without lag" and "Approximation
    accuracy" paragraphs).  Returns arrays of shape (iterations, runs): the
    meta-estimate <F_i>_M, its predicted variance Var[F_i]_M, and Adam's
    bias-corrected first and second moments of the proportional samples."""
    g = np.random.Generator(np.random.PCG64(seed))
    var_F = DecayedMoment((runs,), beta_F)
    var_D = DecayedMoment((runs,), beta_D)
    est = MetaEstimate((runs,))
    m = np.zeros(runs)
    v = np.zeros(runs)
    T = len(schedule)
    F_M, V_M, m_hat, v_hat = (np.zeros((T, runs)) for _ in range(4))
    for i, lam in enumerate(schedule):
        F = toy_grad(np.full(runs, lam), g.random((runs, n)))
        u = g.random((runs, n))  # one set of random numbers at both rates
        var_F.push(F)
        dF = np.zeros(runs)
        var_dF = np.zeros(runs)
        if i >= 1 and lam != schedule[i - 1]:
            norm = abs(lam - schedule[i - 1])
            dF = toy_grad(np.full(runs, lam), u) - toy_grad(np.full(runs, schedule[i - 1]), u)
            var_D.push(dF / norm)
            var_dF = var_D.estimate * norm * norm
        est.update(F, dF, var_F.estimate, var_dF)
        m = beta1 * m + (1 - beta1) * F
        v = beta2 * v + (1 - beta2) * F * F
        F_M[i], V_M[i] = est.F_M, est.V_M
        m_hat[i] = m / (1 - beta1 ** (i + 1))
        v_hat[i] = v / (1 - beta2 ** (i + 1))
    return F_M, V_M, m_hat, v_hat
