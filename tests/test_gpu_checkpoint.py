"""Checkpoint and resume through jso_get_state / jso_set_state: the optimiser
state read back after a restore is bit-identical to the checkpoint, and a
run resumed from a checkpoint at iteration i (in a freshly loaded problem, as
after a restart) continues like the uninterrupted run: the random streams are
keyed by the iteration index, so both trace the same paths, and the states
agree up to the order of the FP32 gradient atomics."""
import sys

import numpy as np
import pytest

from paper_2309_15676_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_15676_amd.problem import Context
    c = Context(0)
    yield c
    c.close()


STATE_KEYS = ("params", "params_prev", "mean", "var", "alpha_prev", "m2_F", "m2_D", "adam_m",
              "adam_v")


def _problem(ctx, spec, T):
    from paper_2309_15676_amd.problem import Problem
    p = Problem(spec, context=ctx)
    p.set_target(T)
    return p


@pytest.mark.parametrize("optimizer", ["meta", "adam"])
def test_resume_from_checkpoint_matches_uninterrupted_run(ctx, optimizer):
    from paper_2309_15676_amd import _lib as L
    _say("checkpoint/resume", optimizer)
    spec = I.scene_textured(48, 40, 16, seed=3, depth=5, rr_start=3)
    gt, init = I.fourier_params(spec, 1), I.uniform_params(spec, 2, 0.2, 0.8)
    T = I.target_image_synthetic(spec, 4)
    opt = L.JSO_OPT_META if optimizer == "meta" else L.JSO_OPT_ADAM
    opts = L.step_opts(optimizer=opt, eta=0.02, adam_spp=3, seed=31)
    a = _problem(ctx, spec, T)
    a.set_params(init)
    for _ in range(4):
        a.grad_step(opts)
    ck = a.get_state()
    assert ck["iteration"] == 4
    for _ in range(3):
        a.grad_step(opts)
    # a fresh problem (as after a restart) resumed from the checkpoint
    b = _problem(ctx, spec, T)
    b.set_state(ck)
    back = b.get_state()
    for k in STATE_KEYS:
        assert np.array_equal(np.asarray(back[k]), np.asarray(ck[k])), k
    for k in ("iteration", "count_F", "count_D", "adam_t", "step_norm2"):
        assert back[k] == ck[k], k
    for _ in range(3):
        b.grad_step(opts)
    sa, sb = a.get_state(), b.get_state()
    assert sa["iteration"] == sb["iteration"] == 7
    for k in ("params", "params_prev", "mean", "var", "m2_F", "m2_D", "adam_m", "adam_v"):
        x, y = np.asarray(sa[k], np.float64), np.asarray(sb[k], np.float64)
        scale = max(np.abs(x).max(), 1e-30)
        assert np.abs(x - y).max() <= 1e-5 * scale, (k, np.abs(x - y).max() / scale)
    assert sa["count_F"] == sb["count_F"] and sa["count_D"] == sb["count_D"]
    assert sa["adam_t"] == sb["adam_t"]
