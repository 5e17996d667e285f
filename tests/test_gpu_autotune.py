"""Schedule autotuner: it times every candidate form on the caller's problem, applies the
fastest, and leaves the caller's state and warm-start values as they were; the tuned
problem still matches the untuned one (same iteration, another kernel form)."""
import numpy as np
import pytest
import torch

from paper_2302_14344_amd import scenes as S

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def test_autotuner_picks_a_form_and_restores_the_state():
    from paper_2302_14344_amd import autotune
    from paper_2302_14344_amd.solver import Problem, rigid_state_tensors
    sc = S.legged_scenes(128, seed=S.config_seed(2, 31))
    pr = Problem.from_rigid(sc, dtype=torch.float32)
    st = rigid_state_tensors(sc)
    pr.rigid_step(*st)  # some warm-start values to keep
    z0, u0 = (t.clone() for t in pr.get_warm())
    before = [t.clone() for t in st]
    cfg, times = autotune.tune_rigid(pr, *st, warmup=2, steps=4, use_cache=False)
    print("autotuner:", cfg, {k: round(v, 4) for k, v in times.items()}, flush=True)
    assert 1 <= len(times) <= len(autotune.candidates()) and all(v > 0 for v in times.values())
    assert min(times.values()) == times[tuple(sorted(cfg.items()))]
    for a, b in zip(before, st):
        np.testing.assert_array_equal(_np(a), _np(b))
    z1, u1 = pr.get_warm()
    np.testing.assert_array_equal(_np(z0), _np(z1))
    np.testing.assert_array_equal(_np(u0), _np(u1))
    # the tuned problem steps like a default one (the forms agree to FP32 rounding)
    ref = Problem.from_rigid(sc, dtype=torch.float32)
    st_ref = [t.clone() for t in before]
    ref.set_warm(z0, u0)
    vh0, vh1 = pr.empty(pr.sizes.n_dof), ref.empty(ref.sizes.n_dof)
    pr.rigid_step(*st, v_hat=vh0)
    ref.rigid_step(*st_ref, v_hat=vh1)
    scale = max(float(np.abs(_np(vh1)).max()), sc.gravity * sc.dt)
    assert np.abs(_np(vh0) - _np(vh1)).max() <= 2e-5 * scale


def test_fem_autotuner_picks_a_form_and_restores_the_state():
    from paper_2302_14344_amd import autotune
    from paper_2302_14344_amd.solver import Problem, fem_state_tensors
    fs = S.fem_scene(seed=S.config_seed(3, 11), blocks=(2, 2, 2), nodes_per_block=4)
    pr = Problem.from_fem(fs, dtype=torch.float32)
    st = fem_state_tensors(fs, dtype=torch.float32)
    pr.fem_step(*st, max_iters=400)
    z0, u0 = (t.clone() for t in pr.get_warm())
    before = [t.clone() for t in st]
    cfg, times = autotune.tune_fem(pr, *st, max_iters=400, warmup=1, steps=2, use_cache=False)
    print("FEM autotuner:", cfg, {k: round(v, 4) for k, v in times.items()}, flush=True)
    assert len(times) == 2 and min(times.values()) == times[tuple(sorted(cfg.items()))]
    for a, b in zip(before, st):
        np.testing.assert_array_equal(_np(a), _np(b))
    z1, u1 = pr.get_warm()
    np.testing.assert_array_equal(_np(z0), _np(z1))
    np.testing.assert_array_equal(_np(u0), _np(u1))
    # both forms compute the same products in the same order
    ref = Problem.from_fem(fs, dtype=torch.float32)
    st_ref = [t.clone() for t in before]
    ref.set_warm(z0, u0)
    pr.fem_step(*st, max_iters=400)
    ref.fem_step(*st_ref, max_iters=400)
    for a, b in zip(st, st_ref):
        np.testing.assert_array_equal(_np(a), _np(b))
    pr.check()
    ref.check()
