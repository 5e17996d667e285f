"""The steps' lambda output as the impulse over the step (option IMPULSE_OUTPUT): Eq. (2) puts
lambda at force level, so the impulse is t lambda.  With the option on, every step form returns
exactly t lambda of the same step without it (one rounding of the product in the problem's
precision, reproduced here in that precision), and the state update is unchanged."""
import numpy as np
import pytest
import torch

from paper_2302_14344_amd import scenes as S

pytestmark = pytest.mark.gpu


def _rigid(dtype, form, impulse):
    from paper_2302_14344_amd.solver import Problem, rigid_state_tensors
    sc = S.legged_scenes(16)
    pr = Problem.from_rigid(sc, dtype=dtype)
    st = rigid_state_tensors(sc, dtype=dtype)
    for _ in range(20):
        pr.rigid_step(*st, max_iters=200)
    pr.set_impulse_output(impulse)
    lam = pr.empty(pr.sizes.n_rows)
    if form == "steps":
        pr.rigid_steps(*st, 2, max_iters=200, lam=lam)
    else:
        for _ in range(2 if form == "graph" else 1):
            pr.rigid_step(*st, max_iters=200, lam=lam, graph=form == "graph")
    pr.check()
    return lam.cpu().numpy(), [t.cpu().numpy() for t in st], sc.dt


@pytest.mark.parametrize("form", ["step", "graph", "steps"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_rigid_impulse(dtype, form):
    lam, st, dt = _rigid(dtype, form, False)
    imp, st1, _ = _rigid(dtype, form, True)
    npt = np.float64 if dtype == torch.float64 else np.float32
    assert np.abs(lam).max() > 0
    np.testing.assert_array_equal(imp, lam * npt(dt))
    for a, b in zip(st, st1):
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("graph", [False, True])
def test_fem_impulse(graph):
    from paper_2302_14344_amd.solver import Problem, fem_state_tensors
    fs = S.fem_scene(seed=S.config_seed(3, 11), blocks=(2, 2, 2), nodes_per_block=4)
    out = []
    for impulse in (False, True):
        pr = Problem.from_fem(fs, dtype=torch.float32)
        pr.set_impulse_output(impulse)
        pos, vel = fem_state_tensors(fs, dtype=torch.float32)
        lam = pr.empty(pr.sizes.n_rows)
        for _ in range(2):
            pr.fem_step(pos, vel, max_iters=50, warm="prev", lam=lam, graph=graph)
        pr.check()
        out.append((lam.cpu().numpy(), pos.cpu().numpy()))
    assert np.abs(out[0][0]).max() > 0
    np.testing.assert_array_equal(out[1][0], out[0][0] * np.float32(fs.dt))
    np.testing.assert_array_equal(out[1][1], out[0][1])
