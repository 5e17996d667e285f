"""The granular stirring stand-in (216 spheres, sphere contact links, an arm with a folded
controller and a stirrer) and sphere contacts on the GPU against the oracle.

* Construction of the scene: FP64 1e-12, FP32 2e-7 of the largest entry.
* One step at 60 fixed iterations from the oracle's state and (z, u) three steps into the
  stirring: FP64 1e-9; FP32 velocities 1e-5 of max(g t, |v|), forces 2e-5 of the weight.
* The paper's protocol (2 steps at 30 iterations): per-step errors equal to the oracle's
  (1e-6 relative, FP64).
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import protocol as OP
from paper_2302_14344_amd import scenes as S
from tests.test_gpu_bench_paths import FP32_L_WEIGHT, FP32_V
from tests.test_gpu_parity import model_as, scene_weight

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _solver():
    from paper_2302_14344_amd.solver import Problem, rigid_state_tensors
    return Problem, rigid_state_tensors


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_stir_assemble_parity(dtype):
    Problem, rst = _solver()
    sc = S.stir_scene()
    sck = model_as(sc, dtype)
    pr = Problem.from_rigid(sc, dtype=dtype)
    A, b, J, e = (_np(t) for t in pr.rigid_assemble(*rst(sck, dtype=dtype)))
    rA, rb, rJ, re = O.rigid_assemble(sck)
    tol = 1e-12 if dtype == torch.float64 else 2e-7
    for g, r, nm in ((A, rA, "A"), (b, rb, "b"), (J, rJ, "J"), (e, re, "e")):
        np.testing.assert_allclose(g, r, atol=tol * max(1.0, np.abs(r).max()), err_msg=nm)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_stir_step_fixed_iterations(dtype):
    Problem, rst = _solver()
    sc = S.stir_scene()
    st, z, u = (sc.pos, sc.rot, sc.vel, sc.omega), None, None
    for _ in range(3):
        st, r = O.rigid_step(sc, max_iters=60, tol=0.0, z0=z, u0=u, n_threads=16, state=st)
        z, u = r.z, r.u
    rnd = (lambda a: np.asarray(a, np.float32).astype(np.float64)) if dtype == torch.float32 else np.asarray
    sck = model_as(sc.with_state(*st), dtype)
    z, u = rnd(z), rnd(u)
    _, ref = O.rigid_step(sck, max_iters=60, tol=0.0, z0=z, u0=u, n_threads=16)
    pr = Problem.from_rigid(sc, dtype=dtype)
    s = rst(sck, dtype=dtype)
    pr.set_warm(pr.tensor(z), pr.tensor(u))
    vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
    pr.rigid_step(*s, max_iters=60, tol=0.0, warm="prev", v_hat=vh, lam=lam)
    pr.check()
    ev = np.abs(_np(vh) - ref.v_hat).max() / max(sc.gravity * sc.dt, np.abs(ref.v_hat).max())
    el = np.abs(_np(lam) - ref.lam).max() / max(scene_weight(sc)[0], np.abs(ref.lam).max())
    print(f"  stir {dtype}: v {ev:.3e} lambda {el:.3e}", flush=True)
    if dtype == torch.float64:
        assert ev <= 1e-9 and el <= 1e-9
    else:
        assert ev <= FP32_V and el <= FP32_L_WEIGHT


def test_stir_protocol_errors_match_the_oracle():
    from paper_2302_14344_amd import protocol
    Problem, rst = _solver()
    sc = S.stir_scene()
    pr = Problem.from_rigid(sc, dtype=torch.float64)
    st = rst(sc, dtype=torch.float64)
    r = protocol.run(pr, "rigid", st, 30, 2, warmup=1)
    pr.check()
    s, z, u, errs = (sc.pos, sc.rot, sc.vel, sc.omega), None, None, []
    for k in range(3):
        A, b, J, e = O.rigid_assemble(sc, *s)
        res = O.solve(O.RigidTopo(sc), A, b, J, e, max_iters=30, tol=0.0, z0=z, u0=u, n_threads=16)
        if k >= 1:
            errs.append(OP.constraint_error(sc, J, e, res.v_hat, res.lam, res.beta, kinds=(0, 1, 2)))
        s = O.rigid_advance(sc, res.v_hat, *s)
        z, u = res.z, res.u
    print(f"  stir AA {r['aa']:.3f}; errors GPU {r['errors'].ravel()} oracle {np.ravel(errs)}", flush=True)
    np.testing.assert_allclose(r["errors"], np.array(errs), rtol=1e-6)
