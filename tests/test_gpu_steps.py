"""The multi-step launch (subadmm_rigid_steps: each scene carried through several whole
steps by one workgroup) against repeated single steps and against the oracle.

* n steps in one launch equal n calls of the single step with the same warm mode (FP64:
  1e-12 relative; the factorisation's sums run over another number of threads, so the last
  bits of beta may differ), with the same iteration counts, on the small chain and on legged
  batches, cold and from the previous step;
* the full 1024-scene legged batch (whose 54 largest factorisations exceed the kernel's LDS
  budget and run in global scratch) after 100 steps of the multi-step launch: one more step
  against the oracle from identical inputs (FP64 to 1e-9 under the tight floors; FP32 to the
  tolerances of the benchmark-path tests), FP32 also with the long rows split within the
  workgroup as the benchmark's multi-step schedule runs.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2302_14344_amd import scenes as S
from tests.test_gpu_bench_paths import FP32_L_TIGHT, FP32_L_WEIGHT, FP32_V, _iface_force_max, _rigid_state
from tests.test_gpu_parity import model_as, per_scene_errors, scene_weight

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


CASES = {
    "chain-cold": (lambda: S.chain_scene(S.config_seed(1)), 1e3, "cold", 200, 1e-8, 6),
    "chain-prev": (lambda: S.chain_scene(S.config_seed(1)), 1e3, "prev", 200, 1e-8, 12),
    "legged-prev": (lambda: S.legged_scenes(64, seed=S.config_seed(2, 31)), 0.0, "prev", 1000, 1e-7, 10),
    "legged-cold": (lambda: S.legged_scenes(64, seed=S.config_seed(2, 32)), 0.0, "cold", 1000, 1e-7, 4),
}


@pytest.mark.parametrize("split", [False, "within"])
@pytest.mark.parametrize("case", list(CASES))
def test_steps_equal_repeated_single_steps(case, split):
    """Both with one lane per slot row and with long rows split within the workgroup (the
    same lane map in both launches)."""
    from paper_2302_14344_amd.solver import Problem, rigid_state_tensors
    mk, rho, warm, L, tol, n = CASES[case]
    print(f"case {case} split {split}", flush=True)
    sc = mk()
    out = []
    for multi in (False, True):
        pr = Problem.from_rigid(sc, rho=rho, dtype=torch.float64)
        pr.set_split_rows(split)
        st = rigid_state_tensors(sc, dtype=torch.float64)
        vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
        if multi:
            pr.rigid_steps(*st, n, max_iters=L, tol=tol, warm=warm, v_hat=vh, lam=lam)
        else:
            for _ in range(n):
                pr.rigid_step(*st, max_iters=L, tol=tol, warm=warm, v_hat=vh, lam=lam)
        s = pr.stats()
        z, u = pr.get_warm()
        out.append(([_np(t) for t in (*st, vh, lam, z, u)], s))
        pr.check()
    (a, sa), (b, sb) = out
    print(f"  iterations (single, multi) total {sa['iters_total'].sum()} {sb['iters_total'].sum()}; last step "
          f"max diff {np.abs(sa['iters'] - sb['iters']).max()}", flush=True)
    assert np.abs(sa["iters_total"] - sb["iters_total"]).max() <= n
    np.testing.assert_array_equal(sa["converged"], sb["converged"])
    for x, y, nm in zip(a, b, ("pos", "rot", "vel", "omega", "v_hat", "lambda", "z", "u")):
        np.testing.assert_allclose(y, x, atol=1e-12 * max(1.0, np.abs(x).max()), err_msg=nm)


@pytest.mark.parametrize("dtype,split", [(torch.float64, False), (torch.float32, False), (torch.float32, "within")])
def test_steps_full_batch_against_oracle(dtype, split):
    """The full batch; FP32 also with long rows split within the workgroup, the benchmark's
    multi-step schedule."""
    from paper_2302_14344_amd.solver import Problem, rigid_state_tensors
    print(f"case {dtype} split {split}", flush=True)
    sc = S.legged_scenes(1024)
    topo = O.RigidTopo(sc)
    pr = Problem.from_rigid(sc, dtype=dtype)
    pr.set_split_rows(split)
    st = rigid_state_tensors(sc, dtype=dtype)
    vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
    L, tol = 1000, 1e-6
    pr.rigid_steps(*st, 100, max_iters=L, tol=tol, warm="prev", v_hat=vh, lam=lam)
    s100 = pr.stats()
    print(f"  100 steps: {s100['iters_total'].sum()} iterations, unconverged scene-steps "
          f"{s100['unconverged_total'].sum()}", flush=True)
    state = _rigid_state(st, sc.n_bodies)
    zp, up = (_np(t) for t in pr.get_warm())
    pr.rigid_steps(*st, 1, max_iters=L, tol=tol, warm="prev", v_hat=vh, lam=lam)
    s = pr.stats()
    pr.check()
    sck = model_as(sc.with_state(*state), dtype)
    A, b, J, e = O.rigid_assemble(sck)
    rule = O.solve(topo, A, b, J, e, max_iters=L, tol=tol, z0=zp, u0=up, n_threads=16)
    at = O.solve(topo, A, b, J, e, max_iters=np.maximum(s["iters"], 1), tol=0.0, z0=zp, u0=up, n_threads=16)
    mism = int(np.sum(s["iters"] != rule.iters))
    gv, gl = _np(vh), _np(lam)
    w = scene_weight(sc)
    ev_p, el_p = per_scene_errors(topo, gv, at.v_hat, gl, at.lam, v_floor=sc.gravity * sc.dt, l_floor=w)
    fmax = _iface_force_max(topo, at.lam, sc.n_scenes)
    ev_t, el_t = per_scene_errors(topo, gv, at.v_hat, gl, at.lam, v_floor=1e-6, l_floor=1e-6 * fmax)
    loaded = fmax > 0.1 * w
    print(f"  step 101: iteration counts differ from the oracle's under the same rule in {mism} scenes; physical "
          f"floors v {ev_p.max():.3e} lambda {el_p.max():.3e}; tight floors v {ev_t.max():.3e} lambda (loaded "
          f"{loaded.sum()}) {el_t[loaded].max():.3e}", flush=True)
    if dtype == torch.float64:
        assert mism == 0
        assert ev_t.max() <= 1e-9 and el_t.max() <= 1e-9
    else:
        assert np.abs(s["converged"].mean() - rule.converged.mean()) <= 0.01
        assert ev_p.max() <= FP32_V and ev_t.max() <= FP32_V
        assert el_p.max() <= FP32_L_WEIGHT and el_t[loaded].max() <= FP32_L_TIGHT
    new = O.rigid_advance(sck, gv)
    atol = 1e-12 if dtype == torch.float64 else 2e-6
    for g, r in zip(st, new):
        np.testing.assert_allclose(_np(g), r.reshape(-1), atol=atol * max(1.0, np.abs(r).max()))
