"""Links of the rigid model (soft Cosserat-like couplings, ball joints, no-slip rows) and the
large-scene iteration path against the oracle.

* The large-scene path (one workgroup per scene in one launch, or one launch per phase of
  each iteration) and the per-scene kernel run the same iteration: random assembled problems
  with every interface kind, FP64 to 1e-12 with the same iteration counts, FP32 to 1e-5; the
  two large-path forms bitwise equal; FP64 against the oracle to 1e-9.
* The cable stand-in (640 segments in 160 subsystems plus two bases: one coupled scene of
  ~11k slot rows, so the large-scene path), with every coupling an interface and with the
  within-group couplings folded into the subsystems' dynamics: construction against the
  oracle (FP64 1e-12,
  FP32 2e-7 of the largest entry); a step at the paper's fixed 60 iterations from a state
  three oracle steps into the motion, FP64 to 1e-9 and FP32 to the tolerances of the
  benchmark-path tests (velocity floor 1e-6 m/s; force floor 1e-6 of the largest force).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2302_14344_amd import scenes as S

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _solver():
    from paper_2302_14344_amd.solver import Problem, rigid_state_tensors
    return Problem, rigid_state_tensors


@pytest.mark.parametrize("form", [True, "phases"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_large_path_matches_per_scene_kernel(dtype, form):
    Problem, _ = _solver()
    p = S.random_assembled(131, n_scenes=30, subs_per_scene=(1, 5), ndof=(1, 12), n_if_per_scene=(0, 7),
                           kinds=(0, 1, 2, 3), eq_dim=(1, 6))
    outs = []
    for large in (False, form):
        pr = Problem.from_assembled(p, dtype=dtype)
        pr.set_large_path(large)
        o = pr.solve(pr.tensor(p.A), pr.tensor(p.b), pr.tensor(p.J), pr.tensor(p.e), max_iters=500,
                     tol=1e-10 if dtype == torch.float64 else 1e-6)
        outs.append(({k: _np(v) for k, v in o.items()}, pr.stats()))
        pr.check()
    (a, sa), (b, sb) = outs
    if dtype == torch.float64:
        np.testing.assert_array_equal(sa["iters"], sb["iters"])
        tol = 1e-12
    else:
        assert np.abs(sa["iters"] - sb["iters"]).max() <= 2
        tol = 1e-5
    for k in ("v_hat", "lam", "z", "u"):
        np.testing.assert_allclose(b[k], a[k], atol=tol * max(1.0, np.abs(a[k]).max()), err_msg=k)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_large_path_forms_are_bitwise_equal(dtype):
    """The large-scene path's two forms (one workgroup per scene in one launch, one launch per
    phase per iteration) run the same arithmetic in the same order."""
    Problem, _ = _solver()
    p = S.random_assembled(133, n_scenes=25, subs_per_scene=(1, 6), ndof=(1, 12), n_if_per_scene=(0, 8),
                           kinds=(0, 1, 2, 3), eq_dim=(1, 6), max_members=4)
    outs = []
    for form in (True, "phases"):
        pr = Problem.from_assembled(p, dtype=dtype)
        pr.set_large_path(form)
        o = pr.solve(pr.tensor(p.A), pr.tensor(p.b), pr.tensor(p.J), pr.tensor(p.e), max_iters=300,
                     tol=1e-9 if dtype == torch.float64 else 1e-6)
        outs.append(({k: _np(v) for k, v in o.items()}, pr.stats()))
        pr.check()
    (a, sa), (b, sb) = outs
    np.testing.assert_array_equal(sa["iters"], sb["iters"])
    for k in ("v_hat", "lam", "z", "u"):
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


def test_large_path_fp64_against_oracle():
    Problem, _ = _solver()
    p = S.random_assembled(132, n_scenes=12, subs_per_scene=(1, 5), ndof=(1, 12), n_if_per_scene=(0, 7),
                           kinds=(0, 1, 2, 3), eq_dim=(1, 6))
    ref = O.solve(p, p.A, p.b, p.J, p.e, max_iters=80, tol=0.0)
    pr = Problem.from_assembled(p, dtype=torch.float64)
    pr.set_large_path(True)
    out = pr.solve(pr.tensor(p.A), pr.tensor(p.b), pr.tensor(p.J), pr.tensor(p.e), max_iters=80, tol=0.0)
    st = pr.stats()
    same = st["iters"] == ref.iters
    assert np.all(ref.r_theta[~same] < 1e-14)
    for k, r in (("v_hat", ref.v_hat), ("lam", ref.lam), ("u", ref.u), ("z", ref.z)):
        np.testing.assert_allclose(_np(out[k]), r, atol=1e-9 * max(1.0, np.abs(r).max()), err_msg=k)


def _cable_state(n_pre=3, fold=False):
    sc = S.cable_scene(fold_soft=fold)
    state = (sc.pos, sc.rot, sc.vel, sc.omega)
    z = u = None
    for _ in range(n_pre):
        state, r = O.rigid_step(sc, max_iters=60, tol=0.0, z0=z, u0=u, n_threads=16, state=state)
        z, u = r.z, r.u
    return sc, state, z, u


@pytest.mark.parametrize("fold", [False, True])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_cable_assemble_parity(dtype, fold):
    from tests.test_gpu_parity import model_as
    Problem, rst = _solver()
    sc, state, _, _ = _cable_state(2, fold)
    sck = model_as(sc.with_state(*state), dtype)
    pr = Problem.from_rigid(sc, dtype=dtype)
    assert pr.sizes.max_slot_scene > 512  # one coupled scene beyond the per-scene kernel
    A, b, J, e = (_np(t) for t in pr.rigid_assemble(*rst(sck, dtype=dtype)))
    rA, rb, rJ, re = O.rigid_assemble(sck)
    tol = 1e-12 if dtype == torch.float64 else 2e-7
    for g, r, nm in ((A, rA, "A"), (b, rb, "b"), (J, rJ, "J"), (e, re, "e")):
        np.testing.assert_allclose(g, r, atol=tol * max(1.0, np.abs(r).max()), err_msg=nm)


@pytest.mark.parametrize("fold", [False, True])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_cable_step_fixed_iterations(dtype, fold):
    """One step of the whole cable at 60 iterations (the paper's protocol) from identical
    inputs: the oracle's state and (z, u) three steps into the motion; every coupling an
    interface, or the within-group couplings folded into the subsystems' dynamics."""
    from tests.test_gpu_bench_paths import FP32_L_TIGHT, FP32_V, _iface_force_max
    from tests.test_gpu_parity import model_as, per_scene_errors
    Problem, rst = _solver()
    sc, state, z, u = _cable_state(3, fold)
    rnd = (lambda a: np.asarray(a, np.float32).astype(np.float64)) if dtype == torch.float32 else np.asarray
    sck = model_as(sc.with_state(*state), dtype)
    z, u = rnd(z), rnd(u)
    new_ref, ref = O.rigid_step(sck, max_iters=60, tol=0.0, z0=z, u0=u, n_threads=16)
    pr = Problem.from_rigid(sc, dtype=dtype)
    st = rst(sck, dtype=dtype)
    pr.set_warm(pr.tensor(z), pr.tensor(u))
    vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
    pr.rigid_step(*st, max_iters=60, tol=0.0, warm="prev", v_hat=vh, lam=lam)
    s = pr.stats()
    pr.check()
    assert int(s["iters"][0]) == 60
    topo = O.RigidTopo(sc)
    fmax = _iface_force_max(topo, ref.lam, 1)
    ev, el = per_scene_errors(topo, _np(vh), ref.v_hat, _np(lam), ref.lam, v_floor=1e-6, l_floor=1e-6 * fmax)
    print(f"  cable {dtype} fold {fold}: v {ev.max():.3e} lambda {el.max():.3e} (largest force {fmax[0]:.3e} N)", flush=True)
    if dtype == torch.float64:
        assert ev.max() <= 1e-9 and el.max() <= 1e-9
    else:
        assert ev.max() <= FP32_V and el.max() <= FP32_L_TIGHT
    # the state update of Eq. 2 from the GPU's own v_hat
    new_ref = O.rigid_advance(sck, _np(vh))
    atol = 1e-12 if dtype == torch.float64 else 2e-6
    for g, r in zip(st, new_ref):
        np.testing.assert_allclose(_np(g), r.reshape(-1), atol=atol * max(1.0, np.abs(r).max()))
