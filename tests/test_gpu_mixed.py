"""The large mixed rigid workload (boxes stacked in columns around position-controlled arms:
two-member box-box contact links, ground contacts, arms of revolute joints held by soft
couplings folded into the arm subsystem, velocity rows fixing the arm bases) against the
FP64 oracle.

* Construction of the full batch (64 scenes: 4096 boxes, 64 seven-link arms): FP64 1e-12,
  FP32 2e-7 of the largest entry.
* One step at 100 fixed iterations from identical inputs (the oracle's state and (z, u)
  30 steps into the motion, the boxes settled on each other), four scenes: FP64 1e-9 of the
  scene's largest velocity and force (floors g t and the scene's weight); FP32 with the
  benchmark-path tolerances under the same floors (velocities 1e-5, forces 2e-5).
* The full batch in FP32, one step at the benchmark's rule (tol 1e-6) replayed from a HIP
  graph: the oracle at the GPU's iteration count from the GPU's inputs; forces to 2e-5 of
  the scene's weight, velocities to 2e-5 of g t.  The velocity bound is twice the legged
  batch's: stacked boxes from 0.06 to 54 kg give penalties (Eq. 23) 400 times apart across
  a contact, and up to ~800 FP32 iterations accumulate the z-update's rounding (measured:
  1.3e-5 in the worst of 64 scenes, below 5e-6 in most; the same step in FP64 meets 1e-9).
* A separating contact whose tangential trial value squares below the normal FP32 range
  (regression for the FP32 disc projection).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2302_14344_amd import scenes as S
from tests.test_gpu_bench_paths import FP32_L_WEIGHT, FP32_V
from tests.test_gpu_parity import model_as, per_scene_errors, scene_weight

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _solver():
    from paper_2302_14344_amd.solver import Problem, rigid_state_tensors
    return Problem, rigid_state_tensors


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_mixed_assemble_parity(dtype):
    Problem, rst = _solver()
    sc = S.mixed_scenes()
    print(f"mixed {dtype}: {sc.n_bodies} bodies, {sc.n_sub} subsystems, {sc.n_if} interfaces", flush=True)
    sck = model_as(sc, dtype)
    pr = Problem.from_rigid(sc, dtype=dtype)
    A, b, J, e = (_np(t) for t in pr.rigid_assemble(*rst(sck, dtype=dtype)))
    rA, rb, rJ, re = O.rigid_assemble(sck)
    tol = 1e-12 if dtype == torch.float64 else 2e-7
    for g, r, nm in ((A, rA, "A"), (b, rb, "b"), (J, rJ, "J"), (e, re, "e")):
        np.testing.assert_allclose(g, r, atol=tol * max(1.0, np.abs(r).max()), err_msg=nm)


def _settled(sc, n_pre=30):
    st, z, u = (sc.pos, sc.rot, sc.vel, sc.omega), None, None
    for _ in range(n_pre):
        st, r = O.rigid_step(sc, max_iters=1000, tol=1e-6, z0=z, u0=u, n_threads=16, state=st)
        z, u = r.z, r.u
    return st, z, u


def _errors(sc, gv, gl, ref):
    topo = O.RigidTopo(sc)
    w = scene_weight(sc)
    return per_scene_errors(topo, gv, ref.v_hat, gl, ref.lam, v_floor=sc.gravity * sc.dt, l_floor=w)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_mixed_step_fixed_iterations(dtype):
    Problem, rst = _solver()
    sc = S.mixed_scenes(n_scenes=4, seed=S.config_seed(5, 1))
    state, z, u = _settled(sc)
    rnd = (lambda a: np.asarray(a, np.float32).astype(np.float64)) if dtype == torch.float32 else np.asarray
    sck = model_as(sc.with_state(*state), dtype)
    z, u = rnd(z), rnd(u)
    _, ref = O.rigid_step(sck, max_iters=100, tol=0.0, z0=z, u0=u, n_threads=16)
    pr = Problem.from_rigid(sc, dtype=dtype)
    st = rst(sck, dtype=dtype)
    pr.set_warm(pr.tensor(z), pr.tensor(u))
    vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
    pr.rigid_step(*st, max_iters=100, tol=0.0, warm="prev", v_hat=vh, lam=lam)
    pr.check()
    ev, el = _errors(sc, _np(vh), _np(lam), ref)
    print(f"  mixed {dtype} step 31 at 100 iterations: v {ev.max():.3e} lambda {el.max():.3e}", flush=True)
    if dtype == torch.float64:
        assert ev.max() <= 1e-9 and el.max() <= 1e-9
    else:
        assert ev.max() <= FP32_V and el.max() <= FP32_L_WEIGHT


def test_mixed_full_batch_fp32_benchmark_rule():
    Problem, rst = _solver()
    sc = S.mixed_scenes()
    pr = Problem.from_rigid(sc, dtype=torch.float32)
    st = rst(sc, dtype=torch.float32)
    for _ in range(20):
        pr.rigid_step(*st, max_iters=1000, tol=1e-6, warm="prev", graph=True)
    sc1 = sc.with_state(*(_np(t).reshape(s.shape) for t, s in zip(st, (sc.pos, sc.rot, sc.vel, sc.omega))))
    zp, up = (_np(t) for t in pr.get_warm())
    vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
    pr.rigid_step(*st, max_iters=1000, tol=1e-6, warm="prev", v_hat=vh, lam=lam)
    s = pr.stats()
    pr.check()
    it = s["iters"]
    print(f"  mixed full batch step 21: iterations {it.min()}..{it.max()}, converged {int(s['converged'].sum())} "
          f"of {len(it)}", flush=True)
    sck = model_as(sc1, torch.float32)
    A, b, J, e = O.rigid_assemble(sck)
    ref = O.solve(O.RigidTopo(sc), A, b, J, e, max_iters=np.maximum(it, 1), tol=0.0, z0=zp, u0=up, n_threads=16)
    ev, el = _errors(sc, _np(vh), _np(lam), ref)
    print(f"  v {ev.max():.3e} (median {np.median(ev):.2e}) lambda {el.max():.3e}", flush=True)
    assert ev.max() <= 2 * FP32_V and el.max() <= FP32_L_WEIGHT


@pytest.mark.parametrize("large", [False, True])
def test_separating_contact_with_tiny_tangential_part_fp32(large):
    """A separating contact (lambda_n = 0) whose tangential trial value is ~1e-20: its
    square is below the smallest normal float, where the hardware reciprocal square root
    reads zero; the projection must still give lambda = 0 (regression: 0 * inf = NaN)."""
    Problem, _ = _solver()
    m = 1.0
    p = S.AssembledProblem(
        sub_ndof=np.array([3], np.int32), sub_scene=np.array([0], np.int32),
        if_kind=np.array([S.KIND_CONTACT], np.int32), if_dim=np.array([3], np.int32),
        if_nsub=np.array([1], np.int32), if_sub=np.array([[0, -1]], np.int32), if_mu=np.array([0.5]),
        A=(2000.0 * m * np.eye(3)).reshape(-1), b=np.zeros(3), J=np.eye(3).reshape(-1),
        e=np.array([0.5, 5e-24, -3e-24]))
    pr = Problem.from_assembled(p, dtype=torch.float32)
    pr.set_large_path(large)
    o = pr.solve(pr.tensor(p.A), pr.tensor(p.b), pr.tensor(p.J), pr.tensor(p.e), max_iters=5, tol=0.0)
    pr.check()
    ref = O.solve(p, p.A, p.b, p.J, p.e, max_iters=5, tol=0.0)
    assert np.all(ref.lam == 0.0)
    np.testing.assert_array_equal(np.abs(_np(o["lam"])), 0.0)
    np.testing.assert_allclose(_np(o["v_hat"]), ref.v_hat, atol=1e-12)
