"""Paper-shaped stand-ins under the paper's evaluation protocol (Sec. IV-A, IV-C, Table I):
whole steps at a fixed number of iterations, with the per-step constraint error.

* The 20-piece FEM beam, FP64: warm-up step and four protocol steps at 60 iterations on the
  GPU (``protocol.run``: a timed pass, then the same steps again from the saved state and
  warm start with the error of each) against the oracle's trajectory from the same initial
  state: final state to 1e-9 of its scale, per-step errors to 1e-6 relative.
* The beam in FP32: one step at 60 fixed iterations from the GPU's state against the
  oracle, velocities to 1e-5 of g t, forces to 2e-5 of the beam's weight (the physical
  floors of the benchmark-path tests).
* The 640-segment cable, FP64 (large-scene path, steps replayed from a HIP graph in the
  timed pass): two protocol steps at 30 iterations against the oracle, errors to 1e-6
  relative; FP32 runs the protocol and reports a finite accuracy index.
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import protocol as OP
from paper_2302_14344_amd import scenes as S

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _oracle_fem_run(fs, iters, n_warm, n_steps):
    st, z, u, errs = (fs.pos, fs.vel), None, None, []
    for k in range(n_warm + n_steps):
        A, b, J, e = O.fem_assemble(fs, *st)
        res = O.solve(O.RigidTopo(fs), A, b, J, e, max_iters=iters, tol=0.0, z0=z, u0=u, n_threads=16)
        if k >= n_warm:
            errs.append(OP.constraint_error(fs, J, e, res.v_hat, res.lam, res.beta, kinds=(0, 1, 2)))
        st = O.fem_advance(fs, res.v_hat, *st)
        z, u = res.z, res.u
    return st, np.array(errs)


def _oracle_rigid_run(sc, iters, n_warm, n_steps):
    st, z, u, errs = (sc.pos, sc.rot, sc.vel, sc.omega), None, None, []
    for k in range(n_warm + n_steps):
        A, b, J, e = O.rigid_assemble(sc, *st)
        res = O.solve(O.RigidTopo(sc), A, b, J, e, max_iters=iters, tol=0.0, z0=z, u0=u, n_threads=16)
        if k >= n_warm:
            errs.append((OP.constraint_error(sc, J, e, res.v_hat, res.lam, res.beta, kinds=(0, 1, 2)),
                         OP.constraint_error(sc, J, e, res.v_hat, res.lam, res.beta, kinds=(3,))))
        st = O.rigid_advance(sc, res.v_hat, *st)
        z, u = res.z, res.u
    return st, np.array(errs)


def test_beam_protocol_fp64_against_oracle():
    from paper_2302_14344_amd import protocol
    from paper_2302_14344_amd.solver import Problem, fem_state_tensors
    fs = S.beam_scene()
    print(f"beam: {fs.n_sub} pieces, {int(fs.sub_ndof.sum())} DOF, {fs.n_if} interfaces", flush=True)
    pr = Problem.from_fem(fs, dtype=torch.float64)
    pos, vel = fem_state_tensors(fs, dtype=torch.float64)
    r = protocol.run(pr, "fem", (pos, vel), 60, 4, warmup=1)
    pr.check()
    (rp, rv), rerr = _oracle_fem_run(fs, 60, 1, 4)
    print(f"  GPU AA {r['aa']:.4f}, oracle AA {OP.accuracy_index(rerr):.4f}; errors {r['errors'].ravel()}", flush=True)
    np.testing.assert_allclose(_np(pos), rp.reshape(-1), atol=1e-9 * np.abs(rp).max())
    np.testing.assert_allclose(_np(vel), rv.reshape(-1), atol=1e-9 * max(np.abs(rv).max(), fs.gravity * fs.dt))
    np.testing.assert_allclose(r["errors"], rerr, rtol=1e-6)
    assert abs(r["aa"] - OP.accuracy_index(rerr)) < 1e-6


def test_beam_fp32_step_at_60_iterations():
    from paper_2302_14344_amd.solver import Problem, fem_state_tensors
    fs = S.beam_scene()
    pr = Problem.from_fem(fs, dtype=torch.float32)
    pos, vel = fem_state_tensors(fs, dtype=torch.float32)
    for _ in range(3):
        pr.fem_step(pos, vel, max_iters=60, tol=0.0, warm="prev")
    fs1 = fs.with_state(_np(pos).reshape(-1, 3), _np(vel).reshape(-1, 3))
    zp, up = (_np(t) for t in pr.get_warm())
    vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
    pr.fem_step(pos, vel, max_iters=60, tol=0.0, warm="prev", v_hat=vh, lam=lam)
    pr.check()
    _, ref = O.fem_step(fs1, max_iters=60, tol=0.0, z0=zp, u0=up, n_threads=16)
    X = np.asarray(fs.rest)[np.asarray(fs.tets)]
    vol = np.abs(np.einsum("ij,ij->i", X[:, 1] - X[:, 0], np.cross(X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]))).sum() / 6
    weight = fs.gravity * fs.density * vol
    ev = np.abs(_np(vh) - ref.v_hat).max() / max(fs.gravity * fs.dt, np.abs(ref.v_hat).max())
    el = np.abs(_np(lam) - ref.lam).max() / max(weight, np.abs(ref.lam).max())
    print(f"  beam FP32 step 4 at 60 iterations: v {ev:.3e}, lambda {el:.3e} (weight {weight:.3e} N)", flush=True)
    assert ev <= 1e-5 and el <= 2e-5


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_cable_protocol(dtype):
    from paper_2302_14344_amd import protocol
    from paper_2302_14344_amd.solver import Problem, rigid_state_tensors
    sc = S.cable_scene()
    print(f"cable {dtype}: {sc.n_bodies} bodies, {sc.n_sub} subsystems", flush=True)
    pr = Problem.from_rigid(sc, dtype=dtype)
    st = rigid_state_tensors(sc, dtype=dtype)
    r = protocol.run(pr, "rigid", st, 30, 2, warmup=1)
    pr.check()
    print(f"  {r['ms_per_step']:.3f} ms/step at 30 iterations, AA {r['aa']:.4f}", flush=True)
    assert np.isfinite(r["aa"]) and r["errors"].shape == (2, 1)
    if dtype == torch.float64:
        _, rerr = _oracle_rigid_run(sc, 30, 1, 2)
        print(f"  oracle errors {rerr[:, 0].ravel()} / soft {rerr[:, 1].ravel()}, GPU {r['errors'].ravel()} / "
              f"soft {r['soft_residuals'].ravel()}", flush=True)
        np.testing.assert_allclose(r["errors"], rerr[:, 0], rtol=1e-6)
        np.testing.assert_allclose(r["soft_residuals"], rerr[:, 1], rtol=1e-6)
