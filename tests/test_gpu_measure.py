"""The accuracy measure on the GPU (per-scene constraint error of a step, computed in FP64
from the step's v_hat and lambda) against the oracle's definition on the same arrays.

* Assembled problems with every interface kind (equality, contact, hard, soft), FP64 and
  FP32 solves, all kinds and the two masks (laws, soft), whose squares add up to the whole:
  same v_hat, lambda, J, e and beta on both sides, 1e-10 relative with an absolute floor of
  1e-13 (the sum forming c_j runs in another order on each side).
* The rigid model (legged scenes with contacts) and the FEM lattice after a step: the
  GPU reads the step's own J and e (no J passed) and must match the oracle on the GPU's
  assembly of the pre-step state (J, e equal to the step's), to the same bound.
"""
import copy

import numpy as np
import pytest
import torch

import oracle as O
from oracle import protocol as P
from paper_2302_14344_amd import scenes as S

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _solver():
    from paper_2302_14344_amd.solver import Problem, fem_state_tensors, rigid_state_tensors
    return Problem, fem_state_tensors, rigid_state_tensors


def _close(g, r):
    # c_j = J v_hat + e is summed in another order on each side: rounding of order eps times
    # the terms (|J v| ~ 1), so an absolute floor of 1e-13 beside the relative bound
    np.testing.assert_allclose(g, r, rtol=1e-10, atol=1e-13)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_measure_assembled(dtype):
    print(f"assembled {dtype}", flush=True)
    Problem, _, _ = _solver()
    p = S.random_assembled(141, n_scenes=24, subs_per_scene=(1, 5), ndof=(1, 12), n_if_per_scene=(0, 7),
                           kinds=(0, 1, 2, 3), eq_dim=(1, 6))
    pr = Problem.from_assembled(p, dtype=dtype)
    A, b, J, e = (pr.tensor(x) for x in (p.A, p.b, p.J, p.e))
    # the GPU holds mu, k and alpha in the solve's precision: give the oracle the same values
    q = copy.copy(p)
    for name in ("if_mu", "if_k", "if_alpha"):
        setattr(q, name, _np(pr.tensor(getattr(p, name))))
    for iters in (3, 40):
        o = pr.solve(A, b, J, e, max_iters=iters, tol=0.0)
        g = pr.constraint_error(o["v_hat"], o["lam"], J, e)
        r = P.constraint_error(q, _np(J), _np(e), _np(o["v_hat"]), _np(o["lam"]), _np(pr.beta()))
        assert r.max() > 0
        _close(g, r)
        # the kind masks split the sum of squares: laws (equality, contact, hard) and soft
        gl = pr.constraint_error(o["v_hat"], o["lam"], J, e, kinds=7)
        gs = pr.constraint_error(o["v_hat"], o["lam"], J, e, kinds=8)
        _close(gl, P.constraint_error(q, _np(J), _np(e), _np(o["v_hat"]), _np(o["lam"]), _np(pr.beta()),
                                      kinds=(0, 1, 2)))
        np.testing.assert_allclose(gl ** 2 + gs ** 2, g ** 2, rtol=1e-12, atol=1e-26)
        assert gs.max() > 0 and gl.max() > 0
    pr.check()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_measure_rigid_step(dtype):
    print(f"rigid {dtype}", flush=True)
    Problem, _, rst = _solver()
    sc = S.legged_scenes(16)
    pr = Problem.from_rigid(sc, dtype=dtype)
    st = rst(sc, dtype=dtype)
    for _ in range(30):
        pr.rigid_step(*st, max_iters=200)
    A, b, J, e = pr.rigid_assemble(*st)
    vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
    pr.rigid_step(*st, max_iters=200, v_hat=vh, lam=lam)
    g = pr.constraint_error(vh, lam)
    sq = copy.copy(sc)
    for name in ("if_mu", "if_k", "if_alpha"):
        setattr(sq, name, _np(pr.tensor(getattr(sc, name))))
    r = P.constraint_error(sq, _np(J), _np(e), _np(vh), _np(lam), _np(pr.beta()))
    assert r.max() > 0
    _close(g, r)
    pr.check()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_measure_fem_step(dtype):
    print(f"fem {dtype}", flush=True)
    Problem, fst, _ = _solver()
    fs = S.fem_scene(seed=S.config_seed(3, 11), blocks=(2, 2, 2), nodes_per_block=4)
    pr = Problem.from_fem(fs, dtype=dtype)
    pos, vel = fst(fs, dtype=dtype)
    for _ in range(6):
        pr.fem_step(pos, vel, max_iters=300)
    A, b, J, e = pr.fem_assemble(pos, vel)
    vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
    pr.fem_step(pos, vel, max_iters=40, tol=0.0, v_hat=vh, lam=lam)
    g = pr.constraint_error(vh, lam)
    fq = copy.copy(fs)
    fq.if_mu = _np(pr.tensor(fs.if_mu))
    r = P.constraint_error(fq, _np(J), _np(e), _np(vh), _np(lam), _np(pr.beta()))
    assert r.max() > 0
    _close(g, r)
    pr.check()
