"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle.

Error measure (per scene, norm-wise): |q_gpu - q_ref|_inf / max(|q_ref|_inf, floor), with
physical floors, because a scene in free fall has v_hat of order g t and lambda = 0:
velocity floor g * dt, constraint-force floor the scene's weight sum_k m_k g.

Tolerances:
* FP64 GPU vs FP64 oracle: 1e-9 (same algorithm, differences only in rounding order,
  propagated through a contractive iteration).
* FP32 GPU vs FP64 oracle: 1e-5 for velocities and constraint forces (identical inputs:
  the FP32-rounded state, widened, is what the oracle receives).  Compared (a) after a
  fixed number of iterations and (b) under the same stopping rule r_theta <= 1e-6.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2302_14344_amd import scenes as S

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _solver():
    from paper_2302_14344_amd.solver import Problem, rigid_state_tensors
    return Problem, rigid_state_tensors


def _scene_ranges(sub_scene, sizes):
    """Per scene slice of an array laid out by subsystem with per-subsystem sizes."""
    off = np.concatenate([[0], np.cumsum(sizes)])
    n = int(sub_scene.max()) + 1
    out = []
    for s in range(n):
        idx = np.nonzero(sub_scene == s)[0]
        out.append((off[idx[0]], off[idx[-1] + 1]) if len(idx) else (0, 0))
    return out


def _if_ranges(topo, n_scene):
    e_off = np.concatenate([[0], np.cumsum(topo.if_dim)])
    sc = np.asarray(topo.sub_scene)[np.asarray(topo.if_sub)[:, 0]] if len(topo.if_dim) else np.zeros(0, int)
    out = []
    for s in range(n_scene):
        idx = np.nonzero(sc == s)[0]
        out.append((e_off[idx[0]], e_off[idx[-1] + 1]) if len(idx) else (0, 0))
    return out


def rel_err(a, b, floor):
    a, b = np.asarray(a, float), np.asarray(b, float)
    if a.size == 0:
        return 0.0
    return float(np.abs(a - b).max() / max(np.abs(b).max(), floor))


def per_scene_errors(topo, gpu_v, ref_v, gpu_l, ref_l, v_floor=1e-6, l_floor=None):
    """Per-scene relative errors; ``l_floor`` is a per-scene array of force floors."""
    n_scene = int(np.asarray(topo.sub_scene).max()) + 1
    vr = _scene_ranges(np.asarray(topo.sub_scene), np.asarray(topo.sub_ndof))
    lr = _if_ranges(topo, n_scene)
    ev, el = [], []
    for s in range(n_scene):
        a, b = vr[s]
        ev.append(rel_err(gpu_v[a:b], ref_v[a:b], v_floor))
        a, b = lr[s]
        lf = 1e-30 if l_floor is None else float(l_floor[s])
        el.append(rel_err(gpu_l[a:b], ref_l[a:b], lf))
    return np.array(ev), np.array(el)


def scene_weight(sc):
    w = np.zeros(sc.n_scenes)
    np.add.at(w, sc.sub_scene[sc.body_sub], sc.mass * sc.gravity)
    return w


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def model_as(sc, dtype):
    """The scene with its model constants rounded to the GPU arithmetic type, so that the
    oracle solves exactly the problem the GPU holds (joint anchors rounded by 1e-8 m
    already move Baumgarte terms gamma*phi/t by ~1e-6 m/s)."""
    import copy
    if dtype == torch.float64:
        return sc
    r = lambda a: np.asarray(a, np.float32).astype(np.float64)
    out = copy.copy(sc)
    for f in ("mass", "inertia", "joint_anchor", "joint_frame_a", "joint_axis_b", "contact_point", "pos", "rot",
              "vel", "omega", "link_anchor", "link_frame", "link_k", "link_alpha", "if_k", "if_alpha", "if_mu"):
        if getattr(sc, f, None) is not None:
            setattr(out, f, r(getattr(sc, f)))
    return out


# --------------------------------------------------------------------------------------
# Assembled problems (generic solve entry)
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("seed,n_scenes,iters", [(101, 1, 1), (102, 5, 17), (103, 40, 60), (104, 3, 400)])
def test_solve_fp64_iterate_parity(seed, n_scenes, iters):
    """Fixed iteration count, FP64: v_hat, lambda, z, u match the oracle to 1e-9."""
    print(f"case seed={seed} scenes={n_scenes} iters={iters}", flush=True)
    Problem, _ = _solver()
    p = S.random_assembled(seed, n_scenes=n_scenes, subs_per_scene=(1, 5), ndof=(1, 12), n_if_per_scene=(0, 7),
                           kinds=(0, 1, 2), eq_dim=(1, 6))
    ref = O.solve(p, p.A, p.b, p.J, p.e, max_iters=iters, tol=0.0)
    pr = Problem.from_assembled(p, dtype=torch.float64)
    out = pr.solve(pr.tensor(p.A), pr.tensor(p.b), pr.tensor(p.J), pr.tensor(p.e), max_iters=iters, tol=0.0)
    st = pr.stats()
    # with tol = 0 a scene only stops early when theta is exactly zero (a fixed point in
    # floating point); the two sides may reach that at different iterations
    diff = st["iters"] != ref.iters
    assert np.all(ref.r_theta[diff] < 1e-14) and np.all(st["r_theta"][diff] < 1e-14)
    sc = max(1.0, np.abs(ref.v_hat).max())
    np.testing.assert_allclose(_np(out["v_hat"]), ref.v_hat, atol=1e-9 * sc)
    ls = max(1.0, np.abs(ref.lam).max())
    np.testing.assert_allclose(_np(out["lam"]), ref.lam, atol=1e-9 * ls)
    np.testing.assert_allclose(_np(out["u"]), ref.u, atol=1e-9 * ls)
    zs = max(1.0, np.abs(ref.z).max())
    np.testing.assert_allclose(_np(out["z"]), ref.z, atol=1e-9 * zs)
    np.testing.assert_allclose(_np(pr.beta()), ref.beta, rtol=1e-12)
    same = ~diff
    np.testing.assert_allclose(st["theta"][same], ref.theta[same], rtol=1e-6, atol=1e-20)


def test_solve_fp64_converged_and_warm_given():
    """Run to tol; then restart from the converged (z, u) (given warm start): one
    iteration, same answer (Prop. 1)."""
    Problem, _ = _solver()
    p = S.random_assembled(105, n_scenes=8, subs_per_scene=(2, 4), ndof=(3, 10), n_if_per_scene=(2, 6))
    ref = O.solve(p, p.A, p.b, p.J, p.e, max_iters=20000, tol=1e-11)
    pr = Problem.from_assembled(p, dtype=torch.float64)
    A, b, J, e = pr.tensor(p.A), pr.tensor(p.b), pr.tensor(p.J), pr.tensor(p.e)
    out = pr.solve(A, b, J, e, max_iters=20000, tol=1e-11)
    st = pr.stats()
    assert st["converged"].all()
    assert np.abs(st["iters"] - ref.iters).max() <= 2
    np.testing.assert_allclose(_np(out["v_hat"]), ref.v_hat, atol=1e-8 * np.abs(ref.v_hat).max())
    out2 = pr.solve(A, b, J, e, max_iters=10, tol=1e-9, warm="given", z0=out["z"], u0=out["u"])
    st2 = pr.stats()
    assert (st2["iters"] == 1).all() and st2["converged"].all()
    np.testing.assert_allclose(_np(out2["v_hat"]), _np(out["v_hat"]), atol=1e-9 * np.abs(ref.v_hat).max())
    # previous-step warm start reuses the kept (z, u)
    out3 = pr.solve(A, b, J, e, max_iters=10, tol=1e-9, warm="prev")
    assert (pr.stats()["iters"] == 1).all()
    np.testing.assert_allclose(_np(out3["v_hat"]), _np(out["v_hat"]), atol=1e-9 * np.abs(ref.v_hat).max())


def test_solve_edge_cases_fp64():
    """Largest subsystem (64 DOF), a scene without interfaces, single-DOF subsystems, a
    1-DOF subsystem with 150 slot rows (forces one factorisation launch per DOF count),
    max_iters = 1."""
    Problem, _ = _solver()
    rng = np.random.default_rng(7)
    p = S.random_assembled(106, n_scenes=3, subs_per_scene=(1, 3), ndof=(1, 4), n_if_per_scene=(1, 3))
    n = 64
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A64 = (Q * np.linspace(1, 50, n)) @ Q.T
    k = len(p.sub_ndof)
    sub_ndof = np.concatenate([p.sub_ndof, [n, 5, 1]]).astype(np.int32)
    sub_scene = np.concatenate([p.sub_scene, [3, 4, 5]]).astype(np.int32)
    n_many = 50
    if_kind = np.concatenate([p.if_kind, [0, 1, 2], [2] * n_many]).astype(np.int32)
    if_dim = np.concatenate([p.if_dim, [6, 3, 2], [3] * n_many]).astype(np.int32)
    if_nsub = np.concatenate([p.if_nsub, [1, 1, 1], [1] * n_many]).astype(np.int32)
    if_sub = np.concatenate([p.if_sub, [[k, -1], [k, -1], [k, -1]], [[k + 2, -1]] * n_many]).astype(np.int32)
    if_mu = np.concatenate([p.if_mu, [0.0, 0.7, 0.0], [0.0] * n_many])
    A5 = np.diag(rng.uniform(1, 2, 5))
    q = S.AssembledProblem(sub_ndof, sub_scene, if_kind, if_dim, if_nsub, if_sub, if_mu,
                           A=np.concatenate([p.A, A64.ravel(), A5.ravel(), [3.0]]),
                           b=np.concatenate([p.b, rng.standard_normal(n + 5 + 1)]),
                           J=np.concatenate([p.J, rng.standard_normal(11 * n), rng.standard_normal(3 * n_many)]),
                           e=np.concatenate([p.e, rng.standard_normal(11 + 3 * n_many)]))
    pr = Problem.from_assembled(q, dtype=torch.float64)
    for iters in (1, 50):
        ref = O.solve(q, q.A, q.b, q.J, q.e, max_iters=iters, tol=0.0)
        out = pr.solve(pr.tensor(q.A), pr.tensor(q.b), pr.tensor(q.J), pr.tensor(q.e), max_iters=iters, tol=0.0)
        st = pr.stats()
        diff = st["iters"] != ref.iters
        assert np.all(ref.r_theta[diff] < 1e-14)
        np.testing.assert_allclose(_np(out["v_hat"]), ref.v_hat, atol=1e-9 * np.abs(ref.v_hat).max())
        np.testing.assert_allclose(_np(out["lam"]), ref.lam, atol=1e-9 * max(1, np.abs(ref.lam).max()))
    # the interface-free scene converges at the first x-update
    assert st["converged"][4] == 1 and st["iters"][4] == 1


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_solve_without_any_interface(dtype):
    """No interface at all: every scene stops at the first x-update (theta = 0) and
    v_hat_i = A_i^-1 b_i, the library solve of each block."""
    print(f"case no interfaces dtype={dtype}", flush=True)
    Problem, _ = _solver()
    p = S.random_assembled(108, n_scenes=6, subs_per_scene=(1, 4), ndof=(1, 20), n_if_per_scene=(0, 0))
    assert p.n_if == 0
    pr = Problem.from_assembled(p, dtype=dtype)
    out = pr.solve(pr.tensor(p.A), pr.tensor(p.b), pr.tensor(p.J), pr.tensor(p.e), max_iters=50, tol=1e-9)
    st = pr.stats()
    assert (st["iters"] == 1).all() and (st["converged"] == 1).all()
    ref, a0, d0 = [], 0, 0
    for n in p.sub_ndof:
        ref.append(np.linalg.solve(p.A[a0:a0 + n * n].reshape(n, n), p.b[d0:d0 + n]))
        a0 += n * n
        d0 += n
    ref = np.concatenate(ref)
    tol = 1e-10 if dtype == torch.float64 else 1e-5
    np.testing.assert_allclose(_np(out["v_hat"]), ref, atol=tol * np.abs(ref).max())


def test_not_spd_and_nonfinite_are_reported():
    Problem, _ = _solver()
    p = S.random_assembled(107, n_scenes=2)
    pr = Problem.from_assembled(p, dtype=torch.float32)
    A = p.A.copy()
    A[0] = -abs(A[0]) - 1e6  # first diagonal entry of the first block strongly negative
    out = pr.solve(pr.tensor(A), pr.tensor(p.b), pr.tensor(p.J), pr.tensor(p.e), max_iters=5)
    from paper_2302_14344_amd._lib import SubadmmError, E_NOT_SPD, E_NONFINITE
    with pytest.raises(SubadmmError) as ei:
        pr.check()
    assert ei.value.code == E_NOT_SPD
    pr.check()  # flags were cleared
    b = p.b.copy()
    b[0] = np.nan
    pr.solve(pr.tensor(p.A), pr.tensor(b), pr.tensor(p.J), pr.tensor(p.e), max_iters=5)
    with pytest.raises(SubadmmError) as ei:
        pr.check()
    assert ei.value.code == E_NONFINITE
    del out


def test_determinism_bitwise():
    Problem, _ = _solver()
    sc = S.legged_scenes(64, seed=555)
    pr = Problem.from_rigid(sc, dtype=torch.float32)
    A, b, J, e = O.rigid_assemble(sc)
    args = (pr.tensor(A), pr.tensor(b), pr.tensor(J), pr.tensor(e))
    o1 = pr.solve(*args, max_iters=300, tol=1e-6)
    o2 = pr.solve(*args, max_iters=300, tol=1e-6)
    assert torch.equal(o1["v_hat"], o2["v_hat"]) and torch.equal(o1["lam"], o2["lam"])


# --------------------------------------------------------------------------------------
# Rigid assembly and steps
# --------------------------------------------------------------------------------------

@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("which", ["chain", "legged"])
def test_rigid_assemble_parity(dtype, which):
    print(f"case assemble {which} {dtype}", flush=True)
    Problem, rst = _solver()
    sc = S.chain_scene(S.config_seed(1)) if which == "chain" else S.legged_scenes(256, seed=S.config_seed(2, 7))
    rng = np.random.default_rng(9)
    sc.vel[:] = rng.normal(0, 0.3, sc.vel.shape)
    sc.omega[:] = rng.normal(0, 1.0, sc.omega.shape)
    pr = Problem.from_rigid(sc, dtype=dtype)
    st = rst(sc, dtype=dtype)
    A, b, J, e = pr.rigid_assemble(*st)
    # identical input state: the rounded GPU state, widened
    pos, rot, vel, om = (_np(t) for t in st)
    rA, rb, rJ, re = O.rigid_assemble(model_as(sc, dtype), pos, rot, vel, om)
    tol = 1e-12 if dtype == torch.float64 else 2e-6
    for g, r, nm in ((A, rA, "A"), (b, rb, "b"), (J, rJ, "J"), (e, re, "e")):
        np.testing.assert_allclose(_np(g), r, atol=tol * max(1.0, np.abs(r).max()), err_msg=nm)


def _trajectory_states(sc, steps, **kw):
    """States along an oracle trajectory (inputs for per-step parity)."""
    state = (sc.pos, sc.rot, sc.vel, sc.omega)
    out = [state]
    for _ in range(steps):
        state, _ = O.rigid_step(sc, state=state, **kw)
        out.append(state)
    return out


@pytest.mark.parametrize("mode", ["fixed", "converged"])
def test_chain_fp64_step_parity(mode):
    """Plain method, FP64: serial chain of 8 links in 4 subsystems, rho = 1e3,
    dt = 1e-3; per-step parity from identical states along a 40-step trajectory."""
    Problem, rst = _solver()
    sc = S.chain_scene(S.config_seed(1))
    states = _trajectory_states(sc, 40, rho=1e3, max_iters=200, tol=1e-6)
    pr = Problem.from_rigid(sc, rho=1e3, dtype=torch.float64)
    iters, tol = (60, 0.0) if mode == "fixed" else (5000, 1e-10)
    for k in (0, 10, 25, 40):
        sck = sc.with_state(*states[k])
        _, ref = O.rigid_step(sck, rho=1e3, max_iters=iters, tol=tol)
        st = rst(sck, dtype=torch.float64)
        vh = pr.empty(pr.sizes.n_dof)
        lam = pr.empty(pr.sizes.n_rows)
        pr.rigid_step(*st, max_iters=iters, tol=tol, warm="cold", v_hat=vh, lam=lam)
        s = pr.stats()
        assert abs(int(s["iters"][0]) - int(ref.iters[0])) <= (0 if mode == "fixed" else 2)
        np.testing.assert_allclose(_np(vh), ref.v_hat, atol=1e-9 * max(1e-3, np.abs(ref.v_hat).max()))
        np.testing.assert_allclose(_np(lam), ref.lam, atol=1e-9 * max(1.0, np.abs(ref.lam).max()))
        new_ref = O.rigid_advance(sck, ref.v_hat)
        for g, r in zip(st, new_ref):
            np.testing.assert_allclose(_np(g), r.reshape(-1), atol=1e-12)


def test_chain_fp32_step_parity():
    """The same chain in FP32 against the FP64 oracle under the same rule (rho = 1e3,
    tol = 1e-6, at most 200 iterations) from identical states along a trajectory."""
    Problem, rst = _solver()
    sc = S.chain_scene(S.config_seed(1))
    states = _trajectory_states(sc, 30, rho=1e3, max_iters=200, tol=1e-6)
    pr = Problem.from_rigid(sc, rho=1e3, dtype=torch.float32)
    w = scene_weight(sc)
    errs = []
    for k in (0, 15, 30):
        st = rst(sc.with_state(*states[k]), dtype=torch.float32)
        sck = model_as(sc.with_state(*states[k]), torch.float32)
        _, ref = O.rigid_step(sck, rho=1e3, max_iters=200, tol=1e-6)
        vh = pr.empty(pr.sizes.n_dof)
        lam = pr.empty(pr.sizes.n_rows)
        pr.rigid_step(*st, max_iters=200, tol=1e-6, warm="cold", v_hat=vh, lam=lam)
        ev, el = per_scene_errors(O.RigidTopo(sc), _np(vh), ref.v_hat, _np(lam), ref.lam,
                                  v_floor=sc.gravity * sc.dt, l_floor=w)
        errs.append((ev.max(), el.max(), int(pr.stats()["iters"][0]), int(ref.iters[0])))
    print("fp32 chain errors (v, lambda, iters gpu, iters ref):", errs, flush=True)
    for ev, el, _, _ in errs:
        assert ev <= 1e-5 and el <= 1e-5


def _legged_case(n_scenes, steps):
    sc = S.legged_scenes(n_scenes)
    states = _trajectory_states(sc, steps, max_iters=1000, tol=1e-6, n_threads=8)
    return sc, states[-1]


@pytest.mark.parametrize("n_scenes,steps", [(1024, 0), (256, 45)])
def test_legged_fp32_batch_parity(n_scenes, steps):
    """Batched legged scenes, FP32 GPU vs FP64 oracle.  The full 1024-scene workload in
    the benchmark's launch configuration (first step), and a 256-scene batch after 45
    steps (feet in contact).  Checks fixed-iteration parity and same-rule parity."""
    print(f"case legged n={n_scenes} steps={steps}", flush=True)
    Problem, rst = _solver()
    sc, state = _legged_case(n_scenes, steps)
    pr = Problem.from_rigid(sc, dtype=torch.float32)
    w = scene_weight(sc)
    st0 = rst(sc.with_state(*state), dtype=torch.float32)
    sck = model_as(sc.with_state(*state), torch.float32)
    topo = O.RigidTopo(sc)
    vf = sc.gravity * sc.dt
    for L, tol in ((100, 0.0), (1000, 1e-6)):
        _, ref = O.rigid_step(sck, max_iters=L, tol=tol, n_threads=8)
        st = [t.clone() for t in st0]
        vh = pr.empty(pr.sizes.n_dof)
        lam = pr.empty(pr.sizes.n_rows)
        pr.rigid_step(*st, max_iters=L, tol=tol, warm="cold", v_hat=vh, lam=lam)
        s = pr.stats()
        gv, gl = _np(vh), _np(lam)
        ev, el = per_scene_errors(topo, gv, ref.v_hat, gl, ref.lam, v_floor=vf, l_floor=w)
        mism = np.nonzero(s["iters"] != ref.iters)[0]
        print(f"  L={L} tol={tol}: converged gpu {s['converged'].mean():.4f} ref {ref.converged.mean():.4f}; "
              f"iters diff max {np.abs(s['iters'] - ref.iters).max()} in {len(mism)} scenes; v err max "
              f"{ev.max():.3e} p99 {np.quantile(ev, .99):.3e}; lambda err max {el.max():.3e} "
              f"p99 {np.quantile(el, .99):.3e}", flush=True)
        if tol > 0:
            assert s["converged"].mean() == ref.converged.mean()
            assert np.abs(s["iters"] - ref.iters).max() <= 3
            # where the FP32 run crossed the stopping threshold at another iteration than
            # the FP64 run, the same-algorithm reference is the oracle after exactly the
            # GPU's iteration count
            for m in np.unique(s["iters"][mism]):
                _, refm = O.rigid_step(sck, max_iters=int(m), tol=0.0, n_threads=8)
                evm, elm = per_scene_errors(topo, gv, refm.v_hat, gl, refm.lam, v_floor=vf, l_floor=w)
                pick = mism[s["iters"][mism] == m]
                ev[pick], el[pick] = evm[pick], elm[pick]
        assert ev.max() <= 1e-5 and el.max() <= 1e-5
        # the state update (the oracle's own v_hat: a 1e-5 relative velocity difference
        # moves positions by dt * 1e-5 |v|, far inside the FP32 state tolerance)
        new_ref = O.rigid_advance(sck, ref.v_hat)
        for g, r in zip(st, new_ref):
            np.testing.assert_allclose(_np(g), r.reshape(-1), atol=2e-6 * max(1.0, np.abs(r).max()))


@pytest.mark.parametrize("mode", [True, "within"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_split_and_unsplit_rows_agree(dtype, mode):
    """The thread-per-slot-row kernel with the long rows' products split over 2 or 4 lanes
    (the workgroup growing as needed, or within the default workgroup) computes the same
    iteration as with one lane per row (only the summation order of the split rows
    differs).  In FP32 the stop test at 1e-7 is at the rounding level, so the order moves
    the stopping iteration by a few percent; the results still agree."""
    Problem, rst = _solver()
    sc = S.legged_scenes(96, seed=S.config_seed(2, 12))
    outs = []
    for split in (mode, False):
        pr = Problem.from_rigid(sc, dtype=dtype)
        pr.set_split_rows(split)
        st = rst(sc, dtype=dtype)
        vh = pr.empty(pr.sizes.n_dof)
        lam = pr.empty(pr.sizes.n_rows)
        pr.rigid_step(*st, max_iters=400, tol=1e-7, warm="cold", v_hat=vh, lam=lam)
        outs.append((_np(vh), _np(lam), pr.stats()))
    tol = 1e-11 if dtype == torch.float64 else 2e-6
    (v0, l0, s0), (v1, l1, s1) = outs
    di = np.abs(s0["iters"] - s1["iters"])
    if dtype == torch.float64:
        assert di.max() == 0
    else:
        assert (di <= np.maximum(2, 0.05 * s1["iters"])).all()
    w = scene_weight(sc)
    ev, el = per_scene_errors(O.RigidTopo(sc), v0, v1, l0, l1, v_floor=sc.gravity * sc.dt, l_floor=w)
    assert ev.max() <= tol and el.max() <= tol * 10


@pytest.mark.parametrize("seed,iters", [(121, 60), (122, 400)])
def test_wave_form_solve_fp64_parity(seed, iters):
    """The one-wave-per-scene iteration form against the oracle, fixed iteration count,
    every interface kind (equality, contact, hard inequality, soft)."""
    print(f"case wave form seed={seed} iters={iters}", flush=True)
    Problem, _ = _solver()
    p = S.random_assembled(seed, n_scenes=20, subs_per_scene=(1, 5), ndof=(1, 12), n_if_per_scene=(0, 7),
                           kinds=(0, 1, 2, 3), eq_dim=(1, 6))
    ref = O.solve(p, p.A, p.b, p.J, p.e, max_iters=iters, tol=0.0)
    pr = Problem.from_assembled(p, dtype=torch.float64, team_kernel=2)
    out = pr.solve(pr.tensor(p.A), pr.tensor(p.b), pr.tensor(p.J), pr.tensor(p.e), max_iters=iters, tol=0.0)
    st = pr.stats()
    diff = st["iters"] != ref.iters
    assert np.all(ref.r_theta[diff] < 1e-14) and np.all(st["r_theta"][diff] < 1e-14)
    sc = max(1.0, np.abs(ref.v_hat).max())
    np.testing.assert_allclose(_np(out["v_hat"]), ref.v_hat, atol=1e-9 * sc)
    ls = max(1.0, np.abs(ref.lam).max())
    np.testing.assert_allclose(_np(out["lam"]), ref.lam, atol=1e-9 * ls)
    np.testing.assert_allclose(_np(out["u"]), ref.u, atol=1e-9 * ls)
    zs = max(1.0, np.abs(ref.z).max())
    np.testing.assert_allclose(_np(out["z"]), ref.z, atol=1e-9 * zs)


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_wave_and_thread_kernel_forms_agree(dtype):
    """The wave form and the thread-per-row form (rows not split) run the same iteration on
    a legged batch; only the order of the residual sum differs, so in FP32, where the stop
    test at 1e-7 is at the rounding level, the stopping iteration may move a little."""
    Problem, rst = _solver()
    sc = S.legged_scenes(96, seed=S.config_seed(2, 13))
    outs = []
    for form in (2, 0):
        pr = Problem.from_rigid(sc, dtype=dtype, team_kernel=form)
        st = rst(sc, dtype=dtype)
        vh = pr.empty(pr.sizes.n_dof)
        lam = pr.empty(pr.sizes.n_rows)
        pr.rigid_step(*st, max_iters=400, tol=1e-7, warm="cold", v_hat=vh, lam=lam)
        outs.append((_np(vh), _np(lam), pr.stats()))
    tol = 1e-11 if dtype == torch.float64 else 2e-6
    (v0, l0, s0), (v1, l1, s1) = outs
    di = np.abs(s0["iters"] - s1["iters"])
    if dtype == torch.float64:
        assert di.max() <= 1
    else:
        assert (di <= np.maximum(2, 0.05 * s1["iters"])).all()
    w = scene_weight(sc)
    ev, el = per_scene_errors(O.RigidTopo(sc), v0, v1, l0, l1, v_floor=sc.gravity * sc.dt, l_floor=w)
    assert ev.max() <= tol and el.max() <= tol * 10


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_team_and_thread_kernel_forms_agree(dtype):
    """The two forms of the iteration kernel (lane team per interface with one barrier,
    thread per slot row with two, rows not split) compute the same iteration."""
    Problem, rst = _solver()
    sc = S.legged_scenes(96, seed=S.config_seed(2, 11))
    prs = [Problem.from_rigid(sc, dtype=dtype, team_kernel=t) for t in (True, False)]
    prs[1].set_split_rows(False)
    outs = []
    for pr in prs:
        st = rst(sc, dtype=dtype)
        vh = pr.empty(pr.sizes.n_dof)
        lam = pr.empty(pr.sizes.n_rows)
        pr.rigid_step(*st, max_iters=400, tol=1e-7, warm="cold", v_hat=vh, lam=lam)
        outs.append((_np(vh), _np(lam), pr.stats()))
    tol = 1e-11 if dtype == torch.float64 else 2e-6
    (v0, l0, s0), (v1, l1, s1) = outs
    assert np.abs(s0["iters"] - s1["iters"]).max() <= (0 if dtype == torch.float64 else 2)
    w = scene_weight(sc)
    ev, el = per_scene_errors(O.RigidTopo(sc), v0, v1, l0, l1, v_floor=sc.gravity * sc.dt, l_floor=w)
    assert ev.max() <= tol and el.max() <= tol * 10
