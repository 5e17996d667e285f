"""GPU learned warm start against the oracle (features, targets, the learned start with
its fallback) and the gain of a trained network.

Inputs of both sides come from the oracle: a state one oracle step into a trajectory and
the oracle's final (z, u) of that step as the previous values (rounded to FP32 for the
FP32 path, and the oracle then receives the rounded values).  Tolerances as in the
solver parity tests: FP64 1e-9, FP32 1e-5, relative to the largest reference entry of
the compared group or a physical floor (velocity g * dt).
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import warm as W
from paper_2302_14344_amd import scenes as S

pytestmark = pytest.mark.gpu

from tests.test_gpu_parity import _np, model_as  # noqa: E402

CONTACT_GROUPS = ((0, 1), (1, 4), (4, 7), (7, 10), (10, 11), (11, 12))
JOINT_GROUPS = ((0, 5), (5, 10), (10, 15), (15, 25), (25, 26), (26, 27))


def _solver():
    from paper_2302_14344_amd.solver import Mlp, Problem, rigid_state_tensors
    return Mlp, Problem, rigid_state_tensors


def _case(which, dtype):
    """(scene after the oracle steps, rho, tol, max_iters, z_prev, u_prev) with the
    previous values rounded to the arithmetic type."""
    if which == "chain":
        sc, rho, tol, L, pre = S.chain_scene(S.config_seed(1)), 1e3, 1e-8, 2000, 12
    else:
        sc, rho, tol, L, pre = S.legged_scenes(48, seed=S.config_seed(4, 800)), 0.0, 1e-6, 1000, 30
    state = (sc.pos, sc.rot, sc.vel, sc.omega)
    r = None
    for _ in range(pre):
        state, r = O.rigid_step(sc, rho=rho, max_iters=L, tol=tol, n_threads=8, state=state)
    rnd = (lambda a: np.asarray(a, np.float32).astype(np.float64)) if dtype == torch.float32 else np.asarray
    sc1 = model_as(sc.with_state(*state), dtype)
    return sc, sc1, rho, tol, L, rnd(r.z), rnd(r.u)


def _gpu_problem(sc, sc1, rho, dtype, zp, up):
    _, Problem, rst = _solver()
    pr = Problem.from_rigid(sc, rho=rho, dtype=dtype)
    st = rst(sc1, dtype=dtype)
    pr.set_warm(pr.tensor(zp), pr.tensor(up))
    return pr, st


def _close_groups(g, r, groups, rel, floor, what, mag=None):
    """Per column group: max error <= rel * max(largest reference entry, floor, largest
    entry of ``mag``, the magnitudes of the summands where a column is a sum)."""
    for a, b in groups:
        ref = r[:, a:b]
        scale = max(float(np.abs(ref).max()) if ref.size else 0.0, floor)
        if mag is not None and ref.size:
            scale = max(scale, float(np.abs(mag[:, a:b]).max()))
        err = float(np.abs(g[:, a:b] - ref).max()) if ref.size else 0.0
        assert err <= rel * scale, f"{what} columns {a}:{b}: error {err:.3e} vs scale {scale:.3e}"


@pytest.mark.parametrize("which,dtype", [("chain", torch.float64), ("legged", torch.float32)])
def test_recorded_features_and_targets_match_oracle(which, dtype):
    print(f"case {which} {dtype}", flush=True)
    sc, sc1, rho, tol, L, zp, up = _case(which, dtype)
    pr, st = _gpu_problem(sc, sc1, rho, dtype, zp, up)
    rec = pr.set_recording(True)
    pr.rigid_step(*st, max_iters=L, tol=tol, warm="prev")
    s = pr.stats()
    topo = O.RigidTopo(sc)
    A, b, J, e = O.rigid_assemble(sc1)
    r1 = O.solve(topo, A, b, J, e, rho=rho, max_iters=L, tol=tol, z0=zp, u0=up, n_threads=8)
    xc, xj = W.features(topo, J, e, r1.beta, W.dof_velocity(sc1), zp, up)
    # features, targets and weights are stored in FP32 (the network's input type): with
    # an FP64 solve they carry the FP32 rounding (2^-24 relative), hence 2e-7
    rel = 2e-7 if dtype == torch.float64 else 1e-5
    vf = sc.gravity * sc.dt
    # the constraint velocity c = sum J v is a sum of terms of size |J| |v|: its rounding
    # error scales with sum |J| |v| (the same features from |J| and |v|)
    mc, mj = W.features(topo, np.abs(J), e, r1.beta, np.abs(W.dof_velocity(sc1)), zp, up)
    _close_groups(_np(rec["xc"]), xc, CONTACT_GROUPS, rel, vf, "contact features", mc)
    _close_groups(_np(rec["xj"]), xj, JOINT_GROUPS, rel, vf, "joint features", mj)
    # targets and weights where both sides stopped at the same iteration
    same = s["iters"] == r1.iters
    print(f"  scenes with equal iteration counts: {same.mean():.3f}", flush=True)
    assert same.mean() >= 0.75
    t = W.targets(topo, r1.beta, zp, up, r1.z, r1.u, r1.converged, sc.sub_scene)
    cls, row, _ = W.interface_classes(sc.if_kind, sc.if_dim, sc.if_nsub)
    scene_of_if = sc.sub_scene[sc.if_sub[:, 0]]
    for c, key in ((0, "c"), (1, "j")):
        rows = row[(cls == c) & same[scene_of_if]]
        gt, rt = _np(rec["t" + key])[rows], t["t" + key][rows]
        gw, rw = _np(rec["w" + key])[rows], t["w" + key][rows]
        np.testing.assert_array_equal(gw == 0, rw == 0)
        np.testing.assert_allclose(gw, rw, rtol=2e-7 if dtype == torch.float64 else 2e-6)
        zscale = max(float(np.abs(r1.z).max()), vf)
        lscale = max(float(np.abs(rt[:, :3 if c == 0 else 5]).max()), vf)
        d = 3 if c == 0 else 5
        assert np.abs(gt[:, :d] - rt[:, :d]).max() <= rel * max(lscale, zscale)
        assert np.abs(gt[:, d:] - rt[:, d:]).max() <= rel * zscale


def _constant_nets(pr, yc, yj):
    """One-layer networks with zero weights: the output is the bias, exactly."""
    Mlp, _, _ = _solver()
    nc, nj = pr.warm_class_counts()
    nets = []
    for c, (nin, y, n) in enumerate(((12, yc, nc), (27, yj, nj))):
        net = Mlp([nin, len(y)], max(n, 1))
        net.set_params(np.concatenate([np.zeros(nin * len(y)), np.asarray(y, np.float32)]))
        pr.set_warm_model(c, net)
        nets.append(net)
    return nets


def test_zero_network_is_the_previous_step_start():
    """Zero network output: the learned step is bit for bit the previous-step step."""
    _, Problem, rst = _solver()
    sc, sc1, rho, tol, L, zp, up = _case("legged", torch.float32)
    outs = []
    for warm in ("prev", "learned"):
        pr, st = _gpu_problem(sc, sc1, rho, torch.float32, zp, up)
        nets = _constant_nets(pr, np.zeros(6), np.zeros(15)) if warm == "learned" else None
        vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
        pr.rigid_step(*st, max_iters=L, tol=tol, warm=warm, v_hat=vh, lam=lam)
        z, u = pr.get_warm()
        outs.append([_np(t) for t in (vh, lam, z, u, *st)] + [pr.stats()["iters"]])
        del nets
    for a, b in zip(*outs):
        np.testing.assert_array_equal(a, b)


def _expected_with_fallback(sc, topo, A, b, J, e, rho, tol, L, budget, z0, u0, zp, up):
    """Oracle of the learned step with its fallback: the run from (z0, u0) with the
    budget; scenes that do not converge there are solved from (zp, up) with L."""
    lrn = O.solve(topo, A, b, J, e, rho=rho, max_iters=budget, tol=tol, z0=z0, u0=u0, n_threads=8)
    prev = O.solve(topo, A, b, J, e, rho=rho, max_iters=L, tol=tol, z0=zp, u0=up, n_threads=8)
    fb = lrn.converged == 0
    v = np.where(np.repeat(fb[sc.sub_scene], sc.sub_ndof), prev.v_hat, lrn.v_hat)
    lam = np.where(np.repeat(fb[sc.sub_scene[sc.if_sub[:, 0]]], sc.if_dim), prev.lam, lrn.lam)
    total = np.where(fb, budget + prev.iters, lrn.iters)
    return lrn, prev, fb, v, lam, total


@pytest.mark.parametrize("which", ["chain", "legged"])
def test_constant_network_start_matches_oracle(which):
    """A network with a known constant output: the GPU's learned step equals the oracle
    started from the values that output defines, with plain ADMM from the previous values
    for the scenes that start does not bring to tol (FP64, 1e-9)."""
    sc, sc1, rho, tol, L, zp, up = _case(which, torch.float64)
    rng = np.random.default_rng(7)
    yc = np.asarray(rng.normal(0, 0.01, 6), np.float32)
    yj = np.asarray(rng.normal(0, 0.01, 15), np.float32)
    pr, st = _gpu_problem(sc, sc1, rho, torch.float64, zp, up)
    nets = _constant_nets(pr, yc, yj)
    vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
    pr.rigid_step(*st, max_iters=L, tol=tol, warm="learned", v_hat=vh, lam=lam)
    s = pr.stats()
    topo = O.RigidTopo(sc)
    A, b, J, e = O.rigid_assemble(sc1)
    beta = O.solve(topo, A, b, J, e, rho=rho, max_iters=1, tol=0.0).beta
    nc, nj = pr.warm_class_counts()
    z0, u0 = W.apply(topo, beta, zp, up, np.tile(yc.astype(np.float64), (nc, 1)),
                     np.tile(yj.astype(np.float64), (nj, 1)))
    lrn, _, fb, ref_v, ref_l, total = _expected_with_fallback(sc, topo, A, b, J, e, rho, tol, L, L, z0, u0, zp, up)
    clear = np.abs(lrn.iters - L) > 3
    print(f"  learned start converges in {(~fb).sum()} of {len(fb)} scenes", flush=True)
    assert (~fb).sum() >= len(fb) // 2
    np.testing.assert_array_equal(s["fallback_total"][clear], fb[clear].astype(np.int64))
    assert np.abs(s["iters_total"][clear] - total[clear]).max() <= 2
    from tests.test_gpu_parity import per_scene_errors, scene_weight
    ev, el = per_scene_errors(topo, _np(vh), ref_v, _np(lam), ref_l, v_floor=sc.gravity * sc.dt,
                              l_floor=scene_weight(sc))
    assert ev[clear].max() <= 1e-9 and el[clear].max() <= 1e-9
    del nets


def test_fallback_restarts_from_previous_values():
    """With a learned-run budget below what some scenes need, those scenes are solved
    again from the previous step's values (plain ADMM, full max_iters) and counted; the
    others keep the learned run.  FP64 against the oracle's two runs, scene by scene."""
    sc, sc1, rho, tol, L, zp, up = _case("legged", torch.float64)
    topo = O.RigidTopo(sc)
    A, b, J, e = O.rigid_assemble(sc1)
    rng = np.random.default_rng(8)
    yc = np.asarray(rng.normal(0, 0.02, 6), np.float32)
    yj = np.asarray(rng.normal(0, 0.02, 15), np.float32)
    beta = O.solve(topo, A, b, J, e, rho=rho, max_iters=1, tol=0.0).beta
    _, _, (nc, nj) = W.interface_classes(sc.if_kind, sc.if_dim, sc.if_nsub)
    z0, u0 = W.apply(topo, beta, zp, up, np.tile(yc.astype(np.float64), (nc, 1)),
                     np.tile(yj.astype(np.float64), (nj, 1)))
    full = O.solve(topo, A, b, J, e, rho=rho, max_iters=L, tol=tol, z0=z0, u0=u0, n_threads=8)
    B = int(np.median(full.iters))
    lrn = O.solve(topo, A, b, J, e, rho=rho, max_iters=B, tol=tol, z0=z0, u0=u0, n_threads=8)
    prev = O.solve(topo, A, b, J, e, rho=rho, max_iters=L, tol=tol, z0=zp, u0=up, n_threads=8)
    fb = lrn.converged == 0
    clear = np.abs(full.iters - B) > 3  # decisions away from the budget
    print(f"  budget {B}: learned start fails in {fb.sum()} of {len(fb)} scenes, {clear.sum()} clear", flush=True)
    assert fb[clear].any() and (~fb[clear]).any()
    pr, st = _gpu_problem(sc, sc1, rho, torch.float64, zp, up)
    pr.set_learned_budget(B)
    nets = _constant_nets(pr, yc, yj)
    vh, lam = pr.empty(pr.sizes.n_dof), pr.empty(pr.sizes.n_rows)
    pr.rigid_step(*st, max_iters=L, tol=tol, warm="learned", v_hat=vh, lam=lam)
    s = pr.stats()
    np.testing.assert_array_equal(s["fallback_total"][clear], fb[clear].astype(np.int64))
    from tests.test_gpu_parity import per_scene_errors, scene_weight
    ref_v = np.where(np.repeat(fb[sc.sub_scene], sc.sub_ndof), prev.v_hat, lrn.v_hat)
    ref_l = np.where(np.repeat(fb[sc.sub_scene[sc.if_sub[:, 0]]], sc.if_dim), prev.lam, lrn.lam)
    ev, el = per_scene_errors(topo, _np(vh), ref_v, _np(lam), ref_l, v_floor=sc.gravity * sc.dt,
                              l_floor=scene_weight(sc))
    assert ev[clear].max() <= 1e-9 and el[clear].max() <= 1e-9
    # both runs are counted: the failed learned attempt (B iterations) plus the fallback
    exp_total = np.where(fb, B + prev.iters, lrn.iters)
    assert np.abs(s["iters_total"][clear] - exp_total[clear]).max() <= 2
    assert (s["converged"][clear] == np.where(fb, prev.converged, 1)[clear]).all()
    del nets


def test_trained_network_start_is_closer_to_the_solution():
    """Train both networks on the GPU (the library's BF16 kernels) from plain-ADMM
    trajectories of legged scenes and measure on held-out scenes: the learned start's
    distance to the converged values in the ADMM metric is well below that of the
    previous-step start.  Iterations and steps per second of learned (with fallback)
    versus plain ADMM are measured and printed; the fallback keeps the residual
    guarantee (no more unconverged scene-steps than plain ADMM, within noise)."""
    from paper_2302_14344_amd import warmstart as WS
    train = S.legged_scenes(256, seed=S.config_seed(4, 1))
    held = S.legged_scenes(256, seed=S.config_seed(4, 100))
    data = WS.collect(train, 80, every=2)
    hold = WS.collect(held, 40, every=4)
    trained = []
    for cls in (0, 1):
        tr = WS.fit(data[cls], cls, iters=1500, batch=4096, lr=1e-3)
        hx, ht, hw = hold[cls].cat()
        net = tr.network(hx.shape[0])
        y = net.forward(hx).double().cpu().numpy()
        ht, hw = ht.double().cpu().numpy(), hw.double().cpu().numpy()
        d_prev, d_learned = float((hw * ht ** 2).sum()), float((hw * (y - ht) ** 2).sum())
        print(f"  class {cls}: squared ADMM-metric distance prev {d_prev:.4e} learned {d_learned:.4e} "
              f"ratio {d_learned / d_prev:.3f}", flush=True)
        assert d_learned < 0.5 * d_prev
        trained.append(tr)
    res = {w: WS.evaluate(held, 60, w, trained=trained) for w in ("prev", "learned")}
    for w, r in res.items():
        print(f"  {w}: iterations per scene-step {r['iters_per_scene_step']:.1f}, fallback "
              f"{r['fallback_frac']:.4f}, unconverged {r['unconverged_frac']:.4f}, steps/s {r['steps_per_s']:.1f}",
              flush=True)
    assert res["learned"]["unconverged_frac"] <= res["prev"]["unconverged_frac"] + 0.005
