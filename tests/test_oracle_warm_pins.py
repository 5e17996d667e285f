"""Pins of the oracle's learned-warm-start functions (features, initial values, targets).

The learned start is not in the paper; what is pinned is its definition in terms of the
solver's quantities: the constraint velocity against the global Jacobian of Eq. (8),
the weights against the ADMM metric, the round trip targets -> initial values against
the converged values, and a point mass whose features follow by hand.
"""
import numpy as np
import pytest

import oracle as O
from oracle import warm as W
from paper_2302_14344_amd import scenes as S
from tests import checkers as CK


def _random_state(sc, rng):
    vel = rng.standard_normal((sc.n_bodies, 3))
    omega = rng.standard_normal((sc.n_bodies, 3))
    return vel, omega


def test_point_mass_features_by_hand():
    """One body whose contact point is its centre: c = R v with R the contact frame
    (normal +z first), e_n = height / dt (the gap rate), w_hat = beta, mu as given."""
    m, h, mu, dt = 1.7, 0.004, 0.6, 1e-3
    v = np.array([0.3, -0.2, -0.5])
    sc = S.point_mass_scene(m, v, h, mu, dt=dt)
    A, b, J, e = O.rigid_assemble(sc)
    r = O.solve(O.RigidTopo(sc), A, b, J, e, max_iters=50, tol=1e-10)
    z_prev = np.array([0.1, 0.2, 0.3])
    u_prev = np.array([-2.0, 0.5, 0.25])
    xc, xj = W.features(O.RigidTopo(sc), J, e, r.beta, W.dof_velocity(sc), z_prev, u_prev)
    assert xc.shape == (1, 12) and xj.shape == (0, 27)
    x = xc[0]
    assert x[0] == pytest.approx(h / dt, rel=1e-12)
    assert x[1] == pytest.approx(v[2], abs=1e-14)           # normal velocity
    assert np.linalg.norm(x[1:4]) == pytest.approx(np.linalg.norm(v), rel=1e-12)
    np.testing.assert_allclose(x[4:7], -u_prev / r.beta[0], rtol=1e-14)
    np.testing.assert_array_equal(x[7:10], z_prev)
    assert x[10] == pytest.approx(np.log(r.beta[0]), rel=1e-14)
    assert x[11] == mu


@pytest.mark.parametrize("seed", [0, 1])
def test_constraint_velocity_matches_global_jacobian(seed):
    """c of every class row equals the interface rows of the global Jacobian (Eq. 8,
    the sum over members of their slot rows) times the velocity vector."""
    sc = S.legged_scenes(n_scenes=3, seed=S.config_seed(4, 900 + seed))
    rng = np.random.default_rng(seed)
    vel, omega = _random_state(sc, rng)
    A, b, J, e = O.rigid_assemble(sc, vel=vel, omega=omega)
    v = W.dof_velocity(sc, vel, omega)
    topo = O.RigidTopo(sc)
    _, _, nslot, _ = O.layout_sizes(sc.sub_ndof, sc.if_dim, sc.if_nsub, sc.if_sub)
    beta = rng.uniform(10, 1000, sc.n_sub)
    xc, xj = W.features(topo, J, e, beta, v, np.zeros(nslot), np.zeros(nslot))
    _, _, Jg, _ = CK.global_system(topo, A, b, J)
    cv = Jg @ v
    erow = np.concatenate([[0], np.cumsum(sc.if_dim)])
    cls, row, count = W.interface_classes(sc.if_kind, sc.if_dim, sc.if_nsub)
    assert count[0] == int(np.sum(sc.if_kind == S.KIND_CONTACT)) and count[1] > 0
    for j in range(sc.n_if):
        if cls[j] == 0:
            np.testing.assert_allclose(xc[row[j], 1:4], cv[erow[j]:erow[j] + 3], rtol=1e-12, atol=1e-12)
            assert xc[row[j], 0] == e[erow[j]]
        elif cls[j] == 1:
            np.testing.assert_allclose(xj[row[j], 5:10], cv[erow[j]:erow[j] + 5], rtol=1e-12, atol=1e-12)
            np.testing.assert_array_equal(xj[row[j], 0:5], e[erow[j]:erow[j] + 5])
            assert xj[row[j], 26] == sc.if_nsub[j] - 1
    # previous values absent: those columns are zero
    assert not xc[:, 4:10].any() and not xj[:, 10:25].any()


def _solved(seed):
    sc = S.legged_scenes(n_scenes=2, seed=S.config_seed(4, 950 + seed))
    topo = O.RigidTopo(sc)
    A, b, J, e = O.rigid_assemble(sc)
    r0 = O.solve(topo, A, b, J, e, max_iters=1000, tol=1e-8)
    state, _ = O.rigid_step(sc, max_iters=1000, tol=1e-8)
    A, b, J, e = O.rigid_assemble(sc, *state)
    r1 = O.solve(topo, A, b, J, e, max_iters=1000, tol=1e-8, z0=r0.z, u0=r0.u)
    return sc, topo, r0, r1


def test_targets_round_trip_to_converged_values():
    """apply(targets) starts the iteration at exactly the converged (z*, u*) on every
    slot of a class interface and at the previous values elsewhere."""
    sc, topo, r0, r1 = _solved(0)
    t = W.targets(topo, r1.beta, r0.z, r0.u, r1.z, r1.u, r1.converged, sc.sub_scene)
    z0, u0 = W.apply(topo, r1.beta, r0.z, r0.u, t["tc"], t["tj"])
    cls, _, _ = W.interface_classes(sc.if_kind, sc.if_dim, sc.if_nsub)
    _, _, first, _, _ = W.slots(sc.sub_ndof, sc.if_dim, sc.if_nsub, sc.if_sub)
    contact = np.zeros(len(z0), bool)
    for j in range(sc.n_if):
        if cls[j] == 0:
            contact[first[j, 0]:first[j, 0] + 3] = True
    assert contact.any() and (~contact).any()
    np.testing.assert_allclose(z0, r1.z, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(u0, r1.u, rtol=1e-12, atol=1e-9)
    # without a joint output the joint slots keep the previous values
    z1, u1 = W.apply(topo, r1.beta, r0.z, r0.u, t["tc"], None)
    np.testing.assert_array_equal(z1[~contact], r0.z[~contact])
    np.testing.assert_array_equal(u1[~contact], r0.u[~contact])
    np.testing.assert_array_equal(z1[contact], z0[contact])


def test_weights_give_the_admm_metric():
    """sum w (y - t)^2 over the class rows equals sum_i beta_i |z_i - z*_i|^2 +
    beta_i^-1 |u_i - u*_i|^2 over their slots, for the start that apply builds from y."""
    sc, topo, r0, r1 = _solved(1)
    t = W.targets(topo, r1.beta, r0.z, r0.u, r1.z, r1.u, r1.converged, sc.sub_scene)
    assert r1.converged.all()
    rng = np.random.default_rng(5)
    yc = t["tc"] + rng.standard_normal(t["tc"].shape)
    yj = t["tj"] + rng.standard_normal(t["tj"].shape)
    for k in range(len(yj)):  # absent member: its z outputs carry no weight and no effect
        if t["wj"][k, 10] == 0:
            yj[k, 10:] = 0.0
    lhs = np.sum(t["wc"] * (yc - t["tc"]) ** 2) + np.sum(t["wj"] * (yj - t["tj"]) ** 2)
    z0, u0 = W.apply(topo, r1.beta, r0.z, r0.u, yc, yj)
    _, slot, first, _, _ = W.slots(sc.sub_ndof, sc.if_dim, sc.if_nsub, sc.if_sub)
    cls, _, _ = W.interface_classes(sc.if_kind, sc.if_dim, sc.if_nsub)
    rhs = 0.0
    for j in range(sc.n_if):
        if cls[j] < 0:
            continue
        d = int(sc.if_dim[j])
        for m in range(int(sc.if_nsub[j])):
            i = int(sc.if_sub[j][m])
            g = slice(first[j, m], first[j, m] + d)
            rhs += r1.beta[i] * np.sum((z0[g] - r1.z[g]) ** 2) + np.sum((u0[g] - r1.u[g]) ** 2) / r1.beta[i]
    assert lhs == pytest.approx(rhs, rel=1e-10)


def test_unconverged_scene_has_zero_weight():
    sc, topo, r0, r1 = _solved(0)
    conv = np.array(r1.converged, copy=True)
    conv[0] = 0
    t = W.targets(topo, r1.beta, r0.z, r0.u, r1.z, r1.u, conv, sc.sub_scene)
    cls, row, _ = W.interface_classes(sc.if_kind, sc.if_dim, sc.if_nsub)
    for j in range(sc.n_if):
        if cls[j] < 0:
            continue
        w = t["wc" if cls[j] == 0 else "wj"][row[j]]
        scene = sc.sub_scene[sc.if_sub[j][0]]
        assert (w == 0).all() if scene == 0 else (w[:int(sc.if_dim[j])] > 0).all()


def test_non_finite_output_keeps_previous_values():
    sc, topo, r0, r1 = _solved(0)
    t = W.targets(topo, r1.beta, r0.z, r0.u, r1.z, r1.u, r1.converged, sc.sub_scene)
    yc = t["tc"].copy()
    yc[0, 2] = np.nan
    z0, u0 = W.apply(topo, r1.beta, r0.z, r0.u, yc, None)
    cls, row, _ = W.interface_classes(sc.if_kind, sc.if_dim, sc.if_nsub)
    _, _, first, _, _ = W.slots(sc.sub_ndof, sc.if_dim, sc.if_nsub, sc.if_sub)
    j0 = int(np.nonzero((cls == 0) & (row == 0))[0][0])
    g = slice(first[j0, 0], first[j0, 0] + 3)
    np.testing.assert_array_equal(z0[g], r0.z[g])
    np.testing.assert_array_equal(u0[g], r0.u[g])
