"""Pins of the oracle's link rows (soft couplings of Eq. 3, velocity-level rows, ball joints)
against closed forms and finite differences written here from the definitions:

* a soft linear coupling between two free bodies is a spring integrated by the midpoint
  rule (alpha = t/2): its stretch after N steps is phi_0 cos(N w_d t) with
  tan(w_d t / 2) = w t / 2, w^2 = k / m_red (one subsystem or two);
* a soft angular coupling about a common principal axis is a torsional spring with the
  same discrete phase (reduced moment of inertia);
* a one-body velocity row (no-slip, Eq. 4 at velocity level) gives the mass-metric
  projection of the free velocity onto J v = 0;
* link rows and errors match finite differences of phi along a motion (linear, angular,
  ball joint);
* the whole cable stand-in, soft rows and all, satisfies Eq. (8) with Eq. (3) on its soft
  rows and J v + e = 0 on its equality rows at convergence.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle as O
from paper_2302_14344_amd import scenes as S


def _two_bodies(ty, frame, kind, k, alpha, sep, same_sub, twist=0.0, dt=1e-2, fold=False):
    sc = S._SceneBuilder()
    half = np.array([0.05, 0.02, 0.03])
    Ra = np.eye(3)
    Rb = Rotation.from_rotvec([twist, 0, 0]).as_matrix()
    a = sc.add_body(1.5, half, [0.0, 0.0, 1.0], Ra)
    b = sc.add_body(0.7, half, [0.1 + sep, 0.0, 1.0], Rb)
    sc.add_link(ty, a, b, [0.05, 0, 0], [-0.05, 0, 0], frame, kind, k, alpha)
    part = [0, 0] if same_sub else [0, 1]
    out = S._assemble([sc], [part], dt, {}, fold_soft=fold)
    out.gravity = 0.0
    return out


def _run(sc, steps, tol=1e-13, L=20000, rho=0.0):
    st = (sc.pos, sc.rot, sc.vel, sc.omega)
    z = u = None
    out = [st]
    for _ in range(steps):
        st, r = O.rigid_step(sc, rho=rho, max_iters=L, tol=tol, z0=z, u0=u, state=st)
        assert r.converged.all()
        z, u = r.z, r.u
        out.append(st)
    return out


# The midpoint rule with the spring force of Eq. 3 at alpha = t/2 is the trapezoidal map of
# phi'' = -w^2 phi: it rotates (w phi, phi') by theta = 2 atan(w t / 2) per step, so
# phi_n = phi_0 cos(n theta) + (phi'_0 / w) sin(n theta).  (The bodies start moving: with a
# cold start and no free motion the first x-update leaves y unchanged and Alg. 1 stops
# before any z-update.)
def _phase(phi0, dphi0, w, dt, n):
    th = 2.0 * np.arctan(w * dt / 2.0)
    return phi0 * np.cos(n * th) + dphi0 / w * np.sin(n * th)


@pytest.mark.parametrize("same_sub", [True, False])
def test_soft_linear_spring_discrete_phase(same_sub):
    k, dt, sep = 400.0, 1e-2, 0.004
    sc = _two_bodies(S.LINK_LINEAR, [[1, 0, 0]], S.KIND_SOFT, k, 0.5 * dt, sep, same_sub, dt=dt)
    sc.vel[0, 0], sc.vel[1, 0] = 0.02, -0.03
    traj = _run(sc, 25)
    m_red = 1.5 * 0.7 / 2.2
    w = np.sqrt(k / m_red)
    for n, (pos, rot, vel, om) in enumerate(traj):
        phi = (pos[0, 0] + 0.05) - (pos[1, 0] - 0.05)   # anchor separation along x
        ref = _phase(-sep, 0.05, w, dt, n)
        assert abs(phi - ref) < 1e-9 * sep, (n, phi, ref)
    # momentum is conserved and there is no motion off the axis
    for pos, rot, vel, om in traj:
        np.testing.assert_allclose(1.5 * vel[0, 0] + 0.7 * vel[1, 0], 1.5 * 0.02 - 0.7 * 0.03, atol=1e-12)
        assert np.abs(vel[:, 1:]).max() < 1e-12 and np.abs(om).max() < 1e-12


@pytest.mark.parametrize("same_sub", [True, False])
def test_soft_angular_spring_discrete_phase(same_sub):
    kt, dt, th0 = 0.02, 1e-2, 0.01
    sc = _two_bodies(S.LINK_ANGULAR, [[1, 0, 0]], S.KIND_SOFT, kt, 0.5 * dt, 0.0, same_sub, twist=th0, dt=dt)
    sc.omega[0, 0], sc.omega[1, 0] = 0.3, -0.1
    # a penalty on the scale of the rotational terms (Eq. 23 weighs in the translational
    # mass, which this row does not see); the fixed point does not depend on it
    traj = _run(sc, 25, rho=0.1)
    Ia, Ib = sc.inertia[0, 0], sc.inertia[1, 0]
    w = np.sqrt(kt * (Ia + Ib) / (Ia * Ib))
    for n, (pos, rot, vel, om) in enumerate(traj):
        rel = Rotation.from_matrix(rot[0].T @ rot[1]).as_rotvec()   # angle of b relative to a about x
        ref = _phase(th0, -0.4, w, dt, n)
        assert abs(rel[0] - ref) < 1e-9 * th0, (n, rel[0], ref)
        assert np.abs(rel[1:]).max() < 1e-12


@pytest.mark.parametrize("ty", ["linear", "angular"])
def test_folded_soft_spring_discrete_phase(ty):
    """A soft coupling inside one subsystem folded into its dynamics (A_i += k alpha J^T J,
    b_i -= k J^T phi; no interface, so each step is one linear solve) follows the same
    trapezoidal map exactly."""
    dt = 1e-2
    if ty == "linear":
        k, sep = 400.0, 0.004
        sc = _two_bodies(S.LINK_LINEAR, [[1, 0, 0]], S.KIND_SOFT, k, 0.5 * dt, sep, True, dt=dt, fold=True)
        sc.vel[0, 0], sc.vel[1, 0] = 0.02, -0.03
        w = np.sqrt(k / (1.5 * 0.7 / 2.2))
    else:
        kt, th0 = 0.02, 0.01
        sc = _two_bodies(S.LINK_ANGULAR, [[1, 0, 0]], S.KIND_SOFT, kt, 0.5 * dt, 0.0, True, twist=th0, dt=dt,
                         fold=True)
        sc.omega[0, 0], sc.omega[1, 0] = 0.3, -0.1
        Ia, Ib = sc.inertia[0, 0], sc.inertia[1, 0]
        w = np.sqrt(kt * (Ia + Ib) / (Ia * Ib))
    assert sc.n_if == 0 and sc.link_if[0] == -1
    traj = _run(sc, 25)
    for n, (pos, rot, vel, om) in enumerate(traj):
        if ty == "linear":
            phi = (pos[0, 0] + 0.05) - (pos[1, 0] - 0.05)
            ref = _phase(-0.004, 0.05, w, dt, n)
            assert abs(phi - ref) < 1e-10 * 0.004, (n, phi, ref)
        else:
            rel = Rotation.from_matrix(rot[0].T @ rot[1]).as_rotvec()
            ref = _phase(0.01, -0.4, w, dt, n)
            assert abs(rel[0] - ref) < 1e-10 * 0.01, (n, rel[0], ref)
            assert np.abs(rel[1:]).max() < 1e-12


def _kkt_soft_equality(sc, A, b, J, e):
    """v_hat of Eq. (8) with Eq. (3) on the soft rows and J v_hat + e = 0 on the equality
    rows, by one monolithic solve: (A + J_s^T K_a J_s) v - J_e^T l = b - J_s^T K e_s,
    J_e v = -e_e (dense, written here from the equations)."""
    n = np.asarray(sc.sub_ndof)
    doff = np.concatenate([[0], np.cumsum(n)])
    aoff = np.concatenate([[0], np.cumsum(n * n)])
    N = int(doff[-1])
    Ag = np.zeros((N, N))
    for i in range(len(n)):
        Ag[doff[i]:doff[i + 1], doff[i]:doff[i + 1]] = A[aoff[i]:aoff[i + 1]].reshape(n[i], n[i])
    # global rows: each member's slot rows, in interface order
    nc = np.zeros(len(n), np.int64)
    for j in range(sc.n_if):
        for m in range(int(sc.if_nsub[j])):
            nc[sc.if_sub[j, m]] += sc.if_dim[j]
    joff = np.concatenate([[0], np.cumsum(nc * n)])
    fill = np.zeros(len(n), np.int64)
    rows = []
    for j in range(sc.n_if):
        d = int(sc.if_dim[j])
        Jg = np.zeros((d, N))
        for m in range(int(sc.if_nsub[j])):
            i = int(sc.if_sub[j, m])
            Ji = J[joff[i]:joff[i + 1]].reshape(nc[i], n[i])
            Jg[:, doff[i]:doff[i + 1]] += Ji[fill[i]:fill[i] + d]
            fill[i] += d
        rows.append(Jg)
    eoff = np.concatenate([[0], np.cumsum(sc.if_dim)])
    K, rhs, Je, ee = Ag.copy(), b.copy(), [], []
    for j in range(sc.n_if):
        ej = e[eoff[j]:eoff[j + 1]]
        if sc.if_kind[j] == S.KIND_SOFT:
            K += sc.if_k[j] * sc.if_alpha[j] * rows[j].T @ rows[j]
            rhs -= sc.if_k[j] * rows[j].T @ ej
        else:
            assert sc.if_kind[j] == S.KIND_EQUALITY
            Je.append(rows[j])
            ee.append(ej)
    Je = np.concatenate(Je) if Je else np.zeros((0, N))
    ee = np.concatenate(ee) if ee else np.zeros(0)
    ne = Je.shape[0]
    M = np.block([[K, -Je.T], [Je, np.zeros((ne, ne))]])
    return np.linalg.solve(M, np.concatenate([rhs, -ee]))[:N]


def test_cable_both_soft_forms_reach_the_monolithic_solution():
    """The same 16-segment cable (no contacts) with its within-group couplings folded into the
    subsystems' dynamics and with every coupling a soft interface (the two options of the
    remark after Eq. 6): both assemble to the same monolithic system, and the iteration of
    each reaches that system's solution; a folded coupling with the wrong sign of phi or a
    missing alpha would move the monolithic solution, a wrong soft z-update the iterate."""
    kw = dict(n_segments=16, seg_per_sub=4, length=0.2, contacts=False)
    fa, fb = S.cable_scene(fold_soft=True, **kw), S.cable_scene(fold_soft=False, **kw)
    assert fa.n_if < fb.n_if and np.sum(fa.link_if < 0) == 4 * 3 * 4
    # a moving, bent state: a few steps of the interface form
    st = (fb.pos, fb.rot, fb.vel, fb.omega)
    for _ in range(3):
        st, _ = O.rigid_step(fb, max_iters=3000, tol=1e-12, state=st)
    Aa, ba, Ja, ea = O.rigid_assemble(fa, *st)
    Ab, bb, Jb, eb = O.rigid_assemble(fb, *st)
    va, vb = _kkt_soft_equality(fa, Aa, ba, Ja, ea), _kkt_soft_equality(fb, Ab, bb, Jb, eb)
    scale = np.abs(vb).max()
    np.testing.assert_allclose(va, vb, atol=1e-12 * scale)
    ra = O.solve(O.RigidTopo(fa), Aa, ba, Ja, ea, max_iters=4000, tol=0.0)
    rb = O.solve(O.RigidTopo(fb), Ab, bb, Jb, eb, max_iters=4000, tol=0.0)
    np.testing.assert_allclose(ra.v_hat, va, atol=1e-9 * scale)
    np.testing.assert_allclose(rb.v_hat, vb, atol=1e-9 * scale)


def test_velocity_row_is_the_mass_metric_projection():
    """One body with a no-slip row along its body x at point r: v_hat minimises the kinetic
    metric distance to the free velocity subject to J v_hat = 0."""
    sc = S._SceneBuilder()
    half = np.array([0.3, 0.2, 0.1])
    R = Rotation.from_rotvec([0.1, -0.2, 0.4]).as_matrix()
    a = sc.add_body(20.0, half, [0, 0, 1.0], R)
    r = np.array([0.05, -0.02, -0.1])
    sc.add_link(S.LINK_LINEAR, a, -1, r, [0, 0, 0], [[1, 0, 0]], S.KIND_EQUALITY)
    out = S._assemble([sc], [[0]], 1e-2, {})
    out.gravity = 0.0
    v0 = np.array([0.3, -0.2, 0.1])
    out.vel = v0[None, :].copy()
    _, res = O.rigid_step(out, max_iters=20000, tol=1e-14)
    # hand-written row: world direction d = R e_x; point velocity v + R (w x r) along d
    d = R[:, 0]
    Jrow = np.concatenate([d, np.cross(r, R.T @ d)])
    Minv = np.diag(np.concatenate([np.full(3, 1 / 20.0), 1.0 / out.inertia[0]]))
    vf = np.concatenate([v0, np.zeros(3)])
    expect = vf - Minv @ Jrow * (Jrow @ vf) / (Jrow @ Minv @ Jrow)
    np.testing.assert_allclose(res.v_hat, expect, atol=1e-12)
    assert abs(Jrow @ res.v_hat) < 1e-12


def _phi_links(sc, pos, rot):
    """phi of every link row, from positions and rotations (written from the definitions)."""
    out = []
    for q in range(len(sc.link_type)):
        a, b = sc.link_body[q]
        j = sc.link_if[q]
        dim = sc.if_dim[j]
        Ra = rot[a]
        for k in range(dim):
            f = sc.link_frame[q, k]
            d = Ra @ f
            if b < 0:
                out.append(0.0)
            elif sc.link_type[q] == 0:
                xa = pos[a] + Ra @ sc.link_anchor[q, 0]
                xb = pos[b] + rot[b] @ sc.link_anchor[q, 1]
                out.append((xa - xb) @ d)
            else:
                th = Rotation.from_matrix(Ra.T @ rot[b]).as_rotvec()
                out.append(-(f @ th))
    return np.array(out)


def _link_rows_and_errors(sc, A, b, J, e):
    """Per link row: (interface, row k, full-system Jacobian row, e)."""
    n = sc.sub_ndof.astype(int)
    nc = np.zeros(sc.n_sub, int)
    for j in range(sc.n_if):
        for m in range(sc.if_nsub[j]):
            nc[sc.if_sub[j, m]] += sc.if_dim[j]
    Joff = np.concatenate([[0], np.cumsum(nc * n)])
    doff = np.concatenate([[0], np.cumsum(n)])
    soff = np.concatenate([[0], np.cumsum(nc)])
    eoff = np.concatenate([[0], np.cumsum(sc.if_dim)])
    fill = np.zeros(sc.n_sub, int)
    slot = {}
    for j in range(sc.n_if):
        for m in range(sc.if_nsub[j]):
            i = sc.if_sub[j, m]
            slot[(j, m)] = fill[i]
            fill[i] += sc.if_dim[j]
    rows = []
    for q in range(len(sc.link_type)):
        j = sc.link_if[q]
        for k in range(sc.if_dim[j]):
            full = np.zeros(doff[-1])
            for m in range(sc.if_nsub[j]):
                i = sc.if_sub[j, m]
                Ji = J[Joff[i]:Joff[i + 1]].reshape(nc[i], n[i])
                full[doff[i]:doff[i + 1]] += Ji[slot[(j, m)] + k]
            rows.append((j, k, full, e[eoff[j] + k]))
    return rows


def test_link_rows_are_the_rates_of_their_errors():
    """At a pose where every link is at rest (phi = 0; the small cable turned as a whole by a
    random rotation), J v = d phi / dt for random body velocities (central differences over
    the state update of Eq. 2) for the linear, angular and ball-joint rows; at a perturbed
    pose, e = phi (soft) or gamma phi / t (equality)."""
    sc = S.cable_scene(seed=S.config_seed(6, 3), n_segments=6, seg_per_sub=2)
    rng = np.random.default_rng(4)
    nb = sc.n_bodies
    Rg = Rotation.from_rotvec([0.3, -0.7, 0.5]).as_matrix()
    pos = sc.pos @ Rg.T
    rot = np.array([Rg @ R for R in sc.rot])
    v = rng.normal(0, 0.1, (nb, 3))
    w = rng.normal(0, 0.5, (nb, 3))
    order = np.argsort([sc.body_sub[k] * 1000 + sc.body_local[k] for k in range(nb)], kind="stable")
    vdof = np.concatenate([np.concatenate([v[k], w[k]]) for k in order])
    s1 = sc.with_state(pos, rot, v, w)
    A, b, J, e = O.rigid_assemble(s1)
    rows = _link_rows_and_errors(s1, A, b, J, e)
    assert np.abs(_phi_links(s1, pos, rot)).max() < 1e-12
    h = 1e-6

    def moved(t):
        return pos + t * v, np.array([rot[k] @ Rotation.from_rotvec(t * w[k]).as_matrix() for k in range(nb)])
    dphi = (_phi_links(s1, *moved(h)) - _phi_links(s1, *moved(-h))) / (2 * h)
    link_of_if = {int(sc.link_if[q]): q for q in range(len(sc.link_if))}
    n_checked = 0
    for (j, k, full, ek), dp in zip(rows, dphi):
        if sc.link_body[link_of_if[j], 1] >= 0:
            assert abs(full @ vdof - dp) < 1e-8 * max(1.0, abs(dp)), (j, k, full @ vdof, dp)
            n_checked += 1
    assert n_checked == len(rows) - 2  # every row but the two no-slip rows
    # error terms at a perturbed pose
    pos2 = pos + rng.normal(0, 1e-3, (nb, 3))
    rot2 = np.array([Rotation.from_rotvec(rng.normal(0, 0.05, 3)).as_matrix() @ R for R in rot])
    s2 = sc.with_state(pos2, rot2, v, w)
    A, b, J, e = O.rigid_assemble(s2)
    phi = _phi_links(s2, pos2, rot2)
    for (j, k, full, ek), ph in zip(_link_rows_and_errors(s2, A, b, J, e), phi):
        if sc.if_kind[j] == S.KIND_SOFT:
            assert abs(ek - ph) < 1e-12
        else:
            assert abs(ek - sc.baumgarte * ph / sc.dt) < 1e-10


def test_cable_satisfies_eq8_with_soft_rows_at_convergence():
    """At convergence the cable's v_hat and lambda satisfy A v = b + J^T lambda, the soft rows
    lambda = -k (e + alpha J v) and the equality rows J v + e = 0 (contacts open: no gravity)."""
    sc = S.cable_scene(seed=S.config_seed(6, 4), n_segments=12, seg_per_sub=4, gravity=False, contacts=False)
    A, b, J, e = O.rigid_assemble(sc)
    topo = O.RigidTopo(sc)
    r = O.solve(topo, A, b, J, e, max_iters=200000, tol=1e-14)
    assert r.converged.all()
    rows = _link_rows_and_errors(sc, A, b, J, e)
    for j, k, full, ek in rows:
        c = full @ r.v_hat
        lam = r.lam[np.concatenate([[0], np.cumsum(sc.if_dim)])[j] + k]
        if sc.if_kind[j] == S.KIND_SOFT:
            kk, al = sc.if_k[j], sc.if_alpha[j]
            assert abs(lam + kk * (ek + al * c)) < 1e-8 * max(1.0, abs(lam))
        else:
            assert abs(c + ek) < 1e-9
