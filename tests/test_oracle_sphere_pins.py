"""Pins of the oracle's sphere contact links (link type 2: the normal follows the centres,
or a plane's world normal; the contact points on the spheres along it), written here from
the definitions:

* each row times the bodies' velocities is the relative velocity of the two contact points
  along the row's direction (v + (R omega) x p), the normal error is the gap over t, and the
  normal row is the rate of the gap (central differences over the state update of Eq. 2);
* a sphere resting on the ground: v_hat = 0 and lambda = (m g, 0, 0);
* two spheres meeting head on: one step leaves them with the common velocity of a perfectly
  inelastic contact at the midpoint (momentum conserved, relative normal velocity zero);
* a sphere spinning on the ground with enough friction: the step ends rolling,
  v_hat = (2/7) r omega (the solid sphere's classical result in the midpoint form); spinning
  faster, it slides with the Coulomb force mu m g.
"""
import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle as O
from paper_2302_14344_amd import scenes as S


def _two_spheres(ra=0.02, rb=0.03, gap=0.001, mu=0.5, seed=0, gravity=False):
    rng = np.random.default_rng(seed)
    sc = S._SceneBuilder()
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    pa = np.array([0.1, -0.2, 0.5])
    pb = pa - n * (ra + rb + gap)
    Ra = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    Rb = Rotation.from_rotvec(rng.normal(size=3)).as_matrix()
    a = sc.add_body(0.3, [ra] * 3, pa, Ra, inertia=[0.4 * 0.3 * ra * ra] * 3)
    b = sc.add_body(0.7, [rb] * 3, pb, Rb, inertia=[0.4 * 0.7 * rb * rb] * 3)
    sc.add_link(S.LINK_SPHERE, a, b, [ra, 0, 0], [rb, 0, 0], np.eye(3), S.KIND_CONTACT, mu=mu)
    # a plane through a tilted normal below sphere a
    m = Rotation.from_rotvec([0.3, -0.2, 0.1]).as_matrix()
    off = m[:, 2] @ pa - ra - 0.002
    sc.add_link(S.LINK_SPHERE, a, -1, [ra, 0, 0], [off, 0, 0], [m[:, 2], m[:, 0], m[:, 1]], S.KIND_CONTACT, mu=mu)
    out = S._assemble([sc], [[0, 0]], 1e-2, {})   # one subsystem: one-member interfaces, full rows
    if not gravity:
        out.gravity = 0.0
    return out, n, m


def _full_rows(sc, J):
    n = int(sc.sub_ndof.sum())
    return np.asarray(J).reshape(-1, n)   # one subsystem: the slot rows are the full rows


def _tangents(nv):
    ax = int(np.argmin(np.abs(nv)))
    t1 = np.eye(3)[ax] - nv[ax] * nv
    t1 /= np.linalg.norm(t1)
    return t1, np.cross(nv, t1)


def test_sphere_rows_are_contact_point_velocities():
    sc, n, m = _two_spheres()
    rng = np.random.default_rng(1)
    vel, om = rng.normal(size=(2, 3)), rng.normal(size=(2, 3))
    A, b, J, e = O.rigid_assemble(sc, sc.pos, sc.rot, vel, om)
    rows = _full_rows(sc, J)
    v = np.concatenate([vel[0], om[0], vel[1], om[1]])
    ra, rb = 0.02, 0.03
    # two-sphere contact: normal from b to a, points -ra n on a and +rb n on b
    w = [sc.rot[i] @ om[i] for i in range(2)]
    ca = vel[0] + np.cross(w[0], -ra * n)
    cb = vel[1] + np.cross(w[1], rb * n)
    dirs = [n, *_tangents(n)]
    for k in range(3):
        np.testing.assert_allclose(rows[k] @ v, (ca - cb) @ dirs[k], atol=1e-13)
    np.testing.assert_allclose(e[0] * sc.dt, 0.001, atol=1e-13)
    assert e[1] == 0.0 and e[2] == 0.0
    # the plane: world normal and tangents as given
    cp = vel[0] + np.cross(w[0], -ra * m[:, 2])
    for k, d in enumerate([m[:, 2], m[:, 0], m[:, 1]]):
        np.testing.assert_allclose(rows[3 + k] @ v, cp @ d, atol=1e-13)
    np.testing.assert_allclose(e[3] * sc.dt, 0.002, atol=1e-13)


def test_sphere_normal_row_is_the_gap_rate():
    sc, n, m = _two_spheres(seed=3)
    rng = np.random.default_rng(2)
    vel, om = rng.normal(size=(2, 3)), rng.normal(size=(2, 3))
    A, b, J, e = O.rigid_assemble(sc, sc.pos, sc.rot, vel, om)
    rows = _full_rows(sc, J)
    v = np.concatenate([vel[0], om[0], vel[1], om[1]])
    h = 1e-6

    def gaps(s):
        pos, rot, _, _ = O.rigid_advance(sc, s * v, sc.pos, sc.rot, vel, om)
        _, _, _, ee = O.rigid_assemble(sc, pos, rot, vel, om)
        return ee[[0, 3]] * sc.dt

    rate = (gaps(h / sc.dt) - gaps(-h / sc.dt)) / (2 * h)
    np.testing.assert_allclose(rate, [rows[0] @ v, rows[3] @ v], rtol=1e-6, atol=1e-9)


def _one_sphere(r, mass, mu, vel, omega, gap=0.0):
    sc = S._SceneBuilder()
    a = sc.add_body(mass, [r] * 3, [0.0, 0.0, r + gap], np.eye(3), inertia=[0.4 * mass * r * r] * 3)
    sc.add_link(S.LINK_SPHERE, a, -1, [r, 0, 0], [0.0, 0, 0], np.eye(3)[[2, 0, 1]], S.KIND_CONTACT, mu=mu)
    out = S._assemble([sc], [[0]], 1e-2, {})
    out.vel[0] = vel
    out.omega[0] = omega
    return out


def test_sphere_resting_on_the_ground():
    sc = _one_sphere(0.01, 0.004, 0.5, [0, 0, 0], [0, 0, 0])
    _, r = O.rigid_step(sc, max_iters=20000, tol=1e-13)
    assert r.converged.all()
    np.testing.assert_allclose(r.v_hat, 0.0, atol=1e-12)
    np.testing.assert_allclose(r.lam, [0.004 * sc.gravity, 0.0, 0.0], atol=1e-12)


def test_head_on_spheres_end_with_the_common_velocity():
    sc = S._SceneBuilder()
    a = sc.add_body(0.3, [0.02] * 3, [0.0, 0.0, 0.5], np.eye(3), inertia=[0.4 * 0.3 * 4e-4] * 3)
    b = sc.add_body(0.7, [0.03] * 3, [-0.05, 0.0, 0.5], np.eye(3), inertia=[0.4 * 0.7 * 9e-4] * 3)
    sc.add_link(S.LINK_SPHERE, a, b, [0.02, 0, 0], [0.03, 0, 0], np.eye(3), S.KIND_CONTACT, mu=0.5)
    out = S._assemble([sc], [[0, 1]], 1e-2, {})
    out.gravity = 0.0
    out.vel[0] = [-0.4, 0.0, 0.0]
    out.vel[1] = [0.3, 0.0, 0.0]
    _, r = O.rigid_step(out, max_iters=20000, tol=1e-13)
    assert r.converged.all()
    common = (0.3 * -0.4 + 0.7 * 0.3) / 1.0
    np.testing.assert_allclose(r.v_hat[[0, 6]], [common, common], atol=1e-10)
    np.testing.assert_allclose(r.v_hat[[1, 2, 3, 4, 5, 7, 8, 9, 10, 11]], 0.0, atol=1e-10)


@pytest.mark.parametrize("omega", [10.0, -6.0])
def test_spinning_sphere_ends_the_step_rolling(omega):
    r, mass = 0.01, 0.004
    sc = _one_sphere(r, mass, 1.0, [0.0, 0.0, 0.0], [0.0, omega, 0.0])
    _, res = O.rigid_step(sc, max_iters=50000, tol=1e-13)
    assert res.converged.all()
    vx, wy = res.v_hat[0], res.v_hat[4]
    np.testing.assert_allclose(vx, 2.0 / 7.0 * r * omega, rtol=1e-8)
    np.testing.assert_allclose(vx - r * wy, 0.0, atol=1e-10)   # the contact point is at rest


def test_fast_spinning_sphere_slides_with_coulomb_friction():
    """Spinning too fast for mu m g to stop the slip within the step: the tangential force is
    mu m g against the slip, so v_hat = (t/2) mu g along it and the spin drops by r m v_hat / I."""
    r, mass, mu, omega = 0.01, 0.004, 1.0, -25.0
    sc = _one_sphere(r, mass, mu, [0.0, 0.0, 0.0], [0.0, omega, 0.0])
    _, res = O.rigid_step(sc, max_iters=50000, tol=1e-13)
    assert res.converged.all()
    vx, wy = res.v_hat[0], res.v_hat[4]
    expect = np.sign(omega) * 0.5 * sc.dt * mu * sc.gravity
    np.testing.assert_allclose(vx, expect, rtol=1e-8)
    np.testing.assert_allclose(wy, omega - r * mass * vx / (0.4 * mass * r * r), rtol=1e-8)
    np.testing.assert_allclose(res.lam[0], mass * sc.gravity, rtol=1e-8)
    assert abs(vx - r * wy) > 1e-3    # still slipping
