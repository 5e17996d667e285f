"""Pins of the oracle's co-rotated FEM assembly (Eq. (2) with the elastic potential folded
into A_i, b_i) against what the mechanics fixes: a library polar decomposition, rigid-
motion invariance, the Hessian of an independently written small-strain energy, exact
linearity for rotation-free stretches, mass and gravity totals, and closed-form free fall.
"""
import numpy as np
import pytest
from scipy.linalg import polar as scipy_polar

import oracle as O
from paper_2302_14344_amd import scenes as S


def _rand_rot(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q *= np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def _tet(rng):
    X = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1]], float) * 0.01 + rng.uniform(-1e-3, 1e-3, (4, 3))
    if np.linalg.det((X[1:] - X[0]).T) < 0:
        X[[2, 3]] = X[[3, 2]]
    return X


def test_polar_matches_library():
    rng = np.random.default_rng(0)
    for _ in range(20):
        F = _rand_rot(rng) @ (np.eye(3) + 0.3 * rng.standard_normal((3, 3)))
        if np.linalg.det(F) <= 0:
            continue
        R = O.polar(F)
        U, _ = scipy_polar(F)
        np.testing.assert_allclose(R, U, atol=1e-12)


def _energy_hessian(X, young, poisson):
    """Hessian of V (mu eps:eps + lam/2 tr(eps)^2), eps = sym(sum_a u_a g_a^T), by central
    differences of the energy (written here from the definition)."""
    lam = young * poisson / ((1 + poisson) * (1 - 2 * poisson))
    mu = young / (2 * (1 + poisson))
    Dm = (X[1:] - X[0]).T
    V = np.linalg.det(Dm) / 6
    Gi = np.linalg.inv(Dm)
    g = np.vstack([-Gi.sum(0), Gi])  # rows g_a

    def psi(u):
        H = u.reshape(4, 3).T @ g
        eps = 0.5 * (H + H.T)
        return V * (mu * np.sum(eps * eps) + 0.5 * lam * np.trace(eps) ** 2)

    h = 1e-4
    K = np.zeros((12, 12))
    for i in range(12):
        for j in range(12):
            e_i, e_j = np.eye(12)[i] * h, np.eye(12)[j] * h
            K[i, j] = (psi(e_i + e_j) - psi(e_i - e_j) - psi(-e_i + e_j) + psi(-e_i - e_j)) / (4 * h * h)
    return K


def test_rest_stiffness_is_the_small_strain_energy_hessian():
    rng = np.random.default_rng(1)
    X = _tet(rng)
    for young, poisson in ((1e6, 0.3), (2e5, 0.45)):
        K, f = O.fem_element(X, X, young, poisson)
        np.testing.assert_allclose(f, 0.0, atol=1e-12 * young)
        ref = _energy_hessian(X, young, poisson)
        np.testing.assert_allclose(K, ref, rtol=1e-6, atol=1e-6 * np.abs(ref).max())


def test_rigid_motion_gives_no_force_and_rotated_stiffness():
    rng = np.random.default_rng(2)
    X = _tet(rng)
    K0, _ = O.fem_element(X, X, 1e6, 0.35)
    Q = _rand_rot(rng)
    x = X @ Q.T + rng.standard_normal(3)
    K, f = O.fem_element(X, x, 1e6, 0.35)
    np.testing.assert_allclose(f, 0.0, atol=1e-9 * np.abs(K0).max() * 0.01)
    Qb = np.kron(np.eye(4), Q)
    np.testing.assert_allclose(K, Qb @ K0 @ Qb.T, atol=1e-9 * np.abs(K0).max())


def test_rotation_free_stretch_force_is_linear():
    """F = I + E with E symmetric (positive definite F): the polar rotation is I, so the
    co-rotated force is exactly -K0 (x - X)."""
    rng = np.random.default_rng(3)
    X = _tet(rng)
    E = rng.standard_normal((3, 3)) * 0.02
    E = 0.5 * (E + E.T)
    x = X @ (np.eye(3) + E).T + np.array([0.1, -0.2, 0.3])
    K0, _ = O.fem_element(X, X, 1e6, 0.3)
    K, f = O.fem_element(X, x, 1e6, 0.3)
    np.testing.assert_allclose(K, K0, atol=1e-9 * np.abs(K0).max())
    np.testing.assert_allclose(f, -K0 @ (x - X).reshape(-1), rtol=1e-9, atol=1e-9 * np.abs(f).max())


def test_rest_state_rows_mass_and_gravity():
    """At rest (x = X, v = 0): b holds only the weights (sum = -g rho V_total, with V_total
    exact for an unjittered lattice), nodal-pair errors vanish, contact errors are z / t,
    A is symmetric positive definite with (2/t) M on top of a stiffness that annihilates
    uniform translations, and J rows are unit selections."""
    fs = S.fem_scene(seed=5, blocks=(2, 1, 1), nodes_per_block=3, jitter=0.0, clearance=0.5)
    A, b, J, e = O.fem_assemble(fs)
    h = fs.meta["h"]
    vol = (2 * 2 * h) * (2 * h) * (2 * h)
    np.testing.assert_allclose(b.reshape(-1, 3)[:, :2], 0.0, atol=1e-15)
    assert b.reshape(-1, 3)[:, 2].sum() == pytest.approx(-fs.gravity * fs.density * vol, rel=1e-12)
    n = int(fs.sub_ndof[0])
    t = fs.dt
    erow = np.concatenate([[0], np.cumsum(fs.if_dim)])
    for j in range(fs.n_if):
        ej = e[erow[j]:erow[j] + 3]
        if fs.if_kind[j] == S.KIND_EQUALITY:
            np.testing.assert_allclose(ej, 0.0, atol=1e-15)
        else:
            np.testing.assert_allclose(ej, [fs.pos[fs.if_node[j, 0], 2] / t, 0, 0], rtol=1e-14)
    mass_node = np.zeros(fs.n_nodes)
    # lumped masses from b (weights) for comparison with the A diagonal mass part
    mass_node[:] = -b.reshape(-1, 3)[:, 2] / fs.gravity
    for i in range(fs.n_sub):
        Ai = A[i * n * n:(i + 1) * n * n].reshape(n, n)
        np.testing.assert_allclose(Ai, Ai.T, atol=1e-9 * np.abs(Ai).max())
        assert np.linalg.eigvalsh(Ai).min() > 0
        m_i = np.repeat(mass_node[i * (n // 3):(i + 1) * (n // 3)], 3)
        Kpart = Ai - np.diag(2 / t * m_i)
        for c in range(3):
            np.testing.assert_allclose(Kpart[:, c::3].sum(1), 0.0, atol=1e-9 * np.abs(Kpart).max())
    assert set(np.unique(J)) <= {-1.0, 0.0, 1.0}


def test_free_fall_is_uniform():
    """Blocks at rest with no contact, tied by nodal equalities: the converged step gives
    every node v_hat = -g t / 2 along z and zero interface forces."""
    fs = S.fem_scene(seed=6, blocks=(2, 1, 1), nodes_per_block=3, contacts=False, clearance=5.0)
    A, b, J, e = O.fem_assemble(fs)
    r = O.solve(O.RigidTopo(fs), A, b, J, e, max_iters=20000, tol=1e-13, n_threads=4)
    assert r.converged.all()
    v = r.v_hat.reshape(-1, 3)
    np.testing.assert_allclose(v[:, :2], 0.0, atol=1e-9)
    np.testing.assert_allclose(v[:, 2], -fs.gravity * fs.dt / 2, rtol=1e-8)
    np.testing.assert_allclose(r.lam, 0.0, atol=1e-8 * fs.gravity * fs.density * 1e-6)
    (pos, vel), _ = O.fem_step(fs, max_iters=20000, tol=1e-13, n_threads=4)
    np.testing.assert_allclose(vel[:, 2], -fs.gravity * fs.dt, rtol=1e-8)
    np.testing.assert_allclose(pos - fs.pos, np.outer(np.ones(fs.n_nodes), [0, 0, -fs.gravity * fs.dt ** 2 / 2]),
                               atol=1e-12)


def test_single_block_unconstrained_is_plain_solve():
    """One block without interfaces: v_hat = A^-1 b (library solve) after one x-update."""
    fs = S.fem_scene(seed=7, blocks=(1, 1, 1), nodes_per_block=3, contacts=False)
    rng = np.random.default_rng(7)
    pos = fs.pos + rng.uniform(-1e-4, 1e-4, fs.pos.shape)
    vel = rng.standard_normal(fs.pos.shape) * 0.01
    A, b, J, e = O.fem_assemble(fs, pos, vel)
    r = O.solve(O.RigidTopo(fs), A, b, J, e, max_iters=3, tol=1e-12)
    n = int(fs.sub_ndof[0])
    np.testing.assert_allclose(r.v_hat, np.linalg.solve(A.reshape(n, n), b), rtol=1e-10, atol=1e-14)


def _strain_energy(fs, pos):
    """sum over tetrahedra of V (mu eps:eps + lam/2 tr(eps)^2), eps the small strain of the
    displacement pos - rest (written here from the definition)."""
    total = 0.0
    for k in range(fs.n_tets):
        v = fs.tets[k]
        X = fs.rest[v]
        u = pos[v] - X
        i = int(fs.tet_sub[k])
        E, nu = fs.young[i], fs.poisson[i]
        lam = E * nu / ((1 + nu) * (1 - 2 * nu))
        mu = E / (2 * (1 + nu))
        Dm = (X[1:] - X[0]).T
        Gi = np.linalg.inv(Dm)
        g = np.vstack([-Gi.sum(0), Gi])
        H = u.T @ g
        eps = 0.5 * (H + H.T)
        total += np.linalg.det(Dm) / 6 * (mu * np.sum(eps * eps) + 0.5 * lam * np.trace(eps) ** 2)
    return total


def test_small_oscillation_conserves_energy():
    """The midpoint rule of Eq. (2) with the elastic force linearised about x and the
    (t/2) K implicit term is the implicit midpoint rule for small (rotation-free to first
    order) vibrations, which conserves kinetic plus strain energy."""
    fs = S.fem_scene(seed=8, blocks=(1, 1, 1), nodes_per_block=3, contacts=False, young=(1e6, 1e6))
    fs.gravity = 0.0
    rng = np.random.default_rng(8)
    mass = np.zeros(fs.n_nodes)
    for v in fs.tets:
        X = fs.rest[v]
        mass[v] += fs.density * np.linalg.det((X[1:] - X[0]).T) / 6 / 4
    pos = fs.pos + rng.uniform(-1e-7, 1e-7, fs.pos.shape)
    vel = np.zeros_like(pos)
    energy = lambda p, v: 0.5 * np.sum(mass[:, None] * v * v) + _strain_energy(fs, p)
    e0 = energy(pos, vel)
    kinetic_seen = 0.0
    for _ in range(20):
        (pos, vel), _ = O.fem_step(fs, state=(pos, vel), max_iters=2, tol=0.0)
        kinetic_seen = max(kinetic_seen, 0.5 * np.sum(mass[:, None] * vel * vel))
        assert abs(energy(pos, vel) - e0) <= 1e-4 * e0
    assert kinetic_seen > 0.1 * e0  # the energy really moves between the two forms
