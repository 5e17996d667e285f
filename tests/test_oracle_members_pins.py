"""Pins of the oracle's z-update for interfaces joining more than two subsystems
(|S_j| > 2, Sec. III-B: S_j is the set of subsystems a constraint acts on; the z-update of
Eq. 16-21 then sums over all members).  Each problem has interfaces of two to four members
and is checked against a whole-system definition built here from the blocks:

* equalities: the monolithic KKT solve of Eq. 8 with J v + e = 0;
* hard inequalities and frictionless contacts: 2^m active-set enumeration of the convex QP;
* soft couplings (Eq. 3): one linear solve of Eq. 8 with the soft law;
* a three-member interface whose third member's rows are zero has the converged solution of
  the two-member interface without it.
"""
import numpy as np
import pytest

import oracle as O
from paper_2302_14344_amd import scenes as S
from tests import checkers as CK


def _problem(seed, kinds, **kw):
    p = S.random_assembled(seed, n_scenes=1, subs_per_scene=(3, 4), ndof=(4, 7), n_if_per_scene=(3, 5),
                           kinds=kinds, max_members=4, **kw)
    return p


@pytest.mark.parametrize("seed", [71, 72, 73])
def test_multi_member_equalities_match_monolithic_kkt(seed):
    p = _problem(seed, (S.KIND_EQUALITY,), eq_dim=(1, 2))
    assert p.if_nsub.max() >= 3
    r = O.solve(p, p.A, p.b, p.J, p.e, max_iters=400000, tol=1e-14)
    Ag, bg, Jg, _ = CK.global_system(p, p.A, p.b, p.J)
    v, lam = CK.kkt_equality(Ag, bg, Jg, p.e)
    np.testing.assert_allclose(r.v_hat, v, rtol=1e-8, atol=1e-9 * np.abs(v).max())
    np.testing.assert_allclose(r.lam, lam, rtol=1e-7, atol=1e-8 * np.abs(lam).max())


@pytest.mark.parametrize("seed", [80, 83, 84])
def test_multi_member_hard_inequalities_match_enumeration(seed):
    p = _problem(seed, (S.KIND_HARD_INEQ, S.KIND_HARD_INEQ, S.KIND_EQUALITY), eq_dim=(1, 2), e_scale=0.5)
    assert p.if_nsub[p.if_kind == S.KIND_HARD_INEQ].max() >= 3
    r = O.solve(p, p.A, p.b, p.J, p.e, max_iters=400000, tol=1e-14)
    Ag, bg, Jg, e_off = CK.global_system(p, p.A, p.b, p.J)
    eq_rows, ineq_rows = [], []
    for j in range(p.n_if):
        rows = list(range(e_off[j], e_off[j + 1]))
        (ineq_rows if p.if_kind[j] == S.KIND_HARD_INEQ else eq_rows).extend(rows)
    sols = CK.enumerate_inequalities(Ag, bg, Jg, p.e, eq_rows, ineq_rows)
    assert len(sols) >= 1
    v, lam = sols[0]
    np.testing.assert_allclose(r.v_hat, v, rtol=1e-7, atol=1e-8 * max(1.0, np.abs(v).max()))
    np.testing.assert_allclose(r.lam, lam, rtol=1e-6, atol=1e-7 * max(1.0, np.abs(lam).max()))


@pytest.mark.parametrize("seed", [86, 88, 89])
def test_multi_member_frictionless_contacts_match_enumeration(seed):
    p = _problem(seed, (S.KIND_CONTACT, S.KIND_CONTACT, S.KIND_EQUALITY), eq_dim=(1, 1), mu=(0.0, 0.0),
                 e_scale=0.5)
    assert p.if_nsub[p.if_kind == S.KIND_CONTACT].max() >= 3
    r = O.solve(p, p.A, p.b, p.J, p.e, max_iters=400000, tol=1e-14)
    Ag, bg, Jg, e_off = CK.global_system(p, p.A, p.b, p.J)
    eq_rows, contacts = [], []
    for j in range(p.n_if):
        if p.if_kind[j] == S.KIND_CONTACT:
            contacts.append((e_off[j], e_off[j] + 1, e_off[j] + 2))
        else:
            eq_rows += list(range(e_off[j], e_off[j + 1]))
    sols = CK.enumerate_frictionless(Ag, bg, Jg, p.e, eq_rows, contacts)
    assert len(sols) >= 1
    v, lam = sols[0]
    np.testing.assert_allclose(r.v_hat, v, rtol=1e-7, atol=1e-8 * max(1.0, np.abs(v).max()))
    np.testing.assert_allclose(r.lam, lam, rtol=1e-6, atol=1e-7 * max(1.0, np.abs(lam).max()))


@pytest.mark.parametrize("seed", [85, 86])
def test_multi_member_soft_couplings_match_their_linear_solve(seed):
    p = _problem(seed, (S.KIND_SOFT, S.KIND_SOFT, S.KIND_EQUALITY), eq_dim=(1, 2))
    assert p.if_nsub[p.if_kind == S.KIND_SOFT].max() >= 3
    r = O.solve(p, p.A, p.b, p.J, p.e, max_iters=400000, tol=1e-14)
    assert r.converged.all()
    Ag, bg, Jg, e_off = CK.global_system(p, p.A, p.b, p.J)
    eq_rows, soft_rows, ks, als = [], [], [], []
    for j in range(p.n_if):
        rows = list(range(e_off[j], e_off[j + 1]))
        if p.if_kind[j] == S.KIND_SOFT:
            soft_rows += rows
            ks += [p.if_k[j]] * len(rows)
            als += [p.if_alpha[j]] * len(rows)
        else:
            eq_rows += rows
    v, lam = CK.soft_linear_solve(Ag, bg, Jg, p.e, eq_rows, soft_rows, ks, als)
    np.testing.assert_allclose(r.v_hat, v, rtol=1e-8, atol=1e-9 * max(1.0, np.abs(v).max()))
    np.testing.assert_allclose(r.lam, lam, rtol=1e-7, atol=1e-8 * max(1.0, np.abs(lam).max()))


def test_member_with_zero_rows_leaves_the_solution_unchanged():
    """Interface j joins subsystems 0 and 1; adding subsystem 2 as a third member whose
    rows are zero changes the iteration (its penalty enters the z-update's weights) but not
    the converged v_hat and lambda."""
    rng = np.random.default_rng(5)
    n = [4, 5, 3]
    A, b = [], []
    for ni in n:
        Q, _ = np.linalg.qr(rng.standard_normal((ni, ni)))
        A.append(((Q * rng.uniform(1.0, 5.0, ni)) @ Q.T).ravel())
        b.append(rng.standard_normal(ni))
    d = 2
    J0, J1 = rng.standard_normal((d, n[0])), rng.standard_normal((d, n[1]))
    # subsystem 2 also has a one-member equality of its own, so that it has slot rows
    J2own = rng.standard_normal((1, n[2]))
    e = np.concatenate([rng.standard_normal(d), rng.standard_normal(1)])
    two = S.AssembledProblem(
        sub_ndof=np.array(n, np.int32), sub_scene=np.zeros(3, np.int32),
        if_kind=np.array([0, 0], np.int32), if_dim=np.array([d, 1], np.int32), if_nsub=np.array([2, 1], np.int32),
        if_sub=np.array([[0, 1, -1], [2, -1, -1]], np.int32), if_mu=np.zeros(2), A=np.concatenate(A),
        b=np.concatenate(b), J=np.concatenate([J0.ravel(), J1.ravel(), J2own.ravel()]), e=e)
    three = S.AssembledProblem(
        sub_ndof=two.sub_ndof, sub_scene=two.sub_scene, if_kind=two.if_kind, if_dim=two.if_dim,
        if_nsub=np.array([3, 1], np.int32), if_sub=np.array([[0, 1, 2], [2, -1, -1]], np.int32),
        if_mu=two.if_mu, A=two.A, b=two.b,
        J=np.concatenate([J0.ravel(), J1.ravel(), np.zeros(d * n[2]), J2own.ravel()]), e=e)
    r2 = O.solve(two, two.A, two.b, two.J, two.e, max_iters=200000, tol=1e-14)
    r3 = O.solve(three, three.A, three.b, three.J, three.e, max_iters=200000, tol=1e-14)
    assert r2.converged.all() and r3.converged.all()
    assert r3.iters[0] != r2.iters[0]
    np.testing.assert_allclose(r3.v_hat, r2.v_hat, atol=1e-9 * np.abs(r2.v_hat).max())
    np.testing.assert_allclose(r3.lam, r2.lam, atol=1e-9 * np.abs(r2.lam).max())
