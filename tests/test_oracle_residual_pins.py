"""Pins of the oracle's primal and dual residuals, the stopping pair of ADMM in its standard
form (Boyd et al. 2011, Sec. 3.3), reported per scene beside r_theta (Eq. 22):
r_prim = |x - z'| / max(|x|, |z'|) and r_dual = |beta (z' - z)| / |u'|, where z', u' are the
z-update (Eq. 16-21) and u-update (Eq. 14) that would follow the last x-update (Eq. 15).

* One DOF and one equality row, one iteration from cold, worked by hand: beta = a (Eq. 23),
  x = b / (2a), y = b / 2, lambda = -(b / 2 + a e), z' = -e, u' = b / 2 + a e.
* Against the iteration itself: a run stopped after L x-updates and a run of L + 1 give
  z' = z^{L+1}, u' = u^{L+1} and x - z' = (u^{L+1} - u^L) / beta slot by slot, so both
  residuals follow from the two runs' returned (z, u), on problems with every interface
  kind and interfaces of up to four members.
* At the fixed point both vanish: a converged run's pair is far below its first one.
"""
import types

import numpy as np
import pytest

import oracle as O
from paper_2302_14344_amd import scenes as S


def _one_row(a, b, e):
    t = types.SimpleNamespace(sub_ndof=np.array([1]), sub_scene=np.array([0]), if_kind=np.array([0]),
                              if_dim=np.array([1]), if_nsub=np.array([1]), if_sub=np.array([[0, -1]]),
                              if_mu=np.array([0.0]))
    return t, np.array([a]), np.array([b]), np.array([1.0]), np.array([e])


@pytest.mark.parametrize("a,b,e", [(2.0, 3.0, 0.5), (5.0, -1.0, 0.25), (0.5, 4.0, -3.0)])
def test_one_row_first_iteration_by_hand(a, b, e):
    t, A, bb, J, ee = _one_row(a, b, e)
    r = O.solve(t, A, bb, J, ee, max_iters=1, tol=0.0)
    x, zn, un = b / (2 * a), -e, b / 2 + a * e
    assert r.beta[0] == pytest.approx(a, rel=1e-15)
    assert r.r_prim[0] == pytest.approx(abs(x - zn) / max(abs(x), abs(zn)), rel=1e-13)
    assert r.r_dual[0] == pytest.approx(abs(a * (zn - 0.0)) / abs(un), rel=1e-13)
    # one iteration more takes exactly those updates
    r2 = O.solve(t, A, bb, J, ee, max_iters=2, tol=0.0)
    assert r2.z[0] == pytest.approx(zn, rel=1e-13) and r2.u[0] == pytest.approx(un, rel=1e-13)


def _slot_beta(p, beta):
    """beta of each slot row's subsystem (slot rows are grouped by subsystem)."""
    isub = O.member_table(p.if_sub, len(p.if_dim))
    nc = np.zeros(len(p.sub_ndof), np.int64)
    for j in range(len(p.if_dim)):
        for m in range(int(p.if_nsub[j])):
            nc[isub[j, m]] += int(p.if_dim[j])
    return np.repeat(beta, nc), np.repeat(np.asarray(p.sub_scene), nc)


def _pair_from_two_runs(p, rL, rL1):
    bs, scene = _slot_beta(p, rL.beta)
    dz = bs * (rL1.z - rL.z)
    xz = (rL1.u - rL.u) / bs  # x - z' of the last x-update
    x = rL1.z + xz
    n = len(rL.r_prim)
    rp, rd = np.zeros(n), np.zeros(n)
    for s in range(n):
        m = scene == s
        nx = max(np.linalg.norm(x[m]), np.linalg.norm(rL1.z[m]), 1e-12)
        rp[s] = np.linalg.norm(xz[m]) / nx
        rd[s] = np.linalg.norm(dz[m]) / max(np.linalg.norm(rL1.u[m]), 1e-12)
    return rp, rd


@pytest.mark.parametrize("seed,kinds,members", [
    (301, (S.KIND_EQUALITY, S.KIND_CONTACT), 2),
    (302, (S.KIND_EQUALITY, S.KIND_CONTACT, S.KIND_HARD_INEQ, S.KIND_SOFT), 2),
    (303, (S.KIND_EQUALITY, S.KIND_HARD_INEQ, S.KIND_SOFT), 4),
])
@pytest.mark.parametrize("L", [1, 7, 40])
def test_pair_matches_the_next_iteration(seed, kinds, members, L):
    p = S.random_assembled(seed, n_scenes=5, subs_per_scene=(2, 5), ndof=(2, 7), n_if_per_scene=(2, 6),
                           kinds=kinds, max_members=members)
    rL = O.solve(p, p.A, p.b, p.J, p.e, max_iters=L, tol=0.0)
    rL1 = O.solve(p, p.A, p.b, p.J, p.e, max_iters=L + 1, tol=0.0)
    rp, rd = _pair_from_two_runs(p, rL, rL1)
    assert rL.r_prim.max() > 0 and rL.r_dual.max() > 0
    np.testing.assert_allclose(rL.r_prim, rp, rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(rL.r_dual, rd, rtol=1e-9, atol=1e-14)


def test_pair_vanishes_at_the_fixed_point():
    p = S.random_assembled(311, n_scenes=4, subs_per_scene=(2, 4), ndof=(3, 6), n_if_per_scene=(2, 5),
                           kinds=(S.KIND_EQUALITY, S.KIND_CONTACT, S.KIND_SOFT))
    r0 = O.solve(p, p.A, p.b, p.J, p.e, max_iters=2, tol=0.0)
    r = O.solve(p, p.A, p.b, p.J, p.e, max_iters=200000, tol=1e-13)
    assert r.converged.all()
    assert (r.r_prim < 1e-8).all() and (r.r_dual < 1e-8).all()
    assert (r.r_prim < 1e-5 * r0.r_prim).all()
