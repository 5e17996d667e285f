"""Pins of the constraint-error measure (the paper's accuracy index) from its definition:
zero at exact solutions of the constraint laws, the value of each term where it has a closed
form, and the Fischer-Burmeister function's defining property."""
import numpy as np

import oracle as O
from oracle import protocol as P
from paper_2302_14344_amd import scenes as S


def test_fb_is_zero_exactly_on_the_complementarity_set():
    rng = np.random.default_rng(1)
    a = np.abs(rng.normal(size=100))
    assert np.all(P.fb(a, 0.0 * a) == 0.0) and np.all(P.fb(0.0 * a, a) == 0.0)
    assert np.all(np.abs(P.fb(a, a)) > 0) and np.all(np.abs(P.fb(-a, 0 * a)) > 0)
    # sign: negative where either argument is negative
    assert np.all(P.fb(-a, a) < 0)


class _T:
    pass


def _one(kind, dim, mu=0.5, k=0.0, alpha=0.0):
    t = _T()
    t.sub_ndof = np.array([3])
    t.sub_scene = np.array([0])
    t.if_kind = np.array([kind])
    t.if_dim = np.array([dim])
    t.if_nsub = np.array([1])
    t.if_sub = np.array([[0, -1]])
    t.if_mu = np.array([mu])
    t.if_k = np.array([k])
    t.if_alpha = np.array([alpha])
    return t


def test_terms_match_their_definitions():
    J = np.eye(3).reshape(-1)            # one subsystem of 3 DOF, one interface of 3 rows
    beta = np.array([2.0])                # w = 1/2
    v = np.array([0.3, -0.1, 0.2])
    e = np.array([0.05, 0.0, 0.0])
    # equality: |J v + e|
    lam = np.array([1.0, 2.0, 3.0])
    got = P.constraint_error(_one(0, 3), J, e, v, lam, beta)[0]
    assert abs(got - np.linalg.norm(v + e)) < 1e-15
    # contact sticking exactly (c_t = 0, |lambda_t| <= mu lambda_n, c_n = 0): zero
    v2 = np.array([-0.05, 0.0, 0.0])
    got = P.constraint_error(_one(1, 3, mu=0.5), J, e, v2, np.array([4.0, 1.0, -1.0]), beta)[0]
    assert abs(got) < 1e-15
    # contact sliding exactly (lambda_t = -mu lambda_n c_t/|c_t|, c_n = 0): zero
    ct = np.array([0.3, -0.4])
    lt = -0.5 * 4.0 * ct / np.linalg.norm(ct)
    got = P.constraint_error(_one(1, 3, mu=0.5), J, e, np.array([-0.05, *ct]), np.array([4.0, *lt]), beta)[0]
    assert abs(got) < 1e-14
    # contact open (c_n > 0, lambda = 0): zero; penetrating (c_n < 0, lambda = 0): |c_n| (FB(a, 0) = a - |a|)
    got = P.constraint_error(_one(1, 3), J, e, np.array([0.1, 0.2, 0.0]), np.zeros(3), beta)[0]
    assert abs(got) < 1e-15
    got = P.constraint_error(_one(1, 3), J, e, np.array([-0.2, 0.0, 0.0]), np.zeros(3), beta)[0]
    assert abs(got - 2 * 0.15) < 1e-15
    # soft: exact Eq. 3 gives zero; otherwise w |lambda + k (e + alpha J v)|
    k, al = 50.0, 0.005
    lam_s = -k * (e + al * v)
    assert abs(P.constraint_error(_one(3, 3, k=k, alpha=al), J, e, v, lam_s, beta)[0]) < 1e-13
    got = P.constraint_error(_one(3, 3, k=k, alpha=al), J, e, v, lam_s + 1.0, beta)[0]
    assert abs(got - 0.5 * np.sqrt(3.0)) < 1e-13


def test_converged_steps_have_small_error_and_unconverged_larger():
    sc = S.chain_scene(S.config_seed(1))
    A, b, J, e = O.rigid_assemble(sc)
    topo = O.RigidTopo(sc)
    few = O.solve(topo, A, b, J, e, rho=1e3, max_iters=5, tol=0.0)
    many = O.solve(topo, A, b, J, e, rho=1e3, max_iters=20000, tol=1e-12)
    e_few = P.constraint_error(topo, J, e, few.v_hat, few.lam, few.beta)[0]
    e_many = P.constraint_error(topo, J, e, many.v_hat, many.lam, many.beta)[0]
    assert e_many < 1e-9 * max(1.0, e_few) and e_few > 1e-6
    assert P.accuracy_index([e_many]) > P.accuracy_index([e_few])
