"""FP64 CPU oracle for the per-step subsystem-based ADMM solve (arXiv 2302.14344).

TEST INFRASTRUCTURE ONLY.  This package is the independent reference that the HIP
library is checked against.  Only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import it; the product package never does.  It
shares no code with the HIP library: the C sources in this directory implement every
step (assembly, Eq. (23) penalty, Cholesky, the x/z/u updates of Eq. (12)-(21), the
residual of Eq. (22) and the state update of Eq. (2)) on their own.

The C library ``liboracle.so`` is built by ``oracle/build.py`` (called from
``__graft_entry__.build()``); this wrapper only marshals numpy arrays.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")


def _opt_f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(C.POINTER(C.c_double))


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b
            _b.build()
        L = C.CDLL(path)
        L.oracle_solve.restype = C.c_int
        L.oracle_solve.argtypes = [
            C.c_int32, _i32p, _i32p, C.c_int32, _i32p, _i32p, _i32p, _i32p, _f64p,
            _f64p, _f64p, _f64p, _f64p, C.c_double, C.c_int32, C.c_double,
            C.POINTER(C.c_double), C.POINTER(C.c_double),
            _f64p, _f64p, _f64p, _f64p, _f64p, _i32p, _i32p, _f64p, _f64p, C.c_int32]
        L.oracle_solve_model.restype = C.c_int
        L.oracle_solve_model.argtypes = L.oracle_solve.argtypes[:-1] + [
            _f64p, _f64p,
            C.c_int32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_int32]
        L.oracle_rigid_assemble.restype = C.c_int
        L.oracle_rigid_assemble.argtypes = [
            C.c_int32, _i32p, C.c_int32, _i32p, _i32p, _i32p,
            C.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p,
            C.c_int32, _i32p, _f64p, _f64p, _f64p, _i32p,
            C.c_int32, _i32p, _f64p, _i32p,
            C.c_double, C.c_double, C.c_double, _f64p, _f64p, _f64p, _f64p]
        L.oracle_rigid_links.restype = C.c_int
        L.oracle_rigid_links.argtypes = [
            C.c_int32, _i32p, C.c_int32, _i32p, _i32p, _i32p, _i32p, _i32p, _i32p, _f64p, _f64p,
            C.c_int32, _i32p, _i32p, _f64p, _f64p, _i32p, C.c_double, C.c_double, _f64p, _f64p]
        L.oracle_rigid_fold_soft.restype = C.c_int
        L.oracle_rigid_fold_soft.argtypes = [
            C.c_int32, _i32p, _i32p, _i32p, _f64p, _f64p, C.c_int32, _i32p, _i32p, _f64p, _f64p, _i32p, _i32p,
            _f64p, _f64p, _f64p, _f64p]
        L.oracle_rigid_advance.restype = C.c_int
        L.oracle_rigid_advance.argtypes = [
            C.c_int32, _i32p, _i32p, C.c_int32, _i32p, _f64p, C.c_double,
            _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p, _f64p]
        L.oracle_mlp_forward.restype = C.c_int
        L.oracle_mlp_forward.argtypes = [C.c_int32, _i32p, _f64p, C.c_int32, _f64p, _f64p]
        L.oracle_mlp_backward.restype = C.c_int
        L.oracle_mlp_backward.argtypes = [C.c_int32, _i32p, _f64p, C.c_int32, _f64p, _f64p, _f64p, _f64p,
                                          C.POINTER(C.c_double)]
        L.oracle_fem_assemble.restype = C.c_int
        L.oracle_fem_assemble.argtypes = [
            C.c_int32, _i32p, C.c_int32, _i32p, _i32p, _f64p, _f64p, _f64p, _f64p, _f64p, C.c_double,
            C.c_int32, _i32p, _i32p, _i32p, _i32p, _i32p, C.c_double, C.c_double, C.c_double,
            _f64p, _f64p, _f64p, _f64p]
        L.oracle_fem_element.restype = C.c_int
        L.oracle_fem_element.argtypes = [_f64p, _f64p, C.c_double, C.c_double, _f64p, _f64p]
        L.oracle_polar.restype = C.c_int
        L.oracle_polar.argtypes = [_f64p, _f64p]
        L.oracle_fem_advance.restype = C.c_int
        L.oracle_fem_advance.argtypes = [C.c_int64, _f64p, C.c_double, _f64p, _f64p, _f64p, _f64p]
        _LIB = L
    return _LIB


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def layout_sizes(sub_ndof, if_dim, if_nsub, if_sub):
    """(sum n_i^2, sum nc_i n_i, total slot rows, total interface rows)."""
    sub_ndof = np.asarray(sub_ndof, np.int64)
    nc = np.zeros(len(sub_ndof), np.int64)
    for j in range(len(if_dim)):
        for m in range(int(if_nsub[j])):
            nc[int(if_sub[j][m])] += int(if_dim[j])
    return int((sub_ndof ** 2).sum()), int((nc * sub_ndof).sum()), int(nc.sum()), int(np.sum(if_dim))


@dataclass
class SolveResult:
    v_hat: np.ndarray
    lam: np.ndarray
    z: np.ndarray
    u: np.ndarray
    beta: np.ndarray
    iters: np.ndarray
    converged: np.ndarray
    theta: np.ndarray
    r_theta: np.ndarray
    r_prim: np.ndarray = None  # primal residual of the returned iterate (Boyd et al. 2011, Sec. 3.3)
    r_dual: np.ndarray = None  # dual residual of the returned iterate


MAX_MEMBERS = 4


def member_table(if_sub, n_if):
    """Members of each interface as an (n_if, 4) table (unused entries -1): the solve's
    layout; scenes carry (n_if, 2) tables when no interface has more than two members."""
    t = np.asarray(if_sub, np.int64).reshape(n_if, -1) if n_if else np.zeros((0, 1), np.int64)
    assert t.shape[1] <= MAX_MEMBERS, "at most four members per interface"
    out = np.full((n_if, MAX_MEMBERS), -1, np.int64)
    out[:, :t.shape[1]] = t
    return out


def solve(topo, A, b, J, e, rho=0.0, max_iters=200, tol=1e-6, z0=None, u0=None, n_threads=1, contact_model=0):
    """Algorithm 1 of the paper (construction steps excluded) on an assembled problem.

    ``max_iters``: the iteration bound, one for every scene or an array with one per scene.

    ``topo`` provides sub_ndof, sub_scene, if_kind, if_dim, if_nsub, if_sub, if_mu (if_sub:
    an (n_if, 2) or (n_if, 4) table of members; an interface may join up to four
    subsystems, Sec. III-B).
    Each scene (set of subsystems with equal ``sub_scene``) terminates on its own test.
    ``contact_model``: 0 = exact Signorini-Coulomb projection in the contact z-update
    (Eq. 21), 1 = the relaxed convex model (Euclidean projection onto the friction cone).
    Soft interfaces (kind 3, Eq. 3) take their gain and alpha from ``topo.if_k`` and
    ``topo.if_alpha``.
    The result carries, per scene, ADMM's standard primal and dual residuals of the returned
    iterate (``r_prim``, ``r_dual``: the z- and u-updates that would follow the last
    x-update, taken aside; r_prim = |x - z'| / max(|x|, |z'|), r_dual = |beta (z' - z)| /
    |u'|), reported beside r_theta, which decides the stop.
    """
    sub_ndof, sub_scene = _i32(topo.sub_ndof), _i32(topo.sub_scene)
    if_kind, if_dim, if_nsub = _i32(topo.if_kind), _i32(topo.if_dim), _i32(topo.if_nsub)
    members = member_table(topo.if_sub, len(if_kind))
    if_sub, if_mu = _i32(members.reshape(-1)), _f64(topo.if_mu)
    nA, nJ, nslot, nrow = layout_sizes(sub_ndof, if_dim, if_nsub, members)
    n_scenes = int(sub_scene.max()) + 1
    ndof = int(sub_ndof.sum())
    A, b, J, e = _f64(A), _f64(b), _f64(J), _f64(e)
    assert A.size == nA and b.size == ndof and J.size == nJ and e.size == nrow, "assembled sizes"
    out = SolveResult(np.zeros(ndof), np.zeros(nrow), np.zeros(nslot), np.zeros(nslot),
                      np.zeros(len(sub_ndof)), np.zeros(n_scenes, np.int32), np.zeros(n_scenes, np.int32),
                      np.zeros(n_scenes), np.zeros(n_scenes), np.zeros(n_scenes), np.zeros(n_scenes))
    if z0 is not None:
        z0 = _f64(z0)
        assert z0.size == nslot
    if u0 is not None:
        u0 = _f64(u0)
        assert u0.size == nslot
    if_k, if_alpha = getattr(topo, "if_k", None), getattr(topo, "if_alpha", None)
    if_k = None if if_k is None else _f64(if_k)
    if_alpha = None if if_alpha is None else _f64(if_alpha)
    caps = None
    if np.ndim(max_iters) > 0:
        caps = _i32(max_iters)
        assert caps.size == n_scenes and caps.min() >= 1, "one iteration bound >= 1 per scene"
        max_iters = int(caps.max())
    rc = lib().oracle_solve_model(len(sub_ndof), sub_ndof, sub_scene, len(if_kind), if_kind, if_dim, if_nsub,
                                  if_sub, if_mu, A, b, J, e, float(rho), int(max_iters), float(tol),
                                  _opt_f64(z0), _opt_f64(u0), out.v_hat, out.lam, out.z, out.u, out.beta,
                                  out.iters, out.converged, out.theta, out.r_theta, out.r_prim, out.r_dual,
                                  int(contact_model),
                                  _opt_f64(if_k), _opt_f64(if_alpha),
                                  caps.ctypes.data_as(C.POINTER(C.c_int32)) if caps is not None else None,
                                  int(n_threads))
    if rc != 0:
        raise RuntimeError(f"oracle_solve failed with code {rc}")
    return out


def rigid_assemble(sc, pos=None, rot=None, vel=None, omega=None):
    """Eq. (2)-(5) for a RigidScenes batch at the given (or stored) state: (A, b, J, e)."""
    pos = _f64(sc.pos if pos is None else pos).reshape(-1)
    rot = _f64(sc.rot if rot is None else rot).reshape(-1)
    vel = _f64(sc.vel if vel is None else vel).reshape(-1)
    omega = _f64(sc.omega if omega is None else omega).reshape(-1)
    sub_ndof = _i32(sc.sub_ndof)
    nA, nJ, nslot, nrow = layout_sizes(sub_ndof, sc.if_dim, sc.if_nsub, sc.if_sub)
    A, b, J, e = np.zeros(nA), np.zeros(int(sub_ndof.sum())), np.zeros(nJ), np.zeros(nrow)
    rc = lib().oracle_rigid_assemble(
        sc.n_sub, sub_ndof, sc.n_if, _i32(sc.if_dim), _i32(sc.if_nsub), _i32(sc.if_sub.reshape(-1)),
        sc.n_bodies, _i32(sc.body_sub), _i32(sc.body_local), _f64(sc.mass), _f64(sc.inertia.reshape(-1)),
        pos, rot, vel, omega,
        len(sc.joint_body), _i32(sc.joint_body.reshape(-1)), _f64(sc.joint_anchor.reshape(-1)),
        _f64(sc.joint_frame_a.reshape(-1)), _f64(sc.joint_axis_b.reshape(-1)), _i32(sc.joint_if),
        len(sc.contact_body), _i32(sc.contact_body), _f64(sc.contact_point.reshape(-1)), _i32(sc.contact_if),
        float(sc.dt), float(sc.gravity), float(sc.baumgarte), A, b, J, e)
    if rc != 0:
        raise RuntimeError(f"oracle_rigid_assemble failed with code {rc}")
    nl = n_links(sc)
    if nl:
        rc = lib().oracle_rigid_links(
            sc.n_sub, sub_ndof, sc.n_if, _i32(sc.if_kind), _i32(sc.if_dim), _i32(sc.if_nsub),
            _i32(sc.if_sub.reshape(-1)), _i32(sc.body_sub), _i32(sc.body_local), pos, rot, nl,
            _i32(sc.link_type), _i32(sc.link_body.reshape(-1)), _f64(sc.link_anchor.reshape(-1)),
            _f64(sc.link_frame.reshape(-1)), _i32(sc.link_if), float(sc.dt), float(sc.baumgarte), J, e)
        if rc != 0:
            raise RuntimeError(f"oracle_rigid_links failed with code {rc}")
        if np.any(np.asarray(sc.link_if) < 0):
            rc = lib().oracle_rigid_fold_soft(
                sc.n_sub, sub_ndof, _i32(sc.body_sub), _i32(sc.body_local), pos, rot, nl, _i32(sc.link_type),
                _i32(sc.link_body.reshape(-1)), _f64(sc.link_anchor.reshape(-1)), _f64(sc.link_frame.reshape(-1)),
                _i32(sc.link_if), _i32(sc.link_dim), _f64(sc.link_k), _f64(sc.link_alpha), A, b)
            if rc != 0:
                raise RuntimeError(f"oracle_rigid_fold_soft failed with code {rc}")
    return A, b, J, e


def n_links(sc):
    lt = getattr(sc, "link_type", None)
    return 0 if lt is None else int(len(lt))


def rigid_advance(sc, v_hat, pos=None, rot=None, vel=None, omega=None):
    """State update of Eq. (2): returns (pos, rot, vel, omega) after the step."""
    pos = _f64(sc.pos if pos is None else pos).reshape(-1)
    rot = _f64(sc.rot if rot is None else rot).reshape(-1)
    vel = _f64(sc.vel if vel is None else vel).reshape(-1)
    omega = _f64(sc.omega if omega is None else omega).reshape(-1)
    nb = sc.n_bodies
    po, ro, vo, oo = np.zeros(3 * nb), np.zeros(9 * nb), np.zeros(3 * nb), np.zeros(3 * nb)
    rc = lib().oracle_rigid_advance(nb, _i32(sc.body_sub), _i32(sc.body_local), sc.n_sub, _i32(sc.sub_ndof),
                                    _f64(v_hat), float(sc.dt), pos, rot, vel, omega, po, ro, vo, oo)
    if rc != 0:
        raise RuntimeError(f"oracle_rigid_advance failed with code {rc}")
    return po.reshape(nb, 3), ro.reshape(nb, 3, 3), vo.reshape(nb, 3), oo.reshape(nb, 3)


class RigidTopo:
    """Adapter exposing a RigidScenes batch's topology to ``solve``."""

    def __init__(self, sc):
        self.sub_ndof = sc.sub_ndof
        self.sub_scene = sc.sub_scene
        self.if_kind, self.if_dim, self.if_nsub = sc.if_kind, sc.if_dim, sc.if_nsub
        self.if_sub, self.if_mu = sc.if_sub, sc.if_mu
        self.if_k, self.if_alpha = getattr(sc, "if_k", None), getattr(sc, "if_alpha", None)


def rigid_step(sc, rho=0.0, max_iters=1000, tol=1e-6, z0=None, u0=None, n_threads=1, state=None, contact_model=0):
    """One whole step of Algorithm 1 on a rigid batch: assemble, solve, advance.

    Returns (new_state, SolveResult)."""
    if state is None:
        state = (sc.pos, sc.rot, sc.vel, sc.omega)
    A, b, J, e = rigid_assemble(sc, *state)
    res = solve(RigidTopo(sc), A, b, J, e, rho=rho, max_iters=max_iters, tol=tol, z0=z0, u0=u0,
                contact_model=contact_model,
                n_threads=n_threads)
    new = rigid_advance(sc, res.v_hat, *state)
    return new, res


def mlp_param_count(widths):
    return int(sum(widths[k + 1] * widths[k] + widths[k + 1] for k in range(len(widths) - 1)))


def mlp_forward(widths, params, x):
    """Warm-start network forward pass in FP64 (ReLU hidden layers, linear output)."""
    widths = _i32(widths)
    x = _f64(x)
    batch = x.shape[0]
    out = np.zeros((batch, int(widths[-1])))
    rc = lib().oracle_mlp_forward(len(widths) - 1, widths, _f64(params), batch, x.reshape(-1), out.reshape(-1))
    if rc != 0:
        raise RuntimeError("oracle_mlp_forward failed")
    return out


def mlp_backward(widths, params, x, target, wt=None):
    """(loss, gradient) of 0.5 * sum wt (out - target)^2 in FP64."""
    widths = _i32(widths)
    x, target = _f64(x), _f64(target)
    wt = np.ones_like(target) if wt is None else _f64(wt)
    grad = np.zeros(mlp_param_count(widths))
    loss = C.c_double(0.0)
    rc = lib().oracle_mlp_backward(len(widths) - 1, widths, _f64(params), x.shape[0], x.reshape(-1),
                                   target.reshape(-1), wt.reshape(-1), grad, C.byref(loss))
    if rc != 0:
        raise RuntimeError("oracle_mlp_backward failed")
    return loss.value, grad


def fem_assemble(fs, pos=None, vel=None):
    """Eq. (2) with co-rotated elastic blocks (FemScenes): (A, b, J, e) at the given (or
    stored) state."""
    pos = _f64(fs.pos if pos is None else pos).reshape(-1)
    vel = _f64(fs.vel if vel is None else vel).reshape(-1)
    sub_ndof = _i32(fs.sub_ndof)
    nA, nJ, nslot, nrow = layout_sizes(sub_ndof, fs.if_dim, fs.if_nsub, fs.if_sub)
    A, b, J, e = np.zeros(nA), np.zeros(int(sub_ndof.sum())), np.zeros(nJ), np.zeros(nrow)
    rc = lib().oracle_fem_assemble(
        fs.n_sub, _i32(fs.sub_nodes), fs.n_tets, _i32(fs.tets.reshape(-1)), _i32(fs.tet_sub),
        _f64(fs.rest.reshape(-1)), pos, vel, _f64(fs.young), _f64(fs.poisson), float(fs.density),
        fs.n_if, _i32(fs.if_kind), _i32(fs.if_dim), _i32(fs.if_nsub), _i32(fs.if_sub.reshape(-1)),
        _i32(fs.if_node.reshape(-1)), float(fs.dt), float(fs.gravity), float(fs.baumgarte), A, b, J, e)
    if rc != 0:
        raise RuntimeError(f"oracle_fem_assemble failed with code {rc}")
    return A, b, J, e


def fem_element(X, x, young, poisson):
    """One tetrahedron: (12x12 co-rotated stiffness, 12 elastic forces)."""
    K, f = np.zeros(144), np.zeros(12)
    rc = lib().oracle_fem_element(_f64(X).reshape(-1), _f64(x).reshape(-1), float(young), float(poisson), K, f)
    if rc != 0:
        raise RuntimeError("oracle_fem_element failed")
    return K.reshape(12, 12), f


def polar(F):
    R = np.zeros(9)
    if lib().oracle_polar(_f64(F).reshape(-1), R) != 0:
        raise RuntimeError("oracle_polar failed")
    return R.reshape(3, 3)


def fem_advance(fs, v_hat, pos=None, vel=None):
    pos = _f64(fs.pos if pos is None else pos).reshape(-1)
    vel = _f64(fs.vel if vel is None else vel).reshape(-1)
    po, vo = np.zeros_like(pos), np.zeros_like(vel)
    lib().oracle_fem_advance(fs.n_nodes, _f64(v_hat), float(fs.dt), pos, vel, po, vo)
    return po.reshape(-1, 3), vo.reshape(-1, 3)


def fem_step(fs, rho=0.0, max_iters=1000, tol=1e-6, z0=None, u0=None, n_threads=1, state=None, contact_model=0):
    """One whole step of Algorithm 1 on FEM blocks: assemble, solve, advance.
    Returns ((pos, vel), SolveResult)."""
    pos, vel = (fs.pos, fs.vel) if state is None else state
    A, b, J, e = fem_assemble(fs, pos, vel)
    res = solve(RigidTopo(fs), A, b, J, e, rho=rho, max_iters=max_iters, tol=tol, z0=z0, u0=u0,
                contact_model=contact_model,
                n_threads=n_threads)
    return fem_advance(fs, res.v_hat, pos, vel), res
