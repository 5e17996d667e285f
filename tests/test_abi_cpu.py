"""Host-side checks of the C-ABI library that need no GPU: the shared library loads,
exports every function the public header declares, and setup validates descriptors."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2302_14344_amd import _lib as L
from paper_2302_14344_amd import scenes as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(subadmm_[a-z0-9_]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    declared = _declared_functions()
    assert declared, "no declarations found"
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert declared == set(L.EXPORTS)


def _setup(subs, ifs, rho=0.0, dtype=L.F32):
    sa = (L.Subsystem * max(1, len(subs)))()
    for i, (n, s) in enumerate(subs):
        sa[i].n_dof, sa[i].scene = n, s
    ia = (L.Interface * max(1, len(ifs)))()
    for j, f in enumerate(ifs):
        k, d, ns, a, b, mu = f[:6]
        ia[j].kind, ia[j].dim, ia[j].n_sub = k, d, ns
        ia[j].sub[0], ia[j].sub[1] = a, b
        ia[j].mu = mu
        if len(f) > 6:  # soft interfaces: gain and alpha
            ia[j].k, ia[j].alpha = f[6], f[7]
    h = C.c_void_p()
    rc = L.lib().subadmm_setup(sa, len(subs), ia, len(ifs), rho, dtype, C.byref(h))
    return rc, h


def test_setup_and_sizes_match_layout():
    p = S.random_assembled(5, n_scenes=3)
    subs = [(int(n), int(s)) for n, s in zip(p.sub_ndof, p.sub_scene)]
    ifs = [(int(p.if_kind[j]), int(p.if_dim[j]), int(p.if_nsub[j]), int(p.if_sub[j, 0]), int(p.if_sub[j, 1]),
            float(p.if_mu[j])) for j in range(p.n_if)]
    rc, h = _setup(subs, ifs)
    assert rc == 0
    sz = L.Sizes()
    assert L.lib().subadmm_get_sizes(h, C.byref(sz)) == 0
    nc = S.slot_counts(p.sub_ndof, p.if_dim, p.if_nsub, p.if_sub)
    assert sz.n_dof == p.sub_ndof.sum() and sz.n_slot == nc.sum() and sz.n_rows == p.if_dim.sum()
    assert sz.n_A == (p.sub_ndof.astype(int) ** 2).sum() and sz.n_J == (nc * p.sub_ndof).sum()
    assert sz.n_scene == 3 and sz.n_sub == p.n_sub and sz.n_if == p.n_if
    assert L.lib().subadmm_workspace_bytes(h) > 0
    # solving before binding is refused
    rc = L.lib().subadmm_solve(h, None, None, None, None, 10, 1e-6, 0, None, None, None, None, None, None)
    assert rc == L.E_WORKSPACE
    L.lib().subadmm_destroy(h)


@pytest.mark.parametrize("subs,ifs,why", [
    ([(0, 0)], [], "n_dof 0"),
    ([(769, 0)], [], "n_dof above 768"),
    ([(6, 1)], [], "scenes must start at 0"),
    ([(6, 0), (6, 2)], [], "scene gap"),
    ([(6, 0)], [(1, 2, 1, 0, -1, 0.5)], "contact dim 2"),
    ([(6, 0)], [(0, 7, 1, 0, -1, 0.0)], "dim 7"),
    ([(6, 0)], [(5, 1, 1, 0, -1, 0.0)], "unknown kind"),
    ([(6, 0)], [(3, 1, 1, 0, -1, 0.0, 1.0, 0.0)], "soft alpha 0"),
    ([(6, 0)], [(3, 1, 1, 0, -1, 0.0, -1.0, 0.5)], "soft gain negative"),
    ([(6, 0)], [(3, 1, 1, 0, -1, 0.0, float("inf"), 0.5)], "soft gain infinite"),
    ([(6, 0), (6, 0)], [(0, 1, 2, 0, 0, 0.0)], "same member twice"),
    ([(6, 0), (6, 1)], [(0, 1, 2, 0, 1, 0.0)], "members in different scenes"),
    ([(6, 0)], [(0, 1, 1, 3, -1, 0.0)], "member out of range"),
    ([(6, 0)], [(1, 3, 1, 0, -1, -0.1)], "negative mu"),
    ([(6, 0), (6, 1)], [(0, 1, 1, 1, -1, 0.0), (0, 1, 1, 0, -1, 0.0)], "interfaces out of scene order"),
])
def test_setup_rejects_bad_descriptors(subs, ifs, why):
    rc, h = _setup(subs, ifs)
    assert rc == L.E_ARG, why
    assert not h.value
    assert L.lib().subadmm_last_error(None)


def test_rigid_soft_interfaces_come_from_links():
    assert _setup([(6, 0)], [(3, 2, 1, 0, -1, 0.0, 1.5, 0.5)])[0] == 0
    sc = S.chain_scene(S.config_seed(1))
    subs = [(int(n), int(s)) for n, s in zip(sc.sub_ndof, sc.sub_scene)]
    ifs = [(int(sc.if_kind[j]), int(sc.if_dim[j]), int(sc.if_nsub[j]), int(sc.if_sub[j, 0]), int(sc.if_sub[j, 1]),
            float(sc.if_mu[j])) for j in range(sc.n_if)]
    ifs[0] = (3,) + ifs[0][1:] + (1.0, 0.5)
    rc, h = _setup(subs, ifs, dtype=L.F64)
    assert rc == 0
    a = lambda x, t: np.ascontiguousarray(x, t)
    arrs = [a(sc.body_sub, np.int32), a(sc.body_local, np.int32), a(sc.mass, np.float64),
            a(sc.inertia.reshape(-1), np.float64), a(sc.joint_body.reshape(-1), np.int32),
            a(sc.joint_anchor.reshape(-1), np.float64), a(sc.joint_frame_a.reshape(-1), np.float64),
            a(sc.joint_axis_b.reshape(-1), np.float64), a(sc.joint_if, np.int32), a(sc.contact_body, np.int32),
            a(sc.contact_point.reshape(-1), np.float64), a(sc.contact_if, np.int32)]
    ptr = lambda x: x.ctypes.data_as(L.i32p if x.dtype == np.int32 else L.f64p)
    rc = L.lib().subadmm_rigid_set_model(h, sc.n_bodies, ptr(arrs[0]), ptr(arrs[1]), ptr(arrs[2]), ptr(arrs[3]),
                                         len(sc.joint_if), ptr(arrs[4]), ptr(arrs[5]), ptr(arrs[6]), ptr(arrs[7]),
                                         ptr(arrs[8]), len(sc.contact_if), ptr(arrs[9]), ptr(arrs[10]),
                                         ptr(arrs[11]), sc.gravity, sc.baumgarte)
    assert rc == L.E_ARG  # a joint cannot produce a soft interface
    L.lib().subadmm_destroy(h)
    # the cable's soft couplings, ball joints, no-slip rows and contacts: links before the model
    sc = S.cable_scene(seed=S.config_seed(6, 5), n_segments=8, seg_per_sub=4)
    subs = [(int(n), int(s)) for n, s in zip(sc.sub_ndof, sc.sub_scene)]
    ifs = [(int(sc.if_kind[j]), int(sc.if_dim[j]), int(sc.if_nsub[j]), int(sc.if_sub[j, 0]), int(sc.if_sub[j, 1]),
            float(sc.if_mu[j]), float(sc.if_k[j]), float(sc.if_alpha[j])) for j in range(sc.n_if)]
    rc, h = _setup(subs, ifs, dtype=L.F64)
    assert rc == 0
    lk = [a(sc.link_type, np.int32), a(sc.link_body.reshape(-1), np.int32), a(sc.link_anchor.reshape(-1), np.float64),
          a(sc.link_frame.reshape(-1), np.float64), a(sc.link_if, np.int32), a(sc.link_dim, np.int32),
          a(sc.link_k, np.float64), a(sc.link_alpha, np.float64)]
    assert L.lib().subadmm_rigid_set_links(h, len(sc.link_type), *[ptr(x) for x in lk]) == 0
    arrs = [a(sc.body_sub, np.int32), a(sc.body_local, np.int32), a(sc.mass, np.float64),
            a(sc.inertia.reshape(-1), np.float64), a(np.zeros(0), np.int32), a(np.zeros(0), np.float64),
            a(np.zeros(0), np.float64), a(np.zeros(0), np.float64), a(np.zeros(0), np.int32),
            a(sc.contact_body, np.int32), a(sc.contact_point.reshape(-1), np.float64), a(sc.contact_if, np.int32)]
    rc = L.lib().subadmm_rigid_set_model(h, sc.n_bodies, ptr(arrs[0]), ptr(arrs[1]), ptr(arrs[2]), ptr(arrs[3]),
                                         0, None, None, None, None, None, len(sc.contact_if), ptr(arrs[9]),
                                         ptr(arrs[10]), ptr(arrs[11]), sc.gravity, sc.baumgarte)
    assert rc == 0, L.lib().subadmm_last_error(h)
    assert L.lib().subadmm_workspace_bytes(h) > 0
    # a link whose members do not match its bodies' subsystems is refused by the model
    rc2, h2 = _setup(subs, ifs, dtype=L.F64)
    bad = lk[1].copy()
    bad[0] = int(np.nonzero(sc.body_sub == sc.body_sub[-1])[0][0])  # a base body for a coupling
    assert L.lib().subadmm_rigid_set_links(h2, len(sc.link_type), ptr(lk[0]), ptr(bad), ptr(lk[2]), ptr(lk[3]),
                                           ptr(lk[4]), None, None, None) == 0
    rc = L.lib().subadmm_rigid_set_model(h2, sc.n_bodies, ptr(arrs[0]), ptr(arrs[1]), ptr(arrs[2]), ptr(arrs[3]),
                                         0, None, None, None, None, None, len(sc.contact_if), ptr(arrs[9]),
                                         ptr(arrs[10]), ptr(arrs[11]), sc.gravity, sc.baumgarte)
    assert rc == L.E_ARG and b"link" in L.lib().subadmm_last_error(h2)
    L.lib().subadmm_destroy(h)
    L.lib().subadmm_destroy(h2)


def test_rigid_folded_soft_links_are_checked():
    """Soft links inside one subsystem folded into its dynamics (link_if -1): accepted with
    their rows, k and alpha; refused across subsystems, with alpha <= 0, or without dims."""
    a = np.ascontiguousarray
    ptr = lambda x: None if x is None else x.ctypes.data_as(L.i32p if x.dtype == np.int32 else L.f64p)
    sc = S.cable_scene(seed=S.config_seed(6, 5), n_segments=8, seg_per_sub=4, fold_soft=True)
    assert np.sum(sc.link_if < 0) == 2 * 3 * 4
    subs = [(int(n), int(s)) for n, s in zip(sc.sub_ndof, sc.sub_scene)]
    ifs = [(int(sc.if_kind[j]), int(sc.if_dim[j]), int(sc.if_nsub[j]), int(sc.if_sub[j, 0]), int(sc.if_sub[j, 1]),
            float(sc.if_mu[j]), float(sc.if_k[j]), float(sc.if_alpha[j])) for j in range(sc.n_if)]
    base = [a(sc.link_type, np.int32), a(sc.link_body.reshape(-1), np.int32),
            a(sc.link_anchor.reshape(-1), np.float64), a(sc.link_frame.reshape(-1), np.float64),
            a(sc.link_if, np.int32), a(sc.link_dim, np.int32), a(sc.link_k, np.float64), a(sc.link_alpha, np.float64)]
    arrs = [a(sc.body_sub, np.int32), a(sc.body_local, np.int32), a(sc.mass, np.float64),
            a(sc.inertia.reshape(-1), np.float64), a(sc.contact_body, np.int32), a(sc.contact_point.reshape(-1),
                                                                                    np.float64),
            a(sc.contact_if, np.int32)]

    def attempt(lk):
        rc, h = _setup(subs, ifs, dtype=L.F64)
        assert rc == 0
        rc = L.lib().subadmm_rigid_set_links(h, len(sc.link_type), *[ptr(x) for x in lk])
        if rc == 0:
            rc = L.lib().subadmm_rigid_set_model(h, sc.n_bodies, ptr(arrs[0]), ptr(arrs[1]), ptr(arrs[2]),
                                                 ptr(arrs[3]), 0, None, None, None, None, None, len(sc.contact_if),
                                                 ptr(arrs[4]), ptr(arrs[5]), ptr(arrs[6]), sc.gravity, sc.baumgarte)
        msg = L.lib().subadmm_last_error(h)
        L.lib().subadmm_destroy(h)
        return rc, msg

    assert attempt(base)[0] == 0
    q = int(np.nonzero(sc.link_if < 0)[0][0])
    bad_alpha = list(base)
    bad_alpha[7] = base[7].copy()
    bad_alpha[7][q] = 0.0
    assert attempt(bad_alpha)[0] == L.E_ARG
    no_dims = list(base)
    no_dims[5] = None
    assert attempt(no_dims)[0] == L.E_ARG
    across = list(base)
    across[1] = base[1].copy()
    across[1][2 * q + 1] = int(np.nonzero(sc.body_sub != sc.body_sub[base[1][2 * q]])[0][0])
    rc, msg = attempt(across)
    assert rc == L.E_ARG and b"folded" in msg


def test_setup_rejects_bad_dtype_and_rho():
    assert _setup([(6, 0)], [], dtype=7)[0] == L.E_ARG
    assert _setup([(6, 0)], [], rho=float("nan"))[0] == L.E_ARG


def test_rigid_model_validation():
    sc = S.chain_scene(S.config_seed(1))
    subs = [(int(n), int(s)) for n, s in zip(sc.sub_ndof, sc.sub_scene)]
    ifs = [(int(sc.if_kind[j]), int(sc.if_dim[j]), int(sc.if_nsub[j]), int(sc.if_sub[j, 0]), int(sc.if_sub[j, 1]),
            float(sc.if_mu[j])) for j in range(sc.n_if)]
    rc, h = _setup(subs, ifs, dtype=L.F64)
    assert rc == 0

    def call(body_local=sc.body_local, mass=sc.mass, joint_if=sc.joint_if):
        a = lambda x, t: np.ascontiguousarray(x, t)
        arrs = [a(sc.body_sub, np.int32), a(body_local, np.int32), a(mass, np.float64),
                a(sc.inertia.reshape(-1), np.float64), a(sc.joint_body.reshape(-1), np.int32),
                a(sc.joint_anchor.reshape(-1), np.float64), a(sc.joint_frame_a.reshape(-1), np.float64),
                a(sc.joint_axis_b.reshape(-1), np.float64), a(joint_if, np.int32), a(sc.contact_body, np.int32),
                a(sc.contact_point.reshape(-1), np.float64), a(sc.contact_if, np.int32)]
        ptr = lambda x: x.ctypes.data_as(L.i32p if x.dtype == np.int32 else L.f64p)
        q = [ptr(x) for x in arrs]
        return L.lib().subadmm_rigid_set_model(h, sc.n_bodies, q[0], q[1], q[2], q[3], len(sc.joint_body), q[4], q[5],
                                                q[6], q[7], q[8], len(sc.contact_body), q[9], q[10], q[11], 9.81, 0.2)

    assert call() == 0
    bad_local = sc.body_local.copy()
    bad_local[0] = bad_local[1]
    assert call(body_local=bad_local) == L.E_ARG
    bad_mass = sc.mass.copy()
    bad_mass[2] = -1.0
    assert call(mass=bad_mass) == L.E_ARG
    bad_if = sc.joint_if.copy()
    bad_if[0] = sc.contact_if[0]
    assert call(joint_if=bad_if) == L.E_ARG
    L.lib().subadmm_destroy(h)


def test_set_option_validates_values():
    """Every option takes its documented values only (host logic, no device call)."""
    rc, h = _setup([(6, 0)], [(1, 3, 1, 0, -1, 0.5)])
    assert rc == 0
    lib = L.lib()
    assert lib.subadmm_set_option(h, L.OPT_TEAM_KERNEL, 2) == 0  # wave form: one small scene fits
    assert lib.subadmm_set_option(h, L.OPT_TEAM_KERNEL, 3) == L.E_ARG
    for opt in (L.OPT_FACTOR_FP64, L.OPT_FACTOR_STREAMS, L.OPT_FEM_RESIDENT, L.OPT_CONTACT_MODEL,
                L.OPT_BOYD_RESIDUALS):
        assert lib.subadmm_set_option(h, opt, 0) == 0
        assert lib.subadmm_set_option(h, opt, 1) == 0
        assert lib.subadmm_set_option(h, opt, 2) == L.E_ARG
        assert lib.subadmm_set_option(h, opt, -1) == L.E_ARG
    for opt in (L.OPT_SPLIT_ROWS, L.OPT_LARGE_PATH):
        for v in (0, 1, 2):
            assert lib.subadmm_set_option(h, opt, v) == 0
        assert lib.subadmm_set_option(h, opt, 3) == L.E_ARG
        assert lib.subadmm_set_option(h, opt, -1) == L.E_ARG
    assert lib.subadmm_set_option(h, L.OPT_LEARNED_BUDGET, 300) == 0
    assert lib.subadmm_set_option(h, L.OPT_LEARNED_BUDGET, -5) == L.E_ARG
    for v in (0, 1):
        assert lib.subadmm_set_option(h, L.OPT_IMPULSE_OUTPUT, v) == 0
    assert lib.subadmm_set_option(h, L.OPT_IMPULSE_OUTPUT, 2) == L.E_ARG
    for v in (0, 1, 10000):
        assert lib.subadmm_set_option(h, L.OPT_FEM_KAPPA_MAX, v) == 0
    assert lib.subadmm_set_option(h, L.OPT_FEM_KAPPA_MAX, -1) == L.E_ARG
    assert lib.subadmm_set_option(h, 99, 0) == L.E_ARG
    # the per-block precision record exists only after a FEM factorisation
    assert lib.subadmm_fem_block_precision(h, None, None) in (L.E_STATE, L.E_WORKSPACE, L.E_ARG)
    lib.subadmm_destroy(h)


def _setup_members(subs, members, kind=0, dim=2):
    """One interface per entry of ``members`` (a list of member lists)."""
    sa = (L.Subsystem * len(subs))()
    for i, (n, s) in enumerate(subs):
        sa[i].n_dof, sa[i].scene = n, s
    ia = (L.Interface * max(1, len(members)))()
    for j, mem in enumerate(members):
        ia[j].kind, ia[j].dim, ia[j].n_sub = kind, dim, len(mem)
        for m, i in enumerate(mem[:L.MAX_MEMBERS]):
            ia[j].sub[m] = i
    h = C.c_void_p()
    rc = L.lib().subadmm_setup(sa, len(subs), ia, len(members), 0.0, L.F64, C.byref(h))
    return rc, h


def test_setup_multi_member_interfaces():
    """Interfaces of up to four distinct members of one scene are accepted, with one slot
    block per member; five members, a repeated member or members of two scenes are not; the
    team and wave iteration forms refuse problems with such interfaces."""
    subs = [(4, 0), (3, 0), (5, 0), (2, 0), (6, 1)]
    rc, h = _setup_members(subs, [[0, 1, 2], [1, 2, 3, 0], [3]])
    assert rc == 0
    sz = L.Sizes()
    assert L.lib().subadmm_get_sizes(h, C.byref(sz)) == 0
    assert sz.n_slot == 2 * 3 + 2 * 4 + 2 and sz.n_rows == 6
    assert sz.max_slot_sub == 4 and sz.n_J == 2 * (2 * 4 + 2 * 3 + 2 * 5 + 2 * 2)
    assert L.lib().subadmm_set_option(h, L.OPT_TEAM_KERNEL, 1) == L.E_ARG
    assert L.lib().subadmm_set_option(h, L.OPT_TEAM_KERNEL, 0) == 0
    L.lib().subadmm_destroy(h)
    for members in ([[0, 1, 2, 3, 4]], [[0, 1, 1]], [[0, 1, 4]]):
        rc, h = _setup_members(subs, members)
        assert rc == L.E_ARG, members


def test_large_subsystems_plan_device_memory_factorisation():
    """Subsystems up to 512 DOF set up; those whose FP64 factorisation arrays exceed the LDS
    get device-memory arrays in the workspace (host logic, no device call)."""
    lib = L.lib()
    lib.subadmm_workspace_bytes.restype = C.c_size_t
    rc, h0 = _setup([(300, 0), (8, 0)], [(0, 6, 2, 0, 1, 0.0)])
    assert rc == 0
    rc, h1 = _setup([(30, 0), (8, 0)], [(0, 6, 2, 0, 1, 0.0)])
    assert rc == 0
    ld = 301
    fb = 8 * (ld * 300 + ld * 7 + 600)  # K, J and the 7 right-hand sides, two n-vectors
    assert lib.subadmm_workspace_bytes(h0) - lib.subadmm_workspace_bytes(h1) >= fb
    # beyond 512 DOF the per-subsystem solver is refused at solve time, not at setup
    rc, h2 = _setup([(513, 0)], [(0, 3, 1, 0, -1, 0.0)])
    assert rc == 0
    for h in (h0, h1, h2):
        lib.subadmm_destroy(h)
