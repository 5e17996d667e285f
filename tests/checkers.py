"""Independent checkers for the oracle: plain definitions of the per-step result.

These do not call the oracle's arithmetic; they rebuild the whole-system problem of
Eq. (8) from the per-subsystem blocks and solve it directly (monolithic KKT for
equalities, active-set / mode enumeration for contacts).
"""
from __future__ import annotations

import itertools

import numpy as np

KIND_EQUALITY, KIND_CONTACT, KIND_HARD_INEQ = 0, 1, 2


def slot_layout(sub_ndof, if_dim, if_nsub, if_sub):
    """Slot rows: subsystem i lists, for each interface j containing it (ascending j),
    d_j rows.  Returns (dof_off, slot_off, if_slot[j][m], e_off)."""
    ns = len(sub_ndof)
    nc = np.zeros(ns, np.int64)
    width = max([2] + [int(x) for x in if_nsub])
    if_slot = np.zeros((len(if_dim), width), np.int64)
    for j in range(len(if_dim)):
        for m in range(int(if_nsub[j])):
            i = int(if_sub[j][m])
            if_slot[j, m] = nc[i]  # local for now
            nc[i] += int(if_dim[j])
    dof_off = np.concatenate([[0], np.cumsum(sub_ndof)]).astype(np.int64)
    slot_off = np.concatenate([[0], np.cumsum(nc)]).astype(np.int64)
    for j in range(len(if_dim)):
        for m in range(int(if_nsub[j])):
            if_slot[j, m] += slot_off[int(if_sub[j][m])]
    e_off = np.concatenate([[0], np.cumsum(if_dim)]).astype(np.int64)
    return dof_off, slot_off, if_slot, e_off, nc


def global_system(p, A, b, J):
    """Block-diagonal A (Eq. 7) and the global constraint Jacobian whose row r of
    interface j is sum over members of that member's slot row (Eq. 8)."""
    sub_ndof = np.asarray(p.sub_ndof)
    if_sub = np.asarray(p.if_sub).reshape(len(p.if_dim), -1)
    dof_off, slot_off, if_slot, e_off, nc = slot_layout(sub_ndof, p.if_dim, p.if_nsub, if_sub)
    n = int(dof_off[-1])
    Ag = np.zeros((n, n))
    a0 = 0
    j0 = 0
    Jblocks = []
    for i, ni in enumerate(sub_ndof):
        ni = int(ni)
        Ag[dof_off[i]:dof_off[i] + ni, dof_off[i]:dof_off[i] + ni] = A[a0:a0 + ni * ni].reshape(ni, ni)
        a0 += ni * ni
        Jblocks.append(J[j0:j0 + int(nc[i]) * ni].reshape(int(nc[i]), ni))
        j0 += int(nc[i]) * ni
    m = int(e_off[-1])
    Jg = np.zeros((m, n))
    for j in range(len(p.if_dim)):
        for mm in range(int(p.if_nsub[j])):
            i = int(if_sub[j, mm])
            loc = int(if_slot[j, mm] - slot_off[i])
            d = int(p.if_dim[j])
            Jg[e_off[j]:e_off[j] + d, dof_off[i]:dof_off[i] + int(sub_ndof[i])] += Jblocks[i][loc:loc + d]
    return Ag, np.asarray(b, float).copy(), Jg, e_off


def kkt_equality(Ag, bg, Jg, e):
    """Monolithic KKT of Eq. (8) with every row an equality:
    [A -J^T; J 0] [v; lam] = [b; -e]."""
    n, m = Ag.shape[0], Jg.shape[0]
    K = np.zeros((n + m, n + m))
    K[:n, :n] = Ag
    K[:n, n:] = -Jg.T
    K[n:, :n] = Jg
    rhs = np.concatenate([bg, -np.asarray(e, float)])
    sol = np.linalg.solve(K, rhs)
    return sol[:n], sol[n:]


def _solve_with(Ag, bg, Jg, e, eq_rows, zero_rows, extra=()):
    """Solve A v - J^T lam = b with: rows in eq_rows satisfy J v + e = 0, rows in
    zero_rows have lam = 0, plus extra linear relations (list of (coef over lam, 0)) on
    lam.  Every row is in exactly one of eq_rows / zero_rows / extra."""
    n, m = Ag.shape[0], Jg.shape[0]
    K = np.zeros((n + m, n + m))
    rhs = np.zeros(n + m)
    K[:n, :n] = Ag
    K[:n, n:] = -Jg.T
    rhs[:n] = bg
    r = n
    for row in eq_rows:
        K[r, :n] = Jg[row]
        rhs[r] = -e[row]
        r += 1
    for row in zero_rows:
        K[r, n + row] = 1.0
        r += 1
    for coef in extra:
        K[r, n:] = coef
        r += 1
    assert r == n + m
    try:
        sol = np.linalg.solve(K, rhs)
    except np.linalg.LinAlgError:
        return None
    if not np.all(np.isfinite(sol)):
        return None
    return sol[:n], sol[n:]


def enumerate_frictionless(Ag, bg, Jg, e, eq_rows, contacts, tol=1e-9):
    """All solutions of the frictionless problem by 2^m active-set enumeration.

    ``contacts`` is a list of (normal_row, t1_row, t2_row).  Tangential multipliers are
    zero (mu = 0).  A candidate is kept if lam_n >= 0 on active and J_n v + e_n >= 0 on
    inactive contacts.  Returns a list of (v, lam)."""
    sols = []
    for act in itertools.product([0, 1], repeat=len(contacts)):
        eqr = list(eq_rows)
        zr = []
        for (cn, t1, t2), a in zip(contacts, act):
            zr += [t1, t2]
            (eqr if a else zr).append(cn)
        s = _solve_with(Ag, bg, Jg, e, eqr, zr)
        if s is None:
            continue
        v, lam = s
        c = Jg @ v + e
        scale = max(1.0, np.abs(lam).max())
        ok = True
        for (cn, _, _), a in zip(contacts, act):
            if a and lam[cn] < -tol * scale:
                ok = False
            if not a and c[cn] < -tol * max(1.0, np.abs(c).max()):
                ok = False
        if ok:
            sols.append((v, lam))
    return sols


def soft_linear_solve(Ag, bg, Jg, e, eq_rows, soft_rows, k_rows, alpha_rows):
    """The per-step solution with soft rows, Eq. (3): A v - J^T lam = b (Eq. 8), J_r v = -e_r
    on ``eq_rows`` and lam_r = -k_r (e_r + alpha_r J_r v) on ``soft_rows`` (gain and alpha
    per row), one linear system in (v, lam).  Every row is in one of the two lists."""
    n, m = Ag.shape[0], Jg.shape[0]
    K = np.zeros((n + m, n + m))
    rhs = np.zeros(n + m)
    K[:n, :n] = Ag
    K[:n, n:] = -Jg.T
    rhs[:n] = bg
    r = n
    for row in eq_rows:
        K[r, :n] = Jg[row]
        rhs[r] = -e[row]
        r += 1
    for row, k, a in zip(soft_rows, k_rows, alpha_rows):
        K[r, n + row] = 1.0
        K[r, :n] = k * a * Jg[row]
        rhs[r] = -k * e[row]
        r += 1
    assert r == n + m
    sol = np.linalg.solve(K, rhs)
    return sol[:n], sol[n:]


def enumerate_inequalities(Ag, bg, Jg, e, eq_rows, ineq_rows, tol=1e-9):
    """All solutions with 0 <= lam_r _|_ J_r v + e_r >= 0 on every row of ``ineq_rows`` (the
    hard inequality of Eq. (4), row by row) and J v + e = 0 on ``eq_rows``, by 2^m
    active-set enumeration.  Returns a list of (v, lam)."""
    sols = []
    for act in itertools.product([0, 1], repeat=len(ineq_rows)):
        eqr = list(eq_rows)
        zr = []
        for row, a in zip(ineq_rows, act):
            (eqr if a else zr).append(row)
        s = _solve_with(Ag, bg, Jg, e, eqr, zr)
        if s is None:
            continue
        v, lam = s
        c = Jg @ v + e
        ok = True
        for row, a in zip(ineq_rows, act):
            if a and lam[row] < -tol * max(1.0, np.abs(lam).max()):
                ok = False
            if not a and c[row] < -tol * max(1.0, np.abs(c).max()):
                ok = False
        if ok:
            sols.append((v, lam))
    return sols


def enumerate_planar_coulomb(Ag, bg, Jg, e, eq_rows, contacts, mu, tol=1e-9):
    """All Signorini-Coulomb solutions of a problem symmetric about the plane spanned by
    the normal and t1 (t2 velocities vanish by symmetry) by 4^m mode enumeration:
    open, stick, slip with c_t1 > 0 (lam_t1 = -mu lam_n), slip with c_t1 < 0
    (lam_t1 = +mu lam_n).  Returns a list of (v, lam, modes)."""
    m_rows = Jg.shape[0]
    sols = []
    for modes in itertools.product(range(4), repeat=len(contacts)):
        eqr = list(eq_rows)
        zr = []
        extra = []
        for (cn, t1, t2), md, mk in zip(contacts, modes, mu):
            if md == 0:
                zr += [cn, t1, t2]
            elif md == 1:
                eqr += [cn, t1, t2]
            else:
                eqr.append(cn)
                zr.append(t2)
                coef = np.zeros(m_rows)
                coef[t1] = 1.0
                coef[cn] = mk if md == 2 else -mk   # lam_t1 + mu lam_n = 0  or lam_t1 - mu lam_n = 0
                extra.append(coef)
        s = _solve_with(Ag, bg, Jg, e, eqr, zr, extra)
        if s is None:
            continue
        v, lam = s
        c = Jg @ v + e
        lsc = max(1.0, np.abs(lam).max())
        csc = max(1e-12, np.abs(c).max(), np.abs(Jg @ v).max())
        ok = True
        for (cn, t1, t2), md, mk in zip(contacts, modes, mu):
            if md == 0:
                ok &= c[cn] >= -tol * csc
            else:
                ok &= lam[cn] >= -tol * lsc
                ok &= abs(c[t2]) <= 1e-6 * csc
                if md == 1:
                    ok &= abs(lam[t1]) <= mk * lam[cn] + tol * lsc
                elif md == 2:
                    ok &= c[t1] >= -tol * csc
                else:
                    ok &= c[t1] <= tol * csc
        if ok:
            sols.append((v, lam, modes))
    return sols
