"""Python front end of the HIP subsystem-ADMM library.

PyTorch supplies device memory (the workspace and all arrays) and the stream; every
computation runs in libsubadmm's kernels, called through the C ABI.  There is no CPU
fallback: without a GPU or without the built library these classes raise.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(L.i32p)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(L.f64p)


class Problem:
    """One set of scenes with fixed topology (subsystems + interfaces).

    Parameters mirror ``subadmm_setup``: per-subsystem DOF and scene, per-interface kind,
    dimension, members and friction coefficient, the penalty ``rho`` (<= 0: Eq. (23)),
    and the arithmetic type (torch.float32 or torch.float64).
    """

    def __init__(self, sub_ndof, sub_scene, if_kind, if_dim, if_nsub, if_sub, if_mu, rho=0.0,
                 dtype=torch.float32, device="cuda", rigid=None, fem=None, factor_fp64=True, team_kernel=False,
                 if_k=None, if_alpha=None):
        if dtype not in (torch.float32, torch.float64):
            raise ValueError("dtype must be torch.float32 or torch.float64")
        self.dtype = dtype
        self.device = torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("the HIP library runs on a GPU device only")
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        lib = L.lib()
        ns = len(sub_ndof)
        subs = (L.Subsystem * max(ns, 1))()
        for i in range(ns):
            subs[i].n_dof = int(sub_ndof[i])
            subs[i].scene = int(sub_scene[i])
        ni = len(if_kind)
        ifs = (L.Interface * max(ni, 1))()
        if_sub = np.asarray(if_sub).reshape(ni, -1) if ni else np.zeros((0, 2), np.int32)
        if if_sub.shape[1] > L.MAX_MEMBERS:
            raise ValueError("an interface has at most four members")
        for j in range(ni):
            ifs[j].kind = int(if_kind[j])
            ifs[j].dim = int(if_dim[j])
            ifs[j].n_sub = int(if_nsub[j])
            for m in range(L.MAX_MEMBERS):
                ifs[j].sub[m] = int(if_sub[j, m]) if m < if_sub.shape[1] else -1
            ifs[j].mu = float(if_mu[j])
            ifs[j].k = float(if_k[j]) if if_k is not None else 0.0
            ifs[j].alpha = float(if_alpha[j]) if if_alpha is not None else 0.0
        h = C.c_void_p()
        L.check(lib.subadmm_setup(subs, ns, ifs, ni, float(rho), L.F64 if dtype == torch.float64 else L.F32,
                                  C.byref(h)))
        self._h = h
        L.check(lib.subadmm_set_option(h, L.OPT_FACTOR_FP64, 1 if factor_fp64 else 0), h)
        L.check(lib.subadmm_set_option(h, L.OPT_TEAM_KERNEL, int(team_kernel)), h)  # False/True/2
        if rigid is not None:
            self._set_rigid(rigid)
        if fem is not None:
            self._set_fem(fem)
        sz = L.Sizes()
        L.check(lib.subadmm_get_sizes(h, C.byref(sz)), h)
        self.sizes = sz
        nbytes = int(lib.subadmm_workspace_bytes(h))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        L.check(lib.subadmm_bind(h, _ptr(self.workspace), nbytes, C.c_void_p(self.stream.cuda_stream)), h)

    # -- construction helpers -----------------------------------------------------------
    @classmethod
    def from_assembled(cls, p, rho=0.0, dtype=torch.float32, device="cuda", **kw):
        return cls(p.sub_ndof, p.sub_scene, p.if_kind, p.if_dim, p.if_nsub, p.if_sub, p.if_mu, rho=rho,
                   dtype=dtype, device=device, if_k=getattr(p, "if_k", None), if_alpha=getattr(p, "if_alpha", None),
                   **kw)

    @classmethod
    def from_rigid(cls, sc, rho=0.0, dtype=torch.float32, device="cuda", **kw):
        return cls(sc.sub_ndof, sc.sub_scene, sc.if_kind, sc.if_dim, sc.if_nsub, sc.if_sub, sc.if_mu, rho=rho,
                   dtype=dtype, device=device, rigid=sc, if_k=getattr(sc, "if_k", None),
                   if_alpha=getattr(sc, "if_alpha", None), **kw)

    @classmethod
    def from_fem(cls, fs, rho=0.0, dtype=torch.float32, device="cuda", **kw):
        return cls(fs.sub_ndof, fs.sub_scene, fs.if_kind, fs.if_dim, fs.if_nsub, fs.if_sub, fs.if_mu, rho=rho,
                   dtype=dtype, device=device, fem=fs, **kw)

    def _set_fem(self, fs):
        rest = _f64(fs.rest.reshape(-1))
        tets = _i32(fs.tets.reshape(-1))
        young, poisson = _f64(fs.young), _f64(fs.poisson)
        ifn = _i32(fs.if_node.reshape(-1) if fs.n_if else np.zeros(2))
        L.check(L.lib().subadmm_fem_set_model(self._h, fs.n_nodes, rest[1], fs.n_tets, tets[1], young[1], poisson[1],
                                              float(fs.density), ifn[1], float(fs.gravity), float(fs.baumgarte)),
                self._h)
        self.dt = float(fs.dt)
        self.n_nodes = fs.n_nodes

    def fem_assemble(self, pos, vel, dt=None):
        sz = self.sizes
        dt = self.dt if dt is None else dt
        A, b, J, e = self.empty(sz.n_A), self.empty(sz.n_dof), self.empty(sz.n_J), self.empty(sz.n_rows)
        L.check(L.lib().subadmm_fem_assemble(self._h, _ptr(pos), _ptr(vel), float(dt), _ptr(A), _ptr(b), _ptr(J),
                                             _ptr(e)), self._h)
        return A, b, J, e

    def fem_step(self, pos, vel, dt=None, max_iters=5000, tol=1e-6, warm="prev", v_hat=None, lam=None, graph=False):
        """One FEM time step; updates pos and vel (flat, n_nodes x 3) in place.  ``graph``:
        replay the step from a HIP graph captured on the first call with these arguments."""
        dt = self.dt if dt is None else dt
        mode = {"cold": L.WARM_COLD, "prev": L.WARM_PREV}[warm]
        for t, name in ((pos, "pos"), (vel, "vel")):
            self._check_arr(t, 3 * self.n_nodes, name)
        fn = L.lib().subadmm_fem_step_graph if graph else L.lib().subadmm_fem_step
        L.check(fn(self._h, _ptr(pos), _ptr(vel), float(dt), int(max_iters), float(tol), mode, _ptr(v_hat), _ptr(lam)),
                self._h)

    def _set_rigid(self, sc):
        nl = len(getattr(sc, "link_type", ()))
        if nl:
            lk = [_i32(sc.link_type), _i32(sc.link_body.reshape(-1)), _f64(sc.link_anchor.reshape(-1)),
                  _f64(sc.link_frame.reshape(-1)), _i32(sc.link_if), _i32(sc.link_dim), _f64(sc.link_k),
                  _f64(sc.link_alpha)]
            L.check(L.lib().subadmm_rigid_set_links(self._h, nl, *[x[1] for x in lk]), self._h)
        keep = [
            _i32(sc.body_sub), _i32(sc.body_local), _f64(sc.mass), _f64(sc.inertia.reshape(-1)),
            _i32(sc.joint_body.reshape(-1)), _f64(sc.joint_anchor.reshape(-1)), _f64(sc.joint_frame_a.reshape(-1)),
            _f64(sc.joint_axis_b.reshape(-1)), _i32(sc.joint_if),
            _i32(sc.contact_body), _f64(sc.contact_point.reshape(-1)), _i32(sc.contact_if),
        ]
        p = [k[1] for k in keep]
        L.check(L.lib().subadmm_rigid_set_model(
            self._h, sc.n_bodies, p[0], p[1], p[2], p[3], len(sc.joint_body), p[4], p[5], p[6], p[7], p[8],
            len(sc.contact_body), p[9], p[10], p[11], float(sc.gravity), float(sc.baumgarte)), self._h)
        self.dt = float(sc.dt)

    def close(self):
        """Waits for the problem's stream and frees the host-side problem (its captured
        graph, side streams and events).  Later calls on this object raise."""
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            torch.cuda.synchronize(self.device)
            L.lib().subadmm_destroy(h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tensors ---------------------------------------------------------------------------
    def tensor(self, x):
        return torch.as_tensor(np.asarray(x), dtype=self.dtype, device=self.device).contiguous()

    def empty(self, n):
        return torch.empty(int(n), dtype=self.dtype, device=self.device)

    def _check_arr(self, t, n, name):
        if t.dtype != self.dtype or t.device != self.device or not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"{name}: expected contiguous {self.dtype} tensor of {n} elements on {self.device}")

    # -- entry points ----------------------------------------------------------------------
    def solve(self, A, b, J, e, max_iters=200, tol=1e-6, warm="cold", z0=None, u0=None):
        """Per-step solve of an assembled problem; returns dict of device tensors."""
        sz = self.sizes
        for t, n, name in ((A, sz.n_A, "A"), (b, sz.n_dof, "b"), (J, sz.n_J, "J"), (e, sz.n_rows, "e")):
            self._check_arr(t, n, name)
        mode = {"cold": L.WARM_COLD, "prev": L.WARM_PREV, "given": L.WARM_GIVEN}[warm]
        if mode == L.WARM_GIVEN:
            self._check_arr(z0, sz.n_slot, "z0")
            self._check_arr(u0, sz.n_slot, "u0")
        out = {"v_hat": self.empty(sz.n_dof), "lam": self.empty(sz.n_rows), "z": self.empty(sz.n_slot),
               "u": self.empty(sz.n_slot)}
        L.check(L.lib().subadmm_solve(self._h, _ptr(A), _ptr(b), _ptr(J), _ptr(e), int(max_iters), float(tol), mode,
                                      _ptr(z0), _ptr(u0), _ptr(out["v_hat"]), _ptr(out["lam"]), _ptr(out["z"]),
                                      _ptr(out["u"])), self._h)
        return out

    def solve_scratch(self, A, b, J, e, max_iters=200, tol=1e-6, warm="cold", z0=None, u0=None, out=None,
                      with_stats=False):
        """``solve`` through ``subadmm_solve_scratch``: the library's static device scratch
        replaces the bound workspace, and the call allocates nothing (``out``: optional
        preallocated dict of the four output tensors).  Returns the outputs, and the
        per-scene statistics list when ``with_stats`` (the call then synchronises)."""
        sz = self.sizes
        for t, n, name in ((A, sz.n_A, "A"), (b, sz.n_dof, "b"), (J, sz.n_J, "J"), (e, sz.n_rows, "e")):
            self._check_arr(t, n, name)
        mode = {"cold": L.WARM_COLD, "given": L.WARM_GIVEN}[warm]
        if mode == L.WARM_GIVEN:
            self._check_arr(z0, sz.n_slot, "z0")
            self._check_arr(u0, sz.n_slot, "u0")
        if out is None:
            out = {"v_hat": self.empty(sz.n_dof), "lam": self.empty(sz.n_rows), "z": self.empty(sz.n_slot),
                   "u": self.empty(sz.n_slot)}
        st = (L.Stats * sz.n_scene)() if with_stats else None
        L.check(L.lib().subadmm_solve_scratch(self._h, C.c_void_p(self.stream.cuda_stream), _ptr(A), _ptr(b), _ptr(J),
                                              _ptr(e), int(max_iters), float(tol), mode, _ptr(z0), _ptr(u0),
                                              _ptr(out["v_hat"]), _ptr(out["lam"]), _ptr(out["z"]), _ptr(out["u"]),
                                              st), self._h)
        if with_stats:
            return out, [(a.iters, a.converged, a.theta, a.r_theta) for a in st]
        return out

    def rigid_assemble(self, pos, rot, vel, omega, dt=None):
        sz = self.sizes
        dt = self.dt if dt is None else dt
        A, b, J, e = self.empty(sz.n_A), self.empty(sz.n_dof), self.empty(sz.n_J), self.empty(sz.n_rows)
        L.check(L.lib().subadmm_rigid_assemble(self._h, _ptr(pos), _ptr(rot), _ptr(vel), _ptr(omega), float(dt),
                                               _ptr(A), _ptr(b), _ptr(J), _ptr(e)), self._h)
        return A, b, J, e

    def rigid_step(self, pos, rot, vel, omega, dt=None, max_iters=1000, tol=1e-6, warm="prev", v_hat=None, lam=None,
                   graph=False):
        """One time step; updates the state tensors in place.  ``warm``: "cold", "prev" or
        "learned" (networks attached with ``set_warm_model``).  ``graph``: replay the step
        from a HIP graph captured on the first call with these tensors."""
        dt = self.dt if dt is None else dt
        mode = {"cold": L.WARM_COLD, "prev": L.WARM_PREV, "learned": L.WARM_LEARNED}[warm]
        nb = pos.numel() // 3
        for t, n, name in ((pos, 3 * nb, "pos"), (rot, 9 * nb, "rot"), (vel, 3 * nb, "vel"), (omega, 3 * nb, "omega")):
            self._check_arr(t, n, name)
        fn = L.lib().subadmm_rigid_step_graph if graph else L.lib().subadmm_rigid_step
        L.check(fn(self._h, _ptr(pos), _ptr(rot), _ptr(vel), _ptr(omega), float(dt), int(max_iters), float(tol), mode,
                   _ptr(v_hat), _ptr(lam)), self._h)

    def rigid_steps(self, pos, rot, vel, omega, n_steps, dt=None, max_iters=1000, tol=1e-6, warm="prev", v_hat=None,
                    lam=None):
        """``n_steps`` time steps in one launch (``subadmm_rigid_steps``): the results of
        ``n_steps`` calls of ``rigid_step`` with ``warm`` "cold" or "prev", each scene carried
        through its steps without waiting for the others."""
        dt = self.dt if dt is None else dt
        mode = {"cold": L.WARM_COLD, "prev": L.WARM_PREV}[warm]
        nb = pos.numel() // 3
        for t, n, name in ((pos, 3 * nb, "pos"), (rot, 9 * nb, "rot"), (vel, 3 * nb, "vel"), (omega, 3 * nb, "omega")):
            self._check_arr(t, n, name)
        L.check(L.lib().subadmm_rigid_steps(self._h, _ptr(pos), _ptr(rot), _ptr(vel), _ptr(omega), float(dt),
                                            int(n_steps), int(max_iters), float(tol), mode, _ptr(v_hat), _ptr(lam)),
                self._h)

    def set_scene_order(self, order=None):
        """Scene of each workgroup of the multi-step launch (a permutation; None: identity)."""
        if order is None:
            L.check(L.lib().subadmm_set_scene_order(self._h, None), self._h)
            return
        a, ap = _i32(order)
        L.check(L.lib().subadmm_set_scene_order(self._h, ap), self._h)

    def constraint_error(self, v_hat, lam, J=None, e=None, kinds=15):
        """Per-scene constraint error of a step's (v_hat, lambda) (subadmm_constraint_error): J, e
        of an assembled problem, or None for those of the model's last step; ``kinds``: mask
        of interface kinds (L.ERR_LAWS, L.ERR_SOFT, or 15 for all)."""
        out = np.zeros(self.sizes.n_scene)
        L.check(L.lib().subadmm_constraint_error(self._h, _ptr(J), _ptr(e), _ptr(v_hat), _ptr(lam), int(kinds),
                                                 out.ctypes.data_as(L.f64p)), self._h)
        return out

    def stats(self):
        n = self.sizes.n_scene
        arr = (L.Stats * n)()
        L.check(L.lib().subadmm_read_stats(self._h, arr), self._h)
        return {"iters": np.array([a.iters for a in arr], np.int32),
                "converged": np.array([a.converged for a in arr], np.int32),
                "theta": np.array([a.theta for a in arr]), "r_theta": np.array([a.r_theta for a in arr]),
                "iters_total": np.array([a.iters_total for a in arr], np.int64),
                "unconverged_total": np.array([a.unconverged_total for a in arr], np.int64),
                "fallback_total": np.array([a.fallback_total for a in arr], np.int64),
                "r_prim": np.array([a.r_prim for a in arr]), "r_dual": np.array([a.r_dual for a in arr])}

    def reset_totals(self):
        L.check(L.lib().subadmm_reset_totals(self._h), self._h)

    def timing_begin(self, max_launches):
        L.check(L.lib().subadmm_timing_begin(self._h, int(max_launches)), self._h)

    def timing_end(self):
        """Summed kernel milliseconds and launch counts per kernel since timing_begin."""
        ms = (C.c_double * L.NUM_KERNELS)()
        cnt = (C.c_int32 * L.NUM_KERNELS)()
        L.check(L.lib().subadmm_timing_end(self._h, ms, cnt), self._h)
        names = ("assemble", "factor", "loop", "advance", "steps", "warm")
        return {n: (float(ms[k]), int(cnt[k])) for k, n in enumerate(names)}

    def beta(self):
        out = self.empty(self.sizes.n_sub)
        L.check(L.lib().subadmm_copy_beta(self._h, _ptr(out)), self._h)
        return out

    def check(self):
        L.check(L.lib().subadmm_check(self._h), self._h)

    def set_fem_resident(self, on=True):
        """FEM iteration form: operators kept on chip for the step (default) or read from
        device memory in every iteration."""
        L.check(L.lib().subadmm_set_option(self._h, L.OPT_FEM_RESIDENT, 1 if on else 0), self._h)

    def set_split_rows(self, on=True):
        """Thread-per-slot-row iteration kernel: rows of subsystems with many slot rows split
        over 2 or 4 lanes (True, the workgroup may grow; "within": inside the default
        workgroup, longest rows first), or one or two lanes per row for the whole scene
        (False, the default)."""
        v = 2 if on == "within" else (1 if on else 0)
        L.check(L.lib().subadmm_set_option(self._h, L.OPT_SPLIT_ROWS, v), self._h)

    def set_contact_model(self, relaxed=False):
        """Contact z-update: exact Signorini-Coulomb projection (default) or the relaxed
        convex model (Euclidean projection onto the friction cone)."""
        L.check(L.lib().subadmm_set_option(self._h, L.OPT_CONTACT_MODEL, 1 if relaxed else 0), self._h)

    def set_large_path(self, on=True):
        """Iterate on the large-scene path even when every scene fits the per-scene kernel:
        True (the form chosen by scene size), "phases" (one launch per phase per iteration),
        or False (the default choice)."""
        v = 2 if on == "phases" else (1 if on else 0)
        L.check(L.lib().subadmm_set_option(self._h, L.OPT_LARGE_PATH, v), self._h)

    def set_boyd_residuals(self, on=True):
        """Form ADMM's primal and dual residuals of the returned iterate after every solve and
        rigid step (``stats()["r_prim"]``, ``["r_dual"]``; NaN when off, the default)."""
        L.check(L.lib().subadmm_set_option(self._h, L.OPT_BOYD_RESIDUALS, 1 if on else 0), self._h)

    def set_impulse_output(self, on=True):
        """lambda output of the steps: the impulse over the step, t lambda (True), or the
        constraint force lambda (False, the default)."""
        L.check(L.lib().subadmm_set_option(self._h, L.OPT_IMPULSE_OUTPUT, 1 if on else 0), self._h)

    def set_fem_kappa_max(self, kmax):
        """Precision of the FEM factorisation (FP32 problems): 0 (default) = FP64 for every
        block; k > 0 = an FP32 trial factorisation of every block, FP64 again for blocks whose
        kappa_est = (max L_rr / min L_rr)^2 exceeds k."""
        L.check(L.lib().subadmm_set_option(self._h, L.OPT_FEM_KAPPA_MAX, int(kmax)), self._h)

    def fem_block_precision(self):
        """(kappa_est, fp64) of the last FEM factorisation, per block: float64 and bool
        tensors on the device (copied on the problem's stream)."""
        k = torch.empty(self.sizes.n_sub, dtype=torch.float64, device=self.device)
        f = torch.empty(self.sizes.n_sub, dtype=torch.int32, device=self.device)
        L.check(L.lib().subadmm_fem_block_precision(self._h, _ptr(k), _ptr(f)), self._h)
        return k, f != 0

    def fem_loop_form(self):
        """Operator tiles per wave kept in registers by the last FEM iteration launch (0:
        streamed from device memory; -1: no step yet)."""
        v = C.c_int32()
        L.check(L.lib().subadmm_fem_loop_form(self._h, C.byref(v)), self._h)
        return v.value

    # -- learned warm start ----------------------------------------------------------------
    def set_learned_budget(self, iters):
        """Iteration budget of the learned-start run (0: max_iters)."""
        L.check(L.lib().subadmm_set_option(self._h, L.OPT_LEARNED_BUDGET, int(iters)), self._h)

    def warm_class_counts(self):
        """(number of contact interfaces, number of dim-5 equality interfaces)."""
        a, b = C.c_int32(), C.c_int32()
        L.check(L.lib().subadmm_warm_class_counts(self._h, C.byref(a), C.byref(b)), self._h)
        return a.value, b.value

    def set_warm_model(self, cls, net):
        """Attach (or detach with None) the network of class 0 (contacts) or 1 (joints)."""
        L.check(L.lib().subadmm_set_warm_model(self._h, int(cls), None if net is None else net._h), self._h)
        if not hasattr(self, "_nets"):
            self._nets = {}
        self._nets[int(cls)] = net

    def set_recording(self, on=True):
        """While on, each rigid step writes its training data to device FP32 tensors:
        ``rec["xc"]`` (n_contact, 12), ``rec["xj"]`` (n_joint, 27) features,
        ``rec["tc"]``/``rec["tj"]`` targets (6 / 15 columns) and ``rec["wc"]``/``rec["wj"]``
        their loss weights.  Returns the dict (None when switched off)."""
        if not on:
            L.check(L.lib().subadmm_set_recording(self._h, None, None, None, None, None, None), self._h)
            self.rec = None
            return None
        nc, nj = self.warm_class_counts()
        z = lambda r, c: torch.zeros((r, c), dtype=torch.float32, device=self.device)
        self.rec = {"xc": z(nc, L.CONTACT_IN), "xj": z(nj, L.JOINT_IN), "tc": z(nc, L.CONTACT_OUT),
                    "tj": z(nj, L.JOINT_OUT), "wc": z(nc, L.CONTACT_OUT), "wj": z(nj, L.JOINT_OUT)}
        r = self.rec
        L.check(L.lib().subadmm_set_recording(self._h, _ptr(r["xc"]), _ptr(r["xj"]), _ptr(r["tc"]), _ptr(r["tj"]),
                                              _ptr(r["wc"]), _ptr(r["wj"])), self._h)
        return self.rec

    def get_warm(self):
        z, u = self.empty(self.sizes.n_slot), self.empty(self.sizes.n_slot)
        L.check(L.lib().subadmm_get_warm(self._h, _ptr(z), _ptr(u)), self._h)
        return z, u

    def set_warm(self, z, u):
        self._check_arr(z, self.sizes.n_slot, "z")
        self._check_arr(u, self.sizes.n_slot, "u")
        L.check(L.lib().subadmm_set_warm(self._h, _ptr(z), _ptr(u)), self._h)


def fem_state_tensors(fs, dtype=torch.float32, device="cuda"):
    """(pos, vel) of a FemScenes batch as flat device tensors."""
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=dtype, device=device).contiguous()
    return f(fs.pos), f(fs.vel)


def rigid_state_tensors(sc, dtype=torch.float32, device="cuda"):
    """(pos, rot, vel, omega) of a RigidScenes batch as flat device tensors."""
    f = lambda a: torch.as_tensor(np.ascontiguousarray(a).reshape(-1), dtype=dtype, device=device).contiguous()
    return f(sc.pos), f(sc.rot), f(sc.vel), f(sc.omega)


class Mlp:
    """Warm-start network on the GPU (subadmm_mlp_*): ReLU perceptron, BF16 matrix-core
    products with FP32 accumulation, FP32 master parameters and Adam."""

    def __init__(self, widths, max_batch, device="cuda"):
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        lib = L.lib()
        self.widths = [int(w) for w in widths]
        wa, wp = _i32(self.widths)
        self._keep = wa
        h = C.c_void_p()
        L.check_mlp(lib.subadmm_mlp_create(len(self.widths) - 1, wp, int(max_batch), C.byref(h)))
        self._h = h
        self.max_batch = int(max_batch)
        self.n_params = int(lib.subadmm_mlp_param_count(h))
        nbytes = int(lib.subadmm_mlp_workspace_bytes(h))
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        L.check_mlp(lib.subadmm_mlp_bind(h, _ptr(self.workspace), nbytes, C.c_void_p(self.stream.cuda_stream)), h)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                torch.cuda.synchronize(self.device)
                L.lib().subadmm_mlp_destroy(h)
            except Exception:
                pass
            self._h = None

    def _f32(self, x, n=None):
        t = torch.as_tensor(x, dtype=torch.float32, device=self.device).contiguous()
        if n is not None and t.numel() != n:
            raise ValueError(f"expected {n} elements, got {t.numel()}")
        return t

    def set_params(self, params):
        p = self._f32(params, self.n_params)
        L.check_mlp(L.lib().subadmm_mlp_set_params(self._h, _ptr(p)), self._h)

    def set_input_affine(self, scale, shift):
        """x <- x * scale + shift per input column (FP32, before the BF16 rounding); None
        switches it off."""
        if scale is None:
            L.check_mlp(L.lib().subadmm_mlp_set_input_affine(self._h, None, None), self._h)
            self._aff = None
            return
        self._aff = (self._f32(scale, self.widths[0]), self._f32(shift, self.widths[0]))
        L.check_mlp(L.lib().subadmm_mlp_set_input_affine(self._h, _ptr(self._aff[0]), _ptr(self._aff[1])), self._h)

    def get_params(self):
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.device)
        L.check_mlp(L.lib().subadmm_mlp_get_params(self._h, _ptr(out)), self._h)
        return out

    def forward(self, x):
        x = self._f32(x)
        batch = x.numel() // self.widths[0]
        y = torch.empty((batch, self.widths[-1]), dtype=torch.float32, device=self.device)
        L.check_mlp(L.lib().subadmm_mlp_forward(self._h, batch, _ptr(x), _ptr(y)), self._h)
        return y

    def backward(self, target, wt=None, want_grad=False):
        t = self._f32(target)
        batch = t.numel() // self.widths[-1]
        w = None if wt is None else self._f32(wt, t.numel())
        grad = torch.empty(self.n_params, dtype=torch.float32, device=self.device) if want_grad else None
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        L.check_mlp(L.lib().subadmm_mlp_backward(self._h, batch, _ptr(t), _ptr(w), _ptr(grad), _ptr(loss)), self._h)
        return loss, grad

    def infer(self, x):
        """Inference-only forward (one fused launch); same output as ``forward``, keeps no
        activations for ``backward``."""
        x = self._f32(x)
        batch = x.numel() // self.widths[0]
        y = torch.empty((batch, self.widths[-1]), dtype=torch.float32, device=self.device)
        L.check_mlp(L.lib().subadmm_mlp_infer(self._h, batch, _ptr(x), _ptr(y)), self._h)
        return y

    def gather_rows(self, src, idx, dst):
        """dst[r] = src[idx[r]] on the network's stream (device FP32 2-D src and dst of one
        width, device int32 idx; rows of out-of-range indices become NaN)."""
        assert src.dtype == torch.float32 and dst.dtype == torch.float32 and idx.dtype == torch.int32
        assert src.is_contiguous() and dst.is_contiguous() and idx.is_contiguous()
        assert src.shape[1] == dst.shape[1] and dst.shape[0] == idx.shape[0]
        L.check_mlp(L.lib().subadmm_mlp_gather_rows(self._h, _ptr(src), int(src.shape[0]), int(src.shape[1]),
                                                    _ptr(idx), int(idx.shape[0]), _ptr(dst)), self._h)

    def adam(self, lr, step, beta1=0.9, beta2=0.999, eps=1e-8):
        L.check_mlp(L.lib().subadmm_mlp_adam(self._h, float(lr), float(beta1), float(beta2), float(eps), int(step)),
                    self._h)
