"""Subsystems beyond the LDS factorisation (up to 512 DOF) through the assembled solve,
against the FP64 oracle (Alg. 1 with Eq. 15, 23 on each subsystem's dense K = A + beta J^T J).

Subsystems whose factorisation arrays (K, J and the nc + 1 right-hand sides in FP64) exceed the
LDS are factorised with them in device memory; subsystems of 65 to ~128 DOF with few slot rows
stay in the LDS classes with a thread per column.  Bounds as in the other assembled parity
tests: FP64 1e-9 of the largest reference entry, FP32 (FP64 factorisation, FP32 iteration,
FP32-rounded inputs on both sides) 1e-5.

* Random assembled problems with subsystems of 40 to 320 DOF and every interface kind, after 1
  and 40 iterations and under the stopping rule; the no-allocation entry on the same problem
  equals the bound solve bit for bit.
* The FEM lattice's blocks (375 DOF, ~200-300 slot rows each) given as an assembled problem:
  the oracle's (A, b, J, e) of a deformed, moving state solved by the assembled entry (device-
  memory factorisation; the scene's slot rows exceed the per-scene kernel, so the large-scene
  path iterates).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2302_14344_amd import scenes as S

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy().astype(np.float64)


def _r32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _problem(dtype):
    kinds = (S.KIND_EQUALITY, S.KIND_CONTACT, S.KIND_HARD_INEQ, S.KIND_SOFT)
    p = S.random_assembled(131, n_scenes=4, subs_per_scene=(2, 4), ndof=(40, 320), n_if_per_scene=(3, 10),
                           kinds=kinds, eq_dim=(1, 6))
    if dtype == torch.float32:
        for name in ("A", "b", "J", "e", "if_mu", "if_k", "if_alpha"):
            v = getattr(p, name)
            if v is not None:
                setattr(p, name, _r32(v))
    return p


def _big_count(p):
    nc = S.slot_counts(p.sub_ndof, p.if_dim, p.if_nsub, p.if_sub)
    n = np.asarray(p.sub_ndof, np.int64)
    ld = n | 1
    fb = 8 * (ld * n + ld * (nc + 1) + 2 * n)
    return int((fb > 150 * 1024).sum()), int((n > 64).sum())


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_assembled_large_subsystems(dtype):
    from paper_2302_14344_amd.solver import Problem
    p = _problem(dtype)
    big, over64 = _big_count(p)
    print(f"  {len(p.sub_ndof)} subsystems, {over64} above 64 DOF, {big} factorised in device memory", flush=True)
    assert big >= 2 and over64 > big
    pr = Problem.from_assembled(p, dtype=dtype)
    A, b, J, e = (pr.tensor(x) for x in (p.A, p.b, p.J, p.e))
    tol_rel = 1e-9 if dtype == torch.float64 else 1e-5
    for iters, tol in ((1, 0.0), (40, 0.0), (3000, 1e-7)):
        out = pr.solve(A, b, J, e, max_iters=iters, tol=tol)
        st = pr.stats()
        ref = O.solve(p, p.A, p.b, p.J, p.e, max_iters=iters, tol=tol, n_threads=16)
        if tol > 0.0 and dtype == torch.float64:
            np.testing.assert_array_equal(st["iters"], ref.iters)
        if tol > 0.0 and dtype == torch.float32:
            ref = O.solve(p, p.A, p.b, p.J, p.e, max_iters=st["iters"], tol=0.0, n_threads=16)
        ev = np.abs(_np(out["v_hat"]) - ref.v_hat).max() / np.abs(ref.v_hat).max()
        el = np.abs(_np(out["lam"]) - ref.lam).max() / max(1.0, np.abs(ref.lam).max())
        print(f"  {dtype} iters {iters} tol {tol}: v {ev:.2e} lambda {el:.2e}", flush=True)
        assert ev <= tol_rel and el <= tol_rel
    pr.check()
    # the no-allocation entry: the same kernels from the library's static scratch
    o1 = pr.solve(A, b, J, e, max_iters=40, tol=0.0)
    o2 = pr.solve_scratch(A, b, J, e, max_iters=40, tol=0.0)
    for k in ("v_hat", "lam", "z", "u"):
        np.testing.assert_array_equal(_np(o1[k]), _np(o2[k]))


def test_fem_blocks_through_the_assembled_solve():
    from paper_2302_14344_amd.solver import Problem
    fs = S.fem_scene(seed=S.config_seed(3, 12), blocks=(2, 2, 2), nodes_per_block=5)
    rng = np.random.default_rng(5)
    fs = fs.with_state(fs.pos + rng.uniform(-0.02, 0.02, fs.pos.shape) * fs.meta["h"],
                       rng.normal(0, 0.05, fs.pos.shape))
    A, b, J, e = O.fem_assemble(fs)
    p = S.AssembledProblem(np.asarray(fs.sub_ndof, np.int32), np.asarray(fs.sub_scene, np.int32),
                           np.asarray(fs.if_kind, np.int32), np.asarray(fs.if_dim, np.int32),
                           np.asarray(fs.if_nsub, np.int32), np.asarray(fs.if_sub, np.int32),
                           np.asarray(fs.if_mu, np.float64), A, b, J, e)
    nc = S.slot_counts(p.sub_ndof, p.if_dim, p.if_nsub, p.if_sub)
    print(f"  {p.n_sub} blocks of {int(p.sub_ndof.max())} DOF, {int(nc.min())}-{int(nc.max())} slot rows each",
          flush=True)
    pr = Problem.from_assembled(p, dtype=torch.float64)
    out = pr.solve(*(pr.tensor(x) for x in (A, b, J, e)), max_iters=40, tol=0.0)
    ref = O.solve(p, A, b, J, e, max_iters=40, tol=0.0, n_threads=16)
    ev = np.abs(_np(out["v_hat"]) - ref.v_hat).max() / np.abs(ref.v_hat).max()
    el = np.abs(_np(out["lam"]) - ref.lam).max() / max(1.0, np.abs(ref.lam).max())
    print(f"  FEM blocks, 40 iterations: v {ev:.2e} lambda {el:.2e}", flush=True)
    assert ev <= 1e-9 and el <= 1e-9
    pr.check()


def _one_big(n, n_if, seed):
    """One scene: a subsystem of n DOF (condition 10) and a small one, coupled by equalities
    and with contacts on the big one."""
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * np.linspace(1.0, 10.0, n)) @ Q.T
    kinds = [S.KIND_EQUALITY if j % 2 == 0 else S.KIND_CONTACT for j in range(n_if)]
    dims = [4 if k == S.KIND_EQUALITY else 3 for k in kinds]
    nsub = [2 if k == S.KIND_EQUALITY else 1 for k in kinds]
    subs = [[0, 1] if k == S.KIND_EQUALITY else [0, -1] for k in kinds]
    nc = S.slot_counts(np.array([n, 6]), np.array(dims), np.array(nsub), np.array(subs))
    return S.AssembledProblem(np.array([n, 6], np.int32), np.array([0, 0], np.int32), np.array(kinds, np.int32),
                              np.array(dims, np.int32), np.array(nsub, np.int32), np.array(subs, np.int32),
                              np.array([0.0 if k == S.KIND_EQUALITY else 0.6 for k in kinds]),
                              np.concatenate([A.ravel(), np.diag(rng.uniform(1, 2, 6)).ravel()]),
                              rng.standard_normal(n + 6), rng.standard_normal(int(nc[0]) * n + int(nc[1]) * 6),
                              rng.standard_normal(int(sum(dims))))


def test_largest_subsystem_and_the_limit():
    """A 512-DOF subsystem (the largest the factorisation takes: a thread per column of its
    first step) against the oracle, FP64, 30 iterations; 513 DOF is refused at solve."""
    from paper_2302_14344_amd import _lib as L
    from paper_2302_14344_amd.solver import Problem
    p = _one_big(512, 8, 41)
    pr = Problem.from_assembled(p, dtype=torch.float64)
    out = pr.solve(*(pr.tensor(x) for x in (p.A, p.b, p.J, p.e)), max_iters=30, tol=0.0)
    ref = O.solve(p, p.A, p.b, p.J, p.e, max_iters=30, tol=0.0)
    ev = np.abs(_np(out["v_hat"]) - ref.v_hat).max() / np.abs(ref.v_hat).max()
    el = np.abs(_np(out["lam"]) - ref.lam).max() / max(1.0, np.abs(ref.lam).max())
    print(f"  512 DOF: v {ev:.2e} lambda {el:.2e}", flush=True)
    assert ev <= 1e-9 and el <= 1e-9
    pr.check()
    q = _one_big(513, 4, 42)
    pq = Problem.from_assembled(q, dtype=torch.float64)
    with pytest.raises(L.SubadmmError, match="512 DOF"):
        pq.solve(*(pq.tensor(x) for x in (q.A, q.b, q.J, q.e)), max_iters=5, tol=0.0)
