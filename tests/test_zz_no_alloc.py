"""subadmm_solve_scratch, the solve that allocates nothing (its tables and per-step arrays
live in the library's static device scratch), against subadmm_solve on a bound workspace:
the same kernels on the same inputs give bit-identical outputs and statistics, on calls in
a row where a smaller problem follows a larger one (and the larger one comes back), with a
cold and a given warm start.  A problem larger than the scratch is refused on the host."""
import numpy as np
import pytest
import torch

from paper_2302_14344_amd import _lib as L
from paper_2302_14344_amd import scenes as S

pytestmark = pytest.mark.gpu


def _np(t):
    return t.detach().cpu().numpy()


def _problem(n_scenes, seed, dtype):
    from paper_2302_14344_amd.solver import Problem
    p = S.random_assembled(seed, n_scenes=n_scenes, subs_per_scene=(1, 5), ndof=(1, 12), n_if_per_scene=(0, 7),
                           kinds=(0, 1, 2), eq_dim=(1, 6))
    pr = Problem.from_assembled(p, dtype=dtype)
    return p, pr, tuple(pr.tensor(x) for x in (p.A, p.b, p.J, p.e))


def _same(ref, got, st_ref, st_got, what):
    for k in ("v_hat", "lam", "z", "u"):
        np.testing.assert_array_equal(_np(got[k]), _np(ref[k]), err_msg=f"{what}: {k}")
    np.testing.assert_array_equal(np.array([s[0] for s in st_got]), st_ref["iters"], err_msg=f"{what}: iters")
    np.testing.assert_array_equal(np.array([s[1] for s in st_got]), st_ref["converged"], err_msg=f"{what}: conv")
    np.testing.assert_array_equal(np.array([s[2] for s in st_got]), st_ref["theta"], err_msg=f"{what}: theta")


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_scratch_solve_matches_bound_solve(dtype):
    tol = 1e-10 if dtype == torch.float64 else 1e-6
    big = _problem(3000, 201, dtype)
    small = _problem(30, 202, dtype)
    assert big[1].sizes.n_scene == 3000 and small[1].sizes.n_scene == 30
    for what, (p, pr, arrs) in (("large", big), ("smaller", small), ("large again", big)):
        print(f"scratch solve {what} {dtype}", flush=True)
        ref = pr.solve(*arrs, max_iters=400, tol=tol, warm="cold")
        st_ref = pr.stats()
        got, st = pr.solve_scratch(*arrs, max_iters=400, tol=tol, warm="cold", with_stats=True)
        torch.cuda.synchronize()
        _same(ref, got, st_ref, st, f"{what} cold")
        pr.check()
    # given warm start: from the converged values of a shorter run, on the smaller problem
    p, pr, arrs = small
    start = pr.solve(*arrs, max_iters=25, tol=0.0, warm="cold")
    ref = pr.solve(*arrs, max_iters=400, tol=tol, warm="given", z0=start["z"], u0=start["u"])
    st_ref = pr.stats()
    got, st = pr.solve_scratch(*arrs, max_iters=400, tol=tol, warm="given", z0=start["z"], u0=start["u"],
                               with_stats=True)
    _same(ref, got, st_ref, st, "given")


def test_scratch_solve_refuses_a_problem_larger_than_the_scratch():
    p, pr, arrs = _problem(20000, 203, torch.float64)
    assert pr.workspace.numel() > L.SCRATCH_BYTES
    with pytest.raises(L.SubadmmError) as ei:
        pr.solve_scratch(*arrs, max_iters=10, tol=0.0)
    assert ei.value.code == L.E_WORKSPACE
    with pytest.raises(L.SubadmmError) as ei:  # the previous-step start is not offered
        L.check(L.lib().subadmm_solve_scratch(pr._h, None, None, None, None, None, 10, 0.0, L.WARM_PREV, None, None,
                                              None, None, None, None, None), pr._h)
    assert ei.value.code == L.E_ARG
