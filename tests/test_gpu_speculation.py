"""Speculative ADMM iterations against the synchronous loop. Needs an MI355X.

Between two residual checks the solver launches ADMM iterations without waiting for their PCG
solves (settings.speculate = 1). When a PCG solve needs more iterations than were launched for
it, a single-workgroup kernel that runs after the iteration's last direction update raises a
device flag, the rest of the speculation is skipped, and the host finishes that solve from the
state the kernels left. With speculate = 0 the host waits for every PCG solve instead (the
synchronous loop of Section 6.3.3). The two run the same kernels on the same data in the same
order, so x, y, z and every count must agree bitwise.

The instance is large (n > 256·1024, so the vector kernels run 1024 workgroups) and a
portfolio QP, whose PCG iteration counts change from one ADMM iteration to the next, so the
resumption path is taken many times.
"""
import sys

import numpy as np
import pytest

from paper_1912_04263_amd import problems as pr
from paper_1912_04263_amd import qpg

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_speculative_solve_equals_synchronous_solve(precision):
    p = pr.portfolio_qp(300_000, 100, 0.05, seed=777)
    out = {}
    for spec in (1, 0):
        say("speculation", precision, "speculate", spec, "n", p.n, "m", p.m, "nnz(A)", p.A.nnz)
        with qpg.Solver.from_qp(p, eps_abs=1e-4, eps_rel=1e-4, precision=precision, speculate=spec) as s:
            info = s.solve()
            out[spec] = (info, s.x(), s.y(), s.z())
    (i1, x1, y1, z1), (i0, x0, y0, z0) = out[1], out[0]
    say("speculative", i1)
    say("synchronous", i0)
    assert i1.status == "solved" and i0.status == "solved"
    assert i1.spec_resumes > 0, "the resumption path was not exercised"
    assert i0.spec_resumes == 0
    assert (i1.iter, i1.pcg_iter_total, i1.pcg_iter_max, i1.rho_updates) == \
        (i0.iter, i0.pcg_iter_total, i0.pcg_iter_max, i0.rho_updates)
    assert np.array_equal(x1, x0) and np.array_equal(y1, y0) and np.array_equal(z1, z0)
