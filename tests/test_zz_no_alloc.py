"""qpg_hutchinson_noalloc (the allocation-free Hutchinson estimate) against qpg_hutchinson. Needs an
MI355X.

Both calls run the same kernels in the same order on the same probes, so the estimates must agree
bitwise. The no-alloc call keeps its accumulator and probe in one static device array shared by
every call on the device: two calls in a row, the second on a smaller problem with fewer probes,
check that nothing of the first call leaks into the second. The small problem is also checked
against the oracle's diag(K⁻¹) estimate with a dense inverse (1e-8, as for qpg_hutchinson).
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import hutchinson as o_hutch
from oracle import pcg as o_pcg
from paper_1912_04263_amd import problems as pr
from paper_1912_04263_amd import qpg

pytestmark = pytest.mark.gpu


def say(*a):
    print("[case]", *a, file=sys.stderr, flush=True)


def probes(seed, s, n):
    rng = np.random.default_rng(seed)
    return rng.choice(np.array([-1, 1], dtype=np.int8), size=(s, n))


def test_noalloc_hutchinson_equals_the_allocating_call_twice_in_a_row():
    rho = 0.3
    big, small = pr.make("svm_small"), pr.make("random_c0")
    assert small.n < big.n
    say("noalloc hutchinson, first call", big.name, big.n)
    with qpg.Solver.from_qp(big) as s:
        z = probes(5, 4, big.n)
        ref = s.hutchinson(z, rho, eps=1e-12)
        got = s.hutchinson_noalloc(z, rho, eps=1e-12)
        assert np.all(np.isfinite(got))
        np.testing.assert_array_equal(got, ref)
    say("noalloc hutchinson, second call", small.name, small.n)
    with qpg.Solver.from_qp(small) as s:
        z = probes(6, 3, small.n)
        got = s.hutchinson_noalloc(z, rho, eps=1e-12)
        ref = s.hutchinson(z, rho, eps=1e-12)
        np.testing.assert_array_equal(got, ref)
        D, E, c = s.scaling()
        Pb = (c * sp.diags(D) @ small.P_full() @ sp.diags(D)).tocsr()
        Ab = (sp.diags(E) @ sp.csr_matrix(small.A) @ sp.diags(D)).tocsr()
        Kinv = np.linalg.inv(o_pcg.reduced_kkt_dense(Pb, Ab, 1e-6, rho))
        want = o_hutch.estimate(lambda v: Kinv @ v, z)
        assert np.max(np.abs(got - want)) <= 1e-8 * np.max(np.abs(want))
        # the handle's ρ̄ is restored: the solve is unaffected by the estimate
        assert s.solve().status == "solved"


def test_noalloc_hutchinson_rejects_n_beyond_the_scratch():
    n = qpg.QPG_NOALLOC_MAX_N + 1
    say("noalloc hutchinson size limit, n =", n)
    P = sp.identity(n, format="csc")
    A = sp.csc_matrix((np.ones(1), (np.zeros(1, int), np.zeros(1, int))), shape=(1, n))
    with qpg.Solver(P, np.zeros(n), A, -np.ones(1), np.ones(1)) as s:
        with pytest.raises(qpg.QpgError) as e:
            s.hutchinson_noalloc(np.ones((1, n), np.int8), 0.1)
        assert e.value.code == qpg.QPG_ERR_SIZE
