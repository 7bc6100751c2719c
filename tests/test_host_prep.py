"""Input validation and CSC → CSR conversion of qpg_setup (csrc/host_prep.cpp), on the CPU, under
AddressSanitizer and UndefinedBehaviorSanitizer.

tests/native/prep_check.cpp runs the library's prepare() on a problem given in the C ABI's
convention (P as its upper triangle in CSC, A in CSC) and writes the converted arrays back. They
are compared with SciPy's own conversion: A in CSR (Section 6.2 stores A and Aᵀ), the full P from
its upper triangle, B = [P | Aᵀ] row by row with the split point of each row, and the bounds with
infinities clamped to ±1e20. Malformed inputs must be rejected with the documented code, before
any conversion. The harness is built with -fsanitize=address,undefined (a memory error or
undefined behaviour aborts it), once per test session.
"""
import functools
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1912_04263_amd", "csrc")
ERR_ARG, ERR_DATA = -1, -2
INF = 1e20


@functools.lru_cache(maxsize=None)
def harness(tmpdir, shuffled=False):
    exe = os.path.join(tmpdir, "prep_check_shuffled" if shuffled else "prep_check")
    par = (os.path.join(ROOT, "tests", "native", "parallel_shuffled.cpp") if shuffled
           else os.path.join(CSRC, "host_parallel.cpp"))
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-I", CSRC, os.path.join(ROOT, "tests", "native", "prep_check.cpp"),
                    os.path.join(CSRC, "host_prep.cpp"), par, "-lpthread", "-o", exe], check=True)
    return exe


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    return harness(str(tmp_path_factory.mktemp("prep")))


def run(exe, d, P_triu, q, A, l, u, rho_vector=0, raw=None, threads=None):
    """Write the problem, run prepare() under the sanitizers, return (rc, message, outputs)."""
    P_triu = sp.csc_matrix(P_triu)
    A = sp.csc_matrix(A)
    arrays = {"pcp": P_triu.indptr, "pri": P_triu.indices, "pv": P_triu.data, "acp": A.indptr, "ari": A.indices,
              "av": A.data}
    if raw:
        arrays.update(raw)
    for k, v in arrays.items():
        np.asarray(v, dtype=np.float64 if k in ("pv", "av") else np.int32).tofile(os.path.join(d, k + ".bin"))
    for k, v in (("q", q), ("l", l), ("u", u)):
        np.asarray(v, dtype=np.float64).tofile(os.path.join(d, k + ".bin"))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    if threads is not None:
        env["QPG_TEST_THREADS"] = str(threads)
    r = subprocess.run([exe, d, str(A.shape[1]), str(A.shape[0]), str(rho_vector)], capture_output=True, text=True,
                       env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.split("\n")
    rc = int(lines[0].split()[1])
    out = {}
    if rc == 0:
        for k, dt in (("a_ptr", np.int32), ("a_col", np.int32), ("a_val", np.float64), ("b_ptr", np.int32),
                      ("b_split", np.int32), ("b_col", np.int32), ("b_val", np.float64), ("lb", np.float64),
                      ("ub", np.float64), ("eqrow", np.uint8)):
            out[k] = np.fromfile(os.path.join(d, f"out_{k}.bin"), dtype=dt)
    return rc, lines[1], out


def random_problem(seed, n, m, dens):
    """Empty rows and columns of A, a variable absent from P, a missing diagonal, one-sided,
    free and equality rows, infinite bounds."""
    rng = np.random.default_rng(seed)
    M = sp.random(n, n, density=dens, random_state=rng, format="csr")
    P = (M @ M.T).tocsr()
    P.setdiag(np.where(rng.random(n) < 0.8, 1.0 + rng.random(n), 0.0))
    P = P.tocsr()
    P.eliminate_zeros()
    A = sp.random(m, n, density=dens, random_state=rng, format="csr")
    A = A.tolil()
    A[min(3, m - 1), :] = 0          # an empty row
    A[:, min(5, n - 1)] = 0          # an empty column
    A = A.tocsc()
    A.eliminate_zeros()
    l = -rng.random(m)
    u = rng.random(m)
    u[::7] = l[::7]                  # equalities
    l[1::5] = -np.inf                # one-sided
    u[2::9] = np.inf
    l[4::11], u[4::11] = -np.inf, np.inf
    q = rng.standard_normal(n)
    return sp.triu(P).tocsc(), P, q, A, l, u


# the last two: more than 2^18 entries, so the conversion splits the columns into parts, and rows
# spanning several 4096-row buckets (8192 rows: the last bucket is empty)
@pytest.mark.parametrize("seed, n, m, dens, rv", [(0, 40, 60, 0.1, 0), (1, 300, 200, 0.05, 1),
                                                  (2, 3000, 5000, 0.03, 0), (4, 2000, 8192, 0.02, 0)])
def test_conversion_matches_scipy(exe, tmp_path, seed, n, m, dens, rv):
    Pt, P, q, A, l, u = random_problem(seed, n, m, dens)
    rc, msg, o = run(exe, str(tmp_path), Pt, q, A, l, u, rho_vector=rv)
    assert rc == 0, msg
    Ar = sp.csr_matrix(A)
    Ar.sort_indices()
    np.testing.assert_array_equal(o["a_ptr"], Ar.indptr)
    np.testing.assert_array_equal(o["a_col"], Ar.indices)
    np.testing.assert_array_equal(o["a_val"], Ar.data)
    Pf = sp.csr_matrix(Pt + sp.triu(Pt, k=1).T)
    Pf.sort_indices()
    B = sp.hstack([Pf, sp.csr_matrix(A.T)]).tocsr()
    B.sort_indices()
    np.testing.assert_array_equal(o["b_ptr"], B.indptr)
    np.testing.assert_array_equal(o["b_col"], B.indices)
    np.testing.assert_array_equal(o["b_val"], B.data)
    np.testing.assert_array_equal(o["b_split"], B.indptr[:-1] + np.diff(Pf.indptr))
    np.testing.assert_array_equal(o["lb"], np.maximum(l, -INF))
    np.testing.assert_array_equal(o["ub"], np.minimum(u, INF))
    if rv:
        np.testing.assert_array_equal(o["eqrow"], (l == u).astype(np.uint8))
    else:
        assert o["eqrow"].size == 0


def _bad_cases():
    Pt, _, q, A, l, u = random_problem(3, 12, 10, 0.3)
    A = sp.csc_matrix(A)
    Pt = sp.csc_matrix(Pt)
    j = int(np.argmax(np.diff(A.indptr)))  # a column with at least two entries
    a, b = A.indptr[j], A.indptr[j + 1]
    assert b - a >= 2
    ri = A.indices.copy()
    ri[a], ri[a + 1] = ri[a + 1], ri[a]
    yield "unsorted row indices", dict(raw={"ari": ri}), ERR_ARG
    ri = A.indices.copy()
    ri[a + 1] = ri[a]
    yield "duplicate row index", dict(raw={"ari": ri}), ERR_ARG
    ri = A.indices.copy()
    ri[b - 1] = A.shape[0]
    yield "row index out of range", dict(raw={"ari": ri}), ERR_ARG
    ri = A.indices.copy()
    ri[a] = -1
    yield "negative row index", dict(raw={"ari": ri}), ERR_ARG
    cp = A.indptr.copy()
    cp[j + 1] = cp[j] - 1 if cp[j] > 0 else cp[j + 1]
    if cp[j] > 0:
        yield "colptr not monotone", dict(raw={"acp": cp}), ERR_ARG
    cp = A.indptr.copy()
    cp[0] = 1
    yield "colptr does not start at 0", dict(raw={"acp": cp}), ERR_ARG
    low = sp.csc_matrix(Pt.T)  # strictly below the diagonal where Pt has off-diagonal entries
    yield "entry below the diagonal of P_triu", dict(P=low), ERR_ARG
    av = A.data.copy()
    av[a] = np.nan
    yield "NaN in A", dict(raw={"av": av}), ERR_DATA
    av = A.data.copy()
    av[a] = np.inf
    yield "inf in A", dict(raw={"av": av}), ERR_DATA
    q2 = q.copy()
    q2[0] = np.inf
    yield "inf in q", dict(q=q2), ERR_DATA
    l2 = l.copy()
    l2[0] = np.nan
    yield "NaN in l", dict(l=l2), ERR_DATA
    l2, u2 = l.copy(), u.copy()
    l2[2], u2[2] = 1.0, 0.5
    yield "l > u", dict(l=l2, u=u2), ERR_DATA


@pytest.mark.parametrize("case", list(_bad_cases()), ids=lambda c: c[0])
def test_malformed_inputs_are_rejected(exe, tmp_path, case):
    _, kw, code = case
    Pt, _, q, A, l, u = random_problem(3, 12, 10, 0.3)
    args = dict(P_triu=kw.get("P", Pt), q=kw.get("q", q), A=A, l=kw.get("l", l), u=kw.get("u", u))
    rc, msg, _ = run(exe, str(tmp_path), args["P_triu"], args["q"], args["A"], args["l"], args["u"],
                     raw=kw.get("raw"))
    assert rc == code, (case[0], rc, msg)
    assert msg


def skewed_problem(seed, n_dense=12, n=700, m=3000):
    """A few dense columns of A that hold most of its entries (as the feature columns of the SVM
    QP do) beside many columns of one or two entries: the column checks and B's rows are cut into
    parts of equal entry counts, so a part boundary falls inside the dense run and the long tail
    of short columns spreads over many parts."""
    rng = np.random.default_rng(seed)
    dense = sp.random(m, n_dense, density=0.6, random_state=rng, format="csc")
    rows = rng.integers(0, m, size=n - n_dense)
    tail = sp.csc_matrix((rng.standard_normal(n - n_dense), (rows, np.arange(n - n_dense))), shape=(m, n - n_dense))
    A = sp.hstack([dense, tail]).tocsc()
    A.sort_indices()
    Pt = sp.diags(1.0 + rng.random(n)).tocsc()
    l = -rng.random(m)
    u = rng.random(m)
    return Pt, rng.standard_normal(n), A, l, u


def test_conversion_of_skewed_columns(exe, tmp_path):
    Pt, q, A, l, u = skewed_problem(5)
    assert np.diff(A.indptr)[:12].sum() > 0.9 * A.nnz
    rc, msg, o = run(exe, str(tmp_path), Pt, q, A, l, u)
    assert rc == 0, msg
    Ar = sp.csr_matrix(A)
    Ar.sort_indices()
    np.testing.assert_array_equal(o["a_ptr"], Ar.indptr)
    np.testing.assert_array_equal(o["a_col"], Ar.indices)
    np.testing.assert_array_equal(o["a_val"], Ar.data)
    B = sp.hstack([sp.csr_matrix(Pt), sp.csr_matrix(A.T)]).tocsr()
    B.sort_indices()
    np.testing.assert_array_equal(o["b_ptr"], B.indptr)
    np.testing.assert_array_equal(o["b_col"], B.indices)
    np.testing.assert_array_equal(o["b_val"], B.data)


@pytest.mark.parametrize("where", ["first dense column", "inside the dense run", "last column"])
def test_skewed_columns_bad_index_is_found(exe, tmp_path, where):
    """A row index out of range is reported wherever the parts of the column check cut."""
    Pt, q, A, l, u = skewed_problem(6)
    j = {"first dense column": 0, "inside the dense run": 7, "last column": A.shape[1] - 1}[where]
    ri = A.indices.copy()
    ri[A.indptr[j + 1] - 1] = A.shape[0]
    rc, msg, _ = run(exe, str(tmp_path), Pt, q, A, l, u, raw={"ari": ri})
    assert rc == ERR_ARG, (where, rc, msg)
    assert "A" in msg


@pytest.mark.parametrize("threads", [1, 3, 8])
def test_conversion_does_not_depend_on_the_host_threads(tmp_path_factory, tmp_path, threads):
    """The harness linked against a stand-in thread pool (tests/native/parallel_shuffled.cpp):
    the given number of threads take the chunks of every parallel pass in a scrambled order, and
    the converted arrays still match SciPy's, on the skewed matrix and on a random one."""
    exe = harness(str(tmp_path_factory.mktemp("prep_shuffled")), shuffled=True)
    Pt, q, A, l, u = skewed_problem(7)
    rc, msg, o = run(exe, str(tmp_path), Pt, q, A, l, u, threads=threads)
    assert rc == 0, msg
    Ar = sp.csr_matrix(A)
    Ar.sort_indices()
    B = sp.hstack([sp.csr_matrix(Pt), sp.csr_matrix(A.T)]).tocsr()
    B.sort_indices()
    for k, ref in (("a_ptr", Ar.indptr), ("a_col", Ar.indices), ("a_val", Ar.data), ("b_ptr", B.indptr),
                   ("b_col", B.indices), ("b_val", B.data)):
        np.testing.assert_array_equal(o[k], ref, err_msg=k)
    Pt, P, q, A, l, u = random_problem(2, 3000, 5000, 0.03)
    rc, msg, o = run(exe, str(tmp_path), Pt, q, A, l, u, threads=threads)
    assert rc == 0, msg
    Ar = sp.csr_matrix(A)
    Ar.sort_indices()
    np.testing.assert_array_equal(o["a_col"], Ar.indices)
    np.testing.assert_array_equal(o["a_val"], Ar.data)
