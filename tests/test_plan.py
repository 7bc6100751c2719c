"""Host logic of the SpMV work lists (csrc/tiles.cpp), checked on the CPU.

tests/native/plan_check.cpp is built with g++ against tiles.cpp; on each matrix it checks every
bound the SpMV kernels rely on (rows, sub-runs, row starts, split positions, LDS windows, partial
and combine slots), that the entry order is a permutation, that every entry is streamed exactly
once, and that the row sums formed the kernels' way match a plain CSR product to 1e-12.
"""
import functools
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

from paper_1912_04263_amd import problems as pr

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1912_04263_amd", "csrc")


SANITIZE = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"]


@functools.lru_cache(maxsize=None)
def checker(tmpdir, sanitize=False, shuffled=False):
    exe = os.path.join(tmpdir, "plan_check_asan" if sanitize else "plan_check_shuffled" if shuffled else "plan_check")
    opt = SANITIZE if sanitize else ["-O2"]
    par = (os.path.join(ROOT, "tests", "native", "parallel_shuffled.cpp") if shuffled
           else os.path.join(CSRC, "host_parallel.cpp"))
    subprocess.run(["g++", *opt, "-std=c++17", "-I", CSRC, os.path.join(ROOT, "tests", "native", "plan_check.cpp"),
                    os.path.join(CSRC, "tiles.cpp"), par, "-lpthread", "-o", exe],
                   check=True)
    return exe


@pytest.fixture(scope="module")
def exe(tmp_path_factory):
    return checker(str(tmp_path_factory.mktemp("plan")))


@pytest.fixture(scope="module")
def exe_sanitized(tmp_path_factory):
    """The same checker built with AddressSanitizer and UndefinedBehaviorSanitizer: an
    out-of-bounds access, an overflow of the 16-bit window offsets' arithmetic or any other
    undefined behaviour in the planner aborts it."""
    return checker(str(tmp_path_factory.mktemp("plan_asan")), sanitize=True)


@pytest.fixture(scope="module")
def exe_shuffled(tmp_path_factory):
    """The checker linked against a stand-in for the host thread pool whose thread count is set
    by QPG_TEST_THREADS and which runs the chunks in a scrambled order."""
    return checker(str(tmp_path_factory.mktemp("plan_shuffled")), shuffled=True)


def stats(out):
    """Fields of the first output line (window size wcap) as a dict of ints/floats."""
    f = out.splitlines()[0].replace("%", "").split()
    return {f[i]: float(f[i + 1]) for i in range(0, len(f) - 1, 2)}


def run(exe, tmp_path, M, nsplit=None, tile_nnz=32768, plain_nnz=8192, wcap=8192, env=None):
    M = sp.csr_matrix(M)
    M.sort_indices()
    pre = str(tmp_path / "m")
    M.indptr.astype(np.int32).tofile(pre + "_ptr.bin")
    M.indices.astype(np.int32).tofile(pre + "_col.bin")
    ncols = M.shape[1]
    out = subprocess.run([exe, pre, str(ncols), str(ncols if nsplit is None else nsplit), str(tile_nnz),
                          str(plain_nnz), str(wcap)], capture_output=True, text=True,
                         env=None if env is None else dict(os.environ, **env))
    assert out.returncode == 0, out.stdout + out.stderr
    return out.stdout


def reduced_pair(p):
    A = sp.csr_matrix(p.A)
    B = sp.hstack([p.P_full().tocsr(), A.T.tocsr()]).tocsr()
    return A, B


@pytest.mark.parametrize("name", ["random_c0", "random_small", "lasso_small", "portfolio_small", "svm_small",
                                  "random2_small"])
@pytest.mark.parametrize("wcap", [1024, 8192])
def test_work_lists_of_the_generated_workloads(exe, tmp_path, name, wcap):
    p = pr.make(name)
    A, B = reduced_pair(p)
    run(exe, tmp_path, A, wcap=wcap)
    run(exe, tmp_path, B, nsplit=p.n, wcap=wcap)


@pytest.mark.parametrize("name", ["random_c0", "lasso_small", "portfolio_small", "random2_small"])
def test_work_lists_under_sanitizers(exe_sanitized, tmp_path, name):
    p = pr.make(name)
    A, B = reduced_pair(p)
    for wcap in (1024, 8192):
        run(exe_sanitized, tmp_path, A, wcap=wcap)
        run(exe_sanitized, tmp_path, B, nsplit=p.n, wcap=wcap)


def test_edge_matrices_under_sanitizers(exe_sanitized, tmp_path):
    run(exe_sanitized, tmp_path, sp.csr_matrix((5, 7)))
    run(exe_sanitized, tmp_path, sp.csr_matrix(([2.0], ([3], [6])), shape=(5, 7)), nsplit=4)
    rng = np.random.default_rng(4)
    M = sp.random(500, 400000, density=100 / 400000, random_state=rng, format="csr")
    run(exe_sanitized, tmp_path, M, nsplit=50000)
    M = sp.random(100, 100000, density=0.02, random_state=rng, format="csr")
    run(exe_sanitized, tmp_path, M, nsplit=30000, tile_nnz=1024, plain_nnz=1024, wcap=2048)


def test_single_segment_rows_with_consecutive_slots_take_run_items(exe, tmp_path):
    # SVM's B: its t rows (one entry of Aᵀ each) are single-segment rows, numbered in row order
    # within their tiles, so the combine takes them as K = 1 runs; the random QP has none
    p = pr.make("svm_small")
    _, B = reduced_pair(p)
    st = stats(run(exe, tmp_path, B, nsplit=p.n))
    assert st["run_rows"] >= p.meta["n_points"]
    p = pr.make("random_small")
    _, B = reduced_pair(p)
    assert stats(run(exe, tmp_path, B, nsplit=p.n))["run_rows"] == 0


def test_wide_rows_take_the_multi_range_layout(exe, tmp_path):
    rng = np.random.default_rng(1)
    M = sp.random(200, 100000, density=0.02, random_state=rng, format="csr")
    st = stats(run(exe, tmp_path, M, nsplit=30000))
    # every row is cut at the window boundaries: many slots per row, all entries in LDS windows
    assert st["slots"] >= 10 * 200 and st["windowed"] >= 10 and st["in-window"] > 95


def test_long_rows_in_a_narrow_band_and_empty_rows(exe, tmp_path):
    rng = np.random.default_rng(2)
    rows, cols = [], []
    for r in range(60):
        if r % 7 == 3:
            continue  # empty row
        n = 6000 if r % 2 else int(rng.integers(1, 40))
        c0 = int(rng.integers(0, 2000))
        rows += [r] * n
        cols += list(range(c0, c0 + n))
    M = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(60, 9000))
    st = stats(run(exe, tmp_path, M, nsplit=4000))
    assert st["slots"] > 60  # the 6000-entry rows are cut into several segments


def test_empty_and_one_entry_matrices(exe, tmp_path):
    run(exe, tmp_path, sp.csr_matrix((5, 7)))
    run(exe, tmp_path, sp.csr_matrix(([2.0], ([3], [6])), shape=(5, 7)), nsplit=4)


def test_small_work_units_on_a_random_matrix(exe, tmp_path):
    rng = np.random.default_rng(3)
    M = sp.random(3000, 50000, density=2e-3, random_state=rng, format="csr")
    run(exe, tmp_path, M, nsplit=20000, tile_nnz=1024, plain_nnz=1024, wcap=2048)


def test_sparse_wide_rows_take_the_l2_range_layout(exe, tmp_path):
    # 100 entries per row over 400,000 columns: too sparse for an LDS window (≈ 2 per 8192
    # columns) but ≈ 33 per 2^17-column range, so the rows are cut at those ranges
    rng = np.random.default_rng(4)
    M = sp.random(3000, 400000, density=100 / 400000, random_state=rng, format="csr")
    st = stats(run(exe, tmp_path, M, nsplit=50000))
    assert st["windowed"] == 0 and st["slots"] >= 3 * 3000


def test_random_rows_take_the_grid_layout(exe, tmp_path):
    # 20 entries per row spread uniformly over 4000 columns: ≈ 5 per 1024-column window, too few
    # for the multi-range layout but enough for the grid (one segment per row and window)
    rng = np.random.default_rng(5)
    M = sp.random(50000, 4000, density=20 / 4000, random_state=rng, format="csr")
    st = stats(run(exe, tmp_path, M, nsplit=1500, wcap=1024))
    # runs of rows of similar length decide the layout; the few rows far from 20 entries form
    # short runs of their own, which may take another layout
    assert st["grid_rows"] >= 0.9 * 50000 and st["in-window"] > 95
    # a few entries outside every qualifying window: those rows' blocks fall back, the rest stay
    M = M.tolil()
    M[7, 3999] = 1.0
    st = stats(run(exe, tmp_path, M.tocsr(), nsplit=1500, wcap=1024))
    assert st["grid_rows"] > 0


def test_grid_layout_under_sanitizers(exe_sanitized, tmp_path):
    rng = np.random.default_rng(6)
    M = sp.random(20000, 3000, density=8 / 3000, random_state=rng, format="csr")
    run(exe_sanitized, tmp_path, M, nsplit=1000, wcap=1024)


def fingerprints(out):
    return [line.split()[-1] for line in out.splitlines() if line.startswith("fingerprint")]


@pytest.mark.parametrize("case", ["svm_small B", "portfolio_small A", "lasso_small B", "grid", "skewed"])
def test_work_lists_do_not_depend_on_the_host_threads(exe, exe_shuffled, tmp_path, case):
    """The planner's parallel passes write disjoint parts and its lists are assembled in block
    order, so every array of the work list is the same for any number of host threads and any
    order in which the threads take the chunks (1, 3 and 8 threads, scrambled, against the
    library's own pool)."""
    rng = np.random.default_rng(11)
    nsplit = None
    if case == "grid":
        M = sp.random(30000, 4000, density=20 / 4000, random_state=rng, format="csr")
        wcap = 1024
    elif case == "skewed":  # a few long rows among many short ones, wide and narrow
        M = sp.vstack([sp.random(40, 50000, density=0.2, random_state=rng),
                       sp.random(20000, 50000, density=3 / 50000, random_state=rng)]).tocsr()
        wcap = 8192
    else:
        name, which = case.split()
        p = pr.make(name)
        A, B = reduced_pair(p)
        M, nsplit, wcap = (A, None, 8192) if which == "A" else (B, p.n, 8192)
    ref = fingerprints(run(exe, tmp_path, M, nsplit=nsplit, wcap=wcap))
    assert len(ref) == 2
    for threads in (1, 3, 8):
        got = fingerprints(run(exe_shuffled, tmp_path, M, nsplit=nsplit, wcap=wcap,
                               env={"QPG_TEST_THREADS": str(threads)}))
        assert got == ref, (case, threads)
