"""C-ABI checks that need no GPU: exported symbols, struct layout, host-side validation."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.sparse as sp

from paper_1912_04263_amd import qpg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "qpg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qpg_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = qpg.lib()
    names = declared_functions()
    assert len(names) >= 24
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(qpg.SIGNATURES)


def test_struct_layout_matches_header():
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "qpg.h"
int main(void) {
  printf("%zu %zu %zu\n", sizeof(qpg_csc), sizeof(qpg_settings), sizeof(qpg_info));
  printf("%zu %zu %zu %zu\n", offsetof(qpg_settings, pcg_max_iter), offsetof(qpg_settings, stream),
         offsetof(qpg_settings, verbose), offsetof(qpg_settings, rho_update_gate));
  printf("%zu %zu %zu %zu\n", offsetof(qpg_info, obj_val), offsetof(qpg_info, solve_time),
         offsetof(qpg_info, scaling_passes), offsetof(qpg_info, precond_switches));
  printf("%zu %zu %zu\n", offsetof(qpg_settings, precond_weights), offsetof(qpg_settings, precond_trial),
         offsetof(qpg_settings, spmv_plain_nnz));
  printf("%zu %zu %zu %zu\n", offsetof(qpg_settings, eps_prim_inf), offsetof(qpg_settings, eps_dual_inf),
         offsetof(qpg_settings, rho_vector), offsetof(qpg_settings, pcg_eps_schedule));
  printf("%zu %d %d\n", offsetof(qpg_info, infeas_checks), QPG_PRIMAL_INFEASIBLE, QPG_DUAL_INFEASIBLE);
  printf("%zu %zu\n", offsetof(qpg_settings, speculate), offsetof(qpg_info, spec_resumes));
  printf("%zu %zu\n", offsetof(qpg_settings, spmv_window_cols), offsetof(qpg_settings, spmv_min_seg));
  printf("%d\n", QPG_NET_NPARAMS);
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split()
    got = [int(v) for v in out]
    S, I = qpg.Settings, qpg.Info
    want = [C.sizeof(qpg.Csc), C.sizeof(S), C.sizeof(I),
            S.pcg_max_iter.offset, S.stream.offset, S.verbose.offset, S.rho_update_gate.offset,
            I.obj_val.offset, I.solve_time.offset, I.scaling_passes.offset, I.precond_switches.offset,
            S.precond_weights.offset, S.precond_trial.offset, S.spmv_plain_nnz.offset,
            S.eps_prim_inf.offset, S.eps_dual_inf.offset, S.rho_vector.offset, S.pcg_eps_schedule.offset,
            I.infeas_checks.offset, qpg.QPG_PRIMAL_INFEASIBLE, qpg.QPG_DUAL_INFEASIBLE,
            S.speculate.offset, I.spec_resumes.offset, S.spmv_window_cols.offset, S.spmv_min_seg.offset,
            qpg.QPG_NET_NPARAMS]
    assert got == want


def test_parameter_count_matches_oracle_layout():
    from oracle import mpnn
    assert mpnn.nparams() == qpg.QPG_NET_NPARAMS


def test_default_settings_follow_the_paper():
    s = qpg.default_settings()
    assert (s.rho, s.sigma, s.alpha) == (0.1, 1e-6, 1.6)          # Section 3.4
    assert (s.pcg_lambda, s.pcg_eps_min) == (0.15, 1e-7)          # Section 6.3.3
    assert (s.check_every, s.rho_update_every) == (5, 10)         # Section 6.3.2–6.3.3, Table 1
    assert s.precision == qpg.QPG_FP64 and s.pcg_rel_test == 1
    assert s.rho_vector == 0 and s.pcg_eps_schedule == 0                # R = ρ̄I (Section 6.3)
    assert (s.eps_prim_inf, s.eps_dual_inf) == (1e-4, 1e-4)


def _tiny():
    P = sp.csc_matrix(np.array([[2.0, 0.5], [0.0, 1.0]]))
    A = sp.csc_matrix(np.array([[1.0, 1.0], [1.0, 0.0]]))
    return P, np.array([1.0, -1.0]), A, np.array([-1.0, 0.0]), np.array([1.0, 0.5])


@pytest.mark.parametrize("mutate, code", [
    (lambda d: d["q"].__setitem__(0, np.nan), qpg.QPG_ERR_DATA),
    (lambda d: d["l"].__setitem__(1, 2.0), qpg.QPG_ERR_DATA),                 # l > u
    (lambda d: d.__setitem__("P", sp.csc_matrix(np.array([[2.0, 0.0], [0.5, 1.0]]))), qpg.QPG_ERR_ARG),
    (lambda d: d["A"].data.__setitem__(0, np.inf), qpg.QPG_ERR_DATA),
    (lambda d: d["u"].__setitem__(0, np.nan), qpg.QPG_ERR_DATA),
])
def test_setup_rejects_bad_data_before_touching_the_device(mutate, code):
    P, q, A, l, u = _tiny()
    d = dict(P=P, q=q, A=A, l=l, u=u)
    mutate(d)
    with pytest.raises(qpg.QpgError) as e:
        qpg.Solver(d["P"], d["q"], d["A"], d["l"], d["u"])
    assert e.value.code == code


def test_setup_rejects_unsorted_indices_and_bad_settings():
    P, q, A, l, u = _tiny()
    L = qpg.lib()
    colptr = np.array([0, 2, 3], np.int32)
    rowidx = np.array([1, 0, 0], np.int32)  # column 0 rows not increasing
    val = np.ones(3)
    Ac = qpg.Csc(2, 2, 3, qpg._iptr(colptr), qpg._iptr(rowidx), qpg._dptr(val))
    Pc = qpg._CscArrays(P)
    s = qpg.default_settings()
    h = C.c_void_p()
    rc = L.qpg_setup(C.byref(h), C.byref(Pc.c), qpg._dptr(q), C.byref(Ac), qpg._dptr(l), qpg._dptr(u), C.byref(s))
    assert rc == qpg.QPG_ERR_ARG and b"increasing" in L.qpg_last_error(None)
    w = np.zeros(qpg.QPG_NET_NPARAMS, np.float32)
    for bad in (dict(alpha=2.0), dict(rho=0.0), dict(check_every=0), dict(precision=7),
                dict(eps_prim_inf=-1.0), dict(eps_dual_inf=np.inf), dict(rho_vector=2),
                dict(rho_vector=1, precond="learned", precond_weights=w), dict(pcg_eps_schedule=3)):
        with pytest.raises(qpg.QpgError) as e:
            qpg.Solver(P, q, A, l, u, **bad)
        assert e.value.code == qpg.QPG_ERR_ARG


def test_header_constants_match_binding():
    """Every #define QPG_* with an integer value in the header has the same value in qpg.py."""
    text = open(HEADER).read()
    defs = dict(re.findall(r"#define\s+(QPG_[A-Z0-9_]+)\s+\(?(-?\d+)\)?", text))
    assert "QPG_ERR_HOST" in defs and len(defs) > 20
    for name, value in defs.items():
        assert getattr(qpg, name) == int(value), name


def test_error_strings_and_null_handles():
    L = qpg.lib()
    assert L.qpg_error_string(qpg.QPG_ERR_DATA) == b"invalid problem data"
    codes = [qpg.QPG_ERR_ARG, qpg.QPG_ERR_DATA, qpg.QPG_ERR_SIZE, qpg.QPG_ERR_DEVICE, qpg.QPG_ERR_OOM,
             qpg.QPG_ERR_STATE, qpg.QPG_ERR_HOST]
    texts = [L.qpg_error_string(c) for c in codes]
    assert len(set(texts)) == len(codes) and b"unknown error" not in texts
    assert L.qpg_cleanup(None) == 0
    assert L.qpg_solve(None) == qpg.QPG_ERR_ARG
    assert L.qpg_get_x(None, None) == qpg.QPG_ERR_ARG
