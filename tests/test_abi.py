"""The C-ABI library loads and exports every entry point include/fsi.h declares.

CPU-only: argument validation paths return before any HIP call, so they run
without a GPU.  The library must have been built (python -m paper_1907_01252_amd.build).
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fsi.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:fsi_status|void|const char\*)\s+(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    from paper_1907_01252_amd import fsi
    return fsi.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("fsi_setup", "fine_propagate", "coarse_propagate", "parareal_run", "fsi_destroy"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n


def test_no_undeclared_c_symbol_is_exported(lib):
    """The library's unmangled (C linkage) dynamic symbols are exactly the header's functions."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    out = subprocess.run([nm, "-D", "--defined-only", lib._name], capture_output=True, text=True, check=True).stdout
    c_syms = {ln.split()[-1] for ln in out.splitlines()
              if len(ln.split()) == 3 and ln.split()[1] == "T" and not ln.split()[-1].startswith("_")}
    assert c_syms == set(declared_functions()), c_syms ^ set(declared_functions())


def test_binding_matches_header():
    from paper_1907_01252_amd import fsi
    assert set(fsi.EXPORTS) == set(declared_functions())


def test_params_struct_matches_header_field_order():
    from paper_1907_01252_amd import fsi
    src = open(HEADER).read()
    body = src[src.index("typedef struct {\n  int32_t dim;"):src.index("} fsi_params;")]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl or decl.startswith("typedef"):
            decl = decl.replace("typedef struct {", "").strip()
            if not decl:
                continue
        toks = decl.split(None, 1)
        for name in toks[1].split(","):
            fields.append(re.sub(r"\[.*", "", name.strip()))
    assert [f[0] for f in fsi.Params._fields_] == fields


def test_status_strings(lib):
    from paper_1907_01252_amd import fsi
    for code in (fsi.FSI_OK, fsi.FSI_ERR_ARG, fsi.FSI_ERR_NEWTON, fsi.FSI_ERR_NONFINITE, fsi.FSI_ERR_PARAREAL):
        assert lib.fsi_status_string(code)
    assert lib.fsi_status_string(-99) == b"unknown status"


def test_argument_errors_without_gpu(lib):
    from paper_1907_01252_amd import fsi
    import synth
    h = C.c_void_p()
    assert lib.fsi_setup(None, C.byref(h)) == fsi.FSI_ERR_ARG
    # invalid parameter sets are rejected before any device allocation
    for bad in (dict(level=0), dict(dim=4), dict(max_batch=0), dict(gmres_restart=100), dict(precond_lag=5),
                dict(lin_rtol_first=0.0), dict(lin_rtol_first=1.0), dict(parareal_theta=3),
                dict(theta_ref_k=-1.0), dict(parareal_pipeline=-1), dict(parareal_pipeline=3),
                dict(mu_s=0.0), dict(lambda_s=-1.0), dict(lambda_s=float("nan")), dict(inflow_peak=float("inf")),
                dict(theta0=-0.5), dict(lps_alpha0=-1.0), dict(cip_gamma=-1e-4), dict(vanka_omega=0.0),
                dict(vanka_omega=2.0), dict(newton_rtol=0.0), dict(lin_rtol=1.0), dict(rho_s=float("nan")),
                dict(batch_split=-1), dict(batch_split=9), dict(batch_split=3), dict(newton_res_rtol=0.0),
                dict(newton_res_rtol=1.0), dict(newton_res_rtol=float("nan")), dict(newton_guess=-1),
                dict(newton_guess=4), dict(precond_lps_scale=-1.0),
                dict(precond_lps_scale=float("nan"))):
        p = fsi.make_params(synth.workload("c1"), max_batch=2)
        for k, v in bad.items():
            setattr(p, k, v)
        assert lib.fsi_setup(C.byref(p), C.byref(h)) == fsi.FSI_ERR_ARG, bad
    p = fsi.make_params(synth.workload("c1"), max_batch=2)
    p.rho_f = -1.0
    assert lib.fsi_setup(C.byref(p), C.byref(h)) == fsi.FSI_ERR_ARG
    st = fsi.Stats()
    t0 = (C.c_double * 1)(0.0)
    assert lib.fine_propagate(None, 1, t0, 0.1, 2, None, None, C.byref(st), None) == fsi.FSI_ERR_ARG
    assert lib.coarse_propagate(None, 1, t0, 0.1, 2, None, None, None, None) == fsi.FSI_ERR_ARG
    assert lib.parareal_run(None, 1.0, 2, 2, 1, 1e-8, 2, None, None, None, None) == fsi.FSI_ERR_ARG
    lib.fsi_destroy(None)


def test_batch_split_defaults():
    """Three concurrent slice groups by default, never more groups than slices; an explicit value is kept."""
    from paper_1907_01252_amd import fsi
    import synth
    w = synth.workload("c1")
    assert fsi.make_params(w, max_batch=8).batch_split == 3
    assert fsi.make_params(w, max_batch=2).batch_split == 2
    assert fsi.make_params(w, max_batch=1).batch_split == 0
    assert fsi.make_params(w, max_batch=8, batch_split=0).batch_split == 0
    assert fsi.make_params(w, max_batch=8, batch_split=4).batch_split == 4


def test_tuned_choices_are_applied(tmp_path, monkeypatch):
    """make_params applies the autotuner's stored choices for the problem's key, unless the caller
    sets a choice itself or asks for tuned=False."""
    import json
    import synth
    from paper_1907_01252_amd import autotune, fsi
    w = synth.workload("c1")
    key = autotune.table_key(2, w["level"], "fp64", 8)
    path = tmp_path / "tuned.json"
    path.write_text(json.dumps({key: {"choice": {"batch_split": 2, "spmv_slice_fast": 0, "vanka_slice_fast": 1}}}))
    monkeypatch.setattr(autotune, "TABLE", str(path))
    p = fsi.make_params(w, max_batch=8)
    assert (p.batch_split, p.spmv_slice_fast, p.vanka_slice_fast) == (2, 0, 1)
    p = fsi.make_params(w, max_batch=8, spmv_slice_fast=1)
    assert (p.batch_split, p.spmv_slice_fast) == (2, 1)
    p = fsi.make_params(w, max_batch=8, tuned=False)
    assert (p.batch_split, p.spmv_slice_fast, p.vanka_slice_fast) == (3, -1, -1)
    p = fsi.make_params(w, max_batch=4)   # another key: the table does not apply
    assert (p.batch_split, p.spmv_slice_fast) == (3, -1)


def test_tuned_choices_follow_the_hardware_queues(tmp_path, monkeypatch):
    """An entry tuned with more hardware queues applies only to a process that has them; the
    default-queue entry serves every other count."""
    import json
    import synth
    from paper_1907_01252_amd import autotune, fsi
    w = synth.workload("c1")
    k4 = autotune.table_key(2, w["level"], "fp64", 8)
    k8 = autotune.table_key(2, w["level"], "fp64", 8, 8)
    assert k8 == k4 + "-q8"
    path = tmp_path / "tuned.json"
    path.write_text(json.dumps({k4: {"choice": {"batch_split": 2}}, k8: {"choice": {"batch_split": 4}}}))
    monkeypatch.setattr(autotune, "TABLE", str(path))
    monkeypatch.delenv("GPU_MAX_HW_QUEUES", raising=False)
    assert fsi.make_params(w, max_batch=8).batch_split == 2
    monkeypatch.setenv("GPU_MAX_HW_QUEUES", "8")
    assert fsi.make_params(w, max_batch=8).batch_split == 4
    monkeypatch.setenv("GPU_MAX_HW_QUEUES", "16")   # no entry of its own: the default one
    assert fsi.make_params(w, max_batch=8).batch_split == 2
    assert 4 in autotune.candidates(2, 8)["batch_split"] and 4 not in autotune.candidates(2, 4)["batch_split"]


def test_solver_defaults_by_precision_and_degree():
    """make_params: the measured solver defaults per dimension, precision and element degree, and
    the caller's settings over them."""
    import synth
    from paper_1907_01252_amd import fsi

    def mp(name, **kw):
        return fsi.make_params(synth.workload(name), **kw)
    p = mp("c2")                                    # 2d FP64
    assert (p.lin_rtol, p.vanka_sweeps, p.vanka_sweeps_coarse, p.newton_guess) == (1e-5, 2, 1, 3)
    assert abs(p.vanka_omega - 0.9) < 1e-15
    p = mp("c3")                                    # 2d mixed
    assert (p.lin_rtol, p.vanka_sweeps, p.vanka_sweeps_coarse, p.newton_guess) == (1e-3, 1, 2, 3)
    p = mp("c5")                                    # 3d mixed
    assert (p.lin_rtol, p.vanka_sweeps, p.vanka_sweeps_coarse, p.newton_guess) == (1e-4, 1, 1, 1)
    assert abs(p.vanka_omega - 0.6) < 1e-15
    p = mp("c5", precision="fp64")                  # 3d FP64
    assert (p.lin_rtol, p.vanka_sweeps) == (1e-5, 2)
    p = mp("c2q2")                                  # Q2 FP64
    assert (p.degree, p.vanka_sweeps, p.precond_lps_scale, p.lin_rtol) == (2, 1, 2.0, 1e-5)
    p = mp("c3q2")                                  # Q2 mixed
    assert (p.degree, p.vanka_sweeps, p.vanka_sweeps_coarse, p.lin_rtol) == (2, 1, 2, 1e-3)
    p = mp("c3", lin_rtol=1e-6, vanka_sweeps=2)     # the caller's settings win
    assert (p.lin_rtol, p.vanka_sweeps, p.vanka_sweeps_coarse) == (1e-6, 2, 2)
