"""Host-side checks of the C-ABI library: it loads, exports every declared
symbol, and its host-only entry points agree with the oracle (no GPU calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2006_05186_amd import cqm as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "cqm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(?:int|const char\*)\s+(cqm_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = C.load_library()
    names = declared_functions()
    assert len(names) >= 16
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(C.EXPORTED_SYMBOLS) <= set(names)


def test_binding_signatures_match_the_header():
    src = open(os.path.join(ROOT, "include", "cqm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    decls = re.findall(r"\b(int|const char\*)\s+(cqm_\w+)\s*\(([^)]*)\)\s*;", src)
    assert len(decls) == len(declared_functions())
    L = C.load_library()
    for ret, name, args in decls:
        args = args.strip()
        nargs = 0 if args in ("", "void") else len(args.split(","))
        f = getattr(L, name)
        assert f.argtypes is not None and len(f.argtypes) == nargs, name
        assert f.restype is (ctypes.c_char_p if ret == "const char*" else ctypes.c_int), name


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    # no fallback: every entry point goes through load_library, which raises
    monkeypatch.setattr(C, "_lib", None)
    monkeypatch.setattr(C, "library_path", lambda: str(tmp_path / "libcqm.so"))
    for call in (lambda: C.cqm_frequencies(8, 1.0), C.cqm_default_options,
                 lambda: C.cqm_ctx_create(0)):
        with pytest.raises(C.CqmError) as e:
            call()
        assert "not built" in str(e.value)


@pytest.mark.parametrize("N,T", [(8, 2.0), (32, 4.0), (64, 4.0), (128, 6.0), (256, 6.0)])
def test_host_frequencies_match_oracle(N, T):
    s = C.cqm_frequencies(N, T)
    ref, _, _ = O.frequencies(N, T)
    assert np.max(np.abs(s - ref) / np.abs(ref)) < 1e-14


@pytest.mark.parametrize("N,T,rho", [(16, 2.0, 0.5), (33, 4.0, 0.97), (64, 4.0, 10 ** (-8 / 64))])
def test_host_frequencies_with_explicit_radius(N, T, rho):
    s = C.cqm_frequencies(N, T, rho)
    ref, r, _ = O.frequencies(N, T, rho)
    assert r == rho
    assert np.max(np.abs(s - ref) / np.abs(ref)) < 1e-14


@pytest.mark.parametrize("N,T,rho", [(8, 1.0, 1.0), (8, 1.0, -0.1), (8, 0.0, 0.5), (8, -1.0, 0.0)])
def test_host_frequencies_reject_bad_arguments(N, T, rho):
    with pytest.raises(C.CqmError) as e:
        C.cqm_frequencies(N, T, rho)
    assert e.value.code == C.CQM_EINVAL


def test_host_argument_errors():
    with pytest.raises(C.CqmError) as e:
        C.cqm_frequencies(0, 1.0)
    assert e.value.code == C.CQM_EINVAL
    o = C.cqm_default_options()
    assert (o.gmres_restart, o.n_min, o.cheb_m, o.q_duffy) == (30, 32, 4, 5)
    assert o.eps_aca == 1e-6 and o.eta == 1.0 and o.outer_tol == 1e-15
    assert o.autotune == 1 and o.arnoldi_layout == C.CQM_ARNOLDI_AUTO and o.graphs == 0
    assert o.precond == C.CQM_PRECOND_BLOCK_JACOBI
    assert (o.cutoff_inner, o.cutoff_outer) == (18.0, 45.0)
    assert o.refine_plain == 1 and o.formulation == C.CQM_FORMULATION_INDIRECT


def test_server_default_options_as_documented():
    o = C.cqm_server_default_options()
    assert (o.max_active, o.cache_operators, o.large_lane, o.large_bytes) == (16, 1, 0, 0)
    d = C.cqm_default_options()
    # the solver defaults are the library's, with operator reuse switched on
    for name, _ in C.cqm_options._fields_:
        if name in ("reserved", "reuse_operator"):
            continue
        assert getattr(o.solver, name) == getattr(d, name), name
    assert o.solver.reuse_operator == 1
    with pytest.raises(C.CqmError):
        C._check(C.load_library().cqm_server_default_options(None))


def test_every_declaration_names_its_passage():
    # each function declaration (or a run of declarations with no blank line
    # between them) is preceded by a comment naming the paper's section or
    # equation it implements, or stating that it is plumbing with no passage
    src = open(os.path.join(ROOT, "include", "cqm.h")).read()
    body = src.split("extern \"C\" {", 1)[1]
    last_comment, missing = "", []
    for chunk in re.split(r"(/\*.*?\*/)", body, flags=re.S):
        if chunk.startswith("/*"):
            last_comment = chunk
            continue
        # a blank line ends the comment's scope
        for k, seg in enumerate(re.split(r"\n[ \t]*\n", chunk)):
            for name in re.findall(r"\b(?:int|const char\*)\s+(cqm_\w+)\s*\(", seg):
                if k > 0 or not re.search(r"Section \d|Paper: no passage|cannot allocate", last_comment):
                    missing.append(name)
    assert not missing, missing
    # the computing entry points cite a section, not "no passage"
    for name in ("cqm_frequencies", "cqm_apply_V", "cqm_near_entries", "cqm_solve",
                 "cqm_set_plane_wave", "cqm_problem_create", "cqm_operator_stats"):
        m = re.search(r"(/\*(?:(?!\*/).)*?\*/)\s*(?:(?:int|const char\*)\s+cqm_\w+\([^;]*;\s*)*"
                      r"(?:int|const char\*)\s+" + name + r"\s*\(", body, flags=re.S)
        assert m and re.search(r"Section \d", m.group(1)), name


def test_library_marks_its_stages_for_the_profiler():
    """Named stage ranges (roctx) around the solve's stages: the library
    imports the range calls, so rocprofv3 --marker-trace records them."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm missing")
    out = subprocess.run([nm, "-D", C.library_path()], capture_output=True, text=True).stdout
    assert "roctxRangePushA" in out and "roctxRangePop" in out
