"""The C-ABI library builds for gfx950, loads without a GPU and exports every entry point that
include/hipsso.h declares (no compute calls here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hipsso.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sso_[a-z_]+)\s*\(", text)))


def _lib_path():
    from paper_2407_20026_amd import LIB_PATH
    if not os.path.exists(LIB_PATH):
        from paper_2407_20026_amd import build
        build.build()
    return LIB_PATH


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("sso_problem_create", "sso_problem_update", "sso_solve", "sso_objective",
              "sso_adjoint", "sso_pattern", "sso_strerror", "sso_problem_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(_lib_path())
    for n in _declared():
        assert hasattr(lib, n), n


def test_binding_names_match_header():
    import paper_2407_20026_amd as sso
    assert sorted(sso.EXPORTS) == _declared()
    lib = sso.load_library()
    assert lib.sso_strerror(-5).decode().startswith("PCG breakdown")
    assert lib.sso_strerror(0).decode() == "ok"


def test_create_rejects_bad_arguments_without_touching_the_gpu():
    """Argument checks that happen before any device call."""
    import paper_2407_20026_amd as sso
    lib = sso.load_library()
    h = ctypes.c_void_p()
    m = sso.sso_mesh()
    m.n_nodes = 0
    assert lib.sso_problem_create(ctypes.byref(m), None, None, ctypes.byref(h)) == sso.SSO_EINVAL
    m.n_nodes = 4
    m.n_beams = -1
    assert lib.sso_problem_create(ctypes.byref(m), None, None, ctypes.byref(h)) == sso.SSO_EINVAL
    assert lib.sso_solve(None, None, None) == sso.SSO_EINVAL
    assert lib.sso_adjoint(None, 0, None, None, None, None, None) == sso.SSO_EINVAL
    assert lib.sso_batch_profile(None, 1, 8) == sso.SSO_EINVAL
    assert lib.sso_batch_timing(None, None, None, None, None) == sso.SSO_EINVAL


def test_struct_layouts_match_the_header(tmp_path):
    """sizeof and every member offset of sso_mesh, sso_options and sso_stats as the C compiler
    lays them out from include/hipsso.h, against the ctypes structures of the binding."""
    import shutil
    import subprocess
    import pytest
    import paper_2407_20026_amd as sso
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "hipsso.h"',
             "int main(void) {"]
    structs = (sso.sso_mesh, sso.sso_options, sso.sso_stats)
    for st in structs:
        name = st.__name__
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for f, _ in st._fields_:
            lines.append(f'  printf("{name}.{f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    "-I" + os.path.join(ROOT, "include"), "-o", str(exe), str(src)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], check=True, capture_output=True,
                                                 text=True).stdout.splitlines())
    for st in structs:
        name = st.__name__
        assert int(got[name]) == ctypes.sizeof(st), name
        for f, _ in st._fields_:
            assert int(got[f"{name}.{f}"]) == getattr(st, f).offset, (name, f)


def test_library_exports_the_ceiling_probes():
    text = open(os.path.join(ROOT, "include", "hipsso_ceiling.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = sorted(set(re.findall(r"\b(hipsso_ceiling_[a-z_]+)\s*\(", text)))
    from paper_2407_20026_amd import ceiling
    assert names == sorted(ceiling.EXPORTS)
    lib = ctypes.CDLL(_lib_path())
    for n in names:
        assert hasattr(lib, n), n


def test_size_penalty_update_matches_the_oracle_rule():
    """The host-only penalty rule of the C ABI against the oracle's (no GPU call)."""
    import paper_2407_20026_amd as sso
    from oracle import extras
    for eps1, violated, kappa in ((2.0, True, 1.015), (2.03, False, 1.015), (1.0, True, 1.1),
                                  (0.0, True, 1.015), (5.0, False, 2.0)):
        assert sso.Problem.update_eps1(eps1, violated, kappa) == \
            extras.update_eps1(eps1, violated, kappa)
    lib = sso.load_library()
    out = ctypes.c_double()
    for bad in ((-1.0, 1, 1.015), (1.0, 1, 0.0), (float("nan"), 0, 1.015),
                (1.0, 0, float("inf"))):
        assert lib.sso_size_penalty_update(*bad, ctypes.byref(out)) == sso.SSO_EINVAL
    assert lib.sso_size_penalty_update(1.0, 1, 1.015, None) == sso.SSO_EINVAL
