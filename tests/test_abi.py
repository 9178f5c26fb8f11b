"""Host-side checks of the C ABI: the library loads and exports every symbol
the header declares, and the ctypes layouts match the header's structs."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chisao.h")


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(chisao_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("chisao_init", "chisao_cycle", "chisao_modes"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2606_26164_amd import _lib

    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libchisao.so is not built; run `python -m paper_2606_26164_amd.build`")
    lib = C.CDLL(_lib.LIB_PATH)
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert set(_declared_functions()) == set(_lib.EXPORTS)


def test_header_constants_match_the_binding():
    """Every integer #define of the header has the same value in _lib."""
    from paper_2606_26164_amd import _lib

    text = open(HEADER).read()
    defs = dict(re.findall(r"#define CHISAO_([A-Z0-9_]+)\s+\(?(-?\d+)u?\)?", text))
    assert len(defs) >= 20
    for name, val in defs.items():
        if name in ("PROF_CLASSES",):
            assert _lib.PROF_CLASSES == int(val)
            continue
        if name.startswith("PROF_"):
            assert _lib.PROF_NAMES[int(val)] == name[5:].lower(), name
            continue
        if name == "TUNE_VARIANTS":
            assert _lib.TUNE_VARIANTS == int(val)
            continue
        assert hasattr(_lib, name), name
        assert getattr(_lib, name) == int(val), name


def test_ctypes_struct_layouts_match_header():
    """Compile a tiny C program that prints sizeof/offsetof of the header's
    structs and compare with the ctypes declarations."""
    import subprocess
    import tempfile

    from paper_2606_26164_amd import _lib

    m = {"chisao_problem": _lib.Problem, "chisao_config": _lib.Config, "chisao_cycle_stats": _lib.CycleStats,
         "chisao_state": _lib.State, "chisao_kernel_profile": _lib.KernelProfile,
         "chisao_tuning_entry": _lib.TuningEntry}
    lines = []
    for t, cls in m.items():
        lines.append(f'  printf("{t} size %zu\\n", sizeof({t}));')
        lines += [f"  P({t}, {f})" for f, _ in cls._fields_]
    src = ("#include <stddef.h>\n#include <stdio.h>\n#include \"chisao.h\"\n"
           "#define P(T, f) printf(#T \" \" #f \" %zu\\n\", offsetof(T, f));\n"
           "int main(void) {\n" + "\n".join(lines) + "\n  return 0;\n}\n")
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "l.c")
        open(c, "w").write(src)
        exe = os.path.join(td, "l")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln.strip():
            t, f, v = ln.split()
            got[(t, f)] = int(v)
    assert len(got) == sum(len(c._fields_) + 1 for c in m.values())
    for (t, f), v in got.items():
        cls = m[t]
        if f == "size":
            assert C.sizeof(cls) == v, (t, C.sizeof(cls), v)
        else:
            assert getattr(cls, f).offset == v, (t, f)
