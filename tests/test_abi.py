"""The C-ABI library loads and exports every entry point include/csp.h
declares; the binding's constants agree with the header.  No GPU calls."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "csp.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(csp_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_1511_06441_amd import csp
    lib = ctypes.CDLL(csp.LIB_PATH)
    names = _declared()
    assert "csp_solve_dev" in names and len(names) >= 8
    for nm in names:
        assert hasattr(lib, nm), nm
    assert sorted(csp.EXPORTED) == names


def test_header_constants_match_binding():
    from paper_1511_06441_amd import csp
    text = open(HEADER).read()
    for nm in ("CSP_OK", "CSP_EINVAL", "CSP_ENOMEM", "CSP_EDEVICE", "CSP_EOVERFLOW", "CSP_ECANCELED"):
        m = re.search(rf"{nm}\s*=\s*(-?\d+)", text)
        assert m and int(m.group(1)) == getattr(csp, nm), nm
    m = re.search(r"#define CSP_MAX_M (0x[0-9A-Fa-f]+)u", text)
    assert int(m.group(1), 16) == csp.CSP_MAX_M
    m = re.search(r"#define CSP_SCRATCH_BYTES \((\d+)ull << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == csp.CSP_SCRATCH_BYTES


def test_result_struct_layout():
    from paper_1511_06441_amd import csp
    assert ctypes.sizeof(csp.csp_result) == 5 * 8
    assert ctypes.sizeof(csp.csp_counters) == 7 * 8


def test_product_path_has_no_oracle_dependency():
    """The package and the C ABI never import, include or load the oracle."""
    pat = re.compile(r"^\s*(from\s+oracle|import\s+oracle|#include\s+.*oracle)|csp_oracle|libcsp_oracle",
                     re.M)
    for base in ("paper_1511_06441_amd", "include"):
        for dirpath, _, files in os.walk(os.path.join(ROOT, base)):
            for f in files:
                if f.endswith((".py", ".hip", ".h", ".cpp")):
                    text = open(os.path.join(dirpath, f)).read()
                    assert not pat.search(text), os.path.join(dirpath, f)


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Sizes and field offsets of every struct the binding mirrors, as the C
    compiler lays them out from the header."""
    import subprocess
    from paper_1511_06441_amd import csp
    structs = {"csp_result": csp.csp_result, "csp_counters": csp.csp_counters,
               "csp_problem": csp.csp_problem, "csp_request": csp.csp_request,
               "csp_completion": csp.csp_completion}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "csp.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name} {fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert got[(name, fname)] == getattr(cls, fname).offset, (name, fname)
