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
