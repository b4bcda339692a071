"""The C-ABI library loads and exports every function include/frmi.h declares
(CPU only: no GPU call is made)."""

import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "frmi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fr_[a-zA-Z0-9_]+)\s*\(", src)))


def test_header_declares_the_hot_path_calls():
    names = declared_functions()
    for n in ["fr_degrid", "fr_grid", "fr_make_psf_kernel", "fr_apply_RNR_approx",
              "fr_apply_RNR_exact", "fr_likelihood_grad", "fr_cg_solve"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2406_09144_amd import _lib
    lib = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the Python binding covers the same set
    assert set(declared_functions()) == set(_lib.SIGNATURES)


def test_version_and_error_string_without_gpu():
    from paper_2406_09144_amd import _lib
    lib = _lib.load(import_torch=False)
    assert lib.fr_version().startswith(b"frmi")
    assert lib.fr_last_error() is not None


def test_plan_info_binding_matches_header():
    """The ctypes fr_plan_info lists the header's fields, in order, with C types of
    the same size (a drifted layout would misread every field after the change)."""
    from paper_2406_09144_amd import _lib
    src = open(os.path.join(ROOT, "include", "frmi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct(?:\s+fr_plan_info)?\s*\{(.*?)\}\s*fr_plan_info\s*;", src, flags=re.S).group(1)
    sizes = {"int64_t": 8, "int": 4, "double": 8, "size_t": 8}
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        ctype, names = decl.split(None, 1)
        for name in names.split(","):
            fields.append((name.strip(), sizes[ctype]))
    binding = [(name, ctypes.sizeof(t)) for name, t in _lib.fr_plan_info._fields_]
    assert binding == fields


def test_binding_constants_match_header():
    """Status codes, plan flags and mode enums of the binding equal the header's."""
    from paper_2406_09144_amd import _lib
    src = open(os.path.join(ROOT, "include", "frmi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    consts = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(FR_[A-Z0-9_]+)\s*=\s*(-?\d+)", src)}
    assert len(consts) >= 20
    for name, value in consts.items():
        assert getattr(_lib, name) == value, name
