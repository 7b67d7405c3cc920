"""The C-ABI library builds for gfx950, loads on the host and exports every
function declared in include/ttipm.h (no GPU work is launched here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "ttipm.h")).read()
    return sorted(set(re.findall(r"TTIPM_API\s+[\w\s\*]+?\b((?:tt|ttipm)_\w+)\s*\(", src)))


def test_header_declares_the_six_calls():
    names = _declared()
    for n in ["tt_contract_interfaces", "tt_local_matvec", "tt_local_solve", "tt_round", "ttipm_step",
              "ttipm_solve"]:
        assert n in names


def test_library_exports_all_declared_symbols():
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2509_11890_amd", "libttipm.so"))
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    lib.tt_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.tt_version()


def test_binding_structs_match_header_fields():
    """The ctypes mirror of ttipm_params / ttipm_step_info lists the header's fields in order."""
    import paper_2509_11890_amd.binding as B
    src = open(os.path.join(ROOT, "include", "ttipm.h")).read()

    def fields(struct):
        end = src.index("} " + struct + ";")
        start = src.rindex("typedef struct {", 0, end) + len("typedef struct {")
        body = src[start:end]
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        names = []
        for decl in body.split(";"):
            decl = decl.strip()
            if not decl:
                continue
            decl = re.sub(r"^(const\s+)?\w+\s*\**", "", decl)
            names += [x.strip().lstrip("*") for x in decl.split(",")]
        return names

    assert fields("ttipm_params") == [f[0] for f in B.ttipm_params._fields_]
    assert fields("ttipm_step_info") == [f[0] for f in B.ttipm_step_info._fields_]
    assert fields("ttipm_result") == [f[0] for f in B.ttipm_result._fields_]


def test_struct_sizes_match_library():
    """sizeof of every caller-visible struct agrees between the compiled library
    and the ctypes mirrors (a field of the wrong type or in the wrong place
    changes the size or the padding)."""
    import paper_2509_11890_amd.binding as B
    assert B.abi_mismatches() == []
    out = (ctypes.c_size_t * 2)()
    assert B.lib.tt_abi_sizes(out, 2) == len(B.ABI_STRUCTS)
    assert out[0] == ctypes.sizeof(B.tt_view)
