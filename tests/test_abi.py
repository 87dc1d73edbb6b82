"""CPU-side checks of the C ABI: the library loads, exports every function
the headers declare, and its host-only logic (workspace sizing) behaves.
No GPU work is launched here."""
import ctypes
import os
import re

import pytest

import paper_2207_00514_amd as emst

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", h)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(emst_[a-z_0-9]+)\s*\(", text)
    return sorted(set(names))


def test_headers_declare_the_binding_exports():
    assert set(declared_functions()) == set(emst.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(emst.LIB_PATH)
    for name in declared_functions():
        assert hasattr(L, name), name


def test_library_is_built_for_gfx950():
    data = open(emst.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_workspace_bytes():
    wb = emst.workspace_bytes
    assert wb(-1, 3) == 0 and wb(10, 4) == 0 and wb(10, 1) == 0 and wb(2 ** 31, 3) == 0
    assert wb(0, 3) > 0 and wb(1, 2) > 0
    prev = 0
    for n in (2, 10, 1000, 10 ** 5, 10 ** 6, 37 * 10 ** 6):
        b = wb(n, 3)
        assert b > prev and b % 256 == 0
        prev = b
    # linear growth, about 225 bytes per 3D point
    per_pt = (wb(10 ** 7, 3) - wb(10 ** 6, 3)) / 9e6
    assert 120 < per_pt < 260
    assert wb(10 ** 6, 2) < wb(10 ** 6, 3)


def test_error_strings_without_a_context():
    L = emst.lib()
    assert L.emst_last_error(None) == b"null context"
    assert L.emst_build(None, None, 0, 3, None, None, None, None, 0, None) == -1


def test_oracle_is_not_imported_by_the_product_path():
    src = open(os.path.join(ROOT, "paper_2207_00514_amd", "__init__.py")).read()
    assert "oracle" not in src.replace("no CPU fallback", "")
    for f in os.listdir(os.path.join(ROOT, "paper_2207_00514_amd", "csrc")):
        assert "oracle" not in open(os.path.join(ROOT, "paper_2207_00514_amd", "csrc", f)).read().lower()


def test_stats_struct_matches_the_header(tmp_path):
    """The binding's emst_stats mirror has the C struct's size and offsets."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    fields = [f for f, _ in emst.Stats._fields_]
    src = tmp_path / "sz.c"
    src.write_text(
        '#include <stddef.h>\n#include <stdio.h>\n#include "emst.h"\nint main(void){\n'
        '  printf("%zu\\n", sizeof(emst_stats));\n'
        + "".join(f'  printf("%zu\\n", offsetof(emst_stats, {f}));\n' for f in fields)
        + "  return 0;\n}\n")
    exe = tmp_path / "sz"
    subprocess.check_call([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert out[0] == ctypes.sizeof(emst.Stats)
    assert out[1:] == [getattr(emst.Stats, f).offset for f in fields]


def test_noalloc_limit_matches_the_header():
    """The binding's copy of EMST_NOALLOC_WORKSPACE_BYTES equals the header's,
    and the entry point rejects a missing context before any device work."""
    text = open(os.path.join(ROOT, "include", "emst.h")).read()
    m = re.search(r"#define EMST_NOALLOC_WORKSPACE_BYTES \((\d+)u << (\d+)\)", text)
    assert m, "EMST_NOALLOC_WORKSPACE_BYTES not found"
    assert emst.NOALLOC_WORKSPACE_BYTES == int(m.group(1)) << int(m.group(2))
    L = emst.lib()
    assert L.emst_build_noalloc(None, None, 10, 3, None, None, None, None) == -1
    # the documented capacity: about 280,000 3D and 300,000 2D points
    wb = emst.workspace_bytes
    assert wb(270_000, 3) <= emst.NOALLOC_WORKSPACE_BYTES < wb(290_000, 3)
    assert wb(290_000, 2) <= emst.NOALLOC_WORKSPACE_BYTES < wb(320_000, 2)
