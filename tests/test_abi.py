"""The C ABI: the built library loads (no GPU needed) and exports every function
declared in include/*.h; the binding's structures match the header layouts."""
import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def _declared():
    names = set()
    for h in (ROOT / "include").glob("*.h"):
        text = re.sub(r"/\*.*?\*/", "", h.read_text(), flags=re.S)
        names.update(re.findall(r"\b(wally_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    from paper_2406_06761_amd.wally import LIB_PATH, SYMBOLS

    if not LIB_PATH.exists():
        pytest.fail("libwally.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(str(LIB_PATH))
    declared = _declared()
    assert declared, "no declarations found"
    assert declared == set(SYMBOLS)
    for name in declared:
        assert hasattr(lib, name), name


def test_struct_layouts_match_header():
    from paper_2406_06761_amd import wally

    # wally_query: two uint32 then five pointers
    assert ctypes.sizeof(wally.Query) == 48
    assert wally.Query.ct.offset == 8 and wally.Query.out.offset == 32 and wally.Query.key_fold.offset == 40
    # wally_params_desc: 10 x 32-bit fields then the 64-bit budget
    assert ctypes.sizeof(wally.ParamsDesc) == 48 and wally.ParamsDesc.hbm_budget.offset == 40
    assert wally.ParamsInfo.q.offset == 24


def test_struct_layouts_match_a_c_compiler(tmp_path):
    """Every field offset and structure size of the binding equals what a C
    compiler gives for include/wally.h."""
    import subprocess

    from paper_2406_06761_amd import wally

    structs = {"wally_params_desc": wally.ParamsDesc, "wally_params_info": wally.ParamsInfo,
               "wally_query": wally.Query, "wally_tune_entry": wally.TuneEntry}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "wally.h"', '#include "wally_diag.h"',
             "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    dtypes = {"wally_query": wally.QUERY_DTYPE, "wally_pir_query": wally.PIR_QUERY_DTYPE,
              "wally_pir_query2": wally.PIR_QUERY2_DTYPE}
    for cname, dt in dtypes.items():
        lines.append(f'printf("np_{cname} size %zu\\n", sizeof({cname}));')
        for fname in dt.names:
            lines.append(f'printf("np_{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", str(ROOT / "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(ln.split()[:2]): int(ln.split()[2]) for ln in out if ln}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)
    for cname, dt in dtypes.items():  # the numpy record layouts the binding passes as arrays
        assert got[("np_" + cname, "size")] == dt.itemsize, cname
        for fname in dt.names:
            assert got[("np_" + cname, fname)] == dt.fields[fname][1], (cname, fname)


def test_error_strings_and_null_handling():
    from paper_2406_06761_amd import wally

    lib = wally.load()
    assert lib.wally_strerror(-3) == b"admission refused, retry later"
    assert lib.wally_params_init(None, None) == wally.EINVAL
    lib.wally_destroy(None)  # no-op
    assert lib.wally_last_error(None) == b"null context"
    assert lib.wally_pir_set_linear(None, 1) == wally.EINVAL
    # unsupported sizes are rejected before any device call
    d = wally.ParamsDesc(11, 3, 36, 20, 64, 0, 0, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    assert lib.wally_params_init(ctypes.byref(d), ctypes.byref(h)) == wally.EINVAL
    d = wally.ParamsDesc(12, 3, 36, 20, 4096, 0, 0, 0, 0, 0, 0)  # d_pad does not divide n/2
    assert lib.wally_params_init(ctypes.byref(d), ctypes.byref(h)) == wally.EINVAL
    d = wally.ParamsDesc(12, 3, 36, 20, 64, 0, 0, 32769, 0, 0, 0)  # wave beyond the grid limits
    assert lib.wally_params_init(ctypes.byref(d), ctypes.byref(h)) == wally.EINVAL
    d = wally.ParamsDesc(12, 3, 36, 20, 64, 0, 0, 0, 0, 8, 0)  # fold_max outside the folded layout
    assert lib.wally_params_init(ctypes.byref(d), ctypes.byref(h)) == wally.EINVAL
    d = wally.ParamsDesc(12, 3, 36, 20, 64, wally.LAYOUT_FOLDED, 0, 0, 0, 12, 0)  # not a power of two
    assert lib.wally_params_init(ctypes.byref(d), ctypes.byref(h)) == wally.EINVAL
    # dimensions whose baby-step count has no giant-step sum kernel (g = 1 and g = 64)
    for dim in (1, 1025, 2048):
        d = wally.ParamsDesc(13, 3, 36, 20, dim, 0, 0, 0, 0, 0, 0)
        assert lib.wally_params_init(ctypes.byref(d), ctypes.byref(h)) == wally.EINVAL, dim
        assert not h.value


def test_library_is_newer_than_its_sources():
    """A failed rebuild leaves the previous library in place; catch it here
    rather than measuring or testing stale code."""
    from paper_2406_06761_amd.wally import LIB_PATH

    if not LIB_PATH.exists():
        pytest.skip("library not built")
    root = Path(__file__).resolve().parents[1]
    sources = list((root / "paper_2406_06761_amd" / "csrc").glob("*")) + list((root / "include").glob("*.h"))
    newest = max(p.stat().st_mtime for p in sources)
    assert LIB_PATH.stat().st_mtime >= newest, "libwally.so is older than its sources: rebuild failed or was skipped"
