"""Host-side checks of the C ABI: the library loads, exports every entry
point include/dmpt.h declares, and rejects bad arguments before touching a
device.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dmpt.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dmpt_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1503_07037_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    return _lib.load()


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("dmpt_init", "dmpt_fermi_recursion", "dmpt_response", "dmpt_mu_newton",
              "dmpt_backward", "dmpt_mu_newton_batched", "dmpt_finalize", "dmpt_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_default_options(lib):
    from paper_1503_07037_amd import _lib as L
    o = L.Options()
    lib.dmpt_default_options(ctypes.byref(o))
    assert o.prec == 0 and o.solver == 0 and o.max_newton == 50 and o.max_cg == 60
    assert o.staged == 1 and o.ckpt_every == 5


def test_null_context_is_rejected(lib):
    from paper_1503_07037_amd import _lib as L
    s = L.Stats()
    assert lib.dmpt_fermi_recursion(None, 4, None, 1.0, 0.0, 10, None, ctypes.byref(s)) == L.DMPT_ERR_ARG
    assert lib.dmpt_mu_newton(None, 4, None, 0, None, None, None, 1.0, 2.0, 10, 0, None, None, None,
                              None, None, None) == L.DMPT_ERR_ARG
    assert lib.dmpt_backward(None, 4, None, 1.0, 2.0, 10, None, None, None, None) == L.DMPT_ERR_ARG
    assert lib.dmpt_congruence(None, 4, None, None, None, 0, None) == L.DMPT_ERR_ARG
    assert lib.dmpt_finalize(None) == L.DMPT_OK
    assert lib.dmpt_last_error(None)


def test_init_argument_checks(lib):
    from paper_1503_07037_amd import _lib as L
    h = ctypes.c_void_p()
    assert lib.dmpt_init(None, 0, 128, 1, None, None) == L.DMPT_ERR_ARG
    assert lib.dmpt_init(ctypes.byref(h), 0, 0, 1, None, None) == L.DMPT_ERR_ARG
    assert b"n_max" in lib.dmpt_last_error(None)
    assert lib.dmpt_init(ctypes.byref(h), 0, 128, 99, None, None) == L.DMPT_ERR_ARG
    o = L.Options()
    lib.dmpt_default_options(ctypes.byref(o))
    o.prec = 17
    assert lib.dmpt_init(ctypes.byref(h), 0, 128, 1, ctypes.byref(o), None) == L.DMPT_ERR_ARG
    assert not h.value


def _c_layout(struct, fields):
    """sizeof and offsetof of a header struct, from a C program compiled with gcc."""
    import json
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        pytest.skip("no C compiler")
    body = ",".join(f'\\"{f}\\":%zu' for f in fields)
    args = ", ".join(f"offsetof({struct}, {f})" for f in fields)
    src = f"""#include <stddef.h>
#include <stdio.h>
#include "dmpt.h"
int main(void) {{ printf("{{\\"size\\":%zu,{body}}}", sizeof({struct}), {args}); return 0; }}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(c, "w").write(src)
        subprocess.run([cc, "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        return json.loads(subprocess.run([exe], check=True, stdout=subprocess.PIPE, text=True).stdout)


@pytest.mark.parametrize("struct,pyname", [("dmpt_stats", "Stats"), ("dmpt_options", "Options"), ("dmpt_sparse_stats", "SparseStats"),
                                           ("dmpt_profile_data", "ProfileData")])
def test_struct_layouts_match_the_header(struct, pyname):
    """The binding's ctypes structures have the header's size and field offsets."""
    from paper_1503_07037_amd import _lib as L
    cls = getattr(L, pyname)
    names = [f[0] for f in cls._fields_]
    lay = _c_layout(struct, names)
    assert lay["size"] == ctypes.sizeof(cls)
    for n in names:
        assert lay[n] == getattr(cls, n).offset, n


def _c_values(names):
    """Values of header enumerators, from a C program compiled with gcc."""
    import json
    import shutil
    import subprocess
    import tempfile
    cc = shutil.which("gcc") or shutil.which("cc")
    if not cc:
        pytest.skip("no C compiler")
    body = ",".join(f'\\"{n}\\":%d' for n in names)
    args = ", ".join(f"(int){n}" for n in names)
    src = f"""#include <stdio.h>
#include "dmpt.h"
int main(void) {{ printf("{{{body}}}", {args}); return 0; }}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "values.c")
        exe = os.path.join(d, "values")
        open(c, "w").write(src)
        subprocess.run([cc, "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        return json.loads(subprocess.run([exe], check=True, stdout=subprocess.PIPE, text=True).stdout)


def test_binding_enum_values_match_the_header():
    """The binding's names for precision modes, solvers and guesses map to the header's values, and every
    enumerator of those enums has a name in the binding."""
    from paper_1503_07037_amd import _lib as L
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    groups = {"dmpt_prec": (L.PREC, {"fp64": "DMPT_FP64", "fp32": "DMPT_FP32", "bf16x3": "DMPT_BF16X3",
                                      "bf16x6": "DMPT_BF16X6", "int8x13": "DMPT_INT8X13", "int8x6": "DMPT_INT8X6"}),
              "dmpt_solver": (L.SOLVER, {"cg": "DMPT_SOLVER_CG", "ns": "DMPT_SOLVER_NS",
                                         "hybrid": "DMPT_SOLVER_HYBRID"}),
              "dmpt_guess": (L.GUESS, {"prev": "DMPT_GUESS_PREV", "taylor": "DMPT_GUESS_TAYLOR"})}
    for enum, (pymap, cnames) in groups.items():
        body = re.search(r"typedef enum \{([^}]*)\}\s*" + enum + r"\s*;", text).group(1)
        declared = re.findall(r"\b(DMPT_[A-Z0-9_]+)\s*=", body)
        assert sorted(declared) == sorted(cnames.values()), (enum, declared)
        vals = _c_values(list(cnames.values()))
        for py, cn in cnames.items():
            assert pymap[py] == vals[cn], (enum, py, cn)
