"""Host-side checks of the C ABI: the library loads and exports every entry
point include/tgks.h declares; parameter defaults carry the paper's
constants.  No kernel is launched."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tgks.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|int64_t|void)\s+(tgks_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2309_10534_amd import tgks
    if not os.path.exists(tgks.LIB_PATH):
        pytest.skip("libtgks.so not built")
    return tgks.lib()


def test_header_declares_entry_points():
    names = declared()
    for n in ("tgks_create", "tgks_step", "tgks_run", "tgks_cfl_dt", "tgks_status", "tgks_destroy",
              "tgks_batch_create", "tgks_batch_run", "tgks_batch_status", "tgks_batch_tune"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_params_default_constants(lib):
    from paper_2309_10534_amd import tgks
    p = tgks.tgks_params_default(2, [8, 8], [0.1, 0.1])
    assert p.gamma == 1.4 and p.c1 == 0.01 and p.c2 == 1.0
    assert p.ct1 == 1e-7 and p.ct2 == 1e-5 and p.eps == 1e-40 and p.q == 7
    assert p.tau_mode == tgks.TAU_INVISCID and p.bc_lo[0] == tgks.BC_TRANSMISSIVE
    assert ctypes.sizeof(p) == ctypes.sizeof(tgks.TgksParams)


def test_create_rejects_invalid_parameters_without_device(lib):
    from paper_2309_10534_amd import tgks
    h = ctypes.c_void_p()
    for bad in ({"ndim": 4}, {"n": (2, 1, 1)}, {"gamma": 1.0}):
        p = tgks.tgks_params_default(1, [10], [0.1])
        for k, v in bad.items():
            if k == "n":
                p.n[0] = v[0]
            else:
                setattr(p, k, v)
        assert lib.tgks_create(ctypes.byref(p), None, ctypes.byref(h)) == -1
    p = tgks.tgks_params_default(1, [10], [0.1])
    p.bc_lo[0], p.bc_hi[0] = tgks.BC_PERIODIC, tgks.BC_TRANSMISSIVE
    assert lib.tgks_create(ctypes.byref(p), None, ctypes.byref(h)) == -1


def test_reconstruction_variables_option(lib):
    """Characteristic variables: accepted in 1-D and 2-D, rejected in 3-D
    and for unknown values (before any device work); the operation counts
    move the normal reconstruction into the per-face work."""
    from paper_2309_10534_amd import tgks
    h = ctypes.c_void_p()
    for nd, recon in ((3, 1), (2, 2), (1, -1)):
        p = tgks.tgks_params_default(nd, [8] * nd, [0.1] * nd, recon=recon)
        assert lib.tgks_create(ctypes.byref(p), None, ctypes.byref(h)) == -1
    for nd in (1, 2):
        cons = tgks.tgks_flop_counts(tgks.tgks_params_default(nd, [8] * nd, [0.1] * nd))
        char = tgks.tgks_flop_counts(tgks.tgks_params_default(nd, [8] * nd, [0.1] * nd, recon=1))
        assert char["normal"] == 0.0 and cons["normal"] > 0.0
        assert char["face"] > cons["face"] + 2 * (nd + 2) * cons["normal"]


def _c_layout(src, struct, fields, tmp_path):
    """sizeof and offsetof of a C struct, from a program compiled with gcc."""
    import subprocess
    prog = tmp_path / "layout.c"
    body = "".join(f'  printf("%zu\\n", offsetof({struct}, {f}));\n' for f in fields)
    prog.write_text(f'#include <stdio.h>\n#include <stddef.h>\n{src}\nint main(void) {{\n'
                    f'  printf("%zu\\n", sizeof({struct}));\n{body}  return 0;\n}}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-o", str(exe), str(prog)], check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    return int(out[0]), [int(x) for x in out[1:]]


def test_params_layout_matches_header(tmp_path):
    """The ctypes mirror of tgks_params has the C struct's size and field
    offsets (a mismatch would let tgks_params_default write past it)."""
    from paper_2309_10534_amd import tgks
    fields = [f for f, _ in tgks.TgksParams._fields_]
    size, offs = _c_layout(f'#include "{HEADER}"', "tgks_params", fields, tmp_path)
    assert size == ctypes.sizeof(tgks.TgksParams)
    assert offs == [getattr(tgks.TgksParams, f).offset for f in fields]


def test_oracle_params_layout(tmp_path):
    """Same for the oracle's parameter structure and its ctypes mirror."""
    from oracle import oracle as orc
    src = open(os.path.join(ROOT, "oracle", "gks_oracle.cpp")).read()
    start = src.index("typedef struct {", src.index('extern "C" {'))
    decl = src[start:src.index("} orc_params;", start) + len("} orc_params;")]
    decl = re.sub(r"//[^\n]*", "", decl)
    fields = [f for f, _ in orc.OrcParams._fields_]
    size, offs = _c_layout(decl, "orc_params", fields, tmp_path)
    assert size == ctypes.sizeof(orc.OrcParams)
    assert offs == [getattr(orc.OrcParams, f).offset for f in fields]


def test_prescribed_and_fallback_checks_without_device(lib):
    """Prescribed sides on 3-D grids, far kinds other than transmissive /
    reflective / state B, a NaN line and unknown fallback values are
    rejected before any device work."""
    from paper_2309_10534_amd import tgks
    h = ctypes.c_void_p()
    bad = [tgks.tgks_params_default(3, [8] * 3, [0.1] * 3, bc=[("prescribed", "transmissive")] * 3),
           tgks.tgks_params_default(2, [8, 8], [0.1, 0.1], fallback=2)]
    p = tgks.tgks_params_default(2, [8, 8], [0.1, 0.1], bc=[("prescribed", "transmissive")] * 2)
    p.bc_far[0][0] = tgks.BC_NOSLIP
    bad.append(p)
    p = tgks.tgks_params_default(2, [8, 8], [0.1, 0.1], bc=[("prescribed", "transmissive")] * 2)
    p.bc_line[0][0][1] = float("nan")
    bad.append(p)
    for q in bad:
        assert lib.tgks_create(ctypes.byref(q), None, ctypes.byref(h)) == -1
