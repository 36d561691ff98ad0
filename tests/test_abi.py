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
