"""CPU checks of the C ABI: the library loads, exports every function that
include/pic.h declares, and validates configurations on the host."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "pic.h")).read()
    return sorted(set(re.findall(r"^(?:pic_status|const char \*)\s*(pic_\w+)\s*\(", src, re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1906_06306_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libpic.so not built: run __graft_entry__.build()")
    return _lib


def test_exports_match_header(lib):
    names = declared_functions()
    assert len(names) >= 10
    L = ctypes.CDLL(lib.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(lib.EXPORTS)


def test_constants_match_header(lib):
    src = open(os.path.join(ROOT, "include", "pic.h")).read()
    seen = 0
    for name, val in re.findall(r"^#define (PIC_\w+) (\(1 << \d+\)|\d+)u?\b", src, re.M):
        v = 1 << int(val[6:-1]) if val.startswith("(") else int(val)
        if hasattr(lib, name):
            assert getattr(lib, name) == v, name
            seen += 1
    assert seen >= 20 and lib.PIC_DEPOSIT_CURL_E == 8


def make_cfg(lib, D=2, n=(64, 64, 1), T=(16, 16, 1), prec=0, cfl=0.45, ns=2):
    cells = np.array([list(n)], dtype=np.int32)
    q = np.array([[-1e-3, 1e-3][:ns]], dtype=np.float64)
    s = np.array([[-1.0, 1.0][:ns]], dtype=np.float64)
    m = np.abs(q)
    cfg = lib.PicConfig()
    cfg.dim, cfg.precision, cfg.n_species, cfg.n_boxes = D, prec, ns, 1
    for d in range(3):
        cfg.tile[d] = T[d]
    cfg.cfl = cfl
    cfg.box_cells, cfg.charge, cfg.qm, cfg.mass = (cells.ctypes.data, q.ctypes.data, s.ctypes.data,
                                                   m.ctypes.data)
    return cfg, (cells, q, s, m)


def query(lib, cfg, counts):
    lay = lib.PicLayout()
    code = lib.lib().pic_query(ctypes.byref(cfg), counts.ctypes.data, ctypes.byref(lay))
    return code, lay


def test_query_layout(lib):
    cfg, keep = make_cfg(lib)
    counts = np.array([[4096 * 4, 4096 * 4]], dtype=np.int64)
    code, lay = query(lib, cfg, counts)
    assert code == 0
    assert lay.cells_total == 64 * 64 and lay.tiles_total == 16
    assert lay.elem_bytes == 4
    # capacity: ceil(1.25 * 1024) + 64 rounded up to the push group of
    # 256 threads x 1 particle, per tile and species
    per = -(-int(np.ceil(1.25 * 1024) + 64) // 256) * 256
    assert lay.capacity_total == per * 16 * 2
    offs = [lay.off_E, lay.off_B, lay.off_J, lay.off_pos, lay.off_u, lay.off_xold, lay.off_seg_offset,
            lay.off_seg_capacity, lay.off_seg_count, lay.off_error, lay.off_flags]
    assert all(o % 256 == 0 for o in offs)
    assert offs == sorted(offs) and lay.total_bytes > offs[-1]
    assert lay.off_B - lay.off_E >= 3 * 4096 * 4


@pytest.mark.parametrize("change,msg", [
    (dict(D=4), "dim"),
    (dict(T=(15, 16, 1)), "even"),
    (dict(T=(24, 16, 1)), "divide"),
    (dict(cfl=0.8), "cfl"),
    (dict(ns=0), "n_species"),
])
def test_query_rejects_bad_config(lib, change, msg):
    kw = dict(D=2, n=(64, 64, 1), T=(16, 16, 1), cfl=0.45, ns=2)
    kw.update(change)
    cfg, keep = make_cfg(lib, **kw)
    code, _ = query(lib, cfg, np.array([[100, 100]], dtype=np.int64))
    assert code == lib.PIC_E_ARG
    assert msg in lib.lib().pic_last_error().decode()


def test_null_context_is_an_argument_error(lib):
    L = lib.lib()
    assert L.pic_step(None, 0) == lib.PIC_E_ARG
    assert L.pic_error(None) == lib.PIC_E_ARG
    assert L.pic_destroy(None) == 0
