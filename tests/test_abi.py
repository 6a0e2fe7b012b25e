"""The C-ABI library loads and exports every symbol include/frmi.h declares; host-side
argument checks (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "frmi.h")
LIB = os.path.join(ROOT, "paper_2408_16509_amd", "libfrmi.so")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(fr_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_four_entry_points():
    names = declared()
    for n in ("fr_setup_mesh", "fr_rhs", "fr_rk_step", "fr_filter"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfrmi.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfrmi.so not built")
def test_binding_covers_header_and_argument_errors():
    from paper_2408_16509_amd import frmi
    assert set(frmi.EXPORTS) == set(declared())
    p = frmi.default_params()
    assert p.struct_size == ctypes.sizeof(frmi.FrParams) and p.order == 3 and abs(p.gamma - 1.4) < 1e-15
    lib = frmi.lib()
    h = ctypes.c_void_p()
    # NULL arrays -> FR_ERR_ARG before any device work
    assert lib.fr_setup_mesh(ctypes.byref(p), 0, None, None, 0, None, None, None, ctypes.byref(h)) == 1
    assert b"empty" in lib.fr_last_error(None)
    bad = frmi.default_params()
    bad.struct_size = 3
    assert lib.fr_setup_mesh(ctypes.byref(bad), 1, None, None, 1, None, None, None, ctypes.byref(h)) == 1
    # NULL context calls fail cleanly
    assert lib.fr_rhs(None, None, None) == 1
    assert lib.fr_sync(None) == 1
    ap = frmi.FrAdaptiveParams()
    lib.fr_default_adaptive_params(ctypes.byref(ap))
    assert ap.atol == 1e-6 and ap.fac_max == 2.5 and ap.max_attempts == 100000
    assert lib.fr_rk_adaptive(None, None, 1.0, 0.1, ctypes.byref(ap), None) == 1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfrmi.so not built")
def test_mesh_errors_are_reported_before_device_work():
    from paper_2408_16509_amd import frmi, inputs
    lib = frmi.lib()

    def setup(m, **kw):
        p = frmi.default_params(**kw)
        h = ctypes.c_void_p()
        xyz = np.ascontiguousarray(m.xyz)
        per = np.ascontiguousarray(m.period, dtype=np.float64)
        et = np.ascontiguousarray(m.etype, dtype=np.int32)
        en = np.ascontiguousarray(m.enodes, dtype=np.int64)
        st = lib.fr_setup_mesh(ctypes.byref(p), xyz.shape[0], xyz.ctypes.data, per.ctypes.data, et.shape[0],
                               et.ctypes.data, en.ctypes.data, None, ctypes.byref(h))
        return st, lib.fr_last_error(None).decode()

    m = inputs.hex_box((2, 2, 2))
    m.period = np.zeros(3)                       # not periodic -> boundary faces unpaired
    st, msg = setup(m)
    assert st == 2 and "partner" in msg
    m = inputs.hex_box((2, 2, 2))
    m.enodes[0] = m.enodes[0][[1, 0, 3, 2, 5, 4, 7, 6]]   # mirrored element: J < 0
    st, msg = setup(m)
    assert st == 2 and "J <= 0" in msg
    st, msg = setup(inputs.hex_box((2, 2, 2)), order=5)
    assert st == 7
    st, msg = setup(inputs.kuhn_split(inputs.hex_box((1, 1, 1))), order=3)
    assert st == 7 and "order 4" in msg
    m = inputs.hex_box((2, 2, 2))
    m.enodes[0, 0] = 10 ** 6
    st, msg = setup(m)
    assert st == 1
    # pyramids: meshes of pyramids only, order 4, affine (parallelogram) bases
    st, msg = setup(inputs.transition_box((4, 1, 1)), order=4)
    assert st == 7 and "pyramids only" in msg
    st, msg = setup(inputs.pyramid_box((2, 2, 2)), order=3)
    assert st == 7 and "order 4" in msg
    m = inputs.pyramid_box((2, 2, 2))
    m.xyz = m.xyz.copy()
    m.xyz[m.enodes[0, 2]] += np.array([0.0, 0.0, 0.05])
    st, msg = setup(m, order=4)
    assert st == 2 and "parallelogram" in msg
    m = inputs.pyramid_box((2, 2, 2))
    m.etype = m.etype.copy()
    m.etype[0] = 3
    st, msg = setup(m, order=4)
    assert st == 1 and "unknown element type" in msg
    # parameter errors
    for kw, word in ((dict(filt_bits=31), "filt_bits"), (dict(filt_zeta_max_coef=0.0), "zeta"),
                     (dict(filt_eps_s=-1.0), "tolerance"), (dict(gamma=1.0), "gamma"),
                     (dict(precision=1, u_ref=(1.0, 0.5, 0.0, 0.0, 2.5)), "rest"), (dict(elem_order=3), "elem_order")):
        st, msg = setup(inputs.hex_box((1, 1, 1)), **kw)
        assert st == 1 and word in msg, (kw, msg)
    # the BF16x3 split products exist for the dense tetrahedral operators only
    st, msg = setup(inputs.hex_box((2, 2, 2)), precision=2, u_ref=(1.0, 0.0, 0.0, 0.0, 2.5))
    assert st == 7 and "tetrahedra" in msg


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfrmi.so not built")
def test_curved_setup_errors_before_device_work():
    from paper_2408_16509_amd import frmi, inputs
    lib = frmi.lib()

    def setup(m, q=None, **kw):
        p = frmi.default_params(**kw)
        h = ctypes.c_void_p()
        xyz = np.ascontiguousarray(m.xyz)
        per = np.ascontiguousarray(m.period, dtype=np.float64)
        ho = np.ascontiguousarray(m.ho_enodes, dtype=np.int64)
        st = lib.fr_setup_mesh_curved(ctypes.byref(p), m.geo_order if q is None else q, xyz.shape[0],
                                      xyz.ctypes.data, per.ctypes.data, ho.shape[0], ho.ctypes.data, None,
                                      ctypes.byref(h))
        return st, lib.fr_last_error(None).decode()

    m = inputs.curved_hex_box((2, 2, 2), q=3)
    assert setup(m, order=2)[0] == 7                        # q above the solution order
    assert setup(m, q=0, order=3)[0] == 7
    assert setup(inputs.curved_hex_box((1, 1, 1), q=4), q=5, order=4)[0] == 7
    st, msg = setup(m, order=3, hex_metric=2)
    assert st == 1 and "hex_metric" in msg
    bad = inputs.curved_hex_box((2, 2, 2), q=2)
    bad.ho_enodes[1, 4] = -1
    assert setup(bad, order=3)[0] == 1
    # a folded element (displacement gradient above 1): J <= 0 somewhere
    st, msg = setup(inputs.curved_hex_box((2, 2, 2), q=2, amp=1.5), order=3)
    assert st == 2 and "J <= 0" in msg
    h = ctypes.c_void_p()
    assert lib.fr_setup_mesh_curved(None, 2, 0, None, None, 0, None, None, ctypes.byref(h)) == 1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfrmi.so not built")
def test_curved_tet_setup_errors_before_device_work():
    from paper_2408_16509_amd import frmi, inputs
    lib = frmi.lib()

    def setup(m, q=None, **kw):
        p = frmi.default_params(**kw)
        h = ctypes.c_void_p()
        xyz = np.ascontiguousarray(m.xyz)
        per = np.ascontiguousarray(m.period, dtype=np.float64)
        ho = np.ascontiguousarray(m.ho_enodes, dtype=np.int64)
        st = lib.fr_setup_mesh_curved_tet(ctypes.byref(p), m.geo_order if q is None else q, xyz.shape[0],
                                          xyz.ctypes.data, per.ctypes.data, ho.shape[0], ho.ctypes.data, None,
                                          ctypes.byref(h))
        return st, lib.fr_last_error(None).decode()

    m = inputs.curved_tet_box((2, 2, 2), q=3)
    st, msg = setup(m, order=3)                              # tetrahedra exist at order 4 only
    assert st == 7 and "order 4" in msg
    assert setup(m, q=0, order=4)[0] == 7
    assert setup(m, q=5, order=4)[0] == 7
    st, msg = setup(m, order=4, hex_metric=2)
    assert st == 1 and "hex_metric" in msg
    bad = inputs.curved_tet_box((2, 2, 2), q=2)
    bad.ho_enodes[3, 5] = bad.xyz.shape[0]
    assert setup(bad, order=4)[0] == 1
    # a folded element (displacement gradient above 1): J <= 0 somewhere
    st, msg = setup(inputs.curved_tet_box((2, 2, 2), q=2, amp=1.5), order=4)
    assert st == 2 and "J <= 0" in msg
    h = ctypes.c_void_p()
    assert lib.fr_setup_mesh_curved_tet(None, 2, 0, None, None, 0, None, None, ctypes.byref(h)) == 1
