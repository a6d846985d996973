"""C ABI without a GPU: the library loads, exports every function the
header declares, and rejects bad inputs with the documented status codes
before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_0712_1695_amd as bs
import workloads as W

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "bs.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(bs_\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = bs.load_library()
    declared = _declared_functions()
    assert sorted(bs.EXPORTS) == declared
    for name in declared:
        assert hasattr(L, name), name


def test_policy_defaults_and_status_strings():
    p = bs.bs_policy_default()
    assert (p.kind, p.n_phi, p.n_theta, p.precision) == (bs.BS_POLICY_FIXED, 16, 16, bs.BS_PREC_FP32_COMP)
    assert (p.near_cut, p.d_g11, p.d_g4) == (2.0, 4.0, 8.0)
    for code in (0, -1, -2, -3, -4, -5, -6, -7, -8):
        assert bs.status_string(code)
    assert bs.status_string(-99) == "unknown status"


def _upload_status(xyz, om, tets, flags=0):
    L = bs.load_library()
    d = bs.MeshDesc(xyz.shape[0], xyz.ctypes.data, om.ctypes.data, tets.shape[0], tets.ctypes.data, flags, None)
    h = ctypes.c_void_p()
    rc = L.bs_mesh_upload(ctypes.byref(d), ctypes.byref(h))
    if rc == 0:
        L.bs_mesh_free(h)
    return rc, L.bs_last_error().decode()


def test_upload_rejects_bad_inputs():
    m = W.make_config("C1", scale=(2, 2, 2))
    xyz, om, tets = m.xyz.copy(), m.omega.copy(), m.tets.copy()
    L = bs.load_library()
    assert L.bs_mesh_upload(None, None) == bs.BS_E_ARG
    bad = tets.copy()
    bad[3, 1] = m.n_nodes
    rc, msg = _upload_status(xyz, om, bad)
    assert rc == bs.BS_E_INDEX and "tetrahedron 3" in msg
    bad = tets.copy()
    bad[5, 2] = bad[5, 0]
    rc, msg = _upload_status(xyz, om, bad)
    assert rc == bs.BS_E_INDEX and "repeats" in msg
    x2 = xyz.copy()
    x2[7, 1] = np.nan
    assert _upload_status(x2, om, tets)[0] == bs.BS_E_NONFINITE
    o2 = om.copy()
    o2[2, 0] = np.inf
    assert _upload_status(xyz, o2, tets)[0] == bs.BS_E_NONFINITE
    x3 = xyz.copy()
    t = tets[4]
    x3[t[3]] = x3[t[0]] + 0.5 * (x3[t[1]] - x3[t[0]]) + 0.5 * (x3[t[2]] - x3[t[0]])  # flatten tet 4
    rc, msg = _upload_status(x3, om, tets)
    assert rc == bs.BS_E_DEGENERATE and "tetrahedron" in msg
    assert _upload_status(xyz, om, tets, flags=8)[0] == bs.BS_E_ARG


def test_calls_on_null_mesh():
    L = bs.load_library()
    p = bs.bs_policy_default()
    assert L.bs_set_policy(None, ctypes.byref(p)) == bs.BS_E_STATE
    assert L.bs_eval_velocity(None, None, 0, None, None) == bs.BS_E_STATE
    assert L.bs_mesh_update(None, None, None, 0, None) == bs.BS_E_STATE
    assert L.bs_advect_heun(None, 0.1, 1, None, 0, None, None, None) == bs.BS_E_STATE
    assert L.bs_eval_points(None, 1, None, None, 0, None, None) == bs.BS_E_STATE
    assert L.bs_velocity_gradient(None, None, None, 0, None) == bs.BS_E_STATE
    assert L.bs_mesh_read(None, None, None, 0, None) == bs.BS_E_STATE
    assert L.bs_stretching_rate(None, None, None, 0, None) == bs.BS_E_STATE
    assert L.bs_eval_velocity_noalloc(None, None, 0, None) == bs.BS_E_STATE
    L.bs_mesh_free(None)


def _no_gpu():
    try:
        import torch

        return not torch.cuda.is_available()
    except Exception:
        return True


@pytest.mark.skipif(not _no_gpu(), reason="checks the no-device error path")
def test_valid_mesh_without_device_reports_device_error():
    m = W.make_config("C1", scale=(2, 2, 2))
    rc, msg = _upload_status(m.xyz, m.omega, m.tets)
    assert rc == bs.BS_E_DEVICE, msg


def test_upload_rejects_meshes_beyond_32_bit_node_indexing():
    """The kernels index the node arrays as c * npad + i in 32 bits, so the
    library refuses more than 2^29 node slots and 2^29 tets before reading
    any array (the pointers here cover one node only)."""
    L = bs.load_library()
    xyz = np.zeros((1, 3))
    tets = np.zeros((1, 4), dtype=np.int32)
    for n_nodes, n_tets in (((1 << 29) + 1, 1), (1 << 30, 1), (4, (1 << 29) + 1)):
        d = bs.MeshDesc(n_nodes, xyz.ctypes.data, xyz.ctypes.data, n_tets, tets.ctypes.data, 0, None)
        h = ctypes.c_void_p()
        assert L.bs_mesh_upload(ctypes.byref(d), ctypes.byref(h)) == bs.BS_E_ARG
        assert "32-bit" in L.bs_last_error().decode()
        assert not h.value
