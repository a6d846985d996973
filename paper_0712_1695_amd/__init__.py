"""Python binding of libbs.so, the MI355X Biot-Savart node-velocity library.

Argument marshalling only: every step of an evaluation runs in the HIP
library.  The function names are those of the C ABI (include/bs.h):

    m = bs_mesh_upload(xyz, omega, tets)          # numpy (host) or torch (device)
    bs_set_policy(m, kind=BS_POLICY_FIXED, n_phi=16, n_theta=16, ...)
    v = bs_eval_velocity(m)                      # numpy [n,3] float64
    bs_eval_velocity(m, out=torch_tensor)        # into device memory
    bs_mesh_update(m, xyz=..., omega=...)        # same connectivity
    bs_mesh_free(m)

torch is used only for device memory and the current HIP stream.  There is
no fallback: if libbs.so is missing or no gfx950 device is present the calls
raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbs.so")

BS_OK = 0
BS_E_ARG = -1
BS_E_INDEX = -2
BS_E_DEGENERATE = -3
BS_E_NONFINITE = -4
BS_E_STATE = -5
BS_E_DEVICE = -6
BS_E_NOMEM = -7
BS_E_POLICY = -8

BS_PTR_HOST = 0
BS_PTR_DEVICE = 1
BS_EVAL_VALU_FAR = 0x10
BS_EVAL_SERIAL = 0x20
BS_ADVECT_STRETCH = 0x40

BS_RULE_G1, BS_RULE_G4, BS_RULE_G11, BS_RULE_RT = 0, 1, 2, 3
BS_POLICY_FIXED, BS_POLICY_PURE_RT, BS_POLICY_GAUSS_ONLY, BS_POLICY_LEARNED = 0, 1, 2, 3
BS_PREC_FP32_NAIVE, BS_PREC_FP32_COMP, BS_PREC_FP64 = 0, 1, 2
BS_FAR_ALL_PAIRS, BS_FAR_TREECODE = 0, 1


class MeshDesc(ctypes.Structure):
    _fields_ = [
        ("n_nodes", ctypes.c_int64),
        ("xyz", ctypes.c_void_p),
        ("omega", ctypes.c_void_p),
        ("n_tets", ctypes.c_int64),
        ("tets", ctypes.c_void_p),
        ("flags", ctypes.c_uint32),
        ("stream", ctypes.c_void_p),
    ]


class Policy(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("n_phi", ctypes.c_int),
        ("n_theta", ctypes.c_int),
        ("near_cut", ctypes.c_double),
        ("d_g11", ctypes.c_double),
        ("d_g4", ctypes.c_double),
        ("gauss_rule", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("mlp_bf16", ctypes.c_void_p),
        ("mlp_len", ctypes.c_int64),
        ("conf_min", ctypes.c_float),
        ("far_field", ctypes.c_int),
        ("tree_theta", ctypes.c_double),
        ("tree_order", ctypes.c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("t_eval_s", ctypes.c_double),
        ("t_kernel_s", ctypes.c_double * 4),
        ("pairs", ctypes.c_int64),
        ("pairs_by_rule", ctypes.c_int64 * 4),
        ("rt_hit_lines", ctypes.c_int64),
        ("fp64_retests", ctypes.c_int64),
        ("reoriented", ctypes.c_int64),
        ("nonfinite_out", ctypes.c_int32),
        ("hbar", ctypes.c_double),
        ("tree_expansions", ctypes.c_int64),
        ("tree_direct", ctypes.c_int64),
        ("tree_covered", ctypes.c_int64),
        ("rt_walk_nodes", ctypes.c_int64),
        ("rt_candidate_nodes", ctypes.c_int64),
    ]

    def as_dict(self):
        return dict(t_eval_s=self.t_eval_s, t_kernel_s=list(self.t_kernel_s), pairs=self.pairs,
                    pairs_by_rule=list(self.pairs_by_rule), rt_hit_lines=self.rt_hit_lines,
                    fp64_retests=self.fp64_retests, reoriented=self.reoriented,
                    nonfinite_out=self.nonfinite_out, hbar=self.hbar, tree_expansions=self.tree_expansions,
                    tree_direct=self.tree_direct, tree_covered=self.tree_covered,
                    rt_walk_nodes=self.rt_walk_nodes, rt_candidate_nodes=self.rt_candidate_nodes)


# every symbol include/bs.h declares
EXPORTS = ["bs_mesh_upload", "bs_mesh_update", "bs_mesh_free", "bs_policy_default", "bs_set_policy",
           "bs_eval_velocity", "bs_eval_velocity_noalloc", "bs_eval_points", "bs_advect_heun", "bs_velocity_gradient",
           "bs_stretching_rate", "bs_mesh_read",
           "bs_learn_sample_pairs", "bs_learn_pairs", "bs_mlp_train",
           "bs_mlp_grad", "bs_mlp_logits", "bs_status_string", "bs_last_error"]

BS_MLP_BLOB_LEN = 5540


class TrainCfg(ctypes.Structure):
    _fields_ = [
        ("epochs", ctypes.c_int),
        ("batch", ctypes.c_int),
        ("lr", ctypes.c_float),
        ("beta1", ctypes.c_float),
        ("beta2", ctypes.c_float),
        ("eps", ctypes.c_float),
        ("class_w", ctypes.c_float * 4),
        ("seed", ctypes.c_uint64),
    ]


class BsError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {detail or 'error'} (status {status})")
        self.status = status


_lib = None


def load_library(path: Optional[str] = None) -> ctypes.CDLL:
    """Load libbs.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} not found: build it with `python -m paper_0712_1695_amd.build`")
    # torch first: its HIP runtime is then the one the library binds to, so
    # torch's streams and device memory are valid arguments of every call
    import torch  # noqa: F401

    L = ctypes.CDLL(p)
    vp = ctypes.c_void_p
    L.bs_mesh_upload.argtypes = [ctypes.POINTER(MeshDesc), ctypes.POINTER(vp)]
    L.bs_mesh_upload.restype = ctypes.c_int
    L.bs_mesh_update.argtypes = [vp, vp, vp, ctypes.c_uint32, vp]
    L.bs_mesh_update.restype = ctypes.c_int
    L.bs_mesh_free.argtypes = [vp]
    L.bs_mesh_free.restype = None
    L.bs_policy_default.argtypes = [ctypes.POINTER(Policy)]
    L.bs_policy_default.restype = None
    L.bs_set_policy.argtypes = [vp, ctypes.POINTER(Policy)]
    L.bs_set_policy.restype = ctypes.c_int
    L.bs_eval_velocity.argtypes = [vp, vp, ctypes.c_uint32, vp, ctypes.POINTER(Stats)]
    L.bs_eval_velocity.restype = ctypes.c_int
    L.bs_eval_velocity_noalloc.argtypes = [vp, vp, ctypes.c_uint32, vp]
    L.bs_eval_velocity_noalloc.restype = ctypes.c_int
    L.bs_eval_points.argtypes = [vp, ctypes.c_int64, vp, vp, ctypes.c_uint32, vp, ctypes.POINTER(Stats)]
    L.bs_eval_points.restype = ctypes.c_int
    L.bs_advect_heun.argtypes = [vp, ctypes.c_double, ctypes.c_int, vp, ctypes.c_uint32, vp, vp,
                                 ctypes.POINTER(Stats)]
    L.bs_advect_heun.restype = ctypes.c_int
    L.bs_velocity_gradient.argtypes = [vp, vp, vp, ctypes.c_uint32, vp]
    L.bs_velocity_gradient.restype = ctypes.c_int
    L.bs_stretching_rate.argtypes = [vp, vp, vp, ctypes.c_uint32, vp]
    L.bs_stretching_rate.restype = ctypes.c_int
    L.bs_mesh_read.argtypes = [vp, vp, vp, ctypes.c_uint32, vp]
    L.bs_mesh_read.restype = ctypes.c_int
    L.bs_learn_sample_pairs.argtypes = [vp, ctypes.c_int64, ctypes.c_uint64, vp, ctypes.POINTER(ctypes.c_int64)]
    L.bs_learn_sample_pairs.restype = ctypes.c_int
    L.bs_learn_pairs.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_double, vp, vp, vp, vp]
    L.bs_learn_pairs.restype = ctypes.c_int
    L.bs_mlp_train.argtypes = [vp, vp, ctypes.c_int64, ctypes.POINTER(TrainCfg), vp, vp, vp]
    L.bs_mlp_train.restype = ctypes.c_int
    L.bs_mlp_grad.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp, vp, vp]
    L.bs_mlp_grad.restype = ctypes.c_int
    L.bs_mlp_logits.argtypes = [vp, vp, ctypes.c_int64, vp, vp]
    L.bs_mlp_logits.restype = ctypes.c_int
    L.bs_status_string.argtypes = [ctypes.c_int]
    L.bs_status_string.restype = ctypes.c_char_p
    L.bs_last_error.argtypes = []
    L.bs_last_error.restype = ctypes.c_char_p
    if path is None:
        _lib = L
    return L


def _check(rc: int, where: str):
    if rc != BS_OK:
        L = load_library()
        raise BsError(rc, where, L.bs_last_error().decode())


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _stream_handle(stream):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    try:
        import torch

        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return ctypes.c_void_p(0)


def _ptr(a, dtype):
    """(pointer, is_device, keepalive) for a numpy array or torch tensor."""
    if a is None:
        return None, False, None
    if _is_torch(a):
        import torch

        want = {np.float64: torch.float64, np.int32: torch.int32}[dtype]
        t = a.contiguous()
        if t.dtype != want:
            t = t.to(want)
        return ctypes.c_void_p(t.data_ptr()), t.is_cuda, t
    arr = np.ascontiguousarray(a, dtype=dtype)
    return ctypes.c_void_p(arr.ctypes.data), False, arr


class BsMesh:
    """Owning handle of a bs_mesh (freed by bs_mesh_free or on collection)."""

    def __init__(self, handle: ctypes.c_void_p, n_nodes: int, n_tets: int):
        self.handle = handle
        self.n_nodes = n_nodes
        self.n_tets = n_tets

    def __del__(self):
        try:
            bs_mesh_free(self)
        except Exception:
            pass


def bs_mesh_upload(xyz, omega, tets, stream=None) -> BsMesh:
    """Copy a mesh (xyz, omega: [n,3] float64; tets: [T,4] int32; numpy on
    the host or torch tensors on the device) into the library."""
    L = load_library()
    px, dx, kx = _ptr(xyz, np.float64)
    pw, dw, kw = _ptr(omega, np.float64)
    pt, dt, kt = _ptr(tets, np.int32)
    if len({dx, dw, dt}) != 1:
        raise ValueError("xyz, omega and tets must all be host arrays or all device tensors")
    n = int(kx.shape[0])
    T = int(kt.shape[0])
    d = MeshDesc(n, px, pw, T, pt, BS_PTR_DEVICE if dx else BS_PTR_HOST, _stream_handle(stream))
    h = ctypes.c_void_p()
    _check(L.bs_mesh_upload(ctypes.byref(d), ctypes.byref(h)), "bs_mesh_upload")
    return BsMesh(h, n, T)


def bs_mesh_update(mesh: BsMesh, xyz=None, omega=None, stream=None):
    L = load_library()
    px, dx, kx = _ptr(xyz, np.float64)
    pw, dw, kw = _ptr(omega, np.float64)
    dev = dx if xyz is not None else dw
    if xyz is not None and omega is not None and dx != dw:
        raise ValueError("xyz and omega must both be host arrays or both device tensors")
    _check(L.bs_mesh_update(mesh.handle, px, pw, BS_PTR_DEVICE if dev else BS_PTR_HOST, _stream_handle(stream)),
           "bs_mesh_update")


def bs_mesh_free(mesh: BsMesh):
    if mesh is not None and mesh.handle:
        load_library().bs_mesh_free(mesh.handle)
        mesh.handle = ctypes.c_void_p()


def bs_policy_default() -> Policy:
    p = Policy()
    load_library().bs_policy_default(ctypes.byref(p))
    return p


def bs_set_policy(mesh: BsMesh, policy: Optional[Policy] = None, **kw):
    """Install a policy: a Policy struct, or the defaults updated with kw
    (kind, n_phi, n_theta, near_cut, d_g11, d_g4, gauss_rule, precision,
    mlp_bf16 (uint16 numpy array), conf_min, far_field ("all_pairs",
    "treecode" or BS_FAR_*), tree_theta, tree_order)."""
    L = load_library()
    p = policy if policy is not None else bs_policy_default()
    keep = None
    for k, v in kw.items():
        if k == "mlp_bf16":
            keep = np.ascontiguousarray(v, dtype=np.uint16)
            p.mlp_bf16 = keep.ctypes.data
            p.mlp_len = keep.size
        elif k == "far_field" and isinstance(v, str):
            p.far_field = {"all_pairs": BS_FAR_ALL_PAIRS, "treecode": BS_FAR_TREECODE}[v]
        else:
            setattr(p, k, v)
    _check(L.bs_set_policy(mesh.handle if mesh is not None else None, ctypes.byref(p)), "bs_set_policy")
    return p


def bs_eval_velocity(mesh: BsMesh, out=None, stream=None, stats: bool = False, valu_far: bool = False,
                     serial: bool = False):
    """Velocity at every node ([n,3] float64, input node order).  out: a
    device torch tensor to fill (returned), else a new numpy array.
    valu_far: far field on the vector ALUs instead of the matrix cores;
    serial: every kernel on one stream (per-kernel times of each alone)."""
    L = load_library()
    st = Stats() if stats else None
    extra = (BS_EVAL_VALU_FAR if valu_far else 0) | (BS_EVAL_SERIAL if serial else 0)
    if out is None:
        vel = np.empty((mesh.n_nodes, 3), dtype=np.float64)
        rc = L.bs_eval_velocity(mesh.handle, ctypes.c_void_p(vel.ctypes.data), BS_PTR_HOST | extra,
                                _stream_handle(stream),
                                ctypes.byref(st) if st is not None else None)
    else:
        if not (_is_torch(out) and out.is_cuda and out.dtype.__str__() == "torch.float64" and out.is_contiguous()):
            raise ValueError("out must be a contiguous float64 device tensor")
        if tuple(out.shape) != (mesh.n_nodes, 3):
            raise ValueError("out must have shape [n_nodes, 3]")
        vel = out
        rc = L.bs_eval_velocity(mesh.handle, ctypes.c_void_p(out.data_ptr()), BS_PTR_DEVICE | extra,
                                _stream_handle(stream), ctypes.byref(st) if st is not None else None)
    _check(rc, "bs_eval_velocity")
    return (vel, st.as_dict()) if stats else vel


def bs_eval_velocity_noalloc(mesh: BsMesh, out, stream=None, valu_far: bool = False):
    """bs_eval_velocity into the device tensor `out` ([n,3] float64,
    contiguous) without any allocation (the library's static scratch)."""
    L = load_library()
    if not (_is_torch(out) and out.is_cuda and str(out.dtype) == "torch.float64" and out.is_contiguous()):
        raise ValueError("out must be a contiguous float64 device tensor")
    if tuple(out.shape) != (mesh.n_nodes, 3):
        raise ValueError("out must have shape [n_nodes, 3]")
    flags = BS_PTR_DEVICE | (BS_EVAL_VALU_FAR if valu_far else 0)
    _check(L.bs_eval_velocity_noalloc(mesh.handle, ctypes.c_void_p(out.data_ptr()), flags, _stream_handle(stream)),
           "bs_eval_velocity_noalloc")
    return out


def bs_eval_points(mesh: BsMesh, pts, out=None, stream=None, stats: bool = False, valu_far: bool = False,
                   serial: bool = False):
    """Velocity at arbitrary points pts ([k,3] float64: numpy, or a device
    tensor, then out must be a device tensor too).  Returns [k,3] (numpy, or
    `out`)[, stats dict]."""
    L = load_library()
    st = Stats() if stats else None
    extra = (BS_EVAL_VALU_FAR if valu_far else 0) | (BS_EVAL_SERIAL if serial else 0)
    if _is_torch(pts) and pts.is_cuda:
        if out is None or not (_is_torch(out) and out.is_cuda and out.is_contiguous()):
            raise ValueError("device points need a contiguous device output tensor")
        if tuple(out.shape) != tuple(pts.shape):
            raise ValueError("out must have the shape of pts")
        p = pts.contiguous()
        rc = L.bs_eval_points(mesh.handle, int(p.shape[0]), ctypes.c_void_p(p.data_ptr()),
                              ctypes.c_void_p(out.data_ptr()), BS_PTR_DEVICE | extra, _stream_handle(stream),
                              ctypes.byref(st) if st is not None else None)
        vel = out
    else:
        p = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 3)
        vel = np.empty_like(p)
        rc = L.bs_eval_points(mesh.handle, int(p.shape[0]), ctypes.c_void_p(p.ctypes.data),
                              ctypes.c_void_p(vel.ctypes.data), BS_PTR_HOST | extra, _stream_handle(stream),
                              ctypes.byref(st) if st is not None else None)
    _check(rc, "bs_eval_points")
    return (vel, st.as_dict()) if stats else vel


def bs_advect_heun(mesh: BsMesh, dt: float, steps: int, out=None, stream=None, stats: bool = False,
                   stretch: bool = False):
    """Advance the mesh nodes `steps` Heun steps of size dt (positions kept in
    the mesh; with stretch the nodal vorticity too, by (w . grad) v).
    Returns (positions [n,3] numpy or the device tensor `out`, per-step
    seconds [steps] numpy[, stats dict])."""
    L = load_library()
    st = Stats() if stats else None
    secs = np.zeros(max(int(steps), 1), dtype=np.float64)
    if out is None:
        pos = np.empty((mesh.n_nodes, 3), dtype=np.float64)
        ptr, flags = ctypes.c_void_p(pos.ctypes.data), BS_PTR_HOST
    else:
        if not (_is_torch(out) and out.is_cuda and str(out.dtype) == "torch.float64" and out.is_contiguous()):
            raise ValueError("out must be a contiguous float64 device tensor")
        pos, ptr, flags = out, ctypes.c_void_p(out.data_ptr()), BS_PTR_DEVICE
    flags |= BS_ADVECT_STRETCH if stretch else 0
    _check(L.bs_advect_heun(mesh.handle, float(dt), int(steps), ptr, flags, _stream_handle(stream),
                            ctypes.c_void_p(secs.ctypes.data), ctypes.byref(st) if st is not None else None),
           "bs_advect_heun")
    secs = secs[: int(steps)]
    return (pos, secs, st.as_dict()) if stats else (pos, secs)


def bs_velocity_gradient(mesh: BsMesh, vel=None, out=None, stream=None):
    """Nodal velocity gradient [n,3,3] (g[i,a,b] = dv_a/dx_b) of the
    piecewise-linear interpolant of vel ([n,3] float64 numpy array or device
    tensor; None: the last bs_eval_velocity).  Returns numpy, or the device
    tensor `out` (contiguous float64 [n,3,3])."""
    L = load_library()
    pv, dv, kv = _ptr(vel, np.float64)
    if vel is not None and tuple(vel.shape) != (mesh.n_nodes, 3):
        raise ValueError("vel must be [n_nodes, 3]")
    if out is None:
        g = np.empty((mesh.n_nodes, 3, 3), dtype=np.float64)
        pg, dev = ctypes.c_void_p(g.ctypes.data), False
    else:
        if not (_is_torch(out) and out.is_cuda and str(out.dtype) == "torch.float64" and out.is_contiguous()
                and tuple(out.shape) == (mesh.n_nodes, 3, 3)):
            raise ValueError("out must be a contiguous float64 device tensor [n_nodes, 3, 3]")
        g, pg, dev = out, ctypes.c_void_p(out.data_ptr()), True
    if vel is not None and dv != dev:
        raise ValueError("vel and out must both be host arrays or both device tensors")
    _check(L.bs_velocity_gradient(mesh.handle, pv, pg, BS_PTR_DEVICE if dev else BS_PTR_HOST,
                                  _stream_handle(stream)), "bs_velocity_gradient")
    return g


def bs_stretching_rate(mesh: BsMesh, vel=None, out=None, stream=None):
    """Vortex stretching rate (omega . grad) v [n,3] with the mesh's nodal
    vorticity and the gradient of vel ([n,3] float64 numpy array or device
    tensor; None: the last bs_eval_velocity).  Returns numpy, or the device
    tensor `out` (contiguous float64 [n,3])."""
    L = load_library()
    pv, dv, kv = _ptr(vel, np.float64)
    if vel is not None and tuple(vel.shape) != (mesh.n_nodes, 3):
        raise ValueError("vel must be [n_nodes, 3]")
    if out is None:
        r = np.empty((mesh.n_nodes, 3), dtype=np.float64)
        pr, dev = ctypes.c_void_p(r.ctypes.data), False
    else:
        if not (_is_torch(out) and out.is_cuda and str(out.dtype) == "torch.float64" and out.is_contiguous()
                and tuple(out.shape) == (mesh.n_nodes, 3)):
            raise ValueError("out must be a contiguous float64 device tensor [n_nodes, 3]")
        r, pr, dev = out, ctypes.c_void_p(out.data_ptr()), True
    if vel is not None and dv != dev:
        raise ValueError("vel and out must both be host arrays or both device tensors")
    _check(L.bs_stretching_rate(mesh.handle, pv, pr, BS_PTR_DEVICE if dev else BS_PTR_HOST, _stream_handle(stream)),
           "bs_stretching_rate")
    return r


def bs_mesh_read(mesh: BsMesh):
    """The mesh's current FP64 positions and nodal vorticity (numpy [n,3] each)."""
    L = load_library()
    x = np.empty((mesh.n_nodes, 3), dtype=np.float64)
    w = np.empty((mesh.n_nodes, 3), dtype=np.float64)
    _check(L.bs_mesh_read(mesh.handle, ctypes.c_void_p(x.ctypes.data), ctypes.c_void_p(w.ctypes.data), BS_PTR_HOST,
                          None), "bs_mesh_read")
    return x, w


def _dev(t, dtype_name):
    if not (_is_torch(t) and t.is_cuda and str(t.dtype) == dtype_name and t.is_contiguous()):
        raise ValueError(f"expected a contiguous {dtype_name} device tensor")
    return ctypes.c_void_p(t.data_ptr())


def bs_learn_sample_pairs(mesh: BsMesh, max_pairs: int, seed: int = 0) -> np.ndarray:
    """Pairs (input node, input tet) of the ray-traced band, non-incident."""
    L = load_library()
    out = np.zeros((max(int(max_pairs), 1), 2), dtype=np.int32)
    n = ctypes.c_int64()
    _check(L.bs_learn_sample_pairs(mesh.handle, int(max_pairs), int(seed), ctypes.c_void_p(out.ctypes.data),
                                   ctypes.byref(n)), "bs_learn_sample_pairs")
    return out[: n.value]


def bs_learn_pairs(mesh: BsMesh, pairs, tau: float, stream=None):
    """Features, labels and Gauss-rule errors of the given pairs (device
    tensors: float32 [n,16], int8 [n], float32 [n,3])."""
    import torch

    L = load_library()
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
    n = pr.shape[0]
    dev = torch.device("cuda", torch.cuda.current_device())
    feats = torch.empty((n, 16), dtype=torch.float32, device=dev)
    labels = torch.empty((n,), dtype=torch.int8, device=dev)
    errs = torch.empty((n, 3), dtype=torch.float32, device=dev)
    _check(L.bs_learn_pairs(mesh.handle, ctypes.c_void_p(pr.ctypes.data), n, float(tau),
                            ctypes.c_void_p(feats.data_ptr()), ctypes.c_void_p(labels.data_ptr()),
                            ctypes.c_void_p(errs.data_ptr()), _stream_handle(stream)), "bs_learn_pairs")
    return feats, labels, errs


def bs_mlp_train(feats, labels, epochs=4, batch=4096, lr=2e-3, beta1=0.9, beta2=0.999, eps=1e-8,
                 class_w=(1.0, 1.0, 1.0, 1.0), seed=0, stream=None):
    """Train on device tensors; returns (blob uint16 [5540], epoch losses)."""
    L = load_library()
    cfg = TrainCfg(int(epochs), int(batch), lr, beta1, beta2, eps, (ctypes.c_float * 4)(*class_w), int(seed))
    blob = np.zeros(BS_MLP_BLOB_LEN, dtype=np.uint16)
    losses = np.zeros(max(int(epochs), 1), dtype=np.float32)
    _check(L.bs_mlp_train(_dev(feats, "torch.float32"), _dev(labels, "torch.int8"), int(feats.shape[0]),
                          ctypes.byref(cfg), ctypes.c_void_p(blob.ctypes.data), ctypes.c_void_p(losses.ctypes.data),
                          _stream_handle(stream)), "bs_mlp_train")
    return blob, losses[: int(epochs)]


def bs_mlp_grad(blob, feats, labels, class_w=(1.0, 1.0, 1.0, 1.0), stream=None):
    """(loss, gradients [5508] float32) of one forward/backward pass."""
    L = load_library()
    b = np.ascontiguousarray(blob, dtype=np.uint16)
    cw = np.ascontiguousarray(class_w, dtype=np.float32)
    grads = np.zeros(BS_MLP_BLOB_LEN - 32, dtype=np.float32)
    loss = ctypes.c_float()
    _check(L.bs_mlp_grad(ctypes.c_void_p(b.ctypes.data), _dev(feats, "torch.float32"), _dev(labels, "torch.int8"),
                         int(feats.shape[0]), ctypes.c_void_p(cw.ctypes.data), ctypes.byref(loss),
                         ctypes.c_void_p(grads.ctypes.data), _stream_handle(stream)), "bs_mlp_grad")
    return float(loss.value), grads


def bs_mlp_logits(blob, feats, stream=None):
    import torch

    L = load_library()
    b = np.ascontiguousarray(blob, dtype=np.uint16)
    out = torch.empty((feats.shape[0], 4), dtype=torch.float32, device=feats.device)
    _check(L.bs_mlp_logits(ctypes.c_void_p(b.ctypes.data), _dev(feats, "torch.float32"), int(feats.shape[0]),
                           ctypes.c_void_p(out.data_ptr()), _stream_handle(stream)), "bs_mlp_logits")
    return out


def status_string(status: int) -> str:
    return load_library().bs_status_string(int(status)).decode()
