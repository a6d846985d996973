"""FP64 CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package.  It is independent of the GPU
library: nothing here imports ``paper_0712_1695_amd`` and nothing there
imports this.

``bs_oracle.c`` holds the method (plain C, FP64, OpenMP over target nodes);
``references.py`` holds exact references used to pin it (closed forms,
brute-force integration of single tetrahedra, analytic line sums).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "bs_oracle.c")
_LIB = os.path.join(_HERE, "libbs_oracle.so")

RULE_G1, RULE_G4, RULE_G11, RULE_RT = 0, 1, 2, 3
POLICY_FIXED, POLICY_PURE_RT, POLICY_GAUSS_ONLY, POLICY_EXPLICIT = 0, 1, 2, 3


class Policy(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int),
        ("n_phi", ctypes.c_int),
        ("n_theta", ctypes.c_int),
        ("near_cut", ctypes.c_double),
        ("d_g11", ctypes.c_double),
        ("d_g4", ctypes.c_double),
        ("gauss_rule", ctypes.c_int),
        ("precheck", ctypes.c_int),
        ("neumaier", ctypes.c_int),
        ("pair_rules", ctypes.c_void_p),
    ]


class Counters(ctypes.Structure):
    _fields_ = [
        ("pairs_by_rule", ctypes.c_int64 * 4),
        ("rt_lines", ctypes.c_int64),
        ("rt_hit_lines", ctypes.c_int64),
        ("rt_face_hits", ctypes.c_int64),
        ("algo_flops", ctypes.c_double),
        ("hbar", ctypes.c_double),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, no fast-math, no FMA
    contraction, portable x86-64 code)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
               "-fno-fast-math", "-march=x86-64-v2", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.bso_gauss_legendre.argtypes = [ctypes.c_int, dp, dp]
        L.bso_tet_rule.argtypes = [ctypes.c_int, dp, dp]
        L.bso_angular_tables.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp]
        L.bso_mean_edge.restype = ctypes.c_double
        L.bso_mean_edge.argtypes = [ctypes.c_int64, dp, ctypes.c_int64, ctypes.c_void_p]
        L.bso_eval.argtypes = [ctypes.c_int64, dp, dp, ctypes.c_int64, ctypes.c_void_p, ctypes.POINTER(Policy),
                               ctypes.c_int64, ctypes.c_void_p, dp, ctypes.c_void_p, ctypes.POINTER(Counters)]
        L.bso_pair.argtypes = [dp, ctypes.c_int64, dp, dp, dp, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                               ctypes.c_int, ctypes.c_int, dp]
        L.bso_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def gauss_legendre(n: int):
    t = np.zeros(n)
    w = np.zeros(n)
    if lib().bso_gauss_legendre(n, _dp(t), _dp(w)) != 0:
        raise ValueError(n)
    return t, w


def tet_rule(k: int):
    lam = np.zeros((k, 4))
    w = np.zeros(k)
    if lib().bso_tet_rule(k, _dp(lam), _dp(w)) != 0:
        raise ValueError(k)
    return lam, w


def angular_tables(N: int, M: int):
    s = np.zeros((N * M, 3))
    k = np.zeros(N * M)
    if lib().bso_angular_tables(N, M, _dp(s), _dp(k)) != 0:
        raise ValueError((N, M))
    return s, k


def mean_edge(xyz, tets) -> float:
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    return float(lib().bso_mean_edge(xyz.shape[0], _dp(xyz), tets.shape[0], tets.ctypes.data))


def make_policy(kind="fixed", n_phi=16, n_theta=16, near_cut=2.0, d_g11=4.0, d_g4=8.0, gauss_rule=RULE_G1,
                precheck=True, neumaier=False):
    kinds = {"fixed": POLICY_FIXED, "pure_rt": POLICY_PURE_RT, "gauss_only": POLICY_GAUSS_ONLY,
             "explicit": POLICY_EXPLICIT}
    return dict(kind=kinds[kind] if isinstance(kind, str) else int(kind), n_phi=n_phi, n_theta=n_theta,
                near_cut=near_cut, d_g11=d_g11, d_g4=d_g4, gauss_rule=gauss_rule, precheck=int(precheck),
                neumaier=int(neumaier))


def evaluate(xyz, omega, tets, policy: Optional[dict] = None, targets=None, return_rules=False,
             pair_rules=None, return_counters=False):
    """Velocity at the target nodes (all nodes by default), FP64.

    policy: dict from make_policy(); pair_rules: int8 [n_targets, n_tets]
    for the explicit policy.  Returns vel [n_targets, 3] (and the rule
    array / counters on request)."""
    pol = dict(make_policy() if policy is None else policy)
    xyz = np.ascontiguousarray(xyz, dtype=np.float64)
    omega = np.ascontiguousarray(omega, dtype=np.float64)
    tets = np.ascontiguousarray(tets, dtype=np.int32)
    n = xyz.shape[0]
    if targets is None:
        tg = None
        nt = n
    else:
        tg = np.ascontiguousarray(targets, dtype=np.int64)
        nt = tg.size
    pr = None
    if pair_rules is not None:
        pr = np.ascontiguousarray(pair_rules, dtype=np.int8)
        assert pr.shape == (nt, tets.shape[0])
        pol["kind"] = POLICY_EXPLICIT
    P = Policy(pol["kind"], pol["n_phi"], pol["n_theta"], pol["near_cut"], pol["d_g11"], pol["d_g4"],
               pol["gauss_rule"], pol["precheck"], pol["neumaier"], pr.ctypes.data if pr is not None else None)
    vel = np.zeros((nt, 3))
    rules = np.zeros((nt, tets.shape[0]), dtype=np.int8) if return_rules else None
    C = Counters()
    rc = lib().bso_eval(n, _dp(xyz), _dp(omega), tets.shape[0], tets.ctypes.data, ctypes.byref(P), nt,
                        tg.ctypes.data if tg is not None else None, _dp(vel),
                        rules.ctypes.data if rules is not None else None, ctypes.byref(C))
    if rc != 0:
        raise RuntimeError("oracle evaluation failed")
    out = [vel]
    if return_rules:
        out.append(rules)
    if return_counters:
        out.append(dict(pairs_by_rule=list(C.pairs_by_rule), rt_lines=C.rt_lines, rt_hit_lines=C.rt_hit_lines,
                        rt_face_hits=C.rt_face_hits, algo_flops=C.algo_flops, hbar=C.hbar))
    return out[0] if len(out) == 1 else tuple(out)


def pair(x, tet_xyz, tet_omega, rule, N=16, M=16, precheck=True, self_index=-1, ids=None, omega_x=None):
    """Contribution of one tetrahedron (4x3 vertices, 4x3 vorticity) to the
    velocity at point x by one rule.  When x is vertex j of the tetrahedron
    pass ids (4 ints) with self_index == ids[j] and omega_x."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    tv = np.ascontiguousarray(tet_xyz, dtype=np.float64)
    tw = np.ascontiguousarray(tet_omega, dtype=np.float64)
    ox = np.ascontiguousarray(np.zeros(3) if omega_x is None else omega_x, dtype=np.float64)
    idv = None if ids is None else np.ascontiguousarray(ids, dtype=np.int32)
    out = np.zeros(3)
    rc = lib().bso_pair(_dp(x), int(self_index), _dp(ox), _dp(tv), _dp(tw),
                        idv.ctypes.data if idv is not None else None, int(rule), int(N), int(M), int(precheck),
                        _dp(out))
    if rc != 0:
        raise RuntimeError("oracle pair failed")
    return out


def num_threads() -> int:
    return int(lib().bso_num_threads())
