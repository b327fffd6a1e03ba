"""CPU oracle for the sparse IDP DG stage -- TEST INFRASTRUCTURE ONLY.

A plain, slow FP64 implementation (``idp_ref.c``) of one limited SSP-RK
stage of the method of Pazner, arXiv 2004.08503, written from the paper and
independent of the GPU library: the two share no source, header, table or
helper.  Only the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product
path never does.

Problem descriptions are duck-typed: any object with the attributes
``dim, nx, ny, lx, ly, p, eq, vel, gamma, limiter`` (``eq`` and ``limiter``
as the integer codes below; ``gmin, gmax`` too for SUBCELL_SI) is accepted,
e.g. the seeded workload objects.  ADVECTION_FIELD takes the nodal
velocity from ``beta`` (shape (2, Nn)) when the object has one, else from
the per-row / per-column samples ``vrows``, ``vcols``.  Open directions
(``bc``) take their per-node boundary conditions from ``bnd`` (a
``workloads.Boundary``).
State arrays are float64 of shape ``(nc, Nn)`` in the layout ``u[c][e][b][a]``.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "idp_ref.c")
_LIB_PATH = os.path.join(_HERE, "libidp_ref.so")

ADVECTION, BURGERS, EULER, ADVECTION_FIELD = 0, 1, 2, 3
SUBCELL, TARGET, LOW, SUBCELL_SI, ELEMENTWISE = 0, 1, 2, 3, 4


def build():
    """Compile the oracle with gcc (plain FP64, no FMA contraction)."""
    # written under a temporary name and renamed into place, so that a
    # process loading the library never sees a partly written file
    tmp = "%s.%d.tmp" % (_LIB_PATH, os.getpid())
    cmd = ["gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
    try:
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    finally:
        if os.path.exists(tmp):
            os.remove(tmp)
    global _lib
    _lib = None


class _Desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("p", ctypes.c_int), ("eq", ctypes.c_int),
                ("vel", ctypes.c_double * 2), ("gamma", ctypes.c_double),
                ("limiter", ctypes.c_int),
                ("gmin", ctypes.c_double), ("gmax", ctypes.c_double),
                ("beta", ctypes.POINTER(ctypes.c_double)),
                ("bc", ctypes.c_int * 2),
                ("bc_type", ctypes.c_void_p * 4),
                ("bc_state", ctypes.c_void_p * 4),
                ("metric", ctypes.POINTER(ctypes.c_double))]


class _Trace(ctypes.Structure):
    _fields_ = [(n, ctypes.POINTER(ctypes.c_double)) for n in
                ("uL", "uH", "rH", "rL", "rbar", "umin", "umax", "kmin",
                 "alpha_z", "alpha")]


_lib = None
_DP = ctypes.POINTER(ctypes.c_double)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    D = ctypes.POINTER(_Desc)
    sig = {
        "idp_ref_set_threads": (ctypes.c_int, [ctypes.c_int]),
        "idp_ref_check": (ctypes.c_int, [D]),
        "idp_ref_num_nodes": (ctypes.c_long, [D]),
        "idp_ref_num_comp": (ctypes.c_int, [D]),
        "idp_ref_gl": (ctypes.c_int, [ctypes.c_int, _DP, _DP]),
        "idp_ref_dmat": (ctypes.c_int, [ctypes.c_int, _DP]),
        "idp_ref_dhat": (ctypes.c_int, [ctypes.c_int, _DP]),
        "idp_ref_flux": (ctypes.c_int, [D, _DP, _DP]),
        "idp_ref_lambda": (ctypes.c_double, [D, _DP, _DP, _DP]),
        "idp_ref_fe": (ctypes.c_int, [D, _DP, _DP, ctypes.c_double,
                                      ctypes.POINTER(_Trace)]),
        "idp_ref_stage": (ctypes.c_int, [D, _DP, _DP, _DP, ctypes.c_double,
                                         ctypes.c_int]),
        "idp_ref_step": (ctypes.c_int, [D, _DP, ctypes.c_double]),
        "idp_ref_max_dt": (ctypes.c_int, [D, _DP, _DP]),
        "idp_ref_smoothness": (ctypes.c_int, [D, _DP, _DP]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _desc(prob):
    d = _Desc()
    d.dim, d.nx, d.ny = int(prob.dim), int(prob.nx), int(prob.ny)
    d.lx, d.ly = float(prob.lx), float(prob.ly)
    d.p, d.eq = int(prob.p), int(prob.eq)
    v = list(prob.vel) + [0.0] * (2 - len(prob.vel))
    d.vel[0], d.vel[1] = float(v[0]), float(v[1])
    d.gamma = float(prob.gamma)
    d.limiter = int(prob.limiter)
    d.gmin = float(getattr(prob, "gmin", 0.0))
    d.gmax = float(getattr(prob, "gmax", 0.0))
    keep = []
    if d.eq == ADVECTION_FIELD:
        beta = nodal_velocity(prob)
        d.beta = _ptr(beta)
        keep.append(beta)
    bc = tuple(getattr(prob, "bc", (0, 0)))
    d.bc[0], d.bc[1] = int(bc[0]), int(bc[1])
    bnd = getattr(prob, "bnd", None)
    if bnd is not None:
        for side in range(4):
            if bnd.type[side] is not None:
                t = np.ascontiguousarray(bnd.type[side], dtype=np.int8)
                d.bc_type[side] = t.ctypes.data
                keep.append(t)
            if bnd.state[side] is not None:
                st = np.ascontiguousarray(bnd.state[side], dtype=np.float64)
                d.bc_state[side] = st.ctypes.data
                keep.append(st)
    if getattr(prob, "coords", None) is not None:   # curved mesh: metric terms (oracle.metric)
        from . import metric as _metric
        met = _metric.metric_terms(prob)
        d.metric = _ptr(met)
        keep.append(met)
    d._keep = keep          # the arrays live as long as the descriptor
    return d


def nodal_velocity(prob):
    """The velocity at every node, shape (2, Nn): ``prob.beta`` if given,
    else beta_x from the node's row sample and beta_y from its column
    sample (node i of element e = ey*nx + ex at local (a, b) sits on row
    ey*(p+1) + b and column ex*(p+1) + a)."""
    beta = getattr(prob, "beta", None)
    if beta is not None:
        return np.ascontiguousarray(beta, dtype=np.float64).reshape(2, -1)
    n1 = prob.p + 1
    vr = np.asarray(prob.vrows, dtype=np.float64)
    vc = np.asarray(prob.vcols, dtype=np.float64)
    if vr.size != prob.ny * n1 or vc.size != prob.nx * n1:
        return np.full((2, prob.nx * prob.ny * n1 * n1), np.nan)
    ey, ex, b, a = np.meshgrid(np.arange(prob.ny), np.arange(prob.nx), np.arange(n1),
                               np.arange(n1), indexing="ij")
    return np.ascontiguousarray(np.stack([vr[(ey * n1 + b).reshape(-1)],
                                          vc[(ex * n1 + a).reshape(-1)]]))


def _ptr(a):
    return a.ctypes.data_as(_DP)


def _arr(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def set_threads(n):
    """Threads of the oracle's node and element loops (results do not
    depend on the number); returns the number in use."""
    return _load().idp_ref_set_threads(int(n))


def check(prob):
    return _load().idp_ref_check(ctypes.byref(_desc(prob)))


def sizes(prob):
    d = _desc(prob)
    lib = _load()
    if lib.idp_ref_check(ctypes.byref(d)):
        raise ValueError("invalid problem description")
    return lib.idp_ref_num_comp(ctypes.byref(d)), lib.idp_ref_num_nodes(ctypes.byref(d))


def gl(p):
    """Gauss-Lobatto nodes and weights on [0,1]."""
    xi = np.zeros(p + 1)
    w = np.zeros(p + 1)
    if _load().idp_ref_gl(p, _ptr(xi), _ptr(w)):
        raise ValueError("bad p")
    return xi, w


def dmat(p):
    D = np.zeros((p + 1, p + 1))
    if _load().idp_ref_dmat(p, _ptr(D)):
        raise ValueError("bad p")
    return D


def dhat(p):
    D = np.zeros((p + 1, p + 1))
    if _load().idp_ref_dhat(p, _ptr(D)):
        raise ValueError("bad p")
    return D


def flux(prob, u):
    """F(u) for one state vector u (nc,), returned as (dim, nc)."""
    nc, _ = sizes(prob)
    u = _arr(u)
    F = np.zeros((prob.dim, nc))
    _load().idp_ref_flux(ctypes.byref(_desc(prob)), _ptr(u), _ptr(F))
    return F


def lam(prob, uL, uR, n):
    uL, uR = _arr(uL), _arr(uR)
    n = _arr(list(n) + [0.0] * (2 - len(n)))
    return _load().idp_ref_lambda(ctypes.byref(_desc(prob)), _ptr(uL), _ptr(uR), _ptr(n))


def smoothness(prob, u):
    """Smoothness factor eps_K of every element (Sec. 4.4) for the limited
    component of u (u, or rho for Euler); shape (nx*ny,)."""
    nc, nn = sizes(prob)
    u = _arr(u).reshape(nc, nn)
    eps = np.empty(int(prob.nx) * int(prob.ny))
    rc = _load().idp_ref_smoothness(ctypes.byref(_desc(prob)), _ptr(u), _ptr(eps))
    if rc:
        raise ValueError("idp_ref_smoothness failed with %d" % rc)
    return eps


def fe(prob, u, dt, trace=False):
    """One forward-Euler sub-step; with trace=True also returns a dict of the
    per-node intermediate arrays (uL, uH, rH, rL, rbar, umin, umax, kmin,
    alpha_z, alpha)."""
    nc, nn = sizes(prob)
    u = _arr(u).reshape(nc, nn)
    out = np.empty((nc, nn))
    tr = None
    arrays = {}
    if trace:
        dim = prob.dim
        shapes = {"uL": (nc, nn), "uH": (nc, nn), "rH": (dim, nc, nn),
                  "rL": (dim, nc, nn), "rbar": (dim, nc, nn), "umin": (nn,),
                  "umax": (nn,), "kmin": (nn,), "alpha_z": (nn,), "alpha": (nn,)}
        tr = _Trace()
        for k, s in shapes.items():
            arrays[k] = np.zeros(s)
            setattr(tr, k, _ptr(arrays[k]))
    rc = _load().idp_ref_fe(ctypes.byref(_desc(prob)), _ptr(u), _ptr(out),
                            float(dt), ctypes.byref(tr) if trace else None)
    if rc:
        raise ValueError("idp_ref_fe failed with %d" % rc)
    return (out, arrays) if trace else out


def stage(prob, u_n, u_s, dt, s):
    nc, nn = sizes(prob)
    u_s = _arr(u_s).reshape(nc, nn)
    un = None if u_n is None else _arr(u_n).reshape(nc, nn)
    out = np.empty((nc, nn))
    rc = _load().idp_ref_stage(ctypes.byref(_desc(prob)),
                               None if un is None else _ptr(un), _ptr(u_s),
                               _ptr(out), float(dt), int(s))
    if rc:
        raise ValueError("idp_ref_stage failed with %d" % rc)
    return out


def step(prob, u, dt):
    nc, nn = sizes(prob)
    v = _arr(u).reshape(nc, nn).copy()
    rc = _load().idp_ref_step(ctypes.byref(_desc(prob)), _ptr(v), float(dt))
    if rc:
        raise ValueError("idp_ref_step failed with %d" % rc)
    return v


def max_dt(prob, u):
    nc, nn = sizes(prob)
    u = _arr(u).reshape(nc, nn)
    dt = np.zeros(1)
    rc = _load().idp_ref_max_dt(ctypes.byref(_desc(prob)), _ptr(u), _ptr(dt))
    if rc:
        raise ValueError("idp_ref_max_dt failed with %d" % rc)
    return float(dt[0])
