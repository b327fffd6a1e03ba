"""ctypes binding of libidp_dg.so (include/idp_dg.h).

Argument marshalling only: every step of the stage runs in the library's
HIP kernels.  States are torch float64 CUDA tensors of shape (nc, Nn)
(contiguous, layout u[c][e][b][a]); work is enqueued on the torch stream
that was current when the Solver was created.  The library must have been
built (``python -m paper_2004_08503_amd.build``); importing this module
raises if it is missing.
"""
import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libidp_dg.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "idp_dg.h")

ADVECTION, BURGERS, EULER, ADVECTION_FIELD = 0, 1, 2, 3
SUBCELL, TARGET_ONLY, LOW_ONLY, SUBCELL_SI, ELEMENTWISE = 0, 1, 2, 3, 4
EINVAL, ENOMEM, EHIP = -1, -2, -3


class Desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("lx", ctypes.c_double), ("ly", ctypes.c_double),
                ("p", ctypes.c_int), ("eq", ctypes.c_int),
                ("velocity", ctypes.c_double * 2), ("gamma", ctypes.c_double),
                ("limiter", ctypes.c_int), ("gmin", ctypes.c_double), ("gmax", ctypes.c_double),
                ("vel_rows", ctypes.POINTER(ctypes.c_double)),
                ("vel_cols", ctypes.POINTER(ctypes.c_double)),
                ("bc", ctypes.c_int * 2)]


class Diag(ctypes.Structure):
    _fields_ = [("limited_nodes", ctypes.c_longlong), ("entropy_nodes", ctypes.c_longlong),
                ("bad_input", ctypes.c_int), ("low_order_violation", ctypes.c_int)]


_VP = ctypes.c_void_p
_DPP = ctypes.POINTER(ctypes.c_void_p)


def _declare(lib):
    H = ctypes.c_void_p
    sig = {
        "idp_dg_create": (ctypes.c_int, [ctypes.POINTER(Desc), _VP, ctypes.POINTER(H)]),
        "idp_dg_workspace_bytes": (ctypes.c_longlong, [ctypes.POINTER(Desc)]),
        "idp_dg_create_in": (ctypes.c_int, [ctypes.POINTER(Desc), _VP, _VP, ctypes.c_longlong,
                                            ctypes.POINTER(H)]),
        "idp_dg_destroy": (None, [H]),
        "idp_dg_num_nodes": (ctypes.c_long, [H]),
        "idp_dg_num_comp": (ctypes.c_int, [H]),
        "idp_dg_stage": (ctypes.c_int, [H, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int]),
        "idp_dg_stage_trace": (ctypes.c_int, [H, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int, _VP]),
        "idp_dg_step": (ctypes.c_int, [H, _VP, ctypes.c_double]),
        "idp_dg_step_noalloc": (ctypes.c_int, [ctypes.POINTER(Desc), _VP, ctypes.c_double, _VP]),
        "idp_dg_step_cfl": (ctypes.c_int, [H, _VP, ctypes.c_double]),
        "idp_dg_last_dt": (ctypes.c_int, [H, ctypes.POINTER(ctypes.c_double)]),
        "idp_dg_max_dt": (ctypes.c_int, [H, _VP, ctypes.POINTER(ctypes.c_double)]),
        "idp_dg_max_dt_async": (ctypes.c_int, [H, _VP, _VP]),
        "idp_dg_stage_dt": (ctypes.c_int, [H, _VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int]),
        "idp_dg_tune": (ctypes.c_int, [H, _VP, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int)]),
        "idp_dg_tile_shape": (ctypes.c_int, [H]),
        "idp_dg_tile_elems": (ctypes.c_int, [H]),
        "idp_dg_tile_dims": (ctypes.c_int, [H, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
        "idp_dg_set_tile_shape": (ctypes.c_int, [H, ctypes.c_int]),
        "idp_dg_batch_tune": (ctypes.c_int, [H, ctypes.POINTER(_VP), ctypes.c_double, ctypes.c_int]),
        "idp_dg_diagnostics": (ctypes.c_int, [H, ctypes.POINTER(Diag)]),
        "idp_dg_set_boundary": (ctypes.c_int, [H, ctypes.c_int, _VP, _VP]),
        "idp_dg_set_mesh": (ctypes.c_int, [H, _VP]),
        "idp_dg_mesh_metric": (ctypes.c_int, [ctypes.POINTER(Desc), _VP, _VP]),
        "idp_dg_last_error": (ctypes.c_char_p, [H]),
        "idp_dg_build_hash": (ctypes.c_char_p, []),
        "idp_dg_batch_create": (ctypes.c_int, [ctypes.POINTER(H), ctypes.c_int, _VP, ctypes.POINTER(H)]),
        "idp_dg_batch_destroy": (None, [H]),
        "idp_dg_batch_update": (ctypes.c_int, [H, ctypes.POINTER(H), ctypes.c_int]),
        "idp_dg_batch_num_items": (ctypes.c_int, [H]),
        "idp_dg_batch_step": (ctypes.c_int, [H, ctypes.POINTER(_VP), ctypes.POINTER(ctypes.c_double)]),
        "idp_dg_batch_step_cfl": (ctypes.c_int, [H, ctypes.POINTER(_VP), ctypes.c_double]),
        "idp_dg_batch_last_dt": (ctypes.c_int, [H, ctypes.POINTER(ctypes.c_double)]),
        "idp_dg_batch_last_error": (ctypes.c_char_p, [H]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


# torch bundles its own HIP runtime (SONAME libamdhip64.so.7, loaded by
# torch under another file name).  Loading torch first makes this library
# bind to that same runtime by SONAME; loading this library first would put
# a second HIP/HSA runtime into the process, and device initialisation in
# one of them fails.
import torch  # noqa: E402,F401

if not os.path.exists(LIB_PATH):
    raise ImportError("libidp_dg.so is not built (run python -m paper_2004_08503_amd.build)")
lib = _declare(ctypes.CDLL(LIB_PATH))


def mesh_metric(prob, coords=None):
    """idp_dg_mesh_metric: the (9, Nn) metric array the library computes for
    a curved mesh (host only, no GPU needed)."""
    import numpy as np
    xy = np.ascontiguousarray(prob.coords if coords is None else coords, dtype=np.float64)
    desc = make_desc(prob)
    out = np.empty((9, prob.num_nodes))
    if xy.shape != (2, prob.num_nodes):
        raise ValueError("coords must have shape (2, %d)" % prob.num_nodes)
    rc = lib.idp_dg_mesh_metric(ctypes.byref(desc), ctypes.c_void_p(xy.ctypes.data),
                                ctypes.c_void_p(out.ctypes.data))
    if rc:
        raise IdpError(rc, lib.idp_dg_last_error(None).decode())
    return out


def build_hash():
    """The source hash the loaded library was built from."""
    return lib.idp_dg_build_hash().decode()


# a library built from other sources than the ones beside it is refused
from . import build as _build  # noqa: E402
if build_hash() != _build.source_hash():
    raise ImportError("libidp_dg.so was built from other sources (library %s, sources %s): rebuild it "
                      "(python -m paper_2004_08503_amd.build)" % (build_hash(), _build.source_hash()))


def header_symbols():
    """Function names declared in include/idp_dg.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(idp_dg_\w+)\s*\(", text)))


class IdpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("idp_dg error %d: %s" % (code, msg))
        self.code = code


def make_desc(prob):
    d = Desc()
    d.dim, d.nx, d.ny = int(prob.dim), int(prob.nx), int(prob.ny)
    d.lx, d.ly = float(prob.lx), float(prob.ly)
    d.p, d.eq = int(prob.p), int(prob.eq)
    v = list(prob.vel) + [0.0] * (2 - len(prob.vel))
    d.velocity[0], d.velocity[1] = float(v[0]), float(v[1])
    d.gamma = float(prob.gamma)
    d.limiter = int(prob.limiter)
    d.gmin = float(getattr(prob, "gmin", 0.0))
    d.gmax = float(getattr(prob, "gmax", 0.0))
    if d.eq == ADVECTION_FIELD:
        import numpy as np
        rows = np.ascontiguousarray(getattr(prob, "vrows", ()), dtype=np.float64)
        cols = np.ascontiguousarray(getattr(prob, "vcols", ()), dtype=np.float64)
        n1 = d.p + 1
        if rows.size != d.ny * n1 or cols.size != d.nx * n1:
            raise ValueError("vrows / vcols need ny*(p+1) / nx*(p+1) samples")
        dp = ctypes.POINTER(ctypes.c_double)
        d.vel_rows = rows.ctypes.data_as(dp)
        d.vel_cols = cols.ctypes.data_as(dp)
        d._keep = (rows, cols)   # alive as long as the descriptor
    bc = tuple(getattr(prob, "bc", (0, 0)))
    d.bc[0], d.bc[1] = int(bc[0]), int(bc[1])
    return d


NOALLOC_MAX_DOUBLES = 4 << 20


def step_noalloc(prob, u, dt):
    """idp_dg_step_noalloc: one step of u (float64 CUDA tensor (nc, Nn),
    contiguous) in place on the current torch stream, with the library's
    static stage buffers; raises IdpError on a non-zero return."""
    d = make_desc(prob)
    n1 = d.p + 1
    nn = d.nx * d.ny * (n1 * n1 if d.dim == 2 else n1)
    nc = d.dim + 2 if d.eq == EULER else 1
    if not (isinstance(u, torch.Tensor) and u.is_cuda and u.dtype == torch.float64
            and u.is_contiguous() and u.numel() == nc * nn):
        raise ValueError("u must be a contiguous float64 CUDA tensor of %d values" % (nc * nn))
    stream = torch.cuda.current_stream(u.device).cuda_stream
    rc = lib.idp_dg_step_noalloc(ctypes.byref(d), ctypes.c_void_p(u.data_ptr()), float(dt),
                                 ctypes.c_void_p(stream))
    if rc:
        raise IdpError(rc, lib.idp_dg_last_error(None).decode())


def family_of(prob):
    """Batches group solves of one kernel family: equation (Euler split by
    gamma = 7/5, 5/3 or other) and dimension."""
    eq = int(prob.eq)
    if eq == EULER:
        g = float(prob.gamma)
        eq = 10 + (0 if g == 1.4 else 1 if abs(g - 5.0 / 3.0) < 1e-15 else 2)
    return eq * 10 + int(prob.dim)


def _torch():
    import torch
    return torch


class Solver:
    """One problem on the current device and torch stream."""

    def __init__(self, prob, stream=None, workspace=False):
        """workspace=True places the handle's device buffers in a torch
        allocation (stream-ordered, no hipMalloc/hipFree by the library)."""
        torch = _torch()
        self.prob = prob
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self._h = ctypes.c_void_p()
        self._ws = None
        desc = make_desc(prob)
        if workspace:
            nbytes = lib.idp_dg_workspace_bytes(ctypes.byref(desc))
            if nbytes < 0:
                raise IdpError(int(nbytes), lib.idp_dg_last_error(None).decode())
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            base = self._ws.data_ptr()
            ofs = (-base) % 256
            rc = lib.idp_dg_create_in(ctypes.byref(desc), ctypes.c_void_p(stream.cuda_stream),
                                      ctypes.c_void_p(base + ofs), nbytes, ctypes.byref(self._h))
        else:
            rc = lib.idp_dg_create(ctypes.byref(desc), ctypes.c_void_p(stream.cuda_stream),
                                   ctypes.byref(self._h))
        if rc:
            raise IdpError(rc, lib.idp_dg_last_error(None).decode())
        self.nc = lib.idp_dg_num_comp(self._h)
        self.nn = lib.idp_dg_num_nodes(self._h)
        self._bnd = {}
        if getattr(prob, "coords", None) is not None:   # curved mesh: node coordinates (2, Nn)
            self.set_mesh(prob.coords)
        bnd = getattr(prob, "bnd", None)
        if bnd is not None:   # the problem's own boundary data, copied to the device
            for side in range(4):
                if bnd.type[side] is not None:
                    t = torch.as_tensor(bnd.type[side], dtype=torch.int8).to("cuda")
                    st = None if bnd.state[side] is None else \
                        torch.as_tensor(bnd.state[side], dtype=torch.float64).to("cuda").contiguous()
                    self.set_boundary(side, t, st)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h:
            lib.idp_dg_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._ws = None   # torch frees it in stream order

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc:
            raise IdpError(rc, lib.idp_dg_last_error(self._h).decode())

    def _ptr(self, t, name):
        torch = _torch()
        if t is None:
            return None
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and t.is_contiguous() and t.numel() == self.nc * self.nn):
            raise ValueError("%s must be a contiguous float64 CUDA tensor of %d values"
                             % (name, self.nc * self.nn))
        return ctypes.c_void_p(t.data_ptr())

    def set_boundary(self, side, type_t, state_t=None):
        """idp_dg_set_boundary: int8 CUDA tensor of per-node codes and an
        optional float64 CUDA tensor (nc, n) of prescribed states.  The
        tensors are kept referenced until replaced; their contents may be
        rewritten between launches."""
        torch = _torch()
        if not (isinstance(type_t, torch.Tensor) and type_t.is_cuda and type_t.dtype == torch.int8
                and type_t.is_contiguous()):
            raise ValueError("type must be a contiguous int8 CUDA tensor")
        sp = None
        if state_t is not None:
            if not (isinstance(state_t, torch.Tensor) and state_t.is_cuda
                    and state_t.dtype == torch.float64 and state_t.is_contiguous()):
                raise ValueError("state must be a contiguous float64 CUDA tensor")
            sp = ctypes.c_void_p(state_t.data_ptr())
        self._check(lib.idp_dg_set_boundary(self._h, int(side), ctypes.c_void_p(type_t.data_ptr()), sp))
        self._bnd[side] = (type_t, state_t)

    def set_mesh(self, coords):
        """idp_dg_set_mesh: host float64 node coordinates of shape (2, Nn),
        x then y, in state order."""
        import numpy as np
        xy = np.ascontiguousarray(coords, dtype=np.float64)
        if xy.shape != (2, self.nn):
            raise ValueError("coords must have shape (2, %d)" % self.nn)
        self._check(lib.idp_dg_set_mesh(self._h, ctypes.c_void_p(xy.ctypes.data)))

    def empty(self):
        torch = _torch()
        return torch.empty((self.nc, self.nn), dtype=torch.float64, device="cuda")

    def stage(self, u_n, u_s, u_out, dt, stage):
        self._check(lib.idp_dg_stage(self._h, self._ptr(u_n, "u_n"), self._ptr(u_s, "u_s"),
                                     self._ptr(u_out, "u_out"), float(dt), int(stage)))

    def stage_trace(self, u_n, u_s, u_out, dt, stage):
        """idp_dg_stage plus the limiter intermediates: returns a (5, Nn)
        tensor [umin, umax, kmin, alpha_z, alpha]."""
        torch = _torch()
        tr = torch.empty((5, self.nn), dtype=torch.float64, device="cuda")
        self._check(lib.idp_dg_stage_trace(self._h, self._ptr(u_n, "u_n"), self._ptr(u_s, "u_s"),
                                           self._ptr(u_out, "u_out"), float(dt), int(stage),
                                           ctypes.c_void_p(tr.data_ptr())))
        return tr

    def step(self, u, dt):
        self._check(lib.idp_dg_step(self._h, self._ptr(u, "u"), float(dt)))

    def step_cfl(self, u, cfl):
        self._check(lib.idp_dg_step_cfl(self._h, self._ptr(u, "u"), float(cfl)))

    def last_dt(self):
        v = ctypes.c_double()
        self._check(lib.idp_dg_last_dt(self._h, ctypes.byref(v)))
        return v.value

    def max_dt(self, u):
        v = ctypes.c_double()
        self._check(lib.idp_dg_max_dt(self._h, self._ptr(u, "u"), ctypes.byref(v)))
        return v.value

    def max_dt_async(self, u, dt_dev):
        """Write the CFL bound of u into the one-element float64 CUDA tensor
        dt_dev without synchronising."""
        self._check(lib.idp_dg_max_dt_async(self._h, self._ptr(u, "u"), self._scalar(dt_dev)))

    def stage_dt(self, u_n, u_s, u_out, dt_dev, cfl, stage):
        """idp_dg_stage with dt = cfl * dt_dev[0] read on the device."""
        self._check(lib.idp_dg_stage_dt(self._h, self._ptr(u_n, "u_n"), self._ptr(u_s, "u_s"),
                                        self._ptr(u_out, "u_out"), self._scalar(dt_dev),
                                        float(cfl), int(stage)))


    NUM_TILE_SHAPES = 2

    def tune(self, u, cfl=0.5, reps=5):
        """idp_dg_tune: time `reps` device-timestepped steps of u (only read)
        under each tile shape, keep the fastest and return it."""
        out = ctypes.c_int(-1)
        self._check(lib.idp_dg_tune(self._h, self._ptr(u, "u"), float(cfl), int(reps), ctypes.byref(out)))
        return out.value

    @property
    def tile_shape(self):
        return lib.idp_dg_tile_shape(self._h)

    @property
    def tile_elems(self):
        """Elements per workgroup of the current tile shape."""
        return lib.idp_dg_tile_elems(self._h)

    @property
    def tile_dims(self):
        """(elements per tile in x, in y) of the current tile shape."""
        tx, ty = ctypes.c_int(), ctypes.c_int()
        self._check(lib.idp_dg_tile_dims(self._h, ctypes.byref(tx), ctypes.byref(ty)))
        return tx.value, ty.value

    def set_tile_shape(self, shape):
        self._check(lib.idp_dg_set_tile_shape(self._h, int(shape)))
    def _scalar(self, t):
        torch = _torch()
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64
                and t.numel() >= 1):
            raise ValueError("dt_dev must be a float64 CUDA tensor")
        return ctypes.c_void_p(t.data_ptr())

    def diagnostics(self):
        d = Diag()
        self._check(lib.idp_dg_diagnostics(self._h, ctypes.byref(d)))
        return {"limited_nodes": d.limited_nodes, "entropy_nodes": d.entropy_nodes,
                "bad_input": bool(d.bad_input), "low_order_violation": bool(d.low_order_violation)}


class Batch:
    """Many solves of one equation family stepped together: per RK stage,
    one work-list launch per degree over all their element tiles."""

    def __init__(self, solvers, stream=None):
        torch = _torch()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.solvers = list(solvers)
        self.n = len(self.solvers)
        hs = (ctypes.c_void_p * self.n)(*[s.handle for s in self.solvers])
        self._b = ctypes.c_void_p()
        rc = lib.idp_dg_batch_create(hs, self.n, ctypes.c_void_p(stream.cuda_stream),
                                     ctypes.byref(self._b))
        if rc:
            raise IdpError(rc, lib.idp_dg_batch_last_error(None).decode())
        self.num_items = lib.idp_dg_batch_num_items(self._b)

    def close(self):
        if self._b:
            lib.idp_dg_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc:
            raise IdpError(rc, lib.idp_dg_batch_last_error(self._b).decode())

    def update(self, solvers):
        """Change the member solves, keeping the batch's device storage."""
        solvers = list(solvers)
        hs = (ctypes.c_void_p * len(solvers))(*[s.handle for s in solvers])
        self._check(lib.idp_dg_batch_update(self._b, hs, len(solvers)))
        self.solvers = solvers
        self.n = len(solvers)
        self.num_items = lib.idp_dg_batch_num_items(self._b)

    def _ptrs(self, us):
        if len(us) != self.n:
            raise ValueError("need %d states" % self.n)
        return (ctypes.c_void_p * self.n)(*[s._ptr(u, "u[%d]" % i).value
                                            for i, (s, u) in enumerate(zip(self.solvers, us))])

    def step(self, us, dts):
        d = (ctypes.c_double * self.n)(*[float(x) for x in dts])
        self._check(lib.idp_dg_batch_step(self._b, self._ptrs(us), d))

    def step_cfl(self, us, cfl):
        self._check(lib.idp_dg_batch_step_cfl(self._b, self._ptrs(us), float(cfl)))

    def prepare(self, us):
        """The checked state-pointer array of `us`, for repeated
        step_cfl_prepared calls while the members and their state tensors
        stay the same (the tensors must stay alive)."""
        return self._ptrs(us)

    def step_cfl_prepared(self, ptrs, cfl):
        self._check(lib.idp_dg_batch_step_cfl(self._b, ptrs, float(cfl)))

    def tune(self, us, cfl=0.5, reps=5):
        """idp_dg_batch_tune: per degree, the tile shape idp_dg_tune picks on
        that degree's largest member (states only read)."""
        self._check(lib.idp_dg_batch_tune(self._b, self._ptrs(us), float(cfl), int(reps)))

    def last_dt(self):
        d = (ctypes.c_double * self.n)()
        self._check(lib.idp_dg_batch_last_dt(self._b, d))
        return list(d)
