"""Seeded synthetic workloads for the IDP DG stage.

This module only builds problem descriptions and initial states; it holds
none of the method's arithmetic and imports neither the GPU binding nor the
oracle, so both sides can take their inputs from it.

All problems are periodic on [0,1]^d, FP64, in the state layout
``u[c][e][b][a]`` (component, element e = ey*nx + ex, y node, x node).
Node coordinates use the Gauss-Lobatto points of the element, computed here
with numpy's Legendre class (a third, independent source of the points).

Workload recipes (the paper's test problems are analytic; there is no
dataset):
  * ``advection_1d``  -- u_t + u_x = 0, 64 elements, p = 3, sin(2 pi x) plus
    a unit pulse on [0.3, 0.5]; dt = 0.2 of the low-order CFL bound.
  * ``burgers_2d``    -- u_t + (u^2/2)_x + (u^2/2)_y = 0 on 128^2, p = 3:
    0.5 + 0.5 sin(2 pi x) sin(2 pi y) + 0.05 U(-1,1) per node + a step of 0.5
    on the elements whose centre has x > 0.5.
  * ``euler_2d``      -- Euler, gamma = 1.4, 256^2, p = 4: four quadrants
    (by element centre) with (rho, p) ~ U[0.1, 1.5]^2 and v ~ U[-0.8, 0.8]^2
    per quadrant, node density times (1 + 0.01 U(-1,1)).
  * ``batch_mix``     -- many Euler solves of uneven n in [32, 256] and p in
    {2..6}, each with its own quadrant data.
  * ``solid_body``    -- u_t + div(beta u) = 0 on [0,1]^2 with the rotation
    field beta = 2 pi (1/2 - y, x - 1/2), 64^2, p = 3: a smooth bump, a cone
    and a slotted cylinder of radius 0.15 (the paper's Sec. 5 test); one
    revolution takes t = 1.
"""
from dataclasses import dataclass, field
from typing import List, Tuple

import numpy as np

ADVECTION, BURGERS, EULER, ADVECTION_FIELD = 0, 1, 2, 3
SUBCELL, TARGET, LOW, SUBCELL_SI, ELEMENTWISE = 0, 1, 2, 3, 4
BC_STATE, BC_OUTFLOW, BC_SLIP = 1, 2, 3      # per-node conditions of an open side
EQ_NAMES = {"advection": ADVECTION, "burgers": BURGERS, "euler": EULER,
            "advection_field": ADVECTION_FIELD}
LIMITER_NAMES = {"subcell": SUBCELL, "target": TARGET, "low": LOW, "subcell_si": SUBCELL_SI,
                 "elementwise": ELEMENTWISE}


@dataclass
class Problem:
    dim: int
    nx: int
    ny: int
    p: int
    eq: int
    lx: float = 1.0
    ly: float = 1.0
    vel: Tuple[float, float] = (1.0, 1.0)
    gamma: float = 1.4
    limiter: int = SUBCELL
    gmin: float = 0.0     # global bounds of the limited component (SUBCELL_SI)
    gmax: float = 0.0
    # ADVECTION_FIELD: the velocity beta = (beta_x(y), beta_y(x)) sampled on
    # the node rows (beta_x at y = (ey + xi_b) hy, index ey*(p+1) + b) and
    # the node columns (beta_y at x = (ex + xi_a) hx, index ex*(p+1) + a)
    vrows: Tuple[float, ...] = ()
    vcols: Tuple[float, ...] = ()
    # per direction (x, y): 0 periodic, 1 open; the open sides' per-node
    # conditions in bnd (a Boundary)
    bc: Tuple[int, int] = (0, 0)
    bnd: object = None
    # curved meshes (2-D, periodic): the physical coordinates of every node,
    # a float64 array (2, Nn) in state order; None: the Cartesian mesh of
    # lx/nx x ly/ny elements
    coords: object = None

    @property
    def nc(self) -> int:
        return self.dim + 2 if self.eq == EULER else 1

    @property
    def nodes_per_element(self) -> int:
        return (self.p + 1) ** self.dim

    @property
    def num_nodes(self) -> int:
        return self.nx * self.ny * self.nodes_per_element

    def replace(self, **kw) -> "Problem":
        d = dict(self.__dict__)
        d.update(kw)
        return Problem(**d)


@dataclass
class Boundary:
    """Per-node conditions of the open sides of a problem, sides ordered
    x = 0, x = lx, y = 0, y = ly.  type[side] is an int8 array with one code
    (BC_STATE, BC_OUTFLOW, BC_SLIP) per boundary node, in node-row order
    ey*(p+1) + b on x-sides and node-column order ex*(p+1) + a on y-sides
    (one node per side in 1-D);
    state[side] is None or a float64 array (nc, n) of prescribed states.
    Periodic sides hold None."""
    type: list
    state: list


def side_nodes(prob: Problem, side: int) -> int:
    """Boundary nodes of one side: one in 1-D."""
    if prob.dim == 1:
        return 1
    return (prob.ny if side < 2 else prob.nx) * (prob.p + 1)


def uniform_boundary(prob: Problem, codes, states=None) -> Boundary:
    """One condition per open side: codes[side] (None for periodic sides),
    states[side] a length-nc vector for BC_STATE sides."""
    types, sts = [None] * 4, [None] * 4
    for side in range(4):
        if codes[side] is None:
            continue
        n = side_nodes(prob, side)
        types[side] = np.full(n, codes[side], dtype=np.int8)
        if states is not None and states[side] is not None:
            v = np.asarray(states[side], dtype=np.float64).reshape(-1, 1)
            sts[side] = np.ascontiguousarray(np.repeat(v, n, axis=1))
    return Boundary(types, sts)


@dataclass
class Workload:
    name: str
    prob: Problem
    u0: np.ndarray            # (nc, Nn) float64
    cfl: float                # dt = cfl * (low-order CFL bound)
    steps: int
    seed: int = 0
    meta: dict = field(default_factory=dict)


def gl_points(p: int) -> np.ndarray:
    """Gauss-Lobatto points on [0,1] (end points and roots of P_p')."""
    inner = np.polynomial.legendre.Legendre.basis(p).deriv().roots()
    x = np.concatenate([[-1.0], np.sort(inner.real), [1.0]])
    return 0.5 * (x + 1.0)


def node_coords(prob: Problem):
    """Physical node coordinates (x, y) in state order; y is None in 1-D."""
    xi = gl_points(prob.p)
    hx = prob.lx / prob.nx
    n1 = prob.p + 1
    if prob.dim == 1:
        ex = np.arange(prob.nx)[:, None]
        x = (ex + xi[None, :]) * hx
        return x.reshape(-1), None, (ex[:, 0] + 0.5) * hx
    hy = prob.ly / prob.ny
    ey, ex = np.meshgrid(np.arange(prob.ny), np.arange(prob.nx), indexing="ij")
    ey = ey.reshape(-1)[:, None, None]
    ex = ex.reshape(-1)[:, None, None]
    b = np.arange(n1)[None, :, None]
    a = np.arange(n1)[None, None, :]
    x = (ex + xi[a]) * hx + 0.0 * b
    y = (ey + xi[b]) * hy + 0.0 * a
    return x.reshape(-1), y.reshape(-1), None


def perturbed_coords(prob: Problem, amp: float = 0.05):
    """Node coordinates of a smoothly curved periodic mesh: the Cartesian
    nodes (X, Y) moved by amp (lx, ly) sin(2 pi X/lx) sin(2 pi Y/ly) in both
    directions (an invertible map for amp < 1/(2 pi)).  The periodic copies
    of a point differ by the box lengths, so neighbouring elements share
    their face nodes."""
    X, Y, _ = node_coords(prob)
    s = np.sin(2 * np.pi * X / prob.lx) * np.sin(2 * np.pi * Y / prob.ly)
    return np.ascontiguousarray(np.stack([X + amp * prob.lx * s, Y + amp * prob.ly * s]))


def rotated_coords(prob: Problem, theta: float):
    """Node coordinates of the Cartesian mesh rotated by theta about the
    origin (an affine mesh whose faces are not aligned with the axes)."""
    X, Y, _ = node_coords(prob)
    c, s = np.cos(theta), np.sin(theta)
    return np.ascontiguousarray(np.stack([c * X - s * Y, s * X + c * Y]))


def _element_centres(prob: Problem):
    n1 = prob.p + 1
    hx = prob.lx / prob.nx
    if prob.dim == 1:
        return ((np.arange(prob.nx) + 0.5) * hx).repeat(n1), None
    hy = prob.ly / prob.ny
    ey, ex = np.meshgrid(np.arange(prob.ny), np.arange(prob.nx), indexing="ij")
    xc = ((ex.reshape(-1) + 0.5) * hx).repeat(n1 * n1)
    yc = ((ey.reshape(-1) + 0.5) * hy).repeat(n1 * n1)
    return xc, yc


def advection_1d(nx: int = 64, p: int = 3, limiter: int = SUBCELL) -> Workload:
    prob = Problem(dim=1, nx=nx, ny=1, p=p, eq=ADVECTION, vel=(1.0, 0.0),
                   limiter=limiter)
    x, _, _ = node_coords(prob)
    xc, _ = _element_centres(prob)
    # a node on an element face takes the value from inside its own element
    xe = xc + (x - xc) * (1.0 - 1e-9)
    u = np.sin(2 * np.pi * x) + ((xe >= 0.3) & (xe <= 0.5)).astype(np.float64)
    return Workload("advection_1d", prob, u[None, :].copy(), cfl=0.2, steps=200)


def burgers_2d(n: int = 128, p: int = 3, seed: int = 2,
               limiter: int = SUBCELL) -> Workload:
    prob = Problem(dim=2, nx=n, ny=n, p=p, eq=BURGERS, vel=(1.0, 1.0),
                   limiter=limiter)
    rng = np.random.default_rng(seed)
    x, y, _ = node_coords(prob)
    xc, _ = _element_centres(prob)
    u = 0.5 + 0.5 * np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y)
    u = u + 0.05 * rng.uniform(-1.0, 1.0, size=u.shape)
    u = u + 0.5 * (xc > 0.5)
    return Workload("burgers_2d", prob, u[None, :].copy(), cfl=0.5, steps=100,
                    seed=seed)


def euler_quadrants(prob: Problem, rng) -> np.ndarray:
    """Four-quadrant piecewise-constant Riemann data with 1% density noise,
    returned in conserved variables (rho, rho v, rho E)."""
    g = prob.gamma
    rho_p = rng.uniform(0.1, 1.5, size=(4, 2))
    vel = rng.uniform(-0.8, 0.8, size=(4, 2))
    xc, yc = _element_centres(prob)
    if prob.dim == 1:
        q = (xc > 0.5).astype(int)
    else:
        q = (xc > 0.5).astype(int) + 2 * (yc > 0.5).astype(int)
    rho = rho_p[q, 0] * (1.0 + 0.01 * rng.uniform(-1.0, 1.0, size=q.shape))
    pr = rho_p[q, 1]
    d = prob.dim
    u = np.empty((d + 2, q.size))
    u[0] = rho
    kin = np.zeros(q.size)
    for k in range(d):
        u[1 + k] = rho * vel[q, k]
        kin += vel[q, k] ** 2
    u[d + 1] = pr / (g - 1.0) + 0.5 * rho * kin
    return u


def euler_2d(n: int = 256, p: int = 4, seed: int = 3,
             limiter: int = SUBCELL) -> Workload:
    prob = Problem(dim=2, nx=n, ny=n, p=p, eq=EULER, gamma=1.4, limiter=limiter)
    rng = np.random.default_rng(seed)
    u = euler_quadrants(prob, rng)
    return Workload("euler_2d", prob, u, cfl=0.5, steps=50, seed=seed)


def euler_1d(n: int = 64, p: int = 3, seed: int = 5,
             limiter: int = SUBCELL) -> Workload:
    prob = Problem(dim=1, nx=n, ny=1, p=p, eq=EULER, gamma=1.4, limiter=limiter)
    rng = np.random.default_rng(seed)
    u = euler_quadrants(prob, rng)
    return Workload("euler_1d", prob, u, cfl=0.5, steps=50, seed=seed)


def batch_mix(count: int = 64, n_range=(32, 256), p_choices=(2, 3, 4, 5, 6),
              seed: int = 4) -> List[Workload]:
    """Independent Euler solves of uneven mesh size and degree."""
    rng = np.random.default_rng(seed)
    out = []
    for s in range(count):
        n = int(rng.integers(n_range[0], n_range[1] + 1))
        p = int(rng.choice(p_choices))
        prob = Problem(dim=2, nx=n, ny=n, p=p, eq=EULER, gamma=1.4)
        u = euler_quadrants(prob, np.random.default_rng([seed, s]))
        out.append(Workload("euler_2d_batch", prob, u, cfl=0.5, steps=50,
                            seed=seed, meta={"index": s}))
    return out


def rotation_lines(prob: Problem, omega: float = 2.0 * np.pi, centre=(0.5, 0.5)):
    """The solid-body rotation field beta = omega (c_y - y, x - c_x) on the
    node rows and columns of prob (see Problem.vrows / vcols)."""
    xi = gl_points(prob.p)
    hx, hy = prob.lx / prob.nx, prob.ly / prob.ny
    y = ((np.arange(prob.ny)[:, None] + xi[None, :]) * hy).reshape(-1)
    x = ((np.arange(prob.nx)[:, None] + xi[None, :]) * hx).reshape(-1)
    return tuple(omega * (centre[1] - y)), tuple(omega * (x - centre[0]))


def solid_body_state(x, y):
    """The three bodies at points (x, y): bump at (0.25, 0.5), cone at
    (0.5, 0.25), slotted cylinder at (0.5, 0.75), radius 0.15, zero
    elsewhere."""
    r0 = 0.15
    u = np.zeros_like(x)
    r = np.hypot(x - 0.25, y - 0.5) / r0
    u = np.where(r <= 1.0, 0.25 * (1.0 + np.cos(np.pi * r)), u)
    r = np.hypot(x - 0.5, y - 0.25) / r0
    u = np.where(r <= 1.0, 1.0 - r, u)
    r = np.hypot(x - 0.5, y - 0.75) / r0
    cyl = (np.abs(x - 0.5) >= 0.025) | (y >= 0.85)
    u = np.where(r <= 1.0, cyl.astype(np.float64), u)
    return u


def solid_body(n: int = 64, p: int = 3, limiter: int = SUBCELL) -> Workload:
    prob = Problem(dim=2, nx=n, ny=n, p=p, eq=ADVECTION_FIELD, limiter=limiter)
    vr, vc = rotation_lines(prob)
    prob = prob.replace(vrows=vr, vcols=vc)
    x, y, _ = node_coords(prob)
    return Workload("solid_body", prob, solid_body_state(x, y)[None, :].copy(), cfl=0.5,
                    steps=0, meta={"t_end": 1.0})


def small_cases():
    """A handful of small problems spanning the equations, dimensions and
    a ragged element count, for parity checks."""
    return [
        advection_1d(),
        burgers_2d(n=16, p=3),
        euler_2d(n=16, p=4),
    ]


# ---------------------------------------------------------------------------
# Serving workload: a seeded Poisson stream of solve requests (Burgers and
# Euler), with initial states generated on the device so that admitting a
# large request does not stall on the host.
# ---------------------------------------------------------------------------

@dataclass
class Request:
    rid: int
    kind: str           # "euler" or "burgers"
    n: int              # elements per direction
    p: int
    steps: int
    arrival: float      # seconds after the start of the stream
    seed: int

    def problem(self) -> Problem:
        if self.kind == "euler":
            return Problem(dim=2, nx=self.n, ny=self.n, p=self.p, eq=EULER, gamma=1.4)
        return Problem(dim=2, nx=self.n, ny=self.n, p=self.p, eq=BURGERS, vel=(1.0, 1.0))


def request_stream(count: int, rate: float, n_range=(16, 512), p_range=(2, 6),
                   steps_range=(20, 200), seed: int = 5) -> List[Request]:
    """Poisson arrivals at `rate` requests/s; half Burgers, half Euler."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        out.append(Request(rid=i, kind="euler" if rng.random() < 0.5 else "burgers",
                           n=int(rng.integers(n_range[0], n_range[1] + 1)),
                           p=int(rng.integers(p_range[0], p_range[1] + 1)),
                           steps=int(rng.integers(steps_range[0], steps_range[1] + 1)),
                           arrival=t, seed=int(rng.integers(1 << 31))))
    return out


def initial_state_device(req: Request, device="cuda"):
    """The request's initial state, generated with torch on the device:
    Euler four-quadrant data with 1% density noise, or the Burgers recipe
    (0.5 + 0.5 sin sin + 0.05 noise + 0.5 step)."""
    import torch
    prob = req.problem()
    n1 = prob.p + 1
    xi = torch.tensor(gl_points(prob.p), dtype=torch.float64, device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(req.seed)
    h = 1.0 / req.n
    e = torch.arange(req.n, dtype=torch.float64, device=device)
    # node coordinates in layout [ey][ex][b][a]
    x = ((e[None, :, None, None] + xi[None, None, None, :]) * h).expand(req.n, req.n, n1, n1)
    y = ((e[:, None, None, None] + xi[None, None, :, None]) * h).expand(req.n, req.n, n1, n1)
    xc = ((e[None, :, None, None] + 0.5) * h).expand(req.n, req.n, n1, n1)
    yc = ((e[:, None, None, None] + 0.5) * h).expand(req.n, req.n, n1, n1)
    if req.kind == "burgers":
        u = 0.5 + 0.5 * torch.sin(2 * np.pi * x) * torch.sin(2 * np.pi * y)
        u = u + 0.05 * (2 * torch.rand(u.shape, generator=gen, dtype=torch.float64, device=device) - 1)
        u = u + 0.5 * (xc > 0.5).double()
        return u.reshape(1, -1).contiguous()
    rng = np.random.default_rng(req.seed)
    rho_p = torch.tensor(rng.uniform(0.1, 1.5, size=(4, 2)), dtype=torch.float64, device=device)
    vel = torch.tensor(rng.uniform(-0.8, 0.8, size=(4, 2)), dtype=torch.float64, device=device)
    q = ((xc > 0.5).long() + 2 * (yc > 0.5).long()).reshape(-1)
    noise = 2 * torch.rand(q.shape, generator=gen, dtype=torch.float64, device=device) - 1
    rho = rho_p[q, 0] * (1.0 + 0.01 * noise)
    pr = rho_p[q, 1]
    u = torch.empty((4, q.numel()), dtype=torch.float64, device=device)
    u[0] = rho
    u[1] = rho * vel[q, 0]
    u[2] = rho * vel[q, 1]
    u[3] = pr / (prob.gamma - 1.0) + 0.5 * rho * (vel[q, 0] ** 2 + vel[q, 1] ** 2)
    return u
