"""Seeded synthetic inputs (initial states, potentials, boundary settings).

This module only *describes problems*: grids, initial primitive fields, the
potential psi and the boundary kinds.  It holds none of the method's arithmetic
and imports neither the HIP library nor the CPU oracle, so both of them can be
fed exactly the same arrays.

Fields are numpy float64, structure of arrays, x fastest:
``prim[5, nz, ny, nx] = (rho, u, v, w, p)``, ``psi[nz, ny, nx]``.

Random numbers come from SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the k-th
output (k = 1, 2, ...) of the stream seeded with s is mix(s + k * 0x9E3779B97F4A7C15).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Dict, Optional, Tuple

import numpy as np

PERIODIC, OUTFLOW, INFLOW, REFLECT = 0, 1, 2, 3

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, index) -> np.ndarray:
    """Outputs number index+1 of the SplitMix64 stream seeded with ``seed``."""
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (idx + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, index) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of SplitMix64."""
    return (splitmix64(seed, index) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


@dataclass
class Problem:
    name: str
    shape: Tuple[int, int, int]          # (nx, ny, nz)
    h: float
    gamma: float
    cfl: float
    bc: Tuple[int, int, int, int, int, int]
    prim: np.ndarray                     # [5, nz, ny, nx]
    psi: Optional[np.ndarray] = None     # [nz, ny, nx] or None (psi = 0)
    inflow: Dict[int, Tuple[float, float, float, float, float]] = field(default_factory=dict)
    origin: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    rho_vac: float = 1e-10
    t_end: float = math.inf
    steps: Optional[int] = None
    nu: float = 0.0                      # kinematic viscosity (0: inviscid)
    grav: float = 0.0                    # G of the gas's self-gravity (0: none)
    src: Optional[np.ndarray] = None     # mass source rate per cell [nz, ny, nx] (< 0: sink)
    eps_src: float = 0.0                 # specific internal energy of injected gas

    @property
    def cells(self) -> int:
        return self.shape[0] * self.shape[1] * self.shape[2]

    def inflow_list(self):
        return [tuple(self.inflow.get(f, (0.0, 0.0, 0.0, 0.0, 0.0))) for f in range(6)]


def centres(shape, h, origin=(0.0, 0.0, 0.0)):
    """Cell-centre coordinates x, y, z, each broadcastable to [nz, ny, nx]."""
    nx, ny, nz = shape
    x = origin[0] + (np.arange(nx) + 0.5) * h
    y = origin[1] + (np.arange(ny) + 0.5) * h
    z = origin[2] + (np.arange(nz) + 0.5) * h
    return x[None, None, :], y[None, :, None], z[:, None, None]


def _prim(shape):
    nx, ny, nz = shape
    return np.zeros((5, nz, ny, nx))


# --------------------------------------------------------------------------
# shock tube and friends
# --------------------------------------------------------------------------
def riemann_tube(n=128, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), gamma=1.4, axis=0,
                 transverse=4, x0=0.5, t_end=0.2, cfl=0.4, name="sod") -> Problem:
    """A 1D Riemann problem along ``axis`` on a unit length; left/right = (rho, u_n, p).

    The discontinuity sits at x0 (on a cell face when n*x0 is an integer)."""
    shape = [transverse] * 3
    shape[axis] = n
    shape = tuple(shape)
    h = 1.0 / n
    prim = _prim(shape)
    coords = centres(shape, h)
    s = np.broadcast_to(coords[axis], prim.shape[1:])
    L = s < x0
    prim[0] = np.where(L, left[0], right[0])
    prim[1 + axis] = np.where(L, left[1], right[1])
    prim[4] = np.where(L, left[2], right[2])
    bc = [PERIODIC] * 6
    bc[2 * axis] = bc[2 * axis + 1] = OUTFLOW
    return Problem(name, shape, h, gamma, cfl, tuple(bc), prim, t_end=t_end)


def sod(n=128, axis=0, transverse=4) -> Problem:
    """Sod's tube: (1, 0, 1) | (0.125, 0, 0.1), gamma 1.4, to t = 0.2."""
    return riemann_tube(n, axis=axis, transverse=transverse)


def vacuum_tube(n=100, gamma=5.0 / 3.0, transverse=4, t_end=0.1) -> Problem:
    """Gas (rho = p = 1, u = 0) on the left of x0 = 0.5, vacuum on the right."""
    return riemann_tube(n, left=(1.0, 0.0, 1.0), right=(0.0, 0.0, 0.0), gamma=gamma,
                        transverse=transverse, t_end=t_end, name="vacuum")


# --------------------------------------------------------------------------
# potential well
# --------------------------------------------------------------------------
def gaussian_well(shape, h, psi0=1.0, a=0.1, centre=(0.5, 0.5, 0.5)):
    x, y, z = centres(shape, h)
    r2 = (x - centre[0]) ** 2 + (y - centre[1]) ** 2 + (z - centre[2]) ** 2
    return np.ascontiguousarray(np.broadcast_to(-psi0 * np.exp(-r2 / (a * a)),
                                                (shape[2], shape[1], shape[0])))


def well_flow(n=256, mach=2.0, gamma=5.0 / 3.0, psi0=1.0, a=0.1, cfl=0.4, steps=100) -> Problem:
    """Supersonic flow through a Gaussian well psi = -psi0 exp(-r^2/a^2) on the unit box.

    Uniform initial state = inflow state rho = 1, p = 1/gamma (sound speed 1),
    u = (mach, 0, 0); inflow at -x, outflow at +x, periodic in y and z."""
    shape = (n, n, n)
    h = 1.0 / n
    psi = gaussian_well(shape, h, psi0, a)
    prim = _prim(shape)
    state = (1.0, mach, 0.0, 0.0, 1.0 / gamma)
    for v in range(5):
        prim[v] = state[v]
    bc = (INFLOW, OUTFLOW, PERIODIC, PERIODIC, PERIODIC, PERIODIC)
    return Problem("well_flow", shape, h, gamma, cfl, bc, prim, psi, inflow={0: state},
                   steps=steps)


def well_rest(n=64, gamma=5.0 / 3.0, psi0=1.0, a=0.1, cfl=0.4, bc=None, steps=100,
              shape=None) -> Problem:
    """Hydrostatic rest in the same well: rho = 1 - psi, p = rho^2 / 2, u = 0."""
    shape = shape or (n, n, n)
    h = 1.0 / shape[0]
    psi = gaussian_well(shape, h, psi0, a)
    prim = _prim(shape)
    prim[0] = 1.0 - psi
    prim[4] = 0.5 * prim[0] ** 2
    bc = bc or (PERIODIC,) * 6
    return Problem("well_rest", shape, h, gamma, cfl, tuple(bc), prim, psi, steps=steps)


def isothermal_rest(n=32, gamma=5.0 / 3.0, psi0=1.0, a=0.1, cfl=0.4, steps=100) -> Problem:
    """Isothermal hydrostatic state rho = p = exp(-psi) in the same well (a control)."""
    shape = (n, n, n)
    h = 1.0 / n
    psi = gaussian_well(shape, h, psi0, a)
    prim = _prim(shape)
    prim[0] = np.exp(-psi)
    prim[4] = prim[0]
    return Problem("isothermal_rest", shape, h, gamma, cfl, (PERIODIC,) * 6, prim, psi,
                   steps=steps)


# --------------------------------------------------------------------------
# self-bound cloud with a gas-vacuum edge
# --------------------------------------------------------------------------
def cloud(n=384, seed=0, R=0.3, eps=0.05, rho_c=1.0, amp=0.01, gamma=5.0 / 3.0, cfl=0.4,
          steps=200, rho_vac=1e-6) -> Problem:
    """Polytrope-like cloud rho = rho_c (1 - r^2/R^2)(1 + amp*zeta) inside R, vacuum outside,
    in the Plummer potential psi = -1/sqrt(r^2 + eps^2); zeta in [-1, 1) from SplitMix64
    of (seed, linear cell index).  The pressure is hydrostatic for the unperturbed
    density: p(r) = rho_c [G(R) - G(r)],
    G(s) = -(1 + eps^2/R^2)/sqrt(s^2 + eps^2) - sqrt(s^2 + eps^2)/R^2.
    Cells below rho_vac = 1e-6 rho_c count as vacuum: with a much lower floor, cells
    holding ~1e-8 of the mass reach speeds ~1e3 and set the CFL step."""
    shape = (n, n, n)
    h = 1.0 / n
    x, y, z = centres(shape, h)
    r2 = np.broadcast_to((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2, (n, n, n))
    psi = -1.0 / np.sqrt(r2 + eps * eps)
    zeta = 2.0 * uniform01(seed, np.arange(n * n * n, dtype=np.uint64)).reshape(n, n, n) - 1.0

    def Gf(s2):
        q = np.sqrt(s2 + eps * eps)
        return -(1.0 + eps * eps / (R * R)) / q - q / (R * R)

    inside = r2 < R * R
    prim = _prim(shape)
    prim[0] = np.where(inside, rho_c * (1.0 - r2 / (R * R)) * (1.0 + amp * zeta), 0.0)
    prim[4] = np.where(inside, rho_c * (Gf(R * R) - Gf(r2)), 0.0)
    return Problem("cloud", shape, h, gamma, cfl, (OUTFLOW,) * 6, prim,
                   np.ascontiguousarray(psi), steps=steps, rho_vac=rho_vac * rho_c)


def cold_sphere(n=16, R=0.3, G=1.0, rho_in=1.0, p_in=1e-6, gamma=5.0 / 3.0, cfl=0.4,
                rho_vac=1e-7) -> Problem:
    """A cold uniform sphere of radius R (rho_in, pressure p_in) in near vacuum
    (rho = 1e-8 rho_in, p = 0) with its own gravity on an isolated box (every
    face OUTFLOW).  At first every shell falls at -(4/3) pi G rho_in r."""
    shape = (n, n, n)
    h = 1.0 / n
    x, y, z = centres(shape, h)
    r = np.broadcast_to(np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2), shape[::-1])
    prim = _prim(shape)
    prim[0] = np.where(r < R, rho_in, 1e-8 * rho_in)
    prim[4] = np.where(r < R, p_in, 0.0)
    return Problem("cold_sphere", shape, h, gamma, cfl, (OUTFLOW,) * 6, prim, grav=G,
                   rho_vac=rho_vac * rho_in)


def z_cut(arr, k0: int, planes: int, overlap: int = 3) -> np.ndarray:
    """Planes k0 - overlap .. k0 + planes + overlap - 1 of a z-periodic array
    [..., nz, ny, nx], taken through the periodic wrap."""
    nz = arr.shape[-3]
    ks = np.arange(k0 - overlap, k0 + planes + overlap) % nz
    return np.ascontiguousarray(np.take(arr, ks, axis=-3))


def z_slab(prob: Problem, k0: int, planes: int, overlap: int = 3) -> Problem:
    """One GPU's share of a z-periodic problem split into z-slabs: the owned
    planes k0 .. k0+planes-1 plus ``overlap`` planes on either side taken
    through the periodic wrap, with OUTFLOW z faces standing in for the halo.
    One step of the method reads U^n at most 3 cells away along an axis, so
    with overlap >= 3 the owned planes advance exactly as in the whole grid
    (given the same dt); afterwards the overlap planes are stale and would be
    refreshed from the neighbours."""
    assert prob.bc[4] == PERIODIC and prob.bc[5] == PERIODIC
    nx, ny, nz = prob.shape
    shape = (nx, ny, planes + 2 * overlap)
    bc = prob.bc[:4] + (OUTFLOW, OUTFLOW)
    psi = None if prob.psi is None else z_cut(prob.psi, k0, planes, overlap)
    origin = (prob.origin[0], prob.origin[1], prob.origin[2] + (k0 - overlap) * prob.h)
    return Problem(prob.name + "_slab", shape, prob.h, prob.gamma, prob.cfl, bc,
                   z_cut(prob.prim, k0, planes, overlap), psi, inflow=dict(prob.inflow),
                   origin=origin, rho_vac=prob.rho_vac, nu=prob.nu)


# --------------------------------------------------------------------------
# point blast
# --------------------------------------------------------------------------
def sedov(shape=(64, 64, 64), gamma=1.4, energy=1.0, rho0=1.0, p0=1e-5, cfl=0.4,
          steps=100) -> Problem:
    """Energy ``energy`` deposited uniformly in the 2x2x2 cells around the box centre
    (h = 1/nx; all extents even), ambient rho0, p0, u = 0, outflow on every face."""
    nx, ny, nz = shape
    assert nx % 2 == 0 and ny % 2 == 0 and nz % 2 == 0
    h = 1.0 / nx
    prim = _prim(shape)
    prim[0] = rho0
    prim[4] = p0
    e_cell = energy / (8.0 * h ** 3)  # energy per unit volume added to each of the 8 cells
    sl = (slice(nz // 2 - 1, nz // 2 + 1), slice(ny // 2 - 1, ny // 2 + 1),
          slice(nx // 2 - 1, nx // 2 + 1))
    prim[4][sl] = p0 + (gamma - 1.0) * e_cell
    return Problem("sedov", shape, h, gamma, cfl, (OUTFLOW,) * 6, prim, steps=steps)


# --------------------------------------------------------------------------
# smooth flows and invariants
# --------------------------------------------------------------------------
def acoustic_wave(n=128, eps=1e-6, rho0=1.0, p0=1.0, u0=0.5, gamma=1.4, transverse=4,
                  t_end=None, cfl=0.4) -> Problem:
    """Right-going acoustic simple wave on a background flow u0 along x (periodic):
    rho' = eps rho0 s, u' = eps c s, p' = eps gamma p0 s, s = sin(2 pi x)."""
    shape = (n, transverse, transverse)
    h = 1.0 / n
    c = math.sqrt(gamma * p0 / rho0)
    x, _, _ = centres(shape, h)
    s = np.broadcast_to(np.sin(2.0 * math.pi * x), (transverse, transverse, n))
    prim = _prim(shape)
    prim[0] = rho0 * (1.0 + eps * s)
    prim[1] = u0 + eps * c * s
    prim[4] = p0 * (1.0 + eps * gamma * s)
    if t_end is None:
        t_end = 1.0 / (u0 + c)
    return Problem("acoustic", shape, h, gamma, cfl, (PERIODIC,) * 6, prim, t_end=t_end)


def advected_density(n=128, amp=0.2, u=(1.0, 0.0, 0.0), p0=1.0, gamma=1.4, transverse=4,
                     t_end=1.0, cfl=0.4) -> Problem:
    """rho = 1 + amp sin(2 pi x) carried by a uniform velocity at uniform pressure."""
    shape = (n, transverse, transverse)
    h = 1.0 / n
    x, _, _ = centres(shape, h)
    prim = _prim(shape)
    prim[0] = np.broadcast_to(1.0 + amp * np.sin(2.0 * math.pi * x), prim.shape[1:])
    for d in range(3):
        prim[1 + d] = u[d]
    prim[4] = p0
    return Problem("advected_density", shape, h, gamma, cfl, (PERIODIC,) * 6, prim, t_end=t_end)


def jeans_wave(n=64, G=1.5, delta=1e-5, rho0=1.0, gamma=5.0 / 3.0, axis=0, transverse=4,
               t_end=0.5, cfl=0.4) -> Problem:
    """A self-gravitating gas at rest with a standing density wave of one period on
    the unit box along `axis` (periodic): rho = rho0 (1 + delta s), p = p0 + c^2
    rho0 delta s, s = cos(2 pi x_axis), p0 = rho0 / gamma (sound speed c = 1)."""
    shape = [transverse] * 3
    shape[axis] = n
    shape = tuple(shape)
    h = 1.0 / n
    xs = centres(shape, h)
    s = np.broadcast_to(np.cos(2.0 * math.pi * xs[axis]), (shape[2], shape[1], shape[0]))
    p0 = rho0 / gamma
    prim = _prim(shape)
    prim[0] = rho0 * (1.0 + delta * s)
    prim[4] = p0 + rho0 * delta * s
    return Problem("jeans_wave", shape, h, gamma, cfl, (PERIODIC,) * 6, prim, t_end=t_end,
                   grav=G)


def uniform_flow(shape=(8, 8, 8), u=(0.3, -0.2, 0.1), rho=1.0, p=1.0, gamma=1.4) -> Problem:
    h = 1.0 / shape[0]
    prim = _prim(shape)
    prim[0] = rho
    for d in range(3):
        prim[1 + d] = u[d]
    prim[4] = p
    return Problem("uniform", tuple(shape), h, gamma, 0.4, (PERIODIC,) * 6, prim)


def random_state(shape=(32, 32, 32), seed=1, gamma=1.4, potential=False, bc=None) -> Problem:
    """Seeded non-smooth state: rho, p in [0.5, 1.5], u in [-0.5, 0.5]^3 (periodic)."""
    nx, ny, nz = shape
    N = nx * ny * nz
    idx = np.arange(5 * N, dtype=np.uint64)
    r = uniform01(seed, idx).reshape(5, nz, ny, nx)
    prim = np.empty((5, nz, ny, nx))
    prim[0] = 0.5 + r[0]
    prim[1:4] = r[1:4] - 0.5
    prim[4] = 0.5 + r[4]
    h = 1.0 / nx
    psi = None
    if potential:
        psi = 0.3 * (uniform01(seed + 1, np.arange(N, dtype=np.uint64)).reshape(nz, ny, nx) - 0.5)
    return Problem("random", tuple(shape), h, gamma, 0.4, tuple(bc or (PERIODIC,) * 6), prim, psi)


def smooth_state(shape=(16, 12, 10), seed=0, gamma=1.4, bc=None, potential=True) -> Problem:
    """Seeded smooth state: every primitive variable is a constant plus one
    low-wavenumber sine per axis with seeded phases (rho, p in [0.7, 1.3],
    |u| <= 0.3); psi likewise (amplitude 0.2) when ``potential``."""
    nx, ny, nz = shape
    h = 1.0 / nx
    x, y, z = centres(shape, h)
    ph = uniform01(seed, np.arange(24, dtype=np.uint64)) * 2 * math.pi

    def wave(q, amp):
        return amp * (np.sin(2 * math.pi * x + ph[3 * q]) * np.cos(2 * math.pi * y + ph[3 * q + 1])
                      * np.cos(2 * math.pi * z + ph[3 * q + 2]))
    prim = _prim(shape)
    prim[0] = 1.0 + wave(0, 0.3)
    prim[1] = wave(1, 0.3)
    prim[2] = wave(2, 0.2)
    prim[3] = wave(3, 0.2)
    prim[4] = 1.0 + wave(4, 0.3)
    psi = wave(5, 0.2) if potential else None
    return Problem("smooth", tuple(shape), h, gamma, 0.4, tuple(bc or (PERIODIC,) * 6), prim, psi)


# --------------------------------------------------------------------------
# batched and serving workloads
# --------------------------------------------------------------------------
BATCH_EDGES = (32, 48, 64, 96)


def batch_shape(master_seed: int, k: int):
    """(nx, ny, nz) and the kind ('sedov' or 'sod') of instance k of the batched
    workload, without building it."""
    r = splitmix64(master_seed, np.arange(4 * k, 4 * k + 4, dtype=np.uint64))
    shape = tuple(BATCH_EDGES[int(r[a] % np.uint64(4))] for a in range(3))
    return shape, ("sedov" if int(r[3]) & 1 else "sod")


def batch_instance(master_seed: int, k: int, gamma=1.4, steps=100) -> Problem:
    """Instance k of the batched workload: edges uniform in {32, 48, 64, 96} per axis,
    a Sod tube along x or a Sedov blast chosen by one hash bit (h = 1/nx, psi = 0)."""
    (nx, ny, nz), kind = batch_shape(master_seed, k)
    if kind == "sedov":
        p = sedov((nx, ny, nz), gamma=gamma, steps=steps)
    else:
        p = riemann_tube(nx, gamma=gamma)
        # a tube with independent transverse extents
        shape = (nx, ny, nz)
        h = 1.0 / nx
        prim = _prim(shape)
        x, _, _ = centres(shape, h)
        L = np.broadcast_to(x < 0.5, prim.shape[1:])
        prim[0] = np.where(L, 1.0, 0.125)
        prim[4] = np.where(L, 1.0, 0.1)
        p = Problem("sod", shape, h, gamma, 0.4, (OUTFLOW, OUTFLOW) + (PERIODIC,) * 4, prim,
                    steps=steps)
    p.steps = steps
    p.t_end = math.inf
    return p


SERVE_EDGES = (64, 96, 128, 160, 192, 224, 256)
SERVE_TYPES = ("sod", "sedov", "well", "cloud")


@dataclass
class Request:
    rid: int
    arrival: float          # seconds after the start of the stream
    edge: int
    kind: str
    dtype: str              # "f32" or "f64"
    steps: int


def serve_requests(count=500, rate=10.0, seed=0, edges=SERVE_EDGES, max_steps=500,
                   min_steps=50):
    """A Poisson stream: exponential inter-arrival times at ``rate`` per second."""
    out = []
    t = 0.0
    for k in range(count):
        r = uniform01(seed, np.arange(5 * k, 5 * k + 5, dtype=np.uint64))
        t += -math.log(1.0 - r[0]) / rate
        edge = edges[min(int(r[1] * len(edges)), len(edges) - 1)]
        kind = SERVE_TYPES[min(int(r[2] * 4), 3)]
        dtype = "f32" if r[3] < 0.5 else "f64"
        steps = min_steps + min(int(r[4] * (max_steps - min_steps + 1)), max_steps - min_steps)
        out.append(Request(k, t, edge, kind, dtype, steps))
    return out


def serve_problem(req: Request) -> Problem:
    n = req.edge
    if req.kind == "sod":
        p = riemann_tube(n, transverse=n)
        p.t_end = math.inf
    elif req.kind == "sedov":
        p = sedov((n, n, n))
    elif req.kind == "well":
        p = well_flow(n)
    else:
        p = cloud(n, seed=req.rid)
    p.steps = req.steps
    return p
