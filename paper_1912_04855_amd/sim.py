"""Python face of the library: ``Sim`` (one simulation) and helpers.

Every step of the method runs in the HIP kernels behind the C ABI; this module
only marshals arguments.  Device memory can be lent by PyTorch (``torch=True``:
a uint8 CUDA tensor sized by ``csph_required_bytes``) and work can be issued on
torch's current stream, so the library interoperates with torch code.
"""
import ctypes as C
import math

import numpy as np

from . import _lib
from ._lib import CONSERVED, F32, F64, PRIMITIVE, check


def _dtype_code(dtype):
    if dtype in ("f32", "float32", F32, np.float32):
        return F32
    if dtype in ("f64", "float64", F64, np.float64):
        return F64
    raise ValueError(f"dtype must be f32 or f64, got {dtype!r}")


def make_desc(shape, h, gamma=1.4, cfl=0.4, rho_vac=1e-10, dtype="f64", origin=(0.0, 0.0, 0.0)):
    d = _lib.GridDesc()
    d.nx, d.ny, d.nz = (int(v) for v in shape)
    d.h = float(h)
    for a in range(3):
        d.origin[a] = float(origin[a])
    d.gamma, d.cfl, d.rho_vac = float(gamma), float(cfl), float(rho_vac)
    d.dtype = _dtype_code(dtype)
    return d


def required_bytes(shape, h=1.0, dtype="f64", **kw) -> int:
    d = make_desc(shape, h, dtype=dtype, **kw)
    return int(_lib.load().csph_required_bytes(C.byref(d)))


def _ptr(a: np.ndarray):
    return C.c_void_p(a.ctypes.data)


class Sim:
    """One CSPH-TVD simulation on the current HIP device.

    shape = (nx, ny, nz).  Arrays are numpy float64, [5, nz, ny, nx] for states.
    ``torch=True`` allocates the device buffer as a torch tensor and issues work on
    torch's current stream."""

    def __init__(self, shape, h, gamma=1.4, cfl=0.4, rho_vac=1e-10, dtype="f64",
                 origin=(0.0, 0.0, 0.0), torch=False, stream=None, static=False):
        L = _lib.load()
        self.shape = (int(shape[2]), int(shape[1]), int(shape[0]))  # (nz, ny, nx)
        self.dtype = _dtype_code(dtype)
        self.desc = make_desc(shape, h, gamma, cfl, rho_vac, dtype, origin)
        self.gamma = gamma
        self._buf = None
        self._h = C.c_void_p()
        if static:
            # the library's static device array (csph_create_static): no allocation
            check(L.csph_create_static(C.byref(self.desc), C.c_void_p(stream or 0), C.byref(self._h)),
                  "csph_create_static")
        elif torch:
            import torch as _t
            nbytes = int(L.csph_required_bytes(C.byref(self.desc)))
            if nbytes == 0:
                raise ValueError("invalid grid description")
            # 256-byte alignment: torch's caching allocator returns 512-byte aligned blocks
            self._buf = _t.empty(nbytes, dtype=_t.uint8, device="cuda")
            if stream is None:
                stream = _t.cuda.current_stream().cuda_stream
            check(L.csph_create_in(C.byref(self.desc), C.c_void_p(stream),
                                   C.c_void_p(self._buf.data_ptr()), nbytes, C.byref(self._h)),
                  "csph_create_in")
        else:
            check(L.csph_create(C.byref(self.desc), C.c_void_p(stream or 0), C.byref(self._h)),
                  "csph_create")

    # ------------------------------------------------------------------ lifetime
    def close(self):
        if self._h:
            # refused (and nothing freed) while the sim is a batch member
            check(_lib.load().csph_destroy(self._h), "csph_destroy")
            self._h = C.c_void_p()
        self._buf = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def handle(self):
        return self._h

    # ------------------------------------------------------------------ setup
    def set_boundary(self, face, kind, inflow=None):
        arr = None
        if inflow is not None:
            arr = np.ascontiguousarray(inflow, dtype=np.float64)
            assert arr.shape == (5,)
        check(_lib.load().csph_set_boundary(self._h, int(face), int(kind),
                                            _ptr(arr) if arr is not None else None),
              "csph_set_boundary")

    def set_state(self, arr, vars=PRIMITIVE):
        a = np.ascontiguousarray(arr, dtype=np.float64)
        assert a.shape == (5,) + self.shape, a.shape
        check(_lib.load().csph_set_state(self._h, int(vars), _ptr(a)), "csph_set_state")

    def set_primitive(self, W):
        self.set_state(W, PRIMITIVE)

    def set_conserved(self, U):
        self.set_state(U, CONSERVED)

    def set_potential(self, psi):
        if psi is None:
            check(_lib.load().csph_set_potential(self._h, None), "csph_set_potential")
            return
        a = np.ascontiguousarray(psi, dtype=np.float64)
        assert a.shape == self.shape
        check(_lib.load().csph_set_potential(self._h, _ptr(a)), "csph_set_potential")

    # ------------------------------------------------------------------ stepping
    def step(self, dt_max=0.0, sync=True) -> float:
        dt = C.c_double()
        check(_lib.load().csph_step(self._h, float(dt_max), C.byref(dt) if sync else None),
              "csph_step")
        return dt.value

    def advance(self, t_end=math.inf, max_steps=2**62) -> int:
        n = C.c_int64()
        check(_lib.load().csph_advance(self._h, float(t_end), int(max_steps), C.byref(n)),
              "csph_advance")
        return n.value

    # ------------------------------------------------------------------ read back
    def get_state(self, vars=CONSERVED) -> np.ndarray:
        out = np.empty((5,) + self.shape)
        check(_lib.load().csph_get_state(self._h, int(vars), _ptr(out)), "csph_get_state")
        return out

    def conserved(self):
        return self.get_state(CONSERVED)

    def primitive(self):
        return self.get_state(PRIMITIVE)

    def time(self):
        t, n = C.c_double(), C.c_int64()
        check(_lib.load().csph_get_time(self._h, C.byref(t), C.byref(n)), "csph_get_time")
        return t.value, n.value

    def set_time(self, t, nsteps):
        check(_lib.load().csph_set_time(self._h, float(t), int(nsteps)), "csph_set_time")

    def totals(self) -> np.ndarray:
        out = np.zeros(5)
        check(_lib.load().csph_totals(self._h, _ptr(out)), "csph_totals")
        return out

    PROFILE_GROUPS = ["stage_p", "stage_c", "stage_e", "ghost_fill", "bookkeeping", "self_gravity"]

    def profile(self, on=True):
        check(_lib.load().csph_profile_enable(self._h, int(bool(on))), "csph_profile_enable")

    def profile_read(self):
        """{group: (average ms per launch, launches)} of the steps since profile(True)."""
        k = len(self.PROFILE_GROUPS)
        ms = np.zeros(k)
        n = np.zeros(k, dtype=np.int64)
        check(_lib.load().csph_profile_read(self._h, _ptr(ms), _ptr(n), k), "csph_profile_read")
        return {g: (float(ms[q]), int(n[q])) for q, g in enumerate(self.PROFILE_GROUPS) if n[q] or q < 5}

    # ------------------------------------------------------------------ scheme
    def set_scheme(self, limiter=_lib.LIM_MINMOD, flux=_lib.FLUX_SWEPT_AV):
        """TVD limiter and face flux of the Eulerian stage (``_lib.LIM_*``, ``_lib.FLUX_*``)."""
        check(_lib.load().csph_set_scheme(self._h, int(limiter), int(flux)), "csph_set_scheme")

    def set_viscosity(self, nu):
        """Uniform kinematic viscosity of the Lagrangian stage (0: inviscid)."""
        check(_lib.load().csph_set_viscosity(self._h, float(nu)), "csph_set_viscosity")

    def fill_state(self, state, vars=PRIMITIVE):
        """Every cell set to one state (5 values), on the device."""
        st = np.ascontiguousarray(state, dtype=np.float64)
        assert st.shape == (5,)
        check(_lib.load().csph_fill_state(self._h, int(vars), _ptr(st)), "csph_fill_state")

    def set_box(self, lo, arr, vars=PRIMITIVE):
        """Write a box of the interior: lo = (i, j, k) of its first cell, arr
        [5, n_z, n_y, n_x]."""
        arr = np.ascontiguousarray(arr, dtype=np.float64)
        assert arr.ndim == 4 and arr.shape[0] == 5
        lo_ = (C.c_int32 * 3)(*[int(v) for v in lo])
        n_ = (C.c_int32 * 3)(arr.shape[3], arr.shape[2], arr.shape[1])
        check(_lib.load().csph_set_state_box(self._h, int(vars), lo_, n_, _ptr(arr)), "csph_set_state_box")

    def get_box(self, lo, n, vars=CONSERVED) -> np.ndarray:
        """Read a box of the interior: lo = (i, j, k) of its first cell, n = (n_x,
        n_y, n_z); returns [5, n_z, n_y, n_x]."""
        out = np.empty((5, int(n[2]), int(n[1]), int(n[0])))
        lo_ = (C.c_int32 * 3)(*[int(v) for v in lo])
        n_ = (C.c_int32 * 3)(*[int(v) for v in n])
        check(_lib.load().csph_get_state_box(self._h, int(vars), lo_, n_, _ptr(out)), "csph_get_state_box")
        return out

    def set_source(self, q, eps=0.0):
        """Mass source rate per cell [nz, ny, nx] (< 0: sink) and the injected gas's
        specific internal energy; None removes the sources."""
        if q is None:
            check(_lib.load().csph_set_source(self._h, None, 0.0), "csph_set_source")
            return
        q = np.ascontiguousarray(np.broadcast_to(q, self.shape), dtype=np.float64)
        check(_lib.load().csph_set_source(self._h, _ptr(q), float(eps)), "csph_set_source")

    def set_self_gravity(self, G):
        """Self-gravity with constant G (0: off): on a periodic box (all six
        faces PERIODIC) by the discrete Poisson equation, on an isolated box (no
        face PERIODIC) as the free-space potential of the cells."""
        check(_lib.load().csph_set_self_gravity(self._h, float(G)), "csph_set_self_gravity")

    def scheme(self):
        lim, flux = C.c_int32(), C.c_int32()
        check(_lib.load().csph_get_scheme(self._h, C.byref(lim), C.byref(flux)), "csph_get_scheme")
        return lim.value, flux.value

    # ------------------------------------------------------------------ tiling
    @property
    def tile_depth(self) -> tuple:
        """Tile depths of the stage P, C and E sweeps."""
        tz = (C.c_int32 * 3)()
        check(_lib.load().csph_get_tile_depths(self._h, tz), "csph_get_tile_depths")
        return tuple(int(v) for v in tz)

    @tile_depth.setter
    def tile_depth(self, tz):
        """One depth for every stage, or three (stage P, C, E)."""
        if np.ndim(tz) == 0:
            check(_lib.load().csph_set_tile_depth(self._h, int(tz)), "csph_set_tile_depth")
            return
        v = [int(x) for x in tz]
        if len(v) != 3:
            raise ValueError("tile depth: one value or three (stage P, C, E)")
        check(_lib.load().csph_set_tile_depths(self._h, (C.c_int32 * 3)(*v)), "csph_set_tile_depths")

    def autotune(self, trial_steps=3):
        """Pick each stage's fastest tile depth by timing trial steps on a copy
        of this simulation (which is not advanced).  Returns ((P, C, E) depths,
        ms per step at those depths)."""
        tz, ms = (C.c_int32 * 3)(), C.c_double()
        check(_lib.load().csph_autotune(self._h, int(trial_steps), tz, C.byref(ms)), "csph_autotune")
        return tuple(int(v) for v in tz), ms.value

    STAGE_FIELDS = ["msx", "msy", "msz", "Es", "xsx", "xsy", "xsz",
                    "mtx", "mty", "mtz", "Et", "xtx", "xty", "xtz", "phis", "psi", "psih"]

    def stage(self, name) -> np.ndarray:
        out = np.empty(self.shape)
        check(_lib.load().csph_get_stage(self._h, self.STAGE_FIELDS.index(name), _ptr(out)),
              "csph_get_stage")
        return out


def from_problem(prob, dtype="f64", torch=False, stream=None) -> Sim:
    """A Sim set up from a ``problems.Problem`` description."""
    s = Sim(prob.shape, prob.h, gamma=prob.gamma, cfl=prob.cfl, rho_vac=prob.rho_vac,
            dtype=dtype, origin=prob.origin, torch=torch, stream=stream)
    for f in range(6):
        s.set_boundary(f, prob.bc[f], prob.inflow.get(f) if prob.bc[f] == _lib.INFLOW else None)
    s.set_potential(prob.psi)
    s.set_primitive(prob.prim)
    if prob.nu:
        s.set_viscosity(prob.nu)
    if prob.grav:
        s.set_self_gravity(prob.grav)
    if prob.src is not None:
        s.set_source(prob.src, prob.eps_src)
    return s


class Batch:
    """Simulations of one dtype advanced together: one launch per stage for all
    members, k steps captured in a HIP graph and replayed.  Members keep their own
    dt, t and step target; the batch references sims, it does not own them."""

    def __init__(self, dtype="f32", budget_bytes=0, stream=None):
        self.dtype = _dtype_code(dtype)
        self._h = C.c_void_p()
        check(_lib.load().csph_batch_create(self.dtype, C.c_void_p(stream or 0),
                                            int(budget_bytes), C.byref(self._h)),
              "csph_batch_create")
        self.members = {}

    def add(self, sim: Sim, steps: int, t_end=math.inf) -> int:
        slot = C.c_int32()
        check(_lib.load().csph_batch_add(self._h, sim.handle, int(steps), float(t_end),
                                         C.byref(slot)), "csph_batch_add")
        self.members[slot.value] = sim
        return slot.value

    def try_add(self, sim: Sim, steps: int, t_end=math.inf):
        """add(), or None when the device-memory budget is exhausted."""
        try:
            return self.add(sim, steps, t_end)
        except _lib.CsphError as e:
            if e.code == _lib.ERR_BUDGET:
                return None
            raise

    def advance(self, k: int, sync=False) -> int:
        n = C.c_int32()
        check(_lib.load().csph_batch_advance(self._h, int(k), C.byref(n) if sync else None),
              "csph_batch_advance")
        return n.value

    def autotune(self, trial_steps=3):
        """Pick the fastest tile depth for every member by timing trial steps of
        the whole batch; members are restored afterwards.  Returns (depth, ms per
        batch step)."""
        tz, ms = C.c_int32(), C.c_double()
        check(_lib.load().csph_batch_autotune(self._h, int(trial_steps), C.byref(tz),
                                              C.byref(ms)), "csph_batch_autotune")
        return tz.value, ms.value

    def poll(self):
        cap = max(1, len(self.members))
        out = np.zeros(cap, dtype=np.int32)
        n = C.c_int32()
        check(_lib.load().csph_batch_poll(self._h, _ptr(out), cap, C.byref(n)), "csph_batch_poll")
        return [int(v) for v in out[:min(n.value, cap)]]

    def remove(self, slot: int) -> Sim:
        check(_lib.load().csph_batch_remove(self._h, int(slot)), "csph_batch_remove")
        return self.members.pop(slot)

    def close(self):
        if self._h:
            _lib.load().csph_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
