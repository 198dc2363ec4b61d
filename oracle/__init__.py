"""CPU FP64 oracle of the CSPH-TVD step -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it.

``OracleSim`` wraps the C oracle (``csph_oracle.c``) through ctypes; arrays are
numpy float64, structure of arrays, x fastest: state ``[5, nz, ny, nx]``.
"""
import ctypes as C
import math

import numpy as np

from .build import ensure_built

PERIODIC, OUTFLOW, INFLOW, REFLECT = 0, 1, 2, 3
POS_LAGRANGE, POS_DISPLACED, POS_LATTICE = 0, 1, 2
BASE_POST, BASE_MID = 0, 1
LIM_MINMOD, LIM_MC, LIM_VANLEER, LIM_SUPERBEE = 0, 1, 2, 3
FLUX_SWEPT, FLUX_LF, FLUX_SWEPT_AV = 0, 1, 2
FACE_FOOT, FACE_PARTICLE = 0, 1

FIELDS = ["msx", "msy", "msz", "Es", "xsx", "xsy", "xsz",
          "mtx", "mty", "mtz", "Et", "xtx", "xty", "xtz", "psis", "vol", "phis", "psi",
          "psih"]

ERRORS = {0: "ok", 1: "bad argument", 2: "out of memory", 5: "non-finite value",
          6: "negative density", 7: "no signal speed (need dt_max)"}


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("h", C.c_double), ("origin", C.c_double * 3), ("gamma", C.c_double),
                ("cfl", C.c_double), ("rho_vac", C.c_double), ("bc", C.c_int32 * 6),
                ("inflow", (C.c_double * 5) * 6), ("pos_mode", C.c_int32),
                ("base_mode", C.c_int32), ("limiter", C.c_int32), ("flux", C.c_int32),
                ("face_mode", C.c_int32), ("nu", C.c_double), ("grav", C.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(ensure_built())
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        vp = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(_Params), C.POINTER(vp)]
        L.orc_destroy.argtypes = [vp]
        L.orc_destroy.restype = None
        L.orc_set_conserved.argtypes = [vp, dp]
        L.orc_set_primitive.argtypes = [vp, dp]
        L.orc_set_potential.argtypes = [vp, vp]
        L.orc_get_conserved.argtypes = [vp, dp]
        L.orc_get_field.argtypes = [vp, C.c_int, dp]
        L.orc_step.argtypes = [vp, C.c_double, C.c_double, C.POINTER(C.c_double)]
        L.orc_advance.argtypes = [vp, C.c_double, C.c_int64, C.POINTER(C.c_int64)]
        L.orc_get_time.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
        L.orc_get_time.restype = None
        L.orc_set_time.argtypes = [vp, C.c_double, C.c_int64]
        L.orc_set_time.restype = None
        L.orc_totals.argtypes = [vp, dp]
        L.orc_totals.restype = None
        L.orc_cfl_dt.argtypes = [vp]
        L.orc_cfl_dt.restype = C.c_double
        L.orc_kappa.argtypes = []
        L.orc_kappa.restype = C.c_double
        L.orc_kernel_grad.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, dp]
        L.orc_kernel_grad.restype = None
        L.orc_limiter.argtypes = [C.c_int, C.c_double, C.c_double]
        L.orc_limiter.restype = C.c_double
        L.orc_lattice_gradient.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_double, dp, dp]
        L.orc_interp_psi.argtypes = [vp, dp, dp]
        L.orc_self_potential.argtypes = [vp, dp, dp]
        L.orc_self_potential_at.argtypes = [vp, dp, C.POINTER(C.c_int32), C.c_int64, dp]
        L.orc_set_source.argtypes = [vp, vp, C.c_double]
        L.orc_fill_ghosts_padded.argtypes = [vp, dp, C.c_int, C.c_double]
        _lib = L
    return _lib


class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"oracle {where}: {ERRORS.get(code, code)}")
        self.code = code


def _check(code, where):
    if code != 0:
        raise OracleError(code, where)


def kappa() -> float:
    return lib().orc_kappa()


def kernel_grad(d, h) -> np.ndarray:
    out = np.zeros(3)
    lib().orc_kernel_grad(float(d[0]), float(d[1]), float(d[2]), float(h), out)
    return out


def limiter(kind, a, b) -> float:
    return lib().orc_limiter(int(kind), float(a), float(b))


def lattice_gradient(f: np.ndarray, h: float) -> np.ndarray:
    """(1/h) sum_o w_|o| (f_{i+o} - f_{i-o}) o on a periodic grid; f is [nz, ny, nx]."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    nz, ny, nx = f.shape
    out = np.zeros((3, nz, ny, nx))
    _check(lib().orc_lattice_gradient(nx, ny, nz, float(h), f, out), "lattice_gradient")
    return out


class OracleSim:
    """One CSPH-TVD simulation on the CPU (FP64, single thread)."""

    def __init__(self, shape, h, gamma=1.4, cfl=0.4, rho_vac=1e-10, bc=(PERIODIC,) * 6,
                 inflow=None, origin=(0.0, 0.0, 0.0), pos_mode=POS_LAGRANGE,
                 base_mode=BASE_POST, limiter=LIM_MINMOD, flux=FLUX_SWEPT_AV,
                 face_mode=FACE_FOOT, nu=0.0, grav=0.0):
        nx, ny, nz = shape
        p = _Params()
        p.nx, p.ny, p.nz = nx, ny, nz
        p.h = h
        for a in range(3):
            p.origin[a] = origin[a]
        p.gamma, p.cfl, p.rho_vac = gamma, cfl, rho_vac
        for f in range(6):
            p.bc[f] = bc[f]
            st = (inflow or {}).get(f, (0, 0, 0, 0, 0)) if isinstance(inflow, dict) else \
                (inflow[f] if inflow is not None else (0, 0, 0, 0, 0))
            for v in range(5):
                p.inflow[f][v] = st[v]
        p.pos_mode, p.base_mode, p.limiter, p.flux = pos_mode, base_mode, limiter, flux
        p.face_mode = face_mode
        p.nu = nu
        p.grav = grav
        self.params = p
        self.shape = (nz, ny, nx)
        self.h = h
        self.gamma = gamma
        self._h = C.c_void_p()
        _check(lib().orc_create(C.byref(p), C.byref(self._h)), "create")

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_conserved(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        assert U.shape == (5,) + self.shape
        _check(lib().orc_set_conserved(self._h, U), "set_conserved")

    def set_primitive(self, W):
        W = np.ascontiguousarray(W, dtype=np.float64)
        assert W.shape == (5,) + self.shape
        _check(lib().orc_set_primitive(self._h, W), "set_primitive")

    def set_potential(self, psi):
        if psi is None:
            _check(lib().orc_set_potential(self._h, None), "set_potential")
            return
        psi = np.ascontiguousarray(psi, dtype=np.float64)
        assert psi.shape == self.shape
        self._psi_keep = psi
        _check(lib().orc_set_potential(self._h, psi.ctypes.data), "set_potential")

    def conserved(self) -> np.ndarray:
        out = np.empty((5,) + self.shape)
        _check(lib().orc_get_conserved(self._h, out), "get_conserved")
        return out

    def primitive(self) -> np.ndarray:
        U = self.conserved()
        rho = U[0]
        with np.errstate(divide="ignore", invalid="ignore"):
            vac = rho <= self.params.rho_vac
            u = np.where(vac, 0.0, U[1:4] / np.where(vac, 1.0, rho))
        p = (self.gamma - 1.0) * (U[4] - 0.5 * np.sum(U[1:4] * u, axis=0))
        return np.concatenate([rho[None], u, np.maximum(p, 0.0)[None]])

    def field(self, name) -> np.ndarray:
        out = np.empty(self.shape)
        _check(lib().orc_get_field(self._h, FIELDS.index(name), out), "get_field")
        return out

    def step(self, dt_max=0.0, t_end=math.inf) -> float:
        dt = C.c_double()
        _check(lib().orc_step(self._h, float(dt_max), float(t_end), C.byref(dt)), "step")
        return dt.value

    def advance(self, t_end=math.inf, max_steps=2**62) -> int:
        n = C.c_int64()
        _check(lib().orc_advance(self._h, float(t_end), int(max_steps), C.byref(n)), "advance")
        return n.value

    def time(self):
        t, n = C.c_double(), C.c_int64()
        lib().orc_get_time(self._h, C.byref(t), C.byref(n))
        return t.value, n.value

    def set_time(self, t, nsteps):
        lib().orc_set_time(self._h, float(t), int(nsteps))

    def totals(self) -> np.ndarray:
        out = np.zeros(5)
        lib().orc_totals(self._h, out)
        return out

    def cfl_dt(self) -> float:
        return lib().orc_cfl_dt(self._h)

    def interp_psi(self, off) -> np.ndarray:
        off = np.ascontiguousarray(off, dtype=np.float64)
        out = np.empty(self.shape)
        _check(lib().orc_interp_psi(self._h, off, out), "interp_psi")
        return out

    def set_source(self, q, eps=0.0):
        """Mass source rate per cell [nz, ny, nx] (< 0: sink), injected gas's specific
        internal energy eps; None removes the sources."""
        if q is None:
            _check(lib().orc_set_source(self._h, None, 0.0), "set_source")
            return
        q = np.ascontiguousarray(np.broadcast_to(q, self.shape), dtype=np.float64)
        _check(lib().orc_set_source(self._h, q.ctypes.data_as(C.c_void_p), float(eps)), "set_source")

    def self_potential(self, rho) -> np.ndarray:
        """The self-gravity potential the step would compute from this density."""
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        out = np.empty(self.shape)
        _check(lib().orc_self_potential(self._h, rho, out), "self_potential")
        return out

    def self_potential_at(self, rho, cells) -> np.ndarray:
        """Isolated box: the self potential of rho at the cells (i, j, k) given,
        each by its direct sum."""
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        cells = np.ascontiguousarray(cells, dtype=np.int32).reshape(-1, 3)
        out = np.empty(len(cells))
        _check(lib().orc_self_potential_at(self._h, rho, cells.ctypes.data_as(C.POINTER(C.c_int32)),
                                           len(cells), out), "self_potential_at")
        return out

    def fill_ghosts_padded(self, padded, role, dt=0.0):
        assert padded.dtype == np.float64 and padded.flags.c_contiguous
        _check(lib().orc_fill_ghosts_padded(self._h, padded, int(role), float(dt)), "fill_ghosts")
        return padded
