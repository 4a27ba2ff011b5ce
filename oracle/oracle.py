"""ctypes wrapper of the FP64 CPU oracle (``btdf_oracle.c``).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's
CPU-baseline leg use this module. Nothing here is shared with the HIP
library; the two meet only through the seeded inputs of ``btdf_workloads``.
"""
import ctypes
import os

import numpy as np

from . import build as _build

PERIODIC, VELOCITY_INLET, ZERO_GRADIENT_OUTLET, BOUNCEBACK_WALL = 0, 1, 2, 3
LINEAR2, ROMA3, PESKIN4, COS4 = 2, 3, 4, 5

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)


def _ptr(a):
    return a.ctypes.data_as(_dp)


def lib():
    """Load the oracle library, building it with gcc if it is not there."""
    global _lib
    if _lib is None:
        path = os.environ.get("ORACLE_LIBRARY")  # another build (the sanitizer build of the tests)
        if not path:
            path = _build.LIB
            if not os.path.exists(path):
                _build.build()
        L = ctypes.CDLL(path)
        L.oracle_create.restype = ctypes.c_void_p
        L.oracle_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                    ctypes.c_double, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                    ctypes.c_double]
        L.oracle_destroy.argtypes = [ctypes.c_void_p]
        L.oracle_add_body.restype = ctypes.c_int
        L.oracle_add_body.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp, _dp,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.oracle_set_marker_velocity.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
        L.oracle_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        L.oracle_init_equilibrium.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.oracle_get_populations.argtypes = [ctypes.c_void_p, _dp]
        L.oracle_set_populations.argtypes = [ctypes.c_void_p, _dp]
        L.oracle_get_macroscopic.argtypes = [ctypes.c_void_p, _dp, _dp, _dp]
        L.oracle_marker_data.argtypes = [ctypes.c_void_p, _dp, _dp, _dp, _dp, _dp]
        L.oracle_marker_corrected_velocity.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.oracle_get_force_field.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.oracle_body_forces.argtypes = [ctypes.c_void_p, _dp]
        L.oracle_unstable.restype = ctypes.c_int
        L.oracle_unstable.argtypes = [ctypes.c_void_p]
        L.oracle_steps.restype = ctypes.c_long
        L.oracle_steps.argtypes = [ctypes.c_void_p]
        L.oracle_num_markers.restype = ctypes.c_int
        L.oracle_num_markers.argtypes = [ctypes.c_void_p]
        L.oracle_num_bodies.restype = ctypes.c_int
        L.oracle_num_bodies.argtypes = [ctypes.c_void_p]
        L.oracle_delta.restype = ctypes.c_double
        L.oracle_delta.argtypes = [ctypes.c_int, ctypes.c_double]
        L.oracle_delta_halfwidth.restype = ctypes.c_double
        L.oracle_delta_halfwidth.argtypes = [ctypes.c_int]
        L.oracle_set_forcing_passes.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.oracle_set_forcing_method.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.oracle_set_body_motion.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_double]
        L.oracle_body_state.argtypes = [ctypes.c_void_p, ctypes.c_int, _dp]
        L.oracle_get_marker_positions.argtypes = [ctypes.c_void_p, _dp]
        L.oracle_delta_deriv.restype = ctypes.c_double
        L.oracle_delta_deriv.argtypes = [ctypes.c_int, ctypes.c_double]
        L.oracle_adjoint.restype = ctypes.c_int
        L.oracle_adjoint.argtypes = [ctypes.c_void_p, ctypes.c_long, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def num_threads():
    """Threads the oracle's parallel loops use."""
    return int(lib().oracle_num_threads())


def set_num_threads(n):
    """Threads of the oracle's parallel loops from now on (results do not depend on it)."""
    lib().oracle_set_num_threads(int(n))


def delta(kind, r):
    """Regularised delta function phi(r) of Section 4.3 (vectorised over r)."""
    L = lib()
    r = np.asarray(r, dtype=np.float64)
    return np.vectorize(lambda v: L.oracle_delta(int(kind), float(v)))(r).astype(np.float64)


def delta_deriv(kind, r):
    """phi'(r) of the delta functions (vectorised over r)."""
    L = lib()
    r = np.asarray(r, dtype=np.float64)
    return np.vectorize(lambda v: L.oracle_delta_deriv(int(kind), float(v)))(r).astype(np.float64)


class OracleSim:
    """One FP64 BTDF-IB-LBM simulation on the host (Algorithm 1, NF = 1)."""

    def __init__(self, nx, ny, bc, tau, kind, thickening, G=(0.0, 0.0),
                 inflow=(0.0, 0.0), init=(1.0, 0.0, 0.0)):
        self.nx, self.ny = int(nx), int(ny)
        self.kind = int(kind)
        bc_arr = (ctypes.c_int * 4)(*[int(b) for b in bc])
        self._h = lib().oracle_create(self.nx, self.ny, bc_arr, float(tau), self.kind,
                                      float(thickening), float(G[0]), float(G[1]),
                                      float(inflow[0]), float(inflow[1]),
                                      float(init[0]), float(init[1]), float(init[2]))
        if not self._h:
            raise MemoryError("oracle_create failed")
        self.body_sizes = []

    def close(self):
        if self._h:
            lib().oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def add_body(self, xy, uv=None, cx=0.0, cy=0.0, ds=None):
        xy = np.ascontiguousarray(xy, dtype=np.float64).reshape(-1, 2)
        n = xy.shape[0]
        if ds is None:
            # polygon perimeter / n
            d = np.roll(xy, -1, axis=0) - xy
            ds = float(np.sum(np.hypot(d[:, 0], d[:, 1])) / n)
        if uv is None:
            uvp = ctypes.cast(None, _dp)
        else:
            uv = np.ascontiguousarray(uv, dtype=np.float64).reshape(n, 2)
            uvp = _ptr(uv)
        b = lib().oracle_add_body(self._h, n, _ptr(xy), uvp, float(cx), float(cy), float(ds))
        if b < 0:
            raise MemoryError("oracle_add_body failed")
        self.body_sizes.append(n)
        return b

    def set_forcing_passes(self, nf):
        """Forcing passes per step (Algorithm 1 step 3; eqs 29-31 for nf > 1)."""
        lib().oracle_set_forcing_passes(self._h, int(nf))

    def set_body_motion(self, b, vx, vy, omega):
        """Rigid motion of body b from now on (eq 4 for a rigid body)."""
        lib().oracle_set_body_motion(self._h, int(b), float(vx), float(vy), float(omega))

    def body_state(self, b):
        out = np.empty(6)
        lib().oracle_body_state(self._h, int(b), _ptr(out))
        return out

    def marker_positions(self):
        out = np.empty((lib().oracle_num_markers(self._h), 2))
        lib().oracle_get_marker_positions(self._h, _ptr(out))
        return out

    DIRECT, IMPLICIT, RKPM = 0, 1, 2

    def set_forcing_method(self, method):
        """DIRECT (eq 20), IMPLICIT (eq 17; = IVC, eqs 32-35) or RKPM (eq 36 / B54)."""
        lib().oracle_set_forcing_method(self._h, int(method))

    def set_marker_velocity(self, b, uv):
        uv = np.ascontiguousarray(uv, dtype=np.float64).reshape(-1, 2)
        lib().oracle_set_marker_velocity(self._h, int(b), _ptr(uv))

    def step(self, n=1):
        lib().oracle_step(self._h, int(n))

    def init_equilibrium(self, ux, uy, rho=None):
        ux = np.ascontiguousarray(ux, dtype=np.float64).reshape(self.ny, self.nx)
        uy = np.ascontiguousarray(uy, dtype=np.float64).reshape(self.ny, self.nx)
        rp = ctypes.cast(None, _dp)
        if rho is not None:
            rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(self.ny, self.nx)
            rp = _ptr(rho)
        lib().oracle_init_equilibrium(self._h, rp, _ptr(ux), _ptr(uy))

    def populations(self):
        out = np.empty((9, self.ny, self.nx), dtype=np.float64)
        lib().oracle_get_populations(self._h, _ptr(out))
        return out

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64).reshape(9, self.ny, self.nx)
        lib().oracle_set_populations(self._h, _ptr(f))

    def macroscopic(self):
        r = np.empty((self.ny, self.nx))
        u = np.empty((self.ny, self.nx))
        v = np.empty((self.ny, self.nx))
        lib().oracle_get_macroscopic(self._h, _ptr(r), _ptr(u), _ptr(v))
        return r, u, v

    def marker_data(self):
        m = lib().oracle_num_markers(self._h)
        arrs = [np.empty(m) for _ in range(5)]
        lib().oracle_marker_data(self._h, *[_ptr(a) for a in arrs])
        return dict(zip(["rho", "ux", "uy", "Fx", "Fy"], arrs))

    def marker_corrected_velocity(self):
        m = lib().oracle_num_markers(self._h)
        u, v = np.empty(m), np.empty(m)
        lib().oracle_marker_corrected_velocity(self._h, _ptr(u), _ptr(v))
        return u, v

    def force_field(self):
        fx = np.empty((self.ny, self.nx))
        fy = np.empty((self.ny, self.nx))
        lib().oracle_get_force_field(self._h, _ptr(fx), _ptr(fy))
        return fx, fy

    def forces(self):
        nb = lib().oracle_num_bodies(self._h)
        out = np.empty((nb, 3))
        if nb:
            lib().oracle_body_forces(self._h, _ptr(out))
        return out

    @property
    def unstable(self):
        return lib().oracle_unstable(self._h)

    @property
    def steps(self):
        return lib().oracle_steps(self._h)

    def adjoint(self, n, hist_bar):
        """Run n steps (the state advances by n), then the reverse sweep for
        J = sum(hist_bar * history of these n steps); hist_bar is [n][nb][3].
        Returns dJ/d(initial populations, inflow, body force, marker
        positions, marker velocities, body centres)."""
        nb = lib().oracle_num_bodies(self._h)
        nm = lib().oracle_num_markers(self._h)
        hb = np.ascontiguousarray(hist_bar, dtype=np.float64).reshape(int(n), nb, 3)
        if hb.size == 0:
            hb = np.zeros(1)
        out = dict(populations=np.empty((9, self.ny, self.nx)), inflow=np.empty(2), body_force=np.empty(2),
                   xy=np.empty((max(nm, 1), 2)), uv=np.empty((max(nm, 1), 2)), centres=np.empty((max(nb, 1), 2)))
        rc = lib().oracle_adjoint(self._h, int(n), _ptr(hb), _ptr(out["populations"]), _ptr(out["inflow"]),
                                  _ptr(out["body_force"]), _ptr(out["xy"]), _ptr(out["uv"]), _ptr(out["centres"]))
        if rc != 0:
            raise RuntimeError("oracle_adjoint failed (memory or an unstable forward run)")
        out["xy"], out["uv"], out["centres"] = out["xy"][:nm], out["uv"][:nm], out["centres"][:nb]
        return out
