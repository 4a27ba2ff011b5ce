"""Python names of the C ABI (include/btdf.h), one function per C call.

Each function converts its arguments (numpy arrays, tuples, ints) into the
C types, calls the library, raises ``BtdfError`` / ``BtdfUnstable`` on a
non-zero status and converts the outputs back into numpy arrays.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import btdf_gradients, btdf_grid, check, dptr, f64, load


def btdf_create(nx, ny, tau, delta_kind, thickening, bc=(0, 0, 0, 0), inflow=(0.0, 0.0),
                body_force=(0.0, 0.0), init=(1.0, 0.0, 0.0), precision=8, history_capacity=0,
                stream=None):
    g = btdf_grid(nx=int(nx), ny=int(ny), bc_west=int(bc[0]), bc_east=int(bc[1]),
                  bc_south=int(bc[2]), bc_north=int(bc[3]),
                  inflow_ux=float(inflow[0]), inflow_uy=float(inflow[1]),
                  body_force_x=float(body_force[0]), body_force_y=float(body_force[1]),
                  rho0=float(init[0]), ux0=float(init[1]), uy0=float(init[2]),
                  precision=int(precision), history_capacity=int(history_capacity),
                  hip_stream=stream, flags=0)
    h = ctypes.c_void_p()
    check(load().btdf_create(ctypes.byref(g), float(tau), int(delta_kind), float(thickening),
                             ctypes.byref(h)))
    return h.value


def btdf_destroy(h):
    return check(load().btdf_destroy(h))


def btdf_workspace_bytes(h):
    return int(load().btdf_workspace_bytes(h))


def btdf_bind_workspace(h, dev_ptr, nbytes):
    return check(load().btdf_bind_workspace(h, dev_ptr, int(nbytes)))


def btdf_set_stream(h, stream_ptr):
    return check(load().btdf_set_stream(h, stream_ptr))


def btdf_add_body(h, xy, uv=None, cx=0.0, cy=0.0, ds=0.0):
    xy = f64(xy, (-1, 2))
    n = xy.shape[0]
    uvp = None
    if uv is not None:
        uv = f64(uv, (n, 2))
        uvp = dptr(uv)
    bid = ctypes.c_int(-1)
    check(load().btdf_add_body(h, n, dptr(xy), uvp, float(cx), float(cy), float(ds), ctypes.byref(bid)))
    return bid.value


def btdf_set_marker_velocity(h, body, uv):
    uv = f64(uv, (-1, 2))
    return check(load().btdf_set_marker_velocity(h, int(body), dptr(uv)))


def btdf_step(h, n):
    return check(load().btdf_step(h, int(n)))


def btdf_step_timed(h, n):
    a, b = ctypes.c_double(), ctypes.c_double()
    check(load().btdf_step_timed(h, int(n), ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def btdf_counts(h):
    nb, nm, ns = ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
    check(load().btdf_counts(h, ctypes.byref(nb), ctypes.byref(nm), ctypes.byref(ns)))
    return nb.value, nm.value, ns.value


def btdf_forces(h):
    nb = btdf_counts(h)[0]
    out = np.zeros((max(nb, 1), 3))
    check(load().btdf_forces(h, dptr(out), nb))
    return out[:nb]


def btdf_force_history(h, max_steps):
    nb = btdf_counts(h)[0]
    out = np.zeros((max(int(max_steps), 1), max(nb, 1), 3))
    n = ctypes.c_int64()
    check(load().btdf_force_history(h, dptr(out), int(max_steps), ctypes.byref(n)))
    return out[:n.value, :nb]


def btdf_init_equilibrium(h, ux, uy, rho=None):
    ux, uy = f64(ux), f64(uy)
    rho = None if rho is None else f64(rho)
    return check(load().btdf_init_equilibrium(h, dptr(rho), dptr(ux), dptr(uy)))


def btdf_get_macroscopic(h, nx, ny):
    r, u, v = (np.empty((ny, nx)) for _ in range(3))
    check(load().btdf_get_macroscopic(h, dptr(r), dptr(u), dptr(v)))
    return r, u, v


def btdf_get_populations(h, nx, ny):
    f = np.empty((9, ny, nx))
    check(load().btdf_get_populations(h, dptr(f)))
    return f


def btdf_set_populations(h, f):
    f = f64(f)
    return check(load().btdf_set_populations(h, dptr(f)))


def btdf_get_populations_to(h, dst_ptr, dst_on_device):
    """dst_ptr: address (int) of an FP64 [9][ny][nx] array, host or device."""
    return check(load().btdf_get_populations_to(h, ctypes.c_void_p(dst_ptr), int(dst_on_device)))


def btdf_set_populations_from(h, src_ptr, src_on_device):
    return check(load().btdf_set_populations_from(h, ctypes.c_void_p(src_ptr), int(src_on_device)))


def btdf_get_marker_data(h):
    nm = btdf_counts(h)[1]
    arrs = [np.empty(max(nm, 1)) for _ in range(5)]
    check(load().btdf_get_marker_data(h, *[dptr(a) for a in arrs]))
    return dict(zip(["rho", "ux", "uy", "Fx", "Fy"], [a[:nm] for a in arrs]))


def btdf_step_timed_split(h, n):
    out = np.empty(3)
    check(load().btdf_step_timed_split(h, int(n), dptr(out)))
    return tuple(float(v) for v in out)


def btdf_step_timed_pass(h, n):
    out = np.empty(1)
    check(load().btdf_step_timed_pass(h, int(n), dptr(out)))
    return float(out[0])


def btdf_set_body_motion(h, body, vx, vy, omega):
    return check(load().btdf_set_body_motion(h, int(body), float(vx), float(vy), float(omega)))


def btdf_get_body_state(h, body):
    out = np.empty(6)
    check(load().btdf_get_body_state(h, int(body), dptr(out)))
    return out


def btdf_get_marker_positions(h):
    nm = btdf_counts(h)[1]
    out = np.empty((max(nm, 1), 2))
    check(load().btdf_get_marker_positions(h, dptr(out)))
    return out[:nm]


def btdf_marker_velocity(h):
    nm = btdf_counts(h)[1]
    u, v = np.empty(max(nm, 1)), np.empty(max(nm, 1))
    check(load().btdf_marker_velocity(h, dptr(u), dptr(v)))
    return u[:nm], v[:nm]


def btdf_marker_velocity_noalloc(h, ux=None, uy=None):
    """The no-allocation variant; ux, uy: caller-owned float64 arrays of at
    least the marker count (allocated here if not given)."""
    nm = btdf_counts(h)[1]
    u = np.empty(max(nm, 1)) if ux is None else ux
    v = np.empty(max(nm, 1)) if uy is None else uy
    if u.dtype != np.float64 or v.dtype != np.float64 or not u.flags.c_contiguous or not v.flags.c_contiguous:
        raise TypeError("ux and uy must be contiguous float64 arrays")
    if u.size < nm or v.size < nm:
        raise ValueError("ux and uy need room for %d markers" % nm)
    check(load().btdf_marker_velocity_noalloc(h, dptr(u), dptr(v)))
    return u[:nm], v[:nm]


def btdf_state_bytes(h):
    return int(load().btdf_state_bytes(h))


def btdf_save(h):
    n = btdf_state_bytes(h)
    buf = ctypes.create_string_buffer(n)
    check(load().btdf_save(h, ctypes.cast(buf, ctypes.c_void_p), n))
    return buf.raw


def btdf_load(h, state):
    buf = ctypes.create_string_buffer(bytes(state), len(state))
    return check(load().btdf_load(h, ctypes.cast(buf, ctypes.c_void_p), len(state)))


def btdf_set_option(h, key, value):
    return check(load().btdf_set_option(h, int(key), int(value)))


def btdf_get_option(h, key):
    v = ctypes.c_int64()
    check(load().btdf_get_option(h, int(key), ctypes.byref(v)))
    return v.value


def btdf_calibrate_thickening(delta_kind, D, n_markers):
    mean = ctypes.c_double()
    per = np.empty(int(n_markers))
    check(load().btdf_calibrate_thickening(int(delta_kind), float(D), int(n_markers), ctypes.byref(mean),
                                           dptr(per)))
    return mean.value, per


def btdf_calibrate_thickening_markers(delta_kind, xy, ds):
    xy = f64(xy, (-1, 2))
    n = xy.shape[0]
    mean = ctypes.c_double()
    per = np.empty(n)
    check(load().btdf_calibrate_thickening_markers(int(delta_kind), n, dptr(xy), float(ds),
                                                   ctypes.byref(mean), dptr(per)))
    return mean.value, per


def btdf_last_error():
    return _lib.last_error()


def btdf_autotune(h, steps_per_trial):
    v = ctypes.c_int(-1)
    check(load().btdf_autotune(h, int(steps_per_trial), ctypes.byref(v)))
    return v.value


def _grid(nx, ny, bc, inflow, body_force, init, precision, history_capacity, stream):
    return btdf_grid(nx=int(nx), ny=int(ny), bc_west=int(bc[0]), bc_east=int(bc[1]),
                     bc_south=int(bc[2]), bc_north=int(bc[3]),
                     inflow_ux=float(inflow[0]), inflow_uy=float(inflow[1]),
                     body_force_x=float(body_force[0]), body_force_y=float(body_force[1]),
                     rho0=float(init[0]), ux0=float(init[1]), uy0=float(init[2]),
                     precision=int(precision), history_capacity=int(history_capacity),
                     hip_stream=stream, flags=0)


def btdf_batch_create(cases, stream=None):
    """cases: list of dicts with the keyword arguments of btdf_create."""
    n = len(cases)
    grids = (btdf_grid * n)(*[_grid(c["nx"], c["ny"], c.get("bc", (0, 0, 0, 0)), c.get("inflow", (0.0, 0.0)),
                                    c.get("body_force", (0.0, 0.0)), c.get("init", (1.0, 0.0, 0.0)),
                                    c.get("precision", 8), c.get("history_capacity", 0), stream)
                              for c in cases])
    taus = np.array([c["tau"] for c in cases], dtype=np.float64)
    kinds = (ctypes.c_int * n)(*[int(c["delta_kind"]) for c in cases])
    th = np.array([c["thickening"] for c in cases], dtype=np.float64)
    b = ctypes.c_void_p()
    check(load().btdf_batch_create(n, grids, dptr(taus), kinds, dptr(th), ctypes.byref(b)))
    return b.value


def btdf_batch_destroy(b):
    return check(load().btdf_batch_destroy(b))


def btdf_batch_case(b, i):
    h = ctypes.c_void_p()
    check(load().btdf_batch_case(b, int(i), ctypes.byref(h)))
    return h.value


def btdf_batch_add_body(b, case_id, xy, uv=None, cx=0.0, cy=0.0, ds=0.0):
    xy = f64(xy, (-1, 2))
    n = xy.shape[0]
    uvp = None
    if uv is not None:
        uv = f64(uv, (n, 2))
        uvp = dptr(uv)
    bid = ctypes.c_int(-1)
    check(load().btdf_batch_add_body(b, int(case_id), n, dptr(xy), uvp, float(cx), float(cy), float(ds),
                                     ctypes.byref(bid)))
    return bid.value


def btdf_batch_workspace_bytes(b):
    return int(load().btdf_batch_workspace_bytes(b))


def btdf_batch_bind_workspace(b, dev_ptr, nbytes):
    return check(load().btdf_batch_bind_workspace(b, dev_ptr, int(nbytes)))


def btdf_batch_set_stream(b, stream_ptr):
    return check(load().btdf_batch_set_stream(b, stream_ptr))


def btdf_batch_step(b, n):
    return check(load().btdf_batch_step(b, int(n)))


def btdf_batch_step_timed(b, n):
    a, c = ctypes.c_double(), ctypes.c_double()
    check(load().btdf_batch_step_timed(b, int(n), ctypes.byref(a), ctypes.byref(c)))
    return a.value, c.value


def btdf_batch_status(b, n_cases):
    st = (ctypes.c_int * max(1, n_cases))()
    ns = ctypes.c_int64()
    check(load().btdf_batch_status(b, st, ctypes.byref(ns)))
    return np.array(st[:n_cases], dtype=bool), ns.value


def btdf_batch_set_option(b, key, value):
    return check(load().btdf_batch_set_option(b, int(key), int(value)))


def btdf_batch_get_option(b, key):
    v = ctypes.c_int64()
    check(load().btdf_batch_get_option(b, int(key), ctypes.byref(v)))
    return v.value


def btdf_batch_autotune(b, steps_per_trial):
    v = ctypes.c_int(-1)
    check(load().btdf_batch_autotune(b, int(steps_per_trial), ctypes.byref(v)))
    return v.value


def btdf_adjoint_workspace_bytes(h, n_steps, checkpoint_every=0):
    return int(load().btdf_adjoint_workspace_bytes(h, int(n_steps), int(checkpoint_every)))


def btdf_adjoint(h, nx, ny, n_steps, hist_bar, checkpoint_every=0, work=None, work_bytes=0):
    """Returns (gradients dict, (ms forward, ms recompute, ms reverse))."""
    nb, nm, _ = btdf_counts(h)
    hb = None
    if nb:
        hb = f64(hist_bar, (int(n_steps), nb, 3))
    out = dict(populations=np.empty((9, ny, nx)), inflow=np.empty(2), body_force=np.empty(2),
               marker_xy=np.empty((max(nm, 1), 2)), marker_uv=np.empty((max(nm, 1), 2)),
               centres=np.empty((max(nb, 1), 2)))
    g = btdf_gradients(**{k: dptr(v) for k, v in out.items()})
    ms = np.zeros(3)
    check(load().btdf_adjoint(h, int(n_steps), int(checkpoint_every), dptr(hb), ctypes.byref(g), work,
                              int(work_bytes), dptr(ms)))
    out["marker_xy"], out["marker_uv"], out["centres"] = out["marker_xy"][:nm], out["marker_uv"][:nm], \
        out["centres"][:nb]
    return out, tuple(ms)
