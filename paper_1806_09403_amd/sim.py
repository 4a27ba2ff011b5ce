"""``Sim``: one BTDF-IB-LBM simulation on the current GPU.

PyTorch supplies the device memory (one uint8 tensor bound as the
library's workspace, regrown when bodies are added) and the stream (the
current torch stream). All arithmetic of the step runs in the library's
HIP kernels.
"""
import numpy as np

from . import api
from ._lib import COS4, PERIODIC


class Sim:
    def __init__(self, nx, ny, tau, delta_kind=COS4, thickening=2.6, bc=(PERIODIC,) * 4,
                 inflow=(0.0, 0.0), body_force=(0.0, 0.0), init=(1.0, 0.0, 0.0), precision=8,
                 history_capacity=0, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("Sim needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.device = torch.device("cuda" if device is None else device)
        self.nx, self.ny = int(nx), int(ny)
        self.precision = int(precision)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        self.h = api.btdf_create(nx, ny, tau, delta_kind, thickening, bc, inflow, body_force, init,
                                 precision, history_capacity, self.stream.cuda_stream)
        self._ws = None

    @classmethod
    def from_case(cls, case, precision=None, set_init=True, options=None):
        """Build from a ``btdf_workloads.Case`` (bodies and initial flow included);
        options: {BTDF_OPT_* key: value} set before any device memory is made."""
        s = cls(case.nx, case.ny, case.tau, case.kind, case.thickening, case.bc, case.inflow, case.G,
                case.init, case.precision if precision is None else precision)
        for k, v in (options or {}).items():
            s.set_option(k, v)
        for b in case.bodies:
            s.add_body(b.xy, b.uv, b.cx, b.cy, b.ds)
        if set_init and case.init_uy is not None:
            ux, uy = case.init_fields()
            s.init_equilibrium(ux, uy, np.full((case.ny, case.nx), case.init[0]))
        return s

    # -- memory ---------------------------------------------------------------
    def _workspace(self):
        import torch
        need = api.btdf_workspace_bytes(self.h)
        if self._ws is None or self._ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            api.btdf_bind_workspace(self.h, ws.data_ptr(), ws.numel())
            self._ws = ws
        return self.h

    def close(self):
        if getattr(self, "h", None):
            api.btdf_destroy(self.h)
            self.h = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- calls ------------------------------------------------------------------
    def add_body(self, xy, uv=None, cx=0.0, cy=0.0, ds=0.0):
        return api.btdf_add_body(self.h, xy, uv, cx, cy, ds)

    def set_marker_velocity(self, body, uv):
        return api.btdf_set_marker_velocity(self._workspace(), body, uv)

    def step(self, n=1):
        return api.btdf_step(self._workspace(), n)

    def step_timed(self, n):
        return api.btdf_step_timed(self._workspace(), n)

    def forces(self):
        return api.btdf_forces(self._workspace())

    def force_history(self, max_steps):
        return api.btdf_force_history(self._workspace(), max_steps)

    def init_equilibrium(self, ux, uy, rho=None):
        return api.btdf_init_equilibrium(self._workspace(), ux, uy, rho)

    def macroscopic(self):
        return api.btdf_get_macroscopic(self._workspace(), self.nx, self.ny)

    def populations(self):
        return api.btdf_get_populations(self._workspace(), self.nx, self.ny)

    def set_populations(self, f):
        return api.btdf_set_populations(self._workspace(), f)

    def populations_to(self, out):
        """Fill a contiguous FP64 torch tensor of shape (9, ny, nx) on the
        handle's device with the populations, with no copy through the host."""
        import torch
        assert out.dtype == torch.float64 and out.is_cuda and out.is_contiguous()
        assert tuple(out.shape) == (9, self.ny, self.nx)
        return api.btdf_get_populations_to(self._workspace(), out.data_ptr(), 1)

    def set_populations_from(self, src):
        """Set the populations from a contiguous FP64 torch tensor (9, ny, nx)
        on the handle's device."""
        import torch
        assert src.dtype == torch.float64 and src.is_cuda and src.is_contiguous()
        assert tuple(src.shape) == (9, self.ny, self.nx)
        return api.btdf_set_populations_from(self._workspace(), src.data_ptr(), 1)

    def marker_data(self):
        return api.btdf_get_marker_data(self._workspace())

    def step_timed_split(self, n):
        """Per-step ms of (marker kernels, single-step lattice kernels, blocked pass)."""
        return api.btdf_step_timed_split(self._workspace(), n)

    def step_timed_pass(self, n):
        """n steps timing only the blocked pass (ms per step; events around its launches alone)."""
        return api.btdf_step_timed_pass(self._workspace(), n)

    @property
    def steps(self):
        """Steps taken so far."""
        return api.btdf_counts(self.h)[2]

    def set_body_motion(self, body, vx, vy, omega):
        """Rigid motion of a body from the next step on (translation and turn rate per step)."""
        return api.btdf_set_body_motion(self.h, body, vx, vy, omega)

    def body_state(self, body):
        """(cx, cy, theta, vx, vy, omega) of a body."""
        return api.btdf_get_body_state(self.h, body)

    def marker_positions(self):
        return api.btdf_get_marker_positions(self._workspace())

    def marker_velocity(self):
        """(u, v) at every marker after the last step (eq 11 interpolated by eq 12)."""
        return api.btdf_marker_velocity(self._workspace())

    def save(self):
        return api.btdf_save(self._workspace())

    def load(self, state):
        return api.btdf_load(self._workspace(), state)

    def counts(self):
        return api.btdf_counts(self.h)

    def set_option(self, key, value):
        return api.btdf_set_option(self.h, key, value)

    def get_option(self, key):
        return api.btdf_get_option(self.h, key)

    def autotune(self, steps_per_trial=20):
        return api.btdf_autotune(self._workspace(), steps_per_trial)

    def adjoint(self, n_steps, hist_bar, checkpoint_every=0):
        """Take n_steps (as step(n_steps) would) and return the gradients of
        J = sum(hist_bar * force history of these steps) and the timings
        (ms of the forward run, the recomputation and the reverse steps).
        The adjoint's device memory is a torch tensor, freed on return."""
        import torch
        h = self._workspace()
        nbytes = api.btdf_adjoint_workspace_bytes(h, n_steps, checkpoint_every)
        work = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        try:
            return api.btdf_adjoint(h, self.nx, self.ny, n_steps, hist_bar, checkpoint_every,
                                    work.data_ptr(), work.numel())
        finally:
            del work


class _CaseView(Sim):
    """A case of a BatchSim: every state call of Sim, on the batch's memory."""

    def __init__(self, batch, i, nx, ny, precision):
        self._batch = batch
        self.h = api.btdf_batch_case(batch.b, i)
        self.nx, self.ny, self.precision = nx, ny, precision
        self._ws = None

    def _workspace(self):
        self._batch._workspace()
        return self.h

    def close(self):
        self.h = None  # owned by the batch

    def step(self, n=1):
        raise RuntimeError("step the batch, not one of its cases")


class BatchSim:
    """Many independent cases stepped together (one launch per kernel per step)."""

    def __init__(self, cases, precision=4, device=None, options=None):
        """cases: btdf_workloads.Case objects (bodies and initial flow included);
        options: {BTDF_OPT_* key: value} set before any device memory is made."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("BatchSim needs a ROCm GPU")
        self.device = torch.device("cuda" if device is None else device)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        spec = [dict(nx=c.nx, ny=c.ny, tau=c.tau, delta_kind=c.kind, thickening=c.thickening, bc=c.bc,
                     inflow=c.inflow, body_force=c.G, init=c.init, precision=precision) for c in cases]
        self.b = api.btdf_batch_create(spec, self.stream.cuda_stream)
        for k, v in (options or {}).items():
            api.btdf_batch_set_option(self.b, k, v)
        self.n = len(cases)
        self._ws = None
        self.cases = []
        for i, c in enumerate(cases):
            for body in c.bodies:
                api.btdf_batch_add_body(self.b, i, body.xy, body.uv, body.cx, body.cy, body.ds)
            self.cases.append(_CaseView(self, i, c.nx, c.ny, precision))
        for i, c in enumerate(cases):
            if c.init_uy is not None:
                ux, uy = c.init_fields()
                self.cases[i].init_equilibrium(ux, uy, np.full((c.ny, c.nx), c.init[0]))

    def _workspace(self):
        import torch
        need = api.btdf_batch_workspace_bytes(self.b)
        if self._ws is None or self._ws_need != need:
            ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            api.btdf_batch_bind_workspace(self.b, ws.data_ptr(), ws.numel())
            self._ws, self._ws_need = ws, need
        return self.b

    def add_body(self, case_id, xy, uv=None, cx=0.0, cy=0.0, ds=0.0):
        return api.btdf_batch_add_body(self.b, case_id, xy, uv, cx, cy, ds)

    def step(self, n=1):
        return api.btdf_batch_step(self._workspace(), n)

    def step_timed(self, n):
        return api.btdf_batch_step_timed(self._workspace(), n)

    def status(self):
        return api.btdf_batch_status(self._workspace(), self.n)

    def set_option(self, key, value):
        return api.btdf_batch_set_option(self.b, key, value)

    def get_option(self, key):
        return api.btdf_batch_get_option(self.b, key)

    def autotune(self, steps_per_trial=20):
        return api.btdf_batch_autotune(self._workspace(), steps_per_trial)

    def close(self):
        if getattr(self, "b", None):
            api.btdf_batch_destroy(self.b)
            self.b = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
