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
    def from_case(cls, case, precision=None, set_init=True):
        """Build from a ``btdf_workloads.Case`` (bodies and initial flow included)."""
        s = cls(case.nx, case.ny, case.tau, case.kind, case.thickening, case.bc, case.inflow, case.G,
                case.init, case.precision if precision is None else precision)
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

    def marker_data(self):
        return api.btdf_get_marker_data(self._workspace())

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
