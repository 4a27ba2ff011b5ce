"""Write the stored oracle values used by the GPU parity tests.

Calls only the FP64 oracle (``oracle/``) on the seeded workloads of
``btdf_workloads``. Run from the repository root:

    python tests/golden/make_golden.py c2

c2: the 2000x800 Re = 200 channel (cosine 4-point delta, drs = 2.6 dh,
shedding perturbation), 5000 steps from the perturbed uniform start; the
hydrodynamic force on the cylinder (eq 27) is written every 10 steps as
``step Fx Fy Tz`` with 17 significant digits.
"""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import btdf_workloads as W  # noqa: E402
from oracle.oracle import OracleSim  # noqa: E402


def c2_forces(path, steps=5000, every=10):
    c = W.c2()
    s = OracleSim(c.nx, c.ny, c.bc, c.tau, c.kind, c.thickening, c.G, c.inflow, c.init)
    for b in c.bodies:
        s.add_body(b.xy, b.uv, b.cx, b.cy, b.ds)
    ux, uy = c.init_fields()
    s.init_equilibrium(ux, uy, np.full((c.ny, c.nx), c.init[0]))
    rows = []
    t0 = time.time()
    for k in range(steps // every):
        s.step(every)
        F = s.forces()[0]
        rows.append((s.steps, F[0], F[1], F[2]))
        if (k + 1) % 50 == 0:
            print("step %d  %.1f s" % (s.steps, time.time() - t0), flush=True)
    with open(path, "w") as f:
        f.write("# oracle forces on the cylinder of the 2000x800 Re=200 channel (cosine 4-point, drs=2.6)\n")
        f.write("# written by tests/golden/make_golden.py from oracle/ only; columns: step Fx Fy Tz\n")
        for r in rows:
            f.write("%d %.17e %.17e %.17e\n" % r)


if __name__ == "__main__":
    which = sys.argv[1:] or ["c2"]
    if "c2" in which:
        c2_forces(os.path.join(HERE, "c2_oracle_forces_5k.txt"))
