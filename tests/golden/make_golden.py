"""Write the oracle's expected signals for the full-size parity tests.

Calls only the FP64 CPU oracle (oracle/) on the seeded synthetic workloads
(dmri_inputs); nothing here touches the GPU library. Each fixture records
the workload, the solver the oracle used and the signals.

    python tests/golden/make_golden.py [name ...]      (default: all)

Fixtures:
  cylinder_36.json         the two-compartment cylinder box (36^3 cubes,
                           51,408 DOFs), all 8 b-values, full PGSE echo
                           (240 steps)
  cylinder_57_first2.json  the 57^3 batched workload (196,593 DOFs): 6 sampled
                           (b, q) pairs after the first 2 steps (sum w u^2)
  seeded_cells_seed3.json  the smallest seeded-cell geometry, 4 sampled pairs,
                           full echo
"""

from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

# One BLAS thread per worker process; set before numpy is imported (the
# workers are forked from this process).
for _k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
    os.environ[_k] = "1"

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import dmri_inputs as di  # noqa: E402


def _solve(args):
    name, idx, n_steps = args
    from oracle import fem, timestep
    prob, seq, sysl = _workload(name)
    asm = fem.assemble(prob)
    t0 = time.time()
    s = timestep.solve_transformed(asm, seq, float(sysl.b[idx]), sysl.q[idx], n_steps=n_steps,
                                   solver="krylov")
    return idx, complex(s), time.time() - t0, asm.n_dof


def _workload(name):
    if name == "cylinder_36":
        return di.cylinder_36()
    if name == "cylinder_57_first2":
        return di.cylinder_57_batched()
    if name == "seeded_cells_seed3":
        return di.seeded_cells(3)
    raise KeyError(name)


SAMPLES = {
    "cylinder_36": (list(range(8)), None),
    # b in {5000, 2667, 333} x an axis-near, an oblique and an equatorial direction
    "cylinder_57_first2": ([15, 8, 1, 16 * 20 + 15, 16 * 33 + 8, 16 * 63 + 1], 2),
    "seeded_cells_seed3": ([0, 11, 22, 31], None),
}


def make(name, workers=8):
    idxs, n_steps = SAMPLES[name]
    prob, seq, sysl = _workload(name)
    with ProcessPoolExecutor(max_workers=min(workers, len(idxs))) as ex:
        res = list(ex.map(_solve, [(name, i, n_steps) for i in idxs]))
    out = {
        "workload": name,
        "oracle": "FP64 P1/PUFEM assembly, theta-scheme, SciPy CG/GMRES to 1e-13 per step",
        "sequence": {"delta": seq.delta, "Delta": seq.Delta, "dt": seq.dt, "theta": seq.theta},
        "n_steps": n_steps if n_steps is not None else seq.n_steps,
        "n_dof": res[0][3],
        "index": [r[0] for r in res],
        "b": [float(sysl.b[r[0]]) for r in res],
        "q": [list(map(float, sysl.q[r[0]])) for r in res],
        "signal_re": [r[1].real for r in res],
        "signal_im": [r[1].imag for r in res],
        "seconds_per_system": [r[2] for r in res],
    }
    with open(os.path.join(HERE, name + ".json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, "done", flush=True)


if __name__ == "__main__":
    names = sys.argv[1:] or list(SAMPLES)
    for n in names:
        make(n)
