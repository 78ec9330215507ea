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
  cylinder_57_full.json    the 57^3 batched workload: 10 sampled (b, q) pairs at
                           full echo, one in each 128-system tile of the batch
                           ordered by b (b = 333 ... 5000) plus two more at
                           b = 5000 / 4667, over axis-near, oblique and
                           equatorial directions
  seeded_cells_seed2.json  the second-smallest seeded-cell geometry, 4 sampled
                           pairs, full echo
  seeded_cells_first2.json 2 sampled pairs on each of the six other seeded-cell
                           geometries (seeds 0, 1, 4, 5, 6, 7) after the first
                           2 steps (sum w u^2)
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


_ASM = {}


def _solve(args):
    name, idx, n_steps = args
    from oracle import fem, timestep
    prob, seq, sysl = _workload(name, idx)
    key = (name, idx[0] if isinstance(idx, tuple) else None)
    if key not in _ASM:  # one assembly per worker and geometry
        _ASM.clear()
        _ASM[key] = fem.assemble(prob)
    asm = _ASM[key]
    i = idx[1] if isinstance(idx, tuple) else idx
    t0 = time.time()
    s = timestep.solve_transformed(asm, seq, float(sysl.b[i]), sysl.q[i], n_steps=n_steps,
                                   solver="krylov")
    print("  %s %s: %.1fs" % (name, idx, time.time() - t0), flush=True)
    return idx, complex(s), time.time() - t0, asm.n_dof


def _workload(name, idx=None):
    if name == "cylinder_36":
        return di.cylinder_36()
    if name in ("cylinder_57_first2", "cylinder_57_full"):
        return di.cylinder_57_batched()
    if name == "seeded_cells_seed3":
        return di.seeded_cells(3)
    if name == "seeded_cells_seed2":
        return di.seeded_cells(2)
    if name == "seeded_cells_first2":
        return di.seeded_cells(idx[0])
    raise KeyError(name)


SAMPLES = {
    "cylinder_36": (list(range(8)), None),
    # b in {5000, 2667, 333} x an axis-near, an oblique and an equatorial direction
    "cylinder_57_first2": ([15, 8, 1, 16 * 20 + 15, 16 * 33 + 8, 16 * 63 + 1], 2),
    "seeded_cells_seed3": ([0, 11, 22, 31], None),
    # pair = direction * 16 + b index; b index 1, 3, 4, 7, 8, 10, 12, 14, 15
    # covers every 128-system tile of the batch ordered by b
    "cylinder_57_full": ([16 * 0 + 15, 16 * 33 + 15, 16 * 20 + 14, 16 * 63 + 12,
                          16 * 45 + 10, 16 * 10 + 8, 16 * 33 + 7, 16 * 52 + 4,
                          16 * 5 + 3, 16 * 27 + 1], None),
    "seeded_cells_seed2": ([0, 11, 22, 31], None),
    # (seed, pair) after 2 steps
    "seeded_cells_first2": ([(s, i) for s in (0, 1, 4, 5, 6, 7) for i in (3, 28)], 2),
}


def make(name, workers=None):
    workers = workers or int(os.environ.get("GOLDEN_WORKERS", "8"))
    idxs, n_steps = SAMPLES[name]
    prob, seq, sysl = _workload(name, idxs[0])
    with ProcessPoolExecutor(max_workers=min(workers, len(idxs))) as ex:
        res = list(ex.map(_solve, [(name, i, n_steps) for i in idxs]))
    if isinstance(idxs[0], tuple):
        per = [_workload(name, r[0]) for r in res]
        b = [float(w[2].b[r[0][1]]) for w, r in zip(per, res)]
        q = [list(map(float, w[2].q[r[0][1]])) for w, r in zip(per, res)]
        index = [list(r[0]) for r in res]
        n_dof = [r[3] for r in res]
    else:
        b = [float(sysl.b[r[0]]) for r in res]
        q = [list(map(float, sysl.q[r[0]])) for r in res]
        index = [r[0] for r in res]
        n_dof = res[0][3]
    out = {
        "workload": name,
        "oracle": "FP64 P1/PUFEM assembly, theta-scheme, SciPy CG/GMRES to 1e-13 per step",
        "sequence": {"delta": seq.delta, "Delta": seq.Delta, "dt": seq.dt, "theta": seq.theta},
        "n_steps": n_steps if n_steps is not None else seq.n_steps,
        "n_dof": n_dof,
        "index": index,
        "b": b,
        "q": q,
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
