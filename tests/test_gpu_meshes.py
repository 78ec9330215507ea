"""Several meshes of uneven size in one batch (option mesh_merge = 1).

The meshes' operators are concatenated block-diagonally and each tile of
systems belongs to one mesh; every kernel launch covers the tiles of all
meshes, each tile over its own mesh's rows. Checked against the FP64 CPU
oracle (exact sparse solves per mesh, tests' own short PGSE sequence) and
against the same pairs run mesh by mesh (mesh_merge = 0).
"""

import numpy as np
import pytest

import dmri_inputs as di
from oracle import timestep

pytestmark = pytest.mark.gpu

SHORT = di.Sequence(2000.0, 4000.0, 200.0, 0.5)


@pytest.fixture(scope="module")
def Sim():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_01719_amd import Simulator
    return Simulator


def _say(msg):
    print(msg, flush=True)


def _err(sig, ref):
    return np.abs(sig - ref) / np.maximum(np.abs(ref), 1e-8 * np.abs(ref).max())


_CASES = {}


def _periodic_case():
    # Three periodic boxes of different sizes (about 600, 1,000 and 1,600
    # DOFs) with 5, 3 and 13 (b, q) pairs: ragged tiles on every mesh.
    if "periodic" not in _CASES:
        probs = [di.cylinder_box(n=8, half=6.0, r=4.0, kappa=1e-2, D_in=1e-3),
                 di.free_diffusion_10()[0],
                 di.cylinder_box(n=11, half=6.0, r=4.3, kappa=5e-3, D_in=1.5e-3,
                                 T2=(6e4, 4e4), u0=(1.0, 0.7))]
        counts = [5, 3, 13]
        rng = np.random.default_rng(11)
        items = []
        for prob, m in zip(probs, counts):
            b = rng.uniform(0.0, 5000.0, m)
            b[0] = 0.0
            q = di.fibonacci_directions(m + 2)[2:]
            ref = timestep.signals(prob, SHORT, b, q, solver="splu")
            items.append((prob, b, q, ref))
        _CASES["periodic"] = items
    return _CASES["periodic"]


def _walls_case():
    # Two walled boxes (the U-form, solved with COCG) of different sizes.
    if "walls" not in _CASES:
        probs = [di.cylinder_box(n=7, half=6.0, r=4.0, kappa=1e-2, D_in=1e-3, periodic_mask=0),
                 di.cylinder_box(n=10, half=6.0, r=3.5, kappa=2e-3, D_in=2e-3, periodic_mask=0)]
        counts = [4, 9]
        rng = np.random.default_rng(12)
        items = []
        for prob, m in zip(probs, counts):
            b = rng.uniform(500.0, 4000.0, m)
            q = di.fibonacci_directions(m)
            ref = timestep.signals(prob, SHORT, b, q, solver="splu")
            items.append((prob, b, q, ref))
        _CASES["walls"] = items
    return _CASES["walls"]


def _run(Sim, items, **opts):
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(**opts)
        pids = [sim.add_problem(prob) for prob, _, _, _ in items]
        ids = np.concatenate([np.full(len(b), p, np.int32) for p, (_, b, _, _) in zip(pids, items)])
        b = np.concatenate([it[1] for it in items])
        q = np.concatenate([it[2] for it in items])
        sig, st = sim.dmri_run(ids, b, q)
    assert st["status"] == "DMRI_OK"
    return sig, st


@pytest.mark.parametrize("precision,tile", [(0, 0), (0, 16), (1, 0), (1, 8)])
def test_periodic_meshes_one_batch_match_oracle(Sim, precision, tile):
    items = _periodic_case()
    ref = np.concatenate([it[3] for it in items])
    merged, st = _run(Sim, items, rtol=1e-12, precision=precision, sys_tile=tile, mesh_merge=1)
    seq, _ = _run(Sim, items, rtol=1e-12, precision=precision, sys_tile=tile, mesh_merge=0)
    err = _err(merged, ref)
    diff = np.abs(merged - seq).max() / np.abs(ref).max()
    _say("3 meshes in one batch, precision %d, tile %d: max err %.2e, vs mesh by mesh %.2e, "
         "%d iterations" % (precision, tile, err.max(), diff, st["total_iterations"]))
    assert err.max() < 1e-9
    assert diff < 1e-10


@pytest.mark.parametrize("guess", [0, 1])
def test_walled_meshes_one_batch_match_oracle(Sim, guess):
    items = _walls_case()
    ref = np.concatenate([it[3] for it in items])
    sig, _ = _run(Sim, items, rtol=1e-12, guess=guess, mesh_merge=1)
    err = _err(sig, ref)
    _say("2 walled meshes in one batch (COCG), guess %d: max err %.2e" % (guess, err.max()))
    assert err.max() < 1e-9


def test_one_batch_refusals(Sim):
    # Combinations the several-mesh batch does not run are refused with an
    # error, not run another way.
    from paper_1908_01719_amd.binding import DmriError
    items = _periodic_case()[:2]
    for opts in (dict(precision=2), dict(krylov=3), dict(graph=1), dict(lds=1)):
        with pytest.raises(DmriError):
            _run(Sim, items, rtol=1e-10, mesh_merge=1, **opts)
