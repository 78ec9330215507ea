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
        st["n_dof"] = [sim.dmri_problem_info(p)[0] for p in pids]
    assert st["status"] == "DMRI_OK"
    return sig, st


@pytest.mark.parametrize("precision,tile,queue", [(0, 0, 0), (0, 16, 0), (0, 64, 0), (0, 8, 1),
                                                  (1, 0, 0), (1, 8, 0), (1, 16, 1)])
def test_periodic_meshes_one_batch_match_oracle(Sim, precision, tile, queue):
    # Tiles of 8-64 systems (64: one ragged tile per mesh), static row
    # chunks or per-item row queues in the gather kernels.
    items = _periodic_case()
    ref = np.concatenate([it[3] for it in items])
    opts = dict(rtol=1e-12, precision=precision, sys_tile=tile, queue=queue)
    merged, st = _run(Sim, items, mesh_merge=1, **opts)
    seq, _ = _run(Sim, items, mesh_merge=0, **opts)
    err = _err(merged, ref)
    diff = np.abs(merged - seq).max() / np.abs(ref).max()
    _say("3 meshes in one batch, precision %d, tile %d, queue %d: max err %.2e, vs mesh by mesh "
         "%.2e, %d iterations" % (precision, tile, queue, err.max(), diff, st["total_iterations"]))
    assert err.max() < 1e-9
    assert diff < 1e-10
    # Work counters cover the caller's pairs only, each over its own mesh.
    rows = np.concatenate([np.full(len(it[1]), n) for it, n in zip(items, st["n_dof"])])
    iters = np.asarray(st["iters_total"], np.int64)
    assert st["total_iterations"] == iters.sum()
    assert st["spmv_rows"] == int((iters * rows).sum())


@pytest.mark.parametrize("precision", [0, 1])
def test_periodic_meshes_persistent_and_graph(Sim, precision):
    # The three meshes' 21 pairs in 32 slots (tiles of 8) solved by the
    # persistent Krylov kernel: one launch per solve spans every mesh. In
    # FP64 the whole time loop is also captured in a HIP graph, then
    # replayed by a second run; both runs match the oracle within 1e-9 and
    # each other exactly, and the chunked launches within 1e-10.
    items = _periodic_case()
    ref = np.concatenate([it[3] for it in items])
    base = dict(rtol=1e-12, precision=precision, mesh_merge=1)
    chunked, stc = _run(Sim, items, persistent=0, time_kernel=1, **base)
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(persistent=1, graph=1 if precision == 0 else 0, **base)
        pids = [sim.add_problem(prob) for prob, _, _, _ in items]
        ids = np.concatenate([np.full(len(b), p, np.int32)
                              for p, (_, b, _, _) in zip(pids, items)])
        b = np.concatenate([it[1] for it in items])
        q = np.concatenate([it[2] for it in items])
        first, st1 = sim.dmri_run(ids, b, q)
        second, st2 = sim.dmri_run(ids, b, q)
        # Krylov launches counted (no graph): one per solve in the persistent kernel.
        sim.set_options(graph=0, time_kernel=1)
        _, st3 = sim.dmri_run(ids, b, q)
    assert st1["status"] == "DMRI_OK" and st2["status"] == "DMRI_OK"
    err = _err(first, ref)
    diff = np.abs(first - chunked).max() / np.abs(ref).max()
    _say("3 meshes, persistent kernel (precision %d): max err %.2e, vs chunked %.2e"
         % (precision, err.max(), diff))
    assert err.max() < 1e-9
    assert diff < 1e-10
    assert np.array_equal(first, second)
    _say("Krylov launches: persistent %d, chunked %d" % (st3["n_kernel_launches"],
                                                         stc["n_kernel_launches"]))
    if precision == 0:
        assert st3["n_kernel_launches"] == st3["n_steps"]
    assert st3["n_kernel_launches"] * 4 < stc["n_kernel_launches"]


@pytest.mark.parametrize("precision", [0, 1])
def test_periodic_meshes_autotuned(Sim, precision):
    # The several-mesh batch under the autotuner: its trials (tile width,
    # blocks per XCD, persistent kernel) run on the first steps, the choice
    # is cached for the kind of batch; both runs within 1e-9 of the oracle,
    # the second (from the cache, no trials) identical to the first.
    items = _periodic_case()
    ref = np.concatenate([it[3] for it in items])
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        # (sort_systems = 0: both runs fill the slots in the same order)
        sim.set_options(rtol=1e-12, precision=precision, mesh_merge=1, autotune=1,
                        sort_systems=0)
        pids = [sim.add_problem(prob) for prob, _, _, _ in items]
        ids = np.concatenate([np.full(len(b), p, np.int32)
                              for p, (_, b, _, _) in zip(pids, items)])
        b = np.concatenate([it[1] for it in items])
        q = np.concatenate([it[2] for it in items])
        first, st1 = sim.dmri_run(ids, b, q)
        tuned = {k: sim.dmri_get_option(k) for k in ("tuned_sys_tile", "tuned_blocks_per_xcd",
                                                       "tuned_persistent", "tuned_trials")}
        second, st2 = sim.dmri_run(ids, b, q)
    assert st1["status"] == "DMRI_OK" and st2["status"] == "DMRI_OK"
    err = _err(first, ref)
    _say("3 meshes autotuned (precision %d): %s, max err %.2e" % (precision, tuned, err.max()))
    # tiles of 8 (13 pairs at most per mesh): 3 launch shapes + the persistent kernel
    assert tuned["tuned_trials"] == 4
    assert tuned["tuned_sys_tile"] == 8
    assert err.max() < 1e-9
    assert np.array_equal(first, second)


def test_periodic_meshes_fp32(Sim):
    # FP32 throughout (precision 2) over the three meshes in one batch:
    # within 1e-4 of the oracle, as for one mesh.
    items = _periodic_case()
    ref = np.concatenate([it[3] for it in items])
    sig, _ = _run(Sim, items, rtol=1e-6, precision=2, mesh_merge=1)
    err = _err(sig, ref)
    _say("3 meshes in one batch, FP32: max err %.2e" % err.max())
    assert err.max() < 1e-4


@pytest.mark.parametrize("case", ["walls", "periodic"])
def test_meshes_one_batch_gmres(Sim, case):
    # Restarted GMRES(12) over several meshes in one batch (the U-form's
    # cross-check, and on the transformed form): within 1e-9 of the oracle.
    items = _walls_case() if case == "walls" else _periodic_case()
    ref = np.concatenate([it[3] for it in items])
    sig, st = _run(Sim, items, rtol=1e-12, krylov=3, gmres_m=12, mesh_merge=1)
    err = _err(sig, ref)
    _say("%s meshes in one batch, GMRES(12): max err %.2e, %d Arnoldi steps"
         % (case, err.max(), st["total_iterations"]))
    assert err.max() < 1e-9


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
    for opts in (dict(precond=2), dict(lds=1), dict(guess=2)):
        with pytest.raises(DmriError):
            _run(Sim, items, rtol=1e-10, mesh_merge=1, **opts)


def _golden(name):
    import json
    import os
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                           name + ".json")) as f:
        d = json.load(f)
    return d, np.array(d["signal_re"]) + 1j * np.array(d["signal_im"])


def test_seeded_cells_one_batch(Sim):
    # The uneven workload as one batch: the 8 seeded-cell geometries (seeds
    # 0-7, 63k-878k DOFs), 32 (b, q) pairs each, every launch over all 8
    # meshes. Mixed precision at rtol 1e-6 over the full echo: the oracle's
    # full-echo signals of seeds 2 and 3 within 1e-4. All-FP64 at rtol 1e-12
    # for the first two steps: the oracle's sums after two steps on seeds 0,
    # 1 and 4 within 1e-9.
    items = [di.seeded_cells(seed) for seed in range(8)]
    seq = items[0][1]
    out = {}
    with Sim(0) as sim:
        sim.set_sequence(seq)
        pids = [sim.add_problem(prob) for prob, _, _ in items]
        ids = np.concatenate([np.full(len(sl), p, np.int32) for p, (_, _, sl) in zip(pids, items)])
        b = np.concatenate([sl.b for _, _, sl in items])
        q = np.concatenate([sl.q for _, _, sl in items])
        for key, opts in (("mixed", dict(precision=1, rtol=1e-6)),
                          ("first2", dict(precision=0, rtol=1e-12, n_steps=2, signal=0))):
            o = dict(mesh_merge=1, n_steps=0, signal=1)
            o.update(opts)
            sim.set_options(**o)
            sig, st = sim.dmri_run(ids, b, q)
            assert st["status"] == "DMRI_OK"
            out[key] = (sig.reshape(8, 32), st)
    sig, st = out["mixed"]
    errs = []
    for seed in (2, 3):
        d, ref = _golden("seeded_cells_seed%d" % seed)
        errs.append(np.abs(sig[seed][np.array(d["index"])] - ref) / np.abs(ref))
    e_full = np.concatenate(errs).max()
    d, ref = _golden("seeded_cells_first2")
    first = out["first2"][0]
    got = np.array([first[s][i] for s, i in d["index"]])
    e_first = (np.abs(got - ref) / np.abs(ref)).max()
    _say("seeded cells, 8 meshes in one batch: mixed full echo max err %.2e (solve %.1f s, %d "
         "inner iterations); FP64 first two steps max err %.2e"
         % (e_full, st["t_solve_s"], st["total_iterations"], e_first))
    assert e_full < 1e-4
    assert e_first < 1e-9
    assert np.all(np.isfinite(sig))
