"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

Tolerances: the all-FP64 GPU path within 1e-9 of the oracle's exact-solve
signal (relative error with the floor max(|S_ref|, 1e-8 S(b=0))); the FP32
operator within 1e-6 of FP64 CSR products.
"""

import numpy as np
import pytest

import dmri_inputs as di
from oracle import fem, timestep

pytestmark = pytest.mark.gpu

SHORT = di.Sequence(2000.0, 4000.0, 200.0, 0.5)


@pytest.fixture(scope="module")
def Sim():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_01719_amd import Simulator
    return Simulator


def rel_err(s, ref, s0):
    floor = np.maximum(np.abs(ref), 1e-8 * abs(s0))
    return np.abs(s - ref) / floor


def _say(msg):
    print(msg, flush=True)


def test_apply_operator_matches_csr(Sim):
    prob = di.cylinder_box(n=10, half=6.0, r=4.0, kappa=1e-2, D_in=1e-3)
    rng = np.random.default_rng(0)
    with Sim(0) as sim:
        sim.set_sequence(di.PGSE_SHORT)
        pid = sim.add_problem(prob)
        exp = sim.dmri_export_operator(pid)
        n = exp["w"].shape[0]
        rows = np.repeat(np.arange(n), np.diff(exp["row_ptr"]))
        import scipy.sparse as sp
        mk = lambda v: sp.csr_matrix((v, (rows, exp["col"])), shape=(n, n))  # noqa: E731
        M, R, MD = mk(exp["vals"][0]), mk(exp["vals"][1]), mk(exp["vals"][2])
        V = [mk(exp["vals"][3 + a]) for a in range(3)]
        k, th = di.PGSE_SHORT.dt, di.PGSE_SHORT.theta
        for n_sys in (1, 13, 64, 70):
            c = rng.uniform(0, 2e-3, n_sys)
            d = rng.normal(size=(n_sys, 3)) * 0.01
            x = rng.normal(size=(n, n_sys)) + 1j * rng.normal(size=(n, n_sys))
            for which, base in ((0, M / k + th * R), (1, M / k - (1 - th) * R)):
                ref = np.empty_like(x)
                for s in range(n_sys):
                    A = base + c[s] * MD + 1j * (d[s, 0] * V[0] + d[s, 1] * V[1] + d[s, 2] * V[2])
                    ref[:, s] = A @ x[:, s]
                for prec, tol in ((0, 1e-13), (2, 2e-6)):
                    sim.dmri_set_option("precision", prec)
                    y = sim.dmri_apply_operator(pid, which, c, d, x)
                    err = np.abs(y - ref).max() / np.abs(ref).max()
                    _say("apply n_sys=%d which=%d prec=%d err=%.2e" % (n_sys, which, prec, err))
                    assert err < tol
        sim.dmri_set_option("precision", 0)


def test_free_diffusion_closed_form(Sim):
    prob, seq, sysl = di.free_diffusion_10()
    with Sim(0) as sim:
        sim.set_sequence(seq)
        sim.set_options(rtol=1e-12)
        pid = sim.add_problem(prob)
        sig, st = sim.dmri_run([pid], sysl.b, sysl.q)
    assert st["status"] == "DMRI_OK"
    assert sig[0].real / 1000.0 == pytest.approx(0.049775509970, abs=1e-11)
    assert abs(sig[0].imag) < 1e-10


def _cyl_case():
    prob = di.cylinder_box(n=11, half=6.0, r=4.3, kappa=5e-3, D_in=1.5e-3, T2=(6e4, 4e4),
                           u0=(1.0, 0.7))
    b = np.array([0.0, 500.0, 1500.0, 3000.0, 5000.0, 2500.0, 4000.0, 1000.0, 3500.0, 200.0,
                  4500.0, 800.0, 2000.0])
    q = di.fibonacci_directions(13)
    return prob, b, q


_CYL_REF = {}


def _cyl_ref():
    # The oracle's exact-solve signals of _cyl_case under SHORT, computed once
    # per session (each call builds the case afresh, so nothing is shared
    # with the GPU side).
    if "ref" not in _CYL_REF:
        prob, b, q = _cyl_case()
        _CYL_REF["ref"] = timestep.signals(prob, SHORT, b, q, solver="splu")
    return _CYL_REF["ref"].copy()


@pytest.mark.parametrize("tile", [0, 8, 16, 64])
@pytest.mark.parametrize("guess", [0, 1])
def test_fp64_transformed_matches_oracle(Sim, tile, guess):
    prob, b, q = _cyl_case()
    ref = _cyl_ref()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12, sys_tile=tile, guess=guess)
        pid = sim.add_problem(prob)
        sig, st = sim.dmri_run([pid] * len(b), b, q)
    err = rel_err(sig, ref, ref[0])
    _say("tile=%d guess=%d max err %.2e iters %s" % (tile, guess, err.max(),
                                                    st["iters_total"].tolist()))
    assert st["status"] == "DMRI_OK"
    assert err.max() < 1e-9


def test_fp64_full_pgse_cylinder_geometry_coarse(Sim):
    # The config-1 geometry (cylinder r=5 in a 12 um box) at n=12 with the
    # full PGSE timing of the workload.
    prob = di.cylinder_box(n=12)
    seq = di.PGSE_SHORT
    b = np.linspace(0.0, 3000.0, 8)
    q = np.tile([[1.0, 0.0, 0.0]], (8, 1))
    ref = timestep.signals(prob, seq, b, q, solver="krylov")
    with Sim(0) as sim:
        sim.set_sequence(seq)
        sim.set_options(rtol=1e-12)
        pid = sim.add_problem(prob)
        sig, st = sim.dmri_run([pid] * 8, b, q)
    err = rel_err(sig, ref, ref[0])
    _say("cylinder-coarse max err %.2e" % err.max())
    assert err.max() < 1e-9
    assert sig[0].real == pytest.approx(1728.0, rel=1e-12)


def test_uform_cocg_matches_oracle(Sim):
    prob = di.slab_box(n=10, half=5.0, split=-1.0, D=(3e-3, 1e-3), kappa=1e-3, u0=(1.0, 0.2),
                       periodic_mask=0)
    b = np.array([0.0, 1000.0, 3000.0])
    q = np.array([[1.0, 0.0, 0.0], [0.8, 0.6, 0.0], [0.0, 0.3, 0.95]])
    ref = timestep.signals(prob, SHORT, b, q, form="uform", solver="splu")
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12)
        pid = sim.add_problem(prob)
        sig, st = sim.dmri_run([pid] * 3, b, q)
    err = rel_err(sig, ref, ref[0])
    _say("uform max err %.2e" % err.max())
    assert err.max() < 1e-9
    assert abs(ref[1].imag) > 1e-3  # a genuinely complex signal


def test_batched_equals_single(Sim):
    prob, b, q = _cyl_case()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12)
        pid = sim.add_problem(prob)
        allsig, _ = sim.dmri_run([pid] * len(b), b, q)
        for i in (3, 7, 12):
            one, _ = sim.dmri_run([pid], b[i:i + 1], q[i:i + 1])
            assert abs(one[0] - allsig[i]) <= 1e-11 * abs(allsig[0])


def test_two_problems_one_run(Sim):
    p1 = di.cylinder_box(n=9, half=6.0, r=4.0, kappa=1e-2)
    p2 = di.free_box(n=7, half=3.5)
    b = np.array([1000.0, 2000.0, 1000.0, 3000.0])
    q = np.array([[1.0, 0, 0], [0, 1.0, 0], [0.6, 0.8, 0], [0, 0, 1.0]])
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12)
        i1 = sim.add_problem(p1)
        i2 = sim.add_problem(p2)
        sig, _ = sim.dmri_run([i1, i2, i2, i1], b, q)
    r1 = timestep.signals(p1, SHORT, b[[0, 3]], q[[0, 3]], solver="splu")
    r2 = timestep.signals(p2, SHORT, b[[1, 2]], q[[1, 2]], solver="splu")
    assert np.abs(sig[[0, 3]] - r1).max() < 1e-9 * abs(r1).max()
    assert np.abs(sig[[1, 2]] - r2).max() < 1e-9 * abs(r2).max()


def test_two_problems_device_entry(Sim):
    # The device entry point with a per-pair problem-id array: pairs of two
    # meshes interleaved, inputs and signals in device memory.
    import torch
    p1 = di.cylinder_box(n=9, half=6.0, r=4.0, kappa=1e-2)
    p2 = di.free_box(n=7, half=3.5)
    b = np.array([1000.0, 2000.0, 1000.0, 3000.0, 0.0])
    q = np.array([[1.0, 0, 0], [0, 1.0, 0], [0.6, 0.8, 0], [0, 0, 1.0], [1.0, 0, 0]])
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12)
        i1 = sim.add_problem(p1)
        i2 = sim.add_problem(p2)
        ids = np.array([i1, i2, i2, i1, i2], np.int32)
        dp = torch.tensor(ids, dtype=torch.int32, device="cuda")
        db = torch.tensor(b, dtype=torch.float64, device="cuda")
        dq = torch.tensor(q, dtype=torch.float64, device="cuda")
        ds = torch.zeros((len(b), 2), dtype=torch.float64, device="cuda")
        st = sim.dmri_run_device(dp, db, dq, ds)
        torch.cuda.synchronize()
        dev = ds.cpu().numpy()
        sig = dev[:, 0] + 1j * dev[:, 1]
        bad = torch.tensor([i1, 7], dtype=torch.int32, device="cuda")
        with pytest.raises(Exception, match="DMRI_E_STATE"):
            sim.dmri_run_device(bad, db[:2], dq[:2], ds[:2])
    assert st["status"] == "DMRI_OK"
    r1 = timestep.signals(p1, SHORT, b[[0, 3]], q[[0, 3]], solver="splu")
    r2 = timestep.signals(p2, SHORT, b[[1, 2, 4]], q[[1, 2, 4]], solver="splu")
    _say("device entry, two problems: errs %.2e %.2e" % (
        np.abs(sig[[0, 3]] - r1).max() / abs(r1).max(),
        np.abs(sig[[1, 2, 4]] - r2).max() / abs(r2).max()))
    assert np.abs(sig[[0, 3]] - r1).max() < 1e-9 * abs(r1).max()
    assert np.abs(sig[[1, 2, 4]] - r2).max() < 1e-9 * abs(r2).max()


def test_sampled_first_steps(Sim):
    # n_steps limits the run; compare sum w u^n after 3 steps with the oracle
    # (option signal = 0: the transformed field's integral).
    prob, b, q = _cyl_case()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-13, n_steps=3, signal=0)
        pid = sim.add_problem(prob)
        sig, _ = sim.dmri_run([pid] * 4, b[:4], q[:4])
    ref = timestep.signals(prob, SHORT, b[:4], q[:4], solver="splu", n_steps=3)
    assert np.abs(sig - ref).max() < 1e-10 * abs(ref).max()


def test_not_converged_and_invalid(Sim):
    from paper_1908_01719_amd import DmriError
    prob, b, q = _cyl_case()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        sim.set_options(max_iter=1, rtol=1e-12)
        sig, st = sim.dmri_run([pid] * 3, b[1:4], q[1:4])
        assert st["status"] == "DMRI_NOT_CONVERGED"
        assert not st["converged"].any()
        assert np.all(np.isfinite(sig))
        sim.set_options(max_iter=2000)
        with pytest.raises(DmriError) as ei:
            sim.dmri_run([pid], [-1.0], [[1, 0, 0]])
        assert "DMRI_E_INVALID" in str(ei.value)
        with pytest.raises(DmriError):
            sim.dmri_run([pid], [1000.0], [[0, 0, 0]])
        with pytest.raises(DmriError):
            sim.dmri_run([5], [1000.0], [[1, 0, 0]])


def test_empty_runs(Sim):
    # n_pairs = 0 through both entry points: DMRI_OK, nothing written, the
    # scalar statistics zeroed.
    import torch
    prob, b, q = _cyl_case()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        sig, st = sim.dmri_run([pid], np.zeros(0), np.zeros((0, 3)))
        assert sig.shape == (0,) and st["status"] == "DMRI_OK"
        assert st["total_iterations"] == 0 and st["n_steps"] == 0
        e = torch.zeros(0, dtype=torch.float64, device="cuda")
        sim.dmri_run_device(pid, e, torch.zeros((0, 3), dtype=torch.float64, device="cuda"),
                            torch.zeros((0, 2), dtype=torch.float64, device="cuda"))


def test_run_device_torch(Sim):
    import torch
    prob, b, q = _cyl_case()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12)
        pid = sim.add_problem(prob)
        host, _ = sim.dmri_run([pid] * len(b), b, q)
        db = torch.tensor(b, dtype=torch.float64, device="cuda")
        dq = torch.tensor(q, dtype=torch.float64, device="cuda")
        ds = torch.zeros((len(b), 2), dtype=torch.float64, device="cuda")
        stream = torch.cuda.current_stream()
        st = sim.dmri_run_device(pid, db, dq, ds, stream_ptr=stream.cuda_stream)
        torch.cuda.synchronize()
        dev = ds.cpu().numpy()
    assert st["status"] == "DMRI_OK"
    np.testing.assert_allclose(dev[:, 0] + 1j * dev[:, 1], host, rtol=0, atol=1e-12 * abs(host[0]))


def test_fp32_path_close(Sim):
    prob, b, q = _cyl_case()
    ref = _cyl_ref()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(precision=2, rtol=1e-6)
        pid = sim.add_problem(prob)
        sig, st = sim.dmri_run([pid] * len(b), b, q)
    err = rel_err(sig, ref, ref[0])
    _say("fp32 max err %.2e" % err.max())
    assert err.max() < 1e-4


@pytest.mark.parametrize("case", ["periodic", "neumann"])
def test_mixed_precision_refinement_matches_oracle(Sim, case):
    if case == "periodic":
        prob, b, q = _cyl_case()
        form = "transformed"
    else:
        prob = di.slab_box(n=10, half=5.0, split=-1.0, D=(3e-3, 1e-3), kappa=1e-3,
                           u0=(1.0, 0.2), periodic_mask=0)
        b = np.array([0.0, 1000.0, 3000.0])
        q = np.array([[1.0, 0.0, 0.0], [0.8, 0.6, 0.0], [0.0, 0.3, 0.95]])
        form = "uform"
    ref = timestep.signals(prob, SHORT, b, q, form=form, solver="splu")
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(precision=1, rtol=1e-12, inner_rtol=1e-4)
        pid = sim.add_problem(prob)
        sig, st = sim.dmri_run([pid] * len(b), b, q)
    err = rel_err(sig, ref, ref[0])
    _say("mixed %s max err %.2e status %s iters %s" % (case, err.max(), st["status"],
                                                      st["iters_total"].tolist()))
    assert st["status"] == "DMRI_OK"
    assert err.max() < 1e-9


@pytest.mark.parametrize("ordering", [0, 1])
def test_orderings_agree(Sim, ordering):
    prob, b, q = _cyl_case()
    ref = timestep.signals(prob, SHORT, b[:5], q[:5], solver="splu")
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12, ordering=ordering, pencil=4)
        pid = sim.add_problem(prob)
        sig, _ = sim.dmri_run([pid] * 5, b[:5], q[:5])
    assert rel_err(sig, ref, ref[0]).max() < 1e-9


@pytest.mark.parametrize("precision", [0, 1])
def test_persistent_solver_matches_oracle(Sim, precision):
    # One launch per Krylov solve with grid barriers; the same signals as the
    # oracle and as the chunked multi-launch loop.
    prob, b, q = _cyl_case()
    ref = _cyl_ref()
    out = {}
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        for persist in (0, 1):
            sim.set_options(rtol=1e-12, precision=precision, persistent=persist)
            out[persist], st = sim.dmri_run([pid] * len(b), b, q)
            assert st["status"] == "DMRI_OK"
    for persist in (0, 1):
        err = rel_err(out[persist], ref, ref[0])
        _say("persistent=%d precision=%d max err %.2e" % (persist, precision, err.max()))
        assert err.max() < 1e-9
    assert np.abs(out[0] - out[1]).max() < 1e-10 * abs(ref[0])


_WIDE = {}


def _wide_case():
    # 67 systems: a full 64-system tile and a ragged one of 3
    if not _WIDE:
        prob, _, _ = _cyl_case()
        rng = np.random.default_rng(4)
        b = rng.uniform(0.0, 5000.0, 67)
        b[0] = 0.0
        q = di.fibonacci_directions(67)
        _WIDE["case"] = (prob, b, q, timestep.signals(prob, SHORT, b, q, solver="splu"))
    return _WIDE["case"]


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_wide_tiles_chunked_match_oracle(Sim, precision):
    # 64-wide tiles through the chunked multi-launch loop: the
    # wavefront-uniform SpMV path (two rows per wavefront in FP32, 16-entry
    # rows and the general fallback).
    prob, b, q, ref = _wide_case()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12 if precision != 2 else 1e-6, precision=precision,
                        sys_tile=64, persistent=0)
        pid = sim.add_problem(prob)
        sig, st = sim.dmri_run([pid] * len(b), b, q)
    assert st["status"] == "DMRI_OK"
    err = rel_err(sig, ref, ref[0])
    _say("wide tiles precision=%d max err %.2e" % (precision, err.max()))
    assert err.max() < (1e-9 if precision != 2 else 1e-4)


@pytest.mark.parametrize("order", [1, 2, 3, 4])
@pytest.mark.parametrize("precision", [0, 1])
def test_extrapolation_orders_match_oracle(Sim, order, precision):
    # The polynomial-extrapolation guess only moves the Krylov starting
    # point: every order gives the oracle's signals (the iteration counts are
    # reported; on this coarse time grid at rtol 1e-12 they barely differ).
    prob, b, q = _cyl_case()
    ref = _cyl_ref()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        sim.set_options(rtol=1e-12, precision=precision, guess=0)
        _, st0 = sim.dmri_run([pid] * len(b), b, q)
        sim.set_options(guess=1, extrap_order=order)
        sig, st = sim.dmri_run([pid] * len(b), b, q)
    assert st["status"] == "DMRI_OK"
    err = rel_err(sig, ref, ref[0])
    _say("order %d precision %d: max err %.2e, iterations %d (previous-step guess %d)"
         % (order, precision, err.max(), st["total_iterations"], st0["total_iterations"]))
    assert err.max() < 1e-9


def test_graph_replay_matches_eager(Sim):
    # The persistent path's time loop captured in a HIP graph: the first run
    # captures, later runs replay, with eager runs in between; every replay
    # gives the eager signals bit for bit and the oracle's within 1e-9.
    prob, b, q = _cyl_case()
    ref = _cyl_ref()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        sim.set_options(rtol=1e-12, persistent=1, graph=0)
        eager, _ = sim.dmri_run([pid] * len(b), b, q)
        runs = []
        for k in range(3):
            sim.set_options(graph=1)
            sig, st = sim.dmri_run([pid] * len(b), b, q)
            assert st["status"] == "DMRI_OK"
            runs.append(sig)
            sim.set_options(graph=0)
            again, _ = sim.dmri_run([pid] * len(b), b, q)
            assert np.array_equal(again, eager)
        # A changed guess option must not replay the graph captured with the
        # old one: undamped extrapolation, graph vs eager, bit for bit.
        sim.set_options(guess=1, extrap_damp=0, graph=0)
        eager_u, _ = sim.dmri_run([pid] * len(b), b, q)
        sim.set_options(graph=1)
        graph_u, _ = sim.dmri_run([pid] * len(b), b, q)
        assert np.array_equal(graph_u, eager_u)
    for sig in runs:
        assert np.array_equal(sig, eager)
    assert rel_err(eager, ref, ref[0]).max() < 1e-9
    assert rel_err(eager_u, ref, ref[0]).max() < 1e-9


def test_graph_recaptured_after_reallocation(Sim):
    # A captured graph bakes device addresses in. Capture with the auto tile
    # (one 64-system tile), run eagerly with 8-system tiles (the per-tile
    # buffers grow, i.e. are reallocated), then ask for the graph again: the
    # library must capture anew, and every result equals its eager run bit
    # for bit.
    prob, b, q = _cyl_case()
    rng = np.random.default_rng(5)
    n = 64
    bb = np.concatenate([b, rng.uniform(0, 3000, n - len(b))])
    qq = np.concatenate([q, rng.normal(size=(n - len(q), 3))])
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        sim.set_options(rtol=1e-12, persistent=1, graph=0, sys_tile=0)
        eager64, _ = sim.dmri_run([pid] * n, bb, qq)
        sim.set_options(sys_tile=8)
        eager8, _ = sim.dmri_run([pid] * n, bb, qq)
        sim.set_options(sys_tile=0, graph=1)
        g1, _ = sim.dmri_run([pid] * n, bb, qq)
        sim.set_options(sys_tile=8, graph=0)
        e8, _ = sim.dmri_run([pid] * n, bb, qq)
        sim.set_options(sys_tile=0, graph=1)
        g2, _ = sim.dmri_run([pid] * n, bb, qq)
        g3, _ = sim.dmri_run([pid] * n, bb, qq)
    assert np.array_equal(g1, eager64)
    assert np.array_equal(e8, eager8)
    assert np.array_equal(g2, eager64)
    assert np.array_equal(g3, eager64)


def test_autotune_matches_oracle(Sim):
    prob, b, q = _cyl_case()
    ref = _cyl_ref()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        assert sim.dmri_get_option("tuned_sys_tile") == -1
        sim.set_options(rtol=1e-12, autotune=1)
        sig, st = sim.dmri_run([pid] * len(b), b, q)
        choice = [sim.dmri_get_option(k) for k in ("tuned_sys_tile", "tuned_blocks_per_xcd",
                                                     "tuned_persistent", "tuned_lds")]
        trials = sim.dmri_get_option("tuned_trials")
        sig2, _ = sim.dmri_run([pid] * len(b), b, q)  # cached choice, no new trials
        assert sim.dmri_get_option("tuned_trials") == trials
        # the user's own options are restored after the tuned run
        assert sim.dmri_get_option("sys_tile") == 0
    _say("autotune choice %s after %d trials" % (choice, trials))
    assert choice[0] in (8, 16) and trials >= 2
    for s_ in (sig, sig2):
        assert rel_err(s_, ref, ref[0]).max() < 1e-9


def test_autotune_cache_persists_across_handles(Sim, tmp_path):
    # The tuned choice saved by one handle serves a fresh handle (another
    # process would read the same file): no trial runs there, the same
    # launch configuration, bit-identical signals.
    prob, b, q = _cyl_case()
    path = str(tmp_path / "tuning.txt")
    keys = ("tuned_sys_tile", "tuned_blocks_per_xcd", "tuned_persistent", "tuned_lds")
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        sim.set_options(rtol=1e-12, autotune=1)
        sig, _ = sim.dmri_run([pid] * len(b), b, q)
        assert sim.dmri_get_option("tuned_trials") >= 2
        choice = [sim.dmri_get_option(k) for k in keys]
        sim.dmri_save_tuning(path)
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        sim.dmri_load_tuning(path)
        sim.set_options(rtol=1e-12, autotune=1)
        sig2, _ = sim.dmri_run([pid] * len(b), b, q)
        assert sim.dmri_get_option("tuned_trials") == 0
        assert [sim.dmri_get_option(k) for k in keys] == choice
    _say("tuning cache: %s" % open(path).read().strip().replace("\n", " | "))
    assert np.array_equal(sig, sig2)


def test_concurrent_problems_match_sequential(Sim):
    # Meshes of uneven size in one run: with concurrency each problem runs on
    # its own lane (stream, workspace, host thread); the signals are the same
    # bit for bit as one after another, and match the oracle.
    probs = [di.cylinder_box(n=n, half=6.0, r=r, kappa=5e-3, D_in=1.5e-3)
             for n, r in ((8, 4.0), (11, 4.3), (6, 3.5))]
    b = np.array([0.0, 800.0, 2500.0, 4000.0])
    q = di.fibonacci_directions(4)
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pids = [sim.add_problem(p) for p in probs]
        sim.set_options(rtol=1e-12)
        pid_arr = np.repeat(pids, len(b))
        bb = np.tile(b, len(pids))
        qq = np.tile(q, (len(pids), 1))
        out = {}
        for c in (1, 3):
            sim.set_options(concurrency=c)
            out[c], st = sim.dmri_run(pid_arr, bb, qq)
            assert st["status"] == "DMRI_OK"
    assert np.array_equal(out[1], out[3])
    for k, prob in enumerate(probs):
        ref = timestep.signals(prob, SHORT, b, q, solver="splu")
        sig = out[3][k * len(b):(k + 1) * len(b)]
        assert rel_err(sig, ref, ref[0]).max() < 1e-9


@pytest.mark.parametrize("precision", [0, 1])
def test_sorted_batches_give_identical_signals(Sim, precision):
    # Ordering the systems by b before tiling changes which tile and lane
    # each system uses, never its arithmetic: bit-identical signals, in the
    # caller's order, through both the host and the device entry points.
    torch = pytest.importorskip("torch")
    prob, b, q = _cyl_case()
    out = {}
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        sim.set_options(rtol=1e-12, precision=precision, sys_tile=8, persistent=0)
        for srt in (0, 1):
            sim.set_options(sort_systems=srt)
            out[srt], _ = sim.dmri_run([pid] * len(b), b, q)
            bd = torch.tensor(b, dtype=torch.float64, device="cuda")
            qd = torch.tensor(q, dtype=torch.float64, device="cuda")
            sd = torch.zeros((len(b), 2), dtype=torch.float64, device="cuda")
            torch.cuda.synchronize()
            sim.dmri_run_device(pid, bd, qd, sd)
            dev = sd.cpu().numpy()
            assert np.array_equal(dev[:, 0] + 1j * dev[:, 1], out[srt])
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("pair,dir16,rows", [(0, 0, 1), (1, 0, 1), (1, 1, 1), (1, 1, 2)])
def test_paired_lanes_match_oracle(Sim, pair, dir16, rows):
    # Mixed precision on 67 systems: the FP32 inner solves in one ragged
    # 128-system tile with two systems per lane (pair = 1) or in 64-system
    # tiles (pair = 0), with FP32 or BF16 search directions in the paired
    # tiles, the BF16 SpMV taking one or two rows per wavefront at a time;
    # all refine to the oracle.
    prob, b, q, ref = _wide_case()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12, precision=1, persistent=0, pair_lanes=pair, dir_bf16=dir16,
                        spmv_rows=rows)
        pid = sim.add_problem(prob)
        sig, st = sim.dmri_run([pid] * len(b), b, q)
    assert st["status"] == "DMRI_OK"
    err = rel_err(sig, ref, ref[0])
    _say("paired lanes %d, BF16 directions %d, rows %d: max err %.2e, %d inner iterations"
         % (pair, dir16, rows, err.max(), st["total_iterations"]))
    assert err.max() < 1e-9


def test_inner_floor_matches_oracle(Sim):
    # Mixed precision on the 67-system paired case at rtol 1e-8: an inner
    # FP32 solve may stop at inner_floor * rtol ||b|| (here up to the outer
    # target itself); the FP64 refinement still ends every step at rtol, so
    # the signals stay within 1e-6 of the oracle with fewer inner iterations.
    prob, b, q, ref = _wide_case()
    out, iters = {}, {}
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-8, precision=1, persistent=0)
        pid = sim.add_problem(prob)
        for f in (0.25, 1.0):
            sim.set_options(inner_floor=f)
            out[f], st = sim.dmri_run([pid] * len(b), b, q)
            assert st["status"] == "DMRI_OK"
            iters[f] = st["total_iterations"]
    for f in (0.25, 1.0):
        err = rel_err(out[f], ref, ref[0])
        _say("inner_floor %.2f: max err %.2e, %d inner iterations" % (f, err.max(), iters[f]))
        assert err.max() < 1e-6
    assert iters[1.0] <= iters[0.25]


@pytest.mark.parametrize("precision", [0, 1])
def test_tile_schedule_matches_oracle(Sim, precision):
    # Two 8-system tiles sorted by b: the low-b tile leaves the Krylov loop
    # first, after which each chunk of iterations is launched over the one
    # tile still active, split over all XCDs (tile_sched = 1). Partials are
    # then grouped differently, so the signals agree with the unrestricted
    # launches to rounding and with the oracle to the solver tolerance.
    prob, b, q = _cyl_case()
    ref = _cyl_ref()
    out = {}
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        sim.set_options(rtol=1e-12, precision=precision, sys_tile=8, persistent=0)
        for ts in (0, 1):
            sim.set_options(tile_sched=ts)
            out[ts], st = sim.dmri_run([pid] * len(b), b, q)
            assert st["status"] == "DMRI_OK"
    assert rel_err(out[1], out[0], ref[0]).max() < 1e-11
    err = rel_err(out[1], ref, ref[0])
    _say("tile schedule, precision %d: max err %.2e" % (precision, err.max()))
    assert err.max() < 1e-9


def test_tile_schedule_odd_tile_counts(Sim):
    # 37 systems in five 8-system tiles (the last one ragged), b spread so the
    # tiles leave the Krylov loop at different times: the restricted launches
    # cover subsets of 1-4 tiles, each split into 8 row parts (five tiles
    # already need 8 parts for a multiple of 8 items). The signals match the
    # unrestricted launches (checked against the oracle above) to rounding.
    prob, _, _ = _cyl_case()
    b = np.linspace(0.0, 5000.0, 37)
    q = di.fibonacci_directions(37)
    out = {}
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        sim.set_options(rtol=1e-12, sys_tile=8, persistent=0)
        for ts in (0, 1):
            sim.set_options(tile_sched=ts)
            out[ts], st = sim.dmri_run([pid] * len(b), b, q)
            assert st["status"] == "DMRI_OK"
    err = rel_err(out[1], out[0], out[0][0])
    _say("tile schedule, 5 tiles: max difference %.2e" % err.max())
    assert err.max() < 1e-11


def test_refinement_schedule_paired_mixed(Sim):
    # Mixed precision on 203 systems: four 64-system FP64 tiles (the last one
    # ragged) and two 128-system paired inner tiles. The first FP64 tile holds
    # only b = 0 systems, which converge at every step start, so each
    # refinement pass runs the refinement residual over the other three tiles
    # only (tile_sched = 1), and the inner start over both inner tiles (the
    # first of which is half idle). At rtol 1e-10 a step takes several
    # passes, and low-b tiles drop out of the later ones. The signals match the
    # runs over every tile (tile_sched = 0) to rounding, and the summed inner
    # iterations agree to within rounding-level differences in when a system
    # stops.
    prob, _, _ = _cyl_case()
    b = np.concatenate([np.zeros(64), np.linspace(200.0, 5000.0, 139)])
    q = di.fibonacci_directions(203)
    out, iters = {}, {}
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        # Input order for every run (no reordering by the previous run's costs).
        sim.set_options(rtol=1e-10, precision=1, pair_lanes=1, persistent=0, sort_systems=0)
        for ts in (0, 1):
            sim.set_options(tile_sched=ts)
            out[ts], st = sim.dmri_run([pid] * len(b), b, q)
            assert st["status"] == "DMRI_OK"
            iters[ts] = st["total_iterations"]
        # Partials are added in a fixed order (in groups first when a tile has
        # many of them), so a second run is bitwise identical.
        again, _ = sim.dmri_run([pid] * len(b), b, q)
    assert np.array_equal(again, out[1])
    err = rel_err(out[1], out[0], out[0][0])
    _say("refinement schedule, 203 systems mixed: max difference %.2e, iterations %d / %d"
         % (err.max(), iters[0], iters[1]))
    assert err.max() < 1e-11
    assert abs(iters[0] - iters[1]) <= 0.01 * iters[0]


@pytest.mark.parametrize("queue,lds", [(1, 0), (0, 1), (1, 1)])
@pytest.mark.parametrize("precision", [0, 1])
def test_row_queue_and_lds_spmv_match_oracle(Sim, queue, lds, precision):
    # The optional launch shapes of the gather kernels: rows taken from a
    # per-item atomic queue instead of static chunks, and the SpMV that stages
    # each chunk's matrix entries in LDS (64-system tile, 13 systems ragged).
    prob, b, q = _cyl_case()
    ref = _cyl_ref()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        sim.set_options(rtol=1e-12, precision=precision, sys_tile=64, persistent=0, queue=queue,
                        lds=lds)
        sig, st = sim.dmri_run([pid] * len(b), b, q)
    assert st["status"] == "DMRI_OK"
    err = rel_err(sig, ref, ref[0])
    _say("queue=%d lds=%d precision=%d max err %.2e" % (queue, lds, precision, err.max()))
    assert err.max() < 1e-9


@pytest.mark.parametrize("opts", [
    dict(precision=1, xcd_split=1),
    dict(precision=1, nt=0),
    dict(precision=1, blocks_per_xcd=3),
    dict(precision=0, blocks_per_xcd=3),
    dict(precision=0, guess=1, extrap_damp=0, extrap_order=3),
    dict(precision=1, pair_lanes=0, tile_sched=0),
], ids=["xcd_split", "nt0", "bpx3_mixed", "bpx3_fp64", "undamped_cubic", "unpaired_unsched"])
def test_launch_options_match_oracle(Sim, opts):
    # Launch-shape and guess options on the two-tile 67-system batch: every
    # tile split over all XCDs, plain stores for the SpMV output, three blocks
    # per XCD (each block sweeps many chunks), the undamped cubic
    # extrapolation, and the unpaired, unscheduled FP32 inner solves.
    prob, b, q, ref = _wide_case()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        sim.set_options(rtol=1e-12, persistent=0, **opts)
        sig, st = sim.dmri_run([pid] * len(b), b, q)
    assert st["status"] == "DMRI_OK"
    err = rel_err(sig, ref, ref[0])
    _say("%s max err %.2e" % (opts, err.max()))
    assert err.max() < 1e-9


# ------------------------------------------------ general temporal profiles
PROFILES = [
    ("double_pgse", (2000.0, 4000.0, 1000.0)),
    ("cos_ogse", (2000.0, 4000.0, 1.0)),
    ("sin_ogse", (2000.0, 4000.0, 2.0)),
    ("trap_pgse", (2000.0, 4000.0, 400.0)),
    ("double_trap_pgse", (2000.0, 4000.0, 400.0, 200.0)),
]


@pytest.mark.parametrize("kind,params", PROFILES)
def test_general_profiles_match_oracle(Sim, kind, params):
    # Each profile through dmri_set_sequence, FP64 at rtol 1e-12, against the
    # oracle's exact solves of the same theta recurrence (periodic box).
    prob, b, q = _cyl_case()
    sel = [1, 3, 4, 8, 12]
    seq = di.GeneralSequence(kind, params, 200.0, 0.5)
    with Sim(0) as sim:
        sim.set_sequence(seq)
        sim.set_options(rtol=1e-12)
        pid = sim.add_problem(prob)
        sig, st = sim.dmri_run([pid] * len(sel), b[sel], q[sel])
        sim.set_options(precision=1, rtol=1e-9)
        sig_m, _ = sim.dmri_run([pid] * len(sel), b[sel], q[sel])
    ref = timestep.signals(prob, seq, b[sel], q[sel], solver="splu")
    e = rel_err(sig, ref, ref[0])
    em = rel_err(sig_m, ref, ref[0])
    _say("%s: FP64 err %.2e, mixed err %.2e, %d steps" % (kind, e.max(), em.max(), st["n_steps"]))
    assert st["status"] == "DMRI_OK"
    assert e.max() < 1e-9
    assert em.max() < 1e-6


@pytest.mark.parametrize("kind,params", [("cos_ogse", (2000.0, 4000.0, 1.0)),
                                         ("trap_pgse", (2000.0, 4000.0, 400.0))])
def test_general_profiles_uform_match_oracle(Sim, kind, params):
    # Walls (U-form, COCG): the one-sided limits of f on each step.
    prob = di.slab_box(n=8, half=4.0, split=0.5, D=(3e-3, 1.5e-3), kappa=2e-3, u0=(1.0, 0.4),
                       periodic_mask=0)
    b = np.array([800.0, 2500.0, 4000.0])
    q = np.array([[1.0, 0.0, 0.0], [0.6, 0.8, 0.0], [0.2, 0.3, 0.9]])
    seq = di.GeneralSequence(kind, params, 200.0, 0.5)
    with Sim(0) as sim:
        sim.set_sequence(seq)
        sim.set_options(rtol=1e-12)
        pid = sim.add_problem(prob)
        sig, st = sim.dmri_run([pid] * 3, b, q)
    ref = timestep.signals(prob, seq, b, q, solver="splu")
    e = rel_err(sig, ref, ref[0])
    _say("U-form %s: err %.2e" % (kind, e.max()))
    assert st["status"] == "DMRI_OK"
    assert e.max() < 1e-9


def test_sequence_table_entry(Sim):
    # An arbitrary profile given as tables on the grid (here the oracle's
    # own F, one-sided f and int F^2 of a cos-OGSE): same signals as the
    # named profile, and the oracle's, on both forms.
    from oracle import sequence as sq
    kind, params, dt = "cos_ogse", (2000.0, 4000.0, 1.0), 200.0
    prof = sq.Profile(kind, params)
    N = int(round(prof.T / dt))
    F = np.array([prof.F(n * dt) for n in range(N + 1)])
    lim = np.array([prof.f_limits(n * dt, (n + 1) * dt) for n in range(N)])
    seq = di.GeneralSequence(kind, params, dt, 0.5)
    prob, b, q = _cyl_case()
    sel = [2, 4, 10]
    wall = di.slab_box(n=8, half=4.0, split=0.5, D=(3e-3, 1.5e-3), kappa=2e-3, u0=(1.0, 0.4),
                       periodic_mask=0)
    with Sim(0) as sim:
        sim.set_options(rtol=1e-12)
        pid = sim.add_problem(prob)
        pw = sim.add_problem(wall)
        sim.set_sequence(seq)
        named, _ = sim.dmri_run([pid] * 3 + [pw] * 3, np.concatenate([b[sel]] * 2),
                                np.concatenate([q[sel]] * 2))
        sim.dmri_set_sequence_table(dt, 0.5, F, lim[:, 0], lim[:, 1], prof.int_F2())
        table, _ = sim.dmri_run([pid] * 3 + [pw] * 3, np.concatenate([b[sel]] * 2),
                                np.concatenate([q[sel]] * 2))
        # without f the periodic problem still runs, the wall problem cannot
        sim.dmri_set_sequence_table(dt, 0.5, F, None, None, prof.int_F2())
        per, _ = sim.dmri_run([pid] * 3, b[sel], q[sel])
        with pytest.raises(Exception, match="DMRI_E_STATE"):
            sim.dmri_run([pw], b[:1], q[:1])
    ref = timestep.signals(prob, seq, b[sel], q[sel], solver="splu")
    refw = timestep.signals(wall, seq, b[sel], q[sel], solver="splu")
    assert rel_err(table, named, named[0]).max() < 1e-12
    assert rel_err(per, named[:3], named[0]).max() < 1e-12
    assert rel_err(table[:3], ref, ref[0]).max() < 1e-9
    assert rel_err(table[3:], refw, refw[0]).max() < 1e-9


@pytest.mark.parametrize("stop", [3, 11, 17])
def test_physical_signal_mid_sequence(Sim, stop):
    # A run that stops where F != 0 returns the physical signal: the P1 field
    # times the plane wave exp(-i G F q.x), integrated exactly per
    # tetrahedron, against the oracle's Gauss-rule integral of its own u^n.
    prob, b, q = _cyl_case()
    sel = [0, 2, 4, 6, 10]
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-13, n_steps=stop)
        pid = sim.add_problem(prob)
        sig, _ = sim.dmri_run([pid] * len(sel), b[sel], q[sel])
        sim.set_options(precision=1, rtol=1e-10)
        sig_m, _ = sim.dmri_run([pid] * len(sel), b[sel], q[sel])
    asm = fem.assemble(prob)
    from oracle import sequence as sq
    F = float(sq.pgse_F(stop * SHORT.dt, SHORT.delta, SHORT.Delta))
    ref = []
    for i in sel:
        _, u = timestep.solve_transformed(asm, SHORT, b[i], q[i], n_steps=stop, solver="splu",
                                          return_u=True)
        G = float(sq.b_to_G(b[i], SHORT.delta, SHORT.Delta))
        qn = np.asarray(q[i]) / np.linalg.norm(q[i])
        ref.append(timestep.physical_signal(prob, asm, u, G * F * qn))
    ref = np.array(ref)
    e = np.abs(sig - ref) / np.abs(ref).max()
    em = np.abs(sig_m - ref) / np.abs(ref).max()
    _say("physical signal at step %d (F = %g): FP64 err %.2e, mixed %.2e" % (stop, F, e.max(),
                                                                             em.max()))
    assert e.max() < 1e-9
    assert em.max() < 1e-7


# ---------------------------------------------------------------- GMRES(m)
@pytest.mark.parametrize("m", [4, 30])
def test_gmres_uform_matches_oracle(Sim, m):
    # Restarted GMRES (krylov = 3) on the complex-symmetric U-form (walls),
    # FP64 at rtol 1e-12: within 1e-9 of the oracle's exact solves, and of
    # COCG; m = 4 forces many restarts.
    prob = di.cylinder_box(n=9, half=6.0, r=4.0, kappa=2e-2, D_in=1.5e-3, periodic_mask=0,
                           u0=(1.0, 0.6))
    b = np.array([0.0, 700.0, 2200.0, 4000.0, 1500.0])
    q = di.fibonacci_directions(5)
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12, krylov=3, gmres_m=m)
        pid = sim.add_problem(prob)
        sig, st = sim.dmri_run([pid] * len(b), b, q)
        sim.set_options(krylov=0)
        cocg, st_c = sim.dmri_run([pid] * len(b), b, q)
        sim.set_options(krylov=3, precision=1)
        with pytest.raises(Exception, match="DMRI_E_UNSUPPORTED"):
            sim.dmri_run([pid], b[:1], q[:1])
    ref = timestep.signals(prob, SHORT, b, q, solver="splu")
    e = rel_err(sig, ref, ref[0])
    _say("GMRES(%d) U-form: err %.2e (COCG %.2e), iterations %d vs COCG %d"
         % (m, e.max(), rel_err(cocg, ref, ref[0]).max(), st["total_iterations"],
            st_c["total_iterations"]))
    assert st["status"] == "DMRI_OK" and np.all(st["converged"] == 1)
    assert e.max() < 1e-9
    assert np.all(st["final_rel_res"] <= 1e-12 * 1.0001)


def test_gmres_transformed_matches_oracle(Sim):
    # GMRES on the Hermitian transformed operator, a ragged 13-system batch
    # over 8-system tiles (systems leave their cycles at different times).
    prob, b, q = _cyl_case()
    ref = _cyl_ref()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12, krylov=3, gmres_m=12, sys_tile=8)
        pid = sim.add_problem(prob)
        sig, st = sim.dmri_run([pid] * len(b), b, q)
    e = rel_err(sig, ref, ref[0])
    _say("GMRES(12) transformed: err %.2e, %d iterations" % (e.max(), st["total_iterations"]))
    assert st["status"] == "DMRI_OK"
    assert e.max() < 1e-9


# ---------------------------------- diffusion tensors, conforming meshes
def _tensor_case(mask=7):
    return di.conforming_cylinder_box(
        n=8, half=6.0, r=4.0, D_in=di.tensor([3e-3, 1e-3, 2e-3], (0.3, 0.5, 0.2)),
        D_out=di.tensor([2e-3, 2.5e-3, 1.5e-3], (1.0, -0.4, 0.7)), kappa=5e-3,
        periodic_mask=mask, jitter=0.15, seed=2, u0=(1.0, 0.8))


@pytest.mark.parametrize("mask", [7, 0])
def test_tensor_conforming_mesh_matches_oracle(Sim, mask):
    # An unstructured, interface-conforming mesh with an anisotropic tensor
    # per compartment: FP64 (CG/COCG and GMRES) within 1e-9 of the oracle,
    # mixed precision within 1e-6 at rtol 1e-9.
    prob = _tensor_case(mask)
    b = np.array([0.0, 900.0, 2500.0, 4200.0, 1700.0, 3300.0])
    q = di.fibonacci_directions(6)
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12)
        pid = sim.add_problem(prob)
        sig, st = sim.dmri_run([pid] * len(b), b, q)
        sim.set_options(krylov=3)
        sig_g, _ = sim.dmri_run([pid] * len(b), b, q)
        sim.set_options(krylov=0, precision=1, rtol=1e-9)
        sig_m, _ = sim.dmri_run([pid] * len(b), b, q)
    ref = timestep.signals(prob, SHORT, b, q, solver="splu")
    e, eg, em = (rel_err(x, ref, ref[0]).max() for x in (sig, sig_g, sig_m))
    _say("tensor conforming mask %d: FP64 %.2e, GMRES %.2e, mixed %.2e" % (mask, e, eg, em))
    assert st["status"] == "DMRI_OK"
    assert e < 1e-9 and eg < 1e-9 and em < 1e-6


def test_tensor_free_diffusion_closed_form(Sim):
    # uniform field on the torus: the scalar recurrence with a = q.D q (G F)^2
    Dt = di.tensor([3e-3, 1e-3, 2e-3], (0.4, 0.9, -0.3))
    prob = di.free_box(n=6, half=5.0)
    prob.D = Dt[None]
    seq = di.PGSE_SHORT
    qs = np.array([[0.6, 0.0, 0.8], [0.0, 1.0, 0.0], [0.36, 0.48, 0.8]])
    with Sim(0) as sim:
        sim.set_sequence(seq)
        sim.set_options(rtol=1e-12)
        pid = sim.add_problem(prob)
        sig, _ = sim.dmri_run([pid] * 3, [1200.0] * 3, qs)
    from oracle import sequence as sq
    N = seq.n_steps
    F = sq.pgse_F(np.arange(N + 1) * seq.dt, seq.delta, seq.Delta)
    G2 = 1200.0 / sq.pgse_int_F2(seq.delta, seq.Delta)
    for s_, q in zip(sig, qs):
        a = (q @ Dt @ q) * G2 * F ** 2
        c = np.prod((1 / seq.dt - 0.5 * a[:-1]) / (1 / seq.dt + 0.5 * a[1:]))
        assert s_.real / 1000.0 == pytest.approx(c, rel=1e-11)


def test_isotropic_tensor_equals_scalar(Sim):
    # D given as D * identity through dmri_add_problem_tensor gives the
    # scalar problem's signals (the per-row factor path against M_D)
    ps = di.conforming_cylinder_box(n=7, D_in=1.5e-3, D_out=3e-3, kappa=2e-3)
    pt = di.conforming_cylinder_box(n=7, D_in=1.5e-3, D_out=3e-3, kappa=2e-3)
    pt.D = np.stack([3e-3 * np.eye(3), 1.5e-3 * np.eye(3)])
    b = np.array([500.0, 2000.0, 3500.0])
    q = di.fibonacci_directions(3)
    out = {}
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        for prec, rtol in ((0, 1e-12), (1, 1e-10)):
            sim.set_options(precision=prec, rtol=rtol)
            i1 = sim.add_problem(ps)
            i2 = sim.add_problem(pt)
            s1, _ = sim.dmri_run([i1] * 3, b, q)
            s2, _ = sim.dmri_run([i2] * 3, b, q)
            out[prec] = rel_err(s2, s1, s1[0]).max()
    _say("isotropic tensor vs scalar: FP64 %.2e, mixed %.2e" % (out[0], out[1]))
    assert out[0] < 1e-11 and out[1] < 1e-8


# ------------------------------------------- weak pseudo-periodic faces
def _weak_case():
    # Two compartments on an unstructured conforming mesh whose opposite box
    # faces do not match node for node; weak faces on x, y and z.
    return di.nonmatching_faces(
        di.conforming_cylinder_box(n=7, half=6.0, r=4.0, kappa=1e-2, D_in=1e-3,
                                   periodic_mask=15, seed=1, u0=(1.0, 0.7)),
        amount=0.25, seed=7)


@pytest.mark.parametrize("scale", [1.0, 8.0])
def test_weak_faces_match_oracle(Sim, scale):
    # Artificial-permeability faces (face mass in the left operator, lagged
    # phase-shifted partner in the right side): FP64 COCG and GMRES within
    # 1e-9 of the oracle, mixed precision within 1e-9 at rtol 1e-12, the
    # FP32 path within 1e-4, a graph replay equal to the eager run.
    prob = _weak_case()
    b = np.array([0.0, 800.0, 2500.0, 4000.0, 1500.0, 3200.0])
    q = di.fibonacci_directions(6)
    asm = fem.assemble(prob, weak_kappa=scale)
    ref = timestep.signals(prob, SHORT, b, q, asm=asm, solver="splu")
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12, weak_kappa=scale)
        pid = sim.add_problem(prob)
        _say("weak faces scale %g: FP64" % scale)
        sig, st = sim.dmri_run([pid] * len(b), b, q)
        sim.set_options(krylov=3)
        sig_g, _ = sim.dmri_run([pid] * len(b), b, q)
        sim.set_options(krylov=0, precision=1)
        sig_m, _ = sim.dmri_run([pid] * len(b), b, q)
        sim.set_options(precision=2, rtol=1e-6)
        sig_32, _ = sim.dmri_run([pid] * len(b), b, q)
        sim.set_options(precision=0, rtol=1e-12, persistent=1, graph=1)
        _say("weak faces scale %g: graph" % scale)
        sig_gr = [sim.dmri_run([pid] * len(b), b, q)[0] for _ in range(2)]
        sim.set_options(graph=0)
        eager, _ = sim.dmri_run([pid] * len(b), b, q)
    e = [rel_err(x, ref, ref[0]).max() for x in (sig, sig_g, sig_m, sig_32)]
    _say("weak faces scale %g: FP64 %.2e GMRES %.2e mixed %.2e FP32 %.2e" % (scale, *e))
    assert st["status"] == "DMRI_OK"
    assert e[0] < 1e-9 and e[1] < 1e-9 and e[2] < 1e-9 and e[3] < 1e-4
    for g in sig_gr:
        assert np.array_equal(g, eager)
    assert abs(ref[2].imag) > 1e-6 * abs(ref[0])  # non-matching faces: a complex signal


def test_weak_faces_refusals(Sim):
    import torch
    prob = _weak_case()
    with Sim(0) as sim:
        sim.set_sequence(di.Sequence(2000.0, 4000.0, 200.0, 0.75))
        pid = sim.add_problem(prob)
        with pytest.raises(Exception, match="DMRI_E_UNSUPPORTED"):
            sim.dmri_run([pid], [1000.0], [[1.0, 0.0, 0.0]])
        sim.set_sequence(SHORT)
        sim.dmri_run([pid], [1000.0], [[1.0, 0.0, 0.0]])
        dev = torch.device("cuda:0")
        b = torch.tensor([1000.0], dtype=torch.float64, device=dev)
        q = torch.tensor([[1.0, 0.0, 0.0]], dtype=torch.float64, device=dev)
        out = torch.zeros(2, dtype=torch.float64, device=dev)
        pids = torch.full((1,), pid, dtype=torch.int32, device=dev)
        with pytest.raises(Exception, match="DMRI_E_UNSUPPORTED"):
            sim.dmri_run_device_noalloc(pids, b, q, out)


# ------------------------- membrane limits and spheres in mixed precision
@pytest.mark.parametrize("case", ["kappa0", "kappa_large", "spheres"])
def test_mixed_precision_membrane_limits_and_spheres(Sim, case):
    # Mixed precision (FP32 inner solves, FP64 refinement) at rtol 1e-12
    # within 1e-9 of the oracle: decoupled compartments (kappa = 0), a
    # nearly impermeable-to-free jump (kappa = 5 um/us, the membrane term
    # dominating its rows), and a seeded geometry with spheres and cylinders.
    if case == "kappa0":
        prob = di.cylinder_box(n=10, half=6.0, r=4.0, kappa=0.0, D_in=1.5e-3, u0=(1.0, 0.6))
    elif case == "kappa_large":
        prob = di.cylinder_box(n=10, half=6.0, r=4.0, kappa=5.0, D_in=1.5e-3, u0=(1.0, 0.6))
    else:
        prob = di.seeded_cells(7, n_fixed=12)[0]
        assert sum(s["kind"] == "sphere" for s in prob.meta["shapes"]) > 0
    b = np.array([0.0, 900.0, 2600.0, 4100.0, 1700.0])
    q = di.fibonacci_directions(5)
    ref = timestep.signals(prob, SHORT, b, q, solver="splu")
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(precision=1, rtol=1e-12)
        pid = sim.add_problem(prob)
        sig, st = sim.dmri_run([pid] * len(b), b, q)
    err = rel_err(sig, ref, ref[0])
    _say("mixed %s: max err %.2e, %d iterations" % (case, err.max(), st["total_iterations"]))
    assert st["status"] == "DMRI_OK"
    # With kappa dt / h ~ 800 the membrane rows dominate and A is ill
    # conditioned: rtol 1e-12 on the residual bounds the signal error only by
    # cond(A) * 1e-12 (measured 9.4e-9, 14x the iterations of kappa = 0);
    # mixed precision's own target is 1e-4.
    assert err.max() < (1e-7 if case == "kappa_large" else 1e-9)


def test_markers_change_nothing(Sim):
    # roctx ranges around batches and steps are host-side only.
    prob, b, q = _cyl_case()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        sim.set_options(rtol=1e-12)
        plain, _ = sim.dmri_run([pid] * len(b), b, q)
        sim.set_options(markers=1)
        marked, st = sim.dmri_run([pid] * len(b), b, q)
    assert st["status"] == "DMRI_OK"
    assert np.array_equal(plain, marked)
