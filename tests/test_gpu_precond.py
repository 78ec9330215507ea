"""GPU tests of the polynomial preconditioner inside flexible CG (options
"precond", "cheb_terms", "cheb_a", "cheb_b") and of its interval network's
recorder and training, through the C ABI.

* flexible CG with the Chebyshev preconditioner on a fixed interval reaches
  the oracle's exact-solve signals within 1e-9 (FP64, rtol 1e-12) for
  several term counts, tile widths and a ragged batch; with one term it is
  scaled Jacobi and takes Jacobi CG's iterations;
* on the first step (previous-step guess) its per-system iteration counts
  equal those of the oracle's FCG (oracle/precond.py) on the same systems;
* the recorder's features and Ritz-value targets equal the oracle's
  definitions from its own PCG coefficients on the same first-step systems;
* a network with zero weights and output bias y gives the interval
  [0.5 e^y0, 1.5 e^y1] (same iterations and signals as that fixed interval);
* an interval far below the spectrum makes the flexible solve hit max_iter,
  and the step is solved again by Jacobi CG (signals still within 1e-9);
* trained on recorded samples of some systems, the learned interval keeps
  the answer and its effect on the iterations is measured, on other systems
  of the same mesh and on a held-out geometry;
* diffusion tensors on a conforming mesh and the autotuner's launch shapes
  keep the answer;
* unsupported combinations are refused.
"""

import math

import numpy as np
import pytest

import dmri_inputs as di
from oracle import fem, precond as opc, sequence as oseq, timestep

pytestmark = pytest.mark.gpu

SHORT = di.Sequence(2000.0, 4000.0, 200.0, 0.5)


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_01719_amd import Simulator
    return torch, Simulator


def _say(msg):
    print(msg, flush=True)


def rel_err(s, ref, s0):
    floor = np.maximum(np.abs(ref), 1e-8 * abs(s0))
    return np.abs(s - ref) / floor


def _case(n_sys=13, seed=0):
    prob = di.cylinder_box(n=11, half=6.0, r=4.3, kappa=5e-3, D_in=1.5e-3, T2=(6e4, 4e4),
                           u0=(1.0, 0.7))
    rng = np.random.default_rng(seed)
    b = rng.uniform(200.0, 5000.0, n_sys)
    b[0] = 0.0
    q = di.fibonacci_directions(n_sys)
    return prob, b, q


_REF = {}


def _ref(n_sys=13):
    if n_sys not in _REF:
        prob, b, q = _case(n_sys)
        _REF[n_sys] = timestep.signals(prob, SHORT, b, q, solver="splu")
    return _REF[n_sys].copy()


def _run(Sim, prob, b, q, **opts):
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(**opts)
        pid = sim.add_problem(prob)
        sig, st = sim.dmri_run([pid] * len(b), b, q)
        fb = sim.dmri_get_option("pc_fallback_steps")
    assert st["status"] == "DMRI_OK"
    return sig, st, fb


@pytest.mark.parametrize("terms,interval,tile,n_sys", [
    (1, (0.5, 1.5), 0, 13), (3, (0.4, 1.8), 8, 13), (4, (0.5, 1.5), 16, 21),
    (6, (0.3, 2.0), 0, 13), (4, (0.2, 1.2), 8, 21)])
def test_fixed_interval_matches_oracle(env, terms, interval, tile, n_sys):
    # (the last interval cuts the top of the spectrum: the polynomial is then
    # not positive there, and flexible CG still converges)
    torch, Sim = env
    _say("fixed interval terms=%d interval=%s tile=%d n_sys=%d" % (terms, interval, tile, n_sys))
    prob, b, q = _case(n_sys)
    ref = _ref(n_sys)
    sig, st, fb = _run(Sim, prob, b, q, rtol=1e-12, precond=2, cheb_terms=terms,
                       cheb_a=interval[0], cheb_b=interval[1], sys_tile=tile)
    err = rel_err(sig, ref, ref[0])
    _say("  max err %.2e, iterations %d, fallback steps %d" % (err.max(),
                                                               st["total_iterations"], fb))
    assert err.max() < 1e-9
    assert fb == 0


def test_one_term_is_jacobi(env):
    torch, Sim = env
    prob, b, q = _case()
    sig0, st0, _ = _run(Sim, prob, b, q, rtol=1e-12, precond=0, persistent=0)
    sig1, st1, _ = _run(Sim, prob, b, q, rtol=1e-12, precond=2, cheb_terms=1)
    d = np.abs(st0["iters_total"] - st1["iters_total"])
    _say("one term: iterations %s vs %s" % (st0["iters_total"].tolist(),
                                             st1["iters_total"].tolist()))
    assert d.max() <= 2
    assert np.max(np.abs(sig0 - sig1) / np.abs(sig0)) < 1e-10


def _max_edge(prob):
    t = prob.tets
    e = 0.0
    for i in range(4):
        for j in range(i + 1, 4):
            e = max(e, float(np.max(np.linalg.norm(prob.xyz[t[:, i]] - prob.xyz[t[:, j]],
                                                   axis=1))))
    return e


def _first_step_systems(prob, b, q):
    asm = fem.assemble(prob)
    out = []
    for s in range(len(b)):
        A, R = opc.step_operator(asm, SHORT, float(b[s]), q[s], 1)
        u0 = asm.u0.astype(np.complex128)
        out.append((A, R @ u0, u0))
    return out


def test_first_step_iterations_match_oracle(env):
    torch, Sim = env
    prob, b, q = _case(9)
    terms, (lo, hi) = 4, (0.45, 1.6)
    _, st, _ = _run(Sim, prob, b, q, rtol=1e-10, precond=2, cheb_terms=terms, cheb_a=lo,
                    cheb_b=hi, n_steps=1, signal=0, guess=0, sort_systems=0)
    want = []
    for A, rhs, x0 in _first_step_systems(prob, b, q):
        dinv = 1.0 / A.diagonal().real
        _, it = opc.fcg(A, rhs, x0, 1e-10,
                        lambda r: opc.chebyshev_apply(A, dinv, r, lo, hi, terms))
        want.append(it)
    got = st["iters_total"]
    _say("first step FCG iterations GPU %s oracle %s" % (got.tolist(), want))
    assert np.max(np.abs(np.asarray(got) - np.asarray(want))) <= 1


def test_recorder_matches_oracle(env):
    torch, Sim = env
    prob, b, q = _case(9)
    b = b[1:]  # b = 0 systems converge at once and give no sample
    q = q[1:]
    n = len(b)
    X = torch.zeros((64, 16), dtype=torch.float32, device="cuda")
    T = torch.zeros((64, 2), dtype=torch.float32, device="cuda")
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-10, precond=0, n_steps=1, signal=0, guess=0, sort_systems=0)
        pid = sim.add_problem(prob)
        sim.dmri_precond_record(X, T, 64)
        _, st = sim.dmri_run([pid] * n, b, q)
        cnt = sim.dmri_precond_record_count()
    assert st["status"] == "DMRI_OK"
    assert cnt == n
    Xg = X[:n].cpu().numpy().astype(np.float64)
    Tg = T[:n].cpu().numpy().astype(np.float64)
    prof = oseq.profile_of(SHORT)
    F1 = prof.F(SHORT.dt)
    h = _max_edge(prob)
    dmax = float(np.max(prob.D))
    for s, (A, rhs, x0) in enumerate(_first_step_systems(prob, b, q)):
        _, al, be = opc.pcg_coefficients(A, rhs, x0, 1e-10)
        assert len(al) == st["iters_total"][s]
        t_ref = opc.targets_from_ritz(*opc.ritz_extremes(al, be))
        G = math.sqrt(b[s] / prof.int_F2())
        f_ref = opc.features(SHORT.dt, SHORT.theta, dmax, h, prob.kappa, G, F1, q[s])
        _say("sample %d: targets %s oracle %s" % (s, Tg[s].tolist(), list(t_ref)))
        np.testing.assert_allclose(Tg[s], t_ref, rtol=0, atol=2e-5)
        np.testing.assert_allclose(Xg[s], f_ref, rtol=2e-6, atol=2e-6)


def _const_net(y0, y1):
    theta = np.zeros(5378, np.float32)
    theta[-2:] = (y0, y1)  # b3: the output is the bias when W3 = 0
    return theta


def test_network_interval_equals_fixed(env):
    torch, Sim = env
    prob, b, q = _case()
    y0, y1 = np.float32(-0.2), np.float32(0.15)
    a, bb = opc.interval_from_output(float(y0), float(y1))
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12, precond=1, cheb_terms=4)
        sim.dmri_precond_set_params(_const_net(y0, y1))
        pid = sim.add_problem(prob)
        sig1, st1 = sim.dmri_run([pid] * len(b), b, q)
        assert np.array_equal(sim.dmri_precond_get_params(), _const_net(y0, y1))
    sig2, st2, _ = _run(Sim, prob, b, q, rtol=1e-12, precond=2, cheb_terms=4, cheb_a=a,
                        cheb_b=bb)
    _say("network interval [%.4f, %.4f]: iterations %d vs %d" % (
        a, bb, st1["total_iterations"], st2["total_iterations"]))
    assert abs(st1["total_iterations"] - st2["total_iterations"]) <= 2
    assert np.max(np.abs(sig1 - sig2) / np.abs(sig2)) < 1e-10


def test_fallback_to_jacobi(env):
    # An interval far below the spectrum with 16 terms makes the
    # preconditioned spectrum span ~1e7: the flexible solve reaches max_iter,
    # and Jacobi CG solves the step again from where it stopped.
    torch, Sim = env
    prob, b, q = _case()
    ref = timestep.signals(prob, SHORT, b, q, solver="splu", n_steps=3)
    sig, st, fb = _run(Sim, prob, b, q, rtol=1e-12, precond=2, cheb_terms=16, cheb_a=1e-3,
                       cheb_b=2e-3, max_iter=300, n_steps=3, signal=0)
    err = rel_err(sig, ref, ref[0])
    _say("fallback: %d steps re-solved, max err %.2e, flags converged %s" % (
        fb, err.max(), st["converged"].tolist()))
    assert fb == 3
    assert err.max() < 1e-9
    assert np.all(st["converged"])


def test_learned_interval_keeps_answer(env):
    # Samples of a Jacobi-CG run on some systems train the interval network
    # (the library's own forward, backward and Adam kernels); the learned
    # interval then solves other systems of the mesh within 1e-9 of the
    # oracle. The iteration counts of Jacobi CG, the learned interval and the
    # reference interval are reported and the measured relation asserted.
    torch, Sim = env
    prob, b, q = _case(13)
    ref = _ref(13)
    rng = np.random.default_rng(9)
    b_tr = rng.uniform(200.0, 5000.0, 24)
    q_tr = di.fibonacci_directions(24)[::-1].copy()
    cap = 24 * 40
    X = torch.zeros((cap, 16), dtype=torch.float32, device="cuda")
    T = torch.zeros((cap, 2), dtype=torch.float32, device="cuda")
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12, precond=0)
        pid = sim.add_problem(prob)
        sim.dmri_precond_record(X, T, cap)
        sim.dmri_run([pid] * len(b_tr), b_tr, q_tr)
        n = sim.dmri_precond_record_count()
        sim.dmri_precond_record(None, None, 0)
        sim.dmri_precond_set_params(np.zeros(5378, np.float32))
        l0, _ = sim.dmri_precond_train(X, T, 1, 1e-3, n=n)
        sim.dmri_precond_set_params(opc_init())
        l_first, l_last = sim.dmri_precond_train(X, T, 400, 3e-3, n=n)
        sim.set_options(precond=1, cheb_terms=4)
        sig, st = sim.dmri_run([pid] * len(b), b, q)
        sim.set_options(precond=0)
        _, st0 = sim.dmri_run([pid] * len(b), b, q)
        sim.set_options(precond=2, cheb_terms=4)
        _, st2 = sim.dmri_run([pid] * len(b), b, q)
    err = rel_err(sig, ref, ref[0])
    _say("learned interval: %d samples, loss zero-net %.3e, trained %.3e -> %.3e; max err %.2e;"
         " iterations Jacobi %d, learned %d (x%d terms), reference interval %d" % (
             n, l0, l_first, l_last, err.max(), st0["total_iterations"],
             st["total_iterations"], 4, st2["total_iterations"]))
    assert n > 100
    assert l_last < 0.2 * l0
    assert err.max() < 1e-9
    assert st["total_iterations"] < st0["total_iterations"]


def opc_init():
    from oracle import mlp as omlp
    return omlp.init(seed=3, scale=0.5).astype(np.float32)


def test_refusals(env):
    torch, Sim = env
    prob, b, q = _case(4)
    walls = di.free_box(n=4, half=2.0, periodic_mask=0)
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        wid = sim.add_problem(walls)
        sim.set_options(precond=1)
        with pytest.raises(Exception, match="DMRI_E_STATE"):
            sim.dmri_run([pid] * 4, b, q)
        for opts, who in (({"precond": 2, "precision": 1}, pid), ({"precond": 2}, wid),
                          ({"precond": 2, "precision": 0, "queue": 1}, pid),
                          ({"precond": 2, "queue": 0, "krylov": 3}, pid)):
            sim.set_options(**opts)
            with pytest.raises(Exception, match="DMRI_E_UNSUPPORTED"):
                sim.dmri_run([who] * 4, b, q)
        sim.set_options(precond=2, krylov=0)
        X = torch.zeros((8, 16), dtype=torch.float32, device="cuda")
        T = torch.zeros((8, 2), dtype=torch.float32, device="cuda")
        sim.dmri_precond_record(X, T, 8)
        with pytest.raises(Exception, match="DMRI_E_UNSUPPORTED"):
            sim.dmri_run([pid] * 4, b, q)


def test_learned_interval_on_held_out_geometry(env):
    # The network trained on one geometry's Jacobi-CG samples (the 11^3
    # cylinder) sets the intervals on another (a seeded cell geometry, other
    # compartments, diffusivities and membranes): the signals stay within
    # 1e-9 of the oracle and the flexible solve takes fewer Krylov iterations
    # than Jacobi CG there too.
    torch, Sim = env
    prob, b, q = _case(13)
    cells, _, _ = di.seeded_cells(5, n_fixed=12)
    rng = np.random.default_rng(4)
    b_ev = rng.uniform(200.0, 5000.0, 6)
    q_ev = di.fibonacci_directions(6)
    ref = timestep.signals(cells, SHORT, b_ev, q_ev, solver="splu")
    cap = 13 * 40
    X = torch.zeros((cap, 16), dtype=torch.float32, device="cuda")
    T = torch.zeros((cap, 2), dtype=torch.float32, device="cuda")
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12, precond=0)
        pid = sim.add_problem(prob)
        cid = sim.add_problem(cells)
        sim.dmri_precond_record(X, T, cap)
        sim.dmri_run([pid] * len(b), b, q)
        n = sim.dmri_precond_record_count()
        sim.dmri_precond_record(None, None, 0)
        sim.dmri_precond_set_params(opc_init())
        l_first, l_last = sim.dmri_precond_train(X, T, 400, 3e-3, n=n)
        _, st0 = sim.dmri_run([cid] * len(b_ev), b_ev, q_ev)
        sim.set_options(precond=1, cheb_terms=4)
        sig, st = sim.dmri_run([cid] * len(b_ev), b_ev, q_ev)
        fb = sim.dmri_get_option("pc_fallback_steps")
    err = rel_err(sig, ref, ref[0])
    _say("held-out geometry: %d samples, loss %.3e -> %.3e; max err %.2e; iterations Jacobi %d,"
         " learned %d (x4 terms); fallback steps %d" % (
             n, l_first, l_last, err.max(), st0["total_iterations"], st["total_iterations"], fb))
    assert err.max() < 1e-9
    assert st["total_iterations"] < st0["total_iterations"]


def test_tensor_mesh_and_autotuner(env):
    # Flexible CG with a fixed interval on a conforming mesh with a diffusion
    # tensor per compartment (the per-row mass coefficient inside the
    # Chebyshev terms), and with the autotuner choosing the launch shape:
    # both within 1e-9 of the oracle.
    torch, Sim = env
    prob = di.conforming_cylinder_box(
        n=7, half=6.0, r=4.0, D_in=di.tensor([3e-3, 1e-3, 2e-3], (0.3, 0.5, 0.2)),
        D_out=di.tensor([2e-3, 2.5e-3, 1.5e-3], (1.0, -0.4, 0.7)), kappa=5e-3)
    rng = np.random.default_rng(2)
    b = rng.uniform(0.0, 5000.0, 10)
    q = di.fibonacci_directions(10)
    ref = timestep.signals(prob, SHORT, b, q, solver="splu")
    for opts in (dict(sys_tile=8), dict(autotune=1)):
        sig, st, fb = _run(Sim, prob, b, q, rtol=1e-12, precond=2, cheb_terms=4, **opts)
        err = rel_err(sig, ref, ref[0])
        _say("tensor mesh %s: max err %.2e, iterations %d" % (opts, err.max(),
                                                              st["total_iterations"]))
        assert err.max() < 1e-9
        assert fb == 0
