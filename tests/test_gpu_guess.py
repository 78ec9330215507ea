"""GPU tests of the learned initial guess (network kernels through the C ABI).

* forward pass and loss gradient against the FP64 NumPy network of the
  oracle, evaluated on the same BF16-rounded inputs and weights (the kernels
  multiply in BF16 and accumulate in FP32; tolerances follow from BF16's
  2^-9 relative rounding of the hidden activations);
* recorded features and targets against the definitions in include/dmri.h,
  computed from the oracle's solutions u^0, u^1, u^2;
* the learned guess never changes the accepted answer: signals stay within
  1e-9 of the oracle for any network, and a network with non-finite weights
  falls back to the previous step exactly;
* training by the library's own backward and Adam kernels lowers the loss.
"""

import numpy as np
import pytest

import dmri_inputs as di
from oracle import fem, mlp as omlp, sequence as oseq, timestep

pytestmark = pytest.mark.gpu

SHORT = di.Sequence(2000.0, 4000.0, 200.0, 0.5)


@pytest.fixture(scope="module")
def env():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_01719_amd import Simulator
    from paper_1908_01719_amd import learned_guess as lg
    return torch, Simulator, lg


def _say(msg):
    print(msg, flush=True)


def _bf16(a):
    """Round float32 values to BF16 (nearest, ties to even), as float64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _bf16_weights(theta32):
    parts = omlp.unpack(theta32.astype(np.float64))
    for i in (0, 2, 4):  # W1, W2, W3 are BF16 operands; biases stay FP32
        parts[i] = _bf16(parts[i].astype(np.float32))
    return omlp.pack(parts)


def _dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


@pytest.mark.parametrize("n", [1, 63, 1000, 20000])
def test_forward_matches_oracle(env, n):
    torch, Sim, lg = env
    _say("forward n=%d" % n)
    rng = np.random.default_rng(n)
    theta = omlp.init(seed=1).astype(np.float32)
    theta[1024:1088] = rng.normal(size=64) * 0.1  # nonzero biases
    X = rng.normal(size=(n, 16)).astype(np.float32)
    y_ref, _ = omlp.forward(_bf16_weights(theta), _bf16(X))
    with Sim(0) as sim:
        sim.dmri_guess_set_params(theta)
        Xd = _dev(torch, X)
        Yd = torch.zeros((n, 2), dtype=torch.float32, device="cuda")
        sim.dmri_guess_eval(Xd, out_dev=Yd, want_loss=False)
        y = Yd.cpu().numpy().astype(np.float64)
    scale = np.sqrt(np.mean(y_ref ** 2))
    err = np.max(np.abs(y - y_ref)) / scale
    _say("  max |y - y_ref| / rms = %.3e" % err)
    assert err < 2e-2


def test_gradient_matches_oracle(env):
    torch, Sim, lg = env
    rng = np.random.default_rng(5)
    n = 3000
    theta = omlp.init(seed=2).astype(np.float32)
    X = rng.normal(size=(n, 16)).astype(np.float32)
    T = rng.normal(size=(n, 2)).astype(np.float32)
    tb = _bf16_weights(theta)
    g_ref = omlp.gradients(tb, _bf16(X), T.astype(np.float64))
    l_ref = omlp.loss(tb, _bf16(X), T.astype(np.float64))
    with Sim(0) as sim:
        sim.dmri_guess_set_params(theta)
        Xd, Td = _dev(torch, X), _dev(torch, T)
        G1 = torch.zeros(5378, dtype=torch.float32, device="cuda")
        G2 = torch.zeros(5378, dtype=torch.float32, device="cuda")
        loss = sim.dmri_guess_eval(Xd, Td, grad_dev=G1)
        sim.dmri_guess_eval(Xd, Td, grad_dev=G2)
        g = G1.cpu().numpy().astype(np.float64)
        g2 = G2.cpu().numpy()
    # deterministic reduction: bitwise equal on repeat
    assert np.array_equal(g.astype(np.float32), g2)
    assert abs(loss - l_ref) / l_ref < 1e-2
    parts, parts_ref = omlp.unpack(g), omlp.unpack(g_ref)
    for name, a, b in zip(["W1", "b1", "W2", "b2", "W3", "b3"], parts, parts_ref):
        rel = np.linalg.norm(a - b) / np.linalg.norm(b)
        _say("  grad %s rel err %.3e" % (name, rel))
        assert rel < 3e-2, name
    cos = g @ g_ref / (np.linalg.norm(g) * np.linalg.norm(g_ref))
    assert cos > 0.999


def test_training_lowers_loss(env):
    torch, Sim, lg = env
    rng = np.random.default_rng(11)
    n = 16384
    teacher = omlp.init(seed=7)
    X = rng.normal(size=(n, 16))
    T, _ = omlp.forward(teacher, X)
    with Sim(0) as sim:
        sim.dmri_guess_set_params(lg.init_params(0))
        Xd, Td = _dev(torch, X), _dev(torch, T)
        hist = lg.train(sim, Xd, Td, iters=600, lr=3e-3)
    _say("  loss history %s" % np.array2string(np.array(hist), precision=4))
    assert hist[-1] < 0.2 * hist[0]
    assert all(np.isfinite(hist))


def _perm(prob, exp, asm):
    tn, _ = fem.torus_nodes(prob.xyz, prob.box_lo, prob.box_hi, prob.periodic_mask)
    key = {(int(c), int(nd)): i for i, (c, nd) in enumerate(zip(asm.dof_comp, asm.dof_node))}
    return np.array([key[(int(c), int(tn[nd]))] for c, nd in zip(exp["dof_comp"], exp["dof_node"])])


def test_recorded_samples_match_definition(env):
    """Every element of a 3-system batch after step 2, against the features
    and targets recomputed from the oracle's u^0, u^1, u^2."""
    torch, Sim, lg = env
    prob = di.cylinder_box(n=8, half=6.0, r=4.3, kappa=5e-3, D_in=1.5e-3, T2=(6e4, 4e4),
                           u0=(1.0, 0.7))
    b = np.array([800.0, 2500.0, 4000.0])
    q = di.fibonacci_directions(3)
    asm = fem.assemble(prob)
    U = []
    for s in range(3):
        u1 = timestep.solve_transformed(asm, SHORT, b[s], q[s], n_steps=1, return_u=True)[1]
        u2 = timestep.solve_transformed(asm, SHORT, b[s], q[s], n_steps=2, return_u=True)[1]
        U.append((asm.u0.astype(np.complex128), u1, u2))
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-13, n_steps=2, sys_tile=8)
        pid = sim.add_problem(prob)
        exp = sim.dmri_export_operator(pid)
        n_dof = exp["w"].shape[0]
        cap = n_dof * 8
        X = torch.zeros((cap, 16), dtype=torch.float32, device="cuda")
        T = torch.zeros((cap, 2), dtype=torch.float32, device="cuda")
        sim.dmri_guess_record(X, T, cap, 1)
        sim.dmri_run([pid] * 3, b, q)
        assert sim.dmri_guess_record_count() == cap
        X, T = X.cpu().numpy().astype(np.float64), T.cpu().numpy().astype(np.float64)
    perm = _perm(prob, exp, asm)
    # element e of the tile-major batch: row e // 8, system e % 8 (one tile)
    Xr = X.reshape(n_dof, 8, 16)
    Tr = T.reshape(n_dof, 8, 2)
    assert np.all(Xr[:, 3:] == 0) and np.all(Tr[:, 3:] == 0)  # padding systems
    t = oseq.time_grid(SHORT.delta, SHORT.Delta, SHORT.dt)
    F = oseq.pgse_F(t, SHORT.delta, SHORT.Delta)
    D = np.array(prob.D)[exp["dof_comp"]]
    # DOFs whose node lies on a periodic face have an ambiguous position
    tn, _ = fem.torus_nodes(prob.xyz, prob.box_lo, prob.box_hi, prob.periodic_mask)
    xyz = prob.xyz[exp["dof_node"]] - 0.5 * (np.asarray(prob.box_lo) + np.asarray(prob.box_hi))
    inner = np.all(np.abs(np.abs(xyz) - 6.0) > 1e-9, axis=1)
    n_comp_of_node = {}
    for c, nd in zip(asm.dof_comp, asm.dof_node):
        n_comp_of_node[int(nd)] = n_comp_of_node.get(int(nd), 0) + 1
    memb = np.array([1.0 if n_comp_of_node[int(tn[nd])] > 1 else 0.0 for nd in exp["dof_node"]])
    for s in range(3):
        u0, u1, u2 = (v[perm] for v in U[s])
        m = np.abs(u1)
        G = float(oseq.b_to_G(b[s], SHORT.delta, SHORT.Delta))
        g0, g1, g2 = G * F[2], G * F[1], G * F[0]
        f = np.zeros((n_dof, 16))
        f[:, 0], f[:, 1] = ((u1 - u0) / m).real, ((u1 - u0) / m).imag
        f[:, 2], f[:, 3] = (u1 / m).real, (u1 / m).imag
        f[:, 4] = 10 * (g0 - g1)
        f[:, 5] = 10 * (g1 - g2)
        f[:, 6] = g0
        f[:, 7] = SHORT.dt * D * g0 ** 2
        f[:, 8] = 0.1 * xyz @ (q[s] / np.linalg.norm(q[s]))
        f[:, 9] = exp["dof_comp"]
        f[:, 10] = memb
        f[:, 11] = SHORT.dt * D * g1 ** 2
        cols = [c for c in range(16) if c != 8]
        np.testing.assert_allclose(Xr[:, s, cols], f[:, cols], rtol=2e-6, atol=1e-6)
        np.testing.assert_allclose(Xr[inner, s, 8], f[inner, 8], rtol=2e-6, atol=1e-6)
        tgt = 100.0 * (u2 - (2 * u1 - u0)) / m
        tgt = np.stack([tgt.real, tgt.imag], axis=1).clip(-100, 100)
        err = np.max(np.abs(Tr[:, s] - tgt))
        _say("  system %d: max target error %.2e (target rms %.2e)" % (s, err, np.sqrt(np.mean(tgt ** 2))))
        assert err < 1e-4 + 1e-5 * np.max(np.abs(tgt))


def _cyl_case():
    prob = di.cylinder_box(n=11, half=6.0, r=4.3, kappa=5e-3, D_in=1.5e-3, T2=(6e4, 4e4),
                           u0=(1.0, 0.7))
    b = np.array([0.0, 500.0, 1500.0, 3000.0, 5000.0, 2500.0, 4000.0, 1000.0, 3500.0, 200.0])
    q = di.fibonacci_directions(10)
    return prob, b, q


@pytest.mark.parametrize("precision", [0, 1])
def test_learned_guess_keeps_answer(env, precision):
    torch, Sim, lg = env
    prob, b, q = _cyl_case()
    ref = timestep.signals(prob, SHORT, b, q, solver="splu")
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12, precision=precision)
        pid = sim.add_problem(prob)
        sim.set_options(guess=0)
        sig0, st0 = sim.dmri_run([pid] * len(b), b, q)
        sim.set_options(guess=2)
        sim.dmri_guess_set_params(lg.init_params(3, out_scale=1.0))
        sig2, st2 = sim.dmri_run([pid] * len(b), b, q)
        bad = lg.init_params(3)
        bad[-2] = np.nan  # output bias: every prediction is non-finite
        sim.dmri_guess_set_params(bad)
        sign, stn = sim.dmri_run([pid] * len(b), b, q)
    for sig, st in ((sig0, st0), (sig2, st2), (sign, stn)):
        assert st["status"] == "DMRI_OK"
        err = np.abs(sig - ref) / np.maximum(np.abs(ref), 1e-8 * abs(ref[0]))
        assert err.max() < 1e-9, err.max()
    _say("  iterations guess0 %d, random network %d, NaN network %d"
         % (st0["total_iterations"], st2["total_iterations"], stn["total_iterations"]))
    # non-finite network => every element falls back to u^{n-1} (= guess 0)
    assert stn["total_iterations"] == st0["total_iterations"]
    assert np.array_equal(sign, sig0)


def test_guess_api_errors(env, tmp_path):
    torch, Sim, lg = env
    from paper_1908_01719_amd import DmriError
    prob, b, q = _cyl_case()
    with Sim(0) as sim:
        sim.set_sequence(SHORT)
        pid = sim.add_problem(prob)
        sim.set_options(guess=2)
        with pytest.raises(DmriError, match="E_STATE"):
            sim.dmri_run([pid], b[:1], q[:1])
        with pytest.raises(DmriError, match="E_INVALID"):
            sim.dmri_guess_set_params(np.zeros(10, np.float32))
        p = lg.init_params(9)
        sim.dmri_guess_set_params(p)
        path = str(tmp_path / "net.bin")
        sim.dmri_save_guess_model(path)
        sim.dmri_guess_set_params(lg.zero_params())
        sim.dmri_load_guess_model(path)
        assert np.array_equal(sim.dmri_guess_get_params(), p)
        with open(path, "r+b") as fh:
            fh.write(b"XXXX")
        with pytest.raises(DmriError, match="E_INVALID"):
            sim.dmri_load_guess_model(path)
        sim.set_options(precision=2)
        with pytest.raises(DmriError, match="E_UNSUPPORTED"):
            sim.dmri_run([pid], b[:1], q[:1])


def test_trained_network_gain_on_held_out_geometry(env):
    """Train on trajectories of one cylinder geometry, evaluate on another
    (different radius, permeability and b-values): the trained network's
    correction of the linear extrapolation has a lower mean squared error on
    the held-out samples than the zero network (the plain extrapolation), and
    the learned guess keeps the signals. The Krylov iterations of the three
    guesses are reported (the per-element error gain does not by itself
    lower them: the network's error varies from element to element)."""
    torch, Sim, lg = env
    train = di.cylinder_box(n=12, half=6.0, r=4.0, kappa=5e-3, D_in=2e-3, T2=(6e4, 4e4))
    held = di.cylinder_box(n=12, half=6.0, r=3.2, kappa=1e-3, D_in=1.2e-3, T2=(5e4, 5e4))
    seq = di.Sequence(2000.0, 4000.0, 100.0, 0.5)
    bt = np.linspace(500.0, 5000.0, 16)
    qt = di.fibonacci_directions(16)
    bh = np.linspace(700.0, 4500.0, 8)
    qh = di.fibonacci_directions(8)[::-1].copy()
    ref = timestep.signals(held, seq, bh, qh, solver="splu")
    with Sim(0) as sim:
        sim.set_sequence(seq)
        sim.set_options(rtol=1e-10)
        pt, ph = sim.add_problem(train), sim.add_problem(held)
        X, T = lg.record(sim, [(pt, bt, qt)], capacity=400_000, stride=7)
        Xv, Tv = lg.record(sim, [(ph, bh, qh)], capacity=200_000, stride=11)
        sim.dmri_guess_set_params(lg.zero_params())
        l_zero = sim.dmri_guess_eval(Xv, Tv)
        sim.dmri_guess_set_params(lg.init_params(0))
        hist = lg.train(sim, X, T, iters=1500, lr=2e-3)
        l_held = sim.dmri_guess_eval(Xv, Tv)
        its = {}
        for g in (0, 1, 2):
            sim.set_options(guess=g, extrap_order=1)
            sig, st = sim.dmri_run([ph] * len(bh), bh, qh)
            its[g] = st["total_iterations"]
            err = np.abs(sig - ref) / np.maximum(np.abs(ref), 1e-8 * abs(ref[0]))
            assert err.max() < 1e-8, (g, err.max())
    _say("  %d training samples, train loss %.3e -> %.3e; held-out loss: zero network %.3e, "
         "trained %.3e; iterations prev/extrap/learned %s"
         % (X.shape[0], hist[0], hist[-1], l_zero, l_held, its))
    assert l_held < 0.8 * l_zero
