"""The entry point that allocates no device memory (dmri_run_device_noalloc)
against the existing device entry point (dmri_run_device) and the oracle.

Two calls in a row, the second with fewer systems (the array keeps the first
call's contents, so the run must clear what it relies on), each compared
with dmri_run_device on the same pairs (same kernels: within 1e-12) and with
the FP64 oracle's exact-solve signals (within 1e-9). Also the limits: more
than 64 pairs, a precision other than FP64, and a problem whose operators
are not on the device yet.
"""

import numpy as np
import pytest

import dmri_inputs as di
from oracle import timestep

pytestmark = pytest.mark.gpu

SHORT = di.Sequence(2000.0, 4000.0, 200.0, 0.5)


def _case():
    prob = di.cylinder_box(n=11, half=6.0, r=4.3, kappa=5e-3, D_in=1.5e-3, T2=(6e4, 4e4),
                           u0=(1.0, 0.7))
    b = np.array([0.0, 500.0, 1500.0, 3000.0, 5000.0, 2500.0, 4000.0, 1000.0, 3500.0, 200.0,
                  4500.0, 800.0, 2000.0])
    q = di.fibonacci_directions(13)
    return prob, b, q


def _rel(a, ref):
    return np.abs(a - ref) / np.maximum(np.abs(ref), 1e-8 * np.abs(ref).max())


def test_noalloc_matches_device_entry_twice():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_01719_amd import Simulator

    prob, b, q = _case()
    ref = timestep.signals(prob, SHORT, b, q, solver="splu")

    def dev(x, dt):
        return torch.tensor(np.ascontiguousarray(x), dtype=dt, device="cuda")

    with Simulator(0) as sim:
        sim.set_sequence(SHORT)
        sim.set_options(rtol=1e-12, persistent=1)
        pid = sim.add_problem(prob)
        other = sim.add_problem(di.free_box(n=6, half=3.0))
        # Before any run of the problem its operators are not on the device.
        ids = dev(np.full(len(b), pid, np.int32), torch.int32)
        out = torch.zeros((len(b), 2), dtype=torch.float64, device="cuda")
        with pytest.raises(Exception, match="DMRI_E_STATE"):
            sim.dmri_run_device_noalloc(ids, dev(b, torch.float64), dev(q, torch.float64), out)
        for sel in (np.arange(len(b)), np.array([4, 1, 10, 2, 7])):
            n = len(sel)
            ids = dev(np.full(n, pid, np.int32), torch.int32)
            db, dq = dev(b[sel], torch.float64), dev(q[sel], torch.float64)
            s_dev = torch.zeros((n, 2), dtype=torch.float64, device="cuda")
            s_na = torch.full((n, 2), float("nan"), dtype=torch.float64, device="cuda")
            st_dev = sim.dmri_run_device(ids, db, dq, s_dev)
            st_na = sim.dmri_run_device_noalloc(ids, db, dq, s_na)
            torch.cuda.synchronize()
            a = s_dev.cpu().numpy()
            c = s_na.cpu().numpy()
            a = a[:, 0] + 1j * a[:, 1]
            c = c[:, 0] + 1j * c[:, 1]
            e_dev = _rel(c, a).max()
            e_ref = _rel(c, ref[sel]).max()
            print("noalloc n=%d: vs device entry %.2e, vs oracle %.2e, iterations %d vs %d"
                  % (n, e_dev, e_ref, st_na["total_iterations"], st_dev["total_iterations"]),
                  flush=True)
            assert st_na["status"] == "DMRI_OK"
            assert np.all(st_na["converged"] == 1)
            assert e_dev < 1e-12
            assert e_ref < 1e-9
        # limits
        ids65 = dev(np.full(65, pid, np.int32), torch.int32)
        with pytest.raises(Exception, match="DMRI_E_INVALID"):
            sim.dmri_run_device_noalloc(ids65, dev(np.ones(65), torch.float64),
                                        dev(np.ones((65, 3)), torch.float64),
                                        torch.zeros((65, 2), dtype=torch.float64, device="cuda"))
        mixed = dev(np.array([pid, other], np.int32), torch.int32)
        with pytest.raises(Exception, match="DMRI_E_INVALID"):
            sim.dmri_run_device_noalloc(mixed, dev(b[:2], torch.float64), dev(q[:2], torch.float64),
                                        torch.zeros((2, 2), dtype=torch.float64, device="cuda"))
        # a problem with diffusion tensors (per-compartment factor table in
        # the array too)
        pt = di.conforming_cylinder_box(
            n=6, D_in=di.tensor([3e-3, 1e-3, 2e-3], (0.3, 0.5, 0.2)),
            D_out=di.tensor([2e-3, 2e-3, 1e-3]), kappa=5e-3)
        it = sim.add_problem(pt)
        sel = np.array([1, 3, 4])
        idt = dev(np.full(3, it, np.int32), torch.int32)
        db, dq = dev(b[sel], torch.float64), dev(q[sel], torch.float64)
        s_dev = torch.zeros((3, 2), dtype=torch.float64, device="cuda")
        s_na = torch.zeros((3, 2), dtype=torch.float64, device="cuda")
        sim.dmri_run_device(idt, db, dq, s_dev)
        sim.dmri_run_device_noalloc(idt, db, dq, s_na)
        torch.cuda.synchronize()
        a, c = s_dev.cpu().numpy(), s_na.cpu().numpy()
        assert _rel(c[:, 0] + 1j * c[:, 1], a[:, 0] + 1j * a[:, 1]).max() < 1e-12
        sim.set_options(precision=1)
        with pytest.raises(Exception, match="DMRI_E_UNSUPPORTED"):
            sim.dmri_run_device_noalloc(ids[:2], dev(b[:2], torch.float64),
                                        dev(q[:2], torch.float64),
                                        torch.zeros((2, 2), dtype=torch.float64, device="cuda"))
