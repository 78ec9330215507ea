"""Host-side logic of the benchmark and the loader (CPU only).

* `bench.py --gpus N` with N > 1 refuses to run (this build measures one GPU).
* The algorithmic byte counts follow the per-kernel formulas: 2c per DOF and
  system for the SpMV vectors, the matrix once per active tile.
* The committed HBM-counter summary is used only for the workload, precision
  and tolerance it was taken on, and only while the library sources hash to
  the recorded value.
* The binding fails loudly when libdmri.so is missing (there is no CPU path).
"""

import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, timeout=120)
    assert p.returncode == 2
    assert "exactly one GPU" in p.stderr
    assert p.stdout.strip() == ""


def test_spmv_bytes_formula():
    n_dof, nnz, iters, tile = 1000, 15000, 640, 128
    got = bench.kernel_bytes("spmv", n_dof, nnz, iters, tile, 4, 10, 64)
    c = 8
    mat = nnz * (4 + 5 * 4) + 4 * n_dof
    assert got == pytest.approx(2 * c * n_dof * iters + mat * iters / tile)
    # FP64 doubles the vector and value bytes, not the column indices
    got64 = bench.kernel_bytes("spmv", n_dof, nnz, iters, 64, 8, 10, 64)
    assert got64 == pytest.approx(2 * 16 * n_dof * iters + (nnz * 44 + 4 * n_dof) * iters / 64)
    assert bench.kernel_bytes("update", n_dof, nnz, iters, tile, 4, 10, 64) == pytest.approx(
        3 * c * n_dof * iters + n_dof * 20 * iters / tile)
    assert bench.kernel_bytes("pupdate", n_dof, nnz, iters, tile, 4, 10, 64) == pytest.approx(
        5 * c * n_dof * iters + n_dof * 20 * iters / tile)


def _summary():
    path = os.path.join(ROOT, "profiles", "hbm_counters_k_spmv_pair_cylinder_57_batched_mixed.md")
    if not os.path.exists(path):
        pytest.skip("no committed counter summary")
    return open(path).read()


def test_counter_summary_is_tied_to_its_workload():
    text = _summary()
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    assert m
    recorded = re.search(r"csrc_sha256:\s*([0-9a-f]+)", text).group(1)
    got = bench.profiled_traffic("k_spmv_pair", "cylinder_57_batched", "mixed", 1e-6)
    if recorded == bench.csrc_sha256():
        assert got == pytest.approx(float(m.group(1)))
    else:
        assert got is None
    # other tolerance, precision, workload or kernel: no figure
    assert bench.profiled_traffic("k_spmv_pair", "cylinder_57_batched", "mixed", 1e-8) is None
    assert bench.profiled_traffic("k_spmv_pair", "cylinder_57_batched", "fp64", 1e-6) is None
    assert bench.profiled_traffic("k_spmv_pair", "cylinder_36", "mixed", 1e-6) is None
    assert bench.profiled_traffic("k_spmv_dot", "cylinder_57_batched", "mixed", 1e-6) is None


def test_source_hash_covers_the_library_sources(tmp_path, monkeypatch):
    h0 = bench.csrc_sha256()
    assert re.fullmatch(r"[0-9a-f]{64}", h0)
    # a copy of the sources with one byte changed in a host file hashes differently
    csrc = os.path.join(ROOT, "paper_1908_01719_amd", "csrc")
    fake = tmp_path / "paper_1908_01719_amd" / "csrc"
    fake.mkdir(parents=True)
    for f in os.listdir(csrc):
        data = open(os.path.join(csrc, f), "rb").read()
        if f == "capi.hip":
            data += b"\n"
        (fake / f).write_bytes(data)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.csrc_sha256() != h0


def test_binding_fails_loudly_without_library(tmp_path):
    from paper_1908_01719_amd import binding
    with pytest.raises(ImportError, match="not found"):
        binding.load(str(tmp_path / "libdmri.so"))


def test_cpu_sample_spans_the_echo_and_the_b_range():
    import dmri_inputs as di
    _, seq, sysl = di.cylinder_57_batched()
    plan = bench.cpu_sample_plan(sysl, seq.n_steps, 6, 16)
    starts = [s0 for _, s0 in plan]
    bs = sorted(float(sysl.b[i]) for i, _ in plan)
    assert starts[0] == 0 and starts[-1] == seq.n_steps - 6
    assert all(0 <= s <= seq.n_steps - 6 for s in starts)
    assert len(set(starts)) == 16
    assert bs[0] < 500 and bs[-1] > 4500


def test_oracle_start_step_takes_later_steps():
    # start_step s with n steps takes steps s+1 .. s+n from the initial
    # magnetization: s = 0 is the plain run; for free diffusion the state
    # stays uniform and follows the scalar recurrence from that step on.
    import numpy as np
    import dmri_inputs as di
    from oracle import fem, sequence, timestep
    prob, seq, sysl = di.free_diffusion_10()
    asm = fem.assemble(prob)
    s_plain = timestep.solve_transformed(asm, seq, 1000.0, [1, 0, 0], n_steps=5)
    s_zero = timestep.solve_transformed(asm, seq, 1000.0, [1, 0, 0], n_steps=5, start_step=0)
    assert s_plain == s_zero
    s_late = timestep.solve_transformed(asm, seq, 1000.0, [1, 0, 0], n_steps=3,
                                        start_step=100)
    G = float(sequence.b_to_G(1000.0, seq.delta, seq.Delta))
    F = sequence.pgse_F(np.arange(seq.n_steps + 1) * seq.dt, seq.delta, seq.Delta)
    c = 1.0
    a = lambda Fv: prob.D[0] * (G * Fv) ** 2  # noqa: E731
    for n in range(101, 104):
        c *= (1 - 0.5 * seq.dt * a(F[n - 1])) / (1 + 0.5 * seq.dt * a(F[n]))
    vol = 1000.0
    assert abs(s_late / vol - c) < 1e-12
