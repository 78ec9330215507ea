"""Host logic of libdmri on the CPU (host-only context, no device calls).

* the shared library loads and exports every function include/dmri.h declares;
* the C++ assembly (periodic identification, PUFEM DOFs, CSR, element and
  membrane integrals) equals the oracle's operators entry by entry after
  matching DOFs by (compartment, mesh node);
* input validation returns DMRI_E_INVALID / DMRI_E_UNSUPPORTED.
"""

import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

import dmri_inputs as di
from oracle import fem
from paper_1908_01719_amd import binding
from paper_1908_01719_amd.binding import DmriError, Simulator

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    header = open(os.path.join(ROOT, "include", "dmri.h")).read()
    declared = sorted(set(re.findall(r"\b(dmri_[a-z_]+)\s*\(", header)))
    assert declared, "no declarations found"
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(binding.EXPORTED) == declared


def test_library_exports_nothing_else():
    # The C entry points are the whole boundary: the library is built with
    # hidden default visibility, so no C++ internals are exported.
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    header = open(os.path.join(ROOT, "include", "dmri.h")).read()
    declared = set(re.findall(r"\b(dmri_[a-z_]+)\s*\(", header))
    out = subprocess.run([nm, "-D", "--defined-only", binding.LIB_PATH], check=True,
                         stdout=subprocess.PIPE, text=True).stdout
    funcs = {ln.split()[-1] for ln in out.splitlines() if len(ln.split()) == 3
             and ln.split()[1] == "T"}
    assert funcs == declared, sorted(funcs ^ declared)


def _lib_to_oracle_perm(prob, exp, asm):
    tn, _ = fem.torus_nodes(prob.xyz, prob.box_lo, prob.box_hi, prob.periodic_mask)
    key = {(int(c), int(n)): i for i, (c, n) in enumerate(zip(asm.dof_comp, asm.dof_node))}
    return np.array([key[(int(c), int(tn[n]))] for c, n in zip(exp["dof_comp"], exp["dof_node"])])


CASES = {
    "free_periodic": lambda: di.free_box(n=5, half=2.5),
    "cyl_centroid": lambda: di.cylinder_box(n=9, half=6.0, r=4.0, kappa=2e-3, D_in=1e-3,
                                            T2=(5e4, 3e4), u0=(0.5, 1.5)),
    "cyl_cube": lambda: di.cylinder_box(n=8, half=6.0, r=4.0, kappa=0.1, mode="cube"),
    "slab_neumann": lambda: di.slab_box(n=6, half=3.0, split=0.4, D=(3e-3, 1e-3), kappa=1e-2,
                                        periodic_mask=0),
    "seeded_cells": lambda: di.seeded_cells(3, n_fixed=10)[0],
    # unstructured interface-conforming mesh with a diffusion tensor per
    # compartment (through dmri_add_problem_tensor), both forms
    "conforming_tensor": lambda: di.conforming_cylinder_box(
        n=7, half=6.0, r=4.0, D_in=di.tensor([3e-3, 1e-3, 2e-3], (0.3, 0.5, 0.2)),
        D_out=di.tensor([2e-3, 2.5e-3, 1.5e-3], (1.0, -0.4, 0.7)), kappa=5e-3),
    # weak pseudo-periodic faces (the arrays of the faces are compared in
    # test_weak_faces_match_oracle)
    "weak_nonmatching": lambda: di.nonmatching_faces(
        di.conforming_cylinder_box(n=6, half=6.0, r=4.0, kappa=1e-2, D_in=1e-3,
                                   periodic_mask=13, seed=1), axes=(0, 2), amount=0.25, seed=7),
    "conforming_tensor_neumann": lambda: di.conforming_cylinder_box(
        n=7, half=6.0, r=4.0, D_in=di.tensor([3e-3, 1e-3, 2e-3], (0.3, 0.5, 0.2)),
        D_out=di.tensor([2e-3, 2e-3, 2e-3]), periodic_mask=0, kappa=5e-3),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_operators_match_oracle(name):
    prob = CASES[name]()
    with Simulator(-1) as s:
        pid = s.add_problem(prob)
        exp = s.dmri_export_operator(pid)
    asm = fem.assemble(prob)
    n = asm.n_dof
    assert exp["w"].shape[0] == n
    perm = _lib_to_oracle_perm(prob, exp, asm)
    assert sorted(perm) == list(range(n))
    nnz = exp["col"].shape[0]
    rows = np.repeat(np.arange(n), np.diff(exp["row_ptr"]))
    P = sp.csr_matrix((np.ones(n), (np.arange(n), perm)), shape=(n, n))
    V = asm.B if prob.periodic_mask == 7 else asm.J
    refs = [asm.M, asm.S + asm.IG + asm.R2, asm.MD, V[0], V[1], V[2]]
    names = ["M", "R", "MD", "Vx", "Vy", "Vz"]
    for a in range(6):
        mine = sp.csr_matrix((exp["vals"][a], (rows, exp["col"])), shape=(n, n))
        ref = (P @ refs[a] @ P.T).tocsr()
        scale = abs(ref).max()
        diff = abs(mine - ref).max()
        assert diff <= 1e-12 * scale, (names[a], diff, scale)
    np.testing.assert_allclose(exp["w"], asm.w[perm], rtol=1e-13)
    np.testing.assert_allclose(exp["u0"], asm.u0[perm], rtol=0)
    # Every stored row holds its diagonal and the pattern is symmetric.
    pat = sp.csr_matrix((np.ones(nnz), (rows, exp["col"])), shape=(n, n))
    assert (pat != pat.T).nnz == 0
    assert np.all(pat.diagonal() == 1)


WEAK_CASES = {
    "free_matching": lambda: di.free_box(n=4, half=2.0, periodic_mask=15),
    "slab_x": lambda: di.slab_box(n=12, half=5.0, split=10.0, cross=(0.5, 1), periodic_mask=9),
    "nonmatching_cylinder": lambda: di.nonmatching_faces(
        di.conforming_cylinder_box(n=6, half=6.0, r=4.0, kappa=1e-2, D_in=1e-3,
                                   periodic_mask=13, seed=1), axes=(0, 2), amount=0.25, seed=7),
    "nonmatching_tensor": lambda: di.nonmatching_faces(
        di.conforming_cylinder_box(
            n=6, half=6.0, r=4.0, D_in=di.tensor([3e-3, 1e-3, 2e-3], (0.3, 0.5, 0.2)),
            D_out=di.tensor([2e-3, 2.5e-3, 4e-3], (1.0, -0.4, 0.7)), kappa=5e-3,
            periodic_mask=15, seed=3), amount=0.2, seed=2),
}


@pytest.mark.parametrize("name", sorted(WEAK_CASES))
def test_weak_faces_match_oracle(name):
    # kappa_e, the face mass and the partner couplings of weak
    # pseudo-periodic faces (exact overlap integrals on non-matching faces)
    # equal the oracle's entry by entry after matching DOFs.
    prob = WEAK_CASES[name]()
    with Simulator(-1) as s:
        pid = s.add_problem(prob)
        exp = s.dmri_export_operator(pid)
        wk = s.dmri_export_weak(pid)
    asm = fem.assemble(prob)
    n = asm.n_dof
    perm = _lib_to_oracle_perm(prob, exp, asm)
    P = sp.csr_matrix((np.ones(n), (np.arange(n), perm)), shape=(n, n))
    assert wk["kappa_e"] == pytest.approx(asm.kappa_e, rel=1e-13)
    rows = np.repeat(np.arange(n), np.diff(exp["row_ptr"]))
    KB = sp.csr_matrix((wk["face_mass"], (rows, exp["col"])), shape=(n, n))
    ref = (P @ asm.KB @ P.T).tocsr()
    assert abs(KB - ref).max() <= 1e-12 * abs(ref).max()
    slot_rows = np.repeat(wk["rows"], np.diff(wk["ptr"]))
    assert np.all(np.diff(wk["rows"]) > 0)
    axes = {a: (Cms, Csm) for a, Cms, Csm, _ in asm.weak}
    assert sorted(set(wk["code"] % 3)) == sorted(axes)
    for code in range(6):
        sel = wk["code"] == code
        mine = sp.csr_matrix((wk["val"][sel], (slot_rows[sel], wk["col"][sel])), shape=(n, n))
        a = code % 3
        if a not in axes:
            assert sel.sum() == 0
            continue
        ref = (P @ axes[a][0 if code < 3 else 1] @ P.T).tocsr()
        assert abs(mine - ref).max() <= 1e-12 * abs(ref).max(), code


def test_weak_face_validation():
    prob = di.free_box(n=4, half=2.0, periodic_mask=9)
    args = _prob_args(prob)
    with Simulator(-1) as s:
        for mask in (8, 16, 24):
            a = dict(args, periodic_mask=mask)
            with pytest.raises(DmriError, match="DMRI_E_UNSUPPORTED"):
                s.dmri_add_problem(**a)
        # a box face not fully meshed: drop the tets touching part of x = hi
        c = prob.xyz[prob.tets].mean(axis=1)
        keep = ~((c[:, 0] > 1.0) & (c[:, 1] > 1.0) & (c[:, 2] > 1.0))
        a = dict(args, tets=prob.tets[keep].copy(), tet_label=prob.tet_label[keep].copy())
        with pytest.raises(DmriError, match="not fully covered"):
            s.dmri_add_problem(**a)


def _prob_args(prob):
    return dict(xyz=prob.xyz.copy(), tets=prob.tets.copy(), tet_label=prob.tet_label.copy(),
                n_comp=prob.n_comp, D=np.array(prob.D, float), T2=None, u0=None,
                kappa=prob.kappa, box_lo=prob.box_lo, box_hi=prob.box_hi,
                periodic_mask=prob.periodic_mask)


def _expect(status_name, **over):
    prob = di.cylinder_box(n=4, half=6.0, r=4.0, kappa=1e-3)
    args = _prob_args(prob)
    args.update(over)
    with Simulator(-1) as s:
        with pytest.raises(DmriError) as ei:
            s.dmri_add_problem(**args)
    assert ei.value.args[0].startswith(status_name)


def test_validation_errors():
    prob = di.cylinder_box(n=4, half=6.0, r=4.0, kappa=1e-3)
    xyz = prob.xyz.copy()
    xyz[5, 1] = np.nan
    _expect("DMRI_E_INVALID", xyz=xyz)
    _expect("DMRI_E_INVALID", D=np.array([3e-3, 0.0]))
    _expect("DMRI_E_INVALID", D=np.array([3e-3, -1.0]))
    _expect("DMRI_E_INVALID", kappa=-1.0)
    _expect("DMRI_E_INVALID", T2=np.array([1e4, 0.0]))
    lab = prob.tet_label.copy()
    lab[3] = 2
    _expect("DMRI_E_INVALID", tet_label=lab)
    tets = prob.tets.copy()
    tets[7, 2] = prob.n_nodes
    _expect("DMRI_E_INVALID", tets=tets)
    tets = prob.tets.copy()
    tets[0, 1] = tets[0, 0]
    _expect("DMRI_E_INVALID", tets=tets)          # degenerate tetrahedron
    _expect("DMRI_E_UNSUPPORTED", periodic_mask=3)
    # A node of the upper x face moved off the face: opposite faces differ.
    xyz = prob.xyz.copy()
    on_hi = np.nonzero(np.isclose(xyz[:, 0], 6.0))[0]
    xyz[on_hi[4], 1] += 0.25
    _expect("DMRI_E_INVALID", xyz=xyz)
    _expect("DMRI_E_INVALID", box_lo=np.array([0.0, -6, -6]), box_hi=np.array([0.0, 6, 6]))


def test_sequence_and_option_validation():
    with Simulator(-1) as s:
        s.dmri_set_sequence_pgse(10600, 13400, 100, 0.5)
        for bad in [(10600, 13400, 300, 0.5), (10600, 13400, 100, 0.4), (10600, 13400, 0, 0.5),
                    (13400, 10600, 100, 0.5), (float("nan"), 13400, 100, 0.5)]:
            with pytest.raises(DmriError):
                s.dmri_set_sequence_pgse(*bad)
        s.dmri_set_option("rtol", 1e-8)
        assert s.dmri_get_option("rtol") == 1e-8
        assert s.dmri_get_option("inner_floor") == 0.25
        s.dmri_set_option("inner_floor", 1.0)
        assert s.dmri_get_option("inner_floor") == 1.0
        assert s.dmri_get_option("mesh_merge") == 0
        s.dmri_set_option("mesh_merge", 1)
        assert s.dmri_get_option("mesh_merge") == 1
        for k, v in [("rtol", 0.0), ("precision", 5), ("sys_tile", 12), ("nope", 1),
                     ("max_iter", 0), ("inner_floor", 0.0), ("inner_floor", 1.5),
                     ("mesh_merge", 2)]:
            with pytest.raises(DmriError):
                s.dmri_set_option(k, v)
        with pytest.raises(DmriError) as ei:
            s.dmri_run([0], [1000.0], [[1, 0, 0]])
        assert "DMRI_E_STATE" in str(ei.value)


def test_tuning_file_round_trip(tmp_path):
    # The autotuner cache file: entries merge into a handle and are written
    # back unchanged; malformed files are refused without changing anything.
    good = tmp_path / "t.txt"
    good.write_text("dmri-tuning-v1\n"
                    "gfx950_cu256/00ab12cd34ef5678/1024/1/0/0 64 512 0 0 0.125\n"
                    "gfx950_cu256/1111222233334444/32/0/0/0 32 256 1 0 0.0625\n")
    out = tmp_path / "o.txt"
    with Simulator(-1) as s:
        s.dmri_load_tuning(str(good))
        s.dmri_save_tuning(str(out))
        lines = out.read_text().splitlines()
        assert lines[0] == "dmri-tuning-v1"
        assert sorted(lines[1:]) == sorted(good.read_text().splitlines()[1:])
        for text in ["nope\n", "dmri-tuning-v1\nkey 12 512 0 0 0.1\n",
                     "dmri-tuning-v1\nkey 64 512 0 0\n", "dmri-tuning-v1\nkey 64 0 0 0 0.1\n",
                     "dmri-tuning-v1\nkey 64 512 0 0 0.1 extra\n"]:
            bad = tmp_path / "bad.txt"
            bad.write_text(text)
            with pytest.raises(DmriError, match="DMRI_E_INVALID"):
                s.dmri_load_tuning(str(bad))
        with pytest.raises(DmriError, match="DMRI_E_INVALID"):
            s.dmri_load_tuning(str(tmp_path / "missing.txt"))
        s.dmri_save_tuning(str(out))
        assert sorted(out.read_text().splitlines()[1:]) == sorted(lines[1:])


def test_marker_and_weak_options():
    with Simulator(-1) as s:
        for k, good, bad in (("markers", (0, 1), (2, -1, 0.5)), ("dir_bf16", (0, 1), (2, 0.5)),
                             ("spmv_rows", (1, 2), (0, 3, 1.5)),
                             ("weak_kappa", (0.5, 1e6), (0.0, 2e6))):
            for v in good:
                s.dmri_set_option(k, v)
                assert s.dmri_get_option(k) == v
            for v in bad:
                with pytest.raises(DmriError, match="DMRI_E_INVALID"):
                    s.dmri_set_option(k, v)


def test_preconditioner_options():
    # precond, cheb_terms ranges; the fixed interval keeps 0 < a, 1.001 a < b
    with Simulator(-1) as s:
        for k, good, bad in (("precond", (0, 1, 2), (3, -1, 0.5)),
                             ("cheb_terms", (1, 4, 16), (0, 17, 2.5))):
            for v in good:
                s.dmri_set_option(k, v)
                assert s.dmri_get_option(k) == v
            for v in bad:
                with pytest.raises(DmriError, match="DMRI_E_INVALID"):
                    s.dmri_set_option(k, v)
        assert (s.dmri_get_option("cheb_a"), s.dmri_get_option("cheb_b")) == (0.5, 1.5)
        s.dmri_set_option("cheb_b", 3.0)
        s.dmri_set_option("cheb_a", 0.1)
        assert (s.dmri_get_option("cheb_a"), s.dmri_get_option("cheb_b")) == (0.1, 3.0)
        for k, v in (("cheb_a", 3.0), ("cheb_a", 0.0), ("cheb_a", -1.0), ("cheb_b", 0.1),
                     ("cheb_b", 2e6)):
            with pytest.raises(DmriError, match="DMRI_E_INVALID"):
                s.dmri_set_option(k, v)
        assert (s.dmri_get_option("cheb_a"), s.dmri_get_option("cheb_b")) == (0.1, 3.0)
        assert s.dmri_get_option("pc_fallback_steps") == 0
        assert s.dmri_precond_record_count() == 0
