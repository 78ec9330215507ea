"""ctypes binding of libdmri (argument marshalling only).

Every computation runs in the C/HIP library; this module converts NumPy
arrays and PyTorch device tensors to pointers and status codes to
exceptions. Function names follow the C ABI declared in include/dmri.h.
If the shared library is missing the import fails loudly: there is no
Python or CPU fallback.
"""

from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libdmri.so")

DMRI_OK = 0
DMRI_NOT_CONVERGED = 1
STATUS_NAMES = {
    0: "DMRI_OK", 1: "DMRI_NOT_CONVERGED", -1: "DMRI_E_INVALID", -2: "DMRI_E_STATE",
    -3: "DMRI_E_NOMEM", -4: "DMRI_E_DEVICE", -5: "DMRI_E_UNSUPPORTED",
}

# Symbols declared in include/dmri.h (checked by the CPU test suite).
EXPORTED = [
    "dmri_create", "dmri_destroy", "dmri_last_error", "dmri_add_problem",
    "dmri_add_problem_tensor", "dmri_problem_info",
    "dmri_export_operator", "dmri_export_weak", "dmri_set_sequence_pgse", "dmri_set_sequence",
    "dmri_set_sequence_table", "dmri_set_option", "dmri_get_option",
    "dmri_run", "dmri_run_device", "dmri_run_device_noalloc", "dmri_apply_operator",
    "dmri_guess_set_params", "dmri_guess_get_params", "dmri_load_guess_model",
    "dmri_save_guess_model", "dmri_guess_record", "dmri_guess_record_count", "dmri_guess_eval",
    "dmri_guess_train", "dmri_save_tuning", "dmri_load_tuning", "dmri_precond_set_params",
    "dmri_precond_get_params", "dmri_precond_record", "dmri_precond_record_count",
    "dmri_precond_train",
]

SEQ_KINDS = {"pgse": 0, "double_pgse": 1, "cos_ogse": 2, "sin_ogse": 3, "trap_pgse": 4,
             "double_trap_pgse": 5}

GUESS_N_FEATURES = 16
GUESS_N_PARAMS = 5378


class DmriError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class Stats(C.Structure):
    _fields_ = [
        ("n_sys", C.c_int64),
        ("iters_total", C.POINTER(C.c_int32)),
        ("converged", C.POINTER(C.c_uint8)),
        ("final_rel_res", C.POINTER(C.c_double)),
        ("t_setup_s", C.c_double),
        ("t_solve_s", C.c_double),
        ("t_signal_s", C.c_double),
        ("total_iterations", C.c_int64),
        ("spmv_rows", C.c_int64),
        ("n_steps", C.c_int64),
        ("n_kernel_launches", C.c_int64),
        ("t_kernel_s", C.c_double),
    ]


_lib = None


def load(path: Optional[str] = None):
    """Load libdmri.so (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise ImportError("libdmri.so not found at %s: build it with "
                          "`python -c 'import __graft_entry__ as g; g.build()'`" % p)
    lib = C.CDLL(p)
    P = C.POINTER
    dbl, i32, i64 = C.c_double, C.c_int32, C.c_int64
    vp = C.c_void_p
    lib.dmri_create.argtypes = [C.c_int, P(vp)]
    lib.dmri_destroy.argtypes = [vp]
    lib.dmri_destroy.restype = None
    lib.dmri_last_error.argtypes = [vp]
    lib.dmri_last_error.restype = C.c_char_p
    lib.dmri_add_problem.argtypes = [vp, i64, vp, i64, vp, vp, i32, vp, vp, vp, dbl, vp, vp,
                                     C.c_uint32, P(i32)]
    lib.dmri_add_problem_tensor.argtypes = [vp, i64, vp, i64, vp, vp, i32, vp, vp, vp, dbl, vp,
                                            vp, C.c_uint32, P(i32)]
    lib.dmri_problem_info.argtypes = [vp, i32, P(i64), P(i64)]
    lib.dmri_export_operator.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
    lib.dmri_export_weak.argtypes = [vp, i32, P(i64), P(i64), P(dbl), vp, vp, vp, vp, vp, vp]
    lib.dmri_set_sequence_pgse.argtypes = [vp, dbl, dbl, dbl, dbl]
    lib.dmri_set_sequence.argtypes = [vp, i32, vp, i32, dbl, dbl]
    lib.dmri_set_sequence_table.argtypes = [vp, i64, dbl, dbl, vp, vp, vp, dbl]
    lib.dmri_set_option.argtypes = [vp, C.c_char_p, dbl]
    lib.dmri_get_option.argtypes = [vp, C.c_char_p, P(dbl)]
    lib.dmri_guess_set_params.argtypes = [vp, vp, i64]
    lib.dmri_guess_get_params.argtypes = [vp, vp, i64]
    lib.dmri_load_guess_model.argtypes = [vp, C.c_char_p]
    lib.dmri_save_guess_model.argtypes = [vp, C.c_char_p]
    lib.dmri_save_tuning.argtypes = [vp, C.c_char_p]
    lib.dmri_load_tuning.argtypes = [vp, C.c_char_p]
    lib.dmri_guess_record.argtypes = [vp, vp, vp, i64, i64]
    lib.dmri_guess_record_count.argtypes = [vp, P(i64)]
    lib.dmri_guess_eval.argtypes = [vp, i64, vp, vp, vp, vp, P(dbl)]
    lib.dmri_guess_train.argtypes = [vp, i64, vp, vp, i32, dbl, P(dbl), P(dbl)]
    lib.dmri_precond_set_params.argtypes = [vp, vp, i64]
    lib.dmri_precond_get_params.argtypes = [vp, vp, i64]
    lib.dmri_precond_record.argtypes = [vp, vp, vp, i64]
    lib.dmri_precond_record_count.argtypes = [vp, P(i64)]
    lib.dmri_precond_train.argtypes = [vp, i64, vp, vp, i32, dbl, P(dbl), P(dbl)]
    lib.dmri_run.argtypes = [vp, i64, vp, vp, vp, vp, P(Stats)]
    lib.dmri_run_device.argtypes = [vp, vp, i64, vp, vp, vp, vp, P(Stats)]
    lib.dmri_run_device_noalloc.argtypes = [vp, vp, i64, vp, vp, vp, vp, P(Stats)]
    lib.dmri_apply_operator.argtypes = [vp, i32, i32, i64, vp, vp, vp, vp]
    for name in EXPORTED:
        f = getattr(lib, name)
        if name not in ("dmri_destroy", "dmri_last_error"):
            f.restype = C.c_int
    if path is None:
        _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


class Simulator:
    """Owns one dmri_handle. device=-1 gives a host-only context."""

    def __init__(self, device: int = 0):
        self.lib = load()
        h = C.c_void_p()
        st = self.lib.dmri_create(int(device), C.byref(h))
        if st != DMRI_OK:
            raise DmriError(st, self.lib.dmri_last_error(None).decode())
        self.h = h
        self.device = device

    # -- errors -------------------------------------------------------------
    def _check(self, st: int, allow_nc: bool = False) -> int:
        if st == DMRI_OK or (allow_nc and st == DMRI_NOT_CONVERGED):
            return st
        raise DmriError(st, self.lib.dmri_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.dmri_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- problems -----------------------------------------------------------
    def dmri_add_problem(self, xyz, tets, tet_label, n_comp, D, T2=None, u0=None, kappa=0.0,
                         box_lo=(0, 0, 0), box_hi=(1, 1, 1), periodic_mask=7) -> int:
        xyz = _c(xyz, np.float64).reshape(-1, 3)
        tets = _c(tets, np.int32).reshape(-1, 4)
        lab = _c(tet_label, np.int32).reshape(-1)
        D = _c(D, np.float64)
        T2 = _c(T2, np.float64)
        u0 = _c(u0, np.float64)
        lo = _c(box_lo, np.float64)
        hi = _c(box_hi, np.float64)
        pid = C.c_int32(-1)
        self._check(self.lib.dmri_add_problem(
            self.h, xyz.shape[0], _ptr(xyz), tets.shape[0], _ptr(tets), _ptr(lab), int(n_comp),
            _ptr(D), _ptr(T2), _ptr(u0), float(kappa), _ptr(lo), _ptr(hi),
            int(periodic_mask), C.byref(pid)))
        return pid.value

    def dmri_add_problem_tensor(self, xyz, tets, tet_label, n_comp, D_tensor, T2=None, u0=None,
                                kappa=0.0, box_lo=(0, 0, 0), box_hi=(1, 1, 1),
                                periodic_mask=7) -> int:
        """D_tensor: [n_comp][6] (xx, yy, zz, xy, xz, yz) or [n_comp][3][3]."""
        Dt = np.asarray(D_tensor, dtype=np.float64)
        if Dt.ndim == 3:
            Dt = np.stack([Dt[:, 0, 0], Dt[:, 1, 1], Dt[:, 2, 2], Dt[:, 0, 1], Dt[:, 0, 2],
                           Dt[:, 1, 2]], axis=1)
        Dt = _c(Dt.reshape(-1, 6), np.float64)
        xyz = _c(xyz, np.float64).reshape(-1, 3)
        tets = _c(tets, np.int32).reshape(-1, 4)
        lab = _c(tet_label, np.int32).reshape(-1)
        T2 = _c(T2, np.float64)
        u0 = _c(u0, np.float64)
        lo = _c(box_lo, np.float64)
        hi = _c(box_hi, np.float64)
        pid = C.c_int32(-1)
        self._check(self.lib.dmri_add_problem_tensor(
            self.h, xyz.shape[0], _ptr(xyz), tets.shape[0], _ptr(tets), _ptr(lab), int(n_comp),
            _ptr(Dt), _ptr(T2), _ptr(u0), float(kappa), _ptr(lo), _ptr(hi),
            int(periodic_mask), C.byref(pid)))
        return pid.value

    def add_problem(self, prob) -> int:
        """Add a dmri_inputs.Problem-like object (fields as in include/dmri.h);
        a D of shape [n_comp, 3, 3] adds it with diffusion tensors."""
        if np.asarray(prob.D).ndim == 3:
            return self.dmri_add_problem_tensor(prob.xyz, prob.tets, prob.tet_label, prob.n_comp,
                                                prob.D, prob.T2, prob.u0, prob.kappa,
                                                prob.box_lo, prob.box_hi, prob.periodic_mask)
        return self.dmri_add_problem(prob.xyz, prob.tets, prob.tet_label, prob.n_comp, prob.D,
                                     prob.T2, prob.u0, prob.kappa, prob.box_lo, prob.box_hi,
                                     prob.periodic_mask)

    def dmri_problem_info(self, pid: int):
        n, z = C.c_int64(), C.c_int64()
        self._check(self.lib.dmri_problem_info(self.h, int(pid), C.byref(n), C.byref(z)))
        return n.value, z.value

    def dmri_export_operator(self, pid: int) -> dict:
        n, nnz = self.dmri_problem_info(pid)
        out = {
            "row_ptr": np.empty(n + 1, np.int32), "col": np.empty(nnz, np.int32),
            "vals": np.empty((6, nnz), np.float64), "w": np.empty(n, np.float64),
            "u0": np.empty(n, np.float64), "dof_comp": np.empty(n, np.int32),
            "dof_node": np.empty(n, np.int32),
        }
        self._check(self.lib.dmri_export_operator(
            self.h, int(pid), _ptr(out["row_ptr"]), _ptr(out["col"]), _ptr(out["vals"]),
            _ptr(out["w"]), _ptr(out["u0"]), _ptr(out["dof_comp"]), _ptr(out["dof_node"])))
        return out

    def dmri_export_weak(self, pid: int) -> dict:
        ns, ne, ke = C.c_int64(), C.c_int64(), C.c_double()
        self._check(self.lib.dmri_export_weak(self.h, int(pid), C.byref(ns), C.byref(ne),
                                              C.byref(ke), None, None, None, None, None, None))
        _, nnz = self.dmri_problem_info(pid)
        out = {"kappa_e": ke.value, "rows": np.empty(ns.value, np.int32),
               "ptr": np.empty(ns.value + 1, np.int32), "col": np.empty(ne.value, np.int32),
               "code": np.empty(ne.value, np.int32), "val": np.empty(ne.value, np.float64),
               "face_mass": np.zeros(nnz, np.float64)}
        if ns.value == 0:
            return out
        self._check(self.lib.dmri_export_weak(
            self.h, int(pid), C.byref(ns), C.byref(ne), C.byref(ke), _ptr(out["rows"]),
            _ptr(out["ptr"]), _ptr(out["col"]), _ptr(out["code"]), _ptr(out["val"]),
            _ptr(out["face_mass"])))
        return out

    # -- sequence and options -----------------------------------------------
    def dmri_set_sequence_pgse(self, delta, Delta, dt, theta=0.5):
        self._check(self.lib.dmri_set_sequence_pgse(self.h, float(delta), float(Delta),
                                                    float(dt), float(theta)))

    def dmri_set_sequence(self, kind, params, dt, theta=0.5):
        k = SEQ_KINDS[kind] if isinstance(kind, str) else int(kind)
        p = _c(np.atleast_1d(params), np.float64)
        self._check(self.lib.dmri_set_sequence(self.h, k, _ptr(p), p.shape[0], float(dt),
                                               float(theta)))

    def dmri_set_sequence_table(self, dt, theta, F, f_start=None, f_end=None, int_F2=None):
        F = _c(F, np.float64)
        fs = _c(f_start, np.float64)
        fe = _c(f_end, np.float64)
        self._check(self.lib.dmri_set_sequence_table(self.h, F.shape[0] - 1, float(dt),
                                                     float(theta), _ptr(F), _ptr(fs), _ptr(fe),
                                                     float(int_F2)))

    def set_sequence(self, seq):
        """A dmri_inputs.Sequence (PGSE) or GeneralSequence (kind, params)."""
        if hasattr(seq, "kind"):
            self.dmri_set_sequence(seq.kind, seq.params, seq.dt, seq.theta)
        else:
            self.dmri_set_sequence_pgse(seq.delta, seq.Delta, seq.dt, seq.theta)

    def dmri_set_option(self, key: str, value: float):
        self._check(self.lib.dmri_set_option(self.h, key.encode(), float(value)))

    def dmri_get_option(self, key: str) -> float:
        v = C.c_double()
        self._check(self.lib.dmri_get_option(self.h, key.encode(), C.byref(v)))
        return v.value

    def set_options(self, **kw):
        for k, v in kw.items():
            self.dmri_set_option(k, v)

    # -- learned initial guess -----------------------------------------------
    def dmri_guess_set_params(self, params):
        p = _c(params, np.float32).reshape(-1)
        self._check(self.lib.dmri_guess_set_params(self.h, _ptr(p), p.shape[0]))

    def dmri_guess_get_params(self) -> np.ndarray:
        p = np.empty(GUESS_N_PARAMS, np.float32)
        self._check(self.lib.dmri_guess_get_params(self.h, _ptr(p), p.shape[0]))
        return p

    def dmri_load_guess_model(self, path: str):
        self._check(self.lib.dmri_load_guess_model(self.h, os.fsencode(path)))

    def dmri_save_tuning(self, path: str):
        self._check(self.lib.dmri_save_tuning(self.h, os.fsencode(path)))

    def dmri_load_tuning(self, path: str):
        self._check(self.lib.dmri_load_tuning(self.h, os.fsencode(path)))

    def dmri_save_guess_model(self, path: str):
        self._check(self.lib.dmri_save_guess_model(self.h, os.fsencode(path)))

    def dmri_guess_record(self, features_dev, targets_dev, capacity: int, stride: int):
        """Record samples into torch float32 CUDA tensors [capacity, 16] and
        [capacity, 2] during later runs (capacity 0 stops recording)."""
        if capacity > 0:
            _dev_f32(features_dev, (capacity, GUESS_N_FEATURES))
            _dev_f32(targets_dev, (capacity, 2))
        self._check(self.lib.dmri_guess_record(
            self.h, _dptr(features_dev) if capacity > 0 else None,
            _dptr(targets_dev) if capacity > 0 else None, int(capacity), int(stride)))

    def dmri_guess_record_count(self) -> int:
        n = C.c_int64()
        self._check(self.lib.dmri_guess_record_count(self.h, C.byref(n)))
        return n.value

    def dmri_guess_eval(self, features_dev, targets_dev=None, out_dev=None, grad_dev=None,
                        want_loss: bool = True):
        """Network outputs / loss gradient / loss on n device samples."""
        n = int(features_dev.shape[0])
        _dev_f32(features_dev, (n, GUESS_N_FEATURES))
        if targets_dev is not None:
            _dev_f32(targets_dev, (n, 2))
        if out_dev is not None:
            _dev_f32(out_dev, (n, 2))
        if grad_dev is not None:
            _dev_f32(grad_dev, (GUESS_N_PARAMS,))
        loss = C.c_double(float("nan"))
        _sync(features_dev)
        self._check(self.lib.dmri_guess_eval(
            self.h, n, _dptr(features_dev), _dptr(targets_dev), _dptr(out_dev), _dptr(grad_dev),
            C.byref(loss) if want_loss and targets_dev is not None else None))
        return loss.value

    def dmri_guess_train(self, features_dev, targets_dev, n_iters: int, lr: float, n=None):
        """Full-batch Adam steps; returns (loss before the first, before the last step)."""
        n = int(features_dev.shape[0]) if n is None else int(n)
        _dev_f32(features_dev, None)
        _dev_f32(targets_dev, None)
        if n > features_dev.shape[0] or n > targets_dev.shape[0]:
            raise ValueError("n exceeds the sample buffers")
        l0, l1 = C.c_double(), C.c_double()
        _sync(features_dev)
        self._check(self.lib.dmri_guess_train(self.h, n, _dptr(features_dev), _dptr(targets_dev),
                                              int(n_iters), float(lr), C.byref(l0), C.byref(l1)))
        return l0.value, l1.value

    # -- preconditioner network -------------------------------------------
    def dmri_precond_set_params(self, params):
        p = _c(params, np.float32).reshape(-1)
        self._check(self.lib.dmri_precond_set_params(self.h, _ptr(p), p.shape[0]))

    def dmri_precond_get_params(self) -> np.ndarray:
        p = np.empty(GUESS_N_PARAMS, np.float32)
        self._check(self.lib.dmri_precond_get_params(self.h, _ptr(p), p.shape[0]))
        return p

    def dmri_precond_record(self, features_dev, targets_dev, capacity: int):
        """Record (system, step) samples of Jacobi-CG runs into torch float32
        CUDA tensors [capacity, 16] and [capacity, 2] (capacity 0 stops)."""
        if capacity > 0:
            _dev_f32(features_dev, (capacity, GUESS_N_FEATURES))
            _dev_f32(targets_dev, (capacity, 2))
        self._check(self.lib.dmri_precond_record(
            self.h, _dptr(features_dev) if capacity > 0 else None,
            _dptr(targets_dev) if capacity > 0 else None, int(capacity)))

    def dmri_precond_record_count(self) -> int:
        n = C.c_int64()
        self._check(self.lib.dmri_precond_record_count(self.h, C.byref(n)))
        return n.value

    def dmri_precond_train(self, features_dev, targets_dev, n_iters: int, lr: float, n=None):
        """Full-batch Adam steps; returns (loss before the first, before the last step)."""
        n = int(features_dev.shape[0]) if n is None else int(n)
        _dev_f32(features_dev, None)
        _dev_f32(targets_dev, None)
        if n > features_dev.shape[0] or n > targets_dev.shape[0]:
            raise ValueError("n exceeds the sample buffers")
        l0, l1 = C.c_double(), C.c_double()
        _sync(features_dev)
        self._check(self.lib.dmri_precond_train(self.h, n, _dptr(features_dev),
                                                _dptr(targets_dev), int(n_iters), float(lr),
                                                C.byref(l0), C.byref(l1)))
        return l0.value, l1.value

    # -- runs ---------------------------------------------------------------
    def dmri_run(self, problem_id: Sequence[int], b, q, want_stats: bool = True):
        """Signals (complex128 [n]) and a stats dict."""
        b = _c(np.atleast_1d(b), np.float64)
        n = b.shape[0]
        pid = _c(np.broadcast_to(np.asarray(problem_id, dtype=np.int32), (n,)), np.int32)
        q = _c(q, np.float64).reshape(n, 3)
        sig = np.empty((n, 2), np.float64)
        iters = np.zeros(n, np.int32)
        conv = np.zeros(n, np.uint8)
        rres = np.zeros(n, np.float64)
        st = Stats()
        st.iters_total = iters.ctypes.data_as(C.POINTER(C.c_int32))
        st.converged = conv.ctypes.data_as(C.POINTER(C.c_uint8))
        st.final_rel_res = rres.ctypes.data_as(C.POINTER(C.c_double))
        status = self._check(self.lib.dmri_run(self.h, n, _ptr(pid), _ptr(b), _ptr(q),
                                               _ptr(sig), C.byref(st)), allow_nc=True)
        stats = _stats_dict(st, iters, conv, rres, status)
        return sig[:, 0] + 1j * sig[:, 1], stats

    def dmri_run_device(self, pid_dev, b_dev, q_dev, sig_dev, stream_ptr=None):
        """Device-resident run. pid_dev is a torch int32 CUDA tensor [n] (or an
        int: one problem for every pair, placed in a device tensor here);
        b_dev/q_dev/sig_dev are torch float64 CUDA tensors ([n], [n,3], [n,2]);
        stream_ptr is a raw HIP stream handle or None."""
        import torch
        n = int(b_dev.shape[0])
        made = isinstance(pid_dev, (int, np.integer))
        if made:
            pid_dev = torch.full((n,), int(pid_dev), dtype=torch.int32, device=b_dev.device)
        if pid_dev.dtype != torch.int32 or tuple(pid_dev.shape) != (n,):
            raise ValueError("problem ids must be an int32 tensor of shape [n]")
        for t in (pid_dev, b_dev, q_dev, sig_dev):
            if not t.is_contiguous():
                raise ValueError("tensors must be contiguous")
        if made or stream_ptr is None:
            _sync(b_dev)  # torch's pending work, when the library runs on its own stream
        st = Stats()
        status = self._check(self.lib.dmri_run_device(
            self.h, None if stream_ptr is None else C.c_void_p(stream_ptr), n,
            C.c_void_p(pid_dev.data_ptr()), C.c_void_p(b_dev.data_ptr()),
            C.c_void_p(q_dev.data_ptr()), C.c_void_p(sig_dev.data_ptr()), C.byref(st)),
            allow_nc=True)
        return _stats_dict(st, None, None, None, status)

    def dmri_run_device_noalloc(self, pid_dev, b_dev, q_dev, sig_dev, stream_ptr=None):
        """As dmri_run_device, through the entry point that allocates no device
        memory (pid_dev must be an int32 CUDA tensor [n], n <= 64)."""
        import torch
        n = int(b_dev.shape[0])
        if pid_dev.dtype != torch.int32 or tuple(pid_dev.shape) != (n,):
            raise ValueError("problem ids must be an int32 tensor of shape [n]")
        for t in (pid_dev, b_dev, q_dev, sig_dev):
            if not t.is_contiguous():
                raise ValueError("tensors must be contiguous")
        if stream_ptr is None:
            _sync(b_dev)
        iters = np.zeros(n, np.int32)
        conv = np.zeros(n, np.uint8)
        rres = np.zeros(n, np.float64)
        st = Stats()
        st.iters_total = iters.ctypes.data_as(C.POINTER(C.c_int32))
        st.converged = conv.ctypes.data_as(C.POINTER(C.c_uint8))
        st.final_rel_res = rres.ctypes.data_as(C.POINTER(C.c_double))
        status = self._check(self.lib.dmri_run_device_noalloc(
            self.h, None if stream_ptr is None else C.c_void_p(stream_ptr), n,
            C.c_void_p(pid_dev.data_ptr()), C.c_void_p(b_dev.data_ptr()),
            C.c_void_p(q_dev.data_ptr()), C.c_void_p(sig_dev.data_ptr()), C.byref(st)),
            allow_nc=True)
        return _stats_dict(st, iters, conv, rres, status)

    def dmri_apply_operator(self, pid: int, which: int, c, d, x):
        c = _c(c, np.float64).reshape(-1)
        ns = c.shape[0]
        d = _c(d, np.float64).reshape(ns, 3)
        x = np.asarray(x)
        n = x.shape[0]
        xr = np.empty((n, ns, 2), np.float64)
        xr[..., 0] = x.real
        xr[..., 1] = x.imag
        y = np.empty_like(xr)
        self._check(self.lib.dmri_apply_operator(self.h, int(pid), int(which), ns, _ptr(c),
                                                 _ptr(d), _ptr(xr), _ptr(y)))
        return y[..., 0] + 1j * y[..., 1]


def _dptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev_f32(t, shape):
    import torch
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous float32 CUDA tensor")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("expected shape %s, got %s" % (shape, tuple(t.shape)))


def _sync(t):
    """Finish torch's pending work on the tensor's device: the library runs on
    its own stream."""
    import torch
    torch.cuda.current_stream(t.device).synchronize()


def _stats_dict(st, iters, conv, rres, status):
    return {
        "status": STATUS_NAMES.get(status, status),
        "iters_total": iters, "converged": conv, "final_rel_res": rres,
        "total_iterations": st.total_iterations, "spmv_rows": st.spmv_rows,
        "n_steps": st.n_steps, "t_setup_s": st.t_setup_s, "t_solve_s": st.t_solve_s,
        "t_signal_s": st.t_signal_s, "n_kernel_launches": st.n_kernel_launches,
        "t_kernel_s": st.t_kernel_s,
    }
