"""ctypes binding of ``libfracprec.so`` (the C ABI in ``include/fracprec.h``).

Argument marshalling only: every step of the preconditioned solve runs in the
library's HIP kernels.  PyTorch provides device memory and the stream; the
library is bound to ``torch.cuda.current_stream()`` at construction.  There
is no fallback: a missing library or a missing GPU raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfracprec.so")

FPC_HOST, FPC_DEVICE = 0, 1
FPC_TUP, FPC_TPU, FPC_TUP_STAR = 0, 1, 2
FPC_FP64, FPC_FP32_PREC = 0, 1

STATUS = {0: "FPC_OK", 1: "FPC_NOT_CONVERGED", -1: "FPC_ERR_ARG",
          -2: "FPC_ERR_DIM", -3: "FPC_ERR_PATTERN",
          -4: "FPC_ERR_SINGULAR_BLOCK", -5: "FPC_ERR_NOT_SPD",
          -6: "FPC_ERR_NAN", -7: "FPC_ERR_HIP", -8: "FPC_ERR_OOM",
          -9: "FPC_ERR_STATE", -10: "FPC_ERR_UNSUPPORTED"}


class FpcCsr(C.Structure):
    _fields_ = [("nrows", C.c_int64), ("ncols", C.c_int64),
                ("nnz", C.c_int64), ("rowptr", C.c_void_p),
                ("colind", C.c_void_p), ("val", C.c_void_p)]


class FpcBlockSystem(C.Structure):
    _fields_ = [("n_u", C.c_int64), ("n_t", C.c_int64), ("n_p", C.c_int64),
                ("A", FpcCsr), ("C1", FpcCsr), ("Q1", FpcCsr),
                ("C2", FpcCsr), ("H", FpcCsr), ("Q2", FpcCsr),
                ("T", FpcCsr), ("coords", C.c_void_p),
                ("ptr_space", C.c_int)]


class FpcAmgOptions(C.Structure):
    _fields_ = [("max_coarse", C.c_int), ("max_levels", C.c_int),
                ("cheb_degree", C.c_int), ("cheb_ratio", C.c_double),
                ("power_its", C.c_int), ("lam_safety", C.c_double),
                ("omega_factor", C.c_double), ("drop_tol", C.c_double)]


class FpcOptions(C.Structure):
    _fields_ = [("mode", C.c_int), ("precision", C.c_int),
                ("restart", C.c_int), ("maxit", C.c_int),
                ("rtol", C.c_double), ("max_batch", C.c_int),
                ("graphs", C.c_int), ("ortho", C.c_int),
                ("tune", C.c_int), ("amg", FpcAmgOptions)]


class FpcInfo(C.Structure):
    _fields_ = [("iterations", C.c_int), ("restarts", C.c_int),
                ("converged", C.c_int), ("true_rel_residual", C.c_double),
                ("est_rel_residual", C.c_double), ("seconds", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FpcLevelDesc(C.Structure):
    _fields_ = [("n_nodes", C.c_int64), ("n_dofs", C.c_int64),
                ("block", C.c_int), ("nnzb", C.c_int64),
                ("nnz_scalar", C.c_int64), ("p_nnzb", C.c_int64),
                ("r_nnzb", C.c_int64), ("lam_hi", C.c_double),
                ("n_agg", C.c_int64), ("layout", C.c_int * 3),
                ("tune_us", C.c_double * 3)]

    def as_dict(self):
        out = {k: getattr(self, k) for k, _ in self._fields_}
        out["layout"] = list(self.layout)
        out["tune_us"] = list(self.tune_us)
        return out


class FpcPressureDesc(C.Structure):
    _fields_ = [("n_levels", C.c_int), ("n_fronts", C.c_int64),
                ("factor_entries", C.c_int64), ("solve_bytes", C.c_int64),
                ("max_pivots", C.c_int64), ("max_boundary", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FpcFlowGraph(C.Structure):
    _fields_ = [("n_p", C.c_int64), ("n_pairs", C.c_int64),
                ("pair_k", C.c_void_p), ("pair_l", C.c_void_p),
                ("ndir", C.c_void_p), ("upsilon", C.c_void_p)]


EXPORTS = ("fpc_default_options", "fpc_create", "fpc_setup", "fpc_apply_prec",
           "fpc_apply_prec_T", "fpc_matvec", "fpc_vcycle", "fpc_solve",
           "fpc_solve_T", "fpc_solve_batch", "fpc_grad_log_trans",
           "fpc_num_levels", "fpc_level_info", "fpc_export_aggregates",
           "fpc_export_level_matrix", "fpc_setup_times", "fpc_destroy",
           "fpc_status_string", "fpc_last_error", "fpc_hash32_device",
           "fpc_kernel_timer", "fpc_psolve", "fpc_stream_triad",
           "fpc_update_values", "fpc_hierarchy_reused",
           "fpc_grad_log_trans_noalloc", "fpc_pressure_info",
           "fpc_dense_inverse")

_lib = None


def load_library(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build it with __graft_entry__.build() "
            "(hipcc, gfx950)")
    # torch ships its own HIP runtime (soname libamdhip64.so.7, opened by
    # torch under another name): loaded first, it is the one this library
    # binds to, so both share one runtime, its streams and allocations.
    # Loading this library first would bring in a second runtime.
    import torch  # noqa: F401
    lib = C.CDLL(path)
    vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
    H = C.c_void_p
    sig = {
        "fpc_default_options": (None, [C.POINTER(FpcOptions)]),
        "fpc_create": (i32, [C.POINTER(H), C.POINTER(FpcOptions), vp]),
        "fpc_setup": (i32, [H, C.POINTER(FpcBlockSystem)]),
        "fpc_update_values": (i32, [H, C.POINTER(FpcBlockSystem)]),
        "fpc_hierarchy_reused": (i32, [H]),
        "fpc_apply_prec": (i32, [H, vp, vp]),
        "fpc_apply_prec_T": (i32, [H, vp, vp]),
        "fpc_matvec": (i32, [H, i32, vp, vp]),
        "fpc_vcycle": (i32, [H, vp, vp]),
        "fpc_psolve": (i32, [H, i32, vp, vp]),
        "fpc_stream_triad": (i32, [H, i64, vp, vp, dbl, vp]),
        "fpc_solve": (i32, [H, vp, vp, dbl, i32, C.POINTER(FpcInfo)]),
        "fpc_solve_T": (i32, [H, vp, vp, dbl, C.POINTER(FpcInfo)]),
        "fpc_solve_batch": (i32, [H, i32, vp, i64, vp, i64, dbl,
                                  C.POINTER(FpcInfo)]),
        "fpc_grad_log_trans": (i32, [H, C.POINTER(FpcFlowGraph), vp, vp, vp]),
        "fpc_grad_log_trans_noalloc": (i32, [H, C.POINTER(FpcFlowGraph), vp,
                                             vp, vp]),
        "fpc_pressure_info": (i32, [H, C.POINTER(FpcPressureDesc)]),
        "fpc_dense_inverse": (i32, [H, i64, vp]),
        "fpc_num_levels": (i32, [H]),
        "fpc_level_info": (i32, [H, i32, C.POINTER(FpcLevelDesc)]),
        "fpc_export_aggregates": (i32, [H, i32, vp, vp]),
        "fpc_export_level_matrix": (i32, [H, i32, i32, vp, vp, vp]),
        "fpc_setup_times": (i32, [H, vp]),
        "fpc_destroy": (None, [H]),
        "fpc_status_string": (C.c_char_p, [i32]),
        "fpc_last_error": (C.c_char_p, [H]),
        "fpc_hash32_device": (i32, [H, C.c_uint32, i64, vp]),
        "fpc_kernel_timer": (i32, [H, i32, i32, C.POINTER(C.c_int64),
                                   C.POINTER(C.c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class FpcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def default_options(**kw) -> FpcOptions:
    lib = load_library()
    o = FpcOptions()
    lib.fpc_default_options(C.byref(o))
    amg = kw.pop("amg", None) or {}
    for k, v in kw.items():
        if k == "mode":
            v = {"tup": FPC_TUP, "tpu": FPC_TPU,
                 "tup_star": FPC_TUP_STAR}.get(v, v)
        if k == "ortho":
            v = {"cgs2": 0, "mgs": 1, "dcgs2": 2}.get(v, v)
        if k == "precision":
            v = {"fp64": FPC_FP64, "fp32": FPC_FP32_PREC,
                 "fp32prec": FPC_FP32_PREC}.get(v, v)
        setattr(o, k, v)
    for k, v in amg.items():
        setattr(o.amg, k, v)
    return o


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("fracprec needs a ROCm GPU (torch.cuda unavailable)")
    return torch


class Solver:
    """Block-preconditioned FGMRES on one GPU.

    ``blocks`` maps ``A, C1, Q1, C2, H, Q2, T`` to SciPy CSR matrices (host)
    or to ``(rowptr int64, colind int32, val float64)`` CUDA tensors
    (device); ``coords`` is ``(n_u/3, 3)`` or None.
    """

    def __init__(self, blocks: Dict, n_u: int, n_t: int, n_p: int,
                 coords=None, device: int = 0, **opts):
        torch = _torch()
        self.lib = load_library()
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.n_u, self.n_t, self.n_p = int(n_u), int(n_t), int(n_p)
        self.N = self.n_u + self.n_t + self.n_p
        self.opts = default_options(**opts)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
        self.h = C.c_void_p()
        st = self.lib.fpc_create(C.byref(self.h), C.byref(self.opts),
                                 C.c_void_p(self.stream.cuda_stream))
        if st != 0:
            raise FpcError(st, "fpc_create failed")
        self.setup(blocks, coords)

    # -- plumbing ---------------------------------------------------------
    def _check(self, st, what):
        if st < 0:
            msg = self.lib.fpc_last_error(self.h).decode()
            raise FpcError(st, f"{what}: {msg}")
        return st

    def _ptr(self, t):
        if not (t.is_cuda and t.dtype == self.torch.float64
                and t.is_contiguous()):
            raise TypeError("expected a contiguous float64 CUDA tensor")
        return C.c_void_p(t.data_ptr())

    def _vec(self, n=None):
        return self.torch.empty(n or self.N, dtype=self.torch.float64,
                                device=self.device)

    @staticmethod
    def _csr_host(M, keep):
        import scipy.sparse as sp
        M = sp.csr_matrix(M)
        rp = np.ascontiguousarray(M.indptr, dtype=np.int64)
        ci = np.ascontiguousarray(M.indices, dtype=np.int32)
        va = np.ascontiguousarray(M.data, dtype=np.float64)
        keep += [rp, ci, va]
        return FpcCsr(M.shape[0], M.shape[1], M.nnz, rp.ctypes.data,
                      ci.ctypes.data, va.ctypes.data)

    def setup(self, blocks, coords=None):
        """(Re)build the preconditioner for a new Jacobian."""
        sysm, keep = self._system(blocks, coords)
        self._check(self.lib.fpc_setup(self.h, C.byref(sysm)), "fpc_setup")
        del keep

    def update_values(self, blocks):
        """Numeric re-setup for a new Jacobian of the same sizes (next Newton
        or active-set iteration); the setup's coordinates are kept."""
        sysm, keep = self._system(blocks, None)
        self._check(self.lib.fpc_update_values(self.h, C.byref(sysm)),
                    "fpc_update_values")
        del keep

    def hierarchy_reused(self):
        return bool(self.lib.fpc_hierarchy_reused(self.h) == 1)

    def _system(self, blocks, coords):
        keep = []
        first = blocks["A"]
        device = isinstance(first, tuple)
        sysm = FpcBlockSystem()
        sysm.n_u, sysm.n_t, sysm.n_p = self.n_u, self.n_t, self.n_p
        shapes = {"A": (self.n_u, self.n_u), "C1": (self.n_u, self.n_t),
                  "Q1": (self.n_u, self.n_p), "C2": (self.n_t, self.n_u),
                  "H": (self.n_t, self.n_t), "Q2": (self.n_p, self.n_u),
                  "T": (self.n_p, self.n_p)}
        for k in ("A", "C1", "Q1", "C2", "H", "Q2", "T"):
            if device:
                rp, ci, va = blocks[k]
                keep += [rp, ci, va]
                c = FpcCsr(shapes[k][0], shapes[k][1], va.numel(),
                           rp.data_ptr(), ci.data_ptr(), va.data_ptr())
            else:
                c = self._csr_host(blocks[k], keep)
            setattr(sysm, k, c)
        if coords is not None:
            if device:
                keep.append(coords)
                sysm.coords = coords.data_ptr()
            else:
                X = np.ascontiguousarray(coords, dtype=np.float64)
                keep.append(X)
                sysm.coords = X.ctypes.data
        sysm.ptr_space = FPC_DEVICE if device else FPC_HOST
        return sysm, keep

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.lib.fpc_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- operations -------------------------------------------------------
    def apply_prec(self, w, out=None):
        v = self._vec() if out is None else out
        self._check(self.lib.fpc_apply_prec(self.h, self._ptr(w),
                                            self._ptr(v)), "apply_prec")
        return v

    def apply_prec_T(self, w, out=None):
        v = self._vec() if out is None else out
        self._check(self.lib.fpc_apply_prec_T(self.h, self._ptr(w),
                                              self._ptr(v)), "apply_prec_T")
        return v

    def matvec(self, x, trans=False, out=None):
        y = self._vec() if out is None else out
        self._check(self.lib.fpc_matvec(self.h, int(trans), self._ptr(x),
                                        self._ptr(y)), "matvec")
        return y

    def vcycle(self, b, out=None):
        x = self._vec(self.n_u) if out is None else out
        self._check(self.lib.fpc_vcycle(self.h, self._ptr(b), self._ptr(x)),
                    "vcycle")
        return x

    def psolve(self, w, trans=False, out=None):
        """Pressure-block solve of the preconditioner (length n_p)."""
        v = self._vec(self.n_p) if out is None else out
        self._check(self.lib.fpc_psolve(self.h, int(bool(trans)), self._ptr(w),
                                        self._ptr(v)), "psolve")
        return v

    def dense_inverse(self, D):
        """In-place inverse of a square contiguous float64 CUDA tensor by the
        coarsest-level Gauss-Jordan with partial pivoting."""
        self._check(self.lib.fpc_dense_inverse(self.h, D.shape[0],
                                               self._ptr(D)), "dense_inverse")
        return D

    def stream_triad(self, b, c, scalar, out):
        """a = b + scalar c (HBM bandwidth reference)."""
        self._check(self.lib.fpc_stream_triad(self.h, b.numel(), self._ptr(b),
                                              self._ptr(c), float(scalar),
                                              self._ptr(out)), "stream_triad")
        return out

    def solve(self, b, rtol=0.0, x0=None, out=None):
        x = self._vec() if out is None else out
        use = 0
        if x0 is not None:
            x.copy_(x0)
            use = 1
        info = FpcInfo()
        st = self._check(self.lib.fpc_solve(self.h, self._ptr(b),
                                            self._ptr(x), float(rtol), use,
                                            C.byref(info)), "solve")
        d = info.as_dict()
        d["status"] = STATUS[st]
        return x, d

    def solve_T(self, g, rtol=0.0, out=None):
        lam = self._vec() if out is None else out
        info = FpcInfo()
        st = self._check(self.lib.fpc_solve_T(self.h, self._ptr(g),
                                              self._ptr(lam), float(rtol),
                                              C.byref(info)), "solve_T")
        d = info.as_dict()
        d["status"] = STATUS[st]
        return lam, d

    def solve_batch(self, B, rtol=0.0, out=None):
        """B: (k, N) contiguous float64 CUDA tensor, one right-hand side per
        row (column-major in the ABI's sense with ld = N)."""
        k = B.shape[0]
        X = self.torch.empty_like(B) if out is None else out
        infos = (FpcInfo * k)()
        st = self._check(self.lib.fpc_solve_batch(
            self.h, k, self._ptr(B), B.stride(0), self._ptr(X), X.stride(0),
            float(rtol), infos), "solve_batch")
        return X, [i.as_dict() for i in infos], STATUS[st]

    def flow_graph(self, pairs, ndir, upsilon):
        """Device arrays of a fracture flow graph for the gradient calls:
        (FpcFlowGraph, tensors that must stay alive while it is used)."""
        t = self.torch
        pk = pairs[:, 0].to(device=self.device, dtype=t.int32).contiguous()
        pl = pairs[:, 1].to(device=self.device, dtype=t.int32).contiguous()
        nd = ndir.to(device=self.device, dtype=t.int32).contiguous()
        up = upsilon.to(device=self.device, dtype=t.float64).contiguous()
        g = FpcFlowGraph(self.n_p, pk.numel(), pk.data_ptr(), pl.data_ptr(),
                         nd.data_ptr(), up.data_ptr())
        return g, (pk, pl, nd, up)

    def grad_log_trans(self, pairs, ndir, upsilon, lam_p, p, out=None):
        """dL/d log Upsilon from the adjoint pressure (device tensors)."""
        g, keep = self.flow_graph(pairs, ndir, upsilon)
        out = self._vec(self.n_p) if out is None else out
        self._check(self.lib.fpc_grad_log_trans(
            self.h, C.byref(g), self._ptr(lam_p.contiguous()),
            self._ptr(p.contiguous()), self._ptr(out)), "grad_log_trans")
        del keep
        return out

    def grad_log_trans_noalloc(self, graph, lam_p, p, out):
        """fpc_grad_log_trans_noalloc: every argument already on the device
        (graph from flow_graph, contiguous float64 tensors); the library
        allocates nothing."""
        self._check(self.lib.fpc_grad_log_trans_noalloc(
            self.h, C.byref(graph), self._ptr(lam_p), self._ptr(p),
            self._ptr(out)), "grad_log_trans_noalloc")
        return out

    # -- introspection ----------------------------------------------------
    def pressure_info(self):
        d = FpcPressureDesc()
        self._check(self.lib.fpc_pressure_info(self.h, C.byref(d)),
                    "pressure_info")
        return d.as_dict()

    def num_levels(self):
        return self.lib.fpc_num_levels(self.h)

    def level_info(self, level):
        d = FpcLevelDesc()
        self._check(self.lib.fpc_level_info(self.h, level, C.byref(d)),
                    "level_info")
        return d.as_dict()

    def export_aggregates(self, level):
        d = self.level_info(level)
        agg = np.empty(d["n_nodes"], np.int32)
        rank = np.empty(max(d["n_agg"], 1), np.int32)
        self._check(self.lib.fpc_export_aggregates(
            self.h, level, agg.ctypes.data, rank.ctypes.data), "aggregates")
        return agg, rank[:d["n_agg"]]

    def export_level_matrix(self, level, which=0):
        """(rowptr, col, blocks) of A_l (0), P_l (1) or R_l (2)."""
        d = self.level_info(level)
        nb = [d["nnzb"], d["p_nnzb"], d["r_nnzb"]][which]
        bs = d["block"]
        nxt = 6 if which else bs
        if which:
            nxt_l = self.level_info(level + 1)["block"]
            shape = (bs, nxt_l) if which == 1 else (nxt_l, bs)
            nrows = d["n_nodes"] if which == 1 else \
                self.level_info(level + 1)["n_nodes"]
        else:
            shape = (bs, bs)
            nrows = d["n_nodes"]
        del nxt
        rp = np.empty(nrows + 1, np.int64)
        col = np.empty(max(nb, 1), np.int32)
        val = np.empty(max(nb, 1) * shape[0] * shape[1], np.float64)
        self._check(self.lib.fpc_export_level_matrix(
            self.h, level, which, rp.ctypes.data, col.ctypes.data,
            val.ctypes.data), "export_level_matrix")
        return rp, col[:nb], val[:nb * shape[0] * shape[1]].reshape(
            nb, *shape)

    def setup_times(self):
        t = np.zeros(5)
        self._check(self.lib.fpc_setup_times(self.h, t.ctypes.data),
                    "setup_times")
        return dict(total=t[0], upload=t[1], schur=t[2], pressure=t[3],
                    amg=t[4])

    def kernel_timer(self, enable=True, reset=True):
        """(launches, total_ms) of the timed level-0 residual SpMV."""
        n, ms = C.c_int64(), C.c_double()
        self._check(self.lib.fpc_kernel_timer(self.h, int(enable), int(reset),
                                              C.byref(n), C.byref(ms)),
                    "kernel_timer")
        return n.value, ms.value

    def hash32(self, first, n):
        out = self.torch.empty(n, dtype=self.torch.int32, device=self.device)
        self._check(self.lib.fpc_hash32_device(
            self.h, C.c_uint32(first), n, C.c_void_p(out.data_ptr())),
            "hash32")
        return out.cpu().numpy().view(np.uint32)


def solver_from_system(s, **opts) -> Solver:
    """Convenience: a Solver for a ``fracgen.BlockSystem``-like object."""
    return Solver(s.blocks(), s.n_u, s.n_t, s.n_p, coords=s.coords, **opts)
