"""ctypes binding of libpsp (include/psp.h).

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI.  PyTorch supplies device memory (tensors) and the stream
(torch.cuda.current_stream()); the calls are asynchronous on that stream.
If libpsp.so is missing this module raises at load time: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsp.so")

PSP_OK, PSP_E_INVALID, PSP_E_EPS, PSP_E_NOMEM, PSP_E_HIP, PSP_E_STATE, PSP_E_UNSUPPORTED = range(7)
PATHS = {"auto": 0, "dense": 1, "sparse": 2, "sparse_batched": 3, "sparse_lds": 4, "sparse_levels": 5, "sparse_grouped": 6,
         "sparse_steps": 7, "sparse_tail": 8}
PATH_NAMES = {v: k for k, v in PATHS.items()}
ORDERS = {"md": 0, "natural": 1}
EXPORTED = ["psp_last_error", "psp_version", "psp_plan_create", "psp_plan_info", "psp_plan_export",
            "psp_plan_destroy", "psp_plan_device_bytes", "psp_plan_upload", "psp_weights", "psp_workspace_bytes",
            "psp_solve_batched", "psp_solve_batched_noalloc", "psp_solve_adaptive_workspace_bytes",
            "psp_solve_adaptive", "psp_tune", "psp_tune_choice", "psp_set_tune_choice", "psp_factor", "psp_solve", "psp_combine", "psp_grad_values",
            "psp_factors_release", "psp_residual", "psp_group_create", "psp_group_workspace_bytes", "psp_group_run",
            "psp_group_capture", "psp_group_adaptive_workspace_bytes", "psp_group_run_adaptive",
            "psp_group_capture_adaptive", "psp_graph_launch", "psp_graph_destroy", "psp_group_destroy", "psp_pf_device_bytes",
            "psp_pf_create", "psp_pf_destroy", "psp_pf_eval", "psp_pf_workspace_bytes", "psp_pf_newton",
            "psp_estimate_rho_workspace_bytes", "psp_estimate_rho"]
PF_STATUS = {0: "converged", 1: "max_iter", 2: "breakdown", 3: "diverged"}


class PSPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"psp status {status}: {msg}")
        self.status = status


class PlanInfo(C.Structure):
    _fields_ = [("n", C.c_int32), ("nnz", C.c_int32), ("nnz_l", C.c_int64), ("ndense", C.c_int32),
                ("nlev", C.c_int32 * 3), ("flops_dense_factor", C.c_int64), ("flops_sparse_factor", C.c_int64),
                ("steps", C.c_int32), ("steps_packed", C.c_int32), ("steps_lds_bytes", C.c_int64),
                ("steps_per_cu", C.c_int32), ("device_bytes", C.c_int64), ("tail_n", C.c_int32),
                ("tail_fac_levels", C.c_int32), ("tail_tiles", C.c_int32), ("tail_mfma", C.c_int64)]


class TuneChoice(C.Structure):
    _fields_ = [("path", C.c_int32), ("steps_mode", C.c_int32), ("steps_wgcu", C.c_int32), ("ring", C.c_int32),
                ("tail_cols", C.c_int32), ("tail_il", C.c_int32), ("tail_lu", C.c_int32), ("ms", C.c_float), ("source", C.c_int32)]

    def as_dict(self):
        return {"path": PATH_NAMES.get(self.path, self.path), "steps_mode": self.steps_mode,
                "steps_wgcu": self.steps_wgcu, "ring": self.ring, "tail_cols": self.tail_cols, "tail_il": self.tail_il, "tail_lu": self.tail_lu,
                "ms": float(self.ms), "source": {0: "heuristic", 1: "tuned", 2: "cache file"}[self.source]}


class GroupShape(C.Structure):
    _fields_ = [("plan", C.c_void_p), ("batch", C.c_int32), ("path", C.c_int32)]


class GroupTask(C.Structure):
    _fields_ = [("values", C.c_void_p), ("d", C.c_void_p), ("B", C.c_void_p), ("X", C.c_void_p),
                ("info", C.c_void_p)]


class GroupAdapt(C.Structure):
    _fields_ = [("est", C.c_void_p), ("scale", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.psp_last_error.restype = C.c_char_p
        L.psp_version.restype = i32
        L.psp_plan_create.argtypes = [i32, vp, vp, C.c_uint32, C.POINTER(vp)]
        L.psp_plan_info.argtypes = [vp, C.POINTER(PlanInfo)]
        L.psp_plan_export.argtypes = [vp, vp, vp, vp, vp, vp, C.POINTER(vp), C.POINTER(vp)]
        L.psp_plan_destroy.argtypes = [vp]
        L.psp_plan_destroy.restype = None
        L.psp_plan_device_bytes.argtypes = [vp]
        L.psp_plan_device_bytes.restype = C.c_size_t
        L.psp_plan_upload.argtypes = [vp, vp, C.c_size_t, vp]
        L.psp_weights.argtypes = [i32, vp, vp]
        L.psp_workspace_bytes.argtypes = [vp, i32, i32, i32, i32, i32]
        L.psp_workspace_bytes.restype = C.c_size_t
        L.psp_solve_batched.argtypes = [vp, i32, i32, vp, i32, vp, vp, i32, vp, vp, vp, vp, C.c_size_t, vp]
        L.psp_solve_batched_noalloc.argtypes = [vp, i32, vp, i32, vp, vp, vp, vp, vp, vp]
        L.psp_solve_adaptive_workspace_bytes.argtypes = [vp, i32, i32]
        L.psp_solve_adaptive_workspace_bytes.restype = C.c_size_t
        L.psp_solve_adaptive.argtypes = [vp, i32, vp, i32, vp, vp, d, vp, vp, vp, vp, vp, vp, C.c_size_t, vp]
        L.psp_tune_choice.argtypes = [vp, i32, i32, i32, C.POINTER(TuneChoice)]
        L.psp_set_tune_choice.argtypes = [vp, i32, i32, i32, C.POINTER(TuneChoice)]
        L.psp_tune.argtypes = [vp, i32, vp, i32, vp, vp, i32, vp, vp, vp, vp, C.c_size_t, vp, vp, vp]
        L.psp_factor.argtypes = [vp, i32, i32, vp, i32, vp, vp, vp, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.psp_solve.argtypes = [vp, i32, vp, vp, i32, vp]
        L.psp_combine.argtypes = [vp, i32, vp, vp, vp]
        L.psp_grad_values.argtypes = [vp, i32, vp, vp, vp, vp]
        L.psp_factors_release.argtypes = [vp]
        L.psp_residual.argtypes = [vp, i32, vp, i32, vp, vp, vp, vp, vp, vp]
        L.psp_group_create.argtypes = [i32, vp, i32, vp, i32, C.POINTER(vp)]
        L.psp_group_workspace_bytes.argtypes = [vp]
        L.psp_group_workspace_bytes.restype = C.c_size_t
        L.psp_group_run.argtypes = [vp, vp, vp, C.c_size_t, vp]
        L.psp_group_capture.argtypes = [vp, vp, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.psp_group_adaptive_workspace_bytes.argtypes = [vp]
        L.psp_group_adaptive_workspace_bytes.restype = C.c_size_t
        L.psp_group_run_adaptive.argtypes = [vp, vp, vp, d, vp, C.c_size_t, vp]
        L.psp_group_capture_adaptive.argtypes = [vp, vp, vp, d, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.psp_graph_launch.argtypes = [vp, vp]
        L.psp_graph_destroy.argtypes = [vp]
        L.psp_graph_destroy.restype = None
        L.psp_group_destroy.argtypes = [vp]
        L.psp_group_destroy.restype = None
        L.psp_pf_device_bytes.argtypes = [i32, i32]
        L.psp_pf_device_bytes.restype = C.c_size_t
        L.psp_pf_create.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, C.c_size_t, vp, C.POINTER(vp)]
        L.psp_pf_destroy.argtypes = [vp]
        L.psp_pf_destroy.restype = None
        L.psp_pf_eval.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
        L.psp_pf_workspace_bytes.argtypes = [vp, i32, i32, i32]
        L.psp_pf_workspace_bytes.restype = C.c_size_t
        L.psp_pf_newton.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, vp, d, i32, vp, vp, vp, vp, C.c_size_t, vp]
        L.psp_estimate_rho_workspace_bytes.argtypes = [vp, i32]
        L.psp_estimate_rho_workspace_bytes.restype = C.c_size_t
        L.psp_estimate_rho.argtypes = [vp, i32, vp, vp, d, i32, vp, vp, vp, C.c_size_t, vp]
        for f in EXPORTED:
            if f not in ("psp_last_error", "psp_version", "psp_plan_destroy", "psp_plan_device_bytes",
                         "psp_workspace_bytes", "psp_group_workspace_bytes", "psp_graph_destroy",
                         "psp_group_destroy", "psp_group_adaptive_workspace_bytes", "psp_pf_device_bytes", "psp_pf_destroy", "psp_pf_workspace_bytes",
                         "psp_estimate_rho_workspace_bytes", "psp_solve_adaptive_workspace_bytes"):
                getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(status: int):
    if status != PSP_OK:
        raise PSPError(status, lib().psp_last_error().decode())


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _dptr(t):
    """Device pointer of a CUDA tensor (or None)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def weights(eps) -> np.ndarray:
    e = np.ascontiguousarray(eps, dtype=np.float64)
    c = np.zeros_like(e)
    _check(lib().psp_weights(len(e), _np_ptr(e), _np_ptr(c)))
    return c


@dataclass
class SymbolicArrays:
    perm: np.ndarray
    iperm: np.ndarray
    parent: np.ndarray
    l_ptr: np.ndarray
    l_idx: np.ndarray
    levels: tuple   # ((ptr, idx) factor, L-solve, U-solve)


class Plan:
    """Symbolic analysis of one CSR pattern (host), reused by every numeric call."""

    def __init__(self, indptr, indices, order: str = "md"):
        ip = np.ascontiguousarray(indptr, dtype=np.int32)
        ix = np.ascontiguousarray(indices, dtype=np.int32)
        self.n = len(ip) - 1
        self.nnz = int(ip[-1]) if len(ip) else 0
        h = C.c_void_p()
        _check(lib().psp_plan_create(self.n, _np_ptr(ip), _np_ptr(ix), ORDERS[order], C.byref(h)))
        self._h = h
        self._ws = {}
        self._dev = None   # device copy of the plan (a torch uint8 tensor this object owns)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.psp_plan_destroy(h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def device_bytes(self) -> int:
        return int(lib().psp_plan_device_bytes(self._h))

    def upload(self, device=None, stream=None):
        """Copies the plan's device arrays into a tensor on `device` (psp_plan_upload); numeric
        calls do this on first use.  Returns the tensor, which the plan keeps alive."""
        import torch
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        nbytes = self.device_bytes()
        if nbytes == 0:
            raise PSPError(PSP_E_NOMEM, "plan image could not be built")
        with torch.cuda.device(dev):
            buf = torch.empty(nbytes, dtype=torch.uint8, device=dev)
            _check(lib().psp_plan_upload(self._h, _dptr(buf), nbytes, _stream(stream)))
        self._dev = buf
        return buf

    def ensure(self, device):
        """Uploads the plan to `device` unless it already lives there."""
        import torch
        dev = torch.device(device)
        if self._dev is None or self._dev.device != dev:
            self.upload(dev)

    def info(self) -> PlanInfo:
        o = PlanInfo()
        _check(lib().psp_plan_info(self._h, C.byref(o)))
        return o

    def export(self) -> SymbolicArrays:
        inf = self.info()
        n, nl = self.n, int(inf.nnz_l)
        perm, iperm, parent = (np.zeros(n, np.int32) for _ in range(3))
        lp = np.zeros(n + 1, np.int32)
        li = np.zeros(max(nl, 1), np.int32)
        lvp = [np.zeros(inf.nlev[t] + 1, np.int32) for t in range(3)]
        lvi = [np.zeros(n, np.int32) for _ in range(3)]
        P = (C.c_void_p * 3)(*[_np_ptr(a).value for a in lvp])
        I = (C.c_void_p * 3)(*[_np_ptr(a).value for a in lvi])
        _check(lib().psp_plan_export(self._h, _np_ptr(perm), _np_ptr(iperm), _np_ptr(parent), _np_ptr(lp),
                                     _np_ptr(li), P, I))
        return SymbolicArrays(perm, iperm, parent, lp, li[:nl], tuple(zip(lvp, lvi)))

    def workspace_bytes(self, path="auto", batch=1, K=1, nrhs=1, keep=False) -> int:
        return int(lib().psp_workspace_bytes(self._h, PATHS[path], batch, K, nrhs, 1 if keep else 0))

    def workspace(self, nbytes: int, device):
        """Device workspace cached per plan (grown on demand)."""
        import torch
        key = str(device)
        w = self._ws.get(key)
        if w is None or w.numel() < nbytes:
            w = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
            self._ws[key] = w
        return w


def solve_batched(plan: Plan, values, eps, b, path: str = "auto", d=None, workspace=None, stream=None):
    """Alg. 1 steps 1-4 in one fused launch (+ a combine launch).

    values: (batch, nnz) float64 device tensor; b: (batch, n) or (batch, n, nrhs).
    Returns (x, info) with x shaped like b and info (batch, K) int32.
    """
    import torch
    batch = values.shape[0]
    nrhs = 1 if b.dim() == 2 else b.shape[2]
    eps_h = np.ascontiguousarray(eps, dtype=np.float64)
    K = len(eps_h)
    if values.dtype != torch.float64 or b.dtype != torch.float64:
        raise TypeError("values and b must be float64")
    if values.shape[1] != plan.nnz or b.shape[1] != plan.n or b.shape[0] != batch:
        raise ValueError("shape mismatch with the plan")
    plan.ensure(values.device)
    x = torch.empty_like(b)
    info = torch.empty((batch, K), dtype=torch.int32, device=values.device)
    need = plan.workspace_bytes(path, batch, K, nrhs, keep=False)
    ws = plan.workspace(need, values.device) if workspace is None else workspace
    _check(lib().psp_solve_batched(plan.handle, PATHS[path], batch, _dptr(values), K, _np_ptr(eps_h), _dptr(d),
                                   nrhs, _dptr(b.contiguous()), _dptr(x), _dptr(info), _dptr(ws), ws.numel(),
                                   _stream(stream)))
    return x, info


def solve_adaptive(plan: Plan, values, eps, b, tol: float = 1e-10, d=None, workspace=None, stream=None):
    """Alg. 1 with the error test choosing the node size per Jacobian (psp_solve_adaptive).

    values (batch, nnz), b (batch, n) float64 device tensors; eps the first node set (K >= 3).
    Returns (x, info, est, scale): x (batch, n), info (batch, K), the final error estimate and
    the node scale used per Jacobian (1, or a power of two below 1)."""
    import torch
    batch = values.shape[0]
    eps_h = np.ascontiguousarray(eps, dtype=np.float64)
    K = len(eps_h)
    if values.dtype != torch.float64 or b.dtype != torch.float64:
        raise TypeError("values and b must be float64")
    if values.shape[1] != plan.nnz or b.dim() != 2 or b.shape[1] != plan.n or b.shape[0] != batch:
        raise ValueError("shape mismatch with the plan")
    plan.ensure(values.device)
    dev = values.device
    x = torch.empty_like(b)
    info = torch.empty((batch, K), dtype=torch.int32, device=dev)
    est = torch.empty(batch, dtype=torch.float64, device=dev)
    scale = torch.empty(batch, dtype=torch.float64, device=dev)
    need = lib().psp_solve_adaptive_workspace_bytes(plan.handle, batch, K)
    ws = plan.workspace(need, dev) if workspace is None else workspace
    _check(lib().psp_solve_adaptive(plan.handle, batch, _dptr(values), K, _np_ptr(eps_h), _dptr(d), float(tol),
                                    _dptr(b.contiguous()), _dptr(x), _dptr(info), _dptr(est), _dptr(scale),
                                    _dptr(ws), ws.numel(), _stream(stream)))
    return x, info, est, scale


class Group:
    """An uneven batch (psp_group_*): items of Jacobians of different patterns, solved together.

    shapes: list of (plan, batch) or (plan, batch, path name).  run() enqueues every item on the
    group's stream lanes; capture() records the same work into a HIP graph that replay() launches."""

    def __init__(self, shapes, eps, nrhs: int = 1, device=None):
        import torch
        self.eps = np.ascontiguousarray(eps, dtype=np.float64)
        self.K = len(self.eps)
        self.nrhs = nrhs
        self.plans = []
        arr = (GroupShape * len(shapes))()
        dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        for i, sh in enumerate(shapes):
            plan, batch = sh[0], int(sh[1])
            path = sh[2] if len(sh) > 2 else "auto"
            plan.ensure(dev)
            self.plans.append((plan, batch))
            arr[i] = GroupShape(plan.handle.value, batch, PATHS[path])
        h = C.c_void_p()
        _check(lib().psp_group_create(len(shapes), C.byref(arr), self.K, _np_ptr(self.eps), nrhs, C.byref(h)))
        self._h = h
        self.ws = torch.empty(int(lib().psp_group_workspace_bytes(h)), dtype=torch.uint8, device=dev)
        self._graphs = []

    def __del__(self):
        for g in getattr(self, "_graphs", []):
            if _lib is not None:
                _lib.psp_graph_destroy(g)
        self._graphs = []
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.psp_group_destroy(h)
            self._h = None

    def outputs(self, items, d=None):
        """Allocates X and info for items = [(values, b)] and returns (task array, [(x, info)], keep)."""
        import torch
        if len(items) != len(self.plans):
            raise ValueError("one (values, b) pair per group item")
        tasks = (GroupTask * len(items))()
        outs, keep = [], []
        for i, ((plan, batch), (values, b)) in enumerate(zip(self.plans, items)):
            if values.dtype != torch.float64 or b.dtype != torch.float64:
                raise TypeError("values and b must be float64")
            if values.shape != (batch, plan.nnz) or b.shape[0] != batch or b.shape[1] != plan.n:
                raise ValueError(f"item {i}: shape mismatch with its plan")
            if (1 if b.dim() == 2 else b.shape[2]) != self.nrhs:
                raise ValueError(f"item {i}: wrong number of right-hand sides")
            vc, bc = values.contiguous(), b.contiguous()
            x = torch.empty_like(bc)
            info = torch.empty((batch, self.K), dtype=torch.int32, device=values.device)
            keep += [vc, bc]
            tasks[i] = GroupTask(_dptr(vc).value, _dptr(d).value if d is not None else None, _dptr(bc).value,
                                 _dptr(x).value, _dptr(info).value)
            outs.append((x, info))
        return tasks, outs, keep

    def run(self, items, d=None, stream=None):
        """Solves every item; returns [(x_i, info_i)]."""
        tasks, outs, keep = self.outputs(items, d)
        _check(lib().psp_group_run(self._h, C.byref(tasks), _dptr(self.ws), self.ws.numel(), _stream(stream)))
        self._keep = keep
        return outs

    def capture(self, items, d=None, stream=None):
        """Captures the group's work into a HIP graph; returns (graph handle, [(x_i, info_i)]).  The
        output tensors and inputs stay bound to the graph: replay(graph) rewrites the outputs."""
        tasks, outs, keep = self.outputs(items, d)
        if stream is None:
            # the default stream cannot be captured: capture on a side stream ordered after it
            import torch
            stream = torch.cuda.Stream(device=self.ws.device)
            stream.wait_stream(torch.cuda.current_stream(self.ws.device))
            self._capture_streams = getattr(self, "_capture_streams", []) + [stream]
        g = C.c_void_p()
        _check(lib().psp_group_capture(self._h, C.byref(tasks), _dptr(self.ws), self.ws.numel(), _stream(stream),
                                       C.byref(g)))
        self._graphs.append(g)
        self._keep_graph = getattr(self, "_keep_graph", []) + [keep]
        return g, outs

    def replay(self, graph, stream=None):
        _check(lib().psp_graph_launch(graph, _stream(stream)))

    def _adapt_outputs(self, outs):
        import torch
        arr = (GroupAdapt * len(self.plans))()
        res = []
        for i, (plan, batch) in enumerate(self.plans):
            dev = outs[i][0].device
            est = torch.empty(batch, dtype=torch.float64, device=dev)
            scale = torch.empty(batch, dtype=torch.float64, device=dev)
            arr[i] = GroupAdapt(_dptr(est).value, _dptr(scale).value)
            res.append((est, scale))
        if not hasattr(self, "ws_adapt"):
            self.ws_adapt = torch.empty(int(lib().psp_group_adaptive_workspace_bytes(self._h)), dtype=torch.uint8,
                                        device=self.ws.device)
        return arr, res

    def run_adaptive(self, items, tol: float = 1e-10, d=None, stream=None):
        """Every item with the error test (psp_solve_adaptive); returns [(x_i, info_i, est_i, scale_i)]."""
        tasks, outs, keep = self.outputs(items, d)
        arr, res = self._adapt_outputs(outs)
        _check(lib().psp_group_run_adaptive(self._h, C.byref(tasks), C.byref(arr), float(tol), _dptr(self.ws_adapt),
                                            self.ws_adapt.numel(), _stream(stream)))
        self._keep = keep
        return [o + r for o, r in zip(outs, res)]

    def capture_adaptive(self, items, tol: float = 1e-10, d=None, stream=None):
        """capture() of run_adaptive; returns (graph handle, [(x_i, info_i, est_i, scale_i)])."""
        tasks, outs, keep = self.outputs(items, d)
        arr, res = self._adapt_outputs(outs)
        if stream is None:
            import torch
            stream = torch.cuda.Stream(device=self.ws.device)
            stream.wait_stream(torch.cuda.current_stream(self.ws.device))
            self._capture_streams = getattr(self, "_capture_streams", []) + [stream]
        g = C.c_void_p()
        _check(lib().psp_group_capture_adaptive(self._h, C.byref(tasks), C.byref(arr), float(tol),
                                                _dptr(self.ws_adapt), self.ws_adapt.numel(), _stream(stream),
                                                C.byref(g)))
        self._graphs.append(g)
        self._keep_graph = getattr(self, "_keep_graph", []) + [(keep, res)]
        return g, [o + r for o, r in zip(outs, res)]


def solve_group(items, eps, path: str = "auto", d=None, stream=None):
    """Uneven batch in one call: items is a list of (plan, values, b), each values (batch_i, nnz_i)
    and b (batch_i, n_i) or (batch_i, n_i, nrhs).  Returns [(x_i, info_i)]."""
    nrhs = 1 if items[0][2].dim() == 2 else items[0][2].shape[2]
    g = Group([(p, v.shape[0], path) for p, v, _ in items], eps, nrhs=nrhs, device=items[0][1].device)
    outs = g.run([(v, b) for _, v, b in items], d=d, stream=stream)
    # keep the group (its workspace and lanes) until the caller's stream has finished with it
    import torch
    torch.cuda.current_stream(items[0][1].device).synchronize() if stream is None else stream.synchronize()
    return outs


def residual(plan: Plan, values, b, x, keep_r: bool = False, stream=None):
    """Alg. 1 step 5 (optional error test): r = b - A x per Jacobian and RHS column.

    values: (batch, nnz); b, x: (batch, n) or (batch, n, nrhs), float64 device tensors.
    Returns (rnorm, bnorm), each (batch, nrhs) = ||r||_2 and ||b||_2, plus r (shaped like
    b) when keep_r."""
    import torch
    batch = values.shape[0]
    nrhs = 1 if b.dim() == 2 else b.shape[2]
    if values.dtype != torch.float64 or b.dtype != torch.float64 or x.dtype != torch.float64:
        raise TypeError("values, b and x must be float64")
    if values.shape[1] != plan.nnz or b.shape != x.shape or b.shape[0] != batch or b.shape[1] != plan.n:
        raise ValueError("shape mismatch with the plan")
    plan.ensure(values.device)
    rn = torch.empty((batch, nrhs), dtype=torch.float64, device=values.device)
    bn = torch.empty_like(rn)
    r = torch.empty_like(b) if keep_r else None
    _check(lib().psp_residual(plan.handle, batch, _dptr(values), nrhs, _dptr(b.contiguous()), _dptr(x.contiguous()),
                              _dptr(r), _dptr(rn), _dptr(bn), _stream(stream)))
    return (rn, bn, r) if keep_r else (rn, bn)


def tune(plan: Plan, values, eps, b, d=None, stream=None):
    """Autotune the fused call for this (batch, K, nrhs): returns (chosen path name,
    {path name: ms per call}); later solve_batched(..., path="auto") uses the choice."""
    import torch
    batch = values.shape[0]
    nrhs = 1 if b.dim() == 2 else b.shape[2]
    eps_h = np.ascontiguousarray(eps, dtype=np.float64)
    K = len(eps_h)
    plan.ensure(values.device)
    x = torch.empty_like(b)
    info = torch.empty((batch, K), dtype=torch.int32, device=values.device)
    need = plan.workspace_bytes("auto", batch, K, nrhs, keep=False)
    ws = plan.workspace(need, values.device)
    chosen = C.c_int32(-1)
    ms = (C.c_float * len(PATHS))()
    _check(lib().psp_tune(plan.handle, batch, _dptr(values), K, _np_ptr(eps_h), _dptr(d), nrhs, _dptr(b.contiguous()),
                          _dptr(x), _dptr(info), _dptr(ws), ws.numel(), _stream(stream), C.byref(chosen), ms))
    times = {PATH_NAMES[i]: float(ms[i]) for i in range(1, len(PATHS)) if ms[i] >= 0}
    return PATH_NAMES[chosen.value], times


def tune_choice(plan: Plan, batch: int, K: int, nrhs: int = 1) -> dict:
    """The path and launch choices PSP_PATH_AUTO uses for (batch, K, nrhs), and where they come from."""
    c = TuneChoice()
    _check(lib().psp_tune_choice(plan.handle, batch, K, nrhs, C.byref(c)))
    return c.as_dict()


def set_tune_choice(plan: Plan, batch: int, K: int, nrhs: int = 1, path: str = "sparse_steps", steps_mode: int = -1,
                    steps_wgcu: int = 0, ring: int = 7, tail_cols: int = 16, tail_il: int = -1,
                    tail_lu: int = 0) -> None:
    """Pins the path and launch choices of PSP_PATH_AUTO for (batch, K, nrhs)."""
    c = TuneChoice(PATHS[path], steps_mode, steps_wgcu, ring, tail_cols, tail_il, tail_lu, -1.0, 1)
    _check(lib().psp_set_tune_choice(plan.handle, batch, K, nrhs, C.byref(c)))


class Factors:
    """Perturbed factors of batch x K systems kept in a device workspace."""

    def __init__(self, plan: Plan, values, eps, path: str = "auto", d=None, nrhs_cap: int = 64, stream=None):
        import torch
        self.plan = plan
        self.batch = values.shape[0]
        self.eps = np.ascontiguousarray(eps, dtype=np.float64)
        self.K = len(self.eps)
        self.c = weights(self.eps)
        self.device = values.device
        plan.ensure(values.device)
        need = plan.workspace_bytes(path, self.batch, self.K, nrhs_cap, keep=True)
        self.ws = torch.empty(max(need, 256), dtype=torch.uint8, device=values.device)
        self.info = torch.empty((self.batch, self.K), dtype=torch.int32, device=values.device)
        h = C.c_void_p()
        _check(lib().psp_factor(plan.handle, PATHS[path], self.batch, _dptr(values.contiguous()), self.K,
                                _np_ptr(self.eps), _dptr(d), _dptr(self.info), _dptr(self.ws), self.ws.numel(),
                                _stream(stream), C.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.psp_factors_release(h)
            self._h = None

    def solve(self, B, transpose: bool = False, stream=None):
        """Per-system solutions, (batch, K, n, nrhs)."""
        import torch
        B3 = B if B.dim() == 3 else B.unsqueeze(-1)
        nrhs = B3.shape[2]
        Xk = torch.empty((self.batch, self.K, self.plan.n, nrhs), dtype=torch.float64, device=self.device)
        _check(lib().psp_solve(self._h, nrhs, _dptr(B3.contiguous()), _dptr(Xk), 1 if transpose else 0,
                               _stream(stream)))
        return Xk

    def combine(self, Xk, stream=None):
        import torch
        nrhs = Xk.shape[3]
        X = torch.empty((self.batch, self.plan.n, nrhs), dtype=torch.float64, device=self.device)
        _check(lib().psp_combine(self._h, nrhs, _dptr(Xk.contiguous()), _dptr(X), _stream(stream)))
        return X

    def grad_values(self, Lamk, Xk, stream=None):
        import torch
        nrhs = Xk.shape[3]
        gA = torch.empty((self.batch, self.plan.nnz), dtype=torch.float64, device=self.device)
        _check(lib().psp_grad_values(self._h, nrhs, _dptr(Lamk.contiguous()), _dptr(Xk.contiguous()), _dptr(gA),
                                     _stream(stream)))
        return gA


def estimate_rho(plan: Plan, values, v0, d=None, probe: float = 1e-8, iters: int = 24, stream=None):
    """rho(A_s^{-1} D) per Jacobian by power iteration on (A_s + probe D)^{-1} D (psp_estimate_rho).
    values (batch, nnz), v0 (batch, n) start vectors, float64 device tensors; returns (batch,)."""
    import torch
    batch = values.shape[0]
    if values.dtype != torch.float64 or v0.dtype != torch.float64:
        raise TypeError("values and v0 must be float64")
    if values.shape[1] != plan.nnz or tuple(v0.shape) != (batch, plan.n):
        raise ValueError("shape mismatch with the plan")
    plan.ensure(values.device)
    rho = torch.empty(batch, dtype=torch.float64, device=values.device)
    need = int(lib().psp_estimate_rho_workspace_bytes(plan.handle, batch))
    ws = plan.workspace(need, values.device)
    _check(lib().psp_estimate_rho(plan.handle, batch, _dptr(values.contiguous()), _dptr(d), float(probe), int(iters),
                                  _dptr(v0.contiguous()), _dptr(rho), _dptr(ws), ws.numel(), _stream(stream)))
    return rho


class PowerFlow:
    """Newton-Raphson power flow of one network around Alg. 1 (psp_pf_* in include/psp.h).

    x and spec are (batch, n) float64 device tensors laid out [theta | |V| | lambda] and
    [P0 | Q0 or V_set | theta_ref]; part is (batch, nbus)."""

    def __init__(self, plan: Plan, y_indptr, y_indices, g, b, pv):
        yp = np.ascontiguousarray(y_indptr, dtype=np.int32)
        yc = np.ascontiguousarray(y_indices, dtype=np.int32)
        gg = np.ascontiguousarray(g, dtype=np.float64)
        bb = np.ascontiguousarray(b, dtype=np.float64)
        pvv = np.ascontiguousarray(pv, dtype=np.int32)
        self.plan = plan
        self.N = len(yp) - 1
        if len(pvv) != self.N:
            raise ValueError("pv must have one entry per bus")
        import torch
        dev = torch.device("cuda", torch.cuda.current_device())
        plan.ensure(dev)
        nbytes = int(lib().psp_pf_device_bytes(self.N, int(yp[-1])))
        self._dev = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=dev)
        h = C.c_void_p()
        _check(lib().psp_pf_create(plan.handle, self.N, _np_ptr(yp), _np_ptr(yc), _np_ptr(gg), _np_ptr(bb),
                                   _np_ptr(pvv), _dptr(self._dev), self._dev.numel(), _stream(None), C.byref(h)))
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value and _lib is not None:
            _lib.psp_pf_destroy(h)
            self._h = None

    def _shapes(self, x, spec, part):
        import torch
        for t in (x, spec, part):
            if t.dtype != torch.float64:
                raise TypeError("x, spec and part must be float64")
        batch = x.shape[0]
        if x.shape != (batch, self.plan.n) or spec.shape != x.shape or part.shape != (batch, self.N):
            raise ValueError("shape mismatch with the network")
        return batch

    def eval(self, x, spec, part, jacobian: bool = True, stream=None):
        """Returns (F, J or None, fnorm) for every scenario."""
        import torch
        batch = self._shapes(x, spec, part)
        F = torch.empty_like(x)
        J = torch.empty((batch, self.plan.nnz), dtype=torch.float64, device=x.device) if jacobian else None
        fn = torch.empty(batch, dtype=torch.float64, device=x.device)
        _check(lib().psp_pf_eval(self._h, batch, _dptr(x.contiguous()), _dptr(spec.contiguous()),
                                 _dptr(part.contiguous()), _dptr(F), _dptr(J), _dptr(fn), _stream(stream)))
        return F, J, fn

    def workspace_bytes(self, path="auto", batch=1, K=1) -> int:
        return int(lib().psp_pf_workspace_bytes(self._h, PATHS[path], batch, K))

    def newton(self, x0, spec, part, eps, tol: float = 1e-9, max_iter: int = 10, d=None, path: str = "auto",
               workspace=None, stream=None):
        """Returns (x, iters, status, fnorm); status codes in PF_STATUS.  Blocks once per iteration."""
        import torch
        batch = self._shapes(x0, spec, part)
        eps_h = np.ascontiguousarray(eps, dtype=np.float64)
        K = len(eps_h)
        x = x0.clone().contiguous()
        iters = torch.empty(batch, dtype=torch.int32, device=x.device)
        status = torch.empty(batch, dtype=torch.int32, device=x.device)
        fn = torch.empty(batch, dtype=torch.float64, device=x.device)
        need = self.workspace_bytes(path, batch, K)
        ws = self.plan.workspace(need, x.device) if workspace is None else workspace
        _check(lib().psp_pf_newton(self._h, PATHS[path], batch, K, _np_ptr(eps_h), _dptr(d), _dptr(x),
                                   _dptr(spec.contiguous()), _dptr(part.contiguous()), float(tol), int(max_iter),
                                   _dptr(iters), _dptr(status), _dptr(fn), _dptr(ws), ws.numel(), _stream(stream)))
        return x, iters, status, fn
