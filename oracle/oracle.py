"""Python front end of the CPU FP64 oracle (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg import
this module.  It loads ``liboracle.so`` (plain C, built from
``psp_oracle.c`` and ``psp_oracle_sparse.c``) and adds a few helpers that
compose those routines into the paper's Algorithm 1:

1. perturb A by eps_k D for each node eps_k,
2. factor and solve each perturbed system without pivoting,
3.-4. combine the perturbed solutions with the weights of Remark 2,
5. optionally test the error against the pivoted ground truth.

It shares no code with the GPU library and never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SOURCES = [os.path.join(HERE, "psp_oracle.c"), os.path.join(HERE, "psp_oracle_sparse.c")]

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile liboracle.so with gcc (-O2, OpenMP, no FP contraction)."""
    if force or not os.path.exists(LIB_PATH) or any(
            os.path.getmtime(s) > os.path.getmtime(LIB_PATH) for s in SOURCES):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                               "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-o", tmp, *SOURCES, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        L.oracle_weights.argtypes = [C.c_int, _dp, _dp]
        L.oracle_lu_nopiv.argtypes = [C.c_int, _dp, C.c_int]
        for f in ("oracle_fwd_unit_lower", "oracle_back_upper", "oracle_fwd_upper_trans",
                  "oracle_back_lower_trans"):
            getattr(L, f).argtypes = [C.c_int, _dp, C.c_int, _dp]
            getattr(L, f).restype = None
        L.oracle_combine.argtypes = [C.c_int, C.c_int64, _dp, _dp, _dp]
        L.oracle_combine.restype = None
        L.oracle_residual.argtypes = [C.c_int, _ip, _ip, _dp, C.c_int, _dp, _dp, C.c_void_p, _dp, C.c_void_p]
        L.oracle_residual.restype = None
        L.oracle_norm2.argtypes = [C.c_int, _dp]
        L.oracle_norm2.restype = C.c_double
        L.oracle_lu_partial.argtypes = [C.c_int, _dp, C.c_int, _ip]
        L.oracle_lu_partial_solve.argtypes = [C.c_int, _dp, C.c_int, _ip, _dp]
        L.oracle_lu_partial_solve.restype = None
        L.oracle_dense_system.argtypes = [C.c_int, _ip, _ip, _dp, C.c_void_p, C.c_double, C.c_void_p,
                                          C.c_int, _dp, _dp, C.c_void_p]
        L.oracle_dense_batch.argtypes = [C.c_int, _ip, _ip, C.c_int, _dp, C.c_void_p, C.c_int, _dp, _dp,
                                         C.c_void_p, C.c_int, _dp, _dp, C.c_void_p, _ip]
        L.oracle_symbolic.argtypes = [C.c_int, _ip, _ip, C.c_int, C.POINTER(C.c_void_p)]
        L.oracle_symbolic_sizes.argtypes = [C.c_void_p, np.ctypeslib.ndpointer(np.int64)]
        L.oracle_symbolic_sizes.restype = None
        L.oracle_symbolic_get.argtypes = [C.c_void_p] + [_ip] * 11
        L.oracle_symbolic_get.restype = None
        L.oracle_symbolic_free.argtypes = [C.c_void_p]
        L.oracle_symbolic_free.restype = None
        L.oracle_sparse_lu.argtypes = [C.c_int, _ip, _ip, _dp, _ip, _ip, _ip, C.c_double, C.c_void_p,
                                       _dp, _dp, _dp]
        L.oracle_sparse_solve.argtypes = [C.c_int, _ip, _ip, _dp, _dp, _dp, C.c_int, _dp]
        L.oracle_sparse_solve.restype = None
        L.oracle_sparse_system.argtypes = [C.c_int, _ip, _ip, _dp, _ip, _ip, _ip, C.c_double, C.c_void_p,
                                           C.c_int, C.c_int, _dp, _dp, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_sparse_batch.argtypes = [C.c_int, _ip, _ip, C.c_int, _dp, _ip, _ip, _ip, C.c_int, _dp,
                                          _dp, C.c_void_p, C.c_int, C.c_int, _dp, _dp, C.c_void_p, _ip]
        L.oracle_set_threads.argtypes = [C.c_int]
        L.oracle_set_threads.restype = None
        L.oracle_divided_difference.argtypes = [C.c_int, _dp, C.c_int64, _dp, _dp]
        L.oracle_divided_difference.restype = None
        L.oracle_error_estimate.argtypes = [C.c_int, _dp, C.c_int64, _dp, _dp, C.POINTER(C.c_double),
                                            C.POINTER(C.c_double)]
        L.oracle_error_estimate.restype = None
        L.oracle_scale_exponent.argtypes = [C.c_int, _dp, C.c_double, C.c_double]
        L.oracle_grad_values.argtypes = [C.c_int, _ip, _ip, C.c_int, _dp, C.c_int, _dp, _dp, _dp]
        L.oracle_grad_values.restype = None
        _lib = L
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def set_threads(t: int) -> None:
    """OpenMP threads of the batched routines (the host's count: os.cpu_count())."""
    lib().oracle_set_threads(int(t))


# ---------------------------------------------------------------- weights
def weights(eps) -> np.ndarray:
    """c_k = prod_{l != k} eps_l / (eps_l - eps_k) (Remark 2, any distinct nodes)."""
    e = _f64(eps)
    c = np.zeros_like(e)
    if lib().oracle_weights(len(e), e, c) != 0:
        raise ValueError("perturbation nodes must be distinct, nonzero and finite")
    return c


# ---------------------------------------------------------------- dense
def lu_nopiv(A: np.ndarray):
    """Pivot-free LU of a dense matrix.  Returns (LU packed, info)."""
    n = A.shape[0]
    a = np.asfortranarray(A, dtype=np.float64).copy(order="F")
    buf = a.ravel(order="F").copy()
    info = lib().oracle_lu_nopiv(n, buf, n)
    return buf.reshape((n, n), order="F"), info


def _colmajor(LU):
    return np.ascontiguousarray(np.asarray(LU, dtype=np.float64).ravel(order="F"))


def solve_lu(LU: np.ndarray, b: np.ndarray, trans: bool = False) -> np.ndarray:
    n = LU.shape[0]
    buf = _colmajor(LU)
    y = _f64(b).copy()
    if not trans:
        lib().oracle_fwd_unit_lower(n, buf, n, y)
        lib().oracle_back_upper(n, buf, n, y)
    else:
        lib().oracle_fwd_upper_trans(n, buf, n, y)
        lib().oracle_back_lower_trans(n, buf, n, y)
    return y


def combine(c, xk: np.ndarray) -> np.ndarray:
    c = _f64(c)
    xk = _f64(xk)
    K = xk.shape[0]
    out = np.zeros(xk.shape[1:])
    flat = out.reshape(-1)
    lib().oracle_combine(K, flat.size, c, xk.reshape(K, -1), flat)
    return flat.reshape(xk.shape[1:])


def residual(n, indptr, indices, values, b, x):
    """Alg. 1 step 5: r = b - A x (A in CSR), ||r||_2 and ||b||_2 per RHS column.
    b, x: (n,) or (n, nrhs).  Returns (r, rnorm, bnorm) with norms of shape (nrhs,)."""
    b = _f64(b)
    x = _f64(x)
    nrhs = 1 if b.ndim == 1 else b.shape[1]
    r = np.zeros_like(b)
    rn = np.zeros(nrhs)
    bn = np.zeros(nrhs)
    lib().oracle_residual(n, _i32(indptr), _i32(indices), _f64(values), nrhs, b, x, _ptr(r), rn, _ptr(bn))
    return r, rn, bn


def norm2(x) -> float:
    """sqrt of the fma sum of squares in ascending order."""
    x = _f64(np.ravel(x))
    return float(lib().oracle_norm2(len(x), x))


def pivoted_solve(A: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Ground truth x* = A^{-1} b by partial-pivot LU (ties to the lower row)."""
    n = A.shape[0]
    buf = _colmajor(A).copy()
    piv = np.zeros(n, dtype=np.int32)
    if lib().oracle_lu_partial(n, buf, n, piv) != 0:
        raise np.linalg.LinAlgError("singular")
    b = _f64(b)
    if b.ndim == 1:
        y = b.copy()
        lib().oracle_lu_partial_solve(n, buf, n, piv, y)
        return y
    out = np.empty_like(b)
    for r in range(b.shape[1]):
        y = np.ascontiguousarray(b[:, r])
        lib().oracle_lu_partial_solve(n, buf, n, piv, y)
        out[:, r] = y
    return out


def dense_system(n, indptr, indices, values, eps, b, perm=None, d=None, return_lu=False):
    """One perturbed system P(A + eps D)P^T, dense, pivot-free; b is n or n x nrhs."""
    b = _f64(b)
    nrhs = 1 if b.ndim == 1 else b.shape[1]
    x = np.zeros_like(b)
    lu = np.zeros(n * n) if return_lu else None
    info = lib().oracle_dense_system(n, _i32(indptr), _i32(indices), _f64(values),
                                     _ptr(None if perm is None else _i32(perm)), float(eps),
                                     _ptr(None if d is None else _f64(d)), nrhs, b, x, _ptr(lu))
    if return_lu:
        return x, info, lu.reshape((n, n), order="F")
    return x, info


def dense_batch(n, indptr, indices, values, eps, b, perm=None, d=None, keep_xk=False):
    """Algorithm 1 on a batch sharing one pattern (dense path).

    values: (batch, nnz); b: (batch, n) or (batch, n, nrhs).
    Returns (x (batch, ...), info (batch, K), xk or None, threads).
    """
    values = _f64(values)
    b = _f64(b)
    batch = values.shape[0]
    nrhs = 1 if b.ndim == 2 else b.shape[2]
    eps = _f64(eps)
    K = len(eps)
    c = weights(eps)
    x = np.zeros_like(b)
    xk = np.zeros((batch, K) + b.shape[1:]) if keep_xk else None
    info = np.zeros((batch, K), dtype=np.int32)
    thr = lib().oracle_dense_batch(n, _i32(indptr), _i32(indices), batch, values,
                                   _ptr(None if perm is None else _i32(perm)), K, eps, c,
                                   _ptr(None if d is None else _f64(d)), nrhs, b, x, _ptr(xk), info)
    return x, info, xk, thr


# ---------------------------------------------------------------- symbolic
@dataclass
class Symbolic:
    n: int
    perm: np.ndarray
    iperm: np.ndarray
    parent: np.ndarray
    lp: np.ndarray
    li: np.ndarray
    ndense: int
    levels: tuple  # ((ptr, idx) factor, (ptr, idx) L-solve, (ptr, idx) U-solve)

    @property
    def nnzL(self) -> int:
        return int(self.lp[-1])

    def flops_factor(self) -> int:
        """Multiply-add count x2 plus divisions of the sparse LU on this fill."""
        cnt = np.diff(self.lp).astype(np.int64)
        return int(np.sum(2 * cnt * cnt + cnt))


def symbolic(n, indptr, indices, natural=False) -> Symbolic:
    h = C.c_void_p()
    rc = lib().oracle_symbolic(n, _i32(indptr), _i32(indices), 1 if natural else 0, C.byref(h))
    if rc != 0:
        raise ValueError("malformed CSR pattern")
    try:
        sz = np.zeros(6, dtype=np.int64)
        lib().oracle_symbolic_sizes(h, sz)
        nnzL = int(sz[1])
        perm = np.zeros(n, np.int32)
        iperm = np.zeros(n, np.int32)
        parent = np.zeros(n, np.int32)
        lp = np.zeros(n + 1, np.int32)
        li = np.zeros(max(nnzL, 1), np.int32)
        lv = [(np.zeros(int(sz[3 + t]) + 1, np.int32), np.zeros(n, np.int32)) for t in range(3)]
        lib().oracle_symbolic_get(h, perm, iperm, parent, lp, li, lv[0][0], lv[0][1], lv[1][0], lv[1][1],
                                  lv[2][0], lv[2][1])
        return Symbolic(n, perm, iperm, parent, lp, li[:nnzL], int(sz[2]), tuple(lv))
    finally:
        lib().oracle_symbolic_free(h)


# ---------------------------------------------------------------- sparse
def sparse_lu(n, indptr, indices, values, sym: Symbolic, eps, d=None):
    """Returns (udiag, lval, uval, info) on sym's fill pattern."""
    nl = max(sym.nnzL, 1)
    ud, lv, uv = np.zeros(n), np.zeros(nl), np.zeros(nl)
    li = sym.li if sym.nnzL else np.zeros(1, np.int32)
    info = lib().oracle_sparse_lu(n, _i32(indptr), _i32(indices), _f64(values), sym.perm, sym.lp, li,
                                  float(eps), _ptr(None if d is None else _f64(d)), ud, lv, uv)
    return ud, lv[:sym.nnzL], uv[:sym.nnzL], info


def sparse_system(n, indptr, indices, values, sym: Symbolic, eps, b, d=None, trans=False):
    b = _f64(b)
    nrhs = 1 if b.ndim == 1 else b.shape[1]
    x = np.zeros_like(b)
    li = sym.li if sym.nnzL else np.zeros(1, np.int32)
    info = lib().oracle_sparse_system(n, _i32(indptr), _i32(indices), _f64(values), sym.perm, sym.lp, li,
                                      float(eps), _ptr(None if d is None else _f64(d)), nrhs,
                                      1 if trans else 0, b, x, None, None, None)
    return x, info


def sparse_batch(n, indptr, indices, values, sym: Symbolic, eps, b, d=None, trans=False, keep_xk=False):
    values = _f64(values)
    b = _f64(b)
    batch = values.shape[0]
    nrhs = 1 if b.ndim == 2 else b.shape[2]
    eps = _f64(eps)
    K = len(eps)
    c = weights(eps)
    x = np.zeros_like(b)
    xk = np.zeros((batch, K) + b.shape[1:]) if keep_xk else None
    info = np.zeros((batch, K), dtype=np.int32)
    li = sym.li if sym.nnzL else np.zeros(1, np.int32)
    thr = lib().oracle_sparse_batch(n, _i32(indptr), _i32(indices), batch, values, sym.perm, sym.lp, li, K,
                                    eps, c, _ptr(None if d is None else _f64(d)), nrhs, 1 if trans else 0,
                                    b, x, _ptr(xk), info)
    return x, info, xk, thr


def divided_difference(j, eps, xk) -> np.ndarray:
    """f[eps_0..eps_j] of the perturbed solutions xk (K, ...): sum_k x_k / prod_{l != k} (eps_k - eps_l)."""
    xk = _f64(xk)
    out = np.zeros(xk.shape[1:])
    lib().oracle_divided_difference(j, _f64(eps), out.size, xk.reshape(xk.shape[0], -1), out.reshape(-1))
    return out


def error_estimate(eps, xk, x):
    """(est, rho_hat) of one system from its perturbed solutions xk (K, n) and combination x (n):
    est = |prod eps| m_{K-1}^2 / m_{K-2} / ||x||_inf with m_j = ||f[eps_0..eps_j]||_inf."""
    xk = _f64(xk)
    est, rho = C.c_double(), C.c_double()
    lib().oracle_error_estimate(len(eps), _f64(eps), xk[0].size, xk.reshape(xk.shape[0], -1), _f64(x).reshape(-1),
                                C.byref(est), C.byref(rho))
    return est.value, rho.value


def scale_exponent(eps, est: float, rho_hat: float) -> int:
    """j of the node scale 2^-j that balances truncation against rounding (see psp_oracle.c)."""
    return int(lib().oracle_scale_exponent(len(eps), _f64(eps), float(est), float(rho_hat)))


def adaptive_batch(n, indptr, indices, values, sym: Symbolic, eps, b, tol: float, d=None):
    """Alg. 1 with the error test deciding the node size per Jacobian: solve every Jacobian at the
    nodes eps, estimate each combination's error from its perturbed solutions, and solve again the
    Jacobians whose estimate exceeds tol (or is NaN) at the nodes 2^-j eps, j from
    scale_exponent.  Returns (x, info, est, scale): the final combination, its info, its estimate
    and the scale applied (1 where the first solve was kept)."""
    values = _f64(values)
    b = _f64(b)
    eps = _f64(eps)
    batch = values.shape[0]
    x, info, xk, _ = sparse_batch(n, indptr, indices, values, sym, eps, b, d=d, keep_xk=True)
    est = np.zeros(batch)
    rho = np.zeros(batch)
    for s in range(batch):
        est[s], rho[s] = error_estimate(eps, xk[s], x[s])
    scale = np.ones(batch)
    for s in range(batch):
        if not (est[s] <= tol):
            scale[s] = 2.0 ** -scale_exponent(eps, est[s], rho[s])
    for sc in np.unique(scale[scale != 1.0]):
        idx = np.nonzero(scale == sc)[0]
        e2 = eps * sc
        x2, i2, xk2, _ = sparse_batch(n, indptr, indices, values[idx], sym, e2, b[idx], d=d, keep_xk=True)
        x[idx], info[idx] = x2, i2
        for t, s in enumerate(idx):
            est[s], _ = error_estimate(e2, xk2[t], x2[t])
    return x, info, est, scale


def grad_values(n, indptr, indices, c, xk, lamk):
    """dL/dA on pat(A): -sum_k c_k sum_r lam_k[i,r] x_k[j,r]; xk, lamk: (K, n, nrhs)."""
    xk = _f64(xk)
    lamk = _f64(lamk)
    K = xk.shape[0]
    nrhs = 1 if xk.ndim == 2 else xk.shape[2]
    g = np.zeros(int(indptr[-1]))
    lib().oracle_grad_values(n, _i32(indptr), _i32(indices), K, _f64(c), nrhs, xk.reshape(K, -1),
                             lamk.reshape(K, -1), g)
    return g


# ---------------------------------------------------------------- diagnostics
def power_rho(A: np.ndarray, d, probe: float, v0: np.ndarray, iters: int) -> float:
    """The power iteration for rho(A^{-1} D) as the library defines it: M = (A + probe D)^{-1} D,
    v = v0/||v0||, then iters times x = M v (pivoted solve), g = ||x||_2, v = x/g;
    rho = exp(mean log g over the last iters - iters//2 steps)."""
    n = A.shape[0]
    dd = np.ones(n) if d is None else np.asarray(d, dtype=np.float64)
    Ap = A + probe * np.diag(dd)
    v = np.asarray(v0, dtype=np.float64) / np.linalg.norm(v0)
    logs = []
    for _ in range(iters):
        x = pivoted_solve(Ap, dd * v)
        g = np.linalg.norm(x)
        logs.append(np.log(g))
        v = x / g
    return float(np.exp(np.mean(logs[iters // 2:])))


def power_rho_pivot_free(n, indptr, indices, values, sym: Symbolic, d, probe: float, v0, iters: int) -> float:
    """power_rho with the method's own solve: each x = (A + probe D)^{-1} D v comes from the
    pivot-free perturbed sparse factorisation (sparse_system, one node), and every norm is
    norm2.  With a tiny probe the pivot-free solve is only as accurate as its element growth
    allows, so this differs from power_rho by more than rounding; it is the sequence the
    library runs."""
    dd = None if d is None else np.asarray(d, dtype=np.float64)
    v = _f64(v0) / norm2(v0)
    logs = []
    for _ in range(iters):
        x, info = sparse_system(n, indptr, indices, values, sym, probe, v if dd is None else dd * v, d=dd)
        if info != 0:
            return float("nan")
        g = norm2(x)
        logs.append(np.log(g))
        v = x / g
    return float(np.exp(np.mean(logs[iters // 2:])))


def spectral_radius_AinvD(A: np.ndarray, d=None, iters: int = 200, seed: int = 0) -> float:
    """rho(A^{-1} D), the Neumann radius of Sec. II-B, from the growth rate of
    ||(A^{-1} D)^k v|| (pivoted solves).  The mean log growth over the second
    half of the iterations also converges when the dominant eigenvalues are a
    complex pair of equal modulus."""
    n = A.shape[0]
    dd = np.ones(n) if d is None else np.asarray(d, dtype=np.float64)
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(n)
    v /= np.linalg.norm(v)
    logs = []
    for _ in range(iters):
        w = pivoted_solve(A, dd * v)
        lam = np.linalg.norm(w)
        logs.append(np.log(lam))
        v = w / lam
    return float(np.exp(np.mean(logs[iters // 2:])))
