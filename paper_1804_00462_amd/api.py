"""Python binding of the SOR-SVD C ABI (include/sorsvd.h).

PyTorch provides device memory and the current HIP stream; every step of the
computation runs in the library's kernels. Names follow the C entry points.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import (SORSVD_BF16, SORSVD_DIAG, SORSVD_F16, SORSVD_F32, SORSVD_F64, AutoInfo, BoundsInfo, Info,
                   Opts, Problem, check)


def _torch():
    import torch
    return torch


def dtype_code(dtype):
    torch = _torch()
    if dtype == torch.float64:
        return SORSVD_F64
    if dtype == torch.float32:
        return SORSVD_F32
    if dtype == torch.bfloat16:
        return SORSVD_BF16
    if dtype == torch.float16:
        return SORSVD_F16
    raise TypeError(f"unsupported dtype {dtype}")


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _check_matrix(A):
    if A.dim() != 2 or not A.is_cuda:
        raise ValueError("A must be a 2-D device tensor")
    if A.stride(1) != 1:
        raise ValueError("A must be row-major (unit column stride)")


def _info_dict(o):
    return {"a_fro": o.a_fro, "err_fro": o.err_fro, "err_fro_explicit": o.err_fro_explicit,
            "sweeps": o.sweeps, "flags": o.flags, "a_noise_rel": o.a_noise_rel}


def make_opts(l=0, max_sweeps=0, refine=0, residual=0, split=0, tile=0, pass_efficient=0, col_exp=None, literal=0,
              out_f32=0):
    """col_exp: None, or a device int32 tensor of n column exponents (FP16 A;
    the caller keeps it alive while the options are in use)."""
    ce = None
    if col_exp is not None:
        torch = _torch()
        if col_exp.dtype != torch.int32 or not col_exp.is_cuda or not col_exp.is_contiguous():
            raise ValueError("col_exp must be a contiguous int32 device tensor")
        ce = col_exp.data_ptr()
    return Opts(l=l, max_sweeps=max_sweeps, refine=refine, residual=residual, split=split, tile=tile,
                pass_efficient=pass_efficient, col_exp=ce, literal=literal, out_f32=out_f32)


def workspace_bytes(m, n, k, q, dtype_or_code, **opts):
    code = dtype_or_code if isinstance(dtype_or_code, int) else dtype_code(dtype_or_code)
    o = make_opts(**opts)
    return int(_lib.load().sorsvd_workspace_bytes(m, n, k, q, code, ctypes.byref(o)))


class Plan:
    """Outputs and workspace for repeated SOR-SVDs of one shape (no allocation per call)."""

    def __init__(self, m, n, k, q, dtype, device="cuda", **opts):
        torch = _torch()
        self.m, self.n, self.k, self.q = m, n, k, q
        self.code = dtype if isinstance(dtype, int) else dtype_code(dtype)
        self.col_exp = opts.get("col_exp")  # kept alive with the plan
        if self.col_exp is not None and self.col_exp.numel() != n:
            raise ValueError("col_exp needs one exponent per column")
        self.opts = make_opts(**opts)
        lib = _lib.load()
        nbytes = int(lib.sorsvd_workspace_bytes(m, n, k, q, self.code, ctypes.byref(self.opts)))
        if nbytes == 0:
            raise _lib.SorsvdError(-1, "sorsvd_workspace_bytes")
        self.ws_bytes = nbytes
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        out_t = torch.float32 if opts.get("out_f32") else torch.float64
        self.U = torch.empty(m, k, dtype=out_t, device=device)
        self.S = torch.empty(k, dtype=torch.float64, device=device)
        self.V = torch.empty(n, k, dtype=out_t, device=device)

    def run(self, A, seed=0, stream=None):
        if self.code == SORSVD_DIAG:
            if A.dim() != 1 or A.shape[0] != self.n or A.dtype != _torch().float64 or not A.is_cuda:
                raise ValueError("diagonal A must be a 1-D FP64 device tensor of length n")
            lda = self.n
        else:
            _check_matrix(A)
            if tuple(A.shape) != (self.m, self.n) or dtype_code(A.dtype) != self.code:
                raise ValueError("A does not match the plan")
            lda = A.stride(0)
        lib = _lib.load()
        st = lib.sorsvd(_ptr(A), lda, self.code, self.m, self.n, self.k, self.q, seed,
                        _ptr(self.U), self.k, _ptr(self.S), _ptr(self.V), self.k,
                        _ptr(self.ws), self.ws_bytes, _stream(stream), ctypes.byref(self.opts))
        check(st, "sorsvd")
        return self.U, self.S, self.V

    def info(self, stream=None):
        out = Info()
        check(_lib.load().sorsvd_read_info(_ptr(self.ws), ctypes.byref(out), _stream(stream)), "sorsvd_read_info")
        return _info_dict(out)

    def capture(self, A, seed=0):
        """The whole launch sequence of run(A, seed) captured in a HIP graph
        (torch.cuda.CUDAGraph; the sequence holds no host synchronisation, no
        allocation and no memset node). Replaying it recomputes U, S, V of the
        current contents of A into this plan's outputs."""
        torch = _torch()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            self.run(A, seed)  # outside the capture: first-call set-up (occupancy queries)
        torch.cuda.current_stream().wait_stream(side)
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run(A, seed)
        return g


def sorsvd(A, k, q=0, seed=0, **opts):
    """Rank-k SOR-SVD of the device matrix A. Returns (U, S, V, info) as FP64 tensors."""
    plan = Plan(A.shape[0], A.shape[1], k, q, A.dtype, device=A.device, **opts)
    U, S, V = plan.run(A, seed)
    return U, S, V, plan.info()


def pack_f16(A, stream=None):
    """FP16 storage of an FP32 / FP64 device matrix with power-of-two column
    scaling: (A_stored, col_exp) with A = A_stored diag(2^-col_exp), the
    input of sorsvd(A_stored, ..., col_exp=col_exp)."""
    torch = _torch()
    _check_matrix(A)
    m, n = A.shape
    out = torch.empty(m, n, dtype=torch.float16, device=A.device)
    e = torch.empty(n, dtype=torch.int32, device=A.device)
    st = _lib.load().sorsvd_pack_f16(_ptr(A), A.stride(0), dtype_code(A.dtype), m, n, _ptr(out), n, _ptr(e),
                                     _stream(stream))
    check(st, "sorsvd_pack_f16")
    return out, e


def sorsvd_diag(sigma, k, q=0, seed=0, **opts):
    """SOR-SVD of A = diag(sigma) (1-D FP64 device tensor); (U, S, V, info)."""
    n = sigma.shape[0]
    plan = Plan(n, n, k, q, SORSVD_DIAG, device=sigma.device, **opts)
    U, S, V = plan.run(sigma, seed)
    return U, S, V, plan.info()


def philox_normal(seed, rows, cols, stream_id=0, word2=0, device="cuda"):
    """rows x cols N(0,1) draws (element (i, j) = draw i + j*rows), as a device FP64 tensor."""
    torch = _torch()
    out = torch.empty(cols, rows, dtype=torch.float64, device=device)  # column-major storage
    check(_lib.load().sorsvd_philox_normal(seed, stream_id, word2, rows, cols, _ptr(out), _stream()),
          "sorsvd_philox_normal")
    return out.t()


def _step_ws(m, n, l, code, device):
    torch = _torch()
    nbytes = int(_lib.load().sorsvd_step_workspace_bytes(m, n, l, code))
    if nbytes == 0:
        raise _lib.SorsvdError(-1, "sorsvd_step_workspace_bytes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


def step_sketch(A, X):
    """T = A X (X: n x l FP64 device tensor)."""
    torch = _torch()
    _check_matrix(A)
    m, n = A.shape
    l = X.shape[1]
    code = dtype_code(A.dtype)
    X = X.contiguous().to(torch.float64)
    T = torch.empty(m, l, dtype=torch.float64, device=A.device)
    ws, nb = _step_ws(m, n, l, code, A.device)
    check(_lib.load().sorsvd_step_sketch(_ptr(A), A.stride(0), code, m, n, _ptr(X), l, _ptr(T),
                                         _ptr(ws), nb, _stream()), "sorsvd_step_sketch")
    return T


def step_orbit(A, Y):
    """T = A^T Y (Y: m x l FP64 device tensor)."""
    torch = _torch()
    _check_matrix(A)
    m, n = A.shape
    l = Y.shape[1]
    code = dtype_code(A.dtype)
    Y = Y.contiguous().to(torch.float64)
    T = torch.empty(n, l, dtype=torch.float64, device=A.device)
    ws, nb = _step_ws(m, n, l, code, A.device)
    check(_lib.load().sorsvd_step_orbit(_ptr(A), A.stride(0), code, m, n, _ptr(Y), l, _ptr(T),
                                        _ptr(ws), nb, _stream()), "sorsvd_step_orbit")
    return T


def step_qr(T):
    """T = Q R with orthonormal Q and upper-triangular R (positive diagonal)."""
    torch = _torch()
    T = T.contiguous().to(torch.float64)
    rows, l = T.shape
    Q = torch.empty(rows, l, dtype=torch.float64, device=T.device)
    R = torch.empty(l, l, dtype=torch.float64, device=T.device)
    ws, nb = _step_ws(rows, l, l, SORSVD_F64, T.device)
    check(_lib.load().sorsvd_step_qr(_ptr(T), rows, l, _ptr(Q), _ptr(R), _ptr(ws), nb, _stream()),
          "sorsvd_step_qr")
    return Q, R


def step_project(A, Q1, Q2):
    """M = Q1^T A Q2."""
    torch = _torch()
    _check_matrix(A)
    m, n = A.shape
    l = Q1.shape[1]
    code = dtype_code(A.dtype)
    Q1 = Q1.contiguous().to(torch.float64)
    Q2 = Q2.contiguous().to(torch.float64)
    M = torch.empty(l, l, dtype=torch.float64, device=A.device)
    ws, nb = _step_ws(m, n, l, code, A.device)
    check(_lib.load().sorsvd_step_project(_ptr(A), A.stride(0), code, m, n, _ptr(Q1), _ptr(Q2), l,
                                          _ptr(M), _ptr(ws), nb, _stream()), "sorsvd_step_project")
    return M


def step_core_svd(M, k, max_sweeps=0):
    """M = U~ diag(s) V~^T; returns the first k columns of U~, s, V~."""
    torch = _torch()
    M = M.contiguous().to(torch.float64)
    l = M.shape[0]
    Ut = torch.empty(l, k, dtype=torch.float64, device=M.device)
    Vt = torch.empty(l, k, dtype=torch.float64, device=M.device)
    s = torch.empty(k, dtype=torch.float64, device=M.device)
    ws, nb = _step_ws(l, l, l, SORSVD_F64, M.device)
    check(_lib.load().sorsvd_step_core_svd(_ptr(M), l, k, _ptr(Ut), _ptr(s), _ptr(Vt), max_sweeps,
                                           _ptr(ws), nb, _stream()), "sorsvd_step_core_svd")
    info = Info()
    check(_lib.load().sorsvd_read_info(_ptr(ws), ctypes.byref(info), _stream()), "sorsvd_read_info")
    return Ut, s, Vt, {"sweeps": info.sweeps, "flags": info.flags}


def pass_timing(enable, capacity=256):
    """Turn the per-launch event timing of the pass kernel over A on or off."""
    check(_lib.load().sorsvd_pass_timing(1 if enable else 0, capacity if enable else 0), "sorsvd_pass_timing")


def pass_timing_read():
    """(total_ms, launches, algorithmic_bytes, flops) recorded since the last read."""
    ms, n, b, f = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
    check(_lib.load().sorsvd_pass_timing_read(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(b),
                                              ctypes.byref(f)), "sorsvd_pass_timing_read")
    return ms.value, n.value, b.value, f.value


class Batch:
    """A batch of independent SOR-SVDs of uneven sizes, run as one launch per step.

    mats: list of 2-D row-major device tensors of one dtype (float32 or float64);
    ks, qs, seeds, ls: per-problem rank, power steps, Omega seed and sketch width
    (l = 0 means l = k). Allocates the FP64 outputs U_i (m_i x k_i), S_i, V_i
    (n_i x k_i) and the workspace once; run() recomputes them from the current
    contents of mats.
    """

    def __init__(self, mats, ks, qs, seeds, ls=None, max_sweeps=0):
        torch = _torch()
        if not mats:
            raise ValueError("empty batch")
        diag = mats[0].dim() == 1
        code = SORSVD_DIAG if diag else dtype_code(mats[0].dtype)
        count = len(mats)
        ls = ls if ls is not None else [0] * count
        if not (len(ks) == len(qs) == len(seeds) == len(ls) == count):
            raise ValueError("per-problem lists must match the number of matrices")
        self.mats = list(mats)
        self.U, self.S, self.V = [], [], []
        probs = (Problem * count)()
        for i, A in enumerate(mats):
            if diag:
                if A.dim() != 1 or A.dtype != torch.float64 or not A.is_cuda:
                    raise ValueError("diagonal problems are 1-D FP64 device tensors")
                m = n = A.shape[0]
            else:
                _check_matrix(A)
                if dtype_code(A.dtype) != code:
                    raise ValueError("all matrices of a batch share one dtype")
                m, n = A.shape
            k = int(ks[i])
            U = torch.empty(m, k, dtype=torch.float64, device=A.device)
            S = torch.empty(k, dtype=torch.float64, device=A.device)
            V = torch.empty(n, k, dtype=torch.float64, device=A.device)
            self.U.append(U)
            self.S.append(S)
            self.V.append(V)
            probs[i] = Problem(A=A.data_ptr(), lda=n if diag else A.stride(0), m=m, n=n, k=k, l=int(ls[i]), q=int(qs[i]),
                               reserved=0, seed=int(seeds[i]), U=U.data_ptr(), ldu=k, S=S.data_ptr(),
                               V=V.data_ptr(), ldv=k)
        self._probs = probs
        lib = _lib.load()
        handle = ctypes.c_void_p()
        nbytes = ctypes.c_size_t()
        opts = make_opts(max_sweeps=max_sweeps)
        check(lib.sorsvd_batch_create(count, probs, code, ctypes.byref(opts), ctypes.byref(handle),
                                      ctypes.byref(nbytes)), "sorsvd_batch_create")
        self._h = handle
        self.ws_bytes = nbytes.value
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=mats[0].device)
        check(lib.sorsvd_batch_upload(self._h, _ptr(self.ws), self.ws_bytes, _stream()), "sorsvd_batch_upload")
        self._graph = None

    def __len__(self):
        return len(self.mats)

    def run(self, stream=None):
        check(_lib.load().sorsvd_batch_run(self._h, _ptr(self.ws), _stream(stream)), "sorsvd_batch_run")

    def config(self):
        c = (ctypes.c_int32 * 6)()
        check(_lib.load().sorsvd_batch_get_config(self._h, c), "sorsvd_batch_get_config")
        return list(c)

    def set_config(self, cfg):
        c = (ctypes.c_int32 * 6)(*[int(x) for x in cfg])
        check(_lib.load().sorsvd_batch_set_config(self._h, c), "sorsvd_batch_set_config")

    def autotune(self, stream=None):
        c = (ctypes.c_int32 * 6)()
        check(_lib.load().sorsvd_batch_autotune(self._h, _ptr(self.ws), _stream(stream), c),
              "sorsvd_batch_autotune")
        return list(c)

    def info(self, stream=None):
        out = (Info * len(self.mats))()
        check(_lib.load().sorsvd_batch_read_info(self._h, out, _stream(stream)), "sorsvd_batch_read_info")
        return [_info_dict(o) for o in out]

    def capture(self):
        """Capture the run's launch sequence in a HIP graph (replaces an earlier one)."""
        self.release_graph()
        g = ctypes.c_void_p()
        check(_lib.load().sorsvd_batch_graph(self._h, _ptr(self.ws), ctypes.byref(g)), "sorsvd_batch_graph")
        self._graph = g

    def replay(self, stream=None):
        if self._graph is None:
            raise RuntimeError("no graph captured")
        check(_lib.load().sorsvd_graph_launch(self._graph, _stream(stream)), "sorsvd_graph_launch")

    def release_graph(self):
        if self._graph is not None:
            _lib.load().sorsvd_graph_destroy(self._graph)
            self._graph = None

    def close(self):
        self.release_graph()
        if self._h:
            _lib.load().sorsvd_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------ learned (k, q)

def probe_features(A, seed=0):
    """128 FP32 features of A (2-D device matrix, or 1-D FP64 diagonal) from the probe sketch."""
    torch = _torch()
    lib = _lib.load()
    if A.dim() == 1:
        code, m, n, lda = SORSVD_DIAG, A.shape[0], A.shape[0], A.shape[0]
    else:
        _check_matrix(A)
        code, (m, n), lda = dtype_code(A.dtype), A.shape, A.stride(0)
    nbytes = int(lib.sorsvd_probe_workspace_bytes(m, n, code))
    if nbytes == 0:
        raise _lib.SorsvdError(-1, "sorsvd_probe_workspace_bytes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
    feat = torch.empty(128, dtype=torch.float32, device=A.device)
    check(lib.sorsvd_probe_features(_ptr(A), lda, code, m, n, seed, _ptr(feat), _ptr(ws), nbytes, _stream()),
          "sorsvd_probe_features")
    return feat


def mlp_param_count():
    return int(_lib.load().sorsvd_mlp_param_count())


class MLP:
    """Device parameters, Adam moments and scratch of the (k, q) network."""

    def __init__(self, params, max_batch=256):
        torch = _torch()
        self.params = params
        self.m = torch.zeros_like(params)
        self.v = torch.zeros_like(params)
        self.grad = torch.zeros_like(params)
        self.loss = torch.zeros(1, dtype=torch.float32, device=params.device)
        self.max_batch = max_batch
        self.work = torch.empty(int(_lib.load().sorsvd_mlp_work_floats(max_batch)), dtype=torch.float32,
                                device=params.device)
        self.step = 0

    def _check(self, X):
        if X.dtype != _torch().float32 or X.dim() != 2 or X.shape[1] != 128 or X.shape[0] > self.max_batch:
            raise ValueError("X must be B x 128 FP32 with B <= max_batch")
        return X.contiguous()

    def forward(self, X):
        X = self._check(X)
        Y = _torch().empty(X.shape[0], 4, dtype=_torch().float32, device=X.device)
        check(_lib.load().sorsvd_mlp_forward(_ptr(self.params), _ptr(X), X.shape[0], _ptr(Y), _ptr(self.work),
                                             _stream()), "sorsvd_mlp_forward")
        return Y

    def backward(self, X, T):
        X = self._check(X)
        T = T.contiguous()
        check(_lib.load().sorsvd_mlp_backward(_ptr(self.params), _ptr(X), _ptr(T), X.shape[0], _ptr(self.grad),
                                              _ptr(self.loss), _ptr(self.work), _stream()), "sorsvd_mlp_backward")
        return self.grad, self.loss

    def train_step(self, X, T, lr=1e-3):
        X = self._check(X)
        T = T.contiguous()
        self.step += 1
        check(_lib.load().sorsvd_mlp_train_step(_ptr(self.params), _ptr(self.m), _ptr(self.v), _ptr(X), _ptr(T),
                                                X.shape[0], self.step, lr, _ptr(self.grad), _ptr(self.loss),
                                                _ptr(self.work), _stream()), "sorsvd_mlp_train_step")
        return self.loss


def auto(A, tol, params=None, seed=0):
    """Learned (k, q) + judge + fallback (params None: fallback only). Returns (U, S, V, info dict, status)."""
    torch = _torch()
    lib = _lib.load()
    if A.dim() == 1:  # A = diag(sigma), FP64 (the stand-in of the training spectra)
        if A.dtype != torch.float64 or not A.is_cuda:
            raise ValueError("diagonal A must be a 1-D FP64 device tensor")
        code, m, n, lda = SORSVD_DIAG, A.shape[0], A.shape[0], A.shape[0]
    else:
        _check_matrix(A)
        code, (m, n), lda = dtype_code(A.dtype), A.shape, A.stride(0)
    kcap = min(1024, m, n)
    nbytes = int(lib.sorsvd_auto_workspace_bytes(m, n, code))
    if nbytes == 0:
        raise _lib.SorsvdError(-1, "sorsvd_auto_workspace_bytes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
    U = torch.empty(m, kcap, dtype=torch.float64, device=A.device)
    S = torch.empty(kcap, dtype=torch.float64, device=A.device)
    V = torch.empty(n, kcap, dtype=torch.float64, device=A.device)
    out = AutoInfo()
    st = lib.sorsvd_auto(_ptr(A), lda, code, m, n, seed, float(tol),
                         _ptr(params) if params is not None else None, _ptr(U), kcap, _ptr(S), _ptr(V), kcap,
                         _ptr(ws), nbytes, _stream(), ctypes.byref(out))
    if st not in (0, -6):
        check(st, "sorsvd_auto")
    k = out.k_used
    info = {"k_used": k, "q_used": out.q_used, "used_fallback": out.used_fallback, "runs": out.runs,
            "err": out.err, "err_stored": out.err_stored, "k_pred": list(out.k_pred), "flags": out.flags,
            "met": st == 0}
    return U[:, :k], S[:k], V[:, :k], info


def predict_kq(A, params, tol=1e-3, seed=0):
    """The (k, q) sorsvd_auto would run first (probe + network), without running
    it. Returns (k, q, k_pred list, predicted flag)."""
    torch = _torch()
    lib = _lib.load()
    if A.dim() == 1:
        code, m, n, lda = SORSVD_DIAG, A.shape[0], A.shape[0], A.shape[0]
    else:
        _check_matrix(A)
        code, (m, n), lda = dtype_code(A.dtype), A.shape, A.stride(0)
    nbytes = int(lib.sorsvd_auto_workspace_bytes(m, n, code))
    if nbytes == 0:
        raise _lib.SorsvdError(-1, "sorsvd_auto_workspace_bytes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=A.device)
    k, q, kp = ctypes.c_int64(), ctypes.c_int32(), (ctypes.c_double * 4)()
    st = lib.sorsvd_predict_kq(_ptr(A), lda, code, m, n, seed, _ptr(params), float(tol), ctypes.byref(k),
                               ctypes.byref(q), kp, _ptr(ws), nbytes, _stream())
    if st not in (0, -6):
        check(st, "sorsvd_predict_kq")
    return int(k.value), int(q.value), list(kp), st == 0


def bounds(V1, sigma, k, l, p, q=0, seed=0):
    """Th. 4 - Th. 7 for the Omega of seed `seed`: V1 (n x (l - p), FP64 on the
    device) the leading right singular vectors of A, sigma (host, descending)
    its singular values. Returns a dict with omega2_norm, omega1_pinv_norm,
    th4 (k), th5_fro, th5_2, th6 (k), th7_fro, th7_2."""
    torch = _torch()
    lib = _lib.load()
    _check_matrix(V1)
    if V1.dtype != torch.float64:
        raise TypeError("bounds takes FP64 V1")
    n = V1.shape[0]
    sig = np.ascontiguousarray(np.asarray(sigma, dtype=np.float64))
    nbytes = int(lib.sorsvd_bounds_workspace_bytes(n, l, p))
    if nbytes == 0:
        raise _lib.SorsvdError(-1, "sorsvd_bounds_workspace_bytes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=V1.device)
    th4 = np.zeros(k)
    th6 = np.zeros(k)
    out = BoundsInfo()
    dp = ctypes.POINTER(ctypes.c_double)
    check(lib.sorsvd_bounds(_ptr(V1), V1.stride(0), n, l, p, k, q, seed, sig.ctypes.data_as(dp), sig.size,
                            th4.ctypes.data_as(dp), th6.ctypes.data_as(dp), ctypes.byref(out), _ptr(ws), nbytes,
                            _stream()), "sorsvd_bounds")
    return {"omega2_norm": out.omega2_norm, "omega1_pinv_norm": out.omega1_pinv_norm, "th4": th4,
            "th5_fro": out.th5_fro, "th5_2": out.th5_2, "th6": th6, "th7_fro": out.th7_fro, "th7_2": out.th7_2}


def rpca(X, l, q=1, seed=0, tol=1e-7, max_iter=100):
    """Robust PCA X = L + S by the ALM-SOR-SVD iteration (FP64 X on the device).
    Returns (L, S, info dict); info["met"] tells whether the tolerance was met."""
    torch = _torch()
    lib = _lib.load()
    _check_matrix(X)
    if X.dtype != torch.float64:
        raise TypeError("rpca takes FP64 X")
    m, n = X.shape
    nbytes = int(lib.sorsvd_rpca_workspace_bytes(m, n, l, q))
    if nbytes == 0:
        raise _lib.SorsvdError(-1, "sorsvd_rpca_workspace_bytes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=X.device)
    L = torch.empty(m, n, dtype=torch.float64, device=X.device)
    S = torch.empty(m, n, dtype=torch.float64, device=X.device)
    out = _lib.RpcaInfo()
    st = lib.sorsvd_rpca(_ptr(X), X.stride(0), m, n, l, q, seed, float(tol), int(max_iter), _ptr(L), _ptr(S), n,
                         _ptr(ws), nbytes, _stream(), ctypes.byref(out))
    if st not in (0, -6):
        check(st, "sorsvd_rpca")
    info = {"iters": out.iters, "rank": out.rank, "nnz_s": out.nnz_s, "xi": out.xi, "lambda": out.lam,
            "norm2": out.norm2, "met": st == 0}
    return L, S, info

