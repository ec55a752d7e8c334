"""ctypes binding of libspsvm.so (C ABI in include/spsvm.h).

Argument marshalling only: every step of training and prediction runs in the library's HIP kernels.
PyTorch provides device memory (inputs, workspace, outputs) and the stream. If the library is not
built, or a tensor is not on the GPU, the calls raise; there is no CPU fallback.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspsvm.so")

SPSVM_F64, SPSVM_F32, SPSVM_MIXED = 0, 1, 2
SPSVM_DT_F32, SPSVM_DT_F64 = 0, 1
PRECISIONS = {"f64": SPSVM_F64, "f32": SPSVM_F32, "mixed": SPSVM_MIXED}

EXPORTED = (
    "spsvm_options_default",
    "spsvm_train_workspace_bytes",
    "spsvm_fixed_workspace_bytes",
    "spsvm_train",
    "spsvm_train_fixed_basis",
    "spsvm_batch_workspace_bytes",
    "spsvm_train_batch",
    "spsvm_train_shared_workspace_bytes",
    "spsvm_train_shared",
    "spsvm_model_get",
    "spsvm_model_stats",
    "spsvm_model_bias",
    "spsvm_train_csr_workspace_bytes",
    "spsvm_train_csr",
    "spsvm_predict_csr",
    "spsvm_ovo_workspace_bytes",
    "spsvm_train_ovo",
    "spsvm_predict_ovo_workspace_bytes",
    "spsvm_predict_ovo",
    "spsvm_predict",
    "spsvm_model_free",
    "spsvm_status_string",
    "spsvm_last_error",
    "spsvm_rbf_block",
    "spsvm_rbf_block_workspace_bytes",
    "spsvm_newton_solve_workspace_bytes",
    "spsvm_newton_solve",
    "spsvm_candidate_draw",
    "spsvm_score_candidates",
    "spsvm_newton_solve_noalloc",
    "spsvm_score_workspace_bytes",
)


class SpsvmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"spsvm status {status}: {msg}")
        self.status = status


class Options(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("kappa", ctypes.c_int32),
        ("growth", ctypes.c_double),
        ("chunk_cap", ctypes.c_int32),
        ("newton_tol", ctypes.c_double),
        ("newton_ftol", ctypes.c_double),
        ("newton_max_iter", ctypes.c_int32),
        ("precision", ctypes.c_int),
        ("log_level", ctypes.c_int32),
        ("profile", ctypes.c_int32),
        ("refactor_frac", ctypes.c_double),
        ("bias", ctypes.c_int32),
        ("eps_stop", ctypes.c_double),
        ("kxj_host", ctypes.c_int32),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("stages", ctypes.c_int64),
        ("additions", ctypes.c_int64),
        ("newton_iters", ctypes.c_int64),
        ("factorizations", ctypes.c_int64),
        ("score_passes", ctypes.c_int64),
        ("score_passes_active", ctypes.c_int64),
        ("score_slot_passes", ctypes.c_int64),
        ("ls_passes", ctypes.c_int64),
        ("iter_cap_hits", ctypes.c_int64),
        ("stage_redos", ctypes.c_int64),
        ("incremental_factorizations", ctypes.c_int64),
        ("n_sv", ctypes.c_int64),
        ("grad_norm", ctypes.c_double),
        ("seconds_select", ctypes.c_double),
        ("seconds_newton", ctypes.c_double),
        ("kblock_launches", ctypes.c_int64),
        ("kblock_seconds", ctypes.c_double),
        ("kblock_flops", ctypes.c_double),
        ("syrk_launches", ctypes.c_int64),
        ("syrk_seconds", ctypes.c_double),
        ("syrk_flops", ctypes.c_double),
        ("score_launches", ctypes.c_int64),
        ("score_seconds", ctypes.c_double),
        ("score_bytes", ctypes.c_double),
        ("chol_calls", ctypes.c_int64),
        ("chol_seconds", ctypes.c_double),
        ("chol_flops", ctypes.c_double),
        ("kblock_mfma_flops", ctypes.c_double),
        ("jitter_retries", ctypes.c_int64),
        ("stop_reason", ctypes.c_int64),
        ("train_error", ctypes.c_double),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load(path: str = LIB_PATH):
    """Loads the library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run paper_1404_1066_amd.build.build() first")
    lib = ctypes.CDLL(path)
    P, I64, D, VP = ctypes.POINTER, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
    lib.spsvm_options_default.argtypes = [P(Options)]
    lib.spsvm_options_default.restype = None
    lib.spsvm_train_workspace_bytes.argtypes = [I64, I64, I64, ctypes.c_int, P(Options), P(ctypes.c_size_t)]
    lib.spsvm_fixed_workspace_bytes.argtypes = [I64, I64, I64, ctypes.c_int, P(Options), P(ctypes.c_size_t)]
    lib.spsvm_rbf_block_workspace_bytes.argtypes = [I64, I64, ctypes.c_int, P(ctypes.c_size_t)]
    lib.spsvm_train.argtypes = [VP, ctypes.c_int, VP, I64, I64, D, D, I64, P(Options), VP, ctypes.c_size_t, VP, P(VP)]
    lib.spsvm_train_fixed_basis.argtypes = [VP, ctypes.c_int, VP, I64, I64, D, D, P(I64), I64, P(Options), VP,
                                            ctypes.c_size_t, VP, P(VP)]
    lib.spsvm_batch_workspace_bytes.argtypes = [I64, I64, I64, I64, ctypes.c_int, P(Options), P(ctypes.c_size_t)]
    lib.spsvm_train_batch.argtypes = [VP, ctypes.c_int, I64, I64, I64, VP, P(D), P(D), P(I64), I64, P(Options), VP,
                                      ctypes.c_size_t, VP, P(VP)]
    lib.spsvm_train_shared_workspace_bytes.argtypes = [I64, I64, I64, P(D), I64, ctypes.c_int, P(Options),
                                                       P(ctypes.c_size_t)]
    lib.spsvm_train_shared.argtypes = [VP, ctypes.c_int, I64, I64, I64, VP, P(D), P(D), I64, P(Options), VP,
                                       ctypes.c_size_t, VP, P(VP)]
    lib.spsvm_model_get.argtypes = [VP, P(I64), P(I64), P(D), P(D)]
    lib.spsvm_model_stats.argtypes = [VP, P(Stats)]
    lib.spsvm_model_bias.argtypes = [VP, P(D)]
    lib.spsvm_train_csr_workspace_bytes.argtypes = [I64, I64, I64, P(Options), P(ctypes.c_size_t)]
    lib.spsvm_train_csr.argtypes = [VP, VP, VP, I64, I64, VP, D, D, I64, P(Options), VP, ctypes.c_size_t, VP, P(VP)]
    lib.spsvm_predict_csr.argtypes = [VP, VP, VP, VP, I64, VP, VP]
    lib.spsvm_ovo_workspace_bytes.argtypes = [I64, I64, I64, ctypes.c_int, P(Options), P(ctypes.c_size_t)]
    lib.spsvm_train_ovo.argtypes = [VP, ctypes.c_int, VP, I64, I64, ctypes.c_int32, D, D, I64, P(Options), VP,
                                    ctypes.c_size_t, VP, P(VP)]
    lib.spsvm_predict_ovo_workspace_bytes.argtypes = [I64, ctypes.c_int32, P(ctypes.c_size_t)]
    lib.spsvm_predict_ovo.argtypes = [P(VP), ctypes.c_int32, VP, ctypes.c_int, I64, VP, VP, ctypes.c_size_t, VP]
    lib.spsvm_predict.argtypes = [VP, VP, ctypes.c_int, I64, VP, VP]
    lib.spsvm_model_free.argtypes = [VP]
    lib.spsvm_model_free.restype = None
    lib.spsvm_status_string.argtypes = [ctypes.c_int]
    lib.spsvm_status_string.restype = ctypes.c_char_p
    lib.spsvm_last_error.argtypes = []
    lib.spsvm_last_error.restype = ctypes.c_char_p
    lib.spsvm_rbf_block.argtypes = [VP, ctypes.c_int, I64, I64, VP, I64, ctypes.c_int, D, VP, I64, VP,
                                    ctypes.c_size_t, VP]
    lib.spsvm_newton_solve_workspace_bytes.argtypes = [I64, P(ctypes.c_size_t)]
    lib.spsvm_newton_solve.argtypes = [VP, I64, I64, VP, VP, VP, ctypes.c_size_t, VP]
    lib.spsvm_candidate_draw.argtypes = [ctypes.c_uint64, I64, I64, ctypes.c_int32, P(ctypes.c_int32)]
    lib.spsvm_score_workspace_bytes.argtypes = [I64, P(ctypes.c_size_t)]
    lib.spsvm_newton_solve_noalloc.argtypes = [VP, I64, I64, VP, VP, VP]
    I32 = ctypes.c_int32
    lib.spsvm_score_candidates.argtypes = [VP, VP, I64, VP, ctypes.c_int, I64, P(D), I32, D, P(D), P(D), P(I32),
                                           P(I32), P(I32), VP, ctypes.c_size_t, VP]
    for name in ("spsvm_train_shared_workspace_bytes", "spsvm_train_shared", "spsvm_train_csr_workspace_bytes", "spsvm_train_csr", "spsvm_predict_csr", "spsvm_ovo_workspace_bytes", "spsvm_train_ovo", "spsvm_predict_ovo_workspace_bytes",
                 "spsvm_predict_ovo", "spsvm_newton_solve_noalloc", "spsvm_score_candidates", "spsvm_score_workspace_bytes", "spsvm_candidate_draw", "spsvm_rbf_block", "spsvm_rbf_block_workspace_bytes", "spsvm_newton_solve_workspace_bytes", "spsvm_newton_solve",
                 "spsvm_train_workspace_bytes", "spsvm_fixed_workspace_bytes", "spsvm_train",
                 "spsvm_train_fixed_basis", "spsvm_batch_workspace_bytes", "spsvm_train_batch", "spsvm_model_get", "spsvm_model_stats", "spsvm_model_bias", "spsvm_predict"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _check(status: int):
    if status != 0:
        lib = load()
        raise SpsvmError(status, lib.spsvm_last_error().decode() or lib.spsvm_status_string(status).decode())


def options(**kw) -> Options:
    lib = load()
    o = Options()
    lib.spsvm_options_default(ctypes.byref(o))
    for k, v in kw.items():
        if v is None:
            continue
        if k == "precision" and isinstance(v, str):
            v = PRECISIONS[v]
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return SPSVM_DT_F32
    if t.dtype == torch.float64:
        return SPSVM_DT_F64
    raise TypeError("feature matrices must be float32 or float64")


def _need_gpu(t: torch.Tensor, name: str):
    if not (isinstance(t, torch.Tensor) and t.is_cuda):
        raise ValueError(f"{name} must be a tensor on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _stream_ptr(stream) -> Optional[int]:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Model:
    """A trained SP-SVM model (owned by the library; freed with the object)."""

    def __init__(self, ptr: int):
        self._ptr = ctypes.c_void_p(ptr)

    def __del__(self):
        ptr = getattr(self, "_ptr", None)
        # at interpreter exit the module's globals may already be gone; the process frees the memory then
        if ptr is not None and ptr.value and _lib is not None:
            _lib.spsvm_model_free(ptr)
            self._ptr = ctypes.c_void_p(None)

    @property
    def m(self) -> int:
        m = ctypes.c_int64()
        _check(load().spsvm_model_get(self._ptr, ctypes.byref(m), None, None, None))
        return m.value

    def get(self):
        """(J, beta, F): basis row indices in order of addition, coefficients, and F of Eq. 4 (paper scale)."""
        import numpy as np

        m = self.m
        J = np.zeros(m, dtype=np.int64)
        beta = np.zeros(m, dtype=np.float64)
        F = ctypes.c_double()
        _check(load().spsvm_model_get(self._ptr, None, J.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                      beta.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(F)))
        return J, beta, F.value

    @property
    def bias(self) -> float:
        """The offset b of Eq. 4 (0 unless trained with bias=1)."""
        b = ctypes.c_double()
        _check(load().spsvm_model_bias(self._ptr, ctypes.byref(b)))
        return b.value

    def stats(self) -> dict:
        s = Stats()
        _check(load().spsvm_model_stats(self._ptr, ctypes.byref(s)))
        return s.as_dict()

    def predict(self, Xt: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        """Decision values (float64, on the GPU) for the rows of Xt."""
        _need_gpu(Xt, "Xt")
        if out is None:
            out = torch.empty(Xt.shape[0], dtype=torch.float64, device=Xt.device)
        _need_gpu(out, "out")
        _check(load().spsvm_predict(self._ptr, ctypes.c_void_p(Xt.data_ptr()), _dtype_code(Xt), Xt.shape[0],
                                    ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(_stream_ptr(stream))))
        return out


def workspace_bytes(n: int, d: int, J_max: int, fixed: bool = False, dtype=torch.float32, batch: bool = False,
                    problems: int = 1, **opts) -> int:
    """Workspace bytes for train (default), train_fixed_basis (fixed=True) or train_batch (batch=True, with
    `problems` problems on J_max shared basis vectors)."""
    o = options(**opts)
    b = ctypes.c_size_t()
    dt = SPSVM_DT_F64 if dtype == torch.float64 else SPSVM_DT_F32
    if batch:
        _check(load().spsvm_batch_workspace_bytes(n, d, problems, J_max, dt, ctypes.byref(o), ctypes.byref(b)))
    else:
        fn = load().spsvm_fixed_workspace_bytes if fixed else load().spsvm_train_workspace_bytes
        _check(fn(n, d, J_max, dt, ctypes.byref(o), ctypes.byref(b)))
    return b.value


def _workspace(nbytes: int, device, workspace: Optional[torch.Tensor]):
    """(tensor, size in bytes). A caller-given workspace is passed with its own size; the library checks it."""
    if workspace is not None:
        _need_gpu(workspace, "workspace")
        return workspace, workspace.numel() * workspace.element_size()
    # torch's caching allocator returns 512-byte aligned blocks
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


def train(X: torch.Tensor, y: torch.Tensor, C: float, gamma: float, J_max: int, workspace=None, stream=None,
          **opts) -> Model:
    """Greedy SP-SVM training; options as in spsvm_options (seed, kappa, growth, chunk_cap, newton_tol,
    newton_ftol, newton_max_iter, precision in {'f64', 'f32'}, log_level)."""
    _need_gpu(X, "X")
    _need_gpu(y, "y")
    if y.dtype != torch.float32:
        raise TypeError("y must be float32")
    n, d = X.shape
    o = options(**opts)
    ws, nbytes = _workspace(workspace_bytes(n, d, J_max, dtype=X.dtype, **opts), X.device, workspace)
    out = ctypes.c_void_p()
    _check(load().spsvm_train(ctypes.c_void_p(X.data_ptr()), _dtype_code(X), ctypes.c_void_p(y.data_ptr()), n, d,
                              float(C), float(gamma), int(J_max), ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()),
                              nbytes, ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(out)))
    return Model(out.value)


def train_fixed_basis(X: torch.Tensor, y: torch.Tensor, C: float, gamma: float, J: Sequence[int], workspace=None,
                      stream=None, **opts) -> Model:
    """Newton re-optimisation of Eq. 4 on the given basis rows J (no selection), from beta = 0."""
    import numpy as np

    _need_gpu(X, "X")
    _need_gpu(y, "y")
    if y.dtype != torch.float32:
        raise TypeError("y must be float32")
    n, d = X.shape
    Jh = np.ascontiguousarray(np.asarray(J, dtype=np.int64))
    o = options(**opts)
    ws, nbytes = _workspace(workspace_bytes(n, d, Jh.size, fixed=True, dtype=X.dtype, **opts), X.device, workspace)
    out = ctypes.c_void_p()
    _check(load().spsvm_train_fixed_basis(ctypes.c_void_p(X.data_ptr()), _dtype_code(X), ctypes.c_void_p(y.data_ptr()),
                                          n, d, float(C), float(gamma),
                                          Jh.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), Jh.size, ctypes.byref(o),
                                          ctypes.c_void_p(ws.data_ptr()), nbytes,
                                          ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(out)))
    return Model(out.value)


# ------------------------------------------------------------------------------------------- components
def rbf_block(X: torch.Tensor, idx: torch.Tensor, gamma: float, precision: str = "f32", out=None, stream=None):
    """K[i, c] = exp(-gamma |x_i - x_idx[c]|^2) for all rows of X (spsvm_rbf_block)."""
    _need_gpu(X, "X")
    _need_gpu(idx, "idx")
    if idx.dtype != torch.int32:
        raise TypeError("idx must be int32")
    n, d = X.shape
    ncols = idx.numel()
    dt = torch.float64 if precision == "f64" else torch.float32
    if out is None:
        out = torch.empty((n, ncols), dtype=dt, device=X.device)
    _need_gpu(out, "out")
    b = ctypes.c_size_t()
    _check(load().spsvm_rbf_block_workspace_bytes(n, d, _dtype_code(X), ctypes.byref(b)))
    ws = torch.empty(max(b.value, 256), dtype=torch.uint8, device=X.device)
    _check(load().spsvm_rbf_block(ctypes.c_void_p(X.data_ptr()), _dtype_code(X), n, d, ctypes.c_void_p(idx.data_ptr()),
                                  ncols, PRECISIONS[precision], float(gamma), ctypes.c_void_p(out.data_ptr()),
                                  out.stride(0), ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                  ctypes.c_void_p(_stream_ptr(stream))))
    return out


def newton_solve(H: torch.Tensor, g: torch.Tensor, stream=None):
    """x = -H^{-1} g by the library's FP64 Cholesky (H is overwritten by its factor)."""
    _need_gpu(H, "H")
    _need_gpu(g, "g")
    if H.dtype != torch.float64 or g.dtype != torch.float64:
        raise TypeError("H and g must be float64")
    m = H.shape[0]
    b = ctypes.c_size_t()
    _check(load().spsvm_newton_solve_workspace_bytes(m, ctypes.byref(b)))
    ws = torch.empty(b.value, dtype=torch.uint8, device=H.device)
    x = torch.empty(m, dtype=torch.float64, device=H.device)
    _check(load().spsvm_newton_solve(ctypes.c_void_p(H.data_ptr()), H.stride(0), m, ctypes.c_void_p(g.data_ptr()),
                                     ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(ws.data_ptr()), b.value,
                                     ctypes.c_void_p(_stream_ptr(stream))))
    return x


def score_candidates(o: torch.Tensor, y: torch.Tensor, Kc: torch.Tensor, oc, C: float, stream=None):
    """Greedy-selection scores of ncand candidates (spsvm_score_candidates). Kc: ncand x n (row c is candidate c's
    kernel column, row stride >= n), float32 or float64; oc: o at the candidate rows. Returns a dict of numpy
    arrays s, score, status, passes and the winning candidate (-1 if none)."""
    import numpy as np

    for t, name in ((o, "o"), (y, "y"), (Kc, "Kc")):
        _need_gpu(t, name)
    if o.dtype != torch.float64 or y.dtype != torch.float32 or Kc.dim() != 2 or Kc.stride(1) != 1:
        raise TypeError("o must be float64, y float32 and Kc a 2-D tensor with contiguous rows")
    ncand, n = Kc.shape
    och = np.ascontiguousarray(np.asarray(oc, dtype=np.float64).reshape(ncand))
    b = ctypes.c_size_t()
    _check(load().spsvm_score_workspace_bytes(n, ctypes.byref(b)))
    ws = torch.empty(b.value, dtype=torch.uint8, device=o.device)
    s_out = np.zeros(ncand)
    sc_out = np.zeros(ncand)
    st_out = np.zeros(ncand, dtype=np.int32)
    ps_out = np.zeros(ncand, dtype=np.int32)
    win = ctypes.c_int32(-2)
    P, D, I32 = ctypes.POINTER, ctypes.c_double, ctypes.c_int32
    _check(load().spsvm_score_candidates(ctypes.c_void_p(o.data_ptr()), ctypes.c_void_p(y.data_ptr()), n,
                                         ctypes.c_void_p(Kc.data_ptr()), _dtype_code(Kc), Kc.stride(0),
                                         och.ctypes.data_as(P(D)), ncand, float(C), s_out.ctypes.data_as(P(D)),
                                         sc_out.ctypes.data_as(P(D)), st_out.ctypes.data_as(P(I32)),
                                         ps_out.ctypes.data_as(P(I32)), ctypes.byref(win),
                                         ctypes.c_void_p(ws.data_ptr()), b.value, ctypes.c_void_p(_stream_ptr(stream))))
    return {"s": s_out, "score": sc_out, "status": st_out, "passes": ps_out, "winner": int(win.value)}


def newton_solve_noalloc(H: torch.Tensor, g: torch.Tensor, stream=None):
    """newton_solve without a workspace (spsvm_newton_solve_noalloc; m <= 4096, scratch in a static device array)."""
    _need_gpu(H, "H")
    _need_gpu(g, "g")
    if H.dtype != torch.float64 or g.dtype != torch.float64:
        raise TypeError("H and g must be float64")
    m = H.shape[0]
    x = torch.empty(m, dtype=torch.float64, device=H.device)
    _check(load().spsvm_newton_solve_noalloc(ctypes.c_void_p(H.data_ptr()), H.stride(0), m,
                                             ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(x.data_ptr()),
                                             ctypes.c_void_p(_stream_ptr(stream))))
    return x


def candidate_draw(seed: int, t: int, n: int, kappa: int = 59):
    """Host-side candidate rows of addition step t with nothing blocked (spsvm_candidate_draw)."""
    out = (ctypes.c_int32 * 64)()
    _check(load().spsvm_candidate_draw(seed, t, n, kappa, out))
    return [v for v in out if v >= 0]


def _csr_parts(indptr, indices, values):
    for t, name in ((indptr, "indptr"), (indices, "indices"), (values, "values")):
        _need_gpu(t, name)
    if indptr.dtype != torch.int64 or indices.dtype != torch.int32 or values.dtype != torch.float32:
        raise TypeError("CSR arrays: indptr int64, indices int32, values float32")
    return ctypes.c_void_p(indptr.data_ptr()), ctypes.c_void_p(indices.data_ptr()), ctypes.c_void_p(values.data_ptr())


def train_csr(indptr: torch.Tensor, indices: torch.Tensor, values: torch.Tensor, d: int, y: torch.Tensor, C: float,
              gamma: float, J_max: int, workspace=None, stream=None, **opts) -> Model:
    """Greedy SP-SVM training on CSR rows (spsvm_train_csr; FP32)."""
    _need_gpu(y, "y")
    if y.dtype != torch.float32:
        raise TypeError("y must be float32")
    n = indptr.numel() - 1
    o = options(**opts)
    b = ctypes.c_size_t()
    _check(load().spsvm_train_csr_workspace_bytes(n, d, J_max, ctypes.byref(o), ctypes.byref(b)))
    ws, nbytes = _workspace(b.value, y.device, workspace)
    out = ctypes.c_void_p()
    ip, ix, vv = _csr_parts(indptr, indices, values)
    _check(load().spsvm_train_csr(ip, ix, vv, n, d, ctypes.c_void_p(y.data_ptr()), float(C), float(gamma), int(J_max),
                                  ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()), nbytes,
                                  ctypes.c_void_p(_stream_ptr(stream)), ctypes.byref(out)))
    return Model(out.value)


def predict_csr(model: Model, indptr: torch.Tensor, indices: torch.Tensor, values: torch.Tensor, stream=None):
    """Decision values (float64, on the GPU) of CSR rows (spsvm_predict_csr)."""
    n_t = indptr.numel() - 1
    out = torch.empty(n_t, dtype=torch.float64, device=indptr.device)
    if n_t == 0:
        return out
    ip, ix, vv = _csr_parts(indptr, indices, values)
    _check(load().spsvm_predict_csr(model._ptr, ip, ix, vv, n_t, ctypes.c_void_p(out.data_ptr()),
                                    ctypes.c_void_p(_stream_ptr(stream))))
    return out


def train_ovo(X: torch.Tensor, classes: torch.Tensor, K: int, C: float, gamma: float, J_max: int, workspace=None,
              stream=None, **opts):
    """One-vs-one multiclass training (spsvm_train_ovo): K (K - 1) / 2 models, pairs (0, 1), (0, 2), ..."""
    _need_gpu(X, "X")
    _need_gpu(classes, "classes")
    if classes.dtype != torch.int32 or classes.numel() != X.shape[0]:
        raise TypeError("classes must be an int32 tensor with one entry per row of X")
    n, d = X.shape
    counts = torch.bincount(classes.long(), minlength=K).cpu().tolist()
    pair_rows = max(counts[a] + counts[b] for a in range(K) for b in range(a + 1, K))
    o = options(**opts)
    b = ctypes.c_size_t()
    _check(load().spsvm_ovo_workspace_bytes(pair_rows, d, J_max, _dtype_code(X), ctypes.byref(o), ctypes.byref(b)))
    ws, nbytes = _workspace(b.value, X.device, workspace)
    P = K * (K - 1) // 2
    outs = (ctypes.c_void_p * P)()
    _check(load().spsvm_train_ovo(ctypes.c_void_p(X.data_ptr()), _dtype_code(X), ctypes.c_void_p(classes.data_ptr()),
                                  n, d, K, float(C), float(gamma), int(J_max), ctypes.byref(o),
                                  ctypes.c_void_p(ws.data_ptr()), nbytes, ctypes.c_void_p(_stream_ptr(stream)), outs))
    return [Model(outs[p]) for p in range(P)]


def predict_ovo(models, K: int, Xt: torch.Tensor, stream=None) -> torch.Tensor:
    """Classes (int32, on the GPU) of the rows of Xt by one-vs-one voting (spsvm_predict_ovo)."""
    _need_gpu(Xt, "Xt")
    n_t = Xt.shape[0]
    out = torch.empty(n_t, dtype=torch.int32, device=Xt.device)
    if n_t == 0:
        return out
    b = ctypes.c_size_t()
    _check(load().spsvm_predict_ovo_workspace_bytes(n_t, K, ctypes.byref(b)))
    ws = torch.empty(b.value, dtype=torch.uint8, device=Xt.device)
    arr = (ctypes.c_void_p * len(models))(*[m._ptr.value for m in models])
    _check(load().spsvm_predict_ovo(arr, K, ctypes.c_void_p(Xt.data_ptr()), _dtype_code(Xt), n_t,
                                    ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()), b.value,
                                    ctypes.c_void_p(_stream_ptr(stream))))
    return out


def train_shared(X: torch.Tensor, Y: torch.Tensor, C, gamma, J_max: int, workspace=None, stream=None, **opts):
    """Greedy growth of one basis shared by P problems (labels Y[p], C[p], gamma[p]); returns P models on it."""
    import numpy as np

    _need_gpu(X, "X")
    _need_gpu(Y, "Y")
    if Y.dtype != torch.float32 or Y.dim() != 2 or Y.shape[1] != X.shape[0]:
        raise TypeError("Y must be a P x n float32 tensor")
    n, d = X.shape
    P = Y.shape[0]
    Ch = np.ascontiguousarray(np.asarray(C, dtype=np.float64).reshape(P))
    gh = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64).reshape(P))
    o = options(**opts)
    nb = ctypes.c_size_t()
    gp = gh.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    _check(load().spsvm_train_shared_workspace_bytes(n, d, P, gp, int(J_max), _dtype_code(X), ctypes.byref(o),
                                                     ctypes.byref(nb)))
    ws, nbytes = _workspace(nb.value, X.device, workspace)
    outs = (ctypes.c_void_p * P)()
    _check(load().spsvm_train_shared(ctypes.c_void_p(X.data_ptr()), _dtype_code(X), n, d, P,
                                     ctypes.c_void_p(Y.data_ptr()), Ch.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     gp, int(J_max), ctypes.byref(o), ctypes.c_void_p(ws.data_ptr()), nbytes,
                                     ctypes.c_void_p(_stream_ptr(stream)), outs))
    return [Model(outs[p]) for p in range(P)]


def train_batch(X: torch.Tensor, Y: torch.Tensor, C, gamma, J: Sequence[int], workspace=None, stream=None,
                **opts):
    """P Newton re-optimisations sharing X and the basis J: problem p has labels Y[p], C[p], gamma[p]."""
    import numpy as np

    _need_gpu(X, "X")
    _need_gpu(Y, "Y")
    if Y.dtype != torch.float32 or Y.dim() != 2 or Y.shape[1] != X.shape[0]:
        raise TypeError("Y must be a P x n float32 tensor")
    n, d = X.shape
    P = Y.shape[0]
    Ch = np.ascontiguousarray(np.asarray(C, dtype=np.float64).reshape(P))
    gh = np.ascontiguousarray(np.asarray(gamma, dtype=np.float64).reshape(P))
    Jh = np.ascontiguousarray(np.asarray(J, dtype=np.int64))
    o = options(**opts)
    ws, nbytes = _workspace(workspace_bytes(n, d, Jh.size, batch=True, problems=P, dtype=X.dtype, **opts), X.device, workspace)
    outs = (ctypes.c_void_p * P)()
    _check(load().spsvm_train_batch(ctypes.c_void_p(X.data_ptr()), _dtype_code(X), n, d, P,
                                    ctypes.c_void_p(Y.data_ptr()), Ch.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    gh.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    Jh.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), Jh.size, ctypes.byref(o),
                                    ctypes.c_void_p(ws.data_ptr()), nbytes, ctypes.c_void_p(_stream_ptr(stream)), outs))
    return [Model(outs[p]) for p in range(P)]
