"""Python binding of libemu (include/emu.h): FP64 GEMM emulated with INT8
slices on MI355X, and the LU solver that uses it for its Schur update.

Two layers:

* the raw C-ABI functions under their C names (``emu_dgemm``, ``emu_dgetrf``,
  ``emu_dgetrs``, ...), which take integer device addresses and sizes and
  return the library's status code;
* thin torch conveniences (``dgemm``, ``dgetrf``, ``dgetrs``, ...), which only
  marshal arguments: a matrix is a float64 CUDA tensor of shape (rows, cols)
  with stride (1, ld) (column-major; ``colmajor`` builds one), and the call
  runs on torch's current stream.

Every computation runs in the HIP library.  There is no fallback: if
libemu.so is missing or does not load, every call raises ``EmuError``.
"""
from __future__ import annotations

import ctypes
import os

__all__ = [
    "EmuError", "lib", "library_path", "EMU_MAX_SLICES", "EMU_MAX_NB",
    "emu_version", "emu_init", "emu_finalize", "emu_set_stream", "emu_last_error",
    "emu_set_workspace", "emu_workspace_bytes", "emu_getrf_workspace_bytes",
    "emu_getrs_workspace_bytes", "set_workspace", "EMU_INFO_ABORTED", "EMU_ERR_PANEL_WAIT",
    "EMU_STATUS_NONFINITE", "EMU_STATUS_PANEL_WAIT", "EMU_STATUS_SOLVE_WAIT",
    "emu_status", "emu_dgemm", "emu_dgemm_t", "emu_dgetrf", "emu_dgetrs",
    "emu_debug_slices", "emu_debug_products", "emu_profile_start",
    "emu_profile_stop", "emu_profile_read", "profile_read", "PROF_SLICE", "PROF_GEMM",
    "emu_set_param", "emu_dgesv_ir", "set_param", "dgesv_ir",
    "emu_dgetrf_batched", "emu_dgesv_batched", "emu_autotune_batched",
    "dgetrf_batched", "dgesv_batched", "autotune_batched",
    "emu_mlp_nparam", "emu_features", "emu_mlp_train_step", "emu_mlp_grad", "emu_mlp_infer",
    "emu_tile_labels", "emu_dgetrf_adaptive", "features", "mlp_init", "mlp_train_step",
    "emu_refine", "refine", "emu_scaled_residual", "scaled_residual",
    "mlp_grad", "mlp_infer", "tile_labels", "dgetrf_adaptive",
    "colmajor", "dgemm", "dgetrf", "dgetrs", "debug_slices", "debug_products",
    "status", "emu_dgemm_noalloc", "EMU_NOALLOC_SCRATCH_BYTES",
    "emu_dpotrf", "emu_potrf_workspace_bytes", "dpotrf",
    "emu_dgesv_batched_ir", "dgesv_batched_ir", "emu_dgemm_ab",
    "emu_dgetrs_batched", "dgetrs_batched", "emu_autotune_getrf", "autotune_getrf",
]

EMU_MAX_SLICES = 16
EMU_MAX_NB = 2048
EMU_ERR_WORKSPACE = 1002
EMU_ERR_UNSUPPORTED = 1003
EMU_NOALLOC_SCRATCH_BYTES = 64 << 20
EMU_ERR_NOT_CONVERGED = 1004
EMU_ERR_PANEL_WAIT = 1005
EMU_INFO_ABORTED = -1000
EMU_STATUS_NONFINITE = 1
EMU_STATUS_PANEL_WAIT = 2
EMU_STATUS_SOLVE_WAIT = 4
_HERE = os.path.dirname(os.path.abspath(__file__))
library_path = os.path.join(_HERE, "libemu.so")


class EmuError(RuntimeError):
    pass


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double

_SIGNATURES = {
    "emu_version": ([], _I),
    "emu_init": ([], _I),
    "emu_finalize": ([], _I),
    "emu_set_stream": ([_P], _I),
    "emu_set_workspace": ([_P, ctypes.c_size_t], _I),
    "emu_workspace_bytes": ([_I, _I, _I, _I], ctypes.c_size_t),
    "emu_getrf_workspace_bytes": ([_I, _I, _I, _I], ctypes.c_size_t),
    "emu_getrs_workspace_bytes": ([_I, _I], ctypes.c_size_t),
    "emu_last_error": ([], ctypes.c_char_p),
    "emu_status": ([ctypes.POINTER(_I)], _I),
    "emu_dgemm": ([_I, _I, _I, _D, _P, _I, _P, _I, _D, _P, _I, _I], _I),
    "emu_dgemm_noalloc": ([_I, _I, _I, _D, _P, _I, _P, _I, _D, _P, _I, _I], _I),
    "emu_dgemm_ab": ([_I, _I, _I, _D, _P, _I, _P, _I, _D, _P, _I, _I, _I], _I),
    "emu_dpotrf": ([_I, _P, _I, _P, _I, _I], _I),
    "emu_dgesv_batched_ir": ([_I, _P, _P, _P, _P, _P, _P, _P, _P, _I, _I, _D, _I, _P, _P, _P,
                              _P], _I),
    "emu_potrf_workspace_bytes": ([_I, _I, _I], ctypes.c_size_t),
    "emu_dgemm_t": ([_I, _I, _I, _D, _P, _I, _P, _I, _D, _P, _I, _I, _I], _I),
    "emu_dgetrf": ([_I, _I, _P, _I, _P, _P, _I, _I], _I),
    "emu_dgetrs": ([_I, _I, _P, _I, _P, _P, _I], _I),
    "emu_debug_slices": ([_I, _I, _P, _I, _I, _I, _P, _P, _P], _I),
    "emu_debug_products": ([_I, _I, _I, _P, _I, _P, _I, _I, _I, _P], _I),
    "emu_set_param": ([ctypes.c_char_p, ctypes.c_longlong], _I),
    "emu_dgesv_ir": ([_I, _I, _P, _I, _P, _I, _P, _I, _I, _I, _D, _I,
                      ctypes.POINTER(_I), ctypes.POINTER(_D), ctypes.POINTER(_I),
                      ctypes.POINTER(_I)], _I),
    "emu_dgetrf_batched": ([_I, _P, _P, _P, _P, _P, _I, _I], _I),
    "emu_dgesv_batched": ([_I, _P, _P, _P, _P, _P, _P, _P, _P, _I, _I], _I),
    "emu_dgetrs_batched": ([_I, _P, _P, _P, _P, _P, _P, _P], _I),
    "emu_autotune_getrf": ([_I, _I, _P, _I, _I, _P, _I, ctypes.POINTER(_I),
                            ctypes.POINTER(_D)], _I),
    "emu_autotune_batched": ([_I, _P, _P, _P, _P, _P, _P, _I, ctypes.POINTER(_I),
                              ctypes.POINTER(_I), ctypes.POINTER(_D), ctypes.POINTER(_I)], _I),
    "emu_refine": ([_I, _I, _P, _I, _P, _I, _P, _P, _I, _P, _I, _D, _I, ctypes.POINTER(_I),
                    ctypes.POINTER(_D)], _I),
    "emu_scaled_residual": ([_I, _I, _P, _I, _P, _I, _P, _I, ctypes.POINTER(_D)], _I),
    "emu_mlp_nparam": ([], _I),
    "emu_features": ([_I, _I, _I, _P, _I, _P, _I, _P], _I),
    "emu_mlp_train_step": ([_P, _P, _P, _I, _P, _P, _I, ctypes.c_float, _P], _I),
    "emu_mlp_grad": ([_P, _P, _P, _I, _P], _I),
    "emu_mlp_infer": ([_P, _P, _I, _P, _P, ctypes.c_float], _I),
    "emu_tile_labels": ([_I, _I, _I, _P, _I, _P, _I, _I, _I, _D, _P], _I),
    "emu_dgetrf_adaptive": ([_I, _I, _P, _I, _P, _P, _I, _P, _I, ctypes.c_float, _P,
                             ctypes.c_longlong, _P], _I),
    "emu_profile_start": ([], _I),
    "emu_profile_stop": ([], _I),
    "emu_profile_read": ([_I, ctypes.POINTER(_D), ctypes.POINTER(_I)], _I),
}


def lib() -> ctypes.CDLL:
    """Load libemu.so (raises EmuError when it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(library_path):
            raise EmuError(f"{library_path} is not built; run "
                           "`python -m paper_2509_23565_amd.build`")
        try:
            L = ctypes.CDLL(library_path)
        except OSError as e:  # pragma: no cover - depends on the machine
            raise EmuError(f"cannot load {library_path}: {e}") from e
        for name, (args, res) in _SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _raw(name):
    def call(*args):
        return getattr(lib(), name)(*args)
    call.__name__ = name
    return call


emu_version = _raw("emu_version")
emu_init = _raw("emu_init")
emu_finalize = _raw("emu_finalize")
emu_set_stream = _raw("emu_set_stream")
emu_set_workspace = _raw("emu_set_workspace")
emu_workspace_bytes = _raw("emu_workspace_bytes")
emu_getrf_workspace_bytes = _raw("emu_getrf_workspace_bytes")
emu_getrs_workspace_bytes = _raw("emu_getrs_workspace_bytes")
emu_status = _raw("emu_status")
emu_dgemm = _raw("emu_dgemm")
emu_dgemm_noalloc = _raw("emu_dgemm_noalloc")
emu_dgemm_ab = _raw("emu_dgemm_ab")
emu_dpotrf = _raw("emu_dpotrf")
emu_dgesv_batched_ir = _raw("emu_dgesv_batched_ir")
emu_potrf_workspace_bytes = _raw("emu_potrf_workspace_bytes")
emu_dgemm_t = _raw("emu_dgemm_t")
emu_dgetrf = _raw("emu_dgetrf")
emu_dgetrs = _raw("emu_dgetrs")
emu_debug_slices = _raw("emu_debug_slices")
emu_debug_products = _raw("emu_debug_products")
emu_set_param = _raw("emu_set_param")
emu_dgesv_ir = _raw("emu_dgesv_ir")
emu_dgetrf_batched = _raw("emu_dgetrf_batched")
emu_dgesv_batched = _raw("emu_dgesv_batched")
emu_dgetrs_batched = _raw("emu_dgetrs_batched")
emu_autotune_getrf = _raw("emu_autotune_getrf")
emu_autotune_batched = _raw("emu_autotune_batched")
emu_refine = _raw("emu_refine")
emu_scaled_residual = _raw("emu_scaled_residual")
emu_mlp_nparam = _raw("emu_mlp_nparam")
emu_features = _raw("emu_features")
emu_mlp_train_step = _raw("emu_mlp_train_step")
emu_mlp_grad = _raw("emu_mlp_grad")
emu_mlp_infer = _raw("emu_mlp_infer")
emu_tile_labels = _raw("emu_tile_labels")
emu_dgetrf_adaptive = _raw("emu_dgetrf_adaptive")
emu_profile_start = _raw("emu_profile_start")
emu_profile_stop = _raw("emu_profile_stop")
emu_profile_read = _raw("emu_profile_read")

PROF_SLICE = 0
PROF_GEMM = 1


def profile_read(kind: int):
    """(total milliseconds, launches) of one profiled kernel group."""
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int(0)
    _check(emu_profile_read(int(kind), ctypes.byref(ms), ctypes.byref(cnt)),
           "emu_profile_read")
    return ms.value, cnt.value


def emu_last_error() -> str:
    v = lib().emu_last_error()
    return v.decode() if v else ""


def _check(rc: int, name: str) -> None:
    if rc != 0:
        raise EmuError(f"{name} returned {rc}: {emu_last_error()}")


# ------------------------------------------------------------------ torch
def _torch():
    import torch
    return torch


def _bind_stream() -> None:
    torch = _torch()
    _check(emu_set_stream(ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)),
           "emu_set_stream")


def colmajor(x, device="cuda"):
    """float64 column-major device tensor (shape (rows, cols), stride (1, rows))
    from a NumPy array or tensor."""
    torch = _torch()
    t = torch.as_tensor(x, dtype=torch.float64)
    if t.dim() == 1:
        t = t[:, None]
    out = torch.empty((t.shape[1], t.shape[0]), dtype=torch.float64, device=device).t()
    out.copy_(t)
    return out


def _mat(t, name):
    torch = _torch()
    if t.dtype != torch.float64 or not t.is_cuda or t.dim() != 2:
        raise EmuError(f"{name}: expected a 2-D float64 CUDA tensor")
    rows, cols = t.shape
    if cols > 1 and rows > 0 and t.stride(0) != 1:
        raise EmuError(f"{name}: must be column-major (stride(0) == 1)")
    ld = t.stride(1) if cols > 1 else max(rows, 1)
    return t.data_ptr(), max(ld, 1)


def dgemm(A, B, C=None, alpha=1.0, beta=0.0, nslices=7, t=None, nslices_b=None):
    """C <- alpha * emul(A @ B) + beta * C (column-major float64 tensors).
    nslices_b: B's own slice count (unequal splits, emu_dgemm_ab)."""
    torch = _torch()
    m, k = A.shape
    k2, n = B.shape
    if k != k2:
        raise EmuError("dgemm: inner dimensions differ")
    if C is None:
        C = torch.empty((n, m), dtype=torch.float64, device=A.device).t()
        if beta != 0.0:
            raise EmuError("dgemm: beta != 0 needs C")
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    pc, ldc = _mat(C, "C")
    _bind_stream()
    if nslices_b is not None:
        if t is not None:
            raise EmuError("dgemm: nslices_b takes t = nslices + 1")
        rc = emu_dgemm_ab(m, n, k, float(alpha), pa, lda, pb, ldb, float(beta), pc, ldc,
                          int(nslices), int(nslices_b))
    elif t is None:
        rc = emu_dgemm(m, n, k, float(alpha), pa, lda, pb, ldb, float(beta), pc, ldc,
                       int(nslices))
    else:
        rc = emu_dgemm_t(m, n, k, float(alpha), pa, lda, pb, ldb, float(beta), pc, ldc,
                         int(nslices), int(t))
    _check(rc, "emu_dgemm")
    return C


def dgetrf(A, nb=64, nslices=7):
    """In-place LU of A; returns (ipiv, info) as int32 device tensors."""
    torch = _torch()
    m, n = A.shape
    pa, lda = _mat(A, "A")
    ipiv = torch.zeros(max(min(m, n), 1), dtype=torch.int32, device=A.device)
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    _bind_stream()
    _check(emu_dgetrf(m, n, pa, lda, ipiv.data_ptr(), info.data_ptr(), int(nb),
                      int(nslices)), "emu_dgetrf")
    return ipiv[:min(m, n)], info


def dpotrf(A, nb=64, nslices=7):
    """In-place lower Cholesky of A (upper part untouched); returns info as an
    int32 device tensor."""
    torch = _torch()
    n = A.shape[0]
    if A.shape[1] != n:
        raise EmuError("dpotrf: A must be square")
    pa, lda = _mat(A, "A")
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    _bind_stream()
    _check(emu_dpotrf(n, pa, lda, info.data_ptr(), int(nb), int(nslices)), "emu_dpotrf")
    return info


def dgetrs(LU, ipiv, B):
    """Solve in place: B <- A^-1 B from dgetrf's factors."""
    n = LU.shape[0]
    nrhs = B.shape[1]
    pl, lda = _mat(LU, "LU")
    pb, ldb = _mat(B, "B")
    _bind_stream()
    _check(emu_dgetrs(n, nrhs, pl, lda, ipiv.data_ptr(), pb, ldb), "emu_dgetrs")
    return B


def set_workspace(buf=None) -> None:
    """Register a caller-owned device buffer (any CUDA tensor; its bytes) as
    the calling thread's scratch, or go back to library-owned scratch with
    None.  The caller keeps the tensor alive while it is registered."""
    if buf is None:
        _check(emu_set_workspace(None, 0), "emu_set_workspace")
    else:
        nbytes = buf.numel() * buf.element_size()
        _check(emu_set_workspace(ctypes.c_void_p(buf.data_ptr()), nbytes), "emu_set_workspace")


def set_param(key: str, value: int) -> None:
    _check(emu_set_param(key.encode(), int(value)), "emu_set_param")


def dgesv_ir(A, B, X=None, nb=64, nslices=3, tol=1e-15, maxiter=10):
    """Precision-form solve; returns (X, dict(iters, berr, s_final, info, rc)).

    rc is 0 on convergence or EMU_ERR_NOT_CONVERGED (1004); other codes raise.
    """
    torch = _torch()
    n = A.shape[0]
    nrhs = B.shape[1]
    if X is None:
        X = torch.empty((nrhs, n), dtype=torch.float64, device=A.device).t()
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    px, ldx = _mat(X, "X")
    it = ctypes.c_int(0)
    be = ctypes.c_double(0.0)
    sf = ctypes.c_int(0)
    inf = ctypes.c_int(0)
    _bind_stream()
    rc = emu_dgesv_ir(n, nrhs, pa, lda, pb, ldb, px, ldx, int(nb), int(nslices),
                      float(tol), int(maxiter), ctypes.byref(it), ctypes.byref(be),
                      ctypes.byref(sf), ctypes.byref(inf))
    if rc not in (0, 1004):
        _check(rc, "emu_dgesv_ir")
    return X, dict(iters=it.value, berr=be.value, s_final=sf.value, info=inf.value, rc=rc)


class _Batch:
    """Host arrays (sizes, device pointers) of a list of column-major tensors
    (the checks of _mat, in one pass over the list: a batch holds thousands)."""

    def __init__(self, mats, name):
        f64 = _torch().float64
        ptrs, lds = [], []
        for i, t in enumerate(mats):
            if t.dtype is not f64 or not t.is_cuda or t.dim() != 2:
                raise EmuError(f"{name}[{i}]: expected a 2-D float64 CUDA tensor")
            rows, cols = t.shape
            s0, s1 = t.stride()
            if cols > 1 and rows > 0 and s0 != 1:
                raise EmuError(f"{name}[{i}]: must be column-major (stride(0) == 1)")
            ptrs.append(t.data_ptr())
            ld = s1 if cols > 1 else rows
            lds.append(ld if ld > 1 else 1)
        n = len(mats)
        self.ptr = (ctypes.c_void_p * n)(*ptrs)
        self.ld = (ctypes.c_int * n)(*lds)


def _pivot_views(torch, sizes, dev):
    """One int32 allocation for all pivot vectors of a batch, as views."""
    flat = torch.zeros(sum(sizes), dtype=torch.int32, device=dev)
    return list(torch.split(flat, sizes))


def dgesv_batched(As, Bs, nb=32, nslices=5):
    """Factor and solve a batch in place (A_i -> LU_i, B_i -> X_i).

    Returns (ipivs, info) with info an int32 device tensor of length count.
    nb = 0 uses the autotuned block size for this batch shape.
    """
    torch = _torch()
    count = len(As)
    dev = As[0].device
    sizes = [int(a.shape[0]) for a in As]
    n = (ctypes.c_int * count)(*sizes)
    nrhs = (ctypes.c_int * count)(*[int(b.shape[1]) for b in Bs])
    ipivs = _pivot_views(torch, sizes, dev)
    pp = (ctypes.c_void_p * count)(*[p.data_ptr() for p in ipivs])
    info = torch.zeros(count, dtype=torch.int32, device=dev)
    a = _Batch(As, "A")
    b = _Batch(Bs, "B")
    _bind_stream()
    _check(emu_dgesv_batched(count, n, nrhs, a.ptr, a.ld, pp, info.data_ptr(), b.ptr, b.ld,
                             int(nb), int(nslices)), "emu_dgesv_batched")
    return ipivs, info


def dgesv_batched_ir(As, Bs, Xs=None, nb=32, nslices=3, tol=1e-15, maxiter=10):
    """Batched precision form: As, Bs untouched, Xs (allocated when None)
    receive the solutions.  Returns (Xs, dict(rc, iters, berr, s_final, info)
    with per-system lists); rc is 0 or EMU_ERR_NOT_CONVERGED (1004)."""
    torch = _torch()
    count = len(As)
    if Xs is None:
        # one allocation, a column-major view per system
        shapes = [(int(b.shape[0]), int(b.shape[1])) for b in Bs]
        offs, tot = [], 0
        for r, c in shapes:
            offs.append(tot)
            tot += r * c
        Xs = []
        if shapes:
            flat = torch.empty(max(tot, 1), dtype=torch.float64, device=Bs[0].device)
            Xs = [torch.as_strided(flat, (r, c), (1, max(r, 1)), o)
                  for (r, c), o in zip(shapes, offs)]
    n = (ctypes.c_int * count)(*[int(a.shape[0]) for a in As])
    nrhs = (ctypes.c_int * count)(*[int(b.shape[1]) for b in Bs])
    a = _Batch(As, "A")
    b = _Batch(Bs, "B")
    x = _Batch(Xs, "X")
    iters = (ctypes.c_int * count)()
    berr = (ctypes.c_double * count)()
    sfin = (ctypes.c_int * count)()
    info = (ctypes.c_int * count)()
    _bind_stream()
    rc = emu_dgesv_batched_ir(count, n, nrhs, a.ptr, a.ld, b.ptr, b.ld, x.ptr, x.ld, int(nb),
                              int(nslices), float(tol), int(maxiter), iters, berr, sfin, info)
    if rc not in (0, EMU_ERR_NOT_CONVERGED):
        _check(rc, "emu_dgesv_batched_ir")
    return Xs, {"rc": rc, "iters": list(iters), "berr": list(berr), "s_final": list(sfin),
                "info": list(info)}


def dgetrf_batched(As, nb=32, nslices=5):
    """Factor a batch in place; returns (ipivs, info)."""
    torch = _torch()
    count = len(As)
    dev = As[0].device
    sizes = [int(a.shape[0]) for a in As]
    n = (ctypes.c_int * count)(*sizes)
    ipivs = _pivot_views(torch, sizes, dev)
    pp = (ctypes.c_void_p * count)(*[p.data_ptr() for p in ipivs])
    info = torch.zeros(count, dtype=torch.int32, device=dev)
    a = _Batch(As, "A")
    _bind_stream()
    _check(emu_dgetrf_batched(count, n, a.ptr, a.ld, pp, info.data_ptr(), int(nb),
                              int(nslices)), "emu_dgetrf_batched")
    return ipivs, info


def autotune_getrf(A, nslices=3, nbs=None):
    """Time the LU of a copy of A over candidate block sizes (nbs None: 256,
    512, 768, 1024 up to min(m, n)) and record the fastest for nb = 0 calls
    of this shape; returns (nb, ms)."""
    m, n = A.shape
    pa, lda = _mat(A, "A")
    cand = list(nbs) if nbs else []
    arr = (ctypes.c_int * max(len(cand), 1))(*cand) if cand else None
    nb = ctypes.c_int(0)
    ms = ctypes.c_double(0.0)
    _bind_stream()
    _check(emu_autotune_getrf(m, n, pa, lda, int(nslices), arr, len(cand), ctypes.byref(nb),
                              ctypes.byref(ms)), "emu_autotune_getrf")
    return nb.value, ms.value


def dgetrs_batched(LUs, ipivs, Bs):
    """Solve every system of a batch in place (B_i -> X_i) from the factors
    and pivots of dgetrf_batched."""
    count = len(LUs)
    n = (ctypes.c_int * count)(*[int(a.shape[0]) for a in LUs])
    nrhs = (ctypes.c_int * count)(*[int(b.shape[1]) for b in Bs])
    pp = (ctypes.c_void_p * count)(*[p.data_ptr() for p in ipivs])
    a = _Batch(LUs, "LU")
    b = _Batch(Bs, "B")
    _bind_stream()
    _check(emu_dgetrs_batched(count, n, nrhs, a.ptr, a.ld, pp, b.ptr, b.ld),
           "emu_dgetrs_batched")
    return Bs


def autotune_batched(As, Bs, nslices=5, with_tile=False):
    """Tune (nb, grid multiplier, grouped-GEMM tile) for this batch shape;
    returns (nb, mult, ms), and the tile (0: 64 x 128, 1: 64 x 64) last
    when with_tile."""
    count = len(As)
    n = (ctypes.c_int * count)(*[int(a.shape[0]) for a in As])
    nrhs = (ctypes.c_int * count)(*[int(b.shape[1]) for b in Bs])
    a = _Batch(As, "A")
    b = _Batch(Bs, "B")
    bnb, bm, bms = ctypes.c_int(0), ctypes.c_int(0), ctypes.c_double(0.0)
    bt = ctypes.c_int(0)
    _bind_stream()
    _check(emu_autotune_batched(count, n, nrhs, a.ptr, a.ld, b.ptr, b.ld, int(nslices),
                                ctypes.byref(bnb), ctypes.byref(bm), ctypes.byref(bms),
                                ctypes.byref(bt)),
           "emu_autotune_batched")
    if with_tile:
        return bnb.value, bm.value, bms.value, bt.value
    return bnb.value, bm.value, bms.value


def refine(A, LU, ipiv, B, X, tol=1e-15, maxiter=10):
    """Refine X in place with existing factors; returns (rc, iters, berr)."""
    n = A.shape[0]
    nrhs = B.shape[1]
    pa, lda = _mat(A, "A")
    pl, ldl = _mat(LU, "LU")
    pb, ldb = _mat(B, "B")
    px, ldx = _mat(X, "X")
    it = ctypes.c_int(0)
    be = ctypes.c_double(0.0)
    _bind_stream()
    rc = emu_refine(n, nrhs, pa, lda, pl, ldl, ipiv.data_ptr(), pb, ldb, px, ldx, float(tol),
                    int(maxiter), ctypes.byref(it), ctypes.byref(be))
    if rc not in (0, 1004):
        _check(rc, "emu_refine")
    return rc, it.value, be.value


def scaled_residual(A, X, B):
    """Eqn (9) scaled residual of X for A X = B, in FP64 on the GPU (host float)."""
    n = A.shape[0]
    nrhs = B.shape[1]
    pa, lda = _mat(A, "A")
    px, ldx = _mat(X, "X")
    pb, ldb = _mat(B, "B")
    out = ctypes.c_double(0.0)
    _bind_stream()
    _check(emu_scaled_residual(n, nrhs, pa, lda, px, ldx, pb, ldb, ctypes.byref(out)),
           "emu_scaled_residual")
    return out.value


# --------------------------------------------------------------- learned
def _tiles(m, n):
    return ((m + 255) // 256) * ((n + 255) // 256)


def features(L21, U12):
    """float32 device tensor [tiles][16] of the update L21 @ U12."""
    torch = _torch()
    m, k = L21.shape
    n = U12.shape[1]
    pl, ldl = _mat(L21, "L21")
    pu, ldu = _mat(U12, "U12")
    f = torch.zeros((max(_tiles(m, n), 1), 16), dtype=torch.float32, device=L21.device)
    _bind_stream()
    _check(emu_features(m, n, k, pl, ldl, pu, ldu, f.data_ptr()), "emu_features")
    return f[:_tiles(m, n)]


def mlp_init(seed=0, device="cuda"):
    """Xavier-uniform weights, zero biases (float32 device tensor)."""
    import numpy as np
    torch = _torch()
    g = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((64, 16), (64, 64), (7, 64)):
        lim = (6.0 / (fan_in + fan_out)) ** 0.5
        parts.append(g.uniform(-lim, lim, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    p = np.concatenate(parts).astype(np.float32)
    assert p.size == emu_mlp_nparam()
    return torch.as_tensor(p, device=device)


def mlp_train_step(params, X, labels, m, v, step, lr=1e-3, loss=None):
    _bind_stream()
    _check(emu_mlp_train_step(params.data_ptr(), X.data_ptr(), labels.data_ptr(),
                              int(X.shape[0]), m.data_ptr(), v.data_ptr(), int(step),
                              float(lr), loss.data_ptr() if loss is not None else None),
           "emu_mlp_train_step")


def mlp_grad(params, X, labels):
    torch = _torch()
    g = torch.zeros_like(params)
    _bind_stream()
    _check(emu_mlp_grad(params.data_ptr(), X.data_ptr(), labels.data_ptr(), int(X.shape[0]),
                        g.data_ptr()), "emu_mlp_grad")
    return g


def mlp_infer(params, X, conf=0.95):
    torch = _torch()
    B = int(X.shape[0])
    prob = torch.zeros((max(B, 1), 7), dtype=torch.float32, device=X.device)
    s = torch.zeros(max(B, 1), dtype=torch.int32, device=X.device)
    _bind_stream()
    _check(emu_mlp_infer(params.data_ptr(), X.data_ptr(), B, prob.data_ptr(), s.data_ptr(),
                         float(conf)), "emu_mlp_infer")
    return prob[:B], s[:B]


def tile_labels(L21, U12, s_lo=3, s_hi=9, tau=2.0 ** -40):
    torch = _torch()
    m, k = L21.shape
    n = U12.shape[1]
    pl, ldl = _mat(L21, "L21")
    pu, ldu = _mat(U12, "U12")
    lab = torch.zeros(_tiles(m, n), dtype=torch.int32, device=L21.device)
    _bind_stream()
    _check(emu_tile_labels(m, n, k, pl, ldl, pu, ldu, int(s_lo), int(s_hi), float(tau),
                           lab.data_ptr()), "emu_tile_labels")
    return lab


def dgetrf_adaptive(A, params, nb=256, s_full=9, conf=0.95, smaps_cap=1 << 20):
    """In-place LU with per-tile slice counts; returns (ipiv, info, smaps, products)."""
    torch = _torch()
    m, n = A.shape
    pa, lda = _mat(A, "A")
    ipiv = torch.zeros(max(min(m, n), 1), dtype=torch.int32, device=A.device)
    info = torch.zeros(1, dtype=torch.int32, device=A.device)
    smaps = (ctypes.c_int * smaps_cap)()
    prods = (ctypes.c_longlong * 3)()
    _bind_stream()
    _check(emu_dgetrf_adaptive(m, n, pa, lda, ipiv.data_ptr(), info.data_ptr(), int(nb),
                               params.data_ptr(), int(s_full), float(conf), smaps,
                               smaps_cap, prods), "emu_dgetrf_adaptive")
    used, full, ntiles = prods[0], prods[1], prods[2]
    return ipiv[:min(m, n)], info, list(smaps[:min(ntiles, smaps_cap)]), (used, full)


def debug_slices(X, by_rows, nslices):
    """(exps, nonfinite, digits) of one operand; digits has shape
    (nslices, rows, cols) in the operand's own column-major layout."""
    torch = _torch()
    rows, cols = X.shape
    px, ldx = _mat(X, "X")
    lines = rows if by_rows else cols
    exps = torch.zeros(max(lines, 1), dtype=torch.int32, device=X.device)
    bad = torch.zeros(max(lines, 1), dtype=torch.int32, device=X.device)
    dig = torch.zeros((nslices, cols, rows), dtype=torch.int8, device=X.device)
    _bind_stream()
    _check(emu_debug_slices(rows, cols, px, ldx, 1 if by_rows else 0, int(nslices),
                            exps.data_ptr(), bad.data_ptr(), dig.data_ptr()),
           "emu_debug_slices")
    return exps[:lines], bad[:lines], dig.transpose(1, 2)


def debug_products(A, B, nslices, t=None):
    """D_g for g = 2..t as an int64 tensor of shape (t-1, m, n)."""
    torch = _torch()
    m, k = A.shape
    n = B.shape[1]
    t = nslices + 1 if t is None else t
    pa, lda = _mat(A, "A")
    pb, ldb = _mat(B, "B")
    D = torch.zeros((t - 1, n, m), dtype=torch.int64, device=A.device)
    _bind_stream()
    _check(emu_debug_products(m, n, k, pa, lda, pb, ldb, int(nslices), int(t),
                              D.data_ptr()), "emu_debug_products")
    return D.transpose(1, 2)


def status() -> int:
    """Synchronize and return (then clear) the EMU_STATUS_* bits."""
    v = ctypes.c_int(0)
    _bind_stream()
    _check(emu_status(ctypes.byref(v)), "emu_status")
    return v.value
