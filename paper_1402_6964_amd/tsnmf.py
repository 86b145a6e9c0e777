"""Python binding of libtsnmf (ctypes; argument marshalling only).

The functions named like the C entry points (``tsnmf_tsqr_r`` ...) take
torch tensors or raw device addresses and forward them unchanged; every step of
the computation runs in the HIP library.  The convenience wrappers below them
(``tsqr_r`` ...) only allocate outputs with torch and pick flags.

Importing this module loads the in-tree ``libtsnmf.so``; it raises if the
library is missing, so there is no silent fallback.
"""

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtsnmf.so")
if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing; build it with `python -m paper_1402_6964_amd.build`")
_lib = ctypes.CDLL(LIB_PATH)

# ---- flags (mirror include/tsnmf.h) ---------------------------------------------
F64 = 0x1
F32 = 0x2
BF16 = 0x4
ROW_MAJOR = 0x00
COL_MAJOR = 0x10
LEAF_F64 = 0x20
GP_MFMA_BF16 = 0x100
GP_SIMD_F32 = 0x200
MAX_N = 256
MAX_BATCH_N = 128
MAX_BATCH = 4096

_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64


class BatchConfig(ctypes.Structure):
    _fields_ = [("slab_shift", _i32 * 4), ("reserved", _i32 * 4)]


def batch_config(shifts):
    """BatchConfig from four per-class slab shifts (16, 32, <= 64, <= 128)."""
    c = BatchConfig()
    for i, v in enumerate(shifts):
        c.slab_shift[i] = int(v)
    return c


class TsqrConfig(ctypes.Structure):
    _fields_ = [("leaf_rows", _i64), ("tree_arity", _i32), ("rows_per_lane", _i32), ("wy_panel", _i32),
                ("reserved", _i32)]


class _Entry:
    """A C entry point, resolved in the library on its first call (a symbol the
    library lacks raises AttributeError there, naming the function)."""

    def __init__(self, name, res, args):
        self.name, self.res, self.args, self.f = name, res, args, None

    def __call__(self, *a):
        if self.f is None:
            f = getattr(_lib, self.name)
            f.restype = self.res
            f.argtypes = self.args
            self.f = f
        return self.f(*a)


def _sig(name, res, args):
    return _Entry(name, res, args)


_tsqr_r = _sig("tsnmf_tsqr_r", ctypes.c_int, [_vp, _i64, _i64, _i64, _u32, _vp, _vp, _vp])
_tsqr_r_noalloc = _sig("tsnmf_tsqr_r_noalloc", ctypes.c_int, [_vp, _i64, _i64, _i64, _u32, _vp, _vp, _vp])
_tsqr_r_ex = _sig("tsnmf_tsqr_r_ex", ctypes.c_int,
                  [_vp, _i64, _i64, _i64, _u32, _vp, _vp, ctypes.POINTER(TsqrConfig), _vp])
_tsqr_r_kron = _sig("tsnmf_tsqr_r_kron", ctypes.c_int, [_vp, _i64, _i32, _i64, _vp, _vp, _vp])
_tsqr_batched = _sig("tsnmf_tsqr_r_batched", ctypes.c_int, [_i32, _vp, _vp, _vp, _vp, _u32, _vp, _vp, _vp])
_tsqr_batched_ex = _sig("tsnmf_tsqr_r_batched_ex", ctypes.c_int,
                        [_i32, _vp, _vp, _vp, _vp, _u32, _vp, _vp, ctypes.POINTER(BatchConfig), _vp])
_reserve_batched = _sig("tsnmf_reserve_batched", ctypes.c_int, [_i32, _i64])
_gauss_proj = _sig("tsnmf_gauss_proj", ctypes.c_int,
                   [_vp, _i64, _i64, _i64, _u32, _i32, _u64, _i64, _vp, _vp, _vp])
_gauss_colsum = _sig("tsnmf_gauss_colsum", ctypes.c_int, [_i64, _i32, _u64, _i64, _vp, _vp])
_select_spa = _sig("tsnmf_select_spa", ctypes.c_int, [_vp, _i32, _i32, _i32, _vp, _i32, _vp, _vp, _vp, _vp])
_select_xray = _sig("tsnmf_select_xray", ctypes.c_int, [_vp, _i32, _i32, _i32, _i32, _vp, _vp, _vp])
_select_gp = _sig("tsnmf_select_gp", ctypes.c_int, [_vp, _i32, _i32, _i32, _vp, _i32, _vp, _vp, _vp, _vp])
_nnls = _sig("tsnmf_nnls", ctypes.c_int, [_vp, _i32, _i32, _i32, _vp, _i32, _vp, _i32, _vp, _vp, _vp])
_residual = _sig("tsnmf_residual", ctypes.c_int, [_vp, _i32, _i32, _i32, _vp, _i32, _vp, _i32, _vp, _vp])
_rsvd = _sig("tsnmf_rsvd", ctypes.c_int, [_vp, _i32, _i32, _vp, _vp, _i32, _vp, _i32, _vp, _vp])
_rank_sweep = _sig("tsnmf_rank_sweep", ctypes.c_int,
                   [_vp, _i32, _i32, _i32, _vp, _i32, _vp, _vp, _i32, _vp, _vp, _vp])
_onepass_create = _sig("tsnmf_onepass_create", ctypes.c_int, [_i32, _u32, _i32, _u64, ctypes.POINTER(_vp)])
_onepass_push = _sig("tsnmf_onepass_push", ctypes.c_int, [_vp, _vp, _i64, _i64, _vp])
_onepass_push_host = _sig("tsnmf_onepass_push_host", ctypes.c_int, [_vp, _vp, _i64, _i64, _vp])
_onepass_block_rows = _sig("tsnmf_onepass_block_rows", ctypes.c_int, [_vp, ctypes.POINTER(_i64)])
_onepass_rows = _sig("tsnmf_onepass_rows", ctypes.c_int, [_vp, ctypes.POINTER(_i64)])
_onepass_result = _sig("tsnmf_onepass_result", ctypes.c_int, [_vp, _vp, _vp, _vp, _vp])
_onepass_state_bytes = _sig("tsnmf_onepass_state_bytes", ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_size_t)])
_onepass_save = _sig("tsnmf_onepass_save", ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _vp])
_onepass_load = _sig("tsnmf_onepass_load", ctypes.c_int, [_vp, _vp, ctypes.c_size_t, _vp])
_onepass_destroy = _sig("tsnmf_onepass_destroy", ctypes.c_int, [_vp])
_reserve = _sig("tsnmf_reserve", ctypes.c_int, [_i64, _i32, _i32])
_workspace_release = _sig("tsnmf_workspace_release", ctypes.c_int, [])
_tune_load = _sig("tsnmf_tune_load", ctypes.c_int, [ctypes.c_char_p])
_profile_enable = _sig("tsnmf_profile_enable", ctypes.c_int, [ctypes.c_int])
_profile_query = _sig("tsnmf_profile_query", ctypes.c_int,
                      [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)])
_status_string = _sig("tsnmf_status_string", ctypes.c_char_p, [ctypes.c_int])
_last_hip_error = _sig("tsnmf_last_hip_error", ctypes.c_int, [])
_version = _sig("tsnmf_version", ctypes.c_int, [])


class TsnmfError(RuntimeError):
    def __init__(self, fn, status):
        msg = _status_string(status).decode()
        if status == 1:
            msg += f" (hip error {_last_hip_error()})"
        super().__init__(f"{fn} returned {status}: {msg}")
        self.status = status


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    return t.ctypes.data              # numpy array (host memory)


def _stream(stream):
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(fn, st):
    if st != 0:
        raise TsnmfError(fn, st)
    return st


# ---- same-name entry points (marshalling only) ---------------------------------------

def tsnmf_tsqr_r(X, m, n, ld, flags, R, colsum=None, stream=None):
    return _tsqr_r(_ptr(X), m, n, ld, flags, _ptr(R), _ptr(colsum), _stream(stream))


def tsnmf_tsqr_r_noalloc(X, m, n, ld, flags, R, colsum=None, stream=None):
    return _tsqr_r_noalloc(_ptr(X), m, n, ld, flags, _ptr(R), _ptr(colsum), _stream(stream))


def tsnmf_tsqr_r_ex(X, m, n, ld, flags, R, colsum=None, cfg=None, stream=None):
    c = None if cfg is None else ctypes.byref(cfg)
    return _tsqr_r_ex(_ptr(X), m, n, ld, flags, _ptr(R), _ptr(colsum), c, _stream(stream))


def tsnmf_tsqr_r_kron(A, p, q, lda, R, colsum=None, stream=None):
    return _tsqr_r_kron(_ptr(A), p, q, lda, _ptr(R), _ptr(colsum), _stream(stream))


def tsnmf_tsqr_r_batched_ex(batch, X, m, n, ld, flags, R, colsum=None, cfg=None, stream=None):
    c = None if cfg is None else ctypes.byref(cfg)
    return _tsqr_batched_ex(batch, _ptr(X), _ptr(m), _ptr(n), _ptr(ld), flags, _ptr(R), _ptr(colsum), c,
                            _stream(stream))


def tsnmf_tsqr_r_batched(batch, X, m, n, ld, flags, R, colsum=None, stream=None):
    return _tsqr_batched(batch, _ptr(X), _ptr(m), _ptr(n), _ptr(ld), flags, _ptr(R), _ptr(colsum),
                         _stream(stream))


def tsnmf_reserve_batched(max_batch, max_rows):
    return _reserve_batched(max_batch, max_rows)


def tsnmf_gauss_proj(X, m, n, ld, flags, k, seed, row_offset, Y, colsum=None, stream=None):
    return _gauss_proj(_ptr(X), m, n, ld, flags, k, seed, row_offset, _ptr(Y), _ptr(colsum), _stream(stream))


def tsnmf_gauss_colsum(m, k, seed, row_offset, s, stream=None):
    return _gauss_colsum(m, k, seed, row_offset, _ptr(s), _stream(stream))


def tsnmf_select_spa(M, p, n, ldm, colscale, r, K, score, info, stream=None):
    return _select_spa(_ptr(M), p, n, ldm, _ptr(colscale), r, _ptr(K), _ptr(score), _ptr(info), _stream(stream))


def tsnmf_select_xray(M, p, n, ldm, r, K, info, stream=None):
    return _select_xray(_ptr(M), p, n, ldm, r, _ptr(K), _ptr(info), _stream(stream))


def tsnmf_select_gp(Y, k, n, ldy, colscale, r, K, counts, info, stream=None):
    return _select_gp(_ptr(Y), k, n, ldy, _ptr(colscale), r, _ptr(K), _ptr(counts), _ptr(info), _stream(stream))


def tsnmf_nnls(M, p, n, ldm, K, r, H, ldh, resid2=None, info=None, stream=None):
    return _nnls(_ptr(M), p, n, ldm, _ptr(K), r, _ptr(H), ldh, _ptr(resid2), _ptr(info), _stream(stream))


def tsnmf_residual(M, p, n, ldm, K, r, H, ldh, relerr, stream=None):
    return _residual(_ptr(M), p, n, ldm, _ptr(K), r, _ptr(H), ldh, _ptr(relerr), _stream(stream))


def tsnmf_rsvd(R, n, ldr, S, V, ldv, U=None, ldu=0, info=None, stream=None):
    return _rsvd(_ptr(R), n, ldr, _ptr(S), _ptr(V), ldv, _ptr(U), ldu, _ptr(info), _stream(stream))


def tsnmf_rank_sweep(R, p, n, ldr, colscale, rmax, K, H, ldh, resid, info, stream=None):
    return _rank_sweep(_ptr(R), p, n, ldr, _ptr(colscale), rmax, _ptr(K), _ptr(H), ldh, _ptr(resid), _ptr(info),
                       _stream(stream))


def tsnmf_onepass_create(n, flags, k, seed, out):
    """`out` is a ctypes.c_void_p that receives the handle."""
    return _onepass_create(n, flags, k, seed, ctypes.byref(out))


def tsnmf_onepass_push(p, X, rows, ld, stream=None):
    return _onepass_push(p, _ptr(X), rows, ld, _stream(stream))


def tsnmf_onepass_push_host(p, X, rows, ld, stream=None):
    return _onepass_push_host(p, _ptr(X), rows, ld, _stream(stream))


def tsnmf_onepass_block_rows(p, out):
    return _onepass_block_rows(p, ctypes.byref(out))


def tsnmf_onepass_rows(p, out):
    return _onepass_rows(p, ctypes.byref(out))


def tsnmf_onepass_result(p, R, colsum=None, Y=None, stream=None):
    return _onepass_result(p, _ptr(R), _ptr(colsum), _ptr(Y), _stream(stream))


def tsnmf_onepass_state_bytes(p, out):
    return _onepass_state_bytes(p, ctypes.byref(out))


def tsnmf_onepass_save(p, host, nbytes, stream=None):
    return _onepass_save(p, _ptr(host), nbytes, _stream(stream))


def tsnmf_onepass_load(p, host, nbytes, stream=None):
    return _onepass_load(p, _ptr(host), nbytes, _stream(stream))


def tsnmf_onepass_destroy(p):
    return _onepass_destroy(p)


def tsnmf_reserve(max_m, max_n, max_k=0):
    return _reserve(max_m, max_n, max_k)


def tsnmf_workspace_release():
    return _workspace_release()


def tsnmf_tune_load(path):
    return _tune_load(None if path is None else os.fsencode(path))


def tsnmf_profile_enable(on):
    """on: 0/False off, 1/True every stage, 2 the main kernel only."""
    return _profile_enable(on if on in (0, 1, 2) and not isinstance(on, bool) else (1 if on else 0))


def tsnmf_profile_query(stage):
    """(status, total_ms, calls) of a profiling stage; clears it."""
    ms = ctypes.c_double()
    n = _i64()
    st = _profile_query(stage, ctypes.byref(ms), ctypes.byref(n))
    return st, ms.value, n.value


def tsnmf_status_string(status):
    return _status_string(status).decode()


def tsnmf_last_hip_error():
    return _last_hip_error()


def tsnmf_version():
    return _version()


# ---- convenience wrappers (allocate outputs with torch) --------------------------------

def _layout(X):
    """(flags, ld) for a 2-D CUDA tensor that is row-major or column-major."""
    if X.dim() != 2:
        raise ValueError("X must be 2-D")
    m, n = X.shape
    if X.stride(1) == 1 and (X.stride(0) >= n or m == 1):
        return ROW_MAJOR, max(X.stride(0), n)
    if X.stride(0) == 1 and (X.stride(1) >= m or n == 1):
        return COL_MAJOR, max(X.stride(1), m)
    raise ValueError("X must be row-major or column-major with unit inner stride")


_DTYPE_FLAG = {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}


def colmajor_square(buf):
    """Logical view of a column-major square output buffer."""
    return buf.t()


def tsqr_r(X, leaf_f64=False, config=None, stream=None, with_colsum=True):
    """R (n x n, FP64, diag >= 0) and the l1 column sums of a CUDA tensor X.

    config: None (library default), a TsqrConfig, or "tuned" for the entry the
    autotuner (tune.py) recorded for X's shape, if any."""
    m, n = X.shape
    lay, ld = _layout(X)
    if isinstance(config, str):
        if config != "tuned":
            raise ValueError("config must be None, a TsqrConfig or 'tuned'")
        from . import tune
        config = tune.lookup(X, leaf_f64)
    flags = _DTYPE_FLAG[X.dtype] | lay | (LEAF_F64 if leaf_f64 else 0)
    Rbuf = torch.empty((n, n), dtype=torch.float64, device=X.device)
    cs = torch.empty(n, dtype=torch.float64, device=X.device) if with_colsum else None
    if config is None:
        st = tsnmf_tsqr_r(X, m, n, ld, flags, Rbuf, cs, stream)
    else:
        st = tsnmf_tsqr_r_ex(X, m, n, ld, flags, Rbuf, cs, config, stream)
    _check("tsnmf_tsqr_r", st)
    return colmajor_square(Rbuf), cs


def tsqr_r_kron(A, stream=None, with_colsum=True):
    """R and column sums of X = A (x) A for a row-major FP32 CUDA tensor A
    (p x q, q <= 5), without forming X."""
    p, q = A.shape
    lay, lda = _layout(A)
    if lay != ROW_MAJOR or A.dtype != torch.float32:
        raise ValueError("A must be a row-major float32 tensor")
    n = q * q
    Rbuf = torch.empty((n, n), dtype=torch.float64, device=A.device)
    cs = torch.empty(n, dtype=torch.float64, device=A.device) if with_colsum else None
    _check("tsnmf_tsqr_r_kron", tsnmf_tsqr_r_kron(A, p, q, lda, Rbuf, cs, stream))
    return colmajor_square(Rbuf), cs


def gauss_proj(X, k, seed, mode=None, row_offset=0, stream=None, with_colsum=False):
    """Y = G^T X (k x n, FP32) with the library's Philox-defined G."""
    m, n = X.shape
    lay, ld = _layout(X)
    if lay != ROW_MAJOR:
        raise ValueError("gauss_proj expects a row-major X")
    if mode is None:
        mode = GP_MFMA_BF16 if X.dtype == torch.bfloat16 else GP_SIMD_F32
    flags = _DTYPE_FLAG[X.dtype] | mode
    Ybuf = torch.empty((n, k), dtype=torch.float32, device=X.device)   # column-major k x n
    cs = torch.empty(n, dtype=torch.float64, device=X.device) if with_colsum else None
    _check("tsnmf_gauss_proj", tsnmf_gauss_proj(X, m, n, ld, flags, k, seed, row_offset, Ybuf, cs, stream))
    return Ybuf.t(), cs


def gauss_colsum(m, k, seed, row_offset=0, device="cuda", stream=None):
    """G^T 1 (k values) for the projection's G, without reading any X."""
    out = torch.empty(k, dtype=torch.float32, device=device)
    _check("tsnmf_gauss_colsum", tsnmf_gauss_colsum(m, k, seed, row_offset, out, stream))
    return out


def _colmajor_input(M):
    """(buffer, ld) of a logical matrix for the column-major small solvers."""
    if M.stride(0) == 1 and M.stride(1) >= M.shape[0]:
        return M, M.stride(1)
    buf = M.t().contiguous()          # column-major copy
    return buf.t(), M.shape[0]


def select_spa(M, r, colscale=None, stream=None):
    p, n = M.shape
    Mc, ldm = _colmajor_input(M)
    K = torch.empty(r, dtype=torch.int32, device=M.device)
    score = torch.empty(r, dtype=torch.float64, device=M.device)
    info = torch.empty(1, dtype=torch.int32, device=M.device)
    _check("tsnmf_select_spa", tsnmf_select_spa(Mc, p, n, ldm, colscale, r, K, score, info, stream))
    return K, score, info


def select_xray(M, r, stream=None):
    p, n = M.shape
    Mc, ldm = _colmajor_input(M)
    K = torch.empty(r, dtype=torch.int32, device=M.device)
    info = torch.empty(1, dtype=torch.int32, device=M.device)
    _check("tsnmf_select_xray", tsnmf_select_xray(Mc, p, n, ldm, r, K, info, stream))
    return K, info


def select_gp(Y, r, colscale=None, stream=None):
    k, n = Y.shape
    Yc, ldy = _colmajor_input(Y)
    K = torch.empty(r, dtype=torch.int32, device=Y.device)
    counts = torch.empty(n, dtype=torch.int32, device=Y.device)
    info = torch.empty(1, dtype=torch.int32, device=Y.device)
    _check("tsnmf_select_gp", tsnmf_select_gp(Yc, k, n, ldy, colscale, r, K, counts, info, stream))
    return K, counts, info


def nnls(M, K, stream=None):
    p, n = M.shape
    r = K.numel()
    Mc, ldm = _colmajor_input(M)
    Hbuf = torch.empty((n, r), dtype=torch.float64, device=M.device)   # column-major r x n
    res = torch.empty(n, dtype=torch.float64, device=M.device)
    info = torch.empty(n, dtype=torch.int32, device=M.device)
    _check("tsnmf_nnls", tsnmf_nnls(Mc, p, n, ldm, K, r, Hbuf, r, res, info, stream))
    return Hbuf.t(), res, info


def residual(M, K, H, stream=None):
    p, n = M.shape
    r = K.numel()
    Mc, ldm = _colmajor_input(M)
    Hc, ldh = _colmajor_input(H)
    out = torch.empty(1, dtype=torch.float64, device=M.device)
    _check("tsnmf_residual", tsnmf_residual(Mc, p, n, ldm, K, r, Hc, ldh, out, stream))
    return out


def rsvd(R, with_u=True, stream=None):
    """(S, U, V) of an n x n FP64 CUDA matrix R (R = U diag(S) V^T), and the
    number of Jacobi sweeps."""
    n = R.shape[0]
    Rc, ldr = _colmajor_input(R)
    S = torch.empty(n, dtype=torch.float64, device=R.device)
    Vb = torch.empty((n, n), dtype=torch.float64, device=R.device)
    Ub = torch.empty((n, n), dtype=torch.float64, device=R.device) if with_u else None
    info = torch.empty(1, dtype=torch.int32, device=R.device)
    _check("tsnmf_rsvd", tsnmf_rsvd(Rc, n, ldr, S, Vb, n, Ub, n if with_u else 0, info, stream))
    return S, (Ub.t() if with_u else None), Vb.t(), info


def rank_sweep(R, rmax, colscale=None, stream=None):
    """(K, resid, H, info): SPA's rmax picks and the relative residual of the
    NNLS fit on each prefix K[:r], r = 1..rmax; H is the fit at rmax."""
    p, n = R.shape
    Rc, ldr = _colmajor_input(R)
    K = torch.empty(rmax, dtype=torch.int32, device=R.device)
    Hb = torch.empty((n, rmax), dtype=torch.float64, device=R.device)
    resid = torch.empty(rmax, dtype=torch.float64, device=R.device)
    info = torch.empty(1, dtype=torch.int32, device=R.device)
    _check("tsnmf_rank_sweep", tsnmf_rank_sweep(Rc, p, n, ldr, colscale, rmax, K, Hb, rmax, resid, info, stream))
    return K, resid, Hb.t(), info


class OnePass:
    """One pass over a matrix delivered in row blocks (device tensors or host
    arrays): R, column sums and, with k > 0, G^T X over all rows pushed."""

    def __init__(self, n, dtype=torch.float32, col_major=False, k=0, seed=0, mode=None, leaf_f64=False):
        flags = _DTYPE_FLAG[dtype] | (COL_MAJOR if col_major else ROW_MAJOR) | (LEAF_F64 if leaf_f64 else 0)
        if k > 0:
            flags |= GP_SIMD_F32 if mode is None else mode
        self.n, self.k, self.h = n, k, ctypes.c_void_p()
        _check("tsnmf_onepass_create", tsnmf_onepass_create(n, flags, k, seed, self.h))

    def push(self, X, stream=None):
        """A device tensor with the state's dtype and layout (rows x n)."""
        lay, ld = _layout(X)
        _check("tsnmf_onepass_push", tsnmf_onepass_push(self.h, X, X.shape[0], ld, stream))

    def push_host(self, X, stream=None):
        """A row-major host array (numpy array or CPU tensor, pinned or not)."""
        rows = X.shape[0]
        ld = X.stride(0) if isinstance(X, torch.Tensor) else X.strides[0] // X.itemsize
        _check("tsnmf_onepass_push_host", tsnmf_onepass_push_host(self.h, X, rows, ld, stream))

    @property
    def block_rows(self):
        v = _i64()
        _check("tsnmf_onepass_block_rows", tsnmf_onepass_block_rows(self.h, v))
        return v.value

    @property
    def rows(self):
        v = _i64()
        _check("tsnmf_onepass_rows", tsnmf_onepass_rows(self.h, v))
        return v.value

    def result(self, stream=None, device="cuda"):
        n, k = self.n, self.k
        Rb = torch.empty((n, n), dtype=torch.float64, device=device)
        cs = torch.empty(n, dtype=torch.float64, device=device)
        Yb = torch.empty((n, k), dtype=torch.float32, device=device) if k > 0 else None
        _check("tsnmf_onepass_result", tsnmf_onepass_result(self.h, Rb, cs, Yb, stream))
        return colmajor_square(Rb), cs, (Yb.t() if k > 0 else None)

    def save(self, stream=None):
        nb = ctypes.c_size_t()
        _check("tsnmf_onepass_state_bytes", tsnmf_onepass_state_bytes(self.h, nb))
        buf = (ctypes.c_char * nb.value)()
        _check("tsnmf_onepass_save", tsnmf_onepass_save(self.h, ctypes.addressof(buf), nb.value, stream))
        return bytes(buf)

    def load(self, blob, stream=None):
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check("tsnmf_onepass_load", tsnmf_onepass_load(self.h, ctypes.addressof(buf), len(blob), stream))

    def close(self):
        if self.h.value:
            _check("tsnmf_onepass_destroy", tsnmf_onepass_destroy(self.h))
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def reserve(max_m, max_n, max_k=0):
    _check("tsnmf_reserve", tsnmf_reserve(max_m, max_n, max_k))


class Batch:
    """Device arrays for tsnmf_tsqr_r_batched over a list of row-major FP32
    CUDA matrices, with FP64 outputs allocated by torch.  ``run`` enqueues the
    call; the arrays stay valid for replays of a captured graph."""

    def __init__(self, mats, with_colsum=True):
        if not mats:
            raise ValueError("empty batch")
        dev = mats[0].device
        self.mats = list(mats)
        lds = []
        for X in self.mats:
            lay, ld = _layout(X)
            if lay != ROW_MAJOR or X.dtype != torch.float32:
                raise ValueError("the batched call takes row-major float32 matrices")
            lds.append(ld)
        self.Rbuf = [torch.empty((X.shape[1], X.shape[1]), dtype=torch.float64, device=dev) for X in self.mats]
        self.cs = [torch.empty(X.shape[1], dtype=torch.float64, device=dev) for X in self.mats] if with_colsum else None

        def arr(vals):
            return torch.tensor(vals, dtype=torch.int64).to(dev)

        self.X = arr([X.data_ptr() for X in self.mats])
        self.m = arr([X.shape[0] for X in self.mats])
        self.n = arr([X.shape[1] for X in self.mats])
        self.ld = arr(lds)
        self.R = arr([r.data_ptr() for r in self.Rbuf])
        self.colsum = arr([c.data_ptr() for c in self.cs]) if with_colsum else None

    def run(self, stream=None, config=None):
        """config: None (library default or the loaded table) or a BatchConfig."""
        if config is None:
            _check("tsnmf_tsqr_r_batched",
                   tsnmf_tsqr_r_batched(len(self.mats), self.X, self.m, self.n, self.ld, F32, self.R, self.colsum,
                                        stream))
        else:
            _check("tsnmf_tsqr_r_batched_ex",
                   tsnmf_tsqr_r_batched_ex(len(self.mats), self.X, self.m, self.n, self.ld, F32, self.R,
                                           self.colsum, config, stream))

    def results(self):
        """[(R, colsum)] with R the logical n x n view of each output."""
        return [(colmajor_square(r), None if self.cs is None else c)
                for r, c in zip(self.Rbuf, self.cs or [None] * len(self.Rbuf))]


def tsqr_r_batched(mats, with_colsum=True, stream=None, config=None):
    """R factors and column sums of a list of row-major FP32 CUDA matrices."""
    b = Batch(mats, with_colsum)
    b.run(stream, config)
    return b.results()


def reserve_batched(max_batch, max_rows):
    _check("tsnmf_reserve_batched", tsnmf_reserve_batched(max_batch, max_rows))
