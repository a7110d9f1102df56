"""Python binding of libmpr, the MI355X (gfx950) library of exact (min,+)
matrix powers for the Roman domination number of cylinders P_m x C_n
(Martinez, Garzon, Puertas, arXiv 2409.17658).

Argument marshalling only: every function here calls the C ABI declared in
include/mpr.h with device pointers taken from torch tensors; all arithmetic
runs in the HIP kernels of libmpr.so.  torch supplies device memory and
streams.  There is no CPU fallback: if libmpr.so has not been built, or no
gfx950 device is present, the calls raise.

Matrices are 2-D torch.uint16 CUDA tensors with unit column stride; the row
stride (tensor.stride(0)) is the leading dimension.  alloc_matrix() returns
a view of a buffer padded to a multiple of 8 columns (the kernels' fast
path).  Offsets R are int64 CUDA tensors.  0xFFFF is infinity.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmpr.so")

INF = 0xFFFF
FMAX = 0x7FFF
ROW_NONE = (1 << 63) - 1
CHAIN = 0
SQUARE = 1
CHAIN_SPARSE = 2
PERIOD_SPARSE = 1
PERIOD_EXTEND = 2
PERIOD_REUSE_A = 4
PERIOD_PIPELINE = 8
ARITH_U16 = 0
ARITH_F16 = 1

_STATUS = {0: "MPR_OK", 1: "MPR_EINVAL", 2: "MPR_ENOMEM", 3: "MPR_EOVERFLOW",
           4: "MPR_ENOTFOUND", 5: "MPR_EHIP", 6: "MPR_EUNSUPPORTED"}


class MprError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s (%d)" % (where, _STATUS.get(status, "?"), status))


class ChainDesc(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("n", ctypes.c_int64), ("lda", ctypes.c_int64),
                ("e", ctypes.c_int64), ("N_out", ctypes.c_void_p), ("ldo", ctypes.c_int64),
                ("R_out", ctypes.c_void_p)]


class ServerOptions(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("baby", ctypes.c_int), ("max_n", ctypes.c_int64),
                ("max_batch", ctypes.c_int), ("slots", ctypes.c_int), ("hbm_budget_bytes", ctypes.c_size_t),
                ("wide_only", ctypes.c_int), ("busy_poll", ctypes.c_int), ("period_mode", ctypes.c_int),
                ("request_timeout_s", ctypes.c_double)]


class QueryResult(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_int64), ("m", ctypes.c_int), ("n", ctypes.c_int64), ("gamma", ctypes.c_int64),
                ("status", ctypes.c_int), ("cold", ctypes.c_int), ("t_submit_s", ctypes.c_double),
                ("t_start_s", ctypes.c_double), ("t_done_s", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "batches", "max_batch_seen", "builds",
                                             "evictions", "admission_waits", "resident_bytes", "narrow_builds",
                                             "shared_reads", "period_answers", "early_answers")]


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I = ctypes.c_int
_SZ = ctypes.c_size_t

_SIGS = {
    "mpr_version": (_I, []),
    "mpr_status_string": (ctypes.c_char_p, [_I]),
    "mpr_init": (_I, [_I]),
    "mpr_transfer_size": (_I, [_I, _P]),
    "mpr_transfer_words": (_I, [_I, _P, _I64]),
    "mpr_build_transfer": (_I, [_I, _P, _I64, _P]),
    "mpr_build_border_transfer": (_I, [_I, _P, _I64, _P, _P]),
    "mpr_minplus_gemm": (_I, [_I64, _I64, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _P]),
    "mpr_minplus_gemm_spare": (_I, [_I, _I64, _I64, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _P]),
    "mpr_minplus_gemm_cfg": (_I, [_I, _I64, _I64, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _P]),
    "mpr_normalise": (_I, [_I64, _I64, _P, _I64, _P, _P, _P, _P]),
    "mpr_gemm_norm_workspace_size": (_I, [_I64, _I64, _P]),
    "mpr_minplus_gemm_norm": (_I, [_I64, _I64, _I64, _P, _I64, _P, _P, _I64, _P, _P, _I64, _P,
                                   _P, _SZ, _P, _P]),
    "mpr_power_workspace_size": (_I, [_I64, _I64, _I, _P]),
    "mpr_minplus_power": (_I, [_P, _I64, _I64, _I64, _I, _P, _I64, _P, _P, _SZ, _P, _P]),
    "mpr_chain_resume": (_I, [_P, _I64, _I64, _P, _I64, _P, _I64, _I, _P, _I64, _P, _P, _SZ, _P, _P]),
    "mpr_minplus_power_noalloc": (_I, [_P, _I64, _I64, _I64, _I, _P, _I64, _P, _P, _P]),
    "mpr_sparse_plan_bytes": (_I, [_P, _I64, _I64, _P, _P]),
    "mpr_trace_min": (_I, [_P, _I64, _I64, _P, _P, _P]),
    "mpr_trace_of_product": (_I, [_P, _P, _P, _P, _I64, _I64, _P, _P]),
    "mpr_trace_of_product_t": (_I, [_P, _P, _P, _P, _I64, _I64, _P, _P]),
    "mpr_period_workspace_size": (_I, [_I64, _I64, _P]),
    "mpr_find_period": (_I, [_P, _I64, _I64, _I64, _P, _P, _P, _P, _P, _SZ, _P]),
    "mpr_period_workspace_size_ex": (_I, [_I64, _I64, _I, _P]),
    "mpr_find_period_ex": (_I, [_P, _I64, _I64, _I64, _I, _P, _P, _P, _P, _P, _SZ, _P]),
    "mpr_gamma_from_period": (_I, [_I64, _I64, _I64, _P, _I64, _I64, _P]),
    "mpr_set_period_progress": (_I, [_P, _P]),
    "mpr_period_formula": (_I, [_I64, _I64, _I64, _P, _I64, _P]),
    "mpr_batch_workspace_size": (_I, [_P, _I, _P]),
    "mpr_batch_plan": (_I, [_P, _I, _P, _SZ, _P]),
    "mpr_batch_launch": (_I, [_P, _P, _P]),
    "mpr_batch_power": (_I, [_P, _I, _P, _SZ, _P, _P]),
    "mpr_batch_config_count": (_I, []),
    "mpr_batch_config_info": (_I, [_I, _P, _P, _P]),
    "mpr_set_sparse_arith": (_I, [_I]),
    "mpr_set_sparse_form": (_I, [_I]),
    "mpr_set_arith": (_I, [_I]),
    "mpr_get_arith": (_I, []),
    "mpr_set_batch_weights": (_I, [_P, _I]),
    "mpr_get_batch_weights": (_I, [_P, _I]),
    "mpr_batch_plan_info": (_I, [_P, _P, _P, _P]),
    "mpr_set_batch_config": (_I, [_I]),
    "mpr_set_batch_persistent": (_I, [_I]),
    "mpr_batch_graph_create": (_I, [_P, _P, _P, _P]),
    "mpr_graph_launch": (_I, [_P, _P]),
    "mpr_graph_destroy": (_I, [_P]),
    "mpr_server_create": (_I, [_P, _P]),
    "mpr_server_submit": (_I, [_P, _I, _I64, _I64]),
    "mpr_server_poll": (_I, [_P, _P, _I, _P, _I]),
    "mpr_server_stats_get": (_I, [_P, _P]),
    "mpr_server_cancel": (_I, [_P, _I64]),
    "mpr_server_now": (ctypes.c_double, [_P]),
    "mpr_server_ladder_bytes": (_I64, [_I, _I, _I64, _I]),
    "mpr_server_period_bytes": (_I64, [_I]),
    "mpr_server_destroy": (_I, [_P]),
    "mpr_gemm_config_count": (_I, []),
    "mpr_gemm_config_info": (_I, [_I, _P, _P, _P, _P, _P, _P, _P]),
    "mpr_set_tile_table": (_I, [_P, _P, _I]),
    "mpr_gemm_pick_config": (_I, [_I64, _I64, _I64]),
    "mpr_autotune_gemm": (_I, [_I64, _I, _P, _P, _P]),
    "mpr_valu_probe": (_I, [_I, _I, _P, _P, _P]),
}


def lib():
    """The loaded libmpr.so (ctypes), with every C-ABI signature declared."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmpr.so is not built (run paper_2409_17658_amd.build.build()); "
                               "there is no CPU fallback")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return sorted(_SIGS)


def _ok(status: int, where: str):
    if status != 0:
        raise MprError(status, where)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a CUDA (HIP) tensor")
    return ctypes.c_void_p(t.data_ptr())


def _vptr(t, n: int):
    """Device pointer of an int64 vector of at least n entries (None -> NULL)."""
    if t is None:
        return None
    if t.dtype != torch.int64 or t.dim() != 1 or (t.numel() > 1 and t.stride(0) != 1) or t.numel() < n:
        raise ValueError("expected a contiguous int64 vector of at least %d entries" % n)
    return _ptr(t)


def _stream(stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ld(t):
    if t.dim() != 2 or t.stride(1) != 1 or t.dtype != torch.uint16:
        raise ValueError("expected a 2-D uint16 tensor with unit column stride")
    return max(t.stride(0), t.shape[1], 1)


def _status_tensor(device):
    return torch.zeros(1, dtype=torch.int32, device=device)


def check_status(d_status):
    """Raise MprError if a device status word is non-zero (synchronises)."""
    v = int(d_status.item())
    if v != 0:
        raise MprError(v, "device status")


def round_up(x: int, a: int = 8) -> int:
    return (x + a - 1) // a * a


def alloc_matrix(rows: int, cols: int, device="cuda", fill=None):
    """rows x cols uint16 view of a buffer whose row stride is a multiple of 8."""
    buf = torch.empty((rows, round_up(max(cols, 1))), dtype=torch.uint16, device=device)
    if fill is not None:
        buf.view(torch.int16).fill_(np.int16(np.uint16(fill).view(np.int16)).item())
    return buf[:, :cols]


def to_device(a: np.ndarray, device="cuda"):
    """Host uint16 matrix -> padded device view (same values)."""
    a = np.ascontiguousarray(a, dtype=np.uint16)
    out = alloc_matrix(a.shape[0], a.shape[1], device)
    out.copy_(torch.from_numpy(a).to(device))
    return out


def to_host(t) -> np.ndarray:
    return t.cpu().numpy()


def workspace(nbytes: int, device="cuda"):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


# ---------------------------------------------------------------- info
def version() -> int:
    return lib().mpr_version()


def init(device: int = 0, tile_table: bool = True):
    """Checks the device and installs the autotuners' persisted tables
    (tile_table.json: size -> product configuration per arithmetic;
    batch_table.json: weights of the batched-configuration model) when
    there are any."""
    _ok(lib().mpr_init(device), "mpr_init")
    if tile_table:
        from .autotune import load_batch_table, load_table

        load_table()
        load_batch_table()


def transfer_size(m: int) -> int:
    n = ctypes.c_int64()
    _ok(lib().mpr_transfer_size(m, ctypes.byref(n)), "mpr_transfer_size")
    return n.value


def transfer_words(m: int) -> np.ndarray:
    n = transfer_size(m)
    out = np.zeros((n, m), dtype=np.uint8)
    _ok(lib().mpr_transfer_words(m, out.ctypes.data_as(_P), n), "mpr_transfer_words")
    return out


# ---------------------------------------------------------------- kernels
def build_transfer(m: int, out=None, stream=None):
    n = transfer_size(m)
    A = alloc_matrix(n, n) if out is None else out
    _ok(lib().mpr_build_transfer(m, _ptr(A), _ld(A), _stream(stream)), "mpr_build_transfer")
    return A


def build_border_transfer(m: int, out=None, stream=None):
    """(A', shift): the appendix's border matrix with every finite entry
    raised by shift (labels can be negative)."""
    n = transfer_size(m)
    A = alloc_matrix(n, n) if out is None else out
    sh = ctypes.c_int64()
    _ok(lib().mpr_build_border_transfer(m, _ptr(A), _ld(A), ctypes.byref(sh), _stream(stream)),
        "mpr_build_border_transfer")
    return A, sh.value


def minplus_gemm(A, B, C=None, check=True, cfg=-1, stream=None, d_status=None, spare=False):
    """C = A (x) B.  spare=True: the launch that leaves one workgroup slot
    per CU free for other launches while it runs (same bits)."""
    M, K = A.shape
    K2, N = B.shape
    if K != K2:
        raise ValueError("inner dimensions differ")
    if C is None:
        C = alloc_matrix(M, N, A.device)
    st = d_status if d_status is not None else (_status_tensor(A.device) if check else None)
    fn = lib().mpr_minplus_gemm_spare if spare else lib().mpr_minplus_gemm_cfg
    _ok(fn(cfg, M, N, K, _ptr(A), _ld(A), _ptr(B), _ld(B), _ptr(C), _ld(C), _ptr(st), _stream(stream)),
        "mpr_minplus_gemm")
    if check and d_status is None:
        check_status(st)
    return C


def normalise(C, R_in=None, R_out=None, check=True, stream=None):
    M, N = C.shape
    if R_out is None:
        R_out = torch.empty(M, dtype=torch.int64, device=C.device)
    st = _status_tensor(C.device) if check else None
    _ok(lib().mpr_normalise(M, N, _ptr(C), _ld(C), _vptr(R_in, M), _vptr(R_out, M), _ptr(st), _stream(stream)),
        "mpr_normalise")
    if check:
        check_status(st)
    return R_out


def minplus_gemm_norm(A, B, Ra=None, Rb=None, C=None, Rc=None, ws=None, check=True, stream=None):
    M, K = A.shape
    _, N = B.shape
    if C is None:
        C = alloc_matrix(M, N, A.device)
    if Rc is None:
        Rc = torch.empty(M, dtype=torch.int64, device=A.device)
    if ws is None:
        nb = ctypes.c_size_t()
        _ok(lib().mpr_gemm_norm_workspace_size(K, N, ctypes.byref(nb)), "mpr_gemm_norm_workspace_size")
        ws = workspace(nb.value, A.device)
    st = _status_tensor(A.device) if check else None
    _ok(lib().mpr_minplus_gemm_norm(M, N, K, _ptr(A), _ld(A), _vptr(Ra, M), _ptr(B), _ld(B), _vptr(Rb, K), _ptr(C),
                                    _ld(C), _vptr(Rc, M), _ptr(ws), ws.numel(), _ptr(st), _stream(stream)),
        "mpr_minplus_gemm_norm")
    if check:
        check_status(st)
    return C, Rc


def power_workspace_size(n: int, e: int, schedule: int = CHAIN) -> int:
    nb = ctypes.c_size_t()
    _ok(lib().mpr_power_workspace_size(n, e, schedule, ctypes.byref(nb)), "mpr_power_workspace_size")
    return nb.value


def minplus_power(A, e: int, schedule: int = CHAIN, N_out=None, R_out=None, ws=None, check=True, stream=None,
                  d_status=None):
    n = A.shape[0]
    if N_out is None:
        N_out = alloc_matrix(n, n, A.device)
    if R_out is None:
        R_out = torch.empty(n, dtype=torch.int64, device=A.device)
    st = d_status if d_status is not None else (_status_tensor(A.device) if check else None)
    if ws is None:
        if schedule == CHAIN_SPARSE and st is not None and e >= 2:  # the plan sized for this A
            ws = workspace(power_workspace_size(n, e, CHAIN) + 256 + sparse_plan_bytes(A, stream), A.device)
        else:
            ws = workspace(power_workspace_size(n, e, schedule), A.device)
    _ok(lib().mpr_minplus_power(_ptr(A), n, _ld(A), e, schedule, _ptr(N_out), _ld(N_out), _vptr(R_out, n),
                                _ptr(ws), ws.numel(), _ptr(st), _stream(stream)), "mpr_minplus_power")
    if check and d_status is None:
        check_status(st)
    return N_out, R_out


def chain_resume(A, N_k, R_k, steps: int, schedule: int = CHAIN, N_out=None, R_out=None, ws=None, check=True,
                 stream=None, d_status=None):
    """Canonical form of A^(k + steps) from that of A^k, (N_k, R_k), by
    `steps` chain steps (mpr_chain_resume)."""
    n = A.shape[0]
    if N_out is None:
        N_out = alloc_matrix(n, n, A.device)
    if R_out is None:
        R_out = torch.empty(n, dtype=torch.int64, device=A.device)
    st = d_status if d_status is not None else (_status_tensor(A.device) if check else None)
    if ws is None:
        if schedule == CHAIN_SPARSE and st is not None and steps >= 1:
            ws = workspace(power_workspace_size(n, steps + 1, CHAIN) + 256 + sparse_plan_bytes(A, stream), A.device)
        else:
            ws = workspace(power_workspace_size(n, steps + 1, schedule), A.device)
    _ok(lib().mpr_chain_resume(_ptr(A), n, _ld(A), _ptr(N_k), _ld(N_k), _vptr(R_k, n), steps, schedule, _ptr(N_out),
                               _ld(N_out), _vptr(R_out, n), _ptr(ws), ws.numel(), _ptr(st), _stream(stream)),
        "mpr_chain_resume")
    if check and d_status is None:
        check_status(st)
    return N_out, R_out


def save_power(path, N, R, k: int):
    """Checkpoint of a chain: the canonical form (N, R) of A^k and k, written
    to an .npz file (plain arrays, no pickled objects)."""
    np.savez(path, N=to_host(N), R=R.cpu().numpy().astype(np.int64), k=np.int64(k))


def load_power(path, device="cuda"):
    """(N, R, k) of a checkpoint written by save_power, N and R on `device`."""
    with np.load(path, allow_pickle=False) as z:
        N, R, k = z["N"], z["R"], int(z["k"])
    if N.dtype != np.uint16 or R.dtype != np.int64 or N.shape[0] != N.shape[1] or R.shape != (N.shape[0],):
        raise ValueError("not a checkpoint of a canonical power")
    return to_device(N, device), torch.from_numpy(R).to(device), k


NOALLOC_SCRATCH_BYTES = 64 << 20


def minplus_power_noalloc(A, e: int, schedule: int, N_out, R_out, d_status=None, stream=None):
    """mpr_minplus_power on the library's fixed device scratch (no workspace,
    no allocation by the library); N_out / R_out are the caller's."""
    n = A.shape[0]
    _ok(lib().mpr_minplus_power_noalloc(_ptr(A), n, _ld(A), e, schedule, _ptr(N_out), _ld(N_out), _vptr(R_out, n),
                                        _ptr(d_status), _stream(stream)), "mpr_minplus_power_noalloc")
    return N_out, R_out


def sparse_plan_bytes(A, stream=None) -> int:
    """Bytes of the compressed-K plan of A (synchronous)."""
    nb = ctypes.c_size_t()
    _ok(lib().mpr_sparse_plan_bytes(_ptr(A), A.shape[0], _ld(A), ctypes.byref(nb), _stream(stream)),
        "mpr_sparse_plan_bytes")
    return nb.value


def trace_min(N, R, out=None, stream=None):
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=N.device)
    _ok(lib().mpr_trace_min(_ptr(N), N.shape[0], _ld(N), _vptr(R, N.shape[0]), _vptr(out, 1), _stream(stream)), "mpr_trace_min")
    return out


def trace_of_product(X, RX, Y, RY, out=None, stream=None):
    if X.stride(0) != Y.stride(0):
        raise ValueError("X and Y must share a leading dimension")
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=X.device)
    _ok(lib().mpr_trace_of_product(_ptr(X), _vptr(RX, X.shape[0]), _ptr(Y), _vptr(RY, X.shape[0]), X.shape[0], _ld(X), _vptr(out, 1),
                                   _stream(stream)), "mpr_trace_of_product")
    return out


def trace_of_product_t(X, RX, YT, CY, out=None, stream=None):
    """Trace of (RX (+) X) (x) Y with Y given through the canonical form
    (YT, CY) of its transpose: Y[l][i] = CY[i] + YT[i][l]."""
    if X.stride(0) != YT.stride(0):
        raise ValueError("X and YT must share a leading dimension")
    if out is None:
        out = torch.empty(1, dtype=torch.int64, device=X.device)
    _ok(lib().mpr_trace_of_product_t(_ptr(X), _vptr(RX, X.shape[0]), _ptr(YT), _vptr(CY, X.shape[0]), X.shape[0],
                                     _ld(X), _vptr(out, 1), _stream(stream)), "mpr_trace_of_product_t")
    return out


def period_workspace_size(n: int, slots: int, flags: int = 0) -> int:
    nb = ctypes.c_size_t()
    _ok(lib().mpr_period_workspace_size_ex(n, slots, flags, ctypes.byref(nb)), "mpr_period_workspace_size_ex")
    return nb.value


def find_period(A, kmax: int, traces: bool = True, slots: int = 64, ws=None, stream=None, sparse: bool = False,
                extend: bool = False, reuse_a: bool = False, pipeline: bool = False):
    """(mu, lam, c, traces) with traces[k] = trace of A^k for k = 1..kmax
    (None when traces=False); mu is None when no period is confirmed.
    sparse=True runs the chain steps over the compressed rows of A;
    extend=True stops at the confirming power and fills the later traces
    from the period (exact); reuse_a=True (with sparse) lets the search
    overwrite A to confirm a period longer than the ring one period late;
    pipeline=True computes the next power while the host reads the current
    one's class hash (same results)."""
    n = A.shape[0]
    flags = ((PERIOD_SPARSE if sparse else 0) | (PERIOD_EXTEND if extend else 0) |
             (PERIOD_REUSE_A if reuse_a else 0) | (PERIOD_PIPELINE if pipeline else 0))
    if ws is None:  # with sparse=True the plan is sized for this A
        ws = workspace(period_workspace_size(n, slots, flags & (PERIOD_REUSE_A | PERIOD_PIPELINE)) +
                       (sparse_plan_bytes(A, stream) if sparse else 0), A.device)
    mu, lam, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    tr = np.zeros(kmax + 1, dtype=np.int64) if traces else None
    st = lib().mpr_find_period_ex(_ptr(A), n, _ld(A), kmax, flags, ctypes.byref(mu), ctypes.byref(lam),
                                  ctypes.byref(c), tr.ctypes.data_as(_P) if traces else None, _ptr(ws), ws.numel(),
                                  _stream(stream))
    if st == 4:
        return None, None, None, tr
    _ok(st, "mpr_find_period")
    return mu.value, lam.value, c.value, tr


_PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p)
_progress_keep = None


def set_period_progress(fn=None):
    """fn(k, trace) after every power of a period search (None: off)."""
    global _progress_keep
    if fn is None:
        _ok(lib().mpr_set_period_progress(None, None), "mpr_set_period_progress")
        _progress_keep = None
        return
    cb = _PROGRESS_FN(lambda k, t, _u: fn(int(k), int(t)))
    _ok(lib().mpr_set_period_progress(ctypes.cast(cb, ctypes.c_void_p), None), "mpr_set_period_progress")
    _progress_keep = cb  # the C side keeps the pointer: keep the callback alive


def gamma_from_period(mu: int, lam: int, c: int, traces, n: int) -> int:
    """gamma(n) from a period and the traces (Proposition 8)."""
    tr = np.ascontiguousarray(traces, dtype=np.int64)
    g = ctypes.c_int64()
    _ok(lib().mpr_gamma_from_period(mu, lam, c, tr.ctypes.data_as(_P), len(tr) - 1, n, ctypes.byref(g)),
        "mpr_gamma_from_period")
    return g.value


def period_formula(mu: int, lam: int, c: int, traces):
    """numer[r] with gamma(n) = (c n + numer[n mod lam]) / lam for n >= mu."""
    tr = np.ascontiguousarray(traces, dtype=np.int64)
    out = np.zeros(lam, dtype=np.int64)
    _ok(lib().mpr_period_formula(mu, lam, c, tr.ctypes.data_as(_P), len(tr) - 1, out.ctypes.data_as(_P)),
        "mpr_period_formula")
    return out


# ---------------------------------------------------------------- batched chains
def _descs(chains):
    arr = (ChainDesc * len(chains))()
    for i, (A, e, N_out, R_out) in enumerate(chains):
        _ptr(A), _ptr(N_out)  # device tensors
        arr[i] = ChainDesc(A.data_ptr(), A.shape[0], _ld(A), int(e), N_out.data_ptr(), _ld(N_out),
                           _vptr(R_out, A.shape[0]).value)
    return arr


def batch_workspace_size(chains) -> int:
    d = _descs(chains)
    nb = ctypes.c_size_t()
    _ok(lib().mpr_batch_workspace_size(d, len(chains), ctypes.byref(nb)), "mpr_batch_workspace_size")
    return nb.value


def batch_plan(chains, ws, stream=None):
    """chains: list of (A, e, N_out, R_out) device tensors."""
    d = _descs(chains)
    _ok(lib().mpr_batch_plan(d, len(chains), _ptr(ws), ws.numel(), _stream(stream)), "mpr_batch_plan")


def batch_launch(ws, d_status=None, stream=None):
    _ok(lib().mpr_batch_launch(_ptr(ws), _ptr(d_status), _stream(stream)), "mpr_batch_launch")


def batch_power(chains, ws=None, check=True, stream=None):
    if ws is None:
        ws = workspace(batch_workspace_size(chains), chains[0][0].device)
    st = _status_tensor(chains[0][0].device) if check else None
    batch_plan(chains, ws, stream)
    batch_launch(ws, st, stream)
    if check:
        check_status(st)
    return ws


def batch_graph_create(ws, d_status=None, stream=None):
    g = ctypes.c_void_p()
    _ok(lib().mpr_batch_graph_create(_ptr(ws), _ptr(d_status), _stream(stream), ctypes.byref(g)),
        "mpr_batch_graph_create")
    return g


def graph_launch(graph, stream=None):
    _ok(lib().mpr_graph_launch(graph, _stream(stream)), "mpr_graph_launch")


def graph_destroy(graph):
    _ok(lib().mpr_graph_destroy(graph), "mpr_graph_destroy")


def batch_config_count() -> int:
    return lib().mpr_batch_config_count()


def batch_config_info(cfg: int):
    r, t, a = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _ok(lib().mpr_batch_config_info(cfg, ctypes.byref(r), ctypes.byref(t), ctypes.byref(a)),
        "mpr_batch_config_info")
    return {"panel_rows": r.value, "threads": t.value, "arith": "f16" if a.value == ARITH_F16 else "u16"}


def _arith_code(arith: str) -> int:
    if arith not in ("u16", "f16"):
        raise ValueError("arithmetic is 'u16' or 'f16'")
    return ARITH_F16 if arith == "f16" else ARITH_U16


def set_sparse_arith(arith: str):
    """'u16' (default) or 'f16' for the compressed-K chain steps."""
    _ok(lib().mpr_set_sparse_arith(_arith_code(arith)), "mpr_set_sparse_arith")


SPARSE_FORMS = {"auto": 0, "tiles": 1, "entries": 2}


def set_sparse_form(form: str):
    """'auto' (default), 'tiles' or 'entries': the form of the compressed-K
    chain steps (entries: only the finite entries of A, uint16 only)."""
    if form not in SPARSE_FORMS:
        raise ValueError("sparse form is 'auto', 'tiles' or 'entries'")
    _ok(lib().mpr_set_sparse_form(SPARSE_FORMS[form]), "mpr_set_sparse_form")


def set_arith(arith: str):
    """Process-wide arithmetic of the products the library configures:
    'u16' (packed uint16, the default) or 'f16' (the exact f16 form)."""
    _ok(lib().mpr_set_arith(_arith_code(arith)), "mpr_set_arith")


def get_arith() -> str:
    return "f16" if lib().mpr_get_arith() == ARITH_F16 else "u16"


class arith_scope:
    """with arith_scope('f16'): ... -- sets the process-wide arithmetic and
    restores the previous one (and the u16 compressed-K default) on exit."""

    def __init__(self, arith: str):
        self.arith = arith

    def __enter__(self):
        self.prev = get_arith()
        set_arith(self.arith)
        return self

    def __exit__(self, *exc):
        set_arith(self.prev)
        return False


def set_batch_weights(rel=None):
    """Relative throughput per batched configuration for the schedule model
    (None: the compiled-in values)."""
    cnt = batch_config_count()
    if rel is None:
        _ok(lib().mpr_set_batch_weights(None, cnt), "mpr_set_batch_weights")
        return
    if len(rel) != cnt:
        raise ValueError("one weight per batched configuration (%d)" % cnt)
    arr = (ctypes.c_double * cnt)(*[float(x) for x in rel])
    _ok(lib().mpr_set_batch_weights(arr, cnt), "mpr_set_batch_weights")


def get_batch_weights():
    cnt = batch_config_count()
    arr = (ctypes.c_double * cnt)()
    _ok(lib().mpr_get_batch_weights(arr, cnt), "mpr_get_batch_weights")
    return list(arr)


def batch_plan_info(ws):
    """(configuration, workgroups of the grid, panels) of the plan in ws."""
    v = [ctypes.c_int() for _ in range(3)]
    _ok(lib().mpr_batch_plan_info(_ptr(ws), *[ctypes.byref(x) for x in v]), "mpr_batch_plan_info")
    return tuple(x.value for x in v)


def set_batch_config(cfg: int):
    _ok(lib().mpr_set_batch_config(cfg), "mpr_set_batch_config")


def set_batch_persistent(on: bool):
    """Launch form of later batch plans: one workgroup per panel (default) or
    a persistent grid of the resident workgroups."""
    _ok(lib().mpr_set_batch_persistent(1 if on else 0), "mpr_set_batch_persistent")


# ---------------------------------------------------------------- tiles / tuning
def gemm_config_count() -> int:
    return lib().mpr_gemm_config_count()


def gemm_config_info(cfg: int):
    v = [ctypes.c_int() for _ in range(7)]
    _ok(lib().mpr_gemm_config_info(cfg, *[ctypes.byref(x) for x in v]), "mpr_gemm_config_info")
    d = dict(zip(["bm", "bn", "bk", "tm", "tn", "threads", "arith"], [x.value for x in v]))
    d["arith"] = "f16" if d["arith"] == ARITH_F16 else "u16"
    return d


def gemm_pick_config(M: int, N: int, K: int) -> int:
    return lib().mpr_gemm_pick_config(M, N, K)


def set_tile_table(table):
    """table: list of (max_dim, cfg), ascending max_dim."""
    md = (ctypes.c_int64 * len(table))(*[int(a) for a, _ in table])
    cf = (ctypes.c_int * len(table))(*[int(b) for _, b in table])
    _ok(lib().mpr_set_tile_table(md, cf, len(table)), "mpr_set_tile_table")


def autotune_gemm(n: int, reps: int = 3, stream=None):
    cnt = gemm_config_count()
    ms = (ctypes.c_float * cnt)()
    best = ctypes.c_int()
    _ok(lib().mpr_autotune_gemm(n, reps, ms, ctypes.byref(best), _stream(stream)), "mpr_autotune_gemm")
    return best.value, list(ms)


def valu_probe(arith: str = "u16", iters: int = 20000, stream=None):
    """(pairs per second, shader clock in GHz) of the instruction mix of
    arithmetic form `arith`, measured on the device."""
    r, c = ctypes.c_double(), ctypes.c_double()
    _ok(lib().mpr_valu_probe(_arith_code(arith), iters, ctypes.byref(r), ctypes.byref(c), _stream(stream)),
        "mpr_valu_probe")
    return r.value, c.value
