"""Python binding of libhss.so: the C entry points under the same names.

Argument marshalling only: torch tensors (device memory, streams) are turned
into raw pointers and sizes, host arrays into packed FP64 buffers in the layout
that include/hss.h documents. Every step of the computation runs in the HIP
library; if the library is missing the import fails loudly.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhss.so")

HSS_OK = 0
HSS_ERR_INVALID_ARGUMENT = 1
HSS_ERR_NOT_SPD = 2
HSS_ERR_OUT_OF_MEMORY = 3
HSS_ERR_DEVICE = 4
HSS_ERR_BAD_STATE = 5
HSS_ERR_NOT_CONVERGED = 6
HSS_ERR_UNSUPPORTED = 7

KERNELS = {"exponential": 0, "matern32": 1, "gaussian": 2, "laplace2d": 3, "yukawa": 4}
HSS_P_FP64 = 0
HSS_P_FP32 = 1
HSS_P_BF16 = 2
HSS_P_BF16X3 = 3
HSS_COMPRESS_PLAIN = 0
HSS_COMPRESS_SCALED = 1
MODES = {"plain": HSS_COMPRESS_PLAIN, "scaled": HSS_COMPRESS_SCALED}


class HSSError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {msg} (status {status})")
        self.status = status


class hss_kernel(C.Structure):
    _fields_ = [("kind", C.c_int32), ("length", C.c_double), ("sigma2", C.c_double),
                ("nugget", C.c_double), ("alpha", C.c_double), ("eps", C.c_double)]


_ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_size_t, C.c_void_p)
_FREE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p)


class hss_allocator(C.Structure):
    _fields_ = [("alloc", _ALLOC_FN), ("free", _FREE_FN), ("user", C.c_void_p)]


class hss_construct_opts(C.Structure):
    _fields_ = [("leaf_size", C.c_int32), ("levels", C.c_int32), ("rank", C.c_int32),
                ("max_rank", C.c_int32), ("tol", C.c_double), ("mode", C.c_int32),
                ("rank_model", C.c_void_p), ("sample_start", C.c_int32), ("probes", C.c_int32),
                ("judge_factor", C.c_double)]


class hss_construct_stats(C.Structure):
    _fields_ = [("samples", C.c_int32), ("probes", C.c_int32), ("attempts", C.c_int32),
                ("judge_failures", C.c_int32), ("predicted_max", C.c_int32), ("max_rank", C.c_int32),
                ("sample_bytes", C.c_int64)]


class hss_train_opts(C.Structure):
    _fields_ = [("batch", C.c_int32), ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float), ("tau", C.c_float)]


class hss_factor_opts(C.Structure):
    _fields_ = [("precision", C.c_int32)]


class hss_desc(C.Structure):
    _fields_ = [("n", C.c_int64), ("levels", C.c_int32),
                ("leaf_lo", C.POINTER(C.c_int64)), ("rank", C.POINTER(C.c_int32)),
                ("D", C.POINTER(C.c_double)), ("U", C.POINTER(C.c_double)),
                ("E", C.POINTER(C.c_double)), ("S", C.POINTER(C.c_double)),
                ("perm", C.POINTER(C.c_int64))]


class hss_desc_out(C.Structure):
    _fields_ = [("leaf_lo", C.POINTER(C.c_int64)), ("rank", C.POINTER(C.c_int32)),
                ("D", C.POINTER(C.c_double)), ("U", C.POINTER(C.c_double)),
                ("E", C.POINTER(C.c_double)), ("S", C.POINTER(C.c_double)),
                ("perm", C.POINTER(C.c_int64))]


class hss_info(C.Structure):
    _fields_ = [("n", C.c_int64), ("levels", C.c_int32), ("factored", C.c_int32),
                ("precision", C.c_int32), ("max_rank", C.c_int32), ("failed_level", C.c_int32),
                ("failed_node", C.c_int32), ("failed_pivot", C.c_int32),
                ("bytes_representation", C.c_int64), ("bytes_factor", C.c_int64),
                ("factor_ms", C.c_double), ("solve_ms", C.c_double),
                ("systems", C.c_int32), ("failed_system", C.c_int32), ("promoted_nodes", C.c_int32)]


# Every symbol include/hss.h declares, with its ctypes signature.
_P = C.c_void_p
SIGNATURES = {
    "hss_ctx_create": (C.c_int, [C.c_int32, _P, C.POINTER(hss_allocator), C.POINTER(_P)]),
    "hss_ctx_destroy": (C.c_int, [_P]),
    "hss_ctx_set_stream": (C.c_int, [_P, _P]),
    "hss_construct": (C.c_int, [_P, _P, C.c_int64, C.c_int32, C.POINTER(hss_kernel),
                                C.POINTER(hss_construct_opts), _P, C.c_int32, C.POINTER(_P)]),
    "hss_import": (C.c_int, [_P, C.POINTER(hss_desc), C.POINTER(_P)]),
    "hss_export_sizes": (C.c_int, [_P, C.POINTER(C.c_int64)]),
    "hss_export": (C.c_int, [_P, _P, C.POINTER(hss_desc_out)]),
    "hss_ulv_factor": (C.c_int, [_P, _P, C.POINTER(hss_factor_opts)]),
    "hss_ulv_solve": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.c_int64]),
    "hss_ulv_factor_solve": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.c_int64]),
    "hss_ulv_solve_noalloc": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.c_int64]),
    "hss_ulv_solve_refined": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.c_int64, C.c_double, C.c_int32,
                                        C.POINTER(C.c_int32), C.POINTER(C.c_double)]),
    "hss_matvec": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.c_int64]),
    "hss_logdet": (C.c_int, [_P, _P, C.POINTER(C.c_double)]),
    "hss_blr2_factor": (C.c_int, [_P, _P]),
    "hss_blr2_solve": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.c_int64]),
    "hss_blr2_logdet": (C.c_int, [_P, _P, C.POINTER(C.c_double)]),
    "hss_blr2_stats": (C.c_int, [_P, C.POINTER(C.c_int64), C.POINTER(C.c_float)]),
    "hss_get_info": (C.c_int, [_P, C.POINTER(hss_info)]),
    "hss_get_ranks": (C.c_int, [_P, C.POINTER(C.c_int32), C.c_int64, C.POINTER(C.c_int64)]),
    "hss_get_permutation": (C.c_int, [_P, _P, _P]),
    "hss_debug_node_block": (C.c_int, [_P, _P, C.c_int32, C.c_int32, C.POINTER(C.c_double), C.c_int64]),
    "hss_profile_enable": (C.c_int, [_P, C.c_int32]),
    "hss_profile_read": (C.c_int, [_P, C.c_char_p, C.c_int64, C.POINTER(C.c_int64)]),
    "hss_batch_create": (C.c_int, [_P, C.c_int32, C.POINTER(_P), C.POINTER(_P)]),
    "hss_construct_batched": (C.c_int, [_P, C.c_int32, C.POINTER(_P), C.POINTER(C.c_int64), C.c_int32,
                                        C.POINTER(hss_kernel), C.POINTER(hss_construct_opts), C.POINTER(_P),
                                        C.POINTER(C.c_int32), C.POINTER(_P)]),
    "hss_batch_query": (C.c_int, [_P, _P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                  C.POINTER(C.c_double)]),
    "hss_use_graphs": (C.c_int, [_P, _P, C.c_int32]),
    "hss_autotune": (C.c_int, [_P, _P, C.c_int32, C.c_int32, C.POINTER(C.c_float)]),
    "hss_gemm_variants": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_int32), C.c_int64, C.POINTER(C.c_int64)]),
    "hss_get_construct_stats": (C.c_int, [_P, C.POINTER(hss_construct_stats)]),
    "hss_rankmlp_param_count": (C.c_int, [C.POINTER(C.c_int64)]),
    "hss_rank_features": (C.c_int, [_P, _P, C.c_int64, C.c_int32, C.c_int32, C.c_double, C.c_double,
                                    C.POINTER(C.c_float), C.c_int64, C.POINTER(C.c_int64)]),
    "hss_rankmlp_create": (C.c_int, [_P, C.POINTER(_P)]),
    "hss_rankmlp_destroy": (C.c_int, [_P]),
    "hss_rankmlp_set_weights": (C.c_int, [_P, _P, C.POINTER(C.c_float)]),
    "hss_rankmlp_get_weights": (C.c_int, [_P, _P, C.POINTER(C.c_float)]),
    "hss_rankmlp_forward": (C.c_int, [_P, _P, _P, C.c_int64, _P]),
    "hss_rankmlp_predict": (C.c_int, [_P, _P, _P, C.c_int64, C.c_int32, _P]),
    "hss_rankmlp_grad": (C.c_int, [_P, _P, _P, _P, C.c_int64, C.c_float, C.POINTER(C.c_float),
                                   C.POINTER(C.c_float)]),
    "hss_rankmlp_train": (C.c_int, [_P, _P, _P, _P, C.c_int64, _P, C.c_int64, C.POINTER(hss_train_opts),
                                    C.POINTER(C.c_float)]),
    "hss_set_gemm_variants": (C.c_int, [_P, _P, C.c_int32, C.POINTER(C.c_int32), C.c_int64]),
    "hss_matrix_destroy": (C.c_int, [_P]),
    "hss_status_string": (C.c_char_p, [C.c_int]),
    "hss_last_error": (C.c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Loads libhss.so; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2311_00921_amd.build`")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != HSS_OK:
        lib = load()
        raise HSSError(status, where, lib.hss_last_error().decode())


def _ptr(t) -> int:
    return t.data_ptr()


def _stream_ptr(stream) -> int:
    if stream is None:
        import torch

        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


def _colmajor(t, n):
    """View a (n,) or (n, k) tensor as column-major n x k: returns (tensor, k, ld)."""
    if t.dim() == 1:
        return t.contiguous(), 1, n
    if t.stride(0) == 1 and t.shape[1] == 1:
        return t, 1, n  # one column: its stride is never used
    if t.stride(0) == 1 and t.stride(1) >= n:
        return t, t.shape[1], t.stride(1)
    tc = t.t().contiguous().t()
    return tc, t.shape[1], n


def _require(t, name: str, dtype, dims=(1, 2), rows=None, cols=None):
    """Checks that t is a tensor on a GPU with the given dtype, rank and sizes
    before its address goes to the library (a host pointer or a buffer of the
    wrong element size would be read out of bounds by the kernels)."""
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device (cuda) tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() not in dims:
        raise ValueError(f"{name} must have {' or '.join(map(str, dims))} dimensions, got {t.dim()}")
    if rows is not None and t.shape[0] != rows:
        raise ValueError(f"{name} must have {rows} rows, got {t.shape[0]}")
    if cols is not None and t.dim() == 2 and t.shape[1] != cols:
        raise ValueError(f"{name} must have {cols} columns, got {t.shape[1]}")
    if t.numel() == 0:
        raise ValueError(f"{name} is empty")


def _matrix_n(m) -> int:
    return int(hss_get_info(m).n)


def _vec_args(m, b, x, bname="b", xname="x"):
    """Validates a right-hand side block and an optional output of the same
    shape for a matrix of order N; returns (b column-major, nrhs, ld, x)."""
    import torch

    n = _matrix_n(m)
    _require(b, bname, torch.float64, rows=n)
    bc, k, ld = _colmajor(b, n)
    if x is None:
        x = torch.empty_strided(bc.shape, bc.stride(), dtype=torch.float64, device=b.device)
    else:
        _require(x, xname, torch.float64, rows=n)
        if tuple(x.shape) != tuple(bc.shape) or tuple(x.stride()) != tuple(bc.stride()):
            raise ValueError(f"{xname} must have the shape and strides of {bname} "
                             f"({tuple(bc.shape)}, {tuple(bc.stride())})")
    return bc, k, ld, x


# --------------------------------------------------------------------------
# entry points
# --------------------------------------------------------------------------


# The callbacks of every allocator handed to the library stay referenced for
# the life of the process: blocks may be returned to them until then.
_ALLOCATORS = []


def torch_allocator(device: int = 0, stream=None) -> hss_allocator:
    """An hss_allocator backed by PyTorch's caching allocator on `device`
    (blocks associated with `stream`, default the current stream)."""
    import torch

    def alloc(nbytes, user):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), device=device, stream=stream)
        except Exception:  # out of memory: the library reports it
            return None

    def free(ptr, user):
        torch.cuda.caching_allocator_delete(ptr)

    a, f = _ALLOC_FN(alloc), _FREE_FN(free)
    _ALLOCATORS.append((a, f))
    return hss_allocator(a, f, None)


def hss_ctx_create(device: int = 0, stream=None, allocator="torch"):
    """Context on `device` enqueueing on `stream` (default: torch's current
    stream). allocator "torch" (default): the library's device memory comes from
    PyTorch's caching allocator; None: hipMalloc; or an hss_allocator."""
    lib = load()
    out = C.c_void_p()
    if isinstance(allocator, str):
        if allocator != "torch":
            raise ValueError("allocator must be 'torch', None or an hss_allocator")
        allocator = torch_allocator(device, stream)
    aptr = C.byref(allocator) if allocator is not None else None
    _check(lib.hss_ctx_create(device, _stream_ptr(stream), aptr, C.byref(out)), "hss_ctx_create")
    return out


def hss_ctx_destroy(ctx):
    _check(load().hss_ctx_destroy(ctx), "hss_ctx_destroy")


def hss_ctx_set_stream(ctx, stream):
    _check(load().hss_ctx_set_stream(ctx, _stream_ptr(stream)), "hss_ctx_set_stream")


def pack_desc(h: dict):
    """Packs an HSS matrix given per level (dict with n, levels, ranges, rank,
    D, U, E, S as lists; optional perm) into the heap-ordered hss_desc arrays."""
    L = int(h["levels"])
    n = int(h["n"])
    leaf_lo = np.array([lo for lo, _ in h["ranges"][L]] + [n], dtype=np.int64)
    nnodes = 2 ** (L + 1) - 1
    rank = np.zeros(nnodes, dtype=np.int32)
    for l in range(1, L + 1):
        for i in range(2 ** l):
            rank[2 ** l - 1 + i] = int(h["rank"][l][i])

    def cat(mats):
        if not mats:
            return np.zeros(1)
        return np.concatenate([np.asarray(M, dtype=np.float64).ravel(order="F") for M in mats])

    D = cat(h["D"])
    U = cat(h["U"]) if L > 0 else np.zeros(1)
    E = cat([h["E"][l][i] for l in range(1, L) for i in range(2 ** l)]) if L > 1 else np.zeros(1)
    S = cat([h["S"][l][i] for l in range(L) for i in range(2 ** l)]) if L > 0 else np.zeros(1)
    perm = h.get("perm")
    perm = None if perm is None else np.ascontiguousarray(perm, dtype=np.int64)
    return dict(n=n, levels=L, leaf_lo=leaf_lo, rank=rank, D=D, U=U, E=E, S=S, perm=perm)


def hss_import(ctx, h: dict):
    """Uploads an HSS matrix (see pack_desc for the accepted dict)."""
    lib = load()
    p = pack_desc(h)
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    desc = hss_desc(p["n"], p["levels"], p["leaf_lo"].ctypes.data_as(C.POINTER(C.c_int64)),
                    p["rank"].ctypes.data_as(C.POINTER(C.c_int32)), dp(p["D"]), dp(p["U"]), dp(p["E"]),
                    dp(p["S"]),
                    None if p["perm"] is None else p["perm"].ctypes.data_as(C.POINTER(C.c_int64)))
    out = C.c_void_p()
    _check(lib.hss_import(ctx, C.byref(desc), C.byref(out)), "hss_import")
    return out


def hss_export(ctx, m):
    """Downloads the representation: returns dict(n, levels, leaf_lo, rank (heap
    order), D, U, E, S (packed, heap order as in include/hss.h), perm)."""
    lib = load()
    sizes = (C.c_int64 * 7)()
    _check(lib.hss_export_sizes(m, sizes), "hss_export_sizes")
    leaf_lo = np.zeros(sizes[0], np.int64)
    rank = np.zeros(sizes[1], np.int32)
    D = np.zeros(max(sizes[2], 1))
    U = np.zeros(max(sizes[3], 1))
    E = np.zeros(max(sizes[4], 1))
    S = np.zeros(max(sizes[5], 1))
    perm = np.zeros(sizes[6], np.int64)
    dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    o = hss_desc_out(leaf_lo.ctypes.data_as(C.POINTER(C.c_int64)), rank.ctypes.data_as(C.POINTER(C.c_int32)),
                     dp(D), dp(U), dp(E), dp(S), perm.ctypes.data_as(C.POINTER(C.c_int64)))
    _check(lib.hss_export(ctx, m, C.byref(o)), "hss_export")
    info = hss_get_info(m)
    return dict(n=int(info.n), levels=int(info.levels), leaf_lo=leaf_lo, rank=rank, D=D[:sizes[2]],
                U=U[:sizes[3]], E=E[:sizes[4]], S=S[:sizes[5]], perm=perm)


def unpack_desc(p: dict) -> dict:
    """Inverse of pack_desc: per-level lists from the packed heap-order arrays."""
    L, n = p["levels"], p["n"]
    leaf_lo = p["leaf_lo"]
    rank = p["rank"]
    ranges = [[(int(leaf_lo[i * 2 ** (L - l)]), int(leaf_lo[(i + 1) * 2 ** (L - l)])) for i in range(2 ** l)]
              for l in range(L + 1)]
    rk = [[] for _ in range(L + 1)]
    for l in range(1, L + 1):
        rk[l] = [int(rank[2 ** l - 1 + i]) for i in range(2 ** l)]

    def rows(l, i):
        if l == L:
            lo, hi = ranges[L][i]
            return hi - lo
        return rk[l + 1][2 * i] + rk[l + 1][2 * i + 1]

    D, U, E, S = [], [], [[] for _ in range(max(L, 1))], [[] for _ in range(max(L, 1))]
    o = 0
    for i in range(2 ** L):
        k = rows(L, i)
        D.append(p["D"][o:o + k * k].reshape((k, k), order="F"))
        o += k * k
    if L > 0:
        o = 0
        for i in range(2 ** L):
            k, r = rows(L, i), rk[L][i]
            U.append(p["U"][o:o + k * r].reshape((k, r), order="F"))
            o += k * r
        o = 0
        for l in range(1, L):
            for i in range(2 ** l):
                k, r = rows(l, i), rk[l][i]
                E[l].append(p["E"][o:o + k * r].reshape((k, r), order="F"))
                o += k * r
        o = 0
        for l in range(L):
            for i in range(2 ** l):
                a, b = rk[l + 1][2 * i], rk[l + 1][2 * i + 1]
                S[l].append(p["S"][o:o + a * b].reshape((a, b), order="F"))
                o += a * b
    return dict(n=n, levels=L, ranges=ranges, rank=rk, D=D, U=U, E=E, S=S, perm=p.get("perm"))


def hss_construct(ctx, points, kernel: str, leaf: int, rank: int = 0, tol: float = 0.0, max_rank: int = 0,
                  omega=None, length: float = 1.0, nugget: float = 0.0, sigma2: float = 1.0,
                  alpha: float = 1.0, eps: float = 1e-9, levels: int = 0, rank_model=None,
                  sample_start: int = 0, probes: int = 0, judge_factor: float = 0.0, mode: str = "scaled"):
    """Builds the HSS approximation of the kernel matrix on device points (N x dim,
    row-major); mode "scaled" (SPD for any truncation) or "plain" (the paper's)."""
    import torch

    lib = load()
    _require(points, "points", torch.float64, dims=(2,))
    pts = points.contiguous()
    n, dim = pts.shape
    if not 1 <= dim <= 3:
        raise ValueError(f"points must have 1, 2 or 3 columns, got {dim}")
    _require(omega, "omega", torch.float64, rows=n)
    om, s, ld = _colmajor(omega, n)
    if ld != n:
        om = om.t().contiguous().t()
    k = hss_kernel(KERNELS[kernel], length, sigma2, nugget, alpha, eps)
    o = hss_construct_opts(leaf, levels, rank, max_rank, tol, MODES[mode], rank_model, sample_start,
                           probes, judge_factor)
    out = C.c_void_p()
    _check(lib.hss_construct(ctx, _ptr(pts), n, dim, C.byref(k), C.byref(o), _ptr(om), s, C.byref(out)),
           "hss_construct")
    return out


def hss_ulv_factor(ctx, m, precision: int = HSS_P_FP64):
    o = hss_factor_opts(precision)
    _check(load().hss_ulv_factor(ctx, m, C.byref(o)), "hss_ulv_factor")


def hss_ulv_solve(ctx, m, b, x=None):
    """x = A^{-1} b for a (N,) or (N, nrhs) float64 device tensor b."""
    bc, k, ld, x = _vec_args(m, b, x)
    _check(load().hss_ulv_solve(ctx, m, _ptr(bc), _ptr(x), k, ld), "hss_ulv_solve")
    return x


def hss_ulv_solve_noalloc(ctx, m, b, x):
    """x = A^{-1} b like hss_ulv_solve, with the library allocating nothing: the
    output x must be given (same shape and strides as b)."""
    if x is None:
        raise ValueError("hss_ulv_solve_noalloc needs the output tensor x")
    colmajor = (b.dim() == 1 and b.is_contiguous()) or (
        b.dim() == 2 and b.stride(0) == 1 and (b.shape[1] == 1 or b.stride(1) >= b.shape[0]))
    if not colmajor:
        raise ValueError("hss_ulv_solve_noalloc needs b in column-major layout (a copy would allocate)")
    bc, k, ld, x = _vec_args(m, b, x)
    _check(load().hss_ulv_solve_noalloc(ctx, m, _ptr(bc), _ptr(x), k, ld), "hss_ulv_solve_noalloc")
    return x


def hss_ulv_factor_solve(ctx, m, b, x=None):
    """FP64 factorization and x = A^{-1} b in one call (forward sweep overlapped
    with the factorization); b is a (N,) or (N, nrhs) float64 device tensor."""
    bc, k, ld, x = _vec_args(m, b, x)
    _check(load().hss_ulv_factor_solve(ctx, m, _ptr(bc), _ptr(x), k, ld), "hss_ulv_factor_solve")
    return x


def hss_ulv_solve_refined(ctx, m, b, tol: float, max_iters: int = 50, x=None):
    bc, k, ld, x = _vec_args(m, b, x)
    iters = C.c_int32(0)
    rr = C.c_double(0.0)
    st = load().hss_ulv_solve_refined(ctx, m, _ptr(bc), _ptr(x), k, ld, tol, max_iters, C.byref(iters),
                                      C.byref(rr))
    if st not in (HSS_OK, HSS_ERR_NOT_CONVERGED):
        _check(st, "hss_ulv_solve_refined")
    return x, int(iters.value), float(rr.value), st == HSS_OK


def hss_matvec(ctx, m, x, y=None):
    xc, k, ld, y = _vec_args(m, x, y, "x", "y")
    _check(load().hss_matvec(ctx, m, _ptr(xc), _ptr(y), k, ld), "hss_matvec")
    return y


def hss_logdet(ctx, m) -> float:
    out = C.c_double()
    _check(load().hss_logdet(ctx, m, C.byref(out)), "hss_logdet")
    return float(out.value)


def hss_blr2_factor(ctx, m):
    """BLR^2-ULV factorization (Alg. 1) of the matrix's leaf level."""
    _check(load().hss_blr2_factor(ctx, m), "hss_blr2_factor")


def hss_blr2_solve(ctx, m, b, x=None):
    """x = A^{-1} b with the BLR^2-ULV factors (Eq. 14)."""
    bc, k, ld, x = _vec_args(m, b, x)
    _check(load().hss_blr2_solve(ctx, m, _ptr(bc), _ptr(x), k, ld), "hss_blr2_solve")
    return x


def hss_blr2_logdet(ctx, m) -> float:
    out = C.c_double()
    _check(load().hss_blr2_logdet(ctx, m, C.byref(out)), "hss_blr2_logdet")
    return float(out.value)


def hss_blr2_stats(m):
    """(skeleton matrix order K, GPU milliseconds of the last BLR^2 factorization)."""
    k = C.c_int64()
    ms = C.c_float()
    _check(load().hss_blr2_stats(m, C.byref(k), C.byref(ms)), "hss_blr2_stats")
    return int(k.value), float(ms.value)


def hss_get_info(m) -> hss_info:
    info = hss_info()
    _check(load().hss_get_info(m, C.byref(info)), "hss_get_info")
    return info


def hss_get_ranks(m) -> np.ndarray:
    """Basis rank of every node (heap order for a single matrix; 0 at the root)."""
    lib = load()
    need = C.c_int64(0)
    _check(lib.hss_get_ranks(m, None, 0, C.byref(need)), "hss_get_ranks")
    out = np.zeros(max(1, need.value), dtype=np.int32)
    _check(lib.hss_get_ranks(m, out.ctypes.data_as(C.POINTER(C.c_int32)), out.size, C.byref(need)), "hss_get_ranks")
    return out[:need.value]


def hss_get_permutation(ctx, m, out):
    import torch

    _require(out, "out", torch.int64, dims=(1,), rows=_matrix_n(m))
    _check(load().hss_get_permutation(ctx, m, _ptr(out)), "hss_get_permutation")
    return out


def hss_debug_node_block(ctx, m, node: int, what: int, rows: int, cols: int | None = None) -> np.ndarray:
    """One intermediate block of the factorization as a rows x cols (default
    square) column-major host array; `what` as in include/hss.h."""
    cols = rows if cols is None else cols
    buf = np.zeros(max(rows * cols, 1))
    _check(load().hss_debug_node_block(ctx, m, node, what, buf.ctypes.data_as(C.POINTER(C.c_double)), buf.size),
           "hss_debug_node_block")
    return buf[:rows * cols].reshape((rows, cols), order="F")


def hss_profile_enable(ctx, on: bool):
    _check(load().hss_profile_enable(ctx, 1 if on else 0), "hss_profile_enable")


def hss_profile_read(ctx):
    """Returns {(step, level): (launch groups, total ms)} of the recorded launches."""
    lib = load()
    need = C.c_int64(0)
    _check(lib.hss_profile_read(ctx, None, 0, C.byref(need)), "hss_profile_read")
    buf = C.create_string_buffer(int(need.value) + 1)
    _check(lib.hss_profile_read(ctx, buf, len(buf), C.byref(need)), "hss_profile_read")
    out = {}
    for line in buf.value.decode().splitlines():
        name, level, cnt, ms = line.split()
        out[(name, int(level))] = (int(cnt), float(ms))
    return out


def hss_batch_create(ctx, mats):
    """Batch (forest) of single matrices; the inputs stay valid."""
    arr = (C.c_void_p * len(mats))(*[C.c_void_p(m.value if isinstance(m, C.c_void_p) else m) for m in mats])
    out = C.c_void_p()
    _check(load().hss_batch_create(ctx, len(mats), arr, C.byref(out)), "hss_batch_create")
    return out


def hss_construct_batched(ctx, points_list, kernels, leafs, ranks=None, tols=None, max_ranks=None, omegas=None,
                          lengths=None, nuggets=None, sigma2: float = 1.0, alpha: float = 1.0, eps: float = 1e-9):
    """hss_construct of every system (per-system lists), then one batch."""
    lib = load()
    cnt = len(points_list)
    ranks = ranks or [0] * cnt
    tols = tols or [0.0] * cnt
    max_ranks = max_ranks or [0] * cnt
    import torch

    if len(omegas) != cnt:
        raise ValueError("one omega per system is required")
    for i, (p, om) in enumerate(zip(points_list, omegas)):
        _require(p, f"points[{i}]", torch.float64, dims=(2,))
        _require(om, f"omegas[{i}]", torch.float64, rows=p.shape[0])
        if p.shape[1] != points_list[0].shape[1]:
            raise ValueError("every system must have the same point dimension")
    pts = [p.contiguous() for p in points_list]
    dim = pts[0].shape[1]
    keep = []
    oms, ss = [], []
    for p, om in zip(pts, omegas):
        n = p.shape[0]
        oc, s, ld = _colmajor(om, n)
        if ld != n:
            oc = oc.t().contiguous().t()
        keep.append(oc)
        oms.append(_ptr(oc))
        ss.append(s)
    P = (C.c_void_p * cnt)(*[_ptr(p) for p in pts])
    N = (C.c_int64 * cnt)(*[p.shape[0] for p in pts])
    K = (hss_kernel * cnt)(*[hss_kernel(KERNELS[kernels[i]], lengths[i], sigma2, nuggets[i], alpha, eps)
                             for i in range(cnt)])
    O = (hss_construct_opts * cnt)(*[hss_construct_opts(leafs[i], 0, ranks[i], max_ranks[i], tols[i],
                                                         HSS_COMPRESS_SCALED, None, 0, 0, 0.0) for i in range(cnt)])
    OM = (C.c_void_p * cnt)(*oms)
    S = (C.c_int32 * cnt)(*ss)
    out = C.c_void_p()
    _check(lib.hss_construct_batched(ctx, cnt, P, N, dim, K, O, OM, S, C.byref(out)), "hss_construct_batched")
    return out


def hss_batch_query(ctx, m, count: int, factored: bool = True):
    """Returns (offsets[count + 1], failed[count] or None, logdets[count] or None)."""
    off = (C.c_int64 * (count + 1))()
    if not factored:
        _check(load().hss_batch_query(ctx, m, count, off, None, None), "hss_batch_query")
        return np.array(off[:], dtype=np.int64), None, None
    fl = (C.c_int32 * count)()
    ld = (C.c_double * count)()
    _check(load().hss_batch_query(ctx, m, count, off, fl, ld), "hss_batch_query")
    return np.array(off[:], dtype=np.int64), np.array(fl[:], dtype=np.int32), np.array(ld[:])


def hss_use_graphs(ctx, m, on: bool):
    _check(load().hss_use_graphs(ctx, m, 1 if on else 0), "hss_use_graphs")


GEMM_TILES = ("64x64x16", "32x32x16", "128x64x16", "64x128x16", "32x32x64", "64x64x32", "64x96x16", "96x96x16")


def hss_autotune(ctx, m, precision: int = HSS_P_FP64, reps: int = 2):
    """Tunes the GEMM tile shapes; returns the GEMM ms per factorization for
    each uniform shape (GEMM_TILES order) and for the tuned choice (last)."""
    rep = (C.c_float * (len(GEMM_TILES) + 1))()
    _check(load().hss_autotune(ctx, m, precision, reps, rep), "hss_autotune")
    return list(rep)


def hss_gemm_variants(m, precision: int = HSS_P_FP64):
    lib = load()
    need = C.c_int64(0)
    _check(lib.hss_gemm_variants(m, precision, None, 0, C.byref(need)), "hss_gemm_variants")
    buf = (C.c_int32 * max(1, need.value))()
    _check(lib.hss_gemm_variants(m, precision, buf, need.value, C.byref(need)), "hss_gemm_variants")
    return list(buf[:need.value])


def hss_set_gemm_variants(ctx, m, variants, precision: int = HSS_P_FP64):
    arr = (C.c_int32 * len(variants))(*variants)
    _check(load().hss_set_gemm_variants(ctx, m, precision, arr, len(variants)), "hss_set_gemm_variants")


def hss_get_construct_stats(m) -> hss_construct_stats:
    st = hss_construct_stats()
    _check(load().hss_get_construct_stats(m, C.byref(st)), "hss_get_construct_stats")
    return st


def hss_rankmlp_param_count() -> int:
    n = C.c_int64(0)
    _check(load().hss_rankmlp_param_count(C.byref(n)), "hss_rankmlp_param_count")
    return int(n.value)


def hss_rank_features(ctx, points, leaf: int, length: float, tol: float) -> np.ndarray:
    """Features of the learned rank model for every non-root node (heap order)."""
    import torch

    lib = load()
    _require(points, "points", torch.float64, dims=(2,))
    pts = points.contiguous()
    n, dim = pts.shape
    need = C.c_int64(0)
    _check(lib.hss_rank_features(ctx, _ptr(pts), n, dim, leaf, length, tol, None, 0, C.byref(need)),
           "hss_rank_features")
    out = np.zeros(max(1, need.value), dtype=np.float32)
    _check(lib.hss_rank_features(ctx, _ptr(pts), n, dim, leaf, length, tol,
                                 out.ctypes.data_as(C.POINTER(C.c_float)), out.size, C.byref(need)),
           "hss_rank_features")
    return out[:need.value].reshape(-1, 7)


def hss_rankmlp_create(ctx):
    out = C.c_void_p()
    _check(load().hss_rankmlp_create(ctx, C.byref(out)), "hss_rankmlp_create")
    return out


def hss_rankmlp_destroy(mlp):
    _check(load().hss_rankmlp_destroy(mlp), "hss_rankmlp_destroy")


def pack_mlp_params(params) -> np.ndarray:
    """[(W (out x in), b)] -> packed float32 vector (every W column-major)."""
    parts = []
    for W, b in params:
        parts.append(np.asarray(W, dtype=np.float64).ravel(order="F"))
        parts.append(np.asarray(b, dtype=np.float64).ravel())
    return np.concatenate(parts).astype(np.float32)


def unpack_mlp_params(vec, sizes=(7, 128, 128, 128, 1)):
    out, o = [], 0
    vec = np.asarray(vec)
    for i, j in zip(sizes[:-1], sizes[1:]):
        W = vec[o:o + i * j].reshape((j, i), order="F")
        o += i * j
        b = vec[o:o + j]
        o += j
        out.append((W, b))
    return out


def hss_rankmlp_set_weights(ctx, mlp, params):
    v = pack_mlp_params(params) if isinstance(params, (list, tuple)) else np.ascontiguousarray(params, np.float32)
    _check(load().hss_rankmlp_set_weights(ctx, mlp, v.ctypes.data_as(C.POINTER(C.c_float))), "hss_rankmlp_set_weights")


def hss_rankmlp_get_weights(ctx, mlp) -> np.ndarray:
    v = np.zeros(hss_rankmlp_param_count(), dtype=np.float32)
    _check(load().hss_rankmlp_get_weights(ctx, mlp, v.ctypes.data_as(C.POINTER(C.c_float))), "hss_rankmlp_get_weights")
    return v


def hss_rankmlp_forward(ctx, mlp, feats):
    import torch

    _require(feats, "feats", torch.float32, dims=(2,), cols=7)
    f = feats.contiguous()
    out = torch.empty(f.shape[0], dtype=torch.float32, device=f.device)
    _check(load().hss_rankmlp_forward(ctx, mlp, _ptr(f), f.shape[0], _ptr(out)), "hss_rankmlp_forward")
    return out


def hss_rankmlp_predict(ctx, mlp, feats, cap: int):
    import torch

    _require(feats, "feats", torch.float32, dims=(2,), cols=7)
    f = feats.contiguous()
    out = torch.empty(f.shape[0], dtype=torch.int32, device=f.device)
    _check(load().hss_rankmlp_predict(ctx, mlp, _ptr(f), f.shape[0], cap, _ptr(out)), "hss_rankmlp_predict")
    return out


def hss_rankmlp_grad(ctx, mlp, feats, targets, tau: float = 0.9):
    import torch

    _require(feats, "feats", torch.float32, dims=(2,), cols=7)
    _require(targets, "targets", torch.float32, dims=(1,), rows=feats.shape[0])
    f = feats.contiguous()
    t = targets.contiguous()
    g = np.zeros(hss_rankmlp_param_count(), dtype=np.float32)
    loss = C.c_float(0.0)
    _check(load().hss_rankmlp_grad(ctx, mlp, _ptr(f), _ptr(t), f.shape[0], tau,
                                   g.ctypes.data_as(C.POINTER(C.c_float)), C.byref(loss)), "hss_rankmlp_grad")
    return float(loss.value), g


def hss_rankmlp_train(ctx, mlp, feats, targets, order, batch: int, lr: float = 1e-3, tau: float = 0.9,
                      beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8, record_losses: bool = True):
    import torch

    _require(feats, "feats", torch.float32, dims=(2,), cols=7)
    _require(targets, "targets", torch.float32, dims=(1,), rows=feats.shape[0])
    _require(order, "order", torch.int64, dims=(1,))
    f = feats.contiguous()
    t = targets.contiguous()
    o = order.contiguous()
    steps = (o.shape[0] + batch - 1) // batch
    losses = np.zeros(steps, dtype=np.float32)
    opts = hss_train_opts(batch, lr, beta1, beta2, eps, tau)
    _check(load().hss_rankmlp_train(ctx, mlp, _ptr(f), _ptr(t), f.shape[0], _ptr(o), o.shape[0], C.byref(opts),
                                    losses.ctypes.data_as(C.POINTER(C.c_float)) if record_losses else None),
           "hss_rankmlp_train")
    return losses if record_losses else None


def hss_matrix_destroy(m):
    _check(load().hss_matrix_destroy(m), "hss_matrix_destroy")


def hss_status_string(status: int) -> str:
    return load().hss_status_string(status).decode()


def hss_last_error() -> str:
    return load().hss_last_error().decode()
