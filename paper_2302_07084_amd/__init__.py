"""Python binding of liblne.so (include/lne.h): argument marshalling only.

Every step of the embedding runs in the library's HIP kernels; this module
turns torch tensors into device pointers, forwards torch's caching allocator
and current stream to the library, and raises on a non-zero status.  It
never falls back to a CPU path: if the library is missing, ``load`` raises.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblne.so")

F64, F32, BF16, U64 = 0, 1, 2, 3
FLAG_NO_FINAL_EIGSVD = 1
FLAG_VANILLA_RSVD = 2
FLAG_SPARSE_OMEGA = 4
FLAG_HOST_SPARSIFIER = 8
_PREC = {"f64": F64, "f32": F32, "bf16": BF16}

STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENUMERIC", -5: "EUNSUPPORTED"}


class LneError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_arcs", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("weight", ctypes.c_void_p), ("index_bits", ctypes.c_int32)]


class Params(ctypes.Structure):
    _fields_ = [("T", ctypes.c_int32), ("s", ctypes.c_double * 16), ("M", ctypes.c_uint64),
                ("b", ctypes.c_uint32), ("C", ctypes.c_double), ("d", ctypes.c_int32),
                ("oversample", ctypes.c_int32), ("q", ctypes.c_int32),
                ("cheb_k", ctypes.c_int32), ("theta", ctypes.c_double),
                ("mu", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("precision", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class CsrStruct(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("val", ctypes.c_void_p),
                ("val_type", ctypes.c_int32)]


class TrialStruct(ctypes.Structure):
    _fields_ = [("s", ctypes.c_double * 16), ("cheb_k", ctypes.c_int32),
                ("theta", ctypes.c_double), ("mu", ctypes.c_double)]


def make_trial(s, k, theta, mu) -> TrialStruct:
    t = TrialStruct()
    for i, x in enumerate(np.asarray(s, np.float64)):
        t.s[i] = float(x)
    t.cheb_k, t.theta, t.mu = int(k), float(theta), float(mu)
    return t


class Stats(ctypes.Structure):
    _fields_ = [("attempted", ctypes.c_uint64), ("accepted", ctypes.c_uint64),
                ("nnz_counts", ctypes.c_uint64), ("nnz_log", ctypes.c_uint64),
                ("shifted", ctypes.c_uint32), ("reserved", ctypes.c_uint32),
                ("entries", ctypes.c_uint64)]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_ if k != "reserved"}


_ALLOC_T = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
_FREE_T = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

# (name, restype, argtypes) of every exported function
_P, _I32, _I64, _U64, _D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                            ctypes.c_double)
SIGNATURES = [
    ("lne_ctx_create", _I32, [_P, _P, _ALLOC_T, _FREE_T, _P]),
    ("lne_ctx_destroy", None, [_P]),
    ("lne_last_error", ctypes.c_char_p, [_P]),
    ("lne_version", ctypes.c_char_p, []),
    ("lne_prof_enable", _I32, [_P, _I32]),
    ("lne_prof_get", _I32, [_P, ctypes.c_char_p, _P, _P]),
    ("lne_prof_reset", _I32, [_P]),
    ("lne_philox", _I32, [_P, _U64, _P, _I64, _P]),
    ("lne_gaussian", _I32, [_P, _I64, _I32, _I64, _U64, _I32, _P]),
    ("lne_sparse_omega", _I32, [_P, _I64, _I32, _U64, _P]),
    ("lne_spmm_sparse_omega", _I32, [_P, _P, _P, _P, _I64, _I32, _I32]),
    ("lne_slots_per_edge", _I64, [_P, _I64]),
    ("lne_sampler_plan", _I32, [_P, _I64, _P, _P, _P]),
    ("lne_sample_slots", _I32, [_P, _P, _P, _I64, _I64, _P, _P, _P, _P]),
    ("lne_sparsify", _I32, [_P, _P, _P, _P, _P]),
    ("lne_trunc_log", _I32, [_P, _P, _P, _P, _P]),
    ("lne_sparsify_log", _I32, [_P, _P, _P, _P, _P]),
    ("lne_csr_copy", _I32, [_P, _P, _P, _P, _P]),
    ("lne_csr_free", None, [_P, _P]),
    ("lne_spmm", _I32, [_P, _P, _P, _I64, _P, _I64, _I32, _I32]),
    ("lne_eigsvd", _I32, [_P, _P, _I64, _I32, _I64, _I32, _P, _I64, _P, _P]),
    ("lne_eigsvd_noalloc", _I32, [_P, _P, _I64, _I32, _I64, _I32, _P, _I64, _P, _P]),
    ("lne_orthonormalize", _I32, [_P, _P, _I64, _I32, _I64, _I32]),
    ("lne_rsvd", _I32, [_P, _P, _P, _P, _P, _P, _P]),
    ("lne_propagate", _I32, [_P, _P, _P, _P, _P]),
    ("lne_graph_spmm", _I32, [_P, _P, _P, _I64, _I32, _I32, ctypes.c_double, ctypes.c_double,
                              _P]),
    ("lne_embed", _I32, [_P, _P, _P, _P, _P]),
    ("lne_sparsify_channels", _I32, [_P, _P, _P, _P, _P]),
    ("lne_trial_matrix", _I32, [_P, _P, _P, _P, _P, _P]),
    ("lne_embed_batch", _I32, [_P, _P, _P, _P, _I32, _P, _P]),
    ("lne_sparsify_rows", _I32, [_P, _P, _P, _I64, _I64, _P, _P]),
    ("lne_batch_create", _I32, [_P, _P, _P, _I32, _P, _P]),
    ("lne_batch_run", _I32, [_P, _P, _I32, _I32, _P, _P]),
    ("lne_batch_info", _I32, [_P, _P, _P, _P, _P]),
    ("lne_batch_resample", _I32, [_P, _P, _P]),
    ("lne_batch_spmm", _I32, [_P, _P, _I32, _P, _I64, _I64, _P, _I64, _I64, _I32]),
    ("lne_batch_destroy", None, [_P]),
    ("lne_mlp_param_count", _I64, [_I32, _I32]),
    ("lne_mlp_init", _I32, [_P, _I32, _I32, _U64, _P]),
    ("lne_mlp_forward", _I32, [_P, _I32, _I32, _P, _P, _I64, _P]),
    ("lne_mlp_grad", _I32, [_P, _I32, _I32, _P, _P, _P, _I64, _P, _P]),
    ("lne_mlp_adam", _I32, [_P, _I64, _P, _P, _P, _P, _I64, ctypes.c_float, ctypes.c_float,
                            ctypes.c_float, ctypes.c_float]),
    ("lne_score_micro_f1", _I32, [_P, _P, _I64, _I32, _P, _I32, _P, _I64, _P, _I64, _I32,
                                  ctypes.c_float, ctypes.c_float, _P]),
    ("lne_score_micro_f1_batch", _I32, [_P, _P, _I32, _I64, _I32, _P, _I32, _P, _I64, _P, _I64,
                                        _I32, ctypes.c_float, ctypes.c_float, _P]),
    ("lne_link_rank", _I32, [_P, _P, _I64, _I32, _I64, _I32, _P, _I64, _P, _I32, _I32, _P, _P,
                             _P]),
    ("lne_graph_stats", _I32, [_P, _P, _U64, _I32, _I32, _P]),
]

_lib = None


def _hip_runtime():
    """Makes one HIP runtime globally visible before liblne binds to it.

    torch carries its own libamdhip64; a second runtime from /opt/rocm in the
    same process would not share torch's device state.  liblne leaves the HIP
    symbols undefined and binds to whichever runtime is promoted here."""
    try:
        import torch  # noqa: F401  (loads torch's HIP runtime)
        from .build import hip_runtime_dir
        path = os.path.join(hip_runtime_dir(), "libamdhip64.so")
        if not os.path.exists(path):
            path = "/opt/rocm/lib/libamdhip64.so"
    except ImportError:
        path = "/opt/rocm/lib/libamdhip64.so"
    ctypes.CDLL(path, mode=os.RTLD_GLOBAL | os.RTLD_NOW)


def load(path: str = LIB_PATH):
    """Loads liblne.so; raises if it is missing (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise ImportError(f"{path} is missing: build it with "
                              "`python -m paper_2302_07084_amd.build` (gfx950 hipcc)")
        _hip_runtime()
        L = ctypes.CDLL(path, mode=os.RTLD_NOW)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def version() -> str:
    return load().lne_version().decode()


def make_params(p: dict, **override) -> Params:
    p = dict(p)
    p.update(override)
    out = Params()
    T = int(p["T"])
    s = np.asarray(p["s"] if p.get("s") is not None else np.full(T, 1.0 / T), dtype=np.float64)
    out.T = T
    for i in range(T):
        out.s[i] = float(s[i])
    out.M = int(p["M"])
    out.b = int(p.get("b", 1))
    C = p.get("C")
    out.C = math.inf if C is None else float(C)
    out.d = int(p.get("d", 1))
    out.oversample = int(p.get("oversample", 0))
    out.q = int(p.get("q", 1))
    out.cheb_k = int(p.get("cheb_k", 0))
    out.theta = float(p.get("theta", 0.0))
    out.mu = float(p.get("mu", 0.0))
    out.seed = int(p.get("seed", 0))
    prec = p.get("precision", "f64")
    out.precision = _PREC[prec] if isinstance(prec, str) else int(prec)
    out.flags = int(p.get("flags", 0))
    return out


def _torch_dtype(code):
    import torch
    return {F64: torch.float64, F32: torch.float32, BF16: torch.bfloat16, U64: torch.int64}[code]


def _code_of(t):
    import torch
    return {torch.float64: F64, torch.float32: F32, torch.bfloat16: BF16}[t.dtype]


class Context:
    """A library context bound to torch's current stream and caching allocator."""

    def __init__(self, device=None, use_torch_allocator: bool = True):
        import torch
        self.L = load()
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.stream = torch.cuda.current_stream(self.device)
        dev_index = self.device.index
        stream = self.stream

        def _alloc(size, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(size), dev_index, stream)
            except Exception:
                return None

        _delete = torch.cuda.caching_allocator_delete

        def _free(ptr, user):
            try:
                _delete(ptr)
            except Exception:   # interpreter shutdown: torch is already torn down
                pass

        if use_torch_allocator:
            self._alloc = _ALLOC_T(_alloc)
            self._free = _FREE_T(_free)
        else:
            self._alloc = ctypes.cast(None, _ALLOC_T)
            self._free = ctypes.cast(None, _FREE_T)
        h = ctypes.c_void_p()
        rc = self.L.lne_ctx_create(ctypes.byref(h), ctypes.c_void_p(stream.cuda_stream),
                                   self._alloc, self._free, None)
        if rc != 0:
            raise LneError(rc, "lne_ctx_create")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.L.lne_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def check(self, rc, what):
        if rc != 0:
            raise LneError(rc, f"{what}: {self.L.lne_last_error(self.h).decode()}")

    # ---- profiling ------------------------------------------------------
    def prof_enable(self, on=True):
        self.check(self.L.lne_prof_enable(self.h, 1 if on else 0), "prof_enable")

    def prof_get(self, name):
        ms = ctypes.c_double()
        cnt = ctypes.c_int64()
        self.check(self.L.lne_prof_get(self.h, name.encode(), ctypes.byref(ms), ctypes.byref(cnt)),
                   "prof_get")
        return ms.value, cnt.value

    def prof_reset(self):
        self.check(self.L.lne_prof_reset(self.h), "prof_reset")


def graph_struct(rowptr, col, weight=None):
    """lne_graph over device tensors (int64 or int32 row offsets, int32
    columns and, for a weighted graph, int32 positive arc weights read as
    uint32)."""
    import torch
    assert rowptr.is_cuda and col.is_cuda
    assert rowptr.dtype in (torch.int64, torch.int32) and col.dtype == torch.int32
    assert rowptr.is_contiguous() and col.is_contiguous()
    g = Graph()
    g.n = rowptr.numel() - 1
    g.n_arcs = col.numel()
    g.row_ptr = rowptr.data_ptr()
    g.index_bits = 32 if rowptr.dtype == torch.int32 else 64
    g.col = col.data_ptr() if col.numel() else None
    g.weight = None
    if weight is not None:
        assert weight.is_cuda and weight.is_contiguous() and weight.numel() == col.numel()
        assert weight.dtype in (torch.int32, torch.uint32)
        g.weight = weight.data_ptr() if weight.numel() else None
    return g


class Csr:
    """A CSR matrix owned by the library (freed with the object)."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self.s = CsrStruct()

    @property
    def nnz(self):
        return int(self.s.nnz)

    def to_torch(self):
        import torch
        n = self.s.n_rows
        rp = torch.empty(n + 1, dtype=torch.int64, device=self.ctx.device)
        col = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=self.ctx.device)
        val = torch.empty(max(self.nnz, 1), dtype=_torch_dtype(self.s.val_type), device=self.ctx.device)
        self.ctx.check(self.ctx.L.lne_csr_copy(self.ctx.h, ctypes.byref(self.s), rp.data_ptr(),
                                               col.data_ptr(), val.data_ptr()), "csr_copy")
        return rp, col[:self.nnz], val[:self.nnz]

    def free(self):
        if self.s.row_ptr:
            self.ctx.L.lne_csr_free(self.ctx.h, ctypes.byref(self.s))

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


# ---- entry points (same names as the C ABI, without the prefix) ----------
def philox(ctx: Context, seed: int, ctr):
    import torch
    out = torch.empty_like(ctr)
    ctx.check(ctx.L.lne_philox(ctx.h, seed, ctr.data_ptr(), ctr.numel() // 4, out.data_ptr()),
              "philox")
    return out


def gaussian(ctx: Context, n: int, k: int, seed: int, dtype=None, ld=None):
    import torch
    dtype = dtype or torch.float64
    ld = ld or k
    out = torch.empty((n, ld), dtype=dtype, device=ctx.device)
    ctx.check(ctx.L.lne_gaussian(ctx.h, n, k, ld, seed, _code_of(out), out.data_ptr()), "gaussian")
    return out[:, :k]


def slots_per_edge(params: dict, n_arcs: int) -> int:
    p = make_params(params)
    return int(load().lne_slots_per_edge(ctypes.byref(p), n_arcs))


def sampler_plan(params: dict, n_arcs: int):
    p = make_params(params)
    base = ctypes.c_uint64()
    thr = ctypes.c_uint64()
    theta = (ctypes.c_uint64 * 16)()
    rc = load().lne_sampler_plan(ctypes.byref(p), n_arcs, ctypes.byref(base), ctypes.byref(thr),
                                 theta)
    if rc != 0:
        raise LneError(rc, "sampler_plan")
    return int(base.value), int(thr.value), np.array(theta[:p.T], dtype=np.uint64)


def sample_slots(ctx: Context, rowptr, col, params: dict, e_begin: int, e_end: int, weight=None):
    import torch
    g = graph_struct(rowptr, col, weight)
    p = make_params(params)
    S = int(ctx.L.lne_slots_per_edge(ctypes.byref(p), g.n_arcs))
    cnt = max((e_end - e_begin) * S, 1)
    dev = ctx.device
    a = torch.empty(cnt, dtype=torch.int32, device=dev)
    b = torch.empty(cnt, dtype=torch.int32, device=dev)
    w = torch.empty(cnt, dtype=torch.int64, device=dev)
    r = torch.empty(cnt, dtype=torch.uint8, device=dev)
    ctx.check(ctx.L.lne_sample_slots(ctx.h, ctypes.byref(g), ctypes.byref(p), e_begin, e_end,
                                     a.data_ptr(), b.data_ptr(), w.data_ptr(), r.data_ptr()),
              "sample_slots")
    k = (e_end - e_begin) * S
    return dict(S=S, a=a[:k], b=b[:k], w=w[:k], r=r[:k])


def sparsify(ctx: Context, rowptr, col, params: dict, weight=None):
    g = graph_struct(rowptr, col, weight)
    p = make_params(params)
    out = Csr(ctx)
    st = Stats()
    ctx.check(ctx.L.lne_sparsify(ctx.h, ctypes.byref(g), ctypes.byref(p), ctypes.byref(out.s),
                                 ctypes.byref(st)), "sparsify")
    return out, st.as_dict()


def sparsify_rows(ctx: Context, rowptr, col, params: dict, row_lo: int, row_hi: int, weight=None):
    """Rows [row_lo, row_hi) of the count matrix (all samples walked)."""
    g = graph_struct(rowptr, col, weight)
    p = make_params(params)
    out = Csr(ctx)
    st = Stats()
    ctx.check(ctx.L.lne_sparsify_rows(ctx.h, ctypes.byref(g), ctypes.byref(p), row_lo, row_hi,
                                      ctypes.byref(out.s), ctypes.byref(st)), "sparsify_rows")
    return out, st.as_dict()


def trunc_log(ctx: Context, rowptr, col, params: dict, counts: Csr, weight=None):
    g = graph_struct(rowptr, col, weight)
    p = make_params(params)
    out = Csr(ctx)
    ctx.check(ctx.L.lne_trunc_log(ctx.h, ctypes.byref(g), ctypes.byref(p), ctypes.byref(counts.s),
                                  ctypes.byref(out.s)), "trunc_log")
    return out


def sparsify_log(ctx: Context, rowptr, col, params: dict, weight=None):
    """The truncated-log matrix as the embedding builds it (lne_sparsify_log)."""
    g = graph_struct(rowptr, col, weight)
    p = make_params(params)
    out = Csr(ctx)
    st = Stats()
    ctx.check(ctx.L.lne_sparsify_log(ctx.h, ctypes.byref(g), ctypes.byref(p),
                                     ctypes.byref(out.s), ctypes.byref(st)), "sparsify_log")
    return out, st.as_dict()


def spmm(ctx: Context, A: Csr, X):
    import torch
    n, k = X.shape
    Y = torch.empty((A.s.n_rows, k), dtype=X.dtype, device=X.device)
    ctx.check(ctx.L.lne_spmm(ctx.h, ctypes.byref(A.s), X.data_ptr(), X.stride(0), Y.data_ptr(),
                             Y.stride(0), k, _code_of(X)), "spmm")
    return Y


def eigsvd(ctx: Context, Y):
    import torch
    n, k = Y.shape
    ut = torch.float32 if Y.dtype == torch.bfloat16 else Y.dtype
    U = torch.empty((n, k), dtype=ut, device=Y.device)
    S = torch.empty(k, dtype=torch.float64, device=Y.device)
    V = torch.empty((k, k), dtype=torch.float64, device=Y.device)
    ctx.check(ctx.L.lne_eigsvd(ctx.h, Y.data_ptr(), n, k, Y.stride(0), _code_of(Y), U.data_ptr(),
                               U.stride(0), S.data_ptr(), V.data_ptr()), "eigsvd")
    return U, S, V


def orthonormalize(ctx: Context, Y):
    n, k = Y.shape
    ctx.check(ctx.L.lne_orthonormalize(ctx.h, Y.data_ptr(), n, k, Y.stride(0), _code_of(Y)),
              "orthonormalize")
    return Y


def rsvd(ctx: Context, M: Csr, params: dict, want=("U", "S", "V", "X0")):
    """Fast (or, with FLAG_VANILLA_RSVD, vanilla) randomized SVD of M:
    (U, S, V, X0); outputs not in `want` are not computed (None)."""
    import torch
    p = make_params(params)
    n, d = M.s.n_rows, p.d
    dt = torch.float64 if p.precision == F64 else torch.float32
    dev = ctx.device
    U = torch.empty((n, d), dtype=dt, device=dev) if "U" in want else None
    V = torch.empty((n, d), dtype=dt, device=dev) if "V" in want else None
    X0 = torch.empty((n, d), dtype=dt, device=dev) if "X0" in want else None
    S = torch.empty(d, dtype=torch.float64, device=dev) if "S" in want else None
    ptr = lambda t: t.data_ptr() if t is not None else None
    ctx.check(ctx.L.lne_rsvd(ctx.h, ctypes.byref(M.s), ctypes.byref(p), ptr(U), ptr(S),
                             ptr(V), ptr(X0)), "rsvd")
    return U, S, V, X0


def propagate(ctx: Context, rowptr, col, params: dict, X0, weight=None):
    import torch
    g = graph_struct(rowptr, col, weight)
    p = make_params(params)
    X = torch.empty_like(X0)
    ctx.check(ctx.L.lne_propagate(ctx.h, ctypes.byref(g), ctypes.byref(p), X0.data_ptr(),
                                  X.data_ptr()), "propagate")
    return X


def graph_spmm(ctx: Context, rowptr, col, Z, a: float, b: float, weight=None):
    """out = a Z + b D^-1 A Z (one product of the propagation recurrence).
    Z: device n x k (row stride a multiple of 16 bytes), F64 or F32."""
    import torch
    g = graph_struct(rowptr, col, weight)
    n, k = Z.shape
    out = torch.empty((n, Z.stride(0)), dtype=Z.dtype, device=Z.device)[:, :k]
    ctx.check(ctx.L.lne_graph_spmm(ctx.h, ctypes.byref(g), Z.data_ptr(), Z.stride(0), k,
                                   _code_of(Z), ctypes.c_double(a), ctypes.c_double(b),
                                   out.data_ptr()), "graph_spmm")
    return out


def embed(ctx: Context, rowptr, col, params: dict, out=None, weight=None):
    import torch
    g = graph_struct(rowptr, col, weight)
    p = make_params(params)
    dt = torch.float64 if p.precision == F64 else torch.float32
    X = out if out is not None else torch.empty((g.n, p.d), dtype=dt, device=ctx.device)
    st = Stats()
    ctx.check(ctx.L.lne_embed(ctx.h, ctypes.byref(g), ctypes.byref(p), X.data_ptr(),
                              ctypes.byref(st)), "embed")
    return X, st.as_dict()


# ---- batched trials ----------------------------------------------------------
def sparsify_channels(ctx: Context, rowptr, col, params: dict):
    g = graph_struct(rowptr, col)
    p = make_params(params)
    out = Csr(ctx)
    st = Stats()
    ctx.check(ctx.L.lne_sparsify_channels(ctx.h, ctypes.byref(g), ctypes.byref(p),
                                          ctypes.byref(out.s), ctypes.byref(st)),
              "sparsify_channels")
    return out, st.as_dict()


def trial_matrix(ctx: Context, rowptr, col, params: dict, channels: Csr, trial: dict):
    g = graph_struct(rowptr, col)
    p = make_params(params)
    t = make_trial(trial["s"], trial.get("k", 0), trial.get("theta", 0.0), trial.get("mu", 0.0))
    out = Csr(ctx)
    ctx.check(ctx.L.lne_trial_matrix(ctx.h, ctypes.byref(g), ctypes.byref(p),
                                     ctypes.byref(channels.s), ctypes.byref(t),
                                     ctypes.byref(out.s)), "trial_matrix")
    return out


def _trial_array(trials):
    return (TrialStruct * len(trials))(*[make_trial(t["s"], t["k"], t["theta"], t["mu"])
                                         for t in trials])


def embed_batch(ctx: Context, rowptr, col, params: dict, trials):
    """Embeddings of several trials (dicts with s, k, theta, mu) from one
    shared sampling pass; returns (n_trials x n x d FP32, stats)."""
    import torch
    g = graph_struct(rowptr, col)
    p = make_params(params, precision="f32")
    arr = _trial_array(trials)
    X = torch.empty((len(trials), g.n, p.d), dtype=torch.float32, device=ctx.device)
    st = Stats()
    ctx.check(ctx.L.lne_embed_batch(ctx.h, ctypes.byref(g), ctypes.byref(p), arr, len(trials),
                                    X.data_ptr(), ctypes.byref(st)), "embed_batch")
    return X, st.as_dict()


BATCH_EAGER, BATCH_GRAPH = 0, 1


class Batch:
    """Persistent per-graph state of the batched trials (lne_batch_*): one
    channel sampling pass at construction (lengths drawn from params["s"]),
    then any number of runs of up to `max_trials` trials.  Holds references
    to the graph tensors, which the library reads on every run."""

    def __init__(self, ctx: Context, rowptr, col, params: dict, max_trials: int):
        self.ctx = ctx
        self._rp, self._col = rowptr, col
        self._g = graph_struct(rowptr, col)
        self._p = make_params(params, precision="f32")
        self.max_trials = max_trials
        self.h = ctypes.c_void_p()
        st = Stats()
        ctx.check(ctx.L.lne_batch_create(ctx.h, ctypes.byref(self._g), ctypes.byref(self._p),
                                         max_trials, ctypes.byref(self.h), ctypes.byref(st)),
                  "batch_create")
        self.stats = st.as_dict()

    def run(self, trials, graph: bool = False, out=None):
        import torch
        n, d = self._g.n, self._p.d
        X = out if out is not None else torch.empty((len(trials), n, d), dtype=torch.float32,
                                                    device=self.ctx.device)
        arr = _trial_array(trials)
        st = Stats()
        self.ctx.check(self.ctx.L.lne_batch_run(self.h, arr, len(trials),
                                                BATCH_GRAPH if graph else BATCH_EAGER,
                                                X.data_ptr(), ctypes.byref(st)), "batch_run")
        return X, st.as_dict()

    def resample(self, pi):
        """New channel pass with length distribution pi (the trials' s must
        be covered by it)."""
        T = self._p.T
        arr = (ctypes.c_double * 16)(*[float(x) for x in np.asarray(pi, np.float64)[:T]])
        st = Stats()
        self.ctx.check(self.ctx.L.lne_batch_resample(self.h, arr, ctypes.byref(st)),
                       "batch_resample")
        for i in range(T):
            self._p.s[i] = arr[i]
        self.stats = st.as_dict()
        return self.stats

    def spmm(self, trials, X):
        """Y[t] = M_t X[t] (X: n_trials x n x k, or n x k shared by all trials)."""
        import torch
        X = X.contiguous()
        k = X.shape[-1]
        n = self._g.n
        xs = 0 if X.dim() == 2 else n * k
        Y = torch.empty((len(trials), n, k), dtype=torch.float32, device=X.device)
        arr = _trial_array(trials)
        self.ctx.check(self.ctx.L.lne_batch_spmm(self.h, arr, len(trials), X.data_ptr(), k, xs,
                                                 Y.data_ptr(), k, n * k, k), "batch_spmm")
        return Y

    def info(self):
        sv, gv, cap = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        nnz = ctypes.c_int64()
        self.ctx.check(self.ctx.L.lne_batch_info(self.h, ctypes.byref(sv), ctypes.byref(gv),
                                                 ctypes.byref(nnz), ctypes.byref(cap)),
                       "batch_info")
        return {"spmm_variant": sv.value, "graph_spmm_variant": gv.value,
                "channel_nnz": nnz.value, "graph_captures": cap.value}

    def close(self):
        if self.h:
            self.ctx.L.lne_batch_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- surrogate network and scorer ------------------------------------------
def mlp_param_count(in_dim: int, hidden: int) -> int:
    return int(load().lne_mlp_param_count(in_dim, hidden))


def mlp_init(ctx: Context, in_dim: int, hidden: int, seed: int):
    import torch
    p = torch.empty(mlp_param_count(in_dim, hidden), dtype=torch.float32, device=ctx.device)
    ctx.check(ctx.L.lne_mlp_init(ctx.h, in_dim, hidden, seed, p.data_ptr()), "mlp_init")
    return p


def mlp_forward(ctx: Context, in_dim: int, hidden: int, params, X):
    import torch
    X = X.contiguous()
    y = torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    ctx.check(ctx.L.lne_mlp_forward(ctx.h, in_dim, hidden, params.data_ptr(), X.data_ptr(),
                                    X.shape[0], y.data_ptr()), "mlp_forward")
    return y


def mlp_grad(ctx: Context, in_dim: int, hidden: int, params, X, target):
    import torch
    X = X.contiguous()
    t = target.contiguous()
    g = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    ctx.check(ctx.L.lne_mlp_grad(ctx.h, in_dim, hidden, params.data_ptr(), X.data_ptr(),
                                 t.data_ptr(), X.shape[0], g.data_ptr(), loss.data_ptr()),
              "mlp_grad")
    return g, loss


def mlp_adam(ctx: Context, params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999,
             eps=1e-8):
    ctx.check(ctx.L.lne_mlp_adam(ctx.h, params.numel(), params.data_ptr(), grad.data_ptr(),
                                 m.data_ptr(), v.data_ptr(), step, lr, beta1, beta2, eps),
              "mlp_adam")


def score_micro_f1(ctx: Context, X, labels, train, test, epochs=300, lr=0.05, l2=None):
    """micro-F1 of one-vs-rest logistic regression trained on rows `train`.
    X: n x d (one embedding, returns a float) or t x n x d (returns a list)."""
    import torch
    # every converted tensor stays referenced until the library call returns:
    # a temporary would go back to torch's allocator, which the library's own
    # scratch allocation may then reuse
    Xf = X.float().contiguous()
    lab = labels.to(torch.uint8).contiguous()
    tr = train.to(torch.int32).contiguous()
    te = test.to(torch.int32).contiguous()
    single = Xf.dim() == 2
    ntr = 1 if single else Xf.shape[0]
    n, d = Xf.shape[-2:]
    L = lab.shape[1]
    l2 = (1.0 / len(tr)) if l2 is None else l2
    f1 = (ctypes.c_double * ntr)()
    ctx.check(ctx.L.lne_score_micro_f1_batch(ctx.h, Xf.data_ptr(), ntr, n, d, lab.data_ptr(), L,
                                             tr.data_ptr(), len(tr), te.data_ptr(), len(te),
                                             epochs, lr, l2, f1), "score_micro_f1")
    return f1[0] if single else list(f1)


def graph_stats(ctx: Context, rowptr, col, seed: int = 0, wedges: int = 2000, iters: int = 200):
    """The eight graph descriptors of lne_graph_stats (log n, log m, log mean
    degree, degree coefficient of variation, log max degree, Hill tail
    exponent, wedge clustering, spectral gap) as a numpy array."""
    out = (ctypes.c_double * 8)()
    g = graph_struct(rowptr, col)
    ctx.check(ctx.L.lne_graph_stats(ctx.h, ctypes.byref(g), seed, wedges, iters, out),
              "graph_stats")
    return np.array(list(out))


def link_rank(ctx: Context, X, pos, neg, hits_k: int = 10):
    """Link-prediction ranks of held-out edges pos (h x 2) against corrupted
    edges (u, neg[i, j]) (neg: h x K) by embedding inner products.  Returns
    (metrics dict: mean_rank, mrr, hits, auc; above; ties), the last two as
    device uint32 tensors (per edge: corrupted edges scoring above / equal)."""
    import torch
    assert X.dim() == 2 and X.stride(1) == 1 and X.dtype in (torch.float32, torch.float64)
    p = pos.to(torch.int32).contiguous()
    q = neg.to(torch.int32).contiguous()
    h, K = q.shape
    assert p.shape == (h, 2)
    above = torch.empty(h, dtype=torch.int32, device=X.device)
    ties = torch.empty(h, dtype=torch.int32, device=X.device)
    m = torch.empty(4, dtype=torch.float64, device=X.device)
    ctx.check(ctx.L.lne_link_rank(ctx.h, X.data_ptr(), X.shape[0], X.shape[1], X.stride(0),
                                  _code_of(X), p.data_ptr(), h, q.data_ptr(), K, hits_k,
                                  above.data_ptr(), ties.data_ptr(), m.data_ptr()), "link_rank")
    mv = m.cpu().tolist()
    return (dict(mean_rank=mv[0], mrr=mv[1], hits=mv[2], auc=mv[3]), above, ties)


def sparse_omega(ctx: Context, n: int, k: int, seed: int):
    """Sparse-sign test matrix: (n, 8) int16 entries sign * (column + 1)."""
    import torch
    out = torch.empty((n, 8), dtype=torch.int16, device=ctx.device)
    ctx.check(ctx.L.lne_sparse_omega(ctx.h, n, k, seed, out.data_ptr()), "sparse_omega")
    return out


def spmm_sparse_omega(ctx: Context, A: Csr, om, k: int, dtype=None):
    """Y = A Omega for a sparse-sign Omega (sparse_omega)."""
    import torch
    dtype = dtype or (torch.float64 if A.s.val_type == F64 else torch.float32)
    Y = torch.empty((A.s.n_rows, k), dtype=dtype, device=ctx.device)
    ctx.check(ctx.L.lne_spmm_sparse_omega(ctx.h, ctypes.byref(A.s), om.data_ptr(), Y.data_ptr(),
                                          Y.stride(0), k, _code_of(Y)), "spmm_sparse_omega")
    return Y

