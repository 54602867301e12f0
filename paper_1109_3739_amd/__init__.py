"""spx: sparse matrix multiplication, indexing and assignment on an MI355X.

Thin ctypes binding over ``libspx.so`` (the C ABI declared in
``include/spx.h``).  This module only marshals arguments: every step of
every operation runs in the library's HIP kernels.  PyTorch provides device
memory (its caching allocator backs the library's scratch allocations) and
the current HIP stream.

The library is required: :func:`load` raises if ``libspx.so`` has not been
built (``python -m paper_1109_3739_amd.build``); there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspx.so")

# ---- codes (include/spx.h) ---------------------------------------------
SPX_OK, SPX_EINVAL, SPX_ENOMEM, SPX_EOVERFLOW, SPX_EUNSUPPORTED, SPX_EDEVICE = range(6)
CSC, DCSC = 0, 1
PTR_I32, PTR_I64 = 0, 1
VAL_F32, VAL_F64, VAL_I64, VAL_BOOL = 0, 1, 2, 3
SEMIRINGS = {"plus_times": 0, "min_plus": 1, "select2nd": 2, "or_and": 3, "select1st": 4}
ERRORS = {1: "EINVAL", 2: "ENOMEM", 3: "EOVERFLOW", 4: "EUNSUPPORTED", 5: "EDEVICE"}

EXPORTS = [
    "spx_spgemm_plan", "spx_spgemm_exec", "spx_spgemm", "spx_plan_get_info", "spx_plan_destroy", "spx_plan_get_times",
    "spx_default_tuning", "spx_spref_plan", "spx_spref_exec", "spx_spasgn_plan", "spx_spasgn_exec",
    "spx_extend_add_plan", "spx_extend_add_exec", "spx_spgemm_sum_plan", "spx_spgemm_sum_exec",
    "spx_contract_plan", "spx_contract_exec", "spx_spref", "spx_spasgn", "spx_extend_add", "spx_batch_spgemm",
    "spx_count_nonempty", "spx_csc_to_dcsc", "spx_dcsc_to_csc", "spx_check", "spx_last_error", "spx_version",
    "spx_batch_plan", "spx_batch_exec", "spx_batch_capture", "spx_batch_replay", "spx_csc_to_dcsc_noalloc",
]


class SpxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"spx error {ERRORS.get(code, code)}: {msg}")
        self.code = code


class spx_mat(ctypes.Structure):
    _fields_ = [
        ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("nzc", ctypes.c_int64),
        ("fmt", ctypes.c_int32), ("ptr_t", ctypes.c_int32), ("val_t", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("jc", ctypes.c_void_p), ("cp", ctypes.c_void_p), ("ir", ctypes.c_void_p), ("num", ctypes.c_void_p),
    ]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class spx_ctx(ctypes.Structure):
    _fields_ = [
        ("stream", ctypes.c_void_p), ("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p),
        ("validate", ctypes.c_int32), ("profile", ctypes.c_int32),
    ]


class spx_tuning(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in (
        "tiny_max", "hash_count_max", "single_part_max", "part_lds_bytes", "count_threads", "bitmap_threads",
        "part_threads", "single_threads", "bitmap_chunk_log2", "xcd_slices", "bitmap_store_mb", "range_chunk", "bucket_parts", "force_off64")]


class spx_plan_info(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in
                ("mults", "nnz", "nzc", "cols_empty", "cols_tiny", "cols_medium", "cols_heavy", "heavy_parts",
                 "nnz_tiny", "nnz_multi", "multi_parts")]


class spx_times(ctypes.Structure):
    _fields_ = [(k, ctypes.c_float) for k in ("symbolic_ms", "numeric_parts_ms", "numeric_multi_ms", "numeric_tiny_ms",
                                              "pointers_ms")]


_lib = None


def load():
    """Load libspx.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1109_3739_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P, I64, I32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    M = ctypes.POINTER(spx_mat)
    C = ctypes.POINTER(spx_ctx)
    PP = ctypes.POINTER(ctypes.c_void_p)
    PI64 = ctypes.POINTER(ctypes.c_int64)
    sig = {
        "spx_spgemm_plan": ([C, M, M, I32, I32, ctypes.POINTER(spx_tuning), PP, PI64, PI64], ctypes.c_int),
        "spx_spgemm_exec": ([P, M], ctypes.c_int),
        "spx_spgemm": ([C, M, M, I32, I32, M], ctypes.c_int),
        "spx_plan_get_info": ([P, ctypes.POINTER(spx_plan_info)], ctypes.c_int),
        "spx_plan_destroy": ([P], None),
        "spx_plan_get_times": ([P, ctypes.POINTER(spx_times)], ctypes.c_int),
        "spx_default_tuning": ([ctypes.POINTER(spx_tuning)], None),
        "spx_spref_plan": ([C, M, P, I64, P, I64, PP, PI64], ctypes.c_int),
        "spx_spref_exec": ([P, M], ctypes.c_int),
        "spx_spasgn_plan": ([C, M, P, I64, P, I64, M, PP, PI64], ctypes.c_int),
        "spx_spasgn_exec": ([P, M], ctypes.c_int),
        "spx_extend_add_plan": ([C, M, P, I64, P, I64, M, ctypes.c_int32, PP, PI64], ctypes.c_int),
        "spx_extend_add_exec": ([P, M], ctypes.c_int),
        "spx_spgemm_sum_plan": ([C, I32, M, M, I32, I32, ctypes.POINTER(spx_tuning), PP, PI64, PI64], ctypes.c_int),
        "spx_spgemm_sum_exec": ([P, M], ctypes.c_int),
        "spx_contract_plan": ([C, M, P, I64, P, I64, I32, I32, ctypes.POINTER(spx_tuning), PP, PI64, PI64],
                              ctypes.c_int),
        "spx_contract_exec": ([P, M], ctypes.c_int),
        "spx_spref": ([C, M, P, I64, P, I64, M], ctypes.c_int),
        "spx_spasgn": ([C, M, P, I64, P, I64, M, M], ctypes.c_int),
        "spx_extend_add": ([C, M, P, I64, P, I64, M, I32, M], ctypes.c_int),
        "spx_batch_spgemm": ([C, I32, M, M, I32, ctypes.POINTER(spx_tuning), M], ctypes.c_int),
        "spx_count_nonempty": ([C, M, PI64], ctypes.c_int),
        "spx_csc_to_dcsc": ([C, M, M], ctypes.c_int),
        "spx_dcsc_to_csc": ([C, M, M], ctypes.c_int),
        "spx_csc_to_dcsc_noalloc": ([C, M, M, P], ctypes.c_int),
        "spx_check": ([C, M, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
        "spx_batch_plan": ([C, I32, M, M, I32, ctypes.POINTER(spx_tuning), PP, PI64, PI64], ctypes.c_int),
        "spx_batch_exec": ([P, P, P, P, M], ctypes.c_int),
        "spx_batch_capture": ([P, P, P, P, M], ctypes.c_int),
        "spx_batch_replay": ([P], ctypes.c_int),
        "spx_last_error": ([], ctypes.c_char_p),
        "spx_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(rc: int):
    if rc != SPX_OK:
        raise SpxError(rc, _lib.spx_last_error().decode())


# ---- device memory through torch's caching allocator ---------------------
_torch = None


def _t():
    global _torch
    if _torch is None:
        import torch
        _torch = torch
    return _torch


@ALLOC_FN
def _alloc_cb(nbytes, user):
    try:
        torch = _t()
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(),
                                                  torch.cuda.current_stream())
    except Exception:
        return None


@FREE_FN
def _free_cb(ptr, user):
    _t().cuda.caching_allocator_delete(ptr)


def make_ctx(stream=None, validate: bool = False, profile: bool = False) -> spx_ctx:
    torch = _t()
    s = stream if stream is not None else torch.cuda.current_stream()
    return spx_ctx(ctypes.c_void_p(s.cuda_stream), _alloc_cb, _free_cb, None, int(validate), int(profile))


# ---- matrices ------------------------------------------------------------
_VAL_OF = {"float32": VAL_F32, "float64": VAL_F64, "int64": VAL_I64}


@dataclasses.dataclass
class SpMat:
    """A CSC or DCSC matrix held in torch device tensors.

    ``cp``: int32/int64 [n+1] (CSC) or [nzc+1] (DCSC); ``ir``: int32 rows;
    ``num``: values or None (pattern); ``jc``: int32 [nzc] for DCSC.
    """
    m: int
    n: int
    cp: "object"
    ir: "object"
    num: Optional["object"] = None
    jc: Optional["object"] = None
    fmt: int = CSC

    @property
    def nnz(self) -> int:
        return int(self.ir.numel())

    @property
    def nzc(self) -> int:
        return int(self.jc.numel()) if self.jc is not None else 0

    @property
    def val_t(self) -> int:
        return VAL_BOOL if self.num is None else _VAL_OF[str(self.num.dtype).replace("torch.", "")]

    def desc(self) -> spx_mat:
        torch = _t()
        ptr_t = PTR_I64 if self.cp.dtype == torch.int64 else PTR_I32
        return spx_mat(self.m, self.n, self.nnz, self.nzc, self.fmt, ptr_t, self.val_t, 0,
                       _ptr(self.jc), _ptr(self.cp), _ptr(self.ir), _ptr(self.num))

    def to_host(self):
        """(cp, ir, num) as numpy arrays (CSC or DCSC pointers as stored)."""
        torch = _t()
        torch.cuda.synchronize()
        cp = self.cp.cpu().numpy().astype(np.int64)
        ir = self.ir.cpu().numpy()
        num = None if self.num is None else self.num.cpu().numpy()
        return cp, ir, num

    def to_host_csc(self):
        """Host object with m, n, cp (int64 [n+1]), ir, num (expands DCSC)."""
        from types import SimpleNamespace
        cp, ir, num = self.to_host()
        if self.fmt == DCSC:
            jc = self.jc.cpu().numpy()
            full = np.zeros(self.n + 1, dtype=np.int64)
            counts = np.zeros(self.n, dtype=np.int64)
            counts[jc] = np.diff(cp)
            np.cumsum(counts, out=full[1:])
            cp = full
        return SimpleNamespace(m=self.m, n=self.n, cp=cp, ir=ir, num=num)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def from_host(M, device="cuda", ptr_dtype=None, values: bool = True) -> SpMat:
    """Copy a host CSC (object with m, n, cp, ir, num) to the device."""
    torch = _t()
    if ptr_dtype is None:
        ptr_dtype = torch.int64
    cp = torch.from_numpy(np.ascontiguousarray(M.cp, dtype=np.int64)).to(device=device, dtype=ptr_dtype)
    ir = torch.from_numpy(np.ascontiguousarray(M.ir, dtype=np.int32)).to(device)
    num = None
    if values and M.num is not None:
        num = torch.from_numpy(np.ascontiguousarray(M.num)).to(device)
    return SpMat(int(M.m), int(M.n), cp, ir, num)


def _empty(n, dtype):
    torch = _t()
    return torch.empty(max(int(n), 0), dtype=dtype, device="cuda")


_TORCH_VAL = {VAL_F32: "float32", VAL_F64: "float64", VAL_I64: "int64"}


def _val_tensor(val_t, n):
    if val_t == VAL_BOOL:
        return None
    return _empty(n, getattr(_t(), _TORCH_VAL[val_t]))


# ---- SpGEMM --------------------------------------------------------------
def default_tuning() -> spx_tuning:
    t = spx_tuning()
    load().spx_default_tuning(ctypes.byref(t))
    return t


class GemmPlan:
    """Symbolic phase of C = A*B; ``execute()`` runs the numeric phase."""

    def __init__(self, A: SpMat, B: SpMat, semiring: str = "plus_times", out_fmt: int = CSC, tuning=None,
                 stream=None, profile: bool = False, validate: bool = False):
        lib = load()
        self._keep = (A, B)
        self.ctx = make_ctx(stream, validate=validate, profile=profile)
        self.A, self.B = A.desc(), B.desc()
        self.m, self.n, self.out_fmt = A.m, B.n, out_fmt
        self.handle = ctypes.c_void_p()
        nnz, nzc = ctypes.c_int64(), ctypes.c_int64()
        tp = ctypes.byref(tuning) if tuning is not None else None
        _check(lib.spx_spgemm_plan(ctypes.byref(self.ctx), ctypes.byref(self.A), ctypes.byref(self.B),
                                   SEMIRINGS[semiring], out_fmt, tp, ctypes.byref(self.handle), ctypes.byref(nnz),
                                   ctypes.byref(nzc)))
        self.nnz, self.nzc = nnz.value, nzc.value
        self.semiring = semiring
        self.val_t = self._result_val(A, B, semiring)

    @staticmethod
    def _result_val(A, B, semiring):
        if semiring == "or_and":
            return VAL_BOOL
        if semiring == "select2nd":
            return B.val_t
        if semiring == "select1st":
            return A.val_t
        return A.val_t

    def info(self) -> dict:
        inf = spx_plan_info()
        _check(load().spx_plan_get_info(self.handle, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in spx_plan_info._fields_}

    def times(self) -> dict:
        """Per-phase device milliseconds (plan created with profile=True)."""
        t = spx_times()
        _check(load().spx_plan_get_times(self.handle, ctypes.byref(t)))
        return {k: float(getattr(t, k)) for k, _ in spx_times._fields_}

    def alloc_output(self, ptr_dtype=None) -> SpMat:
        torch = _t()
        if ptr_dtype is None:
            ptr_dtype = torch.int64
        ncp = (self.n if self.out_fmt == CSC else self.nzc) + 1
        return SpMat(self.m, self.n, _empty(ncp, ptr_dtype), _empty(self.nnz, torch.int32),
                     _val_tensor(self.val_t, self.nnz),
                     _empty(self.nzc, torch.int32) if self.out_fmt == DCSC else None, self.out_fmt)

    def execute(self, C: Optional[SpMat] = None) -> SpMat:
        if C is None:
            C = self.alloc_output()
        d = C.desc()
        _check(load().spx_spgemm_exec(self.handle, ctypes.byref(d)))
        return C

    def close(self):
        if self.handle:
            load().spx_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def spgemm(A: SpMat, B: SpMat, semiring: str = "plus_times", out_fmt: int = CSC, tuning=None) -> SpMat:
    """C = A*B over ``semiring`` (plan + exec)."""
    p = GemmPlan(A, B, semiring, out_fmt, tuning)
    try:
        return p.execute()
    finally:
        p.close()


# ---- batched SpGEMM ------------------------------------------------------
class StageSumPlan(GemmPlan):
    """C = sum_k A_k * B_k: one processor's Sparse SUMMA stages computed as one
    product over the concatenated inner dimension (see spx_spgemm_sum_plan)."""

    def __init__(self, As, Bs, semiring: str = "plus_times", out_fmt: int = CSC, tuning=None, stream=None,
                 profile: bool = False, validate: bool = False):
        lib = load()
        if len(As) != len(Bs) or not As:
            raise ValueError("need equally many A_k and B_k")
        self._keep = (list(As), list(Bs))
        self.count = len(As)
        self.ctx = make_ctx(stream, validate=validate, profile=profile)
        arr = spx_mat * self.count
        self.A = arr(*[a.desc() for a in As])
        self.B = arr(*[b.desc() for b in Bs])
        self.m, self.n, self.out_fmt = As[0].m, Bs[0].n, out_fmt
        self.handle = ctypes.c_void_p()
        nnz, nzc = ctypes.c_int64(), ctypes.c_int64()
        tp = ctypes.byref(tuning) if tuning is not None else None
        _check(lib.spx_spgemm_sum_plan(ctypes.byref(self.ctx), self.count, self.A, self.B, SEMIRINGS[semiring],
                                       out_fmt, tp, ctypes.byref(self.handle), ctypes.byref(nnz),
                                       ctypes.byref(nzc)))
        self.nnz, self.nzc = nnz.value, nzc.value
        self.semiring = semiring
        self.val_t = self._result_val(As[0], Bs[0], semiring)

    def execute(self, C: Optional[SpMat] = None) -> SpMat:
        if C is None:
            C = self.alloc_output()
        d = C.desc()
        _check(load().spx_spgemm_sum_exec(self.handle, ctypes.byref(d)))
        return C


class ContractPlan(GemmPlan):
    """C = S_r * A * S_c^T for unit aggregation operators S_r(row_agg[u], u),
    S_c(col_agg[v], v) (see spx_contract_plan); None: identity on that side."""

    def __init__(self, A: SpMat, row_agg=None, m_coarse: int = 0, col_agg=None, n_coarse: int = 0,
                 semiring: str = "plus_times", out_fmt: int = CSC, tuning=None, stream=None, profile: bool = False):
        lib = load()
        ra = None if row_agg is None else _idx(row_agg)
        ca = None if col_agg is None else _idx(col_agg)
        self._keep = (A, ra, ca)
        self.ctx = make_ctx(stream, profile=profile)
        self.A = A.desc()
        self.m = A.m if ra is None else int(m_coarse)
        self.n = A.n if ca is None else int(n_coarse)
        self.out_fmt = out_fmt
        self.handle = ctypes.c_void_p()
        nnz, nzc = ctypes.c_int64(), ctypes.c_int64()
        tp = ctypes.byref(tuning) if tuning is not None else None
        _check(lib.spx_contract_plan(ctypes.byref(self.ctx), ctypes.byref(self.A), _ptr(ra), self.m, _ptr(ca),
                                     self.n, SEMIRINGS[semiring], out_fmt, tp, ctypes.byref(self.handle),
                                     ctypes.byref(nnz), ctypes.byref(nzc)))
        self.nnz, self.nzc = nnz.value, nzc.value
        self.semiring = semiring
        self.val_t = VAL_BOOL if semiring == "or_and" else A.val_t

    def execute(self, C: Optional[SpMat] = None) -> SpMat:
        if C is None:
            C = self.alloc_output()
        d = C.desc()
        _check(load().spx_contract_exec(self.handle, ctypes.byref(d)))
        return C


def contract(A: SpMat, row_agg=None, m_coarse: int = 0, col_agg=None, n_coarse: int = 0,
             semiring: str = "plus_times", out_fmt: int = CSC) -> SpMat:
    """C = S_r * A * S_c^T with S(agg[v], v) = 1 on each side given (plan + exec)."""
    p = ContractPlan(A, row_agg, m_coarse, col_agg, n_coarse, semiring, out_fmt)
    try:
        return p.execute()
    finally:
        p.close()


def restriction_map(n: int, order: int, device="cuda"):
    """agg[v] = v // order: the restriction operator of the given order
    (S is ceil(n / order) x n with one unit entry per column)."""
    torch = _t()
    return torch.div(torch.arange(n, dtype=torch.int32, device=device), order, rounding_mode="floor")


def restrict(A: SpMat, order: int, semiring: str = "plus_times", out_fmt: int = CSC) -> SpMat:
    """S * A * S^T for the restriction operator of ``order`` (A square)."""
    if A.m != A.n:
        raise ValueError("restriction on both sides needs a square matrix")
    agg = restriction_map(A.n, order)
    nc = -(-A.n // order)
    return contract(A, agg, nc, agg, nc, semiring, out_fmt)


def spgemm_sum(As, Bs, semiring: str = "plus_times", out_fmt: int = CSC, tuning=None) -> SpMat:
    """C = sum_k A_k * B_k over ``semiring`` (plan + exec)."""
    p = StageSumPlan(As, Bs, semiring, out_fmt, tuning)
    try:
        return p.execute()
    finally:
        p.close()


class BatchPlan:
    """C_i = A_i * B_i for all i in one symbolic pass and one persistent
    numeric launch (see spx_batch_plan).  Outputs are views into pools."""

    def __init__(self, As, Bs, semiring: str = "plus_times", tuning=None, stream=None):
        lib = load()
        if len(As) != len(Bs) or not As:
            raise ValueError("need equally many A_i and B_i")
        self._keep = (list(As), list(Bs))
        self.count = len(As)
        self.ctx = make_ctx(stream)
        arr = spx_mat * self.count
        self.A = arr(*[a.desc() for a in As])
        self.B = arr(*[b.desc() for b in Bs])
        self.handle = ctypes.c_void_p()
        nnz, cpt = ctypes.c_int64(), ctypes.c_int64()
        tp = ctypes.byref(tuning) if tuning is not None else None
        _check(lib.spx_batch_plan(ctypes.byref(self.ctx), self.count, self.A, self.B, SEMIRINGS[semiring], tp,
                                  ctypes.byref(self.handle), ctypes.byref(nnz), ctypes.byref(cpt)))
        self.nnz_total, self.cp_total = nnz.value, cpt.value
        self.val_t = GemmPlan._result_val(As[0], Bs[0], semiring)
        self.shapes = [(a.m, b.n) for a, b in zip(As, Bs)]
        self.pools = None
        self.C = (spx_mat * self.count)()

    def alloc_pools(self):
        torch = _t()
        self.pools = (_empty(self.cp_total, torch.int64), _empty(self.nnz_total, torch.int32),
                      _val_tensor(self.val_t, self.nnz_total))
        return self.pools

    def _views(self):
        cpp, irp, nump = self.pools
        out = []
        for i, (m, n) in enumerate(self.shapes):
            d = self.C[i]
            c0 = (d.cp - cpp.data_ptr()) // 8
            e0 = (d.ir - irp.data_ptr()) // 4 if d.nnz else 0
            out.append(SpMat(m, n, cpp[c0:c0 + n + 1], irp[e0:e0 + d.nnz],
                             None if nump is None else nump[e0:e0 + d.nnz]))
        return out

    def _args(self):
        cpp, irp, nump = self.pools
        return _ptr(cpp), _ptr(irp), _ptr(nump)

    def execute(self):
        if self.pools is None:
            self.alloc_pools()
        _check(load().spx_batch_exec(self.handle, *self._args(), self.C))
        return self._views()

    def capture(self):
        """Record execute() into a HIP graph (on the plan's stream)."""
        if self.pools is None:
            self.alloc_pools()
        _check(load().spx_batch_capture(self.handle, *self._args(), self.C))
        return self._views()

    def replay(self):
        _check(load().spx_batch_replay(self.handle))

    def close(self):
        if self.handle:
            load().spx_plan_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_spgemm(As, Bs, semiring: str = "plus_times", tuning=None):
    """[A_i * B_i for i] through one batch plan; returns views into pools."""
    p = BatchPlan(As, Bs, semiring, tuning)
    try:
        return p.execute()
    finally:
        p.close()


# ---- SpRef / SpAsgn ------------------------------------------------------
def _idx(v):
    torch = _t()
    if isinstance(v, np.ndarray):
        v = torch.from_numpy(np.ascontiguousarray(v, dtype=np.int32))
    return v.to(device="cuda", dtype=torch.int32).contiguous()


def spref(A: SpMat, I, J) -> SpMat:
    """B = A(I, J) (rows / columns in the order of I and J, repeats replicate)."""
    lib = load()
    torch = _t()
    I, J = _idx(I), _idx(J)
    ctx = make_ctx()
    a = A.desc()
    h = ctypes.c_void_p()
    nnz = ctypes.c_int64()
    _check(lib.spx_spref_plan(ctypes.byref(ctx), ctypes.byref(a), _ptr(I), I.numel(), _ptr(J), J.numel(),
                              ctypes.byref(h), ctypes.byref(nnz)))
    try:
        B = SpMat(I.numel(), J.numel(), _empty(J.numel() + 1, torch.int64), _empty(nnz.value, torch.int32),
                  _val_tensor(A.val_t, nnz.value))
        d = B.desc()
        _check(lib.spx_spref_exec(h, ctypes.byref(d)))
    finally:
        lib.spx_plan_destroy(h)
    return B


def spasgn(A: SpMat, I, J, B: SpMat) -> SpMat:
    """C = A with A(I, J) replaced by B (last occurrence of a repeated index wins)."""
    lib = load()
    torch = _t()
    I, J = _idx(I), _idx(J)
    ctx = make_ctx()
    a, b = A.desc(), B.desc()
    h = ctypes.c_void_p()
    nnz = ctypes.c_int64()
    _check(lib.spx_spasgn_plan(ctypes.byref(ctx), ctypes.byref(a), _ptr(I), I.numel(), _ptr(J), J.numel(),
                               ctypes.byref(b), ctypes.byref(h), ctypes.byref(nnz)))
    try:
        C = SpMat(A.m, A.n, _empty(A.n + 1, torch.int64), _empty(nnz.value, torch.int32),
                  _val_tensor(A.val_t, nnz.value))
        d = C.desc()
        _check(lib.spx_spasgn_exec(h, ctypes.byref(d)))
    finally:
        lib.spx_plan_destroy(h)
    return C


def extend_add(A: SpMat, I, J, B: SpMat, semiring: str = "plus_times") -> SpMat:
    """C = A + R*B*Q (A(I, J) = A(I, J) + B); repeated indices accumulate."""
    lib = load()
    torch = _t()
    I, J = _idx(I), _idx(J)
    ctx = make_ctx()
    a, b = A.desc(), B.desc()
    h = ctypes.c_void_p()
    nnz = ctypes.c_int64()
    _check(lib.spx_extend_add_plan(ctypes.byref(ctx), ctypes.byref(a), _ptr(I), I.numel(), _ptr(J), J.numel(),
                                   ctypes.byref(b), SEMIRINGS[semiring], ctypes.byref(h), ctypes.byref(nnz)))
    try:
        C = SpMat(A.m, A.n, _empty(A.n + 1, torch.int64), _empty(nnz.value, torch.int32),
                  _val_tensor(A.val_t, nnz.value))
        d = C.desc()
        _check(lib.spx_extend_add_exec(h, ctypes.byref(d)))
    finally:
        lib.spx_plan_destroy(h)
    return C


# ---- formats -------------------------------------------------------------
def csc_to_dcsc(A: SpMat) -> SpMat:
    lib = load()
    torch = _t()
    ctx = make_ctx()
    a = A.desc()
    nzc = ctypes.c_int64()
    _check(lib.spx_count_nonempty(ctypes.byref(ctx), ctypes.byref(a), ctypes.byref(nzc)))
    out = SpMat(A.m, A.n, _empty(nzc.value + 1, A.cp.dtype), A.ir, A.num, _empty(nzc.value, torch.int32), DCSC)
    d = out.desc()
    _check(lib.spx_csc_to_dcsc(ctypes.byref(ctx), ctypes.byref(a), ctypes.byref(d)))
    return out


def csc_to_dcsc_noalloc(A: SpMat, nzc: int, nzc_dev=None) -> SpMat:
    """CSC -> DCSC through the entry point that allocates nothing itself (its
    scratch is a static device array); ``nzc`` is the number of nonempty
    columns, ``nzc_dev`` an optional device int64 tensor that receives it."""
    lib = load()
    torch = _t()
    ctx = make_ctx()
    a = A.desc()
    out = SpMat(A.m, A.n, _empty(nzc + 1, A.cp.dtype), A.ir, A.num, _empty(nzc, torch.int32), DCSC)
    d = out.desc()
    _check(lib.spx_csc_to_dcsc_noalloc(ctypes.byref(ctx), ctypes.byref(a), ctypes.byref(d), _ptr(nzc_dev)))
    return out


def dcsc_to_csc(A: SpMat) -> SpMat:
    lib = load()
    ctx = make_ctx()
    a = A.desc()
    out = SpMat(A.m, A.n, _empty(A.n + 1, A.cp.dtype), A.ir, A.num, None, CSC)
    d = out.desc()
    _check(lib.spx_dcsc_to_csc(ctypes.byref(ctx), ctypes.byref(a), ctypes.byref(d)))
    return out


def check(A: SpMat) -> bool:
    lib = load()
    ctx = make_ctx()
    a = A.desc()
    ok = ctypes.c_int32()
    _check(lib.spx_check(ctypes.byref(ctx), ctypes.byref(a), ctypes.byref(ok)))
    return bool(ok.value)


def version() -> str:
    return load().spx_version().decode()
