"""Python binding of libfemasm.so (argument marshalling only).

The functions named ``fem_*`` mirror the C ABI in include/femasm.h one to
one and take raw device pointers (ints) and a stream handle.  The small
classes below (:class:`Plan`, :class:`Batch`) only allocate torch tensors for
outputs and pass their pointers through; every step of the assembly runs in
the HIP library.  There is no CPU fallback: if the shared library is missing
or no GPU is visible, loading raises :class:`FemasmUnavailable`.
"""
from __future__ import annotations

import ctypes as C
import functools
import inspect
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfemasm.so")

FEM_OP = {"MASS": 0, "MASS_W": 1, "STIFF": 2, "ELAS": 3}
# pair layouts the library builds by default: (rows per 3D block, rows per 2D
# block, tasks per wavefront) of the scalar operators and of elasticity
PAIR_LAYOUT_DEFAULT = {0: (64, 128, 2), 1: (64, 128, 2)}
FEM_STATUS = {0: "FEM_OK", 1: "FEM_ERR_ARG", 2: "FEM_ERR_INDEX", 3: "FEM_ERR_DEGENERATE",
              4: "FEM_ERR_OVERFLOW", 5: "FEM_ERR_NOMEM", 6: "FEM_ERR_DEVICE"}


class FemasmUnavailable(RuntimeError):
    pass


class FemError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        self.name = FEM_STATUS.get(code, f"status {code}")
        super().__init__(f"{where}: {self.name}")


_lib = None
P = C.c_void_p
I32 = C.c_int32
I64 = C.c_int64
U32 = C.c_uint32
D = C.c_double

_SIGS = {
    "fem_status_str": ([C.c_int], C.c_char_p),
    "fem_assemble_symbolic": ([I32, I64, I64, P, P, C.POINTER(P)], C.c_int),
    "fem_plan_layouts": ([P, I32, C.POINTER(I32)], C.c_int),
    "fem_plan_query": ([P, I32, C.POINTER(I64), C.POINTER(I64)], C.c_int),
    "fem_plan_info": ([P, C.POINTER(I32), C.POINTER(I64), C.POINTER(I64), C.POINTER(I32)], C.c_int),
    "fem_plan_pattern": ([P, I32, P, P, P], C.c_int),
    "fem_plan_slot_map": ([P, P, P], C.c_int),
    "fem_plan_vjp_positions": ([P, P], C.c_int),
    "fem_assemble_numeric": ([P, I32, P, P, D, D, P, P], C.c_int),
    "fem_assemble_elasticity_nodal": ([P, P, P, P, P, P], C.c_int),
    "fem_assemble_general": ([P, P, P, P, P], C.c_int),
    "fem_assemble_jvp": ([P, I32, P, P, P, P, P, P], C.c_int),
    "fem_assemble_vjp": ([P, I32, P, P, P, P, P, P, P], C.c_int),
    "fem_vjp_work_bytes": ([P, I32, C.POINTER(I64)], C.c_int),
    "fem_assemble_vjp_ws": ([P, I32, P, P, P, P, P, I64, P, P, P], C.c_int),
    "fem_assemble_vjp_noalloc": ([P, I32, P, P, P, P, P, P, P], C.c_int),
    "fem_assemble_backward": ([P, U32, P, P, P, P, P, P, P], C.c_int),
    "fem_csr_bilinear": ([P, I32, P, P, P, P, P], C.c_int),
    "fem_plan_sync_status": ([P, P], C.c_int),
    "fem_plan_destroy": ([P], None),
    "fem_batch_create": ([I32, P, P, P, P, P, C.POINTER(P)], C.c_int),
    "fem_batch_offsets": ([P, I32, P, P, P, P], C.c_int),
    "fem_batch_plan": ([P, I32, C.POINTER(P)], C.c_int),
    "fem_batch_set_params": ([P, I32, I32], C.c_int),
    "fem_batch_set_kernel": ([P, I32], C.c_int),
    "fem_batch_set_pair_layout": ([P, I32, I32, I32, I32], C.c_int),
    "fem_batch_numeric": ([P, I32, P, P, D, D, P, P], C.c_int),
    "fem_batch_sync_status": ([P, P], C.c_int),
    "fem_batch_destroy": ([P], None),
    "fem_pk_symbolic": ([I32, I32, I64, I64, P, P, C.POINTER(P)], C.c_int),
    "fem_pk_query": ([P, C.POINTER(I64), C.POINTER(I64), C.POINTER(I32)], C.c_int),
    "fem_pk_pattern": ([P, P, P, P], C.c_int),
    "fem_pk_mass": ([P, P, P, P], C.c_int),
    "fem_pk_sync_status": ([P, P], C.c_int),
    "fem_pk_destroy": ([P], None),
    "fem_boundary_symbolic": ([I32, I64, I64, P, P, C.POINTER(P)], C.c_int),
    "fem_boundary_mass": ([P, P, P, P, P], C.c_int),
}

EXPORTED = tuple(_SIGS)


def load_library(require_gpu: bool = True):
    """Load libfemasm.so (raises FemasmUnavailable if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise FemasmUnavailable(f"{LIB_PATH} is not built; run python -m paper_1401_3301_amd.build")
    if require_gpu and not torch.cuda.is_available():
        raise FemasmUnavailable("no GPU visible: the HIP library has no CPU path")
    lib = C.CDLL(LIB_PATH)
    for name, (args, res) in _SIGS.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def _check(st: int, where: str):
    if st != 0:
        raise FemError(st, where)


def _stream(stream=None) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


# ---------------------------------------------------------------- raw ABI
def fem_status_str(code: int) -> str:
    return load_library().fem_status_str(code).decode()


def fem_assemble_symbolic(d: int, nq: int, nme: int, me_ptr: int, stream=None) -> int:
    out = P()
    _check(load_library().fem_assemble_symbolic(d, nq, nme, me_ptr, _stream(stream), C.byref(out)),
           "fem_assemble_symbolic")
    return out.value


def fem_plan_layouts(plan: int, wait: bool = False) -> int:
    """State of the plan's block layouts (0 building, 1 ready, 2 none)."""
    st = I32()
    _check(load_library().fem_plan_layouts(plan, 1 if wait else 0, C.byref(st)), "fem_plan_layouts")
    return st.value


def fem_plan_query(plan: int, op: int):
    nr, nz = I64(), I64()
    _check(load_library().fem_plan_query(plan, op, C.byref(nr), C.byref(nz)), "fem_plan_query")
    return nr.value, nz.value


def fem_plan_info(plan: int):
    d, nq, nme, mr = I32(), I64(), I64(), I32()
    _check(load_library().fem_plan_info(plan, C.byref(d), C.byref(nq), C.byref(nme), C.byref(mr)),
           "fem_plan_info")
    return d.value, nq.value, nme.value, mr.value


def fem_plan_pattern(plan: int, op: int, row_ptr: int, col_idx: int, stream=None):
    _check(load_library().fem_plan_pattern(plan, op, row_ptr, col_idx, _stream(stream)),
           "fem_plan_pattern")


def fem_plan_slot_map(plan: int, slot: int, stream=None):
    _check(load_library().fem_plan_slot_map(plan, slot, _stream(stream)), "fem_plan_slot_map")


def fem_plan_vjp_positions(plan: int, stream=None):
    _check(load_library().fem_plan_vjp_positions(plan, _stream(stream)), "fem_plan_vjp_positions")


def fem_assemble_numeric(plan: int, op: int, q: int, w: int | None, lam: float, mu: float,
                         values: int, stream=None):
    _check(load_library().fem_assemble_numeric(plan, op, q, w, lam, mu, values, _stream(stream)),
           "fem_assemble_numeric")


def fem_assemble_elasticity_nodal(plan: int, q: int, lam: int, mu: int, values: int, stream=None):
    _check(load_library().fem_assemble_elasticity_nodal(plan, q, lam, mu, values, _stream(stream)),
           "fem_assemble_elasticity_nodal")


def fem_assemble_general(plan: int, q: int, coef, values: int, stream=None):
    """coef: host sequence of d*d + 2*d + 1 doubles (A row-major, b, c, a0)."""
    arr = (D * len(coef))(*[float(x) for x in coef])
    _check(load_library().fem_assemble_general(plan, q, arr, values, _stream(stream)),
           "fem_assemble_general")


def fem_assemble_jvp(plan: int, op: int, q: int, w: int | None, dq: int, dw: int | None,
                     dvalues: int, stream=None):
    _check(load_library().fem_assemble_jvp(plan, op, q, w, dq, dw, dvalues, _stream(stream)),
           "fem_assemble_jvp")


def fem_assemble_vjp(plan: int, op: int, q: int, w: int | None, G: int, slot: int,
                     dLdq: int | None, dLdw: int | None, stream=None):
    _check(load_library().fem_assemble_vjp(plan, op, q, w, G, slot, dLdq, dLdw, _stream(stream)),
           "fem_assemble_vjp")


def fem_assemble_vjp_noalloc(plan: int, op: int, q: int, w: int | None, G: int, slot: int,
                             dLdq: int, dLdw: int | None, stream=None):
    _check(load_library().fem_assemble_vjp_noalloc(plan, op, q, w, G, slot, dLdq, dLdw,
                                                   _stream(stream)), "fem_assemble_vjp_noalloc")


def fem_vjp_work_bytes(plan: int, op: int) -> int:
    n = I64(0)
    _check(load_library().fem_vjp_work_bytes(plan, op, C.byref(n)), "fem_vjp_work_bytes")
    return int(n.value)


def fem_assemble_vjp_ws(plan: int, op: int, q: int, w: int | None, G: int, slot: int, work: int,
                        work_bytes: int, dLdq: int | None, dLdw: int | None, stream=None):
    _check(load_library().fem_assemble_vjp_ws(plan, op, q, w, G, slot, work, work_bytes, dLdq,
                                              dLdw, _stream(stream)), "fem_assemble_vjp_ws")


def fem_assemble_backward(plan: int, op_mask: int, q: int, w: int | None, a: int, b: int,
                          dJdw: int | None, dJdq: int | None, stream=None):
    _check(load_library().fem_assemble_backward(plan, op_mask, q, w, a, b, dJdw, dJdq,
                                                _stream(stream)), "fem_assemble_backward")


def fem_csr_bilinear(plan: int, op: int, values: int, a: int, b: int, out: int, stream=None):
    _check(load_library().fem_csr_bilinear(plan, op, values, a, b, out, _stream(stream)),
           "fem_csr_bilinear")


def fem_plan_sync_status(plan: int, stream=None) -> int:
    return load_library().fem_plan_sync_status(plan, _stream(stream))


def fem_plan_destroy(plan: int):
    if plan:
        load_library().fem_plan_destroy(plan)


def fem_batch_create(d, nq, nme, me_ptrs, stream=None) -> int:
    n = len(d)
    arr_d = (I32 * n)(*d)
    arr_nq = (I64 * n)(*nq)
    arr_nme = (I64 * n)(*nme)
    arr_me = (P * n)(*me_ptrs)
    out = P()
    _check(load_library().fem_batch_create(n, arr_d, arr_nq, arr_nme, arr_me, _stream(stream),
                                           C.byref(out)), "fem_batch_create")
    return out.value


def fem_batch_offsets(batch: int, op: int, nmesh: int):
    arrs = [(I64 * (nmesh + 1))() for _ in range(4)]
    _check(load_library().fem_batch_offsets(batch, op, *arrs), "fem_batch_offsets")
    return [list(a) for a in arrs]


def fem_batch_plan(batch: int, index: int) -> int:
    out = P()
    _check(load_library().fem_batch_plan(batch, index, C.byref(out)), "fem_batch_plan")
    return out.value


def fem_batch_set_params(batch: int, block_threads: int, wg_per_cu: int):
    _check(load_library().fem_batch_set_params(batch, block_threads, wg_per_cu),
           "fem_batch_set_params")


FEM_BATCH_KERNEL = {"rowgather": 0, "pair": 1, "pair_split": 2}


def fem_batch_set_kernel(batch: int, kernel: int):
    _check(load_library().fem_batch_set_kernel(batch, kernel), "fem_batch_set_kernel")


def fem_batch_set_pair_layout(batch: int, op: int, rows_3d: int, rows_2d: int, slots: int):
    _check(load_library().fem_batch_set_pair_layout(batch, op, rows_3d, rows_2d, slots),
           "fem_batch_set_pair_layout")


def fem_batch_numeric(batch: int, op: int, q_cat: int, w_cat: int | None, lam: float, mu: float,
                      values_cat: int, stream=None):
    _check(load_library().fem_batch_numeric(batch, op, q_cat, w_cat, lam, mu, values_cat,
                                            _stream(stream)), "fem_batch_numeric")


def fem_batch_sync_status(batch: int, stream=None) -> int:
    return load_library().fem_batch_sync_status(batch, _stream(stream))


def fem_batch_destroy(batch: int):
    if batch:
        load_library().fem_batch_destroy(batch)


def fem_pk_symbolic(d: int, k: int, nq: int, nme: int, me_ptr: int, stream=None) -> int:
    out = P()
    _check(load_library().fem_pk_symbolic(d, k, nq, nme, me_ptr, _stream(stream), C.byref(out)),
           "fem_pk_symbolic")
    return out.value


def fem_pk_query(plan: int):
    nr, nz, n = I64(), I64(), I32()
    _check(load_library().fem_pk_query(plan, C.byref(nr), C.byref(nz), C.byref(n)), "fem_pk_query")
    return nr.value, nz.value, n.value


def fem_pk_pattern(plan: int, row_ptr: int, col_idx: int, stream=None):
    _check(load_library().fem_pk_pattern(plan, row_ptr, col_idx, _stream(stream)), "fem_pk_pattern")


def fem_pk_mass(plan: int, q: int, values: int, stream=None):
    _check(load_library().fem_pk_mass(plan, q, values, _stream(stream)), "fem_pk_mass")


def fem_pk_sync_status(plan: int, stream=None) -> int:
    return load_library().fem_pk_sync_status(plan, _stream(stream))


def fem_pk_destroy(plan: int):
    if plan:
        load_library().fem_pk_destroy(plan)


def fem_boundary_symbolic(d: int, nq: int, nf: int, facets_ptr: int, stream=None) -> int:
    out = P()
    _check(load_library().fem_boundary_symbolic(d, nq, nf, facets_ptr, _stream(stream),
                                                C.byref(out)), "fem_boundary_symbolic")
    return out.value


def fem_boundary_mass(plan: int, q: int, w: int | None, values: int, stream=None):
    _check(load_library().fem_boundary_mass(plan, q, w, values, _stream(stream)),
           "fem_boundary_mass")


# ------------------------------------------------------------ torch helpers
def _on_stream(fn):
    """Runs a method with the caller's stream (its `stream` argument, a
    torch.cuda.Stream or a raw handle) current, so that the tensors it
    allocates -- converted inputs, outputs, work arrays -- belong to that
    stream for the caching allocator and are not handed out again before the
    stream's work on them has ended."""
    sig = inspect.signature(fn)

    @functools.wraps(fn)
    def wrapper(*args, **kw):
        bound = sig.bind(*args, **kw)
        stream = bound.arguments.get("stream")
        if stream is None:
            return fn(*args, **kw)
        s = stream if isinstance(stream, torch.cuda.Stream) else torch.cuda.ExternalStream(int(stream))
        bound.arguments["stream"] = s
        with torch.cuda.stream(s):
            return fn(*bound.args, **bound.kwargs)
    return wrapper


def _op(op) -> int:
    return FEM_OP[op] if isinstance(op, str) else int(op)


def _dev_f64(x, device):
    if x is None:
        return None
    t = torch.as_tensor(x, dtype=torch.float64, device=device)
    return t.contiguous()


class Plan:
    """A symbolic plan for one mesh (connectivity ``me`` of shape (d+1, nme))."""

    def __init__(self, me: torch.Tensor, nq: int, stream=None, wait_layouts: bool = True):
        load_library()
        if me.dtype != torch.int32 or not me.is_cuda or me.dim() != 2:
            raise ValueError("me must be a CUDA int32 tensor of shape (d+1, nme)")
        self.me = me.contiguous()
        self.d = self.me.shape[0] - 1
        self.nq = int(nq)
        self.nme = int(self.me.shape[1])
        self.device = self.me.device
        self.handle = fem_assemble_symbolic(self.d, self.nq, self.nme,
                                            self.me.data_ptr() if self.nme else 0, stream)
        self.max_row = fem_plan_info(self.handle)[3]
        # the block layouts are built by a library thread; by default the
        # plan is handed out once they are ready (every later call then runs
        # the same kernel)
        if wait_layouts:
            fem_plan_layouts(self.handle, wait=True)

    def layouts(self, wait=False):
        """0 building, 1 ready (block kernels), 2 none (row-gather only)."""
        return fem_plan_layouts(self.handle, wait)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            fem_plan_destroy(h)
            self.handle = None

    def query(self, op):
        return fem_plan_query(self.handle, _op(op))

    @_on_stream
    def pattern(self, op="STIFF", stream=None):
        nrows, nnz = self.query(op)
        rp = torch.empty(nrows + 1, dtype=torch.int32, device=self.device)
        ci = torch.empty(max(nnz, 1), dtype=torch.int32, device=self.device)
        fem_plan_pattern(self.handle, _op(op), rp.data_ptr(), ci.data_ptr(), stream)
        return rp, ci[:nnz]

    @_on_stream
    def slot_map(self, stream=None):
        n = (self.d + 1) ** 2 * self.nme
        s = torch.empty(max(n, 1), dtype=torch.int32, device=self.device)
        fem_plan_slot_map(self.handle, s.data_ptr(), stream)
        return s[:n]

    @_on_stream
    def numeric(self, op, q, w=None, lam=1.0, mu=0.5, out=None, stream=None):
        nrows, nnz = self.query(op)
        q = _dev_f64(q, self.device)
        w = _dev_f64(w, self.device)
        if out is None:
            out = torch.empty(max(nnz, 1), dtype=torch.float64, device=self.device)
        fem_assemble_numeric(self.handle, _op(op), q.data_ptr(), _ptr(w), float(lam), float(mu),
                             out.data_ptr(), stream)
        return out[:nnz]

    @_on_stream
    def elasticity_nodal(self, q, lam, mu, out=None, stream=None):
        """Elasticity with nodal Lame fields lam, mu (nq values each)."""
        _, nnz = self.query("ELAS")
        q, lam, mu = (_dev_f64(x, self.device) for x in (q, lam, mu))
        if out is None:
            out = torch.empty(max(nnz, 1), dtype=torch.float64, device=self.device)
        fem_assemble_elasticity_nodal(self.handle, q.data_ptr(), lam.data_ptr(), mu.data_ptr(),
                                      out.data_ptr(), stream)
        return out[:nnz]

    @_on_stream
    def general(self, q, coef, out=None, stream=None):
        """General operator with constant coefficients coef = [A, b, c, a0]."""
        _, nnz = self.query("STIFF")
        if len(coef) != self.d * self.d + 2 * self.d + 1:
            raise ValueError("coef must hold d*d + 2*d + 1 values")
        q = _dev_f64(q, self.device)
        if out is None:
            out = torch.empty(max(nnz, 1), dtype=torch.float64, device=self.device)
        fem_assemble_general(self.handle, q.data_ptr(), list(coef), out.data_ptr(), stream)
        return out[:nnz]

    @_on_stream
    def jvp(self, op, q, dq, w=None, dw=None, out=None, stream=None):
        """Directional derivative of the operator's CSR values along (dq, dw)."""
        _, nnz = self.query(op)
        q, dq, w, dw = (_dev_f64(x, self.device) for x in (q, dq, w, dw))
        if out is None:
            out = torch.empty(max(nnz, 1), dtype=torch.float64, device=self.device)
        fem_assemble_jvp(self.handle, _op(op), q.data_ptr(), _ptr(w), dq.data_ptr(), _ptr(dw),
                         out.data_ptr(), stream)
        return out[:nnz]

    def vjp_work_bytes(self, op):
        """Bytes of the work buffer of the workspace VJP for operator `op`."""
        return fem_vjp_work_bytes(self.handle, _op(op))

    @_on_stream
    def vjp(self, op, q, G, w=None, slot=None, want_w=True, stream=None, work=None):
        """Gradient of sum(G * A) with respect to q (d, nq) and, for MASS_W, w.
        With `work` (a device tensor of at least vjp_work_bytes(op) bytes) the
        workspace form runs: the same values, each element evaluated once.
        Without `slot` the kernels address G through the plan's position
        table (built on first use); with it, through that slot map."""
        if slot is None:
            fem_plan_vjp_positions(self.handle, stream)
        q, w, G = (_dev_f64(x, self.device) for x in (q, w, G))
        gq = torch.empty(self.d, self.nq, dtype=torch.float64, device=self.device)
        gw = (torch.empty(self.nq, dtype=torch.float64, device=self.device)
              if (_op(op) == FEM_OP["MASS_W"] and want_w) else None)
        if work is None:
            fem_assemble_vjp(self.handle, _op(op), q.data_ptr(), _ptr(w), G.data_ptr(),
                             _ptr(slot), gq.data_ptr(), _ptr(gw), stream)
        else:
            if not work.is_cuda:
                raise ValueError("work must be a device tensor")
            fem_assemble_vjp_ws(self.handle, _op(op), q.data_ptr(), _ptr(w), G.data_ptr(),
                                _ptr(slot), work.data_ptr(),
                                work.numel() * work.element_size(), gq.data_ptr(), _ptr(gw),
                                stream)
        return gq, gw

    @_on_stream
    def backward(self, q, w, a, b, op_mask=("STIFF", "MASS_W"), want_w=True, want_q=True,
                 stream=None):
        mask = 0
        for o in op_mask:
            mask |= 1 << _op(o)
        q, w, a, b = (_dev_f64(x, self.device) for x in (q, w, a, b))
        gw = torch.empty(self.nq, dtype=torch.float64, device=self.device) if want_w else None
        gq = torch.empty(self.d, self.nq, dtype=torch.float64, device=self.device) if want_q else None
        fem_assemble_backward(self.handle, mask, q.data_ptr(), _ptr(w), a.data_ptr(), b.data_ptr(),
                              _ptr(gw), _ptr(gq), stream)
        return gw, gq

    @_on_stream
    def bilinear(self, op, values, a, b, stream=None):
        out = torch.empty(1, dtype=torch.float64, device=self.device)
        a = _dev_f64(a, self.device)
        b = _dev_f64(b, self.device)
        fem_csr_bilinear(self.handle, _op(op), values.data_ptr(), a.data_ptr(), b.data_ptr(),
                         out.data_ptr(), stream)
        return out

    def sync_status(self, stream=None):
        st = fem_plan_sync_status(self.handle, stream)
        _check(st, "fem_plan_sync_status")


@dataclass
class BatchOffsets:
    q: list
    w: list
    rows: list
    nnz: list


class Batch:
    """Many meshes assembled by one persistent launch."""

    def __init__(self, mes, nqs, stream=None):
        load_library()
        self.mes = [m.contiguous() for m in mes]
        self.d = [int(m.shape[0]) - 1 for m in self.mes]
        self.nq = [int(n) for n in nqs]
        self.nme = [int(m.shape[1]) for m in self.mes]
        self.device = self.mes[0].device
        self.handle = fem_batch_create(self.d, self.nq, self.nme,
                                       [m.data_ptr() for m in self.mes], stream)
        # pair-layout settings per kind (0 scalar operators, 1 elasticity):
        # (rows per 3D block, rows per 2D block, tasks per wavefront), the
        # library's defaults until configured
        self.layout = {0: PAIR_LAYOUT_DEFAULT[0], 1: PAIR_LAYOUT_DEFAULT[1]}
        self.params = ("pair",) + self.layout[0]

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            fem_batch_destroy(h)
            self.handle = None

    def __len__(self):
        return len(self.mes)

    def offsets(self, op) -> BatchOffsets:
        q, w, r, z = fem_batch_offsets(self.handle, _op(op), len(self.mes))
        return BatchOffsets(q, w, r, z)

    def plan_handle(self, index: int) -> int:
        return fem_batch_plan(self.handle, index)

    def set_params(self, block_threads: int, wg_per_cu: int):
        """Tunables of the row-gather launch (the kernel family is unchanged)."""
        fem_batch_set_params(self.handle, block_threads, wg_per_cu)
        self.params = (self.params[0], block_threads, wg_per_cu)

    def configure(self, params, op="STIFF"):
        """params = ("pair" | "pair_split", rows_3d, rows_2d, slots): the
        vertex-pair kernel with that layout for the operators of op's kind
        (rebuilt when it changes), in one launch over both dimensions or one
        per dimension; or ("rowgather", block_threads, wg_per_cu): the
        row-gather launch with those tunables.  Values are the same for every
        setting."""
        kind = 1 if _op(op) == FEM_OP["ELAS"] else 0
        if params[0] in ("pair", "pair_split"):
            layout = tuple(int(x) for x in params[1:4])
            if layout != self.layout[kind]:
                fem_batch_set_pair_layout(self.handle, _op(op), *layout)
                self.layout[kind] = layout
            fem_batch_set_kernel(self.handle, FEM_BATCH_KERNEL[params[0]])
            self.params = (params[0],) + layout
        else:
            kernel, bt, w = params
            fem_batch_set_params(self.handle, bt, w)
            fem_batch_set_kernel(self.handle, FEM_BATCH_KERNEL[kernel])
            self.params = (kernel, bt, w)

    @_on_stream
    def numeric(self, op, q_cat, w_cat=None, lam=1.0, mu=0.5, out=None, stream=None):
        nnz = self.offsets(op).nnz[-1]
        if out is None:
            out = torch.empty(max(nnz, 1), dtype=torch.float64, device=self.device)
        fem_batch_numeric(self.handle, _op(op), q_cat.data_ptr(), _ptr(w_cat), float(lam),
                          float(mu), out.data_ptr(), stream)
        return out[:nnz]

    def sync_status(self, stream=None):
        _check(fem_batch_sync_status(self.handle, stream), "fem_batch_sync_status")


class PkPlan:
    """Symbolic plan of the P_k mass matrix of one P_k mesh (``me`` of shape
    (N, nme), N = (d+k)!/(d! k!), local nodes 0..d the vertices)."""

    def __init__(self, me: torch.Tensor, nq: int, d: int, k: int, stream=None):
        load_library()
        if me.dtype != torch.int32 or not me.is_cuda or me.dim() != 2:
            raise ValueError("me must be a CUDA int32 tensor of shape (N, nme)")
        self.me = me.contiguous()
        self.d, self.k = int(d), int(k)
        self.nq = int(nq)
        self.nme = int(self.me.shape[1])
        self.device = self.me.device
        self.handle = fem_pk_symbolic(self.d, self.k, self.nq, self.nme,
                                      self.me.data_ptr() if self.nme else 0, stream)
        _, self.nnz, self.ndfe = fem_pk_query(self.handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            fem_pk_destroy(h)
            self.handle = None

    @_on_stream
    def pattern(self, stream=None):
        rp = torch.empty(self.nq + 1, dtype=torch.int32, device=self.device)
        ci = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=self.device)
        fem_pk_pattern(self.handle, rp.data_ptr(), ci.data_ptr(), stream)
        return rp, ci[:self.nnz]

    @_on_stream
    def mass(self, q, out=None, stream=None):
        q = _dev_f64(q, self.device)
        if out is None:
            out = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=self.device)
        fem_pk_mass(self.handle, q.data_ptr(), out.data_ptr(), stream)
        return out[:self.nnz]

    def sync_status(self, stream=None):
        _check(fem_pk_sync_status(self.handle, stream), "fem_pk_sync_status")


class BoundaryPlan:
    """Plan of the boundary mass / weighted mass over (d-1)-simplices
    ``facets`` (shape (d, nf)) embedded in R^d."""

    def __init__(self, facets: torch.Tensor, nq: int, stream=None):
        load_library()
        if facets.dtype != torch.int32 or not facets.is_cuda or facets.dim() != 2:
            raise ValueError("facets must be a CUDA int32 tensor of shape (d, nf)")
        self.facets = facets.contiguous()
        self.d = int(self.facets.shape[0])
        self.nq = int(nq)
        self.nf = int(self.facets.shape[1])
        self.device = self.facets.device
        self.handle = fem_boundary_symbolic(self.d, self.nq, self.nf,
                                            self.facets.data_ptr() if self.nf else 0, stream)
        _, self.nnz, _ = fem_pk_query(self.handle)

    def __del__(self):
        h = getattr(self, "handle", None)
        if h and _lib is not None:
            fem_pk_destroy(h)
            self.handle = None

    @_on_stream
    def pattern(self, stream=None):
        rp = torch.empty(self.nq + 1, dtype=torch.int32, device=self.device)
        ci = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=self.device)
        fem_pk_pattern(self.handle, rp.data_ptr(), ci.data_ptr(), stream)
        return rp, ci[:self.nnz]

    @_on_stream
    def mass(self, q, w=None, out=None, stream=None):
        q = _dev_f64(q, self.device)
        w = _dev_f64(w, self.device)
        if out is None:
            out = torch.empty(max(self.nnz, 1), dtype=torch.float64, device=self.device)
        fem_boundary_mass(self.handle, q.data_ptr(), _ptr(w), out.data_ptr(), stream)
        return out[:self.nnz]

    def sync_status(self, stream=None):
        _check(fem_pk_sync_status(self.handle, stream), "fem_pk_sync_status")
