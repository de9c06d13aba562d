"""paper_1705_06661_amd -- spin summations on AMD Instinct MI355X (gfx950).

Thin ctypes binding of ``libspinsum.so`` (C-ABI declared in
``include/spinsum.h``).  Every function here only marshals arguments; all
arithmetic runs in the library's HIP kernels.  torch is used for device
memory and streams only.  There is no CPU fallback: importing this package
without the built library raises ImportError.

Operation (Springer, Matthews, Bientinesi, "Spin Summations: A
High-Performance Perspective", Def. 1-4 and Sec. 4.6.5):
``Out = S_K(...S_1(In))`` with ``S_k = sum_t alpha_t pi_t`` acting on the
trailing ``d`` dimensions of a row-major tensor; a term ``(p, alpha)`` adds
``alpha * In[..., i_{p[0]}, ..., i_{p[d-1]}]`` to ``Out[..., i_0, ..., i_{d-1}]``.
A coefficient set is given as a list of stages, each a list of
``(perm, alpha)`` with 0-based ``perm``; stage 0 is applied first.
"""
from __future__ import annotations

import ctypes
import math
import itertools
import os
from typing import List, Optional, Sequence, Tuple

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspinsum.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python paper_1705_06661_amd/build.py` "
        "(there is no CPU fallback)")

_lib = ctypes.CDLL(LIB_PATH)

# ------------------------------------------------------------ C declarations
SPINSUM_OK = 0
SPINSUM_ERR_INVALID_ARG = -1
SPINSUM_ERR_NOT_PERMUTATION = -2
SPINSUM_ERR_EXTENT_MISMATCH = -3
SPINSUM_ERR_UNSUPPORTED = -4
SPINSUM_ERR_ALIASING = -5
SPINSUM_ERR_MISALIGNED = -6
SPINSUM_ERR_OUT_OF_MEMORY = -7
SPINSUM_ERR_HIP = -8
SPINSUM_ERR_NO_DEVICE = -9

SPINSUM_F64 = 0
SPINSUM_F32 = 1

SPINSUM_FLAG_HOST_ONLY = 0x1
SPINSUM_FLAG_NO_NT_STORES = 0x2
SPINSUM_FLAG_CHAIN_STAGES = 0x4
SPINSUM_FLAG_NO_XCD_REMAP = 0x8
SPINSUM_FLAG_REVERSE_ORDER = 0x10
SPINSUM_FLAG_NO_LDS_PAD = 0x20
SPINSUM_FLAG_NO_DIRECT_LDS = 0x40
SPINSUM_FLAG_INDEX_PAIRS = 0x80
SPINSUM_FLAG_NT_STORES = 0x100
SPINSUM_FLAG_MULTI_PASS = 0x200
SPINSUM_FLAG_FULL_GROUP = 0x400
SPINSUM_FLAG_NO_NT_LOADS = 0x800

SPINSUM_VARIANT_AUTO = 0
SPINSUM_VARIANT_DIRECT_LDS = 1
SPINSUM_VARIANT_REG_PIPELINE = 2
SPINSUM_VARIANT_REG_ONESHOT = 3
SPINSUM_VARIANT_LDS_PIPELINE = 4


class _Tile(ctypes.Structure):
    _fields_ = [("bl", ctypes.c_int), ("cubes_per_wg", ctypes.c_int),
                ("threads", ctypes.c_int), ("lds_pad", ctypes.c_int), ("variant", ctypes.c_int),
                ("item_tiles", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("n", ctypes.c_int), ("ncubes", ctypes.c_int64),
                ("elems", ctypes.c_int64), ("nstages", ctypes.c_int),
                ("nterms_expanded", ctypes.c_int), ("bl", ctypes.c_int), ("nb", ctypes.c_int),
                ("norbits", ctypes.c_int), ("cubes_per_wg", ctypes.c_int),
                ("threads", ctypes.c_int), ("max_tiles", ctypes.c_int), ("variant", ctypes.c_int),
                ("lds_pad", ctypes.c_int),
                ("lds_bytes", ctypes.c_int64), ("nitems", ctypes.c_int64),
                ("nblocks", ctypes.c_int), ("dtype", ctypes.c_int), ("inplace", ctypes.c_int),
                ("vector_width", ctypes.c_int), ("ragged", ctypes.c_int),
                ("fits_lds", ctypes.c_int), ("items_per_cube", ctypes.c_int),
                ("item_tiles", ctypes.c_int), ("chunks_per_thread", ctypes.c_int),
                ("rep_lds_bytes", ctypes.c_int64), ("inner", ctypes.c_int),
                ("pair_extent", ctypes.c_int), ("batch_item_bytes", ctypes.c_int64),
                ("batch_persistent", ctypes.c_int), ("nt_stores", ctypes.c_int),
                ("exec_d", ctypes.c_int), ("exec_group_first", ctypes.c_int),
                ("persistent_per_cu", ctypes.c_int), ("nt_loads", ctypes.c_int),
                ("coef_grad_split", ctypes.c_int), ("unpack_bl", ctypes.c_int),
                ("unpack_persistent", ctypes.c_int), ("unpack_nt_stores", ctypes.c_int)]


_vp = ctypes.c_void_p
_ip = ctypes.POINTER(ctypes.c_int)
_i64p = ctypes.POINTER(ctypes.c_int64)
_dp = ctypes.POINTER(ctypes.c_double)
_st = ctypes.c_int


def _decl(name, argtypes, restype=_st):
    f = getattr(_lib, name)
    f.argtypes = argtypes
    f.restype = restype
    return f


_c_plan = _decl("spinsum_plan", [ctypes.POINTER(_vp), ctypes.c_int, _i64p, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_int, _ip, _ip, _dp, ctypes.c_int,
                                 ctypes.c_int, ctypes.c_uint])
_c_plan_batched = _decl("spinsum_plan_batched",
                        [ctypes.POINTER(_vp), ctypes.c_int, _ip, ctypes.POINTER(_i64p),
                         ctypes.c_int, ctypes.c_int, ctypes.c_int, _ip, _ip, _dp, ctypes.c_int,
                         ctypes.c_int, ctypes.c_uint])
_c_set_tile = _decl("spinsum_plan_set_tile", [_vp, ctypes.POINTER(_Tile)])
_c_get_info = _decl("spinsum_plan_get_info", [_vp, ctypes.POINTER(_Info)])
_c_expanded = _decl("spinsum_plan_expanded", [_vp, ctypes.c_int, _ip, _ip, _dp])
_c_check = _decl("spinsum_plan_check_ownership", [_vp, ctypes.c_int,
                                                  ctypes.POINTER(ctypes.c_char_p)])
_c_exec = _decl("spinsum_exec", [_vp, _vp, _vp, _vp])
_c_exec_batched = _decl("spinsum_exec_batched", [_vp, _vp, _vp, _vp])
_c_adjoint = _decl("spinsum_adjoint", [_vp, _vp, _vp, _vp])
_c_coef_grad = _decl("spinsum_coef_grad", [_vp, _vp, _vp, _vp, _vp])
_c_coef_grad_noalloc = _decl("spinsum_coef_grad_noalloc", [_vp, _vp, _vp, _vp, _vp])
_c_coef_grad_stages = _decl("spinsum_coef_grad_stages", [_vp, _vp, _vp, _vp, _vp, _vp, _vp])
_c_unpack = _decl("spinsum_unpack", [_vp, _vp, _vp, _vp])
_c_pack = _decl("spinsum_pack", [_vp, _vp, _vp, _vp])
_c_graph_create = _decl("spinsum_graph_create", [_vp, _vp, _vp, ctypes.POINTER(_vp)])
_c_graph_launch = _decl("spinsum_graph_launch", [_vp, _vp])
_c_graph_destroy = _decl("spinsum_graph_destroy", [_vp], None)
_c_autotune = _decl("spinsum_autotune", [_vp, _vp, _vp, _vp, ctypes.c_char_p,
                                         ctypes.POINTER(_Tile), ctypes.POINTER(ctypes.c_float)])
_c_copy = _decl("spinsum_stream_copy", [_vp, _vp, ctypes.c_int64, _vp])
_c_last_err = _decl("spinsum_plan_last_hip_error", [_vp], ctypes.c_int)
_c_destroy = _decl("spinsum_plan_destroy", [_vp], None)
_c_status_string = _decl("spinsum_status_string", [ctypes.c_int], ctypes.c_char_p)
_c_version = _decl("spinsum_version", [], ctypes.c_char_p)

EXPORTED = ["spinsum_plan", "spinsum_plan_batched", "spinsum_plan_set_tile",
            "spinsum_plan_get_info", "spinsum_plan_expanded", "spinsum_plan_check_ownership",
            "spinsum_exec", "spinsum_exec_batched", "spinsum_adjoint", "spinsum_coef_grad",
            "spinsum_coef_grad_noalloc", "spinsum_coef_grad_stages", "spinsum_unpack",
            "spinsum_pack",
            "spinsum_graph_create",
            "spinsum_graph_launch", "spinsum_graph_destroy", "spinsum_autotune",
            "spinsum_stream_copy", "spinsum_plan_last_hip_error", "spinsum_plan_destroy",
            "spinsum_status_string", "spinsum_version"]


class SpinSumError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = int(status)
        msg = _c_status_string(int(status)).decode()
        super().__init__(f"{what}: {msg} (status {status})" if what else msg)


def _check(st: int, what: str, plan=None):
    if st != SPINSUM_OK:
        err = SpinSumError(st, what)
        if plan is not None and st == SPINSUM_ERR_HIP:
            err.hip_error = int(_c_last_err(plan._h))
        raise err


def spinsum_status_string(status: int) -> str:
    return _c_status_string(int(status)).decode()


def spinsum_version() -> str:
    return _c_version().decode()


# ------------------------------------------------------------------- plans
_DTYPES = {"f64": SPINSUM_F64, torch.float64: SPINSUM_F64, "f32": SPINSUM_F32,
           torch.float32: SPINSUM_F32}


def _flatten(stages, d):
    nterms = [len(s) for s in stages]
    perms, alpha = [], []
    for s in stages:
        for p, a in s:
            if len(p) != d:
                raise SpinSumError(SPINSUM_ERR_INVALID_ARG, "permutation of wrong degree")
            perms.extend(int(v) for v in p)
            alpha.append(float(a))
    return ((ctypes.c_int * max(1, len(nterms)))(*nterms),
            (ctypes.c_int * max(1, len(perms)))(*perms),
            (ctypes.c_double * max(1, len(alpha)))(*alpha))


class Plan:
    """Owns a spinsum_plan_t (destroyed with the object)."""

    def __init__(self, handle, d, shapes, dtype, inplace, batched, stages, group_first=None):
        self._h = handle
        self.d = d
        self.group_first = group_first
        self.shapes = shapes
        self.dtype = torch.float64 if dtype == SPINSUM_F64 else torch.float32
        self.inplace = bool(inplace)
        self.batched = batched
        self.stages = stages

    @property
    def shape(self):
        return self.shapes[0]

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _c_destroy is not None:  # module globals may be gone at exit
            _c_destroy(h)

    def info(self) -> dict:
        return spinsum_plan_get_info(self)


def spinsum_plan(extents: Sequence[int], group_first: int, d: int, stages, dtype="f64",
                 inplace: bool = False, flags: int = 0) -> Plan:
    """Plan Out = S_K(...S_1(In)) over dims [group_first, group_first + d)."""
    ext = (ctypes.c_int64 * len(extents))(*[int(e) for e in extents])
    nt, pp, aa = _flatten(stages, d)
    h = _vp()
    dt = _DTYPES[dtype]
    _check(_c_plan(ctypes.byref(h), len(extents), ext, int(group_first), int(d), len(stages),
                   nt, pp, aa, dt, int(bool(inplace)), int(flags)), "spinsum_plan")
    return Plan(h, d, [tuple(int(e) for e in extents)], dt, inplace, False, stages,
                int(group_first))


def spinsum_plan_batched(shapes: Sequence[Sequence[int]], d: int, stages, dtype="f64",
                         inplace: bool = False, flags: int = 0, group_first: int = -1) -> Plan:
    """Plan one launch over many tensors: the group is dims [group_first,
    group_first + d) of every block, or its trailing d dims (group_first -1)."""
    nb = len(shapes)
    ndims = (ctypes.c_int * nb)(*[len(s) for s in shapes])
    rows = [(ctypes.c_int64 * len(s))(*[int(e) for e in s]) for s in shapes]
    ptrs = (_i64p * nb)(*[ctypes.cast(r, _i64p) for r in rows])
    nt, pp, aa = _flatten(stages, d)
    h = _vp()
    dt = _DTYPES[dtype]
    _check(_c_plan_batched(ctypes.byref(h), nb, ndims, ptrs, int(group_first), int(d), len(stages),
                           nt, pp, aa, dt, int(bool(inplace)), int(flags)), "spinsum_plan_batched")
    return Plan(h, d, [tuple(int(e) for e in s) for s in shapes], dt, inplace, True, stages)


def spinsum_plan_set_tile(plan: Plan, bl: int, cubes_per_wg: int = 1, lds_pad: int = 1,
                          threads: int = 0, variant: int = SPINSUM_VARIANT_AUTO,
                          item_tiles: int = 0):
    t = _Tile(int(bl), int(cubes_per_wg), int(threads), int(lds_pad), int(variant),
              int(item_tiles))
    _check(_c_set_tile(plan._h, ctypes.byref(t)), "spinsum_plan_set_tile", plan)


def spinsum_plan_get_info(plan: Plan) -> dict:
    info = _Info()
    _check(_c_get_info(plan._h, ctypes.byref(info)), "spinsum_plan_get_info")
    return {k: getattr(info, k) for k, _ in _Info._fields_}


def spinsum_plan_expanded(plan: Plan) -> List[Tuple[Tuple[int, ...], float]]:
    n = ctypes.c_int(0)
    _check(_c_expanded(plan._h, 0, ctypes.byref(n), None, None), "spinsum_plan_expanded")
    cap = n.value
    perms = (ctypes.c_int * max(1, cap * plan.d))()
    alpha = (ctypes.c_double * max(1, cap))()
    _check(_c_expanded(plan._h, cap, ctypes.byref(n), perms, alpha), "spinsum_plan_expanded")
    return [(tuple(perms[k * plan.d:(k + 1) * plan.d]), alpha[k]) for k in range(n.value)]


def spinsum_plan_check_ownership(plan: Plan, block: int = 0) -> Tuple[bool, str]:
    why = ctypes.c_char_p()
    st = _c_check(plan._h, int(block), ctypes.byref(why))
    return st == SPINSUM_OK, (why.value or b"").decode()


def spinsum_plan_last_hip_error(plan: Plan) -> int:
    return int(_c_last_err(plan._h))


def spinsum_plan_destroy(plan: Plan):
    plan.__del__()


# ------------------------------------------------------------------- exec
def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _tensor_ptr(t: torch.Tensor, plan: Plan, shape, what: str) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch tensor")
    if not t.is_cuda:
        raise SpinSumError(SPINSUM_ERR_INVALID_ARG, f"{what} must be a GPU tensor")
    if t.dtype != plan.dtype:
        raise SpinSumError(SPINSUM_ERR_INVALID_ARG, f"{what} has dtype {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise SpinSumError(SPINSUM_ERR_INVALID_ARG, f"{what} has shape {tuple(t.shape)}")
    if not t.is_contiguous():
        raise SpinSumError(SPINSUM_ERR_INVALID_ARG, f"{what} is not contiguous")
    return t.data_ptr()


def spinsum_exec(plan: Plan, inp: torch.Tensor, out: torch.Tensor, stream=None):
    """out = S(inp) (in-place plans: pass the same tensor twice)."""
    a = _tensor_ptr(inp, plan, plan.shape, "input")
    b = _tensor_ptr(out, plan, plan.shape, "output")
    _check(_c_exec(plan._h, a, b, _stream(stream)), "spinsum_exec", plan)
    return out


def spinsum_adjoint(plan: Plan, grad_out: torch.Tensor, grad_in: torch.Tensor, stream=None):
    """grad_in = S^T grad_out."""
    a = _tensor_ptr(grad_out, plan, plan.shape, "grad_out")
    b = _tensor_ptr(grad_in, plan, plan.shape, "grad_in")
    _check(_c_adjoint(plan._h, a, b, _stream(stream)), "spinsum_adjoint", plan)
    return grad_in


def spinsum_coef_grad(plan: Plan, x: torch.Tensor, g: torch.Tensor, stream=None) -> torch.Tensor:
    """<g, pi_r(x)> for every permutation r of the group (lexicographic
    order, d! float64 values on the device): the gradient of <g, S(x)> with
    respect to the coefficient of each permutation."""
    a = _tensor_ptr(x, plan, plan.shape, "x")
    b = _tensor_ptr(g, plan, plan.shape, "g")
    out = torch.empty(math.factorial(plan.d), dtype=torch.float64, device=x.device)
    _check(_c_coef_grad(plan._h, a, b, out.data_ptr(), _stream(stream)), "spinsum_coef_grad", plan)
    return out


def packed_shape(plan: Plan):
    """[outer..., C(N, d), inner...] of a plan's full shape (group_first is
    taken from the plan's stored arguments)."""
    shape = plan.shape
    gf = plan.group_first
    n = shape[gf]
    return tuple(shape[:gf]) + (math.comb(n, plan.d),) + tuple(shape[gf + plan.d:])


def _packed_ptr(t: torch.Tensor, plan: Plan, what: str) -> int:
    return _tensor_ptr(t, plan, packed_shape(plan), what)


def spinsum_unpack(plan: Plan, packed: torch.Tensor, full: torch.Tensor, stream=None):
    """full = S(E(packed)): the values at the strictly increasing group
    positions (lexicographic order) placed and summed over the plan's
    permutations (the antisymmetriser unpacks an antisymmetric tensor)."""
    a = _packed_ptr(packed, plan, "packed")
    b = _tensor_ptr(full, plan, plan.shape, "full")
    _check(_c_unpack(plan._h, a, b, _stream(stream)), "spinsum_unpack", plan)
    return full


def spinsum_pack(plan: Plan, full: torch.Tensor, packed: torch.Tensor, stream=None):
    """packed = E^T S^T full (the adjoint of spinsum_unpack)."""
    a = _tensor_ptr(full, plan, plan.shape, "full")
    b = _packed_ptr(packed, plan, "packed")
    _check(_c_pack(plan._h, a, b, _stream(stream)), "spinsum_pack", plan)
    return packed


def spinsum_coef_grad_stages(plan: Plan, x: torch.Tensor, g: torch.Tensor, work=None,
                             stream=None) -> torch.Tensor:
    """<(S_K..S_{k+1})^T g, pi_r(S_{k-1}..S_1 x)> for every stage k and every
    permutation r of the group (lexicographic order): a (stages, d!) float64
    tensor, the gradient of <g, S(x)> with respect to every stage's
    coefficients.  work: two tensors of the plan's shape and dtype that are
    overwritten (allocated here if None)."""
    a = _tensor_ptr(x, plan, plan.shape, "x")
    b = _tensor_ptr(g, plan, plan.shape, "g")
    K = len(plan.stages)
    if work is None:
        work = (torch.empty_like(x), torch.empty_like(x)) if K > 1 else (None, None)
    wu = _tensor_ptr(work[0], plan, plan.shape, "work") if work[0] is not None else None
    wh = _tensor_ptr(work[1], plan, plan.shape, "work") if work[1] is not None else None
    out = torch.empty((K, math.factorial(plan.d)), dtype=torch.float64, device=x.device)
    _check(_c_coef_grad_stages(plan._h, a, b, out.data_ptr(), wu, wh, _stream(stream)),
           "spinsum_coef_grad_stages", plan)
    return out


def spinsum_coef_grad_noalloc(plan: Plan, x: torch.Tensor, g: torch.Tensor,
                              grad: torch.Tensor, stream=None) -> torch.Tensor:
    """spinsum_coef_grad into a caller-provided ``grad`` (d! float64 values on
    the device), with the library's static partial-sum array: no device
    memory is allocated by this call.  Calls on one GPU must not overlap."""
    a = _tensor_ptr(x, plan, plan.shape, "x")
    b = _tensor_ptr(g, plan, plan.shape, "g")
    if (not isinstance(grad, torch.Tensor) or not grad.is_cuda or grad.dtype != torch.float64
            or grad.numel() != math.factorial(plan.d) or not grad.is_contiguous()):
        raise SpinSumError(SPINSUM_ERR_INVALID_ARG, "grad must be d! contiguous float64 on the GPU")
    _check(_c_coef_grad_noalloc(plan._h, a, b, grad.data_ptr(), _stream(stream)),
           "spinsum_coef_grad_noalloc", plan)
    return grad


class PointerArrays:
    """Device-resident arrays of block pointers for the batched entry points."""

    def __init__(self, plan: Plan, ins: Sequence[torch.Tensor], outs: Sequence[torch.Tensor]):
        if len(ins) != len(plan.shapes) or len(outs) != len(plan.shapes):
            raise SpinSumError(SPINSUM_ERR_INVALID_ARG, "one tensor per block expected")
        pin = [_tensor_ptr(t, plan, s, "input") for t, s in zip(ins, plan.shapes)]
        pout = [_tensor_ptr(t, plan, s, "output") for t, s in zip(outs, plan.shapes)]
        if any(p & 15 for p in pin + pout):
            raise SpinSumError(SPINSUM_ERR_MISALIGNED, "block tensors must be 16-byte aligned")
        for k, (a, b) in enumerate(zip(pin, pout)):
            nbytes = ins[k].numel() * ins[k].element_size()
            if plan.inplace and a != b:
                raise SpinSumError(SPINSUM_ERR_INVALID_ARG, "in-place plan needs in == out")
            if not plan.inplace and nbytes and a < b + nbytes and b < a + nbytes:
                raise SpinSumError(SPINSUM_ERR_ALIASING, f"block {k} overlaps")
        dev = ins[0].device if ins else torch.device("cuda")
        self.d_in = torch.tensor(pin, dtype=torch.int64, device=dev)
        self.d_out = torch.tensor(pout, dtype=torch.int64, device=dev)
        self.keep = (list(ins), list(outs))


def spinsum_exec_batched(plan: Plan, ins, outs, stream=None, arrays: Optional[PointerArrays] = None):
    """One launch over all blocks of a batched plan."""
    arrays = arrays or PointerArrays(plan, ins, outs)
    _check(_c_exec_batched(plan._h, arrays.d_in.data_ptr(), arrays.d_out.data_ptr(),
                           _stream(stream)), "spinsum_exec_batched", plan)
    return arrays


class Graph:
    def __init__(self, handle, keep):
        self._h = handle
        self._keep = keep

    def __del__(self):
        h, self._h = getattr(self, "_h", None), None
        if h and _c_graph_destroy is not None:
            _c_graph_destroy(h)


def spinsum_graph_create(plan: Plan, ins, outs) -> Graph:
    """Capture one exec (batched: one launch) into a hipGraph."""
    h = _vp()
    if plan.batched:
        arrays = PointerArrays(plan, ins, outs)
        _check(_c_graph_create(plan._h, arrays.d_in.data_ptr(), arrays.d_out.data_ptr(),
                               ctypes.byref(h)), "spinsum_graph_create", plan)
        torch.cuda.synchronize()
        return Graph(h, (plan, arrays))
    a = _tensor_ptr(ins, plan, plan.shape, "input")
    b = _tensor_ptr(outs, plan, plan.shape, "output")
    _check(_c_graph_create(plan._h, a, b, ctypes.byref(h)), "spinsum_graph_create", plan)
    return Graph(h, (plan, ins, outs))


def spinsum_graph_launch(graph: Graph, stream=None):
    _check(_c_graph_launch(graph._h, _stream(stream)), "spinsum_graph_launch")


def spinsum_graph_destroy(graph: Graph):
    graph.__del__()


def spinsum_autotune(plan: Plan, inp, out, stream=None, cache_path: Optional[str] = None):
    """Time tile candidates on these buffers (overwritten) and keep the best.
    Batched plans take one tensor per block in `inp` and `out` (lists) and
    tune the whole-cube item size and the persistent launch; the result's
    cubes_per_wg is the item size in KiB and variant 1 the persistent
    launch."""
    keep = None
    if plan.batched:
        keep = PointerArrays(plan, inp, out)
        a, b = keep.d_in.data_ptr(), keep.d_out.data_ptr()
    else:
        a = _tensor_ptr(inp, plan, plan.shape, "input")
        b = _tensor_ptr(out, plan, plan.shape, "output")
    best = _Tile()
    ms = ctypes.c_float(0)
    cp = cache_path.encode() if cache_path else None
    _check(_c_autotune(plan._h, a, b, _stream(stream), cp, ctypes.byref(best), ctypes.byref(ms)),
           "spinsum_autotune", plan)
    return {"bl": best.bl, "cubes_per_wg": best.cubes_per_wg, "threads": best.threads,
            "lds_pad": best.lds_pad, "variant": best.variant,
            "item_tiles": best.item_tiles}, float(ms.value)


def spinsum_stream_copy(inp: torch.Tensor, out: torch.Tensor, stream=None):
    """out <- inp with the kernels' own load/store instructions (HBM ceiling)."""
    nbytes = inp.numel() * inp.element_size()
    if out.numel() * out.element_size() < nbytes or not (inp.is_cuda and out.is_cuda):
        raise SpinSumError(SPINSUM_ERR_INVALID_ARG, "stream copy")
    _check(_c_copy(inp.data_ptr(), out.data_ptr(), nbytes, _stream(stream)), "spinsum_stream_copy")
    return out


# ----------------------------------------------------------- conveniences
def apply(x: torch.Tensor, plan: Plan, out: Optional[torch.Tensor] = None, stream=None):
    """S(x); in-place plans overwrite x and return it."""
    if plan.inplace:
        return spinsum_exec(plan, x, x, stream)
    if out is None:
        out = torch.empty_like(x)
    return spinsum_exec(plan, x, out, stream)


class SpinSumFunction(torch.autograd.Function):
    """Autograd wrapper: forward = spinsum_exec, backward = spinsum_adjoint.
    The map is linear, so nothing is saved for backward."""

    @staticmethod
    def forward(ctx, x, plan: Plan):
        ctx.plan = plan
        if plan.inplace:
            spinsum_exec(plan, x, x)
            ctx.mark_dirty(x)
            return x
        out = torch.empty_like(x)
        spinsum_exec(plan, x, out)
        return out

    @staticmethod
    def backward(ctx, g):
        plan = ctx.plan
        g = g.contiguous()
        if plan.inplace:
            gi = g.clone()
            spinsum_adjoint(plan, gi, gi)
        else:
            gi = torch.empty_like(g)
            spinsum_adjoint(plan, g, gi)
        return gi, None


class SpinSumCoefFunction(torch.autograd.Function):
    """Out = sum_t alpha_t pi_t(x) with the coefficients as a tensor: the
    gradient flows to x (adjoint kernel) and to alpha (coefficient-gradient
    kernel).  perms: the d-tuples of the terms (distinct); a plan is made
    from the current coefficient values on every call (single stage,
    out-of-place)."""

    @staticmethod
    def forward(ctx, x, alpha, perms, group_first):
        d = len(perms[0])
        terms = [(tuple(p), float(a)) for p, a in zip(perms, alpha.detach().cpu().tolist())]
        if len(set(tuple(p) for p in perms)) != len(perms):
            raise SpinSumError(SPINSUM_ERR_INVALID_ARG, "permutations must be distinct")
        plan = spinsum_plan(tuple(x.shape), group_first, d, [terms], dtype=x.dtype, inplace=False)
        out = torch.empty_like(x)
        spinsum_exec(plan, x.contiguous(), out)
        ctx.plan = plan
        ctx.perms = [tuple(p) for p in perms]
        ctx.save_for_backward(x)
        return out

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        plan = ctx.plan
        g = g.contiguous()
        gx = None
        if ctx.needs_input_grad[0]:
            gx = torch.empty_like(g)
            spinsum_adjoint(plan, g, gx)
        ga = None
        if ctx.needs_input_grad[1]:
            c = spinsum_coef_grad(plan, x.contiguous(), g)
            d = len(ctx.perms[0])
            rank = {p: r for r, p in enumerate(itertools.permutations(range(d)))}
            ga = torch.stack([c[rank[p]] for p in ctx.perms]).to(x.dtype)
        return gx, ga, None, None


class SpinSumChainCoefFunction(torch.autograd.Function):
    """Out = S_K(...S_1(x)), S_k = sum_t alpha_{k,t} pi_{k,t}, with every
    stage's coefficients in one flat tensor (stage 0 first, then stage 1, ...):
    the gradient flows to x (adjoint kernel) and to every stage's
    coefficients (spinsum_coef_grad_stages).  perms: one list of distinct
    d-tuples per stage; a plan with `flags` (by default the stages chained in
    registers) is made from the current coefficient values on every call,
    out-of-place."""

    @staticmethod
    def forward(ctx, x, alpha, perms, group_first, flags=SPINSUM_FLAG_CHAIN_STAGES):
        d = len(perms[0][0])
        vals = alpha.detach().cpu().tolist()
        stages, pos = [], 0
        for st in perms:
            if len(set(tuple(p) for p in st)) != len(st):
                raise SpinSumError(SPINSUM_ERR_INVALID_ARG, "permutations of a stage must be distinct")
            stages.append([(tuple(p), float(vals[pos + i])) for i, p in enumerate(st)])
            pos += len(st)
        if pos != alpha.numel():
            raise SpinSumError(SPINSUM_ERR_INVALID_ARG, "one coefficient per term expected")
        plan = spinsum_plan(tuple(x.shape), group_first, d, stages, dtype=x.dtype, inplace=False,
                            flags=flags)
        out = torch.empty_like(x)
        spinsum_exec(plan, x.contiguous(), out)
        ctx.plan = plan
        ctx.perms = [[tuple(p) for p in st] for st in perms]
        ctx.save_for_backward(x)
        return out

    @staticmethod
    def backward(ctx, g):
        (x,) = ctx.saved_tensors
        plan = ctx.plan
        g = g.contiguous()
        gx = None
        if ctx.needs_input_grad[0]:
            gx = torch.empty_like(g)
            spinsum_adjoint(plan, g, gx)
        ga = None
        if ctx.needs_input_grad[1]:
            c = spinsum_coef_grad_stages(plan, x.contiguous(), g)
            d = len(ctx.perms[0][0])
            rank = {p: r for r, p in enumerate(itertools.permutations(range(d)))}
            ga = torch.stack([c[k, rank[p]] for k, st in enumerate(ctx.perms) for p in st]).to(x.dtype)
        return gx, ga, None, None, None


__all__ = EXPORTED + ["Plan", "Graph", "PointerArrays", "SpinSumError", "SpinSumFunction",
                      "SpinSumCoefFunction", "SpinSumChainCoefFunction", "apply"]
