"""CPU oracle for spin summations -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library never imports it, and
the two share no code: not the arithmetic, not the permutation helpers, not
the layout code.

Three independent routes to the same result (Springer, Matthews, Bientinesi,
"Spin Summations: A High-Performance Perspective"):

* ``spinsum`` / ``spinsum_chain`` / ``spinsum_chain_adjoint`` -- plain C
  nested loops (``spinsum_oracle.c``) with long-double accumulation,
  evaluating Def. 2-3 (Eq. 3-4) in the output-linear order of Alg. 1; a
  factorised sum (Def. 4, Eq. 5-6) is evaluated stage by stage through a full
  temporary, innermost factor first, as in Alg. 3.
* ``spinsum_numpy`` -- ``sum_t alpha_t * numpy.transpose(A, axes_t)``.
  ``numpy.transpose(A, q)`` realises the term whose permutation is the
  inverse of ``q``, so ``axes_t`` is the inverse of ``p_t``.
* ``dense_matrix`` -- the explicit matrix of the linear map, built with
  pure-Python loops for tiny tensors only.

Conventions (Def. 1-2): a permutation is a 0-based tuple ``p`` with
``p[m] = phi(m+1) - 1``; a term ``(p, alpha)`` adds
``alpha * A[..., i_{p[0]}, ..., i_{p[d-1]}, ...]`` to
``B[..., i_0, ..., i_{d-1}, ...]``.  Tensors are row-major numpy arrays; the
permuted group is the ``d`` dimensions starting at ``group_first``; the
dimensions before it are outer spectators and those after it inner
spectators.  A stage list is applied first-to-last (stage 0 innermost).

Index-pair form (``pairs=True``): the coupled-cluster quantities the paper's
summations act on (Sec. 1) carry their indices in pairs, e.g. T[a,b,c,i,j,k]
with (a,i), (b,j), (c,k) together.  Then the ``d`` dimensions right before
the group are permuted by the same ``p``:
``B[.., a_0..a_{d-1}, i_0..i_{d-1}, ..] += alpha *
A[.., a_{p[0]}..a_{p[d-1]}, i_{p[0]}..i_{p[d-1]}, ..]``.
"""
from __future__ import annotations

import ctypes
import math
import itertools
import os
import subprocess
from typing import Iterable, List, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "spinsum_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

Term = Tuple[Tuple[int, ...], float]
Stage = List[Term]

_lib = None


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc (no contraction into FMAs, OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-Wall", "-Wextra", "-o", _LIB + ".tmp", _SRC]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        i64p = ctypes.POINTER(ctypes.c_int64)
        ip = ctypes.POINTER(ctypes.c_int)
        dp = ctypes.POINTER(ctypes.c_double)
        for name in ("oracle_spinsum_chain", "oracle_spinsum_chain_adjoint"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          ip, ip, dp, dp, dp, ctypes.c_int]
        for name in ("oracle_spinsum_chain_ex", "oracle_spinsum_chain_adjoint_ex"):
            f = getattr(lib, name)
            f.restype = ctypes.c_int
            f.argtypes = [ctypes.c_int, i64p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                          ctypes.c_int, ip, ip, dp, dp, dp, ctypes.c_int]
        lib.oracle_max_threads.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


# ----------------------------------------------------------------- notation
def perm_from_paper(label: str) -> Tuple[int, ...]:
    """``"2134"`` (the subscript of pi in Def. 1) -> 0-based tuple (1,0,2,3)."""
    return tuple(int(c) - 1 for c in label)


def stage_from_paper(items: Iterable[Tuple[float, str]], d: int) -> Stage:
    """[(coef, "213"), ...] -> stage; a bare number c means c * identity."""
    out: Stage = []
    for coef, label in items:
        p = tuple(range(d)) if label in ("", "id") else perm_from_paper(label)
        if len(p) != d:
            raise ValueError(f"permutation {label!r} is not of degree {d}")
        out.append((p, float(coef)))
    return out


def _flatten(stages: Sequence[Stage], d: int):
    nterms = [len(s) for s in stages]
    perms = [int(v) for s in stages for (p, _) in s for v in p]
    alpha = [float(a) for s in stages for (_, a) in s]
    for s in stages:
        for p, _ in s:
            if len(p) != d:
                raise ValueError("permutation of wrong degree")
    return nterms, perms, alpha


def _call(fn_name: str, x: np.ndarray, stages: Sequence[Stage], group_first: int,
          d: int, nthreads: int, pairs: bool = False) -> np.ndarray:
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.empty_like(x)
    ext = (ctypes.c_int64 * x.ndim)(*x.shape)
    nterms, perms, alpha = _flatten(stages, d)
    nt = (ctypes.c_int * len(nterms))(*nterms)
    pp = (ctypes.c_int * max(1, len(perms)))(*perms)
    aa = (ctypes.c_double * max(1, len(alpha)))(*alpha)
    dp = ctypes.POINTER(ctypes.c_double)
    st = getattr(lib, fn_name + "_ex")(x.ndim, ext, group_first, d, int(bool(pairs)),
                                       len(stages), nt, pp, aa, x.ctypes.data_as(dp),
                                       out.ctypes.data_as(dp), int(nthreads))
    if st != 0:
        raise ValueError(f"{fn_name} failed with status {st}")
    return out


def spinsum(x: np.ndarray, terms: Stage, group_first: int, d: int,
            nthreads: int = 1, pairs: bool = False) -> np.ndarray:
    """B = sum_t alpha_t pi_t(A)  (Def. 3, Eq. 4)."""
    return _call("oracle_spinsum_chain", x, [terms], group_first, d, nthreads, pairs)


def spinsum_chain(x: np.ndarray, stages: Sequence[Stage], group_first: int, d: int,
                  nthreads: int = 1, pairs: bool = False) -> np.ndarray:
    """B = S_K(...S_1(A)) through full temporaries (Def. 4, Eq. 5-6; Alg. 3)."""
    return _call("oracle_spinsum_chain", x, list(stages), group_first, d, nthreads, pairs)


def spinsum_chain_adjoint(g: np.ndarray, stages: Sequence[Stage], group_first: int,
                          d: int, nthreads: int = 1, pairs: bool = False) -> np.ndarray:
    """S^T g for the chain (transpose of the linear map of Def. 3-4)."""
    return _call("oracle_spinsum_chain_adjoint", g, list(stages), group_first, d,
                 nthreads, pairs)


def expanded_terms(stages: Sequence[Stage], d: int) -> Stage:
    """The single sum that a chain of stages equals (Def. 4 multiplied out),
    as ``[(p, alpha_p)]`` over the permutations with nonzero coefficient, in
    lexicographic order.

    Found by applying the chain itself (the C loops above) to one indicator
    tensor: with N = d and In = 1 at the tuple (0, 1, .., d-1) only, an output
    position x that is itself a permutation tuple reads that 1 through the
    term p exactly when x_{p[m]} = m for every m, i.e. p is the inverse of x,
    so Out[x] is the coefficient of inverse(x).  Integer coefficients stay
    exact (long-double accumulation)."""
    shape = (d,) * d
    ind = np.zeros(shape, dtype=np.float64)
    ind[tuple(range(d))] = 1.0
    out = spinsum_chain(ind, stages, 0, d)
    terms = []
    for p in itertools.permutations(range(d)):
        c = float(out[_inverse(p)])
        if c != 0.0:
            terms.append((tuple(p), c))
    return terms


# ------------------------------------------------------------- numpy route
def _inverse(p: Sequence[int]) -> Tuple[int, ...]:
    inv = [0] * len(p)
    for m, v in enumerate(p):
        inv[v] = m
    return tuple(inv)


def coef_grad(x: np.ndarray, g: np.ndarray, group_first: int, d: int,
              nthreads: int = 1, pairs: bool = False) -> np.ndarray:
    """<g, pi_p(x)> for every permutation p of the group in lexicographic
    order: the derivative of <g, S(x)> with respect to the coefficient of p
    (S is linear in its coefficients, Def. 3), each term by the oracle's own
    single-term summation."""
    out = []
    for p in itertools.permutations(range(d)):
        y = spinsum(x, [(p, 1.0)], group_first, d, nthreads, pairs)
        out.append(float(np.sum(np.asarray(g, dtype=np.float64) * y, dtype=np.float64)))
    return np.array(out)


def coef_grad_stages(x: np.ndarray, g: np.ndarray, stages: Sequence[Stage], group_first: int,
                     d: int, nthreads: int = 1, pairs: bool = False) -> np.ndarray:
    """(stages, d!) array: entry (k, r) is the derivative of <g, S(x)> with
    respect to the coefficient of the r-th permutation (lexicographic order)
    in stage k of the chain S = S_K ... S_1 (Def. 4).  The chain is linear in
    each stage's coefficients, so that derivative is <g, chain(x)> with stage
    k replaced by the single term (p_r, 1): evaluated here by the oracle's
    own chain, term by term."""
    g = np.asarray(g, dtype=np.float64)
    out = np.zeros((len(stages), math.factorial(d)))
    for k in range(len(stages)):
        for r, p in enumerate(itertools.permutations(range(d))):
            chain = list(stages[:k]) + [[(p, 1.0)]] + list(stages[k + 1:])
            y = spinsum_chain(x, chain, group_first, d, nthreads, pairs)
            out[k, r] = float(np.sum(g * y, dtype=np.float64))
    return out


# ----------------------------------------------------------- unpacking
def increasing_tuples(n: int, d: int) -> List[Tuple[int, ...]]:
    """The strictly increasing d-tuples over range(n) in lexicographic order:
    the positions of a packed tensor (one value per tuple)."""
    return list(itertools.combinations(range(n), d))


def embed_packed(packed: np.ndarray, shape: Sequence[int], group_first: int,
                 d: int) -> np.ndarray:
    """A full tensor of `shape` that holds the packed values at the strictly
    increasing group positions and zeros elsewhere.  packed has the shape
    [outer..., C(N, d), inner...]."""
    shape = tuple(int(e) for e in shape)
    n = shape[group_first]
    full = np.zeros(shape, dtype=np.float64)
    packed = np.asarray(packed, dtype=np.float64)
    for r, t in enumerate(increasing_tuples(n, d)):
        idx = (slice(None),) * group_first + tuple(t)
        full[idx] = packed[(slice(None),) * group_first + (r,)]
    return full


def unpack(packed: np.ndarray, shape: Sequence[int], stages: Sequence[Stage],
           group_first: int, d: int, nthreads: int = 1) -> np.ndarray:
    """Unpacking as a sum of permutations (tensor unpacking, Sec. 1 and
    Sec. 7): S(E(packed)) with E the embedding above and S the chain; with S
    the antisymmetriser this is the unpacking of an antisymmetric tensor
    from its strictly increasing entries."""
    return spinsum_chain(embed_packed(packed, shape, group_first, d), stages, group_first, d,
                         nthreads)


def pack(full: np.ndarray, stages: Sequence[Stage], group_first: int, d: int,
         nthreads: int = 1) -> np.ndarray:
    """The adjoint of unpack: S^T applied to the full tensor, then its values
    at the strictly increasing group positions gathered in lexicographic
    order ([outer..., C(N, d), inner...])."""
    full = np.asarray(full, dtype=np.float64)
    n = full.shape[group_first]
    y = spinsum_chain_adjoint(full, stages, group_first, d, nthreads)
    tuples = increasing_tuples(n, d)
    out_shape = full.shape[:group_first] + (len(tuples),) + full.shape[group_first + d:]
    out = np.zeros(out_shape, dtype=np.float64)
    for r, t in enumerate(tuples):
        out[(slice(None),) * group_first + (r,)] = y[(slice(None),) * group_first + tuple(t)]
    return out


def spinsum_numpy(x: np.ndarray, terms: Stage, group_first: int, d: int,
                  pairs: bool = False) -> np.ndarray:
    """sum_t alpha_t * transpose(A) in float64 (second, independent route)."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nd = x.ndim
    for p, a in terms:
        if a == 0.0:
            continue
        q = _inverse(p)
        axes = list(range(nd))
        for m in range(d):
            axes[group_first + m] = group_first + q[m]
            if pairs:
                axes[group_first - d + m] = group_first - d + q[m]
        out += a * np.transpose(x, axes)
    return out


def spinsum_chain_numpy(x: np.ndarray, stages: Sequence[Stage], group_first: int,
                        d: int, pairs: bool = False) -> np.ndarray:
    y = np.asarray(x, dtype=np.float64)
    for s in stages:
        y = spinsum_numpy(y, s, group_first, d, pairs)
    return y


# ------------------------------------------------------------ dense matrix
def dense_matrix(shape: Sequence[int], terms: Stage, group_first: int, d: int,
                 pairs: bool = False) -> np.ndarray:
    """Explicit matrix M with vec(B) = M vec(A), row-major vec (tiny shapes).

    Built straight from Eq. 3: for every output multi-index and every term,
    M[out, source] += alpha_t, where source has the group tuple permuted.
    """
    shape = tuple(int(s) for s in shape)
    size = int(np.prod(shape)) if shape else 1
    if size > 4096:
        raise ValueError("dense_matrix is for tiny tensors only")
    M = np.zeros((size, size), dtype=np.float64)
    strides = [1] * len(shape)
    for k in range(len(shape) - 2, -1, -1):
        strides[k] = strides[k + 1] * shape[k + 1]
    for idx in itertools.product(*[range(s) for s in shape]):
        row = sum(i * s for i, s in zip(idx, strides))
        grp = idx[group_first:group_first + d]
        prt = idx[group_first - d:group_first] if pairs else ()
        for p, a in terms:
            src = list(idx)
            for m in range(d):
                src[group_first + m] = grp[p[m]]
                if pairs:
                    src[group_first - d + m] = prt[p[m]]
            col = sum(i * s for i, s in zip(src, strides))
            M[row, col] += a
    return M


def dense_chain_matrix(shape: Sequence[int], stages: Sequence[Stage], group_first: int,
                       d: int, pairs: bool = False) -> np.ndarray:
    size = int(np.prod(shape))
    M = np.eye(size)
    for s in stages:
        M = dense_matrix(shape, s, group_first, d, pairs) @ M
    return M
