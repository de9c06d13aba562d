"""Seeded synthetic inputs and workload definitions for spin summations.

This module holds no arithmetic of the method itself.  It provides:

* a counter-based generator: splitmix64 (Steele, Lea & Flood, "Fast
  splittable pseudorandom number generators", OOPSLA 2014) applied to the
  counter ``(seed << 40) + linear_index``; the top 53 bits of the mixed word
  give u in [0, 1) and the value is ``2u - 1`` in [-1, 1).  The same
  function, written with torch int64 ops (wrap-around multiply, masked
  shifts), runs on the CPU or on a GPU and gives bit-identical values, so a
  test can regenerate any spectator cube of a multi-GB tensor on the host
  without copying the tensor back;
* integer-valued inputs (|x| <= 1024) from the same counter, for which every
  summation order is exact;
* the coefficient sets and shapes of the workloads (Table II of the paper,
  the 3D/4D amplitude-tensor configurations), and the power-law block list
  of the batched workload.

Coefficient sets are given as stages of ``(perm, alpha)`` terms with 0-based
permutations ``p[m] = phi(m+1) - 1`` (Def. 1); stage 0 is applied first.
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Sequence, Tuple

import numpy as np
import torch

Term = Tuple[Tuple[int, ...], float]
Stage = List[Term]

# ---------------------------------------------------------------- generator
_GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_SEED_SHIFT = 40
_CHUNK = 1 << 25


def _i64(c: int) -> int:
    """Unsigned 64-bit constant as the int64 with the same bit pattern."""
    c &= (1 << 64) - 1
    return c - (1 << 64) if c >= (1 << 63) else c


def _lsr(z: torch.Tensor, s: int) -> torch.Tensor:
    """Logical right shift of int64 bit patterns."""
    return torch.bitwise_and(torch.bitwise_right_shift(z, s), (1 << (64 - s)) - 1)


def _mix(idx: torch.Tensor, seed: int) -> torch.Tensor:
    """splitmix64 output for counters (seed << 40) + idx, as int64 bits."""
    if not (0 <= seed < (1 << 23)):
        raise ValueError("seed must be in [0, 2^23)")
    z = (idx + (seed << _SEED_SHIFT) + 1) * _i64(_GOLDEN)
    z = torch.bitwise_xor(z, _lsr(z, 30)) * _i64(_M1)
    z = torch.bitwise_xor(z, _lsr(z, 27)) * _i64(_M2)
    return torch.bitwise_xor(z, _lsr(z, 31))


def _fill(out: torch.Tensor, seed: int, offset: int, kind: str) -> torch.Tensor:
    flat = out.view(-1)
    n = flat.numel()
    for s in range(0, n, _CHUNK):
        e = min(n, s + _CHUNK)
        idx = torch.arange(offset + s, offset + e, dtype=torch.int64, device=out.device)
        z = _mix(idx, seed)
        top = _lsr(z, 11)  # 53 bits
        if kind == "uniform":
            u = top.to(torch.float64) * (2.0 ** -53)
            flat[s:e] = (2.0 * u - 1.0).to(out.dtype)
        else:
            flat[s:e] = (torch.remainder(top, 2049) - 1024).to(out.dtype)
        del idx, z, top
    return out


def fill_uniform(t: torch.Tensor, seed: int, offset: int = 0) -> torch.Tensor:
    """Fill a contiguous tensor in place with the U(-1,1) stream."""
    return _fill(t, seed, offset, "uniform")


def uniform(shape: Sequence[int], seed: int, device="cpu", dtype=torch.float64,
            offset: int = 0) -> torch.Tensor:
    """U(-1,1) values for linear indices offset .. offset+numel-1.

    FP32 tensors hold the FP64 values rounded to nearest.
    """
    out = torch.empty(tuple(shape), dtype=dtype, device=device)
    return _fill(out, seed, offset, "uniform")


def integers(shape: Sequence[int], seed: int, device="cpu", dtype=torch.float64,
             offset: int = 0) -> torch.Tensor:
    """Integer values in [-1024, 1024] stored as floating point."""
    out = torch.empty(tuple(shape), dtype=dtype, device=device)
    return _fill(out, seed, offset, "integers")


def uniform_numpy(n: int, seed: int, offset: int = 0) -> np.ndarray:
    """The same stream computed with numpy uint64 (well-defined wrap-around)."""
    return uniform_numpy_at(np.arange(offset, offset + n, dtype=np.uint64), seed)


def uniform_numpy_at(index: np.ndarray, seed: int) -> np.ndarray:
    """The stream at arbitrary linear indices (any shape)."""
    with np.errstate(over="ignore"):
        k = np.asarray(index, dtype=np.uint64) + np.uint64(
            (seed << _SEED_SHIFT) + 1)
        z = k * np.uint64(_GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return 2.0 * u - 1.0


# --------------------------------------------------------- coefficient sets
def P(label: str) -> Tuple[int, ...]:
    """Paper subscript (Def. 1) -> 0-based permutation tuple."""
    return tuple(int(c) - 1 for c in label)


def stage(*items) -> Stage:
    """stage((2, "123"), (-1, "213")) -> [((0,1,2), 2.0), ((1,0,2), -1.0)]."""
    return [(P(lbl), float(c)) for c, lbl in items]


# The 3D amplitude-tensor coefficient set: identity 4, each transposition -2,
# each 3-cycle +1.  It equals the expansion of Table II case 1.
CONFIG_3D_ALPHA: Stage = stage((4, "123"), (-2, "213"), (-2, "321"), (-2, "132"),
                               (1, "231"), (1, "312"))

# (2 - P_ij)(2 - P_jk), with P_ij = pi_213 and P_jk = pi_132; the right-hand
# factor is applied first.
FACTORED_PIJ_PJK: List[Stage] = [stage((2, "123"), (-1, "132")),
                                 stage((2, "123"), (-1, "213"))]

# Table II, transcribed as printed; each case is a list of stages, innermost
# (right-most parenthesis) first.  "2" is 2 * identity.
_TABLE2_TEXT: Dict[int, List[List[str]]] = {
    1: [["2", "-321", "-132"], ["2", "-213"]],
    2: [["2", "-321", "-132"]],
    3: [["2", "-213", "-132"]],
    4: [["2", "-213", "-321"]],
    5: [["2", "-4231", "-1432", "-1243"], ["2", "-3214", "-1324"], ["2", "-2134"]],
    6: [["2", "-4231", "-1432", "-1243"], ["2", "-3214", "-1324"]],
    7: [["2", "-4231", "-1432", "-1243"], ["2", "-2134", "-1324"]],
    8: [["2", "-4231", "-1432", "-4231"], ["2", "-2134", "-3214"]],
    9: [["2", "-3214", "-1324", "-4231"], ["2", "-4231", "-1432"]],
    10: [["2", "-3214", "-1324", "-4231"], ["2", "-2134", "-1432"]],
    11: [["2", "-3214", "-1324", "-1234"], ["2", "-2134", "-4231"]],
    12: [["2", "-2134", "-1324", "-1432"], ["2", "-4231", "-1243"]],
    13: [["2", "-2134", "-1324", "-1432"], ["2", "-3214", "-1243"]],
    14: [["2", "-2134", "-1324", "-1432"], ["2", "-3214", "-4231"]],
    15: [["2", "-2134", "-3214", "-4231"], ["2", "-1432", "-1243"]],
    16: [["2", "-2134", "-3214", "-4231"], ["2", "-1432", "-1243"]],
    17: [["2", "-2134", "-3214", "-4231"], ["2", "-1432", "-1432"]],
    18: [["2", "-4231", "-1432", "-1243"]],
    19: [["2", "-3214", "-1324", "-1243"]],
    20: [["2", "-2134", "-1324", "-1432"]],
    21: [["2", "-2134", "-3214", "-4231"]],
}


def table2_case(case: int) -> Tuple[int, List[Stage]]:
    """(d, stages) of Table II case ``case`` exactly as printed."""
    text = _TABLE2_TEXT[case]
    d = 3 if case <= 4 else 4
    ident = "".join(str(m + 1) for m in range(d))
    stages = []
    for st in text:
        items = []
        for tok in st:
            if tok == "2":
                items.append((2.0, ident))
            else:
                items.append((-1.0, tok.lstrip("-")))
        stages.append(stage(*items))
    return d, stages


def _parity(p) -> int:
    inv = sum(1 for i in range(len(p)) for j in range(i + 1, len(p)) if p[i] > p[j])
    return -1 if inv % 2 else 1


def symmetrizer(d: int) -> Stage:
    """sum over all permutations of the group (every coefficient +1)."""
    return [(p, 1.0) for p in itertools.permutations(range(d))]


def antisymmetrizer(d: int) -> Stage:
    """sum over all permutations weighted by their sign."""
    return [(p, float(_parity(p))) for p in itertools.permutations(range(d))]


def random_4d_alpha(seed: int) -> Stage:
    """24 integer coefficients in {-2..8} drawn from ``seed`` (numpy PCG64),
    assigned to the permutations of (0,1,2,3) in lexicographic order."""
    rng = np.random.default_rng(seed)
    a = rng.integers(-2, 9, size=24)
    return [(tuple(p), float(c)) for p, c in zip(itertools.permutations(range(4)), a)]


# ------------------------------------------------------------------ shapes
WORKLOADS = {
    # 3D, T[a,b,c,i,j,k], a,b,c in [0,16), i,j,k in [0,8)
    "3d_v16_o8": dict(shape=(16, 16, 16, 8, 8, 8), group_first=3, d=3),
    # 3D slab of the v=64, o=32 tensor: 64 x 64 x 8 x 32^3 (1.07G elements)
    "3d_v64_o32_slab": dict(shape=(64, 64, 8, 32, 32, 32), group_first=3, d=3, nslabs=8),
    # 4D a-slab of the v=24, o=12 tensor: 1 x 24^3 x 12^4 (287M elements)
    "4d_v24_o12_slab": dict(shape=(1, 24, 24, 24, 12, 12, 12, 12), group_first=4, d=4,
                            nslabs=24),
    # 3D v=48, o=24 forward/backward (1.53G elements)
    "3d_v48_o24": dict(shape=(48, 48, 48, 24, 24, 24), group_first=3, d=3),
}


def power_law(rng: np.random.Generator, lo: int, hi: int, expo: float, size: int):
    """Integers in [lo, hi] with P(x) proportional to x^-expo."""
    xs = np.arange(lo, hi + 1, dtype=np.float64)
    w = xs ** (-expo)
    w /= w.sum()
    return rng.choice(np.arange(lo, hi + 1), size=size, p=w)


def batched_blocks(nblocks: int = 200, target_bytes: float = 2.0e9,
                   tol: float = 0.05e9, expo: float = 1.75, first_seed: int = 0,
                   elem_bytes: int = 8):
    """Symmetry blocks [v,v,v,o,o,o] with v in [4,40], o in [2,16] drawn from a
    power law; seeds are searched upward from ``first_seed`` until the total
    size is within ``tol`` of ``target_bytes``.  Returns (seed, [(v, o), ...])."""
    seed = first_seed
    while True:
        rng = np.random.default_rng(seed)
        v = power_law(rng, 4, 40, expo, nblocks)
        o = power_law(rng, 2, 16, expo, nblocks)
        total = float(np.sum(elem_bytes * (v.astype(np.float64) ** 3) * (o.astype(np.float64) ** 3)))
        if abs(total - target_bytes) <= tol:
            return seed, [(int(a), int(b)) for a, b in zip(v, o)]
        seed += 1
        if seed > first_seed + 100000:
            raise RuntimeError("no seed found for the batched block list")
