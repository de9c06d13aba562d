"""Inf and NaN inputs (run on an MI355X).

A permutation whose coefficient is zero is not a term of the sum (Def. 3),
so an Inf or NaN input reaches exactly the outputs whose terms read it.  The
pre-multiplied form (the default) is the single sum the chain multiplies out
to, so its reference is the oracle on that sum (``oracle.expanded_terms``,
computed by the oracle alone); the chained form
(``SPINSUM_FLAG_CHAIN_STAGES``) applies the stages one after the other, so
its reference is the oracle's chain.  The two differ only where a product
cancels (the last operator below).

Bar: the positions of NaN, +Inf and -Inf equal the oracle's exactly, and the
finite outputs are within the normwise tolerance (1e-14 FP64, 2e-6 FP32).
"""
import itertools

import numpy as np
import pytest
import torch

import oracle
import workloads
from workloads import P, stage

pytestmark = pytest.mark.gpu

ss = pytest.importorskip("paper_1705_06661_amd")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")
TOL = {torch.float64: 1e-14, torch.float32: 2e-6}

OPS = {
    "config3d": (3, [workloads.CONFIG_3D_ALPHA]),          # every permutation present
    "factored": (3, workloads.FACTORED_PIJ_PJK),            # 4 of 6, stages of 2
    "table2_1": (3, workloads.table2_case(1)[1]),          # stages with zeros, product full
    "table2_2": (3, workloads.table2_case(2)[1]),
    "table2_5": (4, workloads.table2_case(5)[1]),
    "table2_18": (4, workloads.table2_case(18)[1]),
    "random4d": (4, [workloads.random_4d_alpha(7)]),        # one zero among 24
    "cancelling": (3, [stage((1, "123"), (1, "213")), stage((1, "123"), (-1, "213"))]),
}


def _say(*a):
    print(*a, flush=True)


def poisoned(shape, gf, d, seed, dtype=torch.float64, per_cube=3):
    """U(-1,1) values with a few Inf / -Inf / NaN entries in every cube (the
    group dims of one outer index), some on diagonals (equal group indices)."""
    x = workloads.uniform(shape, seed).numpy()
    rng = np.random.default_rng(seed)
    outer = shape[:gf]
    n = shape[gf]
    inner = shape[gf + d:]
    vals = [np.inf, -np.inf, np.nan]
    for o in itertools.product(*[range(e) for e in outer]):
        for k in range(per_cube):
            g = list(rng.integers(0, n, size=d))
            if k == 0 and d >= 2:
                g[1] = g[0]  # a degenerate element orbit
            r = tuple(int(rng.integers(0, e)) for e in inner)
            x[tuple(o) + tuple(int(v) for v in g) + r] = vals[(k + sum(o)) % 3]
    t = torch.from_numpy(x).to(dtype)
    return t


def reference(xh, stages, gf, d, chain, adjoint=False, pairs=False):
    terms = stages if chain else [oracle.expanded_terms(stages, d)]
    if adjoint:
        return oracle.spinsum_chain_adjoint(xh, terms, gf, d, nthreads=8, pairs=pairs)
    return oracle.spinsum_chain(xh, terms, gf, d, nthreads=8, pairs=pairs)


def same_pattern(got, ref, tol, what=""):
    got = np.asarray(got, dtype=np.float64)
    np.testing.assert_array_equal(np.isnan(got), np.isnan(ref), err_msg=f"NaN {what}")
    np.testing.assert_array_equal(np.isposinf(got), np.isposinf(ref), err_msg=f"+Inf {what}")
    np.testing.assert_array_equal(np.isneginf(got), np.isneginf(ref), err_msg=f"-Inf {what}")
    fin = np.isfinite(ref)
    scale = np.max(np.abs(ref[fin])) if fin.any() else 0.0
    if scale > 0:
        assert np.max(np.abs(got[fin] - ref[fin])) / scale <= tol, what
    return int((~fin).sum())


def run(plan, x, adjoint=False):
    if plan.inplace:
        y = x.clone()
        (ss.spinsum_adjoint if adjoint else ss.spinsum_exec)(plan, y, y)
    else:
        y = torch.empty_like(x)
        (ss.spinsum_adjoint if adjoint else ss.spinsum_exec)(plan, x, y)
    torch.cuda.synchronize()
    return y.cpu()


TILES = {3: [None, (4, 1, 0), (5, 1, 0), (4, 1, ss.SPINSUM_VARIANT_REG_ONESHOT),
             (12, 1, ss.SPINSUM_VARIANT_REG_PIPELINE), (3, 1, ss.SPINSUM_VARIANT_LDS_PIPELINE)],
         4: [None, (3, 1, 0), (4, 1, 0), (2, 1, ss.SPINSUM_VARIANT_REG_ONESHOT),
             (6, 1, ss.SPINSUM_VARIANT_LDS_PIPELINE)]}


@pytest.mark.parametrize("chain", [False, True])
@pytest.mark.parametrize("op", list(OPS))
def test_group_form(op, chain):
    d, stages = OPS[op]
    n = 12 if d == 3 else 6
    shape = (3,) + (n,) * d
    xh = poisoned(shape, 1, d, 300 + len(op))
    ref = reference(xh.numpy(), stages, 1, d, chain)
    x = xh.to(DEV)
    flags = ss.SPINSUM_FLAG_CHAIN_STAGES if chain else 0
    for tile in TILES[d]:
        for inplace in (False, True):
            p = ss.spinsum_plan(shape, 1, d, stages, inplace=inplace, flags=flags)
            if tile is not None:
                ss.spinsum_plan_set_tile(p, tile[0], tile[1], variant=tile[2])
            nf = same_pattern(run(p, x), ref, 1e-14, f"{op} chain={chain} tile={tile} ip={inplace}")
    _say(f"{op} chain={chain}: {nf} non-finite outputs of {ref.size}")


@pytest.mark.parametrize("chain", [False, True])
@pytest.mark.parametrize("op", ["factored", "table2_5", "random4d", "cancelling"])
def test_adjoint(op, chain):
    d, stages = OPS[op]
    n = 12 if d == 3 else 6
    shape = (2,) + (n,) * d
    gh = poisoned(shape, 1, d, 400 + len(op))
    ref = reference(gh.numpy(), stages, 1, d, chain, adjoint=True)
    flags = ss.SPINSUM_FLAG_CHAIN_STAGES if chain else 0
    for inplace in (False, True):
        p = ss.spinsum_plan(shape, 1, d, stages, inplace=inplace, flags=flags)
        same_pattern(run(p, gh.to(DEV), adjoint=True), ref, 1e-14, f"{op} adjoint ip={inplace}")


@pytest.mark.parametrize("chain", [False, True])
def test_fp32(chain):
    d, stages = OPS["factored"]
    shape = (3, 16, 16, 16)
    xh = poisoned(shape, 1, d, 500, dtype=torch.float32)
    ref = reference(xh.to(torch.float64).numpy(), stages, 1, d, chain)
    flags = ss.SPINSUM_FLAG_CHAIN_STAGES if chain else 0
    for tile in (None, (8, 1, 0)):
        p = ss.spinsum_plan(shape, 1, d, stages, dtype=torch.float32, flags=flags)
        if tile is not None:
            ss.spinsum_plan_set_tile(p, tile[0], tile[1], variant=tile[2])
        same_pattern(run(p, xh.to(DEV)), ref, 2e-6, f"fp32 tile={tile}")


@pytest.mark.parametrize("op", ["factored", "random4d", "cancelling"])
def test_inner_runs(op):
    d, stages = OPS[op]
    shape = (2, 6, 6, 6, 3) if d == 3 else (2, 4, 4, 4, 4, 3)
    xh = poisoned(shape, 1, d, 600)
    for chain in (False, True):
        ref = reference(xh.numpy(), stages, 1, d, chain)
        flags = ss.SPINSUM_FLAG_CHAIN_STAGES if chain else 0
        for tile in (None, (2, 1, 0)):
            p = ss.spinsum_plan(shape, 1, d, stages, inplace=True, flags=flags)
            if tile is not None:
                ss.spinsum_plan_set_tile(p, tile[0], tile[1], variant=tile[2])
            same_pattern(run(p, xh.to(DEV)), ref, 1e-14, f"{op} inner chain={chain} tile={tile}")


@pytest.mark.parametrize("op", ["factored", "table2_18", "random4d", "cancelling"])
def test_index_pairs(op):
    d, stages = OPS[op]
    shape = (2, 3, 3, 3, 4, 4, 4) if d == 3 else (2, 2, 2, 2, 2, 3, 3, 3, 3)
    gf = 1 + d
    xh = poisoned(shape, gf, d, 700)
    for chain in (False, True):
        ref = reference(xh.numpy(), stages, gf, d, chain, pairs=True)
        flags = ss.SPINSUM_FLAG_INDEX_PAIRS | (ss.SPINSUM_FLAG_CHAIN_STAGES if chain else 0)
        for inplace in (False, True):
            p = ss.spinsum_plan(shape, gf, d, stages, inplace=inplace, flags=flags)
            same_pattern(run(p, xh.to(DEV)), ref, 1e-14, f"{op} pairs chain={chain} ip={inplace}")
            if not chain:
                refa = reference(xh.numpy(), stages, gf, d, False, adjoint=True, pairs=True)
                same_pattern(run(p, xh.to(DEV), adjoint=True), refa, 1e-14, f"{op} pairs adjoint")


@pytest.mark.parametrize("op", ["factored", "table2_2", "cancelling"])
def test_batched(op):
    d, stages = OPS[op]
    blocks = [(3, 4), (2, 9), (5, 2), (1, 13), (4, 6), (2, 17)]
    shapes = [(v, v, v, o, o, o) for v, o in blocks]
    xs = [poisoned(s, 3, 3, 800 + k) for k, s in enumerate(shapes)]
    refs = [reference(x.numpy(), stages, 3, d, False) for x in xs]
    bp = ss.spinsum_plan_batched(shapes, 3, stages, inplace=True)
    ys = [x.to(DEV) for x in xs]
    ss.spinsum_exec_batched(bp, ys, ys)
    torch.cuda.synchronize()
    for k, (y, r) in enumerate(zip(ys, refs)):
        same_pattern(y.cpu(), r, 1e-14, f"{op} batched block {k}")
