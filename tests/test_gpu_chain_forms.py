"""Chained summations on an MI355X: the multi-pass form (one launch per
stage, Alg. 3 with the output as its temporary) and the gradients with
respect to every stage's coefficients, against the oracle's chain.

Bars: FP64 normwise 1e-14, FP32 2e-6 (against the oracle on the FP32-rounded
input), integer-valued inputs bit for bit.  The multi-pass form and the stages
chained in registers agree bit for bit on integer inputs; on others they may
differ in the last bits at diagonal positions (an element orbit with equal
coordinates holds several register copies of one element, whose rounded
values differ between stages in registers, while memory keeps one).
"""
import itertools

import numpy as np
import pytest
import torch

import oracle
import workloads
from workloads import stage

pytestmark = pytest.mark.gpu

ss = pytest.importorskip("paper_1705_06661_amd")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")
TOL = {torch.float64: 1e-14, torch.float32: 2e-6}

CHAINS = {
    "factored": (3, workloads.FACTORED_PIJ_PJK),
    "table2_1": (3, workloads.table2_case(1)[1]),
    "table2_5": (4, workloads.table2_case(5)[1]),
    "table2_9": (4, workloads.table2_case(9)[1]),
}


def _say(*a):
    print(*a, flush=True)


def nerr(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.max(np.abs(ref))
    return float(np.max(np.abs(got - ref)) / scale) if scale > 0 else float(np.max(np.abs(got)))


def shape_of(d):
    return (3, 12, 12, 12) if d == 3 else (2, 6, 6, 6, 6)


def run(plan, x, adjoint=False):
    f = ss.spinsum_adjoint if adjoint else ss.spinsum_exec
    if plan.inplace:
        y = x.clone()
        f(plan, y, y)
    else:
        y = torch.empty_like(x)
        f(plan, x, y)
    torch.cuda.synchronize()
    return y


@pytest.mark.parametrize("name", list(CHAINS))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_multi_pass_against_oracle(name, dtype):
    d, stages = CHAINS[name]
    shape = shape_of(d)
    n = shape[1]
    x = workloads.uniform(shape, 1200 + d, device=DEV, dtype=dtype)
    xh = x.cpu().to(torch.float64).numpy()
    ref = oracle.spinsum_chain(xh, stages, 1, d, nthreads=8)
    refa = oracle.spinsum_chain_adjoint(xh, stages, 1, d, nthreads=8)
    xi = workloads.integers(shape, 1300 + d, device=DEV, dtype=dtype)
    refi = oracle.spinsum_chain(xi.cpu().to(torch.float64).numpy(), stages, 1, d)
    for tile in (None, (4 if d == 3 else 3, 1)):
        for inplace in (False, True):
            _say(name, dtype, tile, inplace)
            p = ss.spinsum_plan(shape, 1, d, stages, dtype=dtype, inplace=inplace,
                                flags=ss.SPINSUM_FLAG_MULTI_PASS)
            c = ss.spinsum_plan(shape, 1, d, stages, dtype=dtype, inplace=inplace,
                                flags=ss.SPINSUM_FLAG_CHAIN_STAGES)
            if tile is not None:
                ss.spinsum_plan_set_tile(p, *tile)
                ss.spinsum_plan_set_tile(c, *tile)
            y = run(p, x)
            assert nerr(y.cpu().numpy(), ref) <= TOL[dtype]
            assert nerr(run(c, x).cpu().numpy(), y.cpu().numpy()) <= TOL[dtype]
            ya = run(p, x, adjoint=True)
            assert nerr(ya.cpu().numpy(), refa) <= TOL[dtype]
            assert nerr(run(c, x, adjoint=True).cpu().numpy(), ya.cpu().numpy()) <= TOL[dtype]
            yi = run(p, xi)
            np.testing.assert_array_equal(yi.cpu().to(torch.float64).numpy(), refi)
            assert torch.equal(yi, run(c, xi))
    assert n > 0


def test_multi_pass_index_pairs_and_inner_runs():
    st = workloads.FACTORED_PIJ_PJK
    for shape, gf, flags in [((2, 3, 3, 3, 4, 4, 4), 4, ss.SPINSUM_FLAG_INDEX_PAIRS),
                             ((2, 6, 6, 6, 3), 1, 0)]:
        x = workloads.uniform(shape, 1400, device=DEV)
        ref = oracle.spinsum_chain(x.cpu().numpy(), st, gf, 3,
                                   pairs=bool(flags & ss.SPINSUM_FLAG_INDEX_PAIRS))
        for inplace in (False, True):
            p = ss.spinsum_plan(shape, gf, 3, st, inplace=inplace,
                                flags=flags | ss.SPINSUM_FLAG_MULTI_PASS)
            assert nerr(run(p, x).cpu().numpy(), ref) <= 1e-14


def test_multi_pass_rejects_chain_flag():
    with pytest.raises(ss.SpinSumError) as e:
        ss.spinsum_plan((2, 4, 4, 4), 1, 3, workloads.FACTORED_PIJ_PJK,
                        flags=ss.SPINSUM_FLAG_MULTI_PASS | ss.SPINSUM_FLAG_CHAIN_STAGES)
    assert e.value.status == ss.SPINSUM_ERR_INVALID_ARG


def test_multi_pass_non_finite_inputs_follow_the_chain():
    """Each launch skips its own stage's zero coefficients, so Inf/NaN inputs
    give the oracle chain's pattern (as the stages chained in registers)."""
    cancel = [stage((1, "123"), (1, "213")), stage((1, "123"), (-1, "213"))]
    for stages in (workloads.FACTORED_PIJ_PJK, cancel):
        shape = (2, 8, 8, 8)
        xh = workloads.uniform(shape, 1500).numpy()
        xh[0, 1, 2, 3] = np.inf
        xh[1, 4, 4, 0] = np.nan
        xh[1, 7, 2, 2] = -np.inf
        ref = oracle.spinsum_chain(xh, stages, 1, 3)
        p = ss.spinsum_plan(shape, 1, 3, stages, flags=ss.SPINSUM_FLAG_MULTI_PASS)
        y = run(p, torch.from_numpy(xh).to(DEV)).cpu().numpy()
        np.testing.assert_array_equal(np.isnan(y), np.isnan(ref))
        np.testing.assert_array_equal(np.isposinf(y), np.isposinf(ref))
        np.testing.assert_array_equal(np.isneginf(y), np.isneginf(ref))
        fin = np.isfinite(ref)
        assert nerr(y[fin], ref[fin]) <= 1e-14


@pytest.mark.parametrize("name", list(CHAINS))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_coef_grad_stages_against_oracle(name, dtype):
    d, stages = CHAINS[name]
    shape = shape_of(d)
    x = workloads.uniform(shape, 1600 + d, device=DEV, dtype=dtype)
    g = workloads.uniform(shape, 1700 + d, device=DEV, dtype=dtype)
    xh = x.cpu().to(torch.float64).numpy()
    gh = g.cpu().to(torch.float64).numpy()
    ref = oracle.coef_grad_stages(xh, gh, stages, 1, d, nthreads=8)
    for flags in (0, ss.SPINSUM_FLAG_CHAIN_STAGES):
        p = ss.spinsum_plan(shape, 1, d, stages, dtype=dtype, flags=flags)
        got = ss.spinsum_coef_grad_stages(p, x, g).cpu().numpy()
        _say(name, dtype, flags, nerr(got, ref))
        assert nerr(got, ref) <= TOL[dtype]
    # integer inputs: every intermediate and every partial sum is exact
    xi = workloads.integers(shape, 1800 + d, device=DEV, dtype=dtype)
    gi = workloads.integers(shape, 1900 + d, device=DEV, dtype=dtype)
    refi = oracle.coef_grad_stages(xi.cpu().to(torch.float64).numpy(),
                                   gi.cpu().to(torch.float64).numpy(), stages, 1, d, nthreads=8)
    p = ss.spinsum_plan(shape, 1, d, stages, dtype=dtype)
    if dtype == torch.float64:
        np.testing.assert_array_equal(ss.spinsum_coef_grad_stages(p, xi, gi).cpu().numpy(), refi)


def test_coef_grad_stages_one_stage_and_errors():
    shape = (3, 8, 8, 8)
    x = workloads.uniform(shape, 2000, device=DEV)
    g = workloads.uniform(shape, 2001, device=DEV)
    p = ss.spinsum_plan(shape, 1, 3, [workloads.CONFIG_3D_ALPHA])
    a = ss.spinsum_coef_grad_stages(p, x, g)
    b = ss.spinsum_coef_grad(p, x, g)
    assert a.shape == (1, 6)
    assert nerr(a[0].cpu().numpy(), b.cpu().numpy()) <= 1e-14
    q = ss.spinsum_plan(shape, 1, 3, workloads.FACTORED_PIJ_PJK)
    with pytest.raises(ss.SpinSumError) as e:
        ss.spinsum_coef_grad_stages(q, x, g, work=(x, torch.empty_like(x)))
    assert e.value.status == ss.SPINSUM_ERR_ALIASING


@pytest.mark.parametrize("shape,gf,d,name", [((2, 3, 3, 3), 1, 3, "factored"),
                                             ((1, 2, 2, 2, 2), 1, 4, "table2_5")])
def test_chain_coef_autograd(shape, gf, d, name):
    """SpinSumChainCoefFunction: gradcheck through x and every stage's
    coefficients, and both gradients against the dense matrices."""
    _, stages = CHAINS[name]
    merged = []
    for st in stages:  # distinct permutations per stage (duplicates merged)
        m = {}
        for p, a in st:
            m[p] = m.get(p, 0.0) + a
        merged.append(m)
    perms = [list(m) for m in merged]
    alpha0 = [a for m in merged for a in m.values()]
    x = workloads.uniform(shape, 2100, device=DEV).requires_grad_(True)
    alpha = torch.tensor(alpha0, dtype=torch.float64, device=DEV, requires_grad=True)
    for flags in (ss.SPINSUM_FLAG_CHAIN_STAGES, 0, ss.SPINSUM_FLAG_MULTI_PASS):
        f = lambda xx, aa: ss.SpinSumChainCoefFunction.apply(xx, aa, perms, gf, flags)
        assert torch.autograd.gradcheck(f, (x, alpha), eps=1e-3, atol=1e-9, rtol=1e-9)
        g = workloads.uniform(shape, 2200, device=DEV)
        y = f(x, alpha)
        gx, ga = torch.autograd.grad(y, (x, alpha), g)
        st = [[(p, a) for p, a in m.items()] for m in merged]
        M = oracle.dense_chain_matrix(shape, st, gf, d)
        np.testing.assert_allclose(gx.cpu().numpy().ravel(), M.T @ g.cpu().numpy().ravel(),
                                   rtol=0, atol=1e-12)
        want = []
        for k, m in enumerate(merged):
            for p in m:
                mats = [oracle.dense_matrix(shape, s_, gf, d) for s_ in st]
                mats[k] = oracle.dense_matrix(shape, [(p, 1.0)], gf, d)
                T = np.eye(x.numel())
                for mm in mats:
                    T = mm @ T
                want.append(g.cpu().numpy().ravel() @ (T @ x.detach().cpu().numpy().ravel()))
        np.testing.assert_allclose(ga.cpu().numpy(), np.array(want), rtol=1e-12, atol=1e-12)
