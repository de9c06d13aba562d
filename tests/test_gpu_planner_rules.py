"""Parity of the plans the planner's size rules pick, on an MI355X, against
the oracle (Def. 3-4): whole cubes where tiles would be slow (no edge with
16-byte rows, ragged tiles, FP64 partial lines out of place), small tile
orbits on the register path, small whole cubes at least 8 KiB to a work
item, and the coefficient gradient's own tiles where whole cubes are too
large for both tensors.  Each case first checks (on the host) that the plan
is the one the rule describes, then compares forward, adjoint and, where
stated, the coefficient gradient with the oracle.

Bars: FP64 normwise 1e-14, FP32 2e-6 (against the oracle on the
FP32-rounded input); the coefficient gradient relative 1e-12.
"""
import numpy as np
import pytest
import torch

import oracle
import workloads

pytestmark = pytest.mark.gpu

ss = pytest.importorskip("paper_1705_06661_amd")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")
TOL = {torch.float64: 1e-14, torch.float32: 2e-6}


def nerr(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    scale = np.max(np.abs(ref))
    return float(np.max(np.abs(got - ref)) / scale) if scale > 0 else float(np.max(np.abs(got)))


CASES = [
    # (shape, group_first, dtype, inplace, expected bl, expected cubes per
    # workgroup; the small-cube cases have enough cubes for about eight
    # workgroups per CU at that count)
    ((3, 25, 25, 25), 1, torch.float64, True, 25, 1),     # no edge with 16-byte rows: whole
    ((2, 30, 30, 30), 1, torch.float32, False, 30, 1),    # the same in FP32
    ((3, 22, 22, 22), 1, torch.float64, True, 22, 1),     # 8^3 tiles would be ragged: whole
    ((2, 3, 24, 24, 24), 2, torch.float64, False, 24, 1),  # FP64 partial lines out of place
    ((2, 33, 33, 33), 1, torch.float64, True, 7, 1),      # register path, small tile orbits
    ((2, 37, 37, 37), 1, torch.float32, False, 9, 1),     # the same in FP32
    ((6200, 9, 9, 9), 1, torch.float32, True, 9, 3),      # three 9^3 FP32 cubes per item
    ((4200, 11, 11, 11), 1, torch.float32, True, 11, 2),  # two 11^3 FP32 cubes per item
    ((4200, 9, 9, 9), 1, torch.float64, False, 9, 2),     # two 9^3 FP64 cubes per item
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_planner_rule_plans_against_oracle(case):
    shape, gf, dtype, inplace, bl, cpw = CASES[case]
    d = 3
    stages = [workloads.CONFIG_3D_ALPHA] if case % 2 == 0 else workloads.FACTORED_PIJ_PJK
    p = ss.spinsum_plan(shape, gf, d, stages, dtype=dtype, inplace=inplace)
    info = ss.spinsum_plan_get_info(p)
    assert (info["bl"], info["cubes_per_wg"]) == (bl, cpw), info
    x = workloads.uniform(shape, 7100 + case, device=DEV, dtype=dtype)
    xh = x.cpu().to(torch.float64).numpy()
    ref = oracle.spinsum_chain(xh, stages, gf, d)
    y = x.clone() if inplace else torch.empty_like(x)
    ss.spinsum_exec(p, y if inplace else x, y)
    torch.cuda.synchronize()
    assert nerr(y.cpu().to(torch.float64).numpy(), ref) <= TOL[dtype]
    g = workloads.uniform(shape, 7200 + case, device=DEV, dtype=dtype)
    refa = oracle.spinsum_chain_adjoint(g.cpu().to(torch.float64).numpy(), stages, gf, d)
    ga = g.clone() if inplace else torch.empty_like(g)
    ss.spinsum_adjoint(p, ga if inplace else g, ga)
    torch.cuda.synchronize()
    assert nerr(ga.cpu().to(torch.float64).numpy(), refa) <= TOL[dtype]
    # integer-valued inputs: exact in both precisions
    xi = workloads.integers(shape, 7300 + case, device=DEV, dtype=dtype)
    refi = oracle.spinsum_chain(xi.cpu().to(torch.float64).numpy(), stages, gf, d)
    yi = xi.clone() if inplace else torch.empty_like(xi)
    ss.spinsum_exec(p, yi if inplace else xi, yi)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(yi.cpu().to(torch.float64).numpy(), refi)


@pytest.mark.parametrize("shape,gf", [((2, 3, 24, 24, 24), 2), ((3, 26, 26, 26), 1)])
def test_coef_grad_on_its_own_tiles_against_oracle(shape, gf):
    """Out of place, FP64 24^3 and 26^3 cubes are summed whole, too large for
    both tensors of the coefficient gradient in one CU's LDS: the gradient
    runs on tiles of its own, and matches the oracle."""
    d = 3
    p = ss.spinsum_plan(shape, gf, d, [workloads.CONFIG_3D_ALPHA])
    assert ss.spinsum_plan_get_info(p)["bl"] == shape[-1]
    x = workloads.uniform(shape, 7400, device=DEV)
    g = workloads.uniform(shape, 7401, device=DEV)
    got = ss.spinsum_coef_grad(p, x, g).cpu().numpy()
    ref = oracle.coef_grad(x.cpu().numpy(), g.cpu().numpy(), gf, d)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
