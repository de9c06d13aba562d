"""spinsum_coef_grad_noalloc (the coefficient gradient with the library's
static partial-sum array, for callers that cannot allocate) against
spinsum_coef_grad on the same plan, through the C-ABI, on two calls in a row,
the second with a smaller input (run on an MI355X).

Bar: the d! sums are accumulated in double with atomics whose order varies,
so random inputs agree to the normwise FP64 tolerance (1e-14 of the largest
value); integer-valued inputs make every partial sum exact, so there the two
agree bit for bit."""
import numpy as np
import pytest
import torch

import workloads

pytestmark = pytest.mark.gpu

ss = pytest.importorskip("paper_1705_06661_amd")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

DEV = torch.device("cuda:0")


def _both(plan, x, g):
    ref = ss.spinsum_coef_grad(plan, x, g)
    got = torch.full_like(ref, float("nan"))
    ss.spinsum_coef_grad_noalloc(plan, x, g, got)
    torch.cuda.synchronize()
    return got.cpu().numpy(), ref.cpu().numpy()


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_noalloc_matches_coef_grad_twice_shrinking(dtype):
    cases = [((6, 32, 32, 32), 3, workloads.CONFIG_3D_ALPHA),      # tile orbits
             ((3, 8, 8, 8, 8), 4, workloads.random_4d_alpha(7))]   # whole cubes, smaller
    for k, (shape, d, alpha) in enumerate(cases):
        print("case", shape, dtype, flush=True)
        plan = ss.spinsum_plan(shape, 1, d, [alpha], dtype=dtype)
        x = workloads.uniform(shape, 900 + k, device=DEV, dtype=dtype)
        g = workloads.uniform(shape, 950 + k, device=DEV, dtype=dtype)
        got, ref = _both(plan, x, g)
        assert np.all(np.isfinite(got))
        assert np.max(np.abs(got - ref)) <= 1e-14 * np.max(np.abs(ref)), (got, ref)
        xi = workloads.integers(shape, 960 + k, device=DEV, dtype=dtype)
        gi = workloads.integers(shape, 970 + k, device=DEV, dtype=dtype)
        got, ref = _both(plan, xi, gi)
        np.testing.assert_array_equal(got, ref)


def test_noalloc_rejects_what_coef_grad_rejects():
    p = ss.spinsum_plan((3, 3, 3, 4, 4, 4), 3, 3, [workloads.CONFIG_3D_ALPHA],
                        flags=ss.SPINSUM_FLAG_INDEX_PAIRS)
    x = workloads.uniform((3, 3, 3, 4, 4, 4), 98, device=DEV)
    out = torch.empty(6, dtype=torch.float64, device=DEV)
    with pytest.raises(ss.SpinSumError) as e:
        ss.spinsum_coef_grad_noalloc(p, x, x, out)
    assert e.value.status == ss.SPINSUM_ERR_UNSUPPORTED
