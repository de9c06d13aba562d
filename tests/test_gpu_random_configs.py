"""A seeded sweep of random configurations on an MI355X against the oracle.

Each case draws the group size d, the extent N (ragged tiles included), outer
and inner spectator dims, the storage type, in place or not, an operator of
one to three stages with integer coefficients in [-3, 3] over a random subset
of the permutations (zero coefficients included), a random subset of the plan
flags that change the form or the schedule, and sometimes a tile override.
Checked through the C-ABI:
- forward and adjoint against the oracle's chain and its transpose;
- integer-valued inputs bit for bit wherever every intermediate is exact in
  the storage type.

The error is measured against the a-priori scale of a chain of sums,
prod_s(sum_t |alpha_{s,t}|) * max|x|, which bounds every intermediate: a
random operator can cancel to a result far smaller than its terms, where
max|ref| would measure rounding that the terms, not the result, set.
"""
import itertools

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
EXACT = {torch.float64: 2.0 ** 53, torch.float32: 2.0 ** 24}
NCASES = 160

SCHEDULE_FLAGS = ["SPINSUM_FLAG_NO_XCD_REMAP", "SPINSUM_FLAG_REVERSE_ORDER",
                  "SPINSUM_FLAG_NO_LDS_PAD", "SPINSUM_FLAG_NO_DIRECT_LDS",
                  "SPINSUM_FLAG_NO_NT_STORES", "SPINSUM_FLAG_NT_STORES",
                  "SPINSUM_FLAG_NO_NT_LOADS", "SPINSUM_FLAG_FULL_GROUP"]
VARIANTS = [ss.SPINSUM_VARIANT_AUTO, ss.SPINSUM_VARIANT_DIRECT_LDS,
            ss.SPINSUM_VARIANT_REG_PIPELINE, ss.SPINSUM_VARIANT_REG_ONESHOT,
            ss.SPINSUM_VARIANT_LDS_PIPELINE]


def _say(*a):
    print(*a, flush=True)


def draw(case):
    rng = np.random.default_rng(7000 + case)
    d = int(rng.choice([2, 3, 4], p=[0.2, 0.5, 0.3]))
    if rng.random() < 0.3:  # cubes that several work items share
        n = int(rng.integers(1, {2: 160, 3: 48, 4: 20}[d] + 1))
        outer = [int(v) for v in rng.integers(1, 3, size=int(rng.integers(0, 2)))]
    else:
        n = int(rng.integers(1, {2: 40, 3: 17, 4: 9}[d] + 1))
        outer = [int(v) for v in rng.integers(1, 4, size=int(rng.integers(0, 3)))]
    inner = [int(v) for v in rng.integers(1, 6, size=int(rng.integers(0, 2)))]
    perms = list(itertools.permutations(range(d)))
    stages = []
    for _ in range(int(rng.integers(1, 4))):
        k = int(rng.integers(1, len(perms) + 1))
        pick = rng.choice(len(perms), size=k, replace=False)
        stages.append([(perms[i], float(rng.integers(-3, 4))) for i in pick])
    form = rng.choice(["expanded", "chained", "multi_pass"], p=[0.5, 0.3, 0.2])
    flags = {"expanded": 0, "chained": ss.SPINSUM_FLAG_CHAIN_STAGES,
             "multi_pass": ss.SPINSUM_FLAG_MULTI_PASS}[form]
    for name in SCHEDULE_FLAGS:
        if rng.random() < 0.15:
            flags |= getattr(ss, name)
    if flags & ss.SPINSUM_FLAG_NT_STORES:
        flags &= ~ss.SPINSUM_FLAG_NO_NT_STORES
    tile = None
    if rng.random() < 0.3 and n > 0:
        tile = (int(rng.integers(1, n + 1)), int(VARIANTS[rng.integers(0, len(VARIANTS))]))
    return dict(shape=tuple(outer + [n] * d + inner), gf=len(outer), d=d, stages=stages,
                dtype=torch.float64 if rng.random() < 0.6 else torch.float32,
                inplace=bool(rng.random() < 0.5), flags=int(flags), tile=tile)


def make_plan(c):
    p = ss.spinsum_plan(c["shape"], c["gf"], c["d"], c["stages"], dtype=c["dtype"],
                        inplace=c["inplace"], flags=c["flags"])
    if c["tile"] is not None:
        bl, variant = c["tile"]
        try:
            ss.spinsum_plan_set_tile(p, bl, variant=variant)
        except ss.SpinSumError as e:
            # a tile the library refuses (LDS size, row alignment, variant):
            # a clear error, and a fresh plan keeps the default tiling
            assert e.status in (ss.SPINSUM_ERR_UNSUPPORTED, ss.SPINSUM_ERR_INVALID_ARG), e
            p = ss.spinsum_plan(c["shape"], c["gf"], c["d"], c["stages"], dtype=c["dtype"],
                                inplace=c["inplace"], flags=c["flags"])
    return p


def apply(p, x, adjoint=False):
    f = ss.spinsum_adjoint if adjoint else ss.spinsum_exec
    if p.inplace:
        y = x.clone()
        f(p, y, y)
    else:
        y = torch.empty_like(x)
        f(p, x, y)
    torch.cuda.synchronize()
    return y


@pytest.mark.parametrize("case", range(NCASES))
def test_random_configuration(case):
    c = draw(case)
    _say("case", case, {k: c[k] for k in ("shape", "gf", "d", "dtype", "inplace", "flags", "tile")},
         "stages", [len(s) for s in c["stages"]])
    p = make_plan(c)
    gf, d, stages, dtype = c["gf"], c["d"], c["stages"], c["dtype"]
    gain = float(np.prod([sum(abs(a) for _, a in s) for s in stages]))
    x = workloads.uniform(c["shape"], 7100 + case, device=DEV, dtype=dtype)
    if x.numel() == 0:
        assert apply(p, x).numel() == 0
        return
    xh = x.cpu().to(torch.float64).numpy()
    scale = max(gain * float(np.max(np.abs(xh))), np.finfo(np.float64).tiny)
    ref = oracle.spinsum_chain(xh, stages, gf, d, nthreads=8)
    got = apply(p, x).cpu().to(torch.float64).numpy()
    assert np.max(np.abs(got - ref)) <= TOL[dtype] * scale, "forward"
    refa = oracle.spinsum_chain_adjoint(xh, stages, gf, d, nthreads=8)
    gota = apply(p, x, adjoint=True).cpu().to(torch.float64).numpy()
    assert np.max(np.abs(gota - refa)) <= TOL[dtype] * scale, "adjoint"
    if gain * 1024.0 < EXACT[dtype]:
        xi = workloads.integers(c["shape"], 7200 + case, device=DEV, dtype=dtype)
        refi = oracle.spinsum_chain(xi.cpu().to(torch.float64).numpy(), stages, gf, d)
        np.testing.assert_array_equal(apply(p, xi).cpu().to(torch.float64).numpy(), refi)
