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


def random_stages(rng, d, kmax=3):
    perms = list(itertools.permutations(range(d)))
    stages = []
    for _ in range(int(rng.integers(1, kmax + 1))):
        k = int(rng.integers(1, len(perms) + 1))
        pick = rng.choice(len(perms), size=k, replace=False)
        stages.append([(perms[i], float(rng.integers(-3, 4))) for i in pick])
    return stages


def gain_of(stages):
    return float(np.prod([sum(abs(a) for _, a in s) for s in stages]))


@pytest.mark.parametrize("case", range(40))
def test_random_index_pairs(case):
    """Index-pair plans (the d dims before the group permuted with it):
    forward and adjoint against the oracle's pair form, integers bitwise."""
    rng = np.random.default_rng(7300 + case)
    d = int(rng.choice([2, 3, 4], p=[0.3, 0.5, 0.2]))
    v = int(rng.integers(1, {2: 9, 3: 6, 4: 3}[d] + 1))
    n = int(rng.integers(1, {2: 16, 3: 9, 4: 5}[d] + 1))
    outer = [int(e) for e in rng.integers(1, 3, size=int(rng.integers(0, 2)))]
    inner = [int(e) for e in rng.integers(1, 4, size=int(rng.integers(0, 2)))]
    shape = tuple(outer + [v] * d + [n] * d + inner)
    gf = len(outer) + d
    stages = random_stages(rng, d)
    dtype = torch.float64 if rng.random() < 0.6 else torch.float32
    inplace = bool(rng.random() < 0.5)
    flags = ss.SPINSUM_FLAG_INDEX_PAIRS
    if rng.random() < 0.3:
        flags |= ss.SPINSUM_FLAG_CHAIN_STAGES
    for name in ("SPINSUM_FLAG_NO_XCD_REMAP", "SPINSUM_FLAG_REVERSE_ORDER",
                 "SPINSUM_FLAG_NO_NT_STORES"):
        if rng.random() < 0.2:
            flags |= getattr(ss, name)
    _say("pairs", case, shape, gf, d, dtype, inplace, hex(flags), [len(s) for s in stages])
    p = ss.spinsum_plan(shape, gf, d, stages, dtype=dtype, inplace=inplace, flags=flags)
    x = workloads.uniform(shape, 7400 + case, device=DEV, dtype=dtype)
    xh = x.cpu().to(torch.float64).numpy()
    scale = max(gain_of(stages) * float(np.max(np.abs(xh))), np.finfo(np.float64).tiny)
    ref = oracle.spinsum_chain(xh, stages, gf, d, nthreads=8, pairs=True)
    assert np.max(np.abs(apply(p, x).cpu().to(torch.float64).numpy() - ref)) <= TOL[dtype] * scale
    refa = oracle.spinsum_chain_adjoint(xh, stages, gf, d, nthreads=8, pairs=True)
    gota = apply(p, x, adjoint=True).cpu().to(torch.float64).numpy()
    assert np.max(np.abs(gota - refa)) <= TOL[dtype] * scale
    if gain_of(stages) * 1024.0 < EXACT[dtype]:
        xi = workloads.integers(shape, 7500 + case, device=DEV, dtype=dtype)
        refi = oracle.spinsum_chain(xi.cpu().to(torch.float64).numpy(), stages, gf, d, pairs=True)
        np.testing.assert_array_equal(apply(p, xi).cpu().to(torch.float64).numpy(), refi)


@pytest.mark.parametrize("case", range(24))
def test_random_batched(case):
    """Batched plans over 1-6 blocks of random extents (trailing groups or
    groups before an inner run): one launch equals the per-block plans bit
    for bit, and each block matches the oracle."""
    rng = np.random.default_rng(7600 + case)
    d = int(rng.choice([2, 3, 4], p=[0.2, 0.6, 0.2]))
    inner = [int(rng.integers(1, 4))] if rng.random() < 0.3 else []
    nouter = int(rng.integers(0, 3))
    shapes = []
    for _ in range(int(rng.integers(1, 7))):
        v = int(rng.integers(1, 5))
        o = int(rng.integers(1, {2: 40, 3: 18, 4: 9}[d] + 1))
        shapes.append(tuple([v] * nouter + [o] * d + inner))
    gf = nouter
    stages = random_stages(rng, d, kmax=2)
    dtype = torch.float64 if rng.random() < 0.6 else torch.float32
    inplace = bool(rng.random() < 0.5)
    _say("batched", case, shapes, d, dtype, inplace, [len(s) for s in stages])
    # group position: explicit with inner runs, else the trailing d dims
    bp = ss.spinsum_plan_batched(shapes, d, stages, dtype=dtype, inplace=inplace,
                                 group_first=gf if inner else -1)
    xs = [workloads.uniform(s, 7700 + case * 8 + k, device=DEV, dtype=dtype)
          for k, s in enumerate(shapes)]
    ins = [x.clone() for x in xs]
    outs = ins if inplace else [torch.empty_like(x) for x in xs]
    ss.spinsum_exec_batched(bp, ins, outs)
    torch.cuda.synchronize()
    for k, (s, x) in enumerate(zip(shapes, xs)):
        p = ss.spinsum_plan(s, gf, d, stages, dtype=dtype, inplace=inplace)
        assert torch.equal(outs[k], apply(p, x)), k
        xh = x.cpu().to(torch.float64).numpy()
        scale = max(gain_of(stages) * float(np.max(np.abs(xh))) if xh.size else 0.0,
                    np.finfo(np.float64).tiny)
        ref = oracle.spinsum_chain(xh, stages, gf, d, nthreads=8)
        if xh.size:
            assert np.max(np.abs(outs[k].cpu().to(torch.float64).numpy() - ref)) <= TOL[dtype] * scale


@pytest.mark.parametrize("case", range(24))
def test_random_coefficient_gradients(case):
    """Gradients with respect to the coefficients: of one stage
    (spinsum_coef_grad, every permutation of the group) and of every stage of
    a chain (spinsum_coef_grad_stages), against the oracle, measured against
    sum|g| * max|x| times the gain of the other stages."""
    rng = np.random.default_rng(7800 + case)
    d = int(rng.choice([2, 3, 4], p=[0.2, 0.5, 0.3]))
    n = int(rng.integers(1, {2: 40, 3: 20, 4: 10}[d] + 1))
    outer = [int(e) for e in rng.integers(1, 4, size=int(rng.integers(0, 3)))]
    inner = [int(e) for e in rng.integers(1, 4, size=int(rng.integers(0, 2)))]
    shape = tuple(outer + [n] * d + inner)
    gf = len(outer)
    stages = random_stages(rng, d)
    dtype = torch.float64 if rng.random() < 0.6 else torch.float32
    _say("coef grad", case, shape, gf, d, dtype, [len(s) for s in stages])
    x = workloads.uniform(shape, 7900 + case, device=DEV, dtype=dtype)
    g = workloads.uniform(shape, 8000 + case, device=DEV, dtype=dtype)
    xh = x.cpu().to(torch.float64).numpy()
    gh = g.cpu().to(torch.float64).numpy()
    base = float(np.sum(np.abs(gh))) * float(np.max(np.abs(xh)))
    p1 = ss.spinsum_plan(shape, gf, d, stages[:1], dtype=dtype)
    got1 = ss.spinsum_coef_grad(p1, x, g).cpu().numpy()
    ref1 = oracle.coef_grad(xh, gh, gf, d, nthreads=8)
    assert np.max(np.abs(got1 - ref1)) <= TOL[dtype] * max(base, np.finfo(np.float64).tiny)
    pk = ss.spinsum_plan(shape, gf, d, stages, dtype=dtype)
    gotk = ss.spinsum_coef_grad_stages(pk, x, g).cpu().numpy()
    refk = oracle.coef_grad_stages(xh, gh, stages, gf, d, nthreads=8)
    for k in range(len(stages)):
        others = gain_of(stages[:k] + stages[k + 1:])
        bound = TOL[dtype] * max(base * others, np.finfo(np.float64).tiny)
        assert np.max(np.abs(gotk[k] - refk[k])) <= bound, k


@pytest.mark.parametrize("case", range(24))
def test_random_unpack_and_pack(case):
    """Unpacking and packing with random operators and shapes: against the
    oracle (S(E(p)) and its adjoint), integers bitwise where exact; plans
    whose tile rows are not whole 16-byte chunks are refused with
    SPINSUM_ERR_UNSUPPORTED."""
    rng = np.random.default_rng(8100 + case)
    d = int(rng.choice([2, 3, 4], p=[0.2, 0.5, 0.3]))
    n = int(rng.integers(d, {2: 48, 3: 24, 4: 12}[d] + 1))  # C(N, d) > 0 packed values
    outer = [int(e) for e in rng.integers(1, 4, size=int(rng.integers(0, 3)))]
    inner = [int(e) for e in rng.integers(1, 4, size=int(rng.integers(0, 2)))]
    shape = tuple(outer + [n] * d + inner)
    gf = len(outer)
    stages = random_stages(rng, d, kmax=2)
    dtype = torch.float64 if rng.random() < 0.6 else torch.float32
    _say("unpack", case, shape, gf, d, dtype, [len(s) for s in stages])
    p = ss.spinsum_plan(shape, gf, d, stages, dtype=dtype)
    pshape = ss.packed_shape(p)
    pk = workloads.uniform(pshape, 8200 + case, device=DEV, dtype=dtype)
    full = torch.full(shape, float("nan"), dtype=dtype, device=DEV)
    if ss.spinsum_plan_get_info(p)["variant"] != ss.SPINSUM_VARIANT_DIRECT_LDS:
        with pytest.raises(ss.SpinSumError) as e:
            ss.spinsum_unpack(p, pk, full)
        assert e.value.status == ss.SPINSUM_ERR_UNSUPPORTED
        return
    gain = gain_of(stages)
    ss.spinsum_unpack(p, pk, full)
    torch.cuda.synchronize()
    pkh = pk.cpu().to(torch.float64).numpy()
    ref = oracle.unpack(pkh, shape, stages, gf, d)
    scale = max(gain * (float(np.max(np.abs(pkh))) if pkh.size else 0.0), np.finfo(np.float64).tiny)
    assert np.max(np.abs(full.cpu().to(torch.float64).numpy() - ref)) <= TOL[dtype] * scale
    f = workloads.uniform(shape, 8300 + case, device=DEV, dtype=dtype)
    out = torch.full(pshape, float("nan"), dtype=dtype, device=DEV)
    ss.spinsum_pack(p, f, out)
    torch.cuda.synchronize()
    fh = f.cpu().to(torch.float64).numpy()
    refp = oracle.pack(fh, stages, gf, d)
    if out.numel():
        scale = max(gain * float(np.max(np.abs(fh))), np.finfo(np.float64).tiny)
        assert np.max(np.abs(out.cpu().to(torch.float64).numpy() - refp)) <= TOL[dtype] * scale
    if gain * 1024.0 < EXACT[dtype]:
        pki = workloads.integers(pshape, 8400 + case, device=DEV, dtype=dtype)
        ss.spinsum_unpack(p, pki, full)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(
            full.cpu().to(torch.float64).numpy(),
            oracle.unpack(pki.cpu().to(torch.float64).numpy(), shape, stages, gf, d))


@pytest.mark.parametrize("case", range(40))
def test_random_non_finite_inputs(case):
    """Inf, -Inf and NaN planted at random positions (some on diagonals) under
    random operators with zero coefficients, in the three forms: the
    positions of NaN, +Inf and -Inf equal the oracle's exactly -- on the
    pre-multiplied sum (oracle.expanded_terms) for the default form, on the
    chain for the chained and multi-pass forms -- and the finite outputs are
    within the tolerance."""
    rng = np.random.default_rng(8500 + case)
    d = int(rng.choice([2, 3, 4], p=[0.2, 0.5, 0.3]))
    n = int(rng.integers(1, {2: 40, 3: 16, 4: 8}[d] + 1))
    outer = [int(e) for e in rng.integers(1, 4, size=int(rng.integers(0, 3)))]
    inner = [int(e) for e in rng.integers(1, 4, size=int(rng.integers(0, 2)))]
    shape = tuple(outer + [n] * d + inner)
    gf = len(outer)
    stages = random_stages(rng, d)
    form = rng.choice(["expanded", "chained", "multi_pass"], p=[0.5, 0.3, 0.2])
    flags = {"expanded": 0, "chained": ss.SPINSUM_FLAG_CHAIN_STAGES,
             "multi_pass": ss.SPINSUM_FLAG_MULTI_PASS}[form]
    if rng.random() < 0.3:
        flags |= ss.SPINSUM_FLAG_NO_DIRECT_LDS
    dtype = torch.float64 if rng.random() < 0.6 else torch.float32
    inplace = bool(rng.random() < 0.5)
    _say("non-finite", case, shape, gf, d, form, dtype, inplace, [len(s) for s in stages])
    xh = workloads.uniform(shape, 8600 + case, dtype=dtype).to(torch.float64).numpy()
    flat = xh.reshape(-1)
    for k in range(int(rng.integers(1, 6))):
        pos = list(np.unravel_index(int(rng.integers(0, flat.size)), shape))
        if rng.random() < 0.4:  # onto a diagonal: two group indices equal
            a, b = rng.choice(d, size=2, replace=False) if d > 1 else (0, 0)
            pos[gf + int(a)] = pos[gf + int(b)]
        xh[tuple(pos)] = [np.inf, -np.inf, np.nan][k % 3]
    if form == "expanded":
        ref = oracle.spinsum(xh, oracle.expanded_terms(stages, d), gf, d, nthreads=8)
    else:
        ref = oracle.spinsum_chain(xh, stages, gf, d, nthreads=8)
    p = ss.spinsum_plan(shape, gf, d, stages, dtype=dtype, inplace=inplace, flags=flags)
    got = apply(p, torch.from_numpy(xh).to(dtype).to(DEV)).cpu().to(torch.float64).numpy()
    np.testing.assert_array_equal(np.isnan(got), np.isnan(ref))
    np.testing.assert_array_equal(np.isposinf(got), np.isposinf(ref))
    np.testing.assert_array_equal(np.isneginf(got), np.isneginf(ref))
    fin = np.isfinite(ref)
    if fin.any():
        scale = max(gain_of(stages) * float(np.max(np.abs(xh[np.isfinite(xh)]), initial=0.0)),
                    np.finfo(np.float64).tiny)
        assert np.max(np.abs(got[fin] - ref[fin])) <= TOL[dtype] * scale
