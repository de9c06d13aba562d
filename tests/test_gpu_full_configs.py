"""Parity at the full workload sizes, in the launch configuration the
benchmark times (run on an MI355X).

At these sizes the oracle cannot take the whole tensor, so each test
 * compares sampled spectator cubes with the oracle run on that cube alone
   (a cube's output depends only on that cube); the input of a sampled cube
   is regenerated on the host from the counter-based generator, so the
   multi-GB input is never copied back;
 * checks on every cube the sum invariant sum(Out) = (sum of coefficients)
   * sum(In) (exact in exact arithmetic), which fails for any cube that is
   skipped, written twice or mixed with another one.
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


def _say(*a):
    print(*a, flush=True)


def sample_cubes(ncubes, k, seed):
    rng = np.random.default_rng(seed)
    picks = set(int(c) for c in rng.choice(ncubes, size=min(k, ncubes), replace=False))
    picks.update({0, ncubes - 1})
    return sorted(picks)


def check_sampled(out, seed, stages, d, cubes, tol, in_dtype=torch.float64, adjoint=False):
    """out: GPU tensor viewed as (ncubes, n^d); input of cube c = the
    generator stream at offset c * n^d, rounded to in_dtype."""
    n = round(out.shape[-1] ** (1.0 / d))
    cube = n ** d
    worst = 0.0
    for c in cubes:
        x = workloads.uniform_numpy(cube, seed, offset=c * cube)
        if in_dtype == torch.float32:
            x = x.astype(np.float32).astype(np.float64)
        x = x.reshape((1,) + (n,) * d)
        if adjoint:
            ref = oracle.spinsum_chain_adjoint(x, stages, 1, d)
        else:
            ref = oracle.spinsum_chain(x, stages, 1, d)
        got = out[c].to("cpu", torch.float64).numpy().reshape(ref.shape)
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        worst = max(worst, float(err))
    _say(f"  sampled {len(cubes)} cubes, worst normwise error {worst:.3e}")
    assert worst <= tol


def check_cube_sums(out2d, in_sums, coef_sum, rel):
    """|sum(Out_c) - coef_sum * sum(In_c)| <= rel * sum|Out_c| for every cube c."""
    out_sums = out2d.sum(dim=1, dtype=torch.float64)
    abs_sums = out2d.abs().sum(dim=1, dtype=torch.float64)
    bad = (out_sums - coef_sum * in_sums).abs() > rel * abs_sums + 1e-300
    nbad = int(bad.sum())
    _say(f"  cube sums checked on {out2d.shape[0]} cubes, violations {nbad}")
    assert nbad == 0


def expanded_sum(stages):
    return float(np.prod([sum(a for _, a in s) for s in stages]))


@pytest.mark.parametrize("form", ["expanded", "factored_chained", "table2_1_chained",
                                  "antisymmetrizer"])
def test_3d_v64_o32_slab_inplace(form):
    w = workloads.WORKLOADS["3d_v64_o32_slab"]
    shape = w["shape"]
    _say("case 3d_v64_o32_slab", form, shape)
    if form == "expanded":
        stages, flags = [workloads.CONFIG_3D_ALPHA], 0
    elif form == "factored_chained":
        stages, flags = workloads.FACTORED_PIJ_PJK, ss.SPINSUM_FLAG_CHAIN_STAGES
    elif form == "table2_1_chained":
        stages, flags = workloads.table2_case(1)[1], ss.SPINSUM_FLAG_CHAIN_STAGES
    else:
        stages, flags = [workloads.antisymmetrizer(3)], 0
    seed = 1000
    x = workloads.uniform(shape, seed, device=DEV)
    cube = 32 ** 3
    x2 = x.view(-1, cube)
    in_sums = x2.sum(dim=1, dtype=torch.float64)
    p = ss.spinsum_plan(shape, 3, 3, stages, inplace=True, flags=flags)
    ss.spinsum_exec(p, x, x)
    torch.cuda.synchronize()
    check_sampled(x2, seed, stages, 3, sample_cubes(x2.shape[0], 48, 1), 1e-14)
    check_cube_sums(x2, in_sums, expanded_sum(stages), 1e-12)


def test_4d_v24_o12_slab_inplace():
    w = workloads.WORKLOADS["4d_v24_o12_slab"]
    shape = w["shape"]
    _say("case 4d_v24_o12_slab", shape)
    a = workloads.random_4d_alpha(7)
    seed = 2000
    x = workloads.uniform(shape, seed, device=DEV)
    x2 = x.view(-1, 12 ** 4)
    in_sums = x2.sum(dim=1, dtype=torch.float64)
    p = ss.spinsum_plan(shape, 4, 4, [a], inplace=True)
    ss.spinsum_exec(p, x, x)
    torch.cuda.synchronize()
    check_sampled(x2, seed, [a], 4, sample_cubes(x2.shape[0], 32, 2), 1e-14)
    check_cube_sums(x2, in_sums, expanded_sum([a]), 1e-12)


# Operators whose permutations move two of the group's axes (Fig. 1b and
# (2 - pi_2134)), on the full slabs in the configuration the benchmark times:
# the plan runs the two moved axes alone (the subgroup reduction).
SUBGROUP_SLABS = {
    "3d_fig1b": ("3d_v64_o32_slab", 3, [[((0, 1, 2), 1.0), (workloads.P("213"), 1.0)]], 1000),
    "4d_2_minus_p2134": ("4d_v24_o12_slab", 4,
                         [[((0, 1, 2, 3), 2.0), (workloads.P("2134"), -1.0)]], 2000),
}


@pytest.mark.parametrize("form", list(SUBGROUP_SLABS))
def test_subgroup_slabs_inplace(form):
    wname, d, stages, seed = SUBGROUP_SLABS[form]
    shape = workloads.WORKLOADS[wname]["shape"]
    gf = len(shape) - d
    _say("case subgroup slab", form, shape)
    x = workloads.uniform(shape, seed, device=DEV)
    cube = shape[-1] ** d
    x2 = x.view(-1, cube)
    in_sums = x2.sum(dim=1, dtype=torch.float64)
    p = ss.spinsum_plan(shape, gf, d, stages, inplace=True)
    assert ss.spinsum_plan_get_info(p)["exec_d"] == 2
    ss.spinsum_exec(p, x, x)
    torch.cuda.synchronize()
    check_sampled(x2, seed, stages, d, sample_cubes(x2.shape[0], 32, 3), 1e-14)
    check_cube_sums(x2, in_sums, expanded_sum(stages), 1e-12)


def test_3d_v64_o32_unpack_and_pack():
    """Antisymmetric unpacking of the v=64 o=32 slab (C(32, 3) = 4960 packed
    values per cube into 32^3) and packing back, in the benchmark's
    configuration: sampled cubes against the oracle (inputs regenerated on
    the host); unpack then pack with the antisymmetriser gives 3! times the
    packed values on every cube."""
    shape = workloads.WORKLOADS["3d_v64_o32_slab"]["shape"]
    A = [workloads.antisymmetrizer(3)]
    p = ss.spinsum_plan(shape, 3, 3, A)
    pshape = ss.packed_shape(p)
    assert pshape == (64, 64, 8, 4960)
    pk = workloads.uniform(pshape, 3200, device=DEV)
    full = torch.empty(shape, dtype=torch.float64, device=DEV)
    ss.spinsum_unpack(p, pk, full)
    torch.cuda.synchronize()
    f2 = full.view(-1, 32 ** 3)
    worst = 0.0
    for c in sample_cubes(f2.shape[0], 24, 5):
        pc = workloads.uniform_numpy(4960, 3200, offset=c * 4960).reshape(1, 4960)
        ref = oracle.unpack(pc, (1, 32, 32, 32), A, 1, 3)
        got = f2[c].cpu().numpy().reshape(ref.shape)
        worst = max(worst, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
    _say(f"  unpack: worst normwise error {worst:.3e}")
    assert worst <= 1e-14
    back = torch.empty_like(pk)
    ss.spinsum_pack(p, full, back)
    torch.cuda.synchronize()
    err = float((back - 6.0 * pk).abs().max() / (6.0 * pk).abs().max())
    _say(f"  pack(unpack(p)) = 6 p: normwise error {err:.3e}")
    assert err <= 1e-14


def test_3d_inner_run8_inplace():
    """The slab with its group moved in front of an inner spectator run of
    8: [64, 64, 32, 32, 32, 8], group dims 2..4, in place (the bench line)."""
    shape = (64, 64, 32, 32, 32, 8)
    _say("case 3d_inner_run8", shape)
    stages = [workloads.CONFIG_3D_ALPHA]
    seed = 5000
    x = workloads.uniform(shape, seed, device=DEV)
    cube = 32 ** 3 * 8
    x2 = x.view(-1, cube)
    in_sums = x2.sum(dim=1, dtype=torch.float64)
    p = ss.spinsum_plan(shape, 2, 3, stages, inplace=True)
    ss.spinsum_exec(p, x, x)
    torch.cuda.synchronize()
    worst = 0.0
    cubes = sample_cubes(x2.shape[0], 24, 5)
    for c in cubes:
        xc = workloads.uniform_numpy(cube, seed, offset=c * cube).reshape(1, 32, 32, 32, 8)
        ref = oracle.spinsum(xc, stages[0], 1, 3)
        got = x2[c].to("cpu", torch.float64).numpy().reshape(ref.shape)
        worst = max(worst, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
    _say(f"  sampled {len(cubes)} cubes, worst normwise error {worst:.3e}")
    assert worst <= 1e-14
    check_cube_sums(x2, in_sums, expanded_sum(stages), 1e-12)


def test_3d_pairs_v48_o24_inplace():
    """Index-pair form on T[a,b,c,i,j,k], v=48, o=24, in place (the bench
    line).  For a set S of partner values the sub-tensor T[S,S,S,:,:,:] is
    closed under the operator (a permutation of (a,b,c) stays in S^3), so the
    oracle runs on that sub-tensor alone; its input is regenerated on the
    host cube by cube."""
    shape = (48, 48, 48, 24, 24, 24)
    _say("case 3d_pairs_v48_o24", shape)
    terms = workloads.CONFIG_3D_ALPHA
    seed = 5100
    x = workloads.uniform(shape, seed, device=DEV)
    cube = 24 ** 3
    total_in = float(x.sum(dtype=torch.float64))
    p = ss.spinsum_plan(shape, 3, 3, [terms], inplace=True, flags=ss.SPINSUM_FLAG_INDEX_PAIRS)
    ss.spinsum_exec(p, x, x)
    torch.cuda.synchronize()
    worst = 0.0
    for S in ([0, 1, 47], [3, 20], [11], [5, 46, 47], [0, 24, 36]):
        k = len(S)
        xs = np.empty((k, k, k, 24, 24, 24))
        got = np.empty_like(xs)
        for ia, a in enumerate(S):
            for ib, b in enumerate(S):
                for ic, c in enumerate(S):
                    off = ((a * 48 + b) * 48 + c) * cube
                    xs[ia, ib, ic] = workloads.uniform_numpy(cube, seed, offset=off).reshape(24, 24, 24)
                    got[ia, ib, ic] = x[a, b, c].to("cpu", torch.float64).numpy()
        ref = oracle.spinsum(xs, terms, 3, 3, pairs=True, nthreads=8)
        worst = max(worst, float(np.max(np.abs(got - ref)) / np.max(np.abs(ref))))
    _say(f"  sampled partner sets, worst normwise error {worst:.3e}")
    assert worst <= 1e-14
    # whole-tensor sum invariant: sum(Out) = (sum of coefficients) * sum(In)
    total_out = float(x.sum(dtype=torch.float64))
    coef_sum = sum(a for _, a in terms)
    assert abs(total_out - coef_sum * total_in) <= 1e-9 * float(x.abs().sum(dtype=torch.float64))


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_3d_v48_o24_forward_and_adjoint(dtype):
    w = workloads.WORKLOADS["3d_v48_o24"]
    shape = w["shape"]
    _say("case 3d_v48_o24", dtype)
    stages = workloads.FACTORED_PIJ_PJK
    tol = 1e-14 if dtype == torch.float64 else 2e-6
    seed = 4000
    x = workloads.uniform(shape, seed, device=DEV, dtype=dtype)
    y = torch.empty_like(x)
    p = ss.spinsum_plan(shape, 3, 3, stages, dtype=dtype)
    ss.spinsum_exec(p, x, y)
    torch.cuda.synchronize()
    cube = 24 ** 3
    cubes = sample_cubes(x.numel() // cube, 32, 3)
    check_sampled(y.view(-1, cube), seed, stages, 3, cubes, tol, in_dtype=dtype)
    in_sums = x.view(-1, cube).sum(dim=1, dtype=torch.float64)
    check_cube_sums(y.view(-1, cube).to(torch.float64) if dtype == torch.float32 else y.view(-1, cube),
                    in_sums, expanded_sum(stages), 1e-12 if dtype == torch.float64 else 1e-5)
    del y
    # backward: grad_in = S^T g with g the same stream (seed), adjoint form
    g = x
    gi = torch.empty_like(g)
    ss.spinsum_adjoint(p, g, gi)
    torch.cuda.synchronize()
    check_sampled(gi.view(-1, cube), seed, stages, 3, cubes, tol, in_dtype=dtype, adjoint=True)


def test_batched_power_law_blocks():
    seed, blocks = workloads.batched_blocks()
    shapes = [(v, v, v, o, o, o) for v, o in blocks]
    _say("case batched 200 blocks, block seed", seed)
    alpha = [workloads.CONFIG_3D_ALPHA]
    xs = [workloads.uniform(s, 3000 + k, device=DEV) for k, s in enumerate(shapes)]
    ref_out = []
    for s, x in zip(shapes, xs):
        y = torch.empty_like(x)
        ss.spinsum_exec(ss.spinsum_plan(s, 3, 3, alpha), x, y)
        ref_out.append(y)
    bp = ss.spinsum_plan_batched(shapes, 3, alpha, inplace=True)
    # the plan the benchmark times: item size and launch style from the
    # autotuner (which overwrites the buffers it is given)
    scratch = [torch.empty_like(x) for x in xs]
    tuned, _ = ss.spinsum_autotune(bp, scratch, scratch)
    _say("  autotuned", tuned, ss.spinsum_plan_get_info(bp)["batch_item_bytes"])
    del scratch
    graph = ss.spinsum_graph_create(bp, xs, xs)
    ss.spinsum_graph_launch(graph)
    torch.cuda.synchronize()
    for k, (x, y) in enumerate(zip(xs, ref_out)):
        assert torch.equal(x, y), k
    for k in (0, 1, 57, 123, 199):
        v, o = blocks[k]
        check_sampled(xs[k].view(-1, o ** 3), 3000 + k, alpha, 3,
                      sample_cubes(v ** 3, 8, k), 1e-14)


@pytest.mark.slow
def test_3d_v64_o32_whole_tensor_one_launch():
    """All 8.6G elements (68.7 GB) in one launch: element offsets beyond 2^32."""
    shape = (64, 64, 64, 32, 32, 32)
    _say("case whole v64 o32 tensor", shape)
    seed = 1100
    x = workloads.uniform(shape, seed, device=DEV)
    cube = 32 ** 3
    x2 = x.view(-1, cube)
    in_sums = x2.sum(dim=1, dtype=torch.float64)
    p = ss.spinsum_plan(shape, 3, 3, [workloads.CONFIG_3D_ALPHA], inplace=True)
    ss.spinsum_exec(p, x, x)
    torch.cuda.synchronize()
    ncubes = x2.shape[0]
    cubes = sample_cubes(ncubes, 24, 4) + [ncubes // 2, (1 << 31) // cube, (1 << 32) // cube + 1]
    check_sampled(x2, seed, [workloads.CONFIG_3D_ALPHA], 3, sorted(set(cubes)), 1e-14)
    check_cube_sums(x2, in_sums, 0.0, 1e-12)
    del x, x2
    torch.cuda.empty_cache()


# Table II on hyper-square tensors without spectators at the paper's medium
# size (Sec. 5.1: about 320 MiB), in place, in the launch configuration of
# the benchmark's Table II sweep; the oracle takes the whole tensor.
TABLE2_N = {3: 352, 4: 80}


# The small (about 70 MiB) and large (about 1200 MiB) sizes: for a set S of
# indices (with 0 and N-1) the sub-tensor In[S, .., S] is closed under every
# permutation of the group, so Out on it is the oracle on that sub-tensor
# alone; its input is regenerated on the host at those positions.
TABLE2_OTHER = {"small": {3: 208, 4: 54}, "large": {3: 544, 4: 112}}


@pytest.mark.parametrize("size", ["small", "large"])
@pytest.mark.parametrize("case", [1, 3, 5, 9, 18])
def test_table2_small_and_large_inplace(size, case):
    d, stages = workloads.table2_case(case)
    n = TABLE2_OTHER[size][d]
    shape = (n,) * d
    _say(f"case table2 #{case} {size} shape {shape}")
    seed = 6000 + case
    x = workloads.uniform(shape, seed, device=DEV)
    p = ss.spinsum_plan(shape, 0, d, stages, inplace=True)
    ss.spinsum_exec(p, x, x)
    torch.cuda.synchronize()
    rng = np.random.default_rng(case)
    k = 24 if d == 3 else 14
    S = np.unique(np.concatenate([[0, n - 1], rng.choice(n, k - 2, replace=False)]))
    grids = np.meshgrid(*([S] * d), indexing="ij")
    lin = np.zeros(grids[0].shape, dtype=np.int64)
    for gmat in grids:
        lin = lin * n + gmat
    xs = workloads.uniform_numpy_at(lin.astype(np.uint64), seed)
    ref = oracle.spinsum_chain(xs.reshape((1,) + xs.shape), stages, 1, d).reshape(xs.shape)
    idx = torch.from_numpy(lin.reshape(-1)).to(DEV)
    got = x.view(-1)[idx].cpu().numpy().reshape(xs.shape)
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    _say(f"  {len(S)}^{d} sub-tensor, normwise error {err:.3e}")
    assert err <= 1e-14


@pytest.mark.parametrize("case", range(1, 22))
def test_table2_medium_size_inplace(case):
    d, stages = workloads.table2_case(case)
    n = TABLE2_N[d]
    shape = (n,) * d
    _say(f"case table2 #{case} shape {shape}")
    x = workloads.uniform(shape, 5000 + case, device=DEV)
    ref = oracle.spinsum_chain(x.cpu().numpy().reshape((1,) + shape), stages, 1, d).reshape(shape)
    p = ss.spinsum_plan(shape, 0, d, stages, inplace=True)
    ss.spinsum_exec(p, x, x)
    torch.cuda.synchronize()
    got = x.cpu().numpy()
    err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
    _say(f"  normwise error {err:.3e}")
    assert err <= 1e-14


def test_3d_coef_grad_full_size():
    """The coefficient gradient on two full slabs (the bench line): grad_p =
    <g, pi_p(x)> for every permutation p, checked against the plain sum of
    g * x.permute(...) taken in double by the library (the definition of the
    gradient, Def. 2-3, at a size the oracle cannot take)."""
    import itertools
    shape = workloads.WORKLOADS["3d_v64_o32_slab"]["shape"]
    _say("case 3d_coef_grad full slab", shape)
    x = workloads.uniform(shape, 1000, device=DEV)
    g = workloads.uniform(shape, 1001, device=DEV)
    p = ss.spinsum_plan(shape, 3, 3, [workloads.CONFIG_3D_ALPHA])
    got = ss.spinsum_coef_grad(p, x, g).cpu().numpy()
    scale = float((g.abs().sum(dtype=torch.float64) * x.abs().max()).cpu())
    for r, perm in enumerate(itertools.permutations(range(3))):
        q = [0] * 3
        for m, v in enumerate(perm):
            q[v] = m
        y = x.permute(0, 1, 2, 3 + q[0], 3 + q[1], 3 + q[2])
        ref = float((g * y).sum(dtype=torch.float64))
        _say(f"  p={perm} gpu {got[r]:.12e} ref {ref:.12e}")
        assert abs(got[r] - ref) <= 1e-12 * scale


def test_3d_v64_o32_slab_spectrum():
    """The 3D coefficient set acts with eigenvalues 0, 3 and 12 (the trivial,
    standard and sign representations of S_3), so S^3 - 15 S^2 + 36 S = 0
    on any input: checked on the whole 8.6 GB slab with the benchmark's own
    in-place plan, every cube at once (a closed form of the operator, not
    the oracle)."""
    w = workloads.WORKLOADS["3d_v64_o32_slab"]
    shape = w["shape"]
    s = workloads.uniform(shape, 1000, device=DEV)
    p = ss.spinsum_plan(shape, 3, 3, [workloads.CONFIG_3D_ALPHA], inplace=True)
    ss.spinsum_exec(p, s, s)                       # S x
    r = 36.0 * s
    ss.spinsum_exec(p, s, s)                       # S^2 x
    r.add_(s, alpha=-15.0)
    ss.spinsum_exec(p, s, s)                       # S^3 x
    r.add_(s)
    torch.cuda.synchronize()
    scale = float(s.abs().max())
    res = float(r.abs().max())
    _say(f"  max|S^3 - 15 S^2 + 36 S| = {res:.3e} against max|S^3 x| = {scale:.3e}")
    assert scale > 0 and res <= 1e-13 * scale
    del s, r
    torch.cuda.empty_cache()
