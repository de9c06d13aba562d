"""Unpacking and packing on an MI355X against the oracle (oracle.unpack /
oracle.pack: the embedding of the strictly increasing entries followed by
the chain, and its adjoint).

Bars: FP64 normwise 1e-14, FP32 2e-6 (against the oracle on the FP32-rounded
input), integer-valued inputs bit for bit, Inf/NaN patterns exactly.
"""
import itertools
import math

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


OPS = {
    "antisym3": (3, [workloads.antisymmetrizer(3)]),
    "identity3": (3, [[((0, 1, 2), 1.0)]]),
    "config3": (3, [workloads.CONFIG_3D_ALPHA]),
    "antisym4": (4, [workloads.antisymmetrizer(4)]),
    "random4": (4, [workloads.random_4d_alpha(7)]),
    "antisym2": (2, [workloads.antisymmetrizer(2)]),
}
SHAPES = {2: [((3, 33, 33), None), ((4, 16, 16), (8, 1))],
          3: [((3, 12, 12, 12), None), ((2, 16, 16, 16), (4, 1)), ((2, 14, 14, 14), (4, 1)),
              ((2, 8, 8, 8, 3), None)],
          4: [((2, 6, 6, 6, 6), None), ((1, 12, 12, 12, 12), (4, 1)), ((1, 10, 10, 10, 10), (4, 1))]}


def packed_shape(shape, d):
    return (shape[0], math.comb(shape[1], d)) + tuple(shape[1 + d:])


@pytest.mark.parametrize("op", list(OPS))
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_unpack_and_pack_against_oracle(op, dtype):
    d, stages = OPS[op]
    for shape, tile in SHAPES[d]:
        print(op, dtype, shape, tile, flush=True)
        p = ss.spinsum_plan(shape, 1, d, stages, dtype=dtype)
        if tile is not None:
            ss.spinsum_plan_set_tile(p, *tile)
        pk = workloads.uniform(packed_shape(shape, d), 2600 + d, device=DEV, dtype=dtype)
        full = torch.full(shape, float("nan"), dtype=dtype, device=DEV)
        info = ss.spinsum_plan_get_info(p)
        if info["variant"] != ss.SPINSUM_VARIANT_DIRECT_LDS:
            # tile rows that are not whole 16-byte chunks (FP32 rows of 14):
            # unpacking needs the direct-LDS layout
            with pytest.raises(ss.SpinSumError) as e:
                ss.spinsum_unpack(p, pk, full)
            assert e.value.status == ss.SPINSUM_ERR_UNSUPPORTED
            continue
        ss.spinsum_unpack(p, pk, full)
        torch.cuda.synchronize()
        ref = oracle.unpack(pk.cpu().to(torch.float64).numpy(), shape, stages, 1, d)
        assert nerr(full.cpu().numpy(), ref) <= TOL[dtype], (shape, tile)
        f = workloads.uniform(shape, 2700 + d, device=DEV, dtype=dtype)
        out = torch.full(packed_shape(shape, d), float("nan"), dtype=dtype, device=DEV)
        ss.spinsum_pack(p, f, out)
        torch.cuda.synchronize()
        refp = oracle.pack(f.cpu().to(torch.float64).numpy(), stages, 1, d)
        assert nerr(out.cpu().numpy(), refp) <= TOL[dtype], (shape, tile)
        # integer-valued inputs: exact
        pki = workloads.integers(packed_shape(shape, d), 2800 + d, device=DEV, dtype=dtype)
        ss.spinsum_unpack(p, pki, full)
        fi = workloads.integers(shape, 2900 + d, device=DEV, dtype=dtype)
        ss.spinsum_pack(p, fi, out)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(
            full.cpu().to(torch.float64).numpy(),
            oracle.unpack(pki.cpu().to(torch.float64).numpy(), shape, stages, 1, d))
        np.testing.assert_array_equal(
            out.cpu().to(torch.float64).numpy(),
            oracle.pack(fi.cpu().to(torch.float64).numpy(), stages, 1, d))


def test_antisymmetric_round_trip_and_packed_shape_helper():
    """X antisymmetric: packing with the identity gathers its increasing
    entries and unpacking them with the antisymmetriser rebuilds X."""
    d, n = 3, 11
    shape = (4, n, n, n)
    y = workloads.uniform(shape, 3000, device=DEV)
    A = ss.spinsum_plan(shape, 1, d, [workloads.antisymmetrizer(d)])
    x = torch.empty_like(y)
    ss.spinsum_exec(A, y, x)
    x /= math.factorial(d)
    I = ss.spinsum_plan(shape, 1, d, [[((0, 1, 2), 1.0)]])
    assert ss.packed_shape(I) == packed_shape(shape, d)
    pk = torch.empty(ss.packed_shape(I), dtype=torch.float64, device=DEV)
    ss.spinsum_pack(I, x, pk)
    back = torch.empty_like(x)
    ss.spinsum_unpack(A, pk, back)
    torch.cuda.synchronize()
    assert nerr(back.cpu().numpy(), x.cpu().numpy()) <= 1e-14


def test_unpack_non_finite_and_errors():
    d, stages = OPS["antisym3"]
    shape = (2, 9, 9, 9)
    pkh = workloads.uniform(packed_shape(shape, d), 3100).numpy()
    pkh[0, 5] = np.inf
    pkh[1, 17] = np.nan
    ref = oracle.unpack(pkh, shape, stages, 1, d)
    p = ss.spinsum_plan(shape, 1, d, stages)
    full = torch.empty(shape, dtype=torch.float64, device=DEV)
    ss.spinsum_unpack(p, torch.from_numpy(pkh).to(DEV), full)
    torch.cuda.synchronize()
    got = full.cpu().numpy()
    np.testing.assert_array_equal(np.isnan(got), np.isnan(ref))
    np.testing.assert_array_equal(np.isposinf(got), np.isposinf(ref))
    np.testing.assert_array_equal(np.isneginf(got), np.isneginf(ref))
    fin = np.isfinite(ref)
    assert nerr(got[fin], ref[fin]) <= 1e-14
    big = torch.empty(full.numel() * 2, dtype=torch.float64, device=DEV)
    st = ss._c_unpack(p._h, big.data_ptr() + 8, big.data_ptr(), None)
    assert st == ss.SPINSUM_ERR_ALIASING
    pp = ss.spinsum_plan((2, 3, 3, 3, 4, 4, 4), 4, 3, stages, flags=ss.SPINSUM_FLAG_INDEX_PAIRS)
    st = ss._c_unpack(pp._h, big.data_ptr(), big.data_ptr() + 8 * 4096, None)
    assert st == ss.SPINSUM_ERR_UNSUPPORTED


OWN_TILING_CASES = [
    # (shape, group_first, d, dtype): plans whose unpacking runs on its own
    # tiling (whole cubes, or tiles with whole-line rows), unpack_bl != bl
    ((3, 24, 24, 24), 1, 3, torch.float64),      # whole 24^3 cubes
    ((2, 2, 32, 32, 32), 2, 3, torch.float64),   # bl 16: 128-byte rows
    ((2, 32, 32, 32), 1, 3, torch.float32),      # whole 32^3 FP32 cubes
    ((3, 12, 12, 12, 8), 1, 3, torch.float64),   # whole cubes with inner runs (bl 4)
    ((2, 160, 160), 1, 2, torch.float64),         # bl 80 instead of 40
]


@pytest.mark.parametrize("case", range(len(OWN_TILING_CASES)))
def test_unpack_on_its_own_tiling(case):
    """Unpacking on its own tiling (the largest items a CU holds) against the
    oracle, and bit for bit against the sum of the embedded tensor E(packed)
    through spinsum_exec on the plan's tiling: each output is the one product
    a(tau^-1) v either way (the sum adds exact zeros); integers bitwise."""
    shape, gf, d, dtype = OWN_TILING_CASES[case]
    coefs = np.random.default_rng(case).integers(-3, 4, math.factorial(d))
    stages = [workloads.antisymmetrizer(d)] if case % 2 == 0 else [
        [(p, float(c)) for p, c in zip(itertools.permutations(range(d)), coefs)]]
    # in place: the sum's own tiling (out of place, FP64 cubes that fit are
    # whole for the sum as well)
    p = ss.spinsum_plan(shape, gf, d, stages, dtype=dtype, inplace=True)
    info = ss.spinsum_plan_get_info(p)
    assert info["unpack_bl"] != info["bl"], info
    pshape = ss.packed_shape(p)
    pk = workloads.uniform(pshape, 4100 + case, device=DEV, dtype=dtype)
    full = torch.full(shape, float("nan"), dtype=dtype, device=DEV)
    ss.spinsum_unpack(p, pk, full)
    torch.cuda.synchronize()
    pkh = pk.cpu().to(torch.float64).numpy()
    ref = oracle.unpack(pkh, shape, stages, gf, d)
    assert nerr(full.cpu().to(torch.float64).numpy(), ref) <= TOL[dtype]
    emb = torch.from_numpy(oracle.embed_packed(pkh, shape, gf, d)).to(dtype).to(DEV)
    ss.spinsum_exec(p, emb, emb)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(full.cpu().numpy(), emb.cpu().numpy())
    pki = workloads.integers(pshape, 4200 + case, device=DEV, dtype=dtype)
    ss.spinsum_unpack(p, pki, full)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(full.cpu().to(torch.float64).numpy(),
                                  oracle.unpack(pki.cpu().to(torch.float64).numpy(), shape, stages, gf, d))


PERSISTENT_CASES = [
    # (shape, group_first, d, dtype): unpacked by the persistent kernel,
    # several cubes per workgroup
    ((2000, 24, 24, 24), 1, 3, torch.float64),    # whole cubes, about 8 per workgroup
    ((400, 32, 32, 32), 1, 3, torch.float64),     # 16^3 tiles: four templates, 1 or 3 tiles
    ((400, 16, 16, 16, 3), 1, 3, torch.float64),  # inner runs of 3
    ((300, 100, 100), 1, 2, torch.float64),
    ((500, 32, 32, 32), 1, 3, torch.float32),
    ((64, 2, 2, 24, 24, 24), 3, 3, torch.float64),  # several outer axes
]


def _cube_view(shape, gf, d):
    """(outer cubes, N, .., N, inner..) and the packed (outer, C(N, d), inner..)."""
    outer = math.prod(shape[:gf])
    n = shape[gf]
    return (outer,) + (n,) * d + tuple(shape[gf + d:]), (outer, math.comb(n, d)) + tuple(shape[gf + d:])


@pytest.mark.parametrize("case", range(len(PERSISTENT_CASES)))
def test_unpack_persistent(case):
    """Persistent unpacking: bit for bit against the one-item-per-
    workgroup kernel on the same tiling (SPINSUM_FLAG_NO_XCD_REMAP switches
    the persistent launch off; each output is the same one product either
    way), against the oracle on sampled cubes (first, last, and cubes that
    workgroups take second and later), and bitwise on integers."""
    shape, gf, d, dtype = PERSISTENT_CASES[case]
    stages = [workloads.antisymmetrizer(d)] if case % 2 == 0 else [workloads.CONFIG_3D_ALPHA] \
        if d == 3 else [[((0, 1), 2.0), ((1, 0), -0.5)]]
    p = ss.spinsum_plan(shape, gf, d, stages, dtype=dtype)
    q = ss.spinsum_plan(shape, gf, d, stages, dtype=dtype, flags=ss.SPINSUM_FLAG_NO_XCD_REMAP)
    assert ss.spinsum_plan_get_info(p)["unpack_persistent"] == 1
    assert ss.spinsum_plan_get_info(q)["unpack_persistent"] == 0
    cshape, pshape = _cube_view(shape, gf, d)
    ncube = cshape[0]
    sample = sorted(c for c in {0, 1, 31, 32, 33, 257, 300, ncube // 2, ncube - 2, ncube - 1}
                    if c < ncube)
    for kind in ("uniform", "integers"):
        gen = workloads.uniform if kind == "uniform" else workloads.integers
        pk = gen(ss.packed_shape(p), 4300 + case, device=DEV, dtype=dtype)
        a = torch.full(shape, float("nan"), dtype=dtype, device=DEV)
        b = torch.full(shape, float("nan"), dtype=dtype, device=DEV)
        ss.spinsum_unpack(p, pk, a)
        ss.spinsum_unpack(q, pk, b)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        pks = pk.reshape(pshape)[sample].cpu().to(torch.float64).numpy()
        ref = oracle.unpack(pks, (len(sample),) + cshape[1:], stages, 1, d)
        got = a.reshape(cshape)[sample].cpu().to(torch.float64).numpy()
        if kind == "uniform":
            assert nerr(got, ref) <= TOL[dtype]
        else:
            np.testing.assert_array_equal(got, ref)
        del pk, a, b
        torch.cuda.empty_cache()
