"""Host-side tests of libspinsum (no GPU): exported symbols, argument
validation, canonicalisation, the expanded operator, the tile-orbit tables
and the work ownership that makes the in-place form safe.

Plans are made with SPINSUM_FLAG_HOST_ONLY, so no HIP call is made.
"""
import itertools
import math
import os
import re
import ctypes

import numpy as np
import pytest

import oracle
import workloads
import paper_1705_06661_amd as ss
from workloads import P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = ss.SPINSUM_FLAG_HOST_ONLY
VARIANTS_ALL = [ss.SPINSUM_VARIANT_DIRECT_LDS, ss.SPINSUM_VARIANT_REG_PIPELINE,
                ss.SPINSUM_VARIANT_REG_ONESHOT, ss.SPINSUM_VARIANT_LDS_PIPELINE]


def plan(shape, stages, d=None, dtype="f64", inplace=False, flags=0):
    d = d or len(stages[0][0][0])
    return ss.spinsum_plan(shape, len(shape) - d, d, stages, dtype=dtype, inplace=inplace,
                           flags=flags | HOST)


def _rand(shape, seed):
    return workloads.uniform(shape, seed).numpy()


# ------------------------------------------------------------------ ABI
def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "spinsum.h")).read()
    declared = set(re.findall(r"^[A-Za-z_][\w \*]*?\b(spinsum_\w+)\s*\(", hdr, re.M))
    assert len(declared) >= 18
    lib = ctypes.CDLL(ss.LIB_PATH)
    for name in sorted(declared):
        assert hasattr(lib, name), name
    assert set(ss.EXPORTED) == declared


def test_version_and_status_strings():
    assert "spinsum" in ss.spinsum_version()
    for st in range(-9, 1):
        assert ss.spinsum_status_string(st) != "unknown status"


# ------------------------------------------------------------ validation
@pytest.mark.parametrize("shape,stages,d,code", [
    ((4, 3, 3, 3), [[((0, 0, 1), 1.0)]], 3, ss.SPINSUM_ERR_NOT_PERMUTATION),
    ((4, 3, 3, 3), [[((0, 1, 3), 1.0)]], 3, ss.SPINSUM_ERR_NOT_PERMUTATION),
    ((4, 3, 3, 4), [[((0, 1, 2), 1.0)]], 3, ss.SPINSUM_ERR_EXTENT_MISMATCH),
    ((2, 2, 2, 2, 2, 2), [[((0, 1, 2, 3, 4), 1.0)]], 5, ss.SPINSUM_ERR_UNSUPPORTED),
    ((3, 3), [[((0,), 1.0)]], 1, ss.SPINSUM_ERR_UNSUPPORTED),
    ((4, 3, 3, 3), [[((0, 1, 2), float("nan"))]], 3, ss.SPINSUM_ERR_INVALID_ARG),
    ((4, 3, 3, 3), [], 3, ss.SPINSUM_ERR_INVALID_ARG),
    ((-1, 3, 3, 3), [[((0, 1, 2), 1.0)]], 3, ss.SPINSUM_ERR_INVALID_ARG),
])
def test_plan_rejects_bad_arguments(shape, stages, d, code):
    with pytest.raises(ss.SpinSumError) as e:
        ss.spinsum_plan(shape, len(shape) - d, d, stages, flags=HOST)
    assert e.value.status == code


@pytest.mark.parametrize("shape,gf,d,dtype", [
    ((4, 6, 6, 6, 3), 1, 3, "f64"), ((2, 8, 8, 8, 5), 1, 3, "f32"),
    ((3, 5, 5, 5, 5, 2), 1, 4, "f64"), ((3, 7, 7, 2, 3), 1, 2, "f64"),
    ((2, 12, 12, 12, 4), 1, 3, "f64"), ((9, 9, 9, 2), 0, 3, "f32"),
    ((13, 13, 13, 2), 0, 3, "f64"), ((1, 10, 10, 10, 2, 3), 1, 3, "f64"),
])
def test_inner_spectator_addresses_replayed(shape, gf, d, dtype):
    """Groups followed by inner spectator dims: tiles hold runs of `inner`
    elements per group position.  Every tile edge and kernel variant the
    planner accepts has its load/combine/store addresses replayed."""
    terms = [[(p, 1.0 + i) for i, p in enumerate(itertools.permutations(range(d)))]]
    p = ss.spinsum_plan(shape, gf, d, terms, dtype=dtype, flags=HOST)
    ok, why = ss.spinsum_plan_check_ownership(p)
    assert ok, why
    n = shape[gf]
    accepted = 0
    for bl in range(1, n + 1):
        for pad in (0, 1):
            for variant in VARIANTS_ALL:
                try:
                    ss.spinsum_plan_set_tile(p, bl, cubes_per_wg=2, lds_pad=pad, variant=variant)
                except ss.SpinSumError:
                    continue
                accepted += 1
                ok, why = ss.spinsum_plan_check_ownership(p)
                assert ok, (bl, pad, variant, why)
    assert accepted > 0


@pytest.mark.parametrize("shape,gf,d,dtype", [
    ((3, 3, 4, 4), 2, 2, "f64"), ((2, 4, 4, 4, 6, 6, 6), 4, 3, "f64"),
    ((3, 3, 3, 5, 5, 5, 2), 3, 3, "f32"), ((2, 2, 2, 2, 3, 3, 3, 3), 4, 4, "f64"),
    ((4, 4, 4, 12, 12, 12), 3, 3, "f64"), ((3, 3, 3, 3, 6, 6, 6, 6), 4, 4, "f32"),
    ((2, 6, 6, 6, 10, 10, 10, 3), 4, 3, "f64"), ((5, 5, 9, 9), 2, 2, "f32"),
])
def test_index_pair_items_replayed(shape, gf, d, dtype):
    """Index-pair form: every work item's tile list, loads, combine addresses
    and element ownership replayed on the host for every usable tile edge."""
    terms = [[(p, 1.0) for p in itertools.permutations(range(d))]]
    flags = HOST | ss.SPINSUM_FLAG_INDEX_PAIRS
    p = ss.spinsum_plan(shape, gf, d, terms, dtype=dtype, flags=flags)
    info = ss.spinsum_plan_get_info(p)
    V, n = shape[gf - d], shape[gf]
    nb = info["nb"]
    assert info["pair_extent"] == V and info["variant"] == ss.SPINSUM_VARIANT_DIRECT_LDS
    assert info["norbits"] == math.comb(V * nb + d - 1, d)   # multisets of combined blocks
    assert info["elems"] == int(np.prod(shape))
    accepted = 0
    for bl in range(1, n + 1):
        try:
            ss.spinsum_plan_set_tile(p, bl)
        except ss.SpinSumError:
            continue
        accepted += 1
        ok, why = ss.spinsum_plan_check_ownership(p)
        assert ok, (bl, why)
    assert accepted > 0


def test_index_pair_reductions_and_errors():
    terms = [workloads.CONFIG_3D_ALPHA]
    fl = HOST | ss.SPINSUM_FLAG_INDEX_PAIRS
    # V == 1: the ordinary summation over the group
    i1 = ss.spinsum_plan_get_info(ss.spinsum_plan((1, 1, 1, 5, 5, 5), 3, 3, terms, flags=fl))
    assert i1["pair_extent"] == 0 and i1["n"] == 5
    # N == 1: the ordinary summation over the partners
    i2 = ss.spinsum_plan_get_info(ss.spinsum_plan((5, 5, 5, 1, 1, 1), 3, 3, terms, flags=fl))
    assert i2["pair_extent"] == 0 and i2["n"] == 5
    with pytest.raises(ss.SpinSumError) as e:
        ss.spinsum_plan((4, 4, 4, 4, 4), 2, 3, terms, flags=fl)   # no room for partners
    assert e.value.status == ss.SPINSUM_ERR_INVALID_ARG
    with pytest.raises(ss.SpinSumError) as e:
        ss.spinsum_plan((3, 3, 2, 4, 4, 4), 3, 3, terms, flags=fl)
    assert e.value.status == ss.SPINSUM_ERR_EXTENT_MISMATCH
    p = ss.spinsum_plan((3, 3, 3, 4, 4, 4), 3, 3, terms, flags=fl)
    with pytest.raises(ss.SpinSumError) as e:
        ss.spinsum_plan_set_tile(p, 2, variant=ss.SPINSUM_VARIANT_REG_PIPELINE)
    assert e.value.status == ss.SPINSUM_ERR_UNSUPPORTED


def test_store_mode_rule():
    """Non-temporal stores for whole cubes and for tile rows of at least 64
    bytes in cubes of at most 128 tile orbits; cached stores otherwise; the
    flags override the rule."""
    cfg3 = [workloads.CONFIG_3D_ALPHA]
    def nt(shape, gf, d, terms, flags=0, dtype="f64"):
        p = ss.spinsum_plan(shape, gf, d, terms, dtype=dtype, flags=flags | HOST)
        return ss.spinsum_plan_get_info(p)["nt_stores"]
    a4 = [(p, 1.0) for p in itertools.permutations(range(4))]
    assert nt((2, 32, 32, 32), 1, 3, cfg3) == 1              # 64-byte rows, 20 orbits
    assert nt((4, 8, 8, 8), 1, 3, cfg3) == 1                 # whole cubes
    assert nt((2, 12, 12, 12, 12), 1, 4, [a4]) == 0          # 32-byte rows
    assert nt((352, 352, 352), 0, 3, cfg3) == 0              # one cube of 1140 orbits
    assert nt((2, 12, 12, 12, 12), 1, 4, [a4], ss.SPINSUM_FLAG_NT_STORES) == 1
    assert nt((2, 32, 32, 32), 1, 3, cfg3, ss.SPINSUM_FLAG_NO_NT_STORES) == 0


def test_load_policy_rule():
    """Non-temporal tile loads exactly where every work item owns the
    128-byte lines it reads: whole cubes, or tile rows whose stride, length
    and ragged last length are all multiples of 128 bytes; the index-pair
    form and SPINSUM_FLAG_NO_NT_LOADS keep the default policy."""
    cfg3 = [workloads.CONFIG_3D_ALPHA]
    fig1b = [[((0, 1, 2), 1.0), (P("213"), 1.0)]]
    a4 = [(p, 1.0) for p in itertools.permutations(range(4))]
    def info(shape, gf, d, terms, flags=0, dtype="f64"):
        p = ss.spinsum_plan(shape, gf, d, terms, dtype=dtype, flags=flags | HOST)
        return ss.spinsum_plan_get_info(p)
    def ntl(*a, **k):
        return info(*a, **k)["nt_loads"]
    assert ntl((2, 32, 32, 32), 1, 3, cfg3) == 0                 # 64-byte rows
    assert ntl((2, 12, 12, 12, 12), 1, 4, [a4]) == 0             # 48-byte rows
    assert ntl((80, 80, 80, 80), 0, 4, [a4]) == 0                # 32-byte rows
    assert ntl((4, 8, 8, 8), 1, 3, cfg3) == 1                    # whole cubes
    assert ntl((5, 12, 12, 12), 1, 3, cfg3, dtype="f32") == 1    # whole cubes, 48-byte rows
    i = info((2, 3, 16, 16, 16, 8), 2, 3, cfg3)                  # inner runs of 8: 256-byte rows
    assert i["bl"] < 16 and i["nt_loads"] == 1
    i = info((2, 40, 40, 40, 16), 1, 3, cfg3)                    # ragged, rows of 16 k elements
    assert i["ragged"] == 1 and i["nt_loads"] == 1
    assert ntl((2, 40, 40, 40, 3), 1, 3, cfg3) == 0              # 24-byte inner runs
    i = info((2, 3, 16, 16, 16), 2, 3, fig1b)                    # Fig. 1b: last axis as runs
    assert i["exec_d"] == 2 and i["nt_loads"] == 1
    assert ntl((2, 3, 16, 16, 16, 8), 2, 3, cfg3, ss.SPINSUM_FLAG_NO_NT_LOADS) == 0
    assert ntl((4, 8, 8, 8), 1, 3, cfg3, ss.SPINSUM_FLAG_NO_NT_LOADS) == 0
    assert ntl((4, 4, 4, 8, 8, 8), 3, 3, cfg3, ss.SPINSUM_FLAG_INDEX_PAIRS) == 0
    bp = ss.spinsum_plan_batched([(8, 8, 8, 4, 4, 4), (6, 6, 6, 10, 10, 10)], 3, cfg3, flags=HOST)
    assert ss.spinsum_plan_get_info(bp)["nt_loads"] == 1


def test_coef_grad_kernel_rule():
    """The coefficient gradient keeps one tensor in LDS (k_cgrad_split) for
    tiled direct-LDS items of one tile orbit that one workgroup pass covers,
    with at most two element orbits per thread, d <= 3 and no inner runs."""
    cfg3 = [workloads.CONFIG_3D_ALPHA]
    a4 = [(p, 1.0) for p in itertools.permutations(range(4))]
    def split(shape, gf, d, terms, dtype="f64", tile=None, flags=0):
        p = ss.spinsum_plan(shape, gf, d, terms, dtype=dtype, flags=flags | HOST)
        if tile:
            ss.spinsum_plan_set_tile(p, *tile)
        return ss.spinsum_plan_get_info(p)["coef_grad_split"]
    assert split((64, 64, 8, 32, 32, 32), 3, 3, cfg3) == 1      # 8^3 tiles, 256 chunks
    assert split((2, 20, 20, 20), 1, 3, cfg3, tile=(8, 1, 0)) == 1
    assert split((64, 64, 8, 32, 32, 32), 3, 3, cfg3, dtype="f32") == 0  # 1024 chunks a tile
    assert split((4, 8, 8, 8), 1, 3, cfg3) == 0                  # whole cubes
    assert split((2, 16, 16, 16, 3), 1, 3, cfg3) == 0            # inner runs
    assert split((2, 12, 12, 12, 12), 1, 4, [a4]) == 0           # d = 4
    assert split((2, 20, 20, 20), 1, 3, cfg3,                      # register variant
                 tile=(8, 1, 1, 0, ss.SPINSUM_VARIANT_REG_ONESHOT)) == 0
    assert split((4, 4, 4, 24, 24, 24), 3, 3, cfg3, flags=ss.SPINSUM_FLAG_INDEX_PAIRS) == 0
    bp = ss.spinsum_plan_batched([(8, 8, 8, 4, 4, 4)], 3, cfg3, flags=HOST)
    assert ss.spinsum_plan_get_info(bp)["coef_grad_split"] == 0


def test_unpack_tiling_rule():
    """Unpacking runs on the largest items a CU holds: whole cubes where a
    cube and its representative list fit the LDS, else the largest tile
    edge whose rows are whole 128-byte lines and whose items fit; the plan's
    own tiling otherwise (unpack_bl reports it)."""
    as3, as4 = [workloads.antisymmetrizer(3)], [workloads.antisymmetrizer(4)]
    def ub(shape, gf, d, terms, dtype="f64"):
        i = ss.spinsum_plan_get_info(ss.spinsum_plan(shape, gf, d, terms, dtype=dtype, inplace=True,
                                                     flags=HOST))
        return i["bl"], i["unpack_bl"]
    assert ub((64, 64, 8, 32, 32, 32), 3, 3, as3) == (8, 16)       # 256 KiB cubes: 128-byte rows
    assert ub((48, 48, 48, 24, 24, 24), 3, 3, as3) == (8, 24)      # whole 108 KiB cubes
    assert ub((64, 64, 8, 32, 32, 32), 3, 3, as3, "f32") == (16, 32)
    assert ub((3, 16, 16, 16, 4), 1, 3, as3) == (16, 16)           # whole cubes (5 would be ragged)
    assert ub((1, 24, 24, 24, 12, 12, 12, 12), 4, 4, as4) == (6, 6)  # 162 KiB cubes, 48-byte rows
    assert ub((80, 80, 80, 80), 0, 4, as4) == (4, 4)
    assert ub((4, 11, 11, 11), 1, 3, as3) == (11, 11)              # whole cubes already
    assert ub((2, 160, 160), 1, 2, [workloads.antisymmetrizer(2)]) == (40, 80)
    bp = ss.spinsum_plan_batched([(8, 8, 8, 4, 4, 4)], 3, as3, flags=HOST)
    assert ss.spinsum_plan_get_info(bp)["unpack_bl"] == 0
    # unpacking's own items of d <= 3 run persistently where each template is
    # one tile orbit or one whole cube whose units the threads hold; 4D,
    # several cubes per workgroup and the ablation flag do not
    cubes = lambda shape, gf, d, terms, dtype="f64", flags=0: ss.spinsum_plan_get_info(
        ss.spinsum_plan(shape, gf, d, terms, dtype=dtype, flags=HOST | flags))["unpack_persistent"]
    assert cubes((48, 48, 48, 24, 24, 24), 3, 3, as3) == 1
    assert cubes((64, 64, 8, 32, 32, 32), 3, 3, as3, "f32") == 1
    assert cubes((300, 100, 100), 1, 2, [workloads.antisymmetrizer(2)]) == 1
    assert cubes((64, 64, 8, 32, 32, 32), 3, 3, as3) == 1
    assert cubes((60, 160, 160), 1, 2, [workloads.antisymmetrizer(2)]) == 0  # 6400 units
    assert cubes((1, 24, 24, 24, 12, 12, 12, 12), 4, 4, as4) == 0
    assert cubes((4, 11, 11, 11), 1, 3, as3) == 1                   # whole cubes, one per item
    assert cubes((8192, 8, 8, 8), 1, 3, as3) == 0                   # two cubes per workgroup
    assert cubes((48, 48, 48, 24, 24, 24), 3, 3, as3, flags=ss.SPINSUM_FLAG_NO_XCD_REMAP) == 0


def test_inner_spectator_geometry():
    """A cube of [.., N^d, inner] is N^d * inner contiguous elements; rows
    along the last group axis hold bl * inner elements."""
    p = ss.spinsum_plan((2, 32, 32, 32, 3), 1, 3, [workloads.CONFIG_3D_ALPHA], inplace=True,
                        flags=HOST)
    info = ss.spinsum_plan_get_info(p)
    assert info["elems"] == 2 * 32 ** 3 * 3 and info["ncubes"] == 2
    assert info["bl"] < 32 and info["bl"] % 2 == 0      # 16-byte rows: bl * 3 * 8 % 16 == 0
    assert info["vector_width"] == 2
    # an empty inner dim empties the tensor
    p0 = ss.spinsum_plan((3, 4, 4, 4, 0), 1, 3, [workloads.CONFIG_3D_ALPHA], flags=HOST)
    assert ss.spinsum_plan_get_info(p0)["elems"] == 0


def test_host_only_plan_refuses_exec():
    p = plan((4, 3, 3, 3), [workloads.CONFIG_3D_ALPHA])
    st = ss._c_exec(p._h, 256, 4096, None)
    assert st == ss.SPINSUM_ERR_NO_DEVICE
    st = ss._c_adjoint(p._h, 256, 4096, None)
    assert st == ss.SPINSUM_ERR_NO_DEVICE


def test_exec_rejects_null_plan_and_batched_misuse():
    assert ss._c_exec(None, 256, 4096, None) == ss.SPINSUM_ERR_INVALID_ARG
    assert ss._c_exec_batched(None, 256, 4096, None) == ss.SPINSUM_ERR_INVALID_ARG
    bp = ss.spinsum_plan_batched([(2, 3, 3, 3)], 3, [workloads.CONFIG_3D_ALPHA], flags=HOST)
    assert ss._c_exec(bp._h, 256, 4096, None) == ss.SPINSUM_ERR_INVALID_ARG


def test_stream_copy_argument_checks():
    assert ss._c_copy(256, 4096, 15, None) == ss.SPINSUM_ERR_INVALID_ARG
    assert ss._c_copy(256, 4096, 0, None) == ss.SPINSUM_OK
    assert ss._c_copy(8, 4096, 16, None) == ss.SPINSUM_ERR_MISALIGNED


# ------------------------------------------------------- expanded operator
def _as_dict(terms):
    return {tuple(p): a for p, a in terms}


def test_expanded_3d_factorisations():
    d, st1 = workloads.table2_case(1)
    assert _as_dict(ss.spinsum_plan_expanded(plan((2, 4, 4, 4), st1))) == \
        _as_dict(workloads.CONFIG_3D_ALPHA)
    want = {P("123"): 4.0, P("213"): -2.0, P("132"): -2.0, P("231"): 1.0}
    assert _as_dict(ss.spinsum_plan_expanded(plan((2, 4, 4, 4), workloads.FACTORED_PIJ_PJK))) == want
    eq8 = [workloads.stage((1, "123"), (1, "321"), (1, "132")),
           workloads.stage((1, "123"), (1, "213"))]
    assert _as_dict(ss.spinsum_plan_expanded(plan((1, 3, 3, 3), eq8))) == \
        {p: 1.0 for p in itertools.permutations(range(3))}


@pytest.mark.parametrize("case,count", [(1, 6), (2, 3), (5, 24), (6, 12), (8, 9), (9, 10),
                                        (11, 9), (17, 8), (18, 4), (21, 4)])
def test_expanded_term_counts_table2(case, count):
    d, stages = workloads.table2_case(case)
    p = plan((1,) + (3,) * d, stages, d=d)
    assert ss.spinsum_plan_get_info(p)["nterms_expanded"] == count


@pytest.mark.parametrize("case", range(1, 22))
def test_expanded_operator_matches_oracle_chain(case):
    d, stages = workloads.table2_case(case)
    p = plan((2,) + (4,) * d, stages, d=d)
    x = _rand((2,) + (4,) * d, case)
    exp = ss.spinsum_plan_expanded(p)
    np.testing.assert_allclose(oracle.spinsum(x, exp, 1, d), oracle.spinsum_chain(x, stages, 1, d),
                               rtol=0, atol=1e-11)
    # the planner's product, term by term, against the oracle's own
    assert _as_dict(exp) == {tuple(q): a for q, a in oracle.expanded_terms(stages, d)}


def test_duplicates_merge_and_zeros_drop():
    ident = (0, 1, 2)
    p = plan((2, 3, 3, 3), [[(ident, 1.0), (P("213"), 2.0), (ident, -1.0), (P("213"), 0.5)]])
    assert _as_dict(ss.spinsum_plan_expanded(p)) == {P("213"): 2.5}
    z = plan((2, 3, 3, 3), [[(ident, 0.0)]])
    assert ss.spinsum_plan_expanded(z) == []


# --------------------------------------------------------- tile orbits
def _counts():
    rows = {}
    for ln in open(os.path.join(ROOT, "tests", "golden", "counts.txt")):
        if ln.strip() and not ln.startswith("#"):
            tok = ln.split()
            rows.setdefault(tok[0], []).append(dict(kv.split("=") for kv in tok[1:]))
    return rows


def test_task_count_of_sec45():
    """A 40^4 tensor blocked with bl = 8 gives 70 tile orbits (Sec. 4.5)."""
    for r in _counts()["tasks"]:
        d, n, bl = int(r["d"]), int(r["N"]), int(r["bl"])
        p = plan((1,) + (n,) * d, [[(tuple(range(d)), 1.0)]], d=d)
        ss.spinsum_plan_set_tile(p, bl, lds_pad=1)
        assert ss.spinsum_plan_get_info(p)["norbits"] == int(r["count"])


@pytest.mark.parametrize("d,n,bl", [(3, 32, 16), (3, 32, 8), (4, 12, 6), (4, 12, 4), (4, 12, 3),
                                    (3, 24, 12), (3, 24, 8), (2, 10, 5), (3, 13, 4), (4, 7, 3)])
def test_orbit_count_is_multiset_count(d, n, bl):
    """C(nb + d - 1, d) tile orbits for nb blocks per axis (Alg. 5a loop nest)."""
    p = plan((2,) + (n,) * d, [[(tuple(range(d)), 1.0)]], d=d)
    ss.spinsum_plan_set_tile(p, bl)
    nb = -(-n // bl)
    info = ss.spinsum_plan_get_info(p)
    assert info["norbits"] == math.comb(nb + d - 1, d)
    assert info["nb"] == nb
    assert info["max_tiles"] == max(
        len({tuple(B[i] for i in s) for s in itertools.permutations(range(d))})
        for B in itertools.combinations_with_replacement(range(nb), d))


@pytest.mark.parametrize("d,n,bl", [(3, 8, 8), (3, 8, 4), (3, 32, 8), (3, 12, 5), (3, 13, 4),
                                    (4, 12, 6), (4, 12, 4), (4, 7, 3), (4, 5, 5), (2, 9, 4),
                                    (2, 16, 16), (3, 1, 1), (4, 2, 1), (3, 24, 12)])
def test_ownership_every_element_exactly_once(d, n, bl):
    p = plan((1,) + (n,) * d, [[(tuple(range(d)), 1.0)]], d=d)
    ss.spinsum_plan_set_tile(p, bl)
    ok, why = ss.spinsum_plan_check_ownership(p)
    assert ok, why


def test_lds_footprint_matches_eq11():
    """Eq. 11: C_min = bl^d * m * x * 8 B with x = 2 d! blocks per thread.
    The GPU form keeps one copy of the d! tiles of an orbit in LDS and
    overwrites it in place, so an unpadded orbit occupies C_min / 2."""
    for r in _counts()["cmin"]:
        d, bl, kib = int(r["d"]), int(r["bl"]), int(r["kib"])
        assert bl ** d * 1 * (2 * math.factorial(d)) * 8 == kib * 1024
    # checkable sizes that fit the 160 KiB LDS
    for d, bl in [(3, 8), (3, 6), (4, 3), (4, 2)]:
        n = d * bl
        p = plan((1,) + (n,) * d, [[(tuple(range(d)), 1.0)]], d=d,
                 flags=ss.SPINSUM_FLAG_NO_LDS_PAD)
        ss.spinsum_plan_set_tile(p, bl, lds_pad=0)
        cmin = bl ** d * 1 * (2 * math.factorial(d)) * 8
        assert ss.spinsum_plan_get_info(p)["lds_bytes"] == cmin // 2
    # the paper's own choices (3D bl=16, 4D bl=8) do not fit one CU's LDS
    for d, bl in [(3, 16), (4, 8)]:
        n = d * bl
        p = plan((1,) + (n,) * d, [[(tuple(range(d)), 1.0)]], d=d)
        ss.spinsum_plan_set_tile(p, bl, lds_pad=0)
        info = ss.spinsum_plan_get_info(p)
        assert info["lds_bytes"] == bl ** d * math.factorial(d) * 8 and not info["fits_lds"]


@pytest.mark.parametrize("name,bl,whole", [("3d_v16_o8", 8, True), ("3d_v64_o32_slab", 8, False),
                                           ("4d_v24_o12_slab", 6, False), ("3d_v48_o24", 8, False)])
def test_default_tiles_of_the_workloads(name, bl, whole):
    w = workloads.WORKLOADS[name]
    p = ss.spinsum_plan(w["shape"], w["group_first"], w["d"], [workloads.CONFIG_3D_ALPHA] if w["d"] == 3
                        else [workloads.random_4d_alpha(1)], inplace=True, flags=HOST)
    info = ss.spinsum_plan_get_info(p)
    assert info["bl"] == bl
    assert (info["norbits"] == 1) == whole
    assert info["lds_bytes"] <= 160 * 1024
    assert info["vector_width"] == 2
    assert info["elems"] == int(np.prod(w["shape"]))


def test_default_tiles_follow_the_measured_rules():
    """Cubes up to 64 KiB whole (8 KiB per workgroup when small); larger
    cubes in tile orbits of 16-byte-chunk rows within 32 KiB, widest rows
    first (ragged edge tiles allowed)."""
    alpha = [workloads.CONFIG_3D_ALPHA]
    for shape, dtype, bl, cpw in [((64, 64, 64, 8, 8, 8), "f64", 8, 2),
                                  ((48, 48, 48, 24, 24, 24), "f32", 24, 1),
                                  ((40, 40, 40, 20, 20, 20), "f64", 20, 1),
                                  ((32, 32, 32, 28, 28, 28), "f64", 8, 1),
                                  ((16, 16, 16, 40, 40, 40), "f64", 8, 1),
                                  ((64, 64, 8, 32, 32, 32), "f32", 16, 1)]:
        p = plan(shape, alpha, dtype=dtype)
        info = ss.spinsum_plan_get_info(p)
        assert (info["bl"], info["cubes_per_wg"]) == (bl, cpw), shape
        assert info["variant"] == ss.SPINSUM_VARIANT_DIRECT_LDS


@pytest.mark.parametrize("shape,d,dtype,bl,items,tiles", [
    ((3, 12, 12, 12, 12), 4, "f64", 6, 3, 6),     # classes 1+4 | 6 | 4+1 tiles
    ((3, 32, 32, 32), 3, "f32", 16, 2, 4),        # classes 1+3 | 3+1 tiles
])
def test_two_blocks_per_axis_tiles_pack_neighbouring_classes(shape, d, dtype, bl, items, tiles):
    """Where the first default tile has rows shorter than 64 bytes, a tile
    with two blocks per axis and wider rows is taken if two workgroups
    still fit a CU; its orbits (the classes by number of upper blocks) are
    packed in order, neighbouring classes together."""
    terms = [[(tuple(range(d)), 1.0), (tuple(reversed(range(d))), -0.5)]]
    p = plan(shape, terms, d=d, dtype=dtype)
    info = ss.spinsum_plan_get_info(p)
    assert info["bl"] == bl and info["norbits"] == d + 1
    assert info["items_per_cube"] == items and info["item_tiles"] == tiles
    assert info["threads"] == 512 and info["lds_bytes"] <= 80 * 1024
    ok, why = ss.spinsum_plan_check_ownership(p)
    assert ok, why
    # rows of 64 bytes already: no change (3D 24^3 FP64 in place keeps bl = 8)
    p = ss.spinsum_plan((2, 24, 24, 24), 1, 3, [[((0, 1, 2), 1.0)]], inplace=True, flags=HOST)
    assert ss.spinsum_plan_get_info(p)["bl"] == 8


def test_whole_cubes_where_tiles_are_slow():
    """Cubes of d <= 3 that fit a CU's LDS are processed whole where no tile
    edge gives rows of whole 16-byte chunks, where the tiles would be ragged,
    and, out of place, where FP64 tile rows would write partial lines; in
    place with full 64-byte rows, FP32 32^3 cubes and 4D keep their tiles."""
    as3 = [workloads.antisymmetrizer(3)]
    bl = lambda shape, gf, d, terms, dtype="f64", inplace=False: ss.spinsum_plan_get_info(
        ss.spinsum_plan(shape, gf, d, terms, dtype=dtype, inplace=inplace, flags=HOST))["bl"]
    assert bl((48, 48, 48, 24, 24, 24), 3, 3, as3) == 24             # 108 KiB cubes
    assert bl((48, 48, 48, 24, 24, 24), 3, 3, as3, inplace=True) == 8
    assert bl((52, 52, 52, 22, 22, 22), 3, 3, as3) == 22             # ragged bl = 8 otherwise
    assert bl((44, 44, 44, 26, 26, 26), 3, 3, as3) == 26             # 137 KiB + 13 KiB of lists
    assert bl((40, 40, 40, 32, 32, 32), 3, 3, as3, "f32") == 16      # FP32 keeps its tiles
    assert bl((64, 64, 8, 32, 32, 32), 3, 3, as3) == 8               # 256 KiB: does not fit
    assert bl((1, 12, 12, 12, 12), 1, 4, [workloads.antisymmetrizer(4)]) == 6
    # no edge with rows of whole 16-byte chunks, or ragged tiles: whole cubes
    # in place too (the register path ran at a tenth of the speed)
    assert bl((40, 40, 40, 25, 25, 25), 3, 3, as3, inplace=True) == 25
    assert bl((40, 40, 40, 30, 30, 30), 3, 3, as3, "f32", inplace=True) == 30
    assert bl((52, 52, 52, 22, 22, 22), 3, 3, as3, inplace=True) == 22
    assert bl((40, 40, 40, 28, 28, 28), 3, 3, as3, "f32") == 28


def test_small_orbits_are_packed_where_few_workgroups_fit():
    """With fewer than four workgroups per CU (4D, 24-tile orbits of 4^4
    tiles), the planner packs consecutive orbits up to the largest one; an
    explicit tile keeps one orbit per item."""
    p = plan((1, 16, 16, 16, 16), [[((0, 1, 2, 3), 1.0), ((1, 0, 2, 3), 2.0)]], d=4,
             flags=ss.SPINSUM_FLAG_FULL_GROUP)
    info = ss.spinsum_plan_get_info(p)
    assert info["bl"] == 4 and info["item_tiles"] == 24
    assert info["items_per_cube"] < info["norbits"]
    ok, why = ss.spinsum_plan_check_ownership(p)
    assert ok, why
    ss.spinsum_plan_set_tile(p, 4)
    info = ss.spinsum_plan_get_info(p)
    assert info["items_per_cube"] == info["norbits"]


def test_batched_plan_tables():
    seed, blocks = workloads.batched_blocks()
    shapes = [(v, v, v, o, o, o) for v, o in blocks]
    p = ss.spinsum_plan_batched(shapes, 3, [workloads.CONFIG_3D_ALPHA], inplace=True, flags=HOST)
    info = ss.spinsum_plan_get_info(p)
    assert info["nblocks"] == 200
    assert info["elems"] == sum(v ** 3 * o ** 3 for v, o in blocks)
    assert info["lds_bytes"] <= 160 * 1024
    for b in (0, 17, 199):
        ok, why = ss.spinsum_plan_check_ownership(p, b)
        assert ok, why
    # whole cubes are packed up to the largest cube of at most 40 KiB (o = 16
    # here: 32 KiB), one workgroup per item unless a tuned cache says so
    assert info["batch_item_bytes"] == 16 ** 3 * 8 and info["batch_persistent"] == 0


def test_subgroup_reduction():
    """Terms that move only a contiguous run of the group's axes: the plan
    permutes those axes alone (Sec. 4.6.4's connected components), the fixed
    trailing axes moving as inner runs and the leading ones as outer
    spectators; SPINSUM_FLAG_FULL_GROUP keeps S_d.  The expanded operator and
    the ownership replay are those of the executing plan's group."""
    ident = (0, 1, 2)
    cases = [
        # pi_123 + pi_213 (Fig. 1b): axes 0, 1 of the group; axis 2 inner
        ((64, 4, 32, 32, 32), 2, [[(ident, 1.0), (P("213"), 1.0)]], 3, 2, 2, 32),  # first dim 2
        # 2 - pi_132: axes 1, 2; axis 0 an outer spectator
        ((3, 16, 16, 16), 1, [[(ident, 2.0), (P("132"), -1.0)]], 3, 2, 2, 1),  # first dim 2
        # (2 - pi_2134) in 4D: axes 0, 1; the other two inner (144 elements)
        ((1, 24, 12, 12, 12, 12), 2, [[((0, 1, 2, 3), 2.0), ((1, 0, 2, 3), -1.0)]], 4, 2, 2, 144),
        # a chain whose stages move axes (0,1) and (1,2): all three, no reduction
        ((3, 8, 8, 8), 1, workloads.FACTORED_PIJ_PJK, 3, 3, 1, 1),  # first dim 1
        # pi_321 alone moves axes 0 and 2 (not a contiguous run): no reduction
        ((3, 8, 8, 8), 1, [[(P("321"), 1.0)]], 3, 3, 1, 1),
    ]
    for shape, gf, stages, d, want_d, want_first, want_inner in cases:
        p = ss.spinsum_plan(shape, gf, d, stages, flags=HOST)
        info = ss.spinsum_plan_get_info(p)
        assert info["d"] == d and info["exec_d"] == want_d, (shape, info)
        assert info["exec_group_first"] == want_first
        assert info["inner"] == want_inner, info
        assert info["elems"] == int(np.prod(shape))
        ok, why = ss.spinsum_plan_check_ownership(p)
        assert ok, why
        exp = ss.spinsum_plan_expanded(p)
        assert _as_dict(exp) == {tuple(q): a for q, a in oracle.expanded_terms(stages, d)}
        full = ss.spinsum_plan(shape, gf, d, stages, flags=HOST | ss.SPINSUM_FLAG_FULL_GROUP)
        assert ss.spinsum_plan_get_info(full)["exec_d"] == d


def test_batched_plan_with_inner_runs():
    """A group at the same position of every block, inner spectator runs of
    each block's own length behind it: elements and the work decomposition
    of every block (whole cubes and tile orbits)."""
    shapes = [(3, 5, 5, 5, 2), (2, 4, 4, 4, 7), (1, 24, 24, 24, 3), (4, 2, 2, 2, 1), (2, 3, 3, 3, 16),
              (2, 16, 16, 16, 2), (1, 19, 19, 19, 1)]   # the last two: whole cubes of 40-64 KiB
    p = ss.spinsum_plan_batched(shapes, 3, [workloads.CONFIG_3D_ALPHA], inplace=True, flags=HOST,
                                group_first=1)
    info = ss.spinsum_plan_get_info(p)
    assert info["elems"] == sum(int(np.prod(s)) for s in shapes)
    assert info["ncubes"] == sum(s[0] for s in shapes)
    for b in range(len(shapes)):
        ok, why = ss.spinsum_plan_check_ownership(p, b)
        assert ok, (b, why)
    # -1: the trailing group of each block, whatever its rank
    q = ss.spinsum_plan_batched([(2, 4, 4, 4), (3, 2, 5, 5, 5), (2, 18, 18, 18)], 3,
                                [workloads.CONFIG_3D_ALPHA], flags=HOST)
    assert ss.spinsum_plan_get_info(q)["ncubes"] == 2 + 6 + 2
    for b in range(3):
        ok, why = ss.spinsum_plan_check_ownership(q, b)
        assert ok, (b, why)
    with pytest.raises(ss.SpinSumError):
        ss.spinsum_plan_batched([(2, 4, 4, 4)], 3, [workloads.CONFIG_3D_ALPHA], flags=HOST,
                                group_first=2)
    with pytest.raises(ss.SpinSumError) as e:
        ss.spinsum_plan_batched([(2, 2, 2, 4, 4, 4)], 3, [workloads.CONFIG_3D_ALPHA],
                                flags=HOST | ss.SPINSUM_FLAG_INDEX_PAIRS, group_first=3)
    assert e.value.status == ss.SPINSUM_ERR_UNSUPPORTED


def test_batched_plan_reads_a_tuned_cache_line(tmp_path, monkeypatch):
    """A batched cache line (item KiB, persistent flag) is applied when the
    plan is made; other plans' lines are ignored."""
    blocks = [(4, 6), (5, 3), (3, 8)]
    shapes = [(v, v, v, o, o, o) for v, o in blocks]
    elems = sum(v ** 3 * o ** 3 for v, o in blocks)
    cache = tmp_path / "tune.txt"
    cache.write_text(f"batch_b3_e{elems}_d3_f64_ip1_gfx950 16 1 0.5\n"
                     f"batch_b3_e{elems + 1}_d3_f64_ip1_gfx950 24 0 0.5\n")
    monkeypatch.setenv("SPINSUM_AUTOTUNE_CACHE", str(cache))
    p = ss.spinsum_plan_batched(shapes, 3, [workloads.CONFIG_3D_ALPHA], inplace=True, flags=HOST)
    info = ss.spinsum_plan_get_info(p)
    assert info["batch_item_bytes"] == 16 * 1024 and info["batch_persistent"] == 1
    for b in range(3):
        ok, why = ss.spinsum_plan_check_ownership(p, b)
        assert ok, why


def test_set_tile_rebuilds_and_rejects():
    p = plan((3, 16, 16, 16), [workloads.CONFIG_3D_ALPHA])
    for bl, norb in [(16, 1), (8, 4), (4, 20), (5, 20)]:
        ss.spinsum_plan_set_tile(p, bl)
        assert ss.spinsum_plan_get_info(p)["norbits"] == norb
        ok, why = ss.spinsum_plan_check_ownership(p)
        assert ok, why
    with pytest.raises(ss.SpinSumError):
        ss.spinsum_plan_set_tile(p, -3)


def test_fp32_plan_vector_width():
    p = plan((3, 16, 16, 16), [workloads.CONFIG_3D_ALPHA], dtype="f32")
    assert ss.spinsum_plan_get_info(p)["vector_width"] == 4
    q = plan((3, 6, 6, 6), [workloads.CONFIG_3D_ALPHA], dtype="f32")
    assert ss.spinsum_plan_get_info(q)["vector_width"] == 2
    r = plan((3, 5, 5, 5), [workloads.CONFIG_3D_ALPHA])
    assert ss.spinsum_plan_get_info(r)["vector_width"] == 1


@pytest.mark.parametrize("shape,d,tile,dtype", [
    ((5, 8, 8, 8), 3, (8, 2), "f64"), ((7, 8, 8, 8), 3, (8, 4), "f32"),
    ((9, 6, 6, 6), 3, (6, 4), "f32"), ((3, 5, 5, 5, 5), 4, (5, 2), "f64"),
    ((6, 16, 16), 2, (16, 4), "f32"), ((4, 33, 33), 2, (8, 1), "f64"),
    ((2, 32, 32, 32), 3, (8, 1), "f64"), ((2, 32, 32, 32), 3, (16, 1), "f32"),
    ((2, 12, 12, 12, 12), 4, (6, 1), "f64"), ((2, 12, 12, 12, 12), 4, (4, 1), "f32"),
    ((2, 24, 24, 24), 3, (12, 1), "f64"), ((2, 24, 24, 24), 3, (24, 1), "f32"),
    ((3, 13, 13, 13), 3, (4, 1), "f64"), ((2, 12, 12, 12), 3, (5, 1), "f32"),
])
def test_kernel_addresses_replayed_on_host(shape, d, tile, dtype):
    """The checker replays every load/combine/store address of every work
    item (including a partial last item of whole cubes) with the kernels'
    own index functions and checks bounds and consistency."""
    for pad in (1, 0):
        p = plan(shape, [[(tuple(range(d)), 1.0)]], d=d, dtype=dtype)
        ss.spinsum_plan_set_tile(p, tile[0], cubes_per_wg=tile[1], lds_pad=pad)
        ok, why = ss.spinsum_plan_check_ownership(p)
        assert ok, why


def test_direct_lds_variant_uses_dense_tiles():
    """The direct-LDS kernel lands 16-byte rows in chunk order: unpadded."""
    for shape, d, dtype, bl in [((3, 32, 32, 32), 3, "f64", 8), ((2, 12, 12, 12, 12), 4, "f64", 6),
                                ((3, 16, 16, 16), 3, "f32", 8), ((5, 8, 8, 8), 3, "f64", 8)]:
        p = plan(shape, [[(tuple(range(d)), 1.0)]], d=d, dtype=dtype)
        ss.spinsum_plan_set_tile(p, bl, lds_pad=1, variant=ss.SPINSUM_VARIANT_DIRECT_LDS)
        info = ss.spinsum_plan_get_info(p)
        assert info["variant"] == ss.SPINSUM_VARIANT_DIRECT_LDS and info["lds_pad"] == 0
        ok, why = ss.spinsum_plan_check_ownership(p)
        assert ok, why
    # tile rows that are not 16 bytes fall back to the register one-shot kernel
    p = plan((3, 12, 12, 12), [[((0, 1, 2), 1.0)]], dtype="f32")
    ss.spinsum_plan_set_tile(p, 6, variant=ss.SPINSUM_VARIANT_DIRECT_LDS)
    assert ss.spinsum_plan_get_info(p)["variant"] == ss.SPINSUM_VARIANT_REG_ONESHOT
    # whole cubes of any extent are copied as one contiguous run
    for shape, dtype in [((3, 5, 5, 5), "f64"), ((3, 6, 6, 6), "f32"), ((7, 3, 3, 3, 3), "f64")]:
        q = plan(shape, [[(tuple(range(len(shape) - 1)), 1.0)]], d=len(shape) - 1, dtype=dtype)
        info = ss.spinsum_plan_get_info(q)
        assert info["bl"] == shape[1]
        assert info["variant"] == ss.SPINSUM_VARIANT_DIRECT_LDS
        ok, why = ss.spinsum_plan_check_ownership(q)
        assert ok, why


@pytest.mark.parametrize("d,n,bl", [(3, 32, 8), (3, 13, 4), (4, 12, 6), (4, 10, 4), (2, 16, 4),
                                    (3, 24, 6)])
def test_orbit_groups_cover_every_orbit(d, n, bl):
    """Work items are single tile orbits by default; with item_tiles > 0 the
    orbits of a cube are packed into items of at most max(item_tiles,
    largest orbit) tiles, and every element is still owned exactly once."""
    p = plan((2,) + (n,) * d, [[(tuple(range(d)), 1.0)]], d=d)
    ss.spinsum_plan_set_tile(p, bl)
    info = ss.spinsum_plan_get_info(p)
    norb, biggest = info["norbits"], info["max_tiles"]
    assert info["items_per_cube"] == norb
    assert info["nitems"] == 2 * norb
    tiles_per_cube = (-(-n // bl)) ** d
    for cap in (1, biggest, 2 * biggest, 24):
        ss.spinsum_plan_set_tile(p, bl, item_tiles=cap)
        info = ss.spinsum_plan_get_info(p)
        eff = min(max(cap, biggest), 24)
        assert info["item_tiles"] <= eff
        assert info["items_per_cube"] >= -(-tiles_per_cube // eff)
        assert info["items_per_cube"] <= norb
        assert info["norbits"] == norb
        ok, why = ss.spinsum_plan_check_ownership(p)
        assert ok, (cap, why)


def test_lds_pipeline_variant_needs_two_buffers():
    """The double-buffered kernel holds two item buffers plus every
    representative table in LDS; it falls back to the one-shot direct-LDS
    kernel when they do not fit, and to registers without 16-byte rows."""
    V = ss.SPINSUM_VARIANT_LDS_PIPELINE
    p = plan((2, 32, 32, 32), [[((0, 1, 2), 1.0)]])
    ss.spinsum_plan_set_tile(p, 8, lds_pad=1, variant=V)
    info = ss.spinsum_plan_get_info(p)
    assert info["variant"] == V and info["lds_pad"] == 0
    ok, why = ss.spinsum_plan_check_ownership(p)
    assert ok, why
    ss.spinsum_plan_set_tile(p, 16, variant=V)  # 2 x 3 x 32 KiB > 160 KiB
    assert ss.spinsum_plan_get_info(p)["variant"] == ss.SPINSUM_VARIANT_DIRECT_LDS
    q = plan((2, 32, 32, 32), [[((0, 1, 2), 1.0)]], dtype="f32")
    ss.spinsum_plan_set_tile(q, 16, variant=V)  # 2 x 3 x 16 KiB fits
    assert ss.spinsum_plan_get_info(q)["variant"] == V
    r = plan((2, 12, 12, 12), [[((0, 1, 2), 1.0)]])
    ss.spinsum_plan_set_tile(r, 3, variant=V)  # 24-byte rows
    assert ss.spinsum_plan_get_info(r)["variant"] == ss.SPINSUM_VARIANT_REG_ONESHOT
