"""Pins of the CPU oracle to what the paper and the mathematics fix.

Nothing here re-types the oracle's own formula: the expected values come from
subscripts printed in the paper (Def. 1-2 examples, Alg. 1, Alg. 3, Alg. 6,
the Sec. 4.2 / 4.6.4 statements, the Sec. 4.6.2 re-basing example), from
library routines (numpy transpose), from closed forms of the symmetric group
(symmetric / antisymmetric inputs, the eigenvalues of the 3D coefficient set)
and from brute-force explicit matrices.
"""
import itertools
import math
import os
import re

import numpy as np
import pytest

import oracle
import workloads
from workloads import P, stage

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _lines(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.strip() for ln in f if ln.strip() and not ln.startswith("#")]


def _rand(shape, seed):
    return workloads.uniform(shape, seed).numpy()


def _sign(p):
    """Parity of a permutation from its inversion count."""
    inv = sum(1 for a in range(len(p)) for b in range(a + 1, len(p)) if p[a] > p[b])
    return -1 if inv % 2 else 1


# --------------------------------------------------------- Def. 1 / Def. 2
def test_def1_tuple_example():
    """Def. 1: pi_321 maps (i1,i2,i3) to (i3,i2,i1); via Def. 2 the output at
    (i1,i2,i3) reads the input at that permuted tuple."""
    (line,) = [ln for ln in _lines("def1_def2_examples.txt") if ln.startswith("tuple")]
    _, label, *rest = line.split()
    arrow = rest.index("->")
    src_syms, dst_syms = rest[:arrow], rest[arrow + 1:]
    n = 4
    enc = np.fromfunction(lambda a, b, c: 100 * a + 10 * b + c, (n, n, n))
    out = oracle.spinsum(enc, [(P(label), 1.0)], 0, 3)
    for idx in itertools.product(range(n), repeat=3):
        val = dict(zip(src_syms, idx))
        want = 100 * val[dst_syms[0]] + 10 * val[dst_syms[1]] + val[dst_syms[2]]
        assert out[idx] == want


@pytest.mark.parametrize("shape,gf", [((5, 5), 0), ((3, 4, 4), 1), ((4, 4, 2), 0),
                                      ((2, 3, 3, 5), 1)])
def test_def2_transpose_example(shape, gf):
    """Def. 2: B <- pi_21(A) is the matrix transposition."""
    x = _rand(shape, 11)
    out = oracle.spinsum(x, [(P("21"), 1.0)], gf, 2)
    np.testing.assert_array_equal(out, np.swapaxes(x, gf, gf + 1))


# ------------------------------------------------ printed update statements
def _parse_statements():
    ops, stmts = {}, []
    for ln in _lines("subscript_statements.txt"):
        tok = ln.split()
        if tok[0] == "op":
            ops[tok[1]] = [P(t) for t in tok[2:]]
        else:
            name = tok[1]
            lhs, rhs = " ".join(tok[2:]).split("=")
            lsub = lhs.split()[1:]
            reads = [r.split()[1:] for r in rhs.split("+")]
            stmts.append((name, lsub, reads))
    return ops, stmts


def test_printed_update_statements():
    """Alg. 1 line 5, Alg. 3 lines 5 and 10, and the Sec. 4.2 / 4.6.4
    statements, evaluated from their printed subscripts."""
    ops, stmts = _parse_statements()
    n = 4
    x = _rand((n, n, n), 5)
    for name, lsub, reads in stmts:
        out = oracle.spinsum(x, [(p, 1.0) for p in ops[name]], 0, 3)
        for vals in itertools.product(range(n), repeat=3):
            env = dict(zip(("i1", "i2", "i3"), vals))
            pos = tuple(env[s] for s in lsub)
            want = sum(x[tuple(env[s] for s in r)] for r in reads)
            assert abs(out[pos] - want) < 1e-14, (name, pos)


@pytest.mark.parametrize("bl", [2, 3])
def test_alg6_block_statements(bl):
    """Alg. 6: block offsets and intra-block indices permute together."""
    lines = _lines("alg6_block_statements.txt")
    op = [P(t) for t in lines[0].split()[1:]]
    stmts = []
    for ln in lines[1:]:
        lhs, rhs = ln.split("=")
        lt = lhs.split()[1:]
        reads = [r.split()[1:] for r in rhs.split("+")]
        stmts.append((lt, reads))
    n = 3 * bl
    x = _rand((n, n, n), 17)
    out = oracle.spinsum(x, [(p, 1.0) for p in op], 0, 3)
    for tb in itertools.product(range(3), repeat=3):
        for iv in itertools.product(range(bl), repeat=3):
            env = dict(zip(("t1", "t2", "t3"), [b * bl for b in tb]))
            env.update(zip(("i1", "i2", "i3"), iv))

            def at(sub):
                return tuple(env[sub[k]] + env[sub[k + 3]] for k in range(3))

            for lt, reads in stmts:
                want = sum(x[at(r)] for r in reads)
                assert abs(out[at(lt)] - want) < 1e-14


# ------------------------------------------------------ re-basing (Eq. 9-10)
def test_rebasing_example_sec462():
    """Sec. 4.6.2 prints T <- pi_213(A), B <- (a1 pi_213 + a2 pi_123 + a3 pi_231)(T)
    as equal to (a1 pi_123 + a2 pi_213 + a3 pi_321)(A).  The 3-cycle pi_231
    (not pi_312) fixes the direction of composition."""
    lines = _lines("rebasing_example.txt")
    coef = {"a1": 0.7, "a2": -1.3, "a3": 2.9}

    def parse(tokens):
        return [(P(tokens[k + 1]), coef[tokens[k]]) for k in range(0, len(tokens), 2)]

    direct = parse(lines[0].split()[1:])
    rebase = [(P(lines[1].split()[1]), 1.0)]
    then = parse(lines[2].split()[1:])
    x = _rand((2, 5, 5, 5), 3)
    want = oracle.spinsum(x, direct, 1, 3)
    got = oracle.spinsum_chain(x, [rebase, then], 1, 3)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)
    # the other 3-cycle gives a different operator: the pin discriminates
    wrong = [(p if p != P("231") else P("312"), a) for p, a in then]
    bad = oracle.spinsum_chain(x, [rebase, wrong], 1, 3)
    assert np.max(np.abs(bad - want)) > 0.1


def _compose(p1, p2):
    """Permutation of applying operator p1 after operator p2 (checked against
    the Sec. 4.6.2 example above)."""
    return tuple(p1[p2[m]] for m in range(len(p1)))


@pytest.mark.parametrize("d", [3, 4])
def test_eq9_10_rebasing_random(d):
    """Eq. 9-10: S(A) = S'(w(A)) with S' = sum alpha_i (w_i o w^-1)."""
    rng = np.random.default_rng(d)
    perms = list(itertools.permutations(range(d)))
    terms = [(perms[k], float(rng.normal())) for k in rng.choice(len(perms), 5, replace=False)]
    w = perms[rng.integers(len(perms))]
    winv = tuple(int(v) for v in np.argsort(w))
    then = [(_compose(p, winv), a) for p, a in terms]
    x = _rand((3,) + (4,) * d, 9)
    want = oracle.spinsum(x, terms, 1, d)
    got = oracle.spinsum_chain(x, [[(w, 1.0)], then], 1, d)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


# ------------------------------------------------------------ factorisation
def test_eq7_equals_eq8():
    """Eq. 7 (all six permutations) equals the factorised Eq. 8."""
    x = _rand((3, 6, 6, 6), 21)
    eq7 = stage(*[(1, lbl) for lbl in ("123", "132", "213", "231", "312", "321")])
    eq8 = [stage((1, "123"), (1, "321"), (1, "132")), stage((1, "123"), (1, "213"))]
    np.testing.assert_allclose(oracle.spinsum_chain(x, eq8, 1, 3),
                               oracle.spinsum(x, eq7, 1, 3), rtol=0, atol=1e-13)


def test_table2_transcription():
    """workloads.table2_case matches the printed Table II."""
    for ln in _lines("table2.txt"):
        case = int(ln.split()[0])
        factors = re.findall(r"\(([^)]*)\)", ln)
        d, stages = workloads.table2_case(case)
        assert len(stages) == len(factors)
        for st, fac in zip(stages, reversed(factors)):   # right-most acts first
            toks = fac.split()
            assert toks[0] == "2"
            assert st[0] == (tuple(range(d)), 2.0)
            assert [(P(t.lstrip("-")), -1.0) for t in toks[1:]] == st[1:]


def test_table2_case1_is_the_3d_coefficient_set():
    """Table II case 1 expands to: identity 4, transpositions -2, 3-cycles +1."""
    d, stages = workloads.table2_case(1)
    x = _rand((4, 5, 5, 5), 23)
    np.testing.assert_allclose(oracle.spinsum_chain(x, stages, 1, 3),
                               oracle.spinsum(x, workloads.CONFIG_3D_ALPHA, 1, 3),
                               rtol=0, atol=1e-12)


def _as_dict(terms):
    return {tuple(p): a for p, a in terms}


def test_expanded_terms_of_printed_products():
    """oracle.expanded_terms multiplies a chain out: Eq. 8 gives every
    permutation once (Eq. 7), Table II case 1 the 3D coefficient set, and
    (2 - P_ij)(2 - P_jk) gives 4 - 2 pi_213 - 2 pi_132 + pi_231 by hand
    (P_ij pi_132 . x reads x_(p_132 o ..), i.e. pi_231 for the stage order of
    Def. 4); a product that cancels, (1 + pi_213)(1 - pi_213) = 1 - pi_213^2,
    gives no term at all."""
    eq8 = [stage((1, "123"), (1, "321"), (1, "132")), stage((1, "123"), (1, "213"))]
    assert _as_dict(oracle.expanded_terms(eq8, 3)) == {p: 1.0 for p in itertools.permutations(range(3))}
    assert _as_dict(oracle.expanded_terms(workloads.table2_case(1)[1], 3)) == _as_dict(
        workloads.CONFIG_3D_ALPHA)
    assert _as_dict(oracle.expanded_terms(workloads.FACTORED_PIJ_PJK, 3)) == {
        P("123"): 4.0, P("213"): -2.0, P("132"): -2.0, P("231"): 1.0}
    cancel = [stage((1, "123"), (1, "213")), stage((1, "123"), (-1, "213"))]
    assert oracle.expanded_terms(cancel, 3) == []


def test_expanded_terms_agree_with_the_chain():
    """The multiplied-out sum of every Table II case acts like the chain."""
    for case in range(1, 22):
        d, stages = workloads.table2_case(case)
        x = _rand((2,) + (4,) * d, 60 + case)
        np.testing.assert_allclose(oracle.spinsum(x, oracle.expanded_terms(stages, d), 1, d),
                                   oracle.spinsum_chain(x, stages, 1, d), rtol=0, atol=1e-11)


def test_flop_reduction_factors_of_sec6():
    """The FLOP-count reduction the paper states for each group of Table II
    cases follows from the multiplied-out term counts (golden file)."""
    ident = {3: (0, 1, 2), 4: (0, 1, 2, 3)}
    for ln in _lines("flop_reduction.txt"):
        cases, factor = ln.split()
        lo, _, hi = cases.partition("-")
        for case in range(int(lo), int(hi or lo) + 1):
            d, stages = workloads.table2_case(case)
            expanded = [p for p, _ in oracle.expanded_terms(stages, d) if p != ident[d]]
            factor_terms = 0
            for st in stages:
                merged = {}
                for p, a in st:
                    merged[p] = merged.get(p, 0.0) + a
                factor_terms += sum(1 for p, a in merged.items() if a != 0.0 and p != ident[d])
            assert round(len(expanded) / factor_terms) == int(factor), case


@pytest.mark.parametrize("case", [1, 5, 9])
def test_coef_grad_stages_definition(case):
    """Per-stage coefficient gradients of a chain: L(alpha) = <g, S(x)> is
    linear in the coefficients of each stage, so adding 1 to the coefficient
    of permutation p in stage k changes L by exactly the derivative; and the
    derivative equals g^T M_K .. M_{k,p} .. M_1 x with the dense matrix of
    the single term p in place of stage k."""
    d, stages = workloads.table2_case(case)
    shape = (1,) + (3,) * d if d == 4 else (2, 3, 3, 3)
    x = _rand(shape, 70 + case)
    g = _rand(shape, 80 + case)
    got = oracle.coef_grad_stages(x, g, stages, 1, d)
    perms = list(itertools.permutations(range(d)))
    base = float(np.sum(g * oracle.spinsum_chain(x, stages, 1, d)))
    rng = np.random.default_rng(case)
    for k in range(len(stages)):
        for r in rng.choice(len(perms), size=4, replace=False):
            p = perms[r]
            bumped = [list(st) for st in stages]
            bumped[k] = bumped[k] + [(p, 1.0)]
            diff = float(np.sum(g * oracle.spinsum_chain(x, bumped, 1, d))) - base
            assert abs(diff - got[k, r]) <= 1e-12 * max(1.0, abs(diff))
            mats = [oracle.dense_matrix(shape, st, 1, d) for st in stages]
            mats[k] = oracle.dense_matrix(shape, [(p, 1.0)], 1, d)
            M = np.eye(x.size)
            for m in mats:
                M = m @ M
            dense = float(g.ravel() @ (M @ x.ravel()))
            assert abs(dense - got[k, r]) <= 1e-12 * max(1.0, abs(dense))


def test_unpack_worked_example():
    """N = 3, d = 2, the antisymmetriser: packed (a01, a02, a12) unpacks to
    [[0, a01, a02], [-a01, 0, a12], [-a02, -a12, 0]] (by hand, Def. 2)."""
    a01, a02, a12 = 1.5, -2.0, 7.0
    got = oracle.unpack(np.array([[a01, a02, a12]]), (1, 3, 3), [workloads.antisymmetrizer(2)], 1, 2)
    want = np.array([[[0.0, a01, a02], [-a01, 0.0, a12], [-a02, -a12, 0.0]]])
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("d,n", [(2, 5), (3, 5), (4, 5)])
def test_unpack_pack_antisymmetric(d, n):
    """An antisymmetric tensor X (A(Y)/d! of a random Y) is fixed by A/d! and
    is rebuilt by unpacking its strictly increasing entries with A; packing
    with A gives d! times those entries (A is self-adjoint and A X = d! X);
    unpacking gives an antisymmetric tensor with zero diagonals; and pack is
    the transpose of unpack (<U p, f> = <p, P f>)."""
    A = [workloads.antisymmetrizer(d)]
    shape = (2,) + (n,) * d
    y = _rand(shape, 90 + d)
    x = oracle.spinsum(y, A[0], 1, d) / math.factorial(d)
    np.testing.assert_allclose(oracle.spinsum(x, A[0], 1, d) / math.factorial(d), x, atol=1e-14)
    tuples = oracle.increasing_tuples(n, d)
    assert len(tuples) == math.comb(n, d)
    gathered = np.stack([x[(slice(None),) + t] for t in tuples], axis=1)
    np.testing.assert_allclose(oracle.unpack(gathered, shape, A, 1, d), x, atol=1e-14)
    np.testing.assert_allclose(oracle.pack(x, A, 1, d), math.factorial(d) * gathered, atol=1e-13)
    p = _rand((2, len(tuples)), 95 + d)
    u = oracle.unpack(p, shape, A, 1, d)
    for perm in itertools.permutations(range(d)):
        if _sign(perm) < 0:
            np.testing.assert_allclose(np.transpose(u, (0,) + tuple(1 + q for q in perm)), -u,
                                       atol=1e-14)
    f = _rand(shape, 99 + d)
    lhs = float(np.sum(u * f))
    rhs = float(np.sum(p * oracle.pack(f, A, 1, d)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_unpack_with_identity_is_the_embedding():
    """With the identity operator unpacking only places the packed values
    (dense matrix of E checked element by element) and packing gathers."""
    shape = (2, 4, 4, 4, 3)
    p = _rand((2, math.comb(4, 3), 3), 101)
    u = oracle.unpack(p, shape, [[((0, 1, 2), 1.0)]], 1, 3)
    for r, t in enumerate(itertools.combinations(range(4), 3)):
        np.testing.assert_array_equal(u[(slice(None),) + t], p[:, r])
    assert np.count_nonzero(u) == p.size
    np.testing.assert_array_equal(oracle.pack(u, [[((0, 1, 2), 1.0)]], 1, 3), p)


def test_factored_pij_pjk_closed_form():
    """(2 - P_ij)(2 - P_jk) on A[i,j,k] = 100i + 10j + k.
    By hand from Def. 2: T = 2A - A[i,k,j] = 100i + 19j - 8k, then
    B = 2T - T[j,i,k] = 181i - 62j - 8k.  The reversed product gives
    190i - 161j + 82k, so this pins the stage order."""
    n = 5
    enc = np.fromfunction(lambda i, j, k: 100 * i + 10 * j + k, (n, n, n))
    got = oracle.spinsum_chain(enc, workloads.FACTORED_PIJ_PJK, 0, 3)
    want = np.fromfunction(lambda i, j, k: 181 * i - 62 * j - 8 * k, (n, n, n))
    np.testing.assert_array_equal(got, want)
    rev = oracle.spinsum_chain(enc, workloads.FACTORED_PIJ_PJK[::-1], 0, 3)
    np.testing.assert_array_equal(
        rev, np.fromfunction(lambda i, j, k: 190 * i - 161 * j + 82 * k, (n, n, n)))


# ------------------------------------------------------------- library route
@pytest.mark.parametrize("shape,gf,d", [((3, 4, 4, 4), 1, 3), ((4, 4, 4, 2), 0, 3),
                                        ((2, 3, 3, 3, 3), 1, 4), ((2, 5, 5, 3), 1, 2),
                                        ((2, 3, 3, 3, 3, 2), 1, 4)])
def test_oracle_matches_numpy_transpose(shape, gf, d):
    rng = np.random.default_rng(len(shape) * 10 + d)
    perms = list(itertools.permutations(range(d)))
    terms = [(p, float(rng.normal())) for p in perms]
    x = _rand(shape, 31)
    np.testing.assert_allclose(oracle.spinsum(x, terms, gf, d),
                               oracle.spinsum_numpy(x, terms, gf, d), rtol=0, atol=1e-13)


# ---------------------------------------------------------- explicit matrix
@pytest.mark.parametrize("shape,gf,d", [((2, 3, 3, 3), 1, 3), ((1, 2, 2, 2, 2), 1, 4),
                                        ((3, 3, 3, 3), 0, 4), ((2, 1, 1, 1), 1, 3),
                                        ((5, 5, 5), 0, 3), ((2, 3, 3, 2), 1, 2)])
def test_dense_matrix_forward_and_adjoint(shape, gf, d):
    rng = np.random.default_rng(7)
    perms = list(itertools.permutations(range(d)))
    stages = [[(perms[k], float(rng.normal())) for k in rng.choice(len(perms), min(3, len(perms)), replace=False)]
              for _ in range(2)]
    M = oracle.dense_chain_matrix(shape, stages, gf, d)
    x = _rand(shape, 41)
    g = _rand(shape, 42)
    np.testing.assert_allclose(oracle.spinsum_chain(x, stages, gf, d).ravel(), M @ x.ravel(),
                               rtol=0, atol=1e-13)
    np.testing.assert_allclose(oracle.spinsum_chain_adjoint(g, stages, gf, d).ravel(),
                               M.T @ g.ravel(), rtol=0, atol=1e-13)


def test_adjoint_identity():
    """<S x, y> = <x, S^T y> for a 4D chain with spectators on both sides."""
    d, stages = workloads.table2_case(6)
    x = _rand((2, 4, 4, 4, 4, 3), 51)
    y = _rand((2, 4, 4, 4, 4, 3), 52)
    lhs = np.sum(oracle.spinsum_chain(x, stages, 1, 4) * y)
    rhs = np.sum(x * oracle.spinsum_chain_adjoint(y, stages, 1, 4))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


# ------------------------------------------------------------ closed forms
def _symmetrise(x, gf, d, signed):
    out = np.zeros_like(x)
    for q in itertools.permutations(range(d)):
        axes = list(range(gf)) + [gf + v for v in q] + list(range(gf + d, x.ndim))
        out += (_sign(q) if signed else 1) * np.transpose(x, axes)
    return out


@pytest.mark.parametrize("d", [2, 3, 4])
def test_symmetric_and_antisymmetric_inputs(d):
    """On a fully symmetric input every pi acts as the identity: B = (sum a) A.
    On a fully antisymmetric input pi acts as sgn(pi): B = (sum a sgn) A."""
    rng = np.random.default_rng(d + 100)
    perms = list(itertools.permutations(range(d)))
    terms = [(p, float(rng.integers(-3, 4))) for p in perms]
    x = _rand((2,) + (4,) * d, 61)
    ys = _symmetrise(x, 1, d, signed=False)
    ya = _symmetrise(x, 1, d, signed=True)
    sa = sum(a for _, a in terms)
    ssg = sum(a * _sign(p) for p, a in terms)
    np.testing.assert_allclose(oracle.spinsum(ys, terms, 1, d), sa * ys, rtol=0, atol=1e-11)
    np.testing.assert_allclose(oracle.spinsum(ya, terms, 1, d), ssg * ya, rtol=0, atol=1e-11)


def test_3d_coefficient_set_spectrum():
    """The 3D coefficient set is a class function with eigenvalue 0 on the
    trivial, 3 on the standard and 12 on the sign representation of S_3,
    so S^3 - 15 S^2 + 36 S = 0; on symmetric input S = 0 and on
    antisymmetric input S = 12."""
    x = _rand((3, 5, 5, 5), 71)
    a = workloads.CONFIG_3D_ALPHA
    s1 = oracle.spinsum(x, a, 1, 3)
    s2 = oracle.spinsum(s1, a, 1, 3)
    s3 = oracle.spinsum(s2, a, 1, 3)
    res = s3 - 15 * s2 + 36 * s1
    assert np.max(np.abs(res)) <= 1e-12 * np.max(np.abs(s3))
    ys = _symmetrise(x, 1, 3, signed=False)
    assert np.max(np.abs(oracle.spinsum(ys, a, 1, 3))) < 1e-12
    ya = _symmetrise(x, 1, 3, signed=True)
    np.testing.assert_allclose(oracle.spinsum(ya, a, 1, 3), 12 * ya, rtol=0, atol=1e-11)


def test_class_function_commutes_with_permutation():
    """Class-function coefficients: S(pi_t A) = pi_t S(A)."""
    x = _rand((2, 5, 5, 5), 81)
    a = workloads.CONFIG_3D_ALPHA
    for t in (P("231"), P("213")):
        lhs = oracle.spinsum(oracle.spinsum(x, [(t, 1.0)], 1, 3), a, 1, 3)
        rhs = oracle.spinsum(oracle.spinsum(x, a, 1, 3), [(t, 1.0)], 1, 3)
        np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-12)


def test_linearity_and_sum_invariant():
    d, stages = workloads.table2_case(5)
    x = _rand((2, 4, 4, 4, 4), 91)
    y = _rand((2, 4, 4, 4, 4), 92)
    lin = oracle.spinsum_chain(2.5 * x - 0.5 * y, stages, 1, 4)
    np.testing.assert_allclose(lin, 2.5 * oracle.spinsum_chain(x, stages, 1, 4)
                               - 0.5 * oracle.spinsum_chain(y, stages, 1, 4), rtol=0, atol=1e-11)
    # sum of all outputs = (product of the stage coefficient sums) * sum of inputs
    fac = np.prod([sum(a for _, a in st) for st in stages])
    out = oracle.spinsum_chain(x, stages, 1, 4)
    assert abs(out.sum() - fac * x.sum()) < 1e-10 * max(1.0, abs(x).sum())


# ------------------------------------------------------------- edge cases
def test_group_extent_one():
    """N = 1: every permutation reads the same element, B = (sum a) A."""
    x = _rand((7, 1, 1, 1, 3), 101)
    out = oracle.spinsum(x, [(P("123"), 2.0), (P("231"), -0.5), (P("321"), 4.0)], 1, 3)
    np.testing.assert_allclose(out, 5.5 * x, rtol=0, atol=0)


@pytest.mark.parametrize("shape", [(0, 3, 3, 3), (2, 0, 0, 0), (2, 3, 3, 3, 0)])
def test_empty(shape):
    x = np.zeros(shape)
    out = oracle.spinsum(x, workloads.CONFIG_3D_ALPHA, 1, 3)
    assert out.shape == x.shape


def test_fig2_2d_example():
    """Fig. 2: B <- (a1 pi_12 + a2 pi_21)(A) = a1 A + a2 A^T."""
    x = _rand((9, 9), 111)
    out = oracle.spinsum(x, [(P("12"), 0.25), (P("21"), -3.0)], 0, 2)
    np.testing.assert_allclose(out, 0.25 * x - 3.0 * x.T, rtol=0, atol=1e-15)


def test_zero_coefficient_terms_are_skipped():
    x = _rand((3, 3, 3), 121)
    x[1, 2, 0] = np.inf
    out = oracle.spinsum(x, [(P("123"), 1.0), (P("312"), 0.0)], 0, 3)
    assert np.isinf(out[1, 2, 0])
    assert np.isfinite(out).sum() == 26


def test_inplace_semantics_equal_out_of_place():
    """The oracle accepts aliased in/out and gives the out-of-place result."""
    lib = oracle._load()
    import ctypes
    x = _rand((2, 4, 4, 4), 131)
    want = oracle.spinsum(x, workloads.CONFIG_3D_ALPHA, 1, 3)
    buf = x.copy()
    nterms, perms, alpha = oracle._flatten([workloads.CONFIG_3D_ALPHA], 3)
    dp = ctypes.POINTER(ctypes.c_double)
    st = lib.oracle_spinsum_chain(4, (ctypes.c_int64 * 4)(*buf.shape), 1, 3, 1,
                                  (ctypes.c_int * 1)(*nterms), (ctypes.c_int * len(perms))(*perms),
                                  (ctypes.c_double * len(alpha))(*alpha),
                                  buf.ctypes.data_as(dp), buf.ctypes.data_as(dp), 1)
    assert st == 0
    np.testing.assert_array_equal(buf, want)


def test_threads_do_not_change_results():
    x = _rand((8, 5, 5, 5, 5), 141)
    a = workloads.random_4d_alpha(1)
    np.testing.assert_array_equal(oracle.spinsum(x, a, 1, 4, nthreads=1),
                                  oracle.spinsum(x, a, 1, 4, nthreads=4))


def test_invalid_arguments_are_rejected():
    x = _rand((3, 3, 3), 1)
    with pytest.raises(ValueError):
        oracle.spinsum(x, [((0, 0, 1), 1.0)], 0, 3)          # not a bijection
    with pytest.raises(ValueError):
        oracle.spinsum(_rand((3, 3, 4), 1), [((0, 1, 2), 1.0)], 0, 3)  # not hyper-square


# ------------------------------------------------------------ generators
def test_generator_torch_matches_numpy_and_range():
    a = workloads.uniform((4096,), 5, offset=123).numpy()
    b = workloads.uniform_numpy(4096, 5, offset=123)
    np.testing.assert_array_equal(a, b)
    assert a.min() >= -1.0 and a.max() < 1.0 and abs(a.mean()) < 0.05
    c = workloads.uniform((4096,), 6, offset=123).numpy()
    assert not np.array_equal(a, c)
    ints = workloads.integers((4096,), 5).numpy()
    assert np.all(ints == np.round(ints)) and ints.min() >= -1024 and ints.max() <= 1024


def test_batched_block_list():
    seed, blocks = workloads.batched_blocks()
    assert len(blocks) == 200
    total = sum(8 * v ** 3 * o ** 3 for v, o in blocks)
    assert 1.9e9 <= total <= 2.1e9
    assert all(4 <= v <= 40 and 2 <= o <= 16 for v, o in blocks)
    assert workloads.batched_blocks() == (seed, blocks)


@pytest.mark.parametrize("d", [2, 3, 4])
def test_symmetrizer_sets(d):
    """The (anti)symmetrisers of the workloads: outputs are (anti)symmetric
    under every transposition and the operators are d! times idempotent."""
    x = _rand((2,) + (3,) * d, 90 + d)
    fact = math.factorial(d)
    for stage, sign in [(workloads.symmetrizer(d), 1.0), (workloads.antisymmetrizer(d), -1.0)]:
        y = oracle.spinsum(x, stage, 1, d)
        for a, b in itertools.combinations(range(d), 2):
            axes = list(range(d + 1))
            axes[1 + a], axes[1 + b] = axes[1 + b], axes[1 + a]
            np.testing.assert_allclose(np.transpose(y, axes), sign * y, rtol=0, atol=1e-12)
        np.testing.assert_allclose(oracle.spinsum(y, stage, 1, d), fact * y, rtol=0, atol=1e-10)
    # the antisymmetriser annihilates symmetric inputs and vice versa
    ys = oracle.spinsum(x, workloads.symmetrizer(d), 1, d)
    np.testing.assert_allclose(oracle.spinsum(ys, workloads.antisymmetrizer(d), 1, d), 0, atol=1e-10)


@pytest.mark.parametrize("shape,gf,d", [((2, 3, 3, 3), 1, 3), ((1, 2, 2, 2, 2), 1, 4), ((3, 4, 4), 1, 2)])
def test_coef_grad_definition(shape, gf, d):
    """<g, pi_p(x)> equals g^T M_p x with the dense matrix of the single term
    p, and the derivative of the linear map L(alpha) = <g, S_alpha(x)>:
    L(alpha + e_p) - L(alpha) = grad_p exactly (up to rounding)."""
    x = _rand(shape, 17)
    g = _rand(shape, 18)
    grad = oracle.coef_grad(x, g, gf, d)
    perms = list(itertools.permutations(range(d)))
    assert grad.shape == (len(perms),)
    rng = np.random.default_rng(3)
    alpha = rng.integers(-3, 4, len(perms)).astype(float)
    def L(al):
        return float(np.sum(g * oracle.spinsum(x, list(zip(perms, al)), gf, d)))
    for r, p in enumerate(perms):
        M = oracle.dense_matrix(shape, [(p, 1.0)], gf, d)
        assert abs(grad[r] - g.ravel() @ (M @ x.ravel())) <= 1e-12 * max(1.0, abs(grad[r]))
        e = np.zeros(len(perms))
        e[r] = 1.0
        assert abs((L(alpha + e) - L(alpha)) - grad[r]) <= 1e-10


# ------------------------------------------------------- index-pair form
def _interleave(x, first, d):
    """[.., a_0..a_{d-1}, i_0..i_{d-1}, ..] -> [.., (a_0 i_0), .., (a_{d-1} i_{d-1}), ..]:
    each pair (a_m, i_m) becomes one index a_m * N + i_m of extent V * N."""
    nd = x.ndim
    axes = list(range(first))
    for m in range(d):
        axes += [first + m, first + d + m]
    axes += list(range(first + 2 * d, nd))
    y = np.transpose(x, axes)
    V, N = x.shape[first], x.shape[first + d]
    return np.ascontiguousarray(y).reshape(x.shape[:first] + (V * N,) * d + x.shape[first + 2 * d:])


def _deinterleave(y, first, d, V, N):
    shp = y.shape[:first] + tuple(v for _ in range(d) for v in (V, N)) + y.shape[first + d:]
    z = y.reshape(shp)
    nd = z.ndim
    axes = list(range(first)) + [first + 2 * m for m in range(d)] + \
        [first + 2 * m + 1 for m in range(d)] + list(range(first + 2 * d, nd))
    return np.ascontiguousarray(np.transpose(z, axes))


@pytest.mark.parametrize("shape,gf,d", [((3, 3, 2, 2), 2, 2), ((2, 3, 3, 3, 2, 2, 2), 4, 3),
                                        ((2, 2, 2, 2, 2, 2, 2, 2), 4, 4),
                                        ((2, 4, 4, 2, 2, 3), 3, 2), ((1, 3, 3, 3, 3, 3, 3, 2), 4, 3)])
def test_pairs_match_numpy_transpose_and_interleaved_group(shape, gf, d):
    """Index-pair form: (i) the same as the numpy transpose of both index
    sets; (ii) conjugate to the ordinary summation over the combined indices
    c_m = a_m * N + i_m (the pairs (a_m, i_m) permuted together are exactly
    the permuted tuple of combined indices), which pins it to the already
    pinned group form; bitwise, since both evaluate the same terms in the same
    order."""
    rng = np.random.default_rng(sum(shape))
    terms = [(p, float(rng.normal())) for p in itertools.permutations(range(d))]
    x = _rand(shape, 71)
    got = oracle.spinsum(x, terms, gf, d, pairs=True)
    np.testing.assert_allclose(got, oracle.spinsum_numpy(x, terms, gf, d, pairs=True),
                               rtol=0, atol=1e-13)
    first = gf - d
    V, N = shape[first], shape[gf]
    comb = oracle.spinsum(_interleave(x, first, d), terms, first, d)
    np.testing.assert_array_equal(_deinterleave(comb, first, d, V, N), got)
    adj = oracle.spinsum_chain_adjoint(x, [terms], gf, d, pairs=True)
    comb_adj = oracle.spinsum_chain_adjoint(_interleave(x, first, d), [terms], first, d)
    np.testing.assert_array_equal(_deinterleave(comb_adj, first, d, V, N), adj)


@pytest.mark.parametrize("shape,gf,d", [((2, 2, 3, 3), 2, 2), ((2, 2, 2, 2, 2, 2), 3, 3),
                                        ((2, 3, 3, 2, 2, 2), 3, 2)])
def test_pairs_dense_matrix_forward_and_adjoint(shape, gf, d):
    rng = np.random.default_rng(5)
    perms = list(itertools.permutations(range(d)))
    stages = [[(perms[k], float(rng.normal())) for k in rng.choice(len(perms), min(3, len(perms)), replace=False)]
              for _ in range(2)]
    M = oracle.dense_chain_matrix(shape, stages, gf, d, pairs=True)
    x = _rand(shape, 72)
    g = _rand(shape, 73)
    np.testing.assert_allclose(oracle.spinsum_chain(x, stages, gf, d, pairs=True).ravel(),
                               M @ x.ravel(), rtol=0, atol=1e-13)
    np.testing.assert_allclose(oracle.spinsum_chain_adjoint(g, stages, gf, d, pairs=True).ravel(),
                               M.T @ g.ravel(), rtol=0, atol=1e-13)


def test_pairs_worked_example_and_special_cases():
    """A[a,b,i,j] = 1000a + 100b + 10i + j under the swap (21) gives
    B[a,b,i,j] = 1000b + 100a + 10j + i.  With V = 1 the form is the
    ordinary summation; with N = 1 it is the ordinary summation over the
    partner dims."""
    V, N = 3, 4
    enc = np.fromfunction(lambda a, b, i, j: 1000 * a + 100 * b + 10 * i + j, (V, V, N, N))
    got = oracle.spinsum(enc, [(P("21"), 1.0)], 2, 2, pairs=True)
    want = np.fromfunction(lambda a, b, i, j: 1000 * b + 100 * a + 10 * j + i, (V, V, N, N))
    np.testing.assert_array_equal(got, want)
    terms = [(p, float(k + 1)) for k, p in enumerate(itertools.permutations(range(3)))]
    x = _rand((2, 1, 1, 1, 4, 4, 4), 74)
    np.testing.assert_array_equal(oracle.spinsum(x, terms, 4, 3, pairs=True),
                                  oracle.spinsum(x, terms, 4, 3))
    x = _rand((2, 4, 4, 4, 1, 1, 1, 3), 75)
    np.testing.assert_array_equal(oracle.spinsum(x, terms, 4, 3, pairs=True),
                                  oracle.spinsum(x, terms, 1, 3))
