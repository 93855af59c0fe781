"""The contraction-path cost model (section "Tensor Contraction Path
Optimization") against the paper's worked example, its printed paths of the
expression examples, brute force over every pairwise order, and numpy's
einsum for the values along a path (CPU only)."""
import itertools
import random

import numpy as np
import pytest

from paper_2107_04121_amd.contraction import (naive_flops, optimal_path, parse, path_flops,
                                              step_flops)


def test_paper_worked_example():
    # 'ij,jk,kl->il', A 2x2, B 2x5, C 5x2: naive 120, optimized 56, speed-up
    # 2.143, largest intermediate 4, scalings 4 and 3; B and C first
    sizes = dict(i=2, j=2, k=5, l=2)
    p = optimal_path("ij,jk,kl->il", sizes)
    assert p.naive == 120 and p.flops == 56
    assert round(p.speedup, 3) == 2.143
    assert p.largest_intermediate == 4
    assert p.naive_scaling == 4 and p.scaling == 3
    assert p.steps[0][:2] == ("jk", "kl")
    # the other order (A and B first) costs 80
    assert path_flops("ij,jk,kl->il", sizes, [(0, 1), (0, 1)]).flops == 80


PRINTED = [
    # (expression, sizes, path printed in the paper's expression examples)
    ("cq,cqjd,cqje->cde", {"c": 1024, "q": 27, "j": 3, "d": 27, "e": 27}, [(0, 1), (0, 1)]),
    ("cq,qd,ir,qe,is->crdse", {"c": 1024, "q": 8, "d": 8, "i": 3, "r": 3, "e": 8, "s": 3},
     [(2, 4), (0, 1), (0, 2), (0, 1)]),
    ("cq,qd,ir,qe,cie->crd", {"c": 1024, "q": 8, "d": 8, "i": 3, "r": 3, "e": 8},
     [(3, 4), (0, 3), (0, 2), (0, 1)]),
    ("cq,cqje,rjI,cqIK,cqlf,slK->cresf",
     {"c": 1024, "q": 8, "j": 3, "e": 8, "r": 3, "I": 6, "K": 6, "l": 3, "f": 8, "s": 3},
     [(0, 4), (2, 3), (1, 3), (1, 2), (0, 1)]),
]


@pytest.mark.parametrize("expr,sizes,printed", PRINTED)
def test_printed_paths(expr, sizes, printed):
    opt = optimal_path(expr, sizes)
    given = path_flops(expr, sizes, printed)
    assert opt.flops <= given.flops < opt.naive
    if expr.startswith("cq,cqje"):
        # the paper's dynamic-programming path for elasticity is optimal
        assert given.flops == opt.flops


def _all_orders(n):
    """Every sequence of pairwise contractions of n operands (list
    convention: remove the pair, append the product)."""
    if n == 1:
        yield []
        return
    for i, j in itertools.combinations(range(n), 2):
        for rest in _all_orders(n - 1):
            yield [(i, j)] + rest


def _random_expr(rng, n_ops):
    letters = "abcdefg"
    terms = []
    for _ in range(n_ops):
        k = rng.randint(1, 3)
        terms.append("".join(rng.sample(letters, k)))
    used = sorted(set("".join(terms)))
    out = "".join(ch for ch in used if rng.random() < 0.3)
    sizes = {ch: rng.randint(2, 5) for ch in used}
    return ",".join(terms) + "->" + out, sizes


@pytest.mark.parametrize("seed", range(12))
def test_optimal_path_is_brute_force_minimum(seed):
    rng = random.Random(seed)
    expr, sizes = _random_expr(rng, rng.randint(2, 5))
    n = len(parse(expr)[0])
    brute = min(path_flops(expr, sizes, p).flops for p in _all_orders(n))
    assert optimal_path(expr, sizes).flops == brute


@pytest.mark.parametrize("seed", range(8))
def test_path_evaluates_to_the_einsum(seed):
    rng = random.Random(100 + seed)
    expr, sizes = _random_expr(rng, rng.randint(2, 5))
    inputs, out = parse(expr)
    nrng = np.random.default_rng(seed)
    arrays = [nrng.standard_normal([sizes[ch] for ch in t]) for t in inputs]
    info = optimal_path(expr, sizes)
    ops = list(zip(inputs, arrays))
    for (i, j), (a, b, r, _) in zip(info.path, info.steps):
        (ta, xa), (tb, xb) = ops[i], ops[j]
        assert {ta, tb} == {a, b}
        ops = [o for k, o in enumerate(ops) if k not in (i, j)] + [(r, np.einsum(f"{ta},{tb}->{r}", xa, xb))]
    (t, x), = ops
    ref = np.einsum(expr, *arrays)
    np.testing.assert_allclose(np.einsum(f"{t}->{out}", x), ref, rtol=1e-12, atol=1e-12)


def test_step_and_naive_counts():
    s = dict(i=3, j=4)
    assert step_flops(["ij", "j"], "i", s) == 12 * 2      # one multiply, one add per point
    assert step_flops(["ij", "ij"], "ij", s) == 12        # multiply only
    assert naive_flops("ij,jk,kl->il", dict(i=2, j=2, k=5, l=2)) == 120
    with pytest.raises(ValueError):
        parse("ij,jk->iz")
