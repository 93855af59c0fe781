"""Contraction paths of einsum expressions and their flop cost.

The paper (section "Tensor Contraction Path Optimization") compares the
naive evaluation of a multi-operand einsum -- one loop per index, all
operands multiplied at every point of the loop nest -- with an ordered
sequence of pairwise contractions, the contraction path, and gives the
chained product 'ij,jk,kl->il' with A 2x2, B 2x5, C 5x2 as the worked
example: 120 flops naively, 56 along the best path, a speed-up of 2.143, the
largest intermediate 4 elements.

Cost model used here (it reproduces those numbers): a step that multiplies m
operands over the union of their indices runs one loop point per element of
that index space and does m - 1 multiplications per point, plus one addition
per point when the step sums over at least one index.  The naive evaluation
is a single step over all operands.  A path is a list of index pairs into the
current operand list; the two operands are removed and their product is
appended at the end (the convention of the path printouts in the paper's
expression examples).

`optimal_path` searches all pairwise orders by dynamic programming over
subsets of operands (exact for the few operands of a weak form); the
autotuner and the front-end rank kernel variants with these costs.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from itertools import combinations

__all__ = ["parse", "step_flops", "naive_flops", "path_flops", "optimal_path", "PathInfo"]


def parse(expr: str):
    """'ab,bc->ac' -> (['ab', 'bc'], 'ac').  Without '->' the output is the
    letters that appear exactly once, sorted (the implicit einsum rule)."""
    expr = expr.replace(" ", "")
    if "->" in expr:
        lhs, out = expr.split("->")
    else:
        lhs = expr
        letters = lhs.replace(",", "")
        out = "".join(sorted(ch for ch in set(letters) if letters.count(ch) == 1))
    inputs = lhs.split(",")
    for t in inputs + [out]:
        if not all(ch.isalpha() for ch in t):
            raise ValueError(f"bad einsum term {t!r}")
    if len(set(out)) != len(out):
        raise ValueError("repeated output index")
    missing = set(out) - set("".join(inputs))
    if missing:
        raise ValueError(f"output indices {sorted(missing)} appear in no input")
    return inputs, out


def _space(indices, sizes):
    n = 1
    for ch in indices:
        n *= sizes[ch]
    return n


def step_flops(terms, keep, sizes) -> int:
    """Flops of multiplying `terms` (index strings) into the indices `keep`:
    (number of terms - 1) multiplications per loop point, plus one addition
    per point if an index is summed away."""
    loop = set("".join(terms))
    summed = bool(loop - set(keep))
    per_point = max(1, len(terms) - 1) + (1 if summed else 0)
    if len(terms) == 1 and not summed:
        per_point = 0  # a plain copy or transpose
    return _space(loop, sizes) * per_point


def naive_flops(expr: str, sizes: dict) -> int:
    inputs, out = parse(expr)
    return step_flops(inputs, out, sizes)


@dataclass
class PathInfo:
    """A contraction path with its cost breakdown."""
    expr: str
    path: list
    steps: list = field(default_factory=list)  # (term a, term b, result, flops)
    flops: int = 0
    naive: int = 0
    largest_intermediate: int = 0
    naive_scaling: int = 0
    scaling: int = 0

    @property
    def speedup(self) -> float:
        return self.naive / self.flops if self.flops else float("inf")

    def __str__(self):
        lines = [f"  Complete contraction:  {self.expr}",
                 f"         Naive scaling:  {self.naive_scaling}",
                 f"     Optimized scaling:  {self.scaling}",
                 f"      Naive FLOP count:  {self.naive:.3e}",
                 f"  Optimized FLOP count:  {self.flops:.3e}",
                 f"   Theoretical speedup:  {self.speedup:.3e}",
                 f"  Largest intermediate:  {self.largest_intermediate:.3e} elements"]
        for a, b, r, f in self.steps:
            lines.append(f"    {a},{b}->{r}  {f} flops")
        return "\n".join(lines)


def _result_indices(a, b, others, out):
    """Indices of the product of a and b that are still needed: those in the
    output or in any operand not yet contracted, in order of appearance."""
    need = set(out)
    for t in others:
        need |= set(t)
    seen = []
    for ch in a + b:
        if ch in need and ch not in seen:
            seen.append(ch)
    return "".join(seen)


def path_flops(expr: str, sizes: dict, path) -> PathInfo:
    """Cost of a given pairwise path (list of (i, j) positions in the
    current operand list; the pair is removed, the product appended)."""
    inputs, out = parse(expr)
    ops = list(inputs)
    info = PathInfo(expr=expr, path=[tuple(p) for p in path], naive=naive_flops(expr, sizes),
                    naive_scaling=len(set("".join(inputs))))
    for pair in path:
        i, j = sorted(pair)
        if i == j or j >= len(ops):
            raise ValueError(f"bad path step {pair} for {len(ops)} operands")
        a, b = ops[i], ops[j]
        rest = [t for k, t in enumerate(ops) if k not in (i, j)]
        last = not rest
        r = out if last else _result_indices(a, b, rest, out)
        f = step_flops([a, b], r, sizes)
        info.steps.append((a, b, r, f))
        info.flops += f
        info.scaling = max(info.scaling, len(set(a + b)))
        if not last:
            info.largest_intermediate = max(info.largest_intermediate, _space(r, sizes))
        ops = rest + [r]
    if len(ops) != 1:
        raise ValueError("the path leaves more than one operand")
    if ops[0] != out:  # a final transpose costs nothing in this model
        if sorted(ops[0]) != sorted(out):
            raise ValueError("the path does not produce the output indices")
    return info


def optimal_path(expr: str, sizes: dict, max_operands: int = 12) -> PathInfo:
    """Cheapest pairwise path under the cost model, by dynamic programming
    over subsets of operands: best[S] = the cheapest way to reduce the
    operands in S to one intermediate (whose indices are those of S still
    needed outside S or in the output)."""
    inputs, out = parse(expr)
    n = len(inputs)
    if n > max_operands:
        raise ValueError(f"{n} operands: too many for the exhaustive search")
    if n == 1:
        info = PathInfo(expr=expr, path=[], naive=naive_flops(expr, sizes),
                        naive_scaling=len(set(inputs[0])), scaling=len(set(inputs[0])))
        info.flops = step_flops(inputs, out, sizes)
        info.steps = [(inputs[0], "", out, info.flops)]
        return info
    full = (1 << n) - 1

    def indices_of(mask):
        inside = [inputs[k] for k in range(n) if mask >> k & 1]
        outside = [inputs[k] for k in range(n) if not mask >> k & 1]
        if mask == full:
            return out
        need = set(out)
        for t in outside:
            need |= set(t)
        seen = []
        for t in inside:
            for ch in t:
                if ch in need and ch not in seen:
                    seen.append(ch)
        return "".join(seen)

    idx = {1 << k: inputs[k] for k in range(n)}
    best = {1 << k: (0, None) for k in range(n)}  # mask -> (flops, (maskA, maskB))
    for size in range(2, n + 1):
        for members in combinations(range(n), size):
            mask = 0
            for k in members:
                mask |= 1 << k
            res = indices_of(mask)
            idx[mask] = res
            cand = None
            # split mask into two non-empty parts; the part holding the lowest
            # member is A, so each split is visited once
            low = mask & -mask
            sub = (mask - 1) & mask
            while sub:
                if sub & low:
                    other = mask ^ sub
                    if other:
                        c = best[sub][0] + best[other][0] + step_flops([idx[sub], idx[other]], res, sizes)
                        if cand is None or c < cand[0]:
                            cand = (c, (sub, other))
                sub = (sub - 1) & mask
            best[mask] = cand
    # turn the split tree into a sequential path over the list convention
    order = []

    def walk(mask):
        split = best[mask][1]
        if split is None:
            return
        a, b = split
        walk(a)
        walk(b)
        order.append((a, b))

    walk(full)
    live = [1 << k for k in range(n)]
    path = []
    for a, b in order:
        i, j = live.index(a), live.index(b)
        path.append((min(i, j), max(i, j)))
        live = [m for m in live if m not in (a, b)] + [a | b]
    info = path_flops(expr, sizes, path)
    assert info.flops == best[full][0]
    return info
