"""Independent brute force for tiny search spaces (test helper).

Builds candidate expressions as nested tuples by depth, with no notion of
IDs or ordering, evaluates them with numpy and scores them with
numpy.corrcoef.  Shares nothing with the oracle or the GPU library."""
import itertools

import numpy as np

UN = ("exp", "log", "sqrt", "sq", "inv")
BIN = ("add", "sub", "mul", "div", "rdiv")


def trees_by_depth(p, R, ops):
    """Lists of expression trees of depth exactly 0..R.  A binary node joins
    two distinct trees of which at least one has depth r-1; subtraction is
    taken in one orientation and division in both (div and rdiv)."""
    lv = [[("x", i) for i in range(p)]]
    for r in range(1, R + 1):
        prev = lv[r - 1]
        prev_set = set(prev)
        below = [t for d in range(r) for t in lv[d]]
        new = [(u, a) for u in UN if u in ops for a in prev]
        pairs = []
        for a, b in itertools.combinations(below, 2):
            if a in prev_set or b in prev_set:
                pairs.append((a, b))
        for o in BIN:
            if o in ops:
                new += [(o, a, b) for a, b in pairs]
        lv.append(new)
    return lv


def canon(t):
    """Canonical string: commutative operands sorted, subtraction
    orientation-free (|r| does not see the sign), rdiv written as div."""
    if t[0] == "x":
        return "x%d" % t[1]
    if len(t) == 2:
        return "%s(%s)" % (t[0], canon(t[1]))
    a, b = canon(t[1]), canon(t[2])
    if t[0] in ("add", "mul"):
        a, b = sorted((a, b))
        return "%s(%s,%s)" % (t[0], a, b)
    if t[0] == "sub":
        a, b = sorted((a, b))
        return "sub{%s,%s}" % (a, b)
    if t[0] == "div":
        return "div(%s,%s)" % (a, b)
    return "div(%s,%s)" % (b, a)          # rdiv(a, b) = b / a


def evaluate(t, X):
    with np.errstate(all="ignore"):
        if t[0] == "x":
            return X[t[1]].astype(np.float64)
        if len(t) == 2:
            a = evaluate(t[1], X)
            return {"exp": np.exp, "log": np.log, "sqrt": np.sqrt,
                    "sq": lambda v: v * v, "inv": lambda v: 1.0 / v}[t[0]](a)
        a, b = evaluate(t[1], X), evaluate(t[2], X)
        return {"add": a + b, "sub": a - b, "mul": a * b, "div": a / b,
                "rdiv": b / a}[t[0]]


def oracle_tree(space, cid):
    """Tree of an oracle ID via its decoder (for canonical comparison)."""
    from oracle.oracle import OPS, OP_NONE
    r, op, a, b = space.decode(cid)
    if op == OP_NONE:
        return ("x", cid)
    if b < 0:
        return (OPS[op], oracle_tree(space, a))
    return (OPS[op], oracle_tree(space, a), oracle_tree(space, b))
