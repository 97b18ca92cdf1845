"""Physical units as integer exponent vectors (Physics-Informed Constraints:
dimensional consistency through unit-aware operations).

A unit string is parsed into exponents over the seven SI base units
(m, kg, s, A, K, mol, cd).  Only dimensions matter for the method, so
prefixes and scale factors are accepted and dropped ("km" is a length like
"m").  Grammar (whitespace or '*' multiply, '/' divides the next factor or
parenthesised group, '^' or '**' raises to an integer power):

    unit   := term (('*' | '/' | ' ') term)*
    term   := atom (('^' | '**') int)?
    atom   := symbol | '(' unit ')' | '1'

"", "1", "dimensionless" and "-" are dimensionless.  The exponents of a
set of features are then restricted to the base units any of them uses,
which gives the library's [p][B] exponent matrix (B <= 8).
"""
import re

import numpy as np

BASE = ("m", "kg", "s", "A", "K", "mol", "cd")

# symbol -> exponents over BASE
_D = {
    "m": (1, 0, 0, 0, 0, 0, 0), "g": (0, 1, 0, 0, 0, 0, 0), "s": (0, 0, 1, 0, 0, 0, 0),
    "A": (0, 0, 0, 1, 0, 0, 0), "K": (0, 0, 0, 0, 1, 0, 0), "mol": (0, 0, 0, 0, 0, 1, 0),
    "cd": (0, 0, 0, 0, 0, 0, 1),
    "N": (1, 1, -2, 0, 0, 0, 0), "J": (2, 1, -2, 0, 0, 0, 0), "W": (2, 1, -3, 0, 0, 0, 0),
    "Pa": (-1, 1, -2, 0, 0, 0, 0), "Hz": (0, 0, -1, 0, 0, 0, 0), "C": (0, 0, 1, 1, 0, 0, 0),
    "V": (2, 1, -3, -1, 0, 0, 0), "ohm": (2, 1, -3, -2, 0, 0, 0), "Ohm": (2, 1, -3, -2, 0, 0, 0),
    "F": (-2, -1, 4, 2, 0, 0, 0), "T": (0, 1, -2, -1, 0, 0, 0), "Wb": (2, 1, -2, -1, 0, 0, 0),
    "H": (2, 1, -2, -2, 0, 0, 0), "S": (-2, -1, 3, 2, 0, 0, 0), "L": (3, 0, 0, 0, 0, 0, 0),
    "eV": (2, 1, -2, 0, 0, 0, 0), "Da": (0, 1, 0, 0, 0, 0, 0), "u": (0, 1, 0, 0, 0, 0, 0),
    "bar": (-1, 1, -2, 0, 0, 0, 0), "atm": (-1, 1, -2, 0, 0, 0, 0), "cal": (2, 1, -2, 0, 0, 0, 0),
    "min": (0, 0, 1, 0, 0, 0, 0), "h": (0, 0, 1, 0, 0, 0, 0), "Angstrom": (1, 0, 0, 0, 0, 0, 0),
    "angstrom": (1, 0, 0, 0, 0, 0, 0), "rad": (0, 0, 0, 0, 0, 0, 0),
    "sr": (0, 0, 0, 0, 0, 0, 0), "percent": (0, 0, 0, 0, 0, 0, 0), "Hartree": (2, 1, -2, 0, 0, 0, 0),
    "Ry": (2, 1, -2, 0, 0, 0, 0), "bohr": (1, 0, 0, 0, 0, 0, 0),
}
_PREFIX = ("Y", "Z", "E", "P", "T", "G", "M", "k", "h", "da", "d", "c", "m", "u", "µ", "μ", "n", "p",
           "f", "a", "z", "y")
_DIMLESS = {"", "1", "dimensionless", "-", "none"}


class UnitError(ValueError):
    pass


def _symbol(sym):
    if sym in _D:
        return np.array(_D[sym], np.int64)
    for pre in sorted(_PREFIX, key=len, reverse=True):     # longest prefix first ("da")
        if sym.startswith(pre) and sym[len(pre):] in _D and len(sym) > len(pre):
            return np.array(_D[sym[len(pre):]], np.int64)
    raise UnitError("unknown unit symbol %r" % sym)


_TOK = re.compile(r"\s*(\*\*|\^|\*|/|\(|\)|[-+]?\d+|[A-Za-zµμ_]+)")


def _tokens(s):
    out, pos = [], 0
    s = s.strip()
    while pos < len(s):
        m = _TOK.match(s, pos)
        if not m:
            raise UnitError("cannot parse unit %r at %r" % (s, s[pos:]))
        out.append(m.group(1))
        pos = m.end()
    return out


def parse_unit(text):
    """Exponent vector (over BASE) of a unit string."""
    if text is None or str(text).strip().lower() in _DIMLESS:
        return np.zeros(len(BASE), np.int64)
    toks = _tokens(str(text))
    pos = 0

    def atom():
        nonlocal pos
        if pos >= len(toks):
            raise UnitError("unit %r ends early" % text)
        t = toks[pos]
        if t == "(":
            pos += 1
            v = unit()
            if pos >= len(toks) or toks[pos] != ")":
                raise UnitError("unbalanced parentheses in %r" % text)
            pos += 1
            return v
        pos += 1
        if re.fullmatch(r"[-+]?\d+", t):
            if int(t) != 1:
                raise UnitError("a number other than 1 in unit %r" % text)
            return np.zeros(len(BASE), np.int64)
        return _symbol(t)

    def term():
        nonlocal pos
        v = atom()
        if pos < len(toks) and toks[pos] in ("^", "**"):
            pos += 1
            if pos >= len(toks) or not re.fullmatch(r"[-+]?\d+", toks[pos]):
                raise UnitError("non-integer power in unit %r" % text)
            v = v * int(toks[pos])
            pos += 1
        return v

    def unit():
        nonlocal pos
        v = term()
        while pos < len(toks) and toks[pos] != ")":
            t = toks[pos]
            if t == "/":
                pos += 1
                v = v - term()
            elif t == "*":
                pos += 1
                v = v + term()
            else:                                  # juxtaposition multiplies
                v = v + term()
        return v

    v = unit()
    if pos != len(toks):
        raise UnitError("unexpected %r in unit %r" % (toks[pos], text))
    return v


def exponent_matrix(unit_strings):
    """[p][B] int32 exponents of the features' units over the base units any
    of them uses (B <= 8), and the names of those base units.  None when all
    are dimensionless."""
    V = np.array([parse_unit(u) for u in unit_strings], np.int64).reshape(len(unit_strings), len(BASE))
    used = [b for b in range(len(BASE)) if np.any(V[:, b] != 0)]
    if not used:
        return None, []
    return V[:, used].astype(np.int32), [BASE[b] for b in used]


def same_dimension(a, b):
    return bool(np.array_equal(parse_unit(a), parse_unit(b)))
