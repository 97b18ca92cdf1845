"""Host layer of run_discover: the unit parser, the configuration parser and
the rule resolution (no GPU).

The unit parser is pinned by identities of SI derived units that hold by
their definitions (a joule is a newton metre, a volt a watt per ampere, an
ohm a volt per ampere, a farad a coulomb per volt, a tesla a weber per
square metre, a siemens an inverse ohm), each checked between two
different spellings so that a wrong table entry or a wrong operator in the
grammar fails.
"""
import json
import os

import numpy as np
import pytest

from paper_2602_06986_amd import run as R
from paper_2602_06986_amd import units as U


def vec(m=0, kg=0, s=0, A=0, K=0, mol=0, cd=0):
    return np.array([m, kg, s, A, K, mol, cd], np.int64)


@pytest.mark.parametrize("text,want", [
    ("m", vec(m=1)), ("kg", vec(kg=1)), ("s", vec(s=1)), ("A", vec(A=1)), ("K", vec(K=1)),
    ("mol", vec(mol=1)), ("cd", vec(cd=1)),
    ("m/s^2", vec(m=1, s=-2)), ("kg m s^-2", vec(m=1, kg=1, s=-2)), ("m**2", vec(m=2)),
    ("(m/s)^2", vec(m=2, s=-2)), ("kg/m/s", vec(m=-1, kg=1, s=-1)), ("1/s", vec(s=-1)),
    ("mol/L", vec(m=-3, mol=1)), ("km/h", vec(m=1, s=-1)), ("um", vec(m=1)), ("ms", vec(s=1)),
    ("", vec()), ("1", vec()), ("dimensionless", vec()), ("-", vec()), (None, vec()),
])
def test_parse_unit(text, want):
    assert np.array_equal(U.parse_unit(text), want)


@pytest.mark.parametrize("a,b", [
    ("J", "N*m"), ("J", "kg*m^2/s^2"), ("N", "kg m / s^2"), ("W", "J/s"), ("Pa", "N/m^2"),
    ("V", "W/A"), ("ohm", "V/A"), ("F", "C/V"), ("C", "A s"), ("T", "Wb/m^2"), ("Wb", "V s"),
    ("H", "Wb/A"), ("S", "1/ohm"), ("Hz", "1/s"), ("eV", "J"), ("L", "dm^3"), ("bar", "Pa"),
])
def test_derived_unit_identities(a, b):
    assert U.same_dimension(a, b), (a, b)


@pytest.mark.parametrize("a,b", [("J", "N"), ("V", "W"), ("F", "S"), ("Pa", "J")])
def test_different_dimensions(a, b):
    assert not U.same_dimension(a, b)


@pytest.mark.parametrize("bad", ["m^x", "foo", "(m", "m)", "2 m", "m^", "m//s"])
def test_parse_errors(bad):
    with pytest.raises(U.UnitError):
        U.parse_unit(bad)


def test_exponent_matrix_restricts_bases():
    M, names = U.exponent_matrix(["m/s", "kg", "1", "m^2"])
    assert names == ["m", "kg", "s"]
    assert M.dtype == np.int32
    assert M.tolist() == [[1, 0, -1], [0, 1, 0], [0, 0, 0], [2, 0, 0]]
    assert U.exponent_matrix(["", "1"]) == (None, [])


def test_load_data_csv_npz_inline(tmp_path):
    rng = np.random.default_rng(0)
    X = rng.normal(size=(3, 20))
    y = rng.normal(size=20)
    path = tmp_path / "d.csv"
    with open(path, "w") as f:
        f.write("a,y,b,c\n")
        for i in range(20):
            f.write("%r,%r,%r,%r\n" % (float(X[0, i]), float(y[i]), float(X[1, i]), float(X[2, i])))
    Xc, yc, names = R.load_data({"file": "d.csv", "target": "y"}, str(tmp_path))
    assert names == ["a", "b", "c"]
    assert np.array_equal(Xc, X) and np.array_equal(yc, y)
    Xs, _, names2 = R.load_data({"file": str(path), "target": "y", "features": ["c", "a"]})
    assert names2 == ["c", "a"] and np.array_equal(Xs, X[[2, 0]])
    np.savez(tmp_path / "d.npz", X=X.T, y=y, names=np.array(["a", "b", "c"]))
    Xn, yn, nn = R.load_data({"file": "d.npz", "transpose": True}, str(tmp_path))
    assert nn == ["a", "b", "c"] and np.array_equal(Xn, X) and np.array_equal(yn, y)
    Xi, yi, ni = R.load_data({"X": X.tolist(), "y": y.tolist()})
    assert ni == ["x0", "x1", "x2"] and np.array_equal(Xi, X)
    with pytest.raises(R.ConfigError):
        R.load_data({"file": "d.csv", "target": "nope"}, str(tmp_path))
    with pytest.raises(R.ConfigError):
        R.load_data({"X": X.tolist(), "y": y[:5].tolist()})


def test_load_config_json_yaml(tmp_path):
    cfg = {"data": {"X": [[1.0, 2.0]], "y": [1.0, 2.0]}, "search": {"rung": 1, "k": 3}}
    (tmp_path / "c.json").write_text(json.dumps(cfg))
    (tmp_path / "c.yaml").write_text("data:\n  X: [[1.0, 2.0]]\n  y: [1.0, 2.0]\nsearch:\n  rung: 1\n  k: 3\n")
    a, base = R.load_config(str(tmp_path / "c.json"))
    b, _ = R.load_config(str(tmp_path / "c.yaml"))
    assert a == b == cfg
    assert base == os.path.abspath(str(tmp_path))


def test_resolve_rules():
    names = ["T", "P", "V", "n"]
    r = R.resolve_rules({"max_complexity": 2, "forbid_nest": {"exp": ["exp", "log"]},
                         "forbid_pairs": [["T", "V"], ["n", "n"]], "target_unit": "J"},
                        names, ["m", "kg", "s", "mol"])
    assert r["max_complexity"] == 2
    assert r["forbid_nest"] == {"exp": ["exp", "log"]}
    assert r["forbid_pairs"] == [[0, 2], [3, 3]]
    assert r["target_units"] == [2, 1, -2, 0]
    assert R.resolve_rules(None, names, []) is None
    # no feature carries units: every expression is dimensionless
    assert R.resolve_rules({"target_unit": "1"}, names, [])["target_units"] is None
    for bad in ({"forbid_pairs": [["T", "W"]]}, {"forbid_nest": {"exp": ["cosh"]}},
                {"max_complexity": -3}, {"target_unit": "A"}, {"colour": 1},
                {"forbid_pairs": [["T"]]}):
        with pytest.raises(R.ConfigError):
            R.resolve_rules(bad, names, ["m", "kg", "s", "mol"])


def test_expression_names():
    assert R.expression("(x0 * sq(x12))", ["T"] + ["f%d" % i for i in range(1, 13)]) == "(T * sq(f12))"
