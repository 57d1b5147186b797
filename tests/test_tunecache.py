"""The autotune cache's host side (CPU): the problem part of its key, and the
JSON file surviving round trips, concurrent writers and damage."""
import json

import pytest

torch = pytest.importorskip("torch")
cc = pytest.importorskip("paper_1306_6883_amd")
from paper_1306_6883_amd import tunecache as T  # noqa: E402


def test_problem_key_separates_what_shapes_depend_on():
    base = cc.Problem(n=1024, bc="P")
    k = T.problem_key(base)
    assert k == {"n": 1024, "bc": "2222", "prec": cc.FP64, "nu1": 2, "nu2": 2, "singular": True, "helmholtz": False}
    # the right-hand side and tolerance do not enter; size, sides, precision, operator kind do
    assert T.problem_key(cc.Problem(n=1024, bc="P", rtol=1e-6)) == k
    for other in (cc.Problem(n=2048, bc="P"), cc.Problem(n=1024, bc="D"), cc.Problem(n=1024, bc="P", prec=cc.MIXED),
                  cc.Problem(n=1024, bc="P", alpha=1.0, beta=0.1), cc.Problem(n=1024, bc="P", nu1=1)):
        assert T.problem_key(other) != k


def test_store_and_load_round_trip(tmp_path):
    p = str(tmp_path / "sub" / "tune.json")
    assert T._load(p) == {}
    data = {"k1": {"levels": [[64, 1, 128, 2]], "fused64": [164, 1], "fused32": [64, 1]}}
    T._store(p, data)
    assert T._load(p) == data
    data["k2"] = {"levels": [], "fused64": [8, 4], "fused32": [8, 4]}
    T._store(p, data)
    assert set(T._load(p)) == {"k1", "k2"}
    assert not [f for f in (tmp_path / "sub").iterdir() if f.suffix == ".tmp"]


def test_damaged_file_reads_as_empty(tmp_path):
    p = tmp_path / "tune.json"
    p.write_text("{not json")
    assert T._load(str(p)) == {}
    p.write_text(json.dumps([1, 2, 3]))
    assert T._load(str(p)) == {}
