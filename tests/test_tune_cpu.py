"""Autotuner search and cache logic on the CPU (synthetic cost functions)."""
import numpy as np

import graphgen as gg


def test_coordinate_descent_finds_separable_minimum():
    from paper_1505_04086_amd import tune
    space = {"a": [1, 2, 3, 4], "b": [10, 20, 30], "c": [0, 1]}
    target = {"a": 3, "b": 20, "c": 1}

    def cost(o):
        return 1.0 + sum(abs(o.get(k, 0) - v) for k, v in target.items())

    best, t, trials = tune.coordinate_descent(cost, space=space, sweeps=3)
    assert best == target and t == 1.0
    assert len(trials) <= 1 + 3 * sum(len(v) for v in space.values())


def test_signature_and_cache(tmp_path, monkeypatch):
    from paper_1505_04086_amd import tune
    monkeypatch.setenv("RSOC_TUNE_FILE", str(tmp_path / "tune.json"))
    local = tune.signature(*gg.tri_grid(60))
    scrambled = tune.signature(*gg.tri_grid(60, permute_seed=3))
    assert local.endswith("local") and scrambled.endswith("scrambled")
    assert tune.signature(np.zeros(1, np.int32), np.zeros(0, np.int32)) == "empty"
    assert tune.lookup(local) is None
    tune.save(local, {"chunk": 8}, 1.5)
    assert tune.lookup(local) == {"chunk": 8}
