"""The autotuner (slm_autotune_set): measured launch plans are cached per
shape class and written to a file; tree builds with the measured plans, with
the fitted rules, eagerly and replayed as graphs, give bit-identical
classification trees (a plan changes only the launch shape)."""
import json

import numpy as np
import pytest
import torch

from paper_2208_07023_amd import inputs

pytestmark = pytest.mark.gpu


def _tree(api, Xd, yd, use_graph):
    cfg = api.TreeConfig(crit=api.ENTROPY, K=3, max_depth=4, min_node=32, P=64, T=5, bins=64,
                         seed=3, use_graph=use_graph)
    return api.grow_tree(Xd, yd, cfg)


@pytest.mark.parametrize("use_graph", [False, True])
def test_tuned_and_rule_plans_build_identical_trees(gpu_lib, tmp_path, use_graph):
    api = gpu_lib
    X, y = inputs.cluster_mixture(30000, 96, 3, clusters_per_class=2, mean_std=1.0, seed=8)
    Xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()
    path = str(tmp_path / "plans.json")
    try:
        api.autotune(2, path)
        tuned_build = _tree(api, Xd, yd, use_graph)
        plans = json.load(open(path))["plans"]
        assert any(k.startswith("scan/") for k in plans) and any(k.startswith("proj/") for k in plans)
        n = api.autotune(1, path)
        assert n == len(plans)
        cached = _tree(api, Xd, yd, use_graph)
        api.autotune(0)
        rules = _tree(api, Xd, yd, use_graph)
    finally:
        api.autotune(1)
    for k in ("w", "thr", "left", "right", "split_loss", "n"):
        assert np.array_equal(cached[k], rules[k]), k
        assert np.array_equal(tuned_build[k], rules[k]), k
