"""The learned selector: trained on this project's own measured variant timings
(paper_2607_04489_amd/selector_data) by the library's GPU kernels, it must beat
the fixed hash join and the rule planner on the held-out 20% of instances, and
the committed model must be exactly what that training produces."""
import numpy as np
import pytest
import torch

import oracle
import paper_2607_04489_amd as eg
import synth
from paper_2607_04489_amd import selector

pytestmark = pytest.mark.gpu

STEPS, LR, SEED = 2000, 3e-3, 0


@pytest.fixture(scope="module")
def trained(gpu):
    recs = selector.load_records()
    train, test = selector.split(recs, seed=0)
    model = selector.train(train, steps=STEPS, lr=LR, seed=SEED)
    return recs, train, test, model


def test_learned_selector_gains_over_the_method_without_it(trained):
    _, _, test, model = trained
    ev = selector.evaluate(model, test)
    print(ev)
    assert ev["learned"]["sum_ratio"] < ev["fixed_hash"]["sum_ratio"]
    assert ev["learned"]["sum_ratio"] < ev["rule"]["sum_ratio"]
    assert ev["learned"]["geomean"] < ev["fixed_hash"]["geomean"]
    # the target: the selected plans' total time within 10% of the exhaustive best
    assert ev["learned"]["sum_ratio"] <= 1.10


def test_committed_model_is_the_trained_one(trained):
    _, _, _, model = trained
    committed = selector.load_model(install=False)
    assert torch.equal(committed["params"], model["params"].cpu())
    assert np.array_equal(committed["mean"], model["mean"])
    assert np.array_equal(committed["lo"], model["lo"]) and np.array_equal(committed["hi"], model["hi"])


def test_training_instances_lie_inside_the_domain(trained):
    """The library's domain check keeps every training instance on the model."""
    _, train, _, model = trained
    X = np.array([r["features"] for r in train], dtype=np.float32)
    assert ((X >= model["lo"]) & (X <= model["hi"])).all()


def test_training_is_deterministic(trained):
    _, train, _, _ = trained
    a = selector.train(train, steps=50, lr=LR, seed=SEED)
    b = selector.train(train, steps=50, lr=LR, seed=SEED)
    assert torch.equal(a["params"], b["params"])


def test_learned_plans_join_correctly(gpu):
    selector.load_model()
    for i in range(4):
        inp = synth.selector_instance(99, i, device=gpu, max_build_log2=15, max_probe_log2=17)
        plan = eg.join_plan(eg.stats(inp.build_keys), eg.stats(inp.probe_keys), eg.SEL_LEARNED)
        res = eg.join(inp.build_keys, inp.build_payload, inp.probe_keys, inp.probe_payload, plan)
        _, cnt, cs = oracle.join_sortmerge(inp.build_keys, inp.build_payload, inp.probe_keys,
                                           inp.probe_payload, with_pairs=False)
        assert (res.count, res.checksum) == (cnt, cs)
