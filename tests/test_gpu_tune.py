"""Autotuner with the learned cost model: every candidate schedule decodes
bit-exactly, and on workloads held out of training the model-guided choice
(two measurements) is close to exhaustive tuning and well ahead of the
untuned default."""
import math

import numpy as np
import pytest

from tests.gpuutil import say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def tune():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1504_07038_amd import tune

    return tune


def workloads(tune, Ps, codes=((4, 2), (8, 4)), counts=(1, 32, 1024), cap=256 << 20):
    out = []
    for k, m in codes:
        for P in Ps:
            for nb in counts:
                if nb * P * k * 8 <= cap:
                    out.append(tune.Workload(k, m, P, nb, m))
    return out


def test_every_candidate_schedule_decodes_exactly(tune):
    bench = tune.Bench(reps=1)
    for w in [tune.Workload(4, 2, 4096, 3, 2), tune.Workload(8, 4, 1024, 5, 4),
              tune.Workload(6, 3, 700, 9, 3)]:
        for s in tune.candidates(w):
            bench.run(w, s, check=True)


def test_learned_model_tunes_held_out_workloads(tune):
    bench = tune.Bench(reps=3)
    tuner = tune.Tuner(bench)
    train = workloads(tune, [64, 256, 1024, 4096, 16384])
    held = workloads(tune, [128, 512, 2048, 8192])
    table = {w: tuner.measure_all(w) for w in train + held}
    X, y = tuner.dataset({w: table[w] for w in train})
    model = tune.CostModel(hidden=32, seed=0)
    loss = model.fit(X, y, steps=2500, lr=3e-3)
    tuner.model = model
    say(f"tune: {len(X)} training points, final loss {loss:.4f} (standardised log ms)")
    assert model.losses[-1] < model.losses[0]
    r_best, r_default, r_model, r_rule, n_meas = [], [], [], [], 0
    for w in held:
        times = table[w]
        best = min(times.values())
        t_def = times[tune.default_schedule(w)]
        t_rule = times[tune.rule_schedule(w)]
        s, t_mod = tuner.choose(w, budget=2, times=times)
        n_meas += 2
        r_best.append(t_mod / best)
        r_default.append(t_def / t_mod)
        r_model.append(t_def / best)
        r_rule.append(t_rule / t_mod)
    gm = lambda a: float(math.exp(np.mean(np.log(a))))
    say(f"tune: held-out {len(held)} workloads; model/exhaustive {gm(r_best):.3f}, "
        f"default/model {gm(r_default):.2f}x, default/exhaustive {gm(r_model):.2f}x, "
        f"two-line rule/model {gm(r_rule):.2f}x, "
        f"measurements {n_meas} vs {sum(len(table[w]) for w in held)}")
    assert gm(r_best) < 1.15          # within 15% of exhaustive tuning
    assert gm(r_default) > 1.5        # well ahead of the untuned default
    assert gm(r_rule) > 1.0           # and ahead of a two-line rule on P and nblocks
    assert n_meas < sum(len(table[w]) for w in held)
