"""Host accounting of the learned restart: TTS99, the rank AUC and the
validation score that selects the restart threshold."""
import math

import numpy as np
import pytest

from paper_2308_02329_amd import learned


def test_tts99_closed_forms():
    assert learned.tts99(2.0, 0.0) == math.inf
    assert learned.tts99(2.0, 0.995) == 2.0
    # p = 1 - 0.01^(1/k): exactly k attempts reach 99%
    for k in (1.5, 10.0, 1000.0):
        p = 1.0 - 0.01 ** (1.0 / k)
        assert learned.tts99(3.0, p) == pytest.approx(3.0 * k, rel=1e-12)


def test_auc_rank_statistic():
    assert learned.auc([0.1, 0.2, 0.8, 0.9], [0, 0, 1, 1]) == 1.0
    assert learned.auc([0.9, 0.8, 0.2, 0.1], [0, 0, 1, 1]) == 0.0
    assert learned.auc([0.5, 0.5, 0.5, 0.5], [0, 1, 0, 1]) == 0.5  # ties count half
    g = np.random.default_rng(3)
    s, y = g.normal(size=300), g.random(300) < 0.3
    brute = np.mean([(a > b) + 0.5 * (a == b) for a in s[y] for b in s[~y]])
    assert learned.auc(s, y) == pytest.approx(brute, abs=1e-12)
    assert math.isnan(learned.auc([0.1, 0.2], [1, 1]))


def test_validation_score():
    base = [2.0, 8.0, math.inf]
    assert learned.validation_score(base, base) == pytest.approx(4.0)  # geometric mean of the solved ones
    assert learned.validation_score([1.0, 4.0, math.inf], base) == pytest.approx(2.0)
    # losing an instance the plain method solves is infeasible, however fast the rest gets
    assert learned.validation_score([0.01, math.inf, math.inf], base) == math.inf
    # an instance the plain method does not solve does not count
    assert learned.validation_score([1.0, 4.0, 0.5], base) == pytest.approx(2.0)
    assert learned.validation_score([1.0], [math.inf]) == math.inf
    # a median would prefer a policy that loses 2 of 5 instances; the score does not
    b5 = [10.0] * 5
    risky = [1.0, 1.0, 1.0, math.inf, math.inf]
    assert np.median(risky) < np.median(b5)
    assert learned.validation_score(risky, b5) == math.inf


def test_instance_tts_keep_policy():
    import torch

    # one instance, 2 pumps x 10 runs; run time 10 ms per run, the first 10% of it before the checkpoint
    E = torch.tensor([-5, 0, 0, 0, 0, 0, 0, 0, 0, -5] + [0] * 10)
    inst = dict(E=E, t_part_ms=20.0, t_rest_ms=180.0, n_ic=10, n_pumps=2)
    t_full, t_part = 10.0, 1.0
    # plain: pump 0 succeeds 2 of 10
    want = t_full * math.log(0.01) / math.log(0.8)
    assert learned.instance_tts(inst, -5) == pytest.approx(want)
    assert learned.instance_tts(inst, -5, np.zeros(20), 1.0) == pytest.approx(want)
    # keep the top 20% by score: the two successful runs scored highest -> both kept
    q = np.array([0.9, 0.1, 0.2, 0.3, 0.1, 0.2, 0.3, 0.1, 0.2, 0.8] + [0.5] * 10)
    cost = t_part + 0.2 * (t_full - t_part)
    assert learned.instance_tts(inst, -5, q, 0.2) == pytest.approx(cost * math.log(0.01) / math.log(0.8))
    # keep 10%: only run 0 kept, one success in ten attempts
    cost = t_part + 0.1 * (t_full - t_part)
    assert learned.instance_tts(inst, -5, q, 0.1) == pytest.approx(cost * math.log(0.01) / math.log(0.9))
    # scores that rank the successes last lose the instance at small keep fractions
    assert learned.instance_tts(inst, -5, 1.0 - q, 0.2) == math.inf
    # ties are broken by run index (stable)
    assert learned.instance_tts(inst, -5, np.zeros(20), 0.1) == pytest.approx(cost * math.log(0.01) / math.log(0.9))
