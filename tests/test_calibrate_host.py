"""The calibration loop's host logic on a model source (no GPU).

The model stands in for served runs: gas flow = a w T^0.2 and power =
b w T^1.1 (both proportional to the weight, as the lost-particle counts
times the weight are), times a noise factor shared by the points of one
batch (the common random numbers of one seed) and a small independent one.
"""
import math

import numpy as np
import pytest

from paper_1507_03392_amd.calibrate import Targets, calibrate, outputs


class Model:
    def __init__(self, seed=0, common=0.03, own=0.003):
        self.rng = np.random.default_rng(seed)
        self.common, self.own = common, own
        self.calls = 0

    def truth(self, w, te):
        return 2e-10 * w * te ** 0.2, 3e-9 * w * te ** 1.1

    def __call__(self, points):
        self.calls += 1
        c = math.exp(self.common * self.rng.normal())
        out = []
        for w, te in points:
            f, p = self.truth(w, te)
            out.append((f * c * math.exp(self.own * self.rng.normal()), p * c * math.exp(self.own * self.rng.normal())))
        return out


def test_two_targets_move_weight_and_temperature():
    m = Model(seed=1)
    w_true, te_true = 2.5e9, 1800.0
    f, p = m.truth(w_true, te_true)
    res = calibrate(m, Targets(power_W=p, gas_flow_pmA=f, rtol=0.1), w0=6e8, te0_ev=500.0)
    assert res.converged and res.iterations <= 6
    assert abs(res.power_W / p - 1) <= 0.1 and abs(res.gas_flow_pmA / f - 1) <= 0.1
    assert res.w == pytest.approx(w_true, rel=0.3) and res.te_ev == pytest.approx(te_true, rel=0.3)
    assert res.evaluations == 3 * (res.iterations + 1)  # the point and its two probes, concurrently
    assert len(res.history) == res.iterations + 1


def test_one_target_moves_only_the_weight():
    m = Model(seed=2)
    f, p = m.truth(1e9, 1000.0)
    res = calibrate(m, Targets(power_W=p, rtol=0.05), w0=4e10, te0_ev=1000.0)
    assert res.converged
    assert res.te_ev == 1000.0 and all(h.te_ev == 1000.0 for h in res.history)
    assert abs(res.power_W / p - 1) <= 0.05


def test_unreachable_target_reports_not_converged():
    # the model's power / flow ratio is 15 T^0.9: a ratio that needs T far
    # beyond the allowed range cannot be met
    m = Model(seed=3, common=0.0, own=0.0)
    res = calibrate(m, Targets(power_W=1.0, gas_flow_pmA=1e-9, rtol=0.1), w0=1e9, te0_ev=1000.0, max_iter=4,
                    te_bounds=(10.0, 2000.0))
    assert not res.converged and res.iterations == 4
    assert res.te_ev <= 2000.0 * (1 + 1e-12)
    with pytest.raises(ValueError):
        calibrate(m, Targets(), w0=1e9, te0_ev=1000.0)


def test_outputs_from_tallies():
    # hand-computed: 100 extracted Ar1+ and 50 walls of Ar2+ over 1000 steps of 1 ns
    t = dict(extracted=np.zeros((4, 32), np.uint64), wall=np.zeros((4, 32), np.uint64),
             lost_ke=np.zeros(4), steps=1000)
    t["extracted"][0][1] = 100
    t["wall"][0][2] = 50
    t["lost_ke"][0] = 150 * 20 * 1.602176634e-19
    w, dt, te = 1e9, 1e-9, 1000.0
    flow, power = outputs(t, w, dt, te, [[15.76, 27.63]])
    e = 1.602176634e-19
    assert flow == pytest.approx(e * w * 100 / 1e-6 / 1e-3, rel=1e-12)  # the aperture only
    energy = 150 * 20 * e + (100 * 15.76 + 50 * (15.76 + 27.63)) * e + 1.5 * te * e * (100 * 1 + 50 * 2)
    assert power == pytest.approx(w * energy / 1e-6, rel=1e-12)
