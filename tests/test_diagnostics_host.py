"""Host-side scaling of tallies into the paper's outputs (CPU): currents,
gas flow in pmA, mean extraction radius, first-passage times, coupled power
and axis profiles, each against a hand computation on synthetic tallies."""
import math

import numpy as np
import pytest

import workloads as W
from paper_1507_03392_amd import diagnostics as D

E = 1.602176634e-19


def _tallies(steps=1000):
    z = lambda: np.zeros((4, 32), dtype=np.uint64)
    t = dict(extracted=z(), wall=z(), ionized=z(), cx=z(), fpt_n=z(), fpt_sum=z(), fpt_hist=z(),
             extracted_r=np.zeros((4, 32)), lost_ke=np.zeros(4), steps=steps)
    t["extracted"][0][:3] = [4, 10, 5]
    t["extracted_r"][0][:3] = [0.02, 0.03, 0.01]
    t["fpt_n"][0][1:3] = [8, 5]
    t["fpt_sum"][0][1:3] = [800, 2000]
    t["fpt_hist"][0][[0, 6, 8]] = [1, 7, 5]
    t["wall"][0][:3] = [3, 2, 1]
    t["lost_ke"][0] = 1e-17
    return t


def test_currents_and_gas_flow():
    t, w, dt = _tallies(), 2.36e7, 1e-9
    i = D.extracted_currents(t, w, dt)
    assert i[0] == 0.0 and math.isclose(i[1], 1 * E * w * 10 / 1e-6) and math.isclose(i[2], 2 * E * w * 5 / 1e-6)
    assert math.isclose(D.gas_flow_pmA(t, w, dt), E * w * 19 / 1e-6 / 1e-3)


def test_radius_and_first_passage():
    t, dt = _tallies(), 2e-9
    r = D.mean_extraction_radius(t)
    assert r[:3] == pytest.approx([0.005, 0.003, 0.002]) and np.isnan(r[3])
    m = D.mean_first_passage(t, dt)
    assert m[1:3] == pytest.approx([100 * dt, 400 * dt]) and np.isnan(m[0])
    lo, hi, c = D.first_passage_histogram(t, dt)
    assert lo[0] == 0 and hi[0] == 2 * dt and lo[6] == 64 * dt and hi[6] == 128 * dt
    assert c[[0, 6, 8]].tolist() == [1, 7, 5]


def test_coupled_power_hand_computed():
    t, w, dt = _tallies(), 1e7, 1e-9
    ip = W.AR_IP_EV
    lost = np.array([4 + 3, 10 + 2, 5 + 1], dtype=float)  # Q = 0, 1, 2
    pe = np.array([0.0, ip[0], ip[0] + ip[1]]) * E
    energy = 1e-17 + (lost * pe).sum() + 1.5 * 2000.0 * E * (lost * np.arange(3)).sum()
    assert math.isclose(D.coupled_power(t, w, dt, 2000.0, ip), w * energy / 1e-6, rel_tol=1e-12)


def test_axis_profiles_uniform_grid():
    p = W.base_params(10, 4, 4, 8)
    nn = 5 * 5 * 9
    n_field, p_field = np.full(nn, 3.0), np.full(nn, 6.0 * E)
    z, n, pr, temp = D.axis_profiles(p, n_field, p_field, steps=2, weight=1e6)
    vol = (2 * p["R0"] / 4) ** 2 * (p["L"] / 8)
    assert n == pytest.approx(np.full(9, 3.0 * 1e6 / (vol * 2)))
    assert temp == pytest.approx(np.full(9, 2.0))
    assert z[0] == -p["L"] / 2 and z[-1] == pytest.approx(p["L"] / 2)
