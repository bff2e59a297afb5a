"""Pins of the oracle's extended Monte-Carlo collisions (Sec. II):
multiple ionisation Q -> Q+n and elastic ion-atom scattering.

* Multiple ionisation: each step a particle of charge Q goes to Q+n with
  probability P_{Q,n} = 1 - exp(-n_e k_{Q,n} dt) (channels that would pass
  z_max closed), so the charge distribution after K steps is the start
  distribution times M^K, M the one-step transition matrix, and the expected
  number of n-electron events is the sum over steps of (distribution before
  the step) x P_{Q,n}.  Checked per charge and per n at 4.5 sigma, from a
  start that includes charges next to z_max.
* Elastic scattering with a (nearly) cold partner of equal mass, isotropic
  in the centre-of-mass frame: the energy after the collision is uniform on
  [0, E0] (mean E0/2, quartiles E0/4 and 3E0/4), the mean velocity is the
  centre-of-mass velocity v0/2, the charge is kept, and the collision count
  per Q is binomial with P = n0 (Q sigma_el1) v0 dt.
* One uniform decides between channels: with ionisation, charge exchange
  and elastic scattering on together, each kind occurs with its own
  probability.
"""
import math

import numpy as np

import workloads as W
from oracle.binding import MAXN, OracleSim

E = 1.602176634e-19
AMU = 1.66053906660e-27


def _at_rest(n, q_start, p):
    x = np.zeros(n)
    return dict(x=x.copy(), y=x.copy(), z=x.copy(), vx=x.copy(), vy=x.copy(), vz=x.copy(), q=q_start.astype(np.uint8))


def test_multiple_ionisation_markov_chain():
    K = 6
    per = 8000
    starts = [0, 1, 2, 5, 15, 16, 17]
    p = W.base_params(per * len(starts), 4, 4, 8, seed=21)
    p.update(process_mask=W.P_IONIZE, dt=3e-9, ne_in=1e20)
    sp = W.with_extended_mcc(W.argon())
    p["species"] = [sp]
    q0 = np.repeat(np.array(starts), per)
    o = OracleSim(p)
    o.set_state(_at_rest(len(q0), q0, p), step=0)
    o.step(K)
    qK = o.get_state()["q"].astype(int)
    t = o.tallies()
    z = sp["z_max"]
    P = np.zeros((z + 1, MAXN + 1))  # P[Q, n]
    for q in range(z + 1):
        for n in range(1, MAXN + 1):
            k = sp["k_in"][q] if n == 1 else sp["k_multi_in"][n - 2][q]
            P[q, n] = -math.expm1(-p["ne_in"] * k * p["dt"]) if q + n <= z else 0.0
    assert P.sum(axis=1).max() < 0.1
    M = np.zeros((z + 1, z + 1))
    for q in range(z + 1):
        M[q, q] = 1.0 - P[q].sum()
        for n in range(1, MAXN + 1):
            if P[q, n] > 0:
                M[q, q + n] = P[q, n]
    for s0 in starts:
        pi = np.zeros(z + 1)
        pi[s0] = 1.0
        events = np.zeros(MAXN + 1)
        for _ in range(K):
            events += (pi[:, None] * P).sum(axis=0) * per
            pi = pi @ M
        got = np.bincount(qK[q0 == s0], minlength=z + 1)[:z + 1]
        want = per * pi
        sd = np.sqrt(np.maximum(want * (1 - pi), 1.0))
        assert np.all(np.abs(got - want) <= 4.5 * sd + 1), (s0, got, np.round(want, 1))
    # n-electron event counts over all starts
    ev_want = np.zeros(MAXN + 1)
    for s0 in starts:
        pi = np.zeros(z + 1)
        pi[s0] = 1.0
        for _ in range(K):
            ev_want += (pi[:, None] * P).sum(axis=0) * per
            pi = pi @ M
    got_n = t["ionized_n"][0].astype(float)
    for n in range(1, MAXN + 1):
        assert abs(got_n[n - 1] - ev_want[n]) <= 4.5 * math.sqrt(ev_want[n]) + 1, (n, got_n, ev_want)
    assert got_n[3] > 5  # even the rarest channel fired
    assert t["ionized"][0].sum() == got_n.sum()
    assert qK.max() <= z


def test_elastic_scattering_isotropic_in_the_cm_frame():
    per = 60_000
    p = W.base_params(2 * per, 4, 4, 8, seed=22)
    p.update(process_mask=W.P_ELASTIC, dt=2e-9, T_n_eV=1e-6)
    sp = W.with_extended_mcc(W.argon(n0_m3=5e20))
    p["species"] = [sp]
    e0 = 200.0
    m = sp["mass_amu"] * AMU
    v0 = math.sqrt(2 * e0 * E / m)
    q = np.repeat(np.array([1, 3]), per)
    st = _at_rest(2 * per, q, p)
    st["vz"] = np.full(2 * per, v0)
    o = OracleSim(p)
    o.set_state(st, step=4)
    o.step(1)
    after, ev, t = o.get_state(), o.events(), o.tallies()
    assert np.array_equal(after["q"], st["q"])
    hit = ev == W.EV_ELASTIC
    assert np.array_equal(hit, after["vz"] != v0)  # only collided ions change
    for qq in (1, 3):
        sel = q == qq
        pr = p["species"][0]["n0"] * qq * sp["sigma_el1"] * v0 * p["dt"]
        n = int(hit[sel].sum())
        assert abs(n - per * pr) <= 4.5 * math.sqrt(per * pr * (1 - pr)), (qq, n, per * pr)
        assert t["elastic"][0][qq] == n
    ek = 0.5 * m * (after["vx"] ** 2 + after["vy"] ** 2 + after["vz"] ** 2)[hit] / (e0 * E)
    nh = hit.sum()
    assert nh > 2000
    se = math.sqrt(1 / 12 / nh)
    assert abs(ek.mean() - 0.5) <= 4.5 * se
    for qt in (0.25, 0.75):
        f = (ek <= qt).mean()
        assert abs(f - qt) <= 4.5 * math.sqrt(qt * (1 - qt) / nh)
    assert ek.max() <= 1 + 1e-6
    vz = after["vz"][hit] / v0
    vx = after["vx"][hit] / v0
    assert abs(vz.mean() - 0.5) <= 4.5 * vz.std() / math.sqrt(nh)
    assert abs(vx.mean()) <= 4.5 * vx.std() / math.sqrt(nh)


def test_one_uniform_picks_each_channel_with_its_probability():
    n = 90_000
    p = W.base_params(n, 4, 4, 8, seed=23)
    p.update(process_mask=W.P_IONIZE | W.P_CX | W.P_ELASTIC, dt=2e-9, ne_in=2e19, T_n_eV=1e-6)
    sp = W.with_extended_mcc(W.argon(n0_m3=3e20))
    p["species"] = [sp]
    e0 = 100.0
    m = sp["mass_amu"] * AMU
    v0 = math.sqrt(2 * e0 * E / m)
    q = np.full(n, 4)
    st = _at_rest(n, q, p)
    st["vz"] = np.full(n, v0)
    o = OracleSim(p)
    o.set_state(st, step=1)
    o.step(1)
    ev = o.events()
    pion = sum(-math.expm1(-p["ne_in"] * (sp["k_in"][4] if k == 1 else sp["k_multi_in"][k - 2][4]) * p["dt"])
               for k in range(1, MAXN + 1))
    pcx = p["species"][0]["n0"] * 4 * sp["sigma_cx1"] * v0 * p["dt"]
    pel = p["species"][0]["n0"] * 4 * sp["sigma_el1"] * v0 * p["dt"]
    for code, pr in ((W.EV_IONIZE, pion), (W.EV_CX, pcx), (W.EV_ELASTIC, pel)):
        got = int((ev == code).sum())
        assert abs(got - n * pr) <= 4.5 * math.sqrt(n * pr), (code, got, n * pr)
    assert int((ev == W.EV_NONE).sum()) + int((ev != W.EV_NONE).sum()) == n
