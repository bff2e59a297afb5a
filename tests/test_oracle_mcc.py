"""Pins of the oracle's Monte-Carlo collision block (paper Sec. II, Sec. III.B).

* Ionisation Q -> Q+1 of frozen ions: the charge-state populations follow
  the per-step Markov chain exactly; its mean is the matrix power of the
  bidiagonal transition matrix, and the continuous rate equations (Bateman
  chain) agree to O(nu dt).
* The paper's worked example: atoms at the thermal speed 4e4 cm/s in
  n_e = 5e11 cm^-3 with k = 1e-7 cm^3/s have an ionisation mean free path of
  about 1 cm; the neutral Maxwellian at 0.025 eV has a mean speed of about
  4e4 cm/s (tests/golden/paper_numbers.json).
* Charge exchange: Ar2+ never exchanges; Q >= 3 exchange releases 10 eV
  shared equally, so a slow ion hitting a cold neutral leaves with 5 eV in
  an isotropic direction; event counts are binomial in n0 sigma Q v dt.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle.binding import OracleSim

E = 1.602176634e-19
AMU = 1.66053906660e-27
HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_numbers.json")))


def frozen_state(n, q, vx=0.0):
    z = np.zeros(n)
    return dict(x=z.copy(), y=z.copy(), z=z.copy(), vx=np.full(n, vx), vy=z.copy(), vz=z.copy(),
                q=np.full(n, q, dtype=np.uint8))


def test_ionisation_chain_matches_markov_chain_and_bateman():
    n, steps = 20000, 400
    p = W.base_params(n, 8, 8, 16)
    p.update(process_mask=W.P_IONIZE, dt=2e-8)  # frozen particles, all at the origin (inside the zone)
    s = OracleSim(p)
    s.set_state(frozen_state(n, 0))
    k = np.array(p["species"][0]["k_in"])
    ne, dt, zmax = p["ne_in"], p["dt"], p["species"][0]["z_max"]
    P = np.where(np.arange(32) < zmax, 1.0 - np.exp(-ne * k * dt), 0.0)
    T = np.zeros((zmax + 1, zmax + 1))
    for q in range(zmax + 1):
        T[q, q] = 1 - P[q]
        if q < zmax:
            T[q, q + 1] = P[q]
    p0 = np.zeros(zmax + 1)
    p0[0] = 1.0
    checkpoints = [50, 150, 400]
    done = 0
    for c in checkpoints:
        s.step(c - done)
        done = c
        counts = np.bincount(s.get_state()["q"], minlength=zmax + 1)
        pm = p0 @ np.linalg.matrix_power(T, c)
        for q in range(4):
            mean, var = n * pm[q], n * pm[q] * (1 - pm[q])
            if mean > 5:
                assert abs(counts[q] - mean) < 5 * math.sqrt(var), (c, q, counts[q], mean)
        # Bateman (continuous) populations of the first two states
        nu0, nu1 = ne * k[0], ne * k[1]
        t = c * dt
        b0 = math.exp(-nu0 * t)
        b1 = nu0 / (nu1 - nu0) * (math.exp(-nu0 * t) - math.exp(-nu1 * t))
        assert pm[0] == pytest.approx(b0, rel=5 * nu0 * dt * c * nu0 * dt + 1e-12)
        assert pm[1] == pytest.approx(b1, rel=0.02)
    t = s.tallies()
    assert int(t["ionized"][0].sum()) == int(np.dot(np.arange(zmax + 1), np.bincount(s.get_state()["q"], minlength=zmax + 1)))


def test_paper_mean_free_path_of_atoms():
    g = GOLD["atom_ionisation_mean_free_path"]
    v = g["thermal_speed_cm_s"] * 1e-2
    ne = g["ne_cm3"] * 1e6
    kk = g["k0_cm3_s"] * 1e-6
    n = 4000
    p = W.base_params(n, 8, 8, 16)
    sp = dict(p["species"][0])
    sp["k_in"] = [kk] + [0.0] * 31
    p.update(process_mask=W.P_PUSH | W.P_IONIZE, dt=1e-7, ne_in=ne, zone_a=1.0, zone_c=5.0,
             species=[sp], BH=0.0, L=10.0)
    s = OracleSim(p)
    st = frozen_state(n, 0)
    st["z"] = np.full(n, -4.9)
    st["vz"] = np.full(n, v)
    s.set_state(st)
    dist = np.full(n, np.nan)
    for it in range(1, 3000):
        s.step(1)
        q = s.get_state()["q"]
        newly = (q == 1) & np.isnan(dist)
        dist[newly] = it * v * p["dt"]
        if not np.isnan(dist).any():
            break
    mfp_cm = np.nanmean(dist) * 100
    assert mfp_cm == pytest.approx(v / (ne * kk) * 100, rel=0.05)   # exponential law
    lo, hi = g["mfp_cm_range"]
    assert lo <= mfp_cm <= hi                                         # "about 1 cm"


def cx_params(n, n0, q_forbid=True, T_n=0.025):
    p = W.base_params(n, 8, 8, 16)
    sp = dict(p["species"][0])
    sp["n0"] = n0
    sp["sigma_cx1"] = 1e-18
    if not q_forbid:
        sp["cx_forbidden_mask"] = 0
    p.update(process_mask=W.P_CX, species=[sp], T_n_eV=T_n)
    return p


def test_cx_forbidden_for_ar2_and_binomial_counts():
    n, steps, v = 20000, 20, 1000.0
    n0 = 2e21
    p = cx_params(n, n0)
    s = OracleSim(p)
    st = frozen_state(n, 2, vx=v)
    st["q"][: n // 2] = 3
    s.set_state(st)
    s.step(steps)
    t = s.tallies()
    assert t["cx"][0][2] == 0
    P3 = n0 * 1e-18 * 3 * v * p["dt"]
    # every Q=3 ion that exchanges becomes Q=2 and then stays (Ar2+ is forbidden)
    mean = (n // 2) * (1 - (1 - P3) ** steps)
    assert abs(int(t["cx"][0][3]) - mean) < 5 * math.sqrt(mean)
    assert int(t["cx_products"][0]) == int(t["cx"][0][3])


def test_cx_energy_release_shared_equally_and_isotropic():
    n = 20000
    p = cx_params(n, 1e26, T_n=0.0)   # cold neutrals: v_n = 0
    s = OracleSim(p)
    st = frozen_state(n, 5, vx=1.0)   # 1 m/s ions
    s.set_state(st)
    s.step(1)
    out = s.get_state()
    ev = s.events()
    hit = ev == W.EV_CX
    assert hit.sum() > 1000
    M = 39.948 * AMU
    v2 = out["vx"][hit] ** 2 + out["vy"][hit] ** 2 + out["vz"][hit] ** 2
    ke_ev = 0.5 * M * v2 / E
    assert np.abs(ke_ev - 5.0).max() < 2e-3              # dE/2 = 5 eV each
    assert np.all(out["q"][hit] == 4)
    c = out["vz"][hit] / np.sqrt(v2)
    m = hit.sum()
    assert abs(c.mean()) < 5 / math.sqrt(3 * m)
    assert abs((c * c).mean() - 1 / 3) < 5 * math.sqrt(4 / 45 / m)


def test_cx_resonant_q1_takes_neutral_maxwellian_mean_speed():
    g = GOLD["neutral_thermal_speed"]
    n = 20000
    p = cx_params(n, 1e26, T_n=g["T_eV"])
    s = OracleSim(p)
    s.set_state(frozen_state(n, 1, vx=1000.0))
    s.step(1)
    out = s.get_state()
    hit = s.events() == W.EV_CX
    assert hit.sum() > 2000
    assert np.all(out["q"][hit] == 1)
    sp = np.sqrt(out["vx"][hit] ** 2 + out["vy"][hit] ** 2 + out["vz"][hit] ** 2) * 100
    M = 39.948 * AMU
    mean_theory = math.sqrt(8 * g["T_eV"] * E / (math.pi * M)) * 100
    assert sp.mean() == pytest.approx(mean_theory, rel=0.02)
    assert sp.mean() == pytest.approx(g["mean_speed_cm_s"], rel=g["rel_tol"])
