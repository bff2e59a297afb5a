"""Pins of the oracle's electron-ion heating kick (Sec. II).

* Heating rate: the kick is built to reproduce the classical electron-ion
  heating of the NRL Plasma Formulary (Huba), dT_i/dt = nu (T_e - T_i) with
  nu = 1.8e-19 (m_i m_e)^1/2 Z^2 n_e lambda / (m_i T_e + m_e T_i)^3/2 (cgs,
  T in eV).  Ions at rest gain on average 3/2 nu T_e dt in one step; checked
  for two charge states (the Z^2 law) and both electron zones (the
  1/sqrt(T_e) law) within 3.5% (the paper's constant 3.715e-6 sits 1.9%
  below the formulary's rate, sampling adds 0.4%).
* Renormalisation: |dV| = D |R| whatever the bias, so with R uniform in the
  cube [-1/2, 1/2]^3 the fraction of kicks below D/2 is the volume of the
  ball of radius 1/2, pi/6, and no kick exceeds D sqrt(3)/2.
* Diamagnetic bias: with an ion charge density rising linearly along x
  (a + b ix per cell, uniform in y), the printed stencil gives delta =
  (0, -4 b R_L / (a + b ix), 0), and for small delta the mean kick is
  (2/3) D delta (the cube's symmetry gives E[R R^T / |R|^2] = I/3); its sign
  is the electron diamagnetic drift's for B along +z, (dn/dy, -dn/dx).  At
  the mesh edge the missing neighbours count as zero density.
* No kick for atoms, with zero electron density, or with the switch off.
* The isotropic-heating switch (the paper's ablation, Sec. IV) drops the
  bias: the same ramp gives no mean drift, and the same kick magnitudes.
"""
import math

import numpy as np

import workloads as W
from oracle.binding import OracleSim

E = 1.602176634e-19
AMU = 1.66053906660e-27
ME_G = 9.1093837015e-28   # electron mass, g
AMU_G = 1.66053906660e-24


def _nrl_gain_J(a_amu, z, ne_m3, te_ev, lam, dt):
    """3/2 dT_i in one step for ions at rest, from the formulary's rate."""
    mi = a_amu * AMU_G
    nu = 1.8e-19 * math.sqrt(mi * ME_G) * z * z * (ne_m3 * 1e-6) * lam / (mi * te_ev) ** 1.5
    return 1.5 * nu * te_ev * dt * E


def _uniform_b(p):
    p.update(mirror_k=0.0, BH=0.0)  # B = B0 z-hat everywhere
    return p


def test_heating_rate_is_the_formulary_rate():
    n_grp = 30_000
    p = W.base_params(4 * n_grp, 8, 8, 16, seed=11)
    p.update(process_mask=W.P_HEAT, dt=2e-8, zone_a=0.02, zone_c=0.06, ne_in=1.0e18, ne_out=3.0e17,
             Te_in_eV=1500.0, Te_out_eV=5.0)
    # groups: (inside, Q=1) (inside, Q=3) (outside, Q=1) (outside, Q=3), at rest
    pos_in, pos_out = (0.0, 0.0, 0.0), (0.0, 0.0, 0.12)
    groups = [(pos_in, 1), (pos_in, 3), (pos_out, 1), (pos_out, 3)]
    xyz = np.repeat(np.array([g[0] for g in groups]), n_grp, axis=0)
    q = np.repeat(np.array([g[1] for g in groups], dtype=np.uint8), n_grp)
    zeros = np.zeros(len(q))
    st = dict(x=xyz[:, 0].copy(), y=xyz[:, 1].copy(), z=xyz[:, 2].copy(), vx=zeros, vy=zeros, vz=zeros, q=q)
    o = OracleSim(p)
    o.set_state(st, step=5)
    o.step(1)
    after = o.get_state()
    m = p["species"][0]["mass_amu"] * AMU
    ke = 0.5 * m * (after["vx"] ** 2 + after["vy"] ** 2 + after["vz"] ** 2)
    for g, (pos, z) in enumerate(groups):
        inside = pos is pos_in
        ne = p["ne_in"] if inside else p["ne_out"]
        te = p["Te_in_eV"] if inside else p["Te_out_eV"]
        got = ke[g * n_grp:(g + 1) * n_grp].mean()
        want = _nrl_gain_J(p["species"][0]["mass_amu"], z, ne, te, p["lnL_ei"], p["dt"])
        assert abs(got / want - 1.0) < 0.035, (g, got / want)
    # no bias on a uniform background: the mean kick vanishes
    v = np.stack([after["vx"], after["vy"], after["vz"]], axis=1)
    for g in range(4):
        vg = v[g * n_grp:(g + 1) * n_grp]
        assert np.all(np.abs(vg.mean(0)) <= 4.5 * vg.std(0) / math.sqrt(n_grp))


def _gradient_state(p, a, b, band, n_per_charge):
    """Q=1 ions at rest at the centres of the cells of plane iz0, cell (ix, iy)
    holding a + b*ix ions, for ix, iy in band."""
    hx, hy, hz = 2 * p["R0"] / p["nx"], 2 * p["R0"] / p["ny"], p["L"] / p["nz"]
    iz0 = p["nz"] // 2
    xs, ys, cells = [], [], []
    for iy in band:
        for ix in band:
            k = (a + b * ix) * n_per_charge
            xs += [-p["R0"] + (ix + 0.5) * hx] * k
            ys += [-p["R0"] + (iy + 0.5) * hy] * k
            cells += [(ix, iy)] * k
    n = len(xs)
    z = np.full(n, -p["L"] / 2 + (iz0 + 0.5) * hz)
    st = dict(x=np.array(xs), y=np.array(ys), z=z, vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n),
              q=np.ones(n, dtype=np.uint8))
    return st, np.array(cells)


def test_diamagnetic_bias_and_kick_magnitude():
    nx = 16
    p = _uniform_b(W.base_params(1, nx, nx, 16, seed=12))
    p.update(process_mask=W.P_HEAT, self_ne=True, zone_a=1.0, zone_c=1.0, dt=1e-8, weight=2e9,
             Te_in_eV=4000.0, B0=0.25)
    a, b, per = 20, 6, 40
    band = range(2, 14)
    st, cells = _gradient_state(p, a, b, band, per)
    p["n"] = len(st["x"])
    o = OracleSim(p)
    o.set_state(st, step=3)
    o.step(1)
    after = o.get_state()
    hx = 2 * p["R0"] / nx
    vcell = hx * hx * (p["L"] / p["nz"])
    rl = 2.38e-6 * math.sqrt(p["Te_in_eV"]) / (p["B0"] * hx)
    dv = np.stack([after["vx"], after["vy"], after["vz"]], axis=1)
    A = p["species"][0]["mass_amu"]
    checked = 0
    frac_half, n_all = 0, 0
    for ix in range(3, 13):  # interior columns: every neighbour is populated
        sel = (cells[:, 0] == ix) & (cells[:, 1] >= 3) & (cells[:, 1] <= 12)
        chg = (a + b * ix) * per
        ne = p["weight"] * chg / vcell
        D = math.sqrt(3.715e-6 * ne * p["lnL_ei"] * p["dt"] / (A * A * math.sqrt(p["Te_in_eV"])))
        delta_y = -4.0 * b * per * rl / chg
        assert 0.005 < abs(delta_y) < 0.2
        mean = dv[sel].mean(0)
        se = dv[sel].std(0) / math.sqrt(sel.sum())
        assert abs(mean[0]) <= 4.5 * se[0] and abs(mean[2]) <= 4.5 * se[2], ix
        want = (2.0 / 3.0) * D * delta_y  # third-order terms: < 0.5% at these delta
        assert abs(mean[1] - want) <= 4.5 * se[1] + 0.005 * abs(want), (ix, mean[1], want, se[1])
        assert mean[1] < 0  # density rises along +x: electrons drift along -y for B along +z
        mag = np.linalg.norm(dv[sel], axis=1) / D
        assert mag.max() <= math.sqrt(3) / 2 * (1 + 1e-12)
        frac_half += int((mag <= 0.5).sum())
        n_all += int(sel.sum())
        checked += 1
    assert checked == 10
    pf = math.pi / 6
    assert abs(frac_half / n_all - pf) <= 4.5 * math.sqrt(pf * (1 - pf) / n_all)
    # mesh-edge reading: a column of equal charge at ix = 0 sees zero density
    # at ix = -1, so its bracket is 2 n and delta_y = -2 R_L
    p2 = dict(p)
    st2, cells2 = _gradient_state(p2, 30, 0, range(0, 4), per)
    p2["n"] = len(st2["x"])
    o2 = OracleSim(p2)
    o2.set_state(st2, step=3)
    o2.step(1)
    d2 = o2.get_state()
    sel = (cells2[:, 0] == 0) & (cells2[:, 1] >= 1) & (cells2[:, 1] <= 2)
    ne = p2["weight"] * 30 * per / vcell
    D = math.sqrt(3.715e-6 * ne * p2["lnL_ei"] * p2["dt"] / (A * A * math.sqrt(p2["Te_in_eV"])))
    vy = d2["vy"][sel]
    want = (2.0 / 3.0) * D * (-2.0 * rl)
    assert abs(vy.mean() - want) <= 4.5 * vy.std() / math.sqrt(sel.sum()) + 0.005 * abs(want)


def test_no_kick_for_atoms_empty_backgrounds_or_switch_off():
    p = W.base_params(6000, 8, 8, 16, seed=13)
    p.update(process_mask=W.P_HEAT, dt=1e-8, ne_out=0.0)
    st = W.random_state(p, seed=14, q_max=6, frac_atoms=0.3, v_ev=5.0)
    o = OracleSim(p)
    o.set_state(st, step=0)
    o.step(1)
    after = o.get_state()
    x, y, z = st["x"], st["y"], st["z"]
    inside = (x * x + y * y) / p["zone_a"] ** 2 + z * z / p["zone_c"] ** 2 < 1
    still = (st["q"] == 0) | ~inside
    changed = after["vx"] != st["vx"]
    assert np.array_equal(changed, ~still)  # every ion in the zone moves, nothing else
    assert (~still).sum() > 100
    p_off = dict(p, process_mask=W.P_IONIZE & 0)
    o = OracleSim(p_off)
    o.set_state(st, step=0)
    o.step(1)
    assert np.array_equal(o.get_state()["vx"], st["vx"])


def test_isotropic_switch_removes_the_bias_only():
    nx = 16
    p = _uniform_b(W.base_params(1, nx, nx, 16, seed=12))
    p.update(process_mask=W.P_HEAT, self_ne=True, zone_a=1.0, zone_c=1.0, dt=1e-8, weight=2e9,
             Te_in_eV=4000.0, B0=0.25)
    st, cells = _gradient_state(p, 20, 6, range(2, 14), 40)
    p["n"] = len(st["x"])
    out = []
    for iso in (False, True):
        o = OracleSim(dict(p, heat_isotropic=iso))
        o.set_state(st, step=3)
        o.step(1)
        a = o.get_state()
        out.append(np.stack([a["vx"], a["vy"], a["vz"]], axis=1))
    sel = (cells[:, 0] >= 3) & (cells[:, 0] <= 12) & (cells[:, 1] >= 3) & (cells[:, 1] <= 12)
    biased, iso = out[0][sel], out[1][sel]
    se = iso.std(0) / math.sqrt(sel.sum())
    assert np.all(np.abs(iso.mean(0)) <= 4.5 * se)
    assert biased[:, 1].mean() < -4.5 * se[1]
    # |dV| = D |R| either way: the same draws give the same magnitudes
    np.testing.assert_allclose(np.linalg.norm(iso, axis=1), np.linalg.norm(biased, axis=1), rtol=1e-12)
