"""Pins of the oracle's tracked exchange partners (Sec. II: atoms are
tracked macro-particles; an exchange takes an electron from one of them).

With the switch, each charge exchange of an ion of species s takes a tracked
atom of species s from the ion's collision cell at the end of the step; the
atom becomes a Q = 1 ion (event 6) born in that step, and a Q = 1 ion that
exchanges becomes an atom with its own velocity.  So, with atoms to spare,
one step of exchange alone
* conserves the total charge exactly and removes one atom per exchange of a
  Q >= 2 ion;
* makes as many partners as exchanges in every collision cell and species,
  and moves no particle;
* picks the partners uniformly among the cell's atoms (checked by chi-square
  over many steps);
while a cell with fewer atoms than exchanges ionises all of them and counts
the rest as unmatched, and atoms recycled at a wall in the same step are not
partners.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle.binding import OracleSim

E = 1.602176634e-19
AMU = 1.66053906660e-27


def _centre(p, ix, iy, iz):
    hx, hy, hz = 2 * p["R0"] / p["nx"], 2 * p["R0"] / p["ny"], p["L"] / p["nz"]
    return -p["R0"] + (ix + 0.5) * hx, -p["R0"] + (iy + 0.5) * hy, -p["L"] / 2 + (iz + 0.5) * hz


def _cells_state(p, groups, v0):
    """groups: list of (cell, charge, count); every particle at its cell's
    centre, ions moving along z at v0, atoms at rest"""
    x, y, z, vz, q, tag = [], [], [], [], [], []
    for g, (cell, charge, count) in enumerate(groups):
        cx, cy, cz = _centre(p, *cell)
        for _ in range(count):
            x.append(cx), y.append(cy), z.append(cz)
            vz.append(v0 if charge else 0.0)
            q.append(charge)
            tag.append(g)
    n = len(x)
    zeros = np.zeros(n)
    st = dict(x=np.array(x), y=np.array(y), z=np.array(z), vx=zeros.copy(), vy=zeros.copy(), vz=np.array(vz),
              q=np.array(q, dtype=np.uint8))
    return st, np.array(tag)


def _params(n, seed, **kw):
    p = W.base_params(n, 8, 8, 16, seed=seed)
    p.update(process_mask=W.P_CX, dt=2e-9, weight=1e11, self_n0=True, cx_partner=True, T_n_eV=1e-6)
    p["species"] = [W.argon(n0_m3=1e20)]
    p.update(kw)
    return p


def test_charge_and_atoms_are_conserved_per_cell():
    # (Ar2+ never exchanges: the Q = 4 ions stand for Q >= 2)
    groups = [((4, 4, 8), 1, 3000), ((4, 4, 8), 3, 3000), ((4, 4, 8), 0, 4000),
              ((3, 4, 8), 4, 2000), ((3, 4, 8), 0, 3000)]
    p = _params(1, 41, weight=3e11)
    st, tag = _cells_state(p, groups, 3.0e4)
    p["n"] = len(tag)
    o = OracleSim(p)
    o.set_state(st, step=5)
    o.step(1)
    a, ev, t = o.get_state(), o.events(), o.tallies()
    q0, q1 = st["q"].astype(int), a["q"].astype(int)
    ncx = int((ev == W.EV_CX).sum())
    assert ncx > 200
    assert t["cx_unmatched"].sum() == 0
    assert q1.sum() == q0.sum()  # every electron given to an ion came from an atom
    cx_hi = int(((ev == W.EV_CX) & (q0 >= 2)).sum())
    assert (q1 == 0).sum() == (q0 == 0).sum() - cx_hi  # a Q = 1 exchange hands its charge over
    assert int(t["cx_products"].sum()) == cx_hi
    part = ev == W.EV_CX_PARTNER
    assert np.all(q0[part] == 0) and np.all(q1[part] == 1)
    assert np.all(a["birth"][part] == 5)
    for cell in {g[0] for g in groups}:  # as many partners as exchanges in each cell
        sel = np.isin(tag, [k for k, g in enumerate(groups) if g[0] == cell])
        assert (part & sel).sum() == ((ev == W.EV_CX) & sel).sum() > 0, cell
    # resonant exchange: the ion is now an atom with its own velocity; nothing moves
    res = (ev == W.EV_CX) & (q0 == 1)
    assert np.all(q1[res] == 0) and res.sum() > 50
    for k in ("x", "y", "z"):
        assert np.array_equal(a[k], st[k])
    assert np.array_equal(a["vz"][res | part], st["vz"][res | part])
    # the exchange probability is the tracked atoms' (Sec. II): n0 Q sigma v dt per ion
    vcell = (2 * p["R0"] / 8) ** 2 * (p["L"] / 16)
    n0 = p["weight"] * 4000 / vcell
    pr = n0 * 3 * p["species"][0]["sigma_cx1"] * 3.0e4 * p["dt"]
    got = int(((ev == W.EV_CX) & (tag == 1)).sum())
    assert abs(got - 3000 * pr) <= 4.5 * math.sqrt(3000 * pr)


def test_partners_are_drawn_uniformly_from_the_cell():
    m = 8
    groups = [((4, 4, 8), 4, 400), ((4, 4, 8), 0, m)]
    p = _params(1, 42)
    st, tag = _cells_state(p, groups, 3.0e4)
    p["n"] = len(tag)
    # a high cross-section: a few exchanges per step among m atoms
    p["species"] = [W.argon(n0_m3=1e20, sigma_cx1_m2=5e-17)]
    picks = np.zeros(m)
    total = 0
    o = OracleSim(p)
    for step in range(600):
        o.set_state(st, step=step)
        o.step(1)
        ev = o.events()
        k = int((ev == W.EV_CX).sum())
        got = ev[tag == 1] == W.EV_CX_PARTNER
        assert got.sum() == min(k, m)
        picks += got
        total += got.sum()
    assert total > 800
    chi2 = float((((picks - total / m) ** 2) / (total / m)).sum())
    assert chi2 < 24.3, (picks, chi2)  # 7 degrees of freedom, p = 0.001


def test_unmatched_exchanges_and_recycled_atoms():
    # one atom at rest and many fast ions: every exchange beyond the first is unmatched
    groups = [((4, 4, 8), 3, 3000), ((4, 4, 8), 0, 1)]
    p = _params(1, 43, species=[W.argon(n0_m3=1e20, sigma_cx1_m2=5e-16)])
    st, tag = _cells_state(p, groups, 3.0e4)
    p["n"] = len(tag)
    o = OracleSim(p)
    o.set_state(st, step=7)
    o.step(1)
    ev, t, a = o.events(), o.tallies(), o.get_state()
    ncx = int((ev == W.EV_CX).sum())
    assert ncx > 5
    assert ev[tag == 1][0] == W.EV_CX_PARTNER and a["q"][tag == 1][0] == 1
    assert t["cx_unmatched"][0] == ncx - 1
    # atoms that reach the wall in this step are recycled, not partners: the
    # cell at the edge of the mesh holds only such atoms (moving out at 1e6
    # m/s) and slow ions; every exchange there is unmatched
    p2 = _params(1, 44, process_mask=W.P_CX | W.P_PUSH, species=[W.argon(n0_m3=1e20, sigma_cx1_m2=2e-15)])
    hx = 2 * p2["R0"] / 8
    ix = 7
    cx, cy, cz = _centre(p2, ix, 4, 8)
    n_ion, n_at = 4000, 200
    x = np.full(n_ion + n_at, cx)
    x[n_ion:] = math.sqrt(p2["R0"] ** 2 - cy ** 2) - 2e-5  # just inside the radial wall, still in cell ix = 7
    assert int((x[n_ion:][0] + p2["R0"]) / hx) == ix
    y = np.full(n_ion + n_at, cy)
    z = np.full(n_ion + n_at, cz)
    vx = np.zeros(n_ion + n_at)
    vx[n_ion:] = 1e6
    vz = np.zeros(n_ion + n_at)
    vz[:n_ion] = 3.0e4
    q = np.zeros(n_ion + n_at, dtype=np.uint8)
    q[:n_ion] = 3
    p2["n"] = n_ion + n_at
    o2 = OracleSim(p2)
    o2.set_state(dict(x=x, y=y, z=z, vx=vx, vy=np.zeros(n_ion + n_at), vz=vz, q=q), step=3)
    o2.step(1)
    ev2, t2 = o2.events(), o2.tallies()
    assert np.all(ev2[n_ion:] == W.EV_WALL)
    ncx2 = int((ev2 == W.EV_CX).sum())
    assert ncx2 > 5
    assert t2["cx_unmatched"][0] == ncx2
    assert not (ev2 == W.EV_CX_PARTNER).any()


def test_switch_needs_tracked_neutrals():
    p = _params(100, 45, self_n0=False)
    with pytest.raises(Exception):
        OracleSim(p)
