"""Pins of the oracle's tracked-neutral option (Sec. II: atoms are tracked
macro-particles; their local density is the target of charge exchange and
elastic ion-atom scattering).

Ions of one charge move at one speed v0 through cells that hold chosen
numbers of atoms; with exchange and elastic scattering the only processes
nothing moves, so each ion of cell c exchanges with probability
n0(c) Q sigma1 v0 dt and scatters with n0(c) Q sigma_el v0 dt, where
n0(c) = weight x (atoms of the ion's species in c) / cell volume.  The
counts are binomial (checked at 4.5 sigma); a cell whose atoms are all of
another species has none, however large the species' uniform n0; without
the switch the uniform n0 applies everywhere.
"""
import math

import numpy as np

import workloads as W
from oracle.binding import OracleSim

E = 1.602176634e-19
AMU = 1.66053906660e-27


def _centre(p, ix, iy, iz):
    hx, hy, hz = 2 * p["R0"] / p["nx"], 2 * p["R0"] / p["ny"], p["L"] / p["nz"]
    return -p["R0"] + (ix + 0.5) * hx, -p["R0"] + (iy + 0.5) * hy, -p["L"] / 2 + (iz + 0.5) * hz


def _setup(self_n0):
    nx, ny, nz = 8, 8, 16
    n_ion, Q = 6000, 3
    # species 0 (argon): cells A, B, C, D with these atom counts; species 1
    # (oxygen) puts its atoms in D only
    atoms0 = {"A": 1500, "B": 500, "C": 0, "D": 0}
    cells = {"A": (4, 4, 8), "B": (3, 4, 8), "C": (4, 3, 8), "D": (3, 3, 8)}
    n_o = 1500
    n0_total = sum(n_ion + a for a in atoms0.values())
    n = n0_total + n_o
    p = W.base_params(n, nx, ny, nz, seed=31)
    ar = W.with_extended_mcc(W.argon(fraction=n0_total / n, n0_m3=1e21))
    ox = W.oxygen(fraction=1 - n0_total / n, n0_m3=1e21)
    p.update(process_mask=W.P_CX | W.P_ELASTIC, dt=2e-9, weight=2e11, self_n0=self_n0, T_n_eV=1e-6, species=[ar, ox])
    m = ar["mass_amu"] * AMU
    v0 = math.sqrt(2 * 100.0 * E / m)
    x, y, z, vz, q, tag = [], [], [], [], [], []
    for name, (ix, iy, iz) in cells.items():
        cx, cy, cz = _centre(p, ix, iy, iz)
        for i in range(n_ion + atoms0[name]):
            ion = i < n_ion
            x.append(cx), y.append(cy), z.append(cz)
            vz.append(v0 if ion else 0.0)
            q.append(Q if ion else 0)
            tag.append(name if ion else "-")
    cx, cy, cz = _centre(p, *cells["D"])
    for _ in range(n_o):
        x.append(cx), y.append(cy), z.append(cz), vz.append(0.0), q.append(0), tag.append("o")
    zeros = np.zeros(n)
    st = dict(x=np.array(x), y=np.array(y), z=np.array(z), vx=zeros.copy(), vy=zeros.copy(), vz=np.array(vz),
              q=np.array(q, dtype=np.uint8))
    return p, st, np.array(tag), atoms0, v0, Q


def test_collision_rates_follow_the_cell_atoms():
    p, st, tag, atoms0, v0, Q = _setup(True)
    o = OracleSim(p)
    o.set_state(st, step=2)
    o.step(1)
    ev = o.events()
    vcell = (2 * p["R0"] / p["nx"]) * (2 * p["R0"] / p["ny"]) * (p["L"] / p["nz"])
    sp = p["species"][0]
    for name, na in atoms0.items():
        sel = tag == name
        n0c = p["weight"] * na / vcell
        for code, sigma in ((W.EV_CX, sp["sigma_cx1"]), (W.EV_ELASTIC, sp["sigma_el1"])):
            prob = n0c * Q * sigma * v0 * p["dt"]
            got = int((ev[sel] == code).sum())
            if na == 0:
                assert got == 0, (name, code)  # no atoms of the ion's species in the cell
                continue
            assert 0.002 < prob < 0.1, (name, code, prob)
            m = sel.sum()
            assert abs(got - m * prob) <= 4.5 * math.sqrt(m * prob * (1 - prob)), (name, code, got, m * prob)
    assert not (ev[(tag == "-") | (tag == "o")] != W.EV_NONE).any()  # atoms never collide with atoms


def test_uniform_background_without_the_switch():
    p, st, tag, atoms0, v0, Q = _setup(False)
    o = OracleSim(p)
    o.set_state(st, step=2)
    o.step(1)
    ev = o.events()
    sel = tag == "C"  # no atoms here, but the uniform n0 applies
    prob = p["species"][0]["n0"] * Q * p["species"][0]["sigma_cx1"] * v0 * p["dt"]
    got = int((ev[sel] == W.EV_CX).sum())
    assert abs(got - sel.sum() * prob) <= 4.5 * math.sqrt(sel.sum() * prob)
