"""Pins of the oracle's self-consistent electron density (Sec. II: the
electron density equals the ion charge density, cell by cell; warm electron
rates inside the ECR zone, cold outside).

Ions of chosen charges sit at the centres of chosen cells with atoms beside
them; with ionisation as the only process nothing moves, and each atom of
cell c ionises with probability n_e(c) k dt, where n_e(c) = weight x (sum of
the charges in c) / cell volume follows from quasi-neutrality alone.  The
counts per cell are binomial: checked at 4.5 sigma, and exactly zero in a
cell without ions and outside the zone when the cold rate is zero.
"""
import math

import numpy as np

import workloads as W
from oracle.binding import OracleSim


def _cell_centre(p, ix, iy, iz):
    hx, hy, hz = 2 * p["R0"] / p["nx"], 2 * p["R0"] / p["ny"], p["L"] / p["nz"]
    return -p["R0"] + (ix + 0.5) * hx, -p["R0"] + (iy + 0.5) * hy, -p["L"] / 2 + (iz + 0.5) * hz


def test_ionisation_follows_the_cell_charge():
    # cells: A (8 ions of Q = 1), B (8 ions of Q = 5), C (no ions), D (ions,
    # outside the zone), 12 000 atoms in each; the zone holds A, B and C
    nx, ny, nz = 16, 16, 32
    per = 12_000
    n_ion = 8
    cells = {"A": (8, 8, 16, 1), "B": (7, 8, 16, 5), "C": (8, 7, 16, 0), "D": (8, 8, 30, 3)}
    n = 4 * per + 3 * n_ion
    p = W.base_params(n, nx, ny, nz, seed=3)
    p.update(process_mask=W.P_IONIZE, self_ne=True, weight=1e9, dt=1e-8)
    k = list(p["species"][0]["k_in"])
    p["species"] = [dict(p["species"][0], k_in=[kk * 360 for kk in k], k_out=[0.0] * 32)]
    x, y, z, q, tag = [], [], [], [], []
    for name, (ix, iy, iz, qi) in cells.items():
        cx, cy, cz = _cell_centre(p, ix, iy, iz)
        nions = n_ion if qi else 0
        for i in range(per + nions):
            x.append(cx), y.append(cy), z.append(cz)
            q.append(qi if i < nions else 0)
            tag.append(name)
    x, y, z, q, tag = map(np.array, (x, y, z, q, tag))
    st = dict(x=x, y=y, z=z, vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n), q=q.astype(np.uint8))
    o = OracleSim(p)
    o.set_state(st, step=3)
    o.step(1)
    after = o.get_state()["q"]
    vcell = (2 * p["R0"] / nx) * (2 * p["R0"] / ny) * (p["L"] / nz)
    kdt = p["species"][0]["k_in"][0] * p["dt"]
    for name, (_, _, _, qi) in cells.items():
        atoms = (tag == name) & (q == 0)
        got = int((after[atoms] == 1).sum())
        if name in ("C", "D"):
            assert got == 0, name  # no ions in the cell / cold rate zero outside the zone
            continue
        prob = p["weight"] * (n_ion * qi) / vcell * kdt
        mean, sd = per * prob, math.sqrt(per * prob * (1 - prob))
        assert 0.01 < prob < 0.1
        assert abs(got - mean) <= 4.5 * sd, (name, got, mean, sd)


def test_fixed_background_unchanged_without_the_switch():
    # the same state without the switch ionises every cell's atoms at the
    # fixed background's probability, ions present or not
    p = W.base_params(20_000, 8, 8, 16, seed=1)
    p.update(process_mask=W.P_IONIZE, dt=1e-8, zone_a=0.2, zone_c=0.5, ne_in=1e19)
    st = W.random_state(p, seed=2, q_max=1, frac_atoms=0.5, v_ev=0.0)
    o = OracleSim(p)
    o.set_state(st, step=0)
    o.step(1)
    atoms = st["q"] == 0
    got = int((o.get_state()["q"][atoms] == 1).sum())
    prob = -math.expm1(-p["ne_in"] * p["species"][0]["k_in"][0] * p["dt"])
    m = atoms.sum()
    assert abs(got - m * prob) <= 4.5 * math.sqrt(m * prob * (1 - prob))
