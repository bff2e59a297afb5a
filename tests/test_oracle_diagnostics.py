"""Pins of the oracle's loss and extracted-ion diagnostics.

* Birth steps (Sec. III.D: an ion's first-passage time runs from the moment
  it was made by ionising an atom): after one step from a mixed state, every
  particle's birth follows from its event and its charge before the step,
  worked out here independently (ionisation of Q = 0 and resonant Q = 1
  charge exchange set it to the step; a wall or the aperture clears it;
  anything else leaves it).
* First-passage tallies: count, sum and log2 histogram of (step - birth) over
  the extracted ions equal the brute-force sums over the event log.
* Radial size of the extracted beam (Sec. III.B, mean of sqrt(x^2 + y^2) at
  the aperture): for atoms, which move in straight lines, the crossing point
  of the flange is a closed form.
* Lost kinetic energy (the power balance of Sec. II): the Boris rotation
  keeps |v| with no electric field, so each ion lost in a step carries
  1/2 M |v|^2 of its state before the step.
* Ion pressure moment (Sec. III.B, P = sum_Q n_Q T_Q): the optional field
  equals the brute-force tent sums of M |v|^2 / 3, and for the Maxwellian
  initial ions its total over the ion number is k T_i0.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle.binding import BIRTH_NONE, OracleSim

AMU = 1.66053906660e-27


def _mixed(n, seed, step0, **kw):
    p = W.base_params(n, 16, 16, 32, seed=seed)
    p.update(process_mask=W.P_ALL, dt=5e-9, zone_a=0.03, zone_c=0.14, ne_in=1e20)
    p["species"] = [dict(p["species"][0], n0=1e20)]
    p.update(kw)
    st = W.random_state(p, seed=seed + 50, q_max=10, v_ev=200.0, radius_frac=0.9995, frac_atoms=0.3)
    rng = np.random.default_rng(seed)
    st["birth"] = np.where(st["q"] >= 1, rng.integers(0, step0 + 1, n), BIRTH_NONE).astype(np.uint32)
    return p, st


def test_birth_steps_follow_the_events():
    step0 = 40
    p, st = _mixed(20_000, 1, step0)
    o = OracleSim(p)
    o.set_state(st, step=step0)
    o.step(1)
    ev, b = o.events(), o.get_state()["birth"]
    q0, b0 = st["q"], st["birth"]
    expect = b0.copy()
    made = ((ev == W.EV_IONIZE) & (q0 == 0)) | ((ev == W.EV_CX) & (q0 == 1))
    expect[made] = step0
    expect[(ev == W.EV_WALL) | (ev == W.EV_EXTRACT)] = BIRTH_NONE
    assert np.array_equal(b, expect)
    # every case occurred
    assert ((ev == W.EV_IONIZE) & (q0 == 0)).sum() > 20 and ((ev == W.EV_IONIZE) & (q0 >= 1)).sum() > 20
    assert ((ev == W.EV_CX) & (q0 == 1)).sum() > 5 and ((ev == W.EV_CX) & (q0 >= 2)).sum() > 5
    assert (ev == W.EV_WALL).sum() > 20
    # atoms never carry a birth
    assert np.all(b[o.get_state()["q"] == 0] == BIRTH_NONE)


def _extraction_state(n, seed, step0):
    p = W.base_params(n, 16, 16, 32, seed=seed)
    p.update(process_mask=W.P_ALL, dt=2e-9)
    rng = np.random.default_rng(seed)
    r = 1.2 * p["r_ap"] * np.sqrt(rng.random(n))
    th = 2 * np.pi * rng.random(n)
    st = dict(x=r * np.cos(th), y=r * np.sin(th), z=p["L"] / 2 - rng.random(n) * 3e-5,
              vx=rng.normal(size=n) * 300, vy=rng.normal(size=n) * 300, vz=np.abs(rng.normal(size=n)) * 2e4 + 2e4,
              q=rng.integers(0, 9, n).astype(np.uint8))
    birth = rng.integers(0, step0 + 1, n).astype(np.uint32)
    birth[rng.random(n) < 0.2] = BIRTH_NONE  # ions of unknown origin are left out of the first-passage tallies
    st["birth"] = np.where(st["q"] >= 1, birth, BIRTH_NONE).astype(np.uint32)
    return p, st


def test_first_passage_tallies_brute_force():
    step0 = 5000
    p, st = _extraction_state(8000, 3, step0)
    o = OracleSim(p)
    o.set_state(st, step=step0)
    o.step(1)
    ev, t = o.events(), o.tallies()
    n_exp = np.zeros((4, 32), dtype=np.uint64)
    s_exp = np.zeros((4, 32), dtype=np.uint64)
    h_exp = np.zeros((4, 32), dtype=np.uint64)
    for i in np.nonzero(ev == W.EV_EXTRACT)[0]:
        q, b = int(st["q"][i]), int(st["birth"][i])
        if q >= 1 and b != BIRTH_NONE:
            d = step0 - b
            n_exp[0][q] += 1
            s_exp[0][q] += d
            h_exp[0][max(d.bit_length() - 1, 0)] += 1
    assert n_exp.sum() > 1000 and (ev == W.EV_EXTRACT).sum() > n_exp.sum()
    assert np.array_equal(t["fpt_n"], n_exp)
    assert np.array_equal(t["fpt_sum"], s_exp)
    assert np.array_equal(t["fpt_hist"], h_exp)
    assert t["fpt_hist"].sum() == t["fpt_n"].sum()


def test_extracted_radius_of_atoms_closed_form():
    p, st = _extraction_state(6000, 4, 100)
    st["q"][:] = 0  # atoms: straight lines
    st["birth"][:] = BIRTH_NONE
    p["process_mask"] = W.P_PUSH
    o = OracleSim(p)
    o.set_state(st, step=100)
    o.step(1)
    ev, t = o.events(), o.tallies()
    ext = ev == W.EV_EXTRACT
    f = (p["L"] / 2 - st["z"]) / (st["vz"] * p["dt"])
    xc, yc = st["x"] + f * st["vx"] * p["dt"], st["y"] + f * st["vy"] * p["dt"]
    rc = np.hypot(xc, yc)
    assert np.array_equal(ext, rc <= p["r_ap"])
    assert ext.sum() > 1000 and t["extracted"][0][0] == ext.sum()
    assert math.isclose(t["extracted_r"][0][0], rc[ext].sum(), rel_tol=1e-12)
    assert np.all(t["extracted_r"][0][1:] == 0) and np.all(t["lost_ke"] == 0)  # atoms only


def test_lost_kinetic_energy_of_ions():
    step0 = 7
    p, st = _mixed(20_000, 2, step0, process_mask=W.P_PUSH, dt=2e-8)
    o = OracleSim(p)
    o.set_state(st, step=step0)
    o.step(1)
    ev, t = o.events(), o.tallies()
    lost = ((ev == W.EV_WALL) | (ev == W.EV_EXTRACT)) & (st["q"] >= 1)
    assert lost.sum() > 100
    v2 = st["vx"] ** 2 + st["vy"] ** 2 + st["vz"] ** 2
    ke = 0.5 * p["species"][0]["mass_amu"] * AMU * v2[lost].sum()
    assert math.isclose(t["lost_ke"][0], ke, rel_tol=1e-12)


def test_ion_pressure_field_brute_force_and_equipartition():
    # field 3: sum over ions of CIC weight x M |v|^2 / 3; with a Maxwellian at
    # T its total over the nodes is N k T (the CIC weights of a particle sum
    # to 1), so total pressure moment / total ion number = k T
    p = W.base_params(20_000, 8, 8, 16, seed=6)
    p.update(process_mask=W.P_DEPOSIT, deposit_mask=(1 << W.F_ION_N) | (1 << W.F_ION_P))
    o = OracleSim(p)
    o.init_ions()
    o.step(1)
    st = o.get_state()
    dp, steps = o.density(W.F_ION_P)
    dn, _ = o.density(W.F_ION_N)
    assert steps == 1
    m = p["species"][0]["mass_amu"] * AMU
    e = m * (st["vx"] ** 2 + st["vy"] ** 2 + st["vz"] ** 2) / 3.0
    # brute force: every node's tent-function sum
    R0, hL, nx, ny, nz = p["R0"], p["L"] / 2, p["nx"], p["ny"], p["nz"]
    gx = (st["x"] + R0) * nx / (2 * R0)
    gy = (st["y"] + R0) * ny / (2 * R0)
    gz = (st["z"] + hL) * nz / (2 * hL)
    brute = np.zeros((nz + 1, ny + 1, nx + 1))
    for i in range(len(e)):
        ix, iy, iz = min(int(gx[i]), nx - 1), min(int(gy[i]), ny - 1), min(int(gz[i]), nz - 1)
        tx, ty, tz = gx[i] - ix, gy[i] - iy, gz[i] - iz
        for dz, wz in ((0, 1 - tz), (1, tz)):
            for dy, wy in ((0, 1 - ty), (1, ty)):
                for dx, wx in ((0, 1 - tx), (1, tx)):
                    brute[iz + dz, iy + dy, ix + dx] += wx * wy * wz * e[i]
    assert np.abs(dp - brute.ravel()).max() <= 1e-9 * np.abs(brute).max()
    kT = p["Ti0_eV"] * 1.602176634e-19
    assert dn.sum() == pytest.approx(20_000, rel=1e-12)
    assert dp.sum() / dn.sum() == pytest.approx(kT, rel=0.02)
