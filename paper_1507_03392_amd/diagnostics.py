"""Physical outputs of a run from its tallies and density grids (host side).

The paper reports the extracted charge-state distribution as currents, the
gas flow in particle-milliamperes, the mean radial size of the extracted
beam, first-passage times of the extracted ions, the coupled power from the
power balance, and ion pressure and temperature along the axis (Sec. II,
III.B-III.D).  The library tallies the raw sums; these functions scale them.
All inputs are the dicts returned by Run.tallies() and Run.density(), the
macro-particle weight (Run.weight) and the time step; outputs are SI unless
the name says otherwise.
"""
from __future__ import annotations

import numpy as np

E_CHARGE = 1.602176634e-19


def _duration(t, dt):
    if t["steps"] <= 0:
        raise ValueError("no steps in these tallies")
    return t["steps"] * dt


def extracted_currents(t, weight, dt, species=0):
    """Extracted current per charge state Q (A): Q e w count_Q / time."""
    q = np.arange(t["extracted"].shape[1])
    return q * E_CHARGE * weight * t["extracted"][species].astype(np.float64) / _duration(t, dt)


def gas_flow_pmA(t, weight, dt):
    """Particle flux through the aperture in pmA (1 pmA: the particle flux of
    1 mA of singly charged ions), every species and charge, atoms included."""
    return E_CHARGE * weight * float(t["extracted"].sum()) / _duration(t, dt) / 1e-3


def mean_extraction_radius(t, species=0):
    """Mean sqrt(x^2 + y^2) of the extracted particles where they cross the
    flange, per Q (m; NaN where none)."""
    n = t["extracted"][species].astype(np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(n > 0, t["extracted_r"][species] / n, np.nan)


def mean_first_passage(t, dt, species=0):
    """Mean first-passage time of the extracted ions of known birth, per Q (s)."""
    n = t["fpt_n"][species].astype(np.float64)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(n > 0, t["fpt_sum"][species].astype(np.float64) * dt / n, np.nan)


def first_passage_histogram(t, dt, species=0):
    """Histogram of first-passage times (all charges): bin k holds times in
    [2^k, 2^(k+1)) steps (bin 0 also 0 and 1 step).  Returns (lower edges in
    s, upper edges in s, counts)."""
    k = np.arange(t["fpt_hist"].shape[1])
    lo = np.where(k == 0, 0.0, 2.0 ** k) * dt
    return lo, 2.0 ** (k + 1) * dt, t["fpt_hist"][species].astype(np.int64)


def coupled_power(t, weight, dt, te_warm_ev, ip_ev, species=0):
    """Microwave power coupled to the plasma from the power balance (W): per
    unit time, the kinetic energy of the lost ions, their potential energy
    (the sum of the ionisation potentials up to their charge) and 3/2 k T_ew
    for each electron lost with them (one per unit of lost charge).  ip_ev:
    ionisation potentials of the species, Q = 0 -> 1 first."""
    lost = (t["extracted"][species] + t["wall"][species]).astype(np.float64)
    q = np.arange(lost.size)
    pe = np.concatenate([[0.0], np.cumsum(np.asarray(ip_ev, dtype=np.float64))])
    pe = np.pad(pe, (0, max(0, lost.size - pe.size)), mode="edge")[:lost.size] * E_CHARGE
    energy = t["lost_ke"][species] + (lost * pe).sum() + 1.5 * te_warm_ev * E_CHARGE * (q * lost).sum()
    return weight * energy / _duration(t, dt)


def axis_profiles(params, n_field, p_field, steps, weight):
    """Ion density (m^-3), pressure (Pa) and mean temperature (eV) along the
    source axis: the node column nearest x = y = 0 of the time-integrated
    ion-number and ion-pressure grids, divided by the node volume and the
    number of steps.  Returns (z, n, P, T)."""
    nx, ny, nz = params["nx"], params["ny"], params["nz"]
    R0, L = params["R0"], params["L"]
    vol = (2 * R0 / nx) * (2 * R0 / ny) * (L / nz)
    grid_n = np.asarray(n_field).reshape(nz + 1, ny + 1, nx + 1)
    grid_p = np.asarray(p_field).reshape(nz + 1, ny + 1, nx + 1)
    ix, iy = round(nx / 2), round(ny / 2)
    scale = weight / (vol * steps)
    n = grid_n[:, iy, ix] * scale
    p = grid_p[:, iy, ix] * scale
    with np.errstate(invalid="ignore", divide="ignore"):
        temp = np.where(n > 0, p / n / E_CHARGE, np.nan)
    z = -L / 2 + np.arange(nz + 1) * (L / nz)
    return z, n, p, temp
