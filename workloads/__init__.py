"""Synthetic ECRIS-shaped workloads and seeded input generators.

This module is the only code shared by the GPU library's tests/benchmark and
the CPU oracle's tests.  It holds parameter presets and seeded random inputs
and none of the method's arithmetic: every derived constant (ionisation
probabilities, Boris factors, collision constants) is computed by each side
from these raw inputs on its own.

Units are SI: metres, seconds, tesla, m^-3, m^3/s, m^2; temperatures and
energies in eV.  The paper's own inputs (Superfish field maps, rate and
cross-section datasets) are not available, so the presets below are
synthetic stand-ins of the same shape (Sec. II of the paper and Table I):
an analytic minimum-B field, a fixed electron background in an ellipsoidal
ECR zone, argon (and oxygen) ions born Q=1.
"""
from __future__ import annotations

import copy
import math

import numpy as np

# process switches (same bit meaning on both sides of the boundary)
P_PUSH = 1
P_IONIZE = 2
P_CX = 4
P_COULOMB = 8
P_DEPOSIT = 16
P_ALL = P_PUSH | P_IONIZE | P_CX | P_COULOMB | P_DEPOSIT
P_HEAT = 32  # electron-ion heating kick (not in P_ALL: the fixed-background step of the benchmark)
P_ELASTIC = 64  # elastic ion-atom scattering (not in P_ALL)
MAXN = 4  # electrons removed by one ionisation, 1..MAXN
EV_ELASTIC = 5
EV_CX_PARTNER = 6  # a tracked atom made an ion as the partner of an exchange

F_ION_N, F_ION_Q, F_ATOM_N, F_ION_P = 0, 1, 2, 3

EV_NONE, EV_IONIZE, EV_CX, EV_WALL, EV_EXTRACT = 0, 1, 2, 3, 4

PREC_FP64, PREC_FP32 = 0, 1

# Ionisation potentials in eV of Ar^Q+ and O^Q+ (NIST atomic spectra database,
# ground states).  Used only to shape the synthetic rate table below.
AR_IP_EV = [15.760, 27.630, 40.735, 59.58, 74.84, 91.29, 124.41, 143.457, 422.60,
            479.76, 540.4, 619.0, 685.5, 755.13, 855.5, 918.375, 4120.666, 4426.224]
O_IP_EV = [13.618, 35.121, 54.936, 77.414, 113.899, 138.120, 739.293, 871.410]

K0_CM3S = 1.0e-7  # Ar0 -> Ar1+ rate at keV electron temperature quoted in Sec. III.B


def synthetic_rates(ip_ev, k0_cm3s=K0_CM3S, exponent=1.5):
    """Synthetic single-ionisation rate table in m^3/s, one entry per Q.

    The paper's rates come from datasets that are not available here.  This
    stand-in is anchored at k(Q=0) = k0 and falls with the ionisation
    potential as (I_0/I_Q)^1.5; the entry at Q = z_max is 0.  It is a stated
    synthetic input, not physics data.
    """
    z_max = len(ip_ev)
    k = [0.0] * 32
    for q in range(z_max):
        k[q] = k0_cm3s * 1e-6 * (ip_ev[0] / ip_ev[q]) ** exponent
    return k


SIGMA_CX1_M2 = 5.0e-19  # synthetic Ar+ + Ar charge-exchange cross-section (5e-15 cm^2)


def te_scaled(k, ip_ev, te_ev, te_ref_ev=1000.0):
    """The synthetic rate table k (given at te_ref_ev) moved to electron
    temperature te_ev with the temperature shape of a Maxwellian-averaged
    Lotz-type cross-section, k_Q ~ T^-1/2 E1(I_Q / T).  A stated synthetic
    input; the identity at te_ev == te_ref_ev."""
    if te_ev == te_ref_ev:
        return list(k)
    from scipy.special import exp1
    out = list(k)
    for q, ip in enumerate(ip_ev):
        out[q] = k[q] * math.sqrt(te_ref_ev / te_ev) * float(exp1(ip / te_ev) / exp1(ip / te_ref_ev))
    return out


MULTI_RATIOS = (0.10, 0.02, 0.005)  # synthetic k(Q -> Q+n) / k(Q -> Q+1) for n = 2, 3, 4
SIGMA_EL1_M2 = 3.0e-19  # synthetic elastic Ar+ + Ar cross-section (3e-15 cm^2)


def with_extended_mcc(species, ratios=MULTI_RATIOS, sigma_el1_m2=SIGMA_EL1_M2):
    """The species with multiple ionisation and elastic ion-atom scattering.

    The paper takes double ionisation from a fit and n >= 3 from a scaling
    law (datasets not available here); this stand-in sets k(Q -> Q+n) to a
    fixed fraction of the single rate k(Q -> Q+1), zero where Q + n passes
    z_max, and the elastic cross-section of Q = 1 to a synthetic value.
    Stated synthetic inputs, not physics data."""
    sp = dict(species)
    z = sp["z_max"]
    for key, src in (("k_multi_in", "k_in"), ("k_multi_out", "k_out")):
        sp[key] = [[sp[src][q] * r if q + n <= z else 0.0 for q in range(32)] for n, r in zip((2, 3, 4), ratios)]
    sp["sigma_el1"] = sigma_el1_m2
    return sp


def argon(fraction=1.0, n0_m3=1.0e17, sigma_cx1_m2=SIGMA_CX1_M2, outside_rates=False, te_ev=1000.0):
    k = te_scaled(synthetic_rates(AR_IP_EV), AR_IP_EV, te_ev)
    return dict(mass_amu=39.948, z_max=18, cx_forbidden_mask=1 << 2, fraction=fraction,
                k_in=k, k_out=(list(k) if outside_rates else [0.0] * 32),
                sigma_cx1=sigma_cx1_m2, n0=n0_m3)


def oxygen(fraction=1.0, n0_m3=1.0e17, sigma_cx1_m2=SIGMA_CX1_M2, outside_rates=False, te_ev=1000.0):
    k = te_scaled(synthetic_rates(O_IP_EV, k0_cm3s=K0_CM3S * (O_IP_EV[0] / AR_IP_EV[0]) ** -1.5), O_IP_EV, te_ev)
    return dict(mass_amu=15.999, z_max=8, cx_forbidden_mask=0, fraction=fraction,
                k_in=k, k_out=(list(k) if outside_rates else [0.0] * 32),
                sigma_cx1=sigma_cx1_m2, n0=n0_m3)


def base_params(n, nx, ny, nz, seed=0, precision=PREC_FP64):
    """Shared geometry and plasma of every preset (a KVI-AECRIS-sized source)."""
    R0 = 0.035
    return dict(
        precision=precision, process_mask=P_ALL, deposit_mask=(1 << F_ION_N) | (1 << F_ION_Q),
        seed=seed, n=n, dt=1.0e-9, sort_every=50, nx=nx, ny=ny, nz=nz,
        R0=R0, L=0.30, r_ap=0.01, inlet_x=R0 / 2, inlet_y=0.0,
        B0=0.5, mirror_k=3.0, BH=1.0,
        zone_a=0.015, zone_c=0.05, ne_in=1.0e18, ne_out=0.0, Te_in_eV=1000.0, Te_out_eV=5.0,
        Ti0_eV=0.5, T_wall_eV=0.025, T_n_eV=0.025, dE_cx_eV=10.0, lnL=10.0, lnL_ei=17.0, weight=0.0,
        efield=None, species=[argon()], self_ne=False)


def config(name):
    """Named workloads.  Returns (params, steps)."""
    name = name.lower()
    if name == "c1":   # 20k Ar ions, FP64, grid 32x32x64, 1000 steps
        return base_params(20_000, 32, 32, 64), 1000
    if name == "c2":   # 2M Ar ions, FP64, grid 64x64x128, 10k steps, sort every 50
        return base_params(2_000_000, 64, 64, 128), 10_000
    if name == "c3":   # c1 in FP32 push with FP64 accumulators, 10k steps
        return base_params(20_000, 32, 32, 64, precision=PREC_FP32), 10_000
    if name == "c4":   # 10M two-species (70% O, 30% Ar), n0 = 3e11 cm^-3 split 70/30
        p = base_params(10_000_000, 128, 128, 256, precision=PREC_FP32)
        p["species"] = [oxygen(0.7, n0_m3=0.7 * 3e17), argon(0.3, n0_m3=0.3 * 3e17)]
        return p, 5000
    raise KeyError(name)


def c5_trace(n_requests=256, rate_hz=20.0, seed=0, precision=PREC_FP32, steps=2000, n_lo=10_000, n_hi=2_000_000):
    """The serving workload: a parameter scan of n_requests argon runs.

    Drawn in this order from numpy.default_rng(seed), all arrays of length
    n_requests: exponential inter-arrival gaps of mean 1/rate_hz (arrival =
    running sum); particle count log-uniform in [n_lo, n_hi] (gas load);
    neutral density uniform in 3e10..3e11 cm^-3 (gas flow); one power draw u
    uniform in [0, 1) giving T_e = 0.3 + 2.7u keV and n_e = (0.3 + 2.2u)e12
    cm^-3 in the zone (microwave power).  Each run: grid 64x64x128, sort every
    50 steps, seed = request index, weight n_e V_zone / N.
    Returns a list of (arrival_s, params, steps).
    """
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_hz, n_requests)
    counts = np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), n_requests)).astype(np.int64)
    n0_cm3 = rng.uniform(3e10, 3e11, n_requests)
    u = rng.uniform(0.0, 1.0, n_requests)
    arrival = np.cumsum(gaps)
    out = []
    for i in range(n_requests):
        te_ev = (0.3 + 2.7 * u[i]) * 1e3
        p = base_params(int(counts[i]), 64, 64, 128, seed=i, precision=precision)
        p.update(ne_in=(0.3 + 2.2 * u[i]) * 1e18, Te_in_eV=te_ev)
        p["species"] = [argon(n0_m3=n0_cm3[i] * 1e6, te_ev=te_ev)]
        out.append((float(arrival[i]), p, steps))
    return out


def with_(params, **kw):
    q = copy.deepcopy(params)
    q.update(kw)
    return q


def random_state(params, seed, q_max=None, frac_atoms=0.1, v_ev=0.5, radius_frac=0.95, mass_amu=39.948,
                 birth_max=None):
    """Seeded synthetic particle state, indexed by particle id.

    Positions uniform in the cylinder r < radius_frac R0, |z| < radius_frac L/2;
    velocities Maxwellian with sigma = sqrt(v_ev e / m) for a mass of mass_amu;
    charge states uniform in [1, q_max] (default: the smallest z_max of the
    species), then a fraction frac_atoms set to Q = 0.  With birth_max, the
    ions get birth steps uniform in [0, birth_max] (atoms 0xFFFFFFFF).
    """
    rng = np.random.default_rng(seed)
    n = params["n"]
    R0, L = params["R0"], params["L"]
    r = radius_frac * R0 * np.sqrt(rng.random(n))
    th = 2 * np.pi * rng.random(n)
    x = r * np.cos(th)
    y = r * np.sin(th)
    z = (rng.random(n) * 2 - 1) * radius_frac * L / 2
    sig = math.sqrt(v_ev * 1.602176634e-19 / (mass_amu * 1.66053906660e-27))
    vx = rng.normal(size=n) * sig
    vy = rng.normal(size=n) * sig
    vz = rng.normal(size=n) * sig
    qm = min(s["z_max"] for s in params["species"]) if q_max is None else q_max
    q = (1 + np.floor(rng.random(n) * qm)).astype(np.uint8)
    q[rng.random(n) < frac_atoms] = 0
    out = dict(x=x, y=y, z=z, vx=vx, vy=vy, vz=vz, q=q)
    if birth_max is not None:
        b = rng.integers(0, birth_max + 1, n).astype(np.uint32)
        out["birth"] = np.where(q >= 1, b, np.uint32(0xFFFFFFFF)).astype(np.uint32)
    return out
