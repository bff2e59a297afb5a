"""Pins of the oracle's field model and Boris push (paper Sec. II).

The field pins are closed forms of the analytic minimum-B trap: the on-axis
mirror profile, the hexapole magnitude B_H (r/R0)^2, the paper's polar form
of the hexapole, Maxwell's equations in vacuum (div B = curl B = 0, exact for
a quadratic field under central differences), and the off-axis minimum of
|B| on the midplane.  The push pins are exact discrete properties of the
Boris scheme (gyro-circle radius and phase per step, E x B fixed point, speed
conservation) and the guiding-centre mirror bounce.
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle.binding import OracleSim

E = 1.602176634e-19
AMU = 1.66053906660e-27


def sim(**kw):
    p = W.base_params(4, 8, 8, 16)
    p.update(kw)
    return OracleSim(p), p


def test_axis_profile_and_hexapole_magnitude():
    s, p = sim()
    B0, k, L, R0, BH = p["B0"], p["mirror_k"], p["L"], p["R0"], p["BH"]
    for z in np.linspace(-L / 2, L / 2, 13):
        B = s.field(0.0, 0.0, z)
        assert B[0] == 0.0 and B[1] == 0.0
        assert B[2] == pytest.approx(B0 * (1 + k * (2 * z / L) ** 2), rel=1e-15)
    assert s.field(0, 0, L / 2)[2] == pytest.approx(2.0, rel=1e-15)   # 4 B0 at the flanges
    # midplane: the solenoid has no radial part, the transverse field is the hexapole
    rng = np.random.default_rng(0)
    for _ in range(50):
        r, th = R0 * rng.random(), 2 * np.pi * rng.random()
        B = s.field(r * np.cos(th), r * np.sin(th), 0.0)
        assert math.hypot(B[0], B[1]) == pytest.approx(BH * (r / R0) ** 2, rel=1e-13)
    B = s.field(R0, 0.0, 0.0)
    assert math.hypot(B[0], B[1]) == pytest.approx(1.0, rel=1e-15)


def test_hexapole_matches_polar_form_of_the_paper():
    # Bx = Br cos(th) + BH sin(2 th) R^2/R0^2, By = Br sin(th) + BH cos(2 th) R^2/R0^2,
    # with Br of the solenoid from the derivative of its on-axis profile.
    s, p = sim()
    B0, k, L, R0, BH = p["B0"], p["mirror_k"], p["L"], p["R0"], p["BH"]
    axis = lambda z: B0 * (1 + k * (2 * z / L) ** 2)
    rng = np.random.default_rng(1)
    for _ in range(50):
        r, th, z = R0 * rng.random(), 2 * np.pi * rng.random(), (rng.random() - 0.5) * L
        h = 1e-4
        dBdz = (axis(z + h) - axis(z - h)) / (2 * h)
        Br = -0.5 * r * dBdz
        bx = Br * np.cos(th) + BH * np.sin(2 * th) * r * r / R0**2
        by = Br * np.sin(th) + BH * np.cos(2 * th) * r * r / R0**2
        B = s.field(r * np.cos(th), r * np.sin(th), z)
        assert B[0] == pytest.approx(bx, abs=1e-12)
        assert B[1] == pytest.approx(by, abs=1e-12)


def test_divergence_and_curl_free():
    s, p = sim()
    R0, L = p["R0"], p["L"]
    rng = np.random.default_rng(2)
    h = 1e-4
    for _ in range(40):
        x0 = np.array([(rng.random() - 0.5) * R0, (rng.random() - 0.5) * R0, (rng.random() - 0.5) * L * 0.9])
        J = np.zeros((3, 3))
        for j in range(3):
            d = np.zeros(3)
            d[j] = h
            J[:, j] = (s.field(*(x0 + d)) - s.field(*(x0 - d))) / (2 * h)
        scale = np.abs(J).max()
        assert abs(np.trace(J)) < 1e-9 * scale
        curl = np.array([J[2, 1] - J[1, 2], J[0, 2] - J[2, 0], J[1, 0] - J[0, 1]])
        assert np.abs(curl).max() < 1e-9 * scale


def test_midplane_off_axis_minimum_closed_form():
    # |B|^2 = (B0 - a r^2)^2 + (b r^2)^2 on z = 0 with a = 2 k B0 / L^2, b = BH / R0^2:
    # minimum B0 b / sqrt(a^2 + b^2) at r^2 = a B0 / (a^2 + b^2)  (the shallow ring
    # minimum that the paper describes for sources with a strong radial gradient)
    s, p = sim()
    B0, k, L, R0, BH = p["B0"], p["mirror_k"], p["L"], p["R0"], p["BH"]
    a, b = 2 * k * B0 / L**2, BH / R0**2
    r_star = math.sqrt(a * B0 / (a * a + b * b))
    bmin = B0 * b / math.sqrt(a * a + b * b)
    rs = np.linspace(0, 2 * r_star, 4001)
    mags = np.array([np.linalg.norm(s.field(r * math.cos(0.3), r * math.sin(0.3), 0.0)) for r in rs])
    i = int(np.argmin(mags))
    assert mags[i] == pytest.approx(bmin, rel=1e-9)
    assert rs[i] == pytest.approx(r_star, rel=2e-3)
    assert bmin < B0  # a true off-axis minimum


def uniform(qstate=1, B0=0.5, **kw):
    return sim(B0=B0, mirror_k=0.0, BH=0.0, **kw)


def test_boris_gyro_circle_radius_and_phase():
    s, p = uniform()
    q = 1
    M = 39.948 * AMU
    omega = q * E * p["B0"] / M
    dt = p["dt"]
    # drive the push directly with a large step to make the discrete effects visible
    for wdt in (0.05, 0.4, 1.5):
        s2, p2 = uniform(dt=wdt / omega)
        vperp = 2000.0
        x = np.array([0.0, 0.0, 0.0])
        v = np.array([vperp, 0.0, 37.0])
        theta = 2 * math.atan(wdt / 2)  # exact Boris rotation per step
        R = (vperp / omega) * math.sqrt(1 + (wdt / 2) ** 2)
        pts = []
        for n in range(1, 200):
            x, v = s2.boris(0, q, x, v)
            pts.append(x.copy())
            ang = math.atan2(v[1], v[0])
            want = -(n * theta)  # positive ions turn clockwise about +z
            d = (ang - want + math.pi) % (2 * math.pi) - math.pi
            assert abs(d) < 1e-12 * n + 1e-14
            assert math.hypot(v[0], v[1]) == pytest.approx(vperp, rel=1e-14)
            assert v[2] == 37.0
        pts = np.array(pts)
        # circumcentre of three points, then every point on the circle of radius R
        A, Bp, Cp = pts[0, :2], pts[1, :2], pts[2, :2]
        d = 2 * (A[0] * (Bp[1] - Cp[1]) + Bp[0] * (Cp[1] - A[1]) + Cp[0] * (A[1] - Bp[1]))
        ux = ((A @ A) * (Bp[1] - Cp[1]) + (Bp @ Bp) * (Cp[1] - A[1]) + (Cp @ Cp) * (A[1] - Bp[1])) / d
        uy = ((A @ A) * (Cp[0] - Bp[0]) + (Bp @ Bp) * (A[0] - Cp[0]) + (Cp @ Cp) * (Bp[0] - A[0])) / d
        r = np.hypot(pts[:, 0] - ux, pts[:, 1] - uy)
        assert np.abs(r / R - 1).max() < 1e-9
        assert np.allclose(np.diff(pts[:, 2]), 37.0 * p2["dt"], rtol=1e-12)


def test_boris_exb_drift_is_fixed_point():
    nx, ny, nz = 8, 8, 16
    nodes = (nx + 1) * (ny + 1) * (nz + 1)
    Ex = 300.0
    ef = np.zeros((3, nodes))
    ef[0, :] = Ex
    s, p = uniform(efield=ef)
    vd = np.array([0.0, -Ex / p["B0"], 0.0])  # E x B / B^2
    x = np.array([0.001, 0.002, 0.0])
    v = vd.copy()
    for _ in range(500):
        x, v = s.boris(0, 3, x, v, E=[Ex, 0.0, 0.0])
    assert np.abs(v - vd).max() < 1e-12 * abs(vd[1])


def test_mirror_bounce_period_turning_point_and_trapping():
    # B_H = 0, guiding centre on axis in Bz = B0 (1 + 12 z^2/L^2):
    # harmonic bounce with omega_b = sqrt(12) v_perp0 / L, turning point
    # z_t = (L/sqrt(12)) v_par0/v_perp0; trapped iff sin^2(alpha0) > 1/4.
    L = 0.30
    params = W.base_params(1, 8, 8, 16)
    params.update(BH=0.0, process_mask=W.P_PUSH, dt=1e-8, r_ap=0.0)
    s = OracleSim(params)
    M = 39.948 * AMU
    vperp, vpar = 1.0e4, 0.6e4
    st = dict(x=np.array([0.0]), y=np.array([0.0]), z=np.array([0.0]), vx=np.array([vperp]),
              vy=np.array([0.0]), vz=np.array([vpar]), q=np.array([18], dtype=np.uint8))
    # start on the guiding centre: offset by the Larmor radius
    rl = M * vperp / (18 * E * params["B0"])
    st["y"] = np.array([-rl])  # clockwise gyration about +z starting with +x velocity
    s.set_state(st)
    omega_b = math.sqrt(12) * vperp / L
    T = 2 * math.pi / omega_b
    nsteps = int(2.0 * T / params["dt"])
    zs = []
    for _ in range(nsteps):
        s.step(1)
        zs.append(s.get_state()["z"][0])
    zs = np.array(zs)
    zt = L / math.sqrt(12) * vpar / vperp
    assert zs.max() == pytest.approx(zt, rel=0.02)
    assert -zs.min() == pytest.approx(zt, rel=0.02)
    up = np.nonzero((zs[:-1] < 0) & (zs[1:] >= 0))[0]
    assert len(up) >= 1
    t_first_up = (up[0] + 1) * params["dt"]
    assert t_first_up == pytest.approx(T, rel=0.02)

    # an ion with sin^2(alpha) < 1/4 passes the mirror and leaves through the aperture
    params2 = dict(params)
    params2.update(r_ap=0.01, dt=1e-8)
    s2 = OracleSim(params2)
    st2 = dict(st)
    st2["vx"] = np.array([0.4e4])
    st2["vz"] = np.array([1.0e4])  # sin^2 = 0.16/1.16 < 1/4
    st2["y"] = np.array([-M * 0.4e4 / (18 * E * params["B0"])])
    s2.set_state(st2)
    s2.step(int(0.6 * L / 1.0e4 / params2["dt"]) + 2000)
    assert s2.tallies()["extracted"][0][18] == 1
