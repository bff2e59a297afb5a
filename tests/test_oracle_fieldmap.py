"""Pins of the oracle's magnetic field maps (a node grid of B, as a field
solver such as the paper's Superfish writes it, interpolated trilinearly).

* Trilinear interpolation reproduces an affine field exactly: a map of
  B(x) = B0 + A x, laid out [component][node] with x fastest, then y, then
  z, must return the affine formula at random points to rounding (a swapped
  axis, component or node stride fails at once).
* A map of a uniform field gives the orbits of the analytic uniform field
  (solenoid and hexapole coefficients zero) to rounding.
* The heating kick reads |B| at the cell centre from the map.
"""
import numpy as np

import workloads as W
from oracle.binding import OracleSim


def _nodes(p):
    nx, ny, nz = p["nx"], p["ny"], p["nz"]
    xs = -p["R0"] + np.arange(nx + 1) * (2 * p["R0"] / nx)
    ys = -p["R0"] + np.arange(ny + 1) * (2 * p["R0"] / ny)
    zs = -p["L"] / 2 + np.arange(nz + 1) * (p["L"] / nz)
    Z, Y, X = np.meshgrid(zs, ys, xs, indexing="ij")  # node index = ix + (nx+1)(iy + (ny+1) iz)
    return X.ravel(), Y.ravel(), Z.ravel()


def test_affine_map_is_reproduced_exactly():
    p = W.base_params(10, 6, 5, 7)
    X, Y, Z = _nodes(p)
    B0 = np.array([0.1, -0.2, 0.6])
    A = np.array([[1.0, 2.0, -0.5], [-3.0, 0.5, 1.5], [0.25, -1.0, 2.0]])
    grid = np.stack([B0[c] + A[c, 0] * X + A[c, 1] * Y + A[c, 2] * Z for c in range(3)])
    o = OracleSim(dict(p, bfield=grid))
    rng = np.random.default_rng(1)
    for _ in range(200):
        x, y = rng.uniform(-p["R0"], p["R0"], 2)
        z = rng.uniform(-p["L"] / 2, p["L"] / 2)
        got = np.array(o.field(x, y, z))
        want = B0 + A @ np.array([x, y, z])
        assert np.abs(got - want).max() <= 1e-13 * (1 + np.abs(want).max()), (x, y, z, got, want)
    # without a map the analytic field is back
    o2 = OracleSim(p)
    assert not np.allclose(o2.field(0.01, 0.0, 0.05), o.field(0.01, 0.0, 0.05))


def test_uniform_map_orbits_match_the_analytic_uniform_field():
    p = W.base_params(2000, 8, 8, 16, seed=2)
    p.update(process_mask=W.P_PUSH, mirror_k=0.0, BH=0.0, B0=0.7, dt=2e-9)
    st = W.random_state(p, seed=3, q_max=8, v_ev=5.0, radius_frac=0.5)
    nn = (p["nx"] + 1) * (p["ny"] + 1) * (p["nz"] + 1)
    grid = np.zeros((3, nn))
    grid[2] = 0.7
    a, b = OracleSim(p), OracleSim(dict(p, bfield=grid))
    for o in (a, b):
        o.set_state(st, step=0)
        o.step(100)
    sa, sb = a.get_state(), b.get_state()
    assert np.array_equal(a.events(), b.events())
    for k in ("x", "y", "z", "vx", "vy", "vz"):
        scale = p["R0"] if k in "xyz" else 1e3
        assert np.abs(sa[k] - sb[k]).max() <= 1e-12 * max(scale, np.abs(sa[k]).max()), k
    assert np.abs(sa["x"] - st["x"]).max() > 1e-4  # the ions did gyrate


def test_heating_kick_reads_the_map():
    # the kick's bias scales as 1/|B| at the cell centre: a uniform map of
    # twice the field halves the mean drift of a linear density ramp
    import math
    from test_oracle_heating import _gradient_state, _uniform_b
    p = _uniform_b(W.base_params(1, 16, 16, 16, seed=12))
    p.update(process_mask=W.P_HEAT, self_ne=True, zone_a=1.0, zone_c=1.0, dt=1e-8, weight=2e9,
             Te_in_eV=4000.0, B0=0.25)
    st, cells = _gradient_state(p, 20, 6, range(2, 14), 40)
    p["n"] = len(st["x"])
    nn = 17 * 17 * 17
    means = []
    for b in (None, 0.5):
        q = dict(p)
        if b is not None:
            g = np.zeros((3, nn))
            g[2] = b
            q["bfield"] = g
        o = OracleSim(q)
        o.set_state(st, step=3)
        o.step(1)
        sel = (cells[:, 0] >= 3) & (cells[:, 0] <= 12) & (cells[:, 1] >= 3) & (cells[:, 1] <= 12)
        means.append(o.get_state()["vy"][sel].mean())
    assert means[0] < 0 and means[1] < 0
    assert math.isclose(means[1] / means[0], 0.5, rel_tol=0.08)
