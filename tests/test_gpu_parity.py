"""Parity of the HIP library (through its C ABI) with the FP64 CPU oracle.

Bar (binary64 path): from identical input state, per-step event codes,
charge states and integer tallies are bit-exact; positions agree within
1e-12 relative to max(|x|, R0) and velocities within 1e-12 relative to
max(|v|, 1 km/s); density grids within 1e-12 of the largest node value.
Sizes span several workgroups with a ragged tail; the full-size case runs
2M ions in the benchmark's launch configuration and checks whole sampled
collision cells against the oracle.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

XTOL = 1e-12
VSCALE = 1e3


def gpu_run(params, **kw):
    import paper_1507_03392_amd as ecr
    return ecr.Run(params, **kw)


def oracle(params):
    from oracle.binding import OracleSim
    return OracleSim(params)


def assert_state_close(a, b, params, ids=None, what="", tol=XTOL):
    sel = slice(None) if ids is None else ids
    assert np.array_equal(a["q"][sel], b["q"]), f"{what}: charge states differ"
    for k in ("x", "y", "z"):
        d = np.abs(a[k][sel] - b[k]) / np.maximum(np.abs(b[k]), params["R0"])
        assert d.max(initial=0) <= tol, f"{what}: {k} rel err {d.max()}"
    for k in ("vx", "vy", "vz"):
        d = np.abs(a[k][sel] - b[k]) / np.maximum(np.abs(b[k]), VSCALE)
        assert d.max(initial=0) <= tol, f"{what}: {k} rel err {d.max()}"
    assert np.array_equal(a["birth"][sel], b["birth"]), f"{what}: birth steps differ"


def assert_tallies_equal(tg, to, what=""):
    for k in ("extracted", "wall", "ionized", "cx", "cx_products", "fpt_n", "fpt_sum", "fpt_hist", "ionized_n", "elastic",
              "cx_unmatched"):
        assert np.array_equal(tg[k], to[k]), f"{what}: tally {k} differs"
    for k in ("recycled", "anomalies", "steps"):
        assert tg[k] == to[k], f"{what}: {k} {tg[k]} vs {to[k]}"
    # FP64 sums gathered with atomics: the order differs, the terms do not
    for k in ("extracted_r", "lost_ke"):
        np.testing.assert_allclose(tg[k], to[k], rtol=1e-12, atol=1e-300, err_msg=f"{what}: {k}")


def boosted(params, n0=2e19):
    p = W.with_(params)
    sp = dict(p["species"][0])
    sp["n0"] = n0
    p["species"] = [sp]
    return p


def run_pair(params, st, steps, step0=0, cell=None):
    g = gpu_run(params, events=True)
    g.set_state(st, step=step0, cell=cell)
    g.step(steps)
    o = oracle(params)
    o.set_state(st, step=step0, cell=cell)
    o.step(steps)
    return g, o


def test_philox_bitwise():
    import paper_1507_03392_amd as ecr
    from oracle.binding import philox_fill
    for seed, c in ((0, (0, 0, 0, 0)), (0x123456789ABCDEF, (7, 99, 1, 0)), (2**64 - 1, (2**32 - 5000, 2**32 - 1, 4, 3))):
        g = ecr.selftest_philox(seed, c[0], c[1], c[2], c[3], 200_000)
        o = philox_fill(seed, c[0], c[1], c[2], c[3], 200_000)
        assert np.array_equal(g, o)


def test_division_and_sqrt_correctly_rounded():
    import paper_1507_03392_amd as ecr
    rng = np.random.default_rng(0)
    n = 2_000_000
    # operands within e^+-350, so that every quotient is a finite normal
    # number (|ln q| <= 700 < 708): the rounding of the quotient is what is
    # tested, not overflow to inf or underflow to 0
    a = np.exp(rng.uniform(-350, 350, n))
    b = np.exp(rng.uniform(-350, 350, n)) * rng.choice([-1.0, 1.0], n)
    # a few ends of the range: zero, subnormal and largest operands
    a[:6] = [0.0, 1.0, 2.0, 5e-324, 1.7976931348623157e308, 2.2250738585072014e-308]
    b[:6] = [3.0, 3.0, 7.0, 3.0, 3.0, 3.0]
    with np.errstate(over="raise", under="ignore"):
        ref_q = a / b
    assert np.isfinite(ref_q).all()
    q, r = ecr.selftest_divsqrt(a, b)
    assert np.array_equal(q.view(np.uint64), ref_q.view(np.uint64))
    assert np.array_equal(r.view(np.uint64), np.sqrt(a).view(np.uint64))


@pytest.mark.parametrize("n", [1, 257, 20_011])
def test_init_ions_parity(n):
    params = W.base_params(n, 32, 32, 64)
    g = gpu_run(params)
    g.init_ions()
    o = oracle(params)
    o.init_ions()
    a, b = g.get_state(), o.get_state()
    # positions come from + - * only: bit-exact
    for k in ("x", "y", "z"):
        assert np.array_equal(a[k], b[k]), k
    assert_state_close(a, b, params, what="init")
    assert g.weight == o.weight


CASES = {
    "push": dict(mask=W.P_PUSH, v_ev=0.5),
    "push_walls": dict(mask=W.P_PUSH, v_ev=300.0, dt=5e-9, rf=0.9995),
    "ionize": dict(mask=W.P_IONIZE, v_ev=0.5),
    "cx": dict(mask=W.P_CX, v_ev=50.0, n0=1e20),
    "coulomb": dict(mask=W.P_COULOMB, v_ev=0.5),
    "all": dict(mask=W.P_ALL, v_ev=20.0, n0=1e20),
    "all_walls": dict(mask=W.P_ALL, v_ev=200.0, dt=5e-9, rf=0.9995),
    # the default deposit fields only (ion number and charge: the kernels' specialised path)
    "all_nq": dict(mask=W.P_ALL, v_ev=20.0, n0=1e20, dm=3),
    # electrons = ion charge density per cell (Sec. II); a heavy weight so
    # that ionisation fires in one step
    "ionize_self_ne": dict(mask=W.P_IONIZE, v_ev=0.5, self_ne=True, weight=4e12),
    "all_self_ne": dict(mask=W.P_ALL, v_ev=20.0, n0=1e20, self_ne=True, weight=4e12),
    # electron-ion heating kick: zone background (no bias), and the cell
    # density with its diamagnetic bias
    "heat": dict(mask=W.P_HEAT, v_ev=0.5),
    "heat_self_ne": dict(mask=W.P_HEAT, v_ev=0.5, self_ne=True, weight=4e12),
    "heat_iso_self_ne": dict(mask=W.P_HEAT, v_ev=0.5, self_ne=True, weight=4e12, heat_isotropic=True),
    "all_heat_self_ne": dict(mask=W.P_ALL | W.P_HEAT, v_ev=200.0, dt=5e-9, rf=0.9995, self_ne=True, weight=4e12),
    # multiple ionisation (synthetic rates for n = 2..4) and elastic ion-atom scattering
    "multi_ionize": dict(mask=W.P_IONIZE, v_ev=0.5, dt=3e-9, ext=True),
    "elastic": dict(mask=W.P_ELASTIC, v_ev=50.0, n0=1e20, ext=True),
    "all_extended": dict(mask=W.P_ALL | W.P_ELASTIC | W.P_HEAT, v_ev=200.0, dt=5e-9, rf=0.9995, n0=5e18, ext=True),
    "extended_self_ne": dict(mask=W.P_IONIZE | W.P_CX | W.P_ELASTIC, v_ev=50.0, n0=3e19, self_ne=True, weight=4e12,
                             ext=True),
    # the neutral gas from the tracked atoms of the ion's species in its cell
    "cx_self_n0": dict(mask=W.P_CX | W.P_ELASTIC, v_ev=50.0, self_n0=True, weight=1e13, ext=True, fa=0.5),
    "all_self_n0_ne": dict(mask=W.P_ALL | W.P_ELASTIC | W.P_HEAT, v_ev=200.0, dt=5e-9, rf=0.9995, self_ne=True,
                           self_n0=True, weight=4e12, ext=True, n0=5e18),
    # every exchange ionises a tracked atom of the ion's collision cell
    "cx_partner": dict(mask=W.P_CX | W.P_ELASTIC, v_ev=50.0, self_n0=True, weight=1e13, ext=True, fa=0.5,
                       cx_partner=True),
    "all_cx_partner_ne": dict(mask=W.P_ALL | W.P_ELASTIC | W.P_HEAT, v_ev=200.0, dt=5e-9, rf=0.9995, self_ne=True,
                              self_n0=True, weight=4e12, ext=True, n0=5e18, fa=0.5, cx_partner=True),
    # every process with a magnetic field map (the kick reads |B| at cell centres from it)
    "map_all_heat_self_ne": dict(mask=W.P_ALL | W.P_HEAT, v_ev=200.0, dt=5e-9, rf=0.9995, self_ne=True, weight=4e12,
                                 bmap=True),
}


@pytest.mark.parametrize("case", sorted(CASES))
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_single_step_parity(case, seed):
    c = CASES[case]
    params = boosted(W.base_params(20_011, 16, 16, 32, seed=seed), n0=c.get("n0", 2e19))
    params.update(process_mask=c["mask"], dt=c.get("dt", 1e-9), deposit_mask=c.get("dm", 15), weight=c.get("weight", 4e9),
                  self_ne=c.get("self_ne", False), heat_isotropic=c.get("heat_isotropic", False),
                  self_n0=c.get("self_n0", False), cx_partner=c.get("cx_partner", False))
    # a large zone with a dense electron background so ionisation fires in one step
    params.update(zone_a=0.03, zone_c=0.14, ne_in=1e20)
    if c.get("ext"):
        params["species"] = [W.with_extended_mcc(params["species"][0])]
    if c.get("bmap"):
        params["bfield"] = _random_bmap(params, 40 + seed)
    st = W.random_state(params, seed=100 + seed, q_max=12, v_ev=c["v_ev"], radius_frac=c.get("rf", 0.95),
                        birth_max=17 + seed, frac_atoms=c.get("fa", 0.1))
    g, o = run_pair(params, st, 1, step0=17 + seed)
    a, b = g.get_state(), o.get_state()
    assert np.array_equal(g.events(), o.events()), "events differ"
    assert_state_close(a, b, params, what=case)
    assert np.array_equal(a["cell"], b["cell"])
    tg, to = g.tallies(), o.tallies()
    assert_tallies_equal(tg, to, case)
    ev = o.events()
    if case in ("push_walls", "all_walls"):
        assert (ev == W.EV_WALL).sum() > 20
    if case in ("ionize", "all", "ionize_self_ne", "all_self_ne", "all_heat_self_ne"):
        assert (ev == W.EV_IONIZE).sum() > 5
    if case in ("all_heat_self_ne", "all_extended", "map_all_heat_self_ne"):
        assert (ev == W.EV_WALL).sum() > 20
    if case in ("multi_ionize", "all_extended", "extended_self_ne"):
        assert to["ionized_n"][0][1:].sum() > 0 and (ev == W.EV_IONIZE).sum() > 5
    if case in ("elastic", "all_extended", "extended_self_ne", "cx_self_n0", "all_self_n0_ne"):
        assert (ev == W.EV_ELASTIC).sum() > 10
    if case in ("cx_self_n0", "cx_partner"):
        assert (ev == W.EV_CX).sum() > 10
    if case in ("cx_partner", "all_cx_partner_ne"):
        assert (ev == W.EV_CX_PARTNER).sum() > 5
        assert (ev == W.EV_WALL).sum() > 20 or case == "cx_partner"
    if case in ("heat", "heat_self_ne", "heat_iso_self_ne"):
        kicked = (b["vx"] != st["vx"]).sum()
        assert kicked > 2000, kicked
    if case == "cx":
        assert (ev == W.EV_CX).sum() > 10
    if c["mask"] & W.P_COULOMB:
        assert abs(tg["coul_de"]) <= 1e-12 * tg["coul_e"]
        assert tg["coul_e"] == pytest.approx(to["coul_e"], rel=1e-12)
    if c["mask"] & W.P_DEPOSIT:
        for f in (W.F_ION_N, W.F_ION_Q, W.F_ATOM_N, W.F_ION_P):
            dg, sg = g.density(f)
            do, so = o.density(f)
            assert sg == so == 1
            assert np.abs(dg - do).max() <= 1e-12 * max(1.0, np.abs(do).max())


def test_extraction_aperture_parity():
    # ions just below the extraction flange heading out: some through the
    # aperture (recycled at the inlet), some onto the flange around it
    n = 6007
    params = W.base_params(n, 16, 16, 32)
    params.update(process_mask=W.P_ALL, dt=2e-9)
    rng = np.random.default_rng(12)
    r = 2 * params["r_ap"] * np.sqrt(rng.random(n))
    th = 2 * np.pi * rng.random(n)
    st = dict(x=r * np.cos(th), y=r * np.sin(th), z=params["L"] / 2 - rng.random(n) * 4e-5,
              vx=rng.normal(size=n) * 300, vy=rng.normal(size=n) * 300, vz=np.abs(rng.normal(size=n)) * 2e4,
              q=rng.integers(0, 9, n).astype(np.uint8))
    st["birth"] = np.where(st["q"] >= 1, rng.integers(0, 6, n), 0xFFFFFFFF).astype(np.uint32)
    g, o = run_pair(params, st, 2, step0=5)
    ev = o.events()
    assert np.array_equal(g.events(), ev)
    assert_state_close(g.get_state(), o.get_state(), params, what="extract")
    tg, to = g.tallies(), o.tallies()
    assert_tallies_equal(tg, to, "extract")
    assert to["recycled"] > 500 and to["wall"].sum() > 500
    assert to["fpt_n"].sum() > 300 and to["lost_ke"][0] > 0 and to["extracted_r"].sum() > 0


def test_efield_push_parity():
    params = W.base_params(5003, 8, 8, 16)
    nn = 9 * 9 * 17
    rng = np.random.default_rng(3)
    ef = rng.normal(size=(3, nn)) * 2000.0
    params.update(process_mask=W.P_PUSH, efield=ef)
    st = W.random_state(params, seed=5, q_max=10, v_ev=5.0)
    g, o = run_pair(params, st, 3)
    assert_state_close(g.get_state(), o.get_state(), params, what="efield")
    assert np.array_equal(g.events(), o.events())


def _random_bmap(params, seed):
    # a node field map: a uniform 0.5 T along z plus node-to-node noise
    nn = (params["nx"] + 1) * (params["ny"] + 1) * (params["nz"] + 1)
    rng = np.random.default_rng(seed)
    m = rng.normal(size=(3, nn)) * 0.05
    m[2] += 0.5
    return m


@pytest.mark.parametrize("with_e", [False, True])
def test_bfield_map_push_parity(with_e):
    # a magnetic field map in place of the analytic field (and an E grid with it)
    params = W.base_params(5003, 8, 8, 16)
    params.update(process_mask=W.P_PUSH | W.P_DEPOSIT, bfield=_random_bmap(params, 4), dt=1e-8)
    if with_e:
        params["efield"] = np.random.default_rng(3).normal(size=(3, 9 * 9 * 17)) * 2000.0
    st = W.random_state(params, seed=5, q_max=10, v_ev=300.0, radius_frac=0.9995)
    g, o = run_pair(params, st, 3)
    assert_state_close(g.get_state(), o.get_state(), params, what="bfield map")
    assert np.array_equal(g.events(), o.events())
    assert_tallies_equal(g.tallies(), o.tallies(), "bfield map")
    assert o.tallies()["wall"].sum() > 20
    # and the map is what moved them: the analytic field gives other orbits
    a = oracle(dict(params, bfield=None))
    a.set_state(st, step=0)
    a.step(3)
    assert np.abs(a.get_state()["vx"] - o.get_state()["vx"]).max() > 1.0


def test_multi_step_c1_from_init():
    # the C1 workload (20k Ar ions, FP64, grid 32x32x64) for 120 steps, across two sorts
    params, _ = W.config("c1")
    g = gpu_run(params, events=True)
    g.init_ions()
    o = oracle(params)
    o.init_ions()
    for chunk in (1, 49, 1, 69):
        g.step(chunk)
        o.step(chunk)
        a, b = g.get_state(), o.get_state()
        assert np.array_equal(g.events(), o.events())
        assert_state_close(a, b, params, what=f"c1 step {a['step']}")
        assert np.array_equal(a["cell"], b["cell"])
    assert_tallies_equal(g.tallies(), o.tallies(), "c1")
    for f in (W.F_ION_N, W.F_ION_Q):
        dg, _ = g.density(f)
        do, _ = o.density(f)
        assert np.abs(dg - do).max() <= 1e-12 * np.abs(do).max()


@pytest.mark.parametrize("heat", [False, True])
def test_multi_step_c1_self_consistent_electrons(heat):
    # C1 with the electron density taken from the ions' charge cell by cell,
    # 150 steps across three sorts: every step's decisions bit for bit; with
    # the heating kick and its diamagnetic bias as well
    params = W.with_(W.config("c1")[0], self_ne=True)
    if heat:
        params["process_mask"] |= W.P_HEAT
    g = gpu_run(params, events=True)
    g.init_ions()
    o = oracle(params)
    o.init_ions()
    ionized = 0
    for chunk in (1, 49, 50, 50):
        g.step(chunk)
        o.step(chunk)
        a, b = g.get_state(), o.get_state()
        assert np.array_equal(g.events(), o.events())
        assert_state_close(a, b, params, what=f"c1 self-ne step {a['step']}")
    tg = g.tallies()
    assert_tallies_equal(tg, o.tallies(), "c1 self-ne")
    assert tg["ionized"].sum() > 100


def test_multi_step_c1_extended_mcc():
    # C1 with multiple ionisation, elastic ion-atom scattering and the heating
    # kick on top of every default process, a denser neutral background, 120
    # steps across two sorts.  Decisions stay bit for bit.  The scattering
    # directions of charge exchange and elastic collisions go through sin and
    # cos, whose GPU and CPU results may differ in the last bit; with a
    # thousand such collisions here, Coulomb scattering carries those
    # differences to other ions over the steps, so the multi-step bar for x
    # and v is 1e-9 (one step from an identical state keeps 1e-12: the
    # single-step cases above)
    params = boosted(W.config("c1")[0], n0=2e19)
    params["species"] = [W.with_extended_mcc(params["species"][0])]
    params["process_mask"] = W.P_ALL | W.P_ELASTIC | W.P_HEAT
    params["ne_in"] = 1e19
    g = gpu_run(params, events=True)
    g.init_ions()
    o = oracle(params)
    o.init_ions()
    for chunk in (1, 49, 70):
        g.step(chunk)
        o.step(chunk)
        a, b = g.get_state(), o.get_state()
        assert np.array_equal(g.events(), o.events())
        assert_state_close(a, b, params, what=f"c1 extended step {a['step']}", tol=1e-9)
    tg, to = g.tallies(), o.tallies()
    assert_tallies_equal(tg, to, "c1 extended")
    assert to["elastic"].sum() > 15 and to["ionized_n"][0][1:].sum() > 5


def test_multi_step_exchange_partners():
    # tracked exchange partners over 60 steps and three sorts, with every
    # process on: partners, unmatched exchanges and births bit for bit
    params = boosted(W.base_params(20_011, 16, 16, 32, seed=8))
    params["species"] = [W.with_extended_mcc(params["species"][0])]
    params.update(process_mask=W.P_ALL | W.P_ELASTIC | W.P_HEAT, self_ne=True, self_n0=True, cx_partner=True,
                  weight=1e12, sort_every=20, dt=2e-9, zone_a=0.03, zone_c=0.14)
    st = W.random_state(params, seed=81, q_max=8, v_ev=40.0, frac_atoms=0.5)
    g = gpu_run(params, events=True)
    g.set_state(st, step=0)
    o = oracle(params)
    o.set_state(st, step=0)
    partners = 0
    for chunk in (1, 29, 30):
        g.step(chunk)
        o.step(chunk)
        a, b = g.get_state(), o.get_state()
        assert np.array_equal(g.events(), o.events())
        partners += int((o.events() == W.EV_CX_PARTNER).sum())
        assert_state_close(a, b, params, what=f"exchange partners step {a['step']}", tol=1e-9)
    to = o.tallies()
    assert_tallies_equal(g.tallies(), to, "exchange partners")
    assert to["cx"].sum() > 20 and partners > 0


def test_multi_step_tracked_neutrals_and_electrons():
    # half the particles atoms: the collisions' neutral gas and the
    # electrons both follow the particles cell by cell, 60 steps across
    # three sorts, every decision bit for bit
    params = boosted(W.base_params(20_011, 16, 16, 32, seed=6))
    params["species"] = [W.with_extended_mcc(params["species"][0])]
    params.update(process_mask=W.P_ALL | W.P_ELASTIC | W.P_HEAT, self_ne=True, self_n0=True, weight=1e12,
                  sort_every=20, dt=2e-9, zone_a=0.03, zone_c=0.14)
    st = W.random_state(params, seed=61, q_max=8, v_ev=40.0, frac_atoms=0.5)
    g = gpu_run(params, events=True)
    g.set_state(st, step=0)
    o = oracle(params)
    o.set_state(st, step=0)
    for chunk in (1, 29, 30):
        g.step(chunk)
        o.step(chunk)
        a, b = g.get_state(), o.get_state()
        assert np.array_equal(g.events(), o.events())
        assert_state_close(a, b, params, what=f"tracked neutrals step {a['step']}", tol=1e-9)
    to = o.tallies()
    assert_tallies_equal(g.tallies(), to, "tracked neutrals")
    assert to["cx"].sum() > 20 and to["elastic"].sum() > 20 and to["ionized"].sum() > 20


def test_deposit_fused_and_split_agree():
    # deposit inside the push kernel (default) or as its own kernel after it:
    # the same run, densities within FP64 atomic rounding
    params, _ = W.config("c1")
    outs = []
    for kw in (dict(), dict(split=True)):
        g = gpu_run(params, **kw)
        g.init_ions()
        g.step(37)
        g.step(83)
        outs.append((g.get_state(), g.tallies(), [g.density(f) for f in (W.F_ION_N, W.F_ION_Q)]))
    for st, t, d in outs[1:]:
        for k in ("x", "vx", "q", "cell"):
            assert np.array_equal(st[k], outs[0][0][k]), k
        assert_tallies_equal(t, outs[0][1])
        for (a, na), (b, nb) in zip(d, outs[0][2]):
            assert na == nb == 120
            assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()


@pytest.mark.parametrize("dm", [3, 15])
def test_deposit_tiles_that_overflow_the_brick(dm):
    # 6000 ions, cell-sorted: dense clusters at opposite corners of the mesh
    # interleaved so that every 1024-slot tile spans the whole mesh (far more
    # nodes than the LDS brick holds), plus one tile of a single dense cell;
    # the deposit of both kinds of tile against the oracle's brute-force sum
    params = W.base_params(6000, 16, 16, 32, seed=5)
    params.update(process_mask=W.P_DEPOSIT, deposit_mask=dm)
    rng = np.random.default_rng(8)
    h = 2 * params["R0"] / 16, params["L"] / 32
    n = 6000
    corner = np.where(np.arange(n) % 2 == 0, 0, 1)
    corner[5000:] = 2  # one dense cell in the middle: a tile that fits the brick
    cx = np.select([corner == 0, corner == 1], [-params["R0"] + 0.5 * h[0], params["R0"] - 0.5 * h[0]], 0.2 * h[0])
    cz = np.select([corner == 0, corner == 1], [-params["L"] / 2 + 0.5 * h[1], params["L"] / 2 - 0.5 * h[1]], 0.3 * h[1])
    st = dict(x=cx + rng.uniform(-0.4, 0.4, n) * h[0], y=rng.uniform(-0.4, 0.4, n) * h[0],
              z=cz + rng.uniform(-0.4, 0.4, n) * h[1], vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n),
              q=rng.integers(0, 9, n).astype(np.uint8))
    # slot order = the given cells' order: the alternating corners stay interleaved
    cells = np.full(n, 7, dtype=np.uint32)
    g, o = run_pair(params, st, 2, step0=3, cell=cells)
    for f in (W.F_ION_N, W.F_ION_Q, W.F_ATOM_N):
        dg, sg = g.density(f)
        do, so = o.density(f)
        assert sg == so == 2
        assert np.abs(dg - do).max() <= 1e-12 * max(1.0, np.abs(do).max()), f
        if (dm >> f) & 1:
            assert do.max() > 100
        else:
            assert not dg.any()


def test_given_cells_and_resume_bitwise():
    params = boosted(W.base_params(30_000, 16, 16, 32, seed=4))
    params.update(dt=2e-9)
    st = W.random_state(params, seed=9, q_max=8, v_ev=30.0)
    a = gpu_run(params)
    a.set_state(st)
    a.step(130)
    b = gpu_run(params)
    b.set_state(st)
    b.step(70)
    mid = b.get_state()
    c = gpu_run(params)
    c.set_state(mid, step=mid["step"], cell=mid["cell"])
    c.step(60)
    sa, sc = a.get_state(), c.get_state()
    for k in ("x", "y", "z", "vx", "vy", "vz", "q", "cell"):
        assert np.array_equal(sa[k], sc[k]), k


def test_determinism_two_runs():
    params, _ = W.config("c1")
    outs = []
    for _ in range(2):
        g = gpu_run(params)
        g.init_ions()
        g.step(60)
        outs.append((g.get_state(), g.tallies()))
    for k in ("x", "vx", "q"):
        assert np.array_equal(outs[0][0][k], outs[1][0][k])
    assert_tallies_equal(outs[0][1], outs[1][1])


def test_edge_sizes_zero_one_and_tiny_grid():
    for n in (0, 1, 2, 3):
        params = W.base_params(n, 1, 1, 1)
        params.update(process_mask=W.P_ALL)
        g = gpu_run(params, events=True)
        g.init_ions()
        g.step(5)
        t = g.tallies()
        assert t["steps"] == 5
        if n:
            o = oracle(params)
            o.init_ions()
            o.step(5)
            assert_state_close(g.get_state(), o.get_state(), params, what=f"n={n}")
            assert_tallies_equal(t, o.tallies())


def test_edge_sizes_with_exchange_partners():
    # tracked neutrals and exchange partners with 0-3 particles in one cell
    for n in (0, 1, 2, 3):
        params = W.base_params(n, 1, 1, 1)
        params.update(process_mask=W.P_ALL, self_n0=True, cx_partner=True)
        g = gpu_run(params, events=True)
        g.init_ions()
        g.step(5)
        t = g.tallies()
        assert t["steps"] == 5
        if n:
            o = oracle(params)
            o.init_ions()
            o.step(5)
            assert_state_close(g.get_state(), o.get_state(), params, what=f"partners n={n}")
            assert_tallies_equal(t, o.tallies())


def test_edt_rejected_and_bad_state():
    import paper_1507_03392_amd as ecr
    params = boosted(W.base_params(100, 8, 8, 16), n0=1e23)
    with pytest.raises(ecr.EcrError) as e:
        gpu_run(params)
    assert e.value.status == -6
    params = W.base_params(10, 8, 8, 16)
    g = gpu_run(params)
    st = W.random_state(params, seed=1)
    st["q"][3] = 25
    with pytest.raises(ecr.EcrError) as e:
        g.set_state(st)
    assert e.value.status == -1
    st["q"][3] = 1
    st["vx"][4] = np.nan
    g.set_state(st)
    g.step(1)
    with pytest.raises(ecr.EcrError) as e:
        g.tallies(allow_anomalies=False)
    assert e.value.status == -5


def host_cells(params, st, dtype=np.float64):
    """Collision cell of each particle by floor-and-clamp of its position, in
    the arithmetic of the state's precision (binary64, or binary32 for the
    FP32-mixed state): i = clamp(floor((x + R0) * nx / (2 R0)), 0, nx - 1),
    likewise for y, and for z with (z + L/2) * nz / L."""
    R0, hL = params["R0"], 0.5 * params["L"]
    idx = params["nx"] / (2.0 * R0)
    idy = params["ny"] / (2.0 * R0)
    idz = params["nz"] / params["L"]
    t = dtype
    with np.errstate(invalid="ignore"):
        ix = np.clip(np.floor((st["x"].astype(t) + t(R0)) * t(idx)), 0, params["nx"] - 1).astype(np.int64)
        iy = np.clip(np.floor((st["y"].astype(t) + t(R0)) * t(idy)), 0, params["ny"] - 1).astype(np.int64)
        iz = np.clip(np.floor((st["z"].astype(t) + t(hL)) * t(idz)), 0, params["nz"] - 1).astype(np.int64)
    return (ix + params["nx"] * (iy + params["ny"] * iz)).astype(np.uint32)


def test_full_size_c2_sampled_cells():
    # 2M ions on the 64x64x128 grid, the benchmark's launch configuration:
    # after 60 steps, whole collision cells are stepped once more by the oracle
    from oracle.binding import OracleSim
    params, _ = W.config("c2")
    g = gpu_run(params, events=True)
    g.init_ions()
    g.step(50)
    # the sort at step 50 at full size: every particle's collision cell is
    # floor-and-clamp of its position at the start of that step
    s50 = g.get_state()
    g.step(1)
    assert np.array_equal(g.get_state()["cell"], host_cells(params, s50)), "c2 sort cells"
    g.step(9)
    before = g.get_state()
    g.step(1)
    after = g.get_state()
    ev = g.events()
    rng = np.random.default_rng(0)
    cells = np.unique(before["cell"])
    pick = rng.choice(cells, size=min(400, len(cells)), replace=False)
    ids = np.nonzero(np.isin(before["cell"], pick))[0]
    sub = W.with_(params, n=len(ids), weight=g.weight)
    o = OracleSim(sub)
    o.set_ids(ids, before["species"][ids])
    o.set_state({k: before[k][ids] for k in ("x", "y", "z", "vx", "vy", "vz", "q", "birth")}, step=60,
                cell=before["cell"][ids])
    o.step(1)
    ob = o.get_state()
    assert_state_close(after, ob, params, ids=ids, what="c2 sampled")
    assert np.array_equal(ev[ids], o.events())
    assert len(ids) > 10_000
    t = g.tallies()
    assert t["anomalies"] == 0
    # charge bookkeeping over the whole run
    zz = np.arange(32)
    lost = int((zz * (t["extracted"][0] + t["wall"][0])).sum())
    assert int(after["q"].astype(np.int64).sum()) + lost + int(t["cx_products"][0]) == \
        params["n"] + int(t["ionized"][0].sum())


def test_kernel_timing_every_launch_and_sampled():
    # ecr_profile brackets launches with events; ecr_profile_stride keeps
    # one launch in stride of each kind; timing leaves the results unchanged
    params = W.with_(W.config("c1")[0], sort_every=10)
    for split, main in ((False, "step"), (True, "push")):
        a, b = gpu_run(params, split=split), gpu_run(params, split=split)
        a.init_ions()
        b.init_ions()
        a.profile(True)
        a.step(20)
        kt = a.kernel_times()
        assert kt[main][1] == 20 and kt["sort"][1] == 2
        if split:  # the step as separate kernels
            assert kt["coul_order"][1] == kt["coul_pairs"][1] == 20 and kt["step"][1] == 0
        else:  # the whole step in one kernel
            assert kt["coul_order"][1] == kt["coul_pairs"][1] == kt["push_deposit"][1] == 0
        assert all(ms > 0 for ms, c in kt.values() if c)
        a.profile(True, kinds=[main], stride=6)
        a.step(20)
        kt = a.kernel_times()
        assert kt[main][1] == 4 and kt["sort"][1] == 0  # launches 0, 6, 12, 18
        a.profile(False)
        b.step(40)
        sa, sb = a.get_state(), b.get_state()
        for k in ("x", "vx", "q"):
            assert np.array_equal(sa[k], sb[k])
    import paper_1507_03392_amd as ecr
    with pytest.raises(ecr.EcrError):
        a.profile(True, stride=0)


def test_step_batch_matches_separate_steps():
    # ecr_step_batch advances several runs that share a stream: the same
    # state, events and tallies bit for bit as each run stepped alone
    import torch

    import paper_1507_03392_amd as ecr
    stream = torch.cuda.Stream()
    cases = []
    for i, (n, q) in enumerate(((3_001, 3), (20_011, 8), (700, 1))):
        p = boosted(W.base_params(n, 16, 16, 32, seed=40 + i))
        p.update(process_mask=W.P_ALL, sort_every=7)
        cases.append((p, W.random_state(p, seed=90 + i, q_max=q, v_ev=30.0)))
    runs = []
    for p, st in cases:
        r = gpu_run(p, events=True, stream=stream)
        r.set_state(st, step=5)
        runs.append(r)
    ecr.step_batch(runs, 11, stream)
    ecr.step_batch(runs, 9, stream)
    stream.synchronize()
    for (p, st), r in zip(cases, runs):
        alone = gpu_run(p, events=True)
        alone.set_state(st, step=5)
        alone.step(20)
        a, b = r.get_state(), alone.get_state()
        for k in ("x", "y", "z", "vx", "vy", "vz", "q", "cell", "birth"):
            assert np.array_equal(a[k], b[k]), k
        assert a["step"] == b["step"] == 25
        assert np.array_equal(r.events(), alone.events())
        assert_tallies_equal(r.tallies(), alone.tallies(), "batch vs alone")


def test_step_batch_replays_sort_periods_of_mixed_runs():
    # runs at the start of a common sort period are advanced a period at a
    # time by one captured graph in which every batchable run's step is one
    # shared launch (binary64 and binary32 runs in launches of their own
    # precision; a run with self-consistent electrons keeps its own kernels);
    # the graphs are reused on later periods and forgotten when a run is
    # destroyed.  Each run ends bit for bit where it ends stepped alone.
    import torch

    import paper_1507_03392_amd as ecr
    stream = torch.cuda.Stream()
    cases = []
    for i, (n, q, extra) in enumerate(((3_001, 3, {}), (20_011, 8, {"precision": W.PREC_FP32}),
                                       (4_099, 4, {"self_ne": True}), (700, 1, {}), (61_001, 6, {}))):
        p = boosted(W.base_params(n, 16, 16, 32, seed=60 + i))
        p.update(process_mask=W.P_ALL, sort_every=7, **extra)
        cases.append((p, W.random_state(p, seed=70 + i, q_max=q, v_ev=30.0)))

    def batch(runs, calls):
        for k in calls:
            ecr.step_batch(runs, k, stream)
        stream.synchronize()

    def check(case_runs, steps, step0):
        for (p, st), r in case_runs:
            alone = gpu_run(p, events=True)
            alone.set_state(st, step=step0)
            alone.step(steps)
            a, b = r.get_state(), alone.get_state()
            for k in ("x", "y", "z", "vx", "vy", "vz", "q", "cell", "birth"):
                assert np.array_equal(a[k], b[k]), (p["n"], k)
            assert a["step"] == b["step"] == step0 + steps
            assert np.array_equal(r.events(), alone.events())
            assert_tallies_equal(r.tallies(), alone.tallies(), "batch vs alone")
            da, db = r.density(W.F_ION_Q)[0], alone.density(W.F_ION_Q)[0]
            assert np.allclose(da, db, rtol=0, atol=1e-12 * max(1.0, np.abs(db).max()))

    runs = []
    for p, st in cases:
        r = gpu_run(p, events=True, stream=stream)
        r.set_state(st, step=14)
        runs.append(r)
    # 4 whole periods (the first eagerly, then one graph per buffer, the
    # first of them replayed), then 5 single steps
    batch(runs, (30, 3))
    check(list(zip(cases, runs)), 33, 14)
    # a run leaves and another joins: the new set's graphs, not the old ones
    runs[1].close()
    p, st = cases[1]
    r = gpu_run(p, events=True, stream=stream)
    r.set_state(st, step=40)
    r.step(7)
    stream.synchronize()
    # all at step 47: two single steps; the new set's first period eagerly,
    # its next two captured (one per buffer), the fourth replayed
    batch([runs[0], r, runs[3]], (30,))
    check([(cases[0], runs[0]), (cases[3], runs[3])], 33 + 30, 14)
    check([((p, st), r)], 37, 40)


def test_exchange_partners_in_a_chunk_beyond_the_lds():
    # a cell of 5000 atoms (more slots than the exchange-partner kernel
    # stages in LDS) whose ions exchange charge: the partners are picked
    # from global memory, bit for bit with the oracle
    params = boosted(W.base_params(20_011, 16, 16, 32, seed=9), n0=3e19)
    params.update(process_mask=W.P_CX | W.P_PUSH, self_n0=True, cx_partner=True, weight=4e10)
    st = W.random_state(params, seed=57, q_max=4, v_ev=20.0, frac_atoms=0.2)
    hx, hz = 2 * params["R0"] / 16, params["L"] / 32
    rng = np.random.default_rng(58)
    k = 5600
    st["x"][:k] = -params["R0"] + (8.3 + 0.4 * rng.random(k)) * hx
    st["y"][:k] = -params["R0"] + (8.3 + 0.4 * rng.random(k)) * hx
    st["z"][:k] = -params["L"] / 2 + (1.3 + 0.4 * rng.random(k)) * hz
    st["q"][:5000] = 0
    st["q"][5000:k] = rng.integers(1, 5, k - 5000)
    g, o = run_pair(params, st, 2, step0=3)  # the oracle takes 7 partners in the crowded cell
    a, b = g.get_state(), o.get_state()
    assert np.array_equal(g.events(), o.events())
    assert_state_close(a, b, params, what="partners beyond the LDS")
    tg, to = g.tallies(), o.tallies()
    assert_tallies_equal(tg, to, "partners beyond the LDS")
    assert tg["anomalies"] == 0
    crowded = np.bincount(o.get_state()["cell"].astype(np.int64)).max()
    assert crowded >= 5000
    assert int((o.events()[:k] == W.EV_CX_PARTNER).sum()) > 0  # partners were taken in the crowded cell


@pytest.mark.parametrize("m", [1500, 5001])
def test_coulomb_pool_beyond_a_chunk(m):
    # one cell whose pool holds m ions, more than a chunk of the one-kernel
    # step (1024 slots): its pool is sorted by (key, id) with a bitonic
    # network (in LDS for 1500, in global scratch memory for 5001) and every
    # ion collides, bit for bit with the oracle, whose pool has no size limit
    params = W.base_params(20_011, 16, 16, 32, seed=12)
    params.update(process_mask=W.P_COULOMB | W.P_PUSH | W.P_DEPOSIT, weight=2e9)
    st = W.random_state(params, seed=60 + m % 7, q_max=8, v_ev=5.0, frac_atoms=0.1)
    hx, hz = 2 * params["R0"] / 16, params["L"] / 32
    rng = np.random.default_rng(61)
    st["x"][:m] = -params["R0"] + (5.2 + 0.6 * rng.random(m)) * hx
    st["y"][:m] = -params["R0"] + (9.2 + 0.6 * rng.random(m)) * hx
    st["z"][:m] = -params["L"] / 2 + (20.2 + 0.6 * rng.random(m)) * hz
    st["q"][:m] = rng.integers(1, 9, m)
    g, o = run_pair(params, st, 2, step0=3)
    a, b = g.get_state(), o.get_state()
    assert_state_close(a, b, params, what=f"pool of {m}")
    assert np.bincount(b["cell"].astype(np.int64)).max() >= m
    tg, to = g.tallies(), o.tallies()
    assert tg["anomalies"] == 0
    assert tg["coul_e"] == pytest.approx(to["coul_e"], rel=1e-12)
    for f in (W.F_ION_N, W.F_ION_Q):
        (dg, ng), (do, no) = g.density(f), o.density(f)
        assert ng == no == 2 and np.abs(dg - do).max() <= 1e-12 * np.abs(do).max()
    assert (a["vx"][:m] != st["vx"][:m]).mean() > 0.95  # the crowded cell's ions collided


def test_split_kernels_flag_a_pool_beyond_their_chunk():
    # the per-kernel (split) form orders at most 1024 ions per chunk in
    # LDS: a larger pool skips the step's collisions and the read calls
    # report it (ECR_ENUMERIC); the one-kernel step collides them
    import paper_1507_03392_amd as ecr
    params = W.base_params(4_000, 16, 16, 32, seed=13)
    params.update(process_mask=W.P_COULOMB, weight=2e9)
    st = W.random_state(params, seed=64, q_max=4, v_ev=5.0, frac_atoms=0.0)
    hx, hz = 2 * params["R0"] / 16, params["L"] / 32
    rng = np.random.default_rng(65)
    m = 1500
    st["x"][:m] = -params["R0"] + (5.2 + 0.6 * rng.random(m)) * hx
    st["y"][:m] = -params["R0"] + (9.2 + 0.6 * rng.random(m)) * hx
    st["z"][:m] = -params["L"] / 2 + (20.2 + 0.6 * rng.random(m)) * hz
    g = gpu_run(params, split=True)
    g.set_state(st, step=0)
    g.step(1)
    with pytest.raises(ecr.EcrError) as e:
        g.tallies(allow_anomalies=False)
    assert e.value.status == -5 and "Coulomb chunk" in str(e.value)
    assert (g.get_state()["vx"][:m] == st["vx"][:m]).all()  # the crowded cell did not collide
    f = gpu_run(params)
    f.set_state(st, step=0)
    f.step(1)
    assert f.tallies(allow_anomalies=False)["anomalies"] == 0
    assert (f.get_state()["vx"][:m] != st["vx"][:m]).mean() > 0.95


def test_coulomb_in_a_cell_crowded_with_atoms():
    # over a long run the gas inlet's cell fills with recycled atoms (more
    # than a Coulomb chunk can stage): atoms take no room in the ordering,
    # so a cell of 3000 atoms and 300 ions keeps its collisions, bit for bit
    params = W.base_params(20_011, 16, 16, 32, seed=5)
    params.update(process_mask=W.P_COULOMB, weight=4e9)
    st = W.random_state(params, seed=55, q_max=8, v_ev=5.0, frac_atoms=0.1)
    hx, hz = 2 * params["R0"] / 16, params["L"] / 32
    rng = np.random.default_rng(56)
    k = 3300
    st["x"][:k] = -params["R0"] + (8.2 + 0.6 * rng.random(k)) * hx
    st["y"][:k] = -params["R0"] + (8.2 + 0.6 * rng.random(k)) * hx
    st["z"][:k] = -params["L"] / 2 + (1.2 + 0.6 * rng.random(k)) * hz
    st["q"][:3000] = 0
    st["q"][3000:k] = rng.integers(1, 9, k - 3000)
    g, o = run_pair(params, st, 1, step0=3)
    a, b = g.get_state(), o.get_state()
    assert_state_close(a, b, params, what="crowded cell")
    assert np.bincount(b["cell"].astype(np.int64)).max() >= k
    tg, to = g.tallies(), o.tallies()
    assert tg["anomalies"] == 0  # no chunk overflowed
    assert tg["coul_e"] == pytest.approx(to["coul_e"], rel=1e-12)
    moved = (a["vx"][3000:k] != st["vx"][3000:k]).mean()
    assert moved > 0.9  # the crowded cell's ions did collide


@pytest.mark.parametrize("m,mesh", [(3, (32, 32, 32)), (5, (24, 24, 36)), (7, (20, 20, 36))])
def test_coulomb_chunks_of_odd_pools(m, mesh):
    # every cell holds m ions, so every pool is odd: with 736-slot chunks
    # (from 98 304 particles up) a chunk of 3-ion cells holds about 245
    # triplets, more than three wavefronts of them (every item
    # round-robin); 5- and 7-ion cells give 147 and 105 triplets, whose
    # wavefronts' spare lanes take pairs three at a time before the other
    # wavefronts take the rest; bit for bit against the oracle
    nx, ny, nz = mesh
    n = m * nx * ny * nz
    assert n >= 128 * 768
    params = W.base_params(n, nx, ny, nz, seed=17)
    params.update(process_mask=W.P_COULOMB, weight=2e9)
    st = W.random_state(params, seed=71, q_max=8, v_ev=5.0, frac_atoms=0.0)
    rng = np.random.default_rng(72)
    hx, hy, hz = 2 * params["R0"] / nx, 2 * params["R0"] / ny, params["L"] / nz
    c = np.repeat(np.arange(nx * ny * nz), m)
    ix, iy, iz = c % nx, (c // nx) % ny, c // (nx * ny)
    st["x"][:] = -params["R0"] + (ix + 0.2 + 0.6 * rng.random(n)) * hx
    st["y"][:] = -params["R0"] + (iy + 0.2 + 0.6 * rng.random(n)) * hy
    st["z"][:] = -params["L"] / 2 + (iz + 0.2 + 0.6 * rng.random(n)) * hz
    st["q"][:] = rng.integers(1, 9, n)
    g, o = run_pair(params, st, 1, step0=5)
    a, b = g.get_state(), o.get_state()
    assert_state_close(a, b, params, what=f"cells of {m} ions")
    assert (np.bincount(b["cell"].astype(np.int64), minlength=nx * ny * nz) == m).all()
    tg, to = g.tallies(), o.tallies()
    assert tg["anomalies"] == 0
    assert tg["coul_e"] == pytest.approx(to["coul_e"], rel=1e-12)
    assert abs(tg["coul_de"]) <= 1e-12 * tg["coul_e"]
    assert (a["vx"] != st["vx"]).mean() > 0.95  # every pool collided
