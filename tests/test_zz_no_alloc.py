"""ecr_create_static: the run of ecr_create with its arena replaced by the
library's static device workspace, for callers that cannot allocate device
memory.

Two calls in a row, the second with fewer particles (the workspace keeps the
first run's contents): each static run is stepped from the same state as a
run in a torch arena made by ecr_create, and gives the same results to the
parity bar: positions, velocities, charges, cells, births, events and
integer tallies bit for bit; FP64 sums gathered with atomics within 1e-12
relative; density grids within 1e-12 of the largest node.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = (W.F_ION_N, W.F_ION_Q, W.F_ATOM_N)


def _params(n, seed):
    p = W.base_params(n, 16, 16, 32, seed=seed)
    sp = dict(p["species"][0])
    sp["n0"] = 2e19  # charge exchange fires within the run
    p.update(species=[sp], dt=3e-9, sort_every=20, deposit_mask=7)
    return p


def _run(params, st, steps, static):
    import paper_1507_03392_amd as ecr
    r = ecr.Run(params, events=True, static=static)
    try:
        r.set_state(st, step=3)
        r.step(steps)
        return r.get_state(), r.events(), r.tallies(), [r.density(f) for f in FIELDS]
    finally:
        r.close()


def test_static_workspace_matches_arena_twice():
    for n, steps, seed in ((30_011, 61, 1), (5_003, 23, 2)):
        p = _params(n, seed)
        st = W.random_state(p, seed=10 + seed, q_max=6, v_ev=150.0, frac_atoms=0.3, birth_max=3)
        sa, ea, ta, da = _run(p, st, steps, static=True)
        sb, eb, tb, db = _run(p, st, steps, static=False)
        for k in ("x", "y", "z", "vx", "vy", "vz", "q", "cell", "birth"):
            assert np.array_equal(sa[k], sb[k]), f"n={n}: {k}"
        assert sa["step"] == sb["step"] == 3 + steps
        assert np.array_equal(ea, eb)
        for k in ("extracted", "wall", "ionized", "cx", "cx_products", "fpt_n", "fpt_sum", "fpt_hist"):
            assert np.array_equal(ta[k], tb[k]), f"n={n}: {k}"
        for k in ("recycled", "anomalies", "steps"):
            assert ta[k] == tb[k], f"n={n}: {k}"
        for k in ("extracted_r", "lost_ke"):
            np.testing.assert_allclose(ta[k], tb[k], rtol=1e-12, atol=1e-300)
        np.testing.assert_allclose(ta["coul_e"], tb["coul_e"], rtol=1e-12)
        for (a, na), (b, nb) in zip(da, db):
            assert na == nb == steps
            assert np.abs(a - b).max() <= 1e-12 * max(np.abs(b).max(), 1e-300)
        assert tb["wall"].sum() > 0 and tb["cx"].sum() > 0 and tb["ionized"].sum() > 0


def test_static_workspace_limits():
    import paper_1507_03392_amd as ecr
    big = W.base_params(2_000_000, 64, 64, 128)
    with pytest.raises(ecr.EcrError) as e:
        ecr.Run(big, static=True)
    assert e.value.status == -2 and "static workspace" in str(e.value)
    small = _params(1_000, 3)
    r1 = ecr.Run(small, static=True)
    with pytest.raises(ecr.EcrError) as e:
        ecr.Run(small, static=True)  # the device's workspace holds r1
    assert e.value.status == -4
    r1.close()
    r2 = ecr.Run(small, static=True)
    r2.init_ions()
    r2.step(3)
    assert r2.tallies()["steps"] == 3
    r2.close()
