"""ecr_step_graph (whole sort periods replayed from a captured HIP graph)
against ecr_step, through the C ABI.

The graph path must give the same run as step-by-step launches: state,
event codes and integer tallies bit for bit, density grids within 1e-12 of
the largest node value (FP64 atomics add in a different order).  The graph
is replayed many times, with the program's own eager work and
synchronising read-backs between replays, and every replay is checked.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _runs(params, stream):
    import paper_1507_03392_amd as ecr
    return ecr.Run(params, events=True, stream=stream), ecr.Run(params, events=True, stream=stream)


def _same(a, b, what):
    sa, sb = a.get_state(), b.get_state()
    for k in ("x", "y", "z", "vx", "vy", "vz", "q", "cell"):
        assert np.array_equal(sa[k], sb[k]), f"{what}: {k}"
    assert sa["step"] == sb["step"]
    assert np.array_equal(a.events(), b.events()), what
    ta, tb = a.tallies(), b.tallies()
    for k in ("extracted", "wall", "ionized", "cx", "cx_products", "cx_unmatched"):
        assert np.array_equal(ta[k], tb[k]), f"{what}: {k}"
    for k in ("recycled", "anomalies", "steps"):
        assert ta[k] == tb[k], f"{what}: {k}"
    assert ta["coul_e"] == pytest.approx(tb["coul_e"], rel=1e-12)
    for f in (W.F_ION_N, W.F_ION_Q):
        da, na = a.density(f)
        db, nb = b.density(f)
        assert na == nb
        assert np.abs(da - db).max() <= 1e-12 * max(1.0, np.abs(db).max()), f"{what}: density {f}"


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_FP32])
def test_graph_periods_match_eager(prec):
    import torch
    params = W.with_(W.config("c1")[0], precision=prec, sort_every=20)
    params["species"] = [dict(params["species"][0], n0=1e20)]  # charge exchange fires too
    stream = torch.cuda.Stream()
    a, b = _runs(params, stream)
    a.init_ions()
    b.init_ions()
    # misaligned starts, whole periods, a remainder, then many single periods
    for n in (7, 53, 20, 41, 1, 18, 20, 20, 20, 20, 20, 60):
        a.step(n)
        b.step_graph(n)
        _same(a, b, f"after {a.get_state()['step']} steps")


def test_graph_after_set_state_and_two_runs_on_one_stream():
    import torch
    params = W.with_(W.base_params(30_011, 16, 16, 32, seed=2), sort_every=10, process_mask=W.P_ALL)
    st = W.random_state(params, seed=4, q_max=8, v_ev=30.0)
    stream = torch.cuda.Stream()
    a, b = _runs(params, stream)
    a.set_state(st, step=30)
    b.set_state(st, step=30)
    c, d = _runs(W.with_(params, seed=9), stream)
    c.set_state(st, step=30)
    d.set_state(st, step=30)
    for _ in range(3):
        a.step(40)
        c.step(40)
        b.step_graph(40)
        d.step_graph(40)
        _same(a, b, "run 1")
        _same(c, d, "run 2")
    # the two seeds give different runs
    assert not np.array_equal(a.get_state()["vx"], c.get_state()["vx"])


@pytest.mark.parametrize("heat", [False, True])
def test_graph_self_consistent_electrons_odd_period(heat):
    # the per-cell charge grid alternates between two buffers every step: an
    # odd sort period starts replays on either buffer (the heating kick reads
    # the current one too)
    import torch
    params = W.with_(W.config("c1")[0], self_ne=True, sort_every=15)
    if heat:
        params["process_mask"] |= W.P_HEAT
    stream = torch.cuda.Stream()
    a, b = _runs(params, stream)
    a.init_ions()
    b.init_ions()
    for n in (4, 26, 15, 15, 15, 30, 7):
        a.step(n)
        b.step_graph(n)
        _same(a, b, f"after {a.get_state()['step']} steps")


@pytest.mark.parametrize("partner", [False, True])
def test_graph_tracked_neutrals_odd_period(partner):
    # the cell grids (ion charge and atoms) alternate buffers every step;
    # with exchange partners a kernel after the push edits the next grid
    import torch
    params = W.with_(W.base_params(20_011, 16, 16, 32, seed=7), sort_every=15, self_n0=True, self_ne=True,
                     process_mask=W.P_ALL | W.P_ELASTIC, weight=1e12, dt=2e-9, cx_partner=partner)
    params["species"] = [W.with_extended_mcc(dict(params["species"][0], n0=2e19))]
    st = W.random_state(params, seed=70, q_max=8, v_ev=40.0, frac_atoms=0.5)
    stream = torch.cuda.Stream()
    a, b = _runs(params, stream)
    a.set_state(st, step=0)
    b.set_state(st, step=0)
    for n in (4, 26, 15, 15, 30, 7):
        a.step(n)
        b.step_graph(n)
        _same(a, b, f"after {a.get_state()['step']} steps")
