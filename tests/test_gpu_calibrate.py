"""Outer calibration on the GPU: served runs drive (w, T_ew) to a gas flow
and a coupled power (Sec. II).

The targets are the outputs of a reference run at a known (w, T_ew) of the
hot C1 variant (20k Ar ions, T_i = 30 eV, n_e = 3e12 cm^-3, dt = 5 ns:
hundreds of ions leave through the aperture within the window); started
from a weight 2.5x too large and a temperature 2.5x too small, the loop must
meet both targets within 10% and land near the reference inputs.  The
served warm-up window is checked against two reads of a plain run.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

W_REF, TE_REF = 2.0e9, 1500.0
WARMUP, STEPS = 1000, 3000


def _make(w, te):
    p = W.base_params(20_000, 32, 32, 64, seed=3)
    p.update(Ti0_eV=30.0, dt=5e-9, ne_in=3e18, weight=w, Te_in_eV=te)
    p["species"] = [W.argon(te_ev=te)]
    return p


def test_served_warmup_window_equals_two_reads():
    import paper_1507_03392_amd as ecr
    from paper_1507_03392_amd.serve import Request, Server
    p = _make(W_REF, TE_REF)
    run = ecr.Run(p)
    run.init_ions()
    run.step(WARMUP)
    t0 = run.tallies()
    run.step(500)
    t1 = run.tallies()
    res = Server(8 << 30, max_active=2).serve([Request(0, 0.0, p, WARMUP + 500, warmup=WARMUP),
                                               Request(1, 0.0, p, WARMUP + 500)])
    win, full = res[0].tallies, res[1].tallies
    assert res[0].error is None and res[0].steps_run == WARMUP + 500
    assert win["steps"] == 500 and full["steps"] == WARMUP + 500
    for k in ("extracted", "wall", "ionized", "cx", "fpt_n"):
        assert np.array_equal(win[k], t1[k] - t0[k]), k
        assert np.array_equal(full[k], t1[k]), k
    bad = Server(8 << 30).serve([Request(0, 0.0, p, 100, warmup=100)])
    assert bad[0].error is not None and "warmup" in bad[0].error


def test_calibration_recovers_weight_and_temperature():
    from paper_1507_03392_amd.calibrate import ServedEvaluator, Targets, calibrate
    ev = ServedEvaluator(_make, [W.AR_IP_EV], STEPS, warmup=WARMUP, hbm_budget=8 << 30)
    (flow, power), = ev([(W_REF, TE_REF)])
    assert flow > 0 and power > 0
    res = calibrate(ev, Targets(power_W=power, gas_flow_pmA=flow, rtol=0.1), w0=2.5 * W_REF, te0_ev=TE_REF / 2.5,
                    max_iter=8)
    hist = [(round(h.w / W_REF, 3), round(h.te_ev / TE_REF, 3), round(h.gas_flow_pmA / flow, 3),
             round(h.power_W / power, 3)) for h in res.history]
    print(f"targets: {flow:.4g} pmA, {power:.4g} W; history (w, T_ew, flow, power relative to the reference): {hist}")
    assert res.converged, hist
    assert abs(res.gas_flow_pmA / flow - 1) <= 0.1 and abs(res.power_W / power - 1) <= 0.1
    assert res.w == pytest.approx(W_REF, rel=0.25) and res.te_ev == pytest.approx(TE_REF, rel=0.25)
