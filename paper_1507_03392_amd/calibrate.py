"""Outer calibration of the source model (Sec. II; the gas-flow and power scans of Sec. III).

For a given magnetic configuration the model has two free inputs, the
macro-particle weight w and the warm electron temperature T_ew, and a
converged run is characterised by two outputs, the gas flow out of the
chamber (pmA) and the power carried out of the plasma, which equals the
coupled microwave power.  The paper sets the inputs so that the outputs hit
chosen values within a tolerance (10%, 5% for a fixed power).  With both
targets given, w and T_ew move together; with one target, only w moves and
T_ew stays at its starting value (the paper's scans at fixed T_ew).

Every evaluation of a candidate (w, T_ew) is a served run (serve.Server):
`warmup` steps, then `steps` steps whose tallies give the outputs through
diagnostics.gas_flow_pmA and diagnostics.coupled_power.  An iteration
evaluates the current point and its forward-difference neighbours as one
batch of concurrent requests, all with the same seed, so that their
differences are not drowned in sampling noise (common random numbers).

Update: Newton's method in log space on r = log(output / target), with the
Jacobian d r / d log(input) from forward differences of step h, solved in
the least-squares sense and each component clipped to a factor max_factor.
Both outputs count lost particles times the weight, so they scale about
linearly with w and the iteration settles in a few steps.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from . import diagnostics


@dataclasses.dataclass
class Targets:
    power_W: float | None = None
    gas_flow_pmA: float | None = None
    rtol: float = 0.1

    def names(self):
        out = []
        if self.gas_flow_pmA is not None:
            out.append("gas_flow_pmA")
        if self.power_W is not None:
            out.append("power_W")
        if not out:
            raise ValueError("no calibration target given")
        return out


@dataclasses.dataclass
class Point:
    w: float
    te_ev: float
    gas_flow_pmA: float
    power_W: float


@dataclasses.dataclass
class Calibration:
    w: float
    te_ev: float
    gas_flow_pmA: float
    power_W: float
    converged: bool
    iterations: int
    evaluations: int
    history: list


def outputs(tallies, weight, dt, te_ev, ip_ev):
    """(gas flow in pmA, coupled power in W) of one run's tallies.
    ip_ev: per species, the ionisation potentials from Q = 0 up."""
    flow = diagnostics.gas_flow_pmA(tallies, weight, dt)
    power = sum(diagnostics.coupled_power(tallies, weight, dt, te_ev, ip, species=s) for s, ip in enumerate(ip_ev))
    return flow, power


class ServedEvaluator:
    """Evaluates candidates as concurrent requests on one Server.

    make_params(w, te_ev) -> workload dict of the run at that weight and warm
    electron temperature (its rate tables, heating and zone settings are the
    workload's business); ip_ev: per species ionisation potentials (eV)."""

    def __init__(self, make_params, ip_ev, steps, warmup=0, hbm_budget=32 << 30, max_active=8, device="cuda"):
        from .serve import Server
        self.make_params = make_params
        self.ip_ev = ip_ev
        self.steps = steps
        self.warmup = warmup
        self.server = Server(hbm_budget, max_active=max_active, device=device)
        self.count = 0

    def __call__(self, points):
        from .serve import Request
        reqs, ps = [], []
        for i, (w, te) in enumerate(points):
            p = self.make_params(w, te)
            ps.append(p)
            reqs.append(Request(rid=i, arrival=0.0, params=p, steps=self.warmup + self.steps, warmup=self.warmup))
        res = self.server.serve(reqs)
        self.count += len(reqs)
        out = []
        for r, p, (w, te) in zip(res, ps, points):
            if r.error is not None:
                raise RuntimeError(f"calibration run at w={w:g}, T_ew={te:g} eV failed: {r.error}")
            out.append(outputs(r.tallies, p["weight"], p["dt"], te, self.ip_ev))
        return out


def calibrate(evaluate, targets, w0, te0_ev, max_iter=10, h=0.1, max_factor=3.0, te_bounds=(10.0, 1.0e5)):
    """Drive (w, T_ew) to the targets.  evaluate(list of (w, te)) returns a
    list of (gas flow pmA, power W), one per point."""
    names = targets.names()
    free = ["w"] if len(names) == 1 else ["w", "te"]
    want = np.array([getattr(targets, k) for k in names], dtype=np.float64)
    if np.any(want <= 0):
        raise ValueError("targets must be positive")
    x = np.log(np.array([w0, te0_ev], dtype=np.float64))
    lo, hi = math.log(te_bounds[0]), math.log(te_bounds[1])
    history = []
    evals = 0

    def inputs(p):  # a fixed T_ew is passed through unrounded
        return math.exp(p[0]), (math.exp(p[1]) if len(free) == 2 else float(te0_ev))

    def pick(o):
        d = {"gas_flow_pmA": o[0], "power_W": o[1]}
        return np.array([d[k] for k in names], dtype=np.float64)

    for it in range(max_iter + 1):
        pts = [x.copy()]
        for j in range(len(free)):
            e = x.copy()
            e[j] += h
            pts.append(e)
        # the last iteration only checks the point
        if it == max_iter:
            pts = pts[:1]
        outs = evaluate([inputs(p) for p in pts])
        evals += len(pts)
        y0 = pick(outs[0])
        history.append(Point(*inputs(x), outs[0][0], outs[0][1]))
        if np.all(y0 > 0) and np.all(np.abs(y0 / want - 1.0) <= targets.rtol):
            return Calibration(*inputs(x), outs[0][0], outs[0][1], True, it, evals, history)
        if it == max_iter or np.any(y0 <= 0):
            break
        r = np.log(y0 / want)
        J = np.empty((len(names), len(free)))
        for j in range(len(free)):
            yj = pick(outs[1 + j])
            if np.any(yj <= 0):
                raise RuntimeError("a calibration probe produced no losses: lengthen the runs")
            J[:, j] = (np.log(yj) - np.log(y0)) / h
        dx = np.linalg.lstsq(J, -r, rcond=None)[0]
        dx = np.clip(dx, -math.log(max_factor), math.log(max_factor))
        x[:len(free)] += dx
        x[1] = min(max(x[1], lo), hi)
    last = history[-1]
    return Calibration(last.w, last.te_ev, last.gas_flow_pmA, last.power_W, False, len(history) - 1, evals, history)
