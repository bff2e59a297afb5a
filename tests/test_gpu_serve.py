"""The continuous-batching server (paper_1507_03392_amd.serve) on the GPU.

* alone vs mix: every request of a small scan is served in a mix (several
  runs resident and overlapping on the device) and then alone; its tallies
  are the same bit for bit and its density grids within 1e-12 of the largest
  node value (FP64 atomics add in a different order), and both equal a plain
  step-by-step run of the same request;
* admission: resident runs never exceed the HBM budget, a request that can
  never fit or that the library rejects is answered with an error, and the
  rest complete.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _scan(n_req=6, steps=120, prec=W.PREC_FP64):
    from paper_1507_03392_amd.serve import Request
    rng = np.random.default_rng(5)
    reqs = []
    for i in range(n_req):
        n = int(rng.integers(3_000, 50_000))
        te = float(rng.uniform(300, 3000))
        p = W.base_params(n, 32, 32, 64, seed=100 + i, precision=prec)
        p.update(ne_in=float(rng.uniform(0.3, 2.5)) * 1e18, Te_in_eV=te)
        p["species"] = [W.argon(n0_m3=float(rng.uniform(3e16, 3e17)) * 100, te_ev=te)]
        reqs.append(Request(rid=i, arrival=0.002 * i, params=p, steps=steps))
    return reqs


def _same(r1, r2, what):
    assert r1.error is None and r2.error is None, (r1.error, r2.error)
    for k in ("extracted", "wall", "ionized", "cx", "cx_products"):
        assert np.array_equal(r1.tallies[k], r2.tallies[k]), f"{what}: {k}"
    for k in ("recycled", "anomalies", "steps"):
        assert r1.tallies[k] == r2.tallies[k], f"{what}: {k}"
    assert r1.tallies["coul_e"] == pytest.approx(r2.tallies["coul_e"], rel=1e-12)
    for f, d in r1.density.items():
        e = r2.density[f]
        assert np.abs(d - e).max() <= 1e-12 * max(1.0, np.abs(e).max()), f"{what}: density {f}"


@pytest.mark.parametrize("batched", [False, True])
@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_FP32])
def test_alone_vs_mix(prec, batched):
    import paper_1507_03392_amd as ecr
    from paper_1507_03392_amd.serve import Server, summary
    reqs = _scan(prec=prec)
    fields = (W.F_ION_N, W.F_ION_Q)
    # batched: the requests below 30k particles share one batch
    srv = Server(hbm_budget=1 << 34, max_active=4, density_fields=fields, batch_max_n=30_000 if batched else 0)
    mix = srv.serve(reqs)
    if batched:
        assert sum(r.params["n"] <= 30_000 for r in reqs) >= 2
    assert max(e[3] for e in srv.log) >= 2, "no two runs were ever resident together"
    s = summary(mix)
    assert s["completed"] == len(reqs) and s["p99_s"] >= s["p50_s"] > 0
    for r in reqs:
        alone = Server(hbm_budget=1 << 34, max_active=1, density_fields=fields).serve([r])[0]
        _same(mix[r.rid], alone, f"request {r.rid} mix vs alone")
        plain = ecr.Run(r.params)
        plain.init_ions()
        plain.step(r.steps)
        ref = type(alone)(rid=r.rid, n=r.params["n"], arrival=0.0, tallies=plain.tallies(),
                          density={f: plain.density(f)[0] for f in fields})
        _same(alone, ref, f"request {r.rid} served vs plain steps")
        assert alone.tallies["ionized"].sum() > 0


def test_batched_mix_with_large_requests():
    """Requests of 0.5M and 2M particles with their own slots beside a batch
    of small ones (arriving while the large ones run, some warmed up): each
    result equals a plain step-by-step run of its request."""
    import paper_1507_03392_amd as ecr
    from paper_1507_03392_amd.serve import Request, Server
    rng = np.random.default_rng(8)
    reqs = []
    for i, n in enumerate((2_000_000, 500_000, 12_000, 4_000, 60_000, 9_000, 20_000)):
        te = float(rng.uniform(300, 3000))
        p = W.base_params(n, 64, 64, 128, seed=200 + i, precision=W.PREC_FP32 if i % 2 else W.PREC_FP64)
        p.update(ne_in=float(rng.uniform(0.3, 2.5)) * 1e18, Te_in_eV=te)
        p["species"] = [W.argon(n0_m3=float(rng.uniform(3e16, 3e17)), te_ev=te)]
        # the large runs (600 steps, tens of ms) are still resident when the
        # small ones arrive a millisecond apart
        reqs.append(Request(rid=i, arrival=0.0 if i < 2 else 0.001 * i, params=p, steps=600 if i < 2 else 110,
                            warmup=30 if i in (1, 3) else 0))
    fields = (W.F_ION_N, W.F_ION_Q)
    srv = Server(hbm_budget=1 << 34, max_active=2, density_fields=fields, batch_max_n=100_000)
    out = srv.serve(reqs)
    assert max(e[3] for e in srv.log) >= 3
    for r in reqs:
        plain = ecr.Run(r.params)
        plain.init_ions()
        base = None
        if r.warmup:
            plain.step(r.warmup)
            base = plain.tallies()
        plain.step(r.steps - r.warmup)
        t = plain.tallies()
        from paper_1507_03392_amd.serve import tallies_window
        ref = type(out[0])(rid=r.rid, n=r.params["n"], arrival=0.0,
                           tallies=tallies_window(t, base) if base is not None else t,
                           density={f: plain.density(f)[0] for f in fields})
        _same(out[r.rid], ref, f"request {r.rid} ({r.params['n']} particles) served vs plain steps")
        plain.close()


@pytest.mark.parametrize("batch_max_n", [0, 100_000])
def test_admission_by_footprint_and_errors(batch_max_n):
    from paper_1507_03392_amd import footprint
    from paper_1507_03392_amd.serve import Request, Server
    reqs = _scan(n_req=5, steps=60)
    for r in reqs:
        r.arrival = 0.0
    big = max(footprint(r.params) for r in reqs)
    budget = int(2.2 * big)
    huge = W.base_params(4_000_000, 64, 64, 128, seed=7)
    bad = W.with_(reqs[0].params, dt=1e-3)  # rejected by the library (first-order MCC limit)
    reqs += [Request(rid=5, arrival=0.0, params=huge, steps=60), Request(rid=6, arrival=0.0, params=bad, steps=60)]
    srv = Server(hbm_budget=budget, max_active=4, batch_max_n=batch_max_n)
    out = srv.serve(reqs)
    assert sum(footprint(r.params) for r in reqs[:5]) > budget  # the budget binds
    assert all(e[4] <= budget for e in srv.log)
    assert 2 <= max(e[3] for e in srv.log) < 5  # the budget, not the slots, caps the batches
    assert out[5].error and "budget" in out[5].error
    assert out[6].error
    for r in out[:5]:
        assert r.error is None and r.tallies["steps"] == 60


def test_anomalies_are_reported_not_windowed():
    """A run whose state goes non-finite is answered with an error, both
    when it happens inside the warm-up and after it; the anomaly count of
    the result is the run's total, not the warm-up-subtracted window."""
    from paper_1507_03392_amd.serve import Request, Server
    good = _scan(n_req=1, steps=60)[0]
    p = W.base_params(4_000, 16, 16, 32, seed=11)
    st = W.random_state(p, seed=3, q_max=3, v_ev=1.0)
    st["vx"] = st["vx"].copy()
    st["vx"][17] = float("nan")
    reqs = [good,
            Request(rid=1, arrival=0.0, params=p, steps=60, warmup=20, state=st),
            Request(rid=2, arrival=0.0, params=p, steps=60, state=st)]
    out = Server(hbm_budget=1 << 34, max_active=3).serve(reqs)
    assert out[0].error is None
    for r in out[1:]:
        assert r.error is not None and "ECR_ENUMERIC" in r.error, r.error
        assert r.tallies is None or r.tallies["anomalies"] > 0
    # the run without warm-up carries its tallies, anomalies included
    assert out[2].tallies is not None and out[2].tallies["anomalies"] > 0
