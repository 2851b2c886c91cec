"""GPU: the continuous-batching serving loop on small nanotube queries."""
import numpy as np
import pytest

import oracle
from paper_2403_15768_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_15768_amd import lbm, serve as mod

    lbm.load()
    return mod


def small_trace(n=6):
    return inputs.serving_trace(n, rate_per_s=200.0, nx=32, radius_range=(3, 6))


def test_each_result_same_alone_and_in_the_mix(serve):
    trace = small_trace()
    srv = serve.Server(mode="f32", hbm_budget=8 << 30, check_every=512, realtime=False, tune=False)
    mix = {r.qid: r for r in srv.run(trace)}
    assert all(r.status == "ok" for r in mix.values())
    # queries joined and left the running batch: it was never rebuilt
    assert srv.stats["batch_rebuilds"] == 0
    assert srv.stats["joins"] == srv.stats["leaves"] == len(trace)
    for q in trace[:3]:
        alone = serve.Server(mode="f32", hbm_budget=8 << 30, check_every=512, realtime=False,
                             tune=False).run([q])[0]
        assert alone.steps == mix[q.qid].steps
        assert alone.flux == mix[q.qid].flux  # bit for bit


def test_mixed_precision_reaches_the_same_flux(serve):
    trace = small_trace()
    f32 = {r.qid: r for r in serve.Server(mode="f32", hbm_budget=8 << 30, check_every=512,
                                          realtime=False, tune=False).run(trace)}
    mixed = serve.Server(mode="mixed", hbm_budget=8 << 30, check_every=512, realtime=False, tune=False)
    res = mixed.run(trace)
    assert mixed.stats["batch_rebuilds"] == 0
    assert mixed.stats["joins"] == 2 * len(trace)  # the half batch, then the FP32 one
    for r in res:
        assert r.status == "ok" and r.steps_half > 0
        assert abs(r.flux / f32[r.qid].flux - 1) < 1e-5, (r.qid, r.flux, f32[r.qid].flux)
    # same query alone in mixed mode: same result
    alone = serve.Server(mode="mixed", hbm_budget=8 << 30, check_every=512, realtime=False,
                         tune=False).run([trace[2]])[0]
    mixed_map = {r.qid: r for r in res}
    assert alone.flux == mixed_map[trace[2].qid].flux and alone.steps == mixed_map[trace[2].qid].steps


def test_admission_respects_the_budget(serve):
    trace = small_trace(5)
    one = max(serve.footprint(q, "f32") for q in trace)
    srv = serve.Server(mode="f32", hbm_budget=2 * one + 1, check_every=512, realtime=False, tune=True)
    res = srv.run(trace)
    assert srv.stats["max_active"] <= 2
    assert all(r.status == "ok" for r in res) and len(res) == 5
    assert srv.shape in (1, 2, 4, 8)


def test_realtime_trace_latencies(serve):
    trace = small_trace(4)
    srv = serve.Server(mode="f32", hbm_budget=8 << 30, check_every=512, realtime=True, tune=False)
    res = srv.run(trace)
    s = serve.summarize(res, 0.0)
    assert s["converged"] == 4 and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def oracle_tube(q):
    """The oracle's tube for a served query: same geometry, the friction from
    the oracle's own quadrature of the query's spectra at the same per-node
    plasmon frequencies."""
    from paper_2403_15768_amd import serve

    kw = serve.tube_params(q)
    o = oracle.Lattice(19, oracle.TUBE, kw["nx"], kw["ny"], kw["nz"], tau=q.tau,
                       force=(q.g, 0, 0), tube_radius=kw["tube_radius"],
                       tube_cy=kw["tube_cy"], tube_cz=kw["tube_cz"])
    om = inputs.tube_plasmon_frequencies(o.wall_coords(), kw["nx"], q.radius, kw["tube_cy"],
                                         kw["tube_cz"], q.spectral.omega0,
                                         inputs.rng_for("serving", 1000 + q.qid))
    sp = q.spectral
    _, lam = oracle.friction(oracle.Spectral(T=sp.T, omega0=sp.omega0, gamma_s=sp.gamma_s,
                                             omega_l=sp.omega_l, gamma_l=sp.gamma_l, a_l=sp.a_l,
                                             d=sp.d, nq=sp.nq, nw=sp.nw,
                                             lambda_target=sp.lambda_target), om)
    o.set_friction(lam)
    return o


@pytest.mark.parametrize("mode", ["f32", "mixed"])
def test_served_result_matches_the_oracle(serve, mode):
    # a served query (in a mix of four, FP32 storage or half storage handed
    # to FP32) against the oracle stepped the query's own number of steps:
    # flux and axial velocity field within the FP32 bar, 1e-5
    trace = inputs.serving_trace(4, rate_per_s=200.0, nx=32, radius_range=(3, 4))
    srv = serve.Server(mode=mode, hbm_budget=8 << 30, check_every=512, realtime=False,
                       tune=False, keep_fields=True)
    res = {r.qid: r for r in srv.run(trace)}
    q = trace[1]
    r = res[q.qid]
    assert r.status == "ok" and (r.steps_half > 0) == (mode == "mixed")
    o = oracle_tube(q)
    o.step(r.steps)
    qo = o.invariants()[0]
    uo = o.fields()[1]
    ferr = abs(r.flux / qo - 1)
    uerr = np.max(np.abs(r.ux - uo)) / np.max(np.abs(uo))
    print(f"served q{q.qid} R={q.radius} steps={r.steps} half={r.steps_half}: "
          f"flux err {ferr:.2e}, u err {uerr:.2e}", flush=True)
    assert ferr < 1e-5 and uerr < 1e-5
