"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Tolerances: FP64 results within 1e-12 relative of the oracle, FP32 velocity
fields within 1e-5 (normalised by the largest axial velocity), wall geometry
bit-exact.  Inputs are seeded and synthetic (paper_2403_15768_amd.inputs).
"""
import math

import numpy as np
import pytest

import oracle
from paper_2403_15768_amd import inputs

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_15768_amd import lbm as mod

    mod.load()
    return mod


def say(*a):
    print(*a, flush=True)


def vel_err(g, o):
    """max |u_gpu - u_ora| per component over max |u_x,ora| (and rho - 1)."""
    rg, ro = g.fields(), o.fields()
    ref = np.max(np.abs(ro[1]))
    errs = [np.max(np.abs(rg[k] - ro[k])) / ref for k in (1, 2, 3)]
    return max(errs), np.max(np.abs(rg[0] - ro[0]))


def pair(lbm, lattice, geometry, nx, ny, nz, tau, g, precision, **kw):
    G = lbm.Channel(lattice, geometry, nx, ny, nz, tau=tau, force=(g, 0, 0), precision=precision, **kw)
    O = oracle.Lattice(lattice, geometry, nx, ny, nz, tau=tau, force=(g, 0, 0), **kw)
    return G, O


def tube_kw(R):
    ny, nz, cy, cz = inputs.tube_box(R)
    return dict(tube_radius=float(R), tube_cy=cy, tube_cz=cz), ny, nz


# ------------------------------------------------------------------ geometry
@pytest.mark.parametrize("case", ["slab", "duct", "d2q9", "tube8", "tube32_full", "ragged"])
def test_wall_geometry_bit_exact(lbm, case):
    say("geometry", case)
    if case == "slab":
        args = (19, lbm.SLAB, 16, 9, 7, {})
    elif case == "duct":
        args = (19, lbm.DUCT, 16, 9, 7, {})
    elif case == "d2q9":
        args = (9, lbm.SLAB, 64, 30, 1, {})
    elif case == "ragged":
        args = (19, lbm.DUCT, 37, 5, 3, {})
    else:
        R = 8 if case == "tube8" else 32
        kw, ny, nz = tube_kw(R)
        args = (19, lbm.TUBE, 512 if R == 32 else 20, ny, nz, kw)
    q, geom, nx, ny, nz, kw = args
    G = lbm.Channel(q, geom, nx, ny, nz, tau=0.7, precision="f32", **kw)
    O = oracle.Lattice(q, geom, nx, ny, nz, tau=0.7, **kw)
    assert G.fluid_count == O.fluid_count
    assert G.wall_count == O.wall_count
    assert np.array_equal(G.wall_coords(), O.wall_coords())
    lg, lo = G.wall_links(), O.wall_links()
    assert np.array_equal(lg > 0, lo > 0)
    assert np.max(np.abs(lg - lo)) < 1e-14
    if case == "tube32_full":
        assert G.fluid_count == 1652736 and G.wall_count == 129024


# ------------------------------------------------------------------ channel
@pytest.mark.parametrize("lam", [math.inf, 0.025])
def test_channel2d_full_config_fp64(lbm, lam):
    # D2Q9 64 x 32 box (rows 0 and 31 solid), tau 0.8, g 1e-6, 10,000 steps
    say("channel2d fp64 lam", lam)
    G, O = pair(lbm, 9, lbm.SLAB, 64, 30, 1, 0.8, 1e-6, "f64")
    G.set_friction(lam)
    O.set_friction(lam)
    G.step(10000)
    O.step(10000)
    eu, er = vel_err(G, O)
    say("  u err", eu, "rho err", er)
    assert eu < TOL["f64"] and er < 1e-14
    qg, mg, dg = G.invariants()
    qo, mo, do = O.invariants()
    assert abs(qg / qo - 1) < TOL["f64"]
    assert abs(dg - do) < 1e-12
    pg, po = G.populations(), O.get_populations()
    assert np.max(np.abs(pg - po)) < 1e-12 * np.max(np.abs(po))


def test_channel2d_run_to_steady_closed_form(lbm):
    say("channel2d run_to_steady")
    H, tau, g, lam = 30, 0.8, 1e-6, 0.025
    G = lbm.Channel(9, lbm.SLAB, 64, H, 1, tau=tau, force=(g, 0, 0), precision="f64")
    G.set_friction(lam)
    n = G.run_to_steady(rel_tol=1e-12, check_every=1000, max_steps=200000)
    nu = (tau - 0.5) / 3
    y = np.arange(H) - (H - 1) / 2
    ue = g / (2 * nu) * (H * H / 4 - y * y) + g * H / (2 * lam) + g * (16 * (tau - 0.5) ** 2 - 3) / (24 * nu)
    u = G.field(1)[0]
    say("  steps", n, "err", np.max(np.abs(u - ue[:, None])) / ue.max())
    assert np.max(np.abs(u - ue[:, None])) / ue.max() < 1e-9


def test_couette_fp64(lbm):
    say("couette")
    G, O = pair(lbm, 9, lbm.SLAB, 8, 20, 1, 0.9, 0.0, "f64", wall_velocity_top=1e-3)
    G.set_friction(0.05)
    O.set_friction(0.05)
    G.step(3000)
    O.step(3000)
    eu, _ = vel_err(G, O)
    assert eu < TOL["f64"]


# ------------------------------------------------------------------ duct
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_duct_replica_random_friction(lbm, precision):
    say("duct replica", precision)
    nx, ny, nz = 48, 24, 12
    G, O = pair(lbm, 19, lbm.DUCT, nx, ny, nz, 0.7, 1e-6, precision)
    lam = inputs.duct_friction(G.wall_coords(), nx, ny, nz, inputs.rng_for("duct", 11))
    G.set_friction(lam)
    O.set_friction(lam)
    G.step(1000)
    O.step(1000)
    eu, er = vel_err(G, O)
    say("  u err", eu)
    assert eu < TOL[precision]
    qg, _, dg = G.invariants()
    qo, _, do = O.invariants()
    assert abs(qg / qo - 1) < TOL[precision]


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_duct_full_size_truncated(lbm, precision):
    # the 256 x 128 x 64 duct at full size, few steps (oracle cost)
    say("duct full size", precision)
    nx, ny, nz = 256, 128, 64
    G, O = pair(lbm, 19, lbm.DUCT, nx, ny, nz, 0.7, 1e-6, precision)
    lam = inputs.duct_friction(G.wall_coords(), nx, ny, nz, inputs.rng_for("duct", 0))
    G.set_friction(lam)
    O.set_friction(lam)
    G.step(3)
    O.step(3)
    eu, _ = vel_err(G, O)
    say("  u err", eu)
    assert eu < TOL[precision]
    if precision == "f64":
        pg, po = G.populations(), O.get_populations()
        assert np.max(np.abs(pg - po)) < 1e-12 * np.max(np.abs(po))


def test_duct_full_steps_fp32_against_fp64(lbm):
    # 20,000 steps at full size: FP32 against the FP64 GPU path (itself pinned
    # to the oracle above); reported as the FP32 error of the configuration
    say("duct 20000 steps fp32 vs fp64")
    nx, ny, nz = 256, 128, 64
    out = {}
    for prec in ("f64", "f32"):
        G = lbm.Channel(19, lbm.DUCT, nx, ny, nz, tau=0.7, force=(1e-6, 0, 0), precision=prec)
        lam = inputs.duct_friction(G.wall_coords(), nx, ny, nz, inputs.rng_for("duct", 0))
        G.set_friction(lam)
        G.step(20000)
        out[prec] = (G.field(1), G.invariants())
        G.close()
    ref = np.max(np.abs(out["f64"][0]))
    e = np.max(np.abs(out["f32"][0] - out["f64"][0])) / ref
    eq = abs(out["f32"][1][0] / out["f64"][1][0] - 1)
    say("  fp32 field err", e, "flux err", eq)
    assert e < 1e-5 and eq < 1e-5


# ------------------------------------------------------------------ tube
def small_spectral(nq=32, nw=128, seed=3):
    sp = inputs.draw_spectral(inputs.rng_for("tube", seed), nq=nq, nw=nw)
    return sp


def oracle_spectral(sp, **kw):
    return oracle.Spectral(T=sp.T, omega0=sp.omega0, gamma_s=sp.gamma_s, omega_l=sp.omega_l,
                           gamma_l=sp.gamma_l, a_l=sp.a_l, d=sp.d, nq=sp.nq, nw=sp.nw,
                           lambda_target=sp.lambda_target, **kw)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_tube_replica_spectral_friction(lbm, precision):
    say("tube replica", precision)
    R = 10
    kw, ny, nz = tube_kw(R)
    nx = 40
    G, O = pair(lbm, 19, lbm.TUBE, nx, ny, nz, 0.8, 1e-6, precision, **kw)
    sp = small_spectral()
    om = inputs.tube_plasmon_frequencies(G.wall_coords(), nx, R, kw["tube_cy"], kw["tube_cz"],
                                         sp.omega0, inputs.rng_for("tube", 5), sigma=4.0)
    G.set_friction_spectral(sp, om)
    lam_g = G.get_friction()
    _, lam_o = oracle.friction(oracle_spectral(sp), om)
    assert np.max(np.abs(lam_g / lam_o - 1)) < 1e-12
    O.set_friction(lam_o)
    G.step(1000)
    O.step(1000)
    eu, _ = vel_err(G, O)
    say("  u err", eu)
    assert eu < TOL[precision]


def test_tube_full_size_truncated_fp32(lbm):
    say("tube full size fp32")
    R, nx = 32, 512
    kw, ny, nz = tube_kw(R)
    G, O = pair(lbm, 19, lbm.TUBE, nx, ny, nz, 0.8, 1e-6, "f32", **kw)
    sp = inputs.draw_spectral(inputs.rng_for("tube", 0))
    om = inputs.tube_plasmon_frequencies(G.wall_coords(), nx, R, kw["tube_cy"], kw["tube_cz"],
                                         sp.omega0, inputs.rng_for("tube", 1))
    G.set_friction_spectral(sp, om)
    lam_g, raw_g = G.get_friction(raw=True)
    # quadrature parity on sampled wall nodes (the oracle costs ~10 ms a node)
    idx = np.random.default_rng(0).choice(len(om), 48, replace=False)
    raw_o, lam_o = oracle.friction(oracle_spectral(sp), om[idx])
    assert np.max(np.abs(raw_g[idx] / raw_o - 1)) < 1e-12
    assert np.max(np.abs(lam_g[idx] / lam_o - 1)) < 1e-12
    assert abs(raw_g[-1] / oracle.friction_raw(oracle_spectral(sp), sp.omega0) - 1) < 1e-12
    O.set_friction(lam_g)
    G.step(3)
    O.step(3)
    eu, _ = vel_err(G, O)
    say("  u err", eu)
    assert eu < TOL["f32"]


@pytest.mark.parametrize("nq,nw,disp", [(1, 1, 1), (2, 4, 0), (4, 16, 1), (7, 1500, 1), (300, 64, 1)])
def test_quadrature_grids(lbm, nq, nw, disp):
    say("quadrature", nq, nw, disp)
    G = lbm.Channel(19, lbm.DUCT, 3, 4, 4, tau=0.7, precision="f64")
    sp = small_spectral(nq=nq, nw=nw, seed=9)
    sp.dispersion = disp
    om = np.linspace(0.3, 4.0, G.wall_count)
    G.set_friction_spectral(sp, om)
    lam_g, raw_g = G.get_friction(raw=True)
    raw_o, lam_o = oracle.friction(oracle_spectral(sp, dispersion=disp), om)
    assert np.max(np.abs(raw_g[:-1] / raw_o - 1)) < 1e-13
    assert np.max(np.abs(lam_g / lam_o - 1)) < 1e-13


@pytest.mark.parametrize("nq,nw,disp,coupling,v_l", [
    (1, 1, 1, 1, 0.0), (2, 4, 0, 1, 0.5), (4, 16, 1, 0, 0.7), (7, 1500, 1, 1, 0.3),
    (300, 64, 1, 1, 0.0), (256, 1024, 1, 1, 0.4)])
def test_screened_quadrature_grids(lbm, nq, nw, disp, coupling, v_l):
    # the screening denominator and the dispersive liquid mode (complex
    # responses): same sums as the oracle up to summation order
    say("screened quadrature", nq, nw, disp, coupling, v_l)
    G = lbm.Channel(19, lbm.DUCT, 3, 4, 4, tau=0.7, precision="f64")
    sp = small_spectral(nq=nq, nw=nw, seed=9)
    sp.dispersion, sp.coupling, sp.v_l = disp, coupling, v_l
    om = np.linspace(0.3, 4.0, G.wall_count)
    G.set_friction_spectral(sp, om)
    lam_g, raw_g = G.get_friction(raw=True)
    raw_o, lam_o = oracle.friction(oracle_spectral(sp, dispersion=disp, coupling=coupling,
                                                   v_l=v_l), om)
    assert np.max(np.abs(raw_g[:-1] / raw_o - 1)) < 1e-12
    assert np.max(np.abs(lam_g / lam_o - 1)) < 1e-12
    if coupling and nq >= 32:  # the screening changes the result (a one-point
        # grid samples q = q_max / 2, where e^{-2qd} leaves it negligible)
        raw_u, _ = oracle.friction(oracle_spectral(sp, dispersion=disp, v_l=v_l), om)
        assert np.max(np.abs(raw_u / raw_o - 1)) > 1e-3


def test_screened_quadrature_full_tube_sampled(lbm):
    # the R = 32 tube (129,024 wall nodes, 256 x 1024 points): eight nodes
    # and the reference recomputed one by one by the oracle
    say("screened quadrature, full tube")
    R, nx = 32, 512
    kw, ny, nz = tube_kw(R)
    G = lbm.Channel(19, lbm.TUBE, nx, ny, nz, tau=0.8, precision="f32", **kw)
    sp = inputs.draw_spectral(inputs.rng_for("tube", 0))
    sp.coupling, sp.v_l = 1, 0.5
    om = inputs.tube_plasmon_frequencies(G.wall_coords(), nx, R, kw["tube_cy"], kw["tube_cz"],
                                         sp.omega0, inputs.rng_for("tube", 1))
    G.set_friction_spectral(sp, om)
    lam_g, raw_g = G.get_friction(raw=True)
    osp = oracle_spectral(sp, coupling=1, v_l=0.5)
    pick = np.random.default_rng(4).choice(G.wall_count, 8, replace=False)
    for k in pick:
        ref = oracle.friction_raw(osp, om[k])
        assert abs(raw_g[k] / ref - 1) < 1e-12
    assert abs(raw_g[-1] / oracle.friction_raw(osp, sp.omega0) - 1) < 1e-12
    assert np.all(lam_g > 0)


def test_screened_spectral_settings_rejected(lbm):
    G = lbm.Channel(19, lbm.DUCT, 3, 4, 4, tau=0.7, precision="f64")
    om = np.full(G.wall_count, 1.5)
    for coupling, v_l in [(2, 0.0), (-1, 0.0), (1, -0.1), (1, float("nan")), (0, float("inf"))]:
        sp = small_spectral()
        sp.coupling, sp.v_l = coupling, v_l
        with pytest.raises(lbm.LBMError):
            G.set_friction_spectral(sp, om)
    G.step(2)


# ------------------------------------------------------------------ edge cases
@pytest.mark.parametrize("case", ["nx1", "ragged37", "ragged100", "ny1_d2q9", "slab_d3q19",
                                  "tube_r3", "nx600"])
def test_edge_shapes_fp64(lbm, case):
    say("edge", case)
    kw = {}
    if case == "nx1":
        q, geom, nx, ny, nz = 19, lbm.DUCT, 1, 6, 5
    elif case == "ragged37":
        q, geom, nx, ny, nz = 19, lbm.DUCT, 37, 6, 5
    elif case == "ragged100":
        q, geom, nx, ny, nz = 19, lbm.SLAB, 100, 7, 3
    elif case == "ny1_d2q9":
        q, geom, nx, ny, nz = 9, lbm.SLAB, 10, 1, 1
    elif case == "slab_d3q19":
        q, geom, nx, ny, nz = 19, lbm.SLAB, 8, 12, 4
    elif case == "nx600":
        q, geom, nx, ny, nz = 19, lbm.DUCT, 600, 3, 3
    else:
        kw, ny, nz = tube_kw(3)
        q, geom, nx = 19, lbm.TUBE, 5
    G, O = pair(lbm, q, geom, nx, ny, nz, 0.65, 1e-5, "f64", **kw)
    lam = 0.01 + 0.1 * np.random.default_rng(1).random(G.wall_count)
    G.set_friction(lam)
    O.set_friction(lam)
    G.step(150)
    O.step(150)
    eu, er = vel_err(G, O)
    assert eu < TOL["f64"] and er < 1e-13


def test_mass_conservation_fp64(lbm):
    say("mass conservation")
    nx, ny, nz = 64, 20, 16
    G = lbm.Channel(19, lbm.DUCT, nx, ny, nz, tau=0.7, force=(1e-5, 0, 0), precision="f64")
    lam = inputs.duct_friction(G.wall_coords(), nx, ny, nz, inputs.rng_for("duct", 3), std=0.05)
    G.set_friction(lam)
    G.step(2000)
    _, m, dm = G.invariants()
    assert abs(dm) < 1e-15 * G.fluid_count


# ------------------------------------------------------------------ runtime
def test_graph_and_plain_launches_bitwise_equal_and_deterministic(lbm):
    say("determinism")
    nx, ny, nz = 64, 16, 8
    runs = []
    for mode in ("graph", "plain", "graph"):
        G = lbm.Channel(19, lbm.DUCT, nx, ny, nz, tau=0.7, force=(1e-5, 0, 0), precision="f32")
        G.set_friction(inputs.duct_friction(G.wall_coords(), nx, ny, nz, inputs.rng_for("duct", 4)))
        if mode == "graph":
            G.step(200)
        else:
            for _ in range(200):
                G.step(1)
        runs.append((G.get_state()[0], G.invariants()))
        assert G.step_count == 200
    assert np.array_equal(runs[0][0], runs[1][0]) and np.array_equal(runs[0][0], runs[2][0])
    assert runs[0][1] == runs[2][1]


def test_checkpoint_round_trip(lbm):
    say("checkpoint")
    args = (19, lbm.DUCT, 40, 10, 8)
    A = lbm.Channel(*args, tau=0.7, force=(1e-5, 0, 0), precision="f32")
    A.set_friction(0.03)
    A.step(77)
    buf, step = A.get_state()
    A.step(70)
    ref = A.get_state()[0]
    B = lbm.Channel(*args, tau=0.7, force=(1e-5, 0, 0), precision="f32")
    B.set_friction(0.03)
    B.set_state(buf, step)
    B.step(70)
    assert np.array_equal(B.get_state()[0], ref) and B.step_count == 147


def test_error_paths(lbm):
    say("errors")
    G = lbm.Channel(19, lbm.DUCT, 16, 6, 6, tau=0.7, force=(1e-5, 0, 0), precision="f64")
    G.set_friction(0.05)
    with pytest.raises(lbm.LBMError) as e:
        G.set_friction(-1.0)
    assert e.value.status == -1
    lam = np.full(G.wall_count, 0.05)
    lam[3] = np.nan
    with pytest.raises(lbm.LBMError):
        G.set_friction(lam)
    assert np.all(G.get_friction() == 0.05)  # unchanged
    with pytest.raises(lbm.LBMError) as e:
        G.run_to_steady(rel_tol=1e-14, check_every=10, max_steps=30)
    assert e.value.status == -4
    buf, step = G.get_state()
    f = buf.view(np.float64).copy()
    f[5] = np.nan
    G.set_state(f.view(np.uint8), step)
    with pytest.raises(lbm.LBMError) as e:
        G.invariants()
    assert e.value.status == -5


# ------------------------------------------------------------------ precision
def test_fp32_storage_at_steady_state_closed_form(lbm):
    # 60,000 steps is steady for the 30-row channel; float storage with
    # stochastic rounding stays within 2e-6 of the exact discrete profile
    # (round to nearest stalls ~2e-5 short of it)
    say("fp32 steady state")
    H, tau, g, lam = 30, 0.8, 1e-6, 0.025
    G = lbm.Channel(9, lbm.SLAB, 64, H, 1, tau=tau, force=(g, 0, 0), precision="f32")
    G.set_friction(lam)
    G.step(60000)
    nu = (tau - 0.5) / 3
    y = np.arange(H) - (H - 1) / 2
    ue = g / (2 * nu) * (H * H / 4 - y * y) + g * H / (2 * lam) + g * (16 * (tau - 0.5) ** 2 - 3) / (24 * nu)
    u = G.field(1)[0]
    err = np.max(np.abs(u - ue[:, None])) / ue.max()
    q = G.invariants()[0]
    qerr = abs(q / (ue.sum()) - 1)
    say("  field err", err, "flux err", qerr)
    assert err < 2e-6 and qerr < 2e-6


def test_f16s_storage_error_bounded(lbm):
    # half-precision deviations: the error against the FP64 oracle is
    # reported; measured 3.6e-4 of the axial velocity and 3.4e-6 of the flux
    # after 1000 steps, held to about 3x that
    say("f16s replica")
    nx, ny, nz = 48, 24, 12
    G, O = pair(lbm, 19, lbm.DUCT, nx, ny, nz, 0.7, 1e-6, "f16s")
    lam = inputs.duct_friction(G.wall_coords(), nx, ny, nz, inputs.rng_for("duct", 11))
    G.set_friction(lam)
    O.set_friction(lam)
    G.step(1000)
    O.step(1000)
    eu, _ = vel_err(G, O)
    qg, qo = G.invariants()[0], O.invariants()[0]
    say("  f16s u err", eu, "flux err", abs(qg / qo - 1))
    assert eu < 1.1e-3 and abs(qg / qo - 1) < 1e-5


@pytest.mark.parametrize("precision", ["f16s", "f32"])
def test_stored_values_are_stochastically_rounded(lbm, precision):
    # one step from a random state that the storage holds exactly: every
    # stored population against the FP64 oracle's value of the same step,
    # in units of the storage spacing there.  Stochastic rounding keeps each
    # value at one of the two neighbours of the exact one (|r| < 1), with no
    # bias (mean r = 0) and, unlike round-to-nearest (|r| <= 1/2, mean |r| =
    # 1/4), lands on the farther neighbour a quarter of the time (mean |r| =
    # 1/3).  Half storage holds the deviations times 2^12, its arithmetic is
    # float (about 2^-13 of a half spacing off the FP64 value).
    say("stochastic rounding", precision)
    nx, ny, nz = 40, 12, 10
    G, O = pair(lbm, 19, lbm.DUCT, nx, ny, nz, 0.8, 1e-5, precision)
    lam = inputs.duct_friction(G.wall_coords(), nx, ny, nz, inputs.rng_for("duct", 13))
    G.set_friction(lam)
    O.set_friction(lam)
    rng = np.random.default_rng(21)
    g0 = rng.normal(0.0, 1e-3, (19, nz, ny, nx))
    if precision == "f16s":
        scale, st = 4096.0, np.float16
    else:
        scale, st = 1.0, np.float32
    g0 = (g0 * scale).astype(st).astype(np.float64) / scale  # exactly representable
    G.set_populations(g0, step=5)
    O.set_populations(g0, step=5)
    assert np.array_equal(G.populations(), g0)
    G.step(1)
    O.step(1)
    stored = (G.populations() * scale).ravel()
    exact = (O.get_populations() * scale).ravel()
    assert np.array_equal(stored.astype(st).astype(np.float64), stored)
    lo = np.minimum(np.abs(stored), np.abs(exact)).astype(st)
    sp = np.spacing(lo).astype(np.float64)
    # float arithmetic is a few float ulps of the terms it adds off the FP64
    # value: where they cancel to a result near zero that can exceed the
    # (tiny) spacing there, so the bound carries it and the statistics skip
    # those values
    slack = 8 * 2.0**-24 * np.max(np.abs(exact)) if precision == "f16s" else 0.0
    assert np.all(np.abs(stored - exact) <= 1.001 * sp + slack)
    keep = sp > 64 * slack
    r = (stored - exact)[keep] / sp[keep]
    far = np.mean(np.abs(r) > 0.5)
    say("  values", r.size, "max |r|", np.max(np.abs(r)), "mean r", np.mean(r), "mean |r|",
        np.mean(np.abs(r)), "share |r| > 1/2", far)
    assert r.size > stored.size // 2  # measured: 57,158 of 91,200 for half storage
    assert np.max(np.abs(r)) < 1.001
    assert abs(np.mean(r)) < 0.01  # 0.5 / sqrt(45,600) = 0.0023 per standard deviation
    assert 0.31 < np.mean(np.abs(r)) < 0.36
    assert 0.22 < far < 0.28


@pytest.mark.parametrize("nx", [40, 72])  # 72: the half and float x-lines are padded differently
def test_transfer_state_across_precisions(lbm, nx):
    say("transfer", nx)
    ny, nz = 12, 10
    kw = dict(tau=0.75, force=(1e-6, 0, 0))
    H = lbm.Channel(19, lbm.DUCT, nx, ny, nz, precision="f16s", **kw)
    lam = inputs.duct_friction(H.wall_coords(), nx, ny, nz, inputs.rng_for("duct", 12))
    H.set_friction(lam)
    H.step(300)
    F = lbm.Channel(19, lbm.DUCT, nx, ny, nz, precision="f32", **kw)
    F.transfer_from(H)
    assert F.step_count == 300
    assert np.array_equal(F.populations(), H.populations())  # half -> float is exact
    assert np.array_equal(F.get_friction(), H.get_friction())
    # same precision: a transfer then stepping is bit-identical to stepping
    F2 = lbm.Channel(19, lbm.DUCT, nx, ny, nz, precision="f32", **kw)
    F2.transfer_from(F)
    F.step(130)
    F2.step(130)
    assert np.array_equal(F.get_state()[0], F2.get_state()[0])


# ------------------------------------------------------------------ checked steps
@pytest.mark.parametrize("case", ["duct_f64", "duct_f32", "tube_f32", "d2q9_f64", "duct_f16s",
                                  "duct_f32_thermal", "slab_f64_electrons"])
def test_checked_step_equals_invariants_before_the_last_step(lbm, case):
    # a checked step's fused FP64 sums are the invariants of the state it
    # reads: bit for bit where the arithmetic is double, and within the
    # float arithmetic's rounding for half storage; the cases that cannot
    # fuse (noise, electron lines) take a separate moments pass, exactly
    say("checked step", case)
    geom, prec = case.split("_")[0], case.split("_")[1]
    kw = {}
    if geom == "duct":
        args = (19, lbm.DUCT, 48, 20, 12)
    elif geom == "tube":
        kw, ny, nz = tube_kw(7)
        args = (19, lbm.TUBE, 40, ny, nz)
    elif geom == "slab":
        args = (19, lbm.SLAB, 33, 9, 6)
    else:
        args = (9, lbm.SLAB, 64, 30, 1)

    def make():
        G = lbm.Channel(*args, tau=0.75, force=(1e-5, 0, 0), precision=prec, **kw)
        G.set_friction(np.random.default_rng(4).uniform(0.0, 0.2, G.wall_count))
        if case.endswith("thermal"):
            G.set_thermal(1e-7, 2, 3)
        if case.endswith("electrons"):
            G.set_electrons(0.9, 1.0, 0.05, 1e-6)
        return G

    A, B = make(), make()
    for n in (1, 70, 129):
        A.step(n - 1)
        ref = A.invariants()
        A.step(1)
        B.step_checked(n)
        q, m, dm, at = B.checked_invariants()
        assert at == A.step_count - 1 == B.step_count - 1
        assert np.array_equal(A.get_state()[0], B.get_state()[0])  # same steps
        if prec == "f16s":
            assert abs(q / ref[0] - 1) < 1e-6 and abs(dm - ref[2]) < 1e-9 * B.fluid_count
        else:
            assert (q, m, dm) == ref
        assert B.checked_invariants()[:3] == (q, m, dm)  # may be read again
    B.invariants()  # a reduction pass of its own: the checked sums are gone
    with pytest.raises(lbm.LBMError):
        B.checked_invariants()
    with pytest.raises(lbm.LBMError):
        B.step_checked(0)


# ------------------------------------------------------------------ block width
@pytest.mark.parametrize("case", ["duct_f32", "tube_f64", "slab_f16s_thermal", "masked_f32",
                                  "open_f64", "electrons_f32"])
def test_block_width_never_changes_results(lbm, case):
    # the step kernel's block width (set directly, or chosen by the
    # autotuner) changes which threads update which cells, not one bit of
    # the result; reductions keep the default blocks
    say("block width", case)
    geom, prec = case.split("_")[0], case.split("_")[1]
    kw = {}

    def make():
        if geom == "duct" or geom == "open":
            G = lbm.Channel(19, lbm.DUCT, 200, 10, 8, tau=0.7, force=(1e-5, 0, 0), precision=prec)
        elif geom == "tube":
            k, ny, nz = tube_kw(6)
            G = lbm.Channel(19, lbm.TUBE, 150, ny, nz, tau=0.8, force=(1e-5, 0, 0),
                            precision=prec, **k)
        elif geom == "masked":
            solid = inputs.corrugated_mask(300, 20, inputs.rng_for("corrugated", 5), amp=3,
                                           base=3)
            G = lbm.Channel(19, lbm.MASKED, 300, 20, 4, tau=0.7, force=(1e-5, 0, 0),
                            precision=prec, solid=solid)
        else:  # slab (with noise or electron lines)
            G = lbm.Channel(19, lbm.SLAB, 130, 9, 6, tau=0.7, force=(1e-5, 0, 0), precision=prec)
        G.set_friction(np.random.default_rng(9).uniform(0.0, 0.2, G.wall_count))
        if case.endswith("thermal"):
            G.set_thermal(1e-7, 2, 4)
        if geom == "open":
            G.set_open_ends(1.0 + 1e-5, 1.0 - 1e-5)
        if geom == "electrons":
            G.set_electrons(0.9, 1.0, 0.05, 1e-6)
        return G

    ref = make()
    ref.step(70)
    ref.step_checked(3)
    qr = ref.checked_invariants()
    widths = [w for w in (64, 128, 256, 512) if w <= (ref.nx + 63) // 64 * 64]
    default = min((ref.nx + 63) // 64 * 64, 512)  # the plan's width, which the tuner may keep
    for bx in widths + ["tuned"]:
        G = make()
        if bx == "tuned":
            w, us = G.tune(retime=True)
            assert w in widths + [default] and us > 0
            assert G.tune()[1] == 0.0  # the cached choice
        else:
            G.set_block(bx)
        G.step(70)
        G.step_checked(3)
        if bx == "tuned":  # a search between a checked step and its reduction: the
            G.tune(retime=True)  # tuner's steps are undone, the partials kept
            assert G.step_count == ref.step_count
        assert np.array_equal(G.get_state()[0], ref.get_state()[0]), bx
        assert G.checked_invariants() == qr
    with pytest.raises(lbm.LBMError):
        ref.set_block(96)
