"""GPU parity of open x ends (the Neumann-like inlet and outlet) against the
oracle, through the C ABI.

Tolerances as for the periodic channels: FP64 within 1e-12 relative of the
oracle, FP32 storage within 1e-5 of the largest axial velocity, thermal noise
with double storage within 1e-12 (binary64 normals on both sides), half
storage within about 3x its measured error.  Closed form: the pressure-driven
Poiseuille profile of the equivalent body force; on nanotubes, a density
exactly linear along x and a flux free of end effects.  Exact: graph replays
equal plain launches bit for bit.
"""
import math

import numpy as np
import pytest

import oracle
from test_oracle_lb import poiseuille_exact

pytestmark = pytest.mark.gpu


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


# several 64-lane tiles and ragged tails; D3Q19 slabs wrap in z
CASES = {"d2q9": (9, "SLAB", 150, 20, 1), "d3q19": (19, "SLAB", 70, 12, 5),
         "duct": (19, "DUCT", 37, 10, 8), "duct_long": (19, "DUCT", 200, 6, 5)}


def build(lbm, case, precision, rho=(1.0 + 2e-5, 1.0 - 1e-5), force=(1e-6, 0, 0)):
    q, geom, nx, ny, nz = CASES[case]
    G = lbm.Channel(q, getattr(lbm, geom), nx, ny, nz, tau=0.72, force=force, precision=precision)
    O = oracle.Lattice(q, getattr(oracle, geom), nx, ny, nz, tau=0.72, force=force)
    lam = np.random.default_rng(3).uniform(0.0, 0.3, G.wall_count)
    G.set_friction(lam)
    O.set_friction(lam)
    G.set_open_ends(*rho)
    O.set_open_ends(*rho)
    return G, O


def errs(G, O):
    rg, ro = G.fields(), O.fields()
    ref = np.abs(ro[1]).max()
    return (max(np.abs(rg[k] - ro[k]).max() for k in (1, 2, 3)) / ref,
            np.abs(rg[0] - ro[0]).max())


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_parity_over_graph_and_plain_steps(lbm, case, precision):
    say("open ends parity", case, precision)
    G, O = build(lbm, case, precision)
    n = 229  # three 64-step graph replays, then single launches
    G.step(n)
    O.step(n)
    eu, er = errs(G, O)
    qg, mg, _ = G.invariants()
    qo, mo, _ = O.invariants()
    say(f"  u {eu:.2e}  rho {er:.2e}  flux {abs(qg / qo - 1):.2e}  mass {abs(mg / mo - 1):.2e}")
    tol = 1e-12 if precision == "f64" else 1e-5
    assert eu < tol and abs(qg / qo - 1) < tol
    assert er < (1e-14 if precision == "f64" else 1e-6)
    assert abs(mg / mo - 1) < (1e-14 if precision == "f64" else 1e-8)


@pytest.mark.parametrize("precision", ["f64", "f32", "f16s"])
def test_graph_and_plain_launches_bitwise(lbm, precision):
    say("open ends graph = plain", precision)
    A, _ = build(lbm, "duct", precision)
    B, _ = build(lbm, "duct", precision)
    A.step(128)
    for _ in range(128):
        B.step(1)
    assert np.array_equal(A.get_state()[0], B.get_state()[0])


def test_open_ends_with_thermal_noise(lbm):
    say("open ends + thermal")
    G, O = build(lbm, "d3q19", "f64")
    for L in (G, O):
        L.set_thermal(1e-7, 2, 5)
    G.step(101)
    O.step(101)
    eu, _ = errs(G, O)
    say(f"  u {eu:.2e}")
    assert eu < 1e-12  # binary64 normals with double storage


def test_pressure_driven_poiseuille_closed_form(lbm):
    # no body force, a density drop: the discrete Poiseuille profile of the
    # body force c_s^2 (rho_in - rho_out) / (nx + 1)
    say("open ends Poiseuille")
    nx, ny, tau, drho = 64, 16, 0.8, 1e-6
    G = lbm.Channel(9, lbm.SLAB, nx, ny, 1, tau=tau, precision="f64")
    G.set_friction(math.inf)
    G.set_open_ends(1.0 + drho / 2, 1.0 - drho / 2)
    G.step(20032)
    rho, ux, _, _ = G.fields()
    ue = poiseuille_exact(ny, tau, drho / 3.0 / (nx + 1), math.inf)
    q = G.invariants()[0]
    say(f"  flux {q / ue.sum() - 1:.2e}")
    assert abs(q / ue.sum() - 1) < 1e-8
    slope = np.polyfit(np.arange(nx), rho[0].mean(axis=0), 1)[0]
    assert abs(slope / (-drho / (nx + 1)) - 1) < 1e-6


def test_full_size_duct_open_ends_fp64(lbm):
    say("open ends full size duct")
    nx, ny, nz = 256, 128, 64
    G = lbm.Channel(19, lbm.DUCT, nx, ny, nz, tau=0.7, force=(1e-6, 0, 0), precision="f64")
    O = oracle.Lattice(19, oracle.DUCT, nx, ny, nz, tau=0.7, force=(1e-6, 0, 0))
    lam = np.random.default_rng(9).uniform(0.0, 0.1, G.wall_count)
    for L in (G, O):
        L.set_friction(lam)
        L.set_open_ends(1.0 + 1e-5, 1.0 - 1e-5)
    G.step(3)
    O.step(3)
    eu, er = errs(G, O)
    say(f"  u {eu:.2e} rho {er:.2e}")
    assert eu < 1e-12 and er < 1e-14


def test_open_ends_settings(lbm):
    T = lbm.Channel(19, lbm.TUBE, 8, 12, 12, tau=0.8, precision="f64", tube_radius=4.0,
                    tube_cy=5.5, tube_cz=5.5)
    T.set_open_ends(1.0, 1.0)  # tubes take open ends
    solid = np.zeros((6, 8), dtype=bool)
    solid[0] = True
    M = lbm.Channel(9, lbm.MASKED, 8, 6, 1, tau=0.8, precision="f64", solid=solid)
    M.set_open_ends(1.0, 1.0)  # equal first and last rows of the mask
    solid[1, 7] = True
    M = lbm.Channel(9, lbm.MASKED, 8, 6, 1, tau=0.8, precision="f64", solid=solid)
    with pytest.raises(lbm.LBMError):  # the last row differs from the first
        M.set_open_ends(1.0, 1.0)
    S1 = lbm.Channel(9, lbm.SLAB, 1, 6, 1, tau=0.8, precision="f64")
    with pytest.raises(lbm.LBMError):
        S1.set_open_ends(1.0, 1.0)
    S = lbm.Channel(9, lbm.SLAB, 8, 6, 1, tau=0.8, precision="f64", force=(1e-5, 0, 0))
    for bad in [(0.0, 1.0), (1.0, float("nan")), (1.0, -1.0), (float("inf"), 1.0)]:
        with pytest.raises(lbm.LBMError):
            S.set_open_ends(*bad)
    S.set_electrons(0.9, 1.0, 0.1, 0.0)
    with pytest.raises(lbm.LBMError):
        S.set_open_ends(1.0, 1.0)
    S.set_electrons(0.0)
    S.set_open_ends(1.0, 0.999)
    with pytest.raises(lbm.LBMError):
        S.set_electrons(0.9, 1.0, 0.1, 0.0)
    R = lbm.Channel(9, lbm.SLAB, 8, 6, 1, tau=0.8, precision="f64", force=(1e-5, 0, 0))
    with pytest.raises(lbm.LBMError):
        lbm.Batch([R, S])
    # closing again gives back the periodic channel
    S.set_open_ends(1.0, 1.0, open_=False)
    S2 = lbm.Channel(9, lbm.SLAB, 8, 6, 1, tau=0.8, precision="f64", force=(1e-5, 0, 0))
    S.set_state(S2.get_state()[0], 0)
    S.step(70)
    S2.step(70)
    assert np.array_equal(S.get_state()[0], S2.get_state()[0])


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_restart_with_open_ends_bitwise(lbm, precision):
    # a state set from outside (checkpoint restore) continues exactly as the
    # run that wrote it: the ghosts' end-node records are rebuilt from it
    say("open ends restart", precision)
    A, _ = build(lbm, "d3q19", precision)
    A.step(70)
    buf, step = A.get_state()
    B, _ = build(lbm, "d3q19", precision)
    B.set_state(buf, step)
    A.step(131)
    B.step(131)
    assert np.array_equal(A.get_state()[0], B.get_state()[0])


@pytest.mark.parametrize("nx", [2, 3])
@pytest.mark.parametrize("q,geom,ny,nz", [(9, "SLAB", 7, 1), (19, "DUCT", 5, 4)])
def test_shortest_open_channels_fp64(lbm, nx, q, geom, ny, nz):
    # the degenerate lengths: both ends in one or two cells
    say("open ends short", nx, q, geom)
    kw = dict(tau=0.8, force=(1e-6, 0, 0))
    G = lbm.Channel(q, getattr(lbm, geom), nx, ny, nz, precision="f64", **kw)
    O = oracle.Lattice(q, getattr(oracle, geom), nx, ny, nz, **kw)
    for L in (G, O):
        L.set_friction(0.04)
        L.set_open_ends(1.0 + 3e-6, 1.0 - 2e-6)
    G.step(150)
    O.step(150)
    eu, er = errs(G, O)
    assert eu < 1e-12 and er < 1e-14


def test_open_ends_half_storage_tracks_the_oracle(lbm):
    # half storage (float arithmetic): within its field error, as for the
    # periodic channels; measured 4.0e-4 (field) and 1.05e-5 (flux), held to
    # about 3x that
    say("open ends f16s")
    G, O = build(lbm, "duct", "f16s")
    G.step(500)
    O.step(500)
    eu, _ = errs(G, O)
    qg, qo = G.invariants()[0], O.invariants()[0]
    say(f"  u {eu:.2e}  flux {abs(qg / qo - 1):.2e}")
    assert eu < 1.2e-3 and abs(qg / qo - 1) < 3.2e-5


def test_couette_with_open_ends_matches_periodic_fp64(lbm):
    # a moving top wall with equal end densities: the x-uniform Couette flow
    # is a fixed point of the open ends, so the open channel must reproduce
    # the periodic one (itself pinned by the exact Couette profile)
    say("open ends Couette")
    nx, ny, U = 24, 12, 1e-3
    kw = dict(tau=0.9, precision="f64", wall_velocity_top=U)
    A = lbm.Channel(9, lbm.SLAB, nx, ny, 1, **kw)
    B = lbm.Channel(9, lbm.SLAB, nx, ny, 1, **kw)
    for L in (A, B):
        L.set_friction(0.1)
    B.set_open_ends(1.0, 1.0)
    A.step(6000)
    B.step(6000)
    ua, ub = A.field(1), B.field(1)
    err = np.abs(ua - ub).max() / np.abs(ua).max()
    say(f"  {err:.2e}")
    assert np.abs(ua).max() > 1e-4 and err < 1e-12


# ------------------------------------------------------------------ nanotubes
# open ends on the circular tube: the interpolated wall links at the ends
# read the ghosts too (several 64-lane tiles and a ragged tail along x)
def build_tube(lbm, precision, nx=70, R=5.0, rho=(1.0 + 2e-5, 1.0 - 1e-5), force=(1e-6, 0, 0)):
    n = int(2 * R + 4)
    c = (n - 1) / 2
    kw = dict(tau=0.75, force=force, tube_radius=R, tube_cy=c, tube_cz=c)
    G = lbm.Channel(19, lbm.TUBE, nx, n, n, precision=precision, **kw)
    O = oracle.Lattice(19, oracle.TUBE, nx, n, n, **kw)
    lam = np.random.default_rng(5).uniform(0.0, 0.3, G.wall_count)
    for L in (G, O):
        L.set_friction(lam)
        L.set_open_ends(*rho)
    return G, O


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_tube_parity_over_graph_and_plain_steps(lbm, precision):
    say("open tube parity", precision)
    G, O = build_tube(lbm, precision)
    n = 229  # three 64-step graph replays, then single launches
    G.step(n)
    O.step(n)
    eu, er = errs(G, O)
    qg, mg, _ = G.invariants()
    qo, mo, _ = O.invariants()
    say(f"  u {eu:.2e}  rho {er:.2e}  flux {abs(qg / qo - 1):.2e}  mass {abs(mg / mo - 1):.2e}")
    tol = 1e-12 if precision == "f64" else 1e-5
    assert eu < tol and abs(qg / qo - 1) < tol
    assert er < (1e-14 if precision == "f64" else 1e-6)
    assert abs(mg / mo - 1) < (1e-14 if precision == "f64" else 1e-8)


def test_tube_open_ends_with_thermal_noise(lbm):
    say("open tube + thermal")
    G, O = build_tube(lbm, "f64", nx=40)
    for L in (G, O):
        L.set_thermal(1e-7, 1, 6)
    G.step(101)
    O.step(101)
    eu, _ = errs(G, O)
    say(f"  u {eu:.2e}")
    assert eu < 1e-12


@pytest.mark.parametrize("precision", ["f32", "f16s"])
def test_tube_open_graph_plain_and_restart_bitwise(lbm, precision):
    say("open tube graph = plain = restart", precision)
    A, _ = build_tube(lbm, precision)
    B, _ = build_tube(lbm, precision)
    C, _ = build_tube(lbm, precision)
    A.step(70)
    for _ in range(70):
        B.step(1)
    assert np.array_equal(A.get_state()[0], B.get_state()[0])
    buf, step = A.get_state()
    C.set_state(buf, step)  # the end-node records are rebuilt from the state
    A.step(131)
    C.step(131)
    assert np.array_equal(A.get_state()[0], C.get_state()[0])


def test_tube_open_half_storage_tracks_the_oracle(lbm):
    say("open tube f16s")
    G, O = build_tube(lbm, "f16s")
    G.step(500)
    O.step(500)
    eu, _ = errs(G, O)
    qg, qo = G.invariants()[0], O.invariants()[0]
    say(f"  u {eu:.2e}  flux {abs(qg / qo - 1):.2e}")
    # measured 4.4e-4 (field) and 2.1e-5 (flux), held to about 3x that
    assert eu < 1.4e-3 and abs(qg / qo - 1) < 6.5e-5


def test_tube_pressure_drop_linear_and_free_of_end_effects_fp64(lbm):
    # the property the oracle is pinned by, on the GPU at steady state: the
    # density is uniform over every cross-section and linear along x with the
    # ghost planes at the prescribed densities, and the ends add no
    # resistance (flux times (nx + 1) independent of the length)
    say("open tube steady")
    R, drho = 4.0, 1e-6
    flux_len = []
    for nx in (24, 48):
        G = lbm.Channel(19, lbm.TUBE, nx, 12, 12, tau=0.8, precision="f64", tube_radius=R,
                        tube_cy=5.5, tube_cz=5.5)
        G.set_friction(0.05)
        G.set_open_ends(1.0 + drho / 2, 1.0 - drho / 2)
        G.run_to_steady(1e-12, 500, 400_000)
        rho = G.fields()[0]
        fl = np.abs(rho[:, :, nx // 2]) > 0.5
        for x in (0, nx // 3, nx - 1):
            assert np.ptp(rho[:, :, x][fl]) < 1e-7 * drho
        prof = np.array([rho[:, :, x][fl].mean() for x in range(nx)])
        slope, icpt = np.polyfit(np.arange(nx), prof, 1)
        say(f"  nx {nx}: slope {slope / (-drho / (nx + 1)) - 1:.2e}")
        assert abs(slope / (-drho / (nx + 1)) - 1) < 1e-8
        assert abs((icpt - slope) - (1.0 + drho / 2)) < 1e-6 * drho
        assert np.abs(prof - (slope * np.arange(nx) + icpt)).max() < 1e-6 * drho
        flux_len.append(G.invariants()[0] * (nx + 1))
    say(f"  flux x length {flux_len[1] / flux_len[0] - 1:.2e}")
    assert abs(flux_len[1] / flux_len[0] - 1) < 1e-10


def test_full_size_tube_open_ends_fp64(lbm):
    # the 512 x 72 x 72 nanotube (R = 32) with open ends, three steps
    say("open ends full size tube")
    R, nx = 32.0, 512
    kw = dict(tau=0.8, force=(1e-6, 0, 0), tube_radius=R, tube_cy=35.5, tube_cz=35.5)
    G = lbm.Channel(19, lbm.TUBE, nx, 72, 72, precision="f64", **kw)
    O = oracle.Lattice(19, oracle.TUBE, nx, 72, 72, **kw)
    lam = np.random.default_rng(10).uniform(0.0, 0.1, G.wall_count)
    for L in (G, O):
        L.set_friction(lam)
        L.set_open_ends(1.0 + 1e-5, 1.0 - 1e-5)
    G.step(3)
    O.step(3)
    eu, er = errs(G, O)
    say(f"  u {eu:.2e} rho {er:.2e}")
    assert eu < 1e-12 and er < 1e-14
