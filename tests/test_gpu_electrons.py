"""GPU parity of the electron wind (electron lines in the solid next to slab,
duct and tube walls) against the oracle, through the C ABI.

Tolerances: FP64 water fields and electron state within 1e-12 relative of the
oracle (same arithmetic, summation order aside); FP32 water storage within
1e-5 of the largest axial velocity (its stochastic rounding, as for the plain
channel); half storage within about 3x its measured error; with thermal
noise and double storage 1e-12 (both sides draw the normals in binary64).
Exact properties at full size: the one-step axial momentum
bookkeeping of water plus electrons.  Closed form: the coupled steady state.
"""
import numpy as np
import pytest

import oracle
from test_oracle_lb import poiseuille_exact

pytestmark = pytest.mark.gpu

C9X = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
C19X = np.array([0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0])


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


CASES = {"d2q9": (9, 64, 30, 1), "d3q19": (19, 37, 9, 6), "duct": (19, 33, 10, 7)}
ELEC = (0.85, 0.7, 0.03, -1.5e-6)  # tau_e, rho_e0, gamma_e, force_e


def build(lbm, case, precision, fh=2e-6):
    q, nx, ny, nz = CASES[case]
    geom = "DUCT" if case == "duct" else "SLAB"
    G = lbm.Channel(q, getattr(lbm, geom), nx, ny, nz, tau=0.75, force=(fh, 0, 0),
                    precision=precision)
    O = oracle.Lattice(q, getattr(oracle, geom), nx, ny, nz, tau=0.75, force=(fh, 0, 0))
    lam = np.random.default_rng(8).uniform(0.0, 0.3, G.wall_count)
    G.set_friction(lam)
    O.set_friction(lam)
    G.set_electrons(*ELEC)
    O.set_electrons(*ELEC)
    return G, O


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_parity_over_graph_and_plain_steps(lbm, case, precision):
    say("electrons parity", case, precision)
    G, O = build(lbm, case, precision)
    n = 101  # one 64-step graph replay, then single launches
    G.step(n)
    O.step(n)
    rg, ro = G.fields(), O.fields()
    ref = np.abs(ro[1]).max()
    err = max(np.abs(rg[k] - ro[k]).max() for k in (1, 2, 3)) / ref
    ueg, pg = G.electrons()
    ueo, po = O.electrons()
    eerr = np.abs(ueg - ueo).max() / np.abs(ueo).max()
    perr = np.abs(pg - po).max() / np.abs(po).max()
    say(f"  water {err:.2e}  u_e {eerr:.2e}  electron pops {perr:.2e}")
    tol = 1e-12 if precision == "f64" else 1e-5
    assert err < tol and eerr < tol and perr < tol


@pytest.mark.parametrize("case", ["d3q19", "duct"])
@pytest.mark.parametrize("precision", ["f64", "f32", "f16s"])
def test_graph_and_plain_launches_bitwise(lbm, precision, case):
    say("electrons bitwise", precision, case)
    A, _ = build(lbm, case, precision)
    B, _ = build(lbm, case, precision)
    A.step(128)
    for _ in range(128):
        B.step(1)
    assert np.array_equal(A.get_state()[0], B.get_state()[0])
    ua, pa = A.electrons()
    ub, pb = B.electrons()
    assert np.array_equal(ua, ub) and np.array_equal(pa, pb)


def test_coupled_steady_state_closed_form(lbm):
    # pressure-driven water dragging the electrons, opposed by a field drive
    say("electrons steady state")
    H, tau, lam, fh, fe = 30, 0.8, 0.05, 1e-6, -3e-6
    rho_e, gam = 2.0, 0.2
    G = lbm.Channel(9, lbm.SLAB, 4, H, 1, tau=tau, force=(fh, 0, 0), precision="f64")
    G.set_friction(lam)
    G.set_electrons(0.9, rho_e, gam, fe)
    G.step(45056)
    Ue = (fh * H + fe * 2) / (gam * rho_e * 2)
    ue, _ = G.electrons()
    assert np.abs(ue / Ue - 1).max() < 1e-10
    _, ux, uy, _ = G.fields()
    exp = poiseuille_exact(H, tau, fh, lam) + Ue
    assert np.abs(ux[0] - exp[:, None]).max() < 1e-10 * np.abs(exp).max()


@pytest.mark.parametrize("geom", ["SLAB", "DUCT"])
def test_full_size_momentum_bookkeeping_fp64(lbm, geom):
    # 256 x 128 x 64 slab and duct: over one step water plus electrons change
    # axial momentum by exactly the forces minus the lattice drag
    say("electrons full size momentum", geom)
    nx, ny, nz, fh = 256, 128, 64, 2e-6
    tau_e, rho_e, gam, fe = ELEC
    G = lbm.Channel(19, getattr(lbm, geom), nx, ny, nz, tau=0.7, force=(fh, 0, 0),
                    precision="f64")
    G.set_friction(np.random.default_rng(3).uniform(0.0, 0.2, G.wall_count))
    G.set_electrons(tau_e, rho_e, gam, fe)
    G.step(200)

    def totals():
        g = G.populations()
        _, p = G.electrons()
        return float(np.tensordot(C19X, g, axes=(0, 0)).sum()), float((p[1] - p[2]).sum()), p
    w0, e0, p = totals()
    rho = rho_e + p[0] + np.roll(p[1], 1, axis=-1) + np.roll(p[2], -1, axis=-1)
    G.step(1)
    w1, e1, _ = totals()
    ue, _ = G.electrons()
    expect = fh * G.fluid_count + fe * G.shell_count * nx - gam * float((rho * ue).sum())
    say(f"  residual {(w1 + e1) - (w0 + e0) - expect:.3e} of {abs(w0):.3e}")
    assert abs((w1 + e1) - (w0 + e0) - expect) < 1e-12 * abs(w0)
    assert abs((w1 - w0) - fh * G.fluid_count) > 1e-6 * abs(fh * G.fluid_count)


def test_electron_settings_and_batches(lbm):
    # a tube whose wall touches the box's edge has no solid to hold lines there
    D = lbm.Channel(19, lbm.TUBE, 8, 12, 12, tau=0.8, precision="f64", tube_radius=5.9,
                    tube_cy=5.5, tube_cz=5.5)
    with pytest.raises(lbm.LBMError):
        D.set_electrons(*ELEC)
    M = lbm.Channel(9, lbm.MASKED, 8, 6, 1, tau=0.8, precision="f64", solid=np.eye(6, 8) > 0)
    with pytest.raises(lbm.LBMError):
        M.set_electrons(*ELEC)
    S = lbm.Channel(9, lbm.SLAB, 8, 4, 1, tau=0.8, precision="f64")
    for args in [(0.5, 1.0, 0.1, 0.0), (0.8, 0.0, 0.1, 0.0), (0.8, 1.0, -0.1, 0.0),
                 (0.8, 1.0, 0.1, float("nan"))]:
        with pytest.raises(lbm.LBMError):
            S.set_electrons(*args)
    with pytest.raises(lbm.LBMError):
        S.electrons()  # off
    S.set_electrons(*ELEC)
    T = lbm.Channel(9, lbm.SLAB, 8, 4, 1, tau=0.8, precision="f64")
    with pytest.raises(lbm.LBMError):
        lbm.Batch([S, T])
    S.set_electrons(0.0)  # off again: an ordinary slab
    S.step(70)
    T.step(70)
    assert np.array_equal(S.get_state()[0], T.get_state()[0])


def test_electrons_with_thermal_noise_fp64(lbm):
    # both extensions at once: the sheets' walls and the fluctuating update
    say("electrons + thermal noise")
    G, O = build(lbm, "d3q19", "f64")
    for L in (G, O):
        L.set_thermal(1e-7, 2, 31)
    G.step(101)
    O.step(101)
    rg, ro = G.fields(), O.fields()
    err = max(np.abs(rg[k] - ro[k]).max() for k in (1, 2, 3)) / np.abs(ro[1]).max()
    ueg, _ = G.electrons()
    ueo, _ = O.electrons()
    say(f"  water {err:.2e}  u_e {np.abs(ueg - ueo).max() / np.abs(ueo).max():.2e}")
    # binary64 normals on both sides (see the thermal parity tests)
    assert err < 1e-12
    assert np.abs(ueg - ueo).max() < 1e-12 * np.abs(ueo).max()


def test_half_storage_electrons_track_the_oracle(lbm):
    # half-precision water storage (float arithmetic) with the double sheets:
    # the sheets follow the oracle within the water's half-storage error
    # (fields within about 4e-4 of the oracle after 1000 steps on a duct)
    say("electrons half storage")
    G, O = build(lbm, "d2q9", "f16s")
    G.step(300)
    O.step(300)
    ueg, _ = G.electrons()
    ueo, _ = O.electrons()
    e = np.abs(ueg - ueo).max() / np.abs(ueo).max()
    say(f"  u_e {e:.2e}")
    assert e < 1.6e-3  # measured 5.4e-4


PHON = (0.7, 1.3, 0.02, 0.08)  # tau_p, rho_p0, gamma_pc, gamma_ep


@pytest.mark.parametrize("precision", ["f64", "f32"])
@pytest.mark.parametrize("case", sorted(CASES))
def test_phonon_parity_over_graph_and_plain_steps(lbm, case, precision):
    say("phonons parity", case, precision)
    G, O = build(lbm, case, precision)
    for L in (G, O):
        L.set_phonons(*PHON)
    n = 101
    G.step(n)
    O.step(n)
    rg, ro = G.fields(), O.fields()
    err = max(np.abs(rg[k] - ro[k]).max() for k in (1, 2, 3)) / np.abs(ro[1]).max()
    ueg, _ = G.electrons()
    ueo, _ = O.electrons()
    upg, ppg = G.phonons()
    upo, ppo = O.phonons()
    eu = np.abs(ueg - ueo).max() / np.abs(ueo).max()
    ep = np.abs(upg - upo).max() / np.abs(upo).max()
    epp = np.abs(ppg - ppo).max() / np.abs(ppo).max()
    say(f"  water {err:.2e}  u_e {eu:.2e}  u_p {ep:.2e}  phonon pops {epp:.2e}")
    tol = 1e-12 if precision == "f64" else 1e-5
    assert err < tol and eu < tol and ep < tol and epp < tol


def test_phonons_graph_and_plain_launches_bitwise(lbm):
    say("phonons bitwise")
    A, _ = build(lbm, "duct", "f32")
    B, _ = build(lbm, "duct", "f32")
    for L in (A, B):
        L.set_phonons(*PHON)
    A.step(128)
    for _ in range(128):
        B.step(1)
    assert np.array_equal(A.get_state()[0], B.get_state()[0])
    assert np.array_equal(A.phonons()[1], B.phonons()[1])


def test_phonons_steady_state_closed_form(lbm):
    say("phonons steady state")
    H, tau, lam, fh, fe = 30, 0.8, 0.05, 1e-6, 0.0
    rho_e, gam, rho_p, gpc, gep = 2.0, 0.2, 1.5, 0.1, 0.3
    G = lbm.Channel(9, lbm.SLAB, 4, H, 1, tau=tau, force=(fh, 0, 0), precision="f64")
    G.set_friction(lam)
    G.set_electrons(0.9, rho_e, gam, fe)
    G.set_phonons(0.8, rho_p, gpc, gep)
    G.step(45056)
    Gc = gep * rho_e
    kappa = Gc / (Gc + gpc * rho_p)
    Ue = (fh * H + fe * 2) / (2 * (gam * rho_e + gpc * rho_p * kappa))
    ue, _ = G.electrons()
    up, _ = G.phonons()
    assert np.abs(ue / Ue - 1).max() < 1e-10
    assert np.abs(up / (kappa * Ue) - 1).max() < 1e-10


def test_phonons_full_size_momentum_bookkeeping_fp64(lbm):
    say("phonons full size momentum")
    nx, ny, nz, fh = 256, 128, 64, 2e-6
    tau_e, rho_e, gam, fe = ELEC
    tau_p, rho_p, gpc, gep = PHON
    G = lbm.Channel(19, lbm.DUCT, nx, ny, nz, tau=0.7, force=(fh, 0, 0), precision="f64")
    G.set_friction(np.random.default_rng(3).uniform(0.0, 0.2, G.wall_count))
    G.set_electrons(tau_e, rho_e, gam, fe)
    G.set_phonons(tau_p, rho_p, gpc, gep)
    G.step(200)

    def totals():
        g = G.populations()
        _, pe = G.electrons()
        _, pp = G.phonons()
        return (float(np.tensordot(C19X, g, axes=(0, 0)).sum()), float((pe[1] - pe[2]).sum()),
                float((pp[1] - pp[2]).sum()), pe, pp)
    w0, e0, p0, pe, pp = totals()
    re = rho_e + pe[0] + np.roll(pe[1], 1, axis=-1) + np.roll(pe[2], -1, axis=-1)
    rp = rho_p + pp[0] + np.roll(pp[1], 1, axis=-1) + np.roll(pp[2], -1, axis=-1)
    G.step(1)
    w1, e1, p1, _, _ = totals()
    ue, _ = G.electrons()
    up, _ = G.phonons()
    expect = (fh * G.fluid_count + fe * G.shell_count * nx - gam * float((re * ue).sum())
              - gpc * float((rp * up).sum()))
    res = (w1 + e1 + p1) - (w0 + e0 + p0) - expect
    say(f"  residual {res:.3e} of {abs(w0):.3e}")
    assert abs(res) < 1e-12 * abs(w0)
    assert abs(p1 - p0) > 1e-12 * abs(w0)


def test_phonon_settings(lbm):
    S = lbm.Channel(9, lbm.SLAB, 8, 4, 1, tau=0.8, precision="f64")
    with pytest.raises(lbm.LBMError):  # electrons off
        S.set_phonons(*PHON)
    S.set_electrons(*ELEC)
    with pytest.raises(lbm.LBMError):
        S.phonons()  # off
    for bad in [(0.5, 1.0, 0.1, 0.1), (0.8, 0.0, 0.1, 0.1), (0.8, 1.0, -0.1, 0.1),
                (0.8, 1.0, 0.1, float("nan"))]:
        with pytest.raises(lbm.LBMError):
            S.set_phonons(*bad)
    S.set_phonons(*PHON)
    S.set_electrons(*ELEC)  # switches the phonons off
    with pytest.raises(lbm.LBMError):
        S.phonons()


def test_phonons_with_half_storage_water(lbm):
    # half-storage water (float arithmetic) with double electron and phonon
    # lines: the lines follow the oracle within the water's half-storage error
    say("phonons half storage")
    G, O = build(lbm, "d2q9", "f16s")
    for L in (G, O):
        L.set_phonons(*PHON)
    G.step(300)
    O.step(300)
    upg, _ = G.phonons()
    upo, _ = O.phonons()
    ueg, _ = G.electrons()
    ueo, _ = O.electrons()
    e = max(np.abs(upg - upo).max() / np.abs(upo).max(), np.abs(ueg - ueo).max() / np.abs(ueo).max())
    say(f"  u_e, u_p {e:.2e}")
    assert e < 1.8e-3  # measured 5.8e-4


@pytest.mark.parametrize("precision", ["f64", "f16s"])
def test_checkpoint_holds_the_lines(lbm, precision):
    # with electron and phonon lines on, a checkpoint restores water, lines
    # and the lines' last velocities: the restored run continues bit for bit
    say("checkpoint with lines", precision)
    A, _ = build(lbm, "duct", precision)
    A.set_phonons(*PHON)
    A.step(50)
    buf, step = A.get_state()
    B, _ = build(lbm, "duct", precision)
    B.set_phonons(*PHON)
    B.set_state(buf, step)
    for L in (A, B):
        L.step(70)
    assert np.array_equal(A.get_state()[0], B.get_state()[0])
    for fa, fb in ((A.electrons(), B.electrons()), (A.phonons(), B.phonons())):
        assert np.array_equal(fa[0], fb[0]) and np.array_equal(fa[1], fb[1])
    # a state taken with the lines on does not fit a context without them
    C, _ = build(lbm, "duct", precision)
    C.set_electrons(0.0)
    with pytest.raises(lbm.LBMError):
        C.set_state(buf, step)


# ------------------------------------------------------------------ nanotubes
# electron lines in the solid columns around the circular wall (interpolated
# bounce-back with the moving-wall term scaled by 1 - cc)
def build_tube(lbm, precision, nx=37, R=5.0, fh=2e-6):
    n = int(2 * R + 4)
    c = (n - 1) / 2
    kw = dict(tau=0.75, force=(fh, 0, 0), tube_radius=R, tube_cy=c, tube_cz=c)
    G = lbm.Channel(19, lbm.TUBE, nx, n, n, precision=precision, **kw)
    O = oracle.Lattice(19, oracle.TUBE, nx, n, n, **kw)
    lam = np.random.default_rng(8).uniform(0.0, 0.3, G.wall_count)
    for L in (G, O):
        L.set_friction(lam)
        L.set_electrons(*ELEC)
    assert G.shell_count == O.shell_count > 0
    return G, O


@pytest.mark.parametrize("phonons", [False, True])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_tube_parity_over_graph_and_plain_steps(lbm, precision, phonons):
    say("tube electrons parity", precision, "phonons" if phonons else "")
    G, O = build_tube(lbm, precision)
    if phonons:
        for L in (G, O):
            L.set_phonons(*PHON)
    n = 101
    G.step(n)
    O.step(n)
    rg, ro = G.fields(), O.fields()
    err = max(np.abs(rg[k] - ro[k]).max() for k in (1, 2, 3)) / np.abs(ro[1]).max()
    ueg, pg = G.electrons()
    ueo, po = O.electrons()
    eu = np.abs(ueg - ueo).max() / np.abs(ueo).max()
    ep = np.abs(pg - po).max() / np.abs(po).max()
    say(f"  water {err:.2e}  u_e {eu:.2e}  electron pops {ep:.2e}")
    tol = 1e-12 if precision == "f64" else 1e-5
    assert err < tol and eu < tol and ep < tol
    if phonons:
        upg, _ = G.phonons()
        upo, _ = O.phonons()
        assert np.abs(upg - upo).max() < tol * np.abs(upo).max()


@pytest.mark.parametrize("precision", ["f32", "f16s"])
def test_tube_graph_plain_and_restart_bitwise(lbm, precision):
    say("tube electrons bitwise", precision)
    A, _ = build_tube(lbm, precision)
    B, _ = build_tube(lbm, precision)
    C, _ = build_tube(lbm, precision)
    A.step(70)
    for _ in range(70):
        B.step(1)
    assert np.array_equal(A.get_state()[0], B.get_state()[0])
    buf, step = A.get_state()
    C.set_state(buf, step)
    A.step(64)
    C.step(64)
    assert np.array_equal(A.get_state()[0], C.get_state()[0])
    assert np.array_equal(A.electrons()[1], C.electrons()[1])


def test_tube_electrons_with_thermal_noise_fp64(lbm):
    say("tube electrons + thermal")
    G, O = build_tube(lbm, "f64", nx=20)
    for L in (G, O):
        L.set_thermal(1e-7, 1, 33)
    G.step(101)
    O.step(101)
    rg, ro = G.fields(), O.fields()
    err = max(np.abs(rg[k] - ro[k]).max() for k in (1, 2, 3)) / np.abs(ro[1]).max()
    ueg, _ = G.electrons()
    ueo, _ = O.electrons()
    say(f"  water {err:.2e}")
    assert err < 1e-12
    assert np.abs(ueg - ueo).max() < 1e-12 * np.abs(ueo).max()


def test_tube_half_storage_electrons_track_the_oracle(lbm):
    say("tube electrons half storage")
    G, O = build_tube(lbm, "f16s")
    G.step(300)
    O.step(300)
    ueg, _ = G.electrons()
    ueo, _ = O.electrons()
    e = np.abs(ueg - ueo).max() / np.abs(ueo).max()
    say(f"  u_e {e:.2e}")
    assert e < 6.5e-4  # measured 2.1e-4


def test_tube_full_size_momentum_bookkeeping_fp64(lbm):
    # the 512 x 72 x 72 nanotube (R = 32): over one step water plus electron
    # lines change axial momentum by exactly the forces minus the lattice drag
    say("tube electrons full size momentum")
    nx, fh = 512, 2e-6
    tau_e, rho_e, gam, fe = ELEC
    G = lbm.Channel(19, lbm.TUBE, nx, 72, 72, tau=0.8, force=(fh, 0, 0), precision="f64",
                    tube_radius=32.0, tube_cy=35.5, tube_cz=35.5)
    G.set_friction(np.random.default_rng(3).uniform(0.0, 0.2, G.wall_count))
    G.set_electrons(tau_e, rho_e, gam, fe)
    G.step(200)

    def totals():
        g = G.populations()
        _, p = G.electrons()
        return float(np.tensordot(C19X, g, axes=(0, 0)).sum()), float((p[1] - p[2]).sum()), p
    w0, e0, p = totals()
    rho = rho_e + p[0] + np.roll(p[1], 1, axis=-1) + np.roll(p[2], -1, axis=-1)
    G.step(1)
    w1, e1, _ = totals()
    ue, _ = G.electrons()
    expect = fh * G.fluid_count + fe * G.shell_count * nx - gam * float((rho * ue).sum())
    say(f"  shells {G.shell_count}, residual {(w1 + e1) - (w0 + e0) - expect:.3e} of {abs(w0):.3e}")
    assert abs((w1 + e1) - (w0 + e0) - expect) < 1e-12 * abs(w0)
    assert abs((w1 - w0) - fh * G.fluid_count) > 1e-6 * abs(fh * G.fluid_count)
