"""Pins of the oracle's electron wind (no GPU).

The solid's electrons form a second population set (Sec. 3.3; Sec. 4: one set
of distributions per species) coupled to the water by the relative-velocity
drag of Eq. 5 / Eq. 27 (F_kl = -F_lk).  Pins:

* exact momentum bookkeeping: over any single step, water plus electron axial
  momentum changes by exactly the external forces minus the electrons' drag
  on the lattice -- a wrong sign or weight in the reaction force breaks it;
* exact steady states: total momentum balance fixes the electron velocity
  U_e = (F_h N_h + F_e N_e) / (gamma rho_e0 N_e), and the water is the exact
  discrete slip-Poiseuille profile shifted by U_e (a wall moving with the
  electrons) -- pressure-driven water dragging the electrons along, the field
  drive ("electron wind") pulling the water, and the two opposed;
* in a duct (electron lines on all four walls) the steady total balance:
  the lines' lattice drag takes exactly what the forces put in, with U_e
  varying around the perimeter;
* electron mass conserved line by line; settings outside the model rejected;
* on a nanotube (interpolated bounce-back, the electron lines in the solid
  columns around the circular wall): the same exact one-step momentum
  bookkeeping and steady total balance, mirror-symmetric lines moving alike,
  and a uniform flow at the electrons' velocity an exact fixed point -- which
  needs the moving wall's term divided by 2q on the links whose wall lies
  farther than half a link (left undivided, the state drifts by 30 % in 200
  steps).
"""
import numpy as np
import pytest

import oracle
from oracle import DUCT, SLAB, Lattice
from test_oracle_lb import poiseuille_exact

C9X = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
C19X = np.array([0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0])


def axial_momentum(L, q):
    """(water sum g_i c_ix over the box, electron sum e_i c_i) of the current
    state; solid cells hold zeros."""
    cx = C9X if q == 9 else C19X
    g = L.get_populations()
    _, pops = L.electrons()
    return float(np.tensordot(cx, g, axes=(0, 0)).sum()), float((pops[1] - pops[2]).sum())


@pytest.mark.parametrize("q,geom,shape", [(9, SLAB, (16, 12, 1)), (19, SLAB, (10, 8, 5)),
                                          (19, DUCT, (10, 7, 6))])
def test_momentum_balance_is_exact_every_step(q, geom, shape):
    nx, ny, nz = shape
    fh, fe, gam, rho_e = 2e-6, -1.5e-6, 0.03, 0.7
    L = Lattice(q, geom, nx, ny, nz, tau=0.75, force=(fh, 0, 0))
    rng = np.random.default_rng(2)
    L.set_friction(rng.uniform(0.0, 0.3, L.wall_count))
    L.set_electrons(0.85, rho_e, gam, fe)
    L.step(37)  # a transient state
    for _ in range(3):
        w0, e0 = axial_momentum(L, q)
        _, pops = L.electrons()
        # electron density each node sees in the next step (pulled along x)
        rho = rho_e + pops[0] + np.roll(pops[1], 1, axis=-1) + np.roll(pops[2], -1, axis=-1)
        L.step(1)
        w1, e1 = axial_momentum(L, q)
        ue, _ = L.electrons()
        expect = fh * L.fluid_count + fe * L.shell_count * nx - gam * float((rho * ue).sum())
        assert abs((w1 + e1) - (w0 + e0) - expect) < 1e-15 * (abs(w0) + abs(e0) + 1e-3)
        # and the exchange is not trivially zero: each side alone is off
        assert abs((w1 - w0) - fh * L.fluid_count) > 1e-9


@pytest.mark.parametrize("fh,fe", [(1e-6, 0.0), (0.0, 2e-6), (1e-6, -3e-6)])
def test_steady_state_d2q9_exact(fh, fe):
    H, tau, lam = 30, 0.8, 0.05
    rho_e, gam = 2.0, 0.2
    L = Lattice(9, SLAB, 4, H, 1, tau=tau, force=(fh, 0, 0))
    L.set_friction(lam)
    L.set_electrons(0.9, rho_e, gam, fe)
    L.step(45000)  # slowest coupled mode decays over ~1,200 steps
    Ue = (fh * H + fe * 2) / (gam * rho_e * 2)
    ue, pops = L.electrons()
    assert np.abs(ue / Ue - 1).max() < 1e-10
    rho, ux, uy, _ = L.fields()
    exp = (poiseuille_exact(H, tau, fh, lam) if fh else np.zeros(H)) + Ue
    for x in range(4):
        assert np.abs(ux[0, :, x] - exp).max() < 1e-10 * np.abs(exp).max()
    assert np.abs(uy).max() < 1e-15
    # the sign of the coupling: water dragged along by field-driven electrons
    if fh == 0.0:
        assert ux.min() > 0


def test_steady_state_d3q19_slab_exact():
    H, nz, tau, lam, fh = 16, 3, 0.7, 0.1, 1e-6
    rho_e, gam, fe = 1.5, 0.08, 5e-7
    L = Lattice(19, SLAB, 2, H, nz, tau=tau, force=(fh, 0, 0))
    L.set_friction(lam)
    L.set_electrons(0.8, rho_e, gam, fe)
    L.step(30000)
    Ue = (fh * H * nz + fe * 2 * nz) / (gam * rho_e * 2 * nz)
    ue, _ = L.electrons()
    assert np.abs(ue / Ue - 1).max() < 1e-10
    _, ux, _, uz = L.fields()
    exp = poiseuille_exact(H, tau, fh, lam) + Ue
    assert np.abs(ux[:, :, :] - exp[None, :, None]).max() < 1e-10 * exp.max()
    assert np.abs(uz).max() < 1e-15


def test_duct_steady_state_total_balance():
    # four walls of electron lines: at steady state their lattice drag takes
    # exactly what the forces put in; the lines next to the corners see less
    # shear than those in the middle of a wall, so U_e varies around the
    # perimeter, and the sheets move with the water
    nx, ny, nz, fh, fe = 2, 10, 6, 1e-6, 2e-7
    rho_e, gam = 1.5, 0.1
    L = Lattice(19, DUCT, nx, ny, nz, tau=0.8, force=(fh, 0, 0))
    L.set_friction(0.08)
    L.set_electrons(0.9, rho_e, gam, fe)
    assert L.shell_count == 2 * nz + 2 * ny
    L.step(40000)
    ue, _ = L.electrons()
    drag = gam * rho_e * ue.sum()
    put_in = fh * L.fluid_count + fe * L.shell_count * nx
    assert abs(drag / put_in - 1) < 1e-9
    assert ue.min() > 0 and ue.max() / ue.min() > 1.05
    # each line is uniform along x, and mirror shells move alike
    assert np.abs(ue - ue[:, :1]).max() < 1e-12 * ue.max()
    assert np.allclose(ue[:nz], ue[nz:2 * nz], rtol=1e-10)
    assert np.allclose(ue[2 * nz:2 * nz + ny], ue[2 * nz + ny:], rtol=1e-10)


def test_electron_mass_conserved_per_line():
    L = Lattice(9, SLAB, 20, 10, 1, tau=0.7, force=(1e-6, 0, 0))
    L.set_friction(np.random.default_rng(1).uniform(0, 0.2, L.wall_count))
    L.set_electrons(1.1, 0.4, 0.02, 1e-6)
    L.step(500)
    _, pops = L.electrons()
    assert np.abs(pops.sum(axis=(0, 2))).max() < 1e-16


def test_immovable_electrons_give_walls_at_rest():
    # the heavier the sheets, the less they move: the water then approaches
    # the flow between walls at rest, the difference falling as 1 / rho_e0
    def run(rho_e):
        L = Lattice(9, SLAB, 12, 8, 1, tau=0.8, force=(1e-6, 0, 0))
        L.set_friction(0.07)
        if rho_e:
            L.set_electrons(0.9, rho_e, 1.0, 0.0)
        L.step(400)
        return L.fields()[1]
    rest = run(0)
    d = [np.abs(run(r) - rest).max() / np.abs(rest).max() for r in (1e3, 1e6)]
    assert 1e-6 < d[0] < 1e-4
    assert abs(d[1] / d[0] * 1e3 - 1) < 0.01


def tube(nx, R=4.0, n=12, **kw):
    c = (n - 1) / 2
    return Lattice(19, oracle.TUBE, nx, n, n, tube_radius=R, tube_cy=c, tube_cz=c, **kw)


def tube_shells(L, n):
    """(ys, zs) of the tube's shell columns in the oracle's order: solid
    columns with a fluid column next to them along y or z, by y + n z."""
    fluid = L.fields()[0][:, :, 0] != 0  # (z, y)

    def fl(y, z):
        return 0 <= y < n and 0 <= z < n and fluid[z, y]

    return [(y, z) for z in range(n) for y in range(n)
            if not fluid[z, y] and (fl(y - 1, z) or fl(y + 1, z) or fl(y, z - 1) or fl(y, z + 1))]


def test_tube_momentum_balance_is_exact_every_step():
    nx, fh, fe, gam, rho_e = 10, 2e-6, -1.5e-6, 0.03, 0.7
    L = tube(nx, tau=0.75, force=(fh, 0, 0))
    L.set_friction(np.random.default_rng(2).uniform(0.0, 0.3, L.wall_count))
    L.set_electrons(0.85, rho_e, gam, fe)
    assert L.shell_count == len(tube_shells(L, 12)) > 0
    L.step(37)
    for _ in range(3):
        w0, e0 = axial_momentum(L, 19)
        _, pops = L.electrons()
        rho = rho_e + pops[0] + np.roll(pops[1], 1, axis=-1) + np.roll(pops[2], -1, axis=-1)
        L.step(1)
        w1, e1 = axial_momentum(L, 19)
        ue, _ = L.electrons()
        expect = fh * L.fluid_count + fe * L.shell_count * nx - gam * float((rho * ue).sum())
        assert abs((w1 + e1) - (w0 + e0) - expect) < 1e-15 * (abs(w0) + abs(e0) + 1e-3)
        assert abs((w1 - w0) - fh * L.fluid_count) > 1e-9


def test_tube_uniform_flow_is_a_fixed_point():
    # water and electrons moving together at U, no forces: the interpolated
    # moving-wall rule must return every population unchanged (the friction
    # varies around the circumference, uniform along x)
    U, nx, rho_e = 1e-3, 9, 1.3
    L = tube(nx, tau=0.8)
    xyz = L.wall_coords()
    L.set_friction(0.02 + 0.05 * np.abs(np.sin(xyz[:, 1] + 2 * xyz[:, 2])))
    L.set_electrons(0.9, rho_e, 0.0, 0.0)
    fluid = L.fields()[0] != 0
    g = np.zeros((19,) + fluid.shape)
    for i in range(19):
        cu = C19X[i] * U
        w = 1 / 3 if i == 0 else (1 / 18 if i < 7 else 1 / 36)
        g[i] = np.where(fluid, w * (3 * cu + 4.5 * cu * cu - 1.5 * U * U), 0.0)
    L.set_populations(g)
    e = np.zeros((3, L.shell_count, nx))
    for i, (c, w) in enumerate(((0, 2 / 3), (1, 1 / 6), (-1, 1 / 6))):
        e[i] = w * rho_e * (3 * c * U + 4.5 * c * c * U * U - 1.5 * U * U)
    L.set_electron_populations(e)
    L.step(200)
    assert np.abs(L.get_populations() - g).max() < 1e-13 * np.abs(g).max()
    ue, pops = L.electrons()
    assert np.abs(ue / U - 1).max() < 1e-13
    assert np.abs(pops - e).max() < 1e-13 * np.abs(e).max()


def test_tube_steady_state_total_balance():
    # electron lines all around the circular wall: at steady state their
    # lattice drag takes exactly what the forces put in; U_e varies around
    # the circumference (the staircase wall couples each line differently)
    # and mirror-image lines move alike
    nx, fh, fe, rho_e, gam = 2, 1e-6, 2e-7, 1.5, 0.1
    L = tube(nx, tau=0.8, force=(fh, 0, 0))
    L.set_friction(0.08)
    L.set_electrons(0.9, rho_e, gam, fe)
    L.step(8000)
    ue, _ = L.electrons()
    drag = gam * rho_e * ue.sum()
    put_in = fh * L.fluid_count + fe * L.shell_count * nx
    assert abs(drag / put_in - 1) < 1e-12
    assert ue.min() > 0 and ue.max() / ue.min() > 1.2
    assert np.abs(ue - ue[:, :1]).max() < 1e-12 * ue.max()
    shells = tube_shells(L, 12)
    index = {s: k for k, s in enumerate(shells)}
    for k, (y, z) in enumerate(shells):
        for m in ((11 - y, z), (y, 11 - z), (z, y)):
            assert abs(ue[index[m], 0] / ue[k, 0] - 1) < 1e-10


def test_tube_immovable_electrons_give_walls_at_rest():
    def run(rho_e):
        L = tube(6, tau=0.8, force=(1e-6, 0, 0))
        L.set_friction(0.07)
        if rho_e:
            L.set_electrons(0.9, rho_e, 1.0, 0.0)
        L.step(400)
        return L.fields()[1]
    rest = run(0)
    d = [np.abs(run(r) - rest).max() / np.abs(rest).max() for r in (1e3, 1e6)]
    assert 1e-6 < d[0] < 1e-3
    assert abs(d[1] / d[0] * 1e3 - 1) < 0.01


def test_electron_settings_rejected():
    solid = np.zeros((4, 4), dtype=bool)
    solid[0] = True
    for geom, kw in [(oracle.MASKED, {"solid": solid}), (SLAB, {"wall_velocity_top": 1e-3})]:
        L = Lattice(19, geom, 4, 4, 4, tau=0.8, **kw)
        with pytest.raises(oracle.OracleError):
            L.set_electrons(0.8, 1.0, 0.1, 0.0)
    L = Lattice(9, SLAB, 4, 4, 1, tau=0.8)
    for args in [(0.5, 1.0, 0.1, 0.0), (0.8, 0.0, 0.1, 0.0), (0.8, 1.0, -0.1, 0.0),
                 (0.8, 1.0, 0.1, float("nan"))]:
        with pytest.raises(oracle.OracleError):
            L.set_electrons(*args)
