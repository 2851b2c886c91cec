"""Pins of the oracle's open x ends (the Neumann-like inlet and outlet option
of Sec. 4.2): ghost nodes beyond each end copy their neighbour inside the box,
moved along the local equilibrium to a prescribed density.

What fixes it independently of the oracle's own open-end code:
  - with equal densities at both ends and a body force, an x-uniform flow is
    a fixed point, so the open channel must reproduce the periodic one (whose
    profile is pinned by the exact discrete slip-Poiseuille solution);
  - a pressure drop rho_in - rho_out with no body force holds the density
    linear inside the box with slope -(rho_in - rho_out)/(nx + 1) (the ghost
    planes sit at x = -1 and x = nx), and drives the same flow as the body
    force F = c_s^2 (rho_in - rho_out)/(nx + 1): exactly the discrete
    Poiseuille profile between no-slip walls, up to compressibility terms of
    second order in the density drop;
  - in a duct, the pressure-driven flux equals the body-force-driven flux of
    the periodic duct to the same order;
  - in a nanotube (interpolated bounce-back, whose links reach one node
    further along x), a pressure drop must still leave the density exactly
    linear over every cross-section and add no resistance at the ends: the
    flux times (nx + 1) is the same for any tube length.  Reading the node
    behind an interpolated link at the ends from the periodic image instead
    of the ghost breaks both (slope off by 1 %, flux by 2e-4);
  - masked walls continue past an open end as that end's row of the mask
    (first and last rows equal): an x-uniform mask is then the open slab
    shifted, bit for bit; a mask, friction field and drive mirrored in x
    with the end densities swapped give the mirrored flow; through a
    wrinkled channel the pressure drop drives the flux of the equivalent
    body force up to an end effect that halves when the channel doubles,
    and follows lubrication theory to the staircase correction.
"""
import math

import numpy as np
import pytest

import oracle
from test_oracle_lb import poiseuille_exact


def run_steady(L, chunk=1000, tol=1e-11, max_chunks=200):
    prev = None
    for _ in range(max_chunks):
        L.step(chunk)
        q = L.invariants()[0]
        if prev is not None and abs(q - prev) < tol * abs(q):
            return q
        prev = q
    raise AssertionError("not converged")


@pytest.mark.parametrize("q,geom,shape", [(9, oracle.SLAB, (40, 12, 1)),
                                          (19, oracle.DUCT, (9, 8, 6)),
                                          (19, oracle.SLAB, (7, 9, 4))])
def test_equal_densities_reproduce_the_periodic_channel(q, geom, shape):
    # slab: the periodic flow keeps rho = rho0 at every node, so the ghosts
    # equal the periodic neighbours to rounding; in a duct the corners hold
    # density deviations of second order in the velocity, which the open
    # ends pin to rho0 at the ghosts: agreement to that order only
    nx, ny, nz = shape
    A = oracle.Lattice(q, geom, nx, ny, nz, tau=0.8, force=(1e-5, 0, 0))
    B = oracle.Lattice(q, geom, nx, ny, nz, tau=0.8, force=(1e-5, 0, 0))
    B.set_open_ends(1.0, 1.0)
    # one friction value per wall (a friction varying across the section
    # would stir up density deviations of second order, as in the duct)
    xyz = A.wall_coords()
    lam = np.where(xyz[:, 1] == 0, 0.05, 0.12)
    A.set_friction(lam)
    B.set_friction(lam)
    A.step(800)
    B.step(800)
    ra, rb = A.fields(), B.fields()
    ref = np.abs(ra[1]).max()
    assert ref > 1e-4
    tol = 1e-13 if geom == oracle.SLAB else 1e-5
    assert max(np.abs(ra[k] - rb[k]).max() for k in (1, 2, 3)) < tol * ref
    assert np.abs(ra[0] - rb[0]).max() < (1e-15 if geom == oracle.SLAB else 1e-7)


@pytest.mark.parametrize("nx,drho", [(64, 1e-6), (33, 1e-6), (64, 1e-4)])
def test_pressure_driven_poiseuille_exact(nx, drho):
    ny, tau = 16, 0.8
    L = oracle.Lattice(9, oracle.SLAB, nx, ny, 1, tau=tau)
    L.set_friction(math.inf)
    L.set_open_ends(1.0 + drho / 2, 1.0 - drho / 2)
    q = run_steady(L)
    rho, ux, uy, _ = L.fields()
    # density linear inside with the ghost planes at x = -1 and x = nx
    slope, icpt = np.polyfit(np.arange(nx), rho[0].mean(axis=0), 1)
    assert abs(slope / (-drho / (nx + 1)) - 1) < 1e-6
    assert abs((icpt - slope) - (1.0 + drho / 2)) < 1e-3 * drho
    # the flow of the equivalent body force
    G = drho / 3.0 / (nx + 1)
    ue = poiseuille_exact(ny, tau, G, math.inf)
    tol = 1e-8 if drho <= 1e-6 else 2e-6
    assert abs(q / ue.sum() - 1) < tol
    assert np.abs(ux[0, :, nx // 2] / ue - 1).max() < 50 * tol
    assert np.abs(uy).max() < 1e-3 * ue.max()


def test_pressure_drop_matches_body_force_in_a_duct():
    nx, ny, nz, tau, drho = 24, 10, 8, 0.7, 1e-6
    P = oracle.Lattice(19, oracle.DUCT, nx, ny, nz, tau=tau)
    P.set_friction(math.inf)
    P.set_open_ends(1.0 + drho / 2, 1.0 - drho / 2)
    B = oracle.Lattice(19, oracle.DUCT, 2, ny, nz, tau=tau, force=(drho / 3 / (nx + 1), 0, 0))
    B.set_friction(math.inf)
    qp = run_steady(P, chunk=500)
    qb = run_steady(B, chunk=500)
    assert abs(qp / qb - 1) < 1e-7


def test_slip_walls_under_a_pressure_drop():
    # Navier-slip walls: the pressure drop and the equivalent body force give
    # fluxes within 1 % (the wall rule's slip half sees the density gradient
    # of the pressure-driven flow); both well above the no-slip flux
    nx, ny, tau, drho, lam = 64, 16, 0.8, 1e-6, 0.05
    L = oracle.Lattice(9, oracle.SLAB, nx, ny, 1, tau=tau)
    L.set_friction(lam)
    L.set_open_ends(1.0 + drho / 2, 1.0 - drho / 2)
    q = run_steady(L)
    G = drho / 3.0 / (nx + 1)
    qs = poiseuille_exact(ny, tau, G, lam).sum()
    q0 = poiseuille_exact(ny, tau, G, math.inf).sum()
    assert abs(q / qs - 1) < 0.01
    assert q > 1.5 * q0


def tube_fluid_mask(L, nx):
    rho = L.fields()[0]
    return rho, np.abs(rho[:, :, nx // 2]) > 0.5  # solid cells report 0


@pytest.mark.parametrize("lam", [math.inf, 0.05])
def test_tube_pressure_drop_is_linear_and_free_of_end_effects(lam):
    R, tau, drho = 4.0, 0.8, 1e-6
    ny = nz = 12
    flux_len = []
    for nx in (24, 48):
        P = oracle.Lattice(19, oracle.TUBE, nx, ny, nz, tau=tau, tube_radius=R,
                           tube_cy=5.5, tube_cz=5.5)
        P.set_friction(lam)
        P.set_open_ends(1.0 + drho / 2, 1.0 - drho / 2)
        q = run_steady(P, chunk=500)
        rho, fl = tube_fluid_mask(P, nx)
        # uniform over every cross-section, linear along x, the ghost planes
        # at x = -1 and x = nx holding the prescribed densities
        for x in (0, nx // 3, nx - 1):
            assert np.ptp(rho[:, :, x][fl]) < 1e-7 * drho
        prof = np.array([rho[:, :, x][fl].mean() for x in range(nx)])
        slope, icpt = np.polyfit(np.arange(nx), prof, 1)
        assert abs(slope / (-drho / (nx + 1)) - 1) < 1e-8
        assert abs((icpt - slope) - (1.0 + drho / 2)) < 1e-6 * drho
        assert np.abs(prof - (slope * np.arange(nx) + icpt)).max() < 1e-6 * drho
        flux_len.append(q * (nx + 1))
    assert abs(flux_len[1] / flux_len[0] - 1) < 1e-10


def test_tube_pressure_drop_against_body_force():
    # the pressure-driven and the body-force-driven no-slip tube differ by a
    # wall term of first order in the lattice spacing (the interpolated
    # bounce-back sees the density gradient along its links): under 1 % at
    # R = 4, halved at R = 8
    tau, drho, nx = 0.8, 1e-6, 24
    rel = []
    for R in (4.0, 8.0):
        ny = int(2 * R + 4)
        c = (ny - 1) / 2
        P = oracle.Lattice(19, oracle.TUBE, nx, ny, ny, tau=tau, tube_radius=R, tube_cy=c,
                           tube_cz=c)
        P.set_friction(math.inf)
        P.set_open_ends(1.0 + drho / 2, 1.0 - drho / 2)
        B = oracle.Lattice(19, oracle.TUBE, 2, ny, ny, tau=tau, tube_radius=R, tube_cy=c,
                           tube_cz=c, force=(drho / 3 / (nx + 1), 0, 0))
        B.set_friction(math.inf)
        rel.append(run_steady(P, chunk=500) / run_steady(B, chunk=500) - 1)
    assert abs(rel[0]) < 0.01
    assert 1.8 < rel[0] / rel[1] < 2.2


@pytest.mark.parametrize("q,nz", [(9, 1), (19, 4)])
def test_x_uniform_mask_with_open_ends_is_the_open_slab_bitwise(q, nz):
    nx, ny, lo, hi = 13, 14, 3, 2
    solid = np.zeros((ny, nx), dtype=bool)
    solid[:lo] = True
    solid[ny - hi:] = True
    h = ny - lo - hi
    A = oracle.Lattice(q, oracle.SLAB, nx, h, nz, tau=0.9, force=(2e-5, 0, 0))
    B = oracle.Lattice(q, oracle.MASKED, nx, ny, nz, tau=0.9, force=(2e-5, 0, 0), solid=solid)
    lam = np.random.default_rng(2).uniform(0, 0.5, A.wall_count)
    for L in (A, B):
        L.set_friction(lam)
        L.set_open_ends(1.0 + 3e-5, 1.0 - 2e-5)
    A.step(90)
    B.step(90)
    assert np.array_equal(A.get_populations(), B.get_populations()[:, :, lo:ny - hi, :])


@pytest.mark.parametrize("q,nz", [(9, 1), (19, 3)])
def test_masked_open_ends_mirror_x(q, nz):
    nx, ny = 20, 12
    solid = np.zeros((ny, nx), dtype=bool)
    solid[:2] = True
    for x in range(nx):
        d = min(x, nx - 1 - x)
        if 3 <= d <= 6:
            solid[:4, x] = True
        if d == 8:
            solid[ny - 3:, x] = True
    assert np.array_equal(solid, solid[:, ::-1])
    F, rin, rout = 1e-5, 1.0 + 2e-5, 1.0 - 1e-5
    runs = []
    for sgn in (1, -1):
        L = oracle.Lattice(q, oracle.MASKED, nx, ny, nz, tau=0.8, force=(sgn * F, 0, 0),
                           solid=solid)
        xyz = L.wall_coords()
        d = np.minimum(xyz[:, 0], nx - 1 - xyz[:, 0])
        L.set_friction(0.05 + 0.02 * d + 0.01 * xyz[:, 1] + 0.003 * xyz[:, 2])
        L.set_open_ends(*((rin, rout) if sgn > 0 else (rout, rin)))
        L.step(300)
        runs.append(L.fields())
    (ra, uxa, uya, _), (rb, uxb, uyb, _) = runs
    ref = np.abs(uxa).max()
    assert ref > 1e-5
    assert np.abs(uxb + uxa[:, :, ::-1]).max() < 1e-12 * ref
    assert np.abs(uyb - uya[:, :, ::-1]).max() < 1e-12 * ref
    assert np.abs(rb - ra[:, :, ::-1]).max() < 1e-13


def test_pressure_drop_through_wrinkled_walls():
    from test_oracle_masked import corrugated_mask

    ny, tau, drho = 26, 1.0, 1e-6
    nu = (tau - 0.5) / 3
    diff = []
    for period in (128, 256):
        nx = period + 1  # one or two whole wrinkles plus the repeated first row
        solid = corrugated_mask(nx, ny, amp_lo=2.0, amp_hi=2.0, base=3, period=period)
        assert np.array_equal(solid[:, 0], solid[:, -1])
        L = oracle.Lattice(9, oracle.MASKED, nx, ny, 1, tau=tau, solid=solid)
        L.set_friction(math.inf)
        L.set_open_ends(1.0 + drho / 2, 1.0 - drho / 2)
        q = run_steady(L, tol=1e-10)
        G = drho / 3 / (nx + 1)
        P = oracle.Lattice(9, oracle.MASKED, period, ny, 1, tau=tau, force=(G, 0, 0),
                           solid=solid[:, :period])
        P.set_friction(math.inf)
        diff.append(q / run_steady(P, tol=1e-10) - 1)
        h = (~solid).sum(axis=0).astype(float)
        assert abs(q / (G / (12 * nu) / np.mean(h ** -3.0)) - 1) < 0.03
    assert abs(diff[0]) < 0.005
    assert 1.8 < diff[0] / diff[1] < 2.2


def test_open_ends_rejections():
    solid = np.zeros((6, 8), dtype=bool)
    solid[0, :] = solid[-1, :] = True
    solid[1, 3] = True
    M = oracle.Lattice(19, oracle.MASKED, 8, 6, 2, tau=0.8, solid=solid)
    M.set_open_ends(1.0, 1.0)  # equal first and last rows
    solid[1, 7] = True
    M = oracle.Lattice(19, oracle.MASKED, 8, 6, 2, tau=0.8, solid=solid)
    with pytest.raises(oracle.OracleError):  # the last row differs from the first
        M.set_open_ends(1.0, 1.0)
    S = oracle.Lattice(9, oracle.SLAB, 1, 6, 1, tau=0.8)
    with pytest.raises(oracle.OracleError):  # nx = 1
        S.set_open_ends(1.0, 1.0)
    S = oracle.Lattice(9, oracle.SLAB, 8, 6, 1, tau=0.8)
    for bad in [(0.0, 1.0), (1.0, float("nan")), (1.0, -1.0)]:
        with pytest.raises(oracle.OracleError):
            S.set_open_ends(*bad)
    S.set_electrons(0.9, 1.0, 0.1)
    with pytest.raises(oracle.OracleError):
        S.set_open_ends(1.0, 1.0)
    S.set_open_ends(1.0, 1.0, open_=False)  # closing is always allowed
