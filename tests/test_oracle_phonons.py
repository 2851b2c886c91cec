"""Pins of the oracle's phonon lines (Sec. 3.4): a third population set beside
the electron lines, coupled to the electrons by the electron-phonon drag
(equal and opposite on the two, Eq. 27) and damped by the crystal.

* exact momentum bookkeeping: over any single step water, electrons and
  phonons together change axial momentum by exactly the external forces
  minus the two crystal drags -- the electron-phonon drag cancels, and a
  wrong sign or weight in either half of it breaks the balance;
* exact steady state: the phonons' own balance gamma_pc rho_p0 U_p =
  gamma_ep rho_e0 (U_e - U_p) and the total balance fix U_e and U_p, and the
  water is the exact discrete slip-Poiseuille profile shifted by U_e;
* limits: no electron-phonon drag leaves the electrons as without phonons
  (to the rounding of the coupled solve) and the phonons at rest;
* phonon mass conserved line by line; settings outside the model rejected.
"""
import numpy as np
import pytest

from oracle import DUCT, SLAB, Lattice, OracleError
from test_oracle_lb import poiseuille_exact

C9X = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
C19X = np.array([0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0])


def totals(L, q):
    cx = C9X if q == 9 else C19X
    w = float(np.tensordot(cx, L.get_populations(), axes=(0, 0)).sum())
    _, pe = L.electrons()
    _, pp = L.phonons()
    return w, float((pe[1] - pe[2]).sum()), float((pp[1] - pp[2]).sum()), pe, pp


def node_density(rho0, pops):
    return rho0 + pops[0] + np.roll(pops[1], 1, axis=-1) + np.roll(pops[2], -1, axis=-1)


@pytest.mark.parametrize("q,geom,shape", [(9, SLAB, (16, 12, 1)), (19, SLAB, (10, 8, 5)),
                                          (19, DUCT, (10, 7, 6))])
def test_momentum_balance_is_exact_every_step(q, geom, shape):
    nx, ny, nz = shape
    fh, fe, gam, rho_e = 2e-6, -1.5e-6, 0.03, 0.7
    rho_p, gpc, gep = 1.3, 0.02, 0.08
    L = Lattice(q, geom, nx, ny, nz, tau=0.75, force=(fh, 0, 0))
    L.set_friction(np.random.default_rng(2).uniform(0.0, 0.3, L.wall_count))
    L.set_electrons(0.85, rho_e, gam, fe)
    L.set_phonons(0.7, rho_p, gpc, gep)
    L.step(37)
    for _ in range(3):
        w0, e0, p0, pe, pp = totals(L, q)
        re, rp = node_density(rho_e, pe), node_density(rho_p, pp)
        L.step(1)
        w1, e1, p1, _, _ = totals(L, q)
        ue, _ = L.electrons()
        up, _ = L.phonons()
        expect = (fh * L.fluid_count + fe * L.shell_count * nx - gam * float((re * ue).sum())
                  - gpc * float((rp * up).sum()))
        scale = abs(w0) + abs(e0) + abs(p0) + 1e-3
        assert abs((w1 + e1 + p1) - (w0 + e0 + p0) - expect) < 1e-15 * scale
        # the phonons take part: their momentum changes by the drag exchange
        assert abs(p1 - p0) > 1e-9


@pytest.mark.parametrize("fh,fe", [(1e-6, 0.0), (0.0, 2e-6)])
def test_steady_state_d2q9_exact(fh, fe):
    H, tau, lam = 30, 0.8, 0.05
    rho_e, gam, rho_p, gpc, gep = 2.0, 0.2, 1.5, 0.1, 0.3
    L = Lattice(9, SLAB, 4, H, 1, tau=tau, force=(fh, 0, 0))
    L.set_friction(lam)
    L.set_electrons(0.9, rho_e, gam, fe)
    L.set_phonons(0.8, rho_p, gpc, gep)
    L.step(45000)
    G = gep * rho_e
    kappa = G / (G + gpc * rho_p)  # U_p / U_e from the phonons' own balance
    Ue = (fh * H + fe * 2) / (2 * (gam * rho_e + gpc * rho_p * kappa))
    ue, _ = L.electrons()
    up, _ = L.phonons()
    assert np.abs(ue / Ue - 1).max() < 1e-10
    assert np.abs(up / (kappa * Ue) - 1).max() < 1e-10
    _, ux, _, _ = L.fields()
    exp = (poiseuille_exact(H, tau, fh, lam) if fh else np.zeros(H)) + Ue
    assert np.abs(ux[0] - exp[:, None]).max() < 1e-10 * np.abs(exp).max()


def test_without_electron_phonon_drag():
    q, nx, ny, nz = 19, 9, 7, 4
    A = Lattice(q, SLAB, nx, ny, nz, tau=0.8, force=(1e-6, 0, 0))
    B = Lattice(q, SLAB, nx, ny, nz, tau=0.8, force=(1e-6, 0, 0))
    for L in (A, B):
        L.set_friction(0.07)
        L.set_electrons(0.9, 1.1, 0.05, 3e-7)
    B.set_phonons(0.7, 2.0, 0.1, 0.0)
    A.step(300)
    B.step(300)
    ua, _ = A.electrons()
    ub, _ = B.electrons()
    assert np.abs(ua - ub).max() < 1e-13 * np.abs(ua).max()
    up, pp = B.phonons()
    assert np.abs(up).max() == 0.0 and np.abs(pp).max() == 0.0


def test_phonon_mass_conserved_per_line():
    L = Lattice(9, SLAB, 12, 8, 1, tau=0.8, force=(2e-6, 0, 0))
    L.set_friction(0.05)
    L.set_electrons(0.9, 1.0, 0.05, 1e-6)
    L.set_phonons(0.75, 1.0, 0.02, 0.5)
    L.step(500)
    _, pp = L.phonons()
    assert np.abs(pp.sum(axis=(0, 2))).max() < 1e-15


def test_phonon_settings_rejected():
    L = Lattice(9, SLAB, 8, 6, 1, tau=0.8)
    with pytest.raises(OracleError):  # electrons off
        L.set_phonons(0.8, 1.0, 0.1, 0.1)
    L.set_electrons(0.9, 1.0, 0.1)
    for bad in [(0.5, 1.0, 0.1, 0.1), (0.8, 0.0, 0.1, 0.1), (0.8, 1.0, -0.1, 0.1),
                (0.8, 1.0, 0.1, float("nan"))]:
        with pytest.raises(OracleError):
            L.set_phonons(*bad)
    L.set_phonons(0.8, 1.0, 0.1, 0.1)
    L.set_phonons(0.0)
