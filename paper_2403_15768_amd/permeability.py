"""Water permeability of nanotubes against radius and charge-carrier density.

The application of Sec. 5.1: permeability as a function of the tube's
design parameters -- its radius and, through the quantum friction, the
charge-carrier density of the wall.  The density enters as the wall's plasmon
frequency Omega: the friction quadrature (``lbm_set_friction_spectral``)
turns it into the wall's friction lambda, the lattice-Boltzmann channel is run
to steady state, and the flux is compared with that of the same tube with
no-slip walls.  For a Navier-slip wall of slip length L_s = nu / lambda the
continuum answer is

    Q / Q_no-slip = 1 + 4 L_s / R,

so the enhancement falls like 1 / R.  Every number comes from the library's
kernels; this module only sets the channels up and collects the results.

The same section names nano-corrugations and wrinkles of the graphene walls
as the next design parameter: ``wrinkle_sweep`` runs channels whose two walls
are wrinkled along x (masked walls), as a meander of constant gap or as a
gap that narrows and widens, against the flat channel of the same mean gap,
with no-slip or Navier-slip walls.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import inputs, lbm


@dataclass
class TubeResult:
    radius: int
    omega_scale: float     # plasmon frequency / the spectra's reference omega0
    lam: float             # wall friction (lattice units) from the quadrature
    flux: float            # steady flux, friction wall
    flux_noslip: float     # steady flux, no-slip wall
    steps: int             # steps to steady state (friction wall)

    @property
    def enhancement(self) -> float:
        return self.flux / self.flux_noslip

    def slip_length_fit(self) -> float:
        """L_s from the enhancement: R (Q / Q_no-slip - 1) / 4."""
        return self.radius * (self.enhancement - 1.0) / 4.0


def _tube(R: int, nx: int, tau: float, g: float, precision: str):
    ny, nz, cy, cz = inputs.tube_box(R)
    return lbm.Channel(lbm.D3Q19, lbm.TUBE, nx, ny, nz, tau=tau, force=(g, 0.0, 0.0),
                       precision=precision, tube_radius=float(R), tube_cy=cy, tube_cz=cz)


def sweep(radii, omega_scales, spectral=None, nx: int = 16, tau: float = 0.8,
          g: float = 1e-6, precision: str = "f64", rel_tol: float = 1e-9,
          check_every: int = 500, max_steps: int = 2_000_000) -> list[TubeResult]:
    """Steady flux of x-periodic tubes of the given radii with walls of
    uniform plasmon frequency omega_scale * omega0, and of the same tubes with
    no-slip walls.  The flow is x-uniform, so a short periodic tube (nx) gives
    the permeability of a long one."""
    sp = spectral if spectral is not None else inputs.draw_spectral(inputs.rng_for("tube", 0))
    out = []
    for R in radii:
        ref = _tube(R, nx, tau, g, precision)
        ref.run_to_steady(rel_tol=rel_tol, check_every=check_every, max_steps=max_steps)
        q0 = ref.flux()
        ref.close()
        for s in omega_scales:
            ch = _tube(R, nx, tau, g, precision)
            ch.set_friction_spectral(sp, np.full(ch.wall_count, s * sp.omega0))
            lam = float(ch.get_friction()[0])
            n = ch.run_to_steady(rel_tol=rel_tol, check_every=check_every, max_steps=max_steps)
            out.append(TubeResult(R, float(s), lam, ch.flux(), q0, int(n)))
            ch.close()
    return out


@dataclass
class WrinkleResult:
    amplitude: float       # wrinkle amplitude (cells)
    meander: bool          # True: constant gap; False: the gap narrows and widens
    lam: float             # wall friction (lattice units; inf = no slip)
    flux: float            # steady flux, wrinkled walls
    flux_flat: float       # steady flux, flat walls of the same mean gap
    steps: int

    @property
    def relative(self) -> float:
        return self.flux / self.flux_flat


def _wrinkled(nx: int, ny: int, amp: float, wavelength: float, base: int, meander: bool,
              tau: float, g: float, precision: str):
    solid = inputs.corrugated_mask(nx, ny, None, amp=amp, wavelength=wavelength, base=base,
                                   phases=(0.0, np.pi if meander else 0.0))
    return lbm.Channel(lbm.D2Q9, lbm.MASKED, nx, ny, 1, tau=tau, force=(g, 0.0, 0.0),
                       precision=precision, solid=solid)


def wrinkle_sweep(amplitudes, lams, gap: int = 24, nx: int = 128, wavelength: float = 64.0,
                  meanders=(True, False), tau: float = 0.8, g: float = 1e-6,
                  precision: str = "f64", rel_tol: float = 1e-9, check_every: int = 500,
                  max_steps: int = 2_000_000) -> list[WrinkleResult]:
    """Steady flux of D2Q9 channels of mean gap ``gap`` whose walls carry
    wrinkles of the given amplitudes (cells, <= 4) and wavelength, relative to
    the flat channel with the same walls' friction."""
    base = 4
    ny = gap + 2 * base
    out = []
    for lam in lams:
        flat = _wrinkled(nx, ny, 0.0, wavelength, base, True, tau, g, precision)
        flat.set_friction(lam)
        flat.run_to_steady(rel_tol=rel_tol, check_every=check_every, max_steps=max_steps)
        q0 = flat.flux()
        flat.close()
        for meander in meanders:
            for a in amplitudes:
                ch = _wrinkled(nx, ny, a, wavelength, base, meander, tau, g, precision)
                ch.set_friction(lam)
                n = ch.run_to_steady(rel_tol=rel_tol, check_every=check_every,
                                     max_steps=max_steps)
                out.append(WrinkleResult(float(a), bool(meander), float(lam), ch.flux(), q0,
                                         int(n)))
                ch.close()
    return out
