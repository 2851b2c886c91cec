"""The nanotube permeability sweep (Sec. 5.1) on the GPU.

Parity: the enhancement Q / Q_no-slip of an R = 4 tube against the oracle's
(both run to a 1e-10 steady state, FP64; the friction from the quadrature).
Physics: for a Navier-slip wall the continuum enhancement is 1 + 4 L_s / R
with L_s = nu / lambda; the staircase wall and the same-node reflection of
the free-slip half shift the effective slip length by up to ~15 %, so the
test asks for L_s within [0.8, 1.1] of nu / lambda, an enhancement falling
monotonically with R like 1 / R (log-log slope -1 within 0.15), and a larger
enhancement where the quadrature gives less friction.
"""
import numpy as np
import pytest

import oracle
from paper_2403_15768_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_15768_amd import lbm, permeability

    lbm.load()
    return lbm, permeability


def oracle_steady_flux(R, nx, tau, g, lam, tol=1e-10, every=500):
    ny, nz, cy, cz = inputs.tube_box(R)
    O = oracle.Lattice(19, oracle.TUBE, nx, ny, nz, tau=tau, force=(g, 0, 0),
                       tube_radius=float(R), tube_cy=cy, tube_cz=cz)
    if lam is not None:
        O.set_friction(lam)
    q_old = None
    for _ in range(200):
        O.step(every)
        q = O.invariants()[0]
        if q_old is not None and abs(q - q_old) < tol * abs(q):
            return q
        q_old = q
    raise AssertionError("oracle did not reach steady state")


def test_small_tube_enhancement_matches_oracle(mods):
    lbm, perm = mods
    print("permeability parity R = 4", flush=True)
    res = perm.sweep([4], [1.0], nx=4, precision="f64", rel_tol=1e-10)
    r = res[0]
    q_ns = oracle_steady_flux(4, 4, 0.8, 1e-6, None)
    q_sl = oracle_steady_flux(4, 4, 0.8, 1e-6, r.lam)
    assert abs(r.flux_noslip / q_ns - 1) < 1e-8
    assert abs(r.flux / q_sl - 1) < 1e-8
    assert abs(r.enhancement / (q_sl / q_ns) - 1) < 1e-8


def test_enhancement_falls_like_inverse_radius(mods):
    lbm, perm = mods
    print("permeability sweep", flush=True)
    radii = [4, 8, 16, 32]
    res = perm.sweep(radii, [1.0, 2.0], precision="f64")
    nu = (0.8 - 0.5) / 3
    for s in (1.0, 2.0):
        rs = [r for r in res if r.omega_scale == s]
        enh = np.array([r.enhancement for r in rs])
        assert np.all(np.diff(enh) < 0)
        slope = np.polyfit(np.log(radii), np.log(enh - 1), 1)[0]
        print(f"  scale {s}: enhancement {np.round(enh, 4)}, slope {slope:.3f}", flush=True)
        assert abs(slope + 1) < 0.15
        for r in rs:
            assert 0.8 < r.slip_length_fit() / (nu / r.lam) < 1.1
    # more carriers here means less friction and a larger enhancement
    by = {(r.radius, r.omega_scale): r for r in res}
    for R in radii:
        assert (by[(R, 2.0)].lam < by[(R, 1.0)].lam) == (by[(R, 2.0)].enhancement
                                                           > by[(R, 1.0)].enhancement)


def oracle_wrinkled_flux(nx, gap, amp, wavelength, meander, lam, tau=0.8, g=1e-6, tol=1e-10):
    base = 4
    solid = inputs.corrugated_mask(nx, gap + 2 * base, None, amp=amp, wavelength=wavelength,
                                   base=base, phases=(0.0, np.pi if meander else 0.0))
    O = oracle.Lattice(9, oracle.MASKED, nx, gap + 2 * base, 1, tau=tau, force=(g, 0, 0),
                       solid=solid)
    O.set_friction(lam)
    q_old = None
    for _ in range(400):
        O.step(500)
        q = O.invariants()[0]
        if q_old is not None and abs(q - q_old) < tol * abs(q):
            return q
        q_old = q
    raise AssertionError("oracle did not reach steady state")


def test_wrinkled_channel_flux_matches_oracle(mods):
    # the wall-shape sweep of Sec. 5.1 (masked walls): one wrinkled slip
    # channel and its flat reference, both to a 1e-10 steady state
    lbm, perm = mods
    print("wrinkle sweep parity", flush=True)
    res = perm.wrinkle_sweep([2.0], [0.05], gap=24, nx=64, wavelength=32.0, meanders=(True,),
                             precision="f64", rel_tol=1e-10)
    r = res[0]
    q_flat = oracle_wrinkled_flux(64, 24, 0.0, 32.0, True, 0.05)
    q_wr = oracle_wrinkled_flux(64, 24, 2.0, 32.0, True, 0.05)
    print(f"  flat {r.flux_flat / q_flat - 1:.2e}  wrinkled {r.flux / q_wr - 1:.2e}", flush=True)
    assert abs(r.flux_flat / q_flat - 1) < 1e-8
    assert abs(r.flux / q_wr - 1) < 1e-8


def test_wrinkles_reduce_the_flux_more_with_slip(mods):
    # deeper wrinkles carry less water; slip walls lose more to them than
    # no-slip walls (each step of the staircase blocks part of the slip
    # flow), in the meander and in the narrowing-and-widening gap
    lbm, perm = mods
    print("wrinkle sweep physics", flush=True)
    res = perm.wrinkle_sweep([1.0, 2.0, 4.0], [float("inf"), 0.05], precision="f64")
    rel = {(r.meander, r.lam, r.amplitude): r.relative for r in res}
    for meander in (True, False):
        for lam in (float("inf"), 0.05):
            seq = [rel[(meander, lam, a)] for a in (1.0, 2.0, 4.0)]
            print(f"  meander {meander} lambda {lam}: {seq}", flush=True)
            assert 1.0 > seq[0] > seq[1] > seq[2] > 0.2
        for a in (1.0, 2.0, 4.0):
            assert rel[(meander, 0.05, a)] < rel[(meander, float("inf"), a)]
