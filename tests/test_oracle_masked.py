"""Pins of the oracle's masked geometry (walls that vary along x: corrugated,
wrinkled or stepped walls given as a solid mask in the (x, y) plane).

What fixes it independently of the oracle's own masked code:
  - a mask with no solid point is the slab, whose wall rule is pinned by the
    exact discrete slip-Poiseuille profile: both must agree bit for bit;
  - a mask whose solid rows are the same for every x is a narrower slab,
    shifted: bit for bit again;
  - mass is conserved exactly for any mask and any friction field (the slip
    pairing is a bijection of the wall links at every node);
  - a mask and a friction field symmetric under x -> -x (or y -> -y) give a
    mirror-symmetric flow when the drive is mirrored too (the pairing passes
    commute with the mirrors);
  - no-slip flow through a slowly varying channel follows lubrication theory,
    Q = F / (12 nu <h^-3>), to within the staircase and slope corrections.
"""
import numpy as np
import pytest

import oracle


def corrugated_mask(nx, ny, amp_lo=2.0, amp_hi=1.5, base=3, period=None, phase=1.0):
    period = period or nx
    x = np.arange(nx)
    lo = np.round(base + amp_lo * np.sin(2 * np.pi * x / period)).astype(int)
    hi = np.round(base + amp_hi * np.sin(2 * np.pi * x / period + phase)).astype(int)
    solid = np.zeros((ny, nx), dtype=bool)
    for i in range(nx):
        solid[: lo[i], i] = True
        solid[ny - hi[i]:, i] = True
    return solid


@pytest.mark.parametrize("q,shape", [(9, (20, 10, 1)), (19, (9, 7, 5))])
def test_empty_mask_is_the_slab_bitwise(q, shape):
    nx, ny, nz = shape
    A = oracle.Lattice(q, oracle.SLAB, nx, ny, nz, tau=0.8, force=(1e-5, 3e-6, 0))
    B = oracle.Lattice(q, oracle.MASKED, nx, ny, nz, tau=0.8, force=(1e-5, 3e-6, 0),
                       solid=np.zeros((ny, nx)))
    assert A.wall_count == B.wall_count and A.fluid_count == B.fluid_count
    assert np.array_equal(A.wall_coords(), B.wall_coords())
    lam = np.random.default_rng(1).uniform(0, 0.3, A.wall_count)
    A.set_friction(lam)
    B.set_friction(lam)
    A.step(60)
    B.step(60)
    assert np.array_equal(A.get_populations(), B.get_populations())


@pytest.mark.parametrize("q,nz", [(9, 1), (19, 4)])
def test_x_uniform_mask_is_a_shifted_slab_bitwise(q, nz):
    nx, ny, lo, hi = 11, 14, 3, 2
    solid = np.zeros((ny, nx), dtype=bool)
    solid[:lo] = True
    solid[ny - hi:] = True
    h = ny - lo - hi
    A = oracle.Lattice(q, oracle.SLAB, nx, h, nz, tau=0.9, force=(2e-5, 0, 0))
    B = oracle.Lattice(q, oracle.MASKED, nx, ny, nz, tau=0.9, force=(2e-5, 0, 0), solid=solid)
    assert A.wall_count == B.wall_count and A.fluid_count == B.fluid_count
    lam = np.random.default_rng(2).uniform(0, 0.5, A.wall_count)
    A.set_friction(lam)  # canonical order: the same nodes in the same order
    B.set_friction(lam)
    A.step(80)
    B.step(80)
    ga, gb = A.get_populations(), B.get_populations()
    assert np.array_equal(ga, gb[:, :, lo:ny - hi, :])


@pytest.mark.parametrize("q,nz", [(9, 1), (19, 3)])
def test_mass_exact_on_corrugated_walls(q, nz):
    nx, ny = 24, 13
    solid = corrugated_mask(nx, ny, period=12)
    solid[6, 5:8] = True  # a free-standing post as well
    L = oracle.Lattice(q, oracle.MASKED, nx, ny, nz, tau=0.7, force=(1e-4, 3e-5, 0),
                       solid=solid)
    L.set_friction(np.random.default_rng(3).uniform(0, 2, L.wall_count))
    m0 = L.invariants()
    L.step(400)
    m1 = L.invariants()
    assert abs(m0[2]) == 0.0
    assert abs(m1[2]) < 1e-13 * m1[1]
    assert abs(m1[0]) > 1e-4  # the flow is not trivial


def _lam_field(L, f):
    xyz = L.wall_coords()
    return np.array([f(x, y, z) for x, y, z in xyz], dtype=np.float64)


@pytest.mark.parametrize("q,nz", [(9, 1), (19, 3)])
def test_mirror_x(q, nz):
    nx, ny = 20, 12
    # a mask symmetric under x -> nx - 1 - x: raised blocks and a step down
    solid = np.zeros((ny, nx), dtype=bool)
    solid[:2] = True
    for x in range(nx):
        d = min(x, nx - 1 - x)
        if 3 <= d <= 6:
            solid[:4, x] = True
        if d == 8:
            solid[ny - 3:, x] = True
    assert np.array_equal(solid, solid[:, ::-1])
    F = 2e-5

    def lam(x, y, z):
        d = min(x, nx - 1 - x)
        return 0.05 + 0.02 * d + 0.01 * y + 0.003 * z

    runs = []
    for sgn in (1, -1):
        L = oracle.Lattice(q, oracle.MASKED, nx, ny, nz, tau=0.8, force=(sgn * F, 0, 0),
                           solid=solid)
        L.set_friction(_lam_field(L, lam))
        L.step(300)
        runs.append(L.fields())
    (ra, uxa, uya, _), (rb, uxb, uyb, _) = runs
    ref = np.abs(uxa).max()
    assert ref > 1e-5
    assert np.abs(uxb + uxa[:, :, ::-1]).max() < 1e-12 * ref
    assert np.abs(uyb - uya[:, :, ::-1]).max() < 1e-12 * ref
    assert np.abs(rb - ra[:, :, ::-1]).max() < 1e-13


@pytest.mark.parametrize("q,nz", [(9, 1), (19, 3)])
def test_mirror_y(q, nz):
    nx, ny = 24, 15
    half = corrugated_mask(nx, ny, amp_lo=2.0, amp_hi=0.0, base=3, period=8)
    solid = half | half[::-1]
    assert np.array_equal(solid, solid[::-1])

    def lam(x, y, z):
        d = min(y, ny - 1 - y)
        return 0.1 + 0.05 * d + 0.02 * np.sin(x) + 0.004 * z

    L = oracle.Lattice(q, oracle.MASKED, nx, ny, nz, tau=0.75, force=(3e-5, 0, 0), solid=solid)
    L.set_friction(_lam_field(L, lam))
    L.step(300)
    rho, ux, uy, _ = L.fields()
    ref = np.abs(ux).max()
    assert np.abs(ux - ux[:, ::-1, :]).max() < 1e-12 * ref
    assert np.abs(uy + uy[:, ::-1, :]).max() < 1e-12 * ref
    assert np.abs(uy).max() > 1e-3 * ref  # the corrugation bends the flow


def test_no_slip_lubrication_limit():
    # gap h(x) varying by about +-2 cells over 128: lubrication theory to a
    # few per cent (staircase walls and the finite slope)
    nx, ny, tau, F = 128, 26, 1.0, 1e-6
    nu = (tau - 0.5) / 3
    solid = corrugated_mask(nx, ny, amp_lo=2.0, amp_hi=2.0, base=3)
    h = (~solid).sum(axis=0).astype(float)
    L = oracle.Lattice(9, oracle.MASKED, nx, ny, 1, tau=tau, force=(F, 0, 0), solid=solid)
    L.set_friction(np.inf)
    prev = None
    for _ in range(40):
        L.step(1000)
        qf = L.invariants()[0]
        if prev is not None and abs(qf - prev) < 1e-9 * abs(qf):
            break
        prev = qf
    pred = F / (12 * nu) / np.mean(h ** -3.0)
    assert abs(qf / pred - 1) < 0.03


def test_masked_rejections():
    with pytest.raises(oracle.OracleError):  # no mask
        oracle.Lattice(9, oracle.MASKED, 8, 6, 1, tau=0.8)
    with pytest.raises(oracle.OracleError):  # all solid
        oracle.Lattice(9, oracle.MASKED, 8, 6, 1, tau=0.8, solid=np.ones((6, 8)))
    with pytest.raises(oracle.OracleError):  # moving wall
        oracle.Lattice(9, oracle.MASKED, 8, 6, 1, tau=0.8, solid=np.zeros((6, 8)),
                       wall_velocity_top=1e-3)
    L = oracle.Lattice(9, oracle.MASKED, 8, 6, 1, tau=0.8, solid=np.zeros((6, 8)))
    with pytest.raises(oracle.OracleError):
        L.set_electrons(0.9, 1.0, 0.1)


def test_slip_lubrication_limit_converges_with_the_staircase():
    # with Navier slip (L_s = nu / lambda) lubrication theory gives
    # Q = F / (12 nu <1 / (h^3 + 6 L_s h^2)>); each one-cell step of the
    # staircase wall blocks part of the slip flow, so the deficit is
    # proportional to the steps per length: halving the slope (same
    # amplitude, twice the wavelength) halves it
    ny, tau, F, lam = 26, 1.0, 1e-6, 0.1
    nu = (tau - 0.5) / 3
    deficit = []
    for nx in (128, 256):
        solid = corrugated_mask(nx, ny, amp_lo=2.0, amp_hi=2.0, base=3)
        h = (~solid).sum(axis=0).astype(float)
        L = oracle.Lattice(9, oracle.MASKED, nx, ny, 1, tau=tau, force=(F, 0, 0), solid=solid)
        L.set_friction(lam)
        prev = None
        for _ in range(60):
            L.step(1000)
            qf = L.invariants()[0]
            if prev is not None and abs(qf - prev) < 1e-9 * abs(qf):
                break
            prev = qf
        pred = F / (12 * nu) / np.mean(1.0 / (h ** 3 + 6 * (nu / lam) * h ** 2))
        deficit.append(1 - qf / pred)
    assert 0.05 < deficit[0] < 0.2
    assert 0.4 < deficit[1] / deficit[0] < 0.65
