"""Pins of the oracle's one-point closure of the quantum noise (Sec. 4,
Eq. 18): the two-point correlator averaged over lags with weights W_x(r),
W_t(s) scales the variance of each component of the random stress of the
stress-source noise (Eq. 17).

What fixes it independently of the closure code:
  - the noise's second moment at a cell, sum_i xi_i c_ia c_ib, is the random
    stress P_ab itself (fourth-order isotropy of both lattices), so one step
    from the zero state exposes P_ab cell by cell; the closure must scale it
    by exactly sqrt(m_ab) against the classical run with the same seed;
  - for a separable correlator Gamma_ab(r, s) = f_ab(r) g(s) the average is
    the product (sum_r W_x f_ab)(sum_s W_t g) -- with nr != ns and asymmetric
    tables, a transposed or misaligned sum fails it;
  - weights that average a unit correlator give back the classical noise
    bit for bit.
"""
import numpy as np
import pytest

import oracle

C9 = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]])
C19 = np.array([[0, 0, 0], [1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1],
                [1, 1, 0], [-1, -1, 0], [1, -1, 0], [-1, 1, 0], [1, 0, 1], [-1, 0, -1],
                [1, 0, -1], [-1, 0, 1], [0, 1, 1], [0, -1, -1], [0, 1, -1], [0, -1, 1]])
COMP = [(0, 0), (1, 1), (2, 2), (0, 1), (0, 2), (1, 2)]


def stress_moments(L, q):
    """Pi_ab = sum_i g_i c_ia c_ib per cell, for the six components."""
    g = L.get_populations()
    c = C9 if q == 9 else C19
    out = []
    for a, b in COMP:
        if q == 9 and (a == 2 or b == 2):
            out.append(None)
            continue
        w = (c[:, a] * c[:, b]).astype(float)
        out.append(np.tensordot(w, g, axes=(0, 0)))
    return out


def one_step(q, closure=None, seed=11):
    shape = (9, 6, 1) if q == 9 else (5, 6, 4)
    L = oracle.Lattice(q, oracle.SLAB, *shape, tau=0.8)
    L.set_friction(0.0)
    L.set_thermal(1e-6, 1, seed)
    if closure is not None:
        L.set_noise_closure(*closure)
    L.step(1)
    return L


@pytest.mark.parametrize("q", [9, 19])
def test_separable_closure_scales_each_stress_component(q):
    rng = np.random.default_rng(5)
    nr, ns = 3, 5
    f = rng.uniform(0.2, 3.0, (6, nr))
    f[3] = 0.0           # the xy component switched off
    g = rng.uniform(0.1, 1.0, ns)
    wx = rng.uniform(0.1, 1.0, nr)
    wt = rng.uniform(0.1, 1.0, ns)
    gamma = f[:, :, None] * g[None, None, :]
    m = (f @ wx) * (g @ wt)  # the closed form of the separable average
    A = one_step(q)
    B = one_step(q, (gamma, wx, wt))
    pa, pb = stress_moments(A, q), stress_moments(B, q)
    for k, (xa, xb) in enumerate(zip(pa, pb)):
        if xa is None:
            continue
        assert np.abs(xa).max() > 0
        assert np.abs(xb - np.sqrt(m[k]) * xa).max() < 1e-12 * np.abs(xa).max() * max(1, np.sqrt(m[k]))
    assert np.abs(pb[3]).max() < 1e-25  # xy off: no xy stress at any cell
    # mass and momentum stay exactly unforced
    for Lb in (A, B):
        gb = Lb.get_populations()
        assert np.abs(gb.sum(axis=0)).max() < 1e-14 * np.abs(gb).max()


@pytest.mark.parametrize("q", [9, 19])
def test_unit_correlator_is_the_classical_noise_bitwise(q):
    wx = np.array([0.25, 0.75])
    wt = np.array([0.5, 0.125, 0.375])
    gamma = np.ones((6, 2, 3))
    A = one_step(q)
    B = one_step(q, (gamma, wx, wt))
    assert np.array_equal(A.get_populations(), B.get_populations())
    B.set_noise_closure(None)  # and back
    C = one_step(q)
    assert np.array_equal(A.get_populations(), C.get_populations())


def test_closure_rejections():
    L = oracle.Lattice(9, oracle.SLAB, 4, 4, 1, tau=0.8)
    g = np.ones((6, 1, 1))
    g[1] = -1.0
    with pytest.raises(oracle.OracleError):
        L.set_noise_closure(g, [1.0], [1.0])
    g[1] = np.nan
    with pytest.raises(oracle.OracleError):
        L.set_noise_closure(g, [1.0], [1.0])
