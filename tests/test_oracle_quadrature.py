"""Pins of the oracle's friction quadrature (no GPU).

The integrand is a synthetic stand-in for the friction coefficients
the paper's Keldysh analysis produces (appendix, Eq. 27): a q^3 e^{-2qd}
weighted wavevector sum times a frequency sum of Im g_s Im g_l / sinh^2(w/2T).
The full form also divides by the screening denominator |1 - g_s g_l e^{-2qd}|^2
and lets the liquid mode disperse with q.  The pins reach it by other
routes: complex response functions and the Bose occupation identity
1/sinh^2(x/2) = 4 n (n + 1) (brute force on tiny grids), the f-sum rule of a
damped oscillator, Kramers-Kronig for the real parts, the closed form of the
q integral (a double geometric series once screened), the weak-coupling
limit and an adaptive integrator.
"""
import dataclasses
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import Spectral


def brute_force(sp: Spectral, Omega: float) -> float:
    """Independent route: responses as Python complex numbers, thermal factor
    from the Bose occupation number, screening as |1 - z|^2 of a complex z."""
    qmax = 10.0 / sp.d
    wmax = 20.0 * sp.T
    dq, dw = qmax / sp.nq, wmax / sp.nw
    tot = 0.0
    for a in range(sp.nq):
        q = (a + 0.5) * dq
        wp2 = Omega * Omega * (q * sp.d if sp.dispersion else 1.0)
        for b in range(sp.nw):
            w = (b + 0.5) * dw
            gs = wp2 / complex(wp2 - w * w, -sp.gamma_s * w)
            wl2 = sp.omega_l ** 2 + sp.v_l ** 2 * q * q
            gl = sp.a_l * wl2 / complex(wl2 - w * w, -sp.gamma_l * w)
            n = 1.0 / math.expm1(w / sp.T)
            x = math.exp(-2 * q * sp.d)
            screen = abs(1 - x * gs * gl) ** 2 if sp.coupling else 1.0
            tot += dq * dw * q ** 3 * x * gs.imag * gl.imag * 4 * n * (n + 1) / screen
    return tot / (8 * math.pi ** 2 * sp.T)


def spec(**kw):
    base = dict(T=1.05, omega0=1.7, gamma_s=0.45, omega_l=2.6, gamma_l=0.9, a_l=0.5, d=1.0)
    base.update(kw)
    return Spectral(**base)


@pytest.mark.parametrize("full", [(0, 0.0), (1, 0.0), (1, 0.7)])
@pytest.mark.parametrize("nq", [1, 2, 4])
@pytest.mark.parametrize("nw", [1, 4, 16])
@pytest.mark.parametrize("disp", [0, 1])
def test_tiny_grid_brute_force(nq, nw, disp, full):
    sp = spec(nq=nq, nw=nw, dispersion=disp, coupling=full[0], v_l=full[1])
    for Om in (0.9, 1.7, 2.8):
        ref = brute_force(sp, Om)
        got = oracle.friction_raw(sp, Om)
        assert abs(got / ref - 1) < 1e-13


def test_response_functions_match_complex_form():
    sp = spec()
    rng = np.random.default_rng(5)
    for w in rng.uniform(0.01, 20, 50):
        gl = sp.a_l * sp.omega_l ** 2 / complex(sp.omega_l ** 2 - w * w, -sp.gamma_l * w)
        assert abs(oracle.img_l(sp, w) - gl.imag) <= 1e-14 * abs(gl.imag) + 1e-300
        q = rng.uniform(0.01, 10)
        wp2 = 1.7 ** 2 * q
        gs = wp2 / complex(wp2 - w * w, -sp.gamma_s * w)
        assert abs(oracle.img_s(sp, 1.7, q, w) - gs.imag) <= 1e-14 * abs(gs.imag) + 1e-300


@pytest.mark.parametrize("which", ["liquid", "solid"])
def test_f_sum_rule(which):
    # a damped oscillator of strength A w0^2 obeys int_0^inf w Im g dw = pi A w0^2 / 2
    sp = spec()
    if which == "liquid":
        f = lambda w: w * oracle.img_l(sp, w)
        exact = math.pi / 2 * sp.a_l * sp.omega_l ** 2
    else:
        q = 2.3
        f = lambda w: w * oracle.img_s(sp, 1.7, q, w)
        exact = math.pi / 2 * 1.7 ** 2 * q
    val = integrate.quad(f, 0, np.inf, limit=400, epsabs=0, epsrel=1e-12)[0]
    assert abs(val / exact - 1) < 1e-9


def q_integral_truncated(d, qmax):
    # int_0^qmax q^3 e^{-2 q d} dq in closed form
    Q = qmax
    return (3 / 8 - math.exp(-2 * Q * d) * (d ** 3 * Q ** 3 / 2 + 3 * d * d * Q * Q / 4
                                            + 3 * d * Q / 4 + 3 / 8)) / d ** 4


def test_factorised_q_sum_converges_to_closed_form():
    # without the plasmon dispersion the double sum factorises into
    # C * S_q * S_w; S_q tends to the closed-form q integral at O(dq^4)
    T = 1.0
    sp_ref = spec(T=T, dispersion=0, nq=4096, nw=2048)
    Om = 1.7
    # S_w from the adaptive integrator with the oracle's own spectra
    g = lambda w: oracle.img_s(sp_ref, Om, 1.0, w) * oracle.img_l(sp_ref, w) / math.sinh(w / (2 * T)) ** 2
    S_w_mid = sum(g((b + 0.5) * 20 * T / 2048) for b in range(2048)) * 20 * T / 2048
    C = 1 / (8 * math.pi ** 2 * T)
    Sq_exact = q_integral_truncated(1.0, 10.0)
    errs = []
    for nq in (64, 128, 256):
        sp = spec(T=T, dispersion=0, nq=nq, nw=2048)
        errs.append(oracle.friction_raw(sp, Om) / (C * Sq_exact * S_w_mid) - 1)
        # Euler-Maclaurin for the midpoint rule: f'(0) = 0 and f'(q_max) ~ e^-20
        # remove the h^2 term, leaving (7 h^4 / 5760) (f'''(q_max) - f'''(0))
        # with f'''(0) = 6 for f = q^3 exp(-2q)
        h = 10.0 / nq
        predicted = -7.0 * h ** 4 / 5760.0 * 6.0 / Sq_exact
        if nq < 256:
            assert abs(errs[-1] / predicted - 1) < 0.03
    assert abs(errs[-1]) < 1e-7
    assert 15.0 < errs[0] / errs[1] < 17.0
    # and the untruncated integral is 3 / (8 d^4) up to e^{-20}-sized tails
    assert abs(Sq_exact / (3 / 8) - 1) < 1e-5


def test_refinement_against_adaptive_integrator():
    sp = spec(T=1.1, nq=256, nw=1024)
    Om = 2.2
    T = sp.T

    def integrand(w, q):
        wp2 = Om * Om * q
        gs = wp2 / complex(wp2 - w * w, -sp.gamma_s * w)
        gl = sp.a_l * sp.omega_l ** 2 / complex(sp.omega_l ** 2 - w * w, -sp.gamma_l * w)
        return q ** 3 * math.exp(-2 * q) * gs.imag * gl.imag / math.sinh(w / (2 * T)) ** 2

    ref = integrate.dblquad(integrand, 0, 10.0, 0, 20 * T, epsabs=0, epsrel=1e-11)[0]
    ref /= 8 * math.pi ** 2 * T
    e1 = oracle.friction_raw(sp, Om) / ref - 1
    sp2 = spec(T=1.1, nq=512, nw=2048)
    e2 = oracle.friction_raw(sp2, Om) / ref - 1
    # midpoint rule at fourth order: the integrand is even in w (odd Im g
    # times odd Im g over even sinh^2) and q^3 has zero slope at q = 0, so
    # the h^2 Euler-Maclaurin terms vanish at both ends
    assert abs(e1) < 1e-7
    assert 14.0 < e1 / e2 < 18.0


def test_lattice_friction_normalisation_and_sign():
    sp = spec(nq=64, nw=256, lambda_target=0.05)
    Om = np.array([sp.omega0, 0.5 * sp.omega0, 1.5 * sp.omega0, 1.1])
    raw, lat = oracle.friction(sp, Om)
    assert np.all(raw > 0) and np.all(lat > 0)
    assert lat[0] == pytest.approx(0.05, rel=1e-15)
    assert np.allclose(lat / raw, 0.05 / oracle.friction_raw(sp, sp.omega0), rtol=1e-14)


def test_long_double_agrees():
    sp = spec(nq=128, nw=512)
    a = oracle.friction_raw(sp, 1.9)
    b = oracle.friction_raw(sp, 1.9, kind="f80")
    assert abs(a / b - 1) < 1e-13


# --------------------------------------------- coupled (screened) quadrature
# The full form divides by |1 - g_s g_l e^{-2qd}|^2 (the two surfaces screen
# each other repeatedly) and lets the liquid mode disperse,
# omega_l(q)^2 = omega_l^2 + v_l^2 q^2.  It needs the complex responses; their
# real parts are pinned by causality (Kramers-Kronig), the denominator by a
# closed-form series of the q integral.

@pytest.mark.parametrize("which", ["solid", "liquid"])
def test_real_parts_by_kramers_kronig(which):
    # Re g(w) = (1/pi) [PV int_0^inf Im g(u) / (u - w) du + int_0^inf Im g(u) / (u + w) du]
    # for a causal response vanishing at infinity (Im g odd in w), and the
    # static value g(0) = (2/pi) int_0^inf Im g(u) / u du
    sp = spec(v_l=0.7)
    Om, q = 1.9, 1.3
    k = 0 if which == "solid" else 1
    im = lambda u: oracle.response(sp, Om, q, u)[k].imag
    W = 60.0
    for w in (0.4, 1.1, 2.5, 3.7):
        pv = integrate.quad(im, 0, W, weight="cauchy", wvar=w, limit=400, epsabs=0, epsrel=1e-11)[0]
        pv += integrate.quad(lambda u: im(u) / (u - w), W, np.inf, limit=200, epsabs=0, epsrel=1e-11)[0]
        plus = integrate.quad(lambda u: im(u) / (u + w), 0, np.inf, limit=400, epsabs=0, epsrel=1e-11)[0]
        re = oracle.response(sp, Om, q, w)[k].real
        assert abs((pv + plus) / math.pi - re) < 1e-8 * max(1.0, abs(re))
    static = 2 / math.pi * integrate.quad(lambda u: im(u) / u, 0, np.inf, limit=400,
                                           epsabs=0, epsrel=1e-11)[0]
    assert static == pytest.approx(1.0 if which == "solid" else sp.a_l, rel=1e-8)


def test_liquid_dispersion_shifts_the_mode():
    # with v_l the liquid response at q is the q = 0 response of a mode at
    # sqrt(omega_l^2 + v_l^2 q^2); v_l = 0 leaves it independent of q
    sp = spec(v_l=0.8)
    for q in (0.3, 1.0, 4.0):
        shifted = spec(omega_l=math.sqrt(sp.omega_l ** 2 + 0.64 * q * q))
        for w in (0.5, 2.0, 3.3):
            got = oracle.response(sp, 1.7, q, w)[1].imag
            assert got == pytest.approx(oracle.img_l(shifted, w), rel=1e-14)
            assert oracle.response(spec(), 1.7, q, w)[1].imag == pytest.approx(
                oracle.img_l(spec(), w), rel=1e-14)


def q_series(G, d, Q, kmax=200):
    # int_0^Q q^3 x / |1 - x G|^2 dq, x = e^{-2qd}, |G| < 1:
    # 1/|1 - xG|^2 = sum_{m,n} G^m conj(G)^n x^{m+n}, each power integrated
    # in closed form over the truncated range
    tot = 0.0
    for k in range(kmax):
        s = sum(G ** m * np.conj(G) ** (k - m) for m in range(k + 1))
        tot += s.real * q_integral_truncated(d * (1 + k), Q)
    return tot


def test_coupled_q_sum_equals_series_closed_form():
    # one frequency point and no plasmon dispersion: the double sum is the
    # frequency factor times a midpoint q sum of q^3 x / |1 - x G|^2, G = g_s g_l
    T, Om, w0 = 1.05, 0.9, 1.2
    sp = spec(T=T, dispersion=0, coupling=1, nw=1, w_max=2 * w0)
    gs, gl = oracle.response(sp, Om, 1.0, w0)
    G = gs * gl
    assert 0.3 < abs(G) < 0.9
    C = 1 / (8 * math.pi ** 2 * T)
    pref = C * 2 * w0 * gs.imag * gl.imag / math.sinh(w0 / (2 * T)) ** 2
    exact = q_series(G, 1.0, 10.0)
    for nq, tol in ((128, 0.02), (256, 0.05)):
        err = oracle.friction_raw(dataclasses.replace(sp, nq=nq), Om) / pref - exact
        # midpoint rule: f'(0) = 0, so the leading error is
        # (7 h^4 / 5760)(f'''(Q) - f'''(0)) with f'''(0) = 6 / |1 - G|^2
        h = 10.0 / nq
        predicted = -7 * h ** 4 / 5760 * 6 / abs(1 - G) ** 2
        assert abs(err / predicted - 1) < tol
    assert abs(err / exact) < 1e-7
    # the same sum with the screening sign flipped is far off
    assert abs(q_series(-G, 1.0, 10.0) / exact - 1) > 0.1


def test_weak_coupling_limit():
    # the denominator is 1 + O(a_l): the coupled result approaches the
    # unscreened one linearly in the liquid's strength
    dev = []
    for a in (2e-3, 1e-3):
        sp = spec(a_l=a, nq=64, nw=256)
        dev.append(oracle.friction_raw(dataclasses.replace(sp, coupling=1), 1.7)
                   / oracle.friction_raw(sp, 1.7) - 1)
    assert abs(dev[1]) < 1e-2
    assert 1.9 < dev[0] / dev[1] < 2.1


@pytest.mark.parametrize("v_l", [0.0, 0.6])
def test_coupled_refinement_against_adaptive_integrator(v_l):
    sp = spec(T=1.1, coupling=1, v_l=v_l, nq=256, nw=1024)
    Om, T = 2.2, 1.1

    def integrand(w, q):
        gs, gl = oracle.response(sp, Om, q, w)
        x = math.exp(-2 * q)
        return (q ** 3 * x * gs.imag * gl.imag
                / (math.sinh(w / (2 * T)) ** 2 * abs(1 - x * gs * gl) ** 2))

    ref = integrate.dblquad(integrand, 0, 10.0, 0, 20 * T, epsabs=0, epsrel=1e-11)[0]
    ref /= 8 * math.pi ** 2 * T
    e1 = oracle.friction_raw(sp, Om) / ref - 1
    e2 = oracle.friction_raw(dataclasses.replace(sp, nq=512, nw=2048), Om) / ref - 1
    # still fourth order: |1 - z|^2 is even in w (z(-w) = conj z(w))
    assert abs(e1) < 1e-7
    assert 14.0 < e1 / e2 < 18.0


def test_coupled_long_double_agrees():
    sp = spec(nq=128, nw=512, coupling=1, v_l=0.5)
    a = oracle.friction_raw(sp, 1.9)
    b = oracle.friction_raw(sp, 1.9, kind="f80")
    assert abs(a / b - 1) < 1e-13
