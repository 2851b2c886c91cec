"""GPU: the friction quadrature for callers that cannot allocate
(lbm_friction_quadrature_static, its raw sums in a fixed device array)
against the context path (lbm_set_friction_spectral), through the C ABI."""
import ctypes as C

import numpy as np
import pytest

from paper_2403_15768_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2403_15768_amd import lbm as mod

    mod.load()
    return mod


def tube_case(lbm, R, nx, seed, nq, nw, coupling=0, v_l=0.0):
    ny, nz, cy, cz = inputs.tube_box(R)
    ch = lbm.Channel(19, lbm.TUBE, nx, ny, nz, tau=0.8, force=(1e-6, 0, 0), precision="f64",
                     tube_radius=float(R), tube_cy=cy, tube_cz=cz)
    sp = inputs.draw_spectral(inputs.rng_for("tube", 40 + seed), nq=nq, nw=nw)
    sp.coupling, sp.v_l = coupling, v_l
    om = inputs.tube_plasmon_frequencies(ch.wall_coords(), nx, R, cy, cz, sp.omega0,
                                         inputs.rng_for("tube", 50 + seed), sigma=6.0)
    ch.set_friction_spectral(sp, om)
    return ch, sp, om


def static_call(lbm, sp, om, in_place=False):
    import torch

    lib = lbm.load()
    s = lbm.make_spectral(sp)
    d_om = torch.tensor(om, dtype=torch.float64, device="cuda")
    d_lam = d_om if in_place else torch.full_like(d_om, float("nan"))
    stream = torch.cuda.current_stream()
    rc = lib.lbm_friction_quadrature_static(C.byref(s), C.c_void_p(d_om.data_ptr()), len(om),
                                            C.c_void_p(d_lam.data_ptr()),
                                            C.c_void_p(stream.cuda_stream))
    assert rc == 0
    torch.cuda.synchronize()
    return d_lam.cpu().numpy()


def test_static_quadrature_equals_the_context_path_twice(lbm):
    # a large call, then a smaller one on the same GPU (the array keeps the
    # first call's sums beyond the second's nodes): both bit for bit as the
    # context path
    for R, nx, seed, nq, nw, cpl, vl in ((32, 64, 0, 256, 1024, 0, 0.0),
                                         (6, 20, 1, 64, 256, 1, 0.5)):
        ch, sp, om = tube_case(lbm, R, nx, seed, nq, nw, cpl, vl)
        ref = ch.get_friction()
        got = static_call(lbm, sp, om, in_place=(seed == 1))
        print(f"R {R}: {len(om)} nodes, max |d| {np.max(np.abs(got - ref)):.3e}", flush=True)
        assert got.shape == ref.shape and np.array_equal(got, ref)
        ch.close()


def test_static_quadrature_rejects_oversized_and_bad_input(lbm):
    import torch

    lib = lbm.load()
    sp = inputs.draw_spectral(inputs.rng_for("tube", 3), nq=8, nw=16)
    s = lbm.make_spectral(sp)
    d = torch.zeros(4, dtype=torch.float64, device="cuda")
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    big = (1 << 20) + 1
    assert lib.lbm_friction_quadrature_static(C.byref(s), C.c_void_p(d.data_ptr()), big,
                                              C.c_void_p(d.data_ptr()), stream) == -1
    s.nq = 0
    assert lib.lbm_friction_quadrature_static(C.byref(s), C.c_void_p(d.data_ptr()), 4,
                                              C.c_void_p(d.data_ptr()), stream) == -1
    s.nq = 8
    assert lib.lbm_friction_quadrature_static(C.byref(s), None, 4, None, stream) == -1
    assert lib.lbm_friction_quadrature_static(C.byref(s), None, 0, None, stream) == 0
    torch.cuda.synchronize()
