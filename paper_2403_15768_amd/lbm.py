"""Thin ctypes binding of liblbm.so (the C ABI in include/lbm.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies the device arena (a uint8 tensor) and the HIP
stream; nothing here computes on the data.  Loading fails loudly when the
library has not been built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "liblbm.so")

D2Q9, D3Q19 = 9, 19
F64, F32, F16S = 0, 1, 2
SLAB, DUCT, TUBE, MASKED = 0, 1, 2, 3
PRECISION = {"f64": F64, "f32": F32, "f16s": F16S}

STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EDEVICE",
          -4: "LBM_ENOTCONV", -5: "LBM_EDIVERGED", -6: "LBM_ESTATE"}


class LBMError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int), ("precision", C.c_int), ("geometry", C.c_int),
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("tube_radius", C.c_double), ("tube_cy", C.c_double), ("tube_cz", C.c_double),
        ("tau", C.c_double), ("rho0", C.c_double),
        ("force", C.c_double * 3),
        ("wall_velocity_top", C.c_double),
        ("solid", C.c_void_p),
    ]


class Spectral(C.Structure):
    _fields_ = [
        ("T", C.c_double), ("omega0", C.c_double), ("gamma_s", C.c_double),
        ("omega_l", C.c_double), ("gamma_l", C.c_double), ("a_l", C.c_double),
        ("d", C.c_double), ("nq", C.c_int), ("nw", C.c_int),
        ("q_max", C.c_double), ("w_max", C.c_double),
        ("lambda_target", C.c_double), ("dispersion", C.c_int),
        ("coupling", C.c_int), ("v_l", C.c_double),
    ]


# every symbol include/lbm.h declares
EXPORTS = [
    "lbm_footprint", "lbm_create", "lbm_destroy", "lbm_fluid_count", "lbm_wall_count",
    "lbm_wall_coords", "lbm_wall_links", "lbm_set_friction", "lbm_set_friction_spectral",
    "lbm_get_friction", "lbm_step", "lbm_run_to_steady", "lbm_invariants", "lbm_flux",
    "lbm_mass", "lbm_get_field", "lbm_get_populations", "lbm_state_bytes", "lbm_get_state",
    "lbm_set_state", "lbm_step_count", "lbm_sync", "lbm_last_error", "lbm_copy_probe",
    "lbm_transfer_state", "lbm_batch_footprint", "lbm_batch_create", "lbm_batch_destroy",
    "lbm_batch_items", "lbm_batch_step", "lbm_batch_invariants", "lbm_batch_tune",
    "lbm_batch_set_shape", "lbm_batch_set_group_bytes", "lbm_batch_groups", "lbm_batch_set_streams",
    "lbm_batch_last_error", "lbm_set_thermal", "lbm_set_populations", "lbm_set_electrons",
    "lbm_get_electrons", "lbm_set_open_ends", "lbm_set_noise_closure", "lbm_set_phonons",
    "lbm_get_phonons", "lbm_shell_count", "lbm_step_checked", "lbm_checked_invariants",
    "lbm_friction_quadrature_static", "lbm_batch_member_cost", "lbm_batch_spec_footprint",
    "lbm_batch_create_spec", "lbm_batch_add", "lbm_batch_remove", "lbm_batch_size",
    "lbm_batch_settings", "lbm_invariants_async", "lbm_tune", "lbm_set_block",
]

NOISE_STRESS, NOISE_ALL = 1, 2

_lib = None


def load() -> C.CDLL:
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP runtime; it must be loaded before liblbm.so so
    # that the library binds to that runtime (same soname) instead of pulling
    # in a second one whose streams and allocations torch's would not know
    import torch  # noqa: F401

    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(hipcc, gfx950); there is no CPU fallback")
    lib = C.CDLL(LIB_PATH)
    vp, dp, sz, i64 = C.c_void_p, C.POINTER(C.c_double), C.c_size_t, C.c_int64
    pp = C.POINTER(Params)
    sig = {
        "lbm_footprint": [pp, C.POINTER(sz)],
        "lbm_create": [pp, vp, sz, vp, C.POINTER(vp)],
        "lbm_fluid_count": [vp, C.POINTER(sz)],
        "lbm_wall_count": [vp, C.POINTER(sz)],
        "lbm_wall_coords": [vp, C.POINTER(C.c_int32)],
        "lbm_wall_links": [vp, dp],
        "lbm_set_friction": [vp, vp, sz, C.c_int],
        "lbm_set_friction_spectral": [vp, C.POINTER(Spectral), vp, sz, C.c_int],
        "lbm_get_friction": [vp, dp, dp],
        "lbm_step": [vp, i64],
        "lbm_set_thermal": [vp, C.c_double, C.c_int, C.c_uint64],
        "lbm_set_electrons": [vp, C.c_double, C.c_double, C.c_double, C.c_double],
        "lbm_get_electrons": [vp, dp, dp],
        "lbm_set_phonons": [vp, C.c_double, C.c_double, C.c_double, C.c_double],
        "lbm_get_phonons": [vp, dp, dp],
        "lbm_shell_count": [vp, C.POINTER(C.c_size_t)],
        "lbm_set_open_ends": [vp, C.c_int, C.c_double, C.c_double],
        "lbm_set_noise_closure": [vp, dp, C.c_int, C.c_int, dp, dp],
        "lbm_run_to_steady": [vp, C.c_double, i64, i64, C.POINTER(i64)],
        "lbm_step_checked": [vp, i64],
        "lbm_friction_quadrature_static": [C.POINTER(Spectral), vp, sz, vp, vp],
        "lbm_checked_invariants": [vp, dp, C.POINTER(i64)],
        "lbm_invariants": [vp, dp],
        "lbm_invariants_async": [vp, vp],
        "lbm_tune": [vp, C.c_int, C.POINTER(C.c_int), dp],
        "lbm_set_block": [vp, C.c_int],
        "lbm_flux": [vp, dp],
        "lbm_mass": [vp, dp],
        "lbm_get_field": [vp, C.c_int, dp],
        "lbm_get_populations": [vp, dp],
        "lbm_set_populations": [vp, dp, i64],
        "lbm_state_bytes": [vp, C.POINTER(sz)],
        "lbm_get_state": [vp, vp, sz, C.POINTER(i64)],
        "lbm_set_state": [vp, vp, sz, i64],
        "lbm_step_count": [vp, C.POINTER(i64)],
        "lbm_sync": [vp],
        "lbm_copy_probe": [vp, vp, sz, vp],
        "lbm_transfer_state": [vp, vp],
        "lbm_batch_footprint": [vp, C.c_int, C.POINTER(sz)],
        "lbm_batch_create": [vp, C.c_int, vp, sz, vp, C.POINTER(vp)],
        "lbm_batch_items": [vp, C.POINTER(i64)],
        "lbm_batch_step": [vp, i64],
        "lbm_batch_invariants": [vp, dp],
        "lbm_batch_tune": [vp, C.c_int, vp],
        "lbm_batch_settings": [vp, vp],
        "lbm_batch_member_cost": [vp, C.POINTER(i64), C.POINTER(i64)],
        "lbm_batch_spec_footprint": [vp, C.POINTER(sz)],
        "lbm_batch_create_spec": [vp, vp, sz, vp, C.POINTER(vp)],
        "lbm_batch_add": [vp, vp, C.POINTER(C.c_int)],
        "lbm_batch_remove": [vp, vp],
        "lbm_batch_size": [vp, C.POINTER(C.c_int), C.POINTER(C.c_int)],
        "lbm_batch_set_shape": [vp, C.c_int],
        "lbm_batch_set_group_bytes": [vp, sz],
        "lbm_batch_groups": [vp, C.POINTER(C.c_int)],
        "lbm_batch_set_streams": [vp, C.c_int],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.lbm_destroy.argtypes = [vp]
    lib.lbm_destroy.restype = None
    lib.lbm_last_error.argtypes = [vp]
    lib.lbm_last_error.restype = C.c_char_p
    lib.lbm_batch_destroy.argtypes = [vp]
    lib.lbm_batch_destroy.restype = None
    lib.lbm_batch_last_error.argtypes = [vp]
    lib.lbm_batch_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(lattice: int, geometry: int, nx: int, ny: int, nz: int, tau: float,
                force=(0.0, 0.0, 0.0), precision="f32", rho0: float = 1.0,
                tube_radius: float = 0.0, tube_cy: float = 0.0, tube_cz: float = 0.0,
                wall_velocity_top: float = 0.0, solid=None) -> Params:
    """Creation parameters.  ``solid`` (MASKED only): the solid points of the
    (x, y) plane, array-like shaped (ny, nx), nonzero = solid; the Params
    object keeps its own copy alive."""
    p = Params()
    p.lattice, p.geometry = lattice, geometry
    p.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
    p.nx, p.ny, p.nz = nx, ny, nz
    p.tube_radius, p.tube_cy, p.tube_cz = tube_radius, tube_cy, tube_cz
    p.tau, p.rho0 = tau, rho0
    p.force = (C.c_double * 3)(*force)
    p.wall_velocity_top = wall_velocity_top
    if solid is not None:
        mask = np.ascontiguousarray(np.asarray(solid) != 0, dtype=np.uint8)
        if mask.shape != (ny, nx):
            raise ValueError(f"solid mask must be shaped (ny, nx) = {(ny, nx)}")
        p._solid = mask
        p.solid = mask.ctypes.data
    return p


def footprint(params: Params) -> int:
    n = C.c_size_t()
    rc = load().lbm_footprint(C.byref(params), C.byref(n))
    if rc != 0:
        raise LBMError(rc, "lbm_footprint rejected the parameters")
    return int(n.value)


def make_spectral(sp) -> Spectral:
    """From any object with the lbm_spectral fields (q_max/w_max default to
    10/d and 20 T)."""
    s = Spectral()
    for f in ("T", "omega0", "gamma_s", "omega_l", "gamma_l", "a_l", "d", "nq", "nw",
              "lambda_target"):
        setattr(s, f, getattr(sp, f))
    s.q_max = getattr(sp, "q_max", None) or 10.0 / sp.d
    s.w_max = getattr(sp, "w_max", None) or 20.0 * sp.T
    s.dispersion = int(getattr(sp, "dispersion", 1))
    s.coupling = int(getattr(sp, "coupling", 0))
    s.v_l = float(getattr(sp, "v_l", 0.0))
    return s


class Channel:
    """One lattice-Boltzmann channel on the GPU (a context of liblbm)."""

    def __init__(self, lattice: int, geometry: int, nx: int, ny: int, nz: int, tau: float,
                 force=(0.0, 0.0, 0.0), precision="f32", rho0: float = 1.0,
                 tube_radius: float = 0.0, tube_cy: float = 0.0, tube_cz: float = 0.0,
                 wall_velocity_top: float = 0.0, device: str = "cuda", stream=None,
                 solid=None):
        import torch  # device memory and streams only

        self._lib = load()
        self.params = make_params(lattice, geometry, nx, ny, nz, tau, force, precision, rho0,
                                  tube_radius, tube_cy, tube_cz, wall_velocity_top, solid)
        self.nbytes = footprint(self.params)
        dev = torch.device(device)
        self.arena = torch.empty(self.nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = C.c_void_p()
        rc = self._lib.lbm_create(C.byref(self.params), C.c_void_p(self.arena.data_ptr()),
                                  self.nbytes, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != 0:
            raise LBMError(rc, "lbm_create failed")
        self._h = h
        self.q, self.nx, self.ny, self.nz = lattice, nx, ny, nz
        self.shape = (nz, ny, nx)

    def close(self) -> None:
        """Destroy the context and release its device arena (to torch's
        caching allocator)."""
        h = getattr(self, "_h", None)
        if h:
            self._lib.lbm_destroy(h)
            self._h = None
        self.arena = None

    def __del__(self):
        self.close()

    def _ck(self, rc: int, what: str) -> None:
        if rc != 0:
            raise LBMError(rc, f"{what}: {self._lib.lbm_last_error(self._h).decode()}")

    # ---- geometry
    @property
    def fluid_count(self) -> int:
        n = C.c_size_t()
        self._ck(self._lib.lbm_fluid_count(self._h, C.byref(n)), "lbm_fluid_count")
        return int(n.value)

    @property
    def wall_count(self) -> int:
        n = C.c_size_t()
        self._ck(self._lib.lbm_wall_count(self._h, C.byref(n)), "lbm_wall_count")
        return int(n.value)

    def wall_coords(self) -> np.ndarray:
        out = np.zeros((self.wall_count, 3), dtype=np.int32)
        self._ck(self._lib.lbm_wall_coords(self._h, out.ctypes.data_as(C.POINTER(C.c_int32))),
                 "lbm_wall_coords")
        return out

    def wall_links(self) -> np.ndarray:
        out = np.zeros((self.wall_count, self.q), dtype=np.float64)
        self._ck(self._lib.lbm_wall_links(self._h, _dptr(out)), "lbm_wall_links")
        return out

    # ---- friction
    def set_friction(self, lam) -> None:
        """Per wall node (canonical order): numpy array or float (host) or a
        torch CUDA float64 tensor (device)."""
        if hasattr(lam, "is_cuda") and lam.is_cuda:
            assert lam.dtype.itemsize == 8 and lam.is_contiguous()
            self._ck(self._lib.lbm_set_friction(self._h, C.c_void_p(lam.data_ptr()), lam.numel(), 1),
                     "lbm_set_friction")
            return
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(lam, dtype=np.float64),
                                                 (self.wall_count,)))
        self._ck(self._lib.lbm_set_friction(self._h, a.ctypes.data_as(C.c_void_p), a.size, 0),
                 "lbm_set_friction")

    def set_friction_spectral(self, sp, omega) -> None:
        s = make_spectral(sp)
        if hasattr(omega, "is_cuda") and omega.is_cuda:
            self._ck(self._lib.lbm_set_friction_spectral(self._h, C.byref(s),
                                                         C.c_void_p(omega.data_ptr()),
                                                         omega.numel(), 1),
                     "lbm_set_friction_spectral")
            return
        a = np.ascontiguousarray(np.asarray(omega, dtype=np.float64))
        self._ck(self._lib.lbm_set_friction_spectral(self._h, C.byref(s),
                                                     a.ctypes.data_as(C.c_void_p), a.size, 0),
                 "lbm_set_friction_spectral")

    def get_friction(self, raw: bool = False):
        lam = np.zeros(self.wall_count)
        r = np.zeros(self.wall_count + 1) if raw else None
        self._ck(self._lib.lbm_get_friction(self._h, _dptr(lam), _dptr(r) if raw else None),
                 "lbm_get_friction")
        return (lam, r) if raw else lam

    # ---- thermal fluctuations
    def set_thermal(self, kT: float, mode: int = NOISE_ALL, seed: int = 0) -> None:
        """Fluctuating update at lattice temperature kT (0 = off); mode
        NOISE_STRESS (the stress source alone) or NOISE_ALL."""
        self._ck(self._lib.lbm_set_thermal(self._h, float(kT), int(mode), int(seed)),
                 "lbm_set_thermal")

    def set_noise_closure(self, gamma=None, wx=None, wt=None) -> None:
        """One-point closure of the quantum noise (stress-source form): gamma
        shaped (6, nr, ns) for the components xx, yy, zz, xy, xz, yz at lags
        (r, s), weights wx (nr) and wt (ns); None: the classical noise."""
        if gamma is None:
            rc = self._lib.lbm_set_noise_closure(self._h, None, 0, 0, None, None)
        else:
            g = np.ascontiguousarray(gamma, dtype=np.float64)
            a = np.ascontiguousarray(wx, dtype=np.float64)
            b = np.ascontiguousarray(wt, dtype=np.float64)
            if g.shape != (6, a.size, b.size):
                raise ValueError("gamma must be shaped (6, len(wx), len(wt))")
            dpt = C.POINTER(C.c_double)
            rc = self._lib.lbm_set_noise_closure(self._h, g.ctypes.data_as(dpt), a.size, b.size,
                                                 a.ctypes.data_as(dpt), b.ctypes.data_as(dpt))
        self._ck(rc, "lbm_set_noise_closure")

    # ---- open x ends
    def set_open_ends(self, rho_in: float, rho_out: float, open_: bool = True) -> None:
        """Neumann-like inlet and outlet at densities rho_in and rho_out in
        place of periodic x (open_=False: periodic again)."""
        self._ck(self._lib.lbm_set_open_ends(self._h, int(bool(open_)), float(rho_in),
                                             float(rho_out)), "lbm_set_open_ends")

    # ---- electron sheets (slab walls)
    def set_electrons(self, tau_e: float, rho_e0: float = 1.0, gamma_e: float = 0.0,
                      force_e: float = 0.0) -> None:
        """Electron lines in the solid next to every slab or duct wall (tau_e = 0:
        off); resets them to rest."""
        self._ck(self._lib.lbm_set_electrons(self._h, float(tau_e), float(rho_e0),
                                             float(gamma_e), float(force_e)),
                 "lbm_set_electrons")

    @property
    def shell_count(self) -> int:
        """Electron lines: y = -1, y = ny (by z), then for a duct z = -1, z = nz
        (by y); a tube's: its solid columns next to the water along y or z, by
        increasing y + ny z."""
        n = C.c_size_t()
        self._ck(self._lib.lbm_shell_count(self._h, C.byref(n)), "lbm_shell_count")
        return int(n.value)

    def electrons(self):
        """(u_e of the last step [shell][x], populations [i][shell][x])."""
        ue = np.zeros((self.shell_count, self.nx))
        pops = np.zeros((3, self.shell_count, self.nx))
        self._ck(self._lib.lbm_get_electrons(self._h, _dptr(ue), _dptr(pops)),
                 "lbm_get_electrons")
        return ue, pops

    def set_phonons(self, tau_p: float, rho_p0: float = 1.0, gamma_pc: float = 0.0,
                    gamma_ep: float = 0.0) -> None:
        """Phonon lines beside the electron lines (tau_p = 0: off); reset to rest."""
        self._ck(self._lib.lbm_set_phonons(self._h, float(tau_p), float(rho_p0),
                                           float(gamma_pc), float(gamma_ep)), "lbm_set_phonons")

    def phonons(self):
        """(u_p of the last step [shell][x], phonon populations [i][shell][x])."""
        ns = self.shell_count
        up = np.zeros((ns, self.nx))
        pops = np.zeros((3, ns, self.nx))
        dpt = C.POINTER(C.c_double)
        self._ck(self._lib.lbm_get_phonons(self._h, up.ctypes.data_as(dpt),
                                           pops.ctypes.data_as(dpt)), "lbm_get_phonons")
        return up, pops

    # ---- kernel shape
    def tune(self, retime: bool = False):
        """Autotune the step kernel's block width (cached per kind and size of
        channel); returns (width, microseconds per step or 0 if cached)."""
        bx, us = C.c_int(), C.c_double()
        self._ck(self._lib.lbm_tune(self._h, 1 if retime else 0, C.byref(bx), C.byref(us)),
                 "lbm_tune")
        return int(bx.value), float(us.value)

    def set_block(self, bx: int) -> None:
        """Step kernel block width (64, 128, 256, 512; 0 = default)."""
        self._ck(self._lib.lbm_set_block(self._h, int(bx)), "lbm_set_block")

    # ---- time stepping
    def step(self, n: int) -> None:
        self._ck(self._lib.lbm_step(self._h, int(n)), "lbm_step")

    def step_checked(self, n: int) -> None:
        """n >= 1 steps; the last also reduces the invariants of the state it
        reads (asynchronous; collect them with checked_invariants)."""
        self._ck(self._lib.lbm_step_checked(self._h, int(n)), "lbm_step_checked")

    def checked_invariants(self):
        """(flux, mass, mass deviation, step) of the last step_checked's
        reduction: the state one step before that call's end."""
        out = np.zeros(3)
        at = C.c_int64()
        self._ck(self._lib.lbm_checked_invariants(self._h, _dptr(out), C.byref(at)),
                 "lbm_checked_invariants")
        return float(out[0]), float(out[1]), float(out[2]), int(at.value)

    def run_to_steady(self, rel_tol: float = 1e-8, check_every: int = 1000,
                      max_steps: int = 10 ** 7) -> int:
        taken = C.c_int64()
        self._ck(self._lib.lbm_run_to_steady(self._h, rel_tol, check_every, max_steps,
                                             C.byref(taken)), "lbm_run_to_steady")
        return int(taken.value)

    def sync(self) -> None:
        self._ck(self._lib.lbm_sync(self._h), "lbm_sync")

    @property
    def step_count(self) -> int:
        s = C.c_int64()
        self._ck(self._lib.lbm_step_count(self._h, C.byref(s)), "lbm_step_count")
        return int(s.value)

    # ---- outputs
    def invariants(self):
        out = np.zeros(3)
        self._ck(self._lib.lbm_invariants(self._h, _dptr(out)), "lbm_invariants")
        return float(out[0]), float(out[1]), float(out[2])

    def invariants_async(self, out) -> None:
        """Enqueue the invariants (flux, mass, mass deviation) into ``out``, a
        pinned CPU float64 torch tensor of 3 elements, written when the
        stream reaches this point."""
        assert out.dtype.itemsize == 8 and out.numel() >= 3 and out.is_pinned()
        self._ck(self._lib.lbm_invariants_async(self._h, C.c_void_p(out.data_ptr())),
                 "lbm_invariants_async")

    def flux(self) -> float:
        q = C.c_double()
        self._ck(self._lib.lbm_flux(self._h, C.byref(q)), "lbm_flux")
        return q.value

    def mass(self) -> float:
        m = C.c_double()
        self._ck(self._lib.lbm_mass(self._h, C.byref(m)), "lbm_mass")
        return m.value

    def field(self, which: int) -> np.ndarray:
        out = np.zeros(self.shape)
        self._ck(self._lib.lbm_get_field(self._h, int(which), _dptr(out)), "lbm_get_field")
        return out

    def fields(self):
        return tuple(self.field(k) for k in range(4))

    def populations(self) -> np.ndarray:
        out = np.zeros((self.q,) + self.shape)
        self._ck(self._lib.lbm_get_populations(self._h, _dptr(out)), "lbm_get_populations")
        return out

    def set_populations(self, g: np.ndarray, step: int = 0) -> None:
        """Replace the state by dense shifted populations [i][z][y][x]."""
        g = np.ascontiguousarray(g, dtype=np.float64)
        assert g.shape == (self.q,) + self.shape
        self._ck(self._lib.lbm_set_populations(self._h, _dptr(g), int(step)),
                 "lbm_set_populations")

    def get_state(self):
        n = C.c_size_t()
        self._ck(self._lib.lbm_state_bytes(self._h, C.byref(n)), "lbm_state_bytes")
        buf = np.zeros(n.value, dtype=np.uint8)
        step = C.c_int64()
        self._ck(self._lib.lbm_get_state(self._h, buf.ctypes.data_as(C.c_void_p), buf.size,
                                         C.byref(step)), "lbm_get_state")
        return buf, int(step.value)

    def transfer_from(self, other: "Channel") -> None:
        """Take over the state of another channel of the same geometry (any
        storage precision)."""
        self._ck(self._lib.lbm_transfer_state(self._h, other._h), "lbm_transfer_state")

    def set_state(self, buf: np.ndarray, step: int) -> None:
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._ck(self._lib.lbm_set_state(self._h, buf.ctypes.data_as(C.c_void_p), buf.size,
                                         int(step)), "lbm_set_state")


class BatchSpec(C.Structure):
    _fields_ = [("lattice", C.c_int), ("precision", C.c_int), ("tube", C.c_int),
                ("noise", C.c_int), ("open_ends", C.c_int), ("electrons", C.c_int),
                ("max_members", C.c_int),
                ("max_items", C.c_int64), ("max_columns", C.c_int64)]


class Tuning(C.Structure):
    _fields_ = [("waves_per_group", C.c_int), ("group_bytes", C.c_size_t), ("streams", C.c_int),
                ("us_per_step", C.c_double), ("us_per_step_default", C.c_double),
                ("cached", C.c_int), ("repacks", C.c_int64)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


def member_cost(ch: "Channel"):
    """(work items, fluid columns) a channel takes up in a batch."""
    items, cols = C.c_int64(), C.c_int64()
    rc = load().lbm_batch_member_cost(ch._h, C.byref(items), C.byref(cols))
    if rc != 0:
        raise LBMError(rc, "lbm_batch_member_cost")
    return int(items.value), int(cols.value)


class Batch:
    """Many channels advanced by one kernel launch per step (lbm_batch_*).

    ``Batch(channels)`` holds exactly those channels; ``Batch.empty(...)``
    makes a batch of a given capacity that channels join (``add``) and leave
    (``remove``) while it runs.  ``channels`` lists the members by slot
    (None for a free slot)."""

    def __init__(self, channels, stream=None, tune: bool = False):
        import torch

        self._lib = load()
        self.channels = list(channels)
        n = len(self.channels)
        arr = (C.c_void_p * n)(*[ch._h.value for ch in self.channels])
        nb = C.c_size_t()
        rc = self._lib.lbm_batch_footprint(arr, n, C.byref(nb))
        if rc != 0:
            raise LBMError(rc, "lbm_batch_footprint rejected the members")
        dev = self.channels[0].arena.device
        self.arena = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else self.channels[0].stream
        h = C.c_void_p()
        rc = self._lib.lbm_batch_create(arr, n, C.c_void_p(self.arena.data_ptr()), nb.value,
                                        C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != 0:
            raise LBMError(rc, "lbm_batch_create failed")
        self._h = h
        self.shape = None
        self.tuning = None
        if tune:
            self.tune()

    @classmethod
    def empty(cls, lattice: int, precision, tube: bool, max_members: int, max_items: int,
              max_columns: int, noise: int = 0, open_ends: bool = False,
              electrons: bool = False, stream=None, device: str = "cuda") -> "Batch":
        """An empty batch of this kind and capacity (see lbm_batch_create_spec)."""
        import torch

        self = cls.__new__(cls)
        self._lib = load()
        sp = BatchSpec()
        sp.lattice, sp.tube, sp.noise = int(lattice), int(bool(tube)), int(noise)
        sp.open_ends = int(bool(open_ends))
        sp.electrons = int(bool(electrons))
        sp.precision = PRECISION[precision] if isinstance(precision, str) else int(precision)
        sp.max_members, sp.max_items, sp.max_columns = int(max_members), int(max_items), int(max_columns)
        nb = C.c_size_t()
        rc = self._lib.lbm_batch_spec_footprint(C.byref(sp), C.byref(nb))
        if rc != 0:
            raise LBMError(rc, "lbm_batch_spec_footprint rejected the capacity")
        self.arena = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=torch.device(device))
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.arena.device)
        h = C.c_void_p()
        rc = self._lib.lbm_batch_create_spec(C.byref(sp), C.c_void_p(self.arena.data_ptr()),
                                             nb.value, C.c_void_p(self.stream.cuda_stream),
                                             C.byref(h))
        if rc != 0:
            raise LBMError(rc, "lbm_batch_create_spec failed")
        self._h = h
        self.channels = []
        self.shape = None
        self.tuning = None
        return self

    def close(self) -> None:
        """Destroy the batch (members untouched) and release its arena."""
        h = getattr(self, "_h", None)
        if h:
            self._lib.lbm_batch_destroy(h)
            self._h = None
        self.arena = None
        self.channels = []

    def __del__(self):
        self.close()

    def _ck(self, rc: int, what: str) -> None:
        if rc != 0:
            raise LBMError(rc, f"{what}: {self._lib.lbm_batch_last_error(self._h).decode()}")

    def add(self, ch: "Channel") -> int:
        """Channel ch joins at its current step; returns its slot."""
        s = C.c_int()
        self._ck(self._lib.lbm_batch_add(self._h, ch._h, C.byref(s)), "lbm_batch_add")
        k = int(s.value)
        while len(self.channels) <= k:
            self.channels.append(None)
        self.channels[k] = ch
        return k

    def remove(self, ch: "Channel") -> None:
        """Channel ch leaves after the queued steps; it stays usable alone."""
        self._ck(self._lib.lbm_batch_remove(self._h, ch._h), "lbm_batch_remove")
        k = self.channels.index(ch)
        self.channels[k] = None
        while self.channels and self.channels[-1] is None:
            self.channels.pop()

    @property
    def members(self) -> int:
        n = C.c_int()
        self._ck(self._lib.lbm_batch_size(self._h, C.byref(n), None), "lbm_batch_size")
        return int(n.value)

    @property
    def items(self) -> int:
        n = C.c_int64()
        self._ck(self._lib.lbm_batch_items(self._h, C.byref(n)), "lbm_batch_items")
        return int(n.value)

    def step(self, n: int) -> None:
        self._ck(self._lib.lbm_batch_step(self._h, int(n)), "lbm_batch_step")

    def invariants(self, raise_on_divergence: bool = True) -> np.ndarray:
        """(slots, 3): flux, mass, mass deviation per slot (NaN rows for free
        slots).  With raise_on_divergence=False a member whose flux or mass is
        not finite shows up as NaN/Inf in its row instead of raising."""
        ns = C.c_int()
        self._ck(self._lib.lbm_batch_size(self._h, None, C.byref(ns)), "lbm_batch_size")
        out = np.zeros(3 * max(int(ns.value), 1))
        rc = self._lib.lbm_batch_invariants(self._h, _dptr(out))
        if rc != 0 and not (rc == -5 and not raise_on_divergence):
            self._ck(rc, "lbm_batch_invariants")
        return out[: 3 * int(ns.value)].reshape(-1, 3)

    def tune(self, retime: bool = False) -> int:
        """Autotune workgroup shape, group size and streams (cached per kind
        and size of batch); returns the workgroup shape, the full choice in
        ``self.tuning``."""
        t = Tuning()
        self._ck(self._lib.lbm_batch_tune(self._h, 1 if retime else 0, C.byref(t)),
                 "lbm_batch_tune")
        self.tuning = t.as_dict()
        self.shape = int(t.waves_per_group)
        return self.shape

    def settings(self) -> dict:
        t = Tuning()
        self._ck(self._lib.lbm_batch_settings(self._h, C.byref(t)), "lbm_batch_settings")
        return t.as_dict()

    def set_shape(self, waves_per_group: int) -> None:
        self._ck(self._lib.lbm_batch_set_shape(self._h, int(waves_per_group)), "lbm_batch_set_shape")
        self.shape = int(waves_per_group)

    def set_group_bytes(self, nbytes: int) -> None:
        """Largest state of one group of members (0: a single group)."""
        self._ck(self._lib.lbm_batch_set_group_bytes(self._h, int(nbytes)),
                 "lbm_batch_set_group_bytes")

    def set_streams(self, n: int) -> None:
        """Streams the groups are dealt to (1..4)."""
        self._ck(self._lib.lbm_batch_set_streams(self._h, int(n)), "lbm_batch_set_streams")

    @property
    def groups(self) -> int:
        n = C.c_int()
        self._ck(self._lib.lbm_batch_groups(self._h, C.byref(n)), "lbm_batch_groups")
        return int(n.value)


def copy_probe(src, dst, nbytes: int, stream) -> None:
    """Plain streaming copy between two torch CUDA tensors (bandwidth probe)."""
    rc = load().lbm_copy_probe(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), int(nbytes),
                               C.c_void_p(stream.cuda_stream))
    if rc != 0:
        raise LBMError(rc, "lbm_copy_probe")


def no_slip() -> float:
    return math.inf
