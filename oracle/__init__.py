"""CPU oracle for the lattice-Boltzmann nanochannel path (test infrastructure).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check of
``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``.  The product
path never imports it and shares no code with it.

The arithmetic lives in ``lbm_oracle.c`` (plain scalar loops, FP64, or x87
long double for the self-floor check); this module only compiles it with gcc
and marshals arguments through ctypes.  See the C file's header for what is
computed and which passages of the paper each part follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIBS = {
    "f64": os.path.join(_HERE, "liblbm_oracle.so"),
    "f80": os.path.join(_HERE, "liblbm_oracle_ld.so"),
}

SLAB, DUCT, TUBE, MASKED = 0, 1, 2, 3


def build(verbose: bool = False) -> None:
    """Compile both oracle variants with gcc (no FMA contraction, -O2)."""
    for kind, out in _LIBS.items():
        cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
               "-Wall", "-Wextra", "-o", out + ".tmp", _SRC, "-lm"]
        if kind == "f80":
            cmd.insert(1, "-DORACLE_LONG_DOUBLE")
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


class _Params(C.Structure):
    _fields_ = [
        ("lattice", C.c_int), ("precision", C.c_int), ("geometry", C.c_int),
        ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("tube_radius", C.c_double), ("tube_cy", C.c_double), ("tube_cz", C.c_double),
        ("tau", C.c_double), ("rho0", C.c_double),
        ("force", C.c_double * 3),
        ("wall_velocity_top", C.c_double),
        ("solid", C.c_void_p),
    ]


class _Spectral(C.Structure):
    _fields_ = [
        ("T", C.c_double), ("omega0", C.c_double), ("gamma_s", C.c_double),
        ("omega_l", C.c_double), ("gamma_l", C.c_double), ("a_l", C.c_double),
        ("d", C.c_double), ("nq", C.c_int), ("nw", C.c_int),
        ("q_max", C.c_double), ("w_max", C.c_double),
        ("lambda_target", C.c_double), ("dispersion", C.c_int),
        ("coupling", C.c_int), ("v_l", C.c_double),
    ]


_loaded: dict = {}


def _lib(kind: str = "f64") -> C.CDLL:
    if kind in _loaded:
        return _loaded[kind]
    path = _LIBS[kind]
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        build()
    lib = C.CDLL(path)
    vp, dp, lp = C.c_void_p, C.POINTER(C.c_double), C.c_long
    lib.ora_create.argtypes = [C.POINTER(_Params), C.POINTER(vp)]
    lib.ora_create.restype = C.c_int
    lib.ora_destroy.argtypes = [vp]
    lib.ora_wall_count.argtypes = [vp]
    lib.ora_wall_count.restype = lp
    lib.ora_fluid_count.argtypes = [vp]
    lib.ora_fluid_count.restype = lp
    lib.ora_step_count.argtypes = [vp]
    lib.ora_step_count.restype = lp
    lib.ora_wall_coords.argtypes = [vp, C.POINTER(C.c_int32)]
    lib.ora_wall_links.argtypes = [vp, dp]
    lib.ora_set_friction.argtypes = [vp, dp]
    lib.ora_set_friction.restype = C.c_int
    lib.ora_step.argtypes = [vp, lp]
    lib.ora_fields.argtypes = [vp, dp, dp, dp, dp]
    lib.ora_invariants.argtypes = [vp, dp]
    lib.ora_get_populations.argtypes = [vp, dp]
    lib.ora_set_populations.argtypes = [vp, dp, lp]
    sp = C.POINTER(_Spectral)
    lib.ora_img_l.argtypes = [sp, C.c_double]
    lib.ora_img_l.restype = C.c_double
    lib.ora_img_s.argtypes = [sp, C.c_double, C.c_double, C.c_double]
    lib.ora_img_s.restype = C.c_double
    lib.ora_friction_raw.argtypes = [sp, C.c_double]
    lib.ora_friction_raw.restype = C.c_double
    lib.ora_friction.argtypes = [sp, dp, lp, dp, dp]
    lib.ora_response.argtypes = [sp, C.c_double, C.c_double, C.c_double, dp]
    lib.ora_set_electrons.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_double]
    lib.ora_set_electrons.restype = C.c_int
    lib.ora_get_electrons.argtypes = [vp, dp, dp]
    lib.ora_shell_count.argtypes = [vp]
    lib.ora_shell_count.restype = lp
    lib.ora_set_electron_populations.argtypes = [vp, dp]
    lib.ora_set_electron_populations.restype = C.c_int
    lib.ora_sizeof_real.restype = C.c_int
    lib.ora_set_open_ends.argtypes = [vp, C.c_int, C.c_double, C.c_double]
    lib.ora_set_noise_closure.argtypes = [vp, dp, C.c_int, C.c_int, dp, dp]
    lib.ora_set_noise_closure.restype = C.c_int
    lib.ora_set_phonons.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_double]
    lib.ora_set_phonons.restype = C.c_int
    lib.ora_get_phonons.argtypes = [vp, dp, dp]
    lib.ora_set_open_ends.restype = C.c_int
    u64p = C.POINTER(C.c_uint64)
    lib.ora_set_thermal.argtypes = [vp, C.c_double, C.c_int, C.c_uint64]
    lib.ora_set_thermal.restype = C.c_int
    lib.ora_philox4x64.argtypes = [u64p, u64p, u64p]
    lib.ora_thermal_normals.argtypes = [C.c_uint64, lp, lp, C.c_int, dp]
    _loaded[kind] = lib
    return lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


class OracleError(RuntimeError):
    pass


class Lattice:
    """One lattice-Boltzmann channel in the oracle.

    geometry: SLAB (walls on y, periodic z), DUCT (walls on y and z) or TUBE
    (circular cross-section of ``tube_radius`` centred at (tube_cy, tube_cz) in
    the box) or MASKED (a slab whose solid points in the (x, y) plane are
    ``solid``, shaped (ny, nx), the same for every z: corrugated or stepped
    walls).  For SLAB/DUCT the box is all fluid and the walls lie half a link
    outside it.  ``kind`` = "f64" or "f80" (long double).
    """

    def __init__(self, lattice: int, geometry: int, nx: int, ny: int, nz: int,
                 tau: float, force=(0.0, 0.0, 0.0), rho0: float = 1.0,
                 tube_radius: float = 0.0, tube_cy: float = 0.0, tube_cz: float = 0.0,
                 wall_velocity_top: float = 0.0, kind: str = "f64", solid=None):
        self._lib = _lib(kind)
        p = _Params()
        p.lattice, p.precision, p.geometry = lattice, 0, geometry
        p.nx, p.ny, p.nz = nx, ny, nz
        p.tube_radius, p.tube_cy, p.tube_cz = tube_radius, tube_cy, tube_cz
        p.tau, p.rho0 = tau, rho0
        p.force = (C.c_double * 3)(*force)
        p.wall_velocity_top = wall_velocity_top
        mask = None
        if solid is not None:
            mask = np.ascontiguousarray(np.asarray(solid) != 0, dtype=np.uint8)
            assert mask.shape == (ny, nx)
            p.solid = mask.ctypes.data
        h = C.c_void_p()
        rc = self._lib.ora_create(C.byref(p), C.byref(h))
        if rc != 0:
            raise OracleError(f"ora_create failed with {rc}")
        self._h = h
        self.q, self.nx, self.ny, self.nz = lattice, nx, ny, nz
        self.shape = (nz, ny, nx)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.ora_destroy(h)
            self._h = None

    @property
    def wall_count(self) -> int:
        return int(self._lib.ora_wall_count(self._h))

    @property
    def fluid_count(self) -> int:
        return int(self._lib.ora_fluid_count(self._h))

    @property
    def step_count(self) -> int:
        return int(self._lib.ora_step_count(self._h))

    def wall_coords(self) -> np.ndarray:
        out = np.zeros((self.wall_count, 3), dtype=np.int32)
        self._lib.ora_wall_coords(self._h, out.ctypes.data_as(C.POINTER(C.c_int32)))
        return out

    def wall_links(self) -> np.ndarray:
        """Bouzidi fraction per (wall node, direction); 0 where no wall link."""
        out = np.zeros((self.wall_count, 19), dtype=np.float64)
        self._lib.ora_wall_links(self._h, _dptr(out))
        return out[:, : self.q]

    def set_friction(self, lam) -> None:
        lam = np.ascontiguousarray(np.broadcast_to(np.asarray(lam, dtype=np.float64),
                                                   (self.wall_count,)))
        if self._lib.ora_set_friction(self._h, _dptr(lam)) != 0:
            raise OracleError("friction must be >= 0 (inf allowed)")

    def set_thermal(self, kT: float, mode: int = 2, seed: int = 0) -> None:
        """Thermal fluctuations at lattice temperature kT (0 = off); mode 1 =
        the stress source alone, 2 = every non-conserved direction."""
        if self._lib.ora_set_thermal(self._h, float(kT), int(mode), int(seed)) != 0:
            raise OracleError("kT must be finite and >= 0, mode 1 or 2")

    def set_electrons(self, tau_e: float, rho_e0: float, gamma_e: float,
                      force_e: float = 0.0) -> None:
        """Electron lines in the solid columns next to the water (slab, duct
        and tube walls), coupled to the water by the relative-velocity wall
        drag (state reset to rest)."""
        if self._lib.ora_set_electrons(self._h, float(tau_e), float(rho_e0), float(gamma_e),
                                       float(force_e)) != 0:
            raise OracleError("electron sheets need a SLAB, DUCT or TUBE without moving wall "
                              "or open ends, tau_e > 1/2, rho_e0 > 0, gamma_e >= 0")

    def set_electron_populations(self, pops: np.ndarray) -> None:
        """Replace the electron populations (shifted, [i][shell][x])."""
        e = np.ascontiguousarray(pops, dtype=np.float64)
        assert e.shape == (3, self.shell_count, self.nx)
        if self._lib.ora_set_electron_populations(self._h, _dptr(e)) != 0:
            raise OracleError("the electron lines are off")

    def set_noise_closure(self, gamma=None, wx=None, wt=None) -> None:
        """One-point closure of the quantum noise: gamma shaped (6, nr, ns) (the
        correlator of the components xx, yy, zz, xy, xz, yz at lags r, s),
        weights wx (nr) and wt (ns); None restores the classical noise."""
        if gamma is None:
            rc = self._lib.ora_set_noise_closure(self._h, None, 0, 0, None, None)
        else:
            g = np.ascontiguousarray(gamma, dtype=np.float64)
            a = np.ascontiguousarray(wx, dtype=np.float64)
            b = np.ascontiguousarray(wt, dtype=np.float64)
            assert g.shape == (6, a.size, b.size)
            rc = self._lib.ora_set_noise_closure(self._h, _dptr(g), a.size, b.size, _dptr(a),
                                                 _dptr(b))
        if rc != 0:
            raise OracleError("closure factors must be finite and >= 0")

    def set_open_ends(self, rho_in: float, rho_out: float, open_: bool = True) -> None:
        """Open x ends (Neumann-like inlet and outlet at densities rho_in,
        rho_out); open_=False restores periodic x."""
        if self._lib.ora_set_open_ends(self._h, int(bool(open_)), float(rho_in),
                                       float(rho_out)) != 0:
            raise OracleError("open ends need a SLAB, DUCT, TUBE or MASKED channel (a mask "
                              "with equal first and last rows) without electron sheets, "
                              "nx >= 2 and finite densities > 0")

    def set_phonons(self, tau_p: float, rho_p0: float = 1.0, gamma_pc: float = 0.0,
                    gamma_ep: float = 0.0) -> None:
        """Phonon lines beside the electron lines (tau_p = 0: off); reset to rest."""
        if self._lib.ora_set_phonons(self._h, float(tau_p), float(rho_p0), float(gamma_pc),
                                     float(gamma_ep)) != 0:
            raise OracleError("phonons need the electron lines on, tau_p > 1/2, rho_p0 > 0, "
                              "gamma_pc, gamma_ep >= 0")

    def phonons(self):
        """(u_p of the last step [shell][x], populations [i][shell][x])."""
        up = np.zeros((self.shell_count, self.nx))
        pops = np.zeros((3, self.shell_count, self.nx))
        self._lib.ora_get_phonons(self._h, _dptr(up), _dptr(pops))
        return up, pops

    @property
    def shell_count(self) -> int:
        return int(self._lib.ora_shell_count(self._h))

    def electrons(self):
        """(u_e of the last step [shell][x], shifted populations [i][shell][x]);
        shells: y = -1 (by z), y = ny (by z), then for a duct z = -1 (by y),
        z = nz (by y); for a tube the solid columns next to a fluid column
        along y or z, in increasing y + ny z."""
        ue = np.zeros((self.shell_count, self.nx))
        pops = np.zeros((3, self.shell_count, self.nx))
        self._lib.ora_get_electrons(self._h, _dptr(ue), _dptr(pops))
        return ue, pops

    def step(self, n: int) -> None:
        self._lib.ora_step(self._h, int(n))

    def fields(self):
        """(rho, ux, uy, uz), each shaped (nz, ny, nx); zero on solid cells."""
        outs = [np.zeros(self.shape) for _ in range(4)]
        self._lib.ora_fields(self._h, *[_dptr(a) for a in outs])
        return tuple(outs)

    def invariants(self):
        """(flux Q, mass M, mass deviation sum(rho - rho0))."""
        out = np.zeros(3)
        self._lib.ora_invariants(self._h, _dptr(out))
        return float(out[0]), float(out[1]), float(out[2])

    def get_populations(self) -> np.ndarray:
        out = np.zeros((self.q,) + self.shape)
        self._lib.ora_get_populations(self._h, _dptr(out))
        return out

    def set_populations(self, g: np.ndarray, step: int = 0) -> None:
        g = np.ascontiguousarray(g, dtype=np.float64)
        assert g.shape == (self.q,) + self.shape
        self._lib.ora_set_populations(self._h, _dptr(g), int(step))


@dataclass
class Spectral:
    """Synthetic surface-response spectra of the friction quadrature."""
    T: float
    omega0: float
    gamma_s: float
    omega_l: float
    gamma_l: float
    a_l: float = 0.5
    d: float = 1.0
    nq: int = 256
    nw: int = 1024
    q_max: float | None = None
    w_max: float | None = None
    lambda_target: float = 0.05
    dispersion: int = 1
    coupling: int = 0
    v_l: float = 0.0

    def _c(self) -> _Spectral:
        s = _Spectral()
        s.T, s.omega0, s.gamma_s = self.T, self.omega0, self.gamma_s
        s.omega_l, s.gamma_l, s.a_l, s.d = self.omega_l, self.gamma_l, self.a_l, self.d
        s.nq, s.nw = self.nq, self.nw
        s.q_max = self.q_max if self.q_max is not None else 10.0 / self.d
        s.w_max = self.w_max if self.w_max is not None else 20.0 * self.T
        s.lambda_target, s.dispersion = self.lambda_target, self.dispersion
        s.coupling, s.v_l = self.coupling, self.v_l
        return s


def img_l(sp: Spectral, w: float, kind: str = "f64") -> float:
    s = sp._c()
    return _lib(kind).ora_img_l(C.byref(s), float(w))


def img_s(sp: Spectral, Omega: float, q: float, w: float, kind: str = "f64") -> float:
    s = sp._c()
    return _lib(kind).ora_img_s(C.byref(s), float(Omega), float(q), float(w))


def response(sp: Spectral, Omega: float, q: float, w: float, kind: str = "f64"):
    """Complex surface responses (g_s, g_l) at wavevector q and frequency w."""
    s = sp._c()
    out = np.zeros(4)
    _lib(kind).ora_response(C.byref(s), float(Omega), float(q), float(w), _dptr(out))
    return complex(out[0], out[1]), complex(out[2], out[3])


def friction_raw(sp: Spectral, Omega: float, kind: str = "f64") -> float:
    s = sp._c()
    return _lib(kind).ora_friction_raw(C.byref(s), float(Omega))


def friction(sp: Spectral, Omega, kind: str = "f64"):
    """(raw lambda_k, lattice lambda_k) for the plasmon frequencies Omega_k."""
    Om = np.ascontiguousarray(np.atleast_1d(np.asarray(Omega, dtype=np.float64)))
    raw = np.zeros_like(Om)
    lat = np.zeros_like(Om)
    s = sp._c()
    _lib(kind).ora_friction(C.byref(s), _dptr(Om), len(Om), _dptr(raw), _dptr(lat))
    return raw, lat


def philox4x64(ctr, key, kind: str = "f64") -> np.ndarray:
    """Philox4x64-10 of one 256-bit counter under one 128-bit key."""
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint64))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64))
    assert c.shape == (4,) and k.shape == (2,)
    out = np.zeros(4, dtype=np.uint64)
    u64p = C.POINTER(C.c_uint64)
    _lib(kind).ora_philox4x64(c.ctypes.data_as(u64p), k.ctypes.data_as(u64p),
                              out.ctypes.data_as(u64p))
    return out


def thermal_normals(seed: int, cell: int, step: int, count: int, kind: str = "f64") -> np.ndarray:
    """The first ``count`` standard normals the thermal noise of ``cell`` draws at ``step``."""
    out = np.zeros(count)
    _lib(kind).ora_thermal_normals(int(seed), int(cell), int(step), int(count), _dptr(out))
    return out


def sizeof_real(kind: str = "f64") -> int:
    return int(_lib(kind).ora_sizeof_real())
