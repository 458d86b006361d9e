"""ctypes wrapper around the plain C oracle (``pflbm_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle follows the step description of the paper stage by stage
in FP64; this module only marshals arguments.  It shares nothing with the GPU library.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pflbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_pflbm.so")

MAXB = 16
NP = MAXB + 1


class _Config(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("nb", C.c_int32),
        ("tau", C.c_double), ("G", C.c_double), ("rho0", C.c_double),
        ("solid_threshold", C.c_double),
        ("mobility", C.c_double), ("eta", C.c_double),
        ("sigma", C.c_double * (NP * NP)),
        ("rc", C.c_double), ("nexp", C.c_double), ("e0", C.c_double),
        ("RA", C.c_double),
        ("fext", C.c_double * 3),
        ("kinetics", C.c_int32), ("motion", C.c_int32), ("repulsion", C.c_int32),
        ("lattice", C.c_int32),
        ("phi_floor", C.c_double),
        ("volume_after_advection", C.c_int32),
    ]


class _Body(C.Structure):
    _fields_ = [
        ("mass_density", C.c_double), ("wetting_rho", C.c_double),
        ("v", C.c_double * 3), ("w", C.c_double * 3),
        ("fixed", C.c_int32),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP) into an in-tree shared library."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-Wno-unused-variable", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def library_path() -> str:
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = C.CDLL(_LIB)
        P = C.POINTER
        dp = P(C.c_double)
        ip = P(C.c_int32)
        lib.or_create.restype = C.c_void_p
        lib.or_create.argtypes = [P(_Config), P(_Body), dp, dp]
        lib.or_destroy.argtypes = [C.c_void_p]
        lib.or_step.argtypes = [C.c_void_p, C.c_int]
        lib.or_step.restype = C.c_int
        lib.or_set_threads.argtypes = [C.c_int]
        lib.or_max_threads.restype = C.c_int
        for name in ("or_get_rho", "or_get_mom", "or_get_phi", "or_get_f", "or_get_psi",
                     "or_get_force_density", "or_get_diag"):
            getattr(lib, name).argtypes = [C.c_void_p, dp]
        lib.or_set_f.argtypes = [C.c_void_p, dp]
        lib.or_get_mask.argtypes = [C.c_void_p, ip, ip]
        lib.or_get_lattice.argtypes = [C.c_void_p, ip, dp]
        lib.or_num_velocities.argtypes = [C.c_void_p]
        lib.or_num_velocities.restype = C.c_int32
        lib.or_get_bodies.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
        lib.or_get_force_parts.argtypes = [C.c_void_p, dp, dp, dp]
        lib.or_get_body_consts.argtypes = [C.c_void_p, dp, dp, dp]
        lib.or_equilibrium.argtypes = [C.c_void_p, C.c_double, dp, dp]
        lib.or_set_body.argtypes = [C.c_void_p, C.c_int, dp, dp, dp]
        _lib = lib
    return _lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _iptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


class Oracle:
    """One simulation held by the C oracle.

    ``params`` is a dict with the keys of :class:`pflbm_inputs.Params` (``nx, ny, nz, tau, G,
    rho0, solid_threshold, mobility, eta, sigma (nb+1 x nb+1, phase 0 = fluid), rc, nexp, e0,
    RA, fext, kinetics, motion, repulsion``); ``bodies`` a list of dicts with ``mass_density,
    wetting_rho, v, w, fixed``; ``rho0`` a [nz, ny, nx] FP64 array and ``phi0`` [nb, nz, ny, nx].
    """

    def __init__(self, params: dict, bodies: list, rho0: np.ndarray, phi0: np.ndarray, threads: int | None = None):
        lib = _load()
        if threads is not None:
            lib.or_set_threads(int(threads))
        nb = len(bodies)
        if nb > MAXB:
            raise ValueError("too many bodies for the oracle")
        cfg = _Config()
        cfg.nx, cfg.ny, cfg.nz, cfg.nb = int(params["nx"]), int(params["ny"]), int(params["nz"]), nb
        cfg.tau, cfg.G, cfg.rho0 = params["tau"], params["G"], params["rho0"]
        cfg.solid_threshold = params["solid_threshold"]
        cfg.mobility, cfg.eta = params["mobility"], params["eta"]
        sig = np.asarray(params["sigma"], dtype=np.float64)
        for a in range(nb + 1):
            for b in range(nb + 1):
                cfg.sigma[a * NP + b] = float(sig[a, b])
        cfg.rc, cfg.nexp, cfg.e0 = params["rc"], params["nexp"], params["e0"]
        cfg.RA = params["RA"]
        for d in range(3):
            cfg.fext[d] = float(params["fext"][d])
        cfg.kinetics, cfg.motion, cfg.repulsion = int(params["kinetics"]), int(params["motion"]), int(params["repulsion"])
        cfg.lattice = int(params.get("lattice", 19))
        cfg.phi_floor = float(params["phi_floor"])
        cfg.volume_after_advection = int(params.get("volume_after_advection", 0))
        barr = (_Body * max(nb, 1))()
        for i, b in enumerate(bodies):
            barr[i].mass_density = float(b["mass_density"])
            barr[i].wetting_rho = float(b["wetting_rho"])
            for d in range(3):
                barr[i].v[d] = float(b["v"][d])
                barr[i].w[d] = float(b["w"][d])
            barr[i].fixed = int(b.get("fixed", 0))
        self.shape = (cfg.nz, cfg.ny, cfg.nx)
        self.N = cfg.nx * cfg.ny * cfg.nz
        self.nb = nb
        r = np.ascontiguousarray(rho0, dtype=np.float64).reshape(-1)
        p = np.ascontiguousarray(phi0, dtype=np.float64).reshape(-1) if nb else np.zeros(1)
        if r.size != self.N or (nb and p.size != nb * self.N):
            raise ValueError("field sizes do not match the grid")
        self._keep = (cfg, barr, r, p)
        self._h = lib.or_create(C.byref(cfg), barr, _dptr(r), _dptr(p))
        if not self._h:
            raise ValueError("oracle rejected the configuration")
        self._lib = lib

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._lib.or_destroy(h)
            self._h = None

    def step(self, n: int = 1) -> None:
        if self._lib.or_step(self._h, int(n)) != 0:
            raise RuntimeError("oracle step failed")

    # ---- fields --------------------------------------------------------------------------
    def rho(self) -> np.ndarray:
        out = np.empty(self.N)
        self._lib.or_get_rho(self._h, _dptr(out))
        return out.reshape(self.shape)

    def mom(self) -> np.ndarray:
        out = np.empty(3 * self.N)
        self._lib.or_get_mom(self._h, _dptr(out))
        return out.reshape((3,) + self.shape)

    def phi(self) -> np.ndarray:
        out = np.empty(max(self.nb, 1) * self.N)
        self._lib.or_get_phi(self._h, _dptr(out))
        return out[: self.nb * self.N].reshape((self.nb,) + self.shape)

    def mask(self):
        solid = np.empty(self.N, dtype=np.int32)
        owner = np.empty(self.N, dtype=np.int32)
        self._lib.or_get_mask(self._h, _iptr(solid), _iptr(owner))
        return solid.reshape(self.shape), owner.reshape(self.shape)

    @property
    def q(self) -> int:
        return int(self._lib.or_num_velocities(self._h))

    def populations(self) -> np.ndarray:
        out = np.empty(self.q * self.N)
        self._lib.or_get_f(self._h, _dptr(out))
        return out.reshape(self.shape + (self.q,))

    def set_populations(self, f: np.ndarray) -> None:
        a = np.ascontiguousarray(f, dtype=np.float64).reshape(-1)
        self._lib.or_set_f(self._h, _dptr(a))

    def lattice(self):
        c = np.empty(3 * self.q, dtype=np.int32)
        w = np.empty(self.q)
        self._lib.or_get_lattice(self._h, _iptr(c), _dptr(w))
        return c.reshape(self.q, 3), w

    def psi(self) -> np.ndarray:
        out = np.empty(self.N)
        self._lib.or_get_psi(self._h, _dptr(out))
        return out.reshape(self.shape)

    def force_density(self) -> np.ndarray:
        out = np.empty(3 * self.N)
        self._lib.or_get_force_density(self._h, _dptr(out))
        return out.reshape((3,) + self.shape)

    def equilibrium(self, rho: float, u) -> np.ndarray:
        uu = np.asarray(u, dtype=np.float64)
        out = np.empty(self.q)
        self._lib.or_equilibrium(self._h, float(rho), _dptr(uu), _dptr(out))
        return out

    # ---- bodies --------------------------------------------------------------------------
    def bodies(self) -> dict:
        nb = max(self.nb, 1)
        F, T, X, V, W = (np.zeros(3 * nb) for _ in range(5))
        self._lib.or_get_bodies(self._h, _dptr(F), _dptr(T), _dptr(X), _dptr(V), _dptr(W))
        k = 3 * self.nb
        return {"F": F[:k].reshape(-1, 3), "T": T[:k].reshape(-1, 3), "X": X[:k].reshape(-1, 3),
                "V": V[:k].reshape(-1, 3), "W": W[:k].reshape(-1, 3)}

    def force_parts(self) -> dict:
        nb = max(self.nb, 1)
        a, b, c = (np.zeros(3 * nb) for _ in range(3))
        self._lib.or_get_force_parts(self._h, _dptr(a), _dptr(b), _dptr(c))
        k = 3 * self.nb
        return {"me": a[:k].reshape(-1, 3), "sc": b[:k].reshape(-1, 3), "rep": c[:k].reshape(-1, 3)}

    def body_consts(self) -> dict:
        nb = max(self.nb, 1)
        M, I, Vr = np.zeros(nb), np.zeros(9 * nb), np.zeros(nb)
        self._lib.or_get_body_consts(self._h, _dptr(M), _dptr(I), _dptr(Vr))
        return {"M": M[: self.nb], "Iinv": I[: 9 * self.nb].reshape(-1, 3, 3), "Vref": Vr[: self.nb]}

    def set_body(self, b: int, X=None, V=None, W=None) -> None:
        def opt(v):
            if v is None:
                return None
            a = np.ascontiguousarray(v, dtype=np.float64)
            self._keep = self._keep + (a,)
            return _dptr(a)
        self._lib.or_set_body(self._h, int(b), opt(X), opt(V), opt(W))

    def diag(self) -> dict:
        out = np.zeros(4)
        self._lib.or_get_diag(self._h, _dptr(out))
        return {"step": int(out[0]), "lost_mass": out[1], "n_f2s": int(out[2]), "n_s2f": int(out[3])}

    @staticmethod
    def max_threads() -> int:
        return int(_load().or_max_threads())

    @staticmethod
    def set_threads(n: int) -> None:
        _load().or_set_threads(int(n))


def lattice_of(o: Oracle):
    return o.lattice()
