"""FP64 CPU oracle for the colour-gradient LBM with the ghost-node wetting rule.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The GPU library never imports, links
or runs anything in this package, and this package never touches the GPU
library.  See ``lbm_oracle.c`` for what is computed and which passage of the
paper each step follows.

``liblbm_oracle.so`` is compiled from ``lbm_oracle.c`` by ``build()`` (gcc,
OpenMP, FP64, no FP contraction).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

F_N, F_B, F_PHI, F_U, F_P, F_SOLID, F_PHI_STATE, F_RHO, F_FORCE = range(9)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, OpenMP, -ffp-contract=off)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
               "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("rho_l", C.c_double), ("rho_g", C.c_double), ("mu_l", C.c_double), ("mu_g", C.c_double),
                ("sigma", C.c_double), ("W", C.c_double), ("mobility", C.c_double),
                ("g", C.c_double * 3), ("theta_deg", C.c_double), ("ghost_rule", C.c_int32),
                ("probe", C.c_int32), ("fill", C.c_int32)]


class _Solid(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad", C.c_int32), ("c", C.c_double * 3), ("r", C.c_double),
                ("nrm", C.c_double * 3)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        lib.orc_create.restype = C.c_void_p
        lib.orc_create.argtypes = [C.POINTER(_Params), C.POINTER(_Solid), C.c_int, dp, C.c_char_p, C.c_int]
        lib.orc_destroy.argtypes = [C.c_void_p]
        lib.orc_step.argtypes = [C.c_void_p, C.c_long]
        lib.orc_get.argtypes = [C.c_void_p, C.c_int, dp]
        lib.orc_info.argtypes = [C.c_void_p, C.POINTER(C.c_long)]
        lib.orc_ghosts.argtypes = [C.c_void_p, C.POINTER(C.c_long), dp, C.POINTER(C.c_long), dp]
        lib.orc_lattice.argtypes = [C.c_int, C.c_double, C.POINTER(C.c_int), dp, dp, dp, dp]
        lib.orc_equilibrium.argtypes = [C.c_void_p, dp, C.c_double, dp]
        lib.orc_node.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
        lib.orc_scalars.argtypes = [C.c_void_p, dp]
        lib.orc_set_state.argtypes = [C.c_void_p, dp, dp, dp]
        lib.orc_set_theta.argtypes = [C.c_void_p, C.c_double]
        lib.orc_set_variant.argtypes = [C.c_void_p, C.c_int, C.c_int]
        lib.orc_ghost_rule.restype = C.c_double
        lib.orc_ghost_rule.argtypes = [C.c_double, C.c_double, C.c_int]
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def ghost_rule(phiF: float, eps: float, rule: int = 0) -> float:
    """Eq. 9 (rule 0) or Eq. 10, Fakhari et al. (rule 1)."""
    return _load().orc_ghost_rule(float(phiF), float(eps), int(rule))


def lattice_tables(lattice: int, mobility: float = 0.02) -> Dict[str, np.ndarray]:
    lib = _load()
    c = np.zeros((19, 3), dtype=np.int32)
    w = np.zeros(19)
    chi = np.zeros(19)
    M = np.zeros(19 * 19)
    alpha = np.zeros(1)
    Q = lib.orc_lattice(int(lattice), float(mobility), c.ctypes.data_as(C.POINTER(C.c_int)),
                        _dp(w), _dp(chi), _dp(M), _dp(alpha))
    if Q < 0:
        raise ValueError("bad lattice")
    return {"c": c[:Q].astype(np.int64), "w": w[:Q].copy(), "chi": chi[:Q].copy(),
            "M": M[:Q * Q].reshape(Q, Q).copy(), "alpha": float(alpha[0]), "Q": Q}


MACRO_KEYS = ["phi", "grad", "lap", "rho", "nu", "tau", "u0", "p", "F", "u", "Fs", "Fp", "Fv", "Fb"]
_MACRO_SIZES = [1, 3, 1, 1, 1, 1, 3, 1, 3, 3, 3, 3, 3, 3]


class OracleSim:
    """One oracle simulation.

    ``wl`` is any object with the workload attributes (lattice, shape, rho_l,
    rho_g, mu_l, mu_g, sigma, W, mobility, g, theta, ghost_rule, solids with
    kind/center/radius/normal, nodes); ``phi_init`` is the initial colour
    field in flat node order (x fastest)."""

    def __init__(self, wl, phi_init: np.ndarray):
        lib = _load()
        P = _Params()
        P.lattice = int(wl.lattice)
        P.nx, P.ny, P.nz = (int(v) for v in wl.shape)
        P.rho_l, P.rho_g, P.mu_l, P.mu_g = wl.rho_l, wl.rho_g, wl.mu_l, wl.mu_g
        P.sigma, P.W, P.mobility = wl.sigma, wl.W, wl.mobility
        for a in range(3):
            P.g[a] = wl.g[a]
        P.theta_deg = wl.theta
        P.ghost_rule = int(wl.ghost_rule)
        P.probe = int(getattr(wl, "probe", 0))
        P.fill = int(getattr(wl, "fill", 0))
        ns = len(wl.solids)
        arr = (_Solid * max(ns, 1))()
        for k, s in enumerate(wl.solids):
            arr[k].kind = int(s.kind)
            for a in range(3):
                arr[k].c[a] = float(s.center[a])
                arr[k].nrm[a] = float(s.normal[a])
            arr[k].r = float(s.radius)
        phi_init = np.ascontiguousarray(phi_init, dtype=np.float64)
        if phi_init.size != wl.nodes:
            raise ValueError("phi_init has the wrong size")
        err = C.create_string_buffer(256)
        h = lib.orc_create(C.byref(P), arr, ns, _dp(phi_init), err, 256)
        if not h:
            raise ValueError(f"oracle create failed: {err.value.decode()}")
        self._h = h
        self.wl = wl
        self.n = wl.nodes
        self.Q = 19 if wl.lattice == 1 else 9
        self.D = 3 if wl.lattice == 1 else 2

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().orc_destroy(h)
            self._h = None

    def step(self, nsteps: int = 1) -> None:
        _load().orc_step(self._h, int(nsteps))

    def get(self, field: int) -> np.ndarray:
        size = {F_N: self.Q * self.n, F_B: self.Q * self.n, F_U: 3 * self.n, F_FORCE: 3 * self.n}.get(field, self.n)
        out = np.zeros(size)
        if _load().orc_get(self._h, int(field), _dp(out)) != 0:
            raise ValueError("bad field")
        if field in (F_N, F_B):
            return out.reshape(self.Q, self.n)
        if field in (F_U, F_FORCE):
            return out.reshape(3, self.n)
        return out

    def info(self) -> Dict[str, int]:
        out = (C.c_long * 5)()
        _load().orc_info(self._h, out)
        return {"n_solid": out[0], "n_ghost": out[1], "n_links": out[2], "n_fluid_boundary": out[3],
                "step": out[4]}

    def ghosts(self):
        ng = self.info()["n_ghost"]
        ids = np.zeros(max(ng, 1), dtype=np.int64)
        nrm = np.zeros((max(ng, 1), 3))
        corners = np.zeros((max(ng, 1), 8), dtype=np.int64)
        weights = np.zeros((max(ng, 1), 8))
        _load().orc_ghosts(self._h, ids.ctypes.data_as(C.POINTER(C.c_long)), _dp(nrm),
                           corners.ctypes.data_as(C.POINTER(C.c_long)), _dp(weights))
        return ids[:ng], nrm[:ng], corners[:ng], weights[:ng]

    def equilibrium(self, u: Sequence[float], p: float) -> np.ndarray:
        uu = np.zeros(3)
        uu[: len(u)] = u
        out = np.zeros(self.Q)
        _load().orc_equilibrium(self._h, _dp(uu), float(p), _dp(out))
        return out

    def node(self, N: np.ndarray, phi_nb: np.ndarray):
        N = np.ascontiguousarray(N, dtype=np.float64)
        phi_nb = np.ascontiguousarray(phi_nb, dtype=np.float64)
        Ns = np.zeros(self.Q)
        Bs = np.zeros(self.Q)
        rec = np.zeros(30)
        _load().orc_node(self._h, _dp(N), _dp(phi_nb), _dp(Ns), _dp(Bs), _dp(rec))
        out, k = {}, 0
        for key, sz in zip(MACRO_KEYS, _MACRO_SIZES):
            out[key] = rec[k] if sz == 1 else rec[k:k + sz].copy()
            k += sz
        return Ns, Bs, out

    def scalars(self) -> Dict[str, float]:
        out = np.zeros(5)
        _load().orc_scalars(self._h, _dp(out))
        return dict(zip(["alpha", "eps", "exp_eps", "nu_l", "nu_g"], out.tolist()))

    def set_state(self, N: Optional[np.ndarray] = None, B: Optional[np.ndarray] = None,
                  phi_state: Optional[np.ndarray] = None) -> None:
        def conv(a):
            if a is None:
                return None
            return np.ascontiguousarray(a, dtype=np.float64)
        N, B, ps = conv(N), conv(B), conv(phi_state)
        _load().orc_set_state(self._h, _dp(N) if N is not None else None,
                              _dp(B) if B is not None else None,
                              _dp(ps) if ps is not None else None)

    VISC, SEG = 0, 1
    VISC_PAPER, VISC_FLIPPED, VISC_DROPPED, VISC_NO_TAU_FACTOR = 0, 1, 2, 3
    SEG_CLAMPED, SEG_LITERAL = 0, 1

    def set_variant(self, which: int, value: int) -> None:
        """Alternative reading or planted mistake of one term (orc_set_variant):
        VISC: 0 Eq. A11 as read, 1 sign flipped, 2 left out, 3 without the
        (tau - 1/2)/tau factor; SEG: 0 max(phi (1 - phi), 0), 1 the literal
        factor of Eq. A12.  The non-zero VISC values are planted mistakes for
        negative controls of the pins."""
        if _load().orc_set_variant(self._h, int(which), int(value)) != 0:
            raise ValueError("unknown variant")

    def set_theta(self, theta: float) -> None:
        if _load().orc_set_theta(self._h, float(theta)) != 0:
            raise ValueError("theta outside [0, 180]")

    # ---- observables in FP64, fixed node order (the same definitions the
    # library reports)
    def observe(self) -> Dict[str, float]:
        solid = self.get(F_SOLID) > 0.5
        fluid = ~solid
        phi = self.get(F_PHI)
        u = self.get(F_U)
        rho = self.get(F_RHO)
        speed = np.sqrt((u * u).sum(axis=0))
        return {
            "mass_blue": float(phi[fluid].sum()),
            "mass_red": float((1.0 - phi[fluid]).sum()),
            "momentum": [float((rho[fluid] * u[a][fluid]).sum()) for a in range(3)],
            "max_speed": float(speed[fluid].max()) if fluid.any() else 0.0,
            "kinetic_energy": float((0.5 * rho[fluid] * speed[fluid] ** 2).sum()),
        }
