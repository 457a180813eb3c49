"""ctypes binding of liblbm.so (include/lbm.h) with PyTorch-owned device memory.

Argument marshalling only: every step of the update runs in the HIP kernels of
the shared library.  There is no CPU fallback; loading fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional, Sequence

import numpy as np

from . import workloads as W

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

ABI_VERSION = 2
OK, EINVAL, ESTATE, ENOMEM, EHIP, EUNSTABLE = 0, -1, -2, -3, -4, -5
OPT_FUSED = 1
OPT_FLUID_PROBE = 2
OPT_GRAPH = 8
OPT_FILL_DEAD_ENDS = 16
OPT_SPARSE = 32
(FIELD_PHI, FIELD_N, FIELD_B, FIELD_U, FIELD_P, FIELD_SOLID_PHI, FIELD_FLAGS, FIELD_N_OFFSET,
 FIELD_PHI_STATE) = range(9)
FLAG_SOLID, FLAG_NEAR_SOLID, FLAG_GHOST = 1, 2, 4

EXPORTED = ["lbm_create", "lbm_set_geometry", "lbm_device_bytes", "lbm_bind", "lbm_set_wetting",
            "lbm_set_field", "lbm_step", "lbm_step_profiled", "lbm_observe", "lbm_read_field",
            "lbm_lattice", "lbm_destroy", "lbm_last_error", "lbm_batch_table_bytes", "lbm_batch_create",
            "lbm_batch_step", "lbm_batch_destroy", "lbm_batch_last_error", "lbm_hbm_probe",
            "lbm_observe_static"]


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


class lbm_params(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("lattice", C.c_uint32), ("precision", C.c_uint32),
                ("ghost_rule", C.c_uint32), ("n", C.c_int32 * 3), ("options", C.c_int32),
                ("rho_l", C.c_double), ("rho_g", C.c_double), ("mu_l", C.c_double), ("mu_g", C.c_double),
                ("sigma", C.c_double), ("W", C.c_double), ("mobility", C.c_double),
                ("body_accel", C.c_double * 3)]


class lbm_solid(C.Structure):
    _fields_ = [("kind", C.c_uint32), ("pad", C.c_uint32), ("center", C.c_double * 3),
                ("radius", C.c_double), ("normal", C.c_double * 3)]


class lbm_obs(C.Structure):
    _fields_ = [("step", C.c_int64), ("n_fluid", C.c_int64), ("n_solid", C.c_int64),
                ("n_ghost", C.c_int64), ("nonfinite", C.c_int64), ("mass_blue", C.c_double),
                ("mass_red", C.c_double), ("momentum", C.c_double * 3), ("max_speed", C.c_double),
                ("kinetic_energy", C.c_double)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblbm.so (raises if it is missing: there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2605_30878_amd.build_lib`")
    # torch first: its HIP runtime is then the one the library binds to, so
    # device pointers from torch's allocator are known to the library's calls
    import torch  # noqa: F401
    lib = C.CDLL(path)
    vp, dp = C.c_void_p, C.POINTER(C.c_double)
    lib.lbm_create.argtypes = [C.POINTER(lbm_params), C.POINTER(vp)]
    lib.lbm_set_geometry.argtypes = [vp, C.POINTER(lbm_solid), C.c_int32]
    lib.lbm_device_bytes.argtypes = [vp, C.POINTER(C.c_size_t)]
    lib.lbm_bind.argtypes = [vp, vp, C.c_size_t, vp]
    lib.lbm_set_wetting.argtypes = [vp, C.c_double]
    lib.lbm_set_field.argtypes = [vp, C.c_int, dp, C.c_size_t]
    lib.lbm_step.argtypes = [vp, C.c_int64]
    lib.lbm_step_profiled.argtypes = [vp, C.c_int64, dp]
    lib.lbm_observe.argtypes = [vp, C.POINTER(lbm_obs)]
    lib.lbm_observe_static.argtypes = [vp, C.POINTER(lbm_obs)]
    lib.lbm_read_field.argtypes = [vp, C.c_int, dp, C.c_size_t]
    lib.lbm_lattice.argtypes = [C.c_uint32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
    lib.lbm_destroy.argtypes = [vp]
    lib.lbm_last_error.argtypes = [vp]
    lib.lbm_last_error.restype = C.c_char_p
    lib.lbm_batch_table_bytes.argtypes = [C.c_int32, C.POINTER(C.c_size_t)]
    lib.lbm_batch_create.argtypes = [vp, C.c_size_t, vp, C.POINTER(vp)]
    lib.lbm_batch_step.argtypes = [vp, C.POINTER(vp), C.POINTER(C.c_int64), C.c_int32]
    lib.lbm_batch_destroy.argtypes = [vp]
    lib.lbm_batch_last_error.argtypes = [vp]
    lib.lbm_batch_last_error.restype = C.c_char_p
    lib.lbm_hbm_probe.argtypes = [C.c_int32, vp, vp, C.c_size_t, C.c_int32, vp, dp]
    for name in EXPORTED:
        if name not in ("lbm_last_error", "lbm_batch_last_error"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def lattice(lat: int) -> np.ndarray:
    """Velocities [Q][3] in the library's direction order."""
    lib = load_library()
    c = (C.c_int32 * 57)()
    q = C.c_int32()
    rc = lib.lbm_lattice(int(lat), c, C.byref(q))
    if rc != OK:
        raise LbmError(rc, "bad lattice")
    return np.array(c[: 3 * q.value], dtype=np.int64).reshape(q.value, 3)


def make_params(wl: W.Workload, options: int = 0) -> lbm_params:
    p = lbm_params()
    p.options = (int(options) | (OPT_FLUID_PROBE if getattr(wl, "probe", 0) else 0)
                 | (OPT_FILL_DEAD_ENDS if getattr(wl, "fill", 0) else 0))
    p.abi_version = ABI_VERSION
    p.lattice = int(wl.lattice)
    p.precision = int(wl.precision)
    p.ghost_rule = int(wl.ghost_rule)
    for a in range(3):
        p.n[a] = int(wl.shape[a])
        p.body_accel[a] = float(wl.g[a])
    p.rho_l, p.rho_g, p.mu_l, p.mu_g = wl.rho_l, wl.rho_g, wl.mu_l, wl.mu_g
    p.sigma, p.W, p.mobility = wl.sigma, wl.W, wl.mobility
    return p


def make_solids(solids: Sequence[W.Solid]):
    arr = (lbm_solid * max(len(solids), 1))()
    for k, s in enumerate(solids):
        arr[k].kind = int(s.kind)
        for a in range(3):
            arr[k].center[a] = float(s.center[a])
            arr[k].normal[a] = float(s.normal[a])
        arr[k].radius = float(s.radius)
    return arr


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Simulation:
    """One run of the library on a CUDA (HIP) device: create -> set_geometry
    -> bind (torch buffer + current stream) -> set_wetting -> set_field(PHI)."""

    def __init__(self, wl: W.Workload, phi_init: Optional[np.ndarray] = None, device: str = "cuda:0",
                 stream=None, options: int = 0):
        import torch

        lib = load_library()
        self.lib = lib
        self.wl = wl
        self.n = wl.nodes
        self.Q = W.n_directions(wl.lattice)
        h = C.c_void_p()
        params = make_params(wl, options)
        rc = lib.lbm_create(C.byref(params), C.byref(h))
        if rc != OK:
            raise LbmError(rc, lib.lbm_last_error(None).decode())
        self._h = h
        self._check(lib.lbm_set_geometry(h, make_solids(wl.solids), len(wl.solids)))
        nbytes = C.c_size_t()
        self._check(lib.lbm_device_bytes(h, C.byref(nbytes)))
        self.device_bytes = nbytes.value
        self.device = torch.device(device)
        self.buffer = torch.empty(self.device_bytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self.buffer.data_ptr()
        aligned = (ptr + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._streams = [self.stream]   # streams that may still run work on this run (batches add theirs)
        self._check(lib.lbm_bind(h, C.c_void_p(aligned), self.device_bytes, C.c_void_p(self.stream.cuda_stream)))
        self._check(lib.lbm_set_wetting(h, float(wl.theta)))
        if phi_init is None:
            phi_init = W.initial_phi(wl)
        self.set_field(FIELD_PHI, phi_init)

    def _check(self, rc: int):
        if rc != OK:
            raise LbmError(rc, self.lib.lbm_last_error(self._h).decode())

    def close(self):
        """Wait for the run's queued work, destroy the context and release
        the device buffer (the caching allocator tracks only the stream the
        buffer was allocated on, not the run's)."""
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            for stream in getattr(self, "_streams", []):
                stream.synchronize()
            self.lib.lbm_destroy(h)
            self._h = None
            self.buffer = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_wetting(self, theta: float):
        self._check(self.lib.lbm_set_wetting(self._h, float(theta)))

    def set_field(self, field: int, values: np.ndarray):
        v = np.ascontiguousarray(values, dtype=np.float64).reshape(-1)
        self._check(self.lib.lbm_set_field(self._h, int(field), _dp(v), v.size))

    def step(self, nsteps: int = 1):
        self._check(self.lib.lbm_step(self._h, int(nsteps)))

    def step_profiled(self, nsteps: int) -> Dict[str, float]:
        """Step with per-launch HIP events; returns summed ms per phase
        (colour field, ghost update, collide, colour fix-up) and in all."""
        ms = np.zeros(5)
        self._check(self.lib.lbm_step_profiled(self._h, int(nsteps), _dp(ms)))
        return {"colour": ms[0], "ghost": ms[1], "collide": ms[2], "fixup": ms[3], "total": ms[4]}

    def read(self, field: int) -> np.ndarray:
        size = {FIELD_N: self.Q * self.n, FIELD_N_OFFSET: self.Q * self.n, FIELD_B: self.Q * self.n,
                FIELD_U: 3 * self.n}.get(field, self.n)
        out = np.zeros(size, dtype=np.float64)
        self._check(self.lib.lbm_read_field(self._h, int(field), _dp(out), size))
        if field in (FIELD_N, FIELD_N_OFFSET, FIELD_B):
            return out.reshape(self.Q, self.n)
        if field == FIELD_U:
            return out.reshape(3, self.n)
        return out

    def observe(self, allow_unstable: bool = False, static_scratch: bool = False) -> Dict[str, object]:
        """Diagnostics (lbm_observe); with static_scratch, through
        lbm_observe_static, whose reduction scratch is the library's own
        static device array (no caller-provided workspace)."""
        o = lbm_obs()
        fn = self.lib.lbm_observe_static if static_scratch else self.lib.lbm_observe
        rc = fn(self._h, C.byref(o))
        if rc != OK and not (allow_unstable and rc == EUNSTABLE):
            self._check(rc)
        return {"step": o.step, "n_fluid": o.n_fluid, "n_solid": o.n_solid, "n_ghost": o.n_ghost,
                "nonfinite": o.nonfinite, "mass_blue": o.mass_blue, "mass_red": o.mass_red,
                "momentum": [o.momentum[0], o.momentum[1], o.momentum[2]], "max_speed": o.max_speed,
                "kinetic_energy": o.kinetic_energy, "rc": rc}


class Batch:
    """Shared-launch stepping of many Simulations (lbm_batch_*).  The job
    table is a torch device buffer; launches go to `stream` (default: the
    current stream), which every member Simulation must also use."""

    def __init__(self, max_jobs: int = 512, device: str = "cuda:0", stream=None):
        import torch

        lib = load_library()
        self.lib = lib
        nbytes = C.c_size_t()
        rc = lib.lbm_batch_table_bytes(int(max_jobs), C.byref(nbytes))
        if rc != OK:
            raise LbmError(rc, "bad max_jobs")
        self.table = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=torch.device(device))
        aligned = (self.table.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
        h = C.c_void_p()
        rc = lib.lbm_batch_create(C.c_void_p(aligned), nbytes.value, C.c_void_p(self.stream.cuda_stream), C.byref(h))
        if rc != OK:
            raise LbmError(rc, lib.lbm_batch_last_error(None).decode())
        self._h = h

    def step(self, sims: Sequence["Simulation"], steps: Sequence[int]):
        n = len(sims)
        for s in sims:
            if all(t is not self.stream for t in s._streams):
                s._streams.append(self.stream)
        arr = (C.c_void_p * max(n, 1))(*[s._h for s in sims])
        st = (C.c_int64 * max(n, 1))(*[int(k) for k in steps])
        rc = self.lib.lbm_batch_step(self._h, arr, st, n)
        if rc != OK:
            raise LbmError(rc, self.lib.lbm_batch_last_error(self._h).decode())

    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self.stream.synchronize()   # the job table is read by queued launches
            self.lib.lbm_batch_destroy(h)
            self._h = None
            self.table = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PROBE_READ, PROBE_COPY, PROBE_PLANES = 0, 1, 2


def hbm_probe(kind: int, src, dst, repeats: int = 10) -> float:
    """Average milliseconds per launch of one HBM reference kernel
    (lbm_hbm_probe) over `src` (all of it) into `dst`, both torch device
    tensors, on torch's current stream."""
    import torch

    lib = load_library()
    ms = np.zeros(1)
    stream = torch.cuda.current_stream(src.device)
    nbytes = src.numel() * src.element_size()
    rc = lib.lbm_hbm_probe(int(kind), C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes,
                           int(repeats), C.c_void_p(stream.cuda_stream), _dp(ms))
    if rc != OK:
        raise LbmError(rc, "lbm_hbm_probe failed")
    return float(ms[0])
