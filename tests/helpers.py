"""Shared test helpers: run the HIP library and the oracle on the same seeded
workload and compare arrays normwise."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2605_30878_amd import workloads as W


def direction_map(lattice: int) -> np.ndarray:
    """perm[i] = oracle direction index of library direction i."""
    from paper_2605_30878_amd import lbm

    c_lib = lbm.lattice(lattice)
    c_orc = oracle.lattice_tables(lattice)["c"]
    perm = np.zeros(len(c_lib), dtype=np.int64)
    for i, c in enumerate(c_lib):
        m = np.flatnonzero((c_orc == c).all(axis=1))
        assert m.size == 1
        perm[i] = m[0]
    return perm


def rel_linf(a: np.ndarray, b: np.ndarray) -> float:
    """max |a - b| / max |b| (normwise relative L-infinity)."""
    den = float(np.max(np.abs(b)))
    if den == 0.0:
        return float(np.max(np.abs(a)))
    return float(np.max(np.abs(a - b))) / den


def fields_lib(sim, with_b: bool = True):
    """The library's state as FP64 arrays.  with_b=False for runs stepped in
    the collide-colour form, which keep phi and no liquid populations."""
    from paper_2605_30878_amd import lbm

    out = {"N": sim.read(lbm.FIELD_N), "phi": sim.read(lbm.FIELD_PHI), "u": sim.read(lbm.FIELD_U),
           "p": sim.read(lbm.FIELD_P), "solid_phi": sim.read(lbm.FIELD_SOLID_PHI)}
    if with_b:
        out["B"] = sim.read(lbm.FIELD_B)
    return out


def fields_orc(osim, perm):
    solid = osim.get(oracle.F_SOLID) > 0.5
    N = osim.get(oracle.F_N)[perm]
    B = osim.get(oracle.F_B)[perm]
    N[:, solid] = 0.0
    B[:, solid] = 0.0
    return {"N": N, "B": B, "phi": osim.get(oracle.F_PHI), "u": osim.get(oracle.F_U),
            "p": osim.get(oracle.F_P), "solid_phi": osim.get(oracle.F_PHI_STATE), "solid": solid}


def compare(lib_f, orc_f, keys=("N", "B", "phi", "u", "p")):
    """N, B, phi: normwise relative L-infinity.  u and p are sums of
    populations with heavy cancellation (p is ~1e-4 of the populations it is
    formed from), so their error is measured against the population scale
    max |N| of the oracle instead of their own magnitude."""
    solid = orc_f["solid"]
    scale = float(np.max(np.abs(orc_f["N"])))
    out = {}
    for k in keys:
        a, b = lib_f[k], orc_f[k]
        if k in ("u", "p"):
            a = a.copy()
            b = b.copy()
            a[..., solid] = 0.0
            b[..., solid] = 0.0
            out[k] = float(np.max(np.abs(a - b))) / scale
        else:
            out[k] = rel_linf(a, b)
    if "solid_phi" in lib_f:
        out["solid_phi"] = rel_linf(lib_f["solid_phi"][solid], orc_f["solid_phi"][solid]) if solid.any() else 0.0
    return out
