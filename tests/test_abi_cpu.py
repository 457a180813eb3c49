"""The C-ABI library on the host: it loads, exports every symbol include/lbm.h
declares, validates arguments, enforces call order, and its host-side
geometry (node classes) agrees with the oracle's independent one.  No
device calls are made."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
from paper_2605_30878_amd import lbm
from paper_2605_30878_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "lbm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(lbm_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    lib = lbm.load_library()
    names = _declared_symbols()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(names) == sorted(lbm.EXPORTED)


def _create(wl, **override):
    p = lbm.make_params(wl)
    for k, v in override.items():
        setattr(p, k, v)
    h = C.c_void_p()
    rc = lbm.load_library().lbm_create(C.byref(p), C.byref(h))
    return rc, h


@pytest.mark.parametrize("field,value", [("W", 3.9), ("rho_l", 0.0), ("mu_g", -1.0), ("mobility", 0.0),
                                         ("mobility", 0.35), ("lattice", 7), ("precision", 9),
                                         ("ghost_rule", 5), ("abi_version", 99)])
def test_create_rejects_bad_params(field, value):
    rc, h = _create(W.cylinder_d2q9_128(), **{field: value})
    assert rc == lbm.EINVAL
    assert not h.value
    assert lbm.load_library().lbm_last_error(None)


def test_create_rejects_bad_box():
    wl = W.cylinder_d2q9_128()
    p = lbm.make_params(wl)
    p.n[2] = 2  # D2Q9 needs nz = 1
    h = C.c_void_p()
    assert lbm.load_library().lbm_create(C.byref(p), C.byref(h)) == lbm.EINVAL
    p.n[2] = 1
    p.n[0] = 0
    assert lbm.load_library().lbm_create(C.byref(p), C.byref(h)) == lbm.EINVAL
    # one FP32 field plane of more than 4 GiB (2^30 + 2^20 nodes)
    p.precision = W.FP32
    p.n[0], p.n[1] = 1 << 15, (1 << 15) + 32
    assert lbm.load_library().lbm_create(C.byref(p), C.byref(h)) == lbm.EINVAL
    p.n[1] = 1 << 14   # 2^29 nodes: a 2 GiB plane is accepted in FP32 ...
    assert lbm.load_library().lbm_create(C.byref(p), C.byref(h)) == lbm.OK
    assert lbm.load_library().lbm_destroy(h) == lbm.OK
    p.precision = W.FP64   # ... and is a 4 GiB plane in FP64
    assert lbm.load_library().lbm_create(C.byref(p), C.byref(h)) == lbm.EINVAL


def test_call_order_is_enforced():
    lib = lbm.load_library()
    rc, h = _create(W.cylinder_d2q9_128())
    assert rc == lbm.OK
    nbytes = C.c_size_t()
    assert lib.lbm_device_bytes(h, C.byref(nbytes)) == lbm.ESTATE
    assert lib.lbm_step(h, 1) == lbm.ESTATE
    assert lib.lbm_set_wetting(h, 30.0) == lbm.ESTATE
    o = lbm.lbm_obs()
    assert lib.lbm_observe(h, C.byref(o)) == lbm.ESTATE
    wl = W.cylinder_d2q9_128()
    assert lib.lbm_set_geometry(h, lbm.make_solids(wl.solids), len(wl.solids)) == lbm.OK
    assert lib.lbm_set_geometry(h, lbm.make_solids(wl.solids), len(wl.solids)) == lbm.ESTATE
    assert lib.lbm_device_bytes(h, C.byref(nbytes)) == lbm.OK and nbytes.value > 0
    assert lib.lbm_bind(h, None, nbytes.value, None) == lbm.EINVAL
    assert lib.lbm_step(h, 1) == lbm.ESTATE
    buf = np.zeros(9 * wl.nodes)
    ptr = buf.ctypes.data_as(C.POINTER(C.c_double))
    for field in (lbm.FIELD_N, lbm.FIELD_N_OFFSET, lbm.FIELD_B):
        assert lib.lbm_set_field(h, field, ptr, buf.size) == lbm.ESTATE
        assert lib.lbm_read_field(h, field, ptr, buf.size) == lbm.ESTATE
    assert lib.lbm_destroy(h) == lbm.OK


def test_device_bytes_cover_the_state():
    """Two buffers of N (Q planes each), the B plane buffer and two compact
    liquid records (D + 1 planes each), plus the rest."""
    lib = lbm.load_library()
    wl = W.sphere_d3q19(64, precision=W.FP32)
    rc, h = _create(wl)
    assert lib.lbm_set_geometry(h, lbm.make_solids(wl.solids), 1) == lbm.OK
    nbytes = C.c_size_t()
    lib.lbm_device_bytes(h, C.byref(nbytes))
    assert nbytes.value >= (3 * 19 + 2 * 4) * 64 ** 3 * 4
    lib.lbm_destroy(h)


@pytest.mark.parametrize("wl", [
    W.cylinder_d2q9_128(),
    W.sphere_d3q19(64),
    W.plate_d2q9(40, 24, 60.0, 10.0),
    # a disk across the periodic corner and two overlapping primitives
    W.Workload(name="wrap", lattice=W.D2Q9, shape=(37, 29, 1), theta=45.0,
               solids=[W.Solid(0, (1.5, 2.0, 0.0), 7.3), W.Solid(0, (30.0, 20.0, 0.0), 5.0),
                       W.Solid(1, (0.0, 24.5, 0.0), normal=(0.3, -1.0, 0.0))]),
    W.Workload(name="wrap3", lattice=W.D3Q19, shape=(21, 18, 17), theta=45.0,
               solids=[W.Solid(0, (0.0, 17.0, 8.0), 5.5), W.Solid(0, (10.0, 9.0, 8.0), 4.0)]),
    # a packing with its dead-end nodes filled (LBM_OPT_FILL_DEAD_ENDS)
    W.porous_d3q19(n=40, sphere_radius=5.0, porosity=0.40, seed=1, precision=W.FP64, front=10.0),
], ids=["cyl128", "sphere64", "plate", "wrap2d", "wrap3d", "porous40_fill"])
def test_node_classes_match_oracle(wl):
    lib = lbm.load_library()
    rc, h = _create(wl)
    assert rc == lbm.OK
    assert lib.lbm_set_geometry(h, lbm.make_solids(wl.solids), len(wl.solids)) == lbm.OK
    f = np.zeros(wl.nodes)
    assert lib.lbm_read_field(h, lbm.FIELD_FLAGS, f.ctypes.data_as(C.POINTER(C.c_double)), wl.nodes) == lbm.OK
    lib.lbm_destroy(h)
    flags = f.astype(np.int64)
    osim = oracle.OracleSim(wl, W.initial_phi(wl))
    solid = osim.get(oracle.F_SOLID) > 0.5
    assert np.array_equal((flags & lbm.FLAG_SOLID) > 0, solid)
    ids, *_ = osim.ghosts()
    assert np.array_equal(np.flatnonzero(flags & lbm.FLAG_GHOST), ids)
    assert ((flags & lbm.FLAG_NEAR_SOLID) > 0).sum() == osim.info()["n_fluid_boundary"]


def test_lattice_tables():
    c2 = lbm.lattice(W.D2Q9)
    c3 = lbm.lattice(W.D3Q19)
    assert c2.shape == (9, 3) and c3.shape == (19, 3)
    for c in (c2, c3):
        assert len({tuple(v) for v in c}) == len(c)
        assert (c.sum(axis=0) == 0).all()
    assert np.array_equal(c3[:9], c2)


def test_sparse_option_combinations_and_bytes():
    """LBM_OPT_SPARSE excludes the collide-colour form, unused option bits are
    rejected; on a packing
    its device buffer holds one entry per slot (fluid nodes, ghosts and one
    solid slot) plus Q - 1 neighbour slots per fluid node, less than the
    box layout needs."""
    lib = lbm.load_library()
    wl = W.porous_d3q19(n=40, sphere_radius=5.0, porosity=0.40, seed=0, precision=W.FP32, front=10.0)
    for bad in (lbm.OPT_SPARSE | lbm.OPT_FUSED, 4, 1 << 6):   # excluded pair, unused bits
        p = lbm.make_params(wl, bad)
        h = C.c_void_p()
        assert lib.lbm_create(C.byref(p), C.byref(h)) == lbm.EINVAL
    sizes = {}
    for opt in (0, lbm.OPT_SPARSE):
        p = lbm.make_params(wl, opt)
        h = C.c_void_p()
        assert lib.lbm_create(C.byref(p), C.byref(h)) == lbm.OK
        assert lib.lbm_set_geometry(h, lbm.make_solids(wl.solids), len(wl.solids)) == lbm.OK
        nbytes = C.c_size_t()
        assert lib.lbm_device_bytes(h, C.byref(nbytes)) == lbm.OK
        sizes[opt] = nbytes.value
        f = np.zeros(wl.nodes)
        assert lib.lbm_read_field(h, lbm.FIELD_FLAGS, f.ctypes.data_as(C.POINTER(C.c_double)), wl.nodes) == lbm.OK
        lib.lbm_destroy(h)
    flags = f.astype(np.int64)
    nf = int(((flags & lbm.FLAG_SOLID) == 0).sum())
    ng = int(((flags & lbm.FLAG_GHOST) > 0).sum())
    slots = nf + ng + 1
    assert sizes[lbm.OPT_SPARSE] >= (3 * 19 + 2 * 4) * slots * 4 + 18 * nf * 4
    assert sizes[lbm.OPT_SPARSE] < sizes[0]


def _valid(lattice, n, rho_l, rho_g, mu_l, mu_g, sigma, Wd, mob, g, options):
    """The acceptance rules lbm_create documents, restated."""
    import math
    if lattice == W.D2Q9 and n[2] != 1:
        return False
    if min(n) < 1 or n[1] > 65535 or n[2] > 65535:
        return False
    if not (rho_l > 0 and rho_g > 0 and mu_l > 0 and mu_g > 0):
        return False
    if not sigma >= 0 or not Wd >= 4.0 or not mob > 0:
        return False
    if not all(math.isfinite(a) for a in g):
        return False
    if options & 4 or options & ~63:        # bit 2 is unused
        return False
    if options & 32 and options & 1:        # LBM_OPT_SPARSE excludes LBM_OPT_FUSED
        return False
    cs2 = 1.0 / 3.0
    w0 = 4.0 / 9 if lattice == W.D2Q9 else 1.0 / 3
    alpha = 1.0 - 2.0 * mob * (1.0 - w0) / cs2
    if not (alpha >= 0.0 and alpha < 1.0):
        return False
    return (0.5 + (mu_l / rho_l) / cs2 > 0.5) and (0.5 + (mu_g / rho_g) / cs2 > 0.5)


def test_create_accepts_exactly_the_documented_parameters():
    """Seeded random parameter sets, valid and not (zero, negative, NaN and
    infinite values, small and large mobilities, option clashes): lbm_create
    returns OK exactly when the documented rules hold, else LBM_EINVAL with a
    message, and never crashes."""
    lib = lbm.load_library()
    rng = np.random.default_rng(7)
    specials = [0.0, -1.0, float("nan"), float("inf"), 1e-300, 1e300]

    def pick(lo, hi):
        return specials[rng.integers(len(specials))] if rng.uniform() < 0.15 else float(rng.uniform(lo, hi))

    seen = {True: 0, False: 0}
    for _ in range(400):
        lattice = int(rng.integers(2))
        n = [int(rng.integers(0, 40)), int(rng.integers(0, 40)), 1 if lattice == W.D2Q9 else int(rng.integers(0, 40))]
        if lattice == W.D2Q9 and rng.uniform() < 0.1:
            n[2] = 2
        vals = dict(rho_l=pick(0.5, 1000.0), rho_g=pick(0.5, 2.0), mu_l=pick(0.01, 10.0), mu_g=pick(0.01, 1.0),
                    sigma=pick(0.0, 0.1), Wd=pick(3.0, 8.0), mob=pick(0.0, 0.4))
        g = [pick(-1e-5, 1e-5) if rng.uniform() < 0.3 else 0.0 for _ in range(3)]
        options = int(rng.integers(0, 64))
        if rng.uniform() < 0.8:
            options &= ~4          # mostly documented bits; the unused bit 2 now and then
        wl = W.Workload(name="p", lattice=lattice, shape=tuple(max(v, 1) for v in n), rho_l=vals["rho_l"],
                        rho_g=vals["rho_g"], mu_l=vals["mu_l"], mu_g=vals["mu_g"], sigma=vals["sigma"],
                        W=vals["Wd"], mobility=vals["mob"], g=tuple(g))
        p = lbm.make_params(wl, options)
        for a in range(3):
            p.n[a] = n[a]
        h = C.c_void_p()
        rc = lib.lbm_create(C.byref(p), C.byref(h))
        want = _valid(lattice, n, vals["rho_l"], vals["rho_g"], vals["mu_l"], vals["mu_g"], vals["sigma"], vals["Wd"],
                      vals["mob"], g, options)
        assert rc == (lbm.OK if want else lbm.EINVAL), (lattice, n, vals, g, options, rc)
        if rc == lbm.OK:
            assert h.value
            assert lib.lbm_destroy(h) == lbm.OK
        else:
            assert not h.value and lib.lbm_last_error(None)
        seen[want] += 1
    assert seen[True] > 40 and seen[False] > 40


def test_set_geometry_rejects_bad_solids():
    """lbm_set_geometry's documented errors: a negative count or a null list,
    an unknown kind, a ball wider than the box, a negative radius, a zero
    half-space normal; a failed call leaves the context without geometry, so
    a correct call still succeeds afterwards."""
    lib = lbm.load_library()
    wl = W.cylinder_d2q9_128()
    bad = [
        [W.Solid(2, (10.0, 10.0, 0.0), 3.0)],                          # unknown kind
        [W.Solid(0, (64.0, 64.0, 0.0), 64.0)],                         # 2r = 128: not narrower than the box
        [W.Solid(0, (64.0, 64.0, 0.0), -1.0)],                         # negative radius
        [W.Solid(1, (0.0, 10.0, 0.0), normal=(0.0, 0.0, 0.0))],        # zero normal
    ]
    rc, h = _create(wl)
    assert rc == lbm.OK
    assert lib.lbm_set_geometry(h, lbm.make_solids(wl.solids), -1) == lbm.EINVAL
    assert lib.lbm_set_geometry(h, None, 1) == lbm.EINVAL
    for solids in bad:
        assert lib.lbm_set_geometry(h, lbm.make_solids(solids), len(solids)) == lbm.EINVAL, solids
        assert lib.lbm_last_error(h)
    nbytes = C.c_size_t()
    assert lib.lbm_device_bytes(h, C.byref(nbytes)) == lbm.ESTATE
    assert lib.lbm_set_geometry(h, lbm.make_solids(wl.solids), len(wl.solids)) == lbm.OK
    assert lib.lbm_device_bytes(h, C.byref(nbytes)) == lbm.OK
    assert lib.lbm_destroy(h) == lbm.OK


def test_collide_colour_inbox_only_when_the_form_applies():
    """The collide-colour form (LBM_OPT_FUSED) addresses the Q population
    planes from one base with 32-bit offsets, so it steps only boxes tiled by
    64 x 8 whose populations take at most 4 GiB; its inbox is allocated only
    then (other boxes step in the two-pass form)."""
    lib = lbm.load_library()

    def nbytes(shape, options):
        wl = W.Workload(name="box", lattice=W.D3Q19, shape=shape, precision=W.FP32, theta=90.0, solids=[])
        rc, h = _create(wl, options=options)
        assert rc == lbm.OK
        assert lib.lbm_set_geometry(h, lbm.make_solids([]), 0) == lbm.OK
        out = C.c_size_t()
        assert lib.lbm_device_bytes(h, C.byref(out)) == lbm.OK
        lib.lbm_destroy(h)
        return out.value

    # 512 x 512 x 128 FP32: 19 planes of 128 MiB, 2.4 GiB: the form applies
    assert nbytes((512, 512, 128), lbm.OPT_FUSED) > nbytes((512, 512, 128), 0)
    # 512 x 512 x 256: 4.75 GiB of populations: stepped in the two-pass form
    assert nbytes((512, 512, 256), lbm.OPT_FUSED) == nbytes((512, 512, 256), 0)
    # a box not tiled by 64 x 8
    assert nbytes((96, 64, 32), lbm.OPT_FUSED) == nbytes((96, 64, 32), 0)
