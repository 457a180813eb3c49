"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle on
the same seeded inputs.  FP64 runs must match normwise to 1e-12 in every
population array (N, B) and in phi; FP32 runs are checked against the FP64
oracle with a tolerance derived from single-precision rounding."""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_2605_30878_amd import workloads as W

from helpers import compare, direction_map, fields_lib, fields_orc, rel_linf

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


def _lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_30878_amd import lbm

    lbm.load_library()
    return lbm


def _log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run_pair(wl, checkpoints, tol, keys=("N", "B", "phi", "u", "p"), options=0):
    lbm = _lbm()
    phi0 = W.initial_phi(wl)
    _log(f"[parity] {wl.name} shape={wl.shape} prec={wl.precision} theta={wl.theta} steps={checkpoints}")
    sim = lbm.Simulation(wl, phi0, options=options)
    osim = oracle.OracleSim(wl, phi0)
    perm = direction_map(wl.lattice)
    done = 0
    worst = {}
    for t in checkpoints:
        sim.step(t - done)
        osim.step(t - done)
        done = t
        errs = compare(fields_lib(sim, with_b="B" in keys), fields_orc(osim, perm), keys)
        _log(f"  step {t}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
        for k, v in errs.items():
            worst[k] = max(worst.get(k, 0.0), v)
            assert v <= tol[k] if isinstance(tol, dict) else v <= tol, (t, k, v)
    ob = sim.observe()
    oo = osim.observe()
    mtol = 1e-9 if wl.precision == W.FP64 else 1e-5
    assert abs(ob["mass_blue"] - oo["mass_blue"]) <= mtol * max(1.0, abs(oo["mass_blue"]))
    sim.close()
    return worst


def test_cylinder_d2q9_fp64_parity():
    """The D2Q9 drop on a cylinder (128^2, theta 90, 2000 steps)."""
    _run_pair(W.cylinder_d2q9_128(), [1, 10, 100, 2000], TOL64)


@pytest.mark.parametrize("theta", [30.0, 150.0])
def test_cylinder_d2q9_fp64_parity_angles(theta):
    _run_pair(W.cylinder_d2q9_128(theta=theta), [1, 50, 500], TOL64)


def test_sphere_d3q19_fp64_parity_ragged():
    """D3Q19 with density ratio 1000 and viscosity ratio 100 (exercises the
    pressure and viscous correction forces) on a box whose x extent is not a
    multiple of the 64-wide thread rows."""
    wl = W.Workload(name="d3q19_ragged", lattice=W.D3Q19, shape=(45, 38, 33), rho_l=1000.0, rho_g=1.0,
                    mu_l=10.0, mu_g=0.1, sigma=0.01, W=4.0, theta=60.0,
                    solids=[W.Solid(0, (22.0, 19.0, 12.0), 8.5)],
                    liquid=[W.LiquidRegion("ball", (22.0, 19.0, 21.0), 8.0, width=4.0)])
    _run_pair(wl, [1, 20, 200], TOL64)


@pytest.mark.parametrize("case", ["xcd_bands", "plain_order"])
def test_sphere_d3q19_fp64_parity_tiled_colour(case):
    """Boxes taken by the z-marching colour kernel (x a multiple of 64, y of
    8), density ratio 1000: 64 x 64 x 20 deals the tiles to the XCDs in
    y-bands, 128 x 16 x 18 in plain order with a ragged last z-chunk.  (Both
    are well conditioned: perturbing the oracle's initial field by 1e-15
    stays at 1e-15 over 200 steps.  A box whose drop nearly meets its own
    periodic image amplifies 1e-15 to 1e-3 in 25 steps in the oracle itself
    and cannot be compared at 1e-12.)"""
    if case == "xcd_bands":
        shape, sc, rs, lc, rl = (64, 64, 20), (30.0, 31.0, 3.0), 6.5, (30.0, 31.0, 8.0), 6.0
    else:
        shape, sc, rs, lc, rl = (128, 16, 18), (62.0, 7.0, 4.0), 5.0, (62.0, 7.0, 9.5), 4.5
    wl = W.Workload(name="d3q19_tile", lattice=W.D3Q19, shape=shape, rho_l=1000.0, rho_g=1.0,
                    mu_l=10.0, mu_g=0.1, sigma=0.01, W=4.0, theta=60.0,
                    solids=[W.Solid(0, sc, rs)], liquid=[W.LiquidRegion("ball", lc, rl, width=4.0)])
    _run_pair(wl, [1, 2, 25, 200], TOL64)


def _cc_sphere(shape, sc, rs, lc, rl, theta):
    return W.Workload(name="d3q19_cc", lattice=W.D3Q19, shape=shape, rho_l=1000.0, rho_g=1.0, mu_l=10.0,
                      mu_g=0.1, sigma=0.01, W=4.0, theta=theta, solids=[W.Solid(0, sc, rs)],
                      liquid=[W.LiquidRegion("ball", lc, rl, width=4.0)])


def _cc_channel(shape, lc, rl, theta):
    """A drop on the lower of two flat walls (solid rows y = 0 and y = ny - 1)."""
    return W.Workload(name="d3q19_cc_wall", lattice=W.D3Q19, shape=shape, rho_l=1000.0, rho_g=1.0, mu_l=10.0,
                      mu_g=0.1, sigma=0.01, W=4.0, theta=theta,
                      solids=[W.Solid(1, (0.0, 0.5, 0.0), normal=(0.0, 1.0, 0.0)),
                              W.Solid(1, (0.0, shape[1] - 1.5, 0.0), normal=(0.0, -1.0, 0.0))],
                      liquid=[W.LiquidRegion("ball", lc, rl, width=4.0)])


# collide-colour parity boxes: (workload, compared steps).  Boxes thinner
# than a ball's diameter take a drop on a flat wall; those are compared up
# to step 25, while a 1e-15 perturbation of the oracle's initial field
# stays below 1e-14 (by step 200 it grows: see below).
CC_BOXES = {
    # one tile column across x, a short last z-chunk
    "one_column": (lambda: _cc_sphere((64, 32, 22), (30.0, 15.0, 6.0), 6.0, (30.0, 15.0, 12.5), 5.5, 120.0),
                   [1, 2, 25, 200]),
    # two tile columns each way
    "several_columns": (lambda: _cc_sphere((128, 16, 18), (62.0, 7.0, 4.0), 5.0, (62.0, 7.0, 9.5), 4.5, 120.0),
                        [1, 2, 25, 200]),
    # one 64 x 8 tile: its own x and y neighbour; z-chunks of 4, 4 and 1 planes
    "own_neighbour_tile": (lambda: _cc_sphere((64, 8, 9), (30.0, 3.5, 2.0), 2.5, (30.0, 3.5, 5.5), 2.5, 60.0),
                           [1, 2, 25, 200]),
    # a last z-chunk of one plane
    "one_plane_last_chunk": (lambda: _cc_channel((64, 16, 5), (30.0, 3.0, 2.0), 4.0, 120.0), [1, 2, 25]),
    # boxes thinner than a chunk: one chunk of 3, 2 or 1 planes, whose c_z
    # crossings wrap to itself
    "three_planes": (lambda: _cc_channel((64, 16, 3), (30.0, 3.0, 1.0), 4.0, 90.0), [1, 2, 25]),
    "two_planes": (lambda: _cc_channel((64, 16, 2), (30.0, 3.0, 0.5), 4.0, 120.0), [1, 2, 25]),
    "one_plane": (lambda: _cc_channel((64, 16, 1), (30.0, 3.0, 0.0), 4.0, 60.0), [1, 2, 25]),
}


@pytest.mark.parametrize("case", list(CC_BOXES))
def test_sphere_d3q19_fp64_parity_collide_colour(case):
    """Boxes stepped in the collide-colour form (LBM_OPT_FUSED: the collide
    kernel also forms the next step's colour field; values crossing a
    64 x 8 column or z-chunk face go through the inbox and the fix-up),
    density ratio 1000, including the degenerate tilings (a tile that is its
    own neighbour, one-plane chunks, boxes thinner than a chunk).  The runs
    keep no liquid populations, so N, phi, u and p are compared.  Every box
    is well conditioned over the compared steps: a 1e-15 perturbation of
    the oracle's initial field stays below 3e-15 in phi over 200 steps in
    the sphere boxes and below 1e-14 over 50 steps in the wall boxes (the
    interface normal switches off below |grad phi| = 1e-12 (reading R-n), so
    phi of order 1e-12 far from the drop is not a smooth function of the
    state, and some boxes amplify such differences later: with the first
    box's drop 0.5 nodes lower, 6e-14 by step 200)."""
    make, steps = CC_BOXES[case]
    wl = make()
    _run_pair(wl, steps, TOL64, keys=("N", "phi", "u", "p"), options=1)


@pytest.mark.parametrize("prec", [W.FP32, W.FP16_OFS], ids=["f32", "fp16ofs"])
def test_collide_colour_and_two_pass_steps_agree(prec):
    """The collide-colour form and the two-pass form (colour kernel, ghost
    update, collide-stream kernel) compute the same update.  After one step
    from the same state N is identical bit for bit and so is phi at every
    fluid node whose streamed-in populations all come from its own 64 x 8
    column and z-chunk (the two-pass colour kernel's sum in the same order);
    at the other fluid nodes the in-column and inbox parts are summed
    separately, and at ghost nodes phi is interpolated from such nodes, so
    phi agrees there to a few units in the last place.  After 100 steps both runs
    agree to single-precision rounding (64^3 drop on a sphere)."""
    lbm = _lbm()
    wl = W.sphere_d3q19(64, theta=60.0, precision=prec)
    phi0 = W.initial_phi(wl)
    a = lbm.Simulation(wl, phi0, options=lbm.OPT_FUSED)
    b = lbm.Simulation(wl, phi0)
    a.step(1)
    b.step(1)
    assert np.array_equal(a.read(lbm.FIELD_N_OFFSET), b.read(lbm.FIELD_N_OFFSET))
    pa, pb = a.read(lbm.FIELD_PHI), b.read(lbm.FIELD_PHI)
    n = wl.shape[0]
    z, y, x = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    zc = 4   # the z-chunk of a 64^3 box (one 64 x 8 column across x, 8 along y)
    edge = ((x % 64 == 0) | (x % 64 == 63) | (y % 8 == 0) | (y % 8 == 7) | (z % zc == 0) |
            (z % zc == zc - 1)).reshape(-1)
    # ghost nodes take phi from interpolated fluid values, which may be edge nodes
    inner = ~edge & ((a.read(lbm.FIELD_FLAGS).astype(np.int64) & lbm.FLAG_SOLID) == 0)
    _log(f"[collide-colour] inner fluid nodes differing: {int(np.sum(pa[inner] != pb[inner]))}; "
         f"max diff elsewhere {float(np.max(np.abs(pa - pb)[~inner])):.2e}")
    assert np.array_equal(pa[inner], pb[inner])
    assert np.max(np.abs(pa - pb)) <= 8 * np.finfo(np.float32).eps
    a.step(99)
    b.step(99)
    for f in (lbm.FIELD_N, lbm.FIELD_PHI):
        err = rel_linf(a.read(f), b.read(f))
        _log(f"[collide-colour vs two-pass] {W.PRECISION_NAMES[prec]} field {f}: {err:.2e}")
        assert err < (2e-6 if prec == W.FP32 else 2e-4)
    with pytest.raises(lbm.LbmError) as e:
        a.read(lbm.FIELD_B)
    assert e.value.code == lbm.ESTATE
    a.close()
    b.close()


def test_plate_d2q9_fp64_parity_walls_density_ratio():
    """Flat walls (half-space solids), density ratio 10, body force."""
    wl = W.plate_d2q9(70, 36, 120.0, 12.0, rho_ratio=10.0, mu_ratio=10.0).with_(g=(1e-7, -2e-7, 0.0))
    _run_pair(wl, [1, 30, 300], TOL64)


@pytest.mark.parametrize("theta", [60.0, 90.0])
def test_fakhari_rule_fp64_parity(theta):
    """Eq. 10 as the ghost rule (90 deg hits its removable singularity)."""
    wl = W.cylinder_d2q9_128(theta=theta).with_(ghost_rule=1)
    _run_pair(wl, [1, 100, 400], TOL64)


@pytest.mark.parametrize("theta", [0.0, 180.0])
def test_extreme_angles_fp64(theta):
    wl = W.Workload(name="extreme", lattice=W.D2Q9, shape=(50, 44, 1), rho_l=1.0, rho_g=1.0, mu_l=0.1,
                    mu_g=0.1, W=4.0, theta=theta, solids=[W.Solid(0, (25.0, 15.0, 0.0), 9.0)],
                    liquid=[W.LiquidRegion("ball", (25.0, 26.0, 0.0), 8.0, width=4.0)])
    _run_pair(wl, [1, 200], TOL64)


def test_no_solid_and_degenerate_boxes_fp64():
    """No solid at all (empty ghost list), and boxes one node thick."""
    _run_pair(W.free_drop(W.D2Q9, 40, 9.0, rho_ratio=3.0), [1, 100], TOL64)
    thin = W.Workload(name="thin", lattice=W.D2Q9, shape=(1, 40, 1), rho_l=1.0, rho_g=1.0, mu_l=0.1,
                      mu_g=0.1, W=4.0, theta=60.0,
                      solids=[W.Solid(1, (0.0, 0.5, 0.0), normal=(0.0, 1.0, 0.0))],
                      liquid=[W.LiquidRegion("below", axis=1, lo=20.0, width=4.0)])
    _run_pair(thin, [1, 50], TOL64)
    thin3 = W.Workload(name="thin3", lattice=W.D3Q19, shape=(70, 1, 9), rho_l=1.0, rho_g=1.0, mu_l=0.1,
                       mu_g=0.1, W=4.0, theta=45.0,
                       solids=[W.Solid(1, (0.0, 0.0, 1.5), normal=(0.3, 0.0, -1.0))],
                       liquid=[W.LiquidRegion("slab", axis=0, lo=35.0, hi=60.0, width=4.0)])
    _run_pair(thin3, [1, 50], TOL64)


def test_porous_packing_fp64_parity():
    """A seeded packing of non-overlapping spheres (solid fraction 0.6, many
    ghosts, spheres across the periodic edges), wetting liquid in a slab,
    density ratio 10, body force along x."""
    wl = W.porous_d3q19(n=40, sphere_radius=5.0, porosity=0.40, seed=0, precision=W.FP64, front=10.0, probe=0,
                        fill=0)
    wl = wl.with_(g=(1e-5, 0.0, 0.0))
    _run_pair(wl, [1, 30], TOL64)


@pytest.mark.parametrize("seed", [0, 1])
def test_porous_fluid_probe_fp64_parity(seed):
    """The same packing in the porous workload's setting: fluid-only probe
    interpolation (with the fluid-neighbour fallback for probes wholly in
    solid) and dead-end nodes filled.  The library's solid set equals the
    oracle's; 300 steps against the oracle."""
    wl = W.porous_d3q19(n=40, sphere_radius=5.0, porosity=0.40, seed=seed, precision=W.FP64, front=10.0)
    assert wl.probe == 1 and wl.fill == 1
    wl = wl.with_(g=(1e-5, 0.0, 0.0))
    lbm = _lbm()
    sim = lbm.Simulation(wl, W.initial_phi(wl))
    solid = (sim.read(lbm.FIELD_FLAGS).astype(np.int64) & lbm.FLAG_SOLID) > 0
    sim.close()
    osim = oracle.OracleSim(wl, W.initial_phi(wl))
    assert np.array_equal(solid, osim.get(oracle.F_SOLID) > 0.5)
    plain = oracle.OracleSim(wl.with_(fill=0), W.initial_phi(wl))
    assert (osim.get(oracle.F_SOLID) > plain.get(oracle.F_SOLID)).sum() > 0   # the fill is exercised
    del osim, plain
    _run_pair(wl, [1, 30, 300], TOL64)


@pytest.mark.parametrize("theta", [30.0, 150.0])
def test_cylinder_fluid_probe_fp64_parity(theta):
    _run_pair(W.cylinder_d2q9_128(theta=theta).with_(probe=1), [1, 50, 500], TOL64)


def test_sphere_d3q19_fp32_short_against_oracle():
    """FP32 storage and arithmetic against the FP64 oracle over 50 steps at
    density ratio 1000: single-precision rounding only (normwise 1e-5)."""
    wl = W.sphere_d3q19(32, theta=60.0, precision=W.FP32)
    _run_pair(wl, [1, 50], {"N": 1e-5, "B": 1e-5, "phi": 1e-5, "u": 1e-5, "p": 1e-5, "solid_phi": 1e-5})


@pytest.mark.parametrize("prec,tol", [(W.FP16_OFS, 2e-5), (W.BF16_OFS, 2e-4)], ids=["fp16ofs", "bf16ofs"])
def test_sphere_d3q19_16bit_short_against_oracle(prec, tol):
    """Populations stored as 16-bit offsets from the rest state (FP32
    arithmetic) against the FP64 oracle over 50 steps."""
    wl = W.sphere_d3q19(32, theta=60.0, precision=prec)
    _run_pair(wl, [1, 50], {k: tol for k in ("N", "B", "phi", "u", "p", "solid_phi")})


@pytest.mark.parametrize("prec", [W.FP32, W.FP16_OFS, W.BF16_OFS], ids=["f32", "fp16ofs", "bf16ofs"])
def test_reduced_precision_colour_mass(prec):
    """The stored zeroth moment closes to 1 at every node, so the colour
    mass of the reduced-precision runs only drifts by unbiased rounding."""
    lbm = _lbm()
    wl = W.sphere_d3q19(48, theta=45.0, precision=prec)
    sim = lbm.Simulation(wl, W.initial_phi(wl))
    m0 = sim.observe()["mass_blue"]
    sim.step(500)
    o = sim.observe()
    _log(f"[mass] prec={prec} drift={o['mass_blue'] / m0 - 1:.3e}")
    assert o["nonfinite"] == 0
    assert abs(o["mass_blue"] / m0 - 1) < (1e-6 if prec == W.FP32 else 2e-5)


def test_observe_and_mass():
    lbm = _lbm()
    wl = W.cylinder_d2q9_128()
    phi0 = W.initial_phi(wl)
    sim = lbm.Simulation(wl, phi0)
    osim = oracle.OracleSim(wl, phi0)
    o0 = sim.observe()
    sim.step(300)
    osim.step(300)
    o1 = sim.observe()
    oo = osim.observe()
    assert o1["step"] == 300 and o1["nonfinite"] == 0
    assert o1["n_ghost"] == 188 and o1["n_solid"] == 1793
    assert abs(o1["mass_blue"] / o0["mass_blue"] - 1) < 1e-13
    for k in ("mass_blue", "mass_red", "kinetic_energy", "max_speed"):
        assert abs(o1[k] - oo[k]) <= 1e-10 * abs(oo[k]), k
    # momentum is a signed sum that cancels to ~1e-15 in x by symmetry:
    # compare against sum rho |u| <= n_fluid max|u|
    scale = o1["n_fluid"] * oo["max_speed"]
    for a in range(3):
        assert abs(o1["momentum"][a] - oo["momentum"][a]) <= 1e-12 * scale


@pytest.mark.parametrize("prec,n", [(W.FP64, 32), (W.FP32, 32), (W.FP16_OFS, 32), (W.FP32, 64), (W.FP16_OFS, 64)],
                         ids=["f64", "f32", "fp16ofs", "f32_tiled", "fp16ofs_tiled"])
def test_restore_roundtrip_is_bitwise(prec, n):
    """Raw state (populations as stored offsets, liquid populations, solid
    phi) read out and written into a fresh context continues bit-identically
    (checkpoint / resume).  At 64^3 the colour field is formed by the tiled
    colour kernel (z-marching 64 x 8 columns), below by the row kernel."""
    lbm = _lbm()
    wl = W.sphere_d3q19(n, theta=120.0, precision=prec)
    phi0 = W.initial_phi(wl)
    a = lbm.Simulation(wl, phi0)
    a.step(25)
    N, B, S = a.read(lbm.FIELD_N_OFFSET), a.read(lbm.FIELD_B), a.read(lbm.FIELD_SOLID_PHI)
    b = lbm.Simulation(wl, phi0)
    b.set_field(lbm.FIELD_N_OFFSET, N)
    b.set_field(lbm.FIELD_B, B)
    b.set_field(lbm.FIELD_SOLID_PHI, S)
    assert np.array_equal(a.read(lbm.FIELD_N_OFFSET), b.read(lbm.FIELD_N_OFFSET))
    a.step(10)
    b.step(10)
    assert np.array_equal(a.read(lbm.FIELD_N_OFFSET), b.read(lbm.FIELD_N_OFFSET))
    assert np.array_equal(a.read(lbm.FIELD_B), b.read(lbm.FIELD_B))
    # the absolute populations are a per-direction constant (chi_i, summing
    # to 1) plus the offsets
    fluid = (a.read(lbm.FIELD_FLAGS).astype(int) & lbm.FLAG_SOLID) == 0
    d = a.read(lbm.FIELD_N)[:, fluid] - a.read(lbm.FIELD_N_OFFSET)[:, fluid]
    assert float(np.max(d.max(axis=1) - d.min(axis=1))) <= 1e-15
    assert abs(float(d[:, 0].sum()) - 1.0) <= 1e-6


@pytest.mark.parametrize("prec", [W.FP32, W.FP16_OFS], ids=["f32", "fp16ofs"])
def test_collide_colour_restore_roundtrip_is_bitwise(prec):
    """A run in the collide-colour form keeps N and phi: N offsets, the
    colour field (LBM_FIELD_PHI_STATE) and solid phi read out and written
    into a fresh context continue bit-identically."""
    lbm = _lbm()
    wl = W.sphere_d3q19(64, theta=120.0, precision=prec)
    phi0 = W.initial_phi(wl)
    a = lbm.Simulation(wl, phi0, options=lbm.OPT_FUSED)
    a.step(25)
    N, P, S = a.read(lbm.FIELD_N_OFFSET), a.read(lbm.FIELD_PHI_STATE), a.read(lbm.FIELD_SOLID_PHI)
    b = lbm.Simulation(wl, phi0, options=lbm.OPT_FUSED)
    b.set_field(lbm.FIELD_N_OFFSET, N)
    b.set_field(lbm.FIELD_SOLID_PHI, S)
    b.set_field(lbm.FIELD_PHI_STATE, P)
    a.step(10)
    b.step(10)
    for f in (lbm.FIELD_N_OFFSET, lbm.FIELD_PHI, lbm.FIELD_SOLID_PHI):
        assert np.array_equal(a.read(f), b.read(f)), f
    a.close()
    b.close()


def test_nonfinite_is_reported():
    lbm = _lbm()
    wl = W.cylinder_d2q9_128()
    sim = lbm.Simulation(wl, W.initial_phi(wl))
    N = sim.read(lbm.FIELD_N)
    fluid = np.flatnonzero(~((sim.read(lbm.FIELD_FLAGS).astype(int) & 1) > 0))
    N[3, fluid[100]] = np.nan
    sim.set_field(lbm.FIELD_N, N)
    o = sim.observe(allow_unstable=True)
    assert o["rc"] == lbm.EUNSTABLE and o["nonfinite"] >= 1


def test_runtime_argument_errors():
    lbm = _lbm()
    wl = W.cylinder_d2q9_128()
    sim = lbm.Simulation(wl, W.initial_phi(wl))
    with pytest.raises(lbm.LbmError) as e:
        sim.set_wetting(181.0)
    assert e.value.code == lbm.EINVAL
    with pytest.raises(lbm.LbmError):
        sim.step(-1)
    with pytest.raises(lbm.LbmError):
        sim.set_field(lbm.FIELD_PHI, np.zeros(7))
    bad = np.full(wl.nodes, np.nan)
    with pytest.raises(lbm.LbmError):
        sim.set_field(lbm.FIELD_PHI, bad)


@pytest.mark.parametrize("case", ["d2q9_f64", "d3q19_f32", "packing_sparse_f32", "d3q19_f32_collide_colour"])
def test_step_graph_replays_equal_direct_launches(case):
    """With LBM_OPT_GRAPH lbm_step replays a captured two-step HIP graph for
    long runs: every replay, with eager single steps, reads and
    synchronisations in between, matches the same run launched kernel by
    kernel, bit for bit; a wetting change drops the graph and takes effect.
    Also in the fluid-only layout and in the collide-colour form (whose
    inbox the graph's fix-up launches read)."""
    lbm = _lbm()
    extra = 0
    if case == "d2q9_f64":
        wl = W.cylinder_d2q9_128(theta=30.0)
    elif case == "d3q19_f32":
        wl = W.sphere_d3q19(32, theta=60.0, precision=W.FP32)
    elif case == "d3q19_f32_collide_colour":
        wl = W.sphere_d3q19(64, theta=60.0, precision=W.FP32)
        extra = lbm.OPT_FUSED
    else:
        wl = W.porous_d3q19(n=40, sphere_radius=5.0, porosity=0.40, seed=0, precision=W.FP32, front=10.0)
        extra = lbm.OPT_SPARSE
    phi0 = W.initial_phi(wl)
    a = lbm.Simulation(wl, phi0, options=lbm.OPT_GRAPH | extra)   # graphs
    b = lbm.Simulation(wl, phi0, options=extra)                   # direct launches
    plan = [10, 1, 9, 16, 3, 12]
    for k, n in enumerate(plan):
        if k == 3:
            a.set_wetting(wl.theta + 20.0)
            b.set_wetting(wl.theta + 20.0)
        a.step(n)
        b.step(n)
        assert a.observe()["step"] == b.observe()["step"]
        fields = (lbm.FIELD_N_OFFSET, lbm.FIELD_PHI) if extra == lbm.OPT_FUSED else \
            (lbm.FIELD_N_OFFSET, lbm.FIELD_B, lbm.FIELD_PHI)
        for f in fields:
            assert np.array_equal(a.read(f), b.read(f)), (k, f)
    a.close()
    b.close()


def _packing40(prec, probe=1, fill=1, seed=0):
    wl = W.porous_d3q19(n=40, sphere_radius=5.0, porosity=0.40, seed=seed, precision=prec, front=10.0,
                        probe=probe, fill=fill)
    return wl.with_(g=(1e-5, 0.0, 0.0))


@pytest.mark.parametrize("case", ["porous40", "porous40_all_corners", "cyl128"])
def test_sparse_layout_fp64_parity(case):
    """The fluid-only layout (LBM_OPT_SPARSE: planes over fluid and ghost
    slots, neighbours from a slot table) against the oracle: the packing in
    the porous workload's setting, the packing with all probe corners (probes
    then read the shared slot of the non-ghost solid nodes), and the D2Q9
    cylinder."""
    if case == "porous40":
        _run_pair(_packing40(W.FP64), [1, 30, 300], TOL64, options=32)   # LBM_OPT_SPARSE
    elif case == "porous40_all_corners":
        _run_pair(_packing40(W.FP64, probe=0, fill=0), [1, 30], TOL64, options=32)
    else:
        _run_pair(W.cylinder_d2q9_128(theta=30.0), [1, 50, 500], TOL64, options=32)


@pytest.mark.parametrize("case,prec", [("porous40", W.FP32), ("porous40", W.FP16_OFS), ("free_drop", W.FP32),
                                       ("cyl128", W.BF16_OFS)],
                         ids=["porous40_f32", "porous40_fp16ofs", "no_solid_f32", "d2q9_bf16ofs"])
def test_sparse_layout_equals_box_layout(case, prec):
    """Both layouts call the same per-node functions: N (stored offsets), B,
    phi, solid phi, u and p are identical bit for bit after 1 and 60 steps
    (the diagnostics, summed in another order, agree to rounding), on a
    packing, on a box with no solid (every slot fluid, no ghost) and on the
    D2Q9 cylinder.  A state read from the sparse run restores into a fresh
    sparse run that continues bit-identically."""
    lbm = _lbm()
    if case == "porous40":
        wl = _packing40(prec)
    elif case == "free_drop":
        wl = W.free_drop(W.D3Q19, 24, 7.0, rho_ratio=10.0, precision=prec)
    else:
        wl = W.cylinder_d2q9_128(theta=45.0, precision=prec)
    phi0 = W.initial_phi(wl)
    a = lbm.Simulation(wl, phi0)
    b = lbm.Simulation(wl, phi0, options=lbm.OPT_SPARSE)
    if case == "porous40":
        assert b.device_bytes < a.device_bytes
    fields = [lbm.FIELD_N_OFFSET, lbm.FIELD_B, lbm.FIELD_PHI, lbm.FIELD_SOLID_PHI, lbm.FIELD_U, lbm.FIELD_P]
    for n in (1, 59):
        a.step(n)
        b.step(n)
        for f in fields:
            assert np.array_equal(a.read(f), b.read(f)), (n, f)
        oa, ob = a.observe(), b.observe()
        assert oa["n_fluid"] == ob["n_fluid"] and oa["n_ghost"] == ob["n_ghost"]
        for k in ("mass_blue", "mass_red", "kinetic_energy", "max_speed"):
            assert abs(oa[k] - ob[k]) <= 1e-12 * max(abs(oa[k]), 1e-30), (k, oa[k], ob[k])
    N, B, S = b.read(lbm.FIELD_N_OFFSET), b.read(lbm.FIELD_B), b.read(lbm.FIELD_SOLID_PHI)
    c = lbm.Simulation(wl, phi0, options=lbm.OPT_SPARSE)
    c.set_field(lbm.FIELD_N_OFFSET, N)
    c.set_field(lbm.FIELD_B, B)
    c.set_field(lbm.FIELD_SOLID_PHI, S)
    b.step(10)
    c.step(10)
    for f in fields:
        assert np.array_equal(b.read(f), c.read(f)), f
    # The fluid-only layout stores N post-collision at the source slot (pull
    # streaming): setting an arbitrary post-stream N scatters it, reading it
    # gathers it back, and both layouts then step from the same state.
    a.step(10)   # a to b's step, so that the rest of the state agrees
    rng = np.random.default_rng(7)
    Nr = 1e-3 * rng.standard_normal(N.shape)
    for s in (a, b):
        s.set_field(lbm.FIELD_N_OFFSET, Nr)
    assert np.array_equal(a.read(lbm.FIELD_N_OFFSET), b.read(lbm.FIELD_N_OFFSET))
    a.step(3)
    b.step(3)
    for f in fields:
        assert np.array_equal(a.read(f), b.read(f)), ("set N", f)
    # one value for every non-ghost solid node is all the layout keeps
    flags = b.read(lbm.FIELD_FLAGS).astype(np.int64)
    inner = np.flatnonzero(((flags & lbm.FLAG_SOLID) > 0) & ((flags & lbm.FLAG_GHOST) == 0))
    if len(inner) > 1:
        S2 = S.copy()
        S2[inner[0]] += 0.25
        with pytest.raises(lbm.LbmError):
            c.set_field(lbm.FIELD_SOLID_PHI, S2)
    for s in (a, b, c):
        s.close()
