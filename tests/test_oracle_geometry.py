"""Oracle geometry: solid set, ghost (solid boundary) nodes, solid normals,
probe points x_F = x_G + n_s and their interpolation weights.  Checked by
brute force in numpy and by the properties the construction must have."""
import numpy as np
import pytest

import oracle
from paper_2605_30878_amd import workloads as W


def _velocities(lattice):
    return oracle.lattice_tables(lattice)["c"]


def _brute_sets(wl):
    nx, ny, nz = wl.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    solid = np.zeros((nz, ny, nx), bool)
    for s in wl.solids:
        if s.kind == 0:
            d2 = (x - s.center[0]) ** 2 + (y - s.center[1]) ** 2
            if wl.lattice == W.D3Q19:
                d2 = d2 + (z - s.center[2]) ** 2
            solid |= d2 <= s.radius ** 2
        else:
            v = (x - s.center[0]) * s.normal[0] + (y - s.center[1]) * s.normal[1]
            if wl.lattice == W.D3Q19:
                v = v + (z - s.center[2]) * s.normal[2]
            solid |= v <= 0
    c = _velocities(wl.lattice)
    fluid_nb = np.zeros_like(solid)
    solid_nb_links = np.zeros(solid.shape, np.int64)
    for ci in c[1:]:
        sh = np.roll(solid, shift=(-ci[2], -ci[1], -ci[0]), axis=(0, 1, 2))  # solid[x + c]
        fluid_nb |= ~sh
        solid_nb_links += sh
    ghost = solid & fluid_nb
    links = int(solid_nb_links[~solid].sum())
    fb = int(((solid_nb_links > 0) & ~solid).sum())
    return solid.reshape(-1), ghost.reshape(-1), links, fb


@pytest.mark.parametrize("wl", [W.cylinder_d2q9_128(), W.sphere_d3q19(64),
                                W.plate_d2q9(40, 24, 60.0, 10.0)],
                         ids=["cyl128", "sphere64", "plate"])
def test_solid_and_ghost_sets_brute_force(wl):
    sim = oracle.OracleSim(wl, W.initial_phi(wl))
    solid, ghost, links, fb = _brute_sets(wl)
    info = sim.info()
    assert info["n_solid"] == solid.sum()
    assert info["n_ghost"] == ghost.sum()
    assert info["n_links"] == links
    assert info["n_fluid_boundary"] == fb
    ids, nrm, corners, weights = sim.ghosts()
    assert np.array_equal(ids, np.flatnonzero(ghost))
    assert np.array_equal(sim.get(oracle.F_SOLID) > 0.5, solid)


def test_config_counts():
    """Counts for the two main boxes (closed-ball solids)."""
    s1 = oracle.OracleSim(W.cylinder_d2q9_128(), W.initial_phi(W.cylinder_d2q9_128()))
    assert s1.info()["n_solid"] == 1793 and s1.info()["n_ghost"] == 188
    assert s1.info()["n_links"] == 464 and s1.info()["n_fluid_boundary"] == 200
    wl = W.sphere_d3q19(64)
    s2 = oracle.OracleSim(wl, W.initial_phi(wl))
    assert s2.info()["n_solid"] == 7153 and s2.info()["n_ghost"] == 2088
    assert s2.info()["n_links"] == 10242


@pytest.mark.parametrize("wl", [W.cylinder_d2q9_128(), W.sphere_d3q19(64)], ids=["cyl128", "sphere64"])
def test_probe_points_and_weights(wl):
    """n_s is the unit outward normal of the ball; the weights are the
    bi/trilinear weights of x_F = x_G + n_s: non-negative, sum 1, and they
    reproduce x_F (linear fields are interpolated exactly)."""
    sim = oracle.OracleSim(wl, W.initial_phi(wl))
    ids, nrm, corners, weights = sim.ghosts()
    nx, ny, nz = wl.shape
    D = 3 if wl.lattice == W.D3Q19 else 2
    xs = np.stack([ids % nx, (ids // nx) % ny, ids // (nx * ny)], axis=1).astype(float)
    c = np.asarray(wl.solids[0].center)
    r = xs - c
    r[:, D:] = 0
    want_n = r / np.linalg.norm(r, axis=1, keepdims=True)
    assert np.allclose(nrm, want_n, atol=1e-15)
    nc = 2 ** D
    assert np.all(weights[:, :nc] >= 0)
    assert np.allclose(weights[:, :nc].sum(axis=1), 1.0, atol=1e-15)
    xf = xs + nrm
    cx = np.stack([corners % nx, (corners // nx) % ny, corners // (nx * ny)], axis=2).astype(float)
    # unwrap corners to the neighbourhood of x_F
    L = np.array([nx, ny, nz], float)
    d = cx - xf[:, None, :]
    cx = cx - L * np.round(d / L)
    interp = (weights[:, :nc, None] * cx[:, :nc, :]).sum(axis=1)
    assert np.allclose(interp[:, :D], xf[:, :D], atol=1e-13)
    # x_F lies within one node spacing of every corner used
    assert np.all(np.abs(cx[:, :nc, :D] - xf[:, None, :D]) < 1.0 + 1e-12)


def test_flat_wall_probe_is_a_node():
    """On a grid-aligned flat wall x_F is the node one spacing into the fluid
    (weight 1): the flat-wall limit of the curved-boundary rule."""
    wl = W.plate_d2q9(40, 24, 60.0, 10.0)
    sim = oracle.OracleSim(wl, W.initial_phi(wl))
    ids, nrm, corners, weights = sim.ghosts()
    nx = wl.shape[0]
    for g in range(len(ids)):
        k = int(np.argmax(weights[g, :4]))
        assert weights[g, k] == 1.0
        y = ids[g] // nx
        want_y = 1 if y == 0 else wl.shape[1] - 2
        assert corners[g, k] == ids[g] % nx + nx * want_y


@pytest.mark.parametrize("wl", [W.cylinder_d2q9_128(), W.sphere_d3q19(64),
                                W.porous_d3q19(n=40, sphere_radius=5.0, precision=W.FP64, front=10.0)],
                         ids=["cyl128", "sphere64", "porous40"])
def test_fluid_only_probe_weights(wl):
    """The fluid-only probe (option): solid corners get weight 0 and the fluid
    corners keep their bi/trilinear weights in proportion, summing to 1; a
    probe whose corners are all fluid is unchanged.  A probe with no fluid
    corner takes the ghost's fluid lattice neighbours (found here by brute
    force), weighted by w_i and rescaled to sum 1, the axis neighbours alone
    when there are more than 2^D."""
    a = oracle.OracleSim(wl.with_(probe=0), W.initial_phi(wl))
    b = oracle.OracleSim(wl.with_(probe=1), W.initial_phi(wl))
    ids_a, _, corners, wa = a.ghosts()
    ids_b, _, corners_b, wb = b.ghosts()
    assert np.array_equal(ids_a, ids_b)
    solid = a.get(oracle.F_SOLID) > 0.5
    nc = 2 ** (3 if wl.lattice == W.D3Q19 else 2)
    cs = solid[corners[:, :nc]]
    wa, wb = wa[:, :nc], wb[:, :nc]
    corners, corners_b = corners[:, :nc], corners_b[:, :nc]
    fluid_w = np.where(cs, 0.0, wa).sum(axis=1)
    has_fluid = fluid_w > 0
    assert np.array_equal(corners[has_fluid], corners_b[has_fluid])
    assert np.allclose(wb.sum(axis=1), 1.0, atol=1e-15)
    assert np.all(wb[has_fluid][cs[has_fluid]] == 0.0)
    ratio = np.where(cs, 0.0, wa)[has_fluid] / fluid_w[has_fluid, None]
    assert np.allclose(wb[has_fluid], ratio, atol=1e-15)
    all_fluid = ~cs.any(axis=1)
    assert np.array_equal(wb[all_fluid], wa[all_fluid])
    # the rescaling is exercised
    assert (has_fluid & ~all_fluid).sum() > 0
    # the fallback, against a brute-force list of fluid neighbours
    nx, ny, nz = wl.shape
    tab = oracle.lattice_tables(wl.lattice)
    c, wlat = tab["c"], tab["w"]
    for g in np.flatnonzero(~has_fluid):
        gid = int(ids_b[g])
        x, y, z = gid % nx, (gid // nx) % ny, gid // (nx * ny)
        nb = []
        for ci, wi in zip(c[1:], wlat[1:]):
            j = (x + ci[0]) % nx + nx * ((y + ci[1]) % ny + ny * ((z + ci[2]) % nz))
            if not solid[j]:
                nb.append((j, wi, int(np.abs(ci).sum()) == 1))
        assert nb, "a ghost has a fluid neighbour by definition"
        if len(nb) > nc:
            nb = [t for t in nb if t[2]]
        tot = sum(t[1] for t in nb)
        want = sorted((j, wi / tot) for j, wi, _ in nb)
        got = sorted((int(k), float(v)) for k, v in zip(corners_b[g], wb[g]) if v > 0)
        assert [k for k, _ in got] == [k for k, _ in want]
        assert np.allclose([v for _, v in got], [v for _, v in want], atol=1e-15)
        assert not solid[corners_b[g]].any()
    if wl.name.startswith("d3q19_porous"):
        assert (~has_fluid).sum() > 0, "the packing exercises the fallback"


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dead_end_fill(seed):
    """The dead-end fill (option): starting from the plain solid set, fluid
    nodes with at most one fluid lattice neighbour are made solid, all at
    once, pass after pass (brute force in numpy); every fluid node left has
    at least two fluid neighbours, and a filled ghost's normal is the unit
    vector towards its one remaining fluid neighbour."""
    wl = W.porous_d3q19(n=40, sphere_radius=5.0, porosity=0.40, seed=seed, precision=W.FP64, front=10.0)
    assert wl.fill == 1
    plain = oracle.OracleSim(wl.with_(fill=0), W.initial_phi(wl))
    filled = oracle.OracleSim(wl, W.initial_phi(wl))
    shape = tuple(reversed(wl.shape))
    s0 = (plain.get(oracle.F_SOLID) > 0.5).reshape(shape)
    s1 = (filled.get(oracle.F_SOLID) > 0.5).reshape(shape)
    c = _velocities(wl.lattice)

    def fluid_neighbours(solid):
        cnt = np.zeros(solid.shape, np.int64)
        for ci in c[1:]:
            cnt += ~np.roll(solid, shift=(-ci[2], -ci[1], -ci[0]), axis=(0, 1, 2))
        return cnt

    want = s0.copy()
    while True:
        dead = ~want & (fluid_neighbours(want) <= 1)
        if not dead.any():
            break
        want |= dead
    assert np.array_equal(s1, want)
    new = s1 & ~s0
    assert new.sum() > 0
    assert np.all(fluid_neighbours(s1)[~s1] >= 2)
    ids, nrm, _, _ = filled.ghosts()
    nx, ny, nz = wl.shape
    flat_new = new.reshape(-1)
    checked = 0
    for g, gid in enumerate(ids):
        if not flat_new[gid]:
            continue
        x, y, z = gid % nx, (gid // nx) % ny, gid // (nx * ny)
        open_dirs = [ci for ci in c[1:] if not s1[(z + ci[2]) % nz, (y + ci[1]) % ny, (x + ci[0]) % nx]]
        assert len(open_dirs) == 1
        u = np.asarray(open_dirs[0], float)
        assert np.allclose(nrm[g], u / np.linalg.norm(u), atol=1e-15)
        checked += 1
    assert checked > 0
