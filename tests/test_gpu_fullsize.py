"""The benchmark workloads at their full size, in the launch configurations
the benchmark times: the D3Q19 256^3 drop on a sphere (density ratio 1000)
in FP32 and in FP16-offset storage, both in the two-pass form (tiled colour
kernel, row collide-stream kernel) and in the collide-colour form, and the
384^3 sphere packing in the fluid-only layout.  The oracle cannot
run this box end to end in a test, so it checks sampled nodes one by one
with its own per-node functions, in FP64, from the library's state read
back (which FP32 holds exactly in FP64):

- collision, recolouring and push streaming with bounce-back: the
  populations the sampled nodes send out, found after one step at their
  targets (Appendix A, Eq. A1-A17);
- the colour field of the following step at sampled nodes, summed from the
  oracle's post-collision liquid populations of every upstream node
  (Eq. A13 with streaming);
- the ghost update at sampled ghost nodes: trilinear probe at x_G + n_s
  with fluid corners from the new colour field and solid corners from the
  previous step, then Eq. 9.

Samples are seeded and include interface nodes, fluid nodes next to the
solid (on and off the contact line) and bulk nodes.  The FP32 tolerances
are rounding of one step: populations are stored as offsets from the rest
state (at most about 0.05 here), so 1e-7 is about 20 ulps of the largest
offset; the colour field sums 19 terms of at most about 0.35 (1e-6); Eq. 9
is a few operations on values of order one (5e-7).  In 16-bit storage the
stored offsets themselves are rounded at 3e-5."""
import math

import numpy as np
import pytest

import oracle
from paper_2605_30878_amd import workloads as W

from helpers import direction_map

pytestmark = pytest.mark.gpu


def _lbm():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2605_30878_amd import lbm

    lbm.load_library()
    return lbm


CASES = {
    # name: (workload factory, options, tolerances N / phi / ghost phi, check ghosts)
    "sphere256_f32": (lambda: W.sphere_d3q19(256, theta=60.0, precision=W.FP32), 0, (1e-7, 1e-6, 5e-7), True),
    # 16-bit offsets: tolerances from the FP16 spacing of the largest stored
    # offset (computed below)
    "sphere256_fp16ofs": (lambda: W.sphere_d3q19(256, theta=60.0, precision=W.FP16_OFS), 0, (None, None, 5e-7), True),
    # the collide-colour form (LBM_OPT_FUSED), which the benchmark times
    "sphere256_f32_collide_colour": (lambda: W.sphere_d3q19(256, theta=60.0, precision=W.FP32), 1,
                                     (1e-7, 1e-6, 5e-7), True),
    "sphere256_fp16ofs_collide_colour": (lambda: W.sphere_d3q19(256, theta=60.0, precision=W.FP16_OFS), 1,
                                         (None, None, 5e-7), True),
    # the porous workload in the fluid-only layout (its ghost rule, the
    # fluid-only probe, is checked against the oracle on smaller packings)
    "porous384_sparse_f32": (lambda: W.porous_d3q19(384, precision=W.FP32), 32, (1e-7, 1e-6, None), False),
}


@pytest.mark.parametrize("case", list(CASES))
def test_full_size_sampled_against_oracle(case):
    lbm = _lbm()
    make, options, (tol_n, tol_phi, tol_g), check_ghosts = CASES[case]
    wl = make()
    n = wl.shape[0]
    print(f"[fullsize] {case}: {wl.name} shape={wl.shape} theta={wl.theta} options={options}", flush=True)
    sim = lbm.Simulation(wl, W.initial_phi(wl), options=options)
    sim.step(50)
    flags = sim.read(lbm.FIELD_FLAGS).astype(np.int64)
    solid = (flags & lbm.FLAG_SOLID) > 0
    N0 = sim.read(lbm.FIELD_N)              # state entering step 51, library order
    phi1 = sim.read(lbm.FIELD_PHI)          # the colour field step 51 uses (ghosts included)
    prev = sim.read(lbm.FIELD_SOLID_PHI)    # solid values of the state (last step's ghosts)
    sim.step(1)
    N1 = sim.read(lbm.FIELD_N)
    phi2 = sim.read(lbm.FIELD_PHI)          # colour field of step 52 at fluid nodes
    sim_offsets = sim.read(lbm.FIELD_N_OFFSET) if tol_n is None else None
    sim.close()

    perm = direction_map(W.D3Q19)           # perm[lib] = oracle index
    lib_of = np.argsort(perm)               # lib_of[oracle] = library index
    c = oracle.lattice_tables(W.D3Q19)["c"]
    Q = len(c)
    opp = np.array([int(np.flatnonzero((c == -c[i]).all(axis=1))[0]) for i in range(Q)])
    # the per-node functions need the run's constants only, not its box
    node_sim = oracle.OracleSim(wl.with_(precision=W.FP64, shape=(4, 4, 4), solids=[], liquid=[]),
                                np.zeros(64))

    def nid(x, y, z):
        return (x % n) + n * ((y % n) + n * (z % n))

    def coords(k):
        return k % n, (k // n) % n, k // (n * n)

    cache = {}

    def post(k):
        """Oracle post-collision (N*, B*) of fluid node k, oracle order."""
        if k not in cache:
            x, y, z = coords(k)
            Nk = N0[lib_of, k]
            nb = np.array([phi1[nid(x + c[i][0], y + c[i][1], z + c[i][2])] for i in range(Q)])
            Ns, Bs, _ = node_sim.node(Nk, nb)
            cache[k] = (Ns, Bs)
        return cache[k]

    rng = np.random.default_rng(0)
    fluid = ~solid
    near = fluid & ((flags & lbm.FLAG_NEAR_SOLID) > 0)
    iface = fluid & (phi1 > 0.05) & (phi1 < 0.95)
    pools = {"interface": np.flatnonzero(iface & ~near), "contact line": np.flatnonzero(iface & near),
             "near solid": np.flatnonzero(near & ~iface), "bulk": np.flatnonzero(fluid & ~iface & ~near)}
    picks = []
    for name, pool in pools.items():
        assert pool.size > 0, name
        picks += [int(k) for k in rng.choice(pool, size=min(40, pool.size), replace=False)]
    nscale = float(np.max(np.abs(N0[:, fluid])))
    if tol_n is None:
        # offsets are stored as n / 2^-10 in FP16 (10 fraction bits): h, the
        # spacing at the largest offset, bounds twice the rounding of each
        # stored offset; the rest population closes the stored zeroth moment,
        # so it carries the other 18 roundings (at most 9 h); the colour
        # field sums 19 terms phi_src n_i with phi_src <= 1 (at most 18 h)
        off = float(np.max(np.abs(sim_offsets[:, fluid])))
        h = 2.0 ** (math.floor(math.log2(off * 1024.0)) - 10) / 1024.0
        tol_n = 10 * h
        tol_phi = 20 * h + 1e-6

    # collision + streaming: where each population of a sampled node lands
    err_n = 0.0
    for k in picks:
        Ns, _ = post(k)
        x, y, z = coords(k)
        for i in range(Q):
            t = nid(x + c[i][0], y + c[i][1], z + c[i][2])
            got = N1[lib_of[opp[i]], k] if solid[t] else N1[lib_of[i], t]
            err_n = max(err_n, abs(got - Ns[i]))
    # colour field of the next step: sum of the liquid populations streamed in
    err_phi = 0.0
    for k in picks:
        x, y, z = coords(k)
        acc = 0.0
        for i in range(Q):
            s = nid(x - c[i][0], y - c[i][1], z - c[i][2])
            acc += post(k)[1][opp[i]] if solid[s] else post(s)[1][i]
        err_phi = max(err_phi, abs(phi2[k] - acc))
    # ghost update (Eq. 9) at sampled ghosts
    eps = -4.0 / wl.W * math.cos(math.radians(wl.theta))
    centre = np.array(wl.solids[0].center)
    ghosts = np.flatnonzero((flags & lbm.FLAG_GHOST) > 0)
    err_g = 0.0
    for g in (rng.choice(ghosts, size=200, replace=False) if check_ghosts else []):
        pos = np.array(coords(int(g)), float)
        d = pos - centre
        nrm = d / np.linalg.norm(d)
        xf = pos + nrm
        base = np.floor(xf).astype(int)
        fr = xf - base
        phiF = 0.0
        for bz in (0, 1):
            for by in (0, 1):
                for bx in (0, 1):
                    wgt = (fr[0] if bx else 1 - fr[0]) * (fr[1] if by else 1 - fr[1]) * (fr[2] if bz else 1 - fr[2])
                    q = nid(base[0] + bx, base[1] + by, base[2] + bz)
                    phiF += wgt * (prev[q] if solid[q] else phi1[q])
        err_g = max(err_g, abs(phi1[g] - oracle.ghost_rule(phiF, eps, 0)))
    print(f"[fullsize] samples={len(picks)} upstream nodes={len(cache)} max|dN|={err_n:.2e} (tol {tol_n:.1e}, "
          f"scale {nscale:.3f}) max|dphi|={err_phi:.2e} (tol {tol_phi:.1e}) max|dphi_G|={err_g:.2e}", flush=True)
    assert err_n <= tol_n
    assert err_phi <= tol_phi
    if check_ghosts:
        assert err_g <= tol_g
