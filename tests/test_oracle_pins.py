"""Pins of the FP64 oracle's building blocks against what the paper and the
mathematics fix (closed forms, identities, special cases).  CPU only."""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_2605_30878_amd import workloads as W

CS2 = 1.0 / 3.0


def _tiny(lattice, **kw):
    shape = (4, 4, 4) if lattice == W.D3Q19 else (4, 4, 1)
    base = dict(name="tiny", lattice=lattice, shape=shape, rho_l=1000.0, rho_g=1.0, mu_l=10.0,
                mu_g=0.1, sigma=0.01, W=4.0, mobility=0.02, theta=90.0)
    base.update(kw)
    wl = W.Workload(**base)
    return oracle.OracleSim(wl, np.zeros(wl.nodes))


# ------------------------------------------------------------------ lattices
@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_lattice_isotropy(lattice):
    t = oracle.lattice_tables(lattice)
    c, w = t["c"].astype(float), t["w"]
    assert abs(w.sum() - 1.0) < 1e-15
    for a in range(3):
        assert abs((w * c[:, a]).sum()) < 1e-15
    D = 2 if lattice == W.D2Q9 else 3
    for a, b in itertools.product(range(D), repeat=2):
        assert abs((w * c[:, a] * c[:, b]).sum() - CS2 * (a == b)) < 1e-15
    for a, b, g in itertools.product(range(D), repeat=3):
        assert abs((w * c[:, a] * c[:, b] * c[:, g]).sum()) < 1e-15
    for a, b, g, d in itertools.product(range(D), repeat=4):
        want = CS2 ** 2 * ((a == b) * (g == d) + (a == g) * (b == d) + (a == d) * (b == g))
        assert abs((w * c[:, a] * c[:, b] * c[:, g] * c[:, d]).sum() - want) < 1e-15


def test_d2q9_mrt_matrix_structure():
    """Appendix A's M: orthogonal rows with norms (9,36,36,6,12,6,12,4,4);
    row 0 is mass, rows 3 and 5 momentum, rows 7 and 8 (the ones S relaxes
    with 1/tau) the two traceless second moments cx^2-cy^2 and cx cy."""
    t = oracle.lattice_tables(W.D2Q9)
    M, c = t["M"], t["c"].astype(float)
    G = M @ M.T
    assert np.allclose(G - np.diag(np.diag(G)), 0.0, atol=0)
    assert np.array_equal(np.diag(G), [9, 36, 36, 6, 12, 6, 12, 4, 4])
    assert np.array_equal(M[0], np.ones(9))
    assert np.array_equal(M[3], c[:, 0]) and np.array_equal(M[5], c[:, 1])
    assert np.array_equal(M[7], c[:, 0] ** 2 - c[:, 1] ** 2)
    assert np.array_equal(M[8], c[:, 0] * c[:, 1])


def test_d3q19_moment_basis():
    t = oracle.lattice_tables(W.D3Q19)
    M, c = t["M"], t["c"].astype(float)
    G = M @ M.T
    assert np.allclose(G - np.diag(np.diag(G)), 0.0, atol=1e-12)
    assert np.linalg.matrix_rank(M) == 19
    cx, cy, cz = c.T
    stress = np.stack([2 * cx * cx - cy * cy - cz * cz, cy * cy - cz * cz, cx * cy, cy * cz, cx * cz])
    # the five stress rows of the basis span exactly the traceless second moments
    rows = M[[9, 11, 13, 14, 15]]
    for s in stress:
        coef, res, *_ = np.linalg.lstsq(rows.T, s, rcond=None)
        assert np.allclose(rows.T @ coef, s, atol=1e-12)
    assert np.array_equal(M[0], np.ones(19))
    assert np.array_equal(M[3], cx) and np.array_equal(M[5], cy) and np.array_equal(M[7], cz)


@pytest.mark.parametrize("mob", [0.005, 0.02, 0.05])
def test_colour_weights_and_mobility(mob):
    """chi sums to 1; M_phi = (cs^2 dt/2)[9(1-alpha)/5] (Eq. A7 text, p = 0)
    written as (1/2) sum_i chi_i c_ix^2; the D3Q19 reading reduces to the
    D2Q9 weights when summed over c_z."""
    t2 = oracle.lattice_tables(W.D2Q9, mob)
    t3 = oracle.lattice_tables(W.D3Q19, mob)
    for t in (t2, t3):
        assert abs(t["chi"].sum() - 1.0) < 1e-15
        assert abs(0.5 * (t["chi"] * t["c"][:, 0] ** 2).sum() - mob) < 1e-15
    assert abs(CS2 / 2 * 9 * (1 - t2["alpha"]) / 5 - mob) < 1e-15
    c2 = t2["c"]
    for i in range(9):
        m = (t3["c"][:, 0] == c2[i, 0]) & (t3["c"][:, 1] == c2[i, 1])
        assert abs(t3["chi"][m].sum() - t2["chi"][i]) < 1e-15
        assert abs(t3["w"][m].sum() - t2["w"][i]) < 1e-15


# ------------------------------------------------------------------ equilibrium
@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_equilibrium_moments(lattice):
    """Eq. A4: zeroth moment 1, first moment u, second moment
    (chi2 + p) I + u u with chi2 = sum chi c_x^2."""
    s = _tiny(lattice)
    t = oracle.lattice_tables(lattice)
    c = t["c"].astype(float)
    chi2 = (t["chi"] * c[:, 0] ** 2).sum()
    D = 2 if lattice == W.D2Q9 else 3
    rng = np.random.default_rng(1)
    for _ in range(20):
        u = np.zeros(3)
        u[:D] = rng.uniform(-0.1, 0.1, D)
        p = rng.uniform(-0.01, 0.01)
        neq = s.equilibrium(u, p)
        assert abs(neq.sum() - 1.0) < 1e-15
        assert np.allclose(c.T @ neq, u, atol=1e-16, rtol=0)
        second = np.einsum("ia,ib,i->ab", c, c, neq)
        want = (chi2 + p) * np.eye(3) + np.outer(u, u)
        if D == 2:
            want[2, 2] = 0.0
        assert np.allclose(second, want, atol=2e-16, rtol=0)


@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_pressure_inverts_equilibrium(lattice):
    """Eq. A15 applied to N = N^eq(u, p) returns p, and Eq. A14 returns u
    when there is no force (uniform phi, no gravity)."""
    s = _tiny(lattice)
    D = 2 if lattice == W.D2Q9 else 3
    rng = np.random.default_rng(2)
    Q = s.Q
    for _ in range(20):
        u = np.zeros(3)
        u[:D] = rng.uniform(-0.1, 0.1, D)
        p = rng.uniform(-0.01, 0.01)
        neq = s.equilibrium(u, p)
        _, _, m = s.node(neq, np.ones(Q))
        assert abs(m["p"] - p) < 1e-16
        assert np.allclose(m["u0"], u, atol=1e-17) and np.allclose(m["u"], u, atol=1e-17)
        assert np.allclose(m["F"], 0.0, atol=0)


# ------------------------------------------------------------------ collision
def _stress_projector(lattice):
    t = oracle.lattice_tables(lattice)
    c = t["c"].astype(float)
    cx, cy, cz = c.T
    if lattice == W.D2Q9:
        rows = [cx * cx - cy * cy, cx * cy]
    else:
        rows = [2 * cx * cx - cy * cy - cz * cz, cy * cy - cz * cz, cx * cy, cy * cz, cx * cz]
    return sum(np.outer(r, r) / (r @ r) for r in rows)


def _random_node(s, rng, lattice):
    """Populations near equilibrium and a colour stencil across an interface."""
    D = 2 if lattice == W.D2Q9 else 3
    u = np.zeros(3)
    u[:D] = rng.uniform(-0.05, 0.05, D)
    N = s.equilibrium(u, rng.uniform(-0.01, 0.01)) + rng.uniform(-1e-3, 1e-3, s.Q)
    t = oracle.lattice_tables(lattice)
    n = rng.normal(size=3)
    if D == 2:
        n[2] = 0
    n /= np.linalg.norm(n)
    eta0 = rng.uniform(-2, 2)
    eta = eta0 + t["c"].astype(float) @ n
    phi_nb = 0.5 * (1.0 + np.tanh(2.0 * eta / 4.0))
    return N, phi_nb


@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_collision_identities(lattice):
    """Eq. A1-A3: mass sum 1 (every non-stress moment relaxes at rate 1),
    momentum u0 + F/rho, and the matrix form equals
    N^eq + F/2 + (1 - 1/tau) P_sigma (N - N^eq) with P_sigma the orthogonal
    projector onto the traceless second moments -- i.e. only the stress
    moments keep (1 - 1/tau) of their non-equilibrium part."""
    s = _tiny(lattice, g=(1e-5, -2e-5, 3e-5))
    t = oracle.lattice_tables(lattice)
    c, w = t["c"].astype(float), t["w"]
    Ps = _stress_projector(lattice)
    rng = np.random.default_rng(3)
    for _ in range(25):
        N, phi_nb = _random_node(s, rng, lattice)
        Ns, Bs, m = s.node(N, phi_nb)
        a = m["F"] / m["rho"]
        assert abs(Ns.sum() - 1.0) < 1e-14
        assert np.allclose(c.T @ Ns, m["u0"] + a, atol=1e-15, rtol=0)
        neq = s.equilibrium(m["u"], m["p"])
        Fpop = w / CS2 * (c @ a)
        want = neq + 0.5 * Fpop + (1.0 - 1.0 / m["tau"]) * (Ps @ (N - neq))
        assert np.allclose(Ns, want, atol=1e-15, rtol=0)


@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_segregation_identities(lattice):
    """Eq. A12: sum_i B*_i = phi (the recolouring moves no colour mass), and
    the recolouring flux is (2/W) phi (1 - phi) (chi2 + p) n_phi."""
    s = _tiny(lattice)
    t = oracle.lattice_tables(lattice)
    c = t["c"].astype(float)
    chi2 = (t["chi"] * c[:, 0] ** 2).sum()
    rng = np.random.default_rng(4)
    for _ in range(25):
        N, phi_nb = _random_node(s, rng, lattice)
        Ns, Bs, m = s.node(N, phi_nb)
        phi = m["phi"]
        assert abs(Bs.sum() - phi) < 1e-15
        n = m["grad"] / np.linalg.norm(m["grad"])
        flux = c.T @ (Bs - phi * Ns)
        want = 2.0 / 4.0 * phi * (1 - phi) * (chi2 + m["p"]) * n
        assert np.allclose(flux, want, atol=1e-16, rtol=0)


@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_stencils_exact_on_polynomials(lattice):
    """The isotropic gradient stencil is exact for linear fields and the
    Laplacian stencil exact for quadratics (sum w c c = cs^2 I)."""
    s = _tiny(lattice, rho_l=1.0, mu_l=0.1)
    t = oracle.lattice_tables(lattice)
    c = t["c"].astype(float)
    D = 2 if lattice == W.D2Q9 else 3
    rng = np.random.default_rng(5)
    for _ in range(10):
        b = np.zeros(3)
        b[:D] = rng.uniform(-0.1, 0.1, D)
        H = np.zeros((3, 3))
        H[:D, :D] = rng.uniform(-0.01, 0.01, (D, D))
        H = H + H.T
        f = 0.5 + c @ b + 0.5 * np.einsum("ia,ab,ib->i", c, H, c)
        _, _, m = s.node(s.equilibrium([0, 0, 0], 0.0), f)
        assert np.allclose(m["grad"], b, atol=1e-16, rtol=0)
        assert abs(m["lap"] - np.trace(H)) < 1e-15


def test_surface_tension_vanishes_on_flat_equilibrium_profile():
    """Eq. 4 with the profile of Eq. 5: (3W/2) phi'' = -(48/W) phi(1-phi)(phi-1/2),
    so a flat equilibrium interface carries no surface-tension force.  With
    the lattice Laplacian the residual falls as 1/W^2."""
    res = []
    for Wd in (8.0, 16.0, 32.0):
        s = _tiny(W.D2Q9, W=Wd, rho_l=1.0, mu_l=0.1)
        t = oracle.lattice_tables(W.D2Q9)
        c = t["c"].astype(float)
        worst, scale = 0.0, 0.0
        for eta0 in np.linspace(-Wd / 2, Wd / 2, 17):
            phi_nb = 0.5 * (1 + np.tanh(2 * (eta0 + c[:, 0]) / Wd))
            _, _, m = s.node(s.equilibrium([0, 0, 0], 0.0), phi_nb)
            phi = m["phi"]
            term = 0.01 * 48 / Wd * phi * (1 - phi) * abs(phi - 0.5) * abs(m["grad"][0])
            worst = max(worst, abs(m["Fs"][0]))
            scale = max(scale, term)
        res.append(worst / scale)
    assert res[0] < 0.05
    assert res[1] < res[0] / 3.5 and res[2] < res[1] / 3.5


def test_body_and_pressure_forces():
    """F_b = rho g (Eq. 2); F_p = -p grad rho (Eq. A10) with
    rho = rho_l phi + rho_g (1 - phi) (text after Eq. 3)."""
    s = _tiny(W.D2Q9, g=(1e-4, -2e-4, 0.0))
    t = oracle.lattice_tables(W.D2Q9)
    c = t["c"].astype(float)
    rng = np.random.default_rng(6)
    for _ in range(10):
        N, phi_nb = _random_node(s, rng, W.D2Q9)
        _, _, m = s.node(N, phi_nb)
        phi = m["phi"]
        assert abs(m["rho"] - (1000 * phi + (1 - phi))) < 1e-12
        assert np.allclose(m["Fb"], m["rho"] * np.array([1e-4, -2e-4, 0.0]), rtol=1e-15, atol=0)
        assert np.allclose(m["Fp"], -m["p"] * 999.0 * m["grad"], rtol=1e-14, atol=1e-20)
        nu = 1.0 / (phi / 0.01 + (1 - phi) / 0.1)
        assert abs(m["tau"] - (0.5 + 3 * nu)) < 1e-14


# ------------------------------------------------------------------ ghost rule
def test_ghost_rule_is_exact_integral_of_eq8():
    """Eq. 9 is the exact solution of Eq. 8 from x_G to x_F: for a planar
    equilibrium interface (Eq. 5) meeting a flat wall at angle theta the rule
    returns the profile's value at the ghost node."""
    rng = np.random.default_rng(7)
    for _ in range(200):
        theta = rng.uniform(0.0, 180.0)
        Wd = rng.uniform(4.0, 10.0)
        th = math.radians(theta)
        ns = rng.normal(size=2)
        ns /= np.linalg.norm(ns)
        # n_phi with n_s . n_phi = -cos(theta) (Eq. 7)
        perp = np.array([-ns[1], ns[0]])
        nphi = -math.cos(th) * ns + math.sin(th) * perp
        x0 = rng.uniform(-3, 3, 2)
        xg = rng.uniform(-2, 2, 2)
        xf = xg + ns
        prof = lambda x: 0.5 * (1 + math.tanh(2 * float(nphi @ (x - x0)) / Wd))
        eps = -4.0 / Wd * math.cos(th)
        got = oracle.ghost_rule(prof(xf), eps, 0)
        want = prof(xg)
        assert abs(got - want) <= 1e-14 * max(want, 1e-300) + 1e-300


def test_ghost_rule_special_cases():
    """Bulk phases pass unchanged (no mass transfer along the wall), the
    neutral angle is the identity, and values stay in (0, 1) (Eq. 9 text)."""
    for eps in (-1.0, -0.3, 0.0, 0.5, 1.0):
        assert oracle.ghost_rule(0.0, eps) == 0.0
        assert oracle.ghost_rule(1.0, eps) == 1.0
    for phiF in np.linspace(0.01, 0.99, 21):
        assert oracle.ghost_rule(phiF, 0.0) == phiF
        assert oracle.ghost_rule(phiF, 0.0, 1) == phiF
        for eps in (-1.0, -0.2, 0.2, 1.0):
            g = oracle.ghost_rule(phiF, eps)
            assert 0.0 < g < 1.0
            # eps < 0 (theta < 90): the ghost is wetter than the probe
            assert (g > phiF) == (eps < 0)


def test_fakhari_difference_series():
    """Eq. 11: phi_G - phi_G^Fakhari = (eps^3/12)[1 - 3(1-phi)phi]phi(1-phi)
    + O(eps^4); the ratio tends to 1 as eps -> 0."""
    for phiF in (0.1, 0.3, 0.5, 0.7, 0.9):
        prev = None
        for eps in (0.04, 0.02, 0.01):
            for sgn in (1.0, -1.0):
                e = sgn * eps
                diff = oracle.ghost_rule(phiF, e, 0) - oracle.ghost_rule(phiF, e, 1)
                lead = e ** 3 / 12 * (1 - 3 * (1 - phiF) * phiF) * phiF * (1 - phiF)
                ratio = diff / lead
                assert abs(ratio - 1.0) < eps, (phiF, e, ratio)


@pytest.mark.parametrize("lattice", [W.D2Q9, W.D3Q19])
def test_no_recolouring_outside_unit_interval(lattice):
    """Reading of Eq. A12 where the weakly compressible update lets phi leave
    [0, 1]: the recolouring amplitude phi(1 - phi) is clamped at 0, so there
    B*_i = phi N*_i exactly."""
    s = _tiny(lattice)
    rng = np.random.default_rng(8)
    for shift in (1.0005, -0.0005):
        N, phi_nb = _random_node(s, rng, lattice)
        phi_nb = np.full(s.Q, shift) + 1e-6 * rng.normal(size=s.Q)
        Ns, Bs, m = s.node(N, phi_nb)
        assert np.array_equal(Bs, m["phi"] * Ns)


def test_fakhari_rule_literal_form_and_neutral_limit():
    """Eq. 10 as printed, (2/eps)(1 + eps/2 - sqrt((1 + eps/2)^2 - 2 eps phi)) - phi,
    evaluated where it is well conditioned, equals the oracle's rule; near
    eps = 0 the oracle's rule is smooth and tends to phi (the neutral angle)."""
    for phiF in np.linspace(0.0, 1.0, 11):
        for eps in (-1.0, -0.5, -0.2, 0.2, 0.5, 1.0):
            a = 1 + eps / 2
            lit = 2 / eps * (a - math.sqrt(a * a - 2 * eps * phiF)) - phiF
            assert abs(oracle.ghost_rule(phiF, eps, 1) - lit) < 1e-14
        for eps in (1e-17, -4.9e-17, 1e-9, -1e-9):
            assert abs(oracle.ghost_rule(phiF, eps, 1) - phiF) < 1e-8
        assert oracle.ghost_rule(phiF, 0.0, 1) == phiF
