/*
 * lbm_oracle.c -- plain FP64 CPU oracle for the color-gradient lattice
 * Boltzmann update with the ghost-node wetting condition.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * helper with the HIP library: every constant below is written out here.
 *
 * What it computes (paper: "Color-gradient lattice Boltzmann modeling of
 * wetting boundary condition on curved solid boundaries"):
 *   - Appendix A: MRT collision (Eq. A1-A3), velocity-based equilibrium
 *     (Eq. A4-A7), forcing (Eq. A8-A11), segregation (Eq. A12), macroscopic
 *     fields (Eq. A13-A15), propagation of N and B (Eq. A16-A17).
 *   - Section 2: mixture density / viscosity (text after Eq. 3), surface
 *     tension force (Eq. 4), ghost-node rule (Eq. 9) with the probe point
 *     x_F = x_G + n_s (text before Eq. 8) and bilinear interpolation,
 *     Fakhari et al.'s rule (Eq. 10) as a switch.
 *   - Section 3 (opening paragraph): ghost nodes start at (1 + cos theta)/2,
 *     analytic solid normals.
 *
 * Readings where the paper is silent (the step order, the D3Q19 lattice and
 * moment basis, the gradient stencils, p and the viscous correction force)
 * are marked READING below.  Everything is FP64, no fast-math, loops over
 * nodes run in OpenMP but every per-node result is independent of the thread
 * count; reductions are serial in node order.
 *
 * Parity: the per-node building blocks are pinned by closed forms and
 * identities in the CPU test suite (equilibrium moments, Eq. A15 inverting
 * Eq. A4, collision invariants, segregation mass, Eq. 9 against the exact
 * logistic profile).  The whole update is pinned by invariants (colour mass,
 * mirror symmetry), the Laplace law, single-phase closed forms (Taylor-Green
 * decay, Poiseuille flow) and Young's law on a cylinder.  Transient
 * populations have no closed form: beyond those properties they are
 * "parity unpinned".
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define QMAX 19

/* ---------------------------------------------------------------- params */
typedef struct {
    int32_t lattice;      /* 0 = D2Q9, 1 = D3Q19 */
    int32_t nx, ny, nz;   /* nz = 1 for D2Q9; every axis is periodic */
    double rho_l, rho_g;  /* liquid (phi = 1) and gas (phi = 0) densities */
    double mu_l, mu_g;    /* dynamic viscosities */
    double sigma;         /* surface tension */
    double W;             /* interface width */
    double mobility;      /* M_phi, mapped to alpha (Eq. A7 text) */
    double g[3];          /* body acceleration: F_b = rho g (Eq. 2) */
    double theta_deg;     /* contact angle through the liquid (Eq. 7) */
    int32_t ghost_rule;   /* 0 = Eq. 9, 1 = Eq. 10 (Fakhari et al.) */
    int32_t probe;        /* corners of the probe interpolation: 0 = all eight
                             (solid ones from the snapshot), 1 = fluid ones
                             only, weights rescaled to sum 1 (no fluid
                             corner: the ghost's fluid lattice neighbours) */
    int32_t fill;         /* 1: fluid nodes with at most one fluid lattice
                             neighbour become solid, pass after pass */
} orc_params;

typedef struct {
    int32_t kind;         /* 0 = ball/disk |x-c| <= r ; 1 = half-space (x-c).nrm <= 0 */
    int32_t pad;
    double c[3];
    double r;
    double nrm[3];        /* for kind 1: outward normal of the solid */
} orc_solid;

/* ---------------------------------------------------------------- lattices */
/* D2Q9 velocities, weights: Appendix A (matrix c and w_i after Eq. A4). */
static const int C9[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {-1, 0, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, 1, 0}, {-1, -1, 0}, {1, -1, 0}};
static const double W9[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                             1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
/* The MRT transformation matrix M printed in Appendix A (after Eq. A1). */
static const double M9[9][9] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},
    {4, -2, -2, -2, -2, 1, 1, 1, 1},
    {0, 1, 0, -1, 0, 1, -1, -1, 1},
    {0, -2, 0, 2, 0, 1, -1, -1, 1},
    {0, 0, 1, 0, -1, 1, 1, -1, -1},
    {0, 0, -2, 0, 2, 1, 1, -1, -1},
    {0, 1, -1, 1, -1, 0, 0, 0, 0},
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};

/* READING (D3Q19 lattice): rest, 6 face neighbours (w = 1/18), 12 edge
 * neighbours (w = 1/36), cs^2 = 1/3.  The paper is D2Q9 only and says the
 * scheme extends directly to three dimensions (Section 4). */
static const int C19[19][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1}};

typedef struct {
    int D, Q;
    int c[QMAX][3];
    int opp[QMAX];
    double w[QMAX];
    double chi[QMAX];
    double cs2;
    double M[QMAX][QMAX];
    double Minv[QMAX][QMAX];
    int stress[QMAX];     /* 1 if moment row k relaxes with 1/tau */
} lattice_t;

/* READING (D3Q19 moment basis): the classical orthogonal D3Q19 basis
 * (d'Humieres et al. 2002) as polynomials of the velocity.  Rows 9, 11, 13,
 * 14, 15 are the five traceless second-order (stress) moments; as in the
 * D2Q9 matrix S of Appendix A, only those relax with 1/tau, every other
 * moment relaxes with rate 1. */
static void d3q19_moments(const int c[3], double row[19]) {
    double cx = c[0], cy = c[1], cz = c[2];
    double c2 = cx * cx + cy * cy + cz * cz;
    row[0] = 1.0;
    row[1] = 19.0 * c2 - 30.0;
    row[2] = (21.0 * c2 * c2 - 53.0 * c2 + 24.0) / 2.0;
    row[3] = cx;
    row[4] = (5.0 * c2 - 9.0) * cx;
    row[5] = cy;
    row[6] = (5.0 * c2 - 9.0) * cy;
    row[7] = cz;
    row[8] = (5.0 * c2 - 9.0) * cz;
    row[9] = 3.0 * cx * cx - c2;
    row[10] = (3.0 * c2 - 5.0) * (3.0 * cx * cx - c2);
    row[11] = cy * cy - cz * cz;
    row[12] = (3.0 * c2 - 5.0) * (cy * cy - cz * cz);
    row[13] = cx * cy;
    row[14] = cy * cz;
    row[15] = cx * cz;
    row[16] = (cy * cy - cz * cz) * cx;
    row[17] = (cz * cz - cx * cx) * cy;
    row[18] = (cx * cx - cy * cy) * cz;
}

/* Plain Gauss-Jordan inverse with partial pivoting. Returns 0 on success. */
static int invert(int n, double A[QMAX][QMAX], double Ainv[QMAX][QMAX]) {
    double a[QMAX][2 * QMAX];
    for (int i = 0; i < n; i++)
        for (int j = 0; j < 2 * n; j++)
            a[i][j] = (j < n) ? A[i][j] : (j - n == i ? 1.0 : 0.0);
    for (int col = 0; col < n; col++) {
        int piv = col;
        for (int r = col + 1; r < n; r++)
            if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
        if (fabs(a[piv][col]) < 1e-12) return -1;
        if (piv != col)
            for (int j = 0; j < 2 * n; j++) {
                double t = a[col][j]; a[col][j] = a[piv][j]; a[piv][j] = t;
            }
        double d = a[col][col];
        for (int j = 0; j < 2 * n; j++) a[col][j] /= d;
        for (int r = 0; r < n; r++) {
            if (r == col) continue;
            double f = a[r][col];
            if (f != 0.0)
                for (int j = 0; j < 2 * n; j++) a[r][j] -= f * a[col][j];
        }
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) Ainv[i][j] = a[i][j + n];
    return 0;
}

static int lattice_init(lattice_t* L, int lattice, double mobility, double* alpha_out) {
    memset(L, 0, sizeof(*L));
    L->cs2 = 1.0 / 3.0;
    if (lattice == 0) {
        L->D = 2; L->Q = 9;
        for (int i = 0; i < 9; i++) {
            for (int a = 0; a < 3; a++) L->c[i][a] = C9[i][a];
            L->w[i] = W9[i];
            for (int k = 0; k < 9; k++) L->M[k][i] = M9[k][i];
        }
        L->stress[7] = L->stress[8] = 1;   /* S = diag(1,...,1,s7,s8) */
        /* Eq. A7 text: M_phi = (cs^2 dt / 2) [9(1-alpha)/5 + p/cs^2], read
         * with p = 0 (READING R-alpha). */
        double alpha = 1.0 - 2.0 * mobility / (L->cs2 * 9.0 / 5.0);
        /* Eq. A7: chi = (alpha, (1-alpha)/5 x4, (1-alpha)/20 x4). */
        L->chi[0] = alpha;
        for (int i = 1; i <= 4; i++) L->chi[i] = (1.0 - alpha) / 5.0;
        for (int i = 5; i <= 8; i++) L->chi[i] = (1.0 - alpha) / 20.0;
        *alpha_out = alpha;
    } else if (lattice == 1) {
        L->D = 3; L->Q = 19;
        for (int i = 0; i < 19; i++) {
            for (int a = 0; a < 3; a++) L->c[i][a] = C19[i][a];
            int nz = abs(C19[i][0]) + abs(C19[i][1]) + abs(C19[i][2]);
            L->w[i] = nz == 0 ? 1.0 / 3.0 : (nz == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
            double row[19];
            d3q19_moments(C19[i], row);
            for (int k = 0; k < 19; k++) L->M[k][i] = row[k];
        }
        L->stress[9] = L->stress[11] = L->stress[13] = L->stress[14] = L->stress[15] = 1;
        /* READING (D3Q19 colour weights): chi_i = (1-alpha) w_i / (1 - w_0)
         * for i != 0, which is Eq. A7 exactly in D2Q9.  The mobility relation
         * of Eq. A7 written as M_phi = (dt/2)[sum_i chi_i c_ix^2 + p] with
         * p = 0 then gives alpha = 1 - 2 M_phi (1 - w_0) / cs^2. */
        double alpha = 1.0 - 2.0 * mobility * (1.0 - L->w[0]) / L->cs2;
        L->chi[0] = alpha;
        for (int i = 1; i < 19; i++) L->chi[i] = (1.0 - alpha) * L->w[i] / (1.0 - L->w[0]);
        *alpha_out = alpha;
    } else {
        return -1;
    }
    for (int i = 0; i < L->Q; i++)
        for (int j = 0; j < L->Q; j++)
            if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] && L->c[j][2] == -L->c[i][2])
                L->opp[i] = j;
    return invert(L->Q, L->M, L->Minv);
}

/* ---------------------------------------------------------------- sim */
typedef struct {
    orc_params P;
    lattice_t L;
    double alpha, nu_l, nu_g, eps, exp_eps;
    long n;
    uint8_t* solid;        /* 1 = solid node */
    double* nrm;           /* [n][3] solid normal, only meaningful at ghosts */
    long n_ghost;
    long* ghost;           /* ghost node ids, ascending */
    long* corner;          /* [n_ghost][8] corner node ids */
    double* cw;            /* [n_ghost][8] interpolation weights */
    double* N;             /* [Q][n] post-stream colour-blind populations */
    double* B;             /* [Q][n] post-stream blue (liquid) populations */
    double* Nn;
    double* Bn;
    double* phi_state;     /* [n] phi at solid nodes carried between steps */
    double* phi;           /* [n] working colour field of the current step */
    double* snap;          /* [n] snapshot for the Jacobi ghost update */
    long step;
    /* Alternative readings and planted mistakes (orc_set_variant); all 0 is
     * the oracle as it is meant.  visc: 0 Eq. A11 as read (R-visc), 1 its
     * sign flipped, 2 F_visc left out, 3 without the (tau - 1/2)/tau factor
     * (F_visc = -Pi_dev . grad rho).  seg: 0 READING R-seg (amplitude
     * max(phi (1 - phi), 0)), 1 the literal factor phi (1 - phi) of Eq. A12.
     * visc 1-3 exist only so that a test can show its pin fails on them. */
    int visc_variant, seg_variant;
} orc_sim;

static inline long wrap(long v, long n) { v %= n; return v < 0 ? v + n : v; }
static inline long node_id(const orc_sim* s, long x, long y, long z) {
    return x + (long)s->P.nx * (y + (long)s->P.ny * z);
}
static inline long neighbour(const orc_sim* s, long id, const int c[3]) {
    long nx = s->P.nx, ny = s->P.ny, nz = s->P.nz;
    long x = id % nx, y = (id / nx) % ny, z = id / (nx * ny);
    return node_id(s, wrap(x + c[0], nx), wrap(y + c[1], ny), wrap(z + c[2], nz));
}

/* Eq. A4: velocity-based colour-blind equilibrium. */
static void equilibrium(const lattice_t* L, const double u[3], double p, double* neq) {
    double cs2 = L->cs2;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    neq[0] = L->chi[0] - (1.0 - L->w[0]) * p / cs2 - L->w[0] * uu / (2.0 * cs2);
    for (int i = 1; i < L->Q; i++) {
        double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
        neq[i] = L->chi[i] + L->w[i] * (p / cs2 + cu / cs2 + cu * cu / (2.0 * cs2 * cs2) - uu / (2.0 * cs2));
    }
}

/* Eq. 9 (this paper) or Eq. 10 (Fakhari et al.) ghost-node colour rule. */
double orc_ghost_rule(double phiF, double eps, int rule) {
    if (rule == 0) return phiF / (phiF + (1.0 - phiF) * exp(eps));
    /* Eq. 10 has a removable singularity at eps = 0 (the paper notes it needs
     * special care at 90 degrees).  With a = 1 + eps/2, multiplying
     * (a - sqrt(a^2 - 2 eps phiF)) by its conjugate gives
     * 2 eps phiF / (a + sqrt(a^2 - 2 eps phiF)); the factor eps cancels the
     * 2/eps in front, leaving 4 phiF / (a + sqrt(...)) - phiF, which is the
     * same function without the cancellation near eps = 0 (and phiF at 0). */
    double a = 1.0 + eps / 2.0;
    return 4.0 * phiF / (a + sqrt(a * a - 2.0 * eps * phiF)) - phiF;
}

/* Per-node macroscopic quantities shared by the step and the field readout. */
typedef struct {
    double phi, grad[3], lap, rho, nu, tau, u0[3], p, F[3], u[3];
    double Fs[3], Fp[3], Fv[3], Fb[3];
} node_macro;

/* phi_nb[i] = phi(x + c_i).  N = the node's populations. */
static void compute_macro(const orc_sim* s, const double* N, const double* phi_nb, node_macro* m) {
    const lattice_t* L = &s->L;
    const orc_params* P = &s->P;
    int Q = L->Q, D = L->D;
    double cs2 = L->cs2;
    memset(m, 0, sizeof(*m));
    m->phi = phi_nb[0];
    double phi = m->phi;
    /* READING R-grad: second-order isotropic lattice stencils. */
    for (int a = 0; a < 3; a++) {
        double acc = 0.0;
        for (int i = 0; i < Q; i++) acc += L->w[i] * L->c[i][a] * phi_nb[i];
        m->grad[a] = acc / cs2;
    }
    {
        double acc = 0.0;
        for (int i = 1; i < Q; i++) acc += L->w[i] * (phi_nb[i] - phi);
        m->lap = 2.0 * acc / cs2;
    }
    /* Mixture properties (text after Eq. 3). */
    m->rho = P->rho_l * phi + P->rho_g * (1.0 - phi);
    double inv_nu = phi / s->nu_l + (1.0 - phi) / s->nu_g;
    m->nu = 1.0 / inv_nu;
    m->tau = 0.5 + m->nu / cs2;           /* text after Eq. A3, dt = 1 */
    double grad_rho[3];
    for (int a = 0; a < 3; a++) grad_rho[a] = (P->rho_l - P->rho_g) * m->grad[a];
    /* Eq. A14 without the force half-step: u0 = sum_i N_i c_i. */
    for (int a = 0; a < 3; a++) {
        double acc = 0.0;
        for (int i = 0; i < Q; i++) acc += N[i] * L->c[i][a];
        m->u0[a] = acc;
    }
    /* Eq. A15, READING R-p: evaluated with u0 because u itself needs F_p(p). */
    {
        double sum = 0.0;
        for (int i = 1; i < Q; i++) sum += N[i];
        double uu = m->u0[0] * m->u0[0] + m->u0[1] * m->u0[1] + m->u0[2] * m->u0[2];
        m->p = (-L->w[0] / 2.0 * uu - (1.0 - L->chi[0]) * cs2 + sum * cs2) / (1.0 - L->w[0]);
    }
    /* Eq. 4: surface tension force. */
    double mu = -P->sigma * (48.0 / P->W * phi * (1.0 - phi) * (phi - 0.5) + 1.5 * P->W * m->lap);
    for (int a = 0; a < 3; a++) m->Fs[a] = mu * m->grad[a];
    /* Eq. A10: pressure correction force. */
    for (int a = 0; a < 3; a++) m->Fp[a] = -m->p * grad_rho[a];
    /* Eq. A11, READING R-visc: the strain rate (grad u + grad u^T) is taken
     * locally from the traceless non-equilibrium second moment,
     * (grad u + grad u^T) = -Pi_dev / (tau cs^2), with
     * Pi = sum_i c_i c_i (N_i - N_i^eq(u0, p)). */
    {
        double neq[QMAX];
        equilibrium(L, m->u0, m->p, neq);
        double Pi[3][3] = {{0}};
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) {
                double acc = 0.0;
                for (int i = 0; i < Q; i++) acc += L->c[i][a] * L->c[i][b] * (N[i] - neq[i]);
                Pi[a][b] = acc;
            }
        double tr = 0.0;
        for (int a = 0; a < D; a++) tr += Pi[a][a];
        for (int a = 0; a < D; a++) Pi[a][a] -= tr / D;
        double strain[3][3];
        for (int a = 0; a < 3; a++)
            for (int b = 0; b < 3; b++) strain[a][b] = -Pi[a][b] / (m->tau * cs2);
        for (int a = 0; a < 3; a++) {
            double acc = 0.0;
            for (int b = 0; b < 3; b++) acc += strain[a][b] * grad_rho[b];
            m->Fv[a] = cs2 * 1.0 * (m->tau - 0.5) * acc;
            if (s->visc_variant == 1) m->Fv[a] = -m->Fv[a];
            else if (s->visc_variant == 2) m->Fv[a] = 0.0;
            else if (s->visc_variant == 3) m->Fv[a] = cs2 * m->tau * acc;   /* = -Pi_dev . grad rho */
        }
    }
    /* Body force rho g (Eq. 2). */
    for (int a = 0; a < 3; a++) m->Fb[a] = m->rho * P->g[a];
    /* Eq. A9: total force. */
    for (int a = 0; a < 3; a++) m->F[a] = m->Fv[a] + m->Fp[a] + m->Fs[a] + m->Fb[a];
    if (D == 2) { m->F[2] = 0.0; }
    /* Eq. A14: u = sum_i N_i c_i + F dt / (2 rho). */
    for (int a = 0; a < 3; a++) m->u[a] = m->u0[a] + m->F[a] / (2.0 * m->rho);
}

/* One node: collision (Eq. A1) and segregation (Eq. A12).  Outputs the
 * post-collision N* and B*. */
static void collide_node(const orc_sim* s, const double* N, const double* phi_nb,
                         double* Nstar, double* Bstar, node_macro* mo) {
    const lattice_t* L = &s->L;
    int Q = L->Q;
    double cs2 = L->cs2;
    node_macro m;
    compute_macro(s, N, phi_nb, &m);
    /* Eq. A8: forcing populations F_i = (w_i/cs^2)(F dt / rho) . c_i. */
    double Fpop[QMAX];
    for (int i = 0; i < Q; i++) {
        double cf = L->c[i][0] * m.F[0] + L->c[i][1] * m.F[1] + L->c[i][2] * m.F[2];
        Fpop[i] = L->w[i] / cs2 * cf / m.rho;
    }
    /* Eq. A4 at the forced velocity u. */
    double neq[QMAX];
    equilibrium(L, m.u, m.p, neq);
    /* Eq. A2-A3: S = diag(1, ..., 1, 1/tau on the stress moments). */
    double S[QMAX];
    for (int k = 0; k < Q; k++) S[k] = L->stress[k] ? 1.0 / m.tau : 1.0;
    /* Eq. A1: N* = N - M^-1 S M (N - Neq) + M^-1 (I - S/2) M F. */
    double d[QMAX], md[QMAX], mf[QMAX], t1[QMAX], t2[QMAX];
    for (int i = 0; i < Q; i++) d[i] = N[i] - neq[i];
    for (int k = 0; k < Q; k++) {
        double a = 0.0, b = 0.0;
        for (int j = 0; j < Q; j++) { a += L->M[k][j] * d[j]; b += L->M[k][j] * Fpop[j]; }
        md[k] = S[k] * a;
        mf[k] = (1.0 - S[k] / 2.0) * b;
    }
    for (int i = 0; i < Q; i++) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < Q; k++) { a += L->Minv[i][k] * md[k]; b += L->Minv[i][k] * mf[k]; }
        t1[i] = a;
        t2[i] = b;
    }
    for (int i = 0; i < Q; i++) Nstar[i] = N[i] - t1[i] + t2[i];
    /* Eq. A12: segregation of the blue (liquid) populations.
     * READING R-n: n_phi = grad phi / |grad phi| where |grad phi| > 1e-12,
     * otherwise n_phi = 0 (the normal is undefined there, Eq. 3 text).
     * READING R-seg: the recolouring amplitude phi(1 - phi) is taken as
     * max(phi(1 - phi), 0).  phi is a fraction in [0, 1] in the model; the
     * weakly compressible update lets it overshoot by O(Ma^2) in the bulk,
     * where the factor would turn negative and drive a unit-length flux along
     * a rounding-level gradient (an ill-conditioned, chattering term). */
    double gn = sqrt(m.grad[0] * m.grad[0] + m.grad[1] * m.grad[1] + m.grad[2] * m.grad[2]);
    double n[3] = {0.0, 0.0, 0.0};
    if (gn > 1e-12)
        for (int a = 0; a < 3; a++) n[a] = m.grad[a] / gn;
    double zero[3] = {0.0, 0.0, 0.0};
    double neq0[QMAX];
    equilibrium(L, zero, m.p, neq0);
    double phi = m.phi;
    double amp = phi * (1.0 - phi);
    if (amp < 0.0 && s->seg_variant == 0) amp = 0.0;
    for (int i = 0; i < Q; i++) {
        double cn = L->c[i][0] * n[0] + L->c[i][1] * n[1] + L->c[i][2] * n[2];
        Bstar[i] = phi * Nstar[i] + 2.0 * cn / s->P.W * amp * neq0[i];
    }
    (void)cs2;
    if (mo) *mo = m;
}

/* S1 + S2: colour field at fluid nodes (Eq. A13) and the Jacobi ghost update
 * (Eq. 9) from one snapshot.  Writes s->phi; s->phi_state is not changed. */
static void colour_field(orc_sim* s) {
    long n = s->n;
    int Q = s->L.Q;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < n; x++) {
        if (s->solid[x]) {
            s->phi[x] = s->phi_state[x];
        } else {
            double acc = 0.0;
            for (int i = 0; i < Q; i++) acc += s->B[(long)i * n + x];
            s->phi[x] = acc;
        }
    }
    memcpy(s->snap, s->phi, sizeof(double) * n);
    int nc = s->L.D == 2 ? 4 : 8;
#pragma omp parallel for schedule(static)
    for (long g = 0; g < s->n_ghost; g++) {
        double phiF = 0.0;
        for (int k = 0; k < nc; k++) phiF += s->cw[g * 8 + k] * s->snap[s->corner[g * 8 + k]];
        s->phi[s->ghost[g]] = orc_ghost_rule(phiF, s->eps, s->P.ghost_rule);
    }
}

/* ---------------------------------------------------------------- geometry */
/* Displacement from a ball centre to a node under the periodic minimum
 * image (every axis of the box is periodic). */
static double min_image(double d, long n) { return d - (double)n * floor(d / (double)n + 0.5); }

static int in_solid(const orc_solid* sd, double x, double y, double z, int D, const long* box) {
    if (sd->kind == 0) {
        double dx = min_image(x - sd->c[0], box[0]), dy = min_image(y - sd->c[1], box[1]);
        double dz = D == 3 ? min_image(z - sd->c[2], box[2]) : 0.0;
        return dx * dx + dy * dy + dz * dz <= sd->r * sd->r;   /* READING R-solid: closed */
    }
    double v = (x - sd->c[0]) * sd->nrm[0] + (y - sd->c[1]) * sd->nrm[1] +
               (D == 3 ? (z - sd->c[2]) * sd->nrm[2] : 0.0);
    return v <= 0.0;
}

static void free_sim(orc_sim* s) {
    if (!s) return;
    free(s->solid); free(s->nrm); free(s->ghost); free(s->corner); free(s->cw);
    free(s->N); free(s->B); free(s->Nn); free(s->Bn);
    free(s->phi_state); free(s->phi); free(s->snap);
    free(s);
}

void orc_destroy(void* h) { free_sim((orc_sim*)h); }

void* orc_create(const orc_params* P, const orc_solid* solids, int nsolids,
                 const double* phi_init, char* err, int errlen) {
#define FAIL(msg) do { if (err && errlen > 0) snprintf(err, errlen, "%s", msg); free_sim(s); return NULL; } while (0)
    orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
    if (!s) return NULL;
    s->P = *P;
    if (P->lattice == 0) s->P.nz = 1;
    if (P->nx < 1 || P->ny < 1 || s->P.nz < 1) FAIL("bad grid");
    if (P->W < 4.0) FAIL("W < 4");
    if (lattice_init(&s->L, P->lattice, P->mobility, &s->alpha)) FAIL("bad lattice");
    if (s->alpha < 0.0 || s->alpha >= 1.0) FAIL("alpha outside [0,1)");
    if (!(P->theta_deg >= 0.0 && P->theta_deg <= 180.0)) FAIL("theta outside [0,180]");
    s->nu_l = P->mu_l / P->rho_l;
    s->nu_g = P->mu_g / P->rho_g;
    const double pi = 3.14159265358979323846;
    s->eps = -4.0 / P->W * cos(P->theta_deg * pi / 180.0);   /* Eq. 9, dx = 1 */
    s->exp_eps = exp(s->eps);
    long n = (long)P->nx * P->ny * s->P.nz;
    s->n = n;
    int Q = s->L.Q, D = s->L.D;
    s->solid = (uint8_t*)calloc(n, 1);
    s->nrm = (double*)calloc(n * 3, sizeof(double));
    s->N = (double*)calloc((size_t)Q * n, sizeof(double));
    s->B = (double*)calloc((size_t)Q * n, sizeof(double));
    s->Nn = (double*)calloc((size_t)Q * n, sizeof(double));
    s->Bn = (double*)calloc((size_t)Q * n, sizeof(double));
    s->phi_state = (double*)calloc(n, sizeof(double));
    s->phi = (double*)calloc(n, sizeof(double));
    s->snap = (double*)calloc(n, sizeof(double));
    if (!s->solid || !s->nrm || !s->N || !s->B || !s->Nn || !s->Bn || !s->phi_state || !s->phi || !s->snap)
        FAIL("out of memory");
    /* Solid set and the normal of the first primitive that holds the node. */
    const long box[3] = {P->nx, P->ny, s->P.nz};
    for (long id = 0; id < n; id++) {
        long x = id % P->nx, y = (id / P->nx) % P->ny, z = id / ((long)P->nx * P->ny);
        for (int k = 0; k < nsolids; k++) {
            const orc_solid* sd = &solids[k];
            if (!in_solid(sd, (double)x, (double)y, (double)z, D, box)) continue;
            s->solid[id] = 1;
            double v[3];
            if (sd->kind == 0) {
                v[0] = min_image(x - sd->c[0], box[0]);
                v[1] = min_image(y - sd->c[1], box[1]);
                v[2] = D == 3 ? min_image(z - sd->c[2], box[2]) : 0.0;
            } else {
                v[0] = sd->nrm[0]; v[1] = sd->nrm[1]; v[2] = D == 3 ? sd->nrm[2] : 0.0;
            }
            double len = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
            if (len > 0.0)
                for (int a = 0; a < 3; a++) s->nrm[id * 3 + a] = v[a] / len;
            else
                s->nrm[id * 3 + (D == 3 ? 2 : 1)] = 1.0;   /* node at a ball centre */
            break;
        }
    }
    /* READING (dead-end fill, option): a fluid node joined to the rest of
     * the fluid by at most one lattice link (a pocket in the contact between
     * two solids, narrower than a node) is made solid; passes repeat on the
     * new solid set until no such node is left.  A filled node belongs to no
     * primitive: its normal is the direction of the one fluid neighbour it
     * keeps at the end (none: it is interior and needs no normal). */
    if (P->fill == 1) {
        uint8_t* mark = (uint8_t*)calloc(n, 1);
        if (!mark) FAIL("out of memory");
        for (;;) {
            long changed = 0;
            for (long id = 0; id < n; id++) {
                mark[id] = 0;
                if (s->solid[id]) continue;
                int nf = 0;
                for (int i = 1; i < Q; i++)
                    if (!s->solid[neighbour(s, id, s->L.c[i])]) nf++;
                if (nf <= 1) { mark[id] = 1; changed++; }
            }
            if (changed == 0) break;
            for (long id = 0; id < n; id++)
                if (mark[id]) { s->solid[id] = 2; }
        }
        free(mark);
        for (long id = 0; id < n; id++) {
            if (s->solid[id] != 2) continue;
            s->solid[id] = 1;
            for (int a = 0; a < 3; a++) s->nrm[id * 3 + a] = 0.0;
            for (int i = 1; i < Q; i++) {
                if (s->solid[neighbour(s, id, s->L.c[i])]) continue;
                double len = sqrt((double)(s->L.c[i][0] * s->L.c[i][0] + s->L.c[i][1] * s->L.c[i][1] +
                                           s->L.c[i][2] * s->L.c[i][2]));
                for (int a = 0; a < 3; a++) s->nrm[id * 3 + a] = s->L.c[i][a] / len;
            }
        }
    }
    /* Ghost nodes: solid nodes with at least one fluid neighbour (Section 1). */
    long ng = 0;
    for (long id = 0; id < n; id++) {
        if (!s->solid[id]) continue;
        for (int i = 1; i < Q; i++)
            if (!s->solid[neighbour(s, id, s->L.c[i])]) { ng++; break; }
    }
    s->n_ghost = ng;
    s->ghost = (long*)calloc(ng ? ng : 1, sizeof(long));
    s->corner = (long*)calloc((ng ? ng : 1) * 8, sizeof(long));
    s->cw = (double*)calloc((ng ? ng : 1) * 8, sizeof(double));
    if (!s->ghost || !s->corner || !s->cw) FAIL("out of memory");
    ng = 0;
    for (long id = 0; id < n; id++) {
        if (!s->solid[id]) continue;
        int isg = 0;
        for (int i = 1; i < Q; i++)
            if (!s->solid[neighbour(s, id, s->L.c[i])]) { isg = 1; break; }
        if (!isg) continue;
        long x = id % P->nx, y = (id / P->nx) % P->ny, z = id / ((long)P->nx * P->ny);
        /* Probe point x_F = x_G + dx n_s (dx = 1), bi/trilinear weights. */
        double xf[3] = {x + s->nrm[id * 3 + 0], y + s->nrm[id * 3 + 1], z + s->nrm[id * 3 + 2]};
        double fl[3], fr[3];
        for (int a = 0; a < 3; a++) { fl[a] = floor(xf[a]); fr[a] = xf[a] - fl[a]; }
        if (D == 2) { fl[2] = (double)z; fr[2] = 0.0; }
        int nc = D == 2 ? 4 : 8;
        for (int k = 0; k < nc; k++) {
            int bx = k & 1, by = (k >> 1) & 1, bz = (k >> 2) & 1;
            long cx = wrap((long)fl[0] + bx, P->nx);
            long cy = wrap((long)fl[1] + by, P->ny);
            long cz = wrap((long)fl[2] + bz, s->P.nz);
            double wgt = (bx ? fr[0] : 1.0 - fr[0]) * (by ? fr[1] : 1.0 - fr[1]);
            if (D == 3) wgt *= (bz ? fr[2] : 1.0 - fr[2]);
            s->corner[ng * 8 + k] = node_id(s, cx, cy, cz);
            s->cw[ng * 8 + k] = wgt;
        }
        /* READING (alternative probe, option): phi_F is meant to be the fluid's
         * colour at x_F (the text before Eq. 8 places x_F in the fluid), so
         * only fluid corners take part, their weights rescaled to sum to 1.
         * Where x_F has no fluid corner (a ghost in the gap between two
         * touching solids, whose normal points into the other solid), phi_F
         * is taken from the ghost's own fluid lattice neighbours instead,
         * weighted by w_i and rescaled to sum to 1: all of them when there
         * are at most nc, else the axis (face) neighbours alone. */
        if (P->probe == 1) {
            double wf = 0.0;
            for (int k = 0; k < nc; k++)
                if (!s->solid[s->corner[ng * 8 + k]]) wf += s->cw[ng * 8 + k];
            if (wf > 0.0) {
                for (int k = 0; k < nc; k++)
                    s->cw[ng * 8 + k] = s->solid[s->corner[ng * 8 + k]] ? 0.0 : s->cw[ng * 8 + k] / wf;
            } else {
                long nb[QMAX];
                double wn[QMAX];
                int axis[QMAX], nf = 0, naxis = 0;
                for (int i = 1; i < Q; i++) {
                    long y = neighbour(s, id, s->L.c[i]);
                    if (s->solid[y]) continue;
                    nb[nf] = y;
                    wn[nf] = s->L.w[i];
                    axis[nf] = abs(s->L.c[i][0]) + abs(s->L.c[i][1]) + abs(s->L.c[i][2]) == 1;
                    naxis += axis[nf];
                    nf++;
                }
                const int axis_only = nf > nc;
                if (axis_only && naxis == 0) FAIL("ghost with no fluid probe corner and too many diagonal fluid neighbours");
                double wsum = 0.0;
                int k = 0;
                for (int j = 0; j < nf; j++) {
                    if (axis_only && !axis[j]) continue;
                    s->corner[ng * 8 + k] = nb[j];
                    s->cw[ng * 8 + k] = wn[j];
                    wsum += wn[j];
                    k++;
                }
                for (int j = 0; j < k; j++) s->cw[ng * 8 + j] /= wsum;
                for (; k < nc; k++) { s->corner[ng * 8 + k] = nb[0]; s->cw[ng * 8 + k] = 0.0; }
            }
        }
        s->ghost[ng++] = id;
    }
    /* Initial state (READING R-init): u = p = 0 so N_i = chi_i, B_i = phi chi_i
     * at fluid nodes; every solid node starts at (1 + cos theta)/2. */
    double phi_solid = 0.5 * (1.0 + cos(P->theta_deg * pi / 180.0));
    for (long id = 0; id < n; id++) {
        if (s->solid[id]) { s->phi_state[id] = phi_solid; continue; }
        double ph = phi_init[id];
        for (int i = 0; i < Q; i++) {
            s->N[(long)i * n + id] = s->L.chi[i];
            s->B[(long)i * n + id] = ph * s->L.chi[i];
        }
    }
    return s;
#undef FAIL
}

/* One full time step (S1 ... S10). */
static void step_once(orc_sim* s) {
    long n = s->n;
    int Q = s->L.Q;
    colour_field(s);
#pragma omp parallel for schedule(static)
    for (long x = 0; x < n; x++) {
        if (s->solid[x]) continue;
        double N[QMAX], phi_nb[QMAX], Ns[QMAX], Bs[QMAX];
        for (int i = 0; i < Q; i++) {
            N[i] = s->N[(long)i * n + x];
            phi_nb[i] = s->phi[neighbour(s, x, s->L.c[i])];
        }
        collide_node(s, N, phi_nb, Ns, Bs, NULL);
        /* Eq. A16-A17 with halfway bounce-back at solid links (READING R-BB). */
        for (int i = 0; i < Q; i++) {
            long y = neighbour(s, x, s->L.c[i]);
            if (s->solid[y]) {
                int o = s->L.opp[i];
                s->Nn[(long)o * n + x] = Ns[i];
                s->Bn[(long)o * n + x] = Bs[i];
            } else {
                s->Nn[(long)i * n + y] = Ns[i];
                s->Bn[(long)i * n + y] = Bs[i];
            }
        }
    }
    /* The ghost values of this step are carried to the next one. */
    for (long g = 0; g < s->n_ghost; g++) s->phi_state[s->ghost[g]] = s->phi[s->ghost[g]];
    double* t = s->N; s->N = s->Nn; s->Nn = t;
    t = s->B; s->B = s->Bn; s->Bn = t;
    s->step++;
}

int orc_step(void* h, long nsteps) {
    orc_sim* s = (orc_sim*)h;
    for (long k = 0; k < nsteps; k++) step_once(s);
    return 0;
}

/* Field ids for orc_get. */
enum { F_N = 0, F_B = 1, F_PHI = 2, F_U = 3, F_P = 4, F_SOLID = 5, F_PHI_STATE = 6, F_RHO = 7, F_FORCE = 8 };

/* Macroscopic fields of the current state: the phi, u, p, F that the next
 * step would use.  The state is not modified.  Solid nodes get u = p = 0. */
int orc_get(void* h, int field, double* out) {
    orc_sim* s = (orc_sim*)h;
    long n = s->n;
    int Q = s->L.Q;
    switch (field) {
    case F_N: memcpy(out, s->N, sizeof(double) * Q * n); return 0;
    case F_B: memcpy(out, s->B, sizeof(double) * Q * n); return 0;
    case F_SOLID: for (long x = 0; x < n; x++) out[x] = s->solid[x]; return 0;
    case F_PHI_STATE: memcpy(out, s->phi_state, sizeof(double) * n); return 0;
    default: break;
    }
    colour_field(s);
    if (field == F_PHI) { memcpy(out, s->phi, sizeof(double) * n); return 0; }
    if (field != F_U && field != F_P && field != F_RHO && field != F_FORCE) return -1;
#pragma omp parallel for schedule(static)
    for (long x = 0; x < n; x++) {
        node_macro m;
        if (s->solid[x]) {
            memset(&m, 0, sizeof(m));
        } else {
            double N[QMAX], phi_nb[QMAX];
            for (int i = 0; i < Q; i++) {
                N[i] = s->N[(long)i * n + x];
                phi_nb[i] = s->phi[neighbour(s, x, s->L.c[i])];
            }
            compute_macro(s, N, phi_nb, &m);
        }
        if (field == F_U) for (int a = 0; a < 3; a++) out[(long)a * n + x] = m.u[a];
        else if (field == F_FORCE) for (int a = 0; a < 3; a++) out[(long)a * n + x] = m.F[a];
        else if (field == F_P) out[x] = m.p;
        else out[x] = m.rho;
    }
    return 0;
}

/* Geometry counts: [n_solid, n_ghost, n_links, n_fluid_boundary, step]. */
int orc_info(void* h, long* out) {
    orc_sim* s = (orc_sim*)h;
    long ns = 0, nl = 0, nfb = 0;
    for (long x = 0; x < s->n; x++) {
        if (s->solid[x]) { ns++; continue; }
        int b = 0;
        for (int i = 1; i < s->L.Q; i++)
            if (s->solid[neighbour(s, x, s->L.c[i])]) { nl++; b = 1; }
        nfb += b;
    }
    out[0] = ns; out[1] = s->n_ghost; out[2] = nl; out[3] = nfb; out[4] = s->step;
    return 0;
}

/* Ghost list with normals, corners and weights (for geometry tests). */
int orc_ghosts(void* h, long* ids, double* nrm, long* corners, double* weights) {
    orc_sim* s = (orc_sim*)h;
    for (long g = 0; g < s->n_ghost; g++) {
        long id = s->ghost[g];
        ids[g] = id;
        for (int a = 0; a < 3; a++) nrm[g * 3 + a] = s->nrm[id * 3 + a];
        for (int k = 0; k < 8; k++) { corners[g * 8 + k] = s->corner[g * 8 + k]; weights[g * 8 + k] = s->cw[g * 8 + k]; }
    }
    return 0;
}

/* Lattice tables: c [Q][3], w [Q], chi [Q], M [Q][Q]; returns Q. */
int orc_lattice(int lattice, double mobility, int* c, double* w, double* chi, double* M, double* alpha) {
    lattice_t L;
    double a;
    if (lattice_init(&L, lattice, mobility, &a)) return -1;
    for (int i = 0; i < L.Q; i++) {
        for (int k = 0; k < 3; k++) c[i * 3 + k] = L.c[i][k];
        w[i] = L.w[i];
        chi[i] = L.chi[i];
        for (int j = 0; j < L.Q; j++) M[i * L.Q + j] = L.M[i][j];
    }
    *alpha = a;
    return L.Q;
}

/* Equilibrium (Eq. A4) with the lattice of a sim. */
int orc_equilibrium(void* h, const double* u, double p, double* neq) {
    orc_sim* s = (orc_sim*)h;
    equilibrium(&s->L, u, p, neq);
    return 0;
}

/* One isolated node: N [Q], phi_nb [Q] = phi(x + c_i) -> N*, B*, and the
 * macroscopic record [phi, grad(3), lap, rho, nu, tau, u0(3), p, F(3), u(3),
 * Fs(3), Fp(3), Fv(3), Fb(3)]  (30 values). */
int orc_node(void* h, const double* N, const double* phi_nb, double* Nstar, double* Bstar, double* rec) {
    orc_sim* s = (orc_sim*)h;
    node_macro m;
    collide_node(s, N, phi_nb, Nstar, Bstar, &m);
    double* r = rec;
    *r++ = m.phi;
    for (int a = 0; a < 3; a++) *r++ = m.grad[a];
    *r++ = m.lap; *r++ = m.rho; *r++ = m.nu; *r++ = m.tau;
    for (int a = 0; a < 3; a++) *r++ = m.u0[a];
    *r++ = m.p;
    for (int a = 0; a < 3; a++) *r++ = m.F[a];
    for (int a = 0; a < 3; a++) *r++ = m.u[a];
    for (int a = 0; a < 3; a++) *r++ = m.Fs[a];
    for (int a = 0; a < 3; a++) *r++ = m.Fp[a];
    for (int a = 0; a < 3; a++) *r++ = m.Fv[a];
    for (int a = 0; a < 3; a++) *r++ = m.Fb[a];
    return 0;
}

/* Scalars of a sim: [alpha, eps, exp(eps), nu_l, nu_g]. */
int orc_scalars(void* h, double* out) {
    orc_sim* s = (orc_sim*)h;
    out[0] = s->alpha; out[1] = s->eps; out[2] = s->exp_eps; out[3] = s->nu_l; out[4] = s->nu_g;
    return 0;
}

/* Replace the state (N, B at fluid nodes, phi at solid nodes). */
int orc_set_state(void* h, const double* N, const double* B, const double* phi_state) {
    orc_sim* s = (orc_sim*)h;
    long n = s->n;
    int Q = s->L.Q;
    if (N) memcpy(s->N, N, sizeof(double) * Q * n);
    if (B) memcpy(s->B, B, sizeof(double) * Q * n);
    if (phi_state) memcpy(s->phi_state, phi_state, sizeof(double) * n);
    return 0;
}

/* Select an alternative reading or a planted mistake (see orc_sim):
 * which 0 = visc (0..3), 1 = seg (0..1).  Returns -1 for an unknown one. */
int orc_set_variant(void* h, int which, int value) {
    orc_sim* s = (orc_sim*)h;
    if (which == 0 && value >= 0 && value <= 3) s->visc_variant = value;
    else if (which == 1 && value >= 0 && value <= 1) s->seg_variant = value;
    else return -1;
    return 0;
}

int orc_set_theta(void* h, double theta_deg) {
    orc_sim* s = (orc_sim*)h;
    if (!(theta_deg >= 0.0 && theta_deg <= 180.0)) return -1;
    const double pi = 3.14159265358979323846;
    s->P.theta_deg = theta_deg;
    s->eps = -4.0 / s->P.W * cos(theta_deg * pi / 180.0);
    s->exp_eps = exp(s->eps);
    return 0;
}
