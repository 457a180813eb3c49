// api.cpp -- host side of the library: parameter checks, geometry
// preprocessing (solid set, ghost list, probe-point interpolation), carving
// of the caller's device buffer, and the C ABI of include/lbm.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lattice.h"
#include "launch.h"

using namespace lbm;

struct lbm_ctx {
    lbm_params P;
    int D = 0, Q = 0, NC = 0;
    int64_t n = 0, S = 0;
    StepParams sp{};
    double theta = -1.0;
    bool geometry = false, bound = false, wetting = false, started = false;
    std::vector<uint8_t> flags;
    std::vector<int32_t> g_node, g_corner;  // corner: [NC][ng]
    std::vector<double> g_w;                // [NC][ng]
    std::vector<uint8_t> g_mask;
    int64_t n_solid = 0;
    size_t need = 0;
    char* base = nullptr;
    int device = 0;       // device of the bound buffer
    hipStream_t stream = nullptr;
    DevState d{};
    int cur = 0;   // population / compact-record buffer holding the state
    int ps = 0;    // phi buffer holding the solid values of the state
    int liq = LIQ_PLANES; // liquid state entering the next step (Liquid)
    hipStream_t cap_stream = nullptr;               // private stream for graph capture
    hipGraphExec_t graph2[2] = {nullptr, nullptr};  // two-step graphs, by buffer parity
    // Fluid-only layout (LBM_OPT_SPARSE): slots are the fluid nodes, the
    // ghost nodes, then one slot for every other solid node.
    bool sparse = false;
    int64_t M = 0;                     // slots
    std::vector<int32_t> slot_of;      // [n] slot of each node
    std::vector<int32_t> node_of;      // [M - 1] node of each fluid / ghost slot
    std::vector<uint8_t> slot_flags;   // [M]
    std::vector<uint32_t> nbt;         // [Q - 1][n_fluid] slot of fluid slot k + c_i
    std::vector<double> stage;         // [M] host staging of one plane
    std::vector<int32_t> up_node, up_corner;  // slot-mapped ghost list, alive until its upload completes
    int64_t step = 0;
    std::string err;
};

static thread_local std::string g_create_error;

static int fail(lbm_ctx* c, int code, const std::string& msg) {
    if (c) c->err = msg;
    else g_create_error = msg;
    return code;
}

static int hip_fail(lbm_ctx* c, hipError_t e, const char* where) {
    return fail(c, LBM_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIPCHK(ctx, expr, where)                        \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, where); \
    } while (0)

static void lattice_table(int lattice, int& D, int& Q, int& NC, const int (**c)[3], const double** w) {
    if (lattice == LBM_D2Q9) {
        D = LatD2Q9::D; Q = LatD2Q9::Q; NC = LatD2Q9::NC;
        *c = LatD2Q9::c; *w = LatD2Q9::w;
    } else {
        D = LatD3Q19::D; Q = LatD3Q19::Q; NC = LatD3Q19::NC;
        *c = LatD3Q19::c; *w = LatD3Q19::w;
    }
}

// Plane stride of the per-node fields: n rounded up to 128 (planes of 2-,
// 4- and 8-byte values stay 256-byte aligned), plus 128 so that the planes
// of a power-of-two box do not start at power-of-two distances (measured
// on the 256^3 box: 1 to 2 % per step).
static int64_t plane_stride(int64_t n) { return (n + 127) / 128 * 128 + 128; }

// bytes of one stored population, and of every other per-node value
static size_t elem_size(uint32_t prec) { return prec == LBM_FP64 ? 8 : (prec == LBM_FP32 ? 4 : 2); }
static size_t phi_size(uint32_t prec) { return prec == LBM_FP64 ? 8 : 4; }
static size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

// Device bytes of the collide-colour inbox of this run (0 unless its steps
// take the collide-colour form).
static size_t fused_cross_bytes(const lbm_ctx* c) {
    if (!(c->P.options & LBM_OPT_FUSED) || c->sparse) return 0;
    // the collide-colour kernel addresses all Q population planes with one
    // 32-bit byte offset from the buffer's base
    if ((uint64_t)c->Q * (uint64_t)c->S * elem_size(c->P.precision) > 0xFFFFFFFFull) return 0;
    return cross_bytes((int)c->P.lattice, c->P.precision, c->sp);
}

extern "C" {

int lbm_lattice(uint32_t lattice, int32_t* c_out, int32_t* q_out) {
    if (lattice != LBM_D2Q9 && lattice != LBM_D3Q19) return LBM_EINVAL;
    if (!c_out || !q_out) return LBM_EINVAL;
    int D, Q, NC;
    const int(*c)[3];
    const double* w;
    lattice_table((int)lattice, D, Q, NC, &c, &w);
    for (int i = 0; i < Q; i++)
        for (int a = 0; a < 3; a++) c_out[i * 3 + a] = c[i][a];
    *q_out = Q;
    return LBM_OK;
}

// Captured two-step graphs hold the kernel arguments of the moment they
// were captured (eps, pointers); any call that changes state drops them.
static void drop_graphs(lbm_ctx* c) {
    for (int k = 0; k < 2; k++) {
        if (c->graph2[k]) (void)hipGraphExecDestroy(c->graph2[k]);
        c->graph2[k] = nullptr;
    }
}

// The two steps from buffer parity c->cur as one graph (captured on a
// private stream, launched on the bound one), or nullptr to fall back to
// plain launches.
static hipGraphExec_t two_step_graph(lbm_ctx* c) {
    hipGraphExec_t& ge = c->graph2[c->cur & 1];
    if (ge) return ge;
    if (!c->cap_stream && hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        (void)hipGetLastError();
        c->cap_stream = nullptr;
        return nullptr;
    }
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        // both steps enter in the state the run's own steps leave
        const int liq = step_fused((int)c->P.lattice, c->d, c->sp) ? LIQ_PHI : LIQ_RECORD;
        hipError_t e1 = launch_step((int)c->P.lattice, c->P.precision, c->d, c->sp, c->cur, c->ps, liq, c->cap_stream);
        hipError_t e2 = e1 == hipSuccess ? launch_step((int)c->P.lattice, c->P.precision, c->d, c->sp, c->cur ^ 1,
                                                       c->ps ^ 1, liq, c->cap_stream)
                                         : e1;
        e = hipStreamEndCapture(c->cap_stream, &g);
        if (e == hipSuccess) e = e2;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        ge = nullptr;
    }
    return ge;
}

int lbm_create(const lbm_params* P, lbm_ctx** out) {
    if (!P || !out) return fail(nullptr, LBM_EINVAL, "null argument");
    *out = nullptr;
    if (P->abi_version != LBM_ABI_VERSION) return fail(nullptr, LBM_EINVAL, "abi_version mismatch");
    if (P->lattice != LBM_D2Q9 && P->lattice != LBM_D3Q19) return fail(nullptr, LBM_EINVAL, "unknown lattice");
    if (P->precision > LBM_BF16_OFS) return fail(nullptr, LBM_EINVAL, "unknown precision");
    if (P->ghost_rule > LBM_GHOST_FAKHARI) return fail(nullptr, LBM_EINVAL, "unknown ghost rule");
    if (P->n[0] < 1 || P->n[1] < 1 || P->n[2] < 1) return fail(nullptr, LBM_EINVAL, "box sizes must be >= 1");
    if (P->lattice == LBM_D2Q9 && P->n[2] != 1) return fail(nullptr, LBM_EINVAL, "D2Q9 needs n[2] == 1");
    if (P->n[1] > 65535 || P->n[2] > 65535) return fail(nullptr, LBM_EINVAL, "n[1], n[2] must be <= 65535");
    const int64_t n = (int64_t)P->n[0] * P->n[1] * P->n[2];
    if (n > 2147483647LL) return fail(nullptr, LBM_EINVAL, "more than 2^31-1 nodes");
    if (!(P->rho_l > 0) || !(P->rho_g > 0) || !(P->mu_l > 0) || !(P->mu_g > 0))
        return fail(nullptr, LBM_EINVAL, "densities and viscosities must be > 0");
    if (!(P->sigma >= 0)) return fail(nullptr, LBM_EINVAL, "sigma must be >= 0");
    if (!(P->W >= 4.0)) return fail(nullptr, LBM_EINVAL, "W must be >= 4 (|eps| <= 1)");
    if (!(P->mobility > 0)) return fail(nullptr, LBM_EINVAL, "mobility must be > 0");
    for (int a = 0; a < 3; a++)
        if (!std::isfinite(P->body_accel[a])) return fail(nullptr, LBM_EINVAL, "body_accel not finite");
    const int32_t known = LBM_OPT_FUSED | LBM_OPT_FLUID_PROBE | LBM_OPT_GRAPH | LBM_OPT_FILL_DEAD_ENDS | LBM_OPT_SPARSE;
    if (P->options & ~known) return fail(nullptr, LBM_EINVAL, "unknown option bits");
    if ((P->options & LBM_OPT_SPARSE) && (P->options & LBM_OPT_FUSED))
        return fail(nullptr, LBM_EINVAL, "LBM_OPT_SPARSE excludes LBM_OPT_FUSED");

    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(nullptr, LBM_ENOMEM, "host allocation failed");
    c->P = *P;
    c->sparse = (P->options & LBM_OPT_SPARSE) != 0;
    const int(*cv)[3];
    const double* w;
    lattice_table((int)P->lattice, c->D, c->Q, c->NC, &cv, &w);
    c->n = n;
    c->S = plane_stride(n);
    // The kernels address a field plane with 32-bit byte offsets.
    if ((uint64_t)c->S * std::max(elem_size(P->precision), phi_size(P->precision)) > 0xFFFFFFFFull) {
        delete c;
        return fail(nullptr, LBM_EINVAL, "box too large: one field plane must stay below 4 GiB");
    }
    const double cs2 = 1.0 / 3.0;
    // Colour weights (Eq. A7): chi_0 = alpha, chi_i = (1 - alpha) w_i / (1 - w_0),
    // alpha from M_phi = (dt/2) [sum_i chi_i c_ix^2 + p] at p = 0.
    const double alpha = 1.0 - 2.0 * P->mobility * (1.0 - w[0]) / cs2;
    if (!(alpha >= 0.0 && alpha < 1.0)) {
        delete c;
        return fail(nullptr, LBM_EINVAL, "mobility gives alpha outside [0, 1)");
    }
    StepParams& sp = c->sp;
    sp.rho_l = P->rho_l;
    sp.rho_g = P->rho_g;
    const double nu_l = P->mu_l / P->rho_l, nu_g = P->mu_g / P->rho_g;
    sp.inv_nu_l = 1.0 / nu_l;
    sp.inv_nu_g = 1.0 / nu_g;
    if (!(0.5 + nu_l / cs2 > 0.5) || !(0.5 + nu_g / cs2 > 0.5)) {
        delete c;
        return fail(nullptr, LBM_EINVAL, "tau must exceed 1/2");
    }
    sp.sigma = P->sigma;
    sp.W = P->W;
    for (int a = 0; a < 3; a++) sp.g[a] = P->body_accel[a];
    for (int i = 0; i < 19; i++) sp.chi[i] = 0.0;
    sp.chi[0] = alpha;
    for (int i = 1; i < c->Q; i++) sp.chi[i] = (1.0 - alpha) * w[i] / (1.0 - w[0]);
    sp.chi0 = alpha;
    sp.ghost_rule = (int32_t)P->ghost_rule;
    sp.nx = P->n[0];
    sp.ny = P->n[1];
    sp.nz = P->n[2];
    sp.n = n;
    sp.S = c->S;
    *out = c;
    return LBM_OK;
}

int lbm_set_geometry(lbm_ctx* c, const lbm_solid* solids, int32_t count) {
    if (!c) return LBM_EINVAL;
    if (c->geometry) return fail(c, LBM_ESTATE, "geometry already set");
    if (count < 0 || (count > 0 && !solids)) return fail(c, LBM_EINVAL, "bad solid list");
    const int nx = c->P.n[0], ny = c->P.n[1], nz = c->P.n[2];
    const int D = c->D, Q = c->Q, NC = c->NC;
    const int(*cv)[3];
    const double* w;
    int d_, q_, nc_;
    lattice_table((int)c->P.lattice, d_, q_, nc_, &cv, &w);
    for (int k = 0; k < count; k++) {
        const lbm_solid& s = solids[k];
        if (s.kind > 1) return fail(c, LBM_EINVAL, "unknown solid kind");
        if (s.kind == 0) {
            if (!(s.radius >= 0)) return fail(c, LBM_EINVAL, "ball radius must be >= 0");
            const int dims[3] = {nx, ny, nz};
            for (int a = 0; a < D; a++)
                if (!(2.0 * s.radius < dims[a])) return fail(c, LBM_EINVAL, "ball wider than the box");
        } else {
            double len = 0;
            for (int a = 0; a < D; a++) len += s.normal[a] * s.normal[a];
            if (!(len > 0)) return fail(c, LBM_EINVAL, "half-space normal is zero");
        }
    }
    const int64_t n = c->n;
    std::vector<int32_t> owner;
    try {
        c->flags.assign((size_t)n, 0);
        owner.assign((size_t)n, -1);
    } catch (...) {
        return fail(c, LBM_ENOMEM, "host allocation failed");
    }
    auto id_of = [&](int64_t x, int64_t y, int64_t z) { return x + (int64_t)nx * (y + (int64_t)ny * z); };
    auto wrapi = [](int64_t v, int64_t m) { v %= m; return v < 0 ? v + m : v; };
    // Rasterise in list order; the first primitive holding a node owns it.
    for (int k = 0; k < count; k++) {
        const lbm_solid& s = solids[k];
        if (s.kind == 0) {
            const double r = s.radius;
            int64_t lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
            const int dims[3] = {nx, ny, nz};
            for (int a = 0; a < D; a++) {
                lo[a] = (int64_t)std::floor(s.center[a] - r) - 1;
                hi[a] = (int64_t)std::ceil(s.center[a] + r) + 1;
                if (hi[a] - lo[a] + 1 > dims[a]) { lo[a] = 0; hi[a] = dims[a] - 1; }
            }
            for (int64_t z = lo[2]; z <= hi[2]; z++)
                for (int64_t y = lo[1]; y <= hi[1]; y++)
                    for (int64_t x = lo[0]; x <= hi[0]; x++) {
                        const int64_t X = wrapi(x, nx), Y = wrapi(y, ny), Z = D == 3 ? wrapi(z, nz) : 0;
                        const int64_t id = id_of(X, Y, Z);
                        if (owner[id] >= 0) continue;
                        // minimum-image displacement from the centre
                        double dv[3] = {0, 0, 0};
                        const double pos[3] = {(double)X, (double)Y, (double)Z};
                        for (int a = 0; a < D; a++) {
                            const double L = (double)dims[a];
                            double dd = pos[a] - s.center[a];
                            dd -= L * std::floor(dd / L + 0.5);
                            dv[a] = dd;
                        }
                        if (dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2] <= r * r) owner[id] = k;
                    }
        } else {
            for (int64_t z = 0; z < nz; z++)
                for (int64_t y = 0; y < ny; y++)
                    for (int64_t x = 0; x < nx; x++) {
                        const int64_t id = id_of(x, y, z);
                        if (owner[id] >= 0) continue;
                        double v = (x - s.center[0]) * s.normal[0] + (y - s.center[1]) * s.normal[1];
                        if (D == 3) v += (z - s.center[2]) * s.normal[2];
                        if (v <= 0.0) owner[id] = k;
                    }
        }
    }
    if (c->P.options & LBM_OPT_FILL_DEAD_ENDS) {
        // Fluid nodes joined to the other fluid nodes by at most one lattice
        // link become solid (owner -2), pass after pass until none is left.
        std::vector<int64_t> dead;
        for (;;) {
            dead.clear();
            for (int64_t z = 0; z < nz; z++)
                for (int64_t y = 0; y < ny; y++)
                    for (int64_t x = 0; x < nx; x++) {
                        const int64_t id = id_of(x, y, z);
                        if (owner[id] != -1) continue;
                        int open = 0;
                        for (int i = 1; i < Q && open < 2; i++) {
                            const int64_t nb = id_of(wrapi(x + cv[i][0], nx), wrapi(y + cv[i][1], ny),
                                                     D == 3 ? wrapi(z + cv[i][2], nz) : 0);
                            open += owner[nb] == -1 ? 1 : 0;
                        }
                        if (open < 2) dead.push_back(id);
                    }
            if (dead.empty()) break;
            for (int64_t id : dead) owner[id] = -2;
        }
    }
    int64_t nsolid = 0;
    for (int64_t id = 0; id < n; id++)
        if (owner[id] != -1) { c->flags[id] = FLAG_SOLID; nsolid++; }
    c->n_solid = nsolid;
    // Node classes from the lattice stencil.
    std::vector<int64_t> ghosts;
    for (int64_t z = 0; z < nz; z++)
        for (int64_t y = 0; y < ny; y++)
            for (int64_t x = 0; x < nx; x++) {
                const int64_t id = id_of(x, y, z);
                const bool solid = c->flags[id] & FLAG_SOLID;
                bool other = false;
                for (int i = 1; i < Q && !other; i++) {
                    const int64_t nb = id_of(wrapi(x + cv[i][0], nx), wrapi(y + cv[i][1], ny),
                                             D == 3 ? wrapi(z + cv[i][2], nz) : 0);
                    other = ((c->flags[nb] & FLAG_SOLID) != 0) != solid;
                }
                if (other) {
                    if (solid) {
                        c->flags[id] |= FLAG_GHOST;
                        ghosts.push_back(id);
                    } else {
                        c->flags[id] |= FLAG_NEAR_SOLID;
                    }
                }
            }
    const int64_t ng = (int64_t)ghosts.size();
    c->g_node.resize(ng);
    c->g_corner.resize((size_t)ng * NC);
    c->g_w.resize((size_t)ng * NC);
    c->g_mask.resize(ng);
    for (int64_t g = 0; g < ng; g++) {
        const int64_t id = ghosts[g];
        const int64_t x = id % nx, y = (id / nx) % ny, z = id / ((int64_t)nx * ny);
        // Solid normal n_s pointing out of the solid (Eq. 7).  A filled
        // dead-end node has one fluid neighbour left: n_s points to it.
        double nv[3] = {0, 0, 0};
        if (owner[id] == -2) {
            for (int i = 1; i < Q; i++) {
                const int64_t nb = id_of(wrapi(x + cv[i][0], nx), wrapi(y + cv[i][1], ny),
                                         D == 3 ? wrapi(z + cv[i][2], nz) : 0);
                if (!(c->flags[nb] & FLAG_SOLID))
                    for (int a = 0; a < 3; a++) nv[a] = cv[i][a];
            }
        } else if (solids[owner[id]].kind == 0) {
            const lbm_solid& s = solids[owner[id]];
            const int dims[3] = {nx, ny, nz};
            const double pos[3] = {(double)x, (double)y, (double)z};
            for (int a = 0; a < D; a++) {
                const double L = (double)dims[a];
                double dd = pos[a] - s.center[a];
                dd -= L * std::floor(dd / L + 0.5);
                nv[a] = dd;
            }
        } else {
            for (int a = 0; a < D; a++) nv[a] = solids[owner[id]].normal[a];
        }
        double len = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
        if (len > 0) {
            for (int a = 0; a < 3; a++) nv[a] /= len;
        } else {
            nv[0] = nv[1] = nv[2] = 0;
            nv[D - 1] = 1.0;  // node at a ball centre: any unit vector
        }
        // Probe point x_F = x_G + dx n_s and its bi/trilinear cell.
        const double xf[3] = {x + nv[0], y + nv[1], z + nv[2]};
        int64_t base[3];
        double fr[3];
        for (int a = 0; a < 3; a++) {
            const double fl = std::floor(xf[a]);
            base[a] = (int64_t)fl;
            fr[a] = xf[a] - fl;
        }
        if (D == 2) { base[2] = z; fr[2] = 0.0; }
        uint8_t mask = 0;
        for (int k = 0; k < NC; k++) {
            const int bx = k & 1, by = (k >> 1) & 1, bz = (k >> 2) & 1;
            const int64_t cid = id_of(wrapi(base[0] + bx, nx), wrapi(base[1] + by, ny),
                                      D == 3 ? wrapi(base[2] + bz, nz) : 0);
            double wt = (bx ? fr[0] : 1.0 - fr[0]) * (by ? fr[1] : 1.0 - fr[1]);
            if (D == 3) wt *= (bz ? fr[2] : 1.0 - fr[2]);
            c->g_corner[(size_t)k * ng + g] = (int32_t)cid;
            c->g_w[(size_t)k * ng + g] = wt;
            if (c->flags[cid] & FLAG_SOLID) mask |= (uint8_t)(1u << k);
        }
        if (c->P.options & LBM_OPT_FLUID_PROBE) {
            // phi_F from the fluid corners only, weights rescaled to sum 1.
            double wf = 0.0;
            for (int k = 0; k < NC; k++)
                if (!((mask >> k) & 1u)) wf += c->g_w[(size_t)k * ng + g];
            if (wf > 0.0) {
                for (int k = 0; k < NC; k++) {
                    double& wk = c->g_w[(size_t)k * ng + g];
                    wk = ((mask >> k) & 1u) ? 0.0 : wk / wf;
                }
            } else {
                // The probe cell lies wholly in solid (a ghost in the gap
                // between touching solids): phi_F from the ghost's fluid
                // lattice neighbours, weighted by w_i and rescaled to sum 1;
                // the axis neighbours alone when there are more than NC.
                int64_t nb_id[32];
                double nb_w[32];
                bool nb_axis[32];
                int nf = 0, naxis = 0;
                for (int i = 1; i < Q; i++) {
                    const int64_t nb = id_of(wrapi(x + cv[i][0], nx), wrapi(y + cv[i][1], ny),
                                             D == 3 ? wrapi(z + cv[i][2], nz) : 0);
                    if (c->flags[nb] & FLAG_SOLID) continue;
                    nb_id[nf] = nb;
                    nb_w[nf] = w[i];
                    nb_axis[nf] = std::abs(cv[i][0]) + std::abs(cv[i][1]) + std::abs(cv[i][2]) == 1;
                    naxis += nb_axis[nf] ? 1 : 0;
                    nf++;
                }
                const bool axis_only = nf > NC;
                if (axis_only && naxis == 0)
                    return fail(c, LBM_EINVAL, "ghost node whose probe has no fluid corner and more diagonal "
                                                "fluid neighbours than interpolation slots");
                int k = 0;
                double sum = 0.0;
                for (int j = 0; j < nf; j++) {
                    if (axis_only && !nb_axis[j]) continue;
                    c->g_corner[(size_t)k * ng + g] = (int32_t)nb_id[j];
                    c->g_w[(size_t)k * ng + g] = nb_w[j];
                    sum += nb_w[j];
                    k++;
                }
                for (int j = 0; j < k; j++) c->g_w[(size_t)j * ng + g] /= sum;
                for (; k < NC; k++) {
                    c->g_corner[(size_t)k * ng + g] = (int32_t)nb_id[0];
                    c->g_w[(size_t)k * ng + g] = 0.0;
                }
                mask = 0;   // every slot now names a fluid node
            }
        }
        c->g_node[g] = (int32_t)id;
        c->g_mask[g] = mask;
    }
    if (c->sparse) {
        // Slots: fluid nodes, ghost nodes in list order, then the slot of
        // every other solid node.
        const int64_t nf = n - nsolid;
        const int64_t M = nf + ng + 1;
        if ((uint64_t)((M + 127) / 128 * 128) * std::max(elem_size(c->P.precision), phi_size(c->P.precision)) >
                0xFFFFFFFFull ||
            (uint64_t)(Q - 1) * (uint64_t)nf > 0x7FFFFFFFFFFFull)
            return fail(c, LBM_EINVAL, "sparse layout too large");
        try {
            c->slot_of.assign((size_t)n, (int32_t)(M - 1));
            c->node_of.assign((size_t)(M - 1), 0);
            c->slot_flags.assign((size_t)M, FLAG_SOLID);
            c->nbt.assign((size_t)(Q - 1) * (size_t)nf, 0);
        } catch (...) {
            return fail(c, LBM_ENOMEM, "host allocation failed");
        }
        int64_t k = 0;
        auto take = [&](int64_t id) {
            if (c->flags[id] & FLAG_SOLID) return;
            c->slot_of[id] = (int32_t)k;
            c->node_of[k] = (int32_t)id;
            k++;
        };
        // fluid slots in box order: the +-x neighbours are adjacent slots
        // and the +-y neighbours contiguous runs (numbering them brick by
        // brick measured slower)
        for (int64_t id = 0; id < n; id++) take(id);
        for (int64_t g = 0; g < ng; g++) {
            c->slot_of[ghosts[g]] = (int32_t)(nf + g);
            c->node_of[nf + g] = (int32_t)ghosts[g];
        }
        for (int64_t sl = 0; sl < M - 1; sl++) c->slot_flags[sl] = c->flags[c->node_of[sl]];
        for (int64_t f = 0; f < nf; f++) {
            const int64_t id = c->node_of[f];
            const int64_t x = id % nx, y = (id / nx) % ny, z = id / ((int64_t)nx * ny);
            for (int i = 1; i < Q; i++) {
                const int64_t nb = id_of(wrapi(x + cv[i][0], nx), wrapi(y + cv[i][1], ny),
                                         D == 3 ? wrapi(z + cv[i][2], nz) : 0);
                // bit 31 marks a solid neighbour (a bounce-back link); the
                // size check above keeps slots below 2^30
                c->nbt[(size_t)(i - 1) * nf + f] =
                    (uint32_t)c->slot_of[nb] | ((c->flags[nb] & FLAG_SOLID) ? 0x80000000u : 0u);
            }
        }
        c->M = M;
        c->S = plane_stride(M);
        c->sp.n = M;
        c->sp.S = c->S;
    }
    // Device layout (all 256-byte aligned).
    const size_t es = elem_size(c->P.precision), fs = phi_size(c->P.precision);
    const size_t plane = align256((size_t)c->S * es), tplane = align256((size_t)c->S * fs);
    size_t off = 0;
    off += 2 * (size_t)Q * plane;                       // N[2]
    off += (size_t)Q * tplane;                          // B
    off += 2 * (size_t)(D + 1) * tplane;                // G[2]
    off += 2 * align256((size_t)c->S * fs);             // phi[2]
    off += align256((size_t)(c->sparse ? c->M : n));    // flags
    off += align256((size_t)ng * 4);                    // g_node
    off += align256((size_t)ng * NC * 4);               // g_corner
    off += align256((size_t)ng * NC * fs);              // g_w
    off += align256((size_t)ng);                        // g_mask
    off += align256(c->nbt.size() * 4);                 // neighbour slots (sparse layout)
    off += align256(fused_cross_bytes(c));              // collide-colour inbox
    off += 4 * align256((size_t)c->S * 8);              // aux
    off += align256((size_t)REDUCE_BLOCKS * 8 * 8);     // partial
    off += align256(8 * 8);                             // result
    off += align256((size_t)(REDUCE_BLOCKS + 1) * 8);   // nonfinite
    c->need = off;
    c->geometry = true;
    return LBM_OK;
}

int lbm_device_bytes(const lbm_ctx* c, size_t* bytes) {
    if (!c || !bytes) return LBM_EINVAL;
    if (!c->geometry) return fail(const_cast<lbm_ctx*>(c), LBM_ESTATE, "set the geometry first");
    *bytes = c->need;
    return LBM_OK;
}

int lbm_bind(lbm_ctx* c, void* dev, size_t bytes, void* stream) {
    if (!c) return LBM_EINVAL;
    if (!c->geometry) return fail(c, LBM_ESTATE, "set the geometry before binding");
    if (c->bound) return fail(c, LBM_ESTATE, "already bound");
    if (!dev) return fail(c, LBM_EINVAL, "null device pointer");
    if (((uintptr_t)dev) & 255u) return fail(c, LBM_EINVAL, "device buffer must be 256-byte aligned");
    if (bytes < c->need) return fail(c, LBM_ENOMEM, "device buffer smaller than lbm_device_bytes()");
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, dev) != hipSuccess || attr.type != hipMemoryTypeDevice) {
        (void)hipGetLastError();
        return fail(c, LBM_EINVAL, "buffer is not device memory");
    }
    c->base = (char*)dev;
    c->device = attr.device;
    c->stream = (hipStream_t)stream;
    const int Q = c->Q, NC = c->NC;
    const int64_t ng = (int64_t)c->g_node.size();
    const size_t es = elem_size(c->P.precision), fs = phi_size(c->P.precision);
    const size_t plane = align256((size_t)c->S * es), tplane = align256((size_t)c->S * fs);
    char* p = c->base;
    DevState& d = c->d;
    for (int b = 0; b < 2; b++) { d.N[b] = p; p += (size_t)Q * plane; }
    d.B = p; p += (size_t)Q * tplane;
    for (int b = 0; b < 2; b++) { d.G[b] = p; p += (size_t)(c->D + 1) * tplane; }
    for (int b = 0; b < 2; b++) { d.phi[b] = p; p += align256((size_t)c->S * fs); }
    d.flags = (uint8_t*)p; p += align256((size_t)(c->sparse ? c->M : c->n));
    d.g_node = (int32_t*)p; p += align256((size_t)ng * 4);
    d.g_corner = (int32_t*)p; p += align256((size_t)ng * NC * 4);
    d.g_w = p; p += align256((size_t)ng * NC * fs);
    d.g_mask = (uint8_t*)p; p += align256((size_t)ng);
    d.nbt = (uint32_t*)p; p += align256(c->nbt.size() * 4);
    d.cross = p; p += align256(fused_cross_bytes(c));
    d.aux = (double*)p; p += 4 * align256((size_t)c->S * 8);
    d.partial = (double*)p; p += align256((size_t)REDUCE_BLOCKS * 8 * 8);
    d.result = (double*)p; p += align256(8 * 8);
    d.nonfinite = (int64_t*)p; p += align256((size_t)(REDUCE_BLOCKS + 1) * 8);
    d.n_ghost = (int32_t)ng;
    d.fused = fused_cross_bytes(c) > 0 ? 1 : 0;
    d.n_fluid = c->n - c->n_solid;
    d.sparse = c->sparse ? 1 : 0;
    // Upload the geometry (slot-indexed in the sparse layout).
    hipStream_t st = c->stream;
    const int32_t* g_node_src = c->g_node.data();
    const int32_t* g_corner_src = c->g_corner.data();
    if (c->sparse) {
        // kept in the context: an error return below may leave copies pending
        c->up_node.resize(c->g_node.size());
        c->up_corner.resize(c->g_corner.size());
        for (size_t k = 0; k < c->up_node.size(); k++) c->up_node[k] = c->slot_of[c->g_node[k]];
        for (size_t k = 0; k < c->up_corner.size(); k++) c->up_corner[k] = c->slot_of[c->g_corner[k]];
        g_node_src = c->up_node.data();
        g_corner_src = c->up_corner.data();
        HIPCHK(c, hipMemcpyAsync(d.flags, c->slot_flags.data(), (size_t)c->M, hipMemcpyHostToDevice, st),
               "upload flags");
        if (!c->nbt.empty())
            HIPCHK(c, hipMemcpyAsync(d.nbt, c->nbt.data(), c->nbt.size() * 4, hipMemcpyHostToDevice, st),
                   "upload neighbour slots");
    } else {
        HIPCHK(c, hipMemcpyAsync(d.flags, c->flags.data(), (size_t)c->n, hipMemcpyHostToDevice, st), "upload flags");
    }
    if (ng > 0) {
        HIPCHK(c, hipMemcpyAsync(d.g_node, g_node_src, (size_t)ng * 4, hipMemcpyHostToDevice, st), "upload ghosts");
        HIPCHK(c, hipMemcpyAsync(d.g_corner, g_corner_src, (size_t)ng * NC * 4, hipMemcpyHostToDevice, st),
               "upload corners");
        HIPCHK(c, hipMemcpyAsync(d.g_mask, c->g_mask.data(), (size_t)ng, hipMemcpyHostToDevice, st), "upload mask");
        if (c->P.precision == LBM_FP64) {
            HIPCHK(c, hipMemcpyAsync(d.g_w, c->g_w.data(), (size_t)ng * NC * 8, hipMemcpyHostToDevice, st),
                   "upload weights");
            HIPCHK(c, hipStreamSynchronize(st), "sync");
        } else {
            std::vector<float> wf(c->g_w.size());
            for (size_t k = 0; k < wf.size(); k++) wf[k] = (float)c->g_w[k];
            HIPCHK(c, hipMemcpyAsync(d.g_w, wf.data(), wf.size() * 4, hipMemcpyHostToDevice, st), "upload weights");
            HIPCHK(c, hipStreamSynchronize(st), "sync");
        }
    }
    HIPCHK(c, hipStreamSynchronize(st), "sync");
    std::vector<int32_t>().swap(c->up_node);
    std::vector<int32_t>().swap(c->up_corner);
    c->bound = true;
    return LBM_OK;
}

int lbm_set_wetting(lbm_ctx* c, double theta_deg) {
    if (!c) return LBM_EINVAL;
    if (!c->bound) return fail(c, LBM_ESTATE, "bind before setting the wetting angle");
    if (!(theta_deg >= 0.0 && theta_deg <= 180.0)) return fail(c, LBM_EINVAL, "theta must be in [0, 180]");
    const double pi = 3.14159265358979323846;
    const double ct = std::cos(theta_deg * pi / 180.0);
    drop_graphs(c);
    c->theta = theta_deg;
    c->sp.eps = -4.0 / c->P.W * ct;   // Eq. 9 with dx = 1
    c->sp.exp_eps = std::exp(c->sp.eps);
    c->sp.phi_solid = 0.5 * (1.0 + ct);
    if (!c->started || c->step == 0) {
        // Section 3: ghost (and all solid) nodes start at (1 + cos theta)/2.
        HIPCHK(c, launch_solid_phi(c->P.precision, c->d, c->sp, c->stream), "solid phi");
        HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
    }
    c->wetting = true;
    return LBM_OK;
}

// One FP64 plane of `count` = n box values into aux.  The sparse layout
// gathers it into slot order first; the slot of the non-ghost solid nodes
// takes the value of the first such node (uniform = true: all of them must
// hold that value).
static int upload_aux(lbm_ctx* c, const double* src, int64_t count, int64_t plane_off, bool uniform = false) {
    if (!c->sparse) {
        HIPCHK(c, hipMemcpyAsync(c->d.aux + plane_off, src, (size_t)count * 8, hipMemcpyHostToDevice, c->stream),
               "upload");
        return LBM_OK;
    }
    const int64_t M = c->M;
    c->stage.resize((size_t)M);
    for (int64_t sl = 0; sl < M - 1; sl++) c->stage[sl] = src[c->node_of[sl]];
    bool have = false;
    double v = 0.0;
    for (int64_t id = 0; id < count; id++) {
        if (c->slot_of[id] != M - 1) continue;
        if (!have) {
            v = src[id];
            have = true;
            if (!uniform) break;
        } else if (!(src[id] == v)) {
            return fail(c, LBM_EINVAL, "the sparse layout keeps one value for all non-ghost solid nodes");
        }
    }
    c->stage[M - 1] = have ? v : 0.0;
    HIPCHK(c, hipMemcpyAsync(c->d.aux + plane_off, c->stage.data(), (size_t)M * 8, hipMemcpyHostToDevice, c->stream),
           "upload");
    HIPCHK(c, hipStreamSynchronize(c->stream), "sync");   // the staging buffer is reused
    return LBM_OK;
}

// Plane kind of the population fields for launch_plane_in / _out.
static int n_plane_kind(int field) {
    return field == LBM_FIELD_N ? 0 : field == LBM_FIELD_B ? 1 : 3;
}

int lbm_set_field(lbm_ctx* c, int field, const double* src, size_t count) {
    if (!c) return LBM_EINVAL;
    drop_graphs(c);
    if (!c->wetting) return fail(c, LBM_ESTATE, "set geometry, bind and wetting first");
    if (!src) return fail(c, LBM_EINVAL, "null host pointer");
    const int lat = (int)c->P.lattice;
    const uint32_t prec = c->P.precision;
    const int64_t n = c->n;
    int rc;
    switch (field) {
    case LBM_FIELD_PHI:
        if (count != (size_t)n) return fail(c, LBM_EINVAL, "PHI needs n values");
        for (int64_t x = 0; x < n; x++)
            if (!std::isfinite(src[x])) return fail(c, LBM_EINVAL, "non-finite phi");
        c->cur = 0;
        c->ps = 0;
        if ((rc = upload_aux(c, src, n, 0)) != LBM_OK) return rc;
        HIPCHK(c, launch_init(lat, prec, c->d, c->sp, c->cur, c->ps, c->stream), "init");
        HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
        c->liq = LIQ_PLANES;
        c->step = 0;
        c->started = true;
        return LBM_OK;
    case LBM_FIELD_N:
    case LBM_FIELD_N_OFFSET:
    case LBM_FIELD_B:
        if (!c->started) return fail(c, LBM_ESTATE, "set PHI first");
        if (count != (size_t)c->Q * n) return fail(c, LBM_EINVAL, "N/B need Q*n values");
        if (c->liq == LIQ_RECORD) {
            // The compact liquid record depends on N: write B out to the
            // plane buffer first so that it keeps its value.
            for (int i = 0; i < c->Q; i++) {
                HIPCHK(c, launch_plane_out(lat, prec, c->d, c->sp, 1, i, c->cur, c->ps, LIQ_RECORD, c->stream),
                       "B out");
                HIPCHK(c, launch_plane_in(lat, prec, c->d, c->sp, 1, i, c->cur, c->stream), "B in");
            }
            c->liq = LIQ_PLANES;
        }
        // In LIQ_PHI the liquid state is phi itself, which N does not change;
        // setting B replaces it by the B planes.
        if (field == LBM_FIELD_B) c->liq = LIQ_PLANES;
        for (int i = 0; i < c->Q; i++) {
            if ((rc = upload_aux(c, src + (size_t)i * n, n, 0)) != LBM_OK) return rc;
            HIPCHK(c, launch_plane_in(lat, prec, c->d, c->sp, n_plane_kind(field), i, c->cur, c->stream),
                   "plane in");
        }
        HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
        return LBM_OK;
    case LBM_FIELD_PHI_STATE:
        // the colour field of the next step at fluid nodes becomes the
        // liquid state (restore of a run whose last step was collide-colour)
        if (!c->started) return fail(c, LBM_ESTATE, "set PHI first");
        if (count != (size_t)n) return fail(c, LBM_EINVAL, "PHI_STATE needs n values");
        if ((rc = upload_aux(c, src, n, 0)) != LBM_OK) return rc;
        HIPCHK(c, launch_plane_in(lat, prec, c->d, c->sp, 4, 1 - c->ps, c->cur, c->stream), "plane in");
        HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
        c->liq = LIQ_PHI;
        return LBM_OK;
    case LBM_FIELD_SOLID_PHI:
        if (!c->started) return fail(c, LBM_ESTATE, "set PHI first");
        if (count != (size_t)n) return fail(c, LBM_EINVAL, "SOLID_PHI needs n values");
        if ((rc = upload_aux(c, src, n, 0, true)) != LBM_OK) return rc;
        HIPCHK(c, launch_plane_in(lat, prec, c->d, c->sp, 2, 0, c->cur, c->stream), "plane in");
        HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
        return LBM_OK;
    default:
        return fail(c, LBM_EINVAL, "field cannot be set");
    }
}

int lbm_step(lbm_ctx* c, int64_t nsteps) {
    if (!c) return LBM_EINVAL;
    if (!c->started) return fail(c, LBM_ESTATE, "set PHI before stepping");
    if (nsteps < 0) return fail(c, LBM_EINVAL, "nsteps must be >= 0");
    const int after = step_fused((int)c->P.lattice, c->d, c->sp) ? LIQ_PHI : LIQ_RECORD;
    // With LBM_OPT_GRAPH, long runs replay a captured two-step graph (one
    // launch per two steps instead of six) after the first step of a run.
    if ((c->P.options & LBM_OPT_GRAPH) && nsteps >= 8) {
        if (c->liq != after) {
            int rc = lbm_step(c, 1);
            if (rc != LBM_OK) return rc;
            nsteps--;
        }
        const int64_t pairs = nsteps / 2;
        hipGraphExec_t ge = pairs > 0 ? two_step_graph(c) : nullptr;
        if (ge) {
            for (int64_t k = 0; k < pairs; k++) {
                hipError_t e = hipGraphLaunch(ge, c->stream);
                if (e != hipSuccess) return hip_fail(c, e, "graph launch");
            }
            c->step += 2 * pairs;
            nsteps -= 2 * pairs;
        }
    }
    for (int64_t k = 0; k < nsteps; k++) {
        hipError_t e = launch_step((int)c->P.lattice, c->P.precision, c->d, c->sp, c->cur, c->ps, c->liq, c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "step launch");
        c->cur ^= 1;
        c->ps ^= 1;
        c->liq = after;
        c->step++;
    }
    return LBM_OK;
}

int lbm_step_profiled(lbm_ctx* c, int64_t nsteps, double* ms_out) {
    if (!c || !ms_out) return LBM_EINVAL;
    if (!c->started) return fail(c, LBM_ESTATE, "set PHI before stepping");
    if (nsteps < 1) return fail(c, LBM_EINVAL, "nsteps must be >= 1");
    const int NPH = STEP_PHASES;
    const int after = step_fused((int)c->P.lattice, c->d, c->sp) ? LIQ_PHI : LIQ_RECORD;
    std::vector<hipEvent_t> ev((size_t)nsteps * (NPH + 1), nullptr);
    int rc = LBM_OK;
    for (size_t k = 0; k < ev.size(); k++) {
        hipError_t e = hipEventCreate(&ev[k]);
        if (e != hipSuccess) { rc = hip_fail(c, e, "event create"); break; }
    }
    for (int64_t s = 0; s < nsteps && rc == LBM_OK; s++) {
        hipEvent_t* E = &ev[(size_t)s * (NPH + 1)];
        hipError_t e = hipEventRecord(E[0], c->stream);
        for (int ph = 0; ph < NPH && e == hipSuccess; ph++) {
            e = launch_phase((int)c->P.lattice, c->P.precision, ph, c->d, c->sp, c->cur, c->ps, c->liq, c->stream);
            if (e == hipSuccess) e = hipEventRecord(E[ph + 1], c->stream);
        }
        if (e != hipSuccess) { rc = hip_fail(c, e, "profiled step"); break; }
        c->cur ^= 1;
        c->ps ^= 1;
        c->liq = after;
        c->step++;
    }
    if (rc == LBM_OK) {
        hipError_t e = hipEventSynchronize(ev.back());
        if (e != hipSuccess) rc = hip_fail(c, e, "event sync");
    }
    if (rc == LBM_OK) {
        double tot[NPH + 1] = {};
        for (int64_t s = 0; s < nsteps && rc == LBM_OK; s++) {
            hipEvent_t* E = &ev[(size_t)s * (NPH + 1)];
            for (int ph = 0; ph < NPH; ph++) {
                float ms = 0;
                hipError_t e = hipEventElapsedTime(&ms, E[ph], E[ph + 1]);
                if (e != hipSuccess) { rc = hip_fail(c, e, "event time"); break; }
                tot[ph] += ms;
            }
        }
        float all = 0;
        if (rc == LBM_OK && hipEventElapsedTime(&all, ev.front(), ev.back()) != hipSuccess)
            rc = fail(c, LBM_EHIP, "event time");
        for (int ph = 0; ph < NPH; ph++) ms_out[ph] = tot[ph];
        ms_out[NPH] = all;
    }
    for (hipEvent_t e : ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

// Copy the reduced diagnostics out of rs (synchronises) into *out.
static int finish_observe(lbm_ctx* c, const ReduceScratch& rs, lbm_obs* out) {
    double r[8];
    int64_t nf = 0;
    HIPCHK(c, hipMemcpyAsync(r, rs.result, 8 * 8, hipMemcpyDeviceToHost, c->stream), "download");
    HIPCHK(c, hipMemcpyAsync(&nf, rs.nonfinite + REDUCE_BLOCKS, 8, hipMemcpyDeviceToHost, c->stream), "download");
    HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
    std::memset(out, 0, sizeof(*out));
    out->step = c->step;
    out->n_solid = c->n_solid;
    out->n_fluid = c->n - c->n_solid;
    out->n_ghost = (int64_t)c->g_node.size();
    out->nonfinite = nf;
    out->mass_blue = r[0];
    out->mass_red = r[1];
    out->momentum[0] = r[2];
    out->momentum[1] = r[3];
    out->momentum[2] = r[4];
    out->max_speed = r[5];
    out->kinetic_energy = r[6];
    if (nf > 0) return fail(c, LBM_EUNSTABLE, "non-finite values in the state");
    return LBM_OK;
}

int lbm_observe(lbm_ctx* c, lbm_obs* out) {
    if (!c || !out) return LBM_EINVAL;
    if (!c->started) return fail(c, LBM_ESTATE, "set PHI before observing");
    const int lat = (int)c->P.lattice;
    const uint32_t prec = c->P.precision;
    HIPCHK(c, launch_colour(lat, prec, c->d, c->sp, c->cur, c->ps, c->liq, c->stream), "colour");
    HIPCHK(c, launch_macro(lat, prec, c->d, c->sp, c->cur, c->ps, c->stream), "macro");
    const ReduceScratch rs{c->d.partial, c->d.nonfinite, c->d.result};
    HIPCHK(c, launch_reduce(lat, prec, c->d, c->sp, c->cur, c->ps, c->liq, rs, c->stream), "reduce");
    return finish_observe(c, rs, out);
}

int lbm_observe_static(lbm_ctx* c, lbm_obs* out) {
    if (!c || !out) return LBM_EINVAL;
    if (!c->started) return fail(c, LBM_ESTATE, "set PHI before observing");
    const int lat = (int)c->P.lattice;
    const uint32_t prec = c->P.precision;
    ReduceScratch rs;
    HIPCHK(c, static_reduce_scratch(c->device, rs), "static scratch address");
    HIPCHK(c, launch_colour(lat, prec, c->d, c->sp, c->cur, c->ps, c->liq, c->stream), "colour");
    HIPCHK(c, launch_macro(lat, prec, c->d, c->sp, c->cur, c->ps, c->stream), "macro");
    HIPCHK(c, launch_reduce(lat, prec, c->d, c->sp, c->cur, c->ps, c->liq, rs, c->stream), "reduce");
    return finish_observe(c, rs, out);
}

// One FP64 plane of aux to `count` = n box values (scattered from slot
// order in the sparse layout).
static int download(lbm_ctx* c, double* dst, const double* src, int64_t count) {
    if (!c->sparse) {
        HIPCHK(c, hipMemcpyAsync(dst, src, (size_t)count * 8, hipMemcpyDeviceToHost, c->stream), "download");
        HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
        return LBM_OK;
    }
    c->stage.resize((size_t)c->M);
    HIPCHK(c, hipMemcpyAsync(c->stage.data(), src, (size_t)c->M * 8, hipMemcpyDeviceToHost, c->stream), "download");
    HIPCHK(c, hipStreamSynchronize(c->stream), "sync");
    for (int64_t id = 0; id < count; id++) dst[id] = c->stage[c->slot_of[id]];
    return LBM_OK;
}

int lbm_read_field(lbm_ctx* c, int field, double* dst, size_t count) {
    if (!c) return LBM_EINVAL;
    if (!dst) return fail(c, LBM_EINVAL, "null host pointer");
    const int64_t n = c->n;
    const int lat = (int)c->P.lattice;
    const uint32_t prec = c->P.precision;
    if (field == LBM_FIELD_FLAGS) {
        if (!c->geometry) return fail(c, LBM_ESTATE, "no geometry");
        if (count != (size_t)n) return fail(c, LBM_EINVAL, "FLAGS has n values");
        for (int64_t x = 0; x < n; x++) dst[x] = (double)c->flags[x];
        return LBM_OK;
    }
    if (!c->started) return fail(c, LBM_ESTATE, "set PHI first");
    int rc;
    switch (field) {
    case LBM_FIELD_PHI:
    case LBM_FIELD_PHI_STATE:
        if (count != (size_t)n) return fail(c, LBM_EINVAL, "PHI has n values");
        HIPCHK(c, launch_colour(lat, prec, c->d, c->sp, c->cur, c->ps, c->liq, c->stream), "colour");
        HIPCHK(c, launch_plane_out(lat, prec, c->d, c->sp, 2, 1 - c->ps, c->cur, c->ps, c->liq, c->stream),
               "plane out");
        return download(c, dst, c->d.aux, n);
    case LBM_FIELD_SOLID_PHI:
        if (count != (size_t)n) return fail(c, LBM_EINVAL, "SOLID_PHI has n values");
        HIPCHK(c, launch_plane_out(lat, prec, c->d, c->sp, 2, c->ps, c->cur, c->ps, c->liq, c->stream),
               "plane out");
        return download(c, dst, c->d.aux, n);
    case LBM_FIELD_U:
    case LBM_FIELD_P:
        if (count != (size_t)(field == LBM_FIELD_U ? 3 * n : n)) return fail(c, LBM_EINVAL, "wrong count");
        HIPCHK(c, launch_colour(lat, prec, c->d, c->sp, c->cur, c->ps, c->liq, c->stream), "colour");
        HIPCHK(c, launch_macro(lat, prec, c->d, c->sp, c->cur, c->ps, c->stream), "macro");
        if (field == LBM_FIELD_P) return download(c, dst, c->d.aux + 3 * c->S, n);
        for (int a = 0; a < 3; a++)
            if ((rc = download(c, dst + (size_t)a * n, c->d.aux + (size_t)a * c->S, n)) != LBM_OK) return rc;
        return LBM_OK;
    case LBM_FIELD_N:
    case LBM_FIELD_N_OFFSET:
    case LBM_FIELD_B:
        if (count != (size_t)c->Q * n) return fail(c, LBM_EINVAL, "N/B have Q*n values");
        if (field == LBM_FIELD_B && c->liq == LIQ_PHI)
            return fail(c, LBM_ESTATE,
                        "the collide-colour step keeps phi, not B: read B after a step without LBM_OPT_FUSED");
        for (int i = 0; i < c->Q; i++) {
            HIPCHK(c, launch_plane_out(lat, prec, c->d, c->sp, n_plane_kind(field), i, c->cur, c->ps,
                                       c->liq, c->stream),
                   "plane out");
            if ((rc = download(c, dst + (size_t)i * n, c->d.aux, n)) != LBM_OK) return rc;
        }
        return LBM_OK;
    default:
        return fail(c, LBM_EINVAL, "unknown field");
    }
}

// ------------------------------------------------------------------ batches
struct lbm_batch {
    char* table = nullptr;
    size_t bytes = 0;
    hipStream_t stream = nullptr;
    std::vector<char> staging[8];   // one per (lattice, precision) group
    std::string err;
};

static int bfail(lbm_batch* b, int code, const std::string& msg) {
    if (b) b->err = msg;
    else g_create_error = msg;
    return code;
}

int lbm_batch_table_bytes(int32_t max_jobs, size_t* bytes) {
    if (!bytes || max_jobs < 1) return LBM_EINVAL;
    *bytes = batch_table_bytes(max_jobs);
    return LBM_OK;
}

int lbm_batch_create(void* device_table, size_t bytes, void* hip_stream, lbm_batch** out) {
    if (!out) return bfail(nullptr, LBM_EINVAL, "null argument");
    *out = nullptr;
    if (!device_table) return bfail(nullptr, LBM_EINVAL, "null device table");
    if (((uintptr_t)device_table) & 255u) return bfail(nullptr, LBM_EINVAL, "device table must be 256-byte aligned");
    if (bytes < batch_table_bytes(1)) return bfail(nullptr, LBM_ENOMEM, "device table too small");
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return bfail(nullptr, LBM_ENOMEM, "host allocation failed");
    b->table = (char*)device_table;
    b->bytes = bytes;
    b->stream = (hipStream_t)hip_stream;
    *out = b;
    return LBM_OK;
}

int lbm_batch_step(lbm_batch* b, lbm_ctx* const* ctxs, const int64_t* steps, int32_t count) {
    if (!b) return LBM_EINVAL;
    if (count < 0 || (count > 0 && (!ctxs || !steps))) return bfail(b, LBM_EINVAL, "bad job list");
    if (count == 0) return LBM_OK;
    for (int32_t j = 0; j < count; j++) {
        if (!ctxs[j]) return bfail(b, LBM_EINVAL, "null context");
        if (!ctxs[j]->started) return bfail(b, LBM_ESTATE, "every context must be started (PHI set)");
        if (ctxs[j]->sparse) return bfail(b, LBM_EINVAL, "contexts with LBM_OPT_SPARSE step alone (lbm_step)");
        if (steps[j] < 0) return bfail(b, LBM_EINVAL, "steps must be >= 0");
        for (int32_t k = 0; k < j; k++)
            if (ctxs[k] == ctxs[j]) return bfail(b, LBM_EINVAL, "a context appears twice");
    }
    // The staging buffers of the previous call must have reached the device.
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bfail(b, LBM_EHIP, std::string("sync: ") + hipGetErrorString(e));
    size_t off = 0;
    int group = 0;
    for (uint32_t lat = 0; lat < 2; lat++) {
        for (uint32_t prec = 0; prec < 4; prec++) {
            std::vector<BatchJobHost> jobs;
            std::vector<lbm_ctx*> who;
            for (int32_t j = 0; j < count; j++) {
                lbm_ctx* c = ctxs[j];
                if (c->P.lattice != lat || c->P.precision != prec || steps[j] == 0) continue;
                BatchJobHost h;
                h.d = c->d;
                h.p = c->sp;
                h.cur0 = c->cur;
                h.ps0 = c->ps;
                h.planes0 = c->liq;
                h.steps = steps[j];
                jobs.push_back(h);
                who.push_back(c);
            }
            if (jobs.empty()) continue;
            std::vector<size_t> order(jobs.size());
            for (size_t k = 0; k < order.size(); k++) order[k] = k;
            std::stable_sort(order.begin(), order.end(),
                             [&](size_t a, size_t c) { return jobs[a].steps > jobs[c].steps; });
            std::vector<BatchJobHost> sorted;
            int64_t nsteps = 0;
            for (size_t k : order) {
                sorted.push_back(jobs[k]);
                nsteps = std::max(nsteps, jobs[k].steps);
            }
            const size_t need = batch_group_bytes((int)sorted.size());
            if (off + need > b->bytes) return bfail(b, LBM_ENOMEM, "batch table too small for this many jobs");
            e = launch_batch((int)lat, prec, sorted.data(), (int)sorted.size(), b->table + off, need, nsteps, b->stream,
                             b->staging[group]);
            if (e != hipSuccess) return bfail(b, LBM_EHIP, std::string("batch launch: ") + hipGetErrorString(e));
            off += need;
            group++;
            for (size_t k = 0; k < who.size(); k++) {
                lbm_ctx* c = who[k];
                const int64_t n = jobs[k].steps;
                if (n & 1) {
                    c->cur ^= 1;
                    c->ps ^= 1;
                }
                c->liq = LIQ_RECORD;   // the batched collide writes the compact record
                c->step += n;
            }
        }
    }
    return LBM_OK;
}

int lbm_batch_destroy(lbm_batch* b) {
    if (!b) return LBM_EINVAL;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    delete b;
    return LBM_OK;
}

const char* lbm_batch_last_error(const lbm_batch* b) {
    if (!b) return g_create_error.c_str();
    return b->err.c_str();
}

int lbm_destroy(lbm_ctx* c) {
    if (!c) return LBM_EINVAL;
    if (c->bound) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    delete c;
    return LBM_OK;
}

const char* lbm_last_error(const lbm_ctx* c) {
    if (!c) return g_create_error.c_str();
    return c->err.c_str();
}

}  // extern "C"
