// kernels.hip -- HIP kernels (gfx950) of one colour-gradient lattice
// Boltzmann time step with the ghost-node wetting condition.
//
// Per step, on one stream:
//   k_colour_*  phi = sum_i B_i at fluid nodes                      (Eq. A13)
//   k_ghost     phi_G = phi_F / (phi_F + (1 - phi_F) exp(eps))      (Eq. 9)
//               over the compacted ghost list; phi_F interpolated at
//               x_F = x_G + n_s from one snapshot (Jacobi)
//   k_collide   fused: colour stencils, forces (Eq. 4, A9-A11), MRT
//               collision (Eq. A1) in projection form, recolouring
//               (Eq. A12), push streaming (Eq. A16-A17) with halfway
//               bounce-back at solid links
//
// Liquid populations in compact form.  The recolouring of Eq. A12 is
//   B*_i(x) = phi(x) N*_i(x) + (c_i . G(x)) N^eq_i(u = 0, p(x)),
//   G = (2/W) max(phi (1 - phi), 0) n_phi,  N^eq_i(0, p) = chi_i + w_i p / cs^2,
// and streaming moves B*_i(x) to x + c_i exactly as it moves N*_i(x).  So the
// post-stream B_i(y) is fixed by the post-stream N_i(y) and three fields of
// the previous step at the source node y - c_i: phi, G and p.  The fused
// kernel stores G and p (D + 1 values per node) instead of Q streamed B
// planes, and the colour kernel forms B_i(y) from them on the fly.  At a
// bounce-back link the source is y itself with c_i reversed.  This is the
// same arithmetic as storing B (up to rounding); the Q-plane B buffer is only
// read right after the initial state or a restore.
//
// Populations are SoA planes [Q][S], double-buffered; phi is double-buffered
// so that the ghost update reads last step's solid values while writing the
// new ones, and the previous step's phi at fluid nodes stays available for
// the compact B.  Nothing is a dense contraction, so no MFMA is used; HBM
// bandwidth is the roofline.
//
// Launch forms of the colour and collide kernels (one set of per-node
// functions, so every form computes the same values bit for bit):
//   box planes, D3Q19 boxes tiled by 64 x 8: k_colour_tile (z-marching, the
//     compact record of three planes and a one-node ring in LDS) and the
//     row kernel k_collide_stream;
//   box planes otherwise: the row kernels k_colour_compact, k_collide_stream;
//   fluid-only slots (packings): k_colour_sparse, k_collide_sparse, with
//     pull streaming: N holds post-collision populations at their source
//     slot, every reader gathers the post-stream N_i(y) through the
//     neighbour table, and the collide kernel's stores are contiguous;
//   many runs at once: kb_colour, kb_ghost, kb_collide over a job table;
//   the collide-colour step (LBM_OPT_FUSED, D3Q19 boxes tiled by 64 x 8):
//     k_ghost, then k_collide_colour, which also forms the next step's phi
//     from the populations it streams (an LDS hand-over inside 64 x 8 tile
//     columns, an HBM inbox across their faces), then k_colour_fixup.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <type_traits>
#include <utility>

#include "lattice.h"
#include "launch.h"

#ifndef LBM_COLLIDE_BX
#define LBM_COLLIDE_BX 256   // threads per row block of the fused kernel
#endif

namespace lbm {

// ------------------------------------------------------------------ helpers
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// Element idx of a field plane through a 32-bit byte offset from a
// wave-uniform base: the access compiles to a global load/store with a
// scalar base address and one VGPR offset, with no 64-bit address
// arithmetic per access.  Every field plane is below 4 GiB (checked at
// lbm_create), so idx * sizeof(V) fits in 32 bits.
template <class V>
__device__ __forceinline__ V ld(const V* __restrict__ base, uint32_t idx) {
    return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(V));
}
// The same for a population plane that a launch streams through once:
// a non-temporal load, so the streamed planes (far larger than the caches)
// do not evict the colour field and compact record that the stencils and
// gathers reuse (measured 1.6 % faster per step at 256^3, FP32 and FP16).
template <class V>
__device__ __forceinline__ V ld_nt(const V* __restrict__ base, uint32_t idx) {
    return __builtin_nontemporal_load(
        reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + idx * (uint32_t)sizeof(V)));
}
// Element e of a multi-plane array through one 32-bit byte offset from the
// array's base (e = plane * S + node): one wave-uniform base for every
// plane, so a kernel that marches through many planes keeps one scalar
// pointer instead of one per plane.  The caller guarantees that the whole
// array is below 4 GiB.
template <class V>
__device__ __forceinline__ V ld_nt_e(const V* __restrict__ base, uint32_t e) {
    return __builtin_nontemporal_load(
        reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + e * (uint32_t)sizeof(V)));
}
template <class V>
__device__ __forceinline__ void st(V* __restrict__ base, uint32_t idx, V v) {
    *reinterpret_cast<V*>(reinterpret_cast<char*>(base) + idx * (uint32_t)sizeof(V)) = v;
}
// The same as a non-temporal store, for values the launch does not read again.
template <class V>
__device__ __forceinline__ void st_nt(V* __restrict__ base, uint32_t idx, V v) {
    __builtin_nontemporal_store(v, reinterpret_cast<V*>(reinterpret_cast<char*>(base) + idx * (uint32_t)sizeof(V)));
}

// c * v for a lattice component c in {-1, 0, 1}, resolved at compile time.
template <int C, class T>
__device__ __forceinline__ T cmul(T v) {
    if constexpr (C == 1) return v;
    else if constexpr (C == -1) return -v;
    else return T(0);
}

// Storage of the colour-blind populations as offsets from the rest state,
// n_i = N_i - chi_i (every precision).  Near rest the populations differ
// from chi_i by ~1e-6 .. 1e-2, so moments, the equilibrium and the closure
// below work on small numbers: the pressure p (a difference of O(1) sums
// when N_i is carried whole) keeps its relative precision in FP32.  FP64 /
// FP32 runs store n_i itself; 16-bit runs store h_i = n_i / s with a
// power-of-two scale s (FP16 or BF16, rounded to nearest even); arithmetic
// stays FP32.  The rest population closes the zeroth moment of the stored
// values: sum_i N*_i = 1 exactly in the model (Eq. A4 sums to 1 and the
// forcing has no zeroth moment), so n*_0 is written as the closure of the
// other Q - 1 stored values ("off" space: the offset, or the 16-bit code).
template <class T, class SN>
struct NStore {
    static constexpr bool scaled = false;
    __device__ __forceinline__ static T dec(SN h, T) { return h; }
    __device__ __forceinline__ static SN enc(T v, T) { return v; }
    __device__ __forceinline__ static T off(SN h) { return h; }
    __device__ __forceinline__ static SN enc_off(T o) { return o; }
};
template <class SN>
struct NStore16 {
    static constexpr bool scaled = true;
    __device__ __forceinline__ static float dec(SN h, float s) { return s * (float)h; }
    __device__ __forceinline__ static SN enc(float v, float inv_s) { return (SN)(v * inv_s); }
    __device__ __forceinline__ static float off(SN h) { return (float)h; }
    __device__ __forceinline__ static SN enc_off(float o) { return (SN)o; }
};
template <>
struct NStore<float, _Float16> : NStore16<_Float16> {};
template <>
struct NStore<float, __bf16> : NStore16<__bf16> {};

// Arithmetic-type constants of a run.
template <class T, int Q>
struct KParams {
    T rho_g, drho;          // rho = rho_g + drho phi
    T inv_nu_g, dinv_nu;    // 1/nu = inv_nu_g + dinv_nu phi
    T sigma, W, inv_W;
    T g[3];
    T chi[Q];
    T chi_a, chi_d;         // chi_i of the axis (w_1) and the diagonal (w_Q-1) directions: chi_i = (1 - alpha)
                            // w_i / (1 - w_0) takes one value per weight class, so kernels name 3 values, not Q
    T n_thresh2;            // |grad phi|^2 below which n_phi = 0
    T n_s, n_inv_s;         // 16-bit storage scale of N and its inverse
    T n_close;              // target of the closure sum in "off" space: (1 - sum chi) / s
    int nx, ny, nz;
    int64_t S;
};

// Scale of the 16-bit offsets: 2^-10 keeps offsets of 1e-5 .. 1e-2 (the
// range near the rest state) in FP16's normal range.
constexpr double N16_SCALE = 1.0 / 1024.0;

template <class T, class L, class SN>
static KParams<T, L::Q> make_kparams(const StepParams& p) {
    KParams<T, L::Q> k;
    k.rho_g = T(p.rho_g);
    k.drho = T(p.rho_l - p.rho_g);
    k.inv_nu_g = T(p.inv_nu_g);
    k.dinv_nu = T(p.inv_nu_l - p.inv_nu_g);
    k.sigma = T(p.sigma);
    k.W = T(p.W);
    k.inv_W = T(1.0 / p.W);
    for (int a = 0; a < 3; a++) k.g[a] = T(L::D == 2 && a == 2 ? 0.0 : p.g[a]);
    for (int i = 0; i < L::Q; i++) k.chi[i] = T(p.chi[i]);
    k.chi_a = T(p.chi[1]);
    k.chi_d = T(p.chi[L::Q - 1]);
    // |grad phi| > 1e-12 (FP64) or > 1e-7 (FP32) defines the interface normal
    k.n_thresh2 = std::is_same<T, double>::value ? T(1e-24) : T(1e-14);
    const double scale = NStore<T, SN>::scaled ? N16_SCALE : 1.0;
    double sum_chi = 0.0;
    for (int i = 0; i < L::Q; i++) sum_chi += (double)k.chi[i];
    k.n_s = T(scale);
    k.n_inv_s = T(1.0 / scale);
    k.n_close = T((1.0 - sum_chi) / scale);
    k.nx = p.nx;
    k.ny = p.ny;
    k.nz = p.nz;
    k.S = p.S;
    return k;
}

// Planes of the compact liquid record: G (D components) then p.
template <class L>
struct GRec {
    static constexpr int K = L::D + 1;
    static constexpr int P = L::D;   // plane index of p
};

// Isotropic colour gradient grad = 3 sum_i w_i c_i phi_i, summed over
// opposite pairs: 3 sum_pairs w_i c_i (phi_i - phi_opp).  Shared by the
// collision (macro stage) and the colour kernel that re-forms G.
template <class L, class T>
__device__ __forceinline__ void grad_stencil(const T (&ph)[L::Q], T& gx, T& gy, T& gz) {
    gx = gy = gz = T(0);
    static_for<1, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (i < L::opp[i]) {
            constexpr int j = L::opp[i];
            constexpr T wi = T(L::w[i]);
            const T d = wi * (ph[i] - ph[j]);
            if constexpr (L::c[i][0] != 0) gx += cmul<L::c[i][0]>(d);
            if constexpr (L::c[i][1] != 0) gy += cmul<L::c[i][1]>(d);
            if constexpr (L::c[i][2] != 0) gz += cmul<L::c[i][2]>(d);
        }
    });
    gx *= T(3);
    gy *= T(3);
    gz *= T(3);
}

// 1/x and 1/sqrt(x): FP64 divides; FP32 takes the hardware reciprocal and
// reciprocal square root (1 ulp), a tenth of a divide's instructions.
template <class T>
__device__ __forceinline__ T recip(T x) {
    if constexpr (std::is_same<T, float>::value) return __builtin_amdgcn_rcpf(x);
    else return T(1) / x;
}
template <class T>
__device__ __forceinline__ T rsqrt_(T x) {
    if constexpr (std::is_same<T, float>::value) return __builtin_amdgcn_rsqf(x);
    else return T(1) / sqrt(x);
}

// Recolouring vector of Eq. A12, G = (2/W) max(phi (1 - phi), 0) n_phi:
// the normal where |grad phi| is resolved, the amplitude clamped at 0 where
// phi leaves [0, 1].
template <class T>
__device__ __forceinline__ void recolour_vector(T phi, T gx, T gy, T gz, T inv_W, T n_thresh2, T (&G)[3]) {
    const T gn2 = gx * gx + gy * gy + gz * gz;
    T amp = phi * (T(1) - phi);
    amp = amp > T(0) ? amp : T(0);
    G[0] = G[1] = G[2] = T(0);
    if (gn2 > n_thresh2) {
        const T k = T(2) * inv_W * amp * rsqrt_(gn2);
        G[0] = k * gx;
        G[1] = k * gy;
        G[2] = k * gz;
    }
}

// Node output of the macroscopic stage.
template <class T>
struct Macro {
    T phi, rho, inv_tau, p;   // inv_tau = 1 / tau
    T grad[3];
    T u[3];
    T a[3];  // F / rho
};

// Macroscopic stage of one fluid node (N holds offsets n_i = N_i - chi_i):
// colour stencils, mixture properties,
// u0 and p (Eq. A14-A15 with the unforced velocity), forces (Eq. 4, Eq. 2,
// Eq. A9-A11), forced velocity u = u0 + F/(2 rho).  Also returns the raw
// second moments Pi_ab = sum_i c_ia c_ib N_i for the collision.
template <class L, class T>
__device__ __forceinline__ void macro_stage(const T (&N)[L::Q], const T (&ph)[L::Q], const KParams<T, L::Q>& P,
                                            Macro<T>& m, T (&Pi)[6]) {
    constexpr int Q = L::Q;
    constexpr T w0 = T(L::w[0]);
    const T phi = ph[0];
    m.phi = phi;
    // Isotropic stencils, summed over opposite pairs (i, opp i):
    // grad = 3 sum w c phi (grad_stencil),
    // lap = 6 sum_{i>0} w (phi_i - phi) = 6 (sum_pairs w (phi_i + phi_opp) - (1 - w0) phi).
    T gx, gy, gz;
    grad_stencil<L, T>(ph, gx, gy, gz);
    T lap = 0;
    static_for<1, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (i < L::opp[i]) {
            constexpr int j = L::opp[i];
            constexpr T wi = T(L::w[i]);
            lap += wi * (ph[i] + ph[j]);
        }
    });
    lap = T(6) * (lap - (T(1) - w0) * phi);
    m.grad[0] = gx;
    m.grad[1] = gy;
    m.grad[2] = gz;
    // Mixture density and harmonic viscosity (text after Eq. 3).
    const T rho = P.rho_g + P.drho * phi;
    const T inv_nu = P.inv_nu_g + P.dinv_nu * phi;
    // tau = 1/2 + nu / cs^2 = 1/2 + 3 / inv_nu; only 1/tau is used, one division
    const T inv_tau = inv_nu * recip(T(0.5) * inv_nu + T(3));
    m.rho = rho;
    m.inv_tau = inv_tau;
    // Moments of N over opposite pairs: a = n_i + n_opp carries the even
    // moments (zeroth, second), d = n_i - n_opp the odd one (first).
    T jx = 0, jy = 0, jz = 0, s = 0;
    T pxx = 0, pyy = 0, pzz = 0, pxy = 0, pyz = 0, pxz = 0;
    static_for<1, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (i < L::opp[i]) {
            constexpr int j = L::opp[i];
            constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
            const T a = N[i] + N[j];
            const T d = N[i] - N[j];
            s += a;
            if constexpr (cx != 0) jx += cmul<cx>(d);
            if constexpr (cy != 0) jy += cmul<cy>(d);
            if constexpr (cz != 0) jz += cmul<cz>(d);
            if constexpr (cx != 0) pxx += a;
            if constexpr (cy != 0) pyy += a;
            if constexpr (cz != 0) pzz += a;
            if constexpr (cx * cy != 0) pxy += cmul<cx * cy>(a);
            if constexpr (cy * cz != 0) pyz += cmul<cy * cz>(a);
            if constexpr (cx * cz != 0) pxz += cmul<cx * cz>(a);
        }
    });
    Pi[0] = pxx; Pi[1] = pyy; Pi[2] = pzz; Pi[3] = pxy; Pi[4] = pyz; Pi[5] = pxz;
    // Eq. A15 with u0 = sum c N (the forced u needs F_p(p)); s = sum_{i>0} n_i
    // already excludes sum_{i>0} chi_i = 1 - chi_0, and chi has no first
    // moment.  The chi part of Pi is isotropic (chi2 I) and drops out of every
    // use below (deviators and differences of diagonal entries).
    const T uu0 = jx * jx + jy * jy + jz * jz;
    const T p = (s * T(1.0 / 3.0) - T(0.5) * w0 * uu0) / (T(1) - w0);
    m.p = p;
    // Surface tension (Eq. 4): F_s = mu grad phi.
    const T mu = -P.sigma * (T(48) * P.inv_W * phi * (T(1) - phi) * (phi - T(0.5)) + T(1.5) * P.W * lap);
    // Viscous correction (Eq. A11) with grad u + grad u^T = -Pi_dev/(tau cs^2),
    // Pi = sum c c (N - N^eq(u0, p)); N^eq contributes (chi2 + p) I + u0 u0,
    // whose isotropic part drops out of the deviator.
    T dxx = pxx - jx * jx, dyy = pyy - jy * jy, dzz = pzz - jz * jz;
    const T dxy = pxy - jx * jy, dyz = pyz - jy * jz, dxz = pxz - jx * jz;
    T tr;
    if constexpr (L::D == 2) {
        tr = T(0.5) * (dxx + dyy);
        dzz = 0;
    } else {
        tr = (dxx + dyy + dzz) * T(1.0 / 3.0);
        dzz -= tr;
    }
    dxx -= tr;
    dyy -= tr;
    const T kv = T(0.5) * inv_tau - T(1);   // cs^2 (tau - 1/2) * (-1/(tau cs^2)) = -(1 - 1/(2 tau))
    const T grx = P.drho * gx, gry = P.drho * gy, grz = P.drho * gz;   // grad rho
    T Fx = mu * gx - p * grx + kv * (dxx * grx + dxy * gry + dxz * grz) + rho * P.g[0];
    T Fy = mu * gy - p * gry + kv * (dxy * grx + dyy * gry + dyz * grz) + rho * P.g[1];
    T Fz = mu * gz - p * grz + kv * (dxz * grx + dyz * gry + dzz * grz) + rho * P.g[2];
    if constexpr (L::D == 2) Fz = 0;
    const T inv_rho = recip(rho);
    m.a[0] = Fx * inv_rho;
    m.a[1] = Fy * inv_rho;
    m.a[2] = Fz * inv_rho;
    m.u[0] = jx + T(0.5) * m.a[0];
    m.u[1] = jy + T(0.5) * m.a[1];
    m.u[2] = jz + T(0.5) * m.a[2];
}

// Collision in projection form, exactly equal to Eq. A1 with S relaxing the
// traceless second moments at 1/tau and every other moment at 1:
//   N* = N^eq(u, p) + F/2 + (1 - 1/tau) P_sigma (N - N^eq(u, p)),
// returned as offsets Ns_i = N*_i - chi_i.
// Also returns the recolouring vector G = (2/W) max(phi(1 - phi), 0) n_phi
// of Eq. A12.
template <class L, class T>
__device__ __forceinline__ void collide_stage(const Macro<T>& m, const T (&Pi)[6], const KParams<T, L::Q>& P,
                                              T (&Ns)[L::Q], T (&G)[3]) {
    constexpr int Q = L::Q;
    constexpr T w0 = T(L::w[0]);
    const T ux = m.u[0], uy = m.u[1], uz = m.u[2];
    const T uu = ux * ux + uy * uy + uz * uz;
    const T p3 = T(3) * m.p;                      // p / cs^2
    const T omega = T(1) - m.inv_tau;
    // Stress moments of N - N^eq(u, p): N^eq's second moment is
    // (chi2 + p) I + u u, so only u u enters the traceless rows.
    T s1, s2, s3, s4, s5;
    if constexpr (L::D == 2) {
        s1 = omega * ((Pi[0] - Pi[1]) - (ux * ux - uy * uy)) * T(0.25);   // cx^2 - cy^2, |m|^2 = 4
        s2 = omega * (Pi[3] - ux * uy) * T(0.25);                         // cx cy, |m|^2 = 4
        s3 = s4 = s5 = 0;
    } else {
        s1 = omega * ((T(2) * Pi[0] - Pi[1] - Pi[2]) - (T(2) * ux * ux - uy * uy - uz * uz)) * T(1.0 / 36.0);
        s2 = omega * ((Pi[1] - Pi[2]) - (uy * uy - uz * uz)) * T(1.0 / 12.0);
        s3 = omega * (Pi[3] - ux * uy) * T(0.25);
        s4 = omega * (Pi[4] - uy * uz) * T(0.25);
        s5 = omega * (Pi[5] - ux * uz) * T(0.25);
    }
    // Offsets n*_i = N*_i - chi_i.  The rest direction has no stress moment.
    // For an opposite pair the equilibrium's even part, the forcing's odd
    // part and the (even) stress projection give
    //   n*_i, n*_opp = sym +- asym,
    //   sym = w_i (p/cs^2 - 1.5 u.u + 4.5 (c_i.u)^2) + proj_i,
    //   asym = w_i (3 c_i.u + 1.5 c_i.a)     (F_i / 2 = 1.5 w_i c_i.a).
    Ns[0] = -(T(1) - w0) * p3 - w0 * T(1.5) * uu;
    const T A = p3 - T(1.5) * uu;
    static_for<1, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if constexpr (i < L::opp[i]) {
            constexpr int j = L::opp[i];
            constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
            constexpr T wi = T(L::w[i]);
            const T cu = cmul<cx>(ux) + cmul<cy>(uy) + cmul<cz>(uz);
            const T ca = cmul<cx>(m.a[0]) + cmul<cy>(m.a[1]) + cmul<cz>(m.a[2]);
            // projection onto the stress rows, m_k(i) evaluated at compile time
            T proj;
            if constexpr (L::D == 2) {
                proj = T(cx * cx - cy * cy) * s1 + T(cx * cy) * s2;
            } else {
                proj = T(2 * cx * cx - cy * cy - cz * cz) * s1 + T(cy * cy - cz * cz) * s2 + T(cx * cy) * s3 +
                       T(cy * cz) * s4 + T(cx * cz) * s5;
            }
            const T sym = wi * (A + T(4.5) * cu * cu) + proj;
            const T asym = wi * (T(3) * cu + T(1.5) * ca);
            Ns[i] = sym + asym;
            Ns[j] = sym - asym;
        }
    });
    recolour_vector<T>(m.phi, m.grad[0], m.grad[1], m.grad[2], P.inv_W, P.n_thresh2, G);
}

// Neighbour index tables of a node: nb[i] = index of x + c_i (periodic).
// The node index plus wrap-aware offsets along each axis, summed per
// direction (the same indices as wrapping each coordinate).
template <class L, class I>
__device__ __forceinline__ void neighbours(int ix, int iy, int iz, int nx, int ny, int nz, I (&nb)[L::Q]) {
    const I x = (I)ix + (I)nx * ((I)iy + (I)ny * (I)iz);
    const I plane = (I)nx * (I)ny;
    const I oxp = ix == nx - 1 ? (I)0 - (I)(nx - 1) : (I)1, oxm = ix == 0 ? (I)(nx - 1) : (I)0 - (I)1;
    const I oyp = iy == ny - 1 ? (I)0 - (I)(ny - 1) * (I)nx : (I)nx, oym = iy == 0 ? (I)(ny - 1) * (I)nx : (I)0 - (I)nx;
    I ozp = 0, ozm = 0;
    if constexpr (L::D == 3) {
        ozp = iz == nz - 1 ? (I)0 - (I)(nz - 1) * plane : plane;
        ozm = iz == 0 ? (I)(nz - 1) * plane : (I)0 - plane;
    }
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        I o = 0;
        if constexpr (cx > 0) o += oxp;
        if constexpr (cx < 0) o += oxm;
        if constexpr (cy > 0) o += oyp;
        if constexpr (cy < 0) o += oym;
        if constexpr (cz > 0) o += ozp;
        if constexpr (cz < 0) o += ozm;
        nb[i] = x + o;
    });
}

// ------------------------------------------------------------------ kernels
// Row decomposition shared by the stencil kernels: grid (x-blocks, ny, nz).
struct RowIdx {
    int ix, iy, iz;
    int64_t x;
};

__device__ __forceinline__ bool row_index(int nx, int ny, RowIdx& r) {
    r.ix = blockIdx.x * blockDim.x + threadIdx.x;
    if (r.ix >= nx) return false;
    r.iy = blockIdx.y;
    r.iz = blockIdx.z;
    r.x = (int64_t)r.ix + (int64_t)nx * ((int64_t)r.iy + (int64_t)ny * r.iz);
    return true;
}

// Row schedule of the two hot stencil kernels over a 1-D grid of
// xb * ny * nz row blocks.  Consecutive workgroups are dispatched round-robin
// to the 8 XCDs, each with its own L2.  With band > 0 (ny = 8 band) XCD k
// takes rows y in [k band, (k + 1) band) of every plane, plane after plane, so
// the y +- 1 and z +- 1 neighbour rows a stencil reads are mostly in its own
// L2 (the row-major order spreads y-neighbours over three XCDs, each fetching
// the row again).  Any order computes the same result.
// rev: blocks take the rows in reverse order (last plane first).
struct RowSched {
    int xb, ny, band, rev;
};

__device__ __forceinline__ bool row_index_sched(const RowSched& s, int nx, RowIdx& r) {
    const int64_t L = s.rev ? (int64_t)gridDim.x - 1 - blockIdx.x : (int64_t)blockIdx.x;
    int64_t bxi, y, z;
    if (s.band > 0) {
        const int64_t j = L >> 3;
        bxi = j % s.xb;
        const int64_t t = j / s.xb;
        y = (L & 7) * (int64_t)s.band + t % s.band;
        z = t / s.band;
    } else {
        bxi = L % s.xb;
        const int64_t t = L / s.xb;
        y = t % s.ny;
        z = t / s.ny;
    }
    r.ix = (int)bxi * blockDim.x + threadIdx.x;
    if (r.ix >= nx) return false;
    r.iy = (int)y;
    r.iz = (int)z;
    r.x = (int64_t)r.ix + (int64_t)nx * (y + (int64_t)s.ny * z);
    return true;
}

// One term of the compact liquid population: phi(src) N_i(y) +
// sgn (c_i . G(src)) (chi_i + w_i p(src) / cs^2) with N_i = chi_i + n;
// components of G along zero components of c_i are not used.
template <class L, class T, int I>
__device__ __forceinline__ T compact_term(T n, T phi_src, T gx, T gy, T gz, T p, T sgn,
                                          const KParams<T, L::Q>& P) {
    constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
    constexpr T wi = T(L::w[I]);
    T cG = T(0);
    if constexpr (cx != 0) cG += cmul<cx>(gx);
    if constexpr (cy != 0) cG += cmul<cy>(gy);
    if constexpr (cz != 0) cG += cmul<cz>(gz);
    const T sG = sgn * cG;
    const T chi = L::w[I] == L::w[1] ? P.chi_a : P.chi_d;   // equals P.chi[I] (one value per weight class)
    // phi (chi_i + n) + sG (chi_i + 3 w_i p): at one source node phi chi_i
    // and chi_i + 3 w_i p take one value per weight class
    const T pc = phi_src * chi;
    const T k = wi * T(3) * p + chi;
    return (phi_src * n + pc) + sG * k;
}

// Post-stream liquid population B_i(y) from the compact record.  nb[i] is
// y + c_i, so the source y - c_i is nb[opp(i)]; at a bounce-back link the
// source is y with c_i reversed.  PULL (fluid-only layout): N holds
// post-collision populations at their source node, so the post-stream
// N_i(y) is read at the same source as the record: slot i of y - c_i, or
// slot opp(i) of y at a bounce-back link; and the solid links come from
// the neighbour table (`links` bit i: y + c_i is solid), not from flags.
template <class L, class T, class SN, int I, bool PULL = false>
__device__ __forceinline__ T compact_B(const SN* __restrict__ N, const T* __restrict__ phi_prev,
                                       const T* __restrict__ G, const uint8_t* __restrict__ flags,
                                       const KParams<T, L::Q>& P, uint32_t y, const uint32_t (&nb)[L::Q],
                                       bool near_solid, uint32_t links = 0) {
    const int64_t S = P.S;
    if constexpr (I == 0) {
        const T n = NStore<T, SN>::dec(ld(N, y), P.n_s);
        return ld(phi_prev, y) * (P.chi[0] + n);
    } else {
        constexpr int cx = L::c[I][0], cy = L::c[I][1], cz = L::c[I][2];
        uint32_t src = nb[L::opp[I]];
        T sgn = T(1);
        bool bounce;
        if constexpr (PULL) bounce = (links >> L::opp[I]) & 1u;
        else bounce = near_solid && (ld(flags, src) & FLAG_SOLID);
        if (bounce) {
            src = y;
            sgn = T(-1);
        }
        T n;
        if constexpr (PULL)
            n = NStore<T, SN>::dec(bounce ? ld(N + (int64_t)L::opp[I] * S, y) : ld(N + (int64_t)I * S, src), P.n_s);
        else
            n = NStore<T, SN>::dec(ld(N + (int64_t)I * S, y), P.n_s);
        const T gx = cx != 0 ? ld(G, src) : T(0);
        const T gy = cy != 0 ? ld(G + S, src) : T(0);
        const T gz = cz != 0 ? ld(G + 2 * S, src) : T(0);
        return compact_term<L, T, I>(n, ld(phi_prev, src), gx, gy, gz, ld(G + (int64_t)GRec<L>::P * S, src), sgn, P);
    }
}

// phi = sum_i B_i (i ascending) from the Q-plane B buffer (initial state or
// a restore).
template <class L, class T>
__device__ __forceinline__ void colour_planes_node(const T* __restrict__ B, T* __restrict__ phi,
                                                   const uint8_t* __restrict__ flags, int64_t x, int64_t S) {
    if (flags[x] & FLAG_SOLID) return;
    T acc = 0;
#pragma unroll
    for (int i = 0; i < L::Q; i++) acc += B[(int64_t)i * S + x];
    phi[x] = acc;
}

template <class L, class T>
__global__ __launch_bounds__(256) void k_colour_planes(const T* __restrict__ B, T* __restrict__ phi,
                                                       const uint8_t* __restrict__ flags, int64_t n, int64_t S) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    colour_planes_node<L, T>(B, phi, flags, x, S);
}

// phi = sum_i B_i (i ascending) with B_i formed from the compact record, one
// fluid node x with flags f and neighbour indices nb.
template <class L, class T, class SN, bool PULL = false>
__device__ __forceinline__ void colour_compact_core(const SN* __restrict__ N, const T* __restrict__ phi_prev,
                                                    const T* __restrict__ G, const uint8_t* __restrict__ flags,
                                                    T* __restrict__ phi, const KParams<T, L::Q>& P, uint32_t x,
                                                    uint8_t f, const uint32_t (&nb)[L::Q], uint32_t links = 0) {
    const bool near = (f & FLAG_NEAR_SOLID) != 0;
    T acc = 0;
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        acc += compact_B<L, T, SN, i, PULL>(N, phi_prev, G, flags, P, x, nb, near, links);
    });
    st(phi, x, acc);
}

// The same for the node at (ix, iy, iz) of the box layout.
template <class L, class T, class SN>
__device__ __forceinline__ void colour_compact_node(const SN* __restrict__ N, const T* __restrict__ phi_prev,
                                                    const T* __restrict__ G, const uint8_t* __restrict__ flags,
                                                    T* __restrict__ phi, const KParams<T, L::Q>& P, int ix, int iy,
                                                    int iz) {
    const uint32_t x = (uint32_t)ix + (uint32_t)P.nx * ((uint32_t)iy + (uint32_t)P.ny * (uint32_t)iz);
    const uint8_t f = ld(flags, x);
    if (f & FLAG_SOLID) return;
    uint32_t nb[L::Q];
    neighbours<L>(ix, iy, iz, P.nx, P.ny, P.nz, nb);
    colour_compact_core<L, T, SN>(N, phi_prev, G, flags, phi, P, x, f, nb);
}

template <class L, class T, class SN>
__global__ __launch_bounds__(256) void k_colour_compact(const SN* __restrict__ N, const T* __restrict__ phi_prev,
                                                        const T* __restrict__ G, const uint8_t* __restrict__ flags,
                                                        T* __restrict__ phi, KParams<T, L::Q> P, RowSched rs) {
    RowIdx r;
    if (!row_index_sched(rs, P.nx, r)) return;
    colour_compact_node<L, T, SN>(N, phi_prev, G, flags, phi, P, r.ix, r.iy, r.iz);
}

// Colour field of D3Q19 boxes in z-marching tiles: a workgroup owns a
// CTX x CTY (64 x 8) column of nodes and walks up a chunk of planes, keeping the
// compact record (phi_prev, G, p) and flags of three planes of the tile and
// a one-node ring in LDS.  Every record is fetched from memory once per
// workgroup (plus the ring and two prologue planes) instead of once per
// reading node (18 neighbours, 3 to 4 values each); N is read straight into
// registers before the plane's barrier.  Per node the arithmetic is the row
// kernel's: the same compact_term in the same order.
#ifndef LBM_CTX
#define LBM_CTX 64
#endif
#ifndef LBM_CTY
#define LBM_CTY 8
#endif
#ifndef LBM_CT_BLOCKS
#define LBM_CT_BLOCKS 2048
#endif
constexpr int CTX = LBM_CTX, CTY = LBM_CTY;        // tile
// Three record planes in LDS: the plane below, this one and the one above
// (loaded one plane ahead; two barriers per plane).
constexpr int CSL = 3;
__device__ __forceinline__ int slotc(int z) { return (z % CSL + CSL) % CSL; }
constexpr int CRX = CTX + 2, CRY = CTY + 2;       // tile + ring

template <class T>
struct ColourSmem {
    T rec[CSL][5][CRY][CRX];   // phi_prev, Gx, Gy, Gz, p; planes by slotc(z)
    uint8_t fl[CSL][CRY][CRX];
};

__device__ __forceinline__ int wrapc(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Tile schedule over a 1-D grid: XCD k (blocks with id % 8 == k) takes the
// y-band [k yb, (k + 1) yb) of tiles when band > 0, x-tiles fastest, then
// y-tiles of the band, then z-chunks.
struct TileSched {
    int xt, yt, band;  // tiles in x and y; y-tiles per XCD (0: plain order)
};

__device__ __forceinline__ void tile_index(const TileSched& s, int& bx, int& by, int& bz) {
    const int L = blockIdx.x;
    if (s.band > 0) {
        const int j = L >> 3;
        bx = j % s.xt;
        const int t = j / s.xt;
        by = (L & 7) * s.band + t % s.band;
        bz = t / s.band;
    } else {
        bx = L % s.xt;
        const int t = L / s.xt;
        by = t % s.yt;
        bz = t / s.yt;
    }
}

// The record and flags of plane z for the tile and its ring, fetched and
// stored to LDS in one pass (one entry live at a time).
template <class T>
__device__ __forceinline__ void colour_tile_load(ColourSmem<T>& sm, int z, int x0, int y0,
                                                 const T* __restrict__ phi_prev, const T* __restrict__ G,
                                                 const uint8_t* __restrict__ flags, int nx, int ny, int nz,
                                                 int64_t S) {
    const int sl = slotc(z);
    const int Z = wrapc(z, nz);
    for (int k = threadIdx.x; k < CRX * CRY; k += CTX * CTY) {
        const int lx = k % CRX, ly = k / CRX;
        const int X = wrapc(x0 + lx - 1, nx), Y = wrapc(y0 + ly - 1, ny);
        const uint32_t id = (uint32_t)X + (uint32_t)nx * ((uint32_t)Y + (uint32_t)ny * (uint32_t)Z);
        sm.rec[sl][0][ly][lx] = ld(phi_prev, id);
        sm.rec[sl][1][ly][lx] = ld(G, id);
        sm.rec[sl][2][ly][lx] = ld(G + S, id);
        sm.rec[sl][3][ly][lx] = ld(G + 2 * S, id);
        sm.rec[sl][4][ly][lx] = ld(G + 3 * S, id);
        sm.fl[sl][ly][lx] = ld(flags, id);
    }
}

template <class T, class SN>
__global__ __launch_bounds__(CTX * CTY) void k_colour_tile(const SN* __restrict__ N, const T* __restrict__ phi_prev,
                                                           const T* __restrict__ G, const uint8_t* __restrict__ flags,
                                                           T* __restrict__ phi, KParams<T, 19> P, TileSched ts,
                                                           int zc) {
    using L = LatD3Q19;
    __shared__ ColourSmem<T> sm;
    int bx, by, bz;
    tile_index(ts, bx, by, bz);
    const int x0 = bx * CTX, y0 = by * CTY;
    const int z0 = bz * zc;
    const int z1 = min(z0 + zc, P.nz);
    const int tx = threadIdx.x % CTX, ty = threadIdx.x / CTX;
    const int64_t S = P.S;
    const uint32_t xy = (uint32_t)(x0 + tx) + (uint32_t)P.nx * (uint32_t)(y0 + ty);
    const uint32_t plane = (uint32_t)P.nx * (uint32_t)P.ny;
    for (int zz = z0 - 1; zz < z0 + 1; zz++)
        colour_tile_load<T>(sm, zz, x0, y0, phi_prev, G, flags, P.nx, P.ny, P.nz, S);
    SN raw[19];
    for (int z = z0; z < z1; z++) {
        // N of plane z, the record of plane z + 1 into LDS
#pragma unroll
        for (int i = 0; i < 19; i++) raw[i] = ld_nt(N + (int64_t)i * S, xy + plane * (uint32_t)z);
        colour_tile_load<T>(sm, z + 1, x0, y0, phi_prev, G, flags, P.nx, P.ny, P.nz, S);
        __syncthreads();
        const int s0 = slotc(z), sx = tx + 1, sy = ty + 1;
        const uint8_t f = sm.fl[s0][sy][sx];
        if (!(f & FLAG_SOLID)) {
            const bool near = (f & FLAG_NEAR_SOLID) != 0;
            T acc = 0;
            static_for<0, L::Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
                const T n = NStore<T, SN>::dec(raw[i], P.n_s);
                if constexpr (i == 0) {
                    acc += sm.rec[s0][0][sy][sx] * (P.chi[0] + n);
                } else {
                    int sl = slotc(z - cz), qx = sx - cx, qy = sy - cy;
                    T sgn = T(1);
                    if (near && (sm.fl[sl][qy][qx] & FLAG_SOLID)) {
                        sl = s0;
                        qx = sx;
                        qy = sy;
                        sgn = T(-1);
                    }
                    const T gx = cx != 0 ? sm.rec[sl][1][qy][qx] : T(0);
                    const T gy = cy != 0 ? sm.rec[sl][2][qy][qx] : T(0);
                    const T gz = cz != 0 ? sm.rec[sl][3][qy][qx] : T(0);
                    acc += compact_term<L, T, i>(n, sm.rec[sl][0][qy][qx], gx, gy, gz, sm.rec[sl][4][qy][qx], sgn, P);
                }
            });
            st(phi, xy + plane * (uint32_t)z, acc);
        }
        // the next load overwrites the plane below, which this one read
        __syncthreads();
    }
}

// One direction plane of B from the compact record into FP64 (read-out).
template <class L, class T, class SN>
__global__ __launch_bounds__(256) void k_compact_B_plane(const SN* __restrict__ N, const T* __restrict__ phi_prev,
                                                         const T* __restrict__ G, const uint8_t* __restrict__ flags,
                                                         KParams<T, L::Q> P, int dir, double* __restrict__ out) {
    RowIdx r;
    if (!row_index(P.nx, P.ny, r)) return;
    const uint8_t f = flags[r.x];
    if (f & FLAG_SOLID) {
        out[r.x] = 0.0;
        return;
    }
    uint32_t nb[L::Q];
    neighbours<L>(r.ix, r.iy, r.iz, P.nx, P.ny, P.nz, nb);
    const bool near = (f & FLAG_NEAR_SOLID) != 0;
    T v = 0;
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if (i == dir) v = compact_B<L, T, SN, i>(N, phi_prev, G, flags, P, (uint32_t)r.x, nb, near);
    });
    out[r.x] = (double)v;
}

// Ghost update over the compacted list (Jacobi): fluid corners from the
// colour field just written, solid corners from last step's values.
template <class T, int NC>
__device__ __forceinline__ void ghost_one(const int32_t* __restrict__ g_node, const int32_t* __restrict__ g_corner,
                                          const T* __restrict__ g_w, const uint8_t* __restrict__ g_mask, int ng,
                                          const T* __restrict__ phi_prev, T* __restrict__ phi_work, T E, T eps,
                                          int rule, int g) {
    const uint32_t mask = g_mask[g];
    T f = 0;
#pragma unroll
    for (int k = 0; k < NC; k++) {
        const int32_t c = g_corner[(int64_t)k * ng + g];
        const T v = ((mask >> k) & 1u) ? phi_prev[c] : phi_work[c];
        f += g_w[(int64_t)k * ng + g] * v;
    }
    T out;
    if (rule == 0) {
        out = f / (f + (T(1) - f) * E);                    // Eq. 9
    } else {
        // Eq. 10, rationalised: (2/eps)(a - r) = 4 f / (a + r) with
        // a = 1 + eps/2, r = sqrt(a^2 - 2 eps f); no 0/0 at eps = 0.
        const T a = T(1) + T(0.5) * eps;
        out = T(4) * f / (a + sqrt(a * a - T(2) * eps * f)) - f;
    }
    phi_work[g_node[g]] = out;
}

template <class T, int NC>
__global__ __launch_bounds__(256) void k_ghost(const int32_t* __restrict__ g_node, const int32_t* __restrict__ g_corner,
                                               const T* __restrict__ g_w, const uint8_t* __restrict__ g_mask, int ng,
                                               const T* __restrict__ phi_prev, T* __restrict__ phi_work, T E, T eps,
                                               int rule) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    ghost_one<T, NC>(g_node, g_corner, g_w, g_mask, ng, phi_prev, phi_work, E, eps, rule, g);
}

// Fused stencil + forces + collision + recolouring + push streaming with
// halfway bounce-back, one node.  Writes the streamed N* and the node's
// compact liquid record (G, p).  PULL (fluid-only layout): the node gathers
// its post-stream N from the post-collision slots of its sources (slot i of
// x - c_i, or slot opp(i) of x at a bounce-back link) and stores its own
// post-collision N* in its own slots, so the stores are contiguous and the
// scattered accesses are reads.  Its solid links come from the neighbour
// table (`links` bit i: x + c_i is solid).  NT (single runs): N is loaded
// and the record stored non-temporally.
template <class L, class T, class SN, bool NT = true, bool PULL = false>
__device__ __forceinline__ void collide_core(const SN* __restrict__ Nsrc, SN* __restrict__ Ndst,
                                             T* __restrict__ Gdst, const T* __restrict__ phi,
                                             const uint8_t* __restrict__ flags, const KParams<T, L::Q>& P,
                                             uint32_t x, uint8_t f, const uint32_t (&nb)[L::Q],
                                             uint32_t links = 0) {
    constexpr int Q = L::Q;
    using NS = NStore<T, SN>;
    const int64_t S = P.S;
    T N[Q], ph[Q];
    if constexpr (PULL) {
        N[0] = NS::dec(ld(Nsrc, x), P.n_s);
        static_for<1, Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            constexpr int j = L::opp[i];
            const bool bounce = (links >> j) & 1u;
            N[i] = NS::dec(bounce ? ld(Nsrc + (int64_t)j * S, x) : ld(Nsrc + (int64_t)i * S, nb[j]), P.n_s);
        });
    } else {
#pragma unroll
        for (int i = 0; i < Q; i++)
            N[i] = NS::dec(NT ? ld_nt(Nsrc + (int64_t)i * S, x) : ld(Nsrc + (int64_t)i * S, x), P.n_s);
    }
#pragma unroll
    for (int i = 0; i < Q; i++) ph[i] = ld(phi, nb[i]);
    Macro<T> m;
    T Pi[6];
    macro_stage<L, T>(N, ph, P, m, Pi);
    T Ns[Q], G[3];
    collide_stage<L, T>(m, Pi, P, Ns, G);
    // Encode for storage; the rest population closes the stored zeroth moment.
    SN e[Q];
    T closure = P.n_close;
#pragma unroll
    for (int i = 1; i < Q; i++) {
        e[i] = NS::enc(Ns[i], P.n_inv_s);
        closure -= NS::off(e[i]);
    }
    e[0] = NS::enc_off(closure);
    if constexpr (PULL) {
        // whole lines that this launch does not read again: non-temporal,
        // so that they do not push the gathered source lines out of L2
#pragma unroll
        for (int i = 0; i < Q; i++) st_nt(Ndst + (int64_t)i * S, x, e[i]);
    } else if (f & FLAG_NEAR_SOLID) {
        static_for<0, Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if (ld(flags, nb[i]) & FLAG_SOLID) st(Ndst + (int64_t)L::opp[i] * S, x, e[i]);
            else st(Ndst + (int64_t)i * S, nb[i], e[i]);
        });
    } else {
#pragma unroll
        for (int i = 0; i < Q; i++) st(Ndst + (int64_t)i * S, nb[i], e[i]);
    }
    if constexpr (NT) {
        // single runs: the record is read only by the next step's colour
        // pass, after this launch has streamed the whole box
#pragma unroll
        for (int a = 0; a < L::D; a++) st_nt(Gdst + (int64_t)a * S, x, G[a]);
        st_nt(Gdst + (int64_t)GRec<L>::P * S, x, m.p);
    } else {
#pragma unroll
        for (int a = 0; a < L::D; a++) st(Gdst + (int64_t)a * S, x, G[a]);
        st(Gdst + (int64_t)GRec<L>::P * S, x, m.p);
    }
}
template <class L, class T, class SN, bool NT = true>
__device__ __forceinline__ void collide_node(const SN* __restrict__ Nsrc, SN* __restrict__ Ndst,
                                             T* __restrict__ Gdst, const T* __restrict__ phi,
                                             const uint8_t* __restrict__ flags, const KParams<T, L::Q>& P, int ix,
                                             int iy, int iz) {
    const uint32_t x = (uint32_t)ix + (uint32_t)P.nx * ((uint32_t)iy + (uint32_t)P.ny * (uint32_t)iz);
    const uint8_t f = ld(flags, x);
    if (f & FLAG_SOLID) return;
    uint32_t nb[L::Q];
    neighbours<L>(ix, iy, iz, P.nx, P.ny, P.nz, nb);
    collide_core<L, T, SN, NT>(Nsrc, Ndst, Gdst, phi, flags, P, x, f, nb);
}

// One thread per node of an x-row.
template <class L, class T, class SN>
__global__ __launch_bounds__(LBM_COLLIDE_BX) void k_collide_stream(const SN* __restrict__ Nsrc, SN* __restrict__ Ndst,
                                                                   T* __restrict__ Gdst, const T* __restrict__ phi,
                                                                   const uint8_t* __restrict__ flags,
                                                                   KParams<T, L::Q> P, RowSched rs) {
    RowIdx r;
    if (!row_index_sched(rs, P.nx, r)) return;
    collide_node<L, T, SN>(Nsrc, Ndst, Gdst, phi, flags, P, r.ix, r.iy, r.iz);
}

// ------------------------------------------------------------------ collide-colour step
// D3Q19 boxes tiled by KTX x KTY columns run each step as one collide launch
// that also forms the next step's colour field, plus a small fix-up launch.
// Streaming moves the recoloured B*_i(x) to x + c_i exactly as it moves
// N*_i(x), so phi(y) = sum_i B_i(y) of the next step is the sum of the
// recoloured populations arriving at y (Eq. A12, A13, A17).  A workgroup
// owns a KTX x KTY column and marches up a chunk of planes.  Each node
// collides, pushes N* to its neighbours in HBM, forms its B*_i from the
// stored N*_i (the value the two-pass colour kernel reads back) and its own
// phi, G and p, and hands each B*_i to the node it streams to through LDS.
// That node adds what it receives in direction order: the c_z = 0 group when
// its own plane is done, the c_z = +1 group (from the plane below, kept from
// the previous iteration) right after, and the c_z = -1 group when the plane
// above is done, so a node whose sources all lie in its tile gets exactly
// the two-pass sum.  A value whose source lies outside the target's tile or
// z-chunk goes to the target tile's inbox in HBM instead; k_colour_fixup then
// adds those, in direction order, to the in-tile partial sum.  Bounce-back
// links deliver B*_i(x) to x itself in direction opp(i).  No compact record
// is written: the liquid state after such a step is phi itself.
constexpr int KTX = 64, KTY = 8;   // collide-colour tile
constexpr int KNT = KTX * KTY;     // threads per workgroup
constexpr int KRING = 2 * KTX + 2 * (KTY - 2);   // nodes on a tile's lateral edge

// Index of direction I among the five D3Q19 directions with c[I][A] == S.
template <int I, int A, int S>
__device__ __host__ constexpr int cross_k() {
    int k = 0;
    for (int j = 0; j < I; j++)
        if (LatD3Q19::c[j][A] == S) k++;
    return k;
}

// Inbox of one tile-chunk (values of T): for targets on its x faces the
// directions arriving across them ([2 sides][5][zc][KTY]), then the y faces
// ([2][5][zc][KTX]), then the chunk's bottom and top planes ([2][5][KTY][KTX]).
// A value crossing several faces is filed under x, then y, then z.
__host__ __device__ constexpr int64_t cross_tile_vals(int zc) {
    return 10 * (int64_t)zc * (KTX + KTY) + 10 * (int64_t)KNT;
}

// Slot of direction I arriving at local (lx, ly, lz) of a tile-chunk with
// zlen planes, or -1 when its source (lx, ly, lz) - c_I lies in the same
// tile-chunk.
template <int I>
__device__ __forceinline__ int cross_slot(int lx, int ly, int lz, int zc, int zlen) {
    constexpr int cx = LatD3Q19::c[I][0], cy = LatD3Q19::c[I][1], cz = LatD3Q19::c[I][2];
    const int sx = lx - cx, sy = ly - cy, sz = lz - cz;
    if (cx != 0 && (sx < 0 || sx >= KTX)) {
        constexpr int side = cx > 0 ? 0 : 1, k = cross_k<I, 0, cx>();
        return ((side * 5 + k) * zc + lz) * KTY + ly;
    }
    if (cy != 0 && (sy < 0 || sy >= KTY)) {
        constexpr int side = cy > 0 ? 0 : 1, k = cross_k<I, 1, cy>();
        return 10 * zc * KTY + ((side * 5 + k) * zc + lz) * KTX + lx;
    }
    if (cz != 0 && (sz < 0 || sz >= zlen)) {
        constexpr int side = cz > 0 ? 0 : 1, k = cross_k<I, 2, cz>();
        return 10 * zc * (KTX + KTY) + ((side * 5 + k) * KTY + ly) * KTX + lx;
    }
    return -1;
}

struct CrossGeom {
    int xt, yt;    // tiles in x and y
    int zc;        // planes per z-chunk (the last chunk may be shorter)
    int nzc;       // z-chunks
};

// Lateral face-crossing values of one plane are staged in LDS and copied to
// the inbox after the barrier by all threads, coalesced, instead of by the
// few edge lanes of each wave: values leaving through an x face land in two
// halo columns of the hand-over array (so that every lane of a wave stores
// to LDS unconditionally), values leaving through a y face in a y ring
// ([2 faces][5 directions][KTX + 2 target x]; only the two edge rows of the
// tile, each a whole wave, store there).
constexpr int KHX = KTX + 2;                 // hand-over row: the tile and two halo columns
constexpr int YRING = 2 * 5 * KHX;
constexpr int XHALO = 2 * 5 * KTY;           // copy-out entries of the halo columns

// Direction pairs leaving through the faces normal to axis A: pair
// p = side 5 + k is the k-th direction (ascending) with c_A = -1 (side 0)
// or +1 (side 1).  Bit-packed per pair: the direction (5 bits), the other
// components + 1 (2 bits each) and, for A = 1, the direction's index among
// those with its c_x (3 bits; the k of its x-face slot).
constexpr int face_dir(int A, int p) {
    int k = p % 5;
    const int S = p / 5 ? 1 : -1;
    for (int i = 0; i < 19; i++)
        if (LatD3Q19::c[i][A] == S && k-- == 0) return i;
    return -1;
}
constexpr int index_among(int i, int A) {
    int k = 0;
    for (int j = 0; j < i; j++)
        if (LatD3Q19::c[j][A] == LatD3Q19::c[i][A]) k++;
    return k;
}
template <int A>
struct FaceTab {
    static constexpr uint64_t pack_dir() {
        uint64_t v = 0;
        for (int p = 0; p < 10; p++) v |= (uint64_t)face_dir(A, p) << (5 * p);
        return v;
    }
    static constexpr uint32_t pack_comp(int B) {
        uint32_t v = 0;
        for (int p = 0; p < 10; p++) v |= (uint32_t)(LatD3Q19::c[face_dir(A, p)][B] + 1) << (2 * p);
        return v;
    }
    static constexpr uint32_t pack_kx() {
        uint32_t v = 0;
        for (int p = 0; p < 10; p++) v |= (uint32_t)index_among(face_dir(A, p), 0) << (3 * p);
        return v;
    }
    static constexpr uint64_t DIR = pack_dir();
    static constexpr uint32_t CX = pack_comp(0), CY = pack_comp(1), CZ = pack_comp(2), KX = pack_kx();
};

// Target tile-chunk (absolute inbox offset of its block) and local z of a
// value leaving plane lz of chunk bz along c_z = cz (the same chunk unless
// it crosses the chunk's bottom or top plane).
__device__ __forceinline__ void cross_target_z(const CrossGeom& cg, int nz, int bz, int zlen, int lz, int cz, int& tbz,
                                               int& tz, int& tzlen) {
    tbz = bz;
    tz = lz + cz;
    tzlen = zlen;
    if (tz >= zlen) {
        tbz = bz == cg.nzc - 1 ? 0 : bz + 1;
        tz = 0;
        tzlen = min(cg.zc, nz - tbz * cg.zc);
    } else if (tz < 0) {
        tbz = bz == 0 ? cg.nzc - 1 : bz - 1;
        tzlen = min(cg.zc, nz - tbz * cg.zc);
        tz = tzlen - 1;
    }
}

template <class T, class SN>
__global__ __launch_bounds__(KNT, sizeof(T) == 8 ? 2 : 4) void k_collide_colour(const SN* __restrict__ Nsrc, SN* __restrict__ Ndst,
                                                        const T* __restrict__ phi, T* __restrict__ phi_out,
                                                        T* __restrict__ cross, const uint8_t* __restrict__ flags,
                                                        KParams<T, 19> P, TileSched ts, CrossGeom cg) {
    using L = LatD3Q19;
    using NS = NStore<T, SN>;
    constexpr int Q = 19;
    // LDS: the hand-over array [iteration parity][direction - 1][target y]
    // [target x + 1], then the y ring [iteration parity][YRING]
    constexpr int XCH = 2 * (Q - 1) * KTY * KHX;
    __shared__ T sm[XCH + 2 * YRING];
    auto hx = [](int par, int d, int r, int c) { return ((par * (Q - 1) + d) * KTY + r) * KHX + c; };
    auto rg = [](int par, int q) { return XCH + par * YRING + q; };
    int bx, by, bz;
    tile_index(ts, bx, by, bz);
    const int x0 = bx * KTX, y0 = by * KTY, z0 = bz * cg.zc;
    const int z1 = min(z0 + cg.zc, P.nz), zlen = z1 - z0;
    static_assert(KTX == 64, "one tile row per wave: the row index is wave-uniform");
    const int tx = threadIdx.x % KTX;
    const int ty = __builtin_amdgcn_readfirstlane(threadIdx.x / KTX);
    const int ix = x0 + tx, iy = y0 + ty;
    const uint32_t S32 = (uint32_t)P.S;   // plane stride; Q planes of N fit in 4 GiB (checked on the host)
    const int64_t tvals = cross_tile_vals(cg.zc);
    const uint32_t plane = (uint32_t)P.nx * (uint32_t)P.ny;
    const uint32_t xy = (uint32_t)ix + (uint32_t)P.nx * (uint32_t)iy;
    // per thread, fixed for the whole march: bit i of lat_in is set when
    // x - c_i lies in the tile
    uint32_t lat_in = 0;
    static_for<1, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int cx = L::c[i][0], cy = L::c[i][1];
        if (tx - cx >= 0 && tx - cx < KTX && ty - cy >= 0 && ty - cy < KTY) lat_in |= 1u << i;
    });
    // neighbour offsets in x and y (periodic wrap at the box faces)
    const int oxp = ix == P.nx - 1 ? 1 - P.nx : 1, oxm = ix == 0 ? P.nx - 1 : -1;
    const int oyp = iy == P.ny - 1 ? (1 - P.ny) * P.nx : P.nx, oym = iy == 0 ? (P.ny - 1) * P.nx : -P.nx;
    T acc_prev = T(0);      // partial colour sum of (ix, iy, z - 1): c_z = 0 and +1 groups
    uint32_t m_prev = 0;    // bit i: direction i arrives at (ix, iy, z - 1) by bounce-back; bit 31: fluid
    uint8_t f_next = ld(flags, xy + plane * (uint32_t)z0);   // flags one plane ahead
    for (int z = z0; z < z1; z++) {
        const int buf = (z - z0) & 1;
        const int lz = z - z0;
        const uint32_t x = xy + plane * (uint32_t)z;
        const uint8_t f = f_next;
        if (z + 1 < z1) f_next = ld(flags, x + plane);
        const bool fluid = !(f & FLAG_SOLID);
        uint32_t m = fluid ? 0x80000000u : 0u;
        T b0 = T(0);
        if (fluid) {
            const int ozp = z == P.nz - 1 ? (1 - P.nz) * (int)plane : (int)plane;
            const int ozm = z == 0 ? (P.nz - 1) * (int)plane : -(int)plane;
            auto nbr = [&](auto ic) -> uint32_t {
                constexpr int i = decltype(ic)::value;
                constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
                int o = 0;
                if constexpr (cx > 0) o += oxp;
                if constexpr (cx < 0) o += oxm;
                if constexpr (cy > 0) o += oyp;
                if constexpr (cy < 0) o += oym;
                if constexpr (cz > 0) o += ozp;
                if constexpr (cz < 0) o += ozm;
                return x + (uint32_t)o;
            };
            T N[Q], ph[Q];
#pragma unroll
            for (int i = 0; i < Q; i++) N[i] = NS::dec(ld_nt_e(Nsrc, (uint32_t)i * S32 + x), P.n_s);
            ph[0] = ld(phi, x);
            uint32_t bbm = 0;   // bit i: x + c_i is solid (bounce-back link)
            const bool near = (f & FLAG_NEAR_SOLID) != 0;
            static_for<1, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                const uint32_t y = nbr(ic);
                ph[i] = ld(phi, y);
                if (near && (ld(flags, y) & FLAG_SOLID)) bbm |= 1u << i;
            });
            Macro<T> mc;
            T Pi[6];
            macro_stage<L, T>(N, ph, P, mc, Pi);
            T Ns[Q], G[3];
            collide_stage<L, T>(mc, Pi, P, Ns, G);
            SN e[Q];
            T closure = P.n_close;
#pragma unroll
            for (int i = 1; i < Q; i++) {
                e[i] = NS::enc(Ns[i], P.n_inv_s);
                closure -= NS::off(e[i]);
            }
            e[0] = NS::enc_off(closure);
            // N* goes out with non-temporal stores: the launch does not read
            // it again, and the L2 then keeps the inbox values and the colour
            // field that the fix-up reads next
            st_nt(Ndst, x, e[0]);   // the rest population stays at x
            b0 = mc.phi * (P.chi[0] + NS::dec(e[0], P.n_s));
            // every direction streams to x + c_i; where that node is solid
            // the value lands in an entry that nothing reads (a solid node's
            // N, its hand-over slot, an inbox slot the fix-up skips), and the
            // bounce-back pass below delivers it
            static_for<1, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
                const T b = compact_term<L, T, i>(NS::dec(e[i], P.n_s), mc.phi, G[0], G[1], G[2], mc.p, T(1), P);
                st_nt(Ndst, (uint32_t)i * S32 + nbr(ic), e[i]);
                // the branches on ty and lz are wave-uniform
                const bool y_out = cy != 0 && (ty + cy < 0 || ty + cy >= KTY);
                const bool z_out = cz != 0 && (lz + cz < 0 || lz + cz >= zlen);
                if (y_out) {
                    // leaves through a y face (the whole wave of an edge row): the y ring
                    if constexpr (cy != 0) sm[rg(buf, ((cy > 0 ? 5 : 0) + cross_k<i, 1, cy>()) * KHX + tx + cx + 1)] = b;
                } else if (z_out && (cx == 0 || (unsigned)(tx + cx) < (unsigned)KTX)) {
                    // the chunk's bottom or top plane: a target in this tile's
                    // column lies in the neighbouring chunk (inbox)
                    int tbz, tz, tzlen;
                    cross_target_z(cg, P.nz, bz, zlen, lz, cz, tbz, tz, tzlen);
                    const int64_t t = ((int64_t)tbz * cg.yt + by) * cg.xt + bx;
                    cross[t * tvals + cross_slot<i>(tx + cx, ty + cy, tz, cg.zc, tzlen)] = b;
                } else {
                    // in the tile, or a halo column
                    sm[hx(buf, i - 1, ty + cy, tx + cx + 1)] = b;
                }
            });
            if (bbm) {
                // bounce-back links (nodes next to a solid): N*_i and B*_i
                // return to x in direction j = opp(i); B*_i takes x's own slot
                // of direction j (its source is solid, so nothing else is
                // handed to it), in the other buffer when c_z(j) != 0: read
                // with the plane above (c_z = -1) or by this plane's read of
                // the previous buffer (c_z = +1)
                static_for<1, Q>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    constexpr int j = L::opp[i];
                    if ((bbm >> i) & 1u) {
                        const T b =
                            compact_term<L, T, i>(NS::dec(e[i], P.n_s), mc.phi, G[0], G[1], G[2], mc.p, T(1), P);
                        st(Ndst, (uint32_t)j * S32 + x, e[i]);
                        sm[hx(L::c[j][2] == 0 ? buf : buf ^ 1, j - 1, ty, tx + 1)] = b;
                        m |= 1u << j;
                    }
                });
            }
        }
        if (!fluid) {
            // a solid source sends nothing: its off-tile slots get zeros so
            // that the fix-up can add every crossing value (in-tile slots
            // are left alone: they may hold a bounce-back value)
            static_for<1, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
                const bool y_out = cy != 0 && (ty + cy < 0 || ty + cy >= KTY);
                const bool z_out = cz != 0 && (lz + cz < 0 || lz + cz >= zlen);
                const bool x_out = cx != 0 && (tx + cx < 0 || tx + cx >= KTX);
                if (y_out) {
                    if constexpr (cy != 0) sm[rg(buf, ((cy > 0 ? 5 : 0) + cross_k<i, 1, cy>()) * KHX + tx + cx + 1)] = T(0);
                } else if (x_out) {
                    sm[hx(buf, i - 1, ty + cy, tx + cx + 1)] = T(0);
                } else if (z_out) {
                    int tbz, tz, tzlen;
                    cross_target_z(cg, P.nz, bz, zlen, lz, cz, tbz, tz, tzlen);
                    const int64_t t = ((int64_t)tbz * cg.yt + by) * cg.xt + bx;
                    cross[t * tvals + cross_slot<i>(tx + cx, ty + cy, tz, cg.zc, tzlen)] = T(0);
                }
            });
        }
        // c_z = +1 values for this plane, handed over in the previous
        // iteration's buffer (read before this barrier: the next iteration
        // overwrites that buffer only after it)
        T upv[5];
#pragma unroll
        for (int k = 0; k < 5; k++) upv[k] = sm[hx(buf ^ 1, 9 + k - 1, ty, tx + 1)];
        __syncthreads();
        // the staged lateral face-crossing values to the inbox of the tile
        // they enter (solid sources staged zeros; the entry of a bounce-back
        // link holds a stale value, read by no one: its target is solid).  Entry
        // pr of a face's direction pairs is decoded from bit-packed tables.
        for (int k = threadIdx.x; k < XHALO + YRING; k += KNT) {
            T v;
            bool ok;
            int cz, tbx, tby, slot_lo, slot_mul;   // slot = slot_lo + slot_mul * tz
            if (k < XHALO) {
                const int pr = k / KTY, ry = k % KTY;     // pair (side, direction), target row
                const int i = (int)((FaceTab<0>::DIR >> (5 * pr)) & 31u);
                const int cy = (int)((FaceTab<0>::CY >> (2 * pr)) & 3u) - 1;
                cz = (int)((FaceTab<0>::CZ >> (2 * pr)) & 3u) - 1;
                const bool east = pr >= 5;                // c_x = +1
                ok = (unsigned)(ry - cy) < (unsigned)KTY; // a source row of this tile
                v = sm[hx(buf, i - 1, ry, east ? KHX - 1 : 0)];
                tbx = east ? (bx == cg.xt - 1 ? 0 : bx + 1) : (bx == 0 ? cg.xt - 1 : bx - 1);
                tby = by;
                // x-face slot ((side 5 + k) zc + tz) KTY + ly, side 0 for c_x = +1
                slot_lo = (east ? pr - 5 : pr + 5) * cg.zc * KTY + ry;
                slot_mul = KTY;
            } else {
                const int q = k - XHALO;
                const int pr = q / KHX, hx = q % KHX;     // pair (side, direction), target x + 1
                const int cx = (int)((FaceTab<1>::CX >> (2 * pr)) & 3u) - 1;
                cz = (int)((FaceTab<1>::CZ >> (2 * pr)) & 3u) - 1;
                const int kx = (int)((FaceTab<1>::KX >> (3 * pr)) & 7u);
                const bool north = pr >= 5;               // c_y = +1
                const int ttx = hx - 1;
                ok = (unsigned)(ttx - cx) < (unsigned)KTX;  // a source column of this tile
                v = sm[rg(buf, q)];
                const int ly = north ? 0 : KTY - 1;
                tby = north ? (by == cg.yt - 1 ? 0 : by + 1) : (by == 0 ? cg.yt - 1 : by - 1);
                if (ttx < 0 || ttx >= KTX) {
                    // also crosses an x face: filed under x in the diagonal tile
                    const bool east = ttx >= KTX;
                    tbx = east ? (bx == cg.xt - 1 ? 0 : bx + 1) : (bx == 0 ? cg.xt - 1 : bx - 1);
                    slot_lo = ((east ? 0 : 5) + kx) * cg.zc * KTY + ly;
                    slot_mul = KTY;
                } else {
                    // y-face slot 10 zc KTY + ((side 5 + k) zc + tz) KTX + lx, side 0 for c_y = +1
                    tbx = bx;
                    slot_lo = 10 * cg.zc * KTY + (north ? pr - 5 : pr + 5) * cg.zc * KTX + ttx;
                    slot_mul = KTX;
                }
            }
            if (ok) {
                int tbz, tz, tzlen;
                cross_target_z(cg, P.nz, bz, zlen, lz, cz, tbz, tz, tzlen);
                const int64_t t = ((int64_t)tbz * cg.yt + tby) * cg.xt + tbx;
                cross[t * tvals + slot_lo + slot_mul * tz] = v;
            }
        }
        T acc = T(0);
        if (fluid) {
            const uint32_t take = m | lat_in;   // bounce-back, or a source in the tile
            acc = b0;
            // unconditional LDS reads, selected (slots not taken may hold
            // stale values)
            static_for<1, 9>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                const T v = sm[hx(buf, i - 1, ty, tx + 1)];
                acc += ((take >> i) & 1u) ? v : T(0);
            });
            // c_z = +1: a source in the plane below within this chunk, or bounce-back
            const uint32_t up = m | (lz > 0 ? lat_in : 0u);
            static_for<9, 14>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                acc += ((up >> i) & 1u) ? upv[i - 9] : T(0);
            });
        }
        if (m_prev & 0x80000000u) {
            // the plane below is complete with the c_z = -1 values from this plane
            const uint32_t take = m_prev | lat_in;
            T s = acc_prev;
            static_for<14, 19>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                const T v = sm[hx(buf, i - 1, ty, tx + 1)];
                s += ((take >> i) & 1u) ? v : T(0);
            });
            st(phi_out, x - plane, s);
        }
        acc_prev = acc;
        m_prev = m;
    }
    if (m_prev & 0x80000000u) {
        // top plane of the chunk: its c_z = -1 sources lie in the next chunk
        // (bounce-back values were left in the other buffer)
        const int buf = zlen & 1;
        T s = acc_prev;
        static_for<14, 19>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if ((m_prev >> i) & 1u) s += sm[hx(buf, i - 1, ty, tx + 1)];
        });
        st(phi_out, xy + plane * (uint32_t)(z1 - 1), s);
    }
}

// Adds the inbox values (sources outside the target's tile-chunk) to the
// in-tile partial sums, in direction order.  The nodes that have such
// sources are, in each tile-chunk, every node of its first and last plane
// and the KRING nodes on the tile's lateral edge in the planes between.
// They are numbered densely, FIXUP_BLOCKS(zc) workgroups per tile-chunk,
// class by class so that most waves hold one class: the first plane, the
// last plane, the two edge rows (y = 0, KTY - 1) of each inner plane, then
// the edge columns (x = 0, KTX - 1) of each inner plane.  A solid source
// leaves zeros in the inbox, so every crossing value is added.
__host__ __device__ constexpr int fixup_nodes(int zlen) {
    return zlen >= 2 ? 2 * KNT + (zlen - 2) * KRING : KNT;
}

template <class T>
__global__ __launch_bounds__(256) void k_colour_fixup(T* __restrict__ phi_out, const T* __restrict__ cross,
                                                      const uint8_t* __restrict__ flags, int nx, int ny, int nz,
                                                      CrossGeom cg, int blocks_per_chunk) {
    using L = LatD3Q19;
    const int tc = (int)(blockIdx.x / (unsigned)blocks_per_chunk);   // tile-chunk
    const int k = (int)(blockIdx.x % (unsigned)blocks_per_chunk) * 256 + (int)threadIdx.x;
    const int bx = tc % cg.xt, by = (tc / cg.xt) % cg.yt, bz = tc / (cg.xt * cg.yt);
    const int zlen = min(cg.zc, nz - bz * cg.zc);
    if (k >= fixup_nodes(zlen)) return;
    constexpr int EDGE_ROWS = 2 * KTX, EDGE_COLS = 2 * (KTY - 2);
    int lx, ly, lz;
    if (k < KNT) {
        lz = 0;
        lx = k % KTX;
        ly = k / KTX;
    } else if (k < 2 * KNT) {
        lz = zlen - 1;
        lx = (k - KNT) % KTX;
        ly = (k - KNT) / KTX;
    } else if (k < 2 * KNT + (zlen - 2) * EDGE_ROWS) {
        const int r = k - 2 * KNT;
        lz = 1 + r / EDGE_ROWS;
        const int q = r % EDGE_ROWS;
        lx = q % KTX;
        ly = q < KTX ? 0 : KTY - 1;
    } else {
        const int r = k - 2 * KNT - (zlen - 2) * EDGE_ROWS;
        lz = 1 + r / EDGE_COLS;
        const int q = r % EDGE_COLS;
        lx = q < KTY - 2 ? 0 : KTX - 1;
        ly = 1 + q % (KTY - 2);
    }
    const int X = bx * KTX + lx, Y = by * KTY + ly, Z = bz * cg.zc + lz;
    const uint32_t x = (uint32_t)X + (uint32_t)nx * ((uint32_t)Y + (uint32_t)ny * (uint32_t)Z);
    const T* box = cross + (int64_t)tc * cross_tile_vals(cg.zc);
    // the tile faces the node lies on; direction i arrives across a face
    // when its source x - c_i is on the other side
    const bool xlo = lx == 0, xhi = lx == KTX - 1, ylo = ly == 0, yhi = ly == KTY - 1;
    const bool zlo = lz == 0, zhi = lz == zlen - 1;
    const int xrow = lz * KTY + ly, yrow = lz * KTX + lx, zrow = ly * KTX + lx;
    // every load is issued before any of them is used
    const uint8_t fx = ld(flags, x);
    const T part = ld(phi_out, x);
    T v[18];
    static_for<1, 19>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        const bool xc = (cx > 0 && xlo) || (cx < 0 && xhi);
        const bool yc = (cy > 0 && ylo) || (cy < 0 && yhi);
        const bool zc = (cz > 0 && zlo) || (cz < 0 && zhi);
        // slots of cross_slot: x faces, then y faces, then z faces
        int xs = 0, ys = 0, zs = 0;
        if constexpr (cx != 0) xs = ((cx > 0 ? 0 : 5) + cross_k<i, 0, cx>()) * cg.zc * KTY + xrow;
        if constexpr (cy != 0) ys = 10 * cg.zc * KTY + ((cy > 0 ? 0 : 5) + cross_k<i, 1, cy>()) * cg.zc * KTX + yrow;
        if constexpr (cz != 0) zs = 10 * cg.zc * (KTX + KTY) + ((cz > 0 ? 0 : 5) + cross_k<i, 2, cz>()) * KNT + zrow;
        const int slot = xc ? xs : (yc ? ys : zs);
        v[i - 1] = T(0);
        // the inbox's last read this step: non-temporal
        if (xc || yc || zc) v[i - 1] = __builtin_nontemporal_load(box + slot);
    });
    if (fx & FLAG_SOLID) return;
    T add = T(0);
    static_for<1, 19>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        const bool xc = (cx > 0 && xlo) || (cx < 0 && xhi);
        const bool yc = (cy > 0 && ylo) || (cy < 0 && yhi);
        const bool zc = (cz > 0 && zlo) || (cz < 0 && zhi);
        if (xc || yc || zc) add += v[i - 1];
    });
    st(phi_out, x, part + add);
}

// Fluid-only ("sparse") layout for packings: node slots are the fluid nodes
// (ascending box index), then the ghost nodes, then one slot that stands
// for every other solid node; every plane has one entry per slot.
// nbt[(i - 1) n_fluid + k] is the slot of fluid node k + c_i (a ghost slot
// where the neighbour is solid), with NBT_SOLID set where it is solid, so
// that the bounce-back links need no load of the neighbour's flags.  The
// per-node functions are the box layout's, so a step computes the same
// values bit for bit; only the launches cover the fluid slots instead of
// the box.
constexpr uint32_t NBT_SOLID = 0x80000000u, NBT_SLOT = 0x7FFFFFFFu;
template <class L>
__device__ __forceinline__ void sparse_neighbours(const uint32_t* __restrict__ nbt, int64_t nf, uint32_t k,
                                                  uint32_t (&nb)[L::Q], uint32_t& links) {
    nb[0] = k;
    links = 0;
#pragma unroll
    for (int i = 1; i < L::Q; i++) {
        const uint32_t e = nbt[(int64_t)(i - 1) * nf + k];
        nb[i] = e & NBT_SLOT;
        links |= (e >> 31) << i;
    }
}

template <class L, class T, class SN>
__global__ __launch_bounds__(256) void k_colour_sparse(const uint32_t* __restrict__ nbt, int64_t nf,
                                                       const SN* __restrict__ N, const T* __restrict__ phi_prev,
                                                       const T* __restrict__ G, const uint8_t* __restrict__ flags,
                                                       T* __restrict__ phi, KParams<T, L::Q> P) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nf) return;
    uint32_t nb[L::Q], links;
    sparse_neighbours<L>(nbt, nf, (uint32_t)k, nb, links);
    colour_compact_core<L, T, SN, true>(N, phi_prev, G, flags, phi, P, (uint32_t)k, 0, nb, links);
}

template <class L, class T, class SN>
__global__ __launch_bounds__(256) void k_collide_sparse(const uint32_t* __restrict__ nbt, int64_t nf,
                                                        const SN* __restrict__ Nsrc, SN* __restrict__ Ndst,
                                                        T* __restrict__ Gdst, const T* __restrict__ phi,
                                                        const uint8_t* __restrict__ flags, KParams<T, L::Q> P) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nf) return;
    uint32_t nb[L::Q], links;
    sparse_neighbours<L>(nbt, nf, (uint32_t)k, nb, links);
    collide_core<L, T, SN, false, true>(Nsrc, Ndst, Gdst, phi, flags, P, (uint32_t)k, 0, nb, links);
}

// u and p of every slot (solid slots get 0), sparse layout.
template <class L, class T, class SN>
__global__ __launch_bounds__(256) void k_macro_sparse(const uint32_t* __restrict__ nbt, int64_t nf,
                                                      const SN* __restrict__ Nsrc, const T* __restrict__ phi,
                                                      const uint8_t* __restrict__ flags, KParams<T, L::Q> P,
                                                      int64_t n, double* __restrict__ aux) {
    constexpr int Q = L::Q;
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int64_t S = P.S;
    if ((flags[x] & FLAG_SOLID) || x >= nf) {
        aux[x] = 0.0;
        aux[S + x] = 0.0;
        aux[2 * S + x] = 0.0;
        aux[3 * S + x] = 0.0;
        return;
    }
    uint32_t nb[Q], links;
    sparse_neighbours<L>(nbt, nf, (uint32_t)x, nb, links);
    T N[Q], ph[Q];
    // post-stream N gathered from the post-collision slots (pull storage)
    N[0] = NStore<T, SN>::dec(Nsrc[x], P.n_s);
    static_for<1, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int j = L::opp[i];
        const bool bounce = (links >> j) & 1u;
        N[i] = NStore<T, SN>::dec(bounce ? Nsrc[(int64_t)j * S + x] : Nsrc[(int64_t)i * S + nb[j]], P.n_s);
    });
#pragma unroll
    for (int i = 0; i < Q; i++) ph[i] = phi[nb[i]];
    Macro<T> m;
    T Pi[6];
    macro_stage<L, T>(N, ph, P, m, Pi);
    aux[x] = (double)m.u[0];
    aux[S + x] = (double)m.u[1];
    aux[2 * S + x] = (double)m.u[2];
    aux[3 * S + x] = (double)m.p;
}

// One direction plane of B from the compact record into FP64, sparse layout.
template <class L, class T, class SN>
__global__ __launch_bounds__(256) void k_compact_B_sparse(const uint32_t* __restrict__ nbt, int64_t nf,
                                                          const SN* __restrict__ N, const T* __restrict__ phi_prev,
                                                          const T* __restrict__ G, const uint8_t* __restrict__ flags,
                                                          KParams<T, L::Q> P, int dir, int64_t n,
                                                          double* __restrict__ out) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const uint8_t f = flags[x];
    if ((f & FLAG_SOLID) || x >= nf) {
        out[x] = 0.0;
        return;
    }
    uint32_t nb[L::Q], links;
    sparse_neighbours<L>(nbt, nf, (uint32_t)x, nb, links);
    T v = 0;
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if (i == dir) v = compact_B<L, T, SN, i, true>(N, phi_prev, G, flags, P, (uint32_t)x, nb, false, links);
    });
    out[x] = (double)v;
}

// Macroscopic fields (u, p) of every node into FP64 planes; solids get 0.
template <class L, class T, class SN>
__global__ __launch_bounds__(256) void k_macro(const SN* __restrict__ Nsrc, const T* __restrict__ phi,
                                               const uint8_t* __restrict__ flags, KParams<T, L::Q> P,
                                               double* __restrict__ aux) {
    constexpr int Q = L::Q;
    RowIdx r;
    if (!row_index(P.nx, P.ny, r)) return;
    const int64_t x = r.x;
    const int64_t S = P.S;
    if (flags[x] & FLAG_SOLID) {
        aux[x] = 0.0;
        aux[S + x] = 0.0;
        aux[2 * S + x] = 0.0;
        aux[3 * S + x] = 0.0;
        return;
    }
    int64_t nb[Q];
    neighbours<L>(r.ix, r.iy, r.iz, P.nx, P.ny, P.nz, nb);
    T N[Q], ph[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) N[i] = NStore<T, SN>::dec(Nsrc[(int64_t)i * S + x], P.n_s);
#pragma unroll
    for (int i = 0; i < Q; i++) ph[i] = phi[nb[i]];
    Macro<T> m;
    T Pi[6];
    macro_stage<L, T>(N, ph, P, m, Pi);
    aux[x] = (double)m.u[0];
    aux[S + x] = (double)m.u[1];
    aux[2 * S + x] = (double)m.u[2];
    aux[3 * S + x] = (double)m.p;
}

// Reduction of the seven diagnostics (six sums, the maximum at index 5) and
// the non-finite count over a 256-thread block: a butterfly across the 64
// lanes of each wave (__shfl_xor), then the four waves' results in order.
// The order is fixed, so the result is deterministic; valid in thread 0.
__device__ __forceinline__ void block_reduce_diag(double (&v)[7], int64_t& bad) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
        for (int k = 0; k < 7; k++) {
            const double o = __shfl_xor(v[k], off, 64);
            v[k] = k == 5 ? (o > v[k] ? o : v[k]) : v[k] + o;
        }
        bad += (int64_t)__shfl_xor((long long)bad, off, 64);
    }
    __shared__ double wv[4][7];
    __shared__ int64_t wn[4];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
        for (int k = 0; k < 7; k++) wv[w][k] = v[k];
        wn[w] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int j = 1; j < 4; j++) {
#pragma unroll
            for (int k = 0; k < 7; k++) v[k] = k == 5 ? (wv[j][k] > v[k] ? wv[j][k] : v[k]) : v[k] + wv[j][k];
            bad += wn[j];
        }
    }
}

// Diagnostics, stage 1: each block reduces a fixed strided set of nodes in a
// fixed order (deterministic for a fixed grid).  Values: sum phi,
// sum (1 - phi), sum rho u (3), max |u|, sum rho |u|^2 / 2; non-finite count
// over N, the liquid state (B planes or compact record) and phi.
template <class L, class T, class SN>
__global__ __launch_bounds__(256) void k_reduce1(const SN* __restrict__ N, const T* __restrict__ Bstate, int nB,
                                                 const T* __restrict__ phi, const uint8_t* __restrict__ flags,
                                                 const double* __restrict__ aux, int64_t n, int64_t S, double rho_g,
                                                 double drho, double* __restrict__ partial,
                                                 int64_t* __restrict__ nonfinite) {
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    int64_t bad = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n; x += stride) {
        if (flags[x] & FLAG_SOLID) continue;
        const double ph = (double)phi[x];
        const double ux = aux[x], uy = aux[S + x], uz = aux[2 * S + x];
        const double rho = rho_g + drho * ph;
        const double u2 = ux * ux + uy * uy + uz * uz;
        v[0] += ph;
        v[1] += 1.0 - ph;
        v[2] += rho * ux;
        v[3] += rho * uy;
        v[4] += rho * uz;
        const double sp = sqrt(u2);
        v[5] = sp > v[5] ? sp : v[5];
        v[6] += 0.5 * rho * u2;
        if (!isfinite(ph) || !isfinite(u2)) bad++;
        for (int i = 0; i < L::Q; i++)
            if (!isfinite((double)NStore<T, SN>::off(N[(int64_t)i * S + x]))) bad++;
        for (int i = 0; i < nB; i++)
            if (!isfinite((double)Bstate[(int64_t)i * S + x])) bad++;
    }
    block_reduce_diag(v, bad);
    if (threadIdx.x == 0) {
        for (int k = 0; k < 7; k++) partial[(int64_t)blockIdx.x * 8 + k] = v[k];
        nonfinite[blockIdx.x] = bad;
    }
}

// Diagnostics, stage 2: one block folds the partials in a fixed order.
__global__ __launch_bounds__(256) void k_reduce2(const double* __restrict__ partial,
                                                 const int64_t* __restrict__ nonfinite, int nblocks,
                                                 double* __restrict__ result, int64_t* __restrict__ nf_out) {
    const int t = threadIdx.x;
    double v[7] = {0, 0, 0, 0, 0, 0, 0};
    int64_t bad = 0;
    for (int b = t; b < nblocks; b += 256) {
        for (int k = 0; k < 7; k++) {
            const double q = partial[(int64_t)b * 8 + k];
            if (k == 5) v[k] = q > v[k] ? q : v[k];
            else v[k] += q;
        }
        bad += nonfinite[b];
    }
    block_reduce_diag(v, bad);
    if (t == 0) {
        for (int k = 0; k < 7; k++) result[k] = v[k];
        *nf_out = bad;
    }
}

// Start of a run: N = chi, B = phi chi at fluid nodes (u = p = 0), solid
// phi = phi_solid in both colour buffers, compact record zero.
template <class L, class T, class SN>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ phi0, const uint8_t* __restrict__ flags,
                                              SN* __restrict__ N, T* __restrict__ B, T* __restrict__ phiA,
                                              T* __restrict__ phiB, T* __restrict__ G0, T* __restrict__ G1,
                                              KParams<T, L::Q> P, T phi_solid, int64_t n) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int64_t S = P.S;
#pragma unroll
    for (int k = 0; k < GRec<L>::K; k++) {
        G0[(int64_t)k * S + x] = T(0);
        G1[(int64_t)k * S + x] = T(0);
    }
    if (flags[x] & FLAG_SOLID) {
        phiA[x] = phi_solid;
        phiB[x] = phi_solid;
#pragma unroll
        for (int i = 0; i < L::Q; i++) {
            N[(int64_t)i * S + x] = NStore<T, SN>::enc(T(0), P.n_inv_s);
            B[(int64_t)i * S + x] = T(0);
        }
        return;
    }
    const T ph = (T)phi0[x];
    phiA[x] = ph;
    phiB[x] = ph;
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        N[(int64_t)i * S + x] = NStore<T, SN>::enc(T(0), P.n_inv_s);
        B[(int64_t)i * S + x] = ph * P.chi[i];
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_solid_phi(const uint8_t* __restrict__ flags, T* __restrict__ phiA,
                                                   T* __restrict__ phiB, T v, int64_t n) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    if (flags[x] & FLAG_SOLID) {
        phiA[x] = v;
        phiB[x] = v;
    }
}

template <class T>
__global__ __launch_bounds__(256) void k_plane_out(const T* __restrict__ src, const uint8_t* __restrict__ flags,
                                                   int zero_solid, double* __restrict__ dst, int64_t n) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    dst[x] = (zero_solid && (flags[x] & FLAG_SOLID)) ? 0.0 : (double)src[x];
}

// N plane `dir` <-> FP64 (decoding / encoding the storage).
template <class T, class SN>
__global__ __launch_bounds__(256) void k_nplane_out(const SN* __restrict__ src, const uint8_t* __restrict__ flags,
                                                    T chi, T s, double* __restrict__ dst, int64_t n) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    dst[x] = (flags[x] & FLAG_SOLID) ? 0.0 : (double)chi + (double)NStore<T, SN>::dec(src[x], s);
}

template <class T, class SN>
__global__ __launch_bounds__(256) void k_nplane_in(const double* __restrict__ src, SN* __restrict__ dst, T chi,
                                                   T inv_s, int64_t n) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    dst[x] = NStore<T, SN>::enc((T)(src[x] - (double)chi), inv_s);
}

// The same for the fluid-only layout, whose N holds post-collision
// populations at their source slot: the post-stream N_i of fluid slot y is
// slot i of y - c_i (nbo[y], the neighbour table's plane for opp(i)), or
// slot opp(i) of y when y - c_i is solid.  Every stored slot of a fluid node
// is the post-stream value of exactly one (i, y), so the read-out gathers
// and the set scatters, both without arithmetic.  dir 0 has no source.
template <class T, class SN>
__global__ __launch_bounds__(256) void k_nplane_out_pull(const SN* __restrict__ N, const uint32_t* __restrict__ nbo,
                                                         const uint8_t* __restrict__ flags, int dir, int odir,
                                                         int64_t S, int64_t nf, T chi, T s,
                                                         double* __restrict__ dst, int64_t n) {
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= n) return;
    if (y >= nf || (flags[y] & FLAG_SOLID)) {
        dst[y] = 0.0;
        return;
    }
    SN v;
    if (dir == 0) {
        v = N[y];
    } else {
        const uint32_t e = nbo[y];
        v = (e & NBT_SOLID) ? N[(int64_t)odir * S + y] : N[(int64_t)dir * S + (e & NBT_SLOT)];
    }
    dst[y] = (double)chi + (double)NStore<T, SN>::dec(v, s);
}

template <class T, class SN>
__global__ __launch_bounds__(256) void k_nplane_in_pull(const double* __restrict__ src, SN* __restrict__ N,
                                                        const uint32_t* __restrict__ nbo,
                                                        const uint8_t* __restrict__ flags, int dir, int odir,
                                                        int64_t S, int64_t nf, T chi, T inv_s, int64_t n) {
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= n || y >= nf || (flags[y] & FLAG_SOLID)) return;
    const SN v = NStore<T, SN>::enc((T)(src[y] - (double)chi), inv_s);
    if (dir == 0) {
        N[y] = v;
        return;
    }
    const uint32_t e = nbo[y];
    if (e & NBT_SOLID) N[(int64_t)odir * S + y] = v;
    else N[(int64_t)dir * S + (e & NBT_SLOT)] = v;
}

template <class T>
__global__ __launch_bounds__(256) void k_plane_in(const double* __restrict__ src, T* __restrict__ dst, int64_t n) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    dst[x] = (T)src[x];
}

// Fluid entries of one colour buffer from an FP64 plane.
template <class T>
__global__ __launch_bounds__(256) void k_fluid_in(const double* __restrict__ src, const uint8_t* __restrict__ flags,
                                                  T* __restrict__ phi, int64_t n) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    if (!(flags[x] & FLAG_SOLID)) phi[x] = (T)src[x];
}

// Solid entries of both colour buffers from an FP64 plane.
template <class T>
__global__ __launch_bounds__(256) void k_solid_in(const double* __restrict__ src, const uint8_t* __restrict__ flags,
                                                  T* __restrict__ phiA, T* __restrict__ phiB, int64_t n) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    if (flags[x] & FLAG_SOLID) {
        phiA[x] = (T)src[x];
        phiB[x] = (T)src[x];
    }
}

// ------------------------------------------------------------------ batched steps
// Many independent runs advance in shared launches: every workgroup (one
// wave, 64 threads) finds its job by binary search over the jobs' first
// block, then works on one row-block of that job exactly as the single-run
// kernels do.  Jobs are sorted by their sub-step count (largest first), so
// the jobs still active at sub-step k are a prefix and the grid shrinks.
constexpr int BATCH_BX = 64;

template <class L, class T, class SN>
struct BJob {
    KParams<T, L::Q> P;
    const SN* N[2];
    T* G[2];
    T* phi[2];
    const T* B;
    const uint8_t* flags;
    const int32_t* g_node;
    const int32_t* g_corner;
    const T* g_w;
    const uint8_t* g_mask;
    int32_t n_ghost;
    int32_t rule;
    T E, eps;
    int32_t cur0, ps0, planes0, nxb;
};

__device__ __forceinline__ int find_job(const int64_t* __restrict__ start, int njobs, int64_t b) {
    int lo = 0, hi = njobs - 1;   // largest j with start[j] <= b
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <class L, class T, class SN>
__device__ __forceinline__ bool batch_row(const BJob<L, T, SN>& J, int64_t lb, int& ix, int& iy, int& iz) {
    const int64_t row = lb / J.nxb;
    ix = (int)(lb - row * J.nxb) * BATCH_BX + (int)threadIdx.x;
    iy = (int)(row % J.P.ny);
    iz = (int)(row / J.P.ny);
    return ix < J.P.nx;
}

template <class L, class T, class SN>
__global__ __launch_bounds__(BATCH_BX) void kb_colour(const BJob<L, T, SN>* __restrict__ jobs,
                                                      const int64_t* __restrict__ start, int njobs, int64_t k) {
    const int j = find_job(start, njobs, blockIdx.x);
    const BJob<L, T, SN>& J = jobs[j];
    int ix, iy, iz;
    if (!batch_row(J, (int64_t)blockIdx.x - start[j], ix, iy, iz)) return;
    const int par = (int)((J.cur0 + k) & 1), pps = (int)((J.ps0 + k) & 1);
    T* work = J.phi[1 - pps];
    if (k == 0 && J.planes0 == LIQ_PHI) return;   // phi of this sub-step already formed
    if (k == 0 && J.planes0 == LIQ_PLANES) {
        const int64_t x = (int64_t)ix + (int64_t)J.P.nx * ((int64_t)iy + (int64_t)J.P.ny * iz);
        colour_planes_node<L, T>(J.B, work, J.flags, x, J.P.S);
    } else {
        colour_compact_node<L, T, SN>(J.N[par], J.phi[pps], J.G[par], J.flags, work, J.P, ix, iy, iz);
    }
}

template <class L, class T, class SN>
__global__ __launch_bounds__(BATCH_BX) void kb_ghost(const BJob<L, T, SN>* __restrict__ jobs,
                                                     const int64_t* __restrict__ start, int njobs, int64_t k) {
    const int j = find_job(start, njobs, blockIdx.x);
    const BJob<L, T, SN>& J = jobs[j];
    const int g = (int)((int64_t)blockIdx.x - start[j]) * BATCH_BX + (int)threadIdx.x;
    if (g >= J.n_ghost) return;
    const int pps = (int)((J.ps0 + k) & 1);
    ghost_one<T, L::NC>(J.g_node, J.g_corner, J.g_w, J.g_mask, J.n_ghost, J.phi[pps], J.phi[1 - pps], J.E, J.eps,
                        J.rule, g);
}

template <class L, class T, class SN>
__global__ __launch_bounds__(BATCH_BX) void kb_collide(const BJob<L, T, SN>* __restrict__ jobs,
                                                       const int64_t* __restrict__ start, int njobs, int64_t k) {
    const int j = find_job(start, njobs, blockIdx.x);
    const BJob<L, T, SN>& J = jobs[j];
    int ix, iy, iz;
    if (!batch_row(J, (int64_t)blockIdx.x - start[j], ix, iy, iz)) return;
    const int par = (int)((J.cur0 + k) & 1), pps = (int)((J.ps0 + k) & 1);
    // plain loads: the populations of most batched runs fit in the last-level
    // cache and stay there between sub-steps (non-temporal loads give that up)
    collide_node<L, T, SN, false>(J.N[par], const_cast<SN*>(J.N[1 - par]), J.G[1 - par], J.phi[1 - pps], J.flags,
                                  J.P, ix, iy, iz);
}

// ------------------------------------------------------------------ launchers
static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

static inline dim3 row_grid(const StepParams& p, int bx) {
    return dim3((unsigned)((p.nx + bx - 1) / bx), (unsigned)p.ny, (unsigned)p.nz);
}

// Row block: the widest of 256 / 192 / 128 / 64 threads that divides nx
// (no idle lanes), else 256 / 128 / 64 by size.
static inline int row_block(int nx) {
    for (int b : {256, 192, 128, 64})
        if (b <= LBM_COLLIDE_BX && nx % b == 0) return b;
    int b = nx >= 256 ? 256 : (nx >= 128 ? 128 : 64);
    return b > LBM_COLLIDE_BX ? LBM_COLLIDE_BX : b;
}

// Row kernels run in plain row-major block order (a y-band order per XCD,
// each XCD's L2 holding a stencil's y +- 1 rows, measured slower on gfx950
// for both row kernels); colour tiles are dealt to the XCDs in y-bands.
static inline RowSched row_sched(const StepParams& p, int bx) {
    RowSched s;
    s.xb = (p.nx + bx - 1) / bx;
    s.ny = p.ny;
    s.band = 0;
    s.rev = 0;
    return s;
}

static inline dim3 row_grid1(const RowSched& s, const StepParams& p) {
    return dim3((unsigned)((int64_t)s.xb * p.ny * p.nz));
}

// The z-marching colour kernel takes D3Q19 boxes tiled exactly by CTX x CTY.
static inline bool colour_tile_ok(const StepParams& p) {
    return p.nz > 1 && p.nx % CTX == 0 && p.ny % CTY == 0;
}

// z-chunk: about LBM_CT_BLOCKS (2048) workgroups, at least 4 planes each.
static inline int colour_tile_chunk(const StepParams& p) {
    const int64_t cols = (int64_t)(p.nx / CTX) * (p.ny / CTY);
    int64_t zc = (p.nz * cols + LBM_CT_BLOCKS - 1) / LBM_CT_BLOCKS;
    if (zc < 4) zc = 4;
    if (zc > p.nz) zc = p.nz;
    return (int)zc;
}

static inline TileSched tile_sched(const StepParams& p) {
    TileSched s;
    s.xt = p.nx / CTX;
    s.yt = p.ny / CTY;
    s.band = s.yt % 8 == 0 ? s.yt / 8 : 0;
    return s;
}

// The collide-colour step takes D3Q19 boxes tiled exactly by KTX x KTY.
static inline bool cc_ok(const StepParams& p) { return p.nx % KTX == 0 && p.ny % KTY == 0; }

// z-chunk of the collide-colour step: about LBM_CC_BLOCKS workgroups, at
// least 4 planes each.  Shorter chunks balance the 2-workgroups-per-CU
// launch better but give the fix-up more nodes (every node of a chunk's
// first and last plane); on the 256^3 box (FP32) 2048 / 4096 / 6144 / 8192
// workgroups (chunks of 16 / 8 / 6 / 4 planes) measured 0.908 / 0.875 /
// 0.867 / 0.879 ms per step.
#ifndef LBM_CC_BLOCKS
#define LBM_CC_BLOCKS 6144
#endif
static inline CrossGeom cc_geom(const StepParams& p) {
    CrossGeom g;
    g.xt = p.nx / KTX;
    g.yt = p.ny / KTY;
    int64_t zc = ((int64_t)p.nz * g.xt * g.yt + LBM_CC_BLOCKS - 1) / LBM_CC_BLOCKS;
    if (zc < 4) zc = 4;
    if (zc > p.nz) zc = p.nz;
    g.zc = (int)zc;
    g.nzc = (p.nz + g.zc - 1) / g.zc;
    return g;
}

bool step_fused(int lattice, const DevState& d, const StepParams& p) {
    return lattice == 1 && d.fused && !d.sparse && cc_ok(p);
}

size_t cross_bytes(int lattice, uint32_t prec, const StepParams& p) {
    if (lattice != 1 || !cc_ok(p)) return 0;
    const CrossGeom g = cc_geom(p);
    const int64_t chunks = (p.nz + g.zc - 1) / g.zc;
    return (size_t)((int64_t)g.xt * g.yt * chunks * cross_tile_vals(g.zc)) * (prec == P_FP64 ? 8 : 4);
}

template <class L, class T, class SN>
static hipError_t phase_t(int phase, const DevState& d, const StepParams& p, int cur, int ps, int liq,
                          hipStream_t st) {
    T* work = (T*)d.phi[1 - ps];
    const int bx = row_block(p.nx);
    const bool fused = step_fused(L::D == 3 ? 1 : 0, d, p);
    if (phase == 0) {
        if (liq == LIQ_PHI) return hipSuccess;   // formed by the last collide-colour step
        if (liq == LIQ_PLANES) {
            hipLaunchKernelGGL((k_colour_planes<L, T>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st,
                               (const T*)d.B, work, d.flags, p.n, p.S);
        } else {
            const KParams<T, L::Q> kp = make_kparams<T, L, SN>(p);
            if (d.sparse) {
                if (d.n_fluid > 0)
                    hipLaunchKernelGGL((k_colour_sparse<L, T, SN>), dim3(blocks_for(d.n_fluid, 256)), dim3(256), 0,
                                       st, d.nbt, d.n_fluid, (const SN*)d.N[cur], (const T*)d.phi[ps],
                                       (const T*)d.G[cur], d.flags, work, kp);
                return hipGetLastError();
            }
            if constexpr (L::D == 3) {
                if (colour_tile_ok(p)) {
                    const int zc = colour_tile_chunk(p);
                    const TileSched ts = tile_sched(p);
                    const unsigned nb = (unsigned)(ts.xt * ts.yt * ((p.nz + zc - 1) / zc));
                    hipLaunchKernelGGL((k_colour_tile<T, SN>), dim3(nb), dim3(CTX * CTY), 0, st, (const SN*)d.N[cur],
                                       (const T*)d.phi[ps], (const T*)d.G[cur], d.flags, work, kp, ts, zc);
                    return hipGetLastError();
                }
            }
            const RowSched rs = row_sched(p, bx);
            hipLaunchKernelGGL((k_colour_compact<L, T, SN>), row_grid1(rs, p), dim3(bx), 0, st,
                               (const SN*)d.N[cur], (const T*)d.phi[ps], (const T*)d.G[cur], d.flags, work, kp, rs);
        }
    } else if (phase == 1) {
        if (d.n_ghost > 0) {
            hipLaunchKernelGGL((k_ghost<T, L::NC>), dim3(blocks_for(d.n_ghost, 256)), dim3(256), 0, st, d.g_node,
                               d.g_corner, (const T*)d.g_w, d.g_mask, d.n_ghost, (const T*)d.phi[ps], work,
                               (T)p.exp_eps, (T)p.eps, p.ghost_rule);
        }
    } else if (phase == 2) {
        const KParams<T, L::Q> kp = make_kparams<T, L, SN>(p);
        if constexpr (L::D == 3) {
            if (fused) {
                // this step's phi (work) in, the next step's phi into phi[ps]
                const CrossGeom g = cc_geom(p);
                TileSched ts;
                ts.xt = g.xt;
                ts.yt = g.yt;
                ts.band = g.yt % 8 == 0 ? g.yt / 8 : 0;
                const unsigned nb = (unsigned)(g.xt * g.yt * g.nzc);
                hipLaunchKernelGGL((k_collide_colour<T, SN>), dim3(nb), dim3(KNT), 0, st, (const SN*)d.N[cur],
                                   (SN*)d.N[1 - cur], (const T*)work, (T*)d.phi[ps], (T*)d.cross, d.flags, kp, ts, g);
                return hipGetLastError();
            }
        }
        if (d.sparse) {
            if (d.n_fluid > 0)
                hipLaunchKernelGGL((k_collide_sparse<L, T, SN>), dim3(blocks_for(d.n_fluid, 256)), dim3(256), 0, st,
                                   d.nbt, d.n_fluid, (const SN*)d.N[cur], (SN*)d.N[1 - cur], (T*)d.G[1 - cur],
                                   (const T*)work, d.flags, kp);
            return hipGetLastError();
        }
        // rows from the last plane down: the launch ends on the first planes,
        // where the next step's colour pass starts while the last-level
        // cache still holds what was stored there last (N*, the record)
        RowSched rs = row_sched(p, bx);
        rs.rev = 1;
        hipLaunchKernelGGL((k_collide_stream<L, T, SN>), row_grid1(rs, p), dim3(bx), 0, st, (const SN*)d.N[cur],
                           (SN*)d.N[1 - cur], (T*)d.G[1 - cur], (const T*)work, d.flags, kp, rs);
    } else {
        if constexpr (L::D == 3) {
            if (fused) {
                const CrossGeom g = cc_geom(p);
                const int bpc = (fixup_nodes(g.zc) + 255) / 256;
                hipLaunchKernelGGL((k_colour_fixup<T>), dim3((unsigned)(g.xt * g.yt * g.nzc * bpc)), dim3(256), 0, st,
                                   (T*)d.phi[ps], (const T*)d.cross, d.flags, p.nx, p.ny, p.nz, g, bpc);
            }
        }
    }
    return hipGetLastError();
}

template <class L, class T, class SN>
static hipError_t colour_t(const DevState& d, const StepParams& p, int cur, int ps, int liq, hipStream_t st) {
    hipError_t e = phase_t<L, T, SN>(0, d, p, cur, ps, liq, st);
    if (e != hipSuccess) return e;
    return phase_t<L, T, SN>(1, d, p, cur, ps, liq, st);
}

template <class L, class T, class SN>
static hipError_t step_t(const DevState& d, const StepParams& p, int cur, int ps, int liq, hipStream_t st) {
    for (int ph = 0; ph < STEP_PHASES; ph++) {
        hipError_t e = phase_t<L, T, SN>(ph, d, p, cur, ps, liq, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class L, class T, class SN>
static hipError_t macro_t(const DevState& d, const StepParams& p, int cur, int ps, hipStream_t st) {
    const KParams<T, L::Q> kp = make_kparams<T, L, SN>(p);
    if (d.sparse) {
        hipLaunchKernelGGL((k_macro_sparse<L, T, SN>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, d.nbt,
                           d.n_fluid, (const SN*)d.N[cur], (const T*)d.phi[1 - ps], d.flags, kp, p.n, d.aux);
        return hipGetLastError();
    }
    const int bx = row_block(p.nx);
    hipLaunchKernelGGL((k_macro<L, T, SN>), row_grid(p, bx), dim3(bx), 0, st, (const SN*)d.N[cur],
                       (const T*)d.phi[1 - ps], d.flags, kp, d.aux);
    return hipGetLastError();
}

template <class L, class T, class SN>
static hipError_t reduce_t(const DevState& d, const StepParams& p, int cur, int ps, int liq,
                           const ReduceScratch& rs, hipStream_t st) {
    const T* Bstate = liq == LIQ_PLANES ? (const T*)d.B : (const T*)d.G[cur];
    const int nB = liq == LIQ_PLANES ? L::Q : (liq == LIQ_RECORD ? GRec<L>::K : 0);
    hipLaunchKernelGGL((k_reduce1<L, T, SN>), dim3(REDUCE_BLOCKS), dim3(256), 0, st, (const SN*)d.N[cur], Bstate, nB,
                       (const T*)d.phi[1 - ps], d.flags, d.aux, p.n, p.S, p.rho_g, p.rho_l - p.rho_g, rs.partial,
                       rs.nonfinite);
    hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(256), 0, st, rs.partial, rs.nonfinite, REDUCE_BLOCKS, rs.result,
                       rs.nonfinite + REDUCE_BLOCKS);
    return hipGetLastError();
}

template <class L, class T, class SN>
static hipError_t init_t(const DevState& d, const StepParams& p, int cur, int ps, hipStream_t st) {
    const KParams<T, L::Q> kp = make_kparams<T, L, SN>(p);
    hipLaunchKernelGGL((k_init<L, T, SN>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, d.aux, d.flags, (SN*)d.N[cur],
                       (T*)d.B, (T*)d.phi[0], (T*)d.phi[1], (T*)d.G[0], (T*)d.G[1], kp, (T)p.phi_solid, p.n);
    (void)ps;
    return hipGetLastError();
}

// which: 0 = N plane `dir` of buffer cur, 1 = B plane `dir` (planes buffer
// in LIQ_PLANES, formed from the compact record in LIQ_RECORD), 2 = phi buffer `dir`,
// 3 = N plane `dir` as the stored offset N_i - chi_i (exact in FP64).
template <class L, class T, class SN>
static hipError_t plane_out_t(const DevState& d, const StepParams& p, int which, int dir, int cur, int ps, int liq,
                              hipStream_t st) {
    if (which == 1 && liq == LIQ_PHI) return hipErrorInvalidValue;   // no B and no record to form it from
    if (which == 1 && liq == LIQ_RECORD) {
        const KParams<T, L::Q> kp = make_kparams<T, L, SN>(p);
        if (d.sparse) {
            hipLaunchKernelGGL((k_compact_B_sparse<L, T, SN>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, d.nbt,
                               d.n_fluid, (const SN*)d.N[cur], (const T*)d.phi[ps], (const T*)d.G[cur], d.flags, kp,
                               dir, p.n, d.aux);
            return hipGetLastError();
        }
        const int bx = row_block(p.nx);
        hipLaunchKernelGGL((k_compact_B_plane<L, T, SN>), row_grid(p, bx), dim3(bx), 0, st, (const SN*)d.N[cur],
                           (const T*)d.phi[ps], (const T*)d.G[cur], d.flags, kp, dir, d.aux);
        return hipGetLastError();
    }
    if ((which == 0 || which == 3) && d.sparse) {
        const int odir = L::opp[dir];
        hipLaunchKernelGGL((k_nplane_out_pull<T, SN>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st,
                           (const SN*)d.N[cur], d.nbt + (int64_t)(odir > 0 ? odir - 1 : 0) * d.n_fluid, d.flags, dir,
                           odir, p.S, d.n_fluid, which == 0 ? (T)p.chi[dir] : T(0),
                           (T)(NStore<T, SN>::scaled ? N16_SCALE : 1.0), d.aux, p.n);
        return hipGetLastError();
    }
    if (which == 0 || which == 3) {
        hipLaunchKernelGGL((k_nplane_out<T, SN>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st,
                           (const SN*)d.N[cur] + (int64_t)dir * p.S, d.flags, which == 0 ? (T)p.chi[dir] : T(0),
                           (T)(NStore<T, SN>::scaled ? N16_SCALE : 1.0), d.aux, p.n);
        return hipGetLastError();
    }
    const T* src = which == 1 ? (const T*)d.B + (int64_t)dir * p.S : (const T*)d.phi[dir];
    hipLaunchKernelGGL((k_plane_out<T>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, src, d.flags,
                       which < 2 ? 1 : 0, d.aux, p.n);
    return hipGetLastError();
}

// which: 0 = N plane `dir` of buffer cur, 1 = B plane `dir` (planes buffer),
// 2 = solid entries of both phi buffers, 3 = N plane `dir` from offsets,
// 4 = fluid entries of phi buffer `dir`.
template <class L, class T, class SN>
static hipError_t plane_in_t(const DevState& d, const StepParams& p, int which, int dir, int cur, hipStream_t st) {
    if (which == 4) {
        hipLaunchKernelGGL((k_fluid_in<T>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, d.aux, d.flags,
                           (T*)d.phi[dir], p.n);
        return hipGetLastError();
    }
    if (which == 2) {
        hipLaunchKernelGGL((k_solid_in<T>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, d.aux, d.flags,
                           (T*)d.phi[0], (T*)d.phi[1], p.n);
        return hipGetLastError();
    }
    if ((which == 0 || which == 3) && d.sparse) {
        const int odir = L::opp[dir];
        hipLaunchKernelGGL((k_nplane_in_pull<T, SN>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, d.aux,
                           (SN*)d.N[cur], d.nbt + (int64_t)(odir > 0 ? odir - 1 : 0) * d.n_fluid, d.flags, dir, odir,
                           p.S, d.n_fluid, which == 0 ? (T)p.chi[dir] : T(0),
                           (T)(NStore<T, SN>::scaled ? 1.0 / N16_SCALE : 1.0), p.n);
        return hipGetLastError();
    }
    if (which == 0 || which == 3) {
        hipLaunchKernelGGL((k_nplane_in<T, SN>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, d.aux,
                           (SN*)d.N[cur] + (int64_t)dir * p.S, which == 0 ? (T)p.chi[dir] : T(0),
                           (T)(NStore<T, SN>::scaled ? 1.0 / N16_SCALE : 1.0), p.n);
        return hipGetLastError();
    }
    T* dst = (T*)d.B + (int64_t)dir * p.S;
    hipLaunchKernelGGL((k_plane_in<T>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, d.aux, dst, p.n);
    return hipGetLastError();
}

// Dispatch on lattice and arithmetic type.
#define LBM_DISPATCH_L(FN, T, SN, ...)                                                \
    do {                                                                              \
        if (lattice == 0) return FN<LatD2Q9, T, SN>(__VA_ARGS__);                     \
        return FN<LatD3Q19, T, SN>(__VA_ARGS__);                                      \
    } while (0)
#define LBM_DISPATCH(FN, ...)                                                         \
    do {                                                                              \
        switch (prec) {                                                               \
        case P_FP64: LBM_DISPATCH_L(FN, double, double, __VA_ARGS__);                 \
        case P_FP32: LBM_DISPATCH_L(FN, float, float, __VA_ARGS__);                   \
        case P_FP16_OFS: LBM_DISPATCH_L(FN, float, _Float16, __VA_ARGS__);            \
        case P_BF16_OFS: LBM_DISPATCH_L(FN, float, __bf16, __VA_ARGS__);              \
        default: return hipErrorNotSupported;                                         \
        }                                                                             \
    } while (0)

hipError_t launch_step(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int cur, int ps, int liq,
                       hipStream_t st) {
    LBM_DISPATCH(step_t, d, p, cur, ps, liq, st);
}
hipError_t launch_phase(int lattice, uint32_t prec, int phase, const DevState& d, const StepParams& p, int cur,
                        int ps, int liq, hipStream_t st) {
    LBM_DISPATCH(phase_t, phase, d, p, cur, ps, liq, st);
}
hipError_t launch_colour(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int cur, int ps,
                         int liq, hipStream_t st) {
    LBM_DISPATCH(colour_t, d, p, cur, ps, liq, st);
}
hipError_t launch_macro(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int cur, int ps,
                        hipStream_t st) {
    LBM_DISPATCH(macro_t, d, p, cur, ps, st);
}
hipError_t launch_reduce(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int cur, int ps,
                         int liq, const ReduceScratch& rs, hipStream_t st) {
    LBM_DISPATCH(reduce_t, d, p, cur, ps, liq, rs, st);
}

// Scratch of the diagnostics in device memory of the library's own, for
// callers that cannot allocate (lbm_observe_static): the reduction partials,
// the non-finite counters and the result.  Each device holds one copy; in
// host code `scratch` names no device address, so its address is taken with
// hipGetSymbolAddress once per device (device current) and kept.
constexpr size_t SCRATCH_PARTIAL = (size_t)REDUCE_BLOCKS * 8 * sizeof(double);
constexpr size_t SCRATCH_COUNTS = ((size_t)(REDUCE_BLOCKS + 1) * sizeof(int64_t) + 255) / 256 * 256;
constexpr size_t SCRATCH_BYTES = SCRATCH_PARTIAL + SCRATCH_COUNTS + 256;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_addr[MAX_DEVICES] = {};

hipError_t static_reduce_scratch(int device, ReduceScratch& out) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[device]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (prev != device) {
            const hipError_t e2 = hipSetDevice(prev);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        g_scratch_addr[device] = ptr;
    }
    unsigned char* base = (unsigned char*)g_scratch_addr[device];
    out.partial = (double*)base;
    out.nonfinite = (int64_t*)(base + SCRATCH_PARTIAL);
    out.result = (double*)(base + SCRATCH_PARTIAL + SCRATCH_COUNTS);
    return hipSuccess;
}
hipError_t launch_init(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int cur, int ps,
                       hipStream_t st) {
    LBM_DISPATCH(init_t, d, p, cur, ps, st);
}
hipError_t launch_plane_out(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int which, int dir,
                            int cur, int ps, int liq, hipStream_t st) {
    LBM_DISPATCH(plane_out_t, d, p, which, dir, cur, ps, liq, st);
}
hipError_t launch_plane_in(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int which, int dir,
                           int cur, hipStream_t st) {
    LBM_DISPATCH(plane_in_t, d, p, which, dir, cur, st);
}

// Per job: the descriptor and two block offsets; per group: alignment slack.
static size_t batch_job_bytes() { return sizeof(BJob<LatD3Q19, double, double>) + 2 * sizeof(int64_t); }
size_t batch_group_bytes(int njobs) { return (size_t)njobs * batch_job_bytes() + 1024; }
size_t batch_table_bytes(int max_jobs) { return (size_t)max_jobs * batch_job_bytes() + 8 * 1024; }

template <class L, class T, class SN>
static hipError_t batch_t(const BatchJobHost* jobs, int nj, void* table, size_t table_bytes, int64_t nsteps,
                          hipStream_t st, std::vector<char>& staging) {
    using J = BJob<L, T, SN>;
    const size_t jb = ((sizeof(J) * (size_t)nj) + 255) & ~size_t(255);
    const size_t sb = (((size_t)nj + 1) * sizeof(int64_t) + 255) & ~size_t(255);
    const size_t need = jb + 2 * sb;
    if (need > table_bytes) return hipErrorInvalidValue;
    staging.assign(need, 0);
    J* dj = reinterpret_cast<J*>(staging.data());
    int64_t* rs = reinterpret_cast<int64_t*>(staging.data() + jb);
    int64_t* gs = reinterpret_cast<int64_t*>(staging.data() + jb + sb);
    rs[0] = gs[0] = 0;
    for (int j = 0; j < nj; j++) {
        const BatchJobHost& h = jobs[j];
        J& o = dj[j];
        o.P = make_kparams<T, L, SN>(h.p);
        for (int b = 0; b < 2; b++) {
            o.N[b] = (const SN*)h.d.N[b];
            o.G[b] = (T*)h.d.G[b];
            o.phi[b] = (T*)h.d.phi[b];
        }
        o.B = (const T*)h.d.B;
        o.flags = h.d.flags;
        o.g_node = h.d.g_node;
        o.g_corner = h.d.g_corner;
        o.g_w = (const T*)h.d.g_w;
        o.g_mask = h.d.g_mask;
        o.n_ghost = h.d.n_ghost;
        o.rule = h.p.ghost_rule;
        o.E = (T)h.p.exp_eps;
        o.eps = (T)h.p.eps;
        o.cur0 = h.cur0;
        o.ps0 = h.ps0;
        o.planes0 = h.planes0;
        o.nxb = (h.p.nx + BATCH_BX - 1) / BATCH_BX;
        rs[j + 1] = rs[j] + (int64_t)o.nxb * h.p.ny * h.p.nz;
        gs[j + 1] = gs[j] + (h.d.n_ghost + BATCH_BX - 1) / BATCH_BX;
    }
    char* tb = (char*)table;
    hipError_t e = hipMemcpyAsync(tb, staging.data(), need, hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    const J* djd = (const J*)tb;
    const int64_t* rsd = (const int64_t*)(tb + jb);
    const int64_t* gsd = (const int64_t*)(tb + jb + sb);
    int active = nj;
    for (int64_t k = 0; k < nsteps; k++) {
        while (active > 0 && jobs[active - 1].steps <= k) active--;
        if (active == 0) break;
        hipLaunchKernelGGL((kb_colour<L, T, SN>), dim3((unsigned)rs[active]), dim3(BATCH_BX), 0, st, djd, rsd, active,
                           k);
        if (gs[active] > 0)
            hipLaunchKernelGGL((kb_ghost<L, T, SN>), dim3((unsigned)gs[active]), dim3(BATCH_BX), 0, st, djd, gsd,
                               active, k);
        hipLaunchKernelGGL((kb_collide<L, T, SN>), dim3((unsigned)rs[active]), dim3(BATCH_BX), 0, st, djd, rsd,
                           active, k);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_batch(int lattice, uint32_t prec, const BatchJobHost* jobs, int njobs, void* table,
                        size_t table_bytes, int64_t nsteps, hipStream_t st, std::vector<char>& staging) {
    LBM_DISPATCH(batch_t, jobs, njobs, table, table_bytes, nsteps, st, staging);
}

hipError_t launch_solid_phi(uint32_t prec, const DevState& d, const StepParams& p, hipStream_t st) {
    if (prec == P_FP64) {
        hipLaunchKernelGGL((k_solid_phi<double>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, d.flags,
                           (double*)d.phi[0], (double*)d.phi[1], p.phi_solid, p.n);
    } else if (prec == P_FP32 || prec == P_FP16_OFS || prec == P_BF16_OFS) {
        hipLaunchKernelGGL((k_solid_phi<float>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, d.flags,
                           (float*)d.phi[0], (float*)d.phi[1], (float)p.phi_solid, p.n);
    } else {
        return hipErrorNotSupported;
    }
    return hipGetLastError();
}

}  // namespace lbm
