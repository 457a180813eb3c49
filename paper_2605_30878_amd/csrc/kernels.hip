// kernels.hip -- HIP kernels (gfx950) of one colour-gradient lattice
// Boltzmann time step with the ghost-node wetting condition.
//
// Per step, on one stream:
//   k_colour   phi = sum_i B_i at fluid nodes                      (Eq. A13)
//   k_ghost    phi_G = phi_F / (phi_F + (1 - phi_F) exp(eps))      (Eq. 9)
//              over the compacted ghost list; phi_F interpolated at
//              x_F = x_G + n_s from one snapshot (Jacobi)
//   k_collide  fused: colour stencils, forces (Eq. 4, A9-A11), MRT
//              collision (Eq. A1) in projection form, recolouring (Eq. A12),
//              push streaming of N and B (Eq. A16-A17) with halfway
//              bounce-back at solid links
// Populations are SoA planes [Q][S], double-buffered; phi is double-buffered
// so that the ghost update reads last step's solid values while writing the
// new ones.  Every step is HBM-bound (about 4 Q s bytes per fluid node);
// nothing is a dense contraction, so no MFMA is used.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <utility>

#include "lattice.h"
#include "launch.h"

namespace lbm {

// ------------------------------------------------------------------ helpers
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// c * v for a lattice component c in {-1, 0, 1}, resolved at compile time.
template <int C, class T>
__device__ __forceinline__ T cmul(T v) {
    if constexpr (C == 1) return v;
    else if constexpr (C == -1) return -v;
    else return T(0);
}

// Arithmetic-type constants of a run.
template <class T, int Q>
struct KParams {
    T rho_g, drho;          // rho = rho_g + drho phi
    T inv_nu_g, dinv_nu;    // 1/nu = inv_nu_g + dinv_nu phi
    T sigma, W, inv_W;
    T g[3];
    T chi[Q];
    T chi0;
    T n_thresh2;            // |grad phi|^2 below which n_phi = 0
    int nx, ny, nz;
    int64_t S;
};

template <class T, class L>
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
    k.chi0 = T(p.chi0);
    // |grad phi| > 1e-12 (FP64) or > 1e-7 (FP32) defines the interface normal
    k.n_thresh2 = std::is_same<T, double>::value ? T(1e-24) : T(1e-14);
    k.nx = p.nx;
    k.ny = p.ny;
    k.nz = p.nz;
    k.S = p.S;
    return k;
}

// Node output of the macroscopic stage.
template <class T>
struct Macro {
    T phi, rho, tau, p;
    T grad[3];
    T u[3];
    T a[3];  // F / rho
};

// Macroscopic stage of one fluid node: colour stencils, mixture properties,
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
    // Isotropic stencils: grad = 3 sum w c phi ; lap = 6 sum_{i>0} w (phi_i - phi)
    T gx = 0, gy = 0, gz = 0, lap = 0;
    static_for<1, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr T wi = T(L::w[i]);
        gx += cmul<L::c[i][0]>(wi * ph[i]);
        gy += cmul<L::c[i][1]>(wi * ph[i]);
        gz += cmul<L::c[i][2]>(wi * ph[i]);
        lap += wi * ph[i];
    });
    gx *= T(3);
    gy *= T(3);
    gz *= T(3);
    lap = T(6) * (lap - (T(1) - w0) * phi);
    m.grad[0] = gx;
    m.grad[1] = gy;
    m.grad[2] = gz;
    // Mixture density and harmonic viscosity (text after Eq. 3).
    const T rho = P.rho_g + P.drho * phi;
    const T inv_nu = P.inv_nu_g + P.dinv_nu * phi;
    const T tau = T(0.5) + T(3) / inv_nu;
    m.rho = rho;
    m.tau = tau;
    // Moments of N.
    T jx = 0, jy = 0, jz = 0, s = 0;
    T pxx = 0, pyy = 0, pzz = 0, pxy = 0, pyz = 0, pxz = 0;
    static_for<1, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        const T n = N[i];
        s += n;
        jx += cmul<cx>(n);
        jy += cmul<cy>(n);
        jz += cmul<cz>(n);
        if constexpr (cx != 0) pxx += n;
        if constexpr (cy != 0) pyy += n;
        if constexpr (cz != 0) pzz += n;
        if constexpr (cx * cy != 0) pxy += cmul<cx * cy>(n);
        if constexpr (cy * cz != 0) pyz += cmul<cy * cz>(n);
        if constexpr (cx * cz != 0) pxz += cmul<cx * cz>(n);
    });
    Pi[0] = pxx; Pi[1] = pyy; Pi[2] = pzz; Pi[3] = pxy; Pi[4] = pyz; Pi[5] = pxz;
    // Eq. A15 with u0 = sum c N (the forced u needs F_p(p)).
    const T uu0 = jx * jx + jy * jy + jz * jz;
    const T p = ((s - (T(1) - P.chi0)) * T(1.0 / 3.0) - T(0.5) * w0 * uu0) / (T(1) - w0);
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
    const T kv = -(tau - T(0.5)) / tau;     // cs^2 (tau - 1/2) * (-1/(tau cs^2))
    const T grx = P.drho * gx, gry = P.drho * gy, grz = P.drho * gz;   // grad rho
    T Fx = mu * gx - p * grx + kv * (dxx * grx + dxy * gry + dxz * grz) + rho * P.g[0];
    T Fy = mu * gy - p * gry + kv * (dxy * grx + dyy * gry + dyz * grz) + rho * P.g[1];
    T Fz = mu * gz - p * grz + kv * (dxz * grx + dyz * gry + dzz * grz) + rho * P.g[2];
    if constexpr (L::D == 2) Fz = 0;
    const T inv_rho = T(1) / rho;
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
// then recolouring (Eq. A12) with the amplitude max(phi(1 - phi), 0).
template <class L, class T>
__device__ __forceinline__ void collide_stage(const Macro<T>& m, const T (&Pi)[6], const KParams<T, L::Q>& P,
                                              T (&Ns)[L::Q], T (&Bs)[L::Q]) {
    constexpr int Q = L::Q;
    constexpr T w0 = T(L::w[0]);
    const T ux = m.u[0], uy = m.u[1], uz = m.u[2];
    const T uu = ux * ux + uy * uy + uz * uz;
    const T p3 = T(3) * m.p;                      // p / cs^2
    const T omega = T(1) - T(1) / m.tau;
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
    // Recolouring normal and amplitude.
    const T gx = m.grad[0], gy = m.grad[1], gz = m.grad[2];
    const T gn2 = gx * gx + gy * gy + gz * gz;
    T nx = 0, ny = 0, nz = 0;
    if (gn2 > P.n_thresh2) {
        const T inv = T(1) / sqrt(gn2);
        nx = gx * inv;
        ny = gy * inv;
        nz = gz * inv;
    }
    T amp = m.phi * (T(1) - m.phi);
    amp = amp > T(0) ? amp : T(0);
    const T kseg = T(2) * P.inv_W * amp;
    const T phi = m.phi;
    // i = 0
    {
        const T neq = P.chi[0] - (T(1) - w0) * p3 - w0 * T(1.5) * uu;
        T proj = 0;
        if constexpr (L::D == 2) {
            proj = 0;  // rest direction has zero stress moments
        } else {
            proj = 0;
        }
        Ns[0] = neq + omega * proj;
        Bs[0] = phi * Ns[0];
    }
    static_for<1, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        constexpr T wi = T(L::w[i]);
        const T cu = cmul<cx>(ux) + cmul<cy>(uy) + cmul<cz>(uz);
        const T ca = cmul<cx>(m.a[0]) + cmul<cy>(m.a[1]) + cmul<cz>(m.a[2]);
        const T neq = P.chi[i] + wi * (p3 + T(3) * cu + T(4.5) * cu * cu - T(1.5) * uu);
        // projection onto the stress rows, m_k(i) evaluated at compile time
        T proj;
        if constexpr (L::D == 2) {
            proj = T(cx * cx - cy * cy) * s1 + T(cx * cy) * s2;
        } else {
            proj = T(2 * cx * cx - cy * cy - cz * cz) * s1 + T(cy * cy - cz * cz) * s2 + T(cx * cy) * s3 +
                   T(cy * cz) * s4 + T(cx * cz) * s5;
        }
        const T ns = neq + T(1.5) * wi * ca + proj;   // F_i / 2 = (3 w_i a.c_i) / 2
        Ns[i] = ns;
        const T cn = cmul<cx>(nx) + cmul<cy>(ny) + cmul<cz>(nz);
        const T neq0 = P.chi[i] + wi * p3;            // N^eq(u = 0, p), i != 0
        Bs[i] = phi * ns + kseg * cn * neq0;
    });
}

// Neighbour index tables of a node: nb[i] = index of x + c_i (periodic).
template <class L>
__device__ __forceinline__ void neighbours(int ix, int iy, int iz, int nx, int ny, int nz, int64_t (&nb)[L::Q]) {
    const int xm = ix == 0 ? nx - 1 : ix - 1, xp = ix == nx - 1 ? 0 : ix + 1;
    const int ym = iy == 0 ? ny - 1 : iy - 1, yp = iy == ny - 1 ? 0 : iy + 1;
    int zm = 0, zp = 0;
    if constexpr (L::D == 3) {
        zm = iz == 0 ? nz - 1 : iz - 1;
        zp = iz == nz - 1 ? 0 : iz + 1;
    }
    static_for<0, L::Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int cx = L::c[i][0], cy = L::c[i][1], cz = L::c[i][2];
        const int X = cx == 0 ? ix : (cx > 0 ? xp : xm);
        const int Y = cy == 0 ? iy : (cy > 0 ? yp : ym);
        const int Z = cz == 0 ? iz : (cz > 0 ? zp : zm);
        nb[i] = (int64_t)X + (int64_t)nx * ((int64_t)Y + (int64_t)ny * Z);
    });
}

// ------------------------------------------------------------------ kernels
// phi = sum_i B_i (i ascending) at fluid nodes.
template <class L, class T>
__global__ __launch_bounds__(256) void k_colour(const T* __restrict__ B, T* __restrict__ phi,
                                                const uint8_t* __restrict__ flags, int64_t n, int64_t S) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    if (flags[x] & FLAG_SOLID) return;
    T acc = 0;
#pragma unroll
    for (int i = 0; i < L::Q; i++) acc += B[(int64_t)i * S + x];
    phi[x] = acc;
}

// Ghost update over the compacted list (Jacobi): fluid corners from the
// colour field just written, solid corners from last step's values.
template <class T, int NC>
__global__ __launch_bounds__(256) void k_ghost(const int32_t* __restrict__ g_node, const int32_t* __restrict__ g_corner,
                                               const T* __restrict__ g_w, const uint8_t* __restrict__ g_mask, int ng,
                                               const T* __restrict__ phi_prev, T* __restrict__ phi_work, T E, T eps,
                                               int rule) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
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
    } else if (eps == T(0)) {
        out = f;                                           // Eq. 10 at its removable singularity
    } else {
        const T a = T(1) + T(0.5) * eps;                   // Eq. 10
        out = (T(2) / eps) * (a - sqrt(a * a - T(2) * eps * f)) - f;
    }
    phi_work[g_node[g]] = out;
}

// Fused stencil + forces + collision + recolouring + push streaming with
// halfway bounce-back.  One thread per node of an x-row; grid (x-blocks, ny, nz).
template <class L, class T>
__global__ __launch_bounds__(256) void k_collide_stream(const T* __restrict__ Nsrc, T* __restrict__ Ndst,
                                                        T* __restrict__ Bdst, const T* __restrict__ phi,
                                                        const uint8_t* __restrict__ flags, KParams<T, L::Q> P) {
    constexpr int Q = L::Q;
    const int ix = blockIdx.x * blockDim.x + threadIdx.x;
    if (ix >= P.nx) return;
    const int iy = blockIdx.y, iz = blockIdx.z;
    const int64_t x = (int64_t)ix + (int64_t)P.nx * ((int64_t)iy + (int64_t)P.ny * iz);
    const uint8_t f = flags[x];
    if (f & FLAG_SOLID) return;
    int64_t nb[Q];
    neighbours<L>(ix, iy, iz, P.nx, P.ny, P.nz, nb);
    T N[Q], ph[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) N[i] = Nsrc[(int64_t)i * P.S + x];
#pragma unroll
    for (int i = 0; i < Q; i++) ph[i] = phi[nb[i]];
    Macro<T> m;
    T Pi[6];
    macro_stage<L, T>(N, ph, P, m, Pi);
    T Ns[Q], Bs[Q];
    collide_stage<L, T>(m, Pi, P, Ns, Bs);
    const int64_t S = P.S;
    if (f & FLAG_NEAR_SOLID) {
        static_for<0, Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if (flags[nb[i]] & FLAG_SOLID) {
                Ndst[(int64_t)L::opp[i] * S + x] = Ns[i];
                Bdst[(int64_t)L::opp[i] * S + x] = Bs[i];
            } else {
                Ndst[(int64_t)i * S + nb[i]] = Ns[i];
                Bdst[(int64_t)i * S + nb[i]] = Bs[i];
            }
        });
    } else {
#pragma unroll
        for (int i = 0; i < Q; i++) {
            Ndst[(int64_t)i * S + nb[i]] = Ns[i];
            Bdst[(int64_t)i * S + nb[i]] = Bs[i];
        }
    }
}

// Macroscopic fields (u, p) of every node into FP64 planes; solids get 0.
template <class L, class T>
__global__ __launch_bounds__(256) void k_macro(const T* __restrict__ Nsrc, const T* __restrict__ phi,
                                               const uint8_t* __restrict__ flags, KParams<T, L::Q> P,
                                               double* __restrict__ aux) {
    constexpr int Q = L::Q;
    const int ix = blockIdx.x * blockDim.x + threadIdx.x;
    if (ix >= P.nx) return;
    const int iy = blockIdx.y, iz = blockIdx.z;
    const int64_t x = (int64_t)ix + (int64_t)P.nx * ((int64_t)iy + (int64_t)P.ny * iz);
    const int64_t S = P.S;
    if (flags[x] & FLAG_SOLID) {
        aux[x] = 0.0;
        aux[S + x] = 0.0;
        aux[2 * S + x] = 0.0;
        aux[3 * S + x] = 0.0;
        return;
    }
    int64_t nb[Q];
    neighbours<L>(ix, iy, iz, P.nx, P.ny, P.nz, nb);
    T N[Q], ph[Q];
#pragma unroll
    for (int i = 0; i < Q; i++) N[i] = Nsrc[(int64_t)i * S + x];
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

// Diagnostics, stage 1: each block reduces a fixed strided set of nodes in a
// fixed order (deterministic for a fixed grid).  Values: sum phi,
// sum (1 - phi), sum rho u (3), max |u|, sum rho |u|^2 / 2.
template <class L, class T>
__global__ __launch_bounds__(256) void k_reduce1(const T* __restrict__ N, const T* __restrict__ B,
                                                 const T* __restrict__ phi, const uint8_t* __restrict__ flags,
                                                 const double* __restrict__ aux, int64_t n, int64_t S, double rho_g,
                                                 double drho, double* __restrict__ partial,
                                                 int64_t* __restrict__ nonfinite) {
    __shared__ double sh[7][256];
    __shared__ int64_t shn[256];
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
        for (int i = 0; i < L::Q; i++) {
            if (!isfinite((double)N[(int64_t)i * S + x])) bad++;
            if (!isfinite((double)B[(int64_t)i * S + x])) bad++;
        }
    }
    const int t = threadIdx.x;
    for (int k = 0; k < 7; k++) sh[k][t] = v[k];
    shn[t] = bad;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
            for (int k = 0; k < 7; k++) {
                if (k == 5) sh[k][t] = sh[k][t] > sh[k][t + off] ? sh[k][t] : sh[k][t + off];
                else sh[k][t] += sh[k][t + off];
            }
            shn[t] += shn[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        for (int k = 0; k < 7; k++) partial[(int64_t)blockIdx.x * 8 + k] = sh[k][0];
        nonfinite[blockIdx.x] = shn[0];
    }
}

// Diagnostics, stage 2: one block folds the partials in a fixed order.
__global__ __launch_bounds__(256) void k_reduce2(const double* __restrict__ partial,
                                                 const int64_t* __restrict__ nonfinite, int nblocks,
                                                 double* __restrict__ result, int64_t* __restrict__ nf_out) {
    __shared__ double sh[7][256];
    __shared__ int64_t shn[256];
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
    for (int k = 0; k < 7; k++) sh[k][t] = v[k];
    shn[t] = bad;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (t < off) {
            for (int k = 0; k < 7; k++) {
                if (k == 5) sh[k][t] = sh[k][t] > sh[k][t + off] ? sh[k][t] : sh[k][t + off];
                else sh[k][t] += sh[k][t + off];
            }
            shn[t] += shn[t + off];
        }
        __syncthreads();
    }
    if (t == 0) {
        for (int k = 0; k < 7; k++) result[k] = sh[k][0];
        *nf_out = shn[0];
    }
}

// Start of a run: N = chi, B = phi chi at fluid nodes (u = p = 0), solid
// phi = phi_solid in both colour buffers.
template <class L, class T>
__global__ __launch_bounds__(256) void k_init(const double* __restrict__ phi0, const uint8_t* __restrict__ flags,
                                              T* __restrict__ N, T* __restrict__ B, T* __restrict__ phiA,
                                              T* __restrict__ phiB, KParams<T, L::Q> P, T phi_solid, int64_t n) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int64_t S = P.S;
    if (flags[x] & FLAG_SOLID) {
        phiA[x] = phi_solid;
        phiB[x] = phi_solid;
#pragma unroll
        for (int i = 0; i < L::Q; i++) {
            N[(int64_t)i * S + x] = T(0);
            B[(int64_t)i * S + x] = T(0);
        }
        return;
    }
    const T ph = (T)phi0[x];
    phiA[x] = ph;
    phiB[x] = ph;
#pragma unroll
    for (int i = 0; i < L::Q; i++) {
        N[(int64_t)i * S + x] = P.chi[i];
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

template <class T>
__global__ __launch_bounds__(256) void k_plane_in(const double* __restrict__ src, T* __restrict__ dst, int64_t n) {
    const int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    dst[x] = (T)src[x];
}

// ------------------------------------------------------------------ launchers
static inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

static inline dim3 row_grid(const StepParams& p, int bx) {
    return dim3((unsigned)((p.nx + bx - 1) / bx), (unsigned)p.ny, (unsigned)p.nz);
}

static inline int row_block(int nx) { return nx >= 256 ? 256 : (nx >= 128 ? 128 : 64); }

template <class L, class T>
static hipError_t phase_t(int phase, const DevState& d, const StepParams& p, int cur, int ps, hipStream_t st) {
    T* work = (T*)d.phi[1 - ps];
    if (phase == 0) {
        hipLaunchKernelGGL((k_colour<L, T>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, (const T*)d.B[cur], work,
                           d.flags, p.n, p.S);
    } else if (phase == 1) {
        if (d.n_ghost > 0) {
            hipLaunchKernelGGL((k_ghost<T, L::NC>), dim3(blocks_for(d.n_ghost, 256)), dim3(256), 0, st, d.g_node,
                               d.g_corner, (const T*)d.g_w, d.g_mask, d.n_ghost, (const T*)d.phi[ps], work,
                               (T)p.exp_eps, (T)p.eps, p.ghost_rule);
        }
    } else {
        const KParams<T, L::Q> kp = make_kparams<T, L>(p);
        const int bx = row_block(p.nx);
        hipLaunchKernelGGL((k_collide_stream<L, T>), row_grid(p, bx), dim3(bx), 0, st, (const T*)d.N[cur],
                           (T*)d.N[1 - cur], (T*)d.B[1 - cur], (const T*)work, d.flags, kp);
    }
    return hipGetLastError();
}

template <class L, class T>
static hipError_t colour_t(const DevState& d, const StepParams& p, int cur, int ps, hipStream_t st) {
    hipError_t e = phase_t<L, T>(0, d, p, cur, ps, st);
    if (e != hipSuccess) return e;
    return phase_t<L, T>(1, d, p, cur, ps, st);
}

template <class L, class T>
static hipError_t step_t(const DevState& d, const StepParams& p, int cur, int ps, hipStream_t st) {
    for (int ph = 0; ph < 3; ph++) {
        hipError_t e = phase_t<L, T>(ph, d, p, cur, ps, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <class L, class T>
static hipError_t macro_t(const DevState& d, const StepParams& p, int cur, int ps, hipStream_t st) {
    const KParams<T, L::Q> kp = make_kparams<T, L>(p);
    const int bx = row_block(p.nx);
    hipLaunchKernelGGL((k_macro<L, T>), row_grid(p, bx), dim3(bx), 0, st, (const T*)d.N[cur],
                       (const T*)d.phi[1 - ps], d.flags, kp, d.aux);
    return hipGetLastError();
}

template <class L, class T>
static hipError_t reduce_t(const DevState& d, const StepParams& p, int cur, int ps, hipStream_t st) {
    hipLaunchKernelGGL((k_reduce1<L, T>), dim3(REDUCE_BLOCKS), dim3(256), 0, st, (const T*)d.N[cur],
                       (const T*)d.B[cur], (const T*)d.phi[1 - ps], d.flags, d.aux, p.n, p.S, p.rho_g,
                       p.rho_l - p.rho_g, d.partial, d.nonfinite);
    hipLaunchKernelGGL(k_reduce2, dim3(1), dim3(256), 0, st, d.partial, d.nonfinite, REDUCE_BLOCKS, d.result,
                       d.nonfinite + REDUCE_BLOCKS);
    return hipGetLastError();
}

template <class L, class T>
static hipError_t init_t(const DevState& d, const StepParams& p, int cur, int ps, hipStream_t st) {
    const KParams<T, L::Q> kp = make_kparams<T, L>(p);
    hipLaunchKernelGGL((k_init<L, T>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, d.aux, d.flags, (T*)d.N[cur],
                       (T*)d.B[cur], (T*)d.phi[0], (T*)d.phi[1], kp, (T)p.phi_solid, p.n);
    (void)ps;
    return hipGetLastError();
}

template <class L, class T>
static hipError_t plane_out_t(const DevState& d, const StepParams& p, int which, int dir, int cur, hipStream_t st) {
    const T* src = which == 0 ? (const T*)d.N[cur] + (int64_t)dir * p.S
                 : which == 1 ? (const T*)d.B[cur] + (int64_t)dir * p.S
                              : (const T*)d.phi[dir];
    hipLaunchKernelGGL((k_plane_out<T>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, src, d.flags,
                       which < 2 ? 1 : 0, d.aux, p.n);
    return hipGetLastError();
}

template <class L, class T>
static hipError_t plane_in_t(const DevState& d, const StepParams& p, int which, int dir, int cur, hipStream_t st) {
    T* dst = which == 0 ? (T*)d.N[cur] + (int64_t)dir * p.S
           : which == 1 ? (T*)d.B[cur] + (int64_t)dir * p.S
                        : (T*)d.phi[dir];
    hipLaunchKernelGGL((k_plane_in<T>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, d.aux, dst, p.n);
    return hipGetLastError();
}

// Dispatch on lattice and arithmetic type.
#define LBM_DISPATCH(FN, ...)                                                         \
    do {                                                                              \
        if (prec == P_FP64) {                                                         \
            if (lattice == 0) return FN<LatD2Q9, double>(__VA_ARGS__);                \
            return FN<LatD3Q19, double>(__VA_ARGS__);                                 \
        }                                                                             \
        if (prec == P_FP32) {                                                         \
            if (lattice == 0) return FN<LatD2Q9, float>(__VA_ARGS__);                 \
            return FN<LatD3Q19, float>(__VA_ARGS__);                                  \
        }                                                                             \
        return hipErrorNotSupported;                                                  \
    } while (0)

hipError_t launch_step(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int cur, int ps,
                       hipStream_t st) {
    LBM_DISPATCH(step_t, d, p, cur, ps, st);
}
hipError_t launch_phase(int lattice, uint32_t prec, int phase, const DevState& d, const StepParams& p, int cur,
                        int ps, hipStream_t st) {
    LBM_DISPATCH(phase_t, phase, d, p, cur, ps, st);
}
hipError_t launch_colour(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int cur, int ps,
                         hipStream_t st) {
    LBM_DISPATCH(colour_t, d, p, cur, ps, st);
}
hipError_t launch_macro(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int cur, int ps,
                        hipStream_t st) {
    LBM_DISPATCH(macro_t, d, p, cur, ps, st);
}
hipError_t launch_reduce(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int cur, int ps,
                         hipStream_t st) {
    LBM_DISPATCH(reduce_t, d, p, cur, ps, st);
}
hipError_t launch_init(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int cur, int ps,
                       hipStream_t st) {
    LBM_DISPATCH(init_t, d, p, cur, ps, st);
}
hipError_t launch_plane_out(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int which, int dir,
                            int cur, hipStream_t st) {
    LBM_DISPATCH(plane_out_t, d, p, which, dir, cur, st);
}
hipError_t launch_plane_in(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int which, int dir,
                           int cur, hipStream_t st) {
    LBM_DISPATCH(plane_in_t, d, p, which, dir, cur, st);
}
hipError_t launch_solid_phi(uint32_t prec, const DevState& d, const StepParams& p, hipStream_t st) {
    if (prec == P_FP64) {
        hipLaunchKernelGGL((k_solid_phi<double>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, d.flags,
                           (double*)d.phi[0], (double*)d.phi[1], p.phi_solid, p.n);
    } else if (prec == P_FP32) {
        hipLaunchKernelGGL((k_solid_phi<float>), dim3(blocks_for(p.n, 256)), dim3(256), 0, st, d.flags,
                           (float*)d.phi[0], (float*)d.phi[1], (float)p.phi_solid, p.n);
    } else {
        return hipErrorNotSupported;
    }
    return hipGetLastError();
}

}  // namespace lbm
