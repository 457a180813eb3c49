// launch.h -- interface between the host library (api.cpp) and the HIP
// kernels (kernels.hip).  Plain structs, no HIP types beyond the stream.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace lbm {

// Model constants of one run, FP64 on the host; the launchers round them to
// the arithmetic type of the run.
struct StepParams {
    double rho_l, rho_g;
    double inv_nu_l, inv_nu_g;  // 1/nu of each phase
    double sigma, W;
    double g[3];                // body acceleration
    double chi[19];             // colour weights (Eq. A7)
    double chi0;                // chi_0 = alpha
    double eps;                 // -(4/W) cos(theta)
    double exp_eps;             // exp(eps), formed on the host
    double phi_solid;           // (1 + cos theta) / 2
    int32_t ghost_rule;         // 0 = Eq. 9, 1 = Eq. 10
    int32_t nx, ny, nz;
    int64_t n;                  // nodes
    int64_t S;                  // stride between direction planes (elements)
};

// Device memory of one run, carved from the caller's buffer.
struct DevState {
    void* N[2];         // [Q][S] colour-blind populations, ping-pong
    void* B;            // [Q][S] liquid populations of the initial state or a restore
    void* G[2];         // [D+1][S] compact liquid record (G components, p), ping-pong with N
    void* phi[2];       // [S] colour field; phi[state] holds the solid values and
                        //     the previous step's phi at fluid nodes
    uint8_t* flags;     // [S] node classes
    int32_t* g_node;    // [n_ghost]
    int32_t* g_corner;  // [NC][n_ghost] interpolation corners of x_F
    void* g_w;          // [NC][n_ghost] interpolation weights
    uint8_t* g_mask;    // [n_ghost] bit k: corner k is a solid node
    int32_t n_ghost;
    double* aux;        // [4][S] FP64 scratch: u (3 planes) and p, or a field plane
    double* partial;    // [REDUCE_BLOCKS][8] reduction partials
    double* result;     // [8] reduced diagnostics
    int64_t* nonfinite; // [REDUCE_BLOCKS + 1]
    int32_t fused;      // 1: D3Q19 boxes tiled by the collide-colour tile step in the collide-colour form
    void* cross;        // inbox of the collide-colour step (values crossing a tile-chunk face)
    int64_t n_fluid;
    int32_t sparse;     // 1: fluid-only layout: planes hold one entry per slot (fluid nodes,
                        //    then ghost nodes, then one slot for every other solid node)
    uint32_t* nbt;      // [Q-1][n_fluid] sparse layout: slot of fluid node k + c_i
};

constexpr int REDUCE_BLOCKS = 1024;

// Liquid state entering a step.
enum Liquid : int {
    LIQ_RECORD = 0,   // compact record (G, p) of the last collide in G[cur], its phi in phi[ps]
    LIQ_PLANES = 1,   // B planes (initial state or a restore)
    LIQ_PHI = 2       // the step's phi already formed in phi[1 - ps] at fluid nodes (collide-colour step)
};

// Launches of one step, in order: 0 colour field (none in LIQ_PHI), 1 ghost
// update, 2 collide (two-pass collide-stream, or collide-colour), 3 colour
// fix-up (collide-colour form only).
constexpr int STEP_PHASES = 4;

enum Precision : uint32_t { P_FP64 = 0, P_FP32 = 1, P_FP16_OFS = 2, P_BF16_OFS = 3 };

// All launchers enqueue on `stream` and return hipGetLastError().
// `cur` is the population / compact-record buffer holding the state, `ps`
// the phi buffer holding the state's solid values (and, in LIQ_RECORD, the
// previous step's phi at fluid nodes); `liq` is the liquid state (Liquid).
hipError_t launch_step(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int cur, int ps, int liq,
                       hipStream_t stream);
// One phase of a step (STEP_PHASES, in order).
hipError_t launch_phase(int lattice, uint32_t prec, int phase, const DevState& d, const StepParams& p, int cur,
                        int ps, int liq, hipStream_t stream);
// True when a step of this run takes the collide-colour form (it then
// leaves LIQ_PHI, otherwise LIQ_RECORD).
bool step_fused(int lattice, const DevState& d, const StepParams& p);
// Device bytes of the collide-colour inbox (0 when the box does not take it).
size_t cross_bytes(int lattice, uint32_t prec, const StepParams& p);
// Colour field (phase 0) and ghost update into phi[1 - ps] (the phi the next step uses).
hipError_t launch_colour(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int cur, int ps,
                         int liq, hipStream_t stream);
// u and p of every fluid node into aux (after launch_colour).
hipError_t launch_macro(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int cur, int ps,
                        hipStream_t stream);
// Where the diagnostics reduce to: per-block partials [REDUCE_BLOCKS][8],
// non-finite counters [REDUCE_BLOCKS + 1] (the last one the total) and the
// result [8].  Every entry is overwritten by each reduction.
struct ReduceScratch {
    double* partial;
    int64_t* nonfinite;
    double* result;
};
// Diagnostics into rs (after launch_macro).
hipError_t launch_reduce(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int cur, int ps,
                         int liq, const ReduceScratch& rs, hipStream_t stream);
// The library's own reduction scratch on `device` (a static device array;
// its address is looked up once per device).
constexpr int MAX_DEVICES = 64;
hipError_t static_reduce_scratch(int device, ReduceScratch& out);
// Start of a run from the FP64 phi in aux[0]: N = chi, B = phi chi at fluid
// nodes, phi of solid nodes (both buffers) = phi_solid.
hipError_t launch_init(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int cur, int ps,
                       hipStream_t stream);
// Solid nodes of both phi buffers = phi_solid.
hipError_t launch_solid_phi(uint32_t prec, const DevState& d, const StepParams& p, hipStream_t stream);
// One plane to FP64 aux[0].  which: 0 = N plane `dir`, 1 = B plane `dir`
// (the plane buffer in LIQ_PLANES, formed from the compact record in
// LIQ_RECORD, unavailable in LIQ_PHI), 2 = phi buffer `dir`, 3 = N offsets.
hipError_t launch_plane_out(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int which,
                            int dir, int cur, int ps, int liq, hipStream_t stream);
// One plane from FP64 aux[0].  which: 0 = N plane `dir`, 1 = B plane `dir`
// of the plane buffer, 2 = solid entries of both phi buffers, 3 = N offsets,
// 4 = fluid entries of phi buffer `dir`.

hipError_t launch_plane_in(int lattice, uint32_t prec, const DevState& d, const StepParams& p, int which,
                           int dir, int cur, hipStream_t stream);

// One job of a batched step: a started context's device state, constants,
// state buffers at the first sub-step, and how many sub-steps it takes.
struct BatchJobHost {
    DevState d;
    StepParams p;
    int32_t cur0, ps0, planes0;   // planes0: liquid state (Liquid) at the first sub-step
    int64_t steps;
};

// Device bytes of a batch job table for up to max_jobs jobs (all groups),
// and of one (lattice, precision) group of njobs jobs.
size_t batch_table_bytes(int max_jobs);
size_t batch_group_bytes(int njobs);
// Advance every job of one (lattice, precision) group by its `steps`
// (<= nsteps) with one launch per phase and sub-step for the whole group.
// Jobs must be sorted by steps, largest first.  The table is uploaded from
// `staging` (kept alive by the caller until the stream has passed it).
hipError_t launch_batch(int lattice, uint32_t prec, const BatchJobHost* jobs, int njobs, void* table,
                        size_t table_bytes, int64_t nsteps, hipStream_t stream, std::vector<char>& staging);

}  // namespace lbm
