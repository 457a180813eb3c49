/*
 * lbm.h -- C ABI of the MI355X colour-gradient lattice Boltzmann library
 * with the curved-boundary ghost-node wetting condition.
 *
 * One time step (lbm_step) follows the paper's model:
 *   colour field phi = sum_i B_i                       (Appendix A, Eq. A13)
 *   ghost-node colour update at every solid boundary   (Section 2, Eq. 9;
 *     node, phi_G = phi_F / (phi_F + (1-phi_F) e^eps)   Eq. 10 as a switch)
 *     with phi_F interpolated at x_F = x_G + n_s
 *   forces F_s (Eq. 4), F_p (Eq. A10), F_visc (Eq. A11), F_b (Eq. 2)
 *   MRT collision of the colour-blind populations N    (Eq. A1-A3, A4, A8)
 *   recolouring of the liquid populations B            (Eq. A12)
 *   streaming of N and B with halfway bounce-back      (Eq. A16-A17)
 * on a D2Q9 or D3Q19 lattice, every axis periodic; walls are solids.
 *
 * Conventions
 *   - Every function returns an int: LBM_OK (0) or a negative LBM_E* code;
 *     lbm_last_error() then holds a message.  No function aborts.
 *   - A context is not thread-safe; use one thread per context.
 *   - Node (x, y, z) has flat index x + nx*(y + ny*z).  Host arrays passed in
 *     or out are FP64 in that order; per-direction arrays are [Q][nodes] in
 *     the direction order returned by lbm_lattice().
 *   - The library allocates no device memory.  The caller (PyTorch) owns one
 *     device buffer and one HIP stream and hands them over with lbm_bind();
 *     the buffer must stay alive and unused by others until lbm_destroy().
 *   - Device work is enqueued on the bound stream.  lbm_step() does not
 *     synchronise; lbm_observe(), lbm_read_field() and lbm_set_field() do.
 *     A kernel error of lbm_step() is reported by the next synchronising call.
 *   - Call order: lbm_create -> lbm_set_geometry -> lbm_device_bytes ->
 *     lbm_bind -> lbm_set_wetting -> lbm_set_field(LBM_FIELD_PHI) ->
 *     lbm_step / lbm_observe / lbm_read_field ... -> lbm_destroy.
 *     Out-of-order calls return LBM_ESTATE.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 2u

enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,     /* bad argument or parameter */
    LBM_ESTATE = -2,     /* call out of order */
    LBM_ENOMEM = -3,     /* bound buffer too small, or a host allocation failed */
    LBM_EHIP = -4,       /* HIP runtime or kernel error */
    LBM_EUNSTABLE = -5   /* lbm_observe found non-finite values */
};

enum { LBM_D2Q9 = 0, LBM_D3Q19 = 1 };

/* Population storage.  Arithmetic is FP64 for LBM_FP64 and FP32 otherwise. */
enum { LBM_FP64 = 0, LBM_FP32 = 1, LBM_FP16_OFS = 2, LBM_BF16_OFS = 3 };

/* Step forms.  By default every step is three launches: colour field
 * (phi = sum_i B_i, Eq. A13, from N and the compact record of the last
 * collide), ghost update (Eq. 9), and the collide-stream kernel.  With
 * LBM_OPT_FUSED, D3Q19 boxes with n[0] % 64 == 0 and n[1] % 8 == 0 whose
 * 19 population planes take at most 4 GiB run every step as the ghost update, one collide kernel over 64 x 8 columns
 * that also forms the next step's phi from the recoloured populations it
 * streams (Eq. A12, A17), and a small launch that adds the values crossing
 * a column's faces.  N is then read once per step instead of twice, and no
 * compact record is kept: after such a step the liquid state is phi itself,
 * so lbm_read_field(LBM_FIELD_B) returns LBM_ESTATE; a checkpoint is N,
 * LBM_FIELD_PHI_STATE and LBM_FIELD_SOLID_PHI.  Both forms compute the same update; N is bit-identical
 * and phi differs only in the rounding order of the sum at nodes whose
 * streamed-in populations cross a column face.  Other boxes, D2Q9 and
 * LBM_OPT_SPARSE runs ignore the option for stepping. */
#define LBM_OPT_FUSED 1

/* Probe interpolation of the ghost rule.  By default phi_F at
 * x_F = x_G + n_s (text before Eq. 8) interpolates all 2^D corners, solid
 * ones with their current value (ghosts: last step's; deeper solid nodes:
 * (1 + cos theta)/2).  With LBM_OPT_FLUID_PROBE only the fluid corners take
 * part, their weights rescaled to sum 1.  A probe with no fluid corner (a
 * ghost in the gap between touching solids, its normal pointing into the
 * other solid) takes the ghost's fluid lattice neighbours instead, weighted
 * by w_i and rescaled to sum 1 (the axis neighbours alone if there are more
 * than 2^D; lbm_set_geometry returns LBM_EINVAL if none of them is on an
 * axis).  In narrow gaps between solids (packings) the default lets probes
 * read the far solid's (1 + cos theta)/2 and, below 90 degrees at density
 * ratio 10, drives gas nodes there unstable within ~200 steps. */
#define LBM_OPT_FLUID_PROBE 2

/* With LBM_OPT_GRAPH, lbm_step with nsteps >= 8 replays a captured HIP graph
 * of two steps after the first step of a run; the graph is
 * captured once per buffer parity on a private stream of default priority
 * and dropped by lbm_set_wetting and lbm_set_field.  Both forms compute the
 * same update bit for bit.  Off by default: on the paper's small D2Q9 boxes
 * (4e4 to 1.4e6 nodes) the replays measured 3 to 13 % slower than direct
 * launches, the per-kernel cost being on the device, not in the launch. */
#define LBM_OPT_GRAPH 8

/* Geometry conditioning for packings (not in the paper, whose solids are
 * single convex bodies).  With LBM_OPT_FILL_DEAD_ENDS, lbm_set_geometry makes
 * solid every fluid node that has at most one fluid lattice neighbour, and
 * repeats on the new solid set until no such node is left.  Such nodes sit in
 * the contacts between touching solids, narrower than a node; left fluid,
 * they are wedged between the two solids' ghost values and, below 90 degrees,
 * grow a velocity that doubles every few hundred steps.  A filled node that
 * borders the fluid is a ghost node whose normal n_s points to the one fluid
 * neighbour it keeps. */
#define LBM_OPT_FILL_DEAD_ENDS 16

/* Fluid-only storage for mostly solid boxes (packings).  With LBM_OPT_SPARSE
 * every device plane holds one entry per slot instead of per box node.  The
 * slots are the fluid nodes in box order, then the ghost nodes in list
 * order, then one slot that stands for every other solid node.  A table of
 * Q - 1 slot indices per fluid node (4 (Q - 1) bytes, bit 31 marking a
 * solid neighbour) gives each fluid node's neighbours.  Launches cover the fluid slots only, and a step
 * computes the same values as the box layout, bit for bit.  Streaming is
 * pull: the device keeps each node's post-collision populations in its own
 * slots and the next step gathers them (Eq. A16-A17 applied on read).
 * Fields still cross the ABI in box order, and LBM_FIELD_N / _N_OFFSET
 * still mean the post-stream populations (gathered on read, scattered on
 * set).  Restrictions: it excludes LBM_OPT_FUSED
 * (lbm_create returns LBM_EINVAL); such contexts step
 * only through lbm_step (lbm_batch_step returns LBM_EINVAL); setting
 * LBM_FIELD_SOLID_PHI needs one value for all non-ghost solid nodes
 * (LBM_EINVAL otherwise). */
#define LBM_OPT_SPARSE 32

/* Ghost-node rule: Eq. 9 (this paper) or Eq. 10 (Fakhari et al.). */
enum { LBM_GHOST_EQ9 = 0, LBM_GHOST_FAKHARI = 1 };

/* Fields for lbm_set_field / lbm_read_field (all FP64 on the host). */
enum {
    LBM_FIELD_PHI = 0,        /* [nodes] colour field phi.  set: initial phi at
                                 fluid nodes (N_i = chi_i, B_i = phi chi_i, u = p = 0);
                                 read: the phi (fluid and ghost nodes) the next
                                 step will use */
    LBM_FIELD_N = 1,          /* [Q][nodes] colour-blind populations (post-stream) */
    LBM_FIELD_B = 2,          /* [Q][nodes] liquid populations (post-stream); not
                                 readable after a collide-colour step (LBM_OPT_FUSED) */
    LBM_FIELD_U = 3,          /* [3][nodes] velocity u of Eq. A14 (read only) */
    LBM_FIELD_P = 4,          /* [nodes] auxiliary pressure p of Eq. A15 (read only) */
    LBM_FIELD_SOLID_PHI = 5,  /* [nodes] phi carried at solid nodes between steps */
    LBM_FIELD_FLAGS = 6,      /* [nodes] node class: 1 solid, 2 fluid next to a
                                 solid, 4 ghost (read only) */
    LBM_FIELD_N_OFFSET = 7,   /* [Q][nodes] N_i - chi_i as the library stores it
                                 (every precision keeps the offset from the
                                 rest state); exact in FP64 both ways, so a
                                 read-then-set checkpoint resumes bit for bit */
    LBM_FIELD_PHI_STATE = 8   /* [nodes] read: as LBM_FIELD_PHI; set (after
                                 LBM_FIELD_PHI): the fluid entries become the
                                 colour field of the next step, which then
                                 forms no colour field of its own.  With N
                                 (or N_OFFSET) and SOLID_PHI it restores the
                                 state of a run whose last step was
                                 collide-colour (LBM_OPT_FUSED), bit for bit */
};

typedef struct lbm_ctx lbm_ctx;

/* Model parameters, lattice units (dx = dt = 1).  Defaults of the paper's
 * Section 3: rho_l = 1000, rho_g = 1, mu_l = 10, mu_g = 0.1, sigma = 0.01,
 * W = 4, mobility = 0.02. */
typedef struct {
    uint32_t abi_version;   /* LBM_ABI_VERSION */
    uint32_t lattice;       /* LBM_D2Q9 or LBM_D3Q19 */
    uint32_t precision;     /* LBM_FP64 ... */
    uint32_t ghost_rule;    /* LBM_GHOST_EQ9 or LBM_GHOST_FAKHARI */
    int32_t n[3];           /* box nodes; n[2] must be 1 for D2Q9 */
    int32_t options;        /* bit 0 (LBM_OPT_FUSED): collide-colour D3Q19 steps where the box allows;
                               bit 1 (LBM_OPT_FLUID_PROBE): fluid-only probe interpolation;
                               bit 2: unused (LBM_EINVAL);
                               bit 3 (LBM_OPT_GRAPH): captured two-step graphs in lbm_step;
                               bit 4 (LBM_OPT_FILL_DEAD_ENDS): dead-end fluid nodes made solid;
                               bit 5 (LBM_OPT_SPARSE): fluid-only storage */
    double rho_l, rho_g;    /* liquid (phi = 1) and gas (phi = 0) densities, > 0 */
    double mu_l, mu_g;      /* dynamic viscosities, > 0 */
    double sigma;           /* surface tension, >= 0 */
    double W;               /* interface width, >= 4 (Section 2, text after Eq. 9) */
    double mobility;        /* M_phi > 0; sets the colour weights (Eq. A7) */
    double body_accel[3];   /* g of the body force rho g (Eq. 2) */
} lbm_params;

/* Solid primitive.  kind 0: ball (disk in 2D) |x - center| <= radius, closed.
 * kind 1: half-space (x - center) . normal <= 0; normal points out of the
 * solid.  A node's solid normal n_s is that of the first primitive holding it
 * (radial for a ball, `normal` normalised for a half-space). */
typedef struct {
    uint32_t kind;
    uint32_t pad;
    double center[3];
    double radius;
    double normal[3];
} lbm_solid;

/* Diagnostics, FP64, summed over fluid nodes in a fixed order. */
typedef struct {
    int64_t step;            /* steps taken since the last LBM_FIELD_PHI set */
    int64_t n_fluid, n_solid, n_ghost;
    int64_t nonfinite;       /* non-finite N_i, B_i or phi values */
    double mass_blue;        /* sum phi */
    double mass_red;         /* sum (1 - phi) */
    double momentum[3];      /* sum rho u */
    double max_speed;        /* max |u| (spurious-current measure) */
    double kinetic_energy;   /* sum rho |u|^2 / 2 */
} lbm_obs;

/* Validate params and create a context (host memory only).
 * Errors: LBM_EINVAL for W < 4, non-positive densities/viscosities/mobility,
 * tau <= 1/2, alpha outside [0, 1), bad lattice/precision/rule/sizes.
 * Size limits: at most 2^31 - 1 nodes, n[1], n[2] <= 65535, and one field
 * plane (nodes rounded up to 128, times 8 bytes in FP64 and 4 bytes
 * otherwise) below 4 GiB: up to 5.4e8 nodes in FP64, 1.07e9 otherwise. */
int lbm_create(const lbm_params* params, lbm_ctx** out);

/* Rasterise `count` solids (host), classify nodes (solid, ghost = solid with
 * a fluid lattice neighbour, Section 1), and build the ghost list: analytic
 * normal n_s, probe point x_F = x_G + n_s and its 2^D interpolation corners
 * and weights (Section 2, text before Eq. 8).  `solids` is read only during
 * the call.  May be called once, before lbm_bind.  Errors: LBM_ESTATE when
 * called again; LBM_EINVAL for a bad list, an unknown kind, a ball wider than
 * the box, a zero half-space normal, or (LBM_OPT_FLUID_PROBE) a ghost whose
 * probe fallback has no axis neighbour to use; LBM_ENOMEM on host memory. */
int lbm_set_geometry(lbm_ctx* ctx, const lbm_solid* solids, int32_t count);

/* Bytes of device memory lbm_bind needs (known after lbm_set_geometry). */
int lbm_device_bytes(const lbm_ctx* ctx, size_t* bytes);

/* Hand over a device buffer of at least lbm_device_bytes() bytes (256-byte
 * aligned) and the HIP stream (hipStream_t, may be NULL for the null stream)
 * all device work goes to.  Uploads the geometry.  LBM_ENOMEM if too small. */
int lbm_bind(lbm_ctx* ctx, void* device_ptr, size_t bytes, void* hip_stream);

/* Contact angle theta in degrees through the liquid, 0..180 (Eq. 7);
 * eps = -(4/W) cos(theta) and exp(eps) are formed on the host in FP64
 * (Eq. 9).  Before the first step it also sets every solid node to
 * (1 + cos theta)/2 (Section 3); later calls change eps only. */
int lbm_set_wetting(lbm_ctx* ctx, double theta_deg);

/* Write a field from the host (`count` doubles, see the field list).
 * LBM_FIELD_PHI starts a run (step counter 0); LBM_FIELD_N / _N_OFFSET /
 * _B / _SOLID_PHI overwrite raw state (restore; _N_OFFSET is exact in every
 * precision, _N rounds N_i - chi_i once).  Errors: LBM_ESTATE before
 * LBM_FIELD_PHI (for the raw fields), LBM_EINVAL for a wrong count, a
 * non-finite initial phi or a read-only field.  Synchronises the stream. */
int lbm_set_field(lbm_ctx* ctx, int field, const double* host_src, size_t count);

/* Enqueue nsteps >= 0 time steps on the bound stream; returns at once. */
int lbm_step(lbm_ctx* ctx, int64_t nsteps);

/* lbm_step with timing: brackets each launch of every step (0: colour
 * field, 1: ghost update, 2: collide-stream or collide-colour, 3: colour
 * fix-up of the collide-colour form) with HIP events on the bound stream,
 * waits for the last one, and writes the summed milliseconds of each phase
 * to ms_out[0..3] and the elapsed time from the first to the last event to
 * ms_out[4] (five doubles).  A phase a step does not launch reads ~0.
 * nsteps >= 1.  Synchronises. */
int lbm_step_profiled(lbm_ctx* ctx, int64_t nsteps, double* ms_out);

/* Reduce the diagnostics on the device and copy them out (synchronises).
 * Returns LBM_EUNSTABLE (and fills *out) if any value is non-finite. */
int lbm_observe(lbm_ctx* ctx, lbm_obs* out);
/* lbm_observe for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same diagnostics, bit for bit, with the reduction's scratch (1024
 * per-block partials, the non-finite counters and the result, 74 KB) in a
 * static device array of the library instead of the bound buffer.  The
 * array holds no per-node data, so every box size fits it.  Each device
 * holds one copy, shared by every context on it and kept between calls:
 * every call overwrites all of it before reading it, and calls that overlap
 * on one device (contexts on different threads or streams) race.  Its
 * address is looked up once per device at the first call there (the device
 * of the bound buffer); the call makes no allocation.  Synchronises the
 * bound stream.  Errors as lbm_observe, and LBM_EHIP if the address lookup
 * fails. */
int lbm_observe_static(lbm_ctx* ctx, lbm_obs* out);


/* Copy a field to the host as FP64 (`count` doubles; synchronises).  Solid
 * nodes read u = p = 0 and N = B = 0. */
int lbm_read_field(lbm_ctx* ctx, int field, double* host_dst, size_t count);

/* Lattice velocities in the library's direction order: c_out[Q][3] (room for
 * 19 x 3 int32), *q_out = Q.  No context needed. */
int lbm_lattice(uint32_t lattice, int32_t* c_out, int32_t* q_out);

/* ---------------------------------------------------------------- batches
 * Continuous batching of many runs: lbm_batch_step advances a set of started
 * contexts of any sizes, lattices, precisions and angles with shared
 * launches (per sub-step, one launch per phase for all contexts of the same
 * lattice and precision; every workgroup looks its run up in a job table).
 * Each context keeps its own buffer and state, so the set may change from
 * one call to the next (runs join and leave between calls), and every run
 * computes exactly what lbm_step would.  The job table lives in a device
 * buffer the caller provides (no allocation in the library). */
typedef struct lbm_batch lbm_batch;

/* Device bytes of a job table for up to max_jobs contexts in one call. */
int lbm_batch_table_bytes(int32_t max_jobs, size_t* bytes);

/* Create a batch over a caller-owned, 256-byte aligned device table and the
 * stream its launches go to.  Contexts passed to lbm_batch_step must be idle
 * on their own streams or bound to this same stream. */
int lbm_batch_create(void* device_table, size_t bytes, void* hip_stream, lbm_batch** out);

/* Advance ctxs[j] by steps[j] >= 0 steps (count contexts, each at most
 * once).  Waits for the batch stream's previous work first (the table is
 * reused), then enqueues and returns; results appear like lbm_step's.
 * LBM_EINVAL for a null, repeated or LBM_OPT_SPARSE context or a negative
 * step count; LBM_ESTATE for a context that has not started. */
int lbm_batch_step(lbm_batch* batch, lbm_ctx* const* ctxs, const int64_t* steps, int32_t count);

/* Release the batch (host memory only). */
int lbm_batch_destroy(lbm_batch* batch);

/* Last error of a batch call ("" if none). */
const char* lbm_batch_last_error(const lbm_batch* batch);

/* ---------------------------------------------------------------- measurement
 * HBM reference kernels, not part of the time step: the rates plain
 * streaming kernels reach on this device, against which the lattice kernels'
 * bandwidth is read (beside the published peak).  Enqueues `repeats` >= 1
 * launches on hip_stream between two HIP events, waits for the last, and
 * writes the average milliseconds per launch to *ms_out.
 *   kind 0 (read):   every 16-byte vector of src_bytes of src is loaded once;
 *                    dst needs 4 * 4096 bytes (never written for zeroed src)
 *   kind 1 (copy):   dst (src_bytes) = src, 16-byte vectors
 *   kind 2 (planes): src is 19 FP32 planes of n = src_bytes / 76 values,
 *                    dst (n FP32) = their sum, one 4-byte load per lane and
 *                    plane (the colour-field kernel's access pattern)
 * src and dst are device pointers, 16-byte aligned, owned by the caller.
 * Errors: LBM_EINVAL for a bad kind, size, alignment or repeats; LBM_EHIP. */
int lbm_hbm_probe(int32_t kind, const void* src, void* dst, size_t src_bytes, int32_t repeats,
                  void* hip_stream, double* ms_out);

/* Release the context's host memory.  The device buffer stays the caller's. */
int lbm_destroy(lbm_ctx* ctx);

/* Last error message of ctx ("" if none); for ctx == NULL, the last error of
 * a failed lbm_create on this thread. */
const char* lbm_last_error(const lbm_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
