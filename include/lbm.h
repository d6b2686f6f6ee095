/*
 * lbm.h -- C ABI of the MI355X (gfx950) library for the BGK lattice Boltzmann update with the
 * third-order anisotropic equilibrium of "Lattice Boltzmann Methods with Anisotropic
 * Equilibrium Distributions" (arXiv 2605.27004).
 *
 * What the library evolves (the paper's problem statement):
 *   f_i(t+1, x + c_i) = f_i(t, x) + (1/tau) [f^eq_i(t, x) - f_i(t, x)]            (eq:LBE_BGK)
 * on a periodic Cartesian grid with D2Q9, D3Q19 or D3Q27 velocities (App. C), where
 *   f^eq_i = w_i rho [1 + c_i.s/cs^2 + H2_i:(s s + cs^2 K)/(2 cs^4)
 *                     + H3_i:(s s s + cs^2 (K s + K s + K s))/(6 cs^6)]     (eq:3rd_order_equilibrium)
 *   K = A^-1 - I                                                                     (eq:K-term)
 *   rho = sum_i f_i,  rho s = sum_i f_i c_i                    (eq:a0discrete_f, eq:a1discrete_f)
 * with cs^2 = 1/3 and A the symmetric positive-definite matrix of the anisotropic
 * Maxwell-Boltzmann exponent (eq:equil). Order 2 (the paper's comparison case, Sec. 4)
 * drops the H3 term.
 *
 * Conventions shared by every call:
 *  - Grid: nx * ny * nz cells (nz = 1 for D2Q9), x fastest; cell n = (z*ny + y)*nx + x.
 *  - Velocity order: the canonical order returned by lbm_lattice_info (rest first, then
 *    opposite pairs c_{2p-1} = -c_{2p}: axes, face diagonals, body diagonals).
 *  - Fields: rho is FP64 [N]; s (lattice velocity) is FP64 [d][N] (structure of arrays).
 *  - Populations are stored as deviations g_i = f_i - sigma_i from a constant shift sigma_i
 *    (lbm_params.shift_kind) in the storage precision. The two state buffers use a private
 *    blocked layout (q * N elements, no padding); lbm_get_populations / lbm_set_populations
 *    exchange the canonical structure of arrays [q][N].
 *    The canonical state at integer t is the PRE-collision f_i(t, x) of eq:LBE_BGK; every
 *    read-out call refers to it, whatever the library keeps internally.
 *  - Device pointers are HIP device addresses owned by the caller; they must stay valid
 *    for the lifetime of the context. The library allocates no device memory.
 *  - Every call returns LBM_OK (0) or a negative LBM_ERR_* code; no exception crosses the
 *    ABI. lbm_last_error() returns a thread-local message for the last failing call.
 *    Parameter errors are detected on the host before any device work is enqueued.
 *  - All device work is enqueued on the stream given to lbm_init (hipStream_t; NULL is the
 *    default stream) and is asynchronous unless stated otherwise.
 *  - A context is not thread-safe; distinct contexts may share a device and a stream.
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------- */
#define LBM_OK 0
#define LBM_ERR_ARG (-1)         /* invalid argument (NULL, bad enum, bad size, ...)      */
#define LBM_ERR_NOT_SPD (-2)     /* tensor not symmetric or not positive definite        */
#define LBM_ERR_TAU (-3)         /* tau <= 1/2: eta = rho cs^2 (tau - 1/2) must be > 0   */
#define LBM_ERR_ALIGN (-4)       /* a device buffer is not 256-byte aligned              */
#define LBM_ERR_HIP (-5)         /* a HIP runtime call failed (message has its string)   */
#define LBM_ERR_UNSUPPORTED (-6) /* valid request the library does not implement        */
#define LBM_ERR_NONFINITE (-7)   /* a conservation total is NaN or infinite              */
#define LBM_ERR_SIZE (-8)        /* grid too large: 2^31 cells or more, 4 GiB or more of
                                    populations in one z-plane (a whole D2Q9 grid is one
                                    z-plane) or in one batched domain, or a storage-type plane
                                    of 4 GiB or more                                          */

/* ---- enumerations --------------------------------------------------------------------- */
#define LBM_D2Q9 0
#define LBM_D3Q19 1
#define LBM_D3Q27 2

#define LBM_F64 0  /* populations stored as FP64, arithmetic FP64                      */
#define LBM_F32 1  /* populations stored as FP32, arithmetic FP32                      */
#define LBM_F16 2  /* populations stored as IEEE half, arithmetic FP32                 */
#define LBM_BF16 3 /* populations stored as bfloat16, arithmetic FP32                  */

/* How lbm_params.tensor is to be read (d x d leading block of the 3 x 3 array). */
#define LBM_TENSOR_THETA 0  /* tensor = cs^2 A^-1: the equilibrium's second central moment per
                               unit density, rho cs^2 A^-1 being the pressure tensor (App. E,
                               eq:NSprefinal). Used as given: no det normalisation.            */
#define LBM_TENSOR_A 1      /* tensor = A of eq:equil, used as given (the paper asks det A = 1,
                               Sec. 2.2; the update is defined for any SPD A).                 */
#define LBM_TENSOR_ATILDE 2 /* tensor = A~ proportional to A; A = A~ / det(A~)^(1/d) (Sec. 4
                               gives the d = 2 case A = A~ / sqrt(det A~)).                   */

/* Shift sigma_i subtracted from the stored populations (g_i = f_i - sigma_i). */
#define LBM_SHIFT_REST 0   /* sigma_i = rho0 r_i with r_i = f^eq_i(1, 0) = w_i (1 + H2_i:K/(2 cs^2)),
                              the anisotropic rest equilibrium (recommended).               */
#define LBM_SHIFT_WEIGHT 1 /* sigma_i = rho0 w_i (leaves the O(K) part of r_i in storage).  */

typedef struct lbm_params {
    int32_t lattice;     /* LBM_D2Q9 | LBM_D3Q19 | LBM_D3Q27                               */
    int32_t storage;     /* LBM_F64 | LBM_F32 | LBM_F16 | LBM_BF16                          */
    int32_t order;       /* 3 = the method (eq:3rd_order_equilibrium); 2 = without H3      */
    int32_t tensor_kind; /* LBM_TENSOR_*                                                   */
    int32_t shift_kind;  /* LBM_SHIFT_*                                                    */
    int32_t flags;       /* LBM_FLAG_* bits; 0 for a fully periodic fluid grid              */
    int64_t nx, ny, nz;  /* grid extents, each >= 1; nz == 1 for D2Q9; periodic on all faces */
    double tensor[9];    /* 3 x 3 row-major; leading d x d block used; must be symmetric
                            (|T - T^T| <= 1e-12 |T|) and positive definite. It enters as
                            (T + T^T) / 2, so derivatives split evenly over T_ab and T_ba. */
    double tau;          /* BGK relaxation time of eq:LBE_BGK, > 1/2                       */
    double rho0;         /* reference density of the shift sigma_i, > 0 (usually 1)        */
    double force[3];     /* body force F per cell (lattice units, momentum per step), added by
                            the exact-difference method: f* += f^eq(rho, s + F/rho) - f^eq(rho, s);
                            the fluid velocity is then (sum_i f_i c_i + F/2) / rho. Zero: no force.
                            (The paper names forcing as future work, Sec. 5.) The z entry must be
                            0 for D2Q9. */
} lbm_params;

/* lbm_params.flags bits (at most one of the two). */
#define LBM_FLAG_MASK 1 /* a solid mask is passed to lbm_init: cells with mask = 1 are solid and
                           fluid cells see them through halfway bounce-back -- a population
                           leaving x towards a solid x + c_i returns to x as c_opp(i) one step
                           later. Solid cells carry no state (read out as zeros). */
#define LBM_FLAG_GRAY 2 /* a gray field m in [0, 1] (float per cell) is passed to lbm_init: the
                           post-collision populations become (1 - m) f^BGK_i + m f_opp(i), a
                           partial bounce-back on the node that is differentiable in m (m = 1
                           reflects everything). The library keeps its own copy. */

/* Host-side quantities derived from lbm_params (lbm_prepare). All FP64. */
typedef struct lbm_derived {
    int32_t q, d;
    double ainv[9];        /* A^-1, 3 x 3 row-major, zero outside the d x d block          */
    double k[9];           /* K = A^-1 - I (eq:K-term), same layout                        */
    double omega;          /* 1 / tau                                                      */
    double nu;             /* kinematic shear viscosity cs^2 (tau - 1/2) (Sec. 3)          */
    double rest[27];       /* r_i = f^eq_i(rho = 1, s = 0), canonical order                */
    double shift[27];      /* sigma_i of the stored deviations                             */
    double min_rest_ratio; /* min_i r_i / w_i; negative values mean some rest populations
                              are negative (valid SPD tensors can do this; diagnostic only) */
} lbm_derived;

typedef struct lbm_ctx lbm_ctx; /* opaque; host-side metadata only */

/* Canonical velocity set of a lattice (App. C; c in lattice units, cs^2 = 1/3).
 * q, d: out (may be NULL). c: out [q][3] integers (may be NULL). w: out [q] weights (may be
 * NULL). opp: out [q], index of -c_i (may be NULL). Host only; returns LBM_ERR_ARG for an
 * unknown lattice. */
int lbm_lattice_info(int32_t lattice, int32_t *q, int32_t *d, int32_t *c, double *w, int32_t *opp);

/* Validate p and compute the derived quantities (host only, no device work).
 * Errors: LBM_ERR_ARG (enums, extents, rho0, flags, force), LBM_ERR_TAU, LBM_ERR_NOT_SPD (symmetry
 * or Cholesky failure of A^-1), LBM_ERR_SIZE. out may be NULL (validation only). */
int lbm_prepare(const lbm_params *p, lbm_derived *out);

/* Bytes of one population array: q * nx * ny * nz * sizeof(storage). -1 if p is invalid. */
int64_t lbm_pop_bytes(const lbm_params *p);

/* Rows per block of the private population layout (host only): each z-plane is stored as
 * ny / rows blocks of `rows` consecutive y-rows, a block holding its q direction planes one
 * after another; rows is the largest divisor of ny with rows * nx * sizeof(storage) <= 8 KiB
 * (32 KiB for FP64), at least 1. For tests and tools; -1 if p is invalid. */
int64_t lbm_rows_per_block(const lbm_params *p);

/* Bytes of device scratch lbm_init needs (reduction partials, plus 4 bytes per cell of link
 * words or gray fractions when LBM_FLAG_MASK or LBM_FLAG_GRAY is set). -1 if p is invalid. */
int64_t lbm_scratch_bytes(const lbm_params *p);

/* Create a context and write the initial state f_i(0, x) = f^eq_i(rho0(x), s0(x)).
 *   pop_a, pop_b: two device buffers of lbm_pop_bytes(p) each, 256-byte aligned, distinct;
 *                 the library ping-pongs between them (their contents are its state).
 *   scratch:      device buffer of lbm_scratch_bytes(p), 256-byte aligned.
 *   rho0:         device FP64 [N] initial density (read during this call's device work).
 *   s0:           device FP64 [d][N] initial lattice velocity.
 *   mask:         with LBM_FLAG_MASK: device uint8 [N], 1 = solid; with LBM_FLAG_GRAY: device
 *                 float [N], the gray fraction in [0, 1]; NULL otherwise. Read during this
 *                 call's device work only.
 *   stream:       hipStream_t for all work of this context.
 * On success *out receives the context (free with lbm_destroy). Asynchronous. */
int lbm_init(lbm_ctx **out, const lbm_params *p, void *pop_a, void *pop_b, void *scratch, const double *rho0,
             const double *s0, const void *mask, void *stream);

/* Advance by nsteps >= 0 steps of eq:LBE_BGK: one fused kernel per step that gathers the
 * streamed populations, forms rho and s, builds f^eq_i and relaxes with 1/tau.
 * Asynchronous. */
int lbm_step(lbm_ctx *ctx, int64_t nsteps);

/* Moments of the current state (eq:a0discrete_f, eq:a1discrete_f).
 *   rho:    device FP64 [N] or NULL;  s: device FP64 [d][N] or NULL (the fluid velocity,
 *           (sum_i f_i c_i + F/2) / rho). Solid cells read out rho = 0, s = 0.
 *   totals: host FP64 [4] or NULL: sums over fluid cells of rho, rho s_x, rho s_y, rho s_z
 *           (the last zero for D2Q9), reduced on the device in FP64 in a fixed order
 *           (bit-reproducible for a given grid). Passing totals synchronises the stream and
 *           returns LBM_ERR_NONFINITE if any total is NaN or infinite. */
int lbm_moments(lbm_ctx *ctx, double *rho, double *s, double *totals);

/* lbm_moments for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation). Same arguments, results and errors as
 * lbm_moments, bit for bit, but the reduction partials and totals live in a static device array
 * of the library (82,176 bytes, one per device, held until the process ends) instead of the
 * context's scratch; the call allocates nothing. Every call on a device shares that device's
 * array: calls that overlap on one device (different streams, or host threads) race and give
 * wrong totals; calls ordered on one stream do not. With totals == NULL only kernels are
 * enqueued; with totals the stream is synchronised, as in lbm_moments. Errors: LBM_ERR_ARG,
 * LBM_ERR_HIP (the array's address could not be looked up on the stream's device), and
 * LBM_ERR_SIZE if a grid's reduction needed more than the array (not possible for a valid
 * context: the moments launch never uses more than 2048 work-groups). */
int lbm_moments_static(lbm_ctx *ctx, double *rho, double *s, double *totals);

/* Canonical pre-collision deviations g_i(t, x) = f_i(t, x) - sigma_i in the storage precision,
 * device [q][N] (lbm_pop_bytes(p) bytes), for checkpointing. Exact (a permutation); solid
 * cells read out as zeros. */
int lbm_get_populations(lbm_ctx *ctx, void *out);

/* Restore the state from deviations in the layout of lbm_get_populations (exact inverse;
 * solid cells are ignored). The step counter is left unchanged. */
int lbm_set_populations(lbm_ctx *ctx, const void *in);

/* Canonical pre-collision populations f_i(t, x) = g_i + sigma_i in FP64, device [q][N]
 * (zeros on solid cells). */
int lbm_get_f64(lbm_ctx *ctx, double *out);

/* Steps taken since lbm_init (-1 if ctx is NULL). */
int64_t lbm_time(const lbm_ctx *ctx);

/* Step-kernel launch options: work-group shape block_x * block_y cells (block_x a multiple of
 * 64, block_x * block_y <= 256) and flags. The default spans whole x rows up to 256 cells
 * (block_y = 256 / block_x rows); longer rows take the width of 256, 128 or 64 cells that pads
 * the row least, the widest on a tie. */
#define LBM_LAUNCH_XCD_SLABS 1    /* hand each of the 8 XCDs one contiguous slab of tiles */
#define LBM_LAUNCH_SHIFTED_PULL 2 /* pull every population with its own shifted load. By default, when
                                     nx is a multiple of 64 and block_x == nx (work-groups of whole
                                     rows), x-shifted pulls load the lane's own x and move the values
                                     one lane across the wave; other launches always use shifted
                                     loads. */

/* Override the step kernel's launch. Results do not depend on it: every cell is computed by
 * the same arithmetic whatever work-group computes it. */
int lbm_set_launch(lbm_ctx *ctx, int32_t block_x, int32_t block_y, int32_t flags);

/* Gradients by the discrete adjoint of the step (reverse sweep with checkpointing).
 *
 * lbm_grad advances the context by spec->nsteps steps (exactly as lbm_step would), evaluates
 * the objective J on the final state and returns the derivatives of J with respect to the
 * tensor entries, tau and the per-cell gray fraction, the state at the start of the call
 * being held fixed. Objectives (all sums in FP64):
 *   0  mass flux through the plane x = outlet_plane:  J = sum over its cells of (j_x + F_x/2)
 *   1  kinetic energy:                                J = sum over cells of |j + F/2|^2 / (2 rho)
 * with j = sum_i f_i c_i. The forward states are kept every checkpoint_every steps and each
 * segment but the last is recomputed (bit-identically) before its reverse steps; the forward
 * pass writes the last segment's states where the recompute would. The adjoint populations
 * use the arithmetic precision of the storage; the parameter sums are FP64.
 * Supported: every tensor kind (for LBM_TENSOR_ATILDE the derivative includes the det
 * normalisation) and every wall model: none, LBM_FLAG_GRAY, or LBM_FLAG_MASK (halfway
 * bounce-back; the adjoint follows the same links). */
typedef struct lbm_grad_spec {
    int32_t objective;        /* 0 = outlet mass flux, 1 = kinetic energy                    */
    int32_t reserved;         /* must be 0                                                   */
    int64_t nsteps;           /* steps of the forward pass, >= 0                              */
    int64_t checkpoint_every; /* steps per recomputed segment, >= 1                           */
    int64_t outlet_plane;     /* x index of the flux plane (objective 0), 0 <= . < nx         */
} lbm_grad_spec;

/* Device workspace lbm_grad needs for this context and spec (checkpoints, one segment of
 * recomputed states, two adjoint buffers, partial sums); a negative LBM_ERR_* code when the
 * request is invalid or unsupported. LBM_ERR_SIZE when one z-plane of the adjoint
 * populations (q nx ny values in FP32, FP64 for FP64 storage) would reach 4 GiB. */
int64_t lbm_grad_workspace_bytes(const lbm_ctx *ctx, const lbm_grad_spec *spec);

/*   workspace: device buffer of lbm_grad_workspace_bytes, 256-byte aligned.
 *   objective: host out, J.
 *   dtensor:   host out [9] (may be NULL): dJ/dT_ab for the tensor as given, one value per
 *              independent entry (T_ab and T_ba are one entry), written symmetrically: off the
 *              diagonal it is the derivative with respect to v when T_ab = T_ba = v, twice the
 *              derivative with respect to either element alone (the tensor enters as
 *              (T + T^T) / 2).
 *   dtau:      host out (may be NULL): dJ/dtau.
 *   dmask:     device out FP64 [N] (may be NULL): dJ/dm per cell for the gray fraction m of
 *              the partial bounce-back blend. With a gray field it is the derivative at the
 *              given m; otherwise at m = 0 on every fluid cell (the sensitivity to adding a
 *              little gray there), and zero on solid cells.
 * Synchronises the stream before returning. */
int lbm_grad(lbm_ctx *ctx, const lbm_grad_spec *spec, void *workspace, double *objective, double *dtensor,
             double *dtau, double *dmask);

/* The objective J of lbm_grad (objective 0: mass flux through the plane x = outlet_plane;
 * 1: kinetic energy) on the current state, summed in FP64 on the device in a fixed order, with
 * no adjoint work: the same value lbm_grad returns for a final state. value: host out.
 * Synchronises the stream. */
int lbm_objective(lbm_ctx *ctx, int32_t objective, int64_t outlet_plane, double *value);

/* Measurement aid: nsteps passes of free streaming (every population moved along its velocity,
 * no collision) with exactly the step kernel's loads and stores, work-group shape and launch.
 * Its time is the data-movement floor of the step. It changes the state (lbm_time does not
 * advance); periodic grids only (LBM_ERR_UNSUPPORTED with a mask or gray field). */
int lbm_stream_floor(lbm_ctx *ctx, int64_t nsteps);

/* Free a context (NULL is allowed). Does not touch the caller's buffers. */
void lbm_destroy(lbm_ctx *ctx);

/* Thread-local message of the last failing call on this thread ("" if none). */
const char *lbm_last_error(void);

/* Measurement aid: copy nbytes (a multiple of 16) from src to dst with the library's plain
 * streaming copy kernel on stream; the reference for achievable HBM bandwidth. */
int lbm_stream_copy(void *dst, const void *src, int64_t nbytes, void *stream);

/* ---- batches of independent domains ----------------------------------------------------
 *
 * A batch advances many independent periodic domains of uneven sizes together, each with its
 * own tensor and tau, by eq:LBE_BGK with the equilibrium above: every domain follows exactly
 * the update a single-grid context with the same parameters performs (bitwise the same), so
 * the batch is a throughput device for many small problems, not a different method.
 * Shared by all domains: lattice, storage, order, shift kind and rho0. No masks, gray cells
 * or body force in a batch.
 *
 * Layout. Domain d has N_d = nx*ny*nz cells. Per-cell host-visible arrays (rho, s, FP64
 * exports) concatenate the domains in order: domain d starts at cell offset
 * C_d = N_0 + ... + N_{d-1} (lbm_batch_cells); rho is [C], s is [d][C] with C the total. The
 * population arrays are opaque (lbm_batch_pop_bytes each). */
typedef struct lbm_batch lbm_batch;

typedef struct lbm_domain {
    int64_t nx, ny, nz;  /* extents, >= 1 (nz = 1 for D2Q9), N_d < 2^31                  */
    int32_t tensor_kind; /* LBM_TENSOR_*                                                  */
    int32_t reserved;    /* must be 0                                                     */
    double tensor[9];    /* as in lbm_params                                              */
    double tau;          /* > 1/2                                                         */
} lbm_domain;

typedef struct lbm_batch_params {
    int32_t lattice, storage, order, shift_kind; /* as in lbm_params                      */
    double rho0;                                 /* as in lbm_params                      */
    int64_t ndomains;                            /* >= 1                                  */
    const lbm_domain *domains;                   /* host array [ndomains], read during the call */
} lbm_batch_params;

/* Total cells C; with offsets non-NULL also writes offsets[d] = C_d for d <= ndomains (host,
 * [ndomains + 1]). Negative LBM_ERR_* if the parameters are invalid. */
int64_t lbm_batch_cells(const lbm_batch_params *p, int64_t *offsets);
/* Bytes of ONE population array (the batch needs two) and of the device scratch. */
int64_t lbm_batch_pop_bytes(const lbm_batch_params *p);
int64_t lbm_batch_scratch_bytes(const lbm_batch_params *p);

/* Create a batch: validate every domain (as lbm_init does), upload the per-domain constants
 * and tile tables into scratch, and write f(0) = f^eq(rho0, s0) of every domain.
 *   pop_a, pop_b: device, lbm_batch_pop_bytes each, 256-byte aligned.
 *   scratch:      device, lbm_batch_scratch_bytes, 256-byte aligned.
 *   rho0, s0:     device FP64 [C] and [d][C], read during the call.
 * Synchronises the stream before returning. Starts with the step-per-launch schedule. */
int lbm_batch_init(lbm_batch **out, const lbm_batch_params *p, void *pop_a, void *pop_b, void *scratch,
                   const double *rho0, const double *s0, void *hip_stream);

/* How the steps are run. Results never depend on it (bitwise). */
#define LBM_BATCH_STEPWISE 0   /* one launch per step, one work-group per 256-cell tile       */
#define LBM_BATCH_PERSISTENT 1 /* one cooperative launch for all steps of an lbm_batch_step  */
typedef struct lbm_batch_schedule {
    int32_t mode;        /* LBM_BATCH_STEPWISE or LBM_BATCH_PERSISTENT                        */
    int32_t xcd_group;   /* 1: place each domain's work on one XCD (flat work-group b runs
                            on XCD b mod 8); 0: domain-major order                             */
    int32_t wg_per_cu;   /* persistent: resident work-groups per compute unit, 1 .. the
                            kernel's occupancy (lbm_batch_set_schedule checks)                 */
    int32_t reserved;    /* must be 0                                                          */
    int64_t chunk_cells; /* persistent: most cells one work-group takes from one domain per
                            step, a multiple of 256                                            */
    int64_t group_bytes; /* persistent: 0 = every domain in one group; else domains are run
                            in consecutive groups whose two population arrays total at most
                            this many bytes (a lone larger domain forms its own group), each
                            group through all steps before the next                            */
} lbm_batch_schedule;

/* One entry of a persistent schedule's work lists (lbm_batch_plan). */
typedef struct lbm_batch_item {
    int64_t domain;     /* domain index                                                    */
    int64_t first_cell; /* first cell of the run within the domain (a multiple of 256)     */
    int64_t cells;      /* cells in the run                                                */
    int64_t group;      /* group of domains the run belongs to (groups run one after another) */
    int64_t work_group; /* work-group that runs it; flat work-group w runs on XCD w mod 8   */
} lbm_batch_item;

/* Host only, no device work: the work lists the persistent schedule s would use on a device
 * with cu_count compute units. Writes min(count, cap) items (items may be NULL if cap is 0),
 * in the order each work-group runs them, and returns the count, or a negative LBM_ERR_*.
 * Every cell of every domain is in exactly one item of each step. */
int64_t lbm_batch_plan(const lbm_batch_params *p, const lbm_batch_schedule *s, int32_t cu_count,
                       lbm_batch_item *items, int64_t cap);

/* Build and upload the work lists of a schedule (synchronises the stream). */
int lbm_batch_set_schedule(lbm_batch *b, const lbm_batch_schedule *s);
int lbm_batch_get_schedule(const lbm_batch *b, lbm_batch_schedule *s);

/* Measure a fixed set of candidate schedules (step-per-launch with and without XCD
 * placement; persistent over work-groups per CU, chunk sizes and group sizes) on the batch's
 * own state, trial_steps timed steps each after two untimed ones, and keep the fastest. The
 * state is saved to `backup` (device, lbm_batch_pop_bytes, 256-byte aligned) first and
 * restored afterwards, so the batch's time and state are unchanged. best (host, may be NULL)
 * receives the chosen schedule and best_ms (may be NULL) its time per step. Synchronises. */
int lbm_batch_autotune(lbm_batch *b, void *backup, int32_t trial_steps, lbm_batch_schedule *best, double *best_ms);

/* Advance every domain by nsteps (asynchronous). */
int lbm_batch_step(lbm_batch *b, int64_t nsteps);

/* Synchronise and report the outcome of earlier persistent launches: LBM_ERR_HIP if a
 * work-group's bounded wait ran out (the state is then undefined), else LBM_OK. */
int lbm_batch_status(lbm_batch *b);

/* rho [C] and s [d][C] (device FP64, either may be NULL) of the canonical state, and
 * totals (host FP64 [ndomains][4], may be NULL): per domain sum rho and sum rho s. Checks
 * the status as lbm_batch_status does; synchronises when totals is non-NULL. */
int lbm_batch_moments(lbm_batch *b, double *rho, double *s, double *totals);

/* Canonical pre-collision populations in FP64 (sigma added back): device [q * C], domain d
 * at offset q * C_d as [q][N_d] in the canonical velocity order. */
int lbm_batch_get_f64(lbm_batch *b, double *out);

/* Steps taken since lbm_batch_init (-1 if b is NULL). */
int64_t lbm_batch_time(const lbm_batch *b);

/* Set the spin limit of the persistent schedule's bounded waits (polls of a counter; the
 * default covers seconds). A tiny value makes waits give up; tests use it to exercise the
 * failure path. */
int lbm_batch_set_spin_limit(lbm_batch *b, uint32_t polls);

/* Free a batch (NULL is allowed). Does not touch the caller's buffers. */
void lbm_batch_destroy(lbm_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
