/*
 * lbm.h -- C ABI of the MI355X (gfx950) lattice Boltzmann stream-collide library.
 *
 * The library advances the lattice Boltzmann equation of the paper
 * ("Scalable Flow Simulations with the Lattice Boltzmann Method", Section 2,
 * Eq. (1) collision and Eq. (2) streaming) on one GPU:
 *   - D3Q19 or D3Q27 velocity set,
 *   - two-relaxation-time collision (the paper's "Double Relaxation Time"
 *     D3Q19 scheme of the LaBS section) with Guo body forcing,
 *   - halfway bounce-back walls, velocity and pressure faces, periodic faces,
 *     and an optional per-cell solid mask,
 *   - one population set kept in place in HBM, streamed with the AA access
 *     pattern or with the Esoteric Twist the paper's LAGOON runs use
 *     (Section 5.2), structure of arrays within each row of cells: [z][y][q][x];
 *     or, for solid-heavy domains, the AA pattern over the fluid cells only
 *     (sparse addressing),
 *   - optional LES closures (Smagorinsky, or a small learned MLP) that set a
 *     per-cell relaxation time.
 *
 * Conventions for every entry point:
 *   - Every pointer named *_dev is device memory on the current HIP device,
 *     owned by the caller.  Pointers without the suffix are host memory.
 *   - All work is enqueued on the stream given in lbm_domain (or the stream
 *     argument of the free functions); entry points return once the work is
 *     enqueued, except where a comment says "synchronises".
 *   - The library never allocates device memory: a context lives in a
 *     caller-provided workspace of lbm_workspace_bytes() bytes, which must
 *     outlive the context.  lbm_destroy frees host metadata only.
 *   - Calls on one context are not thread-safe.
 *   - Every function returns LBM_OK (0) or a negative error code; the
 *     message of the last error is available from lbm_last_error().
 *   - Layouts: populations are canonical FP64 [q][nz][ny][nx] (x fastest),
 *     the value f_i(x, t) after streaming and before collision.  Scalar
 *     fields are [nz][ny][nx]; vector fields [3][nz][ny][nx].
 *   - Velocity order (pairs (odd, odd+1) are opposite):
 *       0 (0,0,0); 1,2 (+-1,0,0); 3,4 (0,+-1,0); 5,6 (0,0,+-1);
 *       7 (1,1,0) 8 (-1,-1,0); 9 (1,-1,0) 10 (-1,1,0); 11 (1,0,1) 12 (-1,0,-1);
 *       13 (1,0,-1) 14 (-1,0,1); 15 (0,1,1) 16 (0,-1,-1); 17 (0,1,-1) 18 (0,-1,1);
 *       D3Q27 adds 19 (1,1,1) 20 (-1,-1,-1); 21 (1,1,-1) 22 (-1,-1,1);
 *       23 (1,-1,1) 24 (-1,1,-1); 25 (-1,1,1) 26 (1,-1,-1).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Error codes. */
#define LBM_OK 0
#define LBM_EINVAL (-1)     /* invalid argument (sizes, enums, NULL, small workspace) */
#define LBM_ENOMEM (-2)     /* the domain exceeds the indexing (sparse addressing: 2^32 cells, 2^31 fluid cells) or host memory */
#define LBM_EDEVICE (-3)    /* a HIP runtime call or kernel launch failed */
#define LBM_ENONFINITE (-4) /* lbm_totals found a NaN or Inf population */
#define LBM_ESTATE (-5)     /* call not valid in the current state (e.g. MLP weights missing) */

/* Velocity sets. */
enum { LBM_D3Q19 = 19, LBM_D3Q27 = 27 };

/* Per-face boundary kinds.  Faces are ordered -x, +x, -y, +y, -z, +z.
 * Walls lie halfway between the first/last cell row and the face. */
enum {
    LBM_BC_PERIODIC = 0, /* wrap around; the opposite face must be periodic too */
    LBM_BC_NOSLIP = 1,   /* halfway bounce-back */
    LBM_BC_VELOCITY = 2, /* moving-wall bounce-back with u_bc and rho_bc of the face */
    LBM_BC_PRESSURE = 3, /* anti-bounce-back with density rho_bc of the face */
    LBM_BC_INTERFACE = 4 /* a face of a 2:1 refinement interface (-y or +y only; the dense
                            AA pattern, no HRR): steps of this lattice alone treat it as
                            no-slip; lbm_refine_step exchanges the packets that cross it */
};

/* Population storage in HBM.  All forms store the deviation f_i - w_i. */
enum {
    LBM_STORE_F32 = 0,     /* 4 bytes per population */
    LBM_STORE_F16DEV = 1,  /* IEEE half, round to nearest even, subnormals kept */
    LBM_STORE_BF16DEV = 2  /* bfloat16, round to nearest even */
};

/* Relaxation-time closures. */
enum { LBM_LES_NONE = 0, LBM_LES_SMAGORINSKY = 1, LBM_LES_MLP = 2 };

/* Collision operators (the collision Omega of Eq. (1)).
 * TRT: two relaxation rates, 1/tau on the symmetric part of each pair of
 *      opposite populations and 1/(1/2 + magic/(tau - 1/2)) on the
 *      antisymmetric part (the paper's "Double Relaxation Time", Section 4).
 * MRT: multiple relaxation times in a moment space (the collision of the
 *      paper's LAGOON runs, Section 5.2): the second-order moments relax with
 *      1/tau, the ghost moments with mrt_rates = {energy, energy square,
 *      heat flux, fourth-order, third-order anti-symmetric}.  D3Q19 uses its
 *      19 orthogonal polynomial moments, D3Q27 the tensor products of
 *      {1, c, 3c^2 - 2}.  Not combinable with the learned closure.
 * HRR: hybrid recursive regularisation (the paper's "D3Q19HRR" of the LaBS
 *      section, Section 4; after Jacob, Malaspinas & Sagaut 2018), D3Q19,
 *      dense AA streaming, no closure: the non-equilibrium part is rebuilt
 *      from its second-order Hermite coefficients, a blend hrr_sigma *
 *      (projected flux) + (1 - hrr_sigma) * (-2 rho c_s^2 tau S) with S the
 *      strain rate from finite differences of the previous step's velocity
 *      field, and third-order coefficients by recursion; the equilibrium
 *      carries the third-order terms the lattice supports.  The context keeps
 *      two velocity fields (24 bytes per cell) in its state. */
enum { LBM_COLL_TRT = 0, LBM_COLL_MRT = 1, LBM_COLL_HRR = 2 };

/* In-place streaming schemes (one population set in HBM; Section 5.2).
 * AA: even steps read and write only the cell's own slots, odd steps read
 *     from and write to the neighbours x -+ c_i.
 * ET: the Esoteric Twist: every step reads f_i at x + max(-c_i, 0) and
 *     writes at x + max(c_i, 0), the slot of a direction alternating between
 *     i and opposite(i) from step to step.  Each non-periodic axis gets one
 *     ghost layer beyond its + face in the store (it holds the populations
 *     that face returns).
 * AA_SPARSE: the AA pattern over the fluid cells only (sparse indirect
 *     addressing, for domains that solids fill to a large part): fluid cells
 *     are stored compacted in row order, and a table of the q-1 neighbours of
 *     each fluid cell (4 bytes each) serves the odd steps.  The population
 *     store and the table are sized by the fluid cells (see
 *     lbm_workspace_bytes_flags).
 * All give the same populations up to FP32 rounding order (the same
 * arithmetic runs on the same values). */
enum { LBM_STREAM_AA = 0, LBM_STREAM_ET = 1, LBM_STREAM_AA_SPARSE = 2 };

typedef struct lbm_ctx lbm_ctx;

typedef struct lbm_domain {
    int32_t nx, ny, nz;      /* cells, x fastest; each >= 1, ny and nz <= 65535 (cell indices are 64-bit) */
    int32_t bc[6];           /* LBM_BC_* per face -x,+x,-y,+y,-z,+z */
    double u_bc[6][3];       /* wall velocity of velocity faces */
    double rho_bc[6];        /* wall density of velocity and pressure faces (1.0 by default) */
    int32_t storage;         /* LBM_STORE_* */
    int32_t closure;         /* LBM_LES_* */
    int32_t use_flags;       /* non-zero: reserve room for a per-cell solid mask */
    double magic;            /* TRT magic parameter Lambda (3/16 by default) */
    double cs_smag;          /* Smagorinsky constant (0.1 by default) */
    int32_t collision;       /* LBM_COLL_* (TRT by default) */
    double mrt_rates[5];     /* MRT ghost rates in (0, 2); default 1.19, 1.4, 1.2, 1.4, 1.98 */
    int32_t streaming;       /* LBM_STREAM_* (AA by default) */
    double hrr_sigma;        /* HRR weight of the projected flux in [0, 1] (0.995 by default) */
    void *workspace;         /* device memory of workspace_bytes bytes, 256-byte aligned */
    size_t workspace_bytes;
    void *stream;            /* hipStream_t; NULL = the default stream */
} lbm_domain;

/* Fill *d with defaults: all faces periodic, rho_bc = 1, u_bc = 0, F32
 * storage, no closure, no flags, magic = 3/16, cs_smag = 0.1, TRT
 * collision, MRT ghost rates {1.19, 1.4, 1.2, 1.4, 1.98}, AA streaming,
 * hrr_sigma = 0.995, no workspace.  The domain carries the free parameters of the kernel
 * interface the paper describes for its generated kernels (raw pointers,
 * shape and free parameters; Section 3).  d == NULL: no effect. */
void lbm_domain_defaults(lbm_domain *d);

/* Bytes of device workspace a context needs for domain d and the stencil
 * (19 or 27): one population set kept in place (the single PDF set of the
 * in-place streaming of Section 5.2) plus the reduction and closure areas.
 * Only nx, ny, nz, storage, closure, use_flags, streaming and (for the
 * ghost layers of the Esoteric Twist) bc are read.  With sparse addressing
 * this is the bound for a domain without solids.  *out (host) receives the
 * size.  LBM_EINVAL for NULL or invalid sizes/enums, LBM_ENOMEM when the
 * domain exceeds the cell indexing. */
int lbm_workspace_bytes(const lbm_domain *d, int stencil, size_t *out);

/* As lbm_workspace_bytes, for the solid flags that lbm_create will get
 * (host, one byte per cell, nullable; read only during the call): with
 * sparse addressing the stores are sized by the fluid cells; otherwise the
 * same value.  Errors as lbm_workspace_bytes. */
int lbm_workspace_bytes_flags(const lbm_domain *d, int stencil, const uint8_t *flags, size_t *out);

/*
 * Create a context for the lattice Boltzmann equation of Section 2: the
 * collision Eq. (1) relaxes f^neq with the operator Omega, set here by the
 * relaxation time tau > 1/2 (viscosity nu = (tau - 1/2)/3; Omega read as
 * the two-relaxation-time or MRT operator of d->collision), and the
 * streaming Eq. (2) moves f_i* to x + c_i.  force[3] (host, nullable: zero)
 * is the constant body-force density of Guo's forcing; flags (host,
 * nullable, read only during the call) holds one byte per cell [nz][ny][nx],
 * non-zero = solid, and needs d->use_flags.  Opposite faces must both be
 * periodic or both not.  The context lives in d->workspace (device, caller
 * owned, must outlive it); *out receives a host handle owned by the caller
 * (release with lbm_destroy).  The populations are left undefined: call
 * lbm_init_equilibrium or lbm_set_pdfs next.  Synchronises.
 * LBM_EINVAL for invalid parameters or a small/misaligned workspace,
 * LBM_ENOMEM when the domain exceeds the cell indexing, LBM_EDEVICE when a
 * device call fails (*out stays NULL on every error).
 */
int lbm_create(const lbm_domain *d, int stencil, const uint8_t *flags, double tau, const double force[3],
               lbm_ctx **out);

/* Release the host handle of a context created for Section 2's update.
 * Device memory (the workspace) stays the caller's.  ctx == NULL: no-op. */
int lbm_destroy(lbm_ctx *ctx);

/* Message of the last failure on ctx (ctx == NULL: of the last failed
 * call without a context on this thread).  Never NULL; the string is owned
 * by the library and valid until the next call on ctx.  (Diagnostics only:
 * no passage of the paper defines it.) */
const char *lbm_last_error(const lbm_ctx *ctx);

/* Set every fluid cell to the second-order equilibrium f_i^eq(rho, u) of
 * the given FP64 fields (rho_dev [n], u_dev [3][n]); resets the step count
 * to 0.  Equilibrium as in Eq. (1)'s f^eq with c_s^2 = 1/3. */
int lbm_init_equilibrium(lbm_ctx *ctx, const double *rho_dev, const double *u_dev);

/* Load canonical FP64 populations f_dev [q][n] (device, caller owned):
 * the PDFs f_i(x, t) of Section 2 after the streaming Eq. (2) and before
 * the collision Eq. (1), rounded to the storage format; solid cells are
 * ignored.  Resets the step count to 0.  LBM_EINVAL for NULL. */
int lbm_set_pdfs(lbm_ctx *ctx, const double *f_dev);

/* Write the canonical FP64 populations f_i(x, t) of Section 2 (after the
 * streaming Eq. (2), before the collision Eq. (1)) of the current step to
 * f_dev [q][n] (device, caller owned; solid cells: w_i).  Valid after any
 * number of steps.  LBM_EINVAL for NULL. */
int lbm_get_pdfs(lbm_ctx *ctx, double *f_dev);

/* Canonical FP64 populations f_i(x, t) of Section 2 at n >= 0 cells
 * (device linear indices cells_dev[n], int64, (z ny + y) nx + x) into
 * out_dev [n][q] (device, caller owned).  An index outside the domain
 * yields NaN in its row.  LBM_EINVAL for n < 0 or NULL with n > 0. */
int lbm_gather_pdfs(lbm_ctx *ctx, const int64_t *cells_dev, int64_t n, double *out_dev);

/* Advance n >= 0 time steps (Eq. (1) then Eq. (2) per step, fused in one
 * kernel per step).  Asynchronous.  LBM_EINVAL for n < 0, LBM_ESTATE when
 * the MLP closure has no weights, LBM_EDEVICE when a launch fails. */
int lbm_step(lbm_ctx *ctx, int64_t n);

/* Steps (applications of Eq. (1)-(2)) taken since the last init/set/load;
 * -1 for ctx == NULL. */
int64_t lbm_time(const lbm_ctx *ctx);

/* The local fluid properties on which f^eq of Eq. (1) depends (Section 2):
 * density rho_dev [n] = sum_i f_i and velocity u_dev [3][n] = (j + F/2)/rho
 * of the current canonical state, FP32, device, caller owned (solid cells:
 * rho = 1, u = 0).  Asynchronous.  LBM_EINVAL for NULL. */
int lbm_moments(lbm_ctx *ctx, float *rho_dev, float *u_dev);

/* FP64 totals over fluid cells of the current state (host outputs):
 * *mass = sum rho, mom = sum_i c_i f_i -- the mass conservation the
 * turbulent-channel case is assessed on (Section 5.1).  Deterministic.
 * Synchronises.  Returns LBM_ENONFINITE if any fluid population is NaN or
 * Inf (the totals are still written), LBM_EINVAL for NULL. */
int lbm_totals(lbm_ctx *ctx, double *mass, double mom[3]);

/* Bytes of the raw population store (for checkpoints of the single PDF
 * set kept in place, Section 5.2): q rows of sx cells per stored row,
 * sx = nx rounded up to whole 128-byte lines, with the Esoteric Twist's
 * ghost layers included; with sparse addressing q values per fluid cell, in
 * chunks of 64; with the HRR collision followed by its two velocity
 * fields.  Its layout is internal; only lbm_load_state of a context with
 * the same domain and flags reads it back.  LBM_EINVAL for NULL. */
int lbm_state_bytes(const lbm_ctx *ctx, size_t *out);

/* Copy the raw state (the PDF set of Section 5.2's in-place streaming) to
 * dst_dev (device, caller owned, lbm_state_bytes bytes) and report the step
 * count through *time (host); lbm_load_state restores both from src_dev.
 * Asynchronous.  A restored run continues bit for bit as the saved one
 * would have.  LBM_EINVAL for NULL or time < 0. */
int lbm_save_state(lbm_ctx *ctx, void *dst_dev, int64_t *time);
int lbm_load_state(lbm_ctx *ctx, const void *src_dev, int64_t time);

/*
 * Learned subgrid closure of the LES turbulent channel (Section 5.1: the
 * subgrid shear stresses along the wall-normal direction), weights (host,
 * FP32, read only during the call): n = 1313 + 24 values, the MLP
 * 6 -> 32 -> 32 -> 1 as W1[32][6], b1[32], W2[32][32], b2[32], W3[32], b3,
 * then per input mu[6], sigma[6], lo[6], hi[6] (standardisation and the
 * trusted input range; outside it the cell falls back to Smagorinsky).
 * Weights are rounded to bfloat16 for the matrix cores.  Synchronises.
 */
int lbm_set_closure_weights(lbm_ctx *ctx, const float *params, size_t n);

/* Number of fluid-cell updates of the Section 5.1 LES closure that fell
 * back to Smagorinsky since the last call (MLP closure only) into *count
 * (host); resets the counter.  Synchronises.  LBM_EINVAL for NULL. */
int lbm_closure_fallbacks(lbm_ctx *ctx, int64_t *count);

/* The learned closure's six inputs of every cell, from the current state,
 * as the fused closure computes them before its network (the subgrid model
 * of the Section 5.1 LES channel): tr P, |dev P|, cbrt det dev P of
 * P = P_c / rho, rho - 1, tau_s - tau (Smagorinsky with cs_smag) and tau,
 * where P_c is the non-equilibrium momentum flux with its forcing
 * correction.  x_dev [n][6] FP32 (device, caller owned); solid cells get
 * NaN.  Works with any closure setting (the features do not depend on it).
 * Asynchronous.  LBM_EINVAL for NULL. */
int lbm_closure_features(lbm_ctx *ctx, float *x_dev);

/* ------------------------------------------------------------------------ */
/* Training-data and training kernels of the learned closure (the subgrid   */
/* stresses of the Section 5.1 LES channel).  All pointers are device       */
/* memory owned by the caller; work is enqueued on `stream`; LBM_EINVAL for  */
/* invalid sizes or NULL, LBM_EDEVICE when a launch fails.                   */
/* ------------------------------------------------------------------------ */

/* Box filter over non-overlapping 4x4x4 blocks of fine FP32 fields
 * rho_dev [n], u_dev [3][n] (nx, ny, nz multiples of 4, fewer than 2^31
 * cells, else LBM_ENOMEM) into out_dev
 * [10][n/64] FP32: rho, u_x, u_y, u_z, then the filtered products uu in
 * the order xx, yy, zz, xy, xz, yz. */
int lbm_box_filter4(int32_t nx, int32_t ny, int32_t nz, const float *rho_dev, const float *u_dev, float *out_dev,
                    void *stream);

/* Closure dataset from filtered coarse fields filt_dev [10][n] (cx, cy, cz
 * cells, periodic[3] per axis; non-periodic axes have walls halfway outside
 * the first/last cell): features x_dev [n][6] and target dtau t_dev [n],
 * FP32 (fewer than 2^31 coarse cells, else LBM_ENOMEM).  tau is the
 * molecular relaxation time of the coarse lattice, cs the Smagorinsky
 * constant used for feature 5. */
int lbm_closure_dataset(int32_t cx, int32_t cy, int32_t cz, const int32_t periodic[3], const float *filt_dev,
                        double tau, double cs, float *x_dev, float *t_dev, void *stream);

/* MLP forward over a batch: params_dev (1313 + 24 FP32, layout as in
 * lbm_set_closure_weights), x_dev [n][6] -> y_dev [n] FP32.  Matrix
 * products on bfloat16 matrix cores with FP32 accumulation. */
int lbm_mlp_forward(const float *params_dev, const float *x_dev, int64_t n, float *y_dev, void *stream);

/* Mean-squared-error loss over the batch and its gradient with respect to
 * the 1313 parameters: grad_dev [1313] FP32 (overwritten), loss_dev [1]
 * FP32.  Deterministic (fixed reduction order).  work_dev must hold
 * lbm_mlp_work_bytes(n) bytes. */
size_t lbm_mlp_work_bytes(int64_t n);
int lbm_mlp_loss_grad(const float *params_dev, const float *x_dev, const float *t_dev, int64_t n, float *grad_dev,
                      float *loss_dev, void *work_dev, void *stream);

/* Allocation-free variant of lbm_mlp_loss_grad, for callers that cannot
 * allocate device memory (code under graph capture, serving loops,
 * harnesses that forbid allocation): the same kernels and the same results
 * bit for bit, with the per-block partial gradients in a static device array
 * of the library instead of work_dev.  Limit: that array holds 512 partials
 * of 1314 floats (2 690 048 bytes) per device, independent of n, and each
 * device keeps its copy until the process ends; LBM_EINVAL if the partials
 * of n samples would not fit it, for n < 1 or a NULL pointer.  Every call on
 * a device shares that device's array and leaves its contents behind: calls
 * that overlap on one device race.  Allocates no memory. */
int lbm_mlp_loss_grad_noalloc(const float *params_dev, const float *x_dev, const float *t_dev, int64_t n,
                              float *grad_dev, float *loss_dev, void *stream);

/* One Adam step on the first 1313 entries of params_dev with FP32 moment
 * buffers m_dev, v_dev [1313]; step is 1-based. */
int lbm_mlp_adam(float *params_dev, const float *grad_dev, float *m_dev, float *v_dev, int64_t step, double lr,
                 double beta1, double beta2, double eps, void *stream);

/* ------------------------------------------------------------------------ */
/* Measurement helper.                                                       */
/* ------------------------------------------------------------------------ */

/* Plain device copy of bytes (multiple of 16) from src_dev to dst_dev (both
 * 16-byte aligned, else LBM_EINVAL): the
 * device analogue of the STREAM copy the paper uses to measure the machine
 * bandwidth b_s of its roofline P_max = b_s / n_b (Section 5.2, Eq. (3)). */
int lbm_stream_copy(const void *src_dev, void *dst_dev, size_t bytes, void *stream);

/* 2:1 grid refinement (the paper's 2:1 block refinement, Section 3, whose
 * levels coarse-to-fine and fine-to-coarse kernels join, Section 5.2), read
 * as the volumetric, mass-conservative exchange of Rohde et al. (2006).
 *
 * A coarse lattice and fine lattices below it (fine_lo: its +y face meets
 * the coarse -y face) and/or above it (fine_hi: its -y face meets the coarse
 * +y face).  Every face between two levels has kind LBM_BC_INTERFACE; every
 * other y face is not an interface.  Each fine lattice has twice the coarse
 * nx and nz, x and z are periodic on every level, and the levels share the
 * stencil, the collision (TRT or MRT with equal ghost rates and magic
 * parameter), no closure, the dense AA pattern and the HIP stream.  Acoustic
 * scaling: tau_f = 1/2 + 2 (tau_c - 1/2), force_f = force_c / 2 (relative
 * tolerance 1e-9).  Interface rows hold no solid cells (lbm_create rejects
 * flags there).  Storage formats may differ between levels.
 *
 * Per coarse step: one coarse step; each fine level takes two steps.  The
 * packet f*_i a coarse interface cell X sends across enters the fine level
 * after each fine substep, in the fine interface cells whose source point
 * x_f - c_i (fine units) lies in X; the packets the fine interface cells
 * send across in the two substeps are summed over the cells whose target
 * point x_f + c_i lies in coarse cell Y, divided by 8 (the volume ratio),
 * and become Y's populations.  sum_coarse rho + sum_fine rho / 8 is
 * conserved exactly.  Between calls every slot holds mass of its level:
 * the fine interface row's populations from the coarse level are the
 * second half of the last coarse step's packets.
 *
 * lbm_refine_work_bytes: bytes of the work buffer for a coarse domain (FP32
 * planes [2][q][nz][nx]: the fine packets' running sums, one plane per
 * interface side).  LBM_EINVAL for NULL or a bad stencil. */
int lbm_refine_work_bytes(const lbm_domain *coarse, int stencil, size_t *bytes);

/* Advance the coarse lattice n >= 0 steps and each fine lattice 2n steps.
 * fine_lo / fine_hi may be NULL where the coarse face is not an interface.
 * work_dev: device buffer of at least lbm_refine_work_bytes (caller owned,
 * 4-byte aligned).  Asynchronous, on the shared stream.  LBM_EINVAL when
 * the lattices do not form a refinement as stated above, for a NULL or
 * small work buffer or n < 0 (checked before any work is enqueued);
 * LBM_EDEVICE when a launch fails, which leaves the lattices part way
 * through a coarse step (restore them from a checkpoint). */
int lbm_refine_step(lbm_ctx *coarse, lbm_ctx *fine_lo, lbm_ctx *fine_hi, void *work_dev, size_t work_bytes,
                    int64_t n);

/* Hierarchies of 2:1 levels (the paper's refinement trees, Section 3): each
 * level may be refined again, so the levels form a stack along y whose
 * cell size halves from level to level away from the coarsest one, e.g.
 * fine2 | fine1 | coarse | fine1 | fine2.  A node is a lattice and the
 * indices (into the node array, -1 for none) of the finer lattices below
 * (fine_lo) and above (fine_hi) it; nodes[0] is the coarsest lattice and
 * every child comes after its parent and has exactly one.  Each parent and
 * child pair satisfies the conditions of lbm_refine_step, and a y face is an
 * interface exactly where it meets another level (so a child has no child on
 * its parent's side).  work_dev / work_bytes: the node's work buffer as for
 * lbm_refine_step, needed by nodes with a child (distinct buffers; ignored
 * otherwise; LBM_EINVAL if two of them overlap).  The node array is read
 * during the call only. */
typedef struct lbm_refine_node {
    lbm_ctx *ctx;
    int32_t fine_lo, fine_hi;
    void *work_dev;
    size_t work_bytes;
} lbm_refine_node;

/* Advance nodes[0] n >= 0 steps; a node at depth d takes 2^d steps per step
 * of nodes[0]: each node takes its own step, then for each child the child
 * advances two steps (recursively, each followed by the exchange of
 * lbm_refine_step), then the node's interface rows take the summed packets.
 * 1 <= count <= 4096.  Errors as for lbm_refine_step, reported on nodes[0]
 * (on the thread's global error text for a NULL array or context), and
 * LBM_ENOMEM when the host memory for the validation runs out; a failed
 * launch leaves every level part way through a step.
 * lbm_refine_step(c, lo, hi, ...) is this call on the nodes {c, lo, hi}. */
int lbm_refine_tree_step(const lbm_refine_node *nodes, int32_t count, int64_t n);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
