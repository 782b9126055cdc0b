/*
 * libphurbas: the per-particle spatial-derivative stage of the Phurbas
 * adaptive Lagrangian meshless MHD method (McNally, Maron & Mac Low, paper II,
 * arXiv:1110.0836) on one AMD Instinct MI355X (gfx950).
 *
 * The library finds every neighbor inside the sphere of radius
 * r_f,i = 2.3 lambda_i about each particle (Sec. 2 and 2.1), fits a local
 * weighted third-order (20-monomial) moving-least-squares polynomial to each
 * particle's neighborhood (Sec. 2), applies the resulting derivative operator
 * to the carried fields and forms the ideal-MHD Lagrangian time derivatives
 * (Sec. 2; the evolution equations of App. A without viscosity) that drive
 * the second-order predictor-corrector step (Sec. 2).  A hand-written
 * reverse-mode kernel gives gradients of a scalar of those time derivatives.
 *
 * Conventions for every entry point
 *  - Pointers are DEVICE pointers unless marked "host".  phb_params and
 *    phb_ctx are host objects.
 *  - Arrays are structure-of-arrays, FP64 unless stated, in the caller's
 *    particle order, particle index fastest: pos[3][n], lambda[n], fields
 *    q[8][n] = (rho, Vx, Vy, Vz, Bx, By, Bz, sigma).
 *  - Neighbor lists are CSR: offsets int64[n+1] (offsets[0] = 0),
 *    idx int32[nnz]; row i lists, in ascending order, every j (i itself
 *    included) with  d2 < r*r,  where per axis dx = x_j - x_i, then on a
 *    periodic axis dx -= L if dx > L/2, else dx += L if dx < -L/2;
 *    d2 = (dx*dx + dy*dy) + dz*dz evaluated in FP64 without fused
 *    multiply-adds, and r = rf_ratio * lambda_i.  Rows are gathered with the
 *    centre's radius and the relation is not mutual (Sec. 2.1).
 *  - The caller allocates and owns every input and output buffer.  The
 *    library owns only the context, its workspace and its stream binding,
 *    and never frees caller memory.
 *  - Work is enqueued on the context's stream.  Calls that must size their
 *    output (neighbor build, steps) read a few bytes back to the host and so
 *    synchronize that stream; the others return without waiting.
 *  - Return codes: PHB_OK (0) or a negative PHB_E* code.  Nothing throws
 *    across this boundary.  phb_last_error() gives the message of the last
 *    failure on a context.
 *  - Per-particle numerical failure is not an error: status[i] is
 *    PHB_STATUS_OK, PHB_STATUS_TOO_FEW (fewer than 20 neighbors, i itself
 *    included) or PHB_STATUS_SINGULAR (the equilibrated 20x20 moment matrix
 *    has a non-positive pivot or reciprocal condition estimate
 *    (min L_kk / max L_kk)^2 below 1e-12), and that particle's derivative
 *    outputs are NaN.
 *  - Inputs are validated on the device before use: every position must be
 *    finite and inside [0, L) on every axis, every lambda finite and
 *    positive, and rf_ratio * lambda below L/2 on every periodic axis;
 *    otherwise PHB_EINVAL.
 */
#ifndef PHURBAS_H
#define PHURBAS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PHB_OK 0
#define PHB_EINVAL (-1)    /* bad argument or out-of-domain input data */
#define PHB_ENOMEM (-2)    /* workspace allocation failed */
#define PHB_ECAPACITY (-3) /* caller buffer too small; the needed size is reported */
#define PHB_EHIP (-4)      /* HIP runtime error (see phb_last_error) */
#define PHB_ESTATE (-5)    /* call not allowed in the context's current state */
#define PHB_ENOTIMPL (-6)  /* option not built */

#define PHB_FP64 0        /* all arithmetic in FP64 */
#define PHB_MIXED 1       /* without a tape: FP32 assembly and application,
                             FP64 factor and solve, one refinement step (see
                             mixed_refine: by default one Newton step on the
                             operator rows with an FP64 residual product);
                             particles whose FP32 moment matrix is too
                             ill-conditioned for one step are evaluated in
                             FP64 (see mixed_cond_x10).  With a tape (a call
                             the reverse mode follows) the forward is the
                             FP64 form's data form, since the reverse mode
                             needs the FP64 moments and FP32 arithmetic runs
                             no faster than FP64 here, and the reverse mode
                             stores its pair records in FP32 */
#define PHB_W_POLY3 0     /* w = (1 - d^2/r_f^2)^3 */
#define PHB_W_UNIT 1      /* w = 1 */
#define PHB_FIT_FULL20 0  /* all 20 monomials, constant included */
#define PHB_FIT_INTERP19 1 /* interpolating fit (acknowledgements of the paper: the tests
                              use interpolating fits): the 19 monomials without the
                              constant, so the fit passes through the particle's own
                              value; same status rules */

/* Largest number of neighbor entries the reverse mode and the transposed
 * lists handle: their positions (t_src, t_pos) are int32. */
#define PHB_NNZ_MAX 2147483647LL

#define PHB_STATUS_OK 0
#define PHB_STATUS_TOO_FEW 1
#define PHB_STATUS_SINGULAR 2

typedef struct phb_ctx phb_ctx;

typedef struct {
  double L[3];          /* box lengths; positions live in [0, L) */
  int32_t periodic[3];  /* 1: minimum-image periodic axis, 0: open axis */
  double gamma;         /* adiabatic index of P = (gamma - 1) sigma */
  double rf_ratio;      /* r_f / lambda; the paper uses 2.3 */
  int32_t precision;    /* PHB_FP64 or PHB_MIXED */
  int32_t weight;       /* PHB_W_POLY3 or PHB_W_UNIT */
  int32_t fit;          /* PHB_FIT_FULL20 or PHB_FIT_INTERP19 */
  /* Non-ideal stabilisers (Sec. 2: a bulk viscosity with a grid-scale and an
   * adaptive coefficient field, and a diffusive div-B term in the induction
   * equation; App. A: the viscous acceleration grad(zeta div V)).  All zero
   * (the default) is ideal MHD.  With c_f = sqrt((gamma P + B^2) / rho) and
   * s = min(1, (lambda |grad rho| / rho)^2):
   *   zeta = lambda c_f (visc_grid + visc_adapt s),  eta = divb_diff lambda c_f,
   *   dV/dt += zeta grad div V,  dB/dt += eta grad div B,
   *   dsigma/dt += rho zeta (div V)^2,
   * zeta and eta held constant over each neighborhood.  Each must be finite
   * and >= 0 (else PHB_EINVAL).  Every call supports them, in both
   * precisions, the reverse mode included. */
  double visc_grid;
  double visc_adapt;
  double divb_diff;
} phb_params;

/* ---- context ------------------------------------------------------------
 * phb_create: bind a new context to HIP device `device` and stream
 * `hip_stream` (a hipStream_t; NULL = the default stream).  *out receives the
 * context.  EINVAL on a null out or bad device; EHIP on runtime failure. */
int phb_create(phb_ctx** out, int device, void* hip_stream);
/* Release the context and its workspace (waits for its stream first). */
int phb_destroy(phb_ctx* ctx);
/* Rebind the context to another stream of the same device. */
int phb_set_stream(phb_ctx* ctx, void* hip_stream);
/* Grow the workspace for up to n_max particles and nnz_max neighbor entries
 * so that later calls of the neighbor build (also _async), the transpose,
 * phb_mls_derivs, phb_mhd_rhs and the reverse mode (also _async) within
 * those sizes allocate nothing: what a HIP graph capture of them needs. */
int phb_reserve(phb_ctx* ctx, int64_t n_max, int64_t nnz_max);
/* Static text for a return code. */
const char* phb_strerror(int code);
/* Message of the last failure on ctx (never NULL). */
const char* phb_last_error(phb_ctx* ctx);

/* ---- neighbor search (Sec. 2 and 2.1) ------------------------------------
 * Build the CSR neighbor lists of n particles.  offsets: int64[n+1];
 * idx: int32[idx_capacity].  *nnz_out (host) receives the total number of
 * entries.  If it exceeds idx_capacity the call returns PHB_ECAPACITY, fills
 * offsets but leaves idx unspecified; call again with a larger buffer.
 * Synchronizes the context stream once, at the end (nnz and the status are
 * read back).  n < 2^31. */
int phb_neighbors_build(phb_ctx* ctx, const phb_params* p, int64_t n, const double* pos,
                        const double* lambda, int64_t* offsets, int32_t* idx,
                        int64_t idx_capacity, int64_t* nnz_out);
/* The same without any host synchronization, for capture in a HIP graph:
 * nnz_dev (int64, device) receives the total and flag_dev (int32, device)
 * the status: 0, or a combination of PHB_NB_OVERFLOW (more than
 * idx_capacity entries: offsets and nnz are written, idx is not),
 * PHB_NB_INVALID (a position outside [0, L) or not finite, or a lambda that
 * is not positive) and PHB_NB_RADIUS (r_f >= L/2 on a periodic axis); with
 * either of the last two, offsets and nnz are zero.  Asynchronous; it
 * allocates nothing once the workspace covers the set (phb_reserve), so a
 * capture of it needs the workspace reserved first. */
#define PHB_NB_OVERFLOW 1
#define PHB_NB_INVALID 2
#define PHB_NB_RADIUS 4
int phb_neighbors_build_async(phb_ctx* ctx, const phb_params* p, int64_t n, const double* pos,
                              const double* lambda, int64_t* offsets, int32_t* idx,
                              int64_t idx_capacity, int64_t* nnz_dev, int32_t* flag_dev);
/* The lists of the m particles rows[0 .. m) (int32, in [0, n); m may be 0)
 * among all n: offsets int64[m+1], idx as for phb_neighbors_build, rows in
 * the given order, each sorted ascending.  The same errors. */
int phb_neighbors_build_rows(phb_ctx* ctx, const phb_params* p, int64_t n, const double* pos,
                             const double* lambda, int64_t m, const int32_t* rows,
                             int64_t* offsets, int32_t* idx, int64_t idx_capacity,
                             int64_t* nnz_out);

/* Transposed lists for the reverse-mode kernels: t_offsets int64[n+1],
 * t_src int32[nnz] (row j lists, ascending, every i whose row holds j),
 * t_pos int32[nnz] (for forward entry s = (i, j): the index into t_src at
 * which i appears in row j).  nnz = offsets[n], or any bound of it (the
 * idx capacity of a build whose total stays on the device): it only sizes
 * the scratch.  PHB_EINVAL if nnz exceeds PHB_NNZ_MAX (the positions are
 * int32).  Asynchronous. */
int phb_neighbors_transpose(phb_ctx* ctx, int64_t n, int64_t nnz, const int64_t* offsets,
                            const int32_t* idx, int64_t* t_offsets, int32_t* t_src,
                            int32_t* t_pos);

/* A spatially coherent particle order: the Peano-Hilbert order of the
 * particles' cells on a 1024^3 grid over the box (Sec. 2.1 orders particles
 * along the same curve), ties by index.  perm int32[n] lists caller indices
 * in that order; kernels run fastest on data permuted into it.  Positions
 * and lambdas are validated as for the neighbor build.  Synchronizes. */
int phb_spatial_order(phb_ctx* ctx, const phb_params* p, int64_t n, const double* pos,
                      const double* lambda, int32_t* perm);

/* Gather rows: dst[c][k] = src[c][perm[k]] for c < ncomp, k < n.  src and
 * dst must not overlap.  Asynchronous. */
int phb_permute(phb_ctx* ctx, int64_t n, const int32_t* perm, int32_t ncomp, const double* src,
                double* dst);

/* ---- moving-least-squares derivatives (Sec. 2) ---------------------------
 * For each particle fit f_j - f_i over its neighbors with the 20 monomials
 * of xi = (x_j - x_i) / lambda_i (min-image), weighted, and return physical
 * derivatives of nf fields: d1[nf][3][n] (d/dx, d/dy, d/dz) and, when
 * max_order == 2, d2[nf][6][n] (xx, xy, xz, yy, yz, zz; d2 may be NULL when
 * max_order == 1).  status int32[n].  Asynchronous. */
int phb_mls_derivs(phb_ctx* ctx, const phb_params* p, int64_t n, const double* pos,
                   const double* lambda, const int64_t* offsets, const int32_t* idx, int32_t nf,
                   const double* fields, int32_t max_order, double* d1, double* d2,
                   int32_t* status);

/* ---- ideal-MHD time derivatives (Sec. 2; App. A without viscosity) -------
 * rhs[8][n] = d/dt of (rho, V, B, sigma) following the particle:
 *   drho/dt = -rho div V ; dV/dt = (-(gamma-1) grad sigma + (curl B) x B) / rho ;
 *   dB/dt = (B . grad) V - B div V ; dsigma/dt = -gamma sigma div V ;
 * dxdt[3][n] = V.  status int32[n].  tape: NULL or a device buffer of
 * phb_tape_bytes(n) bytes that keeps what the reverse-mode call reuses.
 * First 31 rows of ld doubles each (ld >= n, padded so that the row stride
 * is not a power of two), particle i at [row][i]: rows 0..20 the gradients of
 * V, B, sigma (3 each), 21 the status, 22..30 grad rho, grad div V and
 * grad div B (stabilisers on).  Then
 * PHB_TAPE_AOS doubles per particle (n blocks, particle i at i *
 * PHB_TAPE_AOS), written in the FP64 form: rows 1..3 of the inverse moment
 * matrix A^{-1} (1..9 with the stabilisers), then the fit coefficients
 * C = A^{-1} B of V, B, sigma (of all eight fields with the stabilisers),
 * 20 each; the block's first 200 (340) doubles are used.  So
 * phb_tape_bytes(n) = 8 (31 ld + PHB_TAPE_AOS n).  Asynchronous. */
#define PHB_TAPE_AOS 340
int phb_mhd_rhs(phb_ctx* ctx, const phb_params* p, int64_t n, const double* pos,
                const double* lambda, const int64_t* offsets, const int32_t* idx,
                const double* q, double* rhs, double* dxdt, int32_t* status, void* tape);
int64_t phb_tape_bytes(int64_t n);

/* ---- allocation-free variant ----------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Arguments,
 * results and errors are those of phb_mhd_rhs, computed by the same kernels;
 * every intermediate buffer lives in a file-scope device array of
 * PHB_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it runs on
 * until the process ends.  The call allocates nothing (no device memory, no
 * events, no second stream).  PHB_ECAPACITY when the set
 * needs more scratch than that: about 3.1 KB per particle in the ideal FP64
 * form (n up to about 21,000), 3.6 KB with the stabilisers; the mixed form
 * needs more.  Calls that overlap on one GPU share the array and race
 * (whatever their context or stream): serialize them.  The array keeps the
 * last call's contents, which no later call reads before writing.  (The HIP
 * runtime loads the library's device code at the first launch of its kernels
 * in a process, an allocation of its own: callers that must not allocate at
 * all make one call first, for instance before a graph capture.)
 * Asynchronous. */
#define PHB_NOALLOC_SCRATCH_BYTES (64LL << 20)
int phb_mhd_rhs_noalloc(phb_ctx* ctx, const phb_params* p, int64_t n, const double* pos,
                        const double* lambda, const int64_t* offsets, const int32_t* idx,
                        const double* q, double* rhs, double* dxdt, int32_t* status, void* tape);
/* Active-subset evaluation (Sec. 2: each particle has its own time step, so
 * only some particles need new time derivatives at a time): the time
 * derivatives of the m particles rows[0 .. m) (int32, distinct, in [0, n)),
 * each from its neighbors among all n particles.  offsets int64[m+1] and
 * idx hold the lists of those rows (phb_neighbors_build_rows); rhs[8][m],
 * dxdt[3][m], status int32[m] are per row.  FP64 form only: PHB_ENOTIMPL
 * with PHB_MIXED.  EINVAL for m outside [1, n]. */
int phb_mhd_rhs_rows(phb_ctx* ctx, const phb_params* p, int64_t n, const double* pos,
                     const double* lambda, int64_t m, const int32_t* rows,
                     const int64_t* offsets, const int32_t* idx, const double* q, double* rhs,
                     double* dxdt, int32_t* status);

/* ---- reverse mode --------------------------------------------------------
 * Gradient of  S = sum_i rhs_bar_i . rhs_i + dxdt_bar_i . dxdt_i  with respect
 * to q (q_bar[8][n]) and positions (pos_bar[3][n]), neighbor lists held
 * fixed.  dxdt_bar may be NULL (zero).  t_* come from
 * phb_neighbors_transpose of the same lists.  tape: the buffer filled by
 * phb_mhd_rhs on the same inputs, or NULL to recompute it.  Particles with
 * nonzero status pass no gradient through rhs.  Outputs are overwritten.
 * Deterministic: contributions are summed in a fixed order, without atomics.
 * Asynchronous. */
int phb_mhd_rhs_adjoint(phb_ctx* ctx, const phb_params* p, int64_t n, const double* pos,
                        const double* lambda, const int64_t* offsets, const int32_t* idx,
                        const int64_t* t_offsets, const int32_t* t_src, const int32_t* t_pos,
                        const double* q, const double* rhs_bar, const double* dxdt_bar,
                        double* q_bar, double* pos_bar, const void* tape);
/* The same without reading offsets[n] back (phb_mhd_rhs_adjoint does, to size
 * its pair records): nnz_bound >= offsets[n] sizes them instead, so that the
 * call can be captured in a HIP graph after phb_neighbors_build_async, whose
 * total stays on the device (its idx capacity is such a bound).
 * adj_pairs_mode 0 (one lane per entry, sized by the exact count) runs as 1
 * here. */
int phb_mhd_rhs_adjoint_async(phb_ctx* ctx, const phb_params* p, int64_t n, const double* pos,
                              const double* lambda, const int64_t* offsets, const int32_t* idx,
                              const int64_t* t_offsets, const int32_t* t_src,
                              const int32_t* t_pos, const double* q, const double* rhs_bar,
                              const double* dxdt_bar, double* q_bar, double* pos_bar,
                              const void* tape, int64_t nnz_bound);

/* ---- predictor-corrector step (Sec. 2) -----------------------------------
 * Advance (pos, q) in place by dt with Heun's trapezoidal scheme:
 *   y* = y + dt F(y);  y <- y + dt/2 (F(y) + F(y*)),  y = (x, q),  F = (V, rhs),
 * rebuilding the neighbor lists at the predicted state and wrapping positions
 * into [0, L) on periodic axes after each stage.  On return offsets/idx hold
 * the lists of the predicted state.  status[i] is the larger of the two
 * stages' statuses.  PHB_ECAPACITY (with *nnz_out) when idx is too small;
 * PHB_EINVAL when a particle leaves [0, L) on an open axis.  Synchronizes. */
int phb_pc_step(phb_ctx* ctx, const phb_params* p, int64_t n, double dt, double* pos, double* q,
                const double* lambda, int64_t* offsets, int32_t* idx, int64_t idx_capacity,
                int64_t* nnz_out, int32_t* status);

/* ---- time evolution (Sec. 2; the tests of Sec. 3.1, 3.2) -----------------
 * nsteps predictor-corrector steps of size dt, as phb_pc_step.  frozen: NULL or
 * int32[n]; a particle with frozen[i] != 0 keeps its position and fields (a
 * fixed-value boundary particle, as in the shock-tube and MRI set-ups of
 * Sec. 3.3 and 3.5) but still serves as a neighbor.  status[i]: the largest
 * status over all stages of all steps (0 for frozen particles; 0 everywhere when
 * nsteps == 0).  Errors as phb_pc_step; the state is then that of the last
 * completed step.  Synchronizes. */
int phb_evolve(phb_ctx* ctx, const phb_params* p, int64_t n, double dt, int32_t nsteps,
               double* pos, double* q, const double* lambda, const int32_t* frozen,
               int64_t* offsets, int32_t* idx, int64_t idx_capacity, int64_t* nnz_out,
               int32_t* status);
/* Individual power-of-two time steps (Sec. 2 and 2.1): nblocks periods of
 * dt_max in which particle i takes steps of dt_max / 2^k_i.  k_i is the
 * smallest level in [0, kmax] whose step is at most cfl times i's own
 * Courant step (the expression of phb_courant_dt); neighbors' levels differ
 * by at most one (k_i >= k_j - 1, enforced at i's step ends); a step grows
 * only where the current time is a multiple of the longer step.  Each step is
 * Heun's over the particle's own step, every other particle's state being
 * predicted linearly from its last step start; the particles ending a step
 * at a time are evaluated as a compacted row list (phb_neighbors_build_rows,
 * phb_mhd_rhs_rows).  With one level throughout this is phb_evolve with
 * dt = dt_max.  pos, q: updated in place (all particles end synchronized).
 * offsets int64[n+1], idx int32[idx_capacity]: list scratch, as for
 * phb_pc_step.  status int32[n]: the largest over all evaluations (0 for
 * frozen particles).  level int32[n] or NULL: the levels of the last steps.
 * stats: NULL or host int64[2] = (step-end times, particle evaluations).
 * FP64 form only (PHB_ENOTIMPL otherwise).  Synchronizes repeatedly. */
int phb_evolve_blocks(phb_ctx* ctx, const phb_params* p, int64_t n, double dt_max,
                      int32_t nblocks, double cfl, int32_t kmax, double* pos, double* q,
                      const double* lambda, const int32_t* frozen, int64_t* offsets,
                      int32_t* idx, int64_t idx_capacity, int32_t* status, int32_t* level,
                      int64_t* stats);
/* Courant time step: *dt_out (host) = cfl * min over non-frozen i of
 * lambda_i / (c_f,i (1 + 2 (visc_grid + visc_adapt + divb_diff))),
 * with the fast speed c_f = sqrt((gamma P + |B|^2) / rho), P = (gamma - 1)
 * sigma (the paper's own time-step criteria live in its companion paper;
 * Sec. 2 states that the steps do not depend on the bulk velocity); the
 * stabilisers' diffusivities enter at their largest as the speed
 * 2 (zeta + eta) / lambda.  NaN entries are skipped.
 * EINVAL if every particle is frozen or cfl <= 0.  Synchronizes. */
int phb_courant_dt(phb_ctx* ctx, const phb_params* p, int64_t n, const double* q,
                   const double* lambda, const int32_t* frozen, double cfl, double* dt_out);

/* ---- diagnostics (Sec. 3.3) ----------------------------------------------
 * phb_divb_norm: out[i] = lambda_i (div B)_i / |B_i|, the fractional magnetic
 * field error on the scale of lambda, from the fitted gradients of q rows 4..6
 * (same fit, precision and status rules as phb_mls_derivs).  out double[n];
 * status int32[n]; out is NaN where status != 0 or |B_i| = 0.  Device
 * pointers, asynchronous. */
int phb_divb_norm(phb_ctx* ctx, const phb_params* p, int64_t n, const double* pos,
                  const double* lambda, const int64_t* offsets, const int32_t* idx,
                  const double* q, double* out, int32_t* status);
/* phb_bin_mean: mean of the finite values[i] per bin b = floor((coord[i] - x0)
 * / width), 0 <= b < nbins, taken in FP64 (the paper bins the divergence
 * diagnostic in bins one lambda wide).  mean double[nbins] (NaN for an empty
 * bin), count int64[nbins] or NULL.  The sums are accumulated with atomic
 * adds, so the last bits of a mean may vary from call to call.  EINVAL for
 * nbins <= 0, width <= 0 or non-finite x0, width. */
int phb_bin_mean(phb_ctx* ctx, int64_t n, const double* coord, const double* values, double x0,
                 double width, int32_t nbins, double* mean, int64_t* count);

/* ---- many particle sets in one captured graph -----------------------------
 * Independent particle sets (each with its own neighbor lists; no set sees
 * another) are stored one after the other: set s owns the particles
 * set_offsets[s] .. set_offsets[s+1]-1 of every SoA array, and the CSR lists
 * hold global indices.  Every stage of an evaluation runs as one launch over
 * all sets, and the whole forward (+ reverse) pass is captured once into a
 * HIP graph and replayed with one graph launch.  All sets share phb_params
 * (box, physics, precision).  A batch holds a private stream on which it
 * captures and replays; phb_batch_launch orders the replay after the
 * context stream's earlier work and makes the context stream wait for it.
 *
 * phb_batch_create: n_sets > 0 sets; set_offsets (host) int64[n_sets+1],
 * starting at 0, strictly increasing, total < 2^31.  *out receives the batch.
 * phb_batch_destroy: waits for the batch stream and frees the batch. */
typedef struct phb_batch phb_batch;
int phb_batch_create(phb_ctx* ctx, const phb_params* p, int32_t n_sets,
                     const int64_t* set_offsets, phb_batch** out);
int phb_batch_destroy(phb_batch* b);
/* Neighbor lists of every set (each built as by phb_neighbors_build on that
 * set alone, indices shifted to global), into offsets int64[n_total+1] and
 * idx int32[idx_capacity].  *nnz_out (host): total entries; PHB_ECAPACITY
 * when idx is too small (the batch is then unusable until a call succeeds).
 * Drops a previously captured graph.  Synchronizes. */
int phb_batch_neighbors(phb_ctx* ctx, phb_batch* b, const double* pos, const double* lambda,
                        int64_t* offsets, int32_t* idx, int64_t idx_capacity, int64_t* nnz_out);
/* The buffers of one pass, all over n_total particles, as for phb_mhd_rhs and
 * phb_mhd_rhs_adjoint.  q_bar and pos_bar both NULL: forward only (then
 * rhs_bar, dxdt_bar and the transposed lists may be NULL).  tape may be NULL
 * (the reverse pass then recomputes it). */
typedef struct {
  const double* pos;
  const double* lambda;
  const int64_t* offsets;
  const int32_t* idx;
  const int64_t* t_offsets;
  const int32_t* t_src;
  const int32_t* t_pos;
  const double* q;
  double* rhs;
  double* dxdt;
  int32_t* status;
  void* tape;
  const double* rhs_bar;
  const double* dxdt_bar;
  double* q_bar;
  double* pos_bar;
} phb_batch_io;
/* One eager pass on the context stream (the reference for a replay). */
int phb_batch_run(phb_ctx* ctx, phb_batch* b, const phb_batch_io* io);
/* Run one eager pass (sizing the workspace, synchronizing), then capture the
 * same pass into the batch's graph, bound to these buffers: the caller keeps
 * them alive and in place for as long as it launches the graph.  The graph
 * runs in a workspace of its own (as large as the context's), held by the
 * batch until the next capture, neighbor build or destroy.  The schedule knobs
 * current at capture are baked in.  PHB_ESTATE before the neighbor lists are
 * built. */
int phb_batch_capture(phb_ctx* ctx, phb_batch* b, const phb_batch_io* io);
/* Replay the captured pass (asynchronous).  PHB_ESTATE if none is captured. */
int phb_batch_launch(phb_ctx* ctx, phb_batch* b);

/* ---- schedule knobs (set by the autotuner; every value gives the same
 * results to rounding) ------------------------------------------------------
 * Keys: "cells_per_rf" (1..4: neighbor-grid cells per minimum r_f),
 * "lanes_moments", "lanes_apply", "lanes_adj_y" (1, 2 or 4 lanes sharing one
 * particle's neighbor loop in the moment and application kernels and in the
 * untaped mixed form's residual-product kernel; the FP64 data form sums its
 * moments with four lanes in the factor's kernel whatever lanes_moments
 * says), "lanes_gather" (1, 2 or 4 lanes summing one particle's
 * transposed row in the reverse mode), "adj_pairs_mode" (0: one lane per
 * neighbor entry, 1: one wavefront per owner particle, 2: persistent
 * wavefronts that stage the next owner through direct-to-LDS loads while
 * computing the current one, 3, the default: one block per tile of 128
 * consecutive owners (a batch's sets tiled from their first particles), its
 * four wavefronts taking the owners in ascending order, summing the pair
 * terms whose target lies in the tile in LDS instead of writing them as
 * records), "record_order" (0:
 * pair records written at their transposed position, 1: written in forward
 * order and gathered through the inverse map), "mixed_cond_x10" (-1..120:
 * in the untaped mixed form a particle whose FP32-assembled moment matrix, scaled to
 * unit diagonal, has an estimated ||A^{-1}||_2 above 10^(value / 10) is
 * evaluated in FP64 instead; -1, the default, takes the refinement form's own
 * threshold, 10^2.5 for the operator-level step and 10^2 for the data-level
 * step; this knob moves results within the mixed tolerance, the others only
 * by rounding), "mixed_refine"
 * (the untaped mixed form's refinement step; 1: the rows G~ = E A~^{-1} of the inverse of
 * the FP32-assembled matrix are refined once, G^ = 2 G~ - (G~ A) A~^{-1},
 * with the product G~ A formed in FP64 over the neighbors, and G^ is applied
 * to the fields in FP32 (each operator weight formed in FP64, the sums in
 * FP32); 0: each field's coefficients are solved for and refined once from
 * their residuals at the neighbors, all sums in FP32 (corrected seminormal
 * equations); 2, the default: 1 for the three gradient rows (the ideal
 * right-hand side, first derivatives), 0 with nine rows (the stabilisers,
 * second derivatives); the forms agree within the mixed tolerance),
 * "fit_fields" (2 or 4: fields per lane in the data form's fit right-hand
 * sides), "moments_mfma" (0 or 1: the untaped mixed form's FP32 moments on the
 * matrix cores, 16 x 16 x 4 FP32 products of the weighted monomials),
 * "fp64_cut_x10" (-1..999: in the FP64 form a fit whose equilibrated
 * inverse has an operator row of 2-norm above 10^(value / 10) is refined on
 * the data; -1, the default, takes 10^2.5 with three rows and 10^1.7 with
 * nine, 999 refines none; moves results within the FP64 tolerance).  EINVAL
 * for an unknown key or value. */
int phb_tune_set(phb_ctx* ctx, const char* key, int value);
int phb_tune_get(phb_ctx* ctx, const char* key, int* value);
/* Autotuner: times one forward + reverse pass of the given set (or batch
 * concatenation) for each value of each of lanes_moments, lanes_apply,
 * lanes_adj_y, lanes_gather, adj_pairs_mode, record_order, fit_fields and
 * moments_mfma in turn
 * (coordinate descent from the current values; median of reps timed passes
 * after one warm-up; a value must win by 2% to replace the current one) and
 * leaves the winners set on ctx.  nnz (host) = offsets[n].  cache_path: NULL,
 * or a text file that, when it exists and was written for the same n, nnz,
 * precision and weight, supplies the values without timing, and otherwise
 * receives them.  Allocates its scratch buffers; synchronizes. */
int phb_tune(phb_ctx* ctx, const phb_params* p, int64_t n, const double* pos,
             const double* lambda, const int64_t* offsets, const int32_t* idx,
             const int64_t* t_offsets, const int32_t* t_src, const int32_t* t_pos, int64_t nnz,
             const double* q, int32_t reps, const char* cache_path);

/* ---- instrumentation -----------------------------------------------------
 * phb_profile: enable (1) or disable (0) per-kernel timing on ctx; clears the
 * totals.  While enabled every kernel launch is bracketed by HIP events on the
 * context stream.  phb_profile_read: synchronizes the stream and reports up
 * to max_entries kernels: names (host, 64 chars per entry, NUL-terminated),
 * total_ms and counts (host arrays); *n_out (host) receives the number of
 * distinct kernels seen. */
int phb_profile(phb_ctx* ctx, int enable);
int phb_profile_read(phb_ctx* ctx, int32_t max_entries, char* names, double* total_ms,
                     int32_t* counts, int32_t* n_out);

#ifdef __cplusplus
}
#endif

#endif /* PHURBAS_H */
