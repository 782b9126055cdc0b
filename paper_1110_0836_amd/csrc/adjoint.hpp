// Entry-point bodies built from several kernels: the reverse mode, the
// mixed-precision evaluation and the predictor-corrector step.
#pragma once

#include "internal.hpp"
#include "mls.hpp"

namespace phb {

int adjoint_rhs(phb_ctx* ctx, const EvalArgs& a, const phb_params* p, const int64_t* t_offsets,
                const int32_t* t_src, const int32_t* t_pos, const double* q,
                const double* rhs_bar, const double* dxdt_bar, double* q_bar, double* pos_bar,
                const double* tape, int64_t nnz_known, bool nnz_exact = true,
                const int32_t* tile_start = nullptr, int64_t ntiles = 0);
// Owners per tile of the reverse mode's tile schedule (tile_start above:
// device int32[ntiles + 1], the tiles' first particles and then n; null:
// uniform tiles of this size from particle 0).
int adjoint_pair_tile();
// Workspace bytes of adjoint_rhs (the lane-per-entry schedule's included).
size_t ws_bytes_adjoint(int64_t n, int64_t nnz, const phb_params* p, bool need_tape);

// Time derivatives in the requested precision (FP64 or mixed).
int eval_rhs(phb_ctx* ctx, const EvalArgs& a, const phb_params* p, const double* q, double* rhs,
             double* dxdt, int32_t* status, double* tape);
int eval_args(phb_ctx* ctx, const phb_params* p, int64_t n64, const double* pos,
              const double* lambda, const int64_t* offsets, const int32_t* idx, EvalArgs* a);

size_t mixed_rhs_bytes(int64_t n, bool stab);
// The mixed form without a tape (a taped mixed call runs the FP64 data form).
int mixed_rhs(phb_ctx* ctx, const EvalArgs& a, double gamma, const Stab& sb, const double* q,
              double* rhs, double* dxdt, int32_t* status);

int mixed_derivs(phb_ctx* ctx, const EvalArgs& a, int nf, const double* fields, double* d1,
                 double* d2, int32_t* status);
size_t mixed_derivs_bytes(int64_t n, bool second);

// One Heun step; frozen (nullable) marks particles held fixed; accumulate:
// status keeps the maximum over earlier steps.
int pc_step(phb_ctx* ctx, const phb_params* p, int n, double dt, double* pos, double* q,
            const double* lambda, const int32_t* frozen, int64_t* offsets, int32_t* idx,
            int64_t idx_capacity, int64_t* nnz_out, int32_t* status, int accumulate);
int courant_dt(phb_ctx* ctx, const phb_params* p, int n, const double* q, const double* lambda,
               const int32_t* frozen, double cfl, double* dt_out);
// Lists of rows built by the library itself (no range check of rows).
int neighbors_rows_unchecked(phb_ctx* ctx, const phb_params* p, int64_t n, const double* pos,
                             const double* lambda, int64_t m, const int32_t* rows,
                             int64_t* offsets, int32_t* idx, int64_t idx_capacity,
                             int64_t* nnz_out);
// Individual power-of-two time steps (phb_evolve_blocks).
int evolve_blocks(phb_ctx* ctx, const phb_params* p, int n, double* pos, double* q,
                  const double* lambda, const int32_t* frozen, double dt_max, int nblocks,
                  double cfl, int kmax, int64_t* offsets, int32_t* idx, int64_t idx_capacity,
                  int32_t* status, int32_t* level, int64_t* stats);

}  // namespace phb
