// FP64 refinement of screened (ill-conditioned) fits, and the kernels that
// turn coefficient rows into derivatives or time derivatives.
#pragma once

#include "internal.hpp"
#include "mls.hpp"

namespace phb {

// Most passes of the refinement: the plain solve and up to four corrections
// (each particle stops once converged; the operator rows of the reverse mode
// take up to REFINE_PASSES - 1 steps).
constexpr int REFINE_PASSES = 5;

// Screen cut on the largest 2-norm of a row of the equilibrated inverse
// among the nrows operator rows a factor kernel computes (the context's
// fp64_cut_x10, or the default of the shape: tight_rows for the FP64
// operator form, whose second-derivative rows are held to FP64 accuracy).
double fp64_screen_cut(const phb_ctx* ctx, int nrows, bool tight_rows = true);

// List of screened particles (device count) and the refinement's buffers, by
// list position: coefficients cbuf[f][20][ldc], residual sums dbuf[f][20][ldc],
// the last correction's size prev[f][ldc] (f < 8) and converged flags
// done[ldc].
struct RefineBufs {
  int32_t* list;
  int32_t* count;
  double* cbuf;
  double* dbuf;
  int64_t ldc;
  double* prev;
  int32_t* done;
};
// nf rows of residual sums per particle; with_c: and of coefficients.
void plan_refine(Workspace& ws, int64_t n, int nf, bool with_c = true);
RefineBufs take_refine(Workspace& ws, int64_t n, int nf, bool with_c = true);
// prev and done alone (for callers that lend their own list and buffers).
void plan_refine_state(Workspace& ws, int64_t n);
void take_refine_state(Workspace& ws, int64_t n, RefineBufs& r);

// Refined coefficient vectors (all 20) of nf <= 8 fields of the packed
// records fa[8 j + fb + f] for the listed particles, into r.cbuf.  mom: FP64
// moments [84][soa_ld(n)] by row index.
int refine_fits(phb_ctx* ctx, const EvalArgs& a, const double* fa, int fb, int nf,
                const double* mom, const RefineBufs& r);

// Refinement steps on the operator rows G (nr rows of 20 at the start of each
// listed owner's record of orec_len doubles); r.dbuf holds nr x 20 rows.
int refine_oprows(phb_ctx* ctx, const EvalArgs& a, int nr, const double* mom,
                  const RefineBufs& r, double* orec, int orec_len);

// The tape's AoS block for the listed particles: their refined coefficients
// (r.cbuf, as refine_fits leaves them), then refined operator rows.
int refine_tape(phb_ctx* ctx, const EvalArgs& a, int nr, const double* mom, const RefineBufs& r,
                double* aos);

// Coefficient (field f, monomial 1 + t) of the particle in column col at
// coef[(f * fstride + t0 + t) * cld + col].  list == null: every particle, column
// = particle; else the listed ones, column = list position.
// Time derivatives (and tape) from the gradient rows of V, B, sigma
// (coefficient fields 0..6) or, stab, from the nine rows of all eight fields.
hipError_t launch_rows_rhs_finish(hipStream_t s, const EvalArgs& a, bool stab, const double* coef,
                                  int fstride, int t0, int64_t cld, const int32_t* list,
                                  const int32_t* count, const int32_t* status, double gamma,
                                  const Stab& sb, double* rhs, double* dxdt, double* tape);
// First (and with ng == 9 second) derivatives of fields f0 .. f0 + nfc - 1.
hipError_t launch_rows_derivs_finish(hipStream_t s, const EvalArgs& a, int ng, const double* coef,
                                     int fstride, int t0, int64_t cld, const int32_t* list,
                                     const int32_t* count, const int32_t* status, int nfc, int f0,
                                     double* d1, double* d2);
// fa[8 i + f] = fields[f0 + f][i], f < nfc (zero beyond).
hipError_t launch_pack_chunk(hipStream_t s, int n, const double* fields, int f0, int nfc,
                             double* fa);

}  // namespace phb
