// Launchers of the moving-least-squares and time-derivative kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "phurbas.h"
#include "device.hpp"
#include "mhd.hpp"

namespace phb {

// Geometry and neighbor lists of one evaluation.  geo and fq are the packed
// per-particle records the neighbor loops read: geo[i] = (x, y, z, lambda)
// (32 bytes) and fq[8 i .. 8 i + 7] = the eight fields (64 bytes), so that one
// neighbor costs one or two cache lines instead of one line per array.
struct EvalArgs {
  int n;
  const double* pos;
  const double* lam;
  const int64_t* off;
  const int32_t* idx;
  Box box;
  double rf_ratio;
  int wkind;
  int fit = PHB_FIT_FULL20;  // PHB_FIT_FULL20 or PHB_FIT_INTERP19
  const double4* geo = nullptr;
  const double* fq = nullptr;
  // Row subset: n rows whose own particles are rows[0 .. n) out of n_all
  // (the lists off/idx and every per-row output then have n rows); null
  // rows: row i is particle i and n_all = n.
  const int32_t* rows = nullptr;
  int n_all = 0;
};

// Tape of the forward evaluation.  First TAPE_DOUBLES rows (SoA, leading
// dimension soa_ld(n)): 21 gradients (V, B, sigma x 3), the status, grad rho,
// grad div V and grad div B (written only with the stabilisers on).  Then,
// written by the FP64 form,
// one block of TAPE_AOS doubles per particle (AoS, the reverse mode's
// per-owner data): the operator rows G (rows 1..nr of A^{-1}, nr = 3, or 9
// with the stabilisers) at 0 and the fit coefficients C = A^{-1} B of the
// fields those rows apply to (7 or 8 x 20) at nr x 20.
constexpr int TAPE_STATUS = 21;
constexpr int TAPE_GRHO = 22;
constexpr int TAPE_GDV = 25;
constexpr int TAPE_GDB = 28;
constexpr int TAPE_DOUBLES = 31;
constexpr int TAPE_AOS = (9 + 8) * NBASIS;
// Doubles of a tape of n particles.
__host__ __device__ constexpr int64_t tape_doubles(int64_t n) {
  return n <= 0 ? 0 : (int64_t)TAPE_DOUBLES * soa_ld(n) + (int64_t)TAPE_AOS * n;
}
// The AoS block of the tape.
__host__ __device__ inline double* tape_aos(double* tape, int64_t n) {
  return tape + (size_t)TAPE_DOUBLES * soa_ld(n);
}
__host__ __device__ inline const double* tape_aos(const double* tape, int64_t n) {
  return tape + (size_t)TAPE_DOUBLES * soa_ld(n);
}

// geo (and fq when q != null) from the SoA inputs.
hipError_t launch_pack(hipStream_t s, int n, const double* pos, const double* lam,
                       const double* q, double4* geo, double* fq);
// fp32: accumulate in FP32 (the mixed form); the moments are stored in FP64.
// lanes: 1, 2 or 4 per particle; with fp32, 0 runs the matrix-core kernel.
hipError_t launch_moments(hipStream_t s, const EvalArgs& a, int lanes, double* mom,
                          bool fp32 = false);
// Screen (list != null): status-0 particles whose equilibrated inverse has one
// of its first nscreen operator rows of 2-norm above rcut are appended to
// list[atomicAdd(count)] (count cleared by the caller).
hipError_t launch_factor(hipStream_t s, const EvalArgs& a, int ntargets, const double* mom,
                         double* gop, int32_t* status, int nscreen = 0, double rcut = 0.0,
                         int32_t* list = nullptr, int32_t* count = nullptr);
// Data form of the FP64 fit.  B_f = sum_j w_j p_j (f_j - f_i) for the last nf
// (7 or 8) fields of the packed records, into bout [nf][20][soa_ld(n)]; fpl
// (2 or 4) fields per lane.
hipError_t launch_fit_b(hipStream_t s, const EvalArgs& a, int nf, int fpl, double* bout);
// The FP64 moments (kept in LDS) and their equilibrated Cholesky in one
// pass: status, rows 1..nrows of A^{-1} (3 or 9; nf = 7 or 8 fields to
// match) and C_f = A^{-1} B_f from B in bc [nf][20][soa_ld(n)]; the
// derivative rows (coefficients 1..nrows) in place over bc as
// [nf][nrows][soa_ld(n)].  With aos (the tape's AoS block) G and all of C
// also go there.  Screen (list != null) as for launch_factor; mom
// [84][soa_ld(n)] receives the moments of the listed particles only.
hipError_t launch_moments_factor_fit(hipStream_t s, const EvalArgs& a, int nrows, double* mom,
                                     double* bc, double* aos, int32_t* status, double rcut,
                                     int32_t* list, int32_t* count);
// fp32: the neighbor loop in FP32 (the mixed form).  list, count (device):
// only the particles list[0 .. *count), outputs at their own indices.
hipError_t launch_apply_derivs(hipStream_t s, const EvalArgs& a, int lanes, const double* gop,
                               const int32_t* status, int nf, const double* fields, double* d1,
                               double* d2, bool fp32 = false, const int32_t* list = nullptr,
                               const int32_t* count = nullptr);
// Time derivatives from the operator rows gop: three rows (ideal), nine with
// the stabilisers on, the neighbor loop in FP32 (the mixed form; the FP64
// form solves for the fit coefficients instead).  list, count as for
// launch_apply_derivs (not with a.rows).
hipError_t launch_apply_rhs(hipStream_t s, const EvalArgs& a, int lanes, double gamma,
                            const Stab& sb, const double* gop, const int32_t* status, double* rhs,
                            double* dxdt, double* tape, const int32_t* list = nullptr,
                            const int32_t* count = nullptr);

}  // namespace phb
