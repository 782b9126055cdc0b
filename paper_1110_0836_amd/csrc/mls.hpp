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

// Tape of the forward evaluation, per particle (SoA, n entries each):
// 21 gradients (V, B, sigma x 3), the status, grad rho, grad div V and
// grad div B (written only with the stabilisers on), then the 84 moments,
// FP64-assembled in both forms.
constexpr int TAPE_STATUS = 21;
constexpr int TAPE_GRHO = 22;
constexpr int TAPE_GDV = 25;
constexpr int TAPE_GDB = 28;
constexpr int TAPE_MOM = 31;
constexpr int TAPE_DOUBLES = TAPE_MOM + NMOM;

// geo (and fq when q != null) from the SoA inputs.
hipError_t launch_pack(hipStream_t s, int n, const double* pos, const double* lam,
                       const double* q, double4* geo, double* fq);
// fp32: accumulate in FP32 (the mixed form); the moments are stored in FP64.
hipError_t launch_moments(hipStream_t s, const EvalArgs& a, int lanes, double* mom,
                          bool fp32 = false);
// Screen (list != null): status-0 particles whose equilibrated inverse has one
// of its first nscreen operator rows of 2-norm above rcut are appended to
// list[atomicAdd(count)] (count cleared by the caller).
hipError_t launch_factor(hipStream_t s, const EvalArgs& a, int ntargets, const double* mom,
                         double* gop, int32_t* status, int nscreen = 0, double rcut = 0.0,
                         int32_t* list = nullptr, int32_t* count = nullptr);
// X = A^{-1} R for nr (1..8) right-hand sides given as SoA [nr][20][n].
hipError_t launch_factor_solve(hipStream_t s, int n, const int64_t* off, int nr,
                               const double* mom, const double* rhs, double* x, int32_t* status,
                               int fit);
// fp32: the neighbor loop in FP32 (the mixed form).  list, count (device):
// only the particles list[0 .. *count), outputs at their own indices.
hipError_t launch_apply_derivs(hipStream_t s, const EvalArgs& a, int lanes, const double* gop,
                               const int32_t* status, int nf, const double* fields, double* d1,
                               double* d2, bool fp32 = false, const int32_t* list = nullptr,
                               const int32_t* count = nullptr);
// Time derivatives from the operator rows gop: three rows (ideal), nine with
// the stabilisers on.  fp32: the neighbor loop in FP32 (the mixed form).
// list, count as for launch_apply_derivs (not with a.rows).
hipError_t launch_apply_rhs(hipStream_t s, const EvalArgs& a, int lanes, double gamma,
                            const Stab& sb, const double* gop, const int32_t* status, double* rhs,
                            double* dxdt, double* tape, bool fp32 = false,
                            const int32_t* list = nullptr, const int32_t* count = nullptr);

}  // namespace phb
