// Launchers of the moving-least-squares and time-derivative kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"
#include "mhd.hpp"

namespace phb {

// Geometry and neighbor lists of one evaluation.
struct EvalArgs {
  int n;
  const double* pos;
  const double* lam;
  const int64_t* off;
  const int32_t* idx;
  Box box;
  double rf_ratio;
  int wkind;
};

hipError_t launch_moments(hipStream_t s, const EvalArgs& a, int lanes, double* mom);
hipError_t launch_factor(hipStream_t s, const EvalArgs& a, int ntargets, const double* mom,
                         double* gop, int32_t* status);
hipError_t launch_apply_derivs(hipStream_t s, const EvalArgs& a, int lanes, const double* gop,
                               const int32_t* status, int nf, const double* fields, double* d1,
                               double* d2);
hipError_t launch_apply_rhs(hipStream_t s, const EvalArgs& a, int lanes, double gamma,
                            const double* gop, const int32_t* status, const double* q,
                            double* rhs, double* dxdt, double* tape);

}  // namespace phb
