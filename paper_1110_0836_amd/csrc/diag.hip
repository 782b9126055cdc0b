// Diagnostics of a particle set: the normalized divergence of the magnetic
// field, lambda (div B) / |B| (Sec. 3.3: the fractional field error on the
// scale of lambda), and the mean of a per-particle quantity in bins of one
// coordinate (the paper bins that diagnostic in bins one lambda wide to
// separate its coherent part from the symmetric truncation scatter).
#include <math.h>

#include <algorithm>

#include "adjoint.hpp"
#include "internal.hpp"
#include "mls.hpp"

namespace phb {
namespace {

constexpr int THREADS = 256;

// out_i = lambda_i (div B)_i / |B_i| from d1[f][3][n], the gradients of Bx,
// By, Bz; NaN where the fit failed or |B_i| = 0.
__global__ void __launch_bounds__(THREADS)
    k_divb_norm(int n, const double* __restrict__ q, const double* __restrict__ lam,
                const double* __restrict__ d1, const int32_t* __restrict__ status,
                double* __restrict__ out) {
  const int i = blockIdx.x * THREADS + threadIdx.x;
  if (i >= n) return;
  const double bx = q[4 * (int64_t)n + i], by = q[5 * (int64_t)n + i], bz = q[6 * (int64_t)n + i];
  const double bm = sqrt(bx * bx + by * by + bz * bz);
  const double div = d1[(int64_t)0 * n + i] + d1[(int64_t)4 * n + i] + d1[(int64_t)8 * n + i];
  out[i] = (status[i] == 0 && bm > 0.0) ? lam[i] * div / bm
                                        : __longlong_as_double(0x7ff8000000000000LL);
}

// Per-bin sums of the finite values; bin b = floor((x - x0) / width), taken
// in FP64 as written (the same decision as any FP64 evaluation of it).
__global__ void __launch_bounds__(THREADS)
    k_bin_accum(int n, const double* __restrict__ coord, const double* __restrict__ val,
                double x0, double width, int nbins, double* __restrict__ sum,
                unsigned long long* __restrict__ cnt) {
  for (int i = blockIdx.x * THREADS + threadIdx.x; i < n; i += gridDim.x * THREADS) {
    const double v = val[i];
    if (!(v == v)) continue;
    const double t = floor((coord[i] - x0) / width);
    if (!(t >= 0.0 && t < (double)nbins)) continue;
    const int b = (int)t;
    atomicAdd(&sum[b], v);
    atomicAdd(&cnt[b], 1ULL);
  }
}

__global__ void __launch_bounds__(THREADS)
    k_bin_finish(int nbins, const double* __restrict__ sum,
                 const unsigned long long* __restrict__ cnt, double* __restrict__ mean,
                 int64_t* __restrict__ count) {
  const int b = blockIdx.x * THREADS + threadIdx.x;
  if (b >= nbins) return;
  const unsigned long long c = cnt[b];
  mean[b] = c ? sum[b] / (double)c : __longlong_as_double(0x7ff8000000000000LL);
  if (count) count[b] = (int64_t)c;
}

constexpr int BIN_BLOCKS = 1024;

}  // namespace
}  // namespace phb

using namespace phb;

extern "C" {

int phb_divb_norm(phb_ctx* ctx, const phb_params* p, int64_t n64, const double* pos,
                  const double* lambda, const int64_t* offsets, const int32_t* idx,
                  const double* q, double* out, int32_t* status) {
  if (!ctx) return PHB_EINVAL;
  int rc;
  if ((rc = check_params(ctx, p)) || (rc = check_n(ctx, n64))) return rc;
  if (!pos || !lambda || !offsets || !idx || !q || !out || !status)
    return set_error(ctx, PHB_EINVAL, "null pointer");
  hipSetDevice(ctx->device);
  const int n = (int)n64;
  Workspace ws(ctx);
  ws.plan((size_t)9 * n * sizeof(double));
  const size_t own = ws.total;
  ws.plan(ws_bytes_derivs(n, p, false));
  if ((rc = ws.commit())) return rc;
  double* d1 = ws.take<double>((size_t)9 * n);
  {
    ArenaHold hold(ctx, own);
    if ((rc = phb_mls_derivs(ctx, p, n, pos, lambda, offsets, idx, 3, q + 4 * (size_t)n, 1, d1,
                             nullptr, status)))
      return rc;
  }
  hipLaunchKernelGGL(k_divb_norm, dim3(grid_for(n, THREADS)), dim3(THREADS), 0, ctx->stream, n, q,
                     lambda, d1, status, out);
  return hip_check(ctx, hipGetLastError(), "div B diagnostic");
}

int phb_bin_mean(phb_ctx* ctx, int64_t n64, const double* coord, const double* values,
                 double x0, double width, int32_t nbins, double* mean, int64_t* count) {
  if (!ctx) return PHB_EINVAL;
  int rc;
  if ((rc = check_n(ctx, n64))) return rc;
  if (!coord || !values || !mean || nbins <= 0 || !(width > 0.0) || !isfinite(width) ||
      !isfinite(x0))
    return set_error(ctx, PHB_EINVAL, "bin_mean: bad arguments");
  hipSetDevice(ctx->device);
  Workspace ws(ctx);
  ws.plan((size_t)nbins * sizeof(double));
  ws.plan((size_t)nbins * sizeof(unsigned long long));
  if ((rc = ws.commit())) return rc;
  double* sum = ws.take<double>(nbins);
  unsigned long long* cnt = ws.take<unsigned long long>(nbins);
  hipStream_t s = ctx->stream;
  if ((rc = hip_check(ctx, fill_f64(s, sum, 0.0, nbins), "bin clear"))) return rc;
  // 0.0 is the all-zero bit pattern: the same fill clears the counts
  if ((rc = hip_check(ctx, fill_f64(s, reinterpret_cast<double*>(cnt), 0.0, nbins), "bin clear")))
    return rc;
  const int n = (int)n64;
  const unsigned blocks = std::min<unsigned>(grid_for(n, THREADS), BIN_BLOCKS);
  hipLaunchKernelGGL(k_bin_accum, dim3(blocks), dim3(THREADS), 0, s, n, coord, values, x0, width,
                     (int)nbins, sum, cnt);
  hipLaunchKernelGGL(k_bin_finish, dim3(grid_for(nbins, THREADS)), dim3(THREADS), 0, s,
                     (int)nbins, sum, cnt, mean, count);
  return hip_check(ctx, hipGetLastError(), "bin mean");
}

}  // extern "C"
