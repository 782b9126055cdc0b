// Second-order predictor-corrector step (paper II, Sec. 2), read as Heun's
// trapezoidal scheme with the neighbor lists rebuilt at the predicted state.
#include "adjoint.hpp"
#include "internal.hpp"

#include <algorithm>

namespace phb {
namespace {

constexpr int THREADS = 256;

// y_out = y0 + c1 * f0 (+ c2 * f1 when f1 != null); positions are wrapped on
// periodic axes and flagged when they leave [0, L) on an open axis.
__global__ void __launch_bounds__(THREADS)
    k_axpy_state(int n, Box box, const double* __restrict__ x0, const double* __restrict__ q0,
                 const double* __restrict__ v0, const double* __restrict__ r0,
                 const double* __restrict__ v1, const double* __restrict__ r1, double c1,
                 double c2, double* __restrict__ xo, double* __restrict__ qo,
                 int32_t* __restrict__ flag) {
  const int i = blockIdx.x * THREADS + threadIdx.x;
  if (i >= n) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int64_t k = (int64_t)a * n + i;
    double v = x0[k] + c1 * v0[k];
    if (v1) v = x0[k] + c1 * (v0[k] + v1[k]);
    if (box.periodic[a]) {
      if (v >= box.L[a]) v -= box.L[a];
      if (v < 0.0) v += box.L[a];
    } else if (!(v >= 0.0 && v < box.L[a])) {
      flag[0] = 1;
    }
    xo[k] = v;
  }
#pragma unroll
  for (int f = 0; f < 8; ++f) {
    const int64_t k = (int64_t)f * n + i;
    qo[k] = r1 ? q0[k] + c1 * (r0[k] + r1[k]) : q0[k] + c1 * r0[k];
  }
  (void)c2;
}

__global__ void __launch_bounds__(THREADS)
    k_max_status(int n, const int32_t* __restrict__ a, const int32_t* __restrict__ b,
                 int32_t* __restrict__ out) {
  const int i = blockIdx.x * THREADS + threadIdx.x;
  if (i < n) out[i] = a[i] > b[i] ? a[i] : b[i];
}

}  // namespace

int pc_step(phb_ctx* ctx, const phb_params* p, int n, double dt, double* pos, double* q,
            const double* lambda, int64_t* offsets, int32_t* idx, int64_t idx_capacity,
            int64_t* nnz_out, int32_t* status) {
  const Box box = make_box(p);
  Workspace ws(ctx);
  const size_t n3 = 3 * (size_t)n, n8 = 8 * (size_t)n;
  for (size_t k : {n3, n8, n3, n8, n3, n8}) ws.plan(k * sizeof(double));
  ws.plan((size_t)n * sizeof(int32_t));
  ws.plan((size_t)n * sizeof(int32_t));
  ws.plan(64 * sizeof(int32_t));
  const size_t own = ws.total;
  ws.plan(std::max(ws_bytes_neighbors(n, idx_capacity), ws_bytes_rhs(n, p->precision)));
  int rc;
  if ((rc = ws.commit())) return rc;
  double* xs = ws.take<double>(n3);
  double* qs = ws.take<double>(n8);
  double* v0 = ws.take<double>(n3);
  double* r0 = ws.take<double>(n8);
  double* v1 = ws.take<double>(n3);
  double* r1 = ws.take<double>(n8);
  int32_t* s0 = ws.take<int32_t>(n);
  int32_t* s1 = ws.take<int32_t>(n);
  int32_t* flag = ws.take<int32_t>(64);
  int32_t* hflag = nullptr;
  ArenaHold hold(ctx, own);

  auto read_flag = [&](int32_t* out) -> int {
    int32_t* h = nullptr;
    if (hipHostMalloc((void**)&h, sizeof(int32_t)) != hipSuccess)
      return set_error(ctx, PHB_EHIP, "pinned flag allocation");
    hipError_t e = hipMemcpyAsync(h, flag, sizeof(int32_t), hipMemcpyDeviceToHost, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    *out = *h;
    hipHostFree(h);
    return hip_check(ctx, e, "step flag read-back");
  };
  (void)hflag;
  const unsigned grid = grid_for(n, THREADS);

  // F(y)
  if ((rc = phb_neighbors_build(ctx, p, n, pos, lambda, offsets, idx, idx_capacity, nnz_out)))
    return rc;
  if ((rc = phb_mhd_rhs(ctx, p, n, pos, lambda, offsets, idx, q, r0, v0, s0, nullptr))) return rc;
  // predictor
  if ((rc = hip_check(ctx, fill_i32(ctx->stream, flag, 0, 1), "flag clear"))) return rc;
  hipLaunchKernelGGL(k_axpy_state, dim3(grid), dim3(THREADS), 0, ctx->stream, n, box, pos, q, v0,
                     r0, nullptr, nullptr, dt, 0.0, xs, qs, flag);
  if ((rc = hip_check(ctx, hipGetLastError(), "predictor"))) return rc;
  int32_t left = 0;
  if ((rc = read_flag(&left))) return rc;
  if (left) return set_error(ctx, PHB_EINVAL, "a predicted position left [0, L) on an open axis");
  // F(y*)
  if ((rc = phb_neighbors_build(ctx, p, n, xs, lambda, offsets, idx, idx_capacity, nnz_out)))
    return rc;
  if ((rc = phb_mhd_rhs(ctx, p, n, xs, lambda, offsets, idx, qs, r1, v1, s1, nullptr))) return rc;
  // corrector, in place
  hipLaunchKernelGGL(k_axpy_state, dim3(grid), dim3(THREADS), 0, ctx->stream, n, box, pos, q, v0,
                     r0, v1, r1, 0.5 * dt, 0.0, pos, q, flag);
  hipLaunchKernelGGL(k_max_status, dim3(grid), dim3(THREADS), 0, ctx->stream, n, s0, s1, status);
  if ((rc = hip_check(ctx, hipGetLastError(), "corrector"))) return rc;
  if ((rc = read_flag(&left))) return rc;
  if (left) return set_error(ctx, PHB_EINVAL, "a corrected position left [0, L) on an open axis");
  return PHB_OK;
}

}  // namespace phb
