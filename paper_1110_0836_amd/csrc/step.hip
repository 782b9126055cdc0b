// Second-order predictor-corrector step (paper II, Sec. 2), read as Heun's
// trapezoidal scheme with the neighbor lists rebuilt at the predicted state.
#include "adjoint.hpp"
#include "internal.hpp"

#include <algorithm>

namespace phb {
namespace {

constexpr int THREADS = 256;

// y_out = y0 + c1 * f0, or y0 + c1 * (f0 + f1) when f1 != null; positions are
// wrapped on periodic axes and flagged when they leave [0, L) on an open axis.
// Frozen particles (frozen[i] != 0) keep y0: their time derivatives are zero.
__global__ void __launch_bounds__(THREADS)
    k_axpy_state(int n, Box box, const double* __restrict__ x0, const double* __restrict__ q0,
                 const double* __restrict__ v0, const double* __restrict__ r0,
                 const double* __restrict__ v1, const double* __restrict__ r1, double c1,
                 const int32_t* __restrict__ frozen, double* __restrict__ xo,
                 double* __restrict__ qo, int32_t* __restrict__ flag) {
  const int i = blockIdx.x * THREADS + threadIdx.x;
  if (i >= n) return;
  if (frozen && frozen[i]) {
#pragma unroll
    for (int a = 0; a < 3; ++a) xo[(int64_t)a * n + i] = x0[(int64_t)a * n + i];
#pragma unroll
    for (int f = 0; f < 8; ++f) qo[(int64_t)f * n + i] = q0[(int64_t)f * n + i];
    return;
  }
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
}

// out = max(a, b) (and the previous out when accumulate), 0 for frozen particles.
__global__ void __launch_bounds__(THREADS)
    k_max_status(int n, const int32_t* __restrict__ a, const int32_t* __restrict__ b,
                 const int32_t* __restrict__ frozen, int accumulate, int32_t* __restrict__ out) {
  const int i = blockIdx.x * THREADS + threadIdx.x;
  if (i >= n) return;
  int v = a[i] > b[i] ? a[i] : b[i];
  if (accumulate && out[i] > v) v = out[i];
  out[i] = (frozen && frozen[i]) ? 0 : v;
}

// Per-block minimum of lambda_i / (|V_i| + c_f,i) over non-frozen particles,
// c_f = sqrt((gamma P + |B|^2) / rho), P = (gamma - 1) sigma.
constexpr int DT_BLOCKS = 512;
__global__ void __launch_bounds__(THREADS)
    k_courant(int n, const double* __restrict__ q, const double* __restrict__ lam,
              const int32_t* __restrict__ frozen, double gamma, double cmul,
              double* __restrict__ part) {
  __shared__ double sm[THREADS];
  double m = 1e300;
  for (int i = blockIdx.x * THREADS + threadIdx.x; i < n; i += gridDim.x * THREADS) {
    if (frozen && frozen[i]) continue;
    const double rho = q[i];
    const double bx = q[4 * (int64_t)n + i], by = q[5 * (int64_t)n + i],
                 bz = q[6 * (int64_t)n + i];
    const double pr = (gamma - 1.0) * q[7 * (int64_t)n + i];
    const double cf = sqrt((gamma * pr + bx * bx + by * by + bz * bz) / rho);
    const double t = lam[i] / (cf * cmul);
    m = fmin(m, t);
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

}  // namespace

int pc_step(phb_ctx* ctx, const phb_params* p, int n, double dt, double* pos, double* q,
            const double* lambda, const int32_t* frozen, int64_t* offsets, int32_t* idx,
            int64_t idx_capacity, int64_t* nnz_out, int32_t* status, int accumulate) {
  const Box box = make_box(p);
  Workspace ws(ctx);
  const size_t n3 = 3 * (size_t)n, n8 = 8 * (size_t)n;
  for (size_t k : {n3, n8, n3, n8, n3, n8}) ws.plan(k * sizeof(double));
  ws.plan((size_t)n * sizeof(int32_t));
  ws.plan((size_t)n * sizeof(int32_t));
  ws.plan(64 * sizeof(int32_t));
  const size_t own = ws.total;
  ws.plan(std::max(ws_bytes_neighbors(n, idx_capacity), ws_bytes_rhs(n, p)));
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
                     r0, nullptr, nullptr, dt, frozen, xs, qs, flag);
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
                     r0, v1, r1, 0.5 * dt, frozen, pos, q, flag);
  hipLaunchKernelGGL(k_max_status, dim3(grid), dim3(THREADS), 0, ctx->stream, n, s0, s1, frozen,
                     accumulate, status);
  if ((rc = hip_check(ctx, hipGetLastError(), "corrector"))) return rc;
  if ((rc = read_flag(&left))) return rc;
  if (left) return set_error(ctx, PHB_EINVAL, "a corrected position left [0, L) on an open axis");
  return PHB_OK;
}

int courant_dt(phb_ctx* ctx, const phb_params* p, int n, const double* q, const double* lambda,
               const int32_t* frozen, double cfl, double* dt_out) {
  Workspace ws(ctx);
  ws.plan(DT_BLOCKS * sizeof(double));
  int rc;
  if ((rc = ws.commit())) return rc;
  double* part = ws.take<double>(DT_BLOCKS);
  // the stabilisers' diffusivities (at most lambda c_f times their
  // coefficients) enter as the speed 2 (zeta + eta) / lambda
  const double cmul = 1.0 + 2.0 * (p->visc_grid + p->visc_adapt + p->divb_diff);
  hipLaunchKernelGGL(k_courant, dim3(DT_BLOCKS), dim3(THREADS), 0, ctx->stream, n, q, lambda,
                     frozen, p->gamma, cmul, part);
  if ((rc = hip_check(ctx, hipGetLastError(), "courant"))) return rc;
  double* h = nullptr;
  if (hipHostMalloc((void**)&h, DT_BLOCKS * sizeof(double)) != hipSuccess)
    return set_error(ctx, PHB_EHIP, "pinned allocation");
  hipError_t e = hipMemcpyAsync(h, part, DT_BLOCKS * sizeof(double), hipMemcpyDeviceToHost,
                                ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  double m = 1e300;
  for (int b = 0; b < DT_BLOCKS; ++b) m = std::min(m, h[b]);
  hipHostFree(h);
  if ((rc = hip_check(ctx, e, "courant read-back"))) return rc;
  if (!(m < 1e300)) return set_error(ctx, PHB_EINVAL, "no particle to time-step");
  *dt_out = cfl * m;
  return PHB_OK;
}

}  // namespace phb
