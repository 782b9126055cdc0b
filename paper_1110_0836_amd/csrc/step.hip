// Second-order predictor-corrector step (paper II, Sec. 2), read as Heun's
// trapezoidal scheme with the neighbor lists rebuilt at the predicted state.
#include "adjoint.hpp"
#include "internal.hpp"

#include <algorithm>
#include <climits>
#include <cstring>
#include <vector>

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

// Per-block minimum of lambda_i / (c_f,i cmul) over non-frozen particles,
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

// ---- individual power-of-two time steps ------------------------------------
// Times are integer ticks of dt_max / 2^kmax; a particle on level k has a step
// of T >> k ticks, T = 2^kmax, and starts its current step at t0.

// flag[i] = 1 for the non-frozen particles ending a step at tick (all: every
// non-frozen particle).
__global__ void __launch_bounds__(THREADS)
    k_blk_flags(int n, const int32_t* __restrict__ frozen, const int64_t* __restrict__ t0,
                const int32_t* __restrict__ lev, int64_t T, int64_t tick, int all,
                int32_t* __restrict__ flag) {
  const int i = blockIdx.x * THREADS + threadIdx.x;
  if (i >= n) return;
  const bool fz = frozen && frozen[i];
  flag[i] = (!fz && (all || t0[i] + (T >> lev[i]) == tick)) ? 1 : 0;
}

// rows[pos[i]] = i for flagged particles; rowpos[i] = their row or -1.
__global__ void __launch_bounds__(THREADS)
    k_blk_scatter(int n, const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                  int32_t* __restrict__ rows, int32_t* __restrict__ rowpos) {
  const int i = blockIdx.x * THREADS + threadIdx.x;
  if (i >= n) return;
  if (flag[i]) rows[pos[i]] = i;
  rowpos[i] = flag[i] ? pos[i] : -1;
}

// Per-block minimum of the next step end over non-frozen particles.
__global__ void __launch_bounds__(THREADS)
    k_blk_next(int n, const int32_t* __restrict__ frozen, const int64_t* __restrict__ t0,
               const int32_t* __restrict__ lev, int64_t T, int64_t* __restrict__ part) {
  __shared__ int64_t sm[THREADS];
  int64_t m = INT64_MAX;
  for (int i = blockIdx.x * THREADS + threadIdx.x; i < n; i += gridDim.x * THREADS) {
    if (frozen && frozen[i]) continue;
    const int64_t e = t0[i] + (T >> lev[i]);
    m = e < m ? e : m;
  }
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = THREADS / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w && sm[threadIdx.x + w] < sm[threadIdx.x])
      sm[threadIdx.x] = sm[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__device__ __forceinline__ double wrap_axis(double v, const Box& box, int a, int32_t* flag) {
  if (box.periodic[a]) {
    if (v >= box.L[a]) v -= box.L[a];
    if (v < 0.0) v += box.L[a];
  } else if (!(v >= 0.0 && v < box.L[a])) {
    flag[0] = 1;
  }
  return v;
}

// Every particle's state predicted linearly to tick from its step start.
__global__ void __launch_bounds__(THREADS)
    k_blk_predict(int n, Box box, const double* __restrict__ x0, const double* __restrict__ q0,
                  const double* __restrict__ v0, const double* __restrict__ f0,
                  const int64_t* __restrict__ t0, int64_t tick, double dtick,
                  double* __restrict__ xp, double* __restrict__ qp, int32_t* __restrict__ flag) {
  const int i = blockIdx.x * THREADS + threadIdx.x;
  if (i >= n) return;
  const double tau = (double)(tick - t0[i]) * dtick;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int64_t k = (int64_t)a * n + i;
    xp[k] = wrap_axis(x0[k] + tau * v0[k], box, a, flag);
  }
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int64_t k = (int64_t)c * n + i;
    qp[k] = q0[k] + tau * f0[k];
  }
}

// Heun's corrector for the rows (f, v: their derivatives at the predicted
// state, per row); the corrected state becomes the rows' step start.
__global__ void __launch_bounds__(THREADS)
    k_blk_correct(int m, const int32_t* __restrict__ rows, int n, Box box, int64_t T,
                  const int32_t* __restrict__ lev, double dtick, int64_t tick,
                  const double* __restrict__ f, const double* __restrict__ v,
                  const int32_t* __restrict__ st, const double* __restrict__ f0,
                  const double* __restrict__ v0, double* __restrict__ x0,
                  double* __restrict__ q0, double* __restrict__ xp, double* __restrict__ qp,
                  int64_t* __restrict__ t0, int32_t* __restrict__ stmax,
                  int32_t* __restrict__ flag) {
  const int r = blockIdx.x * THREADS + threadIdx.x;
  if (r >= m) return;
  const int i = rows[r];
  const double dt = (double)(T >> lev[i]) * dtick;
  const double c1 = 0.5 * dt;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    const int64_t k = (int64_t)c * n + i;
    const double y = q0[k] + c1 * (f0[k] + f[(int64_t)c * m + r]);
    q0[k] = y;
    qp[k] = y;
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const int64_t k = (int64_t)a * n + i;
    const double y = wrap_axis(x0[k] + c1 * (v0[k] + v[(int64_t)a * m + r]), box, a, flag);
    x0[k] = y;
    xp[k] = y;
  }
  t0[i] = tick;
  if (st[r] > stmax[i]) stmax[i] = st[r];
}

// The rows' derivatives at their step start.
__global__ void __launch_bounds__(THREADS)
    k_blk_store(int m, const int32_t* __restrict__ rows, int n, const double* __restrict__ f,
                const double* __restrict__ v, const int32_t* __restrict__ st,
                double* __restrict__ f0, double* __restrict__ v0, int32_t* __restrict__ stmax) {
  const int r = blockIdx.x * THREADS + threadIdx.x;
  if (r >= m) return;
  const int i = rows[r];
#pragma unroll
  for (int c = 0; c < 8; ++c) f0[(int64_t)c * n + i] = f[(int64_t)c * m + r];
#pragma unroll
  for (int a = 0; a < 3; ++a) v0[(int64_t)a * n + i] = v[(int64_t)a * m + r];
  if (st[r] > stmax[i]) stmax[i] = st[r];
}

// Courant level of each row: the smallest k in [0, kmax] whose step
// dt_max / 2^k is at most cfl lambda / (c_f cmul).
__global__ void __launch_bounds__(THREADS)
    k_blk_courant(int m, const int32_t* __restrict__ rows, int n, const double* __restrict__ q,
                  const double* __restrict__ lam, double gamma, double cmul, double cfl,
                  double dt_max, int kmax, int32_t* __restrict__ kn) {
  const int r = blockIdx.x * THREADS + threadIdx.x;
  if (r >= m) return;
  const int i = rows[r];
  const double b2 = q[4 * (int64_t)n + i] * q[4 * (int64_t)n + i] +
                    q[5 * (int64_t)n + i] * q[5 * (int64_t)n + i] +
                    q[6 * (int64_t)n + i] * q[6 * (int64_t)n + i];
  const double pr = (gamma - 1.0) * q[7 * (int64_t)n + i];
  const double cf = sqrt((gamma * pr + b2) / q[i]);
  const double dtc = cfl * (lam[i] / (cf * cmul));
  int k = 0;
  while (k < kmax && !(ldexp(dt_max, -k) <= dtc)) ++k;
  kn[r] = k;
}

// One sweep of the limiter k_r >= k_j - 1 over each row's non-frozen
// neighbors (rows' new levels, the others' current ones).  Levels only rise,
// so sweeps repeated until none changes reach the same fixed point in any
// order.
__global__ void __launch_bounds__(THREADS)
    k_blk_limit(int m, const int32_t* __restrict__ rows, const int64_t* __restrict__ off,
                const int32_t* __restrict__ idx, const int32_t* __restrict__ frozen,
                const int32_t* __restrict__ lev, const int32_t* __restrict__ rowpos,
                int32_t* __restrict__ kn, int32_t* __restrict__ changed) {
  const int r = blockIdx.x * THREADS + threadIdx.x;
  if (r >= m) return;
  const int i = rows[r];
  int kr = kn[r];
  const int k_in = kr;
  for (int64_t e = off[r]; e < off[r + 1]; ++e) {
    const int j = idx[e];
    if (j == i || (frozen && frozen[j])) continue;
    const int pj = rowpos[j];
    const int kj = pj >= 0 ? kn[pj] : lev[j];
    if (kj - 1 > kr) kr = kj - 1;
  }
  if (kr > k_in) {
    kn[r] = kr;
    changed[0] = 1;
  }
}

__global__ void __launch_bounds__(THREADS)
    k_blk_set_levels(int m, const int32_t* __restrict__ rows, const int32_t* __restrict__ kn,
                     int ksync, int32_t* __restrict__ lev) {
  const int r = blockIdx.x * THREADS + threadIdx.x;
  if (r >= m) return;
  lev[rows[r]] = kn[r] > ksync ? kn[r] : ksync;
}

__global__ void __launch_bounds__(THREADS)
    k_blk_finish(int n, const int32_t* __restrict__ frozen, const int32_t* __restrict__ stmax,
                 const int32_t* __restrict__ lev, int32_t* __restrict__ status,
                 int32_t* __restrict__ level) {
  const int i = blockIdx.x * THREADS + threadIdx.x;
  if (i >= n) return;
  status[i] = (frozen && frozen[i]) ? 0 : stmax[i];
  if (level) level[i] = lev[i];
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

namespace phb {

// The block scheme of orc_evolve_blocks (see its readings): predict every
// particle to the next step end, evaluate the particles ending a step there,
// correct them, evaluate them again at the corrected state, give them new
// levels; repeat until nblocks periods of dt_max.
int evolve_blocks(phb_ctx* ctx, const phb_params* p, int n, double* pos, double* q,
                  const double* lambda, const int32_t* frozen, double dt_max, int nblocks,
                  double cfl, int kmax, int64_t* offsets, int32_t* idx, int64_t idx_capacity,
                  int32_t* status, int32_t* level, int64_t* stats) {
  const Box box = make_box(p);
  hipStream_t s = ctx->stream;
  const double cmul = 1.0 + 2.0 * (p->visc_grid + p->visc_adapt + p->divb_diff);
  const int64_t T = int64_t(1) << kmax;
  const double dtick = ldexp(dt_max, -kmax);
  const size_t nd = (size_t)n * sizeof(double), ni = (size_t)n * sizeof(int32_t);
  Workspace ws(ctx);
  for (int c : {3, 8, 8, 3, 8, 3}) ws.plan(c * nd);  // xp qp F0 V0 f v
  for (int c = 0; c < 6; ++c) ws.plan(ni);            // st stmax lev kn rows rowpos
  ws.plan(ni + sizeof(int32_t));                      // flags
  ws.plan(ni + sizeof(int32_t));                      // their scan
  ws.plan((size_t)scan_tmp_elems(n) * sizeof(int32_t));
  ws.plan((size_t)n * sizeof(int64_t));               // t0
  ws.plan(DT_BLOCKS * sizeof(int64_t));               // next-tick partials
  ws.plan(64 * sizeof(int32_t));                      // flags for the host
  const size_t own = ws.total;
  ws.plan(std::max(ws_bytes_neighbors(n, idx_capacity), ws_bytes_rhs(n, p)));
  int rc;
  if ((rc = ws.commit())) return rc;
  double* xp = ws.take<double>(3 * (size_t)n);
  double* qp = ws.take<double>(8 * (size_t)n);
  double* F0 = ws.take<double>(8 * (size_t)n);
  double* V0 = ws.take<double>(3 * (size_t)n);
  double* f = ws.take<double>(8 * (size_t)n);
  double* v = ws.take<double>(3 * (size_t)n);
  int32_t* st = ws.take<int32_t>(n);
  int32_t* stmax = ws.take<int32_t>(n);
  int32_t* lev = ws.take<int32_t>(n);
  int32_t* kn = ws.take<int32_t>(n);
  int32_t* rows = ws.take<int32_t>(n);
  int32_t* rowpos = ws.take<int32_t>(n);
  int32_t* flag = ws.take<int32_t>((size_t)n + 1);
  int32_t* fpos = ws.take<int32_t>((size_t)n + 1);
  int32_t* ftmp = ws.take<int32_t>(scan_tmp_elems(n));
  int64_t* t0 = ws.take<int64_t>(n);
  int64_t* part = ws.take<int64_t>(DT_BLOCKS);
  int32_t* hflag = ws.take<int32_t>(64);
  ArenaHold hold(ctx, own);
  const unsigned gn = grid_for(n, THREADS);
  int64_t events = 0, evals = 0;

  if ((rc = ensure_host(ctx, DT_BLOCKS * sizeof(int64_t)))) return rc;
  auto read_back = [&](void* dst, const void* src, size_t bytes) -> int {
    hipError_t e = hipMemcpyAsync(ctx->host, src, bytes, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess) std::memcpy(dst, ctx->host, bytes);
    return hip_check(ctx, e, "block-step read-back");
  };
  // rows <- the flagged particles; returns their count in *m
  auto compact = [&](int64_t tick, int all, int* m) -> int {
    hipLaunchKernelGGL(k_blk_flags, dim3(gn), dim3(THREADS), 0, s, n, frozen, t0, lev, T, tick,
                       all, flag);
    int r2;
    if ((r2 = hip_check(ctx, hipGetLastError(), "active flags"))) return r2;
    if ((r2 = hip_check(ctx, exclusive_scan_i32_to_i32(s, flag, n, fpos, ftmp), "active scan")))
      return r2;
    hipLaunchKernelGGL(k_blk_scatter, dim3(gn), dim3(THREADS), 0, s, n, flag, fpos, rows,
                       rowpos);
    if ((r2 = hip_check(ctx, hipGetLastError(), "active scatter"))) return r2;
    int32_t cnt = 0;
    if ((r2 = read_back(&cnt, fpos + n, sizeof(int32_t)))) return r2;
    *m = cnt;
    return PHB_OK;
  };
  // f, v, st <- the rows' time derivatives at (xp, qp)
  auto eval_rows = [&](int m) -> int {
    int64_t nnz = 0;
    int r2;
    if ((r2 = neighbors_rows_unchecked(ctx, p, n, xp, lambda, m, rows, offsets, idx,
                                       idx_capacity, &nnz)))
      return r2;
    EvalArgs a;
    if ((r2 = eval_args(ctx, p, n, xp, lambda, offsets, idx, &a))) return r2;
    a.n_all = n;
    a.n = m;
    a.rows = rows;
    evals += m;
    return eval_rhs(ctx, a, p, qp, f, v, st, nullptr);
  };
  auto set_levels = [&](int m, int ksync) -> int {
    const unsigned gm = grid_for(m, THREADS);
    hipLaunchKernelGGL(k_blk_courant, dim3(gm), dim3(THREADS), 0, s, m, rows, n, q, lambda,
                       p->gamma, cmul, cfl, dt_max, kmax, kn);
    int r2;
    if ((r2 = hip_check(ctx, hipGetLastError(), "levels"))) return r2;
    for (int sweep = 0; sweep <= kmax + 1; ++sweep) {
      if ((r2 = hip_check(ctx, fill_i32(s, hflag, 0, 1), "limiter flag"))) return r2;
      hipLaunchKernelGGL(k_blk_limit, dim3(gm), dim3(THREADS), 0, s, m, rows, offsets, idx,
                         frozen, lev, rowpos, kn, hflag);
      if ((r2 = hip_check(ctx, hipGetLastError(), "limiter"))) return r2;
      int32_t changed = 0;
      if ((r2 = read_back(&changed, hflag, sizeof(int32_t)))) return r2;
      if (!changed) break;
    }
    hipLaunchKernelGGL(k_blk_set_levels, dim3(gm), dim3(THREADS), 0, s, m, rows, kn, ksync, lev);
    return hip_check(ctx, hipGetLastError(), "set levels");
  };
  auto check_left = [&]() -> int {
    int32_t left = 0;
    int r2;
    if ((r2 = read_back(&left, hflag + 1, sizeof(int32_t)))) return r2;
    if (left) return set_error(ctx, PHB_EINVAL, "a position left [0, L) on an open axis");
    return PHB_OK;
  };

  // zero state: levels, step starts, derivatives, statuses (0.0 and int 0
  // share the all-zero bit pattern)
  if ((rc = hip_check(ctx, fill_i32(s, lev, 0, n), "clear"))) return rc;
  if ((rc = hip_check(ctx, fill_i32(s, stmax, 0, n), "clear"))) return rc;
  if ((rc = hip_check(ctx, fill_f64(s, reinterpret_cast<double*>(t0), 0.0, n), "clear")))
    return rc;
  if ((rc = hip_check(ctx, fill_f64(s, F0, 0.0, 8 * (int64_t)n), "clear"))) return rc;
  if ((rc = hip_check(ctx, fill_f64(s, V0, 0.0, 3 * (int64_t)n), "clear"))) return rc;
  if ((rc = hip_check(ctx, hipMemcpyAsync(xp, pos, 3 * nd, hipMemcpyDeviceToDevice, s), "copy")))
    return rc;
  if ((rc = hip_check(ctx, hipMemcpyAsync(qp, q, 8 * nd, hipMemcpyDeviceToDevice, s), "copy")))
    return rc;
  int m = 0;
  if ((rc = compact(0, 1, &m))) return rc;
  if (m > 0 && nblocks > 0) {
    // time 0: every particle's derivative and level
    if ((rc = eval_rows(m))) return rc;
    hipLaunchKernelGGL(k_blk_store, dim3(grid_for(m, THREADS)), dim3(THREADS), 0, s, m, rows, n,
                       f, v, st, F0, V0, stmax);
    if ((rc = hip_check(ctx, hipGetLastError(), "store"))) return rc;
    if ((rc = set_levels(m, 0))) return rc;
    const int64_t tick_end = (int64_t)nblocks * T;
    for (;;) {
      hipLaunchKernelGGL(k_blk_next, dim3(DT_BLOCKS), dim3(THREADS), 0, s, n, frozen, t0, lev, T,
                         part);
      if ((rc = hip_check(ctx, hipGetLastError(), "next step end"))) return rc;
      std::vector<int64_t> hp(DT_BLOCKS);
      if ((rc = read_back(hp.data(), part, DT_BLOCKS * sizeof(int64_t)))) return rc;
      const int64_t tick = *std::min_element(hp.begin(), hp.end());
      if ((rc = compact(tick, 0, &m))) return rc;
      ++events;
      if ((rc = hip_check(ctx, fill_i32(s, hflag + 1, 0, 1), "flag clear"))) return rc;
      // a predicted position off an open axis fails the list build's input
      // check; the flag is read once, after the corrector
      hipLaunchKernelGGL(k_blk_predict, dim3(gn), dim3(THREADS), 0, s, n, box, pos, q, V0, F0, t0,
                         tick, dtick, xp, qp, hflag + 1);
      if ((rc = hip_check(ctx, hipGetLastError(), "predict"))) return rc;
      if ((rc = eval_rows(m))) return rc;
      hipLaunchKernelGGL(k_blk_correct, dim3(grid_for(m, THREADS)), dim3(THREADS), 0, s, m, rows,
                         n, box, T, lev, dtick, tick, f, v, st, F0, V0, pos, q, xp, qp, t0, stmax,
                         hflag + 1);
      if ((rc = hip_check(ctx, hipGetLastError(), "correct"))) return rc;
      if ((rc = check_left())) return rc;
      if (tick >= tick_end) break;
      if ((rc = eval_rows(m))) return rc;
      hipLaunchKernelGGL(k_blk_store, dim3(grid_for(m, THREADS)), dim3(THREADS), 0, s, m, rows,
                         n, f, v, st, F0, V0, stmax);
      if ((rc = hip_check(ctx, hipGetLastError(), "store"))) return rc;
      int tz = 0;
      while (tz < kmax && ((tick >> tz) & 1) == 0) ++tz;
      if ((rc = set_levels(m, kmax - tz))) return rc;
    }
  }
  hipLaunchKernelGGL(k_blk_finish, dim3(gn), dim3(THREADS), 0, s, n, frozen, stmax, lev, status,
                     level);
  if ((rc = hip_check(ctx, hipGetLastError(), "finish"))) return rc;
  if (stats) {
    stats[0] = events;
    stats[1] = evals;
  }
  return PHB_OK;
}

}  // namespace phb
