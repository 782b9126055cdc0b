// Reverse mode of the MLS / ideal-MHD time derivatives with the neighbor
// lists held fixed.
//
// Forward, per particle i (operator form): A = sum_j w_j p_j p_j^T,
// G = E A^{-1} (E picks the x, y, z monomials), grad f = (1/lambda) sum_j
// w_j (G p_j) (f_j - f_i), then the pointwise right-hand side.
//
// Reverse, per particle i:
//   1. pointwise adjoint of the right-hand side: qbar_i (direct part) and
//      Ubar = grad_bar / lambda  (3 x 7, coefficient space);
//   2. Y = sum_j w_j p_j (Ubar df_j)^T  (20 x 3);
//   3. factor A again, G as in the forward and K = (A^{-1} Y)^T  (3 x 20);
//      with C = A^{-1} B the fit coefficients, K = Ubar C^T, so the adjoint
//      of A is  Abar = -G^T K  and of B is  Bbar = G^T Ubar;
//   4. for each neighbor: a = G p, h = Ubar df, b = h - K p,
//        wbar  = a . b,
//        pbar  = w (G^T b - K^T a),  xibar = (dp/dxi)^T pbar,
//        dfbar = w Ubar^T a,
//        dbar  = xibar / lambda + wbar (dw/dq) 2 d / r_f^2,
//      and the pair contributes +dfbar, +dbar to j and -dfbar, -dbar to i;
//   5. every particle sums the pair records addressed to it (the transposed
//      lists), in a fixed order, plus its own terms.  No atomics.
#include <type_traits>

#include "adjoint.hpp"
#include "mhd.hpp"
#include "neighbors.hpp"

namespace phb {

template <int B, int E, class F>
__device__ __forceinline__ void static_for_a(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for_a<B + 1, E>(f);
  }
}

namespace {

constexpr int THREADS = 256;
constexpr int REC = 10;  // doubles per pair record: dfbar (7), dbar (3)

struct EntryTableA {
  unsigned char v[NBASIS * NBASIS];
};
constexpr EntryTableA make_entry_table_a() {
  EntryTableA t{};
  for (int r = 0; r < NBASIS; ++r)
    for (int c = 0; c < NBASIS; ++c) t.v[r * NBASIS + c] = (unsigned char)entry_moment(r, c);
  return t;
}
__constant__ EntryTableA c_entry_a = make_entry_table_a();

// Pointwise adjoint of particle i; returns Ubar (coefficient space) and adds
// the direct part to qb.  Status != 0: no gradient through rhs.
__device__ __forceinline__ void pointwise_adjoint(int n, int i, const double* __restrict__ q,
                                                  const double* __restrict__ tape,
                                                  const double* __restrict__ rhs_bar,
                                                  const double* __restrict__ dxdt_bar,
                                                  double gamma, double inv_lam, int st,
                                                  double (&qi)[8], double (&ub)[7][3],
                                                  double (&qb)[8]) {
#pragma unroll
  for (int f = 0; f < 8; ++f) {
    qi[f] = q[(int64_t)f * n + i];
    qb[f] = 0.0;
  }
  if (dxdt_bar) {
#pragma unroll
    for (int a = 0; a < 3; ++a) qb[1 + a] += dxdt_bar[(int64_t)a * n + i];
  }
#pragma unroll
  for (int f = 0; f < 7; ++f)
#pragma unroll
    for (int t = 0; t < 3; ++t) ub[f][t] = 0.0;
  if (st != 0) return;
  double grad[7][3], ob[8];
#pragma unroll
  for (int f = 0; f < 7; ++f)
#pragma unroll
    for (int t = 0; t < 3; ++t) grad[f][t] = tape[((int64_t)f * 3 + t) * n + i];
#pragma unroll
  for (int f = 0; f < 8; ++f) ob[f] = rhs_bar[(int64_t)f * n + i];
  double gb[7][3];
  mhd_point_adjoint(qi, grad, gamma, ob, qb, gb);
#pragma unroll
  for (int f = 0; f < 7; ++f)
#pragma unroll
    for (int t = 0; t < 3; ++t) ub[f][t] = gb[f][t] * inv_lam;
}

// ---- 2. Y = sum_j w_j p_j (Ubar df_j)^T, plus Ubar and the direct qbar ------
template <int G>
__global__ void __launch_bounds__(THREADS)
    k_adj_y(int n, const double* __restrict__ pos, const double* __restrict__ lam,
            const int64_t* __restrict__ off, const int32_t* __restrict__ idx, Box box,
            double rf_ratio, int wkind, double gamma, const double* __restrict__ q,
            const double* __restrict__ tape, const double* __restrict__ rhs_bar,
            const double* __restrict__ dxdt_bar, double* __restrict__ ybuf,
            double* __restrict__ ubuf, double* __restrict__ qb_direct) {
  const int tid = blockIdx.x * THREADS + threadIdx.x;
  const int i = tid / G;
  const int l = tid % G;
  const bool valid = i < n;
  const int ii = valid ? i : n - 1;
  const double li = lam[ii];
  const double inv_lam = 1.0 / li;
  const int st = (int)tape[(int64_t)21 * n + ii];
  double qi[8], ub[7][3], qb[8];
  pointwise_adjoint(n, ii, q, tape, rhs_bar, dxdt_bar, gamma, inv_lam, st, qi, ub, qb);
  const double xi = pos[ii], yi = pos[(int64_t)n + ii], zi = pos[2 * (int64_t)n + ii];
  const double r = rf_ratio * li;
  const double inv_r2 = 1.0 / (r * r);
  double y[3][NBASIS];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int b = 0; b < NBASIS; ++b) y[t][b] = 0.0;
  const int64_t s0 = off[ii], s1 = (valid && st == 0) ? off[ii + 1] : s0;
  for (int64_t s = s0 + l; s < s1; s += G) {
    const int j = idx[s];
    const double dx = min_image(pos[j] - xi, box.L[0], box.halfL[0], box.periodic[0]);
    const double dy = min_image(pos[(int64_t)n + j] - yi, box.L[1], box.halfL[1], box.periodic[1]);
    const double dz =
        min_image(pos[2 * (int64_t)n + j] - zi, box.L[2], box.halfL[2], box.periodic[2]);
    const double w = weight_of((dx * dx + dy * dy + dz * dz) * inv_r2, wkind);
    double p[NBASIS];
    basis(p, dx * inv_lam, dy * inv_lam, dz * inv_lam);
    double h[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int f = 0; f < 7; ++f) {
      const double df = q[(int64_t)(f + 1) * n + j] - qi[f + 1];
#pragma unroll
      for (int t = 0; t < 3; ++t) h[t] = fma(ub[f][t], df, h[t]);
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const double wh = w * h[t];
#pragma unroll
      for (int b = 0; b < NBASIS; ++b) y[t][b] = fma(wh, p[b], y[t][b]);
    }
  }
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int b = 0; b < NBASIS; ++b) y[t][b] = group_sum<G>(y[t][b]);
  if (valid) {
#pragma unroll
    for (int t = 0; t < 3; ++t)
#pragma unroll
      for (int b = 0; b < NBASIS; ++b)
        if ((t * NBASIS + b) % G == l) ybuf[((int64_t)t * NBASIS + b) * n + i] = y[t][b];
    if (l == 0) {
#pragma unroll
      for (int f = 0; f < 7; ++f)
#pragma unroll
        for (int t = 0; t < 3; ++t) ubuf[((int64_t)f * 3 + t) * n + i] = ub[f][t];
#pragma unroll
      for (int f = 0; f < 8; ++f) qb_direct[(int64_t)f * n + i] = qb[f];
    }
  }
}

// ---- 3. factor again: G = rows 1..3 of A^{-1}, K_t = A^{-1} Y_t ------------
__host__ __device__ constexpr int aoff_a(int rho) { return 2 * rho * (rho + 1); }

__global__ void __launch_bounds__(THREADS)
    k_adj_factor(int n, const double* __restrict__ mom, const double* __restrict__ ybuf,
                 const double* __restrict__ tape, double* __restrict__ gop,
                 double* __restrict__ kop) {
  const int tid = blockIdx.x * THREADS + threadIdx.x;
  const int i = tid >> 2;
  const int l = tid & 3;
  const bool valid = i < n;
  const int ii = valid ? i : n - 1;
  double a[60];
  double dg[5];
  static_for_a<0, 5>([&](auto R) {
    constexpr int rho = R;
    const int r = 4 * rho + l;
    static_for_a<0, 4 * rho + 4>([&](auto C) {
      constexpr int c = C;
      a[aoff_a(rho) + c] = mom[(int64_t)c_entry_a.v[r * NBASIS + c] * n + ii];
    });
    dg[rho] = mom[(int64_t)c_entry_a.v[r * NBASIS + r] * n + ii];
  });
  double s_own[5];
  static_for_a<0, 5>([&](auto R) {
    constexpr int rho = R;
    s_own[rho] = dg[rho] > 0.0 ? 1.0 / sqrt(dg[rho]) : 1.0;
  });
  double s_all[NBASIS];
  static_for_a<0, NBASIS>([&](auto C) {
    constexpr int c = C;
    s_all[c] = quad_bcast<c & 3>(s_own[c >> 2]);
  });
  static_for_a<0, 5>([&](auto R) {
    constexpr int rho = R;
    static_for_a<0, 4 * rho + 4>([&](auto C) {
      constexpr int c = C;
      a[aoff_a(rho) + c] *= s_own[rho] * s_all[c];
    });
  });
  double inv_ld[NBASIS];
  static_for_a<0, NBASIS>([&](auto K) {
    constexpr int k = K;
    constexpr int o = k & 3;
    constexpr int rk = k >> 2;
    const double dkk = quad_bcast<o>(a[aoff_a(rk) + k]);
    const double inv = 1.0 / sqrt(dkk > 0.0 ? dkk : 1.0);
    inv_ld[k] = inv;
    static_for_a<rk, 5>([&](auto R) {
      constexpr int rho = R;
      a[aoff_a(rho) + k] *= inv;
    });
    double colk[NBASIS];
    static_for_a<k + 1, NBASIS>([&](auto C) {
      constexpr int c = C;
      colk[c] = quad_bcast<c & 3>(a[aoff_a(c >> 2) + k]);
    });
    static_for_a<rk, 5>([&](auto R) {
      constexpr int rho = R;
      static_for_a<k + 1, 4 * rho + 4>([&](auto C) {
        constexpr int c = C;
        a[aoff_a(rho) + c] = fma(-a[aoff_a(rho) + k], colk[c], a[aoff_a(rho) + c]);
      });
    });
  });
  const int st = (int)tape[(int64_t)21 * n + ii];
  // Six right-hand sides: e_1, e_2, e_3 (rows of A^{-1}) and Y_0..Y_2.
  // In equilibrated form A^{-1} b = S A_hat^{-1} (S b).
  static_for_a<0, 6>([&](auto RH) {
    constexpr int rh = RH;
    double y[5];
    static_for_a<0, 5>([&](auto R) {
      constexpr int rho = R;
      const int r = 4 * rho + l;
      double b;
      if constexpr (rh < 3)
        b = (r == 1 + rh) ? s_all[1 + rh] : 0.0;
      else
        b = ybuf[((int64_t)(rh - 3) * NBASIS + r) * n + ii] * s_own[rho];
      y[rho] = b;
    });
    constexpr int k0 = rh < 3 ? 1 + rh : 0;
    static_for_a<k0, NBASIS>([&](auto K) {
      constexpr int k = K;
      constexpr int o = k & 3;
      constexpr int rk = k >> 2;
      const double yk = quad_bcast<o>(y[rk]) * inv_ld[k];
      static_for_a<rk + 1, 5>([&](auto R) {
        constexpr int rho = R;
        y[rho] = fma(-a[aoff_a(rho) + k], yk, y[rho]);
      });
      const double upd = fma(-a[aoff_a(rk) + k], yk, y[rk]);
      y[rk] = (l == o) ? yk : ((l > o) ? upd : y[rk]);
    });
    double x[5];
    static_for_a<0, 5>([&](auto R) { x[R] = y[R]; });
    static_for_a<0, NBASIS>([&](auto KK) {
      constexpr int k = NBASIS - 1 - KK;
      constexpr int o = k & 3;
      constexpr int rk = k >> 2;
      double part = 0.0;
      static_for_a<rk + 1, 5>([&](auto R) {
        constexpr int rho = R;
        part = fma(a[aoff_a(rho) + k], x[rho], part);
      });
      part += (l > o) ? a[aoff_a(rk) + k] * x[rk] : 0.0;
      part = group_sum<4>(part);
      const double xk = (y[rk] - part) * inv_ld[k];
      x[rk] = (l == o) ? xk : x[rk];
    });
    if (valid) {
      static_for_a<0, 5>([&](auto R) {
        constexpr int rho = R;
        const int r = 4 * rho + l;
        const double v = st == 0 ? x[rho] * s_own[rho] : 0.0;
        if constexpr (rh < 3)
          gop[((int64_t)rh * NBASIS + r) * n + i] = v;
        else
          kop[((int64_t)(rh - 3) * NBASIS + r) * n + i] = v;
      });
    }
  });
}

// ---- 4. pair contributions --------------------------------------------------
__global__ void __launch_bounds__(THREADS)
    k_adj_pairs(int n, const double* __restrict__ pos, const double* __restrict__ lam,
                const int64_t* __restrict__ off, const int32_t* __restrict__ idx,
                const int32_t* __restrict__ t_pos, Box box, double rf_ratio, int wkind,
                const double* __restrict__ q, const double* __restrict__ gop,
                const double* __restrict__ kop, const double* __restrict__ ubuf,
                double* __restrict__ rec, double* __restrict__ own) {
  const int i = blockIdx.x * THREADS + threadIdx.x;
  if (i >= n) return;
  double g[3][NBASIS], k[3][NBASIS], ub[7][3], qi[7];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int b = 0; b < NBASIS; ++b) {
      g[t][b] = gop[((int64_t)t * NBASIS + b) * n + i];
      k[t][b] = kop[((int64_t)t * NBASIS + b) * n + i];
    }
#pragma unroll
  for (int f = 0; f < 7; ++f) {
    qi[f] = q[(int64_t)(f + 1) * n + i];
#pragma unroll
    for (int t = 0; t < 3; ++t) ub[f][t] = ubuf[((int64_t)f * 3 + t) * n + i];
  }
  const double xi = pos[i], yi = pos[(int64_t)n + i], zi = pos[2 * (int64_t)n + i];
  const double li = lam[i];
  const double inv_lam = 1.0 / li;
  const double r = rf_ratio * li;
  const double inv_r2 = 1.0 / (r * r);
  double sdf[7] = {0, 0, 0, 0, 0, 0, 0}, sd[3] = {0, 0, 0};
  for (int64_t s = off[i]; s < off[i + 1]; ++s) {
    const int j = idx[s];
    double* out = rec + (int64_t)t_pos[s] * REC;
    if (j == i) {  // the self pair adds and removes the same terms
#pragma unroll
      for (int c = 0; c < REC; ++c) out[c] = 0.0;
      continue;
    }
    const double dx = min_image(pos[j] - xi, box.L[0], box.halfL[0], box.periodic[0]);
    const double dy = min_image(pos[(int64_t)n + j] - yi, box.L[1], box.halfL[1], box.periodic[1]);
    const double dz =
        min_image(pos[2 * (int64_t)n + j] - zi, box.L[2], box.halfL[2], box.periodic[2]);
    const double qd = (dx * dx + dy * dy + dz * dz) * inv_r2;
    const double w = weight_of(qd, wkind);
    const double dw = weight_dq(qd, wkind);
    const double ex = dx * inv_lam, ey = dy * inv_lam, ez = dz * inv_lam;
    double p[NBASIS];
    basis(p, ex, ey, ez);
    double av[3], bv[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      double ga = 0.0, kp = 0.0;
#pragma unroll
      for (int b = 0; b < NBASIS; ++b) {
        ga = fma(g[t][b], p[b], ga);
        kp = fma(k[t][b], p[b], kp);
      }
      av[t] = ga;
      bv[t] = -kp;
    }
    double dfb[7];
#pragma unroll
    for (int f = 0; f < 7; ++f) {
      const double df = q[(int64_t)(f + 1) * n + j] - qi[f];
#pragma unroll
      for (int t = 0; t < 3; ++t) bv[t] = fma(ub[f][t], df, bv[t]);
      dfb[f] = w * (ub[f][0] * av[0] + ub[f][1] * av[1] + ub[f][2] * av[2]);
    }
    const double wbar = av[0] * bv[0] + av[1] * bv[1] + av[2] * bv[2];
    // pbar = w (G^T b - K^T a)
    double pb[NBASIS];
#pragma unroll
    for (int b = 0; b < NBASIS; ++b) {
      double v = 0.0;
#pragma unroll
      for (int t = 0; t < 3; ++t) v = fma(g[t][b], bv[t], fma(-k[t][b], av[t], v));
      pb[b] = w * v;
    }
    double gx[NBASIS], gy[NBASIS], gz[NBASIS];
    basis_grad(gx, gy, gz, ex, ey, ez);
    double xb0 = 0.0, xb1 = 0.0, xb2 = 0.0;
#pragma unroll
    for (int b = 0; b < NBASIS; ++b) {
      xb0 = fma(pb[b], gx[b], xb0);
      xb1 = fma(pb[b], gy[b], xb1);
      xb2 = fma(pb[b], gz[b], xb2);
    }
    const double geo = wbar * dw * 2.0 * inv_r2;
    const double db0 = xb0 * inv_lam + geo * dx;
    const double db1 = xb1 * inv_lam + geo * dy;
    const double db2 = xb2 * inv_lam + geo * dz;
#pragma unroll
    for (int f = 0; f < 7; ++f) {
      out[f] = dfb[f];
      sdf[f] += dfb[f];
    }
    out[7] = db0;
    out[8] = db1;
    out[9] = db2;
    sd[0] += db0;
    sd[1] += db1;
    sd[2] += db2;
  }
#pragma unroll
  for (int f = 0; f < 7; ++f) own[(int64_t)f * n + i] = -sdf[f];
#pragma unroll
  for (int a = 0; a < 3; ++a) own[(int64_t)(7 + a) * n + i] = -sd[a];
}

// ---- 5. gather over the transposed lists ------------------------------------
__global__ void __launch_bounds__(THREADS)
    k_adj_gather(int n, const int64_t* __restrict__ t_off, const double* __restrict__ rec,
                 const double* __restrict__ own, const double* __restrict__ qb_direct,
                 double* __restrict__ q_bar, double* __restrict__ pos_bar) {
  const int j = blockIdx.x * THREADS + threadIdx.x;
  if (j >= n) return;
  double acc[REC];
#pragma unroll
  for (int c = 0; c < REC; ++c) acc[c] = own[(int64_t)c * n + j];
  for (int64_t k = t_off[j]; k < t_off[j + 1]; ++k) {
    const double* r = rec + k * REC;
#pragma unroll
    for (int c = 0; c < REC; ++c) acc[c] += r[c];
  }
  q_bar[j] = qb_direct[j];
#pragma unroll
  for (int f = 0; f < 7; ++f) q_bar[(int64_t)(f + 1) * n + j] = qb_direct[(int64_t)(f + 1) * n + j] + acc[f];
#pragma unroll
  for (int a = 0; a < 3; ++a) pos_bar[(int64_t)a * n + j] = acc[7 + a];
}

template <int G>
hipError_t launch_adj_y_g(hipStream_t s, const EvalArgs& a, double gamma, const double* q,
                          const double* tape, const double* rhs_bar, const double* dxdt_bar,
                          double* ybuf, double* ubuf, double* qbd) {
  hipLaunchKernelGGL((k_adj_y<G>), dim3(grid_for((int64_t)a.n * G, THREADS)), dim3(THREADS), 0, s,
                     a.n, a.pos, a.lam, a.off, a.idx, a.box, a.rf_ratio, a.wkind, gamma, q, tape,
                     rhs_bar, dxdt_bar, ybuf, ubuf, qbd);
  return hipGetLastError();
}

}  // namespace

int adjoint_rhs(phb_ctx* ctx, const EvalArgs& a, const phb_params* p, const int64_t* t_offsets,
                const int32_t* t_src, const int32_t* t_pos, const double* q,
                const double* rhs_bar, const double* dxdt_bar, double* q_bar, double* pos_bar,
                const double* tape_in) {
  (void)t_src;
  const int n = a.n;
  // nnz is needed to size the pair records: read offsets[n] back.
  int rc;
  int64_t nnz = 0;
  {
    int64_t* h = nullptr;
    if (hipHostMalloc((void**)&h, sizeof(int64_t)) != hipSuccess)
      return set_error(ctx, PHB_EHIP, "pinned allocation");
    hipError_t e = hipMemcpyAsync(h, a.off + n, sizeof(int64_t), hipMemcpyDeviceToHost,
                                  ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    nnz = *h;
    hipHostFree(h);
    if ((rc = hip_check(ctx, e, "nnz read-back"))) return rc;
  }
  Workspace ws(ctx);
  const size_t nd = (size_t)n * sizeof(double);
  ws.plan(NMOM * nd);          // moments
  ws.plan(3 * NBASIS * nd);    // Y
  ws.plan(3 * NBASIS * nd);    // G
  ws.plan(3 * NBASIS * nd);    // K
  ws.plan(21 * nd);            // Ubar
  ws.plan(8 * nd);             // direct qbar
  ws.plan(10 * nd);            // own sums
  ws.plan((size_t)std::max<int64_t>(nnz, 1) * REC * sizeof(double));  // pair records
  const bool need_tape = tape_in == nullptr;
  if (need_tape) {
    ws.plan(22 * nd);  // tape
    ws.plan(8 * nd);   // rhs scratch
    ws.plan(3 * nd);   // dxdt scratch
    ws.plan((size_t)n * sizeof(int32_t));
  }
  if ((rc = ws.commit())) return rc;
  double* mom = ws.take<double>((size_t)NMOM * n);
  double* ybuf = ws.take<double>((size_t)3 * NBASIS * n);
  double* gop = ws.take<double>((size_t)3 * NBASIS * n);
  double* kop = ws.take<double>((size_t)3 * NBASIS * n);
  double* ubuf = ws.take<double>((size_t)21 * n);
  double* qbd = ws.take<double>((size_t)8 * n);
  double* own = ws.take<double>((size_t)10 * n);
  double* rec = ws.take<double>((size_t)std::max<int64_t>(nnz, 1) * REC);
  const double* tape = tape_in;
  hipStream_t s = ctx->stream;
  { Prof pf(ctx, "k_moments");
  if ((rc = hip_check(ctx, launch_moments(s, a, ctx->lanes_assemble, mom), "adjoint moments")))
    return rc; }
  if (need_tape) {
    double* tp = ws.take<double>((size_t)22 * n);
    double* rs = ws.take<double>((size_t)8 * n);
    double* dx = ws.take<double>((size_t)3 * n);
    int32_t* st = ws.take<int32_t>(n);
    if ((rc = hip_check(ctx, launch_factor(s, a, 3, mom, gop, st), "adjoint factor"))) return rc;
    if ((rc = hip_check(ctx,
                        launch_apply_rhs(s, a, ctx->lanes_apply, p->gamma, gop, st, q, rs, dx, tp),
                        "adjoint forward")))
      return rc;
    tape = tp;
  }
  { Prof pf(ctx, "k_adj_y");
  switch (ctx->lanes_assemble) {
    case 1: rc = hip_check(ctx, launch_adj_y_g<1>(s, a, p->gamma, q, tape, rhs_bar, dxdt_bar, ybuf, ubuf, qbd), "adjoint Y"); break;
    case 2: rc = hip_check(ctx, launch_adj_y_g<2>(s, a, p->gamma, q, tape, rhs_bar, dxdt_bar, ybuf, ubuf, qbd), "adjoint Y"); break;
    default: rc = hip_check(ctx, launch_adj_y_g<4>(s, a, p->gamma, q, tape, rhs_bar, dxdt_bar, ybuf, ubuf, qbd), "adjoint Y"); break;
  }
  if (rc) return rc; }
  { Prof pf(ctx, "k_adj_factor");
  hipLaunchKernelGGL(k_adj_factor, dim3(grid_for((int64_t)n * 4, THREADS)), dim3(THREADS), 0, s, n,
                     mom, ybuf, tape, gop, kop);
  if ((rc = hip_check(ctx, hipGetLastError(), "adjoint factor"))) return rc; }
  { Prof pf(ctx, "k_adj_pairs");
  hipLaunchKernelGGL(k_adj_pairs, dim3(grid_for(n, THREADS)), dim3(THREADS), 0, s, n, a.pos, a.lam,
                     a.off, a.idx, t_pos, a.box, a.rf_ratio, a.wkind, q, gop, kop, ubuf, rec, own);
  if ((rc = hip_check(ctx, hipGetLastError(), "adjoint pairs"))) return rc; }
  Prof pf(ctx, "k_adj_gather");
  hipLaunchKernelGGL(k_adj_gather, dim3(grid_for(n, THREADS)), dim3(THREADS), 0, s, n, t_offsets,
                     rec, own, qbd, q_bar, pos_bar);
  return hip_check(ctx, hipGetLastError(), "adjoint gather");
}

size_t mixed_rhs_bytes(int64_t n) { return 0; }

int mixed_rhs(phb_ctx* ctx, const EvalArgs& a, double gamma, const double* q, double* rhs,
              double* dxdt, int32_t* status, double* tape) {
  return set_error(ctx, PHB_ENOTIMPL, "mixed precision not built yet");
}

}  // namespace phb
