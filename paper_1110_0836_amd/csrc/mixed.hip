// Mixed-precision moving-least-squares derivatives and time derivatives.
//
// Assembly and field application run in FP32 (displacements and field
// differences are formed in FP64 first, scaled by 1/lambda_i, then rounded),
// the 20x20 factorization and solves stay in FP64, and one data-level
// refinement step follows.  With C~ = A~^{-1} B~ from the FP32 sums, the
// residuals r_j = df_j - p(xi_j) . C~ of every neighbor are summed into
// dB = sum_j w_j p(xi_j) r_j (FP32), and the requested coefficient rows are
// E C = E C~ + G~ dB with G~ = E A~^{-1}.  This is one step of the corrected
// seminormal equations (Bjorck): forming the normal matrix in FP32 costs
// kappa(A) eps_32, while the refined solution only sees the data rounding,
// amplified by kappa(P) = sqrt(kappa(A)).
//
// A particle whose FP32-assembled matrix is too ill-conditioned for one step
// to converge (estimated norm of the inverse of the equilibrated matrix above
// a cut, or a failed pivot) is recomputed entirely in FP64: its moments are
// re-assembled in FP64 and factored again (its status is that of the FP64
// form), and its fit is solved by the FP64 refinement on the data that the
// FP64 form applies to its own ill-conditioned fits.  Such particles are
// collected into a list (order irrelevant: each is processed on its own).
//
// Kernels, per evaluation of up to 8 fields:
//   k_moments<fp32>   84 moments, FP32 accumulation            (mls.hip)
//   k_mixed_b         B~ = sum w p df, quad per particle, lane l owns fields
//                     l and l + 4
//   k_mixed_factor    FP64 equilibrated Cholesky of A~, screening, C~ and G~
//   k_mixed_repair    FP64 moments of the listed particles
//   k_mixed_factor    (list form) FP64 factor and status of the listed ones
//   k_mixed_resid     dB in FP32 and the refined rows E C~ + G~ dB
//   refine_fits       FP64 refinement of the listed fits (refine.hip)
//   finish            scaling by powers of 1/lambda, the MHD right-hand side
#include <algorithm>

#include "adjoint.hpp"
#include "chol.hpp"
#include "internal.hpp"
#include "mhd.hpp"
#include "mls.hpp"
#include "refine.hpp"

namespace phb {
namespace {

constexpr int THREADS = 256;
constexpr int LIST_BLOCKS = 512;  // grid of the list-driven kernels

__constant__ EntryTab c_mtab = make_entry_tab();

// Local frame of particle i: FP64 displacement to a neighbor, then FP32
// weight and scaled coordinates.
struct Frame {
  double x, y, z, inv_lam, inv_r2;
  Box box;
  int wkind;
  __device__ __forceinline__ void at(const double4& gj, float& w, float& xs, float& ys,
                                     float& zs) const {
    const double dx = min_image(gj.x - x, box.L[0], box.halfL[0], box.periodic[0]);
    const double dy = min_image(gj.y - y, box.L[1], box.halfL[1], box.periodic[1]);
    const double dz = min_image(gj.z - z, box.L[2], box.halfL[2], box.periodic[2]);
    w = (float)weight_of((dx * dx + dy * dy + dz * dz) * inv_r2, wkind);
    xs = (float)(dx * inv_lam);
    ys = (float)(dy * inv_lam);
    zs = (float)(dz * inv_lam);
  }
};

__device__ __forceinline__ Frame make_frame(const double4& gi, const Box& box, double rf_ratio,
                                            int wkind) {
  Frame f;
  f.x = gi.x;
  f.y = gi.y;
  f.z = gi.z;
  f.inv_lam = 1.0 / gi.w;
  const double r = rf_ratio * gi.w;
  f.inv_r2 = 1.0 / (r * r);
  f.box = box;
  f.wkind = wkind;
  return f;
}

// B~[f][b] = sum_j w_j p_b(xi_j) (f_j - f_i) in FP32.  Four lanes per
// particle; lane l owns fields l and l + 4 of the records fa[8 j + fb + f].
__global__ void __launch_bounds__(THREADS)
    k_mixed_b(int n, const double4* __restrict__ geo, const int64_t* __restrict__ off,
              const int32_t* __restrict__ idx, Box box, double rf_ratio, int wkind,
              const double* __restrict__ fa, int fb, int nf, double* __restrict__ bout) {
  const int tid = xcd_block() * THREADS + threadIdx.x;
  const int i = tid >> 2;
  const int l = tid & 3;
  if (i >= n) return;
  const bool has0 = l < nf, has1 = l + 4 < nf;
  const int fa0 = fb + (has0 ? l : 0), fa1 = fb + (has1 ? l + 4 : 0);
  const double4 gi = geo[i];
  const Frame fr = make_frame(gi, box, rf_ratio, wkind);
  const double fi0 = fa[8 * (int64_t)i + fa0], fi1 = fa[8 * (int64_t)i + fa1];
  float acc0[NBASIS], acc1[NBASIS];
#pragma unroll
  for (int b = 0; b < NBASIS; ++b) acc0[b] = acc1[b] = 0.f;
  const int64_t s0 = off[i], s1 = off[i + 1];
  int64_t s = s0;
  // the next neighbor's record is fetched one iteration ahead
  double4 gn = gi;
  double vn0 = fi0, vn1 = fi1;
  if (s < s1) {
    const int j = idx[s];
    gn = geo[j];
    vn0 = fa[8 * (int64_t)j + fa0];
    vn1 = fa[8 * (int64_t)j + fa1];
  }
  for (; s < s1; ++s) {
    const double4 gj = gn;
    const double v0 = vn0, v1 = vn1;
    if (s + 1 < s1) {
      const int j = idx[s + 1];
      gn = geo[j];
      vn0 = fa[8 * (int64_t)j + fa0];
      vn1 = fa[8 * (int64_t)j + fa1];
    }
    float w, xs, ys, zs;
    fr.at(gj, w, xs, ys, zs);
    float p[NBASIS];
    basis(p, xs, ys, zs);
    const float d0 = w * (float)(v0 - fi0);
    const float d1 = w * (float)(v1 - fi1);
#pragma unroll
    for (int b = 0; b < NBASIS; ++b) {
      acc0[b] = fmaf(d0, p[b], acc0[b]);
      acc1[b] = fmaf(d1, p[b], acc1[b]);
    }
  }
  if (has0) {
#pragma unroll
    for (int b = 0; b < NBASIS; ++b) bout[((int64_t)l * NBASIS + b) * soa_ld(n) + i] = widen(acc0[b]);
  }
  if (has1) {
#pragma unroll
    for (int b = 0; b < NBASIS; ++b)
      bout[((int64_t)(l + 4) * NBASIS + b) * soa_ld(n) + i] = widen(acc1[b]);
  }
}

// Equilibrated FP64 Cholesky of the moments of particle i (quad lanes),
// C = A^{-1} B for nf fields and G = rows 1..NG of A^{-1}.
//
// Screening form (list_in == null, one quad per particle): a particle with at
// least 20 neighbors whose factorization fails or whose equilibrated matrix
// has an estimated ||A_hat^{-1}|| above ncut is flagged and appended to
// list_out; its outputs are left to the list form.  (The refinement step
// contracts the error by about kappa * eps_32 * sqrt(n); the equilibrated
// matrix has unit diagonal, so kappa <= 20 ||A_hat^{-1}||.)  List form: the
// particles list_in[0 .. *count) (FP64 moments by then).
template <int NG, bool SOLVE, bool LISTED>
__device__ __forceinline__ void mixed_factor_one(int n, int i, int l, const double* __restrict__ mom,
                                                 const int64_t* __restrict__ off, int nf,
                                                 const double* __restrict__ bin,
                                                 double* __restrict__ cfit, double* __restrict__ gt,
                                                 int32_t* __restrict__ status,
                                                 int32_t* __restrict__ flag, double ncut,
                                                 int32_t* __restrict__ list_out,
                                                 int32_t* __restrict__ count, int interp) {
  QuadChol c;
  quad_chol_factor(c, c_mtab, mom, soa_ld(n), i, l, interp != 0);
  const int nnb = (int)(off[i + 1] - off[i]);
  const int st = quad_chol_status(c, nnb);
  if constexpr (!LISTED) {
    const bool bad = nnb >= NBASIS && (st != 0 || !(quad_chol_inv_norm_est(c, l) <= ncut));
    if (l == 0) flag[i] = bad ? 1 : 0;
    if (bad) {
      if (l == 0) list_out[atomicAdd(count, 1)] = i;
      return;
    }
  }
  if (l == 0) status[i] = st;
  if constexpr (SOLVE) {
    for (int f = 0; f < nf; ++f) {
      double b[5], x[5];
      sfor<0, 5>([&](auto R) {
        constexpr int rho = R;
        b[rho] = bin[((int64_t)f * NBASIS + 4 * rho + l) * soa_ld(n) + i];
      });
      quad_chol_apply_inverse(c, l, b, x);
      if (interp && l == 0) x[0] = 0.0;  // no constant term: the residuals see p . c of 19
      sfor<0, 5>([&](auto R) {
        constexpr int rho = R;
        cfit[((int64_t)f * NBASIS + 4 * rho + l) * soa_ld(n) + i] = st == 0 ? x[rho] : 0.0;
      });
    }
  }
  sfor<0, NG>([&](auto TI) {
    constexpr int t = 1 + TI;
    double row[5];
    quad_chol_inverse_row<t>(c, l, row);
    sfor<0, 5>([&](auto R) {
      constexpr int rho = R;
      gt[((int64_t)TI * NBASIS + 4 * rho + l) * soa_ld(n) + i] = st == 0 ? row[rho] : 0.0;
    });
  });
}

// LISTED false: the screening form; LISTED true: the listed particles, quad
// k taking list_in[k] for k < *count (the launch covers n quads; a loop
// instead would double the register footprint).  SOLVE false compiles the
// field solves out (nf must then be 0: the operator-level refinement needs
// only G~).
template <int NG, bool SOLVE, bool LISTED>
__global__ void __launch_bounds__(THREADS)
    k_mixed_factor(int n, const double* __restrict__ mom, const int64_t* __restrict__ off, int nf,
                   const double* __restrict__ bin, double* __restrict__ cfit,
                   double* __restrict__ gt, int32_t* __restrict__ status,
                   int32_t* __restrict__ flag, double ncut, const int32_t* __restrict__ list_in,
                   int32_t* __restrict__ list_out, int32_t* __restrict__ count, int interp) {
  const int tid = blockIdx.x * THREADS + threadIdx.x;
  const int l = tid & 3;
  const int quad = tid >> 2;
  if constexpr (!LISTED) {
    if (quad >= n) return;  // whole quads leave together
    mixed_factor_one<NG, SOLVE, false>(n, quad, l, mom, off, nf, bin, cfit, gt, status, flag, ncut,
                                       list_out, count, interp);
  } else {
    if (quad >= *count) return;
    mixed_factor_one<NG, SOLVE, true>(n, list_in[quad], l, mom, off, nf, bin, cfit, gt, status,
                                      flag, ncut, list_out, count, interp);
  }
}

// FP64 moments and right-hand sides of the listed particles.  Four lanes per
// particle split its neighbor entries; partial sums meet in quad reductions.
// A grid-stride loop over the list (its length is read on the device).
__global__ void __launch_bounds__(THREADS)
    k_mixed_repair(int n, const double4* __restrict__ geo, const int64_t* __restrict__ off,
                   const int32_t* __restrict__ idx, Box box, double rf_ratio, int wkind,
                   const double* __restrict__ fa, int fb, int nf, const int32_t* __restrict__ list,
                   const int32_t* __restrict__ count, double* __restrict__ mom,
                   double* __restrict__ bout) {
  const int tid = blockIdx.x * THREADS + threadIdx.x;
  const int l = tid & 3;
  const int total = *count;
  const int stride = (int)(gridDim.x * (THREADS / 4));
  for (int k = tid >> 2; k < total; k += stride) {
    const int i = list[k];
    const double4 gi = geo[i];
    const double inv_lam = 1.0 / gi.w;
    const double r = rf_ratio * gi.w;
    const double inv_r2 = 1.0 / (r * r);
    const int64_t s0 = off[i], s1 = off[i + 1];
    double m[NMOM];
#pragma unroll
    for (int q = 0; q < NMOM; ++q) m[q] = 0.0;
    for (int64_t s = s0 + l; s < s1; s += 4) {
      const double4 gj = geo[idx[s]];
      const double dx = min_image(gj.x - gi.x, box.L[0], box.halfL[0], box.periodic[0]);
      const double dy = min_image(gj.y - gi.y, box.L[1], box.halfL[1], box.periodic[1]);
      const double dz = min_image(gj.z - gi.z, box.L[2], box.halfL[2], box.periodic[2]);
      const double w = weight_of((dx * dx + dy * dy + dz * dz) * inv_r2, wkind);
      accumulate_moments(m, w, dx * inv_lam, dy * inv_lam, dz * inv_lam);
    }
#pragma unroll
    for (int q = 0; q < NMOM; ++q) {
      const double t = group_sum<4>(m[q]);
      if ((q & 3) == l) mom[(int64_t)q * soa_ld(n) + i] = t;
    }
    for (int f0 = 0; f0 < nf; f0 += 4) {
      double fi[4];
      double acc[4][NBASIS];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        fi[f] = f0 + f < nf ? fa[8 * (int64_t)i + fb + f0 + f] : 0.0;
#pragma unroll
        for (int b = 0; b < NBASIS; ++b) acc[f][b] = 0.0;
      }
      for (int64_t s = s0 + l; s < s1; s += 4) {
        const int j = idx[s];
        const double4 gj = geo[j];
        const double dx = min_image(gj.x - gi.x, box.L[0], box.halfL[0], box.periodic[0]);
        const double dy = min_image(gj.y - gi.y, box.L[1], box.halfL[1], box.periodic[1]);
        const double dz = min_image(gj.z - gi.z, box.L[2], box.halfL[2], box.periodic[2]);
        const double w = weight_of((dx * dx + dy * dy + dz * dz) * inv_r2, wkind);
        double p[NBASIS];
        basis(p, dx * inv_lam, dy * inv_lam, dz * inv_lam);
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const double wd = f0 + f < nf ? w * (fa[8 * (int64_t)j + fb + f0 + f] - fi[f]) : 0.0;
#pragma unroll
          for (int b = 0; b < NBASIS; ++b) acc[f][b] = fma(wd, p[b], acc[f][b]);
        }
      }
#pragma unroll
      for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int b = 0; b < NBASIS; ++b) {
          const double t = group_sum<4>(acc[f][b]);
          if (f0 + f < nf && ((f * NBASIS + b) & 3) == l)
            bout[((int64_t)(f0 + f) * NBASIS + b) * soa_ld(n) + i] = t;
        }
    }
  }
}

// dB = sum_j w_j p(xi_j) (df_j - p(xi_j) . C~) in FP32 for the fields of
// this lane (l and l + 4), then rows[f][t] = C[f][1 + t] + (G~ dB)[t] for
// t < NG (FP64).  Flagged particles and particles with status != 0 skip the
// neighbor loop (dB = 0).
template <int NG>
__global__ void __launch_bounds__(THREADS)
    k_mixed_resid(int n, const double4* __restrict__ geo, const int64_t* __restrict__ off,
                  const int32_t* __restrict__ idx, Box box, double rf_ratio, int wkind,
                  const double* __restrict__ fa, int fb, int nf, const double* __restrict__ cfit,
                  const double* __restrict__ gt, const int32_t* __restrict__ status,
                  const int32_t* __restrict__ flag, double* __restrict__ rows) {
  const int tid = xcd_block() * THREADS + threadIdx.x;
  const int i = tid >> 2;
  const int l = tid & 3;
  if (i >= n) return;
  const bool has0 = l < nf, has1 = l + 4 < nf;
  const int f0 = has0 ? l : 0, f1 = has1 ? l + 4 : 0;
  const double4 gi = geo[i];
  const Frame fr = make_frame(gi, box, rf_ratio, wkind);
  const double fi0 = fa[8 * (int64_t)i + fb + f0], fi1 = fa[8 * (int64_t)i + fb + f1];
  // this lane's two coefficient vectors wait in LDS (csh[b][thread]), re-read
  // every neighbor, instead of holding 40 registers through the loop
  __shared__ float2 csh[NBASIS][THREADS];
  float a0[NBASIS], a1[NBASIS];
#pragma unroll
  for (int b = 0; b < NBASIS; ++b) {
    csh[b][threadIdx.x] = make_float2((float)cfit[((int64_t)f0 * NBASIS + b) * soa_ld(n) + i],
                                      (float)cfit[((int64_t)f1 * NBASIS + b) * soa_ld(n) + i]);
    a0[b] = a1[b] = 0.f;
  }
  const bool refine = status[i] == 0 && flag[i] == 0;
  const int64_t s0 = off[i], s1 = refine ? off[i + 1] : s0;
  int64_t s = s0;
  double4 gn = gi;
  double vn0 = fi0, vn1 = fi1;
  if (s < s1) {
    const int j = idx[s];
    gn = geo[j];
    vn0 = fa[8 * (int64_t)j + fb + f0];
    vn1 = fa[8 * (int64_t)j + fb + f1];
  }
  for (; s < s1; ++s) {
    const double4 gj = gn;
    const double v0 = vn0, v1 = vn1;
    if (s + 1 < s1) {
      const int j = idx[s + 1];
      gn = geo[j];
      vn0 = fa[8 * (int64_t)j + fb + f0];
      vn1 = fa[8 * (int64_t)j + fb + f1];
    }
    float w, xs, ys, zs;
    fr.at(gj, w, xs, ys, zs);
    float p[NBASIS];
    basis(p, xs, ys, zs);
    float fit0 = 0.f, fit1 = 0.f;
    asm volatile("" ::: "memory");
#pragma unroll
    for (int b = 0; b < NBASIS; ++b) {
      const float2 cb = csh[b][threadIdx.x];
      fit0 = fmaf(cb.x, p[b], fit0);
      fit1 = fmaf(cb.y, p[b], fit1);
    }
    const float r0 = w * ((float)(v0 - fi0) - fit0);
    const float r1 = w * ((float)(v1 - fi1) - fit1);
#pragma unroll
    for (int b = 0; b < NBASIS; ++b) {
      a0[b] = fmaf(r0, p[b], a0[b]);
      a1[b] = fmaf(r1, p[b], a1[b]);
    }
  }
#pragma unroll
  for (int t = 0; t < NG; ++t) {
    double u0 = cfit[((int64_t)f0 * NBASIS + 1 + t) * soa_ld(n) + i];
    double u1 = cfit[((int64_t)f1 * NBASIS + 1 + t) * soa_ld(n) + i];
#pragma unroll
    for (int b = 0; b < NBASIS; ++b) {
      const double g = gt[((int64_t)t * NBASIS + b) * soa_ld(n) + i];
      u0 = fma(g, (double)a0[b], u0);
      u1 = fma(g, (double)a1[b], u1);
    }
    if (has0) rows[((int64_t)f0 * NG + t) * soa_ld(n) + i] = u0;
    if (has1) rows[((int64_t)f1 * NG + t) * soa_ld(n) + i] = u1;
  }
}

// ---- operator-level refinement ----------------------------------------------
// With G~ = E A~^{-1} from the FP32-assembled moments, one Newton step on the
// operator rows gives
//   G^ = G~ (2 I - A A~^{-1}) = 2 G~ - (G~ A) A~^{-1},
// whose error is quadratic in that of G~: G^ - E A^{-1} =
// -E (A~^{-1} - A^{-1}) A (A~^{-1} - A^{-1}).  The product G~ A is the
// residual of the step and must be formed more accurately than the error it
// removes, so this pass runs in FP64:
//   M_t = sum_j w_j (G~_t . p_j) p_j^T
// for three rows r0 .. r0 + 2 at a time (60 accumulators per lane).  The
// particle's three rows of G~ wait in LDS.  Particles with a nonzero status
// or on the FP64 list skip the neighbor loop (their rows are final).
template <int G>
__global__ void __launch_bounds__(THREADS)
    k_mixed_gta(int n, const double4* __restrict__ geo, const int64_t* __restrict__ off,
                const int32_t* __restrict__ idx, Box box, double rf_ratio, int wkind,
                const double* __restrict__ gt, int r0, const int32_t* __restrict__ status,
                const int32_t* __restrict__ flag, double* __restrict__ mbuf) {
  const int tid = xcd_block() * THREADS + threadIdx.x;
  const int i = tid / G;
  const int l = tid % G;
  const bool valid = i < n;
  const int ii = valid ? i : n - 1;
  const double4 gi = geo[ii];
  const bool go = valid && status[ii] == 0 && flag[ii] == 0;
  // the first neighbor entry is fetched ahead of the staging and the barrier
  const int64_t s0 = off[ii], s1 = go ? off[ii + 1] : s0;
  int64_t s = s0 + l;
  int jn = ii;
  double4 gn = gi;
  if (s < s1) gn = geo[idx[s]];
  if (s + G < s1) jn = idx[s + G];
  constexpr int PPB = THREADS / G;
  __shared__ double2 gsh[3 * NBASIS / 2][PPB];
  const int pl = threadIdx.x / G;
  for (int k = l; k < 3 * NBASIS / 2; k += G) {
    const int t = (2 * k) / NBASIS, b = (2 * k) % NBASIS;
    gsh[k][pl] = make_double2(gt[((int64_t)(r0 + t) * NBASIS + b) * soa_ld(n) + ii],
                              gt[((int64_t)(r0 + t) * NBASIS + b + 1) * soa_ld(n) + ii]);
  }
  __syncthreads();
  const double inv_lam = 1.0 / gi.w;
  const double r = rf_ratio * gi.w;
  const double inv_r2 = 1.0 / (r * r);
  double m[3][NBASIS];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int b = 0; b < NBASIS; ++b) m[t][b] = 0.0;
  for (; s < s1; s += G) {
    const double4 gj = gn;
    if (s + G < s1) {
      gn = geo[jn];
      if (s + 2 * G < s1) jn = idx[s + 2 * G];
    }
    const double dx = min_image(gj.x - gi.x, box.L[0], box.halfL[0], box.periodic[0]);
    const double dy = min_image(gj.y - gi.y, box.L[1], box.halfL[1], box.periodic[1]);
    const double dz = min_image(gj.z - gi.z, box.L[2], box.halfL[2], box.periodic[2]);
    const double w = weight_of((dx * dx + dy * dy + dz * dz) * inv_r2, wkind);
    double p[NBASIS];
    basis(p, dx * inv_lam, dy * inv_lam, dz * inv_lam);
    asm volatile("" ::: "memory");  // re-read the rows from LDS every iteration
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      double v = 0.0;
#pragma unroll
      for (int b = 0; b < NBASIS; b += 2) {
        const double2 gg = gsh[(t * NBASIS + b) / 2][pl];
        v = fma(gg.x, p[b], v);
        v = fma(gg.y, p[b + 1], v);
      }
      const double a = w * v;
#pragma unroll
      for (int b = 0; b < NBASIS; ++b) m[t][b] = fma(a, p[b], m[t][b]);
    }
  }
  store_rows3<G>(&m[0][0], l, valid, mbuf, r0, soa_ld(n), i);
}

// The Newton step G^_t = 2 G~_t - A~^{-1} M_t for rows 1..NG (quad per
// particle; A~ factored again, as in the screening).  In the interpolating
// fit the constant's row and column of A are the identity's: M_t's constant
// entry is dropped, which keeps G^_t's constant entry at zero.
template <int NG>
__global__ void __launch_bounds__(THREADS)
    k_mixed_refine(int n, const double* __restrict__ mom, const double* __restrict__ mbuf,
                   double* __restrict__ gt, const int32_t* __restrict__ status,
                   const int32_t* __restrict__ flag, int interp) {
  static_assert(NG % 3 == 0, "rows in groups of three");
  const int tid = blockIdx.x * THREADS + threadIdx.x;
  const int l = tid & 3;
  const int i = tid >> 2;
  if (i >= n) return;  // whole quads leave together
  if (status[i] != 0 || flag[i] != 0) return;
  QuadChol c;
  quad_chol_factor(c, c_mtab, mom, soa_ld(n), i, l, interp != 0);
  sfor<0, NG / 3>([&](auto GI) {
    constexpr int t0 = 3 * GI;
    double y[3][5], x[3][5];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int rho = 0; rho < 5; ++rho) {
        const double b = mbuf[((int64_t)(t0 + r) * NBASIS + 4 * rho + l) * soa_ld(n) + i];
        y[r][rho] = (interp && rho == 0 && l == 0) ? 0.0 : b * c.s_own[rho];
      }
    quad_chol_solve_n<0, 3>(c, l, y, x);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int rho = 0; rho < 5; ++rho) {
        const int64_t k = ((int64_t)(t0 + r) * NBASIS + 4 * rho + l) * soa_ld(n) + i;
        gt[k] = fma(-x[r][rho], c.s_own[rho], 2.0 * gt[k]);
      }
  });
}

__global__ void k_zero_i32(int32_t* p, int m) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) p[k] = 0;
}

// Screen threshold on the estimated ||A_hat^{-1}||: 10^(x10 / 10), x10 from
// the context or, when unset (-1), the form's own: one Newton step on the
// operator rows leaves an error quadratic in kappa eps_32 and tolerates
// 10^2.5; the data-level step 10^2.
double screen_cut(const phb_ctx* ctx, int x10_default) {
  const int x10 = ctx->mixed_cond_x10 >= 0 ? ctx->mixed_cond_x10 : x10_default;
  return pow(10.0, 0.1 * x10);
}

struct MixedBufs {
  double* mom;
  double* b;
  double* cfit;
  double* gt;
  double* rows;
  int32_t* flag;
  int32_t* list;
  int32_t* count;
  RefineBufs ref;  // the listed fits' refinement state
};

void plan_mixed(Workspace& ws, int64_t n, int nf, int ng) {
  const size_t nd = (size_t)soa_ld(n) * sizeof(double);  // rows of the padded stride
  ws.plan(NMOM * nd);
  ws.plan((size_t)nf * NBASIS * nd);
  ws.plan((size_t)nf * NBASIS * nd);
  ws.plan((size_t)ng * NBASIS * nd);
  ws.plan((size_t)nf * ng * nd);
  ws.plan((size_t)n * sizeof(int32_t));
  ws.plan((size_t)n * sizeof(int32_t));
  ws.plan(sizeof(int32_t));
  plan_refine_state(ws, n);
}

// The refinement of the listed particles reuses B~ (residual sums) and C~
// (coefficients) once the FP32 fit is done with them.
RefineBufs listed_refine(const MixedBufs& m, int64_t n) {
  RefineBufs r = m.ref;
  r.list = m.list;
  r.count = m.count;
  r.cbuf = m.cfit;
  r.dbuf = m.b;
  r.ldc = soa_ld(n);
  return r;
}

MixedBufs take_mixed(Workspace& ws, int64_t n, int nf, int ng) {
  MixedBufs m;
  const size_t ld = soa_ld(n);
  m.mom = ws.take<double>((size_t)NMOM * ld);
  m.b = ws.take<double>((size_t)nf * NBASIS * ld);
  m.cfit = ws.take<double>((size_t)nf * NBASIS * ld);
  m.gt = ws.take<double>((size_t)ng * NBASIS * ld);
  m.rows = ws.take<double>((size_t)nf * ng * ld);
  m.flag = ws.take<int32_t>(n);
  m.list = ws.take<int32_t>(n);
  m.count = ws.take<int32_t>(1);
  take_refine_state(ws, n, m.ref);
  return m;
}

// Refined coefficient rows 1..NG (unscaled) of nf <= 8 fields stored in the
// records fa[8 j + fb + f] into m.rows; m.mom receives the moments
// (FP32-assembled, FP64 for the listed particles).  The listed particles'
// rows in m.rows are those of the plain FP64 solve; their refined
// coefficients are left in listed_coef() by list position.
template <int NG>
int mixed_fit(phb_ctx* ctx, const EvalArgs& a, const double* fa, int fb, int nf,
              const MixedBufs& m, int32_t* status) {
  hipStream_t s = ctx->stream;
  const int n = a.n;
  const double ncut = screen_cut(ctx, 20);
  const int interp = a.fit == PHB_FIT_INTERP19;
  const unsigned gq = grid_for((int64_t)n * 4, THREADS);
  int rc;
  { Prof pf(ctx, "k_moments<fp32>");
    if ((rc = hip_check(ctx, launch_moments(s, a, ctx->moments_mfma ? 0 : ctx->lanes_assemble, m.mom, true), "moments")))
      return rc; }
  { Prof pf(ctx, "k_mixed_b");
    hipLaunchKernelGGL(k_mixed_b, dim3(gq), dim3(THREADS), 0, s, n, a.geo, a.off, a.idx, a.box,
                       a.rf_ratio, a.wkind, fa, fb, nf, m.b);
    if ((rc = hip_check(ctx, hipGetLastError(), "mixed B"))) return rc; }
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, m.count, 1);
  { Prof pf(ctx, "k_mixed_factor");
    hipLaunchKernelGGL((k_mixed_factor<NG, true, false>), dim3(gq), dim3(THREADS), 0, s, n, m.mom, a.off, nf,
                       m.b, m.cfit, m.gt, status, m.flag, ncut, nullptr, m.list, m.count, interp);
    if ((rc = hip_check(ctx, hipGetLastError(), "mixed factor"))) return rc; }
  { Prof pf(ctx, "k_mixed_repair");
    hipLaunchKernelGGL(k_mixed_repair, dim3(LIST_BLOCKS), dim3(THREADS), 0, s, n, a.geo, a.off,
                       a.idx, a.box, a.rf_ratio, a.wkind, nullptr, 0, 0, m.list, m.count, m.mom,
                       nullptr);
    hipLaunchKernelGGL((k_mixed_factor<NG, true, true>), dim3(gq), dim3(THREADS), 0, s, n, m.mom,
                       a.off, nf, m.b, m.cfit, m.gt, status, m.flag, ncut, m.list, nullptr,
                       m.count, interp);
    if ((rc = hip_check(ctx, hipGetLastError(), "mixed repair"))) return rc; }
  { Prof pf(ctx, "k_mixed_resid");
    hipLaunchKernelGGL((k_mixed_resid<NG>), dim3(gq), dim3(THREADS), 0, s, n, a.geo, a.off, a.idx,
                       a.box, a.rf_ratio, a.wkind, fa, fb, nf, m.cfit, m.gt, status, m.flag,
                       m.rows);
    if ((rc = hip_check(ctx, hipGetLastError(), "mixed residual"))) return rc; }
  // B~ and C~ are dead now: they hold the listed fits' refinement
  return refine_fits(ctx, a, fa, fb, nf, m.mom, listed_refine(m, n));
}

struct OpBufs {
  double* mom;
  double* gt;
  double* mb;
  int32_t* flag;
  int32_t* list;
  int32_t* count;
};

void plan_op(Workspace& ws, int64_t n, int ng) {
  const size_t nd = (size_t)soa_ld(n) * sizeof(double);  // rows of the padded stride
  ws.plan(NMOM * nd);
  ws.plan((size_t)ng * NBASIS * nd);
  ws.plan((size_t)ng * NBASIS * nd);
  ws.plan((size_t)n * sizeof(int32_t));
  ws.plan((size_t)n * sizeof(int32_t));
  ws.plan(sizeof(int32_t));
}

OpBufs take_op(Workspace& ws, int64_t n, int ng) {
  OpBufs m;
  const size_t ld = soa_ld(n);
  m.mom = ws.take<double>((size_t)NMOM * ld);
  m.gt = ws.take<double>((size_t)ng * NBASIS * ld);
  m.mb = ws.take<double>((size_t)ng * NBASIS * ld);
  m.flag = ws.take<int32_t>(n);
  m.list = ws.take<int32_t>(n);
  m.count = ws.take<int32_t>(1);
  return m;
}

template <int G>
void launch_gta(hipStream_t s, const EvalArgs& a, const double* gt, int ng,
                const int32_t* status, const int32_t* flag, double* mb) {
  for (int r0 = 0; r0 < ng; r0 += 3)
    hipLaunchKernelGGL((k_mixed_gta<G>), dim3(grid_for((int64_t)a.n * G, THREADS)), dim3(THREADS), 0,
                       s, a.n, a.geo, a.off, a.idx, a.box, a.rf_ratio, a.wkind, gt, r0, status,
                       flag, mb);
}

// Refined operator rows 1..NG of A^{-1} into m.gt: FP32 moments (FP64 for the
// particles the screen lists), the FP64 factor with the screen, the FP64
// residual product G~ A and the Newton step.
template <int NG>
int mixed_operator(phb_ctx* ctx, const EvalArgs& a, const OpBufs& m, int32_t* status) {
  hipStream_t s = ctx->stream;
  const int n = a.n;
  const double ncut = screen_cut(ctx, 25);
  const int interp = a.fit == PHB_FIT_INTERP19;
  const unsigned gq = grid_for((int64_t)n * 4, THREADS);
  int rc;
  { Prof pf(ctx, "k_moments<fp32>");
    if ((rc = hip_check(ctx, launch_moments(s, a, ctx->moments_mfma ? 0 : ctx->lanes_assemble, m.mom, true), "moments")))
      return rc; }
  hipLaunchKernelGGL(k_zero_i32, dim3(1), dim3(64), 0, s, m.count, 1);
  { Prof pf(ctx, "k_mixed_screen");
    hipLaunchKernelGGL((k_mixed_factor<NG, false, false>), dim3(gq), dim3(THREADS), 0, s, n, m.mom, a.off, 0,
                       nullptr, nullptr, m.gt, status, m.flag, ncut, nullptr, m.list, m.count,
                       interp);
    if ((rc = hip_check(ctx, hipGetLastError(), "mixed factor"))) return rc; }
  { Prof pf(ctx, "k_mixed_repair");
    hipLaunchKernelGGL(k_mixed_repair, dim3(LIST_BLOCKS), dim3(THREADS), 0, s, n, a.geo, a.off,
                       a.idx, a.box, a.rf_ratio, a.wkind, nullptr, 0, 0, m.list, m.count, m.mom,
                       nullptr);
    hipLaunchKernelGGL((k_mixed_factor<NG, false, true>), dim3(gq), dim3(THREADS), 0, s, n, m.mom,
                       a.off, 0, nullptr, nullptr, m.gt, status, m.flag, ncut, m.list, nullptr,
                       m.count, interp);
    if ((rc = hip_check(ctx, hipGetLastError(), "mixed repair"))) return rc; }
  { Prof pf(ctx, "k_mixed_gta");
    // the reverse-mode Y kernel's shape (60 FP64 sums per lane): its lane
    // count applies
    switch (ctx->lanes_adj_y) {
      case 1: launch_gta<1>(s, a, m.gt, NG, status, m.flag, m.mb); break;
      case 2: launch_gta<2>(s, a, m.gt, NG, status, m.flag, m.mb); break;
      default: launch_gta<4>(s, a, m.gt, NG, status, m.flag, m.mb); break;
    }
    if ((rc = hip_check(ctx, hipGetLastError(), "mixed residual product"))) return rc; }
  Prof pf(ctx, "k_mixed_refine");
  hipLaunchKernelGGL((k_mixed_refine<NG>), dim3(gq), dim3(THREADS), 0, s, n, m.mom, m.mb, m.gt,
                     status, m.flag, interp);
  return hip_check(ctx, hipGetLastError(), "mixed refinement");
}

}  // namespace

// Workspace of the operator-level form: its buffers, the packed records and
// the listed fits' refinement (coefficients and residual sums of nf fields).
static void plan_op_form(Workspace& ws, int64_t n, int ng, int nf) {
  plan_op(ws, n, ng);
  ws.plan((size_t)n * sizeof(double4));
  ws.plan((size_t)8 * n * sizeof(double));
  ws.plan((size_t)2 * nf * NBASIS * soa_ld(n) * sizeof(double));
  plan_refine_state(ws, n);
}

static RefineBufs take_op_refine(Workspace& ws, const OpBufs& m, int64_t n, int nf) {
  RefineBufs r;
  r.ldc = soa_ld(n);
  r.list = m.list;
  r.count = m.count;
  r.cbuf = ws.take<double>((size_t)nf * NBASIS * r.ldc);
  r.dbuf = ws.take<double>((size_t)nf * NBASIS * r.ldc);
  take_refine_state(ws, n, r);
  return r;
}

size_t mixed_rhs_bytes(int64_t n, bool stab) {
  phb_ctx dummy;
  const int nf = stab ? 8 : 7, ng = stab ? 9 : 3;
  // the larger of the two refinement forms
  Workspace wd(&dummy);
  plan_mixed(wd, n, nf, ng);
  wd.plan((size_t)n * sizeof(double4));
  wd.plan((size_t)8 * n * sizeof(double));
  Workspace wo(&dummy);
  plan_op_form(wo, n, ng, nf);
  return std::max(wd.total, wo.total);
}

// Operator-level form of mixed_rhs: the refined rows applied in FP32.
static int mixed_rhs_op(phb_ctx* ctx, const EvalArgs& a0, double gamma, const Stab& sb,
                        const double* q, double* rhs, double* dxdt, int32_t* status) {
  const int n = a0.n;
  const bool stab = sb.on();
  const int ng = stab ? 9 : 3, nf = stab ? 8 : 7;
  Workspace ws(ctx);
  plan_op_form(ws, n, ng, nf);
  int rc;
  if ((rc = ws.commit())) return rc;
  OpBufs m = take_op(ws, n, ng);
  double4* geo = ws.take<double4>(n);
  double* fq = ws.take<double>((size_t)8 * n);
  const RefineBufs rb = take_op_refine(ws, m, n, nf);
  EvalArgs a = a0;
  a.geo = geo;
  a.fq = fq;
  { Prof pf(ctx, "k_pack");
    if ((rc = hip_check(ctx, launch_pack(ctx->stream, n, a.pos, a.lam, q, geo, fq), "pack")))
      return rc; }
  rc = stab ? mixed_operator<9>(ctx, a, m, status) : mixed_operator<3>(ctx, a, m, status);
  if (rc) return rc;
  { Prof pf(ctx, stab ? "k_apply_rhs<fp32, stab>" : "k_apply_rhs<fp32>");
    if ((rc = hip_check(ctx,
                        launch_apply_rhs(ctx->stream, a, ctx->lanes_apply, gamma, sb, m.gt,
                                         status, rhs, dxdt, nullptr),
                        "mixed apply")))
      return rc; }
  // the listed (ill-conditioned) particles again, by the FP64 refinement on
  // the data: applied in FP32 their operator would lose kappa eps_32, in
  // FP64 kappa eps_64
  if ((rc = refine_fits(ctx, a, fq, stab ? 0 : 1, nf, m.mom, rb))) return rc;
  Prof pf(ctx, "k_rows_rhs_finish<list>");
  return hip_check(ctx,
                   launch_rows_rhs_finish(ctx->stream, a, stab, rb.cbuf, NBASIS, 1, rb.ldc,
                                          rb.list, rb.count, status, gamma, sb, rhs, dxdt,
                                          nullptr),
                   "mixed rhs (listed)");
}

int mixed_rhs(phb_ctx* ctx, const EvalArgs& a0, double gamma, const Stab& sb, const double* q,
              double* rhs, double* dxdt, int32_t* status) {
  // by shape (2): the operator-level step for the three gradient rows; with
  // the stabilisers' nine rows it needs three residual-product passes, and
  // the data-level step's two passes over the eight fields cost less
  const int form = ctx->mixed_refine == 2 ? (sb.on() ? 0 : 1) : ctx->mixed_refine;
  if (form == 1) return mixed_rhs_op(ctx, a0, gamma, sb, q, rhs, dxdt, status);
  const int n = a0.n;
  const bool stab = sb.on();
  // ideal: V, B, sigma (records 1..7), three rows; stabilised: all eight
  // fields (rho's gradient feeds the sensor), nine rows
  const int nf = stab ? 8 : 7, ng = stab ? 9 : 3;
  Workspace ws(ctx);
  plan_mixed(ws, n, nf, ng);
  ws.plan((size_t)n * sizeof(double4));
  ws.plan((size_t)8 * n * sizeof(double));
  int rc;
  if ((rc = ws.commit())) return rc;
  MixedBufs m = take_mixed(ws, n, nf, ng);
  double4* geo = ws.take<double4>(n);
  double* fq = ws.take<double>((size_t)8 * n);
  EvalArgs a = a0;
  a.geo = geo;
  a.fq = fq;
  { Prof pf(ctx, "k_pack");
    if ((rc = hip_check(ctx, launch_pack(ctx->stream, n, a.pos, a.lam, q, geo, fq), "pack")))
      return rc; }
  // V, B and sigma are entries 1..7 of the packed records (all eight with the
  // stabilisers)
  rc = stab ? mixed_fit<9>(ctx, a, fq, 0, 8, m, status) : mixed_fit<3>(ctx, a, fq, 1, 7, m, status);
  if (rc) return rc;
  const RefineBufs rb = listed_refine(m, n);
  { Prof pf(ctx, stab ? "k_rows_rhs_finish<stab>" : "k_rows_rhs_finish");
    if ((rc = hip_check(ctx,
                        launch_rows_rhs_finish(ctx->stream, a, stab, m.rows, ng, 0, soa_ld(n),
                                               nullptr, nullptr, status, gamma, sb, rhs, dxdt,
                                               nullptr),
                        "mixed rhs")))
      return rc; }
  Prof pf(ctx, "k_rows_rhs_finish<list>");
  return hip_check(ctx,
                   launch_rows_rhs_finish(ctx->stream, a, stab, rb.cbuf, NBASIS, 1, rb.ldc,
                                          rb.list, rb.count, status, gamma, sb, rhs, dxdt,
                                          nullptr),
                   "mixed rhs (listed)");
}

size_t mixed_derivs_bytes(int64_t n, bool second) {
  phb_ctx dummy;
  const int ng = second ? 9 : 3;
  Workspace wd(&dummy);
  plan_mixed(wd, n, 8, ng);
  wd.plan((size_t)n * sizeof(double4));
  wd.plan((size_t)8 * n * sizeof(double));
  Workspace wo(&dummy);
  plan_op_form(wo, n, ng, 8);
  return std::max(wd.total, wo.total);
}

// Operator-level form of mixed_derivs: one refined operator serves every
// field.
static int mixed_derivs_op(phb_ctx* ctx, const EvalArgs& a0, int nf, const double* fields,
                           double* d1, double* d2, int32_t* status) {
  const int n = a0.n;
  const int ng = d2 ? 9 : 3;
  Workspace ws(ctx);
  plan_op_form(ws, n, ng, 8);
  int rc;
  if ((rc = ws.commit())) return rc;
  OpBufs m = take_op(ws, n, ng);
  double4* geo = ws.take<double4>(n);
  double* fa = ws.take<double>((size_t)8 * n);
  const RefineBufs rb = take_op_refine(ws, m, n, 8);
  EvalArgs a = a0;
  a.geo = geo;
  if ((rc = hip_check(ctx, launch_pack(ctx->stream, n, a.pos, a.lam, nullptr, geo, nullptr),
                      "pack")))
    return rc;
  rc = d2 ? mixed_operator<9>(ctx, a, m, status) : mixed_operator<3>(ctx, a, m, status);
  if (rc) return rc;
  if ((rc = hip_check(ctx,
                      launch_apply_derivs(ctx->stream, a, ctx->lanes_apply, m.gt, status, nf,
                                          fields, d1, d2, true),
                      "mixed derivatives")))
    return rc;
  // the listed particles again by the FP64 refinement (as in mixed_rhs_op)
  for (int f0 = 0; f0 < nf; f0 += 8) {
    const int nfc = nf - f0 < 8 ? nf - f0 : 8;
    if ((rc = hip_check(ctx, launch_pack_chunk(ctx->stream, n, fields, f0, nfc, fa), "pack")))
      return rc;
    if ((rc = refine_fits(ctx, a, fa, 0, nfc, m.mom, rb))) return rc;
    if ((rc = hip_check(ctx,
                        launch_rows_derivs_finish(ctx->stream, a, ng, rb.cbuf, NBASIS, 1, rb.ldc,
                                                  rb.list, rb.count, status, nfc, f0, d1, d2),
                        "mixed derivatives (listed)")))
      return rc;
  }
  return PHB_OK;
}

int mixed_derivs(phb_ctx* ctx, const EvalArgs& a0, int nf, const double* fields, double* d1,
                 double* d2, int32_t* status) {
  const int form = ctx->mixed_refine == 2 ? (d2 ? 0 : 1) : ctx->mixed_refine;
  if (form == 1) return mixed_derivs_op(ctx, a0, nf, fields, d1, d2, status);
  const int n = a0.n;
  const int ng = d2 ? 9 : 3;
  Workspace ws(ctx);
  plan_mixed(ws, n, 8, ng);
  ws.plan((size_t)n * sizeof(double4));
  ws.plan((size_t)8 * n * sizeof(double));
  int rc;
  if ((rc = ws.commit())) return rc;
  MixedBufs m = take_mixed(ws, n, 8, ng);
  double4* geo = ws.take<double4>(n);
  double* fa = ws.take<double>((size_t)8 * n);
  const RefineBufs rb = listed_refine(m, n);
  EvalArgs a = a0;
  a.geo = geo;
  if ((rc = hip_check(ctx, launch_pack(ctx->stream, n, a.pos, a.lam, nullptr, geo, nullptr),
                      "pack")))
    return rc;
  for (int f0 = 0; f0 < nf; f0 += 8) {
    const int nfc = nf - f0 < 8 ? nf - f0 : 8;
    if ((rc = hip_check(ctx, launch_pack_chunk(ctx->stream, n, fields, f0, nfc, fa), "pack")))
      return rc;
    // the moments are assembled again per chunk: the list form has replaced
    // the flagged particles' moments by FP64 ones
    rc = ng == 9 ? mixed_fit<9>(ctx, a, fa, 0, nfc, m, status)
                 : mixed_fit<3>(ctx, a, fa, 0, nfc, m, status);
    if (rc) return rc;
    if ((rc = hip_check(ctx,
                        launch_rows_derivs_finish(ctx->stream, a, ng, m.rows, ng, 0, soa_ld(n),
                                                  nullptr, nullptr, status, nfc, f0, d1, d2),
                        "mixed derivatives")) ||
        (rc = hip_check(ctx,
                        launch_rows_derivs_finish(ctx->stream, a, ng, rb.cbuf, NBASIS, 1, rb.ldc,
                                                  rb.list, rb.count, status, nfc, f0, d1, d2),
                        "mixed derivatives (listed)")))
      return rc;
  }
  return PHB_OK;
}

}  // namespace phb
