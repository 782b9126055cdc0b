// Moving-least-squares derivatives and ideal-MHD time derivatives
// (paper II, Sec. 2) in FP64.
//
// Three kernels per evaluation:
//  1. k_moments: for each particle, the 84 distinct weighted moments
//     sum_j w_j xi_j^alpha (|alpha| <= 6) that make up the 20x20 normal
//     matrix A = sum_j w_j p(xi_j) p(xi_j)^T.  G lanes share one particle's
//     neighbor list and combine their partial sums with DPP quad permutes.
//  2. k_factor: four lanes per particle hold A row-cyclically (lane l owns
//     rows l, l+4, ...), Jacobi-equilibrate it, factor it by Cholesky in FP64
//     and solve for the requested rows of A^{-1} (the derivative operator in
//     monomial space): G = E A^{-1}, E selecting the gradient (and Hessian)
//     monomials.
//  3. k_apply_*: for each neighbor, gamma_j = w_j G p(xi_j) are the operator
//     weights; derivatives are sum_j gamma_j (f_j - f_i) scaled by powers of
//     1/lambda_i, followed (for the time derivatives) by the pointwise
//     ideal-MHD right-hand side.
// This "operator" form needs 84 + 3x20 accumulations per neighbor instead of
// the 84 + 20 x nfields of solving for every field's coefficients.
#include <type_traits>

#include "chol.hpp"
#include "internal.hpp"
#include "mls.hpp"

namespace phb {
namespace {

constexpr int THREADS = 256;

// ---------------------------------------------------------------------------
// 1. moments
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(THREADS)
    k_pack(int n, const double* __restrict__ pos, const double* __restrict__ lam,
           const double* __restrict__ q, double4* __restrict__ geo, double* __restrict__ fq) {
  const int i = blockIdx.x * THREADS + threadIdx.x;
  if (i >= n) return;
  geo[i] = make_double4(pos[i], pos[(int64_t)n + i], pos[2 * (int64_t)n + i], lam[i]);
  if (q) {
    double2* o = reinterpret_cast<double2*>(fq + 8 * (int64_t)i);
#pragma unroll
    for (int f = 0; f < 8; f += 2)
      o[f / 2] = make_double2(q[(int64_t)f * n + i], q[(int64_t)(f + 1) * n + i]);
  }
}

// T is the accumulation type: double, or float for the mixed form (the
// displacement, its scaling by 1/lambda and the weight are formed in FP64 and
// only then rounded to FP32).
template <int G, class T = double>
__global__ void __launch_bounds__(THREADS)
    k_moments(int n, const double4* __restrict__ geo, const int64_t* __restrict__ off,
              const int32_t* __restrict__ idx, Box box, double rf_ratio, int wkind,
              double* __restrict__ mom, const int32_t* __restrict__ rows) {
  const int tid = xcd_block() * THREADS + threadIdx.x;
  const int i = tid / G;
  const int l = tid % G;
  const bool valid = i < n;
  const int ii = valid ? i : n - 1;
  T m[NMOM];
#pragma unroll
  for (int k = 0; k < NMOM; ++k) m[k] = T(0);
  const double4 gi = geo[rows ? rows[ii] : ii];  // row ii's own particle
  const double inv_lam = 1.0 / gi.w;
  const double r = rf_ratio * gi.w;
  const double inv_r2 = 1.0 / (r * r);
  const int64_t s0 = off[ii], s1 = valid ? off[ii + 1] : s0;
  // neighbor records are fetched one iteration ahead, indices two ahead
  int64_t s = s0 + l;
  double4 gn = gi;
  int jn = 0;
  if (s < s1) gn = geo[idx[s]];
  if (s + G < s1) jn = idx[s + G];
  for (; s < s1; s += G) {
    const double4 gj = gn;
    if (s + G < s1) {
      gn = geo[jn];
      if (s + 2 * G < s1) jn = idx[s + 2 * G];
    }
    const double dx = min_image(gj.x - gi.x, box.L[0], box.halfL[0], box.periodic[0]);
    const double dy = min_image(gj.y - gi.y, box.L[1], box.halfL[1], box.periodic[1]);
    const double dz = min_image(gj.z - gi.z, box.L[2], box.halfL[2], box.periodic[2]);
    const double qd = (dx * dx + dy * dy + dz * dz) * inv_r2;
    const double w = weight_of(qd, wkind);
    accumulate_moments(m, T(w), T(dx * inv_lam), T(dy * inv_lam), T(dz * inv_lam));
  }
  // lane l of the group ends with the moments l, l + G, ... and stores them
  T mine[NMOM / G];
  group_reduce_scatter<G, NMOM>(m, mine, l);
  if (valid) {
    double* dst = mom + (int64_t)l * soa_ld(n) + i;
#pragma unroll
    for (int k = 0; k < NMOM / G; ++k) dst[(int64_t)(G * k) * soa_ld(n)] = widen(mine[k]);
  }
}

// The FP32 moments on the matrix cores: A = P^T W P (P: the entries' 20
// monomials) as 16 x 16 x 4 FP32 MFMA products over groups of four entries,
// one wavefront per particle.  Lane l feeds monomial l % 16 (and 16 + l % 16,
// the four cubic monomials past the first tile) of entry l / 16 of the group:
// the A operand is p_c(xi), the B operand w p_c(xi), and the 32 x 32 padded
// product needs three tiles by symmetry (rows/columns 0-15 x 0-15, 0-15 x
// 16-31, 16-31 x 16-31), whose valid entries hold every one of the 84
// moments; a table names the lane and register that writes each.  The
// displacement and weight are formed in FP64 and rounded to FP32, as in the
// VALU kernel; the monomials are x^a y^b z^c from per-lane exponents.
struct MfmaMomTab {
  int8_t id[3][4][64];  // moment written by (tile, register, lane), or -1
  int8_t ex[16][3], ex_hi[16][3];  // exponents of monomials c and 16 + c
};

constexpr MfmaMomTab make_mfma_mom_tab() {
  MfmaMomTab t{};
  bool done[NMOM] = {};
  for (int tile = 0; tile < 3; ++tile)
    for (int reg = 0; reg < 4; ++reg)
      for (int lane = 0; lane < 64; ++lane) t.id[tile][reg][lane] = -1;
  const int r0[3] = {0, 0, 16}, c0[3] = {0, 16, 16};
  for (int tile = 0; tile < 3; ++tile)
    for (int lane = 0; lane < 64; ++lane)
      for (int reg = 0; reg < 4; ++reg) {
        const int r = r0[tile] + 4 * (lane / 16) + reg, c = c0[tile] + lane % 16;
        if (r >= NBASIS || c >= NBASIS) continue;
        const int k = entry_moment(r, c);
        if (!done[k]) {
          done[k] = true;
          t.id[tile][reg][lane] = (int8_t)k;
        }
      }
  for (int c = 0; c < 16; ++c) {
    t.ex[c][0] = (int8_t)basis_expo(c).a;
    t.ex[c][1] = (int8_t)basis_expo(c).b;
    t.ex[c][2] = (int8_t)basis_expo(c).c;
    const int h = 16 + c < NBASIS ? 16 + c : 0;
    t.ex_hi[c][0] = (int8_t)(16 + c < NBASIS ? basis_expo(h).a : -1);
    t.ex_hi[c][1] = (int8_t)basis_expo(h).b;
    t.ex_hi[c][2] = (int8_t)basis_expo(h).c;
  }
  return t;
}

__constant__ MfmaMomTab c_mfma_tab = make_mfma_mom_tab();

// x^e for e in 0..3 from precomputed powers
__device__ __forceinline__ float pow3_sel(int e, float x, float x2, float x3) {
  return e == 0 ? 1.0f : (e == 1 ? x : (e == 2 ? x2 : x3));
}

__global__ void __launch_bounds__(THREADS)
    k_moments_mfma(int n, const double4* __restrict__ geo, const int64_t* __restrict__ off,
                   const int32_t* __restrict__ idx, Box box, double rf_ratio, int wkind,
                   double* __restrict__ mom, const int32_t* __restrict__ rows) {
  typedef float float4_t __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x & 63;
  const int i = __builtin_amdgcn_readfirstlane(xcd_block() * (THREADS / 64) + (threadIdx.x >> 6));
  if (i >= n) return;  // whole wavefronts
  const int c = lane & 15, k = lane >> 4;
  const int ea = c_mfma_tab.ex[c][0], eb = c_mfma_tab.ex[c][1], ec = c_mfma_tab.ex[c][2];
  const int ha = c_mfma_tab.ex_hi[c][0], hb = c_mfma_tab.ex_hi[c][1],
            hc = c_mfma_tab.ex_hi[c][2];
  const double4 gi = geo[rows ? rows[i] : i];
  const double inv_lam = 1.0 / gi.w;
  const double r = rf_ratio * gi.w;
  const double inv_r2 = 1.0 / (r * r);
  const int64_t s0 = off[i], s1 = off[i + 1];
  float4_t t00 = {0.f, 0.f, 0.f, 0.f}, t01 = t00, t11 = t00;
  for (int64_t g = s0; g < s1; g += 4) {
    const int64_t s = g + k;
    float w = 0.f, x = 0.f, y = 0.f, z = 0.f;
    if (s < s1) {
      const double4 gj = geo[idx[s]];
      const double dx = min_image(gj.x - gi.x, box.L[0], box.halfL[0], box.periodic[0]);
      const double dy = min_image(gj.y - gi.y, box.L[1], box.halfL[1], box.periodic[1]);
      const double dz = min_image(gj.z - gi.z, box.L[2], box.halfL[2], box.periodic[2]);
      w = (float)weight_of((dx * dx + dy * dy + dz * dz) * inv_r2, wkind);
      x = (float)(dx * inv_lam);
      y = (float)(dy * inv_lam);
      z = (float)(dz * inv_lam);
    }
    const float x2 = x * x, y2 = y * y, z2 = z * z;
    const float plo = pow3_sel(ea, x, x2, x2 * x) * pow3_sel(eb, y, y2, y2 * y) *
                      pow3_sel(ec, z, z2, z2 * z);
    const float phi = ha < 0 ? 0.0f
                             : pow3_sel(ha, x, x2, x2 * x) * pow3_sel(hb, y, y2, y2 * y) *
                                   pow3_sel(hc, z, z2, z2 * z);
    t00 = __builtin_amdgcn_mfma_f32_16x16x4f32(plo, w * plo, t00, 0, 0, 0);
    t01 = __builtin_amdgcn_mfma_f32_16x16x4f32(plo, w * phi, t01, 0, 0, 0);
    t11 = __builtin_amdgcn_mfma_f32_16x16x4f32(phi, w * phi, t11, 0, 0, 0);
  }
  const float4_t tl[3] = {t00, t01, t11};
#pragma unroll
  for (int tile = 0; tile < 3; ++tile)
#pragma unroll
    for (int reg = 0; reg < 4; ++reg) {
      const int m = c_mfma_tab.id[tile][reg][lane];
      if (m >= 0) mom[(int64_t)m * soa_ld(n) + i] = (double)tl[tile][reg];
    }
}

// ---------------------------------------------------------------------------
// 2. factor: equilibrated FP64 Cholesky, four lanes per particle
// ---------------------------------------------------------------------------
__constant__ EntryTab c_tab = make_entry_tab();

// Writes rows 1 .. NT of A^{-1} (the x, y, z monomials first) to
// gop[t][20][n], and the status.  Screen (list != null): a particle with
// status 0 whose equilibrated inverse has a row among the first nscreen
// operator rows of 2-norm above rcut is appended to list (its operator form
// would lose more than the fit's own accuracy; the refinement solves it
// again).
template <int NT>
__global__ void __launch_bounds__(THREADS)
    k_factor(int n, const double* __restrict__ mom, const int64_t* __restrict__ off,
             double* __restrict__ gop, int32_t* __restrict__ status, int interp, int nscreen,
             double rcut, int32_t* __restrict__ list, int32_t* __restrict__ count) {
  const int tid = blockIdx.x * THREADS + threadIdx.x;
  const int i = tid >> 2;
  const int l = tid & 3;
  const bool valid = i < n;
  const int ii = valid ? i : n - 1;
  QuadChol c;
  quad_chol_factor(c, c_tab, mom, soa_ld(n), ii, l, interp != 0);
  const int st = quad_chol_status(c, (int)(off[ii + 1] - off[ii]));
  double rmax2 = 0.0;
  // rows in lockstep groups of three
  sfor<0, NT / 3>([&](auto GI) {
    constexpr int t0 = 1 + 3 * GI;
    double rows[3][5];
    quad_chol_inverse_rows<t0, 3>(c, l, rows);
    if (valid) {
      sfor<0, 3>([&](auto RI) {
        sfor<0, 5>([&](auto R) {
          constexpr int rho = R;
          gop[((int64_t)(3 * GI + RI) * NBASIS + 4 * rho + l) * soa_ld(n) + i] = rows[RI][rho];
        });
      });
    }
    if (list && 3 * GI < nscreen) rmax2 = fmax(rmax2, quad_rows_hat_norm2<t0, 3>(c, l, rows));
  });
  if (valid && l == 0) {
    status[i] = st;
    if (list && st == 0 && !(rmax2 <= rcut * rcut)) list[atomicAdd(count, 1)] = i;
  }
}

// ---------------------------------------------------------------------------
// 2b. data form: right-hand-side moments, the full fit and its tape
// ---------------------------------------------------------------------------
// B_f[b] = sum_j w_j p_b(xi_j) (f_j - f_i) for the NF fields of the packed
// records fq[8 j + 8 - NF + f].  Eight lanes per particle: lane S h + e
// (S = FPL slots) takes the fields FPL h .. FPL h + FPL - 1 for the entries
// e, e + S, ...: FPL x 20 accumulators per lane.  FPL = 4 forms each entry's
// monomials twice per particle, FPL = 2 four times with half the registers.
// The slots' partial sums meet in a reduce-scatter (each slot ends with the
// coefficients it stores).  The next entry's record is fetched one iteration
// ahead, its index two ahead.
// At least two wavefronts per SIMD: unconstrained, the allocator parks one
// value live across the loop in an accumulation register, and the 257
// registers halve the occupancy; held to 256 it keeps that value in 8 bytes
// of scratch, written once before the loop and read once after it.
template <int NF, int FPL>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(2)))
    k_fit_b(int n, const double4* __restrict__ geo, const double* __restrict__ fq,
            const int64_t* __restrict__ off, const int32_t* __restrict__ idx, Box box,
            double rf_ratio, int wkind, const int32_t* __restrict__ rows,
            double* __restrict__ bout) {
  constexpr int S = FPL, G = 8, F0 = 8 - NF;
  static_assert(G / S * FPL >= NF, "field groups");
  const int tid = xcd_block() * THREADS + threadIdx.x;
  const int i = tid / G;
  const int l = tid % G;
  const int h = l / S, e = l % S;
  const bool valid = i < n;
  const int ii = valid ? i : n - 1;
  const int me = rows ? rows[ii] : ii;  // row ii's own particle
  const double4 gi = geo[me];
  const double inv_lam = 1.0 / gi.w;
  const double r = rf_ratio * gi.w;
  const double inv_r2 = 1.0 / (r * r);
  const int fb = F0 + FPL * h;  // this group's first field record
  const int nfh = NF - FPL * h < FPL ? NF - FPL * h : FPL;
  double fi[FPL];
#pragma unroll
  for (int c = 0; c < FPL; ++c) fi[c] = c < nfh ? fq[8 * (int64_t)me + fb + c] : 0.0;
  double acc[FPL][NBASIS];
#pragma unroll
  for (int c = 0; c < FPL; ++c)
#pragma unroll
    for (int b = 0; b < NBASIS; ++b) acc[c][b] = 0.0;
  const int64_t s1 = valid ? off[ii + 1] : off[ii];
  int64_t s = off[ii] + e;
  double4 gn = gi;
  double vn[FPL];
#pragma unroll
  for (int c = 0; c < FPL; ++c) vn[c] = fi[c];
  int jn = me;
  if (s < s1) {
    const int j = idx[s];
    gn = geo[j];
#pragma unroll
    for (int c = 0; c < FPL; ++c) vn[c] = c < nfh ? fq[8 * (int64_t)j + fb + c] : 0.0;
  }
  if (s + S < s1) jn = idx[s + S];
  for (; s < s1; s += S) {
    const double4 gj = gn;
    double vj[FPL];
#pragma unroll
    for (int c = 0; c < FPL; ++c) vj[c] = vn[c];
    if (s + S < s1) {
      gn = geo[jn];
#pragma unroll
      for (int c = 0; c < FPL; ++c) vn[c] = c < nfh ? fq[8 * (int64_t)jn + fb + c] : 0.0;
      if (s + 2 * S < s1) jn = idx[s + 2 * S];
    }
    const double dx = min_image(gj.x - gi.x, box.L[0], box.halfL[0], box.periodic[0]);
    const double dy = min_image(gj.y - gi.y, box.L[1], box.halfL[1], box.periodic[1]);
    const double dz = min_image(gj.z - gi.z, box.L[2], box.halfL[2], box.periodic[2]);
    const double w = weight_of((dx * dx + dy * dy + dz * dz) * inv_r2, wkind);
    double p[NBASIS];
    basis(p, dx * inv_lam, dy * inv_lam, dz * inv_lam);
#pragma unroll
    for (int c = 0; c < FPL; ++c) {
      const double d = w * (vj[c] - fi[c]);
#pragma unroll
      for (int b = 0; b < NBASIS; ++b) acc[c][b] = fma(d, p[b], acc[c][b]);
    }
  }
  // slot e ends with the sums of flat index S m + e: field m / (20 / S),
  // coefficient S (m % (20 / S)) + e
  constexpr int PER = NBASIS / S;
  static_assert(NBASIS % S == 0, "coefficients split evenly over the slots");
  double mine[FPL * PER];
  group_reduce_scatter<S, FPL * NBASIS>(&acc[0][0], mine, e);
  if (valid) {
    const int64_t ld = soa_ld(n);
    double* dst = bout + ((int64_t)FPL * h * NBASIS + e) * ld + i;
#pragma unroll
    for (int m = 0; m < FPL * PER; ++m)
      if (m / PER < nfh) dst[(int64_t)((m / PER) * NBASIS + S * (m % PER)) * ld] = mine[m];
  }
}

// The FP64 moments and the data-form factor in one kernel.  Four lanes per
// particle sum the 84 moments as k_moments<4, double> does (the same sums,
// bit for bit) and leave them in LDS; the quad then factors A from there:
// equilibrated Cholesky, the status, rows 1..NT of A^{-1} (the screen of
// k_factor; with a tape also its G) and C_f = A^{-1} B_f for the
// NT == 9 ? 8 : 7 fields in lockstep pairs.  The derivative rows of C
// (coefficients 1..NT) go in place over B as [NF][NT][ld] (each quad reads a
// pair's B before it writes that pair's rows, which lie below every later
// pair's B), all of C to the tape.  Failed fits write zeros.  Interpolating
// fit: the constant's row and column are the identity's, B's constant entry
// is dropped and C's stays zero.  Only the particles listed for refinement
// write their moments to mom (the refinement reads them), so the moments
// make no round trip through HBM.
template <int NT>
__global__ void __launch_bounds__(THREADS)
    k_moments_factor_fit(int n, const double4* __restrict__ geo, const int64_t* __restrict__ off,
                         const int32_t* __restrict__ idx, Box box, double rf_ratio, int wkind,
                         const int32_t* __restrict__ rows, double* __restrict__ mom, double* bc,
                         double* __restrict__ aos, int32_t* __restrict__ status, int interp,
                         double rcut, int32_t* __restrict__ list, int32_t* __restrict__ count) {
  constexpr int NF = NT == 9 ? 8 : 7;
  constexpr int LEN = TAPE_AOS, COFF = NT * NBASIS, G = 4, PW = 64 / G;
  __shared__ double smom[THREADS / 64][NMOM][PW];
  const int tid = xcd_block() * THREADS + threadIdx.x;
  const int i = tid / G;
  const int l = tid % G;
  const int wv = threadIdx.x >> 6, p = (threadIdx.x & 63) / G;  // particle within the wavefront
  const bool valid = i < n;
  const int ii = valid ? i : n - 1;
  {
    double m[NMOM];
#pragma unroll
    for (int k = 0; k < NMOM; ++k) m[k] = 0.0;
    const double4 gi = geo[rows ? rows[ii] : ii];  // row ii's own particle
    const double inv_lam = 1.0 / gi.w;
    const double r = rf_ratio * gi.w;
    const double inv_r2 = 1.0 / (r * r);
    const int64_t s0 = off[ii], s1 = valid ? off[ii + 1] : s0;
    int64_t s = s0 + l;
    double4 gn = gi;
    int jn = 0;
    if (s < s1) gn = geo[idx[s]];
    if (s + G < s1) jn = idx[s + G];
    for (; s < s1; s += G) {
      const double4 gj = gn;
      if (s + G < s1) {
        gn = geo[jn];
        if (s + 2 * G < s1) jn = idx[s + 2 * G];
      }
      const double dx = min_image(gj.x - gi.x, box.L[0], box.halfL[0], box.periodic[0]);
      const double dy = min_image(gj.y - gi.y, box.L[1], box.halfL[1], box.periodic[1]);
      const double dz = min_image(gj.z - gi.z, box.L[2], box.halfL[2], box.periodic[2]);
      const double qd = (dx * dx + dy * dy + dz * dz) * inv_r2;
      const double w = weight_of(qd, wkind);
      accumulate_moments(m, w, dx * inv_lam, dy * inv_lam, dz * inv_lam);
    }
    double mine[NMOM / G];
    group_reduce_scatter<G, NMOM>(m, mine, l);
#pragma unroll
    for (int k = 0; k < NMOM / G; ++k) smom[wv][l + G * k][p] = mine[k];
  }
  // each wavefront reads only its own particles' moments
  wave_lds_sync();
  QuadChol c;
  quad_chol_factor(c, c_tab, &smom[wv][0][0], PW, p, l, interp != 0);
  const int st = quad_chol_status(c, (int)(off[ii + 1] - off[ii]));
  double* rec = (aos && valid) ? aos + (int64_t)i * LEN : nullptr;
  double rmax2 = 0.0;
  sfor<0, NT / 3>([&](auto GI) {
    constexpr int t0 = 1 + 3 * GI;
    double rws[3][5];
    quad_chol_inverse_rows<t0, 3>(c, l, rws);
    if (rec) {
      sfor<0, 3>([&](auto RI) {
        sfor<0, 5>([&](auto R) {
          constexpr int rho = R;
          rec[(3 * GI + RI) * NBASIS + 4 * rho + l] = st == 0 ? rws[RI][rho] : 0.0;
        });
      });
    }
    if (list) rmax2 = fmax(rmax2, quad_rows_hat_norm2<t0, 3>(c, l, rws));
  });
  constexpr int LS = 2;  // lockstep solves: two keep the kernel within 256 VGPRs
  for (int f0 = 0; f0 < NF; f0 += LS) {
    double y[LS][5], x[LS][5];
#pragma unroll
    for (int r = 0; r < LS; ++r)
#pragma unroll
      for (int rho = 0; rho < 5; ++rho) {
        const double b =
            f0 + r < NF ? bc[((int64_t)(f0 + r) * NBASIS + 4 * rho + l) * soa_ld(n) + ii] : 0.0;
        y[r][rho] = (interp && rho == 0 && l == 0) ? 0.0 : b * c.s_own[rho];
      }
    quad_chol_solve_n<0, LS>(c, l, y, x);
    if (valid) {
#pragma unroll
      for (int r = 0; r < LS; ++r) {
        if (f0 + r >= NF) break;
#pragma unroll
        for (int rho = 0; rho < 5; ++rho) {
          const double v = st == 0 ? x[r][rho] * c.s_own[rho] : 0.0;
          const int cf = 4 * rho + l;  // coefficient index
          if (cf >= 1 && cf <= NT) bc[((int64_t)(f0 + r) * NT + cf - 1) * soa_ld(n) + i] = v;
          if (rec) rec[COFF + (f0 + r) * NBASIS + cf] = v;
        }
      }
    }
  }
  // the quad agrees on the status and on the screen (rmax2 is a quad sum)
  const bool listed = valid && list && st == 0 && !(rmax2 <= rcut * rcut);
  if (listed) {
#pragma unroll
    for (int k = 0; k < NMOM / G; ++k)
      mom[(int64_t)(l + G * k) * soa_ld(n) + i] = smom[wv][l + G * k][p];
  }
  if (valid && l == 0) {
    status[i] = st;
    if (listed) list[atomicAdd(count, 1)] = i;
  }
}

// ---------------------------------------------------------------------------
// 3a. derivatives of up to 8 fields for three operator rows
// ---------------------------------------------------------------------------
constexpr int FCHUNK = 8;

// CT as in k_apply_rhs (float: the mixed form's FP32 application of operator
// weights formed in FP64).
template <int G, class CT = double>
__global__ void __launch_bounds__(THREADS)
    k_apply_derivs(int n, const double* __restrict__ pos, const double* __restrict__ lam,
                   const int64_t* __restrict__ off, const int32_t* __restrict__ idx, Box box,
                   double rf_ratio, int wkind, const double* __restrict__ gop, int row0,
                   const int32_t* __restrict__ status, int nf, int f0,
                   const double* __restrict__ fields, double* __restrict__ out, int out_comp,
                   int comp0, double c0, double c1, double c2, int power,
                   const int32_t* __restrict__ list, const int32_t* __restrict__ count) {
  // list form: only the particles list[0 .. *count) (count read on the
  // device); the launch covers n, and the first blocks the list needs keep
  // the XCD-aware order among themselves
  const int m = count ? *count : n;
  const int nbk = count ? (m + THREADS / G - 1) / (THREADS / G) : (int)gridDim.x;
  if ((int)blockIdx.x >= nbk) return;
  const int tid = xcd_block_of(blockIdx.x, nbk) * THREADS + threadIdx.x;
  const int i = tid / G;
  const int l = tid % G;
  const bool valid = i < m;
  const int ii = list ? list[valid ? i : m - 1] : (valid ? i : m - 1);
  const int st = status[ii];
  double g[3][NBASIS];
#pragma unroll
  for (int t = 0; t < 3; ++t)
#pragma unroll
    for (int b = 0; b < NBASIS; ++b) g[t][b] = gop[((int64_t)(row0 + t) * NBASIS + b) * soa_ld(n) + ii];
  const int nfc = (nf - f0) < FCHUNK ? (nf - f0) : FCHUNK;
  double fi[FCHUNK];
#pragma unroll
  for (int f = 0; f < FCHUNK; ++f) fi[f] = f < nfc ? fields[(int64_t)(f0 + f) * n + ii] : 0.0;
  const double xi = pos[ii], yi = pos[(int64_t)n + ii], zi = pos[2 * (int64_t)n + ii];
  const double li = lam[ii];
  const double inv_lam = 1.0 / li;
  const double r = rf_ratio * li;
  const double inv_r2 = 1.0 / (r * r);
  CT acc[FCHUNK][3];
#pragma unroll
  for (int f = 0; f < FCHUNK; ++f)
#pragma unroll
    for (int t = 0; t < 3; ++t) acc[f][t] = CT(0);
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
    CT gam[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      double v = 0.0;
#pragma unroll
      for (int b = 0; b < NBASIS; ++b) v = fma(g[t][b], p[b], v);
      gam[t] = CT(w * v);
    }
#pragma unroll
    for (int f = 0; f < FCHUNK; ++f) {
      if (f < nfc) {
        const CT df = CT(fields[(int64_t)(f0 + f) * n + j] - fi[f]);
#pragma unroll
        for (int t = 0; t < 3; ++t) acc[f][t] = fma(gam[t], df, acc[f][t]);
      }
    }
  }
  double sum[FCHUNK][3];
#pragma unroll
  for (int f = 0; f < FCHUNK; ++f)
#pragma unroll
    for (int t = 0; t < 3; ++t) sum[f][t] = group_sum<G>(widen(acc[f][t]));
  if (valid && l == 0) {
    const double scale = power == 1 ? inv_lam : inv_lam * inv_lam;
    const double cf[3] = {c0, c1, c2};
    const double nan = __longlong_as_double(0x7ff8000000000000LL);
    for (int f = 0; f < nfc; ++f)
      for (int t = 0; t < 3; ++t)
        out[((int64_t)(f0 + f) * out_comp + comp0 + t) * n + ii] =
            st == 0 ? cf[t] * sum[f][t] * scale : nan;
  }
}

// ---------------------------------------------------------------------------
// 3b. MHD time derivatives
// ---------------------------------------------------------------------------
// Ideal form: the three gradient rows applied to V, B and sigma.  STAB (the
// non-ideal stabilisers): nine rows (gradient, then xx, xy, xz, yy, yz, zz)
// applied to all eight fields' gradients (rho's feeds the change sensor) and
// to grad div V and grad div B, whose entry terms are
//   d_a div V  <-  sum_b h_ab (V_b,j - V_b,i),   h_ab = w row_(ab) . p_j
// with the diagonal rows doubled (d^2/dx_a^2 = 2 c_aa / lambda^2).
// CT: the arithmetic of the field application.  double; float in the mixed
// form, where each operator weight gamma_j is formed in FP64 and rounded once
// (in FP32 its rounding would be amplified by the cancellation inside
// G . p_j, which grows with the condition of the moment matrix), the field
// differences are formed in FP64 and rounded once, the sums over neighbors
// are FP32, and the lanes' partial sums meet in FP64.
template <int G, bool STAB, class CT = double>
__global__ void __launch_bounds__(THREADS)
    __attribute__((amdgpu_waves_per_eu(!STAB && sizeof(CT) == 4 ? 4 : 1)))
    k_apply_rhs(int n, const double4* __restrict__ geo, const double* __restrict__ fq,
                const int64_t* __restrict__ off, const int32_t* __restrict__ idx, Box box,
                double rf_ratio, int wkind, double gamma, Stab sb, const double* __restrict__ gop,
                const int32_t* __restrict__ status, double* __restrict__ rhs,
                double* __restrict__ dxdt, double* __restrict__ tape,
                const int32_t* __restrict__ rows, const int32_t* __restrict__ list,
                const int32_t* __restrict__ count) {
  constexpr int NR = STAB ? 9 : 3;  // operator rows
  constexpr int NF = STAB ? 8 : 7;  // fields with a gradient: the last NF of eight
  constexpr int F0 = 8 - NF;
  constexpr int PPB = THREADS / G;
  // List form: only the particles list[0 .. *count) (count read on the
  // device).  The launch covers n; the first blocks the list needs keep the
  // XCD-aware order among themselves, the rest leave (before the barrier,
  // whole blocks together).
  const int m = count ? *count : n;
  const int nbk = count ? (m + PPB - 1) / PPB : (int)gridDim.x;
  if ((int)blockIdx.x >= nbk) return;
  const int tid = xcd_block_of(blockIdx.x, nbk) * THREADS + threadIdx.x;
  const int i = tid / G;
  const int l = tid % G;
  const bool valid = i < m;
  const int ii = list ? list[valid ? i : m - 1] : (valid ? i : m - 1);
  const int st = status[ii];
  // The particle's operator rows live in LDS, not in each lane's registers:
  // gsh[k][pl] holds entries 2k, 2k+1, and one 16-byte read serves all lanes
  // of a particle (consecutive particles, consecutive addresses: no bank
  // conflicts).
  __shared__ double2 gsh[NR * NBASIS / 2][PPB];
  const int pl = threadIdx.x / G;
  // The lane's own data and its first neighbor entry are fetched before the
  // rows are staged, so that their latency overlaps the staging and the
  // barrier.
  const int me = rows ? rows[ii] : ii;  // row ii's own particle
  const double4 gi = geo[me];
  const int64_t s0 = off[ii], s1 = (valid && st == 0) ? off[ii + 1] : s0;
  int64_t s = s0 + l;
  int jc = me, jn = me;
  double4 gn = gi;
  if (s < s1) {
    jc = idx[s];
    gn = geo[jc];
  }
  if (s + G < s1) jn = idx[s + G];
  double qi[8];
  load_fields(fq, me, qi);
  for (int k = l; k < NR * NBASIS / 2; k += G) {
    const int t = (2 * k) / NBASIS, b = (2 * k) % NBASIS;
    const double sc = (STAB && (t == 3 || t == 6 || t == 8)) ? 2.0 : 1.0;
    gsh[k][pl] = make_double2(sc * gop[((int64_t)t * NBASIS + b) * soa_ld(n) + ii],
                              sc * gop[((int64_t)t * NBASIS + b + 1) * soa_ld(n) + ii]);
  }
  __syncthreads();
  const double inv_lam = 1.0 / gi.w;
  const double r = rf_ratio * gi.w;
  const double inv_r2 = 1.0 / (r * r);
  CT acc[NF][3];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int t = 0; t < 3; ++t) acc[f][t] = CT(0);
  CT adv[3] = {CT(0), CT(0), CT(0)}, adb[3] = {CT(0), CT(0), CT(0)};
  for (; s < s1; s += G) {
    const double4 gj = gn;
    const int j = jc;
    if (s + G < s1) {
      gn = geo[jn];
      jc = jn;
      if (s + 2 * G < s1) jn = idx[s + 2 * G];
    }
    double qj[8];
    load_fields(fq, j, qj);
    const double dx = min_image(gj.x - gi.x, box.L[0], box.halfL[0], box.periodic[0]);
    const double dy = min_image(gj.y - gi.y, box.L[1], box.halfL[1], box.periodic[1]);
    const double dz = min_image(gj.z - gi.z, box.L[2], box.halfL[2], box.periodic[2]);
    const double w = weight_of((dx * dx + dy * dy + dz * dz) * inv_r2, wkind);
    double p[NBASIS];
    basis(p, dx * inv_lam, dy * inv_lam, dz * inv_lam);
    CT gam[NR];
    // re-read the rows from LDS every iteration: hoisted out of the loop they
    // would occupy registers again
    asm volatile("" ::: "memory");
#pragma unroll
    for (int t = 0; t < NR; ++t) {
      double v = 0.0;
#pragma unroll
      for (int b = 0; b < NBASIS; b += 2) {
        const double2 gg = gsh[(t * NBASIS + b) / 2][pl];
        v = fma(gg.x, p[b], v);
        v = fma(gg.y, p[b + 1], v);
      }
      gam[t] = CT(w * v);
    }
    CT df[8];
#pragma unroll
    for (int f = F0; f < 8; ++f) df[f] = CT(qj[f] - qi[f]);
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int t = 0; t < 3; ++t) acc[f][t] = fma(gam[t], df[F0 + f], acc[f][t]);
    if constexpr (STAB) {
      // rows 3..8 = xx, xy, xz, yy, yz, zz
      adv[0] += gam[3] * df[1] + gam[4] * df[2] + gam[5] * df[3];
      adv[1] += gam[4] * df[1] + gam[6] * df[2] + gam[7] * df[3];
      adv[2] += gam[5] * df[1] + gam[7] * df[2] + gam[8] * df[3];
      adb[0] += gam[3] * df[4] + gam[4] * df[5] + gam[5] * df[6];
      adb[1] += gam[4] * df[4] + gam[6] * df[5] + gam[7] * df[6];
      adb[2] += gam[5] * df[4] + gam[7] * df[5] + gam[8] * df[6];
    }
  }
  double grad[NF][3];
#pragma unroll
  for (int f = 0; f < NF; ++f)
#pragma unroll
    for (int t = 0; t < 3; ++t) grad[f][t] = group_sum<G>(widen(acc[f][t])) * inv_lam;
  double gdv[3] = {0.0, 0.0, 0.0}, gdb[3] = {0.0, 0.0, 0.0};
  if constexpr (STAB) {
    const double il2 = inv_lam * inv_lam;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      gdv[a] = group_sum<G>(double(adv[a])) * il2;
      gdb[a] = group_sum<G>(double(adb[a])) * il2;
    }
  }
  if (valid && l == 0) {
    double g7[7][3];
#pragma unroll
    for (int f = 0; f < 7; ++f)
#pragma unroll
      for (int t = 0; t < 3; ++t) g7[f][t] = grad[NF - 7 + f][t];
    double out[8];
    if (st == 0) {
      mhd_point(qi, g7, gamma, out);
      if constexpr (STAB) {
        const double grho[3] = {grad[0][0], grad[0][1], grad[0][2]};
        stab_point(qi, grho, g7[0][0] + g7[1][1] + g7[2][2], gdv, gdb, gi.w, gamma, sb, out);
      }
    } else {
      const double nan = __longlong_as_double(0x7ff8000000000000LL);
#pragma unroll
      for (int f = 0; f < 8; ++f) out[f] = nan;
    }
#pragma unroll
    for (int f = 0; f < 8; ++f) rhs[(int64_t)f * n + ii] = out[f];
#pragma unroll
    for (int a = 0; a < 3; ++a) dxdt[(int64_t)a * n + ii] = qi[1 + a];
    if (tape) {  // what the reverse mode reuses (layout in mls.hpp)
#pragma unroll
      for (int f = 0; f < 7; ++f)
#pragma unroll
        for (int t = 0; t < 3; ++t) tape[((int64_t)f * 3 + t) * soa_ld(n) + ii] = g7[f][t];
      tape[(int64_t)TAPE_STATUS * soa_ld(n) + ii] = (double)st;
      if constexpr (STAB) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          tape[(int64_t)(TAPE_GRHO + a) * soa_ld(n) + ii] = grad[0][a];
          tape[(int64_t)(TAPE_GDV + a) * soa_ld(n) + ii] = gdv[a];
          tape[(int64_t)(TAPE_GDB + a) * soa_ld(n) + ii] = gdb[a];
        }
      }
    }
  }
}

template <int G, class T>
hipError_t launch_moments_g(hipStream_t s, const EvalArgs& a, double* mom) {
  hipLaunchKernelGGL((k_moments<G, T>), dim3(grid_for((int64_t)a.n * G, THREADS)), dim3(THREADS), 0,
                     s, a.n, a.geo, a.off, a.idx, a.box, a.rf_ratio, a.wkind, mom, a.rows);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_moments(hipStream_t s, const EvalArgs& a, int lanes, double* mom, bool fp32) {
  if (fp32) {
    if (lanes == 0) {
      hipLaunchKernelGGL(k_moments_mfma, dim3(grid_for((int64_t)a.n * 64, THREADS)),
                         dim3(THREADS), 0, s, a.n, a.geo, a.off, a.idx, a.box, a.rf_ratio, a.wkind,
                         mom, a.rows);
      return hipGetLastError();
    }
    switch (lanes) {
      case 1: return launch_moments_g<1, float>(s, a, mom);
      case 2: return launch_moments_g<2, float>(s, a, mom);
      default: return launch_moments_g<4, float>(s, a, mom);
    }
  }
  switch (lanes) {
    case 1: return launch_moments_g<1, double>(s, a, mom);
    case 2: return launch_moments_g<2, double>(s, a, mom);
    default: return launch_moments_g<4, double>(s, a, mom);
  }
}

hipError_t launch_factor(hipStream_t s, const EvalArgs& a, int ntargets, const double* mom,
                         double* gop, int32_t* status, int nscreen, double rcut, int32_t* list,
                         int32_t* count) {
  const unsigned grid = grid_for((int64_t)a.n * 4, THREADS);
  const int interp = a.fit == PHB_FIT_INTERP19;
  if (ntargets == 3)
    hipLaunchKernelGGL((k_factor<3>), dim3(grid), dim3(THREADS), 0, s, a.n, mom, a.off, gop, status,
                       interp, nscreen, rcut, list, count);
  else
    hipLaunchKernelGGL((k_factor<9>), dim3(grid), dim3(THREADS), 0, s, a.n, mom, a.off, gop, status,
                       interp, nscreen, rcut, list, count);
  return hipGetLastError();
}

hipError_t launch_fit_b(hipStream_t s, const EvalArgs& a, int nf, int fpl, double* bout) {
  const unsigned grid = grid_for((int64_t)a.n * 8, THREADS);
#define PHB_FIT_B(NF, FPL)                                                                    \
  hipLaunchKernelGGL((k_fit_b<NF, FPL>), dim3(grid), dim3(THREADS), 0, s, a.n, a.geo, a.fq,   \
                     a.off, a.idx, a.box, a.rf_ratio, a.wkind, a.rows, bout)
  if (nf == 8) {
    if (fpl == 2) PHB_FIT_B(8, 2); else PHB_FIT_B(8, 4);
  } else {
    if (fpl == 2) PHB_FIT_B(7, 2); else PHB_FIT_B(7, 4);
  }
#undef PHB_FIT_B
  return hipGetLastError();
}

hipError_t launch_moments_factor_fit(hipStream_t s, const EvalArgs& a, int nrows, double* mom,
                                     double* bc, double* aos, int32_t* status, double rcut,
                                     int32_t* list, int32_t* count) {
  const unsigned grid = grid_for((int64_t)a.n * 4, THREADS);
  const int interp = a.fit == PHB_FIT_INTERP19;
  if (nrows == 3)
    hipLaunchKernelGGL((k_moments_factor_fit<3>), dim3(grid), dim3(THREADS), 0, s, a.n, a.geo,
                       a.off, a.idx, a.box, a.rf_ratio, a.wkind, a.rows, mom, bc, aos, status,
                       interp, rcut, list, count);
  else
    hipLaunchKernelGGL((k_moments_factor_fit<9>), dim3(grid), dim3(THREADS), 0, s, a.n, a.geo,
                       a.off, a.idx, a.box, a.rf_ratio, a.wkind, a.rows, mom, bc, aos, status,
                       interp, rcut, list, count);
  return hipGetLastError();
}

template <int G, class CT>
static hipError_t derivs_g(hipStream_t s, const EvalArgs& a, const double* gop,
                           const int32_t* status, int nf, const double* fields, double* d1,
                           double* d2, const int32_t* list, const int32_t* count) {
  const unsigned grid = grid_for((int64_t)a.n * G, THREADS);
  for (int f0 = 0; f0 < nf; f0 += FCHUNK) {
    hipLaunchKernelGGL((k_apply_derivs<G, CT>), dim3(grid), dim3(THREADS), 0, s, a.n, a.pos, a.lam,
                       a.off, a.idx, a.box, a.rf_ratio, a.wkind, gop, 0, status, nf, f0, fields,
                       d1, 3, 0, 1.0, 1.0, 1.0, 1, list, count);
    if (d2) {
      // rows 4..6: xx (2 c), xy, xz ; rows 7..9: yy (2 c), yz, zz (2 c)
      hipLaunchKernelGGL((k_apply_derivs<G, CT>), dim3(grid), dim3(THREADS), 0, s, a.n, a.pos, a.lam,
                         a.off, a.idx, a.box, a.rf_ratio, a.wkind, gop, 3, status, nf, f0, fields,
                         d2, 6, 0, 2.0, 1.0, 1.0, 2, list, count);
      hipLaunchKernelGGL((k_apply_derivs<G, CT>), dim3(grid), dim3(THREADS), 0, s, a.n, a.pos, a.lam,
                         a.off, a.idx, a.box, a.rf_ratio, a.wkind, gop, 6, status, nf, f0, fields,
                         d2, 6, 3, 2.0, 1.0, 2.0, 2, list, count);
    }
  }
  return hipGetLastError();
}

hipError_t launch_apply_derivs(hipStream_t s, const EvalArgs& a, int lanes, const double* gop,
                               const int32_t* status, int nf, const double* fields, double* d1,
                               double* d2, bool fp32, const int32_t* list, const int32_t* count) {
  if (fp32) {
    switch (lanes) {
      case 1: return derivs_g<1, float>(s, a, gop, status, nf, fields, d1, d2, list, count);
      case 2: return derivs_g<2, float>(s, a, gop, status, nf, fields, d1, d2, list, count);
      default: return derivs_g<4, float>(s, a, gop, status, nf, fields, d1, d2, list, count);
    }
  }
  switch (lanes) {
    case 1: return derivs_g<1, double>(s, a, gop, status, nf, fields, d1, d2, list, count);
    case 2: return derivs_g<2, double>(s, a, gop, status, nf, fields, d1, d2, list, count);
    default: return derivs_g<4, double>(s, a, gop, status, nf, fields, d1, d2, list, count);
  }
}

template <int G, bool STAB, class CT = double>
static hipError_t rhs_g(hipStream_t s, const EvalArgs& a, double gamma, const Stab& sb,
                        const double* gop, const int32_t* status, double* rhs, double* dxdt,
                        double* tape, const int32_t* list, const int32_t* count) {
  hipLaunchKernelGGL((k_apply_rhs<G, STAB, CT>), dim3(grid_for((int64_t)a.n * G, THREADS)),
                     dim3(THREADS), 0, s, a.n, a.geo, a.fq, a.off, a.idx, a.box, a.rf_ratio,
                     a.wkind, gamma, sb, gop, status, rhs, dxdt, tape, a.rows, list, count);
  return hipGetLastError();
}

hipError_t launch_pack(hipStream_t s, int n, const double* pos, const double* lam,
                       const double* q, double4* geo, double* fq) {
  hipLaunchKernelGGL(k_pack, dim3(grid_for(n, THREADS)), dim3(THREADS), 0, s, n, pos, lam, q, geo,
                     fq);
  return hipGetLastError();
}

hipError_t launch_apply_rhs(hipStream_t s, const EvalArgs& a, int lanes, double gamma,
                            const Stab& sb, const double* gop, const int32_t* status, double* rhs,
                            double* dxdt, double* tape, const int32_t* list,
                            const int32_t* count) {
  // nine LDS rows per particle: eight lanes per particle keep a block's rows
  // small enough for several blocks per CU
  if (sb.on()) return rhs_g<8, true, float>(s, a, gamma, sb, gop, status, rhs, dxdt, tape, list, count);
  switch (lanes) {
    case 1: return rhs_g<1, false, float>(s, a, gamma, sb, gop, status, rhs, dxdt, tape, list, count);
    case 2: return rhs_g<2, false, float>(s, a, gamma, sb, gop, status, rhs, dxdt, tape, list, count);
    default: return rhs_g<4, false, float>(s, a, gamma, sb, gop, status, rhs, dxdt, tape, list, count);
  }
}

}  // namespace phb
