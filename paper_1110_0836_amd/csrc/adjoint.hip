// Reverse mode of the MLS / ideal-MHD time derivatives with the neighbor
// lists held fixed.
//
// Forward, per particle i (data form): A = sum_j w_j p_j p_j^T, B_f = sum_j
// w_j p_j (f_j - f_i), C_f = A^{-1} B_f, the derivatives from C's rows 1..NR,
// then the pointwise right-hand side.  The tape keeps G (rows 1..NR of
// A^{-1}) and C per particle.
//
// Reverse, per particle i:
//   1. pointwise adjoint of the right-hand side: qbar_i (direct part) and
//      Ubar = grad_bar / lambda  (NR x NFA, coefficient space);
//   2. K = Ubar C^T  (NR x 20; with C = A^{-1} B this is (A^{-1} Y)^T for
//      Y = sum_j w_j p_j (Ubar df_j)^T, without forming Y or factoring A
//      again), so the adjoint of A is  Abar = -G^T K  and of B is
//      Bbar = G^T Ubar;
//   3. for each neighbor: a = G p, h = Ubar df, b = h - K p,
//        wbar  = a . b,
//        pbar  = w (G^T b - K^T a),  xibar = (dp/dxi)^T pbar,
//        dfbar = w Ubar^T a,
//        dbar  = xibar / lambda + wbar (dw/dq) 2 d / r_f^2,
//      and the pair contributes +dfbar, +dbar to j and -dfbar, -dbar to i;
//   4. every particle sums the pair records addressed to it (the transposed
//      lists), in a fixed order, plus its own terms.  No atomics.  Under the
//      tile schedule (the default) the pairs whose target lies in the
//      owner's tile of consecutive particles are summed on chip instead and
//      arrive with the particle's own terms.
#include <type_traits>

#include "adjoint.hpp"
#include "chol.hpp"
#include "mhd.hpp"
#include "neighbors.hpp"
#include "refine.hpp"

namespace phb {
namespace {

constexpr int THREADS = 256;
// Shapes of the reverse pass.  Ideal MHD: three operator rows (the gradient)
// applied to V, B and sigma.  With the stabilisers: nine rows (the gradient,
// then xx, xy, xz, yy, yz, zz) applied to all eight fields (rho's gradient
// feeds the sensor).  Per-owner record of the pair kernel: G (NR x 20) at 0,
// K (NR x 20) at KOFF, Ubar [NFA][NR] at UOFF; one 1152-byte block per
// particle in the ideal shape, 3456 bytes with the stabilisers.  Pair record:
// dfbar (NFA), dbar (3), padded to an even count for paired stores.
template <bool STAB>
struct Shape {
  static constexpr int NR = STAB ? 9 : 3;
  static constexpr int NFA = STAB ? 8 : 7;
  static constexpr int F0 = 8 - NFA;
  static constexpr int REC = STAB ? 12 : 10;
  static constexpr int KOFF = NR * NBASIS;
  static constexpr int UOFF = 2 * NR * NBASIS;
  static constexpr int OREC = STAB ? 432 : 144;
  static_assert(UOFF + NFA * NR <= OREC && NFA + 3 <= REC && REC % 2 == 0, "record shape");
};
// the ideal shape, used by the lane-per-entry schedule
constexpr int REC = Shape<false>::REC;
constexpr int OREC = Shape<false>::OREC;
constexpr int UOFF = Shape<false>::UOFF;
constexpr int PAIRS_PER_BLOCK = 256;

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
    for (int t = 0; t < 3; ++t) grad[f][t] = tape[((int64_t)f * 3 + t) * soa_ld(n) + i];
#pragma unroll
  for (int f = 0; f < 8; ++f) ob[f] = rhs_bar[(int64_t)f * n + i];
  double gb[7][3];
  mhd_point_adjoint(qi, grad, gamma, ob, qb, gb);
#pragma unroll
  for (int f = 0; f < 7; ++f)
#pragma unroll
    for (int t = 0; t < 3; ++t) ub[f][t] = gb[f][t] * inv_lam;
}

// The same with the stabilisers: Ubar [8][9] (rows: the gradient, then the
// second-derivative rows xx, xy, xz, yy, yz, zz, in coefficient space).  With
// D_k[f] = fac_k (row_k . B_f) / lambda^2 (fac = 2 on the diagonal), grad div V
// is d_a div V = sum_b D_(ab)[V_b]; its adjoint reaches D_(ab)[V_b] and,
// for a != b, D_(ab)[V_a].
__device__ __forceinline__ void pointwise_adjoint_stab(int n, int i, const double* __restrict__ q,
                                                       const double* __restrict__ tape,
                                                       const double* __restrict__ rhs_bar,
                                                       const double* __restrict__ dxdt_bar,
                                                       double gamma, double lam, const Stab& sb,
                                                       int st, double (&qi)[8],
                                                       double (&ub)[8][9], double (&qb)[8]) {
#pragma unroll
  for (int f = 0; f < 8; ++f) {
    qi[f] = q[(int64_t)f * n + i];
    qb[f] = 0.0;
#pragma unroll
    for (int t = 0; t < 9; ++t) ub[f][t] = 0.0;
  }
  if (dxdt_bar) {
#pragma unroll
    for (int a = 0; a < 3; ++a) qb[1 + a] += dxdt_bar[(int64_t)a * n + i];
  }
  if (st != 0) return;
  double grad[7][3], ob[8], grho[3], gdv[3], gdb[3];
#pragma unroll
  for (int f = 0; f < 7; ++f)
#pragma unroll
    for (int t = 0; t < 3; ++t) grad[f][t] = tape[((int64_t)f * 3 + t) * soa_ld(n) + i];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    grho[a] = tape[(int64_t)(TAPE_GRHO + a) * soa_ld(n) + i];
    gdv[a] = tape[(int64_t)(TAPE_GDV + a) * soa_ld(n) + i];
    gdb[a] = tape[(int64_t)(TAPE_GDB + a) * soa_ld(n) + i];
  }
#pragma unroll
  for (int f = 0; f < 8; ++f) ob[f] = rhs_bar[(int64_t)f * n + i];
  double gb[7][3];
  mhd_point_adjoint(qi, grad, gamma, ob, qb, gb);
  double grho_b[3] = {0.0, 0.0, 0.0}, gdv_b[3] = {0.0, 0.0, 0.0}, gdb_b[3] = {0.0, 0.0, 0.0};
  const double divv_b = stab_point_adjoint(qi, grho, grad[0][0] + grad[1][1] + grad[2][2], gdv,
                                           gdb, lam, gamma, sb, ob, qb, grho_b, gdv_b, gdb_b);
  gb[0][0] += divv_b;
  gb[1][1] += divv_b;
  gb[2][2] += divv_b;
  const double inv_lam = 1.0 / lam;
  const double il2 = inv_lam * inv_lam;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    ub[0][t] = grho_b[t] * inv_lam;
#pragma unroll
    for (int f = 0; f < 7; ++f) ub[1 + f][t] = gb[f][t] * inv_lam;
  }
  // second-derivative row k = (a0, a1)
  constexpr int A0[6] = {0, 0, 0, 1, 1, 2}, A1[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double fac = (A0[k] == A1[k] ? 2.0 : 1.0) * il2;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      double cv = 0.0, cb = 0.0;
      if (b == A0[k]) {
        cv += gdv_b[A1[k]];
        cb += gdb_b[A1[k]];
      }
      if (b == A1[k] && A0[k] != A1[k]) {
        cv += gdv_b[A0[k]];
        cb += gdb_b[A0[k]];
      }
      ub[1 + b][3 + k] = fac * cv;
      ub[4 + b][3 + k] = fac * cb;
    }
  }
}

// ---- 1. Ubar [NFA][NR] and the direct qbar, one thread per particle ---------
// Ubar into ubuf[i * ustride + uoff ..] (a compact array).

template <bool STAB>
__global__ void __launch_bounds__(THREADS)
    k_adj_u(int n, const double4* __restrict__ geo, double gamma, Stab sb,
            const double* __restrict__ q, const double* __restrict__ tape,
            const double* __restrict__ rhs_bar, const double* __restrict__ dxdt_bar,
            double* __restrict__ ubuf, int ustride, int uoff, double* __restrict__ qb_direct) {
  const int i = blockIdx.x * THREADS + threadIdx.x;
  if (i >= n) return;
  const int st = (int)tape[(int64_t)TAPE_STATUS * soa_ld(n) + i];
  double qi[8], qb[8];
  double* u = ubuf + (int64_t)i * ustride + uoff;
  if constexpr (STAB) {
    double ub[8][9];
    pointwise_adjoint_stab(n, i, q, tape, rhs_bar, dxdt_bar, gamma, geo[i].w, sb, st, qi, ub, qb);
#pragma unroll
    for (int f = 0; f < 8; ++f)
#pragma unroll
      for (int t = 0; t < 9; ++t) u[f * 9 + t] = ub[f][t];
  } else {
    double ub[7][3];
    pointwise_adjoint(n, i, q, tape, rhs_bar, dxdt_bar, gamma, 1.0 / geo[i].w, st, qi, ub, qb);
#pragma unroll
    for (int f = 0; f < 7; ++f)
#pragma unroll
      for (int t = 0; t < 3; ++t) u[f * 3 + t] = ub[f][t];
  }
#pragma unroll
  for (int f = 0; f < 8; ++f) qb_direct[(int64_t)f * n + i] = qb[f];
}

// Data form: the owner record (G, K = Ubar C^T, Ubar) of the lane-per-entry
// schedule from the tape's G and C and the compact Ubar; one thread per owner
// and row.
template <bool STAB>
__global__ void __launch_bounds__(THREADS)
    k_adj_orec(int n, const double* __restrict__ aos, const double* __restrict__ ubuf,
               double* __restrict__ orec) {
  using SH = Shape<STAB>;
  constexpr int NR = SH::NR, NFA = SH::NFA, LEN = TAPE_AOS;
  const int64_t tid = (int64_t)blockIdx.x * THREADS + threadIdx.x;
  const int i = (int)(tid / NR);
  const int t = (int)(tid % NR);
  if (i >= n) return;
  const double* g = aos + (int64_t)i * LEN;
  const double* u = ubuf + (int64_t)i * NFA * NR;
  double* o = orec + (int64_t)i * SH::OREC;
  for (int b = 0; b < NBASIS; ++b) {
    double k = 0.0;
    for (int f = 0; f < NFA; ++f) k = fma(u[f * NR + t], g[NR * NBASIS + f * NBASIS + b], k);
    o[t * NBASIS + b] = g[t * NBASIS + b];
    o[SH::KOFF + t * NBASIS + b] = k;
  }
  if (t == 0)
    for (int e = 0; e < NFA * NR; ++e) o[SH::UOFF + e] = u[e];
}

// ---- 3. pair contributions ---------------------------------------------------
// Reverse-mode contributions of one neighbor entry (i, j), j != i, given the
// owner record o (G rows 0..59, K rows 60..119, Ubar at UOFF):
//   a = G p, b = Ubar df - K p, dfbar_f = w Ubar_f . a, wbar = a . b,
//   xibar = w sum_t (b_t grad(G_t . p) - a_t grad(K_t . p)),
//   dbar = xibar / lambda + wbar w'(q) 2 d / r^2.
// v receives dfbar (7) and dbar (3).  The owner record is read one
// 20-coefficient row at a time, each row used at once for its value and its
// gradient; the compiler fences keep the rows' loads from being hoisted
// together (a wavefront-uniform record is read through the scalar cache, and
// 141 doubles do not fit the scalar registers).
__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

// Value and gradient of one row's cubic c . p(xi) at xi = (x, y, z), nested
// over the quadratic monomials so that the 20 monomials are never held:
// value c0 + c1 x + c2 y + c3 z + xx (c4 + c10 x + c11 y + c12 z)
//       + xy (c5 + c13 y + c14 z) + xz (c6 + c15 z) + yy (c7 + c16 y + c17 z)
//       + yz (c8 + c18 z) + zz (c9 + c19 z),
// and each gradient component likewise.
template <class CT>
struct CubicAt {
  CT x, y, z, xx, xy, xz, yy, yz, zz, x2, y2, z2, x3, y3, z3;
};
template <class CT>
__device__ __forceinline__ CubicAt<CT> cubic_at(CT x, CT y, CT z) {
  CubicAt<CT> q;
  q.x = x; q.y = y; q.z = z;
  q.xx = x * x; q.xy = x * y; q.xz = x * z; q.yy = y * y; q.yz = y * z; q.zz = z * z;
  q.x2 = x + x; q.y2 = y + y; q.z2 = z + z;
  q.x3 = CT(3) * x; q.y3 = CT(3) * y; q.z3 = CT(3) * z;
  return q;
}
template <class CT>
__device__ __forceinline__ void row_value_grad_q(const CT* __restrict__ c, const CubicAt<CT>& q,
                                                 CT& v, CT (&g)[3]) {
  const CT c0 = c[0], c1 = c[1], c2 = c[2], c3 = c[3], c4 = c[4], c5 = c[5], c6 = c[6];
  const CT c7 = c[7], c8 = c[8], c9 = c[9], c10 = c[10], c11 = c[11], c12 = c[12];
  const CT c13 = c[13], c14 = c[14], c15 = c[15], c16 = c[16], c17 = c[17], c18 = c[18];
  const CT c19 = c[19];
  CT t = fma(c10, q.x, fma(c11, q.y, fma(c12, q.z, c4)));
  v = fma(q.xx, t, fma(c1, q.x, fma(c2, q.y, fma(c3, q.z, c0))));
  v = fma(q.xy, fma(c13, q.y, fma(c14, q.z, c5)), v);
  v = fma(q.xz, fma(c15, q.z, c6), v);
  v = fma(q.yy, fma(c16, q.y, fma(c17, q.z, c7)), v);
  v = fma(q.yz, fma(c18, q.z, c8), v);
  v = fma(q.zz, fma(c19, q.z, c9), v);
  // gx = c1 + x (2 c4 + 3x c10 + 2y c11 + 2z c12) + y (c5 + y c13 + z c14) + z (c6 + z c15)
  t = fma(q.x3, c10, fma(q.y2, c11, fma(q.z2, c12, c4 + c4)));
  g[0] = fma(q.x, t, fma(q.y, fma(q.y, c13, fma(q.z, c14, c5)), fma(q.z, fma(q.z, c15, c6), c1)));
  // gy = c2 + x (c5 + x c11 + 2y c13 + z c14) + y (2 c7 + 3y c16 + 2z c17) + z (c8 + z c18)
  t = fma(q.x, c11, fma(q.y2, c13, fma(q.z, c14, c5)));
  g[1] = fma(q.x, t, fma(q.y, fma(q.y3, c16, fma(q.z2, c17, c7 + c7)), fma(q.z, fma(q.z, c18, c8), c2)));
  // gz = c3 + x (c6 + x c12 + y c14 + 2z c15) + y (c8 + y c17 + 2z c18) + z (2 c9 + 3z c19)
  t = fma(q.x, c12, fma(q.y, c14, fma(q.z2, c15, c6)));
  g[2] = fma(q.x, t, fma(q.y, fma(q.y, c17, fma(q.z2, c18, c8)), fma(q.z, fma(q.z3, c19, c9 + c9), c3)));
}

// CT: the arithmetic type of the pair terms.  The displacement, the weight and
// the field differences are formed in FP64 and rounded once.  STAB: the
// stabilised shape (nine rows, eight fields).
template <class CT, bool STAB = false>
__device__ __forceinline__ void pair_terms(const CT* __restrict__ o, double w, double dw,
                                           double inv_lam, double inv_r2, double dx, double dy,
                                           double dz, const double* __restrict__ fi,
                                           const double* __restrict__ fj,
                                           CT (&v)[Shape<STAB>::REC]) {
  using SH = Shape<STAB>;
  CT h[SH::NR];
#pragma unroll
  for (int t = 0; t < SH::NR; ++t) h[t] = CT(0);
#pragma unroll
  for (int f = 0; f < SH::NFA; ++f) {
    const CT df = CT(fj[SH::F0 + f] - fi[SH::F0 + f]);
#pragma unroll
    for (int t = 0; t < SH::NR; ++t) h[t] = fma(o[SH::UOFF + SH::NR * f + t], df, h[t]);
  }
  const CubicAt<CT> q = cubic_at(CT(dx * inv_lam), CT(dy * inv_lam), CT(dz * inv_lam));
  CT av[SH::NR], bv[SH::NR], xg[3] = {CT(0), CT(0), CT(0)};
#pragma unroll
  for (int t = 0; t < SH::NR; ++t) {
    compiler_fence();
    CT a, ga[3];
    row_value_grad_q(o + t * NBASIS, q, a, ga);
    compiler_fence();
    CT k, gk[3];
    row_value_grad_q(o + SH::KOFF + t * NBASIS, q, k, gk);
    const CT b = h[t] - k;
#pragma unroll
    for (int c = 0; c < 3; ++c) xg[c] = fma(b, ga[c], fma(-a, gk[c], xg[c]));
    av[t] = a;
    bv[t] = b;
  }
  compiler_fence();
  const CT wc = CT(w);
#pragma unroll
  for (int f = 0; f < SH::NFA; ++f) {
    CT u = o[SH::UOFF + SH::NR * f] * av[0];
#pragma unroll
    for (int t = 1; t < SH::NR; ++t) u = fma(o[SH::UOFF + SH::NR * f + t], av[t], u);
    v[f] = wc * u;
  }
  CT wbar = av[0] * bv[0];
#pragma unroll
  for (int t = 1; t < SH::NR; ++t) wbar = fma(av[t], bv[t], wbar);
  const CT geo_f = wbar * CT(dw * 2.0 * inv_r2);
  const CT wl = CT(w * inv_lam);
  v[SH::NFA] = fma(wl, xg[0], geo_f * CT(dx));
  v[SH::NFA + 1] = fma(wl, xg[1], geo_f * CT(dy));
  v[SH::NFA + 2] = fma(wl, xg[2], geo_f * CT(dz));
#pragma unroll
  for (int c = SH::NFA + 3; c < SH::REC; ++c) v[c] = CT(0);
}

// One lane per neighbor entry: a block takes 256 consecutive entries, so
// lanes are never idle at row ends.  The owner records of the rows the block
// touches (at most OWN_MAX of them, contiguous in memory) are staged in LDS
// by one coalesced copy; blocks touching more rows read them from global
// memory.  Owner shares are summed by a segmented scan over each wavefront;
// rows that span wavefronts are finished by k_adj_combine.
constexpr int OWN_MAX = 24;

template <class RT>
__global__ void __launch_bounds__(PAIRS_PER_BLOCK)
    k_adj_pairs(int n, int64_t nnz, const double4* __restrict__ geo,
                const int64_t* __restrict__ off, const int32_t* __restrict__ idx,
                const int32_t* __restrict__ t_pos, Box box, double rf_ratio, int wkind,
                const double* __restrict__ fq, const double* __restrict__ orec,
                RT* __restrict__ rec, double* __restrict__ own, double* __restrict__ wpart,
                int slot_order) {
  __shared__ int64_t sh_off[PAIRS_PER_BLOCK + 1];
  __shared__ int sh_i0, sh_cnt;
  __shared__ double sh_rec[OWN_MAX * OREC];
  const int64_t S0 = (int64_t)blockIdx.x * PAIRS_PER_BLOCK;
  if (threadIdx.x == 0) {  // last row starting at or before S0
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (off[mid] <= S0)
        lo = mid;
      else
        hi = mid - 1;
    }
    sh_i0 = lo;
  }
  __syncthreads();
  const int i0 = sh_i0;
  for (int k = threadIdx.x; k <= PAIRS_PER_BLOCK; k += PAIRS_PER_BLOCK) {
    const int r = i0 + k;
    sh_off[k] = off[r < n ? r : n];
  }
  __syncthreads();
  const int64_t s = S0 + threadIdx.x;
  const bool valid = s < nnz;
  const int lane = threadIdx.x & 63;
  int i = 0x7fffffff;  // owner (sentinel for lanes past the end)
  int lo = 0;
  if (valid) {
    int hi = PAIRS_PER_BLOCK;
    while (lo < hi) {  // last staged row with off <= s
      const int mid = (lo + hi + 1) >> 1;
      if (sh_off[mid] <= s)
        lo = mid;
      else
        hi = mid - 1;
    }
    i = i0 + lo;
    if (lo == PAIRS_PER_BLOCK) {  // only with many empty rows: search the rest
      int a = i, b = n - 1;
      while (a < b) {
        const int mid = (a + b + 1) >> 1;
        if (off[mid] <= s)
          a = mid;
        else
          b = mid - 1;
      }
      i = a;
    }
  }
  // the last valid lane owns the block's last row
  const int64_t last = (nnz - 1 - S0) < (PAIRS_PER_BLOCK - 1) ? (nnz - 1 - S0)
                                                               : (PAIRS_PER_BLOCK - 1);
  if ((int64_t)threadIdx.x == last) sh_cnt = i - i0 + 1;
  __syncthreads();
  const int cnt = sh_cnt;
  const bool staged = cnt <= OWN_MAX;
  if (staged) {
    const double* src = orec + (int64_t)i0 * OREC;
    for (int k = threadIdx.x; k < cnt * OREC; k += PAIRS_PER_BLOCK) sh_rec[k] = src[k];
  }
  __syncthreads();
  double v[REC];
#pragma unroll
  for (int c = 0; c < REC; ++c) v[c] = 0.0;
  if (valid) {
    const int j = idx[s];
    if (j != i) {
      const double4 gi = geo[i], gj = geo[j];
      const double inv_lam = 1.0 / gi.w;
      const double r = rf_ratio * gi.w;
      const double inv_r2 = 1.0 / (r * r);
      const double dx = min_image(gj.x - gi.x, box.L[0], box.halfL[0], box.periodic[0]);
      const double dy = min_image(gj.y - gi.y, box.L[1], box.halfL[1], box.periodic[1]);
      const double dz = min_image(gj.z - gi.z, box.L[2], box.halfL[2], box.periodic[2]);
      const double qd = (dx * dx + dy * dy + dz * dz) * inv_r2;
      const double w = weight_of(qd, wkind);
      const double dw = weight_dq(qd, wkind);
      if (staged)
        pair_terms(sh_rec + (i - i0) * OREC, w, dw, inv_lam, inv_r2, dx, dy, dz,
                   fq + 8 * (int64_t)i, fq + 8 * (int64_t)j, v);
      else
        pair_terms(orec + (int64_t)i * OREC, w, dw, inv_lam, inv_r2, dx, dy, dz,
                   fq + 8 * (int64_t)i, fq + 8 * (int64_t)j, v);
    }
    RT* out = rec + (slot_order ? s : (int64_t)t_pos[s]) * REC;
    if constexpr (sizeof(RT) == 8) {
      double2* o2 = reinterpret_cast<double2*>(out);
#pragma unroll
      for (int c = 0; c < REC; c += 2) o2[c / 2] = make_double2(v[c], v[c + 1]);
    } else {
      float2* o2 = reinterpret_cast<float2*>(out);
#pragma unroll
      for (int c = 0; c < REC; c += 2) o2[c / 2] = make_float2((float)v[c], (float)v[c + 1]);
    }
  }
  // segmented inclusive sum over the wavefront (owners are non-decreasing)
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int ku = __shfl_up(i, d, 64);
    double u[REC];
#pragma unroll
    for (int c = 0; c < REC; ++c) u[c] = __shfl_up(v[c], d, 64);
    if (lane >= d && ku == i) {
#pragma unroll
      for (int c = 0; c < REC; ++c) v[c] += u[c];
    }
  }
  const int knext = __shfl_down(i, 1, 64);
  if (valid && (lane == 63 || knext != i)) {
    const int64_t wfirst = s - lane;
    const int64_t wlast = wfirst + 63;
    const int64_t rs = off[i], re = off[i + 1] - 1;
    if (rs >= wfirst && re <= wlast) {
#pragma unroll
      for (int c = 0; c < REC; ++c) own[(int64_t)c * n + i] = -v[c];
    } else {
      const int64_t wv = wfirst >> 6;
      double* dst = wpart + (wv * 2 + (rs <= wfirst ? 0 : 1)) * REC;
#pragma unroll
      for (int c = 0; c < REC; ++c) dst[c] = v[c];
    }
  }
}

// Owners whose rows span several wavefronts: add the pieces in order.
__global__ void __launch_bounds__(THREADS)
    k_adj_combine(int n, const int64_t* __restrict__ off, const double* __restrict__ wpart,
                  double* __restrict__ own) {
  const int i = blockIdx.x * THREADS + threadIdx.x;
  if (i >= n) return;
  const int64_t rs = off[i], re = off[i + 1] - 1;
  if (re < rs) {  // empty row: nothing owned
#pragma unroll
    for (int c = 0; c < REC; ++c) own[(int64_t)c * n + i] = 0.0;
    return;
  }
  const int64_t w0 = rs >> 6, w1 = re >> 6;
  if (w0 == w1) return;
  double acc[REC];
  const double* first = wpart + (w0 * 2 + (rs == (w0 << 6) ? 0 : 1)) * REC;
#pragma unroll
  for (int c = 0; c < REC; ++c) acc[c] = first[c];
  for (int64_t wv = w0 + 1; wv <= w1; ++wv) {
    const double* pc = wpart + wv * 2 * REC;
#pragma unroll
    for (int c = 0; c < REC; ++c) acc[c] += pc[c];
  }
#pragma unroll
  for (int c = 0; c < REC; ++c) own[(int64_t)c * n + i] = -acc[c];
}

// ---- 3b. pair contributions, one wavefront per owner ------------------------
// The owner's G, K and Ubar are wavefront-uniform and staged in LDS; lanes
// take the owner's neighbor entries 64 at a time (rows longer than 64
// entries loop); the owner's own share is one transposed wavefront sum of the
// record's components at the end.  Each block is one wavefront: the waves
// live for different times (row lengths vary 10x), and a block of several
// holds its slots until the longest of them ends.

// RT: type of the pair records (double; float in the mixed form, where the
// records are an application-level quantity and halve the record traffic).
// CT: arithmetic type of the pair terms.  FP64 in both forms: in FP32 the
// difference b = Ubar df - K p, which is Ubar times the fit's residual, and
// the cancelling sums of the records over a particle's owners lose up to
// 1e-3 of the gradient on the 1M shear layer (sharp layers, 4x lambda range).
//
// aos is the tape's AoS block (G, then the fit coefficients C) and ubuf the
// compact Ubar [n][NFA][NR]; the wavefront stages G and Ubar and forms
// K = Ubar C^T as it stages them (one entry of K per lane and pass, all in
// the one staging phase).
// PAIR_TILE: owners per tile of the tile schedule (its LDS sums).  The
// tiles of a set are fixed by its size alone: a batch tiles each of its
// sets as a call on that set would.
constexpr int PAIR_TILE = 128;

// One owner's pair terms.  TILE = false: every record to its slot and the
// owner's share to own.  TILE = true (the tile schedule): the terms for
// targets j in the wavefront's tile [T0, T1) and the owner's share are
// added to the tile's LDS sums tacc[component][j - T0] instead; a row's
// targets are distinct, so its lanes never add to one sum together, and a
// wavefront's LDS accesses complete in program order.
template <class RT, class CT, bool STAB, bool TILE>
__device__ __forceinline__ void owner_pairs(
    int i, int lane, int n, const double4* __restrict__ geo, const int64_t* __restrict__ off,
    const int32_t* __restrict__ idx, const int32_t* __restrict__ t_pos, const Box& box,
    double rf_ratio, int wkind, const double* __restrict__ fq, const double* __restrict__ aos,
    const double* __restrict__ ubuf, RT* __restrict__ rec, double* __restrict__ own,
    int slot_order, CT* osh, double* tacc, int T0, int T1) {
  using SH = Shape<STAB>;
  constexpr int RC = SH::REC;
  constexpr int NR = SH::NR, NFA = SH::NFA;
  // Each lane's first entry (index, neighbor geometry, transposed position)
  // is fetched before the record is staged, so that this dependent chain of
  // loads overlaps the staging; later entries are fetched one iteration
  // ahead.
  const int64_t rs = off[i], re = off[i + 1];
  const double4 gi = geo[i];
  double4 gjn = make_double4(0.0, 0.0, 0.0, 1.0);
  int jn = 0, tpn = 0;
  if (rs + lane < re) {
    jn = idx[rs + lane];
    gjn = geo[jn];
    if (!slot_order) tpn = t_pos[rs + lane];
  }
  {
    // every load of the staging is issued before the first LDS store, so
    // the record costs one memory latency
    const double* g = aos + (int64_t)i * TAPE_AOS;
    const double* u = ubuf + (int64_t)i * NFA * NR;
    constexpr int NK = (NR * NBASIS + 63) / 64, NU = (NFA * NR + 63) / 64;
    double gv[NK], kv[NK], uv[NU];
#pragma unroll
    for (int r = 0; r < NK; ++r) {
      const int e = lane + 64 * r;
      gv[r] = e < NR * NBASIS ? g[e] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < NU; ++r) {
      const int e = lane + 64 * r;
      uv[r] = e < NFA * NR ? u[e] : 0.0;
    }
    // K_t = sum_f Ubar[f][t] C_f
#pragma unroll
    for (int r = 0; r < NK; ++r) {
      const int e = lane + 64 * r;
      const int t = e / NBASIS, b = e % NBASIS;
      double k = 0.0;
      if (e < NR * NBASIS) {
#pragma unroll
        for (int f = 0; f < NFA; ++f) k = fma(u[f * NR + t], g[NR * NBASIS + f * NBASIS + b], k);
      }
      kv[r] = k;
    }
#pragma unroll
    for (int r = 0; r < NK; ++r) {
      const int e = lane + 64 * r;
      if (e < NR * NBASIS) {
        osh[e] = CT(gv[r]);
        osh[SH::KOFF + e] = CT(kv[r]);
      }
    }
#pragma unroll
    for (int r = 0; r < NU; ++r) {
      const int e = lane + 64 * r;
      if (e < NFA * NR) osh[SH::UOFF + e] = CT(uv[r]);
    }
  }
  // each wavefront reads only its own record: no block barrier
  wave_lds_sync();
  const double inv_lam = 1.0 / gi.w;
  const double r = rf_ratio * gi.w;
  const double inv_r2 = 1.0 / (r * r);
  const CT* o = osh;
  const double* fi = fq + 8 * (int64_t)i;
  double acc[RC];
#pragma unroll
  for (int c = 0; c < RC; ++c) acc[c] = 0.0;
  for (int64_t s = rs + lane; s < re; s += 64) {
    const int j = jn;
    const double4 gj = gjn;
    const int tp = tpn;
    if (s + 64 < re) {
      jn = idx[s + 64];
      gjn = geo[jn];
      if (!slot_order) tpn = t_pos[s + 64];
    }
    CT v[RC];
#pragma unroll
    for (int c = 0; c < RC; ++c) v[c] = CT(0);
    if (j != i) {
      const double dx = min_image(gj.x - gi.x, box.L[0], box.halfL[0], box.periodic[0]);
      const double dy = min_image(gj.y - gi.y, box.L[1], box.halfL[1], box.periodic[1]);
      const double dz = min_image(gj.z - gi.z, box.L[2], box.halfL[2], box.periodic[2]);
      const double qd = (dx * dx + dy * dy + dz * dz) * inv_r2;
      const double w = weight_of(qd, wkind);
      const double dw = weight_dq(qd, wkind);
      pair_terms<CT, STAB>(o, w, dw, inv_lam, inv_r2, dx, dy, dz, fi, fq + 8 * (int64_t)j, v);
    }
    if (TILE && j >= T0 && j < T1) {
#pragma unroll
      for (int c = 0; c < RC; ++c) tacc[c * PAIR_TILE + (j - T0)] += double(v[c]);
    } else {
      RT* out = rec + (slot_order ? s : (int64_t)tp) * RC;
      if constexpr (sizeof(RT) == 8) {
        double2* o2 = reinterpret_cast<double2*>(out);
#pragma unroll
        for (int c = 0; c < RC; c += 2) o2[c / 2] = make_double2(v[c], v[c + 1]);
      } else {
        float2* o2 = reinterpret_cast<float2*>(out);
#pragma unroll
        for (int c = 0; c < RC; c += 2) o2[c / 2] = make_float2((float)v[c], (float)v[c + 1]);
      }
    }
#pragma unroll
    for (int c = 0; c < RC; ++c) acc[c] += v[c];
  }
  double tot;
  int comp;
  wave_sum_transposed<RC>(acc, tot, comp);
  if (comp >= 0) {
    if constexpr (TILE) tacc[comp * PAIR_TILE + (i - T0)] -= tot;
    else own[(int64_t)comp * n + i] = -tot;
  }
}

template <class RT, class CT = double, bool STAB = false>
__global__ void __launch_bounds__(64)
    k_adj_pairs_w(int n, const double4* __restrict__ geo, const int64_t* __restrict__ off,
                  const int32_t* __restrict__ idx, const int32_t* __restrict__ t_pos, Box box,
                  double rf_ratio, int wkind, const double* __restrict__ fq,
                  const double* __restrict__ aos, const double* __restrict__ ubuf,
                  RT* __restrict__ rec, double* __restrict__ own, int slot_order) {
  const int i = __builtin_amdgcn_readfirstlane(xcd_block());
  if (i >= n) return;  // one wavefront per block
  // the owner record (G | K | Ubar) goes to LDS once per wavefront; the pair
  // terms then read it row by row at LDS latency
  __shared__ CT osh[Shape<STAB>::OREC];
  owner_pairs<RT, CT, STAB, false>(i, threadIdx.x & 63, n, geo, off, idx, t_pos, box, rf_ratio,
                                   wkind, fq, aos, ubuf, rec, own, slot_order, osh, nullptr, 0,
                                   0);
}

// ---- 3b'. pair contributions, one block per tile of owners ------------------
// A block of TILE_WAVES wavefronts takes the owners of one tile of
// ts <= PAIR_TILE consecutive particles (consecutive along the Hilbert
// curve: a compact region); wavefront w takes owners w, w + TILE_WAVES, ...
// in ascending order.  Pair terms whose target lies in the tile are summed
// in LDS, in FP64, each wavefront in its own copy of the tile's sums, and
// the copies are added in a fixed order and written once per particle with
// the owner's share (into own, which the gather adds); only the other
// records go to memory, and the gather skips a particle's in-tile owners (a
// contiguous run of its sorted transposed row; tbound gives each particle
// its tile).  The order of every sum is fixed by the tiles: uniform tiles of
// ts owners, or the tile starts tstart[0 .. ntiles] (a batch tiles each set
// from its first particle, as a call on that set alone does, so that its
// results are the same to the last bit).  Several wavefronts per tile keep
// the tiles short, so that
// the tiles in flight on an XCD span a region whose neighbor data stays in
// its L2.
constexpr int TILE_WAVES = 4;

// Three wavefronts per SIMD, as the wavefront-per-owner kernel gets by
// itself (its 64-thread blocks): a 256-thread block lets the compiler take
// more registers and leaves two.
template <class RT, class CT = double, bool STAB = false>
__global__ void __launch_bounds__(64 * TILE_WAVES) __attribute__((amdgpu_waves_per_eu(3)))
    k_adj_pairs_t(int n, int ts, const int32_t* __restrict__ tstart, int2* __restrict__ tbound,
                  const double4* __restrict__ geo,
                  const int64_t* __restrict__ off, const int32_t* __restrict__ idx,
                  const int32_t* __restrict__ t_pos, Box box, double rf_ratio, int wkind,
                  const double* __restrict__ fq, const double* __restrict__ aos,
                  const double* __restrict__ ubuf, RT* __restrict__ rec,
                  double* __restrict__ own, int slot_order) {
  using SH = Shape<STAB>;
  constexpr int RC = SH::REC;
  const int t = xcd_block();
  const int T0 = tstart ? tstart[t] : t * ts;
  if (T0 >= n) return;  // whole blocks leave together
  const int T1 = tstart ? tstart[t + 1] : min(T0 + ts, n);
  // the wavefront's index made uniform, so that the owner index and all it
  // addresses stay in scalar registers
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  __shared__ CT osh[TILE_WAVES][SH::OREC];
  __shared__ double tacc[TILE_WAVES][RC * PAIR_TILE];
  for (int e = lane; e < RC * PAIR_TILE; e += 64) tacc[wv][e] = 0.0;
  for (int i = T0 + wv; i < T1; i += TILE_WAVES)
    owner_pairs<RT, CT, STAB, true>(i, lane, n, geo, off, idx, t_pos, box, rf_ratio, wkind, fq,
                                    aos, ubuf, rec, own, slot_order, osh[wv], tacc[wv], T0, T1);
  __syncthreads();
  for (int e = threadIdx.x; e < T1 - T0; e += 64 * TILE_WAVES) {
#pragma unroll
    for (int c = 0; c < RC; ++c) {
      double sum = tacc[0][c * PAIR_TILE + e];
#pragma unroll
      for (int w = 1; w < TILE_WAVES; ++w) sum += tacc[w][c * PAIR_TILE + e];
      own[(int64_t)c * n + T0 + e] = sum;
    }
    tbound[T0 + e] = make_int2(T0, T1);
  }
}

// ---- 3c. pair contributions, pipelined over owners --------------------------
// A persistent wavefront takes a contiguous range of owners and runs the
// wavefront-per-owner pair terms over it as a two-stage pipeline.  While
// owner k is computed from LDS, gfx950's direct-to-LDS loads bring owner
// k + 1 into the other half of a double buffer (each lane's neighbor
// position and fields, 16 bytes per lane and instruction, and the owner's
// record), and the neighbor indices of owner k + 2 load into registers.  The
// two dependent memory latencies of an owner (its indices, then its
// neighbors) overlap the previous owner's arithmetic; the one-shot schedule
// waits them out with three wavefronts per SIMD to cover them.  Entries past
// a row's 64th are fetched directly (rows that long are rare).
//
// The compiler does not track the direct-to-LDS loads: the wavefront drains
// its vector-memory counter before it reads a stage.
constexpr int PIPE_SLABS = 6;  // 16-byte pieces per entry: x y, z lambda, fields 0-1 .. 6-7

template <bool STAB>
struct PipeShape {
  using SH = Shape<STAB>;
  static constexpr int GC = (SH::NR + SH::NFA) * NBASIS;  // the tape's G and C rows
  static constexpr int UW = SH::NFA * SH::NR;            // compact Ubar
  static constexpr int RAW = GC + UW;                     // doubles staged per owner
  static constexpr int RAW_PAD = (RAW + 1) & ~1;
};

__device__ __forceinline__ void vmem_drain() {
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0); expcnt and lgkmcnt left alone
  asm volatile("" ::: "memory");       // no memory access moves above the wait
}

// The direct-to-LDS loads of one owner into one stage.  len: the row's
// entries in the stage (at most 64); j: this lane's neighbor.
template <bool STAB>
__device__ __forceinline__ void pipe_issue(int i, int len, int j, int lane,
                                           const double4* __restrict__ geo,
                                           const double* __restrict__ fq,
                                           const double* __restrict__ aos,
                                           const double* __restrict__ ubuf,
                                           double (*ent)[64][2], double* raw, double* self) {
  using PS = PipeShape<STAB>;
  // the owner's own position and fields: lanes 0-1 and 2-5
  if (lane < 6) {
    const double* g = lane < 2 ? reinterpret_cast<const double*>(geo + i) + 2 * lane
                               : fq + 8 * (int64_t)i + 2 * (lane - 2);
    __builtin_amdgcn_global_load_lds(g, self, 16, 0, 0);
  }
  if (lane < len) {
    const double* g = reinterpret_cast<const double*>(geo + j);
    const double* f = fq + 8 * (int64_t)j;
    __builtin_amdgcn_global_load_lds(g, &ent[0][0][0], 16, 0, 0);
    __builtin_amdgcn_global_load_lds(g + 2, &ent[1][0][0], 16, 0, 0);
#pragma unroll
    for (int k = 0; k < 4; ++k) __builtin_amdgcn_global_load_lds(f + 2 * k, &ent[2 + k][0][0], 16, 0, 0);
  }
  constexpr int NW = PS::GC;  // even
  const double* src = aos + (int64_t)i * TAPE_AOS;
#pragma unroll
  for (int c = 0; c < (NW + 127) / 128; ++c) {
    const int e = 128 * c + 2 * lane;
    if (e < NW) __builtin_amdgcn_global_load_lds(src + e, raw + 128 * c, 16, 0, 0);
  }
  // Ubar [NFA][NR], four bytes per lane (its rows are 8-byte aligned)
  const uint32_t* u = reinterpret_cast<const uint32_t*>(ubuf + (int64_t)i * PS::UW);
  uint32_t* ru = reinterpret_cast<uint32_t*>(raw + PS::GC);
#pragma unroll
  for (int c = 0; c < (2 * PS::UW + 63) / 64; ++c) {
    const int e = 64 * c + lane;
    if (e < 2 * PS::UW) __builtin_amdgcn_global_load_lds(u + e, ru + 64 * c, 4, 0, 0);
  }
}

template <class RT, bool STAB>
__global__ void __launch_bounds__(64)
    k_adj_pairs_p(int n, const double4* __restrict__ geo, const int64_t* __restrict__ off,
                  const int32_t* __restrict__ idx, const int32_t* __restrict__ t_pos, Box box,
                  double rf_ratio, int wkind, const double* __restrict__ fq,
                  const double* __restrict__ aos, const double* __restrict__ ubuf,
                  RT* __restrict__ rec, double* __restrict__ own, int slot_order) {
  using SH = Shape<STAB>;
  using PS = PipeShape<STAB>;
  constexpr int RC = SH::REC, NR = SH::NR, NFA = SH::NFA;
  __shared__ __align__(16) double s_ent[2][PIPE_SLABS][64][2];
  __shared__ __align__(16) double s_raw[2][PS::RAW_PAD];
  __shared__ double osh[SH::OREC];  // G | K | Ubar, formed from the stage
  __shared__ __align__(16) double s_self[2][12];  // the owner's x y z lambda and eight fields
  const int lane = threadIdx.x;
  const int w = xcd_block(), nw = (int)gridDim.x;
  const int i0 = (int)((int64_t)n * w / nw), i1 = (int)((int64_t)n * (w + 1) / nw);
  if (i0 >= i1) return;
  // owner i0 into stage 0; the indices of owner i0 + 1
  int64_t rs = off[i0], re = off[i0 + 1];
  int jc = i0, tpc = 0;
  if (rs + lane < re) {
    jc = idx[rs + lane];
    if (!slot_order) tpc = t_pos[rs + lane];
  }
  pipe_issue<STAB>(i0, (int)min<int64_t>(re - rs, 64), jc, lane, geo, fq, aos, ubuf, s_ent[0],
                   s_raw[0], s_self[0]);
  int64_t rsn = re, ren = re;
  int jn = 0, tpn = 0;
  if (i0 + 1 < i1) {
    ren = off[i0 + 2];
    if (rsn + lane < ren) {
      jn = idx[rsn + lane];
      if (!slot_order) tpn = t_pos[rsn + lane];
    }
  }
  for (int i = i0; i < i1; ++i) {
    const int c = (i - i0) & 1;
    vmem_drain();  // stage c has landed, the indices of owner i + 1 are in
    if (i + 1 < i1)
      pipe_issue<STAB>(i + 1, (int)min<int64_t>(ren - rsn, 64), jn, lane, geo, fq, aos, ubuf,
                       s_ent[c ^ 1], s_raw[c ^ 1], s_self[c ^ 1]);
    int64_t rsnn = ren, rENN = ren;
    int jnn = 0, tpnn = 0;
    if (i + 2 < i1) {
      rENN = off[i + 3];
      if (rsnn + lane < rENN) {
        jnn = idx[rsnn + lane];
        if (!slot_order) tpnn = t_pos[rsnn + lane];
      }
    }
    // ---- owner i from stage c: G | K | Ubar, K_t = sum_f Ubar[f][t] C_f
    {
      const double* raw = s_raw[c];
#pragma unroll
      for (int r = 0; r < (NR * NBASIS + 63) / 64; ++r) {
        const int e = lane + 64 * r;
        if (e < NR * NBASIS) {
          const int t = e / NBASIS, b = e % NBASIS;
          double k = 0.0;
#pragma unroll
          for (int f = 0; f < NFA; ++f)
            k = fma(raw[PS::GC + f * NR + t], raw[NR * NBASIS + f * NBASIS + b], k);
          osh[e] = raw[e];
          osh[SH::KOFF + e] = k;
        }
      }
      for (int e = lane; e < PS::UW; e += 64) osh[SH::UOFF + e] = raw[PS::GC + e];
      wave_lds_sync();
    }
    const double* o = osh;
    // the owner's own data from the stage too: a global load here would
    // wait for the next owner's loads as well (the counter drains in order)
    const double4 gi = make_double4(s_self[c][0], s_self[c][1], s_self[c][2], s_self[c][3]);
    const double inv_lam = 1.0 / gi.w;
    const double r = rf_ratio * gi.w;
    const double inv_r2 = 1.0 / (r * r);
    const double* fi = &s_self[c][4];
    double acc[RC];
#pragma unroll
    for (int k = 0; k < RC; ++k) acc[k] = 0.0;
    for (int64_t s = rs + lane; s < re; s += 64) {
      int j, tp;
      double4 gj;
      double fj[8];
      if (s - lane == rs) {  // the staged first 64 entries
        j = jc;
        tp = tpc;
        const double2 a = *reinterpret_cast<const double2*>(&s_ent[c][0][lane][0]);
        const double2 b = *reinterpret_cast<const double2*>(&s_ent[c][1][lane][0]);
        gj = make_double4(a.x, a.y, b.x, b.y);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const double2 t = *reinterpret_cast<const double2*>(&s_ent[c][2 + k][lane][0]);
          fj[2 * k] = t.x;
          fj[2 * k + 1] = t.y;
        }
      } else {
        j = idx[s];
        tp = slot_order ? 0 : t_pos[s];
        gj = geo[j];
        load_fields(fq, j, fj);
      }
      double v[RC];
#pragma unroll
      for (int k = 0; k < RC; ++k) v[k] = 0.0;
      if (j != i) {
        const double dx = min_image(gj.x - gi.x, box.L[0], box.halfL[0], box.periodic[0]);
        const double dy = min_image(gj.y - gi.y, box.L[1], box.halfL[1], box.periodic[1]);
        const double dz = min_image(gj.z - gi.z, box.L[2], box.halfL[2], box.periodic[2]);
        const double qd = (dx * dx + dy * dy + dz * dz) * inv_r2;
        const double wt = weight_of(qd, wkind);
        const double dw = weight_dq(qd, wkind);
        pair_terms<double, STAB>(o, wt, dw, inv_lam, inv_r2, dx, dy, dz, fi, fj, v);
      }
      RT* out = rec + (slot_order ? s : (int64_t)tp) * RC;
      if constexpr (sizeof(RT) == 8) {
        double2* o2 = reinterpret_cast<double2*>(out);
#pragma unroll
        for (int k = 0; k < RC; k += 2) o2[k / 2] = make_double2(v[k], v[k + 1]);
      } else {
        float2* o2 = reinterpret_cast<float2*>(out);
#pragma unroll
        for (int k = 0; k < RC; k += 2) o2[k / 2] = make_float2((float)v[k], (float)v[k + 1]);
      }
#pragma unroll
      for (int k = 0; k < RC; ++k) acc[k] += v[k];
    }
    double tot;
    int comp;
    wave_sum_transposed<RC>(acc, tot, comp);
    if (comp >= 0) own[(int64_t)comp * n + i] = -tot;
    // rotate the pipeline
    rs = rsn;
    re = ren;
    jc = jn;
    tpc = tpn;
    rsn = rsnn;
    ren = rENN;
    jn = jnn;
    tpn = tpnn;
  }
}

// Inverse of t_pos: for transposed entry k, the forward entry it came from.
// nnz_true: offsets[n] (the launch covers a bound of it).
__global__ void __launch_bounds__(THREADS)
    k_invert(int64_t nnz, const int64_t* __restrict__ nnz_true, const int32_t* __restrict__ t_pos,
             int32_t* __restrict__ t_slot) {
  const int64_t s = (int64_t)blockIdx.x * THREADS + threadIdx.x;
  if (s < nnz && s < *nnz_true) t_slot[t_pos[s]] = (int32_t)s;
}

// ---- 4. gather over the transposed lists ------------------------------------
// G lanes share one particle's transposed row; their partial sums meet in a
// quad reduction.  The summation order is fixed for a given G.  TILE: the
// pair records of owners in the particle's own tile (tbound) were summed
// into own by the tile schedule and are skipped here (t_src names each
// entry's owner).
template <int G, class RT, bool STAB = false, bool TILE = false>
__global__ void __launch_bounds__(THREADS)
    k_adj_gather(int n, const int2* __restrict__ tbound, const int64_t* __restrict__ t_off,
                 const int32_t* __restrict__ t_slot, const int32_t* __restrict__ t_src,
                 const RT* __restrict__ rec, const double* __restrict__ own,
                 const double* __restrict__ qb_direct, double* __restrict__ q_bar,
                 double* __restrict__ pos_bar) {
  using SH = Shape<STAB>;
  constexpr int REC = SH::REC;
  const int tid = xcd_block() * THREADS + threadIdx.x;
  const int j = tid / G;
  const int l = tid % G;
  const bool valid = j < n;
  const int jj = valid ? j : n - 1;
  const int2 tb = TILE ? tbound[jj] : make_int2(0, 0);
  const int tlo = tb.x, thi = tb.y;
  double acc[REC];
#pragma unroll
  for (int c = 0; c < REC; ++c) acc[c] = 0.0;
  const int64_t k1 = valid ? t_off[jj + 1] : 0;
  for (int64_t k = t_off[jj] + l; k < k1; k += G) {
    if constexpr (TILE) {
      const int src = t_src[k];
      if (src >= tlo && src < thi) continue;
    }
    const RT* r = rec + (t_slot ? (int64_t)t_slot[k] : k) * REC;
    if constexpr (sizeof(RT) == 8) {
      const double2* r2 = reinterpret_cast<const double2*>(r);
#pragma unroll
      for (int c = 0; c < REC; c += 2) {
        const double2 t = r2[c / 2];
        acc[c] += t.x;
        acc[c + 1] += t.y;
      }
    } else {
      const float2* r2 = reinterpret_cast<const float2*>(r);
#pragma unroll
      for (int c = 0; c < REC; c += 2) {
        const float2 t = r2[c / 2];
        acc[c] += (double)t.x;
        acc[c + 1] += (double)t.y;
      }
    }
  }
#pragma unroll
  for (int c = 0; c < REC; ++c) acc[c] = group_sum<G>(acc[c]);
  if (!valid || l != 0) return;
#pragma unroll
  for (int c = 0; c < REC; ++c) acc[c] += own[(int64_t)c * n + j];
  if (SH::F0 == 1) q_bar[j] = qb_direct[j];
#pragma unroll
  for (int f = 0; f < SH::NFA; ++f)
    q_bar[(int64_t)(f + SH::F0) * n + j] = qb_direct[(int64_t)(f + SH::F0) * n + j] + acc[f];
#pragma unroll
  for (int a = 0; a < 3; ++a) pos_bar[(int64_t)a * n + j] = acc[SH::NFA + a];
}

}  // namespace

namespace {

// Launch helpers that pick the template instance from run-time choices.
template <bool STAB, bool TILE, class RT>
void launch_gather_t(hipStream_t s, int gl, int n, const int2* tb, const int64_t* t_off,
                     const int32_t* tsl, const int32_t* t_src, const RT* rec, const double* own,
                     const double* qbd, double* q_bar, double* pos_bar) {
  const unsigned gg = grid_for((int64_t)n * gl, THREADS);
  if (gl == 1)
    hipLaunchKernelGGL((k_adj_gather<1, RT, STAB, TILE>), dim3(gg), dim3(THREADS), 0, s, n, tb,
                       t_off, tsl, t_src, rec, own, qbd, q_bar, pos_bar);
  else if (gl == 2)
    hipLaunchKernelGGL((k_adj_gather<2, RT, STAB, TILE>), dim3(gg), dim3(THREADS), 0, s, n, tb,
                       t_off, tsl, t_src, rec, own, qbd, q_bar, pos_bar);
  else
    hipLaunchKernelGGL((k_adj_gather<4, RT, STAB, TILE>), dim3(gg), dim3(THREADS), 0, s, n, tb,
                       t_off, tsl, t_src, rec, own, qbd, q_bar, pos_bar);
}

// tb: each particle's tile under the tile schedule (its in-tile records are
// skipped), or null.
template <bool STAB, class RT>
void launch_gather(hipStream_t s, int gl, const int2* tb, int n, const int64_t* t_off,
                   const int32_t* tsl, const int32_t* t_src, const RT* rec, const double* own,
                   const double* qbd, double* q_bar, double* pos_bar) {
  if (tb)
    launch_gather_t<STAB, true>(s, gl, n, tb, t_off, tsl, t_src, rec, own, qbd, q_bar, pos_bar);
  else
    launch_gather_t<STAB, false>(s, gl, n, tb, t_off, tsl, t_src, rec, own, qbd, q_bar, pos_bar);
}

template <bool STAB, class RT>
void launch_pairs_w(hipStream_t s, const EvalArgs& a, const double4* geo, const double* fq,
                    const int32_t* t_pos, const double* aos, const double* ubuf, RT* rec,
                    double* own, int slot_order) {
  const dim3 grid(grid_for(a.n, 1));  // one wavefront per owner, one per block
  hipLaunchKernelGGL((k_adj_pairs_w<RT, double, STAB>), grid, dim3(64), 0, s, a.n, geo, a.off,
                     a.idx, t_pos, a.box, a.rf_ratio, a.wkind, fq, aos, ubuf, rec, own,
                     slot_order);
}

template <bool STAB, class RT>
void launch_pairs_t(hipStream_t s, const EvalArgs& a, int ts, const int32_t* tstart,
                    int64_t ntiles, int2* tb, const double4* geo, const double* fq,
                    const int32_t* t_pos, const double* aos, const double* ubuf, RT* rec,
                    double* own, int slot_order) {
  const dim3 grid(tstart ? (unsigned)ntiles : grid_for(a.n, ts));  // one block per tile
  hipLaunchKernelGGL((k_adj_pairs_t<RT, double, STAB>), grid, dim3(64 * TILE_WAVES), 0, s, a.n,
                     ts, tstart, tb, geo,
                     a.off, a.idx, t_pos, a.box, a.rf_ratio, a.wkind, fq, aos, ubuf, rec, own,
                     slot_order);
}

// Persistent pipelined schedule: about 64 owners per wavefront, at most 8192
// wavefronts (several per slot, so that ranges that finish early are
// replaced).
template <bool STAB, class RT>
void launch_pairs_p(hipStream_t s, const EvalArgs& a, const double4* geo, const double* fq,
                    const int32_t* t_pos, const double* aos, const double* ubuf, RT* rec,
                    double* own, int slot_order) {
  const dim3 grid((unsigned)std::max<int64_t>(1, std::min<int64_t>(a.n / 64, 8192)));
  hipLaunchKernelGGL((k_adj_pairs_p<RT, STAB>), grid, dim3(64), 0, s, a.n, geo, a.off, a.idx,
                     t_pos, a.box, a.rf_ratio, a.wkind, fq, aos, ubuf, rec, own, slot_order);
}

}  // namespace

// The owner data: every tape holds each owner's G and fit coefficients C,
// refined for the screened fits (the FP64 form's, and the mixed form's, whose
// taped forward is the FP64 data form), so the reverse pass needs Ubar alone
// before the pairs (K = Ubar C^T is formed in the pair kernel).
// Workspace of the reverse pass (see adjoint_rhs for the pieces).
static void plan_adjoint(Workspace& ws, int64_t n, int64_t nnz, const phb_params* p,
                         bool need_tape, bool lane_pairs) {
  const bool stab = stab_of(p).on();
  const int NRr = stab ? Shape<true>::NR : Shape<false>::NR;
  const int NFAr = stab ? Shape<true>::NFA : Shape<false>::NFA;
  const int ORr = stab ? Shape<true>::OREC : Shape<false>::OREC;
  const int RCr = stab ? Shape<true>::REC : Shape<false>::REC;
  const size_t nd = (size_t)n * sizeof(double);
  const int64_t nwaves = (std::max<int64_t>(nnz, 1) + 63) / 64;
  ws.plan((size_t)n * sizeof(double4));  // packed geometry
  ws.plan(8 * nd);                       // packed fields
  ws.plan(8 * nd);                       // direct qbar
  ws.plan((size_t)RCr * nd);             // own sums
  ws.plan((size_t)std::max<int64_t>(nnz, 1) * RCr * sizeof(double));  // pair records
  ws.plan((size_t)nwaves * 2 * REC * sizeof(double));                 // wavefront partials
  ws.plan((size_t)std::max<int64_t>(nnz, 1) * sizeof(int32_t));       // inverse of t_pos
  ws.plan((size_t)n * sizeof(int2));                                  // tile of each particle
  ws.plan((size_t)NFAr * NRr * nd);               // Ubar
  if (lane_pairs) ws.plan((size_t)ORr * nd);      // owner records
  if (need_tape) {
    ws.plan((size_t)tape_doubles(n) * sizeof(double));  // private tape
    ws.plan(8 * nd);                                     // rhs scratch
    ws.plan(3 * nd);                                     // dxdt scratch
    ws.plan((size_t)n * sizeof(int32_t));                // status scratch
  }
}

int adjoint_pair_tile() { return PAIR_TILE; }

size_t ws_bytes_adjoint(int64_t n, int64_t nnz, const phb_params* p, bool need_tape) {
  phb_ctx dummy;
  Workspace ws(&dummy);
  plan_adjoint(ws, n, nnz, p, need_tape, !stab_of(p).on());
  if (need_tape) {
    phb_params p64 = *p;
    p64.precision = PHB_FP64;
    ws.plan(ws_bytes_rhs(n, &p64));
  }
  return ws.total;
}

int adjoint_rhs(phb_ctx* ctx, const EvalArgs& a, const phb_params* p, const int64_t* t_offsets,
                const int32_t* t_src, const int32_t* t_pos, const double* q,
                const double* rhs_bar, const double* dxdt_bar, double* q_bar, double* pos_bar,
                const double* tape_in, int64_t nnz_known, bool nnz_exact,
                const int32_t* tstart, int64_t ntiles) {
  const int n = a.n;
  const Stab sb = stab_of(p);
  const bool stab = sb.on();
  // record shapes of this pass (see Shape)
  const int NRr = stab ? Shape<true>::NR : Shape<false>::NR;
  const int NFAr = stab ? Shape<true>::NFA : Shape<false>::NFA;
  const int ORr = stab ? Shape<true>::OREC : Shape<false>::OREC;
  const int RCr = stab ? Shape<true>::REC : Shape<false>::REC;
  // nnz sizes the pair records: unless the caller knows it, read offsets[n]
  // back (a synchronization, so captured callers pass it).
  int rc;
  int64_t nnz = nnz_known;
  if (nnz < 0) {
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
  // transposed positions and pair-record slots are int32
  if (nnz > PHB_NNZ_MAX)
    return set_error(ctx, PHB_EINVAL, "nnz exceeds the int32 positions of the transposed lists");
  const bool need_tape = tape_in == nullptr;
  // the lane-per-entry schedule (ideal shape) reads whole owner records and
  // needs the exact entry count
  const bool lane_pairs = !stab && ctx->adj_pairs_mode == 0 && nnz_exact;
  phb_params p64 = *p;
  p64.precision = PHB_FP64;
  Workspace ws(ctx);
  plan_adjoint(ws, n, nnz, p, need_tape, lane_pairs);
  const int64_t nwaves = (std::max<int64_t>(nnz, 1) + 63) / 64;
  const size_t own_bytes = ws.total;
  if (need_tape) ws.plan(ws_bytes_rhs(n, &p64));  // the nested forward
  if ((rc = ws.commit())) return rc;
  double4* geo = ws.take<double4>(n);
  double* fq = ws.take<double>((size_t)8 * n);
  double* qbd = ws.take<double>((size_t)8 * n);
  double* own = ws.take<double>((size_t)RCr * n);
  double* rec = ws.take<double>((size_t)std::max<int64_t>(nnz, 1) * RCr);
  double* wpart = ws.take<double>((size_t)nwaves * 2 * REC);
  int32_t* t_slot = ws.take<int32_t>(std::max<int64_t>(nnz, 1));
  int2* tbound = ws.take<int2>(n);
  double* ubuf = ws.take<double>((size_t)NFAr * NRr * n);
  double* orec = lane_pairs ? ws.take<double>((size_t)ORr * n) : nullptr;
  const int slot_order = ctx->record_order;
  const double* tape = tape_in;
  hipStream_t s = ctx->stream;
  if (need_tape) {  // the FP64 forward fills a private tape
    double* tp = ws.take<double>((size_t)tape_doubles(n));
    double* rs = ws.take<double>((size_t)8 * n);
    double* dx = ws.take<double>((size_t)3 * n);
    int32_t* st = ws.take<int32_t>(n);
    ArenaHold hold(ctx, own_bytes);
    if ((rc = eval_rhs(ctx, a, &p64, q, rs, dx, st, tp))) return rc;
    tape = tp;
  }
  EvalArgs ap = a;
  ap.geo = geo;
  ap.fq = fq;
  { Prof pf(ctx, "k_pack");
  if ((rc = hip_check(ctx, launch_pack(s, n, a.pos, a.lam, q, geo, fq), "pack"))) return rc; }
  const double* aos = tape_aos(tape, n);  // each owner's G and C
  { Prof pf(ctx, stab ? "k_adj_u<stab>" : "k_adj_u");
  if (stab)
    hipLaunchKernelGGL(k_adj_u<true>, dim3(grid_for(n, THREADS)), dim3(THREADS), 0, s, n, geo,
                       p->gamma, sb, q, tape, rhs_bar, dxdt_bar, ubuf, NFAr * NRr, 0, qbd);
  else
    hipLaunchKernelGGL(k_adj_u<false>, dim3(grid_for(n, THREADS)), dim3(THREADS), 0, s, n, geo,
                       p->gamma, sb, q, tape, rhs_bar, dxdt_bar, ubuf, NFAr * NRr, 0, qbd);
  if ((rc = hip_check(ctx, hipGetLastError(), "adjoint Ubar"))) return rc; }
  if (lane_pairs) {
    Prof pf(ctx, "k_adj_orec");
    hipLaunchKernelGGL(k_adj_orec<false>, dim3(grid_for((int64_t)n * NRr, THREADS)),
                       dim3(THREADS), 0, s, n, aos, ubuf, orec);
    if ((rc = hip_check(ctx, hipGetLastError(), "adjoint owner records"))) return rc;
  }
  // FP32 pair records in the mixed form
  const bool rec32 = p->precision == PHB_MIXED;
  float* rec_f = reinterpret_cast<float*>(rec);
  // the pipelined schedule stages 16-byte pieces: the tape's blocks (a
  // caller's tape) must be 16-byte aligned, else the one-shot schedule runs
  const bool piped = !lane_pairs && ctx->adj_pairs_mode == 2 &&
                     (reinterpret_cast<uintptr_t>(aos) & 15) == 0;
  const bool tiled = !lane_pairs && ctx->adj_pairs_mode == 3;
  const int ts = PAIR_TILE;
  if (piped) {
    Prof pf(ctx, stab ? "k_adj_pairs_p<stab>" : "k_adj_pairs_p");
    if (stab) {
      if (rec32) launch_pairs_p<true>(s, a, geo, fq, t_pos, aos, ubuf, rec_f, own, slot_order);
      else launch_pairs_p<true>(s, a, geo, fq, t_pos, aos, ubuf, rec, own, slot_order);
    } else {
      if (rec32) launch_pairs_p<false>(s, a, geo, fq, t_pos, aos, ubuf, rec_f, own, slot_order);
      else launch_pairs_p<false>(s, a, geo, fq, t_pos, aos, ubuf, rec, own, slot_order);
    }
    if ((rc = hip_check(ctx, hipGetLastError(), "adjoint pairs"))) return rc;
  } else if (tiled) {
    Prof pf(ctx, stab ? "k_adj_pairs_t<stab>" : "k_adj_pairs_t");
    if (stab) {
      if (rec32) launch_pairs_t<true>(s, a, ts, tstart, ntiles, tbound, geo, fq, t_pos, aos, ubuf, rec_f, own, slot_order);
      else launch_pairs_t<true>(s, a, ts, tstart, ntiles, tbound, geo, fq, t_pos, aos, ubuf, rec, own, slot_order);
    } else {
      if (rec32) launch_pairs_t<false>(s, a, ts, tstart, ntiles, tbound, geo, fq, t_pos, aos, ubuf, rec_f, own, slot_order);
      else launch_pairs_t<false>(s, a, ts, tstart, ntiles, tbound, geo, fq, t_pos, aos, ubuf, rec, own, slot_order);
    }
    if ((rc = hip_check(ctx, hipGetLastError(), "adjoint pairs"))) return rc;
  } else if (!lane_pairs) {
    // the stabilised shape runs a wavefront-per-owner schedule only
    Prof pf(ctx, stab ? "k_adj_pairs_w<stab>" : "k_adj_pairs_w");
    if (stab) {
      if (rec32) launch_pairs_w<true>(s, a, geo, fq, t_pos, aos, ubuf, rec_f, own, slot_order);
      else launch_pairs_w<true>(s, a, geo, fq, t_pos, aos, ubuf, rec, own, slot_order);
    } else {
      if (rec32) launch_pairs_w<false>(s, a, geo, fq, t_pos, aos, ubuf, rec_f, own, slot_order);
      else launch_pairs_w<false>(s, a, geo, fq, t_pos, aos, ubuf, rec, own, slot_order);
    }
    if ((rc = hip_check(ctx, hipGetLastError(), "adjoint pairs"))) return rc;
  } else {
    if (nnz > 0) {
      Prof pf(ctx, "k_adj_pairs");
      if (rec32)
        hipLaunchKernelGGL((k_adj_pairs<float>), dim3(grid_for(nnz, PAIRS_PER_BLOCK)),
                           dim3(PAIRS_PER_BLOCK), 0, s, n, nnz, geo, a.off, a.idx, t_pos, a.box,
                           a.rf_ratio, a.wkind, fq, orec, rec_f, own, wpart, slot_order);
      else
        hipLaunchKernelGGL((k_adj_pairs<double>), dim3(grid_for(nnz, PAIRS_PER_BLOCK)),
                           dim3(PAIRS_PER_BLOCK), 0, s, n, nnz, geo, a.off, a.idx, t_pos, a.box,
                           a.rf_ratio, a.wkind, fq, orec, rec, own, wpart, slot_order);
      if ((rc = hip_check(ctx, hipGetLastError(), "adjoint pairs"))) return rc;
    }
    Prof pf(ctx, "k_adj_combine");
    hipLaunchKernelGGL(k_adj_combine, dim3(grid_for(n, THREADS)), dim3(THREADS), 0, s, n, a.off,
                       wpart, own);
    if ((rc = hip_check(ctx, hipGetLastError(), "adjoint combine"))) return rc;
  }
  if (slot_order && nnz > 0) {
    Prof pf(ctx, "k_invert");
    hipLaunchKernelGGL(k_invert, dim3(grid_for(nnz, THREADS)), dim3(THREADS), 0, s, nnz,
                       a.off + n, t_pos, t_slot);
    if ((rc = hip_check(ctx, hipGetLastError(), "adjoint invert"))) return rc;
  }
  const int32_t* tsl = slot_order ? t_slot : nullptr;
  Prof pf(ctx, "k_adj_gather");
  const int gl = ctx->lanes_gather;
  if (stab) {
    if (rec32) launch_gather<true>(s, gl, tiled ? tbound : nullptr, n, t_offsets, tsl, t_src, (const float*)rec_f, own, qbd, q_bar, pos_bar);
    else launch_gather<true>(s, gl, tiled ? tbound : nullptr, n, t_offsets, tsl, t_src, (const double*)rec, own, qbd, q_bar, pos_bar);
  } else {
    if (rec32) launch_gather<false>(s, gl, tiled ? tbound : nullptr, n, t_offsets, tsl, t_src, (const float*)rec_f, own, qbd, q_bar, pos_bar);
    else launch_gather<false>(s, gl, tiled ? tbound : nullptr, n, t_offsets, tsl, t_src, (const double*)rec, own, qbd, q_bar, pos_bar);
  }
  return hip_check(ctx, hipGetLastError(), "adjoint gather");
}

}  // namespace phb
