// Equilibrated FP64 Cholesky of one particle's 20x20 moment matrix, held by
// the four lanes of a quad (lane l owns rows l, l+4, l+8, l+12, l+16), and
// the triangular solves against it.  Used by every kernel that needs A^{-1}.
#pragma once

#include <type_traits>

#include "device.hpp"

namespace phb {

template <int B, int E, class F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}

// 1 / sqrt(d) for d > 0 (normal): the hardware estimate, then two Newton
// steps r <- r + (r / 2)(1 - d r^2).  Each step squares the relative error, so
// the result is within a few units in the last place.
__device__ __forceinline__ double rsqrt_nr(double d) {
  double r = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d * r, r, 1.0);
    r = fma(0.5 * r, e, r);
  }
  return r;
}

// Pivots and diagonal entries at or below this are treated as non-positive.
constexpr double CHOL_TINY = 1e-280;

// Row rho of a lane lives at a[aoff(rho) .. aoff(rho) + 4 rho + 3]: the
// longest row any lane can own among rows 4 rho .. 4 rho + 3.  Once the
// factorization is done, the entries on and right of a lane's own diagonal
// are zero (the diagonal's reciprocal is kept in inv_own), so the solves can
// apply every entry of a column without asking which lane owns the pivot.
__host__ __device__ constexpr int chol_aoff(int rho) { return 2 * rho * (rho + 1); }

struct EntryTab {
  unsigned char v[NBASIS * NBASIS];
};
constexpr EntryTab make_entry_tab() {
  EntryTab t{};
  for (int r = 0; r < NBASIS; ++r)
    for (int c = 0; c < NBASIS; ++c) t.v[r * NBASIS + c] = (unsigned char)entry_moment(r, c);
  return t;
}

struct QuadChol {
  double a[60];      // own rows of L (equilibrated)
  double s_own[5];   // equilibration scale of the own rows
  double inv_own[5]; // 1 / L_kk of the own rows
  bool ok;
  double ldmin, ldmax;
};

// Loads A from the moments (SoA [84][ld]), equilibrates A_hat = S A S with
// S = diag(1/sqrt(A_rr)) and factors A_hat = L L^T.  tab is the entry->moment
// table in constant memory.  interp: the 19-monomial interpolating fit (the
// constant's row and column replaced by the identity's).
__device__ __forceinline__ void quad_chol_factor(QuadChol& c, const EntryTab& tab,
                                                 const double* __restrict__ mom, int64_t ld,
                                                 int ii, int l, bool interp = false) {
  double dg[5];
  sfor<0, 5>([&](auto R) {
    constexpr int rho = R;
    const int r = 4 * rho + l;
    sfor<0, 4 * rho + 4>([&](auto C) {
      constexpr int cc = C;
      c.a[chol_aoff(rho) + cc] = mom[(int64_t)tab.v[r * NBASIS + cc] * ld + ii];
    });
    dg[rho] = mom[(int64_t)tab.v[r * NBASIS + r] * ld + ii];
  });
  if (interp) {
    // interpolating fit: the constant monomial leaves the basis.  Its row and
    // column become those of the identity, which decouples the other 19:
    // their block is factored as it is, and every inverse row 1.. has a zero
    // constant entry.
    sfor<0, 5>([&](auto R) {
      constexpr int rho = R;
      c.a[chol_aoff(rho)] = (rho == 0 && l == 0) ? 1.0 : 0.0;
    });
    if (l == 0) dg[0] = 1.0;
  }
  c.ok = true;
  sfor<0, 5>([&](auto R) {
    constexpr int rho = R;
    c.ok = c.ok && (dg[rho] > CHOL_TINY);
    c.s_own[rho] = rsqrt_nr(dg[rho] > CHOL_TINY ? dg[rho] : 1.0);
  });
  c.ok = quad_min(c.ok ? 1.0 : 0.0) > 0.5;  // the same verdict on all four lanes
  {
    double s_all[NBASIS];
    sfor<0, NBASIS>([&](auto C) {
      constexpr int cc = C;
      s_all[cc] = quad_bcast<cc & 3>(c.s_own[cc >> 2]);
    });
    sfor<0, 5>([&](auto R) {
      constexpr int rho = R;
      sfor<0, 4 * rho + 4>([&](auto C) {
        constexpr int cc = C;
        c.a[chol_aoff(rho) + cc] *= c.s_own[rho] * s_all[cc];
      });
    });
  }
  c.ldmin = 1e300;
  c.ldmax = 0.0;
  sfor<0, NBASIS>([&](auto K) {
    constexpr int k = K;
    constexpr int o = k & 3;
    constexpr int rk = k >> 2;
    const double dkk = quad_bcast<o>(c.a[chol_aoff(rk) + k]);
    c.ok = c.ok && (dkk > CHOL_TINY);
    const double dpos = dkk > CHOL_TINY ? dkk : 1.0;
    const double inv = rsqrt_nr(dpos);
    const double lkk = dpos * inv;
    c.ldmin = fmin(c.ldmin, lkk);
    c.ldmax = fmax(c.ldmax, lkk);
    c.inv_own[rk] = (l == o) ? inv : c.inv_own[rk];
    sfor<rk, 5>([&](auto R) {
      constexpr int rho = R;
      c.a[chol_aoff(rho) + k] *= inv;
    });
    double colk[NBASIS];
    sfor<k + 1, NBASIS>([&](auto C) {
      constexpr int cc = C;
      colk[cc] = quad_bcast<cc & 3>(c.a[chol_aoff(cc >> 2) + k]);
    });
    sfor<rk, 5>([&](auto R) {
      constexpr int rho = R;
      sfor<k + 1, 4 * rho + 4>([&](auto C) {
        constexpr int cc = C;
        c.a[chol_aoff(rho) + cc] = fma(-c.a[chol_aoff(rho) + k], colk[cc], c.a[chol_aoff(rho) + cc]);
      });
    });
  });
  // row 4 rho + l keeps columns < 4 rho + l only
  sfor<0, 5>([&](auto R) {
    constexpr int rho = R;
    sfor<0, 4>([&](auto C) {
      constexpr int cc = C;
      if (l <= cc) c.a[chol_aoff(rho) + 4 * rho + cc] = 0.0;
    });
  });
}

// Status of the factorization: too few neighbors, singular, or fine.
__device__ __forceinline__ int quad_chol_status(const QuadChol& c, int nnb) {
  const double rc = c.ldmin / c.ldmax;
  if (nnb < NBASIS) return 1;
  if (!c.ok || !(rc * rc >= 1e-12)) return 2;
  return 0;
}

// x = A_hat^{-1} y for own rows; y is overwritten with the forward solution.
// K0: index of the first possibly nonzero entry of y.  ADAPT: the right-hand
// side is not given but chosen entry by entry as +-1, with the sign that
// makes the forward solution grow most (LINPACK's condition estimator); y
// must enter as zeros.
template <int K0, bool ADAPT = false>
__device__ __forceinline__ void quad_chol_solve(const QuadChol& c, int l, double (&y)[5],
                                                double (&x)[5]) {
  sfor<K0, NBASIS>([&](auto K) {
    constexpr int k = K;
    constexpr int o = k & 3;
    constexpr int rk = k >> 2;
    // the owner lane o holds y_k and 1 / L_kk
    double t = y[rk];
    if constexpr (ADAPT) t += t >= 0.0 ? 1.0 : -1.0;
    const double yk = quad_bcast<o>(t * c.inv_own[rk]);
    sfor<rk + 1, 5>([&](auto R) {
      constexpr int rho = R;
      y[rho] = fma(-c.a[chol_aoff(rho) + k], yk, y[rho]);
    });
    const double upd = fma(-c.a[chol_aoff(rk) + k], yk, y[rk]);  // no change for l < o
    y[rk] = (l == o) ? yk : upd;
  });
  sfor<0, 5>([&](auto R) { x[R] = y[R]; });
  sfor<0, NBASIS>([&](auto KK) {
    constexpr int k = NBASIS - 1 - KK;
    constexpr int o = k & 3;
    constexpr int rk = k >> 2;
    double part = 0.0;
    sfor<rk, 5>([&](auto R) {  // row block rk adds zeros on lanes l <= o
      constexpr int rho = R;
      part = fma(c.a[chol_aoff(rho) + k], x[rho], part);
    });
    part = group_sum<4>(part);
    const double xk = (y[rk] - part) * c.inv_own[rk];  // valid on the owner lane
    x[rk] = (l == o) ? xk : x[rk];
  });
}

// Row t of A^{-1} (own entries): A^{-1} = S A_hat^{-1} S.
template <int T>
__device__ __forceinline__ void quad_chol_inverse_row(const QuadChol& c, int l, double (&out)[5]) {
  double y[5];
  const double sT = quad_bcast<T & 3>(c.s_own[T >> 2]);
  sfor<0, 5>([&](auto R) {
    constexpr int rho = R;
    y[rho] = (4 * rho + l == T) ? sT : 0.0;
  });
  double x[5];
  quad_chol_solve<T>(c, l, y, x);
  sfor<0, 5>([&](auto R) { out[R] = x[R] * c.s_own[R]; });
}

// NR independent solves x_r = A_hat^{-1} y_r in lockstep: each elimination
// step serves all right-hand sides, which gives the scheduler NR independent
// chains between the quad broadcasts.  K0 as in quad_chol_solve.
template <int K0, int NR>
__device__ __forceinline__ void quad_chol_solve_n(const QuadChol& c, int l, double (&y)[NR][5],
                                                  double (&x)[NR][5]) {
  sfor<K0, NBASIS>([&](auto K) {
    constexpr int k = K;
    constexpr int o = k & 3;
    constexpr int rk = k >> 2;
    double yk[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) yk[r] = quad_bcast<o>(y[r][rk] * c.inv_own[rk]);
    sfor<rk + 1, 5>([&](auto R) {
      constexpr int rho = R;
#pragma unroll
      for (int r = 0; r < NR; ++r) y[r][rho] = fma(-c.a[chol_aoff(rho) + k], yk[r], y[r][rho]);
    });
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const double upd = fma(-c.a[chol_aoff(rk) + k], yk[r], y[r][rk]);  // no change for l < o
      y[r][rk] = (l == o) ? yk[r] : upd;
    }
  });
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int rho = 0; rho < 5; ++rho) x[r][rho] = y[r][rho];
  sfor<0, NBASIS>([&](auto KK) {
    constexpr int k = NBASIS - 1 - KK;
    constexpr int o = k & 3;
    constexpr int rk = k >> 2;
    double part[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) part[r] = 0.0;
    sfor<rk, 5>([&](auto R) {  // row block rk adds zeros on lanes l <= o
      constexpr int rho = R;
#pragma unroll
      for (int r = 0; r < NR; ++r) part[r] = fma(c.a[chol_aoff(rho) + k], x[r][rho], part[r]);
    });
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      part[r] = group_sum<4>(part[r]);
      const double xk = (y[r][rk] - part[r]) * c.inv_own[rk];  // valid on the owner lane
      x[r][rk] = (l == o) ? xk : x[r][rk];
    }
  });
}

// Rows T0 .. T0 + NR - 1 of A^{-1} (own entries) by one lockstep solve.
template <int T0, int NR>
__device__ __forceinline__ void quad_chol_inverse_rows(const QuadChol& c, int l,
                                                       double (&out)[NR][5]) {
  double y[NR][5];
  sfor<0, NR>([&](auto RI) {
    constexpr int T = T0 + RI;
    const double sT = quad_bcast<T & 3>(c.s_own[T >> 2]);
    sfor<0, 5>([&](auto R) {
      constexpr int rho = R;
      y[RI][rho] = (4 * rho + l == T) ? sT : 0.0;
    });
  });
  quad_chol_solve_n<T0, NR>(c, l, y, out);
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int rho = 0; rho < 5; ++rho) out[r][rho] *= c.s_own[rho];
}

// Largest squared 2-norm among rows T0 .. T0 + NR - 1 of the equilibrated
// inverse A_hat^{-1}, given those rows of A^{-1} (own entries, as returned by
// quad_chol_inverse_rows): A_hat^{-1}[T][b] = A^{-1}[T][b] / (s_T s_b).  The
// same value on all four lanes.
template <int T0, int NR>
__device__ __forceinline__ double quad_rows_hat_norm2(const QuadChol& c, int l,
                                                      const double (&rows)[NR][5]) {
  double m = 0.0;
  sfor<0, NR>([&](auto RI) {
    constexpr int T = T0 + RI;
    double part = 0.0;
    sfor<0, 5>([&](auto R) {
      const double e = rows[RI][R] / c.s_own[R];
      part = fma(e, e, part);
    });
    part = group_sum<4>(part);
    const double sT = quad_bcast<T & 3>(c.s_own[T >> 2]);
    m = fmax(m, part / (sT * sT));
  });
  return m;
}

// Estimate of the 2-norm of A_hat^{-1} (the equilibrated matrix), from below
// and in practice within a small factor: x = A_hat^{-1} e with the signs of e
// chosen for growth as above, then one power step z = A_hat^{-1} x and
// ||z|| / ||x||.
__device__ __forceinline__ double quad_chol_inv_norm_est(const QuadChol& c, int l) {
  double y[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double x[5], z[5];
  quad_chol_solve<0, true>(c, l, y, x);
  sfor<0, 5>([&](auto R) { y[R] = x[R]; });
  quad_chol_solve<0>(c, l, y, z);
  double xx = 0.0, zz = 0.0;
  sfor<0, 5>([&](auto R) {
    xx = fma(x[R], x[R], xx);
    zz = fma(z[R], z[R], zz);
  });
  xx = group_sum<4>(xx);
  zz = group_sum<4>(zz);
  return sqrt(zz / xx);
}

// A^{-1} b for a general right-hand side b given by its own rows.
__device__ __forceinline__ void quad_chol_apply_inverse(const QuadChol& c, int l,
                                                        const double (&b)[5], double (&out)[5]) {
  double y[5];
  sfor<0, 5>([&](auto R) { y[R] = b[R] * c.s_own[R]; });
  double x[5];
  quad_chol_solve<0>(c, l, y, x);
  sfor<0, 5>([&](auto R) { out[R] = x[R] * c.s_own[R]; });
}

}  // namespace phb
