// Phurbas MLS / ideal-MHD oracle: plain, slow, obviously-checkable CPU FP64 code.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file; only the test-suite, the smoke check and the CPU-baseline
// leg of the benchmark do.  It shares no code, header, table or helper with
// the GPU library.
//
// What it computes (Phurbas paper II, McNally, Maron & Mac Low 2012):
//  * neighbor sets: every particle j (i itself included) inside the sphere of
//    radius r_f,i = 2.3 lambda_i about particle i (Sec. 2, Sec. 2.1: a strict,
//    fixed-radius, non-mutual search);  brute force over all j;
//  * a local third-order polynomial moving-least-squares fit of each field
//    around each particle (Sec. 2), solved by Householder QR of the weighted,
//    column-scaled design matrix (a different algorithm from the GPU's
//    normal-equation Cholesky);
//  * the ideal-MHD Lagrangian time derivatives from the fitted gradients
//    (Sec. 2; the evolution equations of App. A with zero viscosity), and
//    optionally the non-ideal stabilisers of Sec. 2 (bulk viscosity and div-B
//    diffusion, from the fitted second derivatives);
//  * the second-order predictor-corrector step (Sec. 2);
//  * reverse-mode derivatives of the time derivatives (hand-derived matrix
//    calculus in full 20x20 form) and a complex-step forward evaluation used
//    to pin them.
//
// Readings where the paper is silent (weight function, equation of state,
// induction form, predictor-corrector form, singularity tests) are listed in
// the design notes; each place that takes one says so below.
//
// Build: g++ -O2 -std=c++17 -fopenmp -ffp-contract=off -fPIC -shared
// (-ffp-contract=off keeps the neighbor distance test free of fused
// multiply-adds, so it is the exact FP64 expression stated below.)

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <climits>
#include <omp.h>

namespace {

using cd = std::complex<double>;

inline double re(double x) { return x; }
inline double re(const cd& x) { return x.real(); }

// Monomial exponents (a,b,c) of xi^a eta^b zeta^c, degree <= 3, in the order
// 1; x,y,z; xx,xy,xz,yy,yz,zz; xxx,xxy,xxz,xyy,xyz,xzz,yyy,yyz,yzz,zzz.
const int EXPO[20][3] = {
    {0, 0, 0},
    {1, 0, 0}, {0, 1, 0}, {0, 0, 1},
    {2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2},
    {3, 0, 0}, {2, 1, 0}, {2, 0, 1}, {1, 2, 0}, {1, 1, 1},
    {1, 0, 2}, {0, 3, 0}, {0, 2, 1}, {0, 1, 2}, {0, 0, 3}};

struct Setup {
  double L[3];
  int periodic[3];
  double rf_ratio;  // r_f / lambda (2.3 in the paper)
  double gamma;     // adiabatic index
  int weight;       // 0: (1-q)^3 with q = d^2 / r_f^2 ; 1: unit weight
  int fit;          // 0: full 20-monomial fit; 1: 19-monomial interpolating fit
  // Non-ideal stabilisers (Sec. 2): coefficients of the grid-scale and the
  // adaptive bulk viscosity and of the div-B diffusion; all zero is ideal MHD.
  double visc_grid = 0.0, visc_adapt = 0.0, divb_diff = 0.0;
  bool stabilised() const { return visc_grid != 0.0 || visc_adapt != 0.0 || divb_diff != 0.0; }
};

// Minimum-image displacement along one axis: subtract or add one box length
// when the raw difference is beyond half the box.  Comparisons use the real
// part so that a complex-step perturbation never changes the branch.
template <class T>
T min_image(T d, double L, int periodic) {
  if (periodic) {
    if (re(d) > 0.5 * L)
      d -= L;
    else if (re(d) < -0.5 * L)
      d += L;
  }
  return d;
}

// The neighbor predicate, written as the exact FP64 expression:
//   d2 = (dx*dx + dy*dy) + dz*dz ;  r = rf_ratio * lambda_i ;  d2 < r*r
// Strict inequality: a pair at exactly r_f is excluded.  i itself (d2 = 0)
// is included.
bool in_sphere(const double* pos, int64_t n, int64_t i, int64_t j,
               const double* lambda, const Setup& s) {
  double dx = min_image(pos[j] - pos[i], s.L[0], s.periodic[0]);
  double dy = min_image(pos[n + j] - pos[n + i], s.L[1], s.periodic[1]);
  double dz = min_image(pos[2 * n + j] - pos[2 * n + i], s.L[2], s.periodic[2]);
  double d2 = (dx * dx + dy * dy) + dz * dz;
  double r = s.rf_ratio * lambda[i];
  return d2 < r * r;
}

// Value of monomial k at (x, y, z).
template <class T>
T monomial(int k, const T& x, const T& y, const T& z) {
  T v = T(1.0);
  for (int e = 0; e < EXPO[k][0]; ++e) v *= x;
  for (int e = 0; e < EXPO[k][1]; ++e) v *= y;
  for (int e = 0; e < EXPO[k][2]; ++e) v *= z;
  return v;
}

// Partial derivative of monomial k with respect to coordinate `axis`.
template <class T>
T monomial_deriv(int k, int axis, const T& x, const T& y, const T& z) {
  int ex[3] = {EXPO[k][0], EXPO[k][1], EXPO[k][2]};
  if (ex[axis] == 0) return T(0.0);
  T factor = T(double(ex[axis]));
  ex[axis] -= 1;
  T v = factor;
  for (int e = 0; e < ex[0]; ++e) v *= x;
  for (int e = 0; e < ex[1]; ++e) v *= y;
  for (int e = 0; e < ex[2]; ++e) v *= z;
  return v;
}

// Reading of the weight function (Paper I, which defines it, is not part of
// paper II): w = (1 - q)^3 with q = d^2 / r_f^2, positive inside the sphere
// and C^2-smooth to zero at its edge.  Option 1 is unit weight.
template <class T>
T weight_of(const T& q, int kind) {
  if (kind == 1) return T(1.0);
  T u = T(1.0) - q;
  return u * u * u;
}
template <class T>
T weight_deriv(const T& q, int kind) {  // dw/dq
  if (kind == 1) return T(0.0);
  T u = T(1.0) - q;
  return T(-3.0) * u * u;
}

// Geometry of one particle's neighborhood: displacements, scaled coordinates
// xi = d / lambda_i, normalized squared distance q and weight w.
template <class T>
struct Local {
  int m = 0;
  std::vector<int64_t> nb;     // neighbor indices
  std::vector<T> d;            // m x 3 min-image displacements x_j - x_i
  std::vector<T> xi;           // m x 3 scaled coordinates
  std::vector<T> q;            // m normalized squared distances
  std::vector<T> w;            // m weights
};

template <class T>
void build_local(int64_t n, int64_t i, const T* pos, const double* lambda,
                 const int32_t* nb, int m, const Setup& s, Local<T>& loc) {
  loc.m = m;
  loc.nb.assign(nb, nb + m);
  loc.d.assign(3 * m, T(0.0));
  loc.xi.assign(3 * m, T(0.0));
  loc.q.assign(m, T(0.0));
  loc.w.assign(m, T(0.0));
  const double lam = lambda[i];
  const double r = s.rf_ratio * lam;
  for (int k = 0; k < m; ++k) {
    int64_t j = nb[k];
    for (int a = 0; a < 3; ++a) {
      T dd = min_image(pos[a * n + j] - pos[a * n + i], s.L[a], s.periodic[a]);
      loc.d[3 * k + a] = dd;
      loc.xi[3 * k + a] = dd / lam;
    }
    T d2 = loc.d[3 * k] * loc.d[3 * k] + loc.d[3 * k + 1] * loc.d[3 * k + 1] +
           loc.d[3 * k + 2] * loc.d[3 * k + 2];
    loc.q[k] = d2 / (r * r);
    loc.w[k] = weight_of(loc.q[k], s.weight);
  }
}

// Weighted least squares by Householder QR.
//   minimize sum_j w_j (p(xi_j) . c - b_j)^2     over c in R^ncol
// Design matrix M = diag(sqrt(w)) P S, S = diag(1/column norms).  M = Q R.
// Complex-step safe: all "norms" are sqrt(sum x^2) without conjugation and
// every sign choice uses real parts.
template <class T>
struct QR {
  int m = 0, ncol = 0;
  std::vector<T> R;      // ncol x ncol upper triangle
  std::vector<T> scale;  // column scaling S
  int status = 0;        // 0 ok, 1 too few neighbors, 2 singular
};

// Basis columns used by the fit kind: all 20 monomials, or the 19 that
// vanish at the center (interpolating fit).
inline int first_column(int fit) { return fit == 1 ? 1 : 0; }

template <class T>
void wls_solve(const Local<T>& loc, int fit, int nrhs, const std::vector<T>& rhs /* m x nrhs */,
               QR<T>& qr, std::vector<T>& coef /* 20 x nrhs, unused rows zero */) {
  const int m = loc.m;
  const int c0 = first_column(fit);
  const int ncol = 20 - c0;
  qr.m = m;
  qr.ncol = ncol;
  qr.status = 0;
  coef.assign(20 * nrhs, T(0.0));
  // Reading: fewer than 20 samples (the particle itself included) cannot
  // determine the cubic fit; flag it.
  if (m < 20) {
    qr.status = 1;
    return;
  }
  std::vector<T> M(m * ncol), B(m * nrhs);
  for (int k = 0; k < m; ++k) {
    T sw = std::sqrt(loc.w[k]);
    const T& x = loc.xi[3 * k];
    const T& y = loc.xi[3 * k + 1];
    const T& z = loc.xi[3 * k + 2];
    for (int c = 0; c < ncol; ++c) M[k * ncol + c] = sw * monomial(c + c0, x, y, z);
    for (int f = 0; f < nrhs; ++f) B[k * nrhs + f] = sw * rhs[k * nrhs + f];
  }
  qr.scale.assign(ncol, T(1.0));
  for (int c = 0; c < ncol; ++c) {
    T s2 = T(0.0);
    for (int k = 0; k < m; ++k) s2 += M[k * ncol + c] * M[k * ncol + c];
    if (re(s2) <= 0.0) {
      qr.status = 2;
      return;
    }
    T sc = T(1.0) / std::sqrt(s2);
    qr.scale[c] = sc;
    for (int k = 0; k < m; ++k) M[k * ncol + c] *= sc;
  }
  qr.R.assign(ncol * ncol, T(0.0));
  std::vector<T> v(m);
  for (int c = 0; c < ncol; ++c) {
    T nrm2 = T(0.0);
    for (int k = c; k < m; ++k) nrm2 += M[k * ncol + c] * M[k * ncol + c];
    T nrm = std::sqrt(nrm2);
    T alpha = re(M[c * ncol + c]) >= 0.0 ? -nrm : nrm;
    for (int k = 0; k < m; ++k) v[k] = T(0.0);
    for (int k = c; k < m; ++k) v[k] = M[k * ncol + c];
    v[c] -= alpha;
    T vtv = T(0.0);
    for (int k = c; k < m; ++k) vtv += v[k] * v[k];
    if (re(vtv) != 0.0) {
      for (int cc = c; cc < ncol; ++cc) {
        T dot = T(0.0);
        for (int k = c; k < m; ++k) dot += v[k] * M[k * ncol + cc];
        T fac = T(2.0) * dot / vtv;
        for (int k = c; k < m; ++k) M[k * ncol + cc] -= fac * v[k];
      }
      for (int f = 0; f < nrhs; ++f) {
        T dot = T(0.0);
        for (int k = c; k < m; ++k) dot += v[k] * B[k * nrhs + f];
        T fac = T(2.0) * dot / vtv;
        for (int k = c; k < m; ++k) B[k * nrhs + f] -= fac * v[k];
      }
    }
    for (int cc = c; cc < ncol; ++cc) qr.R[c * ncol + cc] = M[c * ncol + cc];
  }
  // Reading of the singularity test: the scaled problem's reciprocal
  // condition estimate (min |R_kk| / max |R_kk|)^2 below 1e-12 flags the fit.
  double dmin = 1e300, dmax = 0.0;
  for (int c = 0; c < ncol; ++c) {
    double a = std::abs(re(qr.R[c * ncol + c]));
    dmin = std::min(dmin, a);
    dmax = std::max(dmax, a);
  }
  if (!(dmax > 0.0) || !(dmin > 0.0) || (dmin / dmax) * (dmin / dmax) < 1e-12) {
    qr.status = 2;
    return;
  }
  // Back substitution R y = (Q^T b)[0:ncol], then c = S y.
  for (int f = 0; f < nrhs; ++f) {
    std::vector<T> y(ncol);
    for (int r = ncol - 1; r >= 0; --r) {
      T acc = B[r * nrhs + f];
      for (int cc = r + 1; cc < ncol; ++cc) acc -= qr.R[r * ncol + cc] * y[cc];
      y[r] = acc / qr.R[r * ncol + r];
    }
    for (int c = 0; c < ncol; ++c) coef[(c + c0) * nrhs + f] = qr.scale[c] * y[c];
  }
}

// Column `col` (basis index) of A^{-1}, A = P^T W P, from the factorization:
// A = S^{-1} R^T R S^{-1}  =>  A^{-1} = S R^{-1} R^{-T} S.  Rows/cols of the
// dropped constant monomial (interpolating fit) are zero.
template <class T>
std::vector<T> ainv_column(const QR<T>& qr, int fit, int col) {
  const int c0 = first_column(fit);
  const int ncol = qr.ncol;
  std::vector<T> out(20, T(0.0));
  if (col < c0) return out;
  const int cc = col - c0;
  // R^T u = S e_cc
  std::vector<T> u(ncol, T(0.0));
  for (int r = 0; r < ncol; ++r) {
    T acc = (r == cc) ? qr.scale[cc] : T(0.0);
    for (int k = 0; k < r; ++k) acc -= qr.R[k * ncol + r] * u[k];
    u[r] = acc / qr.R[r * ncol + r];
  }
  // R v = u
  std::vector<T> v(ncol, T(0.0));
  for (int r = ncol - 1; r >= 0; --r) {
    T acc = u[r];
    for (int k = r + 1; k < ncol; ++k) acc -= qr.R[r * ncol + k] * v[k];
    v[r] = acc / qr.R[r * ncol + r];
  }
  for (int r = 0; r < ncol; ++r) out[r + c0] = qr.scale[r] * v[r];
  return out;
}

// Ideal-MHD Lagrangian time derivatives at one particle from its values and
// physical gradients (Sec. 2; App. A with zero bulk viscosity):
//   drho/dt   = -rho div V
//   dV/dt     = ( -grad P + (curl B) x B ) / rho
//   dB/dt     = (B . grad) V - B div V
//   dsigma/dt = -gamma sigma div V
// Readings: P = (gamma - 1) sigma (sigma is the internal energy density);
// Heaviside-Lorentz units (no 4 pi); the induction equation keeps no
// V (div B) term, so a uniform velocity shift leaves every derivative
// unchanged; no bulk viscosity or div-B diffusion (ideal MHD).
// Field order q = (rho, Vx, Vy, Vz, Bx, By, Bz, sigma); grad[f][b] = d q_f / d x_b.
template <class T>
void mhd_point(const T* qv, const T grad[8][3], double gamma, T* out) {
  const T rho = qv[0];
  const T V[3] = {qv[1], qv[2], qv[3]};
  const T B[3] = {qv[4], qv[5], qv[6]};
  const T sig = qv[7];
  T gV[3][3], gB[3][3], gS[3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      gV[a][b] = grad[1 + a][b];
      gB[a][b] = grad[4 + a][b];
    }
  for (int b = 0; b < 3; ++b) gS[b] = grad[7][b];
  T divV = gV[0][0] + gV[1][1] + gV[2][2];
  T J[3] = {gB[2][1] - gB[1][2], gB[0][2] - gB[2][0], gB[1][0] - gB[0][1]};
  T F[3] = {J[1] * B[2] - J[2] * B[1], J[2] * B[0] - J[0] * B[2], J[0] * B[1] - J[1] * B[0]};
  out[0] = -rho * divV;
  for (int a = 0; a < 3; ++a) out[1 + a] = (-(gamma - 1.0) * gS[a] + F[a]) / rho;
  for (int a = 0; a < 3; ++a) {
    T adv = B[0] * gV[a][0] + B[1] * gV[a][1] + B[2] * gV[a][2];
    out[4 + a] = adv - B[a] * divV;
  }
  out[7] = -gamma * sig * divV;
}

// Reverse mode of mhd_point: given out_bar (8), accumulate into q_bar (8)
// and grad_bar[8][3].  Written term by term from the forward expressions.
void mhd_point_adjoint(const double* qv, const double grad[8][3], double gamma,
                       const double* ob, double* qb, double gb[8][3]) {
  const double rho = qv[0];
  const double B[3] = {qv[4], qv[5], qv[6]};
  const double sig = qv[7];
  double gV[3][3], gB[3][3], gS[3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      gV[a][b] = grad[1 + a][b];
      gB[a][b] = grad[4 + a][b];
    }
  for (int b = 0; b < 3; ++b) gS[b] = grad[7][b];
  double divV = gV[0][0] + gV[1][1] + gV[2][2];
  double J[3] = {gB[2][1] - gB[1][2], gB[0][2] - gB[2][0], gB[1][0] - gB[0][1]};
  double F[3] = {J[1] * B[2] - J[2] * B[1], J[2] * B[0] - J[0] * B[2], J[0] * B[1] - J[1] * B[0]};

  double divV_b = 0.0, rho_b = 0.0, sig_b = 0.0;
  double B_b[3] = {0, 0, 0}, F_b[3] = {0, 0, 0}, J_b[3] = {0, 0, 0};
  double gV_b[3][3] = {{0}}, gB_b[3][3] = {{0}}, gS_b[3] = {0, 0, 0};
  // out[0] = -rho divV
  rho_b += -divV * ob[0];
  divV_b += -rho * ob[0];
  // out[1+a] = (-(g-1) gS[a] + F[a]) / rho
  for (int a = 0; a < 3; ++a) {
    double num = -(gamma - 1.0) * gS[a] + F[a];
    gS_b[a] += -(gamma - 1.0) * ob[1 + a] / rho;
    F_b[a] += ob[1 + a] / rho;
    rho_b += -num / (rho * rho) * ob[1 + a];
  }
  // out[4+a] = sum_b B[b] gV[a][b] - B[a] divV
  for (int a = 0; a < 3; ++a) {
    for (int b = 0; b < 3; ++b) {
      B_b[b] += gV[a][b] * ob[4 + a];
      gV_b[a][b] += B[b] * ob[4 + a];
    }
    B_b[a] += -divV * ob[4 + a];
    divV_b += -B[a] * ob[4 + a];
  }
  // out[7] = -gamma sig divV
  sig_b += -gamma * divV * ob[7];
  divV_b += -gamma * sig * ob[7];
  // F = J x B
  J_b[1] += B[2] * F_b[0];  B_b[2] += J[1] * F_b[0];
  J_b[2] += -B[1] * F_b[0]; B_b[1] += -J[2] * F_b[0];
  J_b[2] += B[0] * F_b[1];  B_b[0] += J[2] * F_b[1];
  J_b[0] += -B[2] * F_b[1]; B_b[2] += -J[0] * F_b[1];
  J_b[0] += B[1] * F_b[2];  B_b[1] += J[0] * F_b[2];
  J_b[1] += -B[0] * F_b[2]; B_b[0] += -J[1] * F_b[2];
  // J = curl B
  gB_b[2][1] += J_b[0]; gB_b[1][2] -= J_b[0];
  gB_b[0][2] += J_b[1]; gB_b[2][0] -= J_b[1];
  gB_b[1][0] += J_b[2]; gB_b[0][1] -= J_b[2];
  // divV
  for (int a = 0; a < 3; ++a) gV_b[a][a] += divV_b;

  qb[0] += rho_b;
  for (int a = 0; a < 3; ++a) qb[4 + a] += B_b[a];
  qb[7] += sig_b;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      gb[1 + a][b] += gV_b[a][b];
      gb[4 + a][b] += gB_b[a][b];
    }
  for (int b = 0; b < 3; ++b) gb[7][b] += gS_b[b];
}

// Second-derivative index of d2/dx_a dx_b in the (xx, xy, xz, yy, yz, zz) order.
const int HIDX[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

// Non-ideal stabilising terms at one particle, added to out.  Sec. 2 names
// them (a bulk viscosity split into a grid-scale and an adaptive coefficient
// field, and a diffusive div-B correction in the induction equation); App. A
// fixes the viscous term, grad(zeta div V) per unit mass, which for constant
// zeta damps compressive modes at the rate zeta k^2 / 2.  The coefficient
// formulas live in the companion paper, which is not available; readings:
//   c_f   = sqrt((gamma P + B^2) / rho)                   fast speed
//   zeta  = lambda c_f (visc_grid + visc_adapt min(1, (lambda |grad rho| / rho)^2))
//   eta   = divb_diff lambda c_f
//   dV/dt     += zeta grad(div V)
//   dB/dt     += eta  grad(div B)
//   dsigma/dt += rho zeta (div V)^2                      viscous heating
// with zeta and eta held constant over the neighborhood (App. A's constant-
// coefficient form; a grad zeta term would need a second neighbor pass).
// gdiv[0][a] = d_a div V, gdiv[1][a] = d_a div B; grad[f][b] = d q_f / d x_b.
template <class T>
void stab_point(const T* qv, const T grad[8][3], const T gdiv[2][3], double lam, const Setup& s,
                T* out) {
  const T rho = qv[0], sig = qv[7];
  const T b2 = qv[4] * qv[4] + qv[5] * qv[5] + qv[6] * qv[6];
  const T cf = sqrt((s.gamma * (s.gamma - 1.0) * sig + b2) / rho);
  const T gr2 = grad[0][0] * grad[0][0] + grad[0][1] * grad[0][1] + grad[0][2] * grad[0][2];
  const T s2 = lam * lam * gr2 / (rho * rho);
  const T sat = re(s2) < 1.0 ? s2 : T(1.0);
  const T zeta = lam * cf * (s.visc_grid + s.visc_adapt * sat);
  const T eta = s.divb_diff * lam * cf;
  const T divV = grad[1][0] + grad[2][1] + grad[3][2];
  for (int a = 0; a < 3; ++a) {
    out[1 + a] += zeta * gdiv[0][a];
    out[4 + a] += eta * gdiv[1][a];
  }
  out[7] += rho * zeta * divV * divV;
}

// Reverse mode of stab_point: accumulates into qb (8), gb[8][3] (adjoint of
// grad) and gdb[2][3] (adjoint of gdiv).  min(1, s2) passes no derivative
// where it is saturated (s2 >= 1).
void stab_point_adjoint(const double* qv, const double grad[8][3], const double gdiv[2][3],
                        double lam, const Setup& s, const double* ob, double* qb,
                        double gb[8][3], double gdb[2][3]) {
  const double g = s.gamma;
  const double rho = qv[0], sig = qv[7];
  const double B[3] = {qv[4], qv[5], qv[6]};
  const double N = g * (g - 1.0) * sig + B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  const double cf = std::sqrt(N / rho);
  const double gr2 = grad[0][0] * grad[0][0] + grad[0][1] * grad[0][1] + grad[0][2] * grad[0][2];
  const double s2 = lam * lam * gr2 / (rho * rho);
  const double sat = s2 < 1.0 ? s2 : 1.0;
  const double zeta = lam * cf * (s.visc_grid + s.visc_adapt * sat);
  const double eta = s.divb_diff * lam * cf;
  const double divV = grad[1][0] + grad[2][1] + grad[3][2];
  double zeta_b = ob[7] * rho * divV * divV, eta_b = 0.0;
  for (int a = 0; a < 3; ++a) {
    zeta_b += ob[1 + a] * gdiv[0][a];
    eta_b += ob[4 + a] * gdiv[1][a];
    gdb[0][a] += zeta * ob[1 + a];
    gdb[1][a] += eta * ob[4 + a];
  }
  qb[0] += ob[7] * zeta * divV * divV;
  const double divV_b = ob[7] * 2.0 * rho * zeta * divV;
  gb[1][0] += divV_b;
  gb[2][1] += divV_b;
  gb[3][2] += divV_b;
  const double cf_b = zeta_b * lam * (s.visc_grid + s.visc_adapt * sat) + eta_b * s.divb_diff * lam;
  if (s2 < 1.0) {
    const double s2_b = zeta_b * lam * cf * s.visc_adapt;
    for (int b = 0; b < 3; ++b) gb[0][b] += s2_b * 2.0 * lam * lam * grad[0][b] / (rho * rho);
    qb[0] += s2_b * (-2.0 * s2 / rho);
  }
  // cf = sqrt(N / rho)
  const double N_b = cf_b / (2.0 * cf * rho);
  qb[0] += -cf_b * cf / (2.0 * rho);
  qb[7] += N_b * g * (g - 1.0);
  for (int a = 0; a < 3; ++a) qb[4 + a] += N_b * 2.0 * B[a];
}

Setup make_setup(const double* L, const int32_t* periodic, double rf_ratio, double gamma,
                 int weight, int fit, const double* stab = nullptr) {
  Setup s;
  if (stab) {
    s.visc_grid = stab[0];
    s.visc_adapt = stab[1];
    s.divb_diff = stab[2];
  }
  for (int a = 0; a < 3; ++a) {
    s.L[a] = L[a];
    s.periodic[a] = periodic[a];
  }
  s.rf_ratio = rf_ratio;
  s.gamma = gamma;
  s.weight = weight;
  s.fit = fit;
  return s;
}

inline int64_t row_of(const int64_t* rows, int64_t r) { return rows ? rows[r] : r; }

// Fit all nf fields around particle i; fills physical first and second
// derivatives.  Returns the status.
template <class T>
int fit_particle(int64_t n, int64_t i, const T* pos, const double* lambda, const int32_t* nb,
                 int m, int nf, const T* fields, const Setup& s, T* d1 /* nf x 3 */,
                 T* d2 /* nf x 6 */, Local<T>* keep_loc, QR<T>* keep_qr,
                 std::vector<T>* keep_coef) {
  Local<T> loc;
  build_local(n, i, pos, lambda, nb, m, s, loc);
  std::vector<T> rhs(m * nf);
  for (int k = 0; k < m; ++k)
    for (int f = 0; f < nf; ++f) rhs[k * nf + f] = fields[f * n + nb[k]] - fields[f * n + i];
  QR<T> qr;
  std::vector<T> coef;
  wls_solve(loc, s.fit, nf, rhs, qr, coef);
  const double lam = lambda[i];
  const double nan = std::nan("");
  if (qr.status != 0) {
    for (int f = 0; f < nf; ++f) {
      for (int a = 0; a < 3; ++a) d1[f * 3 + a] = T(nan);
      if (d2)
        for (int k = 0; k < 6; ++k) d2[f * 6 + k] = T(nan);
    }
  } else {
    // f(x_i + lambda xi) - f_i ~ sum_k c_k p_k(xi):
    //   d f/d x_a = c_{a} / lambda ;  d2 f/dx_a^2 = 2 c_{aa} / lambda^2 ;
    //   d2 f/dx_a dx_b = c_{ab} / lambda^2
    for (int f = 0; f < nf; ++f) {
      for (int a = 0; a < 3; ++a) d1[f * 3 + a] = coef[(1 + a) * nf + f] / lam;
      if (d2) {
        const double fac[6] = {2.0, 1.0, 1.0, 2.0, 1.0, 2.0};
        for (int k = 0; k < 6; ++k) d2[f * 6 + k] = fac[k] * coef[(4 + k) * nf + f] / (lam * lam);
      }
    }
  }
  if (keep_loc) *keep_loc = loc;
  if (keep_qr) *keep_qr = qr;
  if (keep_coef) *keep_coef = coef;
  return qr.status;
}

template <class T>
void rhs_particle(int64_t n, int64_t i, const T* pos, const double* lambda, const int32_t* nb,
                  int m, const T* q, const Setup& s, T* rhs /* 8 */, T* dxdt /* 3 */,
                  int32_t* status) {
  T d1[8 * 3], d2[8 * 6];
  const bool stab = s.stabilised();
  int st = fit_particle<T>(n, i, pos, lambda, nb, m, 8, q, s, d1, stab ? d2 : nullptr, nullptr,
                           nullptr, nullptr);
  *status = st;
  T qv[8];
  for (int f = 0; f < 8; ++f) qv[f] = q[f * n + i];
  for (int a = 0; a < 3; ++a) dxdt[a] = qv[1 + a];
  if (st != 0) {
    for (int f = 0; f < 8; ++f) rhs[f] = T(std::nan(""));
    return;
  }
  T grad[8][3];
  for (int f = 0; f < 8; ++f)
    for (int a = 0; a < 3; ++a) grad[f][a] = d1[f * 3 + a];
  mhd_point(qv, grad, s.gamma, rhs);
  if (stab) {
    // d_a div V = sum_b d2 V_b / dx_a dx_b ;  likewise for B
    T gdiv[2][3];
    for (int g = 0; g < 2; ++g)
      for (int a = 0; a < 3; ++a) {
        T acc = T(0.0);
        for (int b = 0; b < 3; ++b) acc += d2[(1 + 3 * g + b) * 6 + HIDX[a][b]];
        gdiv[g][a] = acc;
      }
    stab_point(qv, grad, gdiv, lambda[i], s, rhs);
  }
}

// Local reverse-mode contributions of particle i.  For each neighbor slot k
// it returns dL/d(x_j) and dL/d(q_j) through particle i's own outputs, and
// the particle's own (pointwise plus "minus" side) contributions.  Neighbor
// sets are held fixed.
struct LocalAdj {
  std::vector<double> xb;  // m x 3 : contribution to x_{nb[k]}
  std::vector<double> qb;  // m x 8 : contribution to q_{nb[k]}
  double xb_self[3];
  double qb_self[8];
  int status;
};

void adjoint_particle(int64_t n, int64_t i, const double* pos, const double* lambda,
                      const int32_t* nb, int m, const double* q, const Setup& s,
                      const double* gbar /* 8 */, const double* xdbar /* 3 or null */,
                      LocalAdj& out) {
  out.xb.assign(3 * m, 0.0);
  out.qb.assign(8 * m, 0.0);
  for (int a = 0; a < 3; ++a) out.xb_self[a] = 0.0;
  for (int f = 0; f < 8; ++f) out.qb_self[f] = 0.0;
  // dx/dt = V is pointwise.
  if (xdbar)
    for (int a = 0; a < 3; ++a) out.qb_self[1 + a] += xdbar[a];

  Local<double> loc;
  QR<double> qr;
  std::vector<double> coef;  // 20 x 8
  double d1[8 * 3], d2[8 * 6];
  const bool stab = s.stabilised();
  int st = fit_particle<double>(n, i, pos, lambda, nb, m, 8, q, s, d1, stab ? d2 : nullptr, &loc,
                                &qr, &coef);
  out.status = st;
  if (st != 0) return;  // NaN outputs: no gradient flows through them

  const int F = 8;
  const double lam = lambda[i];
  const double r = s.rf_ratio * lam;
  double qv[8];
  for (int f = 0; f < F; ++f) qv[f] = q[f * n + i];
  double grad[8][3];
  for (int f = 0; f < F; ++f)
    for (int a = 0; a < 3; ++a) grad[f][a] = d1[f * 3 + a];

  // 1. pointwise adjoint
  double gb[8][3] = {{0}};
  mhd_point_adjoint(qv, grad, s.gamma, gbar, out.qb_self, gb);
  double d2b[8][6] = {{0}};
  if (stab) {
    double gdiv[2][3], gdb[2][3] = {{0}};
    for (int g = 0; g < 2; ++g)
      for (int a = 0; a < 3; ++a) {
        double acc = 0.0;
        for (int b = 0; b < 3; ++b) acc += d2[(1 + 3 * g + b) * 6 + HIDX[a][b]];
        gdiv[g][a] = acc;
      }
    stab_point_adjoint(qv, grad, gdiv, lam, s, gbar, out.qb_self, gb, gdb);
    for (int g = 0; g < 2; ++g)
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) d2b[1 + 3 * g + b][HIDX[a][b]] += gdb[g][a];
  }

  // 2. grad = E C / lambda  =>  Cbar (20 x F) has rows 1..3 = gb^T / lambda;
  //    second derivatives fac C_(ab) / lambda^2 give rows 4..9
  std::vector<double> Cbar(20 * F, 0.0);
  for (int a = 0; a < 3; ++a)
    for (int f = 0; f < F; ++f) Cbar[(1 + a) * F + f] = gb[f][a] / lam;
  if (stab) {
    const double fac[6] = {2.0, 1.0, 1.0, 2.0, 1.0, 2.0};
    for (int k = 0; k < 6; ++k)
      for (int f = 0; f < F; ++f) Cbar[(4 + k) * F + f] = fac[k] * d2b[f][k] / (lam * lam);
  }

  // 3. C = A^{-1} Bm  =>  Bbar = A^{-1} Cbar ;  Abar = -Bbar C^T
  std::vector<double> Ainv(400, 0.0);
  for (int c = 0; c < 20; ++c) {
    std::vector<double> col = ainv_column(qr, s.fit, c);
    for (int r2 = 0; r2 < 20; ++r2) Ainv[r2 * 20 + c] = col[r2];
  }
  std::vector<double> Bbar(20 * F, 0.0), Abar(400, 0.0);
  for (int a = 0; a < 20; ++a)
    for (int f = 0; f < F; ++f) {
      double acc = 0.0;
      for (int b = 0; b < 20; ++b) acc += Ainv[a * 20 + b] * Cbar[b * F + f];
      Bbar[a * F + f] = acc;
    }
  for (int a = 0; a < 20; ++a)
    for (int b = 0; b < 20; ++b) {
      double acc = 0.0;
      for (int f = 0; f < F; ++f) acc += Bbar[a * F + f] * coef[b * F + f];
      Abar[a * 20 + b] = -acc;
    }

  // 4. per neighbor: A = sum w p p^T,  Bm = sum w p df^T
  for (int k = 0; k < m; ++k) {
    const int64_t j = nb[k];
    const double x = loc.xi[3 * k], y = loc.xi[3 * k + 1], z = loc.xi[3 * k + 2];
    double p[20];
    for (int c = 0; c < 20; ++c) p[c] = monomial(c, x, y, z);
    if (s.fit == 1) p[0] = 0.0;  // the interpolating fit has no constant column
    const double w = loc.w[k];
    double df[8];
    for (int f = 0; f < F; ++f) df[f] = q[f * n + j] - q[f * n + i];
    // wbar = p^T Abar p + p^T Bbar df
    double wbar = 0.0;
    double pbar[20];
    for (int a = 0; a < 20; ++a) {
      double Ap = 0.0, ATp = 0.0, Bd = 0.0;
      for (int b = 0; b < 20; ++b) {
        Ap += Abar[a * 20 + b] * p[b];
        ATp += Abar[b * 20 + a] * p[b];
      }
      for (int f = 0; f < F; ++f) Bd += Bbar[a * F + f] * df[f];
      wbar += p[a] * Ap + p[a] * Bd;
      pbar[a] = w * (Ap + ATp) + w * Bd;
    }
    if (s.fit == 1) pbar[0] = 0.0;
    // dfbar = w Bbar^T p
    for (int f = 0; f < F; ++f) {
      double acc = 0.0;
      for (int a = 0; a < 20; ++a) acc += Bbar[a * F + f] * p[a];
      const double dfb = w * acc;
      out.qb[k * 8 + f] += dfb;
      out.qb_self[f] -= dfb;
    }
    // xi = d / lambda ; q = |d|^2 / r^2 ; w = w(q)
    double xibar[3];
    for (int ax = 0; ax < 3; ++ax) {
      double acc = 0.0;
      for (int a = 0; a < 20; ++a) acc += pbar[a] * monomial_deriv(a, ax, x, y, z);
      xibar[ax] = acc;
    }
    const double qbar_geom = wbar * weight_deriv(loc.q[k], s.weight);
    for (int ax = 0; ax < 3; ++ax) {
      const double db = xibar[ax] / lam + qbar_geom * 2.0 * loc.d[3 * k + ax] / (r * r);
      out.xb[k * 3 + ax] += db;
      out.xb_self[ax] -= db;
    }
  }
}

}  // namespace

extern "C" {

// Brute-force neighbor lists.  rows == NULL means all n rows in order.
// offsets has nrows+1 entries; idx receives up to cap entries.  Each row
// lists the qualifying j in ascending order.  Returns the total count; when
// it exceeds cap the idx contents are incomplete.  Returns -1 for invalid
// arguments.
int64_t orc_neighbors(int64_t n, const double* pos, const double* lambda, const double* L,
                      const int32_t* periodic, double rf_ratio, int64_t nrows,
                      const int64_t* rows, int64_t* offsets, int32_t* idx, int64_t cap,
                      int nthreads) {
  if (n <= 0 || !pos || !lambda || !L || !periodic || !offsets) return -1;
  Setup s = make_setup(L, periodic, rf_ratio, 0.0, 0, 0);
  if (nthreads > 0) omp_set_num_threads(nthreads);
  std::vector<int64_t> cnt(nrows, 0);
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = row_of(rows, r);
    int64_t c = 0;
    for (int64_t j = 0; j < n; ++j) c += in_sphere(pos, n, i, j, lambda, s) ? 1 : 0;
    cnt[r] = c;
  }
  offsets[0] = 0;
  for (int64_t r = 0; r < nrows; ++r) offsets[r + 1] = offsets[r] + cnt[r];
  const int64_t total = offsets[nrows];
  if (total > cap || !idx) return total;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = row_of(rows, r);
    int64_t o = offsets[r];
    for (int64_t j = 0; j < n; ++j)
      if (in_sphere(pos, n, i, j, lambda, s)) idx[o++] = (int32_t)j;
  }
  return total;
}

// MLS derivatives of nf fields for the listed rows, from the CSR restricted
// to those rows.  d1: [nf][3][nrows]; d2: [nf][6][nrows] (xx,xy,xz,yy,yz,zz)
// or NULL; status: [nrows].
int orc_mls_derivs(int64_t n, const double* pos, const double* lambda, const double* L,
                   const int32_t* periodic, double rf_ratio, int weight, int fit, int64_t nrows,
                   const int64_t* rows, const int64_t* offsets, const int32_t* idx, int nf,
                   const double* fields, double* d1, double* d2, int32_t* status, int nthreads) {
  if (n <= 0 || nf <= 0 || !pos || !lambda || !offsets || !idx || !fields || !d1 || !status)
    return -1;
  Setup s = make_setup(L, periodic, rf_ratio, 0.0, weight, fit);
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = row_of(rows, r);
    const int m = (int)(offsets[r + 1] - offsets[r]);
    std::vector<double> a1(nf * 3), a2(nf * 6);
    status[r] = fit_particle<double>(n, i, pos, lambda, idx + offsets[r], m, nf, fields, s,
                                     a1.data(), d2 ? a2.data() : nullptr, nullptr, nullptr,
                                     nullptr);
    for (int f = 0; f < nf; ++f) {
      for (int a = 0; a < 3; ++a) d1[(f * 3 + a) * nrows + r] = a1[f * 3 + a];
      if (d2)
        for (int k = 0; k < 6; ++k) d2[(f * 6 + k) * nrows + r] = a2[f * 6 + k];
    }
  }
  return 0;
}

// MHD time derivatives for the listed rows.  rhs: [8][nrows],
// dxdt: [3][nrows], status: [nrows].  stab: NULL (ideal MHD) or the three
// stabiliser coefficients (visc_grid, visc_adapt, divb_diff) of stab_point.
// Every entry point below that takes stab reads it the same way.
int orc_mhd_rhs(int64_t n, const double* pos, const double* lambda, const double* L,
                const int32_t* periodic, double rf_ratio, double gamma, int weight, int fit,
                int64_t nrows, const int64_t* rows, const int64_t* offsets, const int32_t* idx,
                const double* q, double* rhs, double* dxdt, int32_t* status, int nthreads,
                const double* stab) {
  if (n <= 0 || !pos || !lambda || !offsets || !idx || !q || !rhs || !dxdt || !status) return -1;
  Setup s = make_setup(L, periodic, rf_ratio, gamma, weight, fit, stab);
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = row_of(rows, r);
    const int m = (int)(offsets[r + 1] - offsets[r]);
    double o[8], v[3];
    int32_t st;
    rhs_particle<double>(n, i, pos, lambda, idx + offsets[r], m, q, s, o, v, &st);
    status[r] = st;
    for (int f = 0; f < 8; ++f) rhs[f * nrows + r] = o[f];
    for (int a = 0; a < 3; ++a) dxdt[a * nrows + r] = v[a];
  }
  return 0;
}

// Normalized divergence diagnostic of the magnetic field (Sec. 3.3: the
// fractional field error on the scale of lambda), for the listed rows:
//   out = lambda_i (div B)_i / |B_i|
// from the fitted gradients of Bx, By, Bz (q rows 4..6).  NaN where the fit
// failed or |B_i| = 0.  status: [nrows].
int orc_divb_norm(int64_t n, const double* pos, const double* lambda, const double* L,
                  const int32_t* periodic, double rf_ratio, int weight, int fit, int64_t nrows,
                  const int64_t* rows, const int64_t* offsets, const int32_t* idx,
                  const double* q, double* out, int32_t* status, int nthreads) {
  if (n <= 0 || !pos || !lambda || !offsets || !idx || !q || !out || !status) return -1;
  Setup s = make_setup(L, periodic, rf_ratio, 0.0, weight, fit);
  if (nthreads > 0) omp_set_num_threads(nthreads);
  const double* bfield = q + 4 * n;
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = row_of(rows, r);
    const int m = (int)(offsets[r + 1] - offsets[r]);
    double d1[3 * 3];
    const int st = fit_particle<double>(n, i, pos, lambda, idx + offsets[r], m, 3, bfield, s, d1,
                                        nullptr, nullptr, nullptr, nullptr);
    status[r] = st;
    const double bx = bfield[i], by = bfield[n + i], bz = bfield[2 * n + i];
    const double bmag = std::sqrt(bx * bx + by * by + bz * bz);
    const double div = d1[0 * 3 + 0] + d1[1 * 3 + 1] + d1[2 * 3 + 2];
    out[r] = (st == 0 && bmag > 0.0) ? lambda[i] * div / bmag : std::nan("");
  }
  return 0;
}

// Complex-step evaluation: inputs pos + i h dpos, q + i h dq (neighbor sets
// from the real positions, given in the CSR).  Returns Re(rhs) and
// Im(rhs)/h, the directional derivative along (dpos, dq), for all rows.
int orc_mhd_rhs_cstep(int64_t n, const double* pos, const double* lambda, const double* L,
                      const int32_t* periodic, double rf_ratio, double gamma, int weight,
                      int fit, const int64_t* offsets, const int32_t* idx, const double* q,
                      const double* dpos, const double* dq, double h, double* rhs_re,
                      double* rhs_dir, int32_t* status, int nthreads, const double* stab) {
  if (n <= 0 || !pos || !lambda || !offsets || !idx || !q || !rhs_re || !rhs_dir) return -1;
  Setup s = make_setup(L, periodic, rf_ratio, gamma, weight, fit, stab);
  if (nthreads > 0) omp_set_num_threads(nthreads);
  std::vector<cd> cpos(3 * n), cq(8 * n);
  for (int64_t k = 0; k < 3 * n; ++k) cpos[k] = cd(pos[k], dpos ? h * dpos[k] : 0.0);
  for (int64_t k = 0; k < 8 * n; ++k) cq[k] = cd(q[k], dq ? h * dq[k] : 0.0);
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < n; ++i) {
    const int m = (int)(offsets[i + 1] - offsets[i]);
    cd o[8], v[3];
    int32_t st;
    rhs_particle<cd>(n, i, cpos.data(), lambda, idx + offsets[i], m, cq.data(), s, o, v, &st);
    if (status) status[i] = st;
    for (int f = 0; f < 8; ++f) {
      rhs_re[f * n + i] = o[f].real();
      rhs_dir[f * n + i] = o[f].imag() / h;
    }
  }
  return 0;
}

// Reverse-mode gradient of  sum_i rhs_bar_i . rhs_i + dxdt_bar_i . dxdt_i
// with respect to q (8 x n) and pos (3 x n), neighbor sets held fixed.  The
// CSR must hold all n rows.  Particles with nonzero status contribute only
// through dxdt.
int orc_mhd_rhs_adjoint(int64_t n, const double* pos, const double* lambda, const double* L,
                        const int32_t* periodic, double rf_ratio, double gamma, int weight,
                        int fit, const int64_t* offsets, const int32_t* idx, const double* q,
                        const double* rhs_bar, const double* dxdt_bar, double* q_bar,
                        double* pos_bar, int32_t* status, int nthreads, const double* stab) {
  if (n <= 0 || !pos || !lambda || !offsets || !idx || !q || !rhs_bar || !q_bar || !pos_bar)
    return -1;
  Setup s = make_setup(L, periodic, rf_ratio, gamma, weight, fit, stab);
  if (nthreads > 0) omp_set_num_threads(nthreads);
  std::vector<LocalAdj> all(n);
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t i = 0; i < n; ++i) {
    const int m = (int)(offsets[i + 1] - offsets[i]);
    double gb[8], xb[3];
    for (int f = 0; f < 8; ++f) gb[f] = rhs_bar[f * n + i];
    if (dxdt_bar)
      for (int a = 0; a < 3; ++a) xb[a] = dxdt_bar[a * n + i];
    adjoint_particle(n, i, pos, lambda, idx + offsets[i], m, q, s, gb, dxdt_bar ? xb : nullptr,
                     all[i]);
    if (status) status[i] = all[i].status;
  }
  for (int64_t k = 0; k < 8 * n; ++k) q_bar[k] = 0.0;
  for (int64_t k = 0; k < 3 * n; ++k) pos_bar[k] = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    const int m = (int)(offsets[i + 1] - offsets[i]);
    for (int f = 0; f < 8; ++f) q_bar[f * n + i] += all[i].qb_self[f];
    for (int a = 0; a < 3; ++a) pos_bar[a * n + i] += all[i].xb_self[a];
    for (int k = 0; k < (int)all[i].xb.size() / 3 && k < m; ++k) {
      const int64_t j = idx[offsets[i] + k];
      for (int f = 0; f < 8; ++f) q_bar[f * n + j] += all[i].qb[k * 8 + f];
      for (int a = 0; a < 3; ++a) pos_bar[a * n + j] += all[i].xb[k * 3 + a];
    }
  }
  return 0;
}

// Reverse-mode contributions of the listed owner rows only (CSR restricted to
// those rows), accumulated into full q_bar (8 x n) and pos_bar (3 x n), which
// are zeroed first.  With every row listed this is orc_mhd_rhs_adjoint; with a
// sample of rows it is that sample's share of the work.
int orc_adjoint_rows(int64_t n, const double* pos, const double* lambda, const double* L,
                     const int32_t* periodic, double rf_ratio, double gamma, int weight, int fit,
                     int64_t nrows, const int64_t* rows, const int64_t* offsets,
                     const int32_t* idx, const double* q, const double* rhs_bar,
                     const double* dxdt_bar, double* q_bar, double* pos_bar, int nthreads,
                     const double* stab) {
  if (n <= 0 || nrows <= 0 || !rows || !offsets || !idx || !q || !rhs_bar || !q_bar || !pos_bar)
    return -1;
  Setup s = make_setup(L, periodic, rf_ratio, gamma, weight, fit, stab);
  if (nthreads > 0) omp_set_num_threads(nthreads);
  std::vector<LocalAdj> all(nrows);
#pragma omp parallel for schedule(dynamic, 8)
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = rows[r];
    const int m = (int)(offsets[r + 1] - offsets[r]);
    double gb[8], xb[3];
    for (int f = 0; f < 8; ++f) gb[f] = rhs_bar[f * n + i];
    if (dxdt_bar)
      for (int a = 0; a < 3; ++a) xb[a] = dxdt_bar[a * n + i];
    adjoint_particle(n, i, pos, lambda, idx + offsets[r], m, q, s, gb, dxdt_bar ? xb : nullptr,
                     all[r]);
  }
  for (int64_t k = 0; k < 8 * n; ++k) q_bar[k] = 0.0;
  for (int64_t k = 0; k < 3 * n; ++k) pos_bar[k] = 0.0;
  for (int64_t r = 0; r < nrows; ++r) {
    const int64_t i = rows[r];
    for (int f = 0; f < 8; ++f) q_bar[f * n + i] += all[r].qb_self[f];
    for (int a = 0; a < 3; ++a) pos_bar[a * n + i] += all[r].xb_self[a];
    const int m = (int)(offsets[r + 1] - offsets[r]);
    for (int k = 0; k < (int)all[r].xb.size() / 3 && k < m; ++k) {
      const int64_t j = idx[offsets[r] + k];
      for (int f = 0; f < 8; ++f) q_bar[f * n + j] += all[r].qb[k * 8 + f];
      for (int a = 0; a < 3; ++a) pos_bar[a * n + j] += all[r].xb[k * 3 + a];
    }
  }
  return 0;
}

// Gradient entries of the same scalar for a few sampled particles only, at
// any n: finds every particle whose sphere holds the sample (brute force),
// rebuilds those particles' neighbor lists (brute force), and sums their
// local reverse-mode contributions.  q_bar_s: [8][nsamp], pos_bar_s: [3][nsamp].
int orc_adjoint_sampled(int64_t n, const double* pos, const double* lambda, const double* L,
                        const int32_t* periodic, double rf_ratio, double gamma, int weight,
                        int fit, const double* q, const double* rhs_bar,
                        const double* dxdt_bar, int64_t nsamp, const int64_t* samples,
                        double* q_bar_s, double* pos_bar_s, int nthreads, const double* stab) {
  if (n <= 0 || nsamp <= 0 || !samples || !q_bar_s || !pos_bar_s) return -1;
  Setup s = make_setup(L, periodic, rf_ratio, gamma, weight, fit, stab);
  if (nthreads > 0) omp_set_num_threads(nthreads);
  for (int64_t t = 0; t < nsamp; ++t) {
    const int64_t jt = samples[t];
    double qacc[8] = {0}, xacc[3] = {0};
    // owners: every i whose sphere contains jt (jt itself included)
    std::vector<int64_t> owners;
    for (int64_t i = 0; i < n; ++i)
      if (in_sphere(pos, n, i, jt, lambda, s)) owners.push_back(i);
    std::vector<std::vector<double>> part(owners.size(), std::vector<double>(11, 0.0));
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t u = 0; u < (int64_t)owners.size(); ++u) {
      const int64_t i = owners[u];
      std::vector<int32_t> nb;
      for (int64_t j = 0; j < n; ++j)
        if (in_sphere(pos, n, i, j, lambda, s)) nb.push_back((int32_t)j);
      double gb[8], xb[3];
      for (int f = 0; f < 8; ++f) gb[f] = rhs_bar[f * n + i];
      if (dxdt_bar)
        for (int a = 0; a < 3; ++a) xb[a] = dxdt_bar[a * n + i];
      LocalAdj la;
      adjoint_particle(n, i, pos, lambda, nb.data(), (int)nb.size(), q, s, gb,
                       dxdt_bar ? xb : nullptr, la);
      for (size_t k = 0; k < nb.size(); ++k) {
        if (nb[k] != jt) continue;
        for (int f = 0; f < 8; ++f) part[u][f] += la.qb[k * 8 + f];
        for (int a = 0; a < 3; ++a) part[u][8 + a] += la.xb[k * 3 + a];
      }
      if (i == jt) {
        for (int f = 0; f < 8; ++f) part[u][f] += la.qb_self[f];
        for (int a = 0; a < 3; ++a) part[u][8 + a] += la.xb_self[a];
      }
    }
    for (size_t u = 0; u < owners.size(); ++u) {
      for (int f = 0; f < 8; ++f) qacc[f] += part[u][f];
      for (int a = 0; a < 3; ++a) xacc[a] += part[u][8 + a];
    }
    for (int f = 0; f < 8; ++f) q_bar_s[f * nsamp + t] = qacc[f];
    for (int a = 0; a < 3; ++a) pos_bar_s[a * nsamp + t] = xacc[a];
  }
  return 0;
}

// One second-order predictor-corrector step (Sec. 2), in place.
// Reading (the scheme's details are in paper I): Heun's trapezoidal form,
//   y* = y + dt F(y) ;  y_new = y + dt/2 (F(y) + F(y*)),  y = (x, q),
// with neighbor sets rebuilt at the predicted positions and positions
// wrapped back into [0, L) on periodic axes after each stage.
// status[i] is the larger of the two stages' statuses.  Returns -2 when a
// predicted position leaves [0, L) on a non-periodic axis.
// One Heun step (reading of the second-order predictor-corrector, Sec. 2)
// with an optional mask of frozen particles, whose time derivatives are taken
// as zero (fixed-value boundary particles, Sec. 3.3 and 3.5).
static int pc_step_masked(int64_t n, double* pos, double* q, const double* lambda,
                          const double* L, const int32_t* periodic, double rf_ratio, double gamma,
                          int weight, int fit, double dt, const int32_t* frozen, int32_t* status,
                          int nthreads, const double* stab);

int orc_pc_step(int64_t n, double* pos, double* q, const double* lambda, const double* L,
                const int32_t* periodic, double rf_ratio, double gamma, int weight, int fit,
                double dt, int32_t* status, int nthreads, const double* stab) {
  return pc_step_masked(n, pos, q, lambda, L, periodic, rf_ratio, gamma, weight, fit, dt,
                        nullptr, status, nthreads, stab);
}

// nsteps steps of size dt; status = the largest over all stages and steps
// (0 for frozen particles).
int orc_evolve(int64_t n, double* pos, double* q, const double* lambda, const double* L,
               const int32_t* periodic, double rf_ratio, double gamma, int weight, int fit,
               double dt, int nsteps, const int32_t* frozen, int32_t* status, int nthreads,
               const double* stab) {
  if (n <= 0 || !pos || !q || !lambda || nsteps < 0) return -1;
  std::vector<int32_t> st(n, 0), acc(n, 0);
  for (int k = 0; k < nsteps; ++k) {
    int rc = pc_step_masked(n, pos, q, lambda, L, periodic, rf_ratio, gamma, weight, fit, dt,
                            frozen, st.data(), nthreads, stab);
    if (rc) return rc;
    for (int64_t i = 0; i < n; ++i) acc[i] = std::max(acc[i], st[i]);
  }
  if (status)
    for (int64_t i = 0; i < n; ++i) status[i] = (frozen && frozen[i]) ? 0 : acc[i];
  return 0;
}

// Courant step: cfl * min over non-frozen particles of
//   lambda / (c_f (1 + 2 (visc_grid + visc_adapt + divb_diff))),
// c_f = sqrt((gamma P + B^2) / rho) with P = (gamma - 1) sigma (reading: the
// paper's own criteria are in its companion paper; Sec. 2 says the steps do
// not depend on the bulk velocity, so the signal speed is c_f alone).  The
// stabilisers' diffusivities zeta, eta <= lambda c_f (coefficients) enter as
// the speed 2 (zeta + eta) / lambda at their largest, so the step stays
// pointwise.  Returns -1 if no particle qualifies.
double orc_courant_dt(int64_t n, const double* q, const double* lambda, double gamma,
                      const int32_t* frozen, double cfl, const double* stab) {
  const double csum = stab ? stab[0] + stab[1] + stab[2] : 0.0;
  double best = -1.0;
  for (int64_t i = 0; i < n; ++i) {
    if (frozen && frozen[i]) continue;
    const double rho = q[i];
    const double b2 = q[4 * n + i] * q[4 * n + i] + q[5 * n + i] * q[5 * n + i] +
                      q[6 * n + i] * q[6 * n + i];
    const double P = (gamma - 1.0) * q[7 * n + i];
    const double cf = std::sqrt((gamma * P + b2) / rho);
    const double t = lambda[i] / (cf * (1.0 + 2.0 * csum));
    if (std::isnan(t)) continue;
    if (best < 0.0 || t < best) best = t;
  }
  return best < 0.0 ? -1.0 : cfl * best;
}

// Individual power-of-two time steps (Sec. 2 and 2.1: each particle has its
// own step, rounded down to a power of two of the largest in the binary block
// scheme; neighboring steps may differ only so much; a step may grow only
// when the times line up).  Readings, since the scheme's details are in the
// companion paper:
//  * level k_i: step dt_max / 2^k_i, k_i the smallest k in [0, kmax] whose step
//    is at most particle i's own Courant step (orc_courant_dt's expression);
//  * limiter: k_i >= k_j - 1 for every non-frozen neighbor j (neighboring
//    steps differ by a factor of two at most), enforced at i's step ends;
//  * synchronization: at its step end (a multiple of the tick dt_max / 2^kmax),
//    a particle takes at least the level whose step divides the current time;
//  * integration: Heun over each particle's own step, with every other
//    particle's state predicted linearly from its last step start,
//    y_j(t) = y_j(t0_j) + (t - t0_j) F_j(t0_j).  When a set A of particles
//    ends a step at time t: predict all to t, evaluate F at t for A (the
//    Heun predictor's derivative), correct A, then evaluate F at t for A at
//    its corrected state (the next step's starting derivative).
// With one level for all particles this is orc_evolve with dt = dt_max.
// Runs nblocks periods of dt_max.  level: the levels of the last step.
// stats[0]: step-end times, stats[1]: particle evaluations.  Returns -1 for
// bad arguments, -2 when a position leaves [0, L) on an open axis.
int orc_evolve_blocks(int64_t n, double* pos, double* q, const double* lambda, const double* L,
                      const int32_t* periodic, double rf_ratio, double gamma, int weight, int fit,
                      double dt_max, int nblocks, double cfl, int kmax, const int32_t* frozen,
                      int32_t* status, int32_t* level, int64_t* stats, int nthreads,
                      const double* stab) {
  if (n <= 0 || !pos || !q || !lambda || nblocks < 0 || kmax < 0 || kmax > 30 ||
      !(dt_max > 0.0) || !(cfl > 0.0))
    return -1;
  Setup s = make_setup(L, periodic, rf_ratio, gamma, weight, fit, stab);
  if (nthreads > 0) omp_set_num_threads(nthreads);
  const double cmul = 1.0 + 2.0 * (s.visc_grid + s.visc_adapt + s.divb_diff);
  const int64_t T = int64_t(1) << kmax;  // ticks per dt_max
  const double dtick = std::ldexp(dt_max, -kmax);
  auto is_frozen = [&](int64_t i) { return frozen && frozen[i]; };
  auto wrap = [&](double v, int a, bool& ok) {
    if (s.periodic[a]) {
      if (v >= s.L[a]) v -= s.L[a];
      if (v < 0.0) v += s.L[a];
    } else if (v < 0.0 || v >= s.L[a]) {
      ok = false;
    }
    return v;
  };
  auto courant_level = [&](const double* qq, int64_t i) {
    const double b2 = qq[4 * n + i] * qq[4 * n + i] + qq[5 * n + i] * qq[5 * n + i] +
                      qq[6 * n + i] * qq[6 * n + i];
    const double P = (s.gamma - 1.0) * qq[7 * n + i];
    const double cf = std::sqrt((s.gamma * P + b2) / qq[i]);
    const double dtc = cfl * (lambda[i] / (cf * cmul));
    int k = 0;
    while (k < kmax && !(std::ldexp(dt_max, -k) <= dtc)) ++k;
    return k;
  };
  std::vector<double> x0(pos, pos + 3 * n), q0(q, q + 8 * n), xp(x0), qp(q0);
  std::vector<double> F0(8 * n, 0.0), V0(3 * n, 0.0);
  std::vector<int64_t> t0(n, 0);
  std::vector<int32_t> k(n, 0), stmax(n, 0);
  int64_t events = 0, evals = 0;
  // time derivatives of the listed rows at the state (xp, qp)
  auto eval_rows = [&](const std::vector<int64_t>& rows, std::vector<int64_t>& off,
                       std::vector<int32_t>& nb, std::vector<double>& f,
                       std::vector<double>& v, std::vector<int32_t>& st) {
    const int64_t m = (int64_t)rows.size();
    off.assign(m + 1, 0);
    const int64_t nnz = orc_neighbors(n, xp.data(), lambda, L, periodic, rf_ratio, m, rows.data(),
                                      off.data(), nullptr, 0, nthreads);
    nb.assign(std::max<int64_t>(nnz, 1), 0);
    orc_neighbors(n, xp.data(), lambda, L, periodic, rf_ratio, m, rows.data(), off.data(),
                  nb.data(), nnz, nthreads);
    f.assign(8 * m, 0.0);
    v.assign(3 * m, 0.0);
    st.assign(m, 0);
    orc_mhd_rhs(n, xp.data(), lambda, L, periodic, rf_ratio, gamma, weight, fit, m, rows.data(),
                off.data(), nb.data(), qp.data(), f.data(), v.data(), st.data(), nthreads, stab);
    evals += m;
  };
  // levels of the rows (Courant, limiter among them against the others'
  // current levels, synchronization with the time `tick`)
  auto set_levels = [&](const std::vector<int64_t>& rows, const std::vector<int64_t>& off,
                        const std::vector<int32_t>& nb, int64_t tick) {
    const int64_t m = (int64_t)rows.size();
    std::vector<int32_t> kn(m);
    std::vector<int64_t> rpos(n, -1);
    for (int64_t r = 0; r < m; ++r) {
      kn[r] = courant_level(q0.data(), rows[r]);
      rpos[rows[r]] = r;
    }
    bool changed = true;
    while (changed) {
      changed = false;
      for (int64_t r = 0; r < m; ++r)
        for (int64_t e = off[r]; e < off[r + 1]; ++e) {
          const int64_t j = nb[e];
          if (j == rows[r] || is_frozen(j)) continue;
          const int kj = rpos[j] >= 0 ? kn[rpos[j]] : k[j];
          if (kj - 1 > kn[r]) {
            kn[r] = kj - 1;
            changed = true;
          }
        }
    }
    int ksync = 0;
    if (tick > 0) {
      int tz = 0;
      while (tz < kmax && ((tick >> tz) & 1) == 0) ++tz;
      ksync = kmax - tz;
    }
    for (int64_t r = 0; r < m; ++r) k[rows[r]] = std::max(kn[r], ksync);
  };
  std::vector<int64_t> act, off;
  std::vector<int32_t> nb, st;
  std::vector<double> f, v;
  for (int64_t i = 0; i < n; ++i)
    if (!is_frozen(i)) act.push_back(i);
  if (act.empty() || nblocks == 0) {
    if (status) for (int64_t i = 0; i < n; ++i) status[i] = 0;
    if (level) for (int64_t i = 0; i < n; ++i) level[i] = 0;
    if (stats) { stats[0] = 0; stats[1] = 0; }
    return 0;
  }
  // start: every particle's derivative and level at time 0
  eval_rows(act, off, nb, f, v, st);
  for (size_t r = 0; r < act.size(); ++r) {
    const int64_t i = act[r];
    for (int c = 0; c < 8; ++c) F0[c * n + i] = f[c * act.size() + r];
    for (int a = 0; a < 3; ++a) V0[a * n + i] = v[a * act.size() + r];
    stmax[i] = std::max(stmax[i], st[r]);
  }
  set_levels(act, off, nb, 0);
  const int64_t tick_end = (int64_t)nblocks * T;
  for (;;) {
    int64_t tick = INT64_MAX;
    for (int64_t i = 0; i < n; ++i)
      if (!is_frozen(i)) tick = std::min(tick, t0[i] + (T >> k[i]));
    act.clear();
    for (int64_t i = 0; i < n; ++i)
      if (!is_frozen(i) && t0[i] + (T >> k[i]) == tick) act.push_back(i);
    ++events;
    // predict every particle to tick
    bool ok = true;
    for (int64_t i = 0; i < n; ++i) {
      const double tau = (double)(tick - t0[i]) * dtick;
      for (int a = 0; a < 3; ++a) xp[a * n + i] = wrap(x0[a * n + i] + tau * V0[a * n + i], a, ok);
      for (int c = 0; c < 8; ++c) qp[c * n + i] = q0[c * n + i] + tau * F0[c * n + i];
    }
    if (!ok) return -2;
    eval_rows(act, off, nb, f, v, st);
    const int64_t m = (int64_t)act.size();
    for (int64_t r = 0; r < m; ++r) {
      const int64_t i = act[r];
      const double dt = (double)(T >> k[i]) * dtick;
      for (int c = 0; c < 8; ++c) {
        q0[c * n + i] = q0[c * n + i] + 0.5 * dt * (F0[c * n + i] + f[c * m + r]);
        qp[c * n + i] = q0[c * n + i];
      }
      for (int a = 0; a < 3; ++a) {
        x0[a * n + i] = wrap(x0[a * n + i] + 0.5 * dt * (V0[a * n + i] + v[a * m + r]), a, ok);
        xp[a * n + i] = x0[a * n + i];
      }
      t0[i] = tick;
      stmax[i] = std::max(stmax[i], st[r]);
    }
    if (!ok) return -2;
    if (tick >= tick_end) break;
    eval_rows(act, off, nb, f, v, st);
    for (int64_t r = 0; r < m; ++r) {
      const int64_t i = act[r];
      for (int c = 0; c < 8; ++c) F0[c * n + i] = f[c * m + r];
      for (int a = 0; a < 3; ++a) V0[a * n + i] = v[a * m + r];
      stmax[i] = std::max(stmax[i], st[r]);
    }
    set_levels(act, off, nb, tick);
  }
  std::copy(x0.begin(), x0.end(), pos);
  std::copy(q0.begin(), q0.end(), q);
  if (status)
    for (int64_t i = 0; i < n; ++i) status[i] = is_frozen(i) ? 0 : stmax[i];
  if (level)
    for (int64_t i = 0; i < n; ++i) level[i] = k[i];
  if (stats) {
    stats[0] = events;
    stats[1] = evals;
  }
  return 0;
}

static int pc_step_masked(int64_t n, double* pos, double* q, const double* lambda,
                          const double* L, const int32_t* periodic, double rf_ratio, double gamma,
                          int weight, int fit, double dt, const int32_t* frozen, int32_t* status,
                          int nthreads, const double* stab) {
  if (n <= 0 || !pos || !q || !lambda) return -1;
  Setup s = make_setup(L, periodic, rf_ratio, gamma, weight, fit, stab);
  if (nthreads > 0) omp_set_num_threads(nthreads);
  auto wrap = [&](std::vector<double>& x) -> bool {
    bool ok = true;
    for (int a = 0; a < 3; ++a)
      for (int64_t i = 0; i < n; ++i) {
        double& v = x[a * n + i];
        if (s.periodic[a]) {
          if (v >= s.L[a]) v -= s.L[a];
          if (v < 0.0) v += s.L[a];
        } else if (v < 0.0 || v >= s.L[a]) {
          ok = false;
        }
      }
    return ok;
  };
  auto eval = [&](const std::vector<double>& x, const std::vector<double>& qq,
                  std::vector<double>& fq, std::vector<double>& fx, std::vector<int32_t>& st) {
    std::vector<int64_t> off(n + 1);
    int64_t nnz = orc_neighbors(n, x.data(), lambda, L, periodic, rf_ratio, n, nullptr,
                                off.data(), nullptr, 0, nthreads);
    std::vector<int32_t> nb(nnz);
    orc_neighbors(n, x.data(), lambda, L, periodic, rf_ratio, n, nullptr, off.data(), nb.data(),
                  nnz, nthreads);
    orc_mhd_rhs(n, x.data(), lambda, L, periodic, rf_ratio, gamma, weight, fit, n, nullptr,
                off.data(), nb.data(), qq.data(), fq.data(), fx.data(), st.data(), nthreads, stab);
  };
  std::vector<double> x0(pos, pos + 3 * n), q0(q, q + 8 * n);
  std::vector<double> f0(8 * n), v0(3 * n), f1(8 * n), v1(3 * n);
  std::vector<int32_t> s0(n), s1(n);
  auto freeze = [&](std::vector<double>& fq, std::vector<double>& fx) {
    if (!frozen) return;
    for (int64_t i = 0; i < n; ++i)
      if (frozen[i]) {
        for (int f = 0; f < 8; ++f) fq[f * n + i] = 0.0;
        for (int a = 0; a < 3; ++a) fx[a * n + i] = 0.0;
      }
  };
  eval(x0, q0, f0, v0, s0);
  freeze(f0, v0);
  std::vector<double> xs(3 * n), qs(8 * n);
  for (int64_t k = 0; k < 3 * n; ++k) xs[k] = x0[k] + dt * v0[k];
  for (int64_t k = 0; k < 8 * n; ++k) qs[k] = q0[k] + dt * f0[k];
  if (!wrap(xs)) return -2;
  eval(xs, qs, f1, v1, s1);
  freeze(f1, v1);
  for (int64_t k = 0; k < 3 * n; ++k) pos[k] = x0[k] + 0.5 * dt * (v0[k] + v1[k]);
  for (int64_t k = 0; k < 8 * n; ++k) q[k] = q0[k] + 0.5 * dt * (f0[k] + f1[k]);
  std::vector<double> xn(pos, pos + 3 * n);
  bool ok = wrap(xn);
  std::copy(xn.begin(), xn.end(), pos);
  if (status)
    for (int64_t i = 0; i < n; ++i) status[i] = std::max(s0[i], s1[i]);
  return ok ? 0 : -2;
}

}  // extern "C"
