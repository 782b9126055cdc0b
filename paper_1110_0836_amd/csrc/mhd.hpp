// Pointwise ideal-MHD Lagrangian time derivatives (paper II, Sec. 2; the
// evolution equations of App. A without bulk viscosity) and their reverse
// mode.  Field order q = (rho, Vx, Vy, Vz, Bx, By, Bz, sigma);
// grad[f][b] = d q_{f+1} / d x_b for the seven fields V, B, sigma.
// Readings: P = (gamma - 1) sigma; Heaviside-Lorentz units; the induction
// equation without a V (div B) term.
#pragma once

#include <hip/hip_runtime.h>

namespace phb {

__device__ __forceinline__ void mhd_point(const double (&q)[8], const double (&grad)[7][3],
                                          double gamma, double (&out)[8]) {
  const double rho = q[0], sig = q[7];
  const double B0 = q[4], B1 = q[5], B2 = q[6];
  // grad[0..2] = dV_a/dx_b, grad[3..5] = dB_a/dx_b, grad[6] = d sigma/dx_b
  const double divV = grad[0][0] + grad[1][1] + grad[2][2];
  const double J0 = grad[5][1] - grad[4][2];
  const double J1 = grad[3][2] - grad[5][0];
  const double J2 = grad[4][0] - grad[3][1];
  const double F0 = J1 * B2 - J2 * B1;
  const double F1 = J2 * B0 - J0 * B2;
  const double F2 = J0 * B1 - J1 * B0;
  const double inv_rho = 1.0 / rho;
  const double gm1 = gamma - 1.0;
  out[0] = -rho * divV;
  out[1] = (F0 - gm1 * grad[6][0]) * inv_rho;
  out[2] = (F1 - gm1 * grad[6][1]) * inv_rho;
  out[3] = (F2 - gm1 * grad[6][2]) * inv_rho;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    out[4 + a] = B0 * grad[a][0] + B1 * grad[a][1] + B2 * grad[a][2] - q[4 + a] * divV;
  out[7] = -gamma * sig * divV;
}

// Reverse mode of mhd_point.  ob: adjoint of out.  Adds to qb (8) and
// returns gb[7][3], the adjoint of grad.
__device__ __forceinline__ void mhd_point_adjoint(const double (&q)[8],
                                                  const double (&grad)[7][3], double gamma,
                                                  const double (&ob)[8], double (&qb)[8],
                                                  double (&gb)[7][3]) {
  const double rho = q[0], sig = q[7];
  const double B[3] = {q[4], q[5], q[6]};
  const double divV = grad[0][0] + grad[1][1] + grad[2][2];
  const double J[3] = {grad[5][1] - grad[4][2], grad[3][2] - grad[5][0], grad[4][0] - grad[3][1]};
  const double inv_rho = 1.0 / rho;
  const double gm1 = gamma - 1.0;
#pragma unroll
  for (int f = 0; f < 7; ++f)
#pragma unroll
    for (int b = 0; b < 3; ++b) gb[f][b] = 0.0;
  double divb = -rho * ob[0] - gamma * sig * ob[7];
  qb[0] += -divV * ob[0];
  qb[7] += -gamma * divV * ob[7];
  // momentum: out[1+a] = (F_a - gm1 gS_a) / rho
  double Fb[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Fb[a] = ob[1 + a] * inv_rho;
    gb[6][a] += -gm1 * ob[1 + a] * inv_rho;
  }
  {
    const double F0 = J[1] * B[2] - J[2] * B[1];
    const double F1 = J[2] * B[0] - J[0] * B[2];
    const double F2 = J[0] * B[1] - J[1] * B[0];
    const double num0 = F0 - gm1 * grad[6][0];
    const double num1 = F1 - gm1 * grad[6][1];
    const double num2 = F2 - gm1 * grad[6][2];
    qb[0] += -(num0 * ob[1] + num1 * ob[2] + num2 * ob[3]) * inv_rho * inv_rho;
  }
  // F = J x B
  const double Jb0 = B[1] * Fb[2] - B[2] * Fb[1];
  const double Jb1 = B[2] * Fb[0] - B[0] * Fb[2];
  const double Jb2 = B[0] * Fb[1] - B[1] * Fb[0];
  qb[4] += J[2] * Fb[1] - J[1] * Fb[2];
  qb[5] += J[0] * Fb[2] - J[2] * Fb[0];
  qb[6] += J[1] * Fb[0] - J[0] * Fb[1];
  // J = curl B
  gb[5][1] += Jb0; gb[4][2] -= Jb0;
  gb[3][2] += Jb1; gb[5][0] -= Jb1;
  gb[4][0] += Jb2; gb[3][1] -= Jb2;
  // induction: out[4+a] = sum_b B_b gV[a][b] - B_a divV
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double o = ob[4 + a];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      qb[4 + b] += grad[a][b] * o;
      gb[a][b] += B[b] * o;
    }
    qb[4 + a] += -divV * o;
    divb += -B[a] * o;
  }
  gb[0][0] += divb;
  gb[1][1] += divb;
  gb[2][2] += divb;
}

// ---------------------------------------------------------------------------
// Non-ideal stabilisers (Sec. 2: a bulk viscosity whose coefficient has a
// grid-scale and an adaptive part, and a diffusive div-B correction in the
// induction equation; App. A: the viscous acceleration grad(zeta div V), which
// damps compressive modes at zeta k^2 / 2 for constant zeta).  The
// coefficient formulas are readings (the companion paper that defines them is
// not available):
//   c_f  = sqrt((gamma (gamma - 1) sigma + |B|^2) / rho)        fast speed
//   s    = min(1, (lambda |grad rho| / rho)^2)                  change sensor
//   zeta = lambda c_f (grid + adapt s),   eta = divb lambda c_f
//   dV/dt += zeta grad div V,  dB/dt += eta grad div B,  dsigma/dt += rho zeta (div V)^2
// zeta and eta are taken constant over the neighborhood.
// ---------------------------------------------------------------------------
struct Stab {
  double grid = 0.0;   // grid-scale bulk viscosity coefficient
  double adapt = 0.0;  // adaptive bulk viscosity coefficient
  double divb = 0.0;   // div-B diffusion coefficient
  __host__ __device__ bool on() const { return grid != 0.0 || adapt != 0.0 || divb != 0.0; }
};

// Adds the stabilising terms to out.  grho = grad rho, gdv = grad div V,
// gdb = grad div B.
__device__ __forceinline__ void stab_point(const double (&q)[8], const double (&grho)[3],
                                           double divV, const double (&gdv)[3],
                                           const double (&gdb)[3], double lam, double gamma,
                                           const Stab& sb, double (&out)[8]) {
  const double rho = q[0];
  const double inv_rho = 1.0 / rho;
  const double bb = q[4] * q[4] + q[5] * q[5] + q[6] * q[6];
  const double cf = sqrt((gamma * (gamma - 1.0) * q[7] + bb) * inv_rho);
  const double lg = lam * inv_rho;
  const double sens = lg * lg * (grho[0] * grho[0] + grho[1] * grho[1] + grho[2] * grho[2]);
  const double sat = sens < 1.0 ? sens : 1.0;
  const double lcf = lam * cf;
  const double zeta = lcf * (sb.grid + sb.adapt * sat);
  const double eta = sb.divb * lcf;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    out[1 + a] += zeta * gdv[a];
    out[4 + a] += eta * gdb[a];
  }
  out[7] += rho * zeta * divV * divV;
}

// Reverse mode of stab_point: given ob (adjoint of out), adds to qb (8),
// grho_b, gdv_b, gdb_b and returns the adjoint of div V.  The saturated
// sensor (s >= 1) passes no derivative.
__device__ __forceinline__ double stab_point_adjoint(const double (&q)[8], const double (&grho)[3],
                                                     double divV, const double (&gdv)[3],
                                                     const double (&gdb)[3], double lam,
                                                     double gamma, const Stab& sb,
                                                     const double (&ob)[8], double (&qb)[8],
                                                     double (&grho_b)[3], double (&gdv_b)[3],
                                                     double (&gdb_b)[3]) {
  const double rho = q[0];
  const double inv_rho = 1.0 / rho;
  const double gg = gamma * (gamma - 1.0);
  const double bb = q[4] * q[4] + q[5] * q[5] + q[6] * q[6];
  const double cf = sqrt((gg * q[7] + bb) * inv_rho);
  const double lg = lam * inv_rho;
  const double sens = lg * lg * (grho[0] * grho[0] + grho[1] * grho[1] + grho[2] * grho[2]);
  const bool live = sens < 1.0;
  const double sat = live ? sens : 1.0;
  const double lcf = lam * cf;
  const double coef = sb.grid + sb.adapt * sat;
  const double zeta = lcf * coef;
  const double eta = sb.divb * lcf;
  double zb = ob[7] * rho * divV * divV;
  double eb = 0.0;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    zb += ob[1 + a] * gdv[a];
    eb += ob[4 + a] * gdb[a];
    gdv_b[a] += zeta * ob[1 + a];
    gdb_b[a] += eta * ob[4 + a];
  }
  qb[0] += ob[7] * zeta * divV * divV;
  // zeta = lam cf coef, eta = divb lam cf
  const double cfb = lam * (zb * coef + eb * sb.divb);
  if (live) {
    const double sb_ = zb * lcf * sb.adapt;  // adjoint of the sensor
    const double k2 = 2.0 * sb_ * lg * lg;
#pragma unroll
    for (int a = 0; a < 3; ++a) grho_b[a] += k2 * grho[a];
    qb[0] += -2.0 * sb_ * sens * inv_rho;
  }
  // cf^2 = (gg sigma + bb) / rho
  const double c2b = cfb / (2.0 * cf);
  qb[0] += -c2b * cf * cf * inv_rho;
  qb[7] += c2b * gg * inv_rho;
#pragma unroll
  for (int a = 0; a < 3; ++a) qb[4 + a] += c2b * 2.0 * q[4 + a] * inv_rho;
  return ob[7] * 2.0 * rho * zeta * divV;
}

}  // namespace phb
