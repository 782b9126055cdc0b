// Device helpers shared by the gfx950 kernels of libphurbas.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace phb {

// ---------------------------------------------------------------------------
// Polynomial basis.  The 20 monomials of degree <= 3 in xi = (x, y, z), in the
// order 1; x,y,z; xx,xy,xz,yy,yz,zz; xxx,xxy,xxz,xyy,xyz,xzz,yyy,yyz,yzz,zzz.
// The moment matrix A = sum_j w_j p(xi_j) p(xi_j)^T has entries that are
// weighted sums of the 84 distinct monomials of degree <= 6; those sums are
// the "moments".
// ---------------------------------------------------------------------------
struct Expo {
  int a, b, c;
};

__host__ __device__ constexpr Expo basis_expo(int k) {
  constexpr int E[20][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {2, 0, 0},
                            {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2},
                            {3, 0, 0}, {2, 1, 0}, {2, 0, 1}, {1, 2, 0}, {1, 1, 1},
                            {1, 0, 2}, {0, 3, 0}, {0, 2, 1}, {0, 1, 2}, {0, 0, 3}};
  return Expo{E[k][0], E[k][1], E[k][2]};
}

// Index of monomial x^a y^b z^c (a+b+c <= 6) among the 84 moments, ordered
// by a, then b, then c.
__host__ __device__ constexpr int moment_index(int a, int b, int c) {
  int idx = 0;
  for (int aa = 0; aa < a; ++aa) {
    const int m = 6 - aa;
    idx += (m + 1) * (m + 2) / 2;
  }
  for (int bb = 0; bb < b; ++bb) idx += 6 - a - bb + 1;
  return idx + c;
}

constexpr int NMOM = 84;
constexpr int NBASIS = 20;

// Leading dimension of the library's own per-particle SoA arrays (workspace
// and tape; callers' arrays keep n): n rounded up to 64, plus 104.  With a
// power-of-two row stride (n = 2^20: 8 MiB) every row of an array falls on
// the same HBM channels and the kernels that read or write many rows at once
// (the factorizations) slow down by a fifth; the skew of 832 B spreads them.
__host__ __device__ constexpr int64_t soa_ld(int64_t n) { return ((n + 63) / 64) * 64 + 104; }

__host__ __device__ constexpr int entry_moment(int r, int s) {
  return moment_index(basis_expo(r).a + basis_expo(s).a, basis_expo(r).b + basis_expo(s).b,
                      basis_expo(r).c + basis_expo(s).c);
}

// All 84 weighted monomials w x^a y^b z^c accumulated into m[].  Fully
// unrolled: every index is a compile-time constant, so m[] stays in VGPRs.
template <class T>
__device__ __forceinline__ void accumulate_moments(T (&m)[NMOM], T w, T x, T y, T z) {
  T zp[7];
  zp[0] = T(1);
#pragma unroll
  for (int c = 1; c < 7; ++c) zp[c] = zp[c - 1] * z;
  T wx = w;
#pragma unroll
  for (int a = 0; a < 7; ++a) {
    T wxy = wx;
#pragma unroll
    for (int b = 0; b + a < 7; ++b) {
#pragma unroll
      for (int c = 0; a + b + c < 7; ++c) {
        const int k = moment_index(a, b, c);
        if (c == 0)
          m[k] += wxy;
        else
          m[k] = fma(wxy, zp[c], m[k]);
      }
      wxy = wxy * y;
    }
    wx = wx * x;
  }
}

// Widens an FP32 value to FP64 through a register copy.  Without the copy
// the register allocator places every float that is widened at the end of a
// loop in the low half of an aligned pair (the widening's destination), so an
// array of FP32 accumulators occupies twice its registers.
__device__ __forceinline__ double widen(float v) {
  float c;
  asm volatile("v_mov_b32 %0, %1" : "=v"(c) : "v"(v));
  return (double)c;
}
__device__ __forceinline__ double widen(double v) { return v; }

// The 20 basis monomials at (x, y, z).
template <class T>
__device__ __forceinline__ void basis(T (&p)[NBASIS], T x, T y, T z) {
  const T xx = x * x, yy = y * y, zz = z * z;
  p[0] = T(1);
  p[1] = x;
  p[2] = y;
  p[3] = z;
  p[4] = xx;
  p[5] = x * y;
  p[6] = x * z;
  p[7] = yy;
  p[8] = y * z;
  p[9] = zz;
  p[10] = xx * x;
  p[11] = xx * y;
  p[12] = xx * z;
  p[13] = x * yy;
  p[14] = p[5] * z;
  p[15] = x * zz;
  p[16] = yy * y;
  p[17] = yy * z;
  p[18] = y * zz;
  p[19] = zz * z;
}

// ---------------------------------------------------------------------------
// Geometry
// ---------------------------------------------------------------------------
// Workgroups are dispatched to the eight XCDs round-robin (block b runs on
// XCD b % 8) and every XCD has its own L2.  Kernels that gather neighbor
// records number their blocks so that XCD x runs one contiguous range of
// logical blocks: particles stored in spatial order then share neighbors
// inside one L2 instead of spreading every neighborhood over eight.
// A bijection of [0, gridDim.x) for any grid size.
__device__ __forceinline__ int xcd_block_of(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + (x < r ? x : r) + (b >> 3);
}
__device__ __forceinline__ int xcd_block() { return xcd_block_of(blockIdx.x, gridDim.x); }

struct Box {
  double L[3];
  double halfL[3];
  int periodic[3];
};

__device__ __forceinline__ double min_image(double d, double L, double halfL, int periodic) {
  if (periodic) {
    if (d > halfL)
      d -= L;
    else if (d < -halfL)
      d += L;
  }
  return d;
}

// The neighbor predicate's squared distance, evaluated exactly as
// (dx*dx + dy*dy) + dz*dz with no fused multiply-add.
__device__ __forceinline__ double dist2_nofma(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  const double a = dx * dx;
  const double b = dy * dy;
  const double c = dz * dz;
  return (a + b) + c;
}

__device__ __forceinline__ double radius2_nofma(double rf_ratio, double lam) {
#pragma clang fp contract(off)
  const double r = rf_ratio * lam;
  return r * r;
}

// Weight reading: w = (1 - q)^3, q = d^2 / r_f^2 (kind 0) or w = 1 (kind 1).
template <class T>
__device__ __forceinline__ T weight_of(T q, int kind) {
  if (kind == 1) return T(1);
  const T u = T(1) - q;
  return u * u * u;
}
template <class T>
__device__ __forceinline__ T weight_dq(T q, int kind) {
  if (kind == 1) return T(0);
  const T u = T(1) - q;
  return T(-3) * u * u;
}

// ---------------------------------------------------------------------------
// Cross-lane exchange inside groups of 4 lanes (DPP quad permutes).
// ---------------------------------------------------------------------------
// Every pattern used here (quad permutes, row rotations and mirrors, all
// rows and banks enabled) reads a valid lane, so no "old" value is needed:
// mov_dpp with bound_ctrl set is one instruction per 32 bits, where
// update_dpp with an old value first initialises the destination.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, true));
}

// quad_perm selectors: lane l of each quad reads lane sel[l].
constexpr int QP_XOR1 = 0xB1;  // [1,0,3,2]
constexpr int QP_XOR2 = 0x4E;  // [2,3,0,1]
template <int O>
constexpr int qp_bcast() {
  return O * 0x55;
}

template <class T>
__device__ __forceinline__ T quad_xor1(T v);
template <>
__device__ __forceinline__ double quad_xor1(double v) { return dpp_f64<QP_XOR1>(v); }
template <>
__device__ __forceinline__ float quad_xor1(float v) { return dpp_f32<QP_XOR1>(v); }
template <class T>
__device__ __forceinline__ T quad_xor2(T v);
template <>
__device__ __forceinline__ double quad_xor2(double v) { return dpp_f64<QP_XOR2>(v); }
template <>
__device__ __forceinline__ float quad_xor2(float v) { return dpp_f32<QP_XOR2>(v); }

// Eight fields of particle j from the packed records fq[8 j .. 8 j + 7].
__device__ __forceinline__ void load_fields(const double* __restrict__ fq, int j, double (&v)[8]) {
  const double2* p = reinterpret_cast<const double2*>(fq + 8 * (int64_t)j);
#pragma unroll
  for (int f = 0; f < 8; f += 2) {
    const double2 t = p[f / 2];
    v[f] = t.x;
    v[f + 1] = t.y;
  }
}

// DPP row controls: lane l of each 8-lane half row reads lane 7 - l; of each
// 16-lane row, lane 15 - l.
constexpr int ROW_HALF_MIRROR = 0x141;
constexpr int ROW_MIRROR = 0x140;

// Sum over the G consecutive lanes of a group (G = 1, 2, 4, 8 or 16); every
// lane of the group receives the total.  Past the quad, a mirror step pairs
// each lane with one of the other half of its group, whose partial sum is
// already complete.
template <int G, class T>
__device__ __forceinline__ T group_sum(T v) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16, "group of 1..16 lanes");
  if constexpr (G >= 2) v += quad_xor1(v);
  if constexpr (G >= 4) v += quad_xor2(v);
  if constexpr (G >= 8) {
    if constexpr (sizeof(T) == 8) v += dpp_f64<ROW_HALF_MIRROR>(v);
    else v += dpp_f32<ROW_HALF_MIRROR>(v);
  }
  if constexpr (G >= 16) {
    if constexpr (sizeof(T) == 8) v += dpp_f64<ROW_MIRROR>(v);
    else v += dpp_f32<ROW_MIRROR>(v);
  }
  return v;
}

// Reduce-scatter over the G = 1, 2 or 4 lanes of an aligned group: every lane
// holds N partial values a[0 .. N), and lane e of the group receives
// r[m] = the group's sum of a[G m + e], m < N / G.  Each step pairs two of a
// lane's values, keeps the one its half of the group owns and sends the
// other, so a lane sends half of what it holds per step (group_sum sends all
// of it) and ends with only the sums it stores.  Every sum is formed as
// group_sum<G> forms it (the pair's sum, then the sum of the two pair sums;
// the additions commute), so the values are bit-identical to it.
// The pairs retire one at a time: each next pair is tied to the previous
// sum, so the selected and exchanged copies of all values are never live
// together (hoisted, they double the register footprint).
template <int G, int N, class T>
__device__ __forceinline__ void group_reduce_scatter(T* a, T* r, int e) {
  static_assert(G == 1 || G == 2 || G == 4, "group of 1, 2 or 4 lanes");
  static_assert(N % G == 0, "the values split evenly over the group");
  if constexpr (G == 1) {
#pragma unroll
    for (int k = 0; k < N; ++k) r[k] = a[k];
  } else {
    const bool odd = (e & 1) != 0;
    T h[N / 2];
#pragma unroll
    for (int m = 0; m < N / 2; ++m) {
      const T keep = odd ? a[2 * m + 1] : a[2 * m];
      const T send = odd ? a[2 * m] : a[2 * m + 1];
      h[m] = keep + quad_xor1(send);  // the pair's sum of a[2 m + (e & 1)]
      if (m + 1 < N / 2) asm volatile("" : "+v"(a[2 * m + 2]), "+v"(a[2 * m + 3]) : "v"(h[m]));
    }
    if constexpr (G == 2) {
#pragma unroll
      for (int m = 0; m < N / 2; ++m) r[m] = h[m];
    } else {
      const bool up = (e & 2) != 0;
#pragma unroll
      for (int m = 0; m < N / 4; ++m) {
        const T keep = up ? h[2 * m + 1] : h[2 * m];
        const T send = up ? h[2 * m] : h[2 * m + 1];
        r[m] = keep + quad_xor2(send);  // the quad's sum of a[4 m + e]
        if (m + 1 < N / 4) asm volatile("" : "+v"(h[2 * m + 2]), "+v"(h[2 * m + 3]) : "v"(r[m]));
      }
    }
  }
}

// Group sums of three 20-coefficient rows a[t][b] (flat, t-major), stored to
// rows r0 + t of an SoA array buf[row][20][ld], column i.  Lane e of the
// group stores the coefficients b = e, e + G, ... of each row.
template <int G>
__device__ __forceinline__ void store_rows3(double* a, int e, bool valid, double* buf,
                                            int r0, int64_t ld, int i) {
  constexpr int PER = NBASIS / G;
  static_assert(NBASIS % G == 0, "coefficients split evenly over the group");
  double r[3 * PER];
  group_reduce_scatter<G, 3 * NBASIS>(a, r, e);
  if (valid) {
    double* dst = buf + ((int64_t)r0 * NBASIS + e) * ld + i;
#pragma unroll
    for (int m = 0; m < 3 * PER; ++m) dst[(int64_t)((m / PER) * NBASIS + G * (m % PER)) * ld] = r[m];
  }
}

// Makes a wavefront's LDS writes visible to its own later LDS reads from any
// of its lanes (the lanes run in lockstep: the writes only have to complete
// and stay ordered before the reads).  Wavefronts of the same block are not
// waited for.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Lane-half exchanges of gfx950 on a double, one 32-bit half at a time.
// swap32: lanes 32..63 of a trade places with lanes 0..31 of b.  swap16: in
// each half of the wavefront, lanes 16..31 of a trade places with lanes 0..15
// of b.
__device__ __forceinline__ void swap32(double& a, double& b) {
  const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane32_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi =
      __builtin_amdgcn_permlane32_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}
__device__ __forceinline__ void swap16(double& a, double& b) {
  const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
  const auto lo = __builtin_amdgcn_permlane16_swap((unsigned)ua, (unsigned)ub, false, false);
  const auto hi =
      __builtin_amdgcn_permlane16_swap((unsigned)(ua >> 32), (unsigned)(ub >> 32), false, false);
  a = __longlong_as_double((long long)(((unsigned long long)hi[0] << 32) | lo[0]));
  b = __longlong_as_double((long long)(((unsigned long long)hi[1] << 32) | lo[1]));
}

// Sums over the 64 lanes of a wavefront of N = 10 or 12 values per lane,
// transposed on the way so that the additions are shared: a lane-half swap
// pairs values 2k and 2k + 1 (one half of the wavefront then holds partial
// sums of each), a row swap pairs two such registers (each 16-lane row then
// holds one value's partial sums), and three 16-lane row sums finish.  About
// a third of the instructions of N separate wavefront sums.  On return lane
// l holds the total of value comp (comp < 0: none); every value is on
// exactly one lane.
template <int N>
__device__ __forceinline__ void wave_sum_transposed(const double (&v)[N], double& out, int& comp) {
  static_assert(N == 10 || N == 12, "ten or twelve values");
  constexpr int NC = N / 2;
  double c[NC];
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    double x = v[2 * k], y = v[2 * k + 1];
    swap32(x, y);
    c[k] = x + y;  // half 0: value 2k, half 1: value 2k + 1
  }
  double e[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double x = c[2 * k < NC ? 2 * k : NC - 1];
    double y = 2 * k + 1 < NC ? c[2 * k + 1] : x;  // N = 10: c[4] pairs with itself
    swap16(x, y);
    e[k] = x + y;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    double t = e[k];
    t += quad_xor1(t);
    t += quad_xor2(t);
    t += dpp_f64<0x124>(t);  // row_ror:4
    t += dpp_f64<0x128>(t);  // row_ror:8
    e[k] = t;
  }
  const int lane = __lane_id();
  const int q = lane >> 4, p = lane & 15;
  // rows of e[k] for a pair: values 4k, 4k + 2, 4k + 1, 4k + 3
  const int perm = (q == 0) ? 0 : (q == 1) ? 2 : (q == 2) ? 1 : 3;
  out = p == 0 ? e[0] : (p == 1 ? e[1] : e[2]);
  comp = -1;
  if (p < 2 || (p == 2 && N == 12)) comp = 4 * p + perm;
  else if (p == 2 && (q & 1) == 0) comp = 8 + (q >> 1);
}

template <int O>
__device__ __forceinline__ double quad_bcast(double v) {
  return dpp_f64<qp_bcast<O>()>(v);
}

__device__ __forceinline__ double quad_min(double v) {
  v = fmin(v, dpp_f64<QP_XOR1>(v));
  return fmin(v, dpp_f64<QP_XOR2>(v));
}
__device__ __forceinline__ double quad_max(double v) {
  v = fmax(v, dpp_f64<QP_XOR1>(v));
  return fmax(v, dpp_f64<QP_XOR2>(v));
}

}  // namespace phb
