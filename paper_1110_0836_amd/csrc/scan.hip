// Exclusive prefix sums (three passes: block totals, scan of totals, apply)
// and fill kernels.  Used for cell starts, CSR offsets and transposed offsets.
#include "internal.hpp"

namespace phb {
namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

template <class T>
__device__ T block_exclusive(T v, T* sh, T& total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < SCAN_THREADS; d <<= 1) {
    T add = (t >= d) ? sh[t - d] : T(0);
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  total = sh[SCAN_THREADS - 1];
  T incl = sh[t];
  __syncthreads();
  return incl - v;
}

template <class TI, class TO>
__global__ void __launch_bounds__(SCAN_THREADS)
    k_tile_sums(const TI* __restrict__ in, int64_t n, TO* __restrict__ sums) {
  __shared__ TO sh[SCAN_THREADS];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  TO v = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k)
    if (base + k < n) v += (TO)in[base + k];
  TO total;
  block_exclusive<TO>(v, sh, total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block scans the tile totals in place (exclusive) and stores the grand
// total after them.
template <class TO>
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_sums(TO* sums, int64_t nt) {
  __shared__ TO sh[SCAN_THREADS];
  TO carry = 0;
  for (int64_t base = 0; base < nt; base += SCAN_THREADS) {
    const int64_t k = base + threadIdx.x;
    TO v = k < nt ? sums[k] : TO(0);
    TO total;
    TO ex = block_exclusive<TO>(v, sh, total);
    if (k < nt) sums[k] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) sums[nt] = carry;
}

template <class TI, class TO>
__global__ void __launch_bounds__(SCAN_THREADS)
    k_scan_apply(const TI* __restrict__ in, int64_t n, const TO* __restrict__ sums, int64_t nt,
                 TO* __restrict__ out) {
  __shared__ TO sh[SCAN_THREADS];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * SCAN_ITEMS;
  TO vals[SCAN_ITEMS];
  TO v = 0;
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    vals[k] = (base + k < n) ? (TO)in[base + k] : TO(0);
    v += vals[k];
  }
  TO total;
  TO run = block_exclusive<TO>(v, sh, total) + sums[blockIdx.x];
#pragma unroll
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < n) out[base + k] = run;
    run += vals[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[nt];
}

template <class T>
__global__ void k_fill(T* p, T v, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = v;
}

template <class TI, class TO>
hipError_t scan_impl(hipStream_t s, const TI* in, int64_t n, TO* out, TO* tmp) {
  const int64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nt == 0) {
    hipLaunchKernelGGL((k_fill<TO>), dim3(1), dim3(1), 0, s, out, TO(0), (int64_t)1);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_tile_sums<TI, TO>), dim3((unsigned)nt), dim3(SCAN_THREADS), 0, s, in, n,
                     tmp);
  hipLaunchKernelGGL((k_scan_sums<TO>), dim3(1), dim3(SCAN_THREADS), 0, s, tmp, nt);
  hipLaunchKernelGGL((k_scan_apply<TI, TO>), dim3((unsigned)nt), dim3(SCAN_THREADS), 0, s, in, n,
                     tmp, nt, out);
  return hipGetLastError();
}

}  // namespace

int64_t scan_tmp_elems(int64_t n) { return (n + SCAN_TILE - 1) / SCAN_TILE + 1; }

hipError_t exclusive_scan_i32_to_i64(hipStream_t s, const int32_t* in, int64_t n, int64_t* out,
                                     int64_t* tmp) {
  return scan_impl<int32_t, int64_t>(s, in, n, out, tmp);
}
hipError_t exclusive_scan_i32_to_i32(hipStream_t s, const int32_t* in, int64_t n, int32_t* out,
                                     int32_t* tmp) {
  return scan_impl<int32_t, int32_t>(s, in, n, out, tmp);
}

hipError_t fill_i32(hipStream_t s, int32_t* p, int32_t v, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_fill<int32_t>), dim3(grid_for(n, 256) > 4096 ? 4096 : grid_for(n, 256)),
                     dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}
hipError_t fill_f64(hipStream_t s, double* p, double v, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_fill<double>), dim3(grid_for(n, 256) > 4096 ? 4096 : grid_for(n, 256)),
                     dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

}  // namespace phb
