// Fixed-radius, non-mutual neighbor search (paper II, Sec. 2 and 2.1) on a
// uniform cell grid, its transpose, a Peano-Hilbert particle ordering, and the
// gather kernel used to apply an ordering.
//
// Pipeline of the search:
//   validate + min/max lambda (read back)  ->  cell keys  ->  counting sort of
//   particles into cells (positions copied in cell order, 32 B records)  ->
//   per-particle count over the candidate cells  ->  scan to CSR offsets
//   (nnz read back)  ->  fill  ->  per-row sort into ascending order.
// Candidate cells along each axis are those that can hold a point within
// r_f (plus a margin far above rounding) of the particle; the distance test
// itself is the exact FP64 expression of the contract, so the lists match a
// brute-force search bit for bit.
#include "internal.hpp"
#include "neighbors.hpp"

namespace phb {
namespace {

constexpr int NB_THREADS = 256;

// ---- validation and lambda range -----------------------------------------
__global__ void __launch_bounds__(NB_THREADS)
    k_validate(int n, const double* __restrict__ pos, const double* __restrict__ lam, Box box,
               double* __restrict__ part /* 3 per block: min, max, bad */) {
  __shared__ double smin[NB_THREADS], smax[NB_THREADS], sbad[NB_THREADS];
  double mn = 1e300, mx = -1e300, bad = 0.0;
  const int stride = gridDim.x * blockDim.x;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double l = lam[i];
    if (!(l > 0.0) || !isfinite(l)) bad = 1.0;
    mn = fmin(mn, l);
    mx = fmax(mx, l);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double x = pos[(int64_t)a * n + i];
      if (!(x >= 0.0 && x < box.L[a])) bad = 1.0;  // also rejects NaN
    }
  }
  smin[threadIdx.x] = mn;
  smax[threadIdx.x] = mx;
  sbad[threadIdx.x] = bad;
  __syncthreads();
  for (int d = NB_THREADS / 2; d > 0; d >>= 1) {
    if (threadIdx.x < d) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + d]);
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + d]);
      sbad[threadIdx.x] = fmax(sbad[threadIdx.x], sbad[threadIdx.x + d]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[3 * blockIdx.x] = smin[0];
    part[3 * blockIdx.x + 1] = smax[0];
    part[3 * blockIdx.x + 2] = sbad[0];
  }
}

__device__ __forceinline__ int cell_of(double x, double inv_h, int nc) {
  int c = (int)(x * inv_h);  // x >= 0: truncation is floor
  return c < nc - 1 ? c : nc - 1;
}

__global__ void __launch_bounds__(NB_THREADS)
    k_cell_key(int n, const double* __restrict__ pos, Grid g, int32_t* __restrict__ key,
               int32_t* __restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int cx = cell_of(pos[i], g.inv_h[0], g.nc[0]);
  const int cy = cell_of(pos[(int64_t)n + i], g.inv_h[1], g.nc[1]);
  const int cz = cell_of(pos[2 * (int64_t)n + i], g.inv_h[2], g.nc[2]);
  const int k = cx + g.nc[0] * (cy + g.nc[1] * cz);
  key[i] = k;
  atomicAdd(&count[k], 1);
}

__global__ void __launch_bounds__(NB_THREADS)
    k_cell_scatter(int n, const double* __restrict__ pos, const double* __restrict__ lam,
                   const int32_t* __restrict__ key, const int32_t* __restrict__ cell_start,
                   int32_t* __restrict__ cursor, int32_t* __restrict__ sorted_id,
                   double4* __restrict__ spos) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = key[i];
  const int slot = cell_start[k] + atomicAdd(&cursor[k], 1);
  sorted_id[slot] = i;
  spos[slot] = make_double4(pos[i], pos[(int64_t)n + i], pos[2 * (int64_t)n + i], lam[i]);
}

// Candidate cell range on one axis: cells that may hold a point within
// r (+ margin) of x.  On a periodic axis the range may run past either end
// (indices are wrapped by the caller); when it covers the whole axis it is
// clipped to one pass so no cell is visited twice.
struct Range {
  int lo, hi;
};
__device__ __forceinline__ Range axis_range(double x, double r, double margin, double inv_h,
                                            int nc, int periodic) {
  const double a = (x - r) - margin;
  const double b = (x + r) + margin;
  int lo = (int)floor(a * inv_h);
  int hi = (int)floor(b * inv_h);
  if (periodic) {
    if (hi - lo + 1 >= nc) {
      lo = 0;
      hi = nc - 1;
    }
  } else {
    lo = lo < 0 ? 0 : lo;
    hi = hi > nc - 1 ? nc - 1 : hi;
  }
  return Range{lo, hi};
}

__device__ __forceinline__ int wrap_cell(int c, int nc) {
  return c < 0 ? c + nc : (c >= nc ? c - nc : c);
}

// Visits every candidate of particle (xi, yi, zi) with squared radius r2 and
// calls f(slot_index_in_sorted_order, j) for those strictly inside.
template <class F>
__device__ __forceinline__ void for_each_neighbor(double xi, double yi, double zi, double r,
                                                  double r2, const Box& box, const Grid& g,
                                                  const int32_t* __restrict__ cell_start,
                                                  const int32_t* __restrict__ sorted_id,
                                                  const double4* __restrict__ spos, F&& f) {
  const Range ry = axis_range(yi, r, g.margin, g.inv_h[1], g.nc[1], box.periodic[1]);
  const Range rz = axis_range(zi, r, g.margin, g.inv_h[2], g.nc[2], box.periodic[2]);
  // Rows of cells (fixed y and z) are culled to the sphere: a neighbor in a
  // row is at least the row's distance (dy_min, dz_min) away in y and z, so
  // |dx|^2 < r^2 - dy_min^2 - dz_min^2.  Rows where that bound is empty are
  // skipped, the others scan only the cells under the chord.  The bound uses
  // r + margin, which covers the rounding of the cell binning and of the
  // distance test; the lists are those of the full box.
  // A periodic axis whose range was clipped to the whole axis has lost the
  // image each cell index stood for: it is not culled.
  const double hy = 1.0 / g.inv_h[1], hz = 1.0 / g.inv_h[2];
  const bool cull_y = !(box.periodic[1] && ry.lo == 0 && ry.hi == g.nc[1] - 1);
  const bool cull_z = !(box.periodic[2] && rz.lo == 0 && rz.hi == g.nc[2] - 1);
  const double rc = r + g.margin;
  const double rc2 = rc * rc;
  for (int cz = rz.lo; cz <= rz.hi; ++cz) {
    const double z0 = cz * hz;
    const double dzm = cull_z ? fmax(0.0, fmax(z0 - zi, zi - (z0 + hz))) : 0.0;
    const double remz = rc2 - dzm * dzm;
    if (!(remz > 0.0)) continue;
    const int wz = wrap_cell(cz, g.nc[2]);
    for (int cy = ry.lo; cy <= ry.hi; ++cy) {
      const double y0 = cy * hy;
      const double dym = cull_y ? fmax(0.0, fmax(y0 - yi, yi - (y0 + hy))) : 0.0;
      const double rem = remz - dym * dym;
      if (!(rem > 0.0)) continue;
      const Range rx = axis_range(xi, sqrt(rem), g.margin, g.inv_h[0], g.nc[0], box.periodic[0]);
      // x runs: at most two contiguous pieces after wrapping
      int xa0, xb0, xa1 = 0, xb1 = -1;
      if (rx.lo < 0) {
        xa0 = rx.lo + g.nc[0]; xb0 = g.nc[0] - 1; xa1 = 0; xb1 = rx.hi;
      } else if (rx.hi >= g.nc[0]) {
        xa0 = rx.lo; xb0 = g.nc[0] - 1; xa1 = 0; xb1 = rx.hi - g.nc[0];
      } else {
        xa0 = rx.lo; xb0 = rx.hi;
      }
      const int wy = wrap_cell(cy, g.nc[1]);
      const int row = g.nc[0] * (wy + g.nc[1] * wz);
      for (int piece = 0; piece < 2; ++piece) {
        const int a = piece == 0 ? xa0 : xa1;
        const int b = piece == 0 ? xb0 : xb1;
        if (b < a) continue;
        const int s0 = cell_start[row + a];
        const int s1 = cell_start[row + b + 1];
        for (int s = s0; s < s1; ++s) {
          const double4 pj = spos[s];
          const double dx = min_image(pj.x - xi, box.L[0], box.halfL[0], box.periodic[0]);
          const double dy = min_image(pj.y - yi, box.L[1], box.halfL[1], box.periodic[1]);
          const double dz = min_image(pj.z - zi, box.L[2], box.halfL[2], box.periodic[2]);
          if (dist2_nofma(dx, dy, dz) < r2) f(s, sorted_id[s]);
        }
      }
    }
  }
}

// Count (FILL = false) or emit (FILL = true) the neighbors of each particle.
// Thread t handles the particle in sorted slot t, so a wavefront covers
// neighboring cells and shares candidates through the caches.
template <bool FILL>
__global__ void __launch_bounds__(NB_THREADS)
    k_neighbors(int n, Box box, Grid g, double rf_ratio, const int32_t* __restrict__ cell_start,
                const int32_t* __restrict__ sorted_id, const double4* __restrict__ spos,
                int32_t* __restrict__ count, const int64_t* __restrict__ offsets,
                int32_t* __restrict__ out) {
  const int t = xcd_block() * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const double4 pi = spos[t];
  const int i = sorted_id[t];
  const double r2 = radius2_nofma(rf_ratio, pi.w);
  const double r = rf_ratio * pi.w;
  if (!FILL) {
    int c = 0;
    for_each_neighbor(pi.x, pi.y, pi.z, r, r2, box, g, cell_start, sorted_id, spos,
                      [&](int, int) { ++c; });
    count[i] = c;
  } else {
    int64_t o = offsets[i];
    for_each_neighbor(pi.x, pi.y, pi.z, r, r2, box, g, cell_start, sorted_id, spos,
                      [&](int, int j) { out[o++] = j; });
  }
}

// The same for a list of rows: thread r handles particle rows[r] (read from
// the unsorted SoA positions, which the sorted copy holds bit for bit) and
// writes its count or its entries at row r.
template <bool FILL>
__global__ void __launch_bounds__(NB_THREADS)
    k_neighbors_rows(int m, const int32_t* __restrict__ rows, int n,
                     const double* __restrict__ pos, const double* __restrict__ lam, Box box,
                     Grid g, double rf_ratio, const int32_t* __restrict__ cell_start,
                     const int32_t* __restrict__ sorted_id, const double4* __restrict__ spos,
                     int32_t* __restrict__ count, const int64_t* __restrict__ offsets,
                     int32_t* __restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= m) return;
  const int i = rows[r];
  const double xi = pos[i], yi = pos[(int64_t)n + i], zi = pos[2 * (int64_t)n + i];
  const double li = lam[i];
  const double r2 = radius2_nofma(rf_ratio, li);
  const double rad = rf_ratio * li;
  if (!FILL) {
    int c = 0;
    for_each_neighbor(xi, yi, zi, rad, r2, box, g, cell_start, sorted_id, spos,
                      [&](int, int) { ++c; });
    count[r] = c;
  } else {
    int64_t o = offsets[r];
    for_each_neighbor(xi, yi, zi, rad, r2, box, g, cell_start, sorted_id, spos,
                      [&](int, int j) { out[o++] = j; });
  }
}

// ---- per-row ascending sort ------------------------------------------------
// One wavefront per row; rows up to ROW_LDS entries are bitonic-sorted in
// LDS, longer rows by rank counting straight from global memory.
constexpr int ROW_LDS = 1024;

// Rows of up to SHORT_ROW entries, one wavefront each, sorted in registers:
// entry k of the row, padded to m = 2^p slots, sits on lane k % 64 in
// register k / 64, and a bitonic network exchanges partners across lanes
// with shuffles and across registers within a lane (distances 64 and 128).
// Entries are distinct, so the sort is a permutation.
constexpr int SHORT_ROW = 256;

__device__ __forceinline__ int32_t bitonic_keep(int32_t v, int32_t w, int i, int j, int k) {
  const bool lower = (i & j) == 0, up = (i & k) == 0;
  return (lower == up) ? min(v, w) : max(v, w);
}

// compare-exchange of registers a (lower index i) and b (index i + j >= 64)
__device__ __forceinline__ void bitonic_regs(int32_t& a, int32_t& b, int i, int k) {
  const bool up = (i & k) == 0;
  const int32_t lo = min(a, b), hi = max(a, b);
  a = up ? lo : hi;
  b = up ? hi : lo;
}

template <int R>
__device__ __forceinline__ void wave_bitonic(int32_t (&v)[R], int m, int lane) {
  for (int k = 2; k <= m; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= 64) {
        if constexpr (R == 2) {
          bitonic_regs(v[0], v[1], lane, k);
        } else if constexpr (R == 4) {
          if (j == 64) {
            bitonic_regs(v[0], v[1], lane, k);
            bitonic_regs(v[2], v[3], lane + 128, k);
          } else {
            bitonic_regs(v[0], v[2], lane, k);
            bitonic_regs(v[1], v[3], lane + 64, k);
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (64 * r < m) {
            const int32_t w = __shfl_xor(v[r], j, 64);
            v[r] = bitonic_keep(v[r], w, lane + 64 * r, j, k);
          }
        }
      }
    }
  }
}

template <int R>
__device__ __forceinline__ void sort_row_in_registers(const int32_t* __restrict__ in,
                                                      int32_t* __restrict__ out, int64_t b,
                                                      int len, int lane) {
  int m = 1;
  while (m < len) m <<= 1;
  int32_t v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = lane + 64 * r < len ? in[b + 64 * r + lane] : 0x7fffffff;
  wave_bitonic<R>(v, m, lane);
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (lane + 64 * r < len) out[b + 64 * r + lane] = v[r];
}

__global__ void __launch_bounds__(256)
    k_row_sort_short(int64_t nrows, const int64_t* __restrict__ off,
                     const int32_t* __restrict__ in, int32_t* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t r = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); r < nrows;
       r += waves) {
    const int64_t b = off[r];
    const int len = (int)(off[r + 1] - b);  // wavefront-uniform
    if (len <= 64) sort_row_in_registers<1>(in, out, b, len, lane);
    else if (len <= 128) sort_row_in_registers<2>(in, out, b, len, lane);
    else if (len <= SHORT_ROW) sort_row_in_registers<4>(in, out, b, len, lane);
  }
}

__global__ void __launch_bounds__(64)
    k_row_sort(int64_t nrows, const int64_t* __restrict__ off, const int32_t* __restrict__ in,
               int32_t* __restrict__ out, int min_len) {
  __shared__ int32_t buf[ROW_LDS];
  const int lane = threadIdx.x;
  for (int64_t r = blockIdx.x; r < nrows; r += gridDim.x) {
    const int64_t b = off[r];
    const int len = (int)(off[r + 1] - b);
    if (len < min_len) continue;  // sorted by k_row_sort_short
    if (len <= ROW_LDS) {
      int m = 1;
      while (m < len) m <<= 1;
      for (int k = lane; k < m; k += 64) buf[k] = k < len ? in[b + k] : 0x7fffffff;
      __syncthreads();
      for (int k = 2; k <= m; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
          for (int t = lane; t < (m >> 1); t += 64) {
            const int lo = 2 * j * (t / j) + (t % j);
            const int hi = lo + j;
            const bool up = (lo & k) == 0;
            const int32_t a = buf[lo], c = buf[hi];
            if ((a > c) == up) {
              buf[lo] = c;
              buf[hi] = a;
            }
          }
          __syncthreads();
        }
      }
      for (int k = lane; k < len; k += 64) out[b + k] = buf[k];
      __syncthreads();
    } else {
      // entries within a row are distinct, so each value's rank is its slot
      for (int k = lane; k < len; k += 64) {
        const int32_t v = in[b + k];
        int rank = 0;
        for (int u = 0; u < len; ++u) rank += in[b + u] < v ? 1 : 0;
        out[b + rank] = v;
      }
    }
  }
}

// ---- transpose -------------------------------------------------------------
__global__ void __launch_bounds__(NB_THREADS)
    k_t_count(int64_t nnz, const int32_t* __restrict__ idx, int32_t* __restrict__ tcount) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nnz) atomicAdd(&tcount[idx[s]], 1);
}

// k_t_fill and k_t_pos: TL lanes share a row, so that its entries are read
// coalesced and the rows' lengths even out over the lanes.
constexpr int TL = 16;

__global__ void __launch_bounds__(NB_THREADS)
    k_t_fill(int n, const int64_t* __restrict__ off, const int32_t* __restrict__ idx,
             const int64_t* __restrict__ toff, int32_t* __restrict__ cursor,
             int32_t* __restrict__ tmp) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / TL);
  if (i >= n) return;
  for (int64_t s = off[i] + t % TL; s < off[i + 1]; s += TL) {
    const int j = idx[s];
    const int p = atomicAdd(&cursor[j], 1);
    tmp[toff[j] + p] = i;
  }
}

__global__ void __launch_bounds__(NB_THREADS)
    k_t_pos(int n, const int64_t* __restrict__ off, const int32_t* __restrict__ idx,
            const int64_t* __restrict__ toff, const int32_t* __restrict__ tsrc,
            int32_t* __restrict__ tpos) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(t / TL);
  if (i >= n) return;
  for (int64_t s = off[i] + t % TL; s < off[i + 1]; s += TL) {
    const int j = idx[s];
    int64_t lo = toff[j], hi = toff[j + 1] - 1;
    while (lo < hi) {  // first position with tsrc >= i (i is present)
      const int64_t mid = (lo + hi) >> 1;
      if (tsrc[mid] < i)
        lo = mid + 1;
      else
        hi = mid;
    }
    tpos[s] = (int32_t)lo;
  }
}

// ---- Peano-Hilbert ordering ------------------------------------------------
// Each particle's cell on a 2^HB-per-axis grid over the box gets its index
// along the Hilbert curve of that grid.  The index is computed by Skilling's
// transpose method (J. Skilling, "Programming the Hilbert curve", AIP Conf.
// Proc. 707, 381, 2004): the cell coordinates are turned into the curve's
// "transposed" index (undo the rotations level by level, then Gray-encode),
// whose bits, interleaved, are the index.  Consecutive cells along the curve
// share a face, and the top 3k bits of the index are the index of the
// enclosing cell of the 2^k grid, so a counting sort on a prefix followed by a
// sort inside each bin orders by the whole index.
constexpr int HB = 10;                     // bits per axis of the fine grid
constexpr int HB_BIN = 7;                  // bits per axis of the counting-sort bins
constexpr int HB_SHIFT = 3 * (HB - HB_BIN);

__device__ __forceinline__ uint32_t spread3(uint32_t v) {  // 10 bits -> every third bit
  v &= 0x3ff;
  v = (v | (v << 16)) & 0x030000FF;
  v = (v | (v << 8)) & 0x0300F00F;
  v = (v | (v << 4)) & 0x030C30C3;
  v = (v | (v << 2)) & 0x09249249;
  return v;
}

__device__ __forceinline__ uint32_t hilbert_index(uint32_t x, uint32_t y, uint32_t z) {
  uint32_t X[3] = {x, y, z};
  for (uint32_t q = 1u << (HB - 1); q > 1; q >>= 1) {
    const uint32_t low = q - 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (X[a] & q) {
        X[0] ^= low;  // reflect the low bits
      } else {        // swap the low bits of axis 0 and axis a
        const uint32_t t = (X[0] ^ X[a]) & low;
        X[0] ^= t;
        X[a] ^= t;
      }
    }
  }
  X[1] ^= X[0];
  X[2] ^= X[1];
  uint32_t t = 0;
  for (uint32_t q = 1u << (HB - 1); q > 1; q >>= 1)
    if (X[2] & q) t ^= q - 1;
  X[0] ^= t;
  X[1] ^= t;
  X[2] ^= t;
  return (spread3(X[0]) << 2) | (spread3(X[1]) << 1) | spread3(X[2]);
}

// key = the full Hilbert index; the bin counted is its top 3 HB_BIN bits.
__global__ void __launch_bounds__(NB_THREADS)
    k_hilbert_key(int n, const double* __restrict__ pos, Grid g, int32_t* __restrict__ key,
                  int32_t* __restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const uint32_t cx = cell_of(pos[i], g.inv_h[0], g.nc[0]);
  const uint32_t cy = cell_of(pos[(int64_t)n + i], g.inv_h[1], g.nc[1]);
  const uint32_t cz = cell_of(pos[2 * (int64_t)n + i], g.inv_h[2], g.nc[2]);
  const int k = (int)hilbert_index(cx, cy, cz);
  key[i] = k;
  atomicAdd(&count[k >> HB_SHIFT], 1);
}

__global__ void __launch_bounds__(NB_THREADS)
    k_bin_scatter(int n, const int32_t* __restrict__ key, const int32_t* __restrict__ start,
                  int32_t* __restrict__ cursor, int32_t* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int k = key[i] >> HB_SHIFT;
  out[start[k] + atomicAdd(&cursor[k], 1)] = i;
}

// Sort the members of each bin by (key, index) (bins hold a handful of
// entries).
__global__ void __launch_bounds__(NB_THREADS)
    k_bin_sort_small(int nbins, const int32_t* __restrict__ start, const int32_t* __restrict__ key,
                     int32_t* __restrict__ v) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= nbins) return;
  const int s0 = start[b], s1 = start[b + 1];
  for (int k = s0 + 1; k < s1; ++k) {  // insertion sort
    const int32_t x = v[k];
    const int32_t kx = key[x];
    int u = k - 1;
    while (u >= s0) {
      const int32_t y = v[u];
      const int32_t ky = key[y];
      if (ky < kx || (ky == kx && y < x)) break;
      v[u + 1] = y;
      --u;
    }
    v[u + 1] = x;
  }
}

__global__ void __launch_bounds__(NB_THREADS)
    k_permute(int n, int ncomp, const int32_t* __restrict__ perm, const double* __restrict__ src,
              double* __restrict__ dst) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int i = perm[k];
  for (int c = 0; c < ncomp; ++c) dst[(int64_t)c * n + k] = src[(int64_t)c * n + i];
}

}  // namespace

hipError_t launch_validate(hipStream_t s, int n, const double* pos, const double* lam,
                           const Box& box, double* part, int nblocks) {
  hipLaunchKernelGGL(k_validate, dim3(nblocks), dim3(NB_THREADS), 0, s, n, pos, lam, box, part);
  return hipGetLastError();
}

hipError_t launch_cell_sort(hipStream_t s, int n, const double* pos, const double* lam,
                            const Grid& g, int32_t* key, int32_t* cell_count,
                            int32_t* cell_start, int32_t* scan_tmp, int32_t* sorted_id,
                            double4* spos) {
  const int64_t ncell = (int64_t)g.nc[0] * g.nc[1] * g.nc[2];
  hipError_t e = fill_i32(s, cell_count, 0, ncell);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cell_key, dim3(grid_for(n, NB_THREADS)), dim3(NB_THREADS), 0, s, n, pos, g,
                     key, cell_count);
  e = exclusive_scan_i32_to_i32(s, cell_count, ncell, cell_start, scan_tmp);
  if (e != hipSuccess) return e;
  e = fill_i32(s, cell_count, 0, ncell);  // reused as the scatter cursor
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cell_scatter, dim3(grid_for(n, NB_THREADS)), dim3(NB_THREADS), 0, s, n,
                     pos, lam, key, cell_start, cell_count, sorted_id, spos);
  return hipGetLastError();
}

hipError_t launch_neighbor_count(hipStream_t s, int n, const Box& box, const Grid& g,
                                 double rf_ratio, const int32_t* cell_start,
                                 const int32_t* sorted_id, const double4* spos, int32_t* count) {
  hipLaunchKernelGGL((k_neighbors<false>), dim3(grid_for(n, NB_THREADS)), dim3(NB_THREADS), 0, s,
                     n, box, g, rf_ratio, cell_start, sorted_id, spos, count, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_neighbor_fill(hipStream_t s, int n, const Box& box, const Grid& g,
                                double rf_ratio, const int32_t* cell_start,
                                const int32_t* sorted_id, const double4* spos,
                                const int64_t* offsets, int32_t* tmp) {
  hipLaunchKernelGGL((k_neighbors<true>), dim3(grid_for(n, NB_THREADS)), dim3(NB_THREADS), 0, s,
                     n, box, g, rf_ratio, cell_start, sorted_id, spos, nullptr, offsets, tmp);
  return hipGetLastError();
}

hipError_t launch_neighbor_count_rows(hipStream_t s, int m, const int32_t* rows, int n,
                                      const double* pos, const double* lam, const Box& box,
                                      const Grid& g, double rf_ratio, const int32_t* cell_start,
                                      const int32_t* sorted_id, const double4* spos,
                                      int32_t* count) {
  hipLaunchKernelGGL((k_neighbors_rows<false>), dim3(grid_for(m, NB_THREADS)), dim3(NB_THREADS),
                     0, s, m, rows, n, pos, lam, box, g, rf_ratio, cell_start, sorted_id, spos,
                     count, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_neighbor_fill_rows(hipStream_t s, int m, const int32_t* rows, int n,
                                     const double* pos, const double* lam, const Box& box,
                                     const Grid& g, double rf_ratio, const int32_t* cell_start,
                                     const int32_t* sorted_id, const double4* spos,
                                     const int64_t* offsets, int32_t* tmp) {
  hipLaunchKernelGGL((k_neighbors_rows<true>), dim3(grid_for(m, NB_THREADS)), dim3(NB_THREADS),
                     0, s, m, rows, n, pos, lam, box, g, rf_ratio, cell_start, sorted_id, spos,
                     nullptr, offsets, tmp);
  return hipGetLastError();
}

hipError_t launch_row_sort(hipStream_t s, int64_t nrows, const int64_t* off, const int32_t* in,
                           int32_t* out) {
  const int64_t sblocks = std::min<int64_t>(std::max<int64_t>((nrows + 3) / 4, 1), 65536);
  hipLaunchKernelGGL(k_row_sort_short, dim3((unsigned)sblocks), dim3(256), 0, s, nrows, off, in,
                     out);
  // rows longer than SHORT_ROW are rare: a small grid strides over all rows
  // and sorts only those
  const int64_t blocks = std::min<int64_t>(std::max<int64_t>(nrows, 1), 2048);
  hipLaunchKernelGGL(k_row_sort, dim3((unsigned)blocks), dim3(64), 0, s, nrows, off, in, out,
                     SHORT_ROW + 1);
  return hipGetLastError();
}

hipError_t launch_transpose(hipStream_t s, int n, int64_t nnz, const int64_t* off,
                            const int32_t* idx, int64_t* toff, int32_t* tsrc, int32_t* tpos,
                            int32_t* count, int64_t* scan_tmp, int32_t* tmp) {
  hipError_t e = fill_i32(s, count, 0, n);
  if (e != hipSuccess) return e;
  if (nnz > 0)
    hipLaunchKernelGGL(k_t_count, dim3(grid_for(nnz, NB_THREADS)), dim3(NB_THREADS), 0, s, nnz,
                       idx, count);
  e = exclusive_scan_i32_to_i64(s, count, n, toff, scan_tmp);
  if (e != hipSuccess) return e;
  e = fill_i32(s, count, 0, n);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_t_fill, dim3(grid_for((int64_t)n * TL, NB_THREADS)), dim3(NB_THREADS), 0, s,
                     n, off, idx, toff, count, tmp);
  e = launch_row_sort(s, n, toff, tmp, tsrc);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_t_pos, dim3(grid_for((int64_t)n * TL, NB_THREADS)), dim3(NB_THREADS), 0, s,
                     n, off, idx, toff, tsrc, tpos);
  return hipGetLastError();
}

hipError_t launch_hilbert_order(hipStream_t s, int n, const double* pos, const double* L,
                                int32_t* key, int32_t* bin_count, int32_t* bin_start,
                                int32_t* scan_tmp, int32_t* perm) {
  Grid g;
  for (int a = 0; a < 3; ++a) {
    g.nc[a] = 1 << HB;
    g.inv_h[a] = g.nc[a] / L[a];
  }
  g.margin = 0.0;
  const int nbins = 1 << (3 * HB_BIN);
  hipError_t e = fill_i32(s, bin_count, 0, nbins);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_hilbert_key, dim3(grid_for(n, NB_THREADS)), dim3(NB_THREADS), 0, s, n, pos,
                     g, key, bin_count);
  e = exclusive_scan_i32_to_i32(s, bin_count, nbins, bin_start, scan_tmp);
  if (e != hipSuccess) return e;
  e = fill_i32(s, bin_count, 0, nbins);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bin_scatter, dim3(grid_for(n, NB_THREADS)), dim3(NB_THREADS), 0, s, n, key,
                     bin_start, bin_count, perm);
  hipLaunchKernelGGL(k_bin_sort_small, dim3(grid_for(nbins, NB_THREADS)), dim3(NB_THREADS), 0, s,
                     nbins, bin_start, key, perm);
  return hipGetLastError();
}

hipError_t launch_permute(hipStream_t s, int n, int ncomp, const int32_t* perm, const double* src,
                          double* dst) {
  hipLaunchKernelGGL(k_permute, dim3(grid_for(n, NB_THREADS)), dim3(NB_THREADS), 0, s, n, ncomp,
                     perm, src, dst);
  return hipGetLastError();
}

}  // namespace phb
