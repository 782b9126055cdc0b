// Fixed-radius, non-mutual neighbor search (paper II, Sec. 2 and 2.1) on a
// uniform cell grid, its transpose, a Peano-Hilbert particle ordering, and the
// gather kernel used to apply an ordering.
//
// Pipeline of the search, all on the device (no host synchronization):
//   validate + lambda range  ->  grid sized from the smallest r_f (one
//   thread)  ->  cell keys  ->  counting sort of particles into cells
//   (positions copied in cell order, 32 B records)  ->  per-row count over
//   the candidate cells  ->  scan to CSR offsets  ->  capacity check  ->
//   fill, each row sorted ascending in registers and written once.
// A status word carries invalid input and overflow from kernel to kernel;
// every kernel after the check it concerns leaves at once when it is set.
// Candidate cells along each axis are those that can hold a point within
// r_f (plus a margin far above rounding) of the particle; the distance test
// itself is the exact FP64 expression of the contract, so the lists match a
// brute-force search bit for bit.
#include <algorithm>

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
    k_cell_key(int n, const double* __restrict__ pos, const Grid* __restrict__ gp,
               const int32_t* __restrict__ flag, int32_t* __restrict__ key,
               int32_t* __restrict__ count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || *flag) return;
  const Grid g = *gp;
  const int cx = cell_of(pos[i], g.inv_h[0], g.nc[0]);
  const int cy = cell_of(pos[(int64_t)n + i], g.inv_h[1], g.nc[1]);
  const int cz = cell_of(pos[2 * (int64_t)n + i], g.inv_h[2], g.nc[2]);
  const int k = cx + g.nc[0] * (cy + g.nc[1] * cz);
  key[i] = k;
  atomicAdd(&count[k], 1);
}

__global__ void __launch_bounds__(NB_THREADS)
    k_cell_scatter(int n, const double* __restrict__ pos, const double* __restrict__ lam,
                   const int32_t* __restrict__ flag, const int32_t* __restrict__ key,
                   const int32_t* __restrict__ cell_start, int32_t* __restrict__ cursor,
                   int32_t* __restrict__ sorted_id, double4* __restrict__ spos) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || *flag) return;
  const int k = key[i];
  const int slot = cell_start[k] + atomicAdd(&cursor[k], 1);
  sorted_id[slot] = i;
  spos[slot] = make_double4(pos[i], pos[(int64_t)n + i], pos[2 * (int64_t)n + i], lam[i]);
}

// The lambda range and validity of the inputs (from k_validate's per-block
// partials), then the cell grid, by one wavefront: cells of side
// r_f,min / cells_per_rf, coarsened by 1.26 per axis until at most
// max_cells.  Status: PHB_NB_INVALID for a position outside [0, L) or not
// finite or a lambda that is not positive, PHB_NB_RADIUS for r_f,max >= L/2
// on a periodic axis.
__global__ void __launch_bounds__(64)
    k_nb_setup(const double* __restrict__ part, int nblocks, Box box, double rf_ratio,
               int cells_per_rf, int64_t max_cells, int max_per_axis, Grid* __restrict__ gout,
               int32_t* __restrict__ flag, double* __restrict__ lrange) {
  const int lane = threadIdx.x;
  double mn = 1e300, mx = -1e300, bad = 0.0;
  for (int b = lane; b < nblocks; b += 64) {
    mn = fmin(mn, part[3 * b]);
    mx = fmax(mx, part[3 * b + 1]);
    bad = fmax(bad, part[3 * b + 2]);
  }
  for (int d = 32; d > 0; d >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, d, 64));
    mx = fmax(mx, __shfl_xor(mx, d, 64));
    bad = fmax(bad, __shfl_xor(bad, d, 64));
  }
  if (lane != 0) return;
  lrange[0] = mn;
  lrange[1] = mx;
  int st = bad != 0.0 ? PHB_NB_INVALID : 0;
  for (int a = 0; a < 3; ++a)
    if (box.periodic[a] && !(rf_ratio * mx < box.halfL[a])) st |= PHB_NB_RADIUS;
  *flag = st;
  if (st) return;
  Grid g;
  double h = rf_ratio * mn / (cells_per_rf > 1 ? cells_per_rf : 1);
  for (;;) {
    int64_t total = 1;
    for (int a = 0; a < 3; ++a) {
      double c = floor(box.L[a] / h);
      if (c < 1) c = 1;
      if (c > max_per_axis) c = max_per_axis;
      g.nc[a] = (int)c;
      total *= g.nc[a];
    }
    if (total <= max_cells) break;
    h *= 1.26;
  }
  double hmin = 1e300;
  for (int a = 0; a < 3; ++a) {
    g.inv_h[a] = g.nc[a] / box.L[a];
    hmin = fmin(hmin, box.L[a] / g.nc[a]);
  }
  g.margin = 1e-6 * hmin;
  *gout = g;
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

// ---- per-row ascending sort ------------------------------------------------
// One wavefront per row; rows up to ROW_LDS entries are bitonic-sorted in
// LDS, longer rows by rank counting straight from global memory.
constexpr int ROW_LDS = 1024;

// In-register sort of a row of up to 256 entries, one wavefront: entry k of
// the row, padded to m = 2^p slots, sits on lane k % 64 in register k / 64,
// and a bitonic network exchanges partners across lanes with shuffles and
// across registers within a lane (distances 64 and 128).  Entries are
// distinct, so the sort is a permutation.

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

// The rows list[0 .. *count) (one block of one wavefront per row, the grid
// striding over the list).
__global__ void __launch_bounds__(64)
    k_row_sort(const int32_t* __restrict__ list, const int32_t* __restrict__ count,
               const int64_t* __restrict__ off, const int32_t* __restrict__ in,
               int32_t* __restrict__ out, const int32_t* __restrict__ flag) {
  __shared__ int32_t buf[ROW_LDS];
  const int lane = threadIdx.x;
  if (*flag) return;
  const int nl = *count;
  for (int q = blockIdx.x; q < nl; q += gridDim.x) {
    const int r = list[q];
    const int64_t b = off[r];
    const int len = (int)(off[r + 1] - b);
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

// ---- the search: one wavefront per row ----------------------------------
// Row k of cells (fixed y and z) in the candidate block of a particle, as at
// most two contiguous runs of cell-sorted slots [s0a, s0a + lena),
// [s0b, s0b + lenb) (an x range that wraps is two pieces).  Rows of cells
// are culled to the sphere: a neighbor in a row is at least the row's
// distance (dy_min, dz_min) away in y and z, so |dx|^2 < r^2 - dy_min^2 -
// dz_min^2; rows where that bound is empty hold no candidates, the others
// only the cells under the chord.  The bound uses r + margin, which covers
// the rounding of the cell binning and of the distance test: the lists are
// those of the full box.  A periodic axis whose range was clipped to the
// whole axis has lost the image each cell index stood for: it is not culled.
struct CellRows {
  Range ry, rz;
  int ny, nrows;
  bool cull_y, cull_z;
};

__device__ __forceinline__ CellRows cell_rows(double yi, double zi, double r, const Box& box,
                                              const Grid& g) {
  CellRows c;
  c.ry = axis_range(yi, r, g.margin, g.inv_h[1], g.nc[1], box.periodic[1]);
  c.rz = axis_range(zi, r, g.margin, g.inv_h[2], g.nc[2], box.periodic[2]);
  c.ny = c.ry.hi - c.ry.lo + 1;
  c.nrows = c.ny * (c.rz.hi - c.rz.lo + 1);
  c.cull_y = !(box.periodic[1] && c.ry.lo == 0 && c.ry.hi == g.nc[1] - 1);
  c.cull_z = !(box.periodic[2] && c.rz.lo == 0 && c.rz.hi == g.nc[2] - 1);
  return c;
}

__device__ __forceinline__ void cell_row_runs(int k, const CellRows& c, double xi, double yi,
                                              double zi, double r, const Box& box,
                                              const Grid& g,
                                              const int32_t* __restrict__ cell_start, int& s0a,
                                              int& lena, int& s0b, int& lenb) {
  s0a = lena = s0b = lenb = 0;
  const int cz = c.rz.lo + k / c.ny, cy = c.ry.lo + k % c.ny;
  const double hy = 1.0 / g.inv_h[1], hz = 1.0 / g.inv_h[2];
  const double rc = r + g.margin;
  const double z0 = cz * hz, y0 = cy * hy;
  const double dzm = c.cull_z ? fmax(0.0, fmax(z0 - zi, zi - (z0 + hz))) : 0.0;
  const double dym = c.cull_y ? fmax(0.0, fmax(y0 - yi, yi - (y0 + hy))) : 0.0;
  const double rem = (rc * rc - dzm * dzm) - dym * dym;
  if (!(rc * rc - dzm * dzm > 0.0) || !(rem > 0.0)) return;
  const Range rx = axis_range(xi, sqrt(rem), g.margin, g.inv_h[0], g.nc[0], box.periodic[0]);
  int xa0, xb0, xa1 = 0, xb1 = -1;
  if (rx.lo < 0) {
    xa0 = rx.lo + g.nc[0]; xb0 = g.nc[0] - 1; xa1 = 0; xb1 = rx.hi;
  } else if (rx.hi >= g.nc[0]) {
    xa0 = rx.lo; xb0 = g.nc[0] - 1; xa1 = 0; xb1 = rx.hi - g.nc[0];
  } else {
    xa0 = rx.lo; xb0 = rx.hi;
  }
  const int row = g.nc[0] * (wrap_cell(cy, g.nc[1]) + g.nc[1] * wrap_cell(cz, g.nc[2]));
  s0a = cell_start[row + xa0];
  lena = cell_start[row + xb0 + 1] - s0a;
  if (xb1 >= xa1) {
    s0b = cell_start[row + xa1];
    lenb = cell_start[row + xb1 + 1] - s0b;
  }
}

// Inclusive maximum over lanes 0..lane.
__device__ __forceinline__ int wave_inclusive_max(int v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(v, d, 64);
    if (lane >= d) v = max(v, t);
  }
  return v;
}

__device__ __forceinline__ int wave_inclusive_scan(int v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// Rows of up to NB_ROW entries are collected in LDS and sorted in registers.
constexpr int NB_WAVES = NB_THREADS / 64;
constexpr int NB_ROW = 256;
constexpr int NB_LONG_BLOCKS = 64;  // grid of the passes over the long rows

template <int R>
__device__ __forceinline__ void sort_lds_row(const int32_t* buf, int32_t* __restrict__ out,
                                             int64_t o, int len, int lane) {
  int mm = 1;
  while (mm < len) mm <<= 1;
  int32_t v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = lane + 64 * r < len ? buf[lane + 64 * r] : 0x7fffffff;
  wave_bitonic<R>(v, mm, lane);
#pragma unroll
  for (int r = 0; r < R; ++r)
    if (lane + 64 * r < len) out[o + 64 * r + lane] = v[r];
}

// Row r's neighbors: the particle in cell-sorted slot r (rows == null; the
// row is its particle index) or particle rows[r] (read from the SoA inputs,
// which the sorted copy holds bit for bit).  The lanes take the candidate
// block's rows of cells 64 at a time; their runs, prefix-summed over the
// wavefront, flatten the candidates into one index range that the lanes
// then test, NB_U candidates per lane at a time (one: with more, rows of
// fewer candidates leave more of each pass's lanes idle), a ballot
// compacting the hits.  Consecutive rows are spatial
// neighbors (cell order): the XCD-aware block order keeps them in one L2.
//   LONG = false: count the row; a row of up to NB_ROW entries is collected
//   in LDS, sorted in registers and written once, coalesced, to its slot of
//   the padded scratch (NB_ROW entries per row), to be copied to its CSR
//   place after the scan.
//   LONG = true: the rows longer than NB_ROW, listed by the first pass
//   (long_slot: their r, long_row: their output row), again, written unsorted
//   at their CSR place in long_tmp (for k_row_sort); the wavefronts stride
//   over the list.
constexpr int NB_U = 1;

template <bool LONG>
__global__ void __launch_bounds__(NB_THREADS)
    k_nb_wave(int m, const int32_t* __restrict__ rows, int n, const double* __restrict__ pos,
              const double* __restrict__ lam, Box box, const Grid* __restrict__ gp,
              double rf_ratio, const int32_t* __restrict__ cell_start,
              const int32_t* __restrict__ sorted_id, const double4* __restrict__ spos,
              const int32_t* __restrict__ flag, int32_t* __restrict__ count,
              int32_t* __restrict__ scratch, const int64_t* __restrict__ offsets,
              int32_t* __restrict__ long_tmp, int32_t* __restrict__ long_slot,
              int32_t* __restrict__ long_row, int32_t* __restrict__ long_count) {
  __shared__ int sh_start[NB_WAVES][64], sh_s0a[NB_WAVES][64], sh_lena[NB_WAVES][64],
      sh_s0b[NB_WAVES][64], sh_mark[NB_WAVES][NB_U][64];
  __shared__ int32_t sh_row[LONG ? 1 : NB_WAVES][LONG ? 1 : NB_ROW];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int w0 = __builtin_amdgcn_readfirstlane(xcd_block() * NB_WAVES + wv);
  const int fl = *flag;
  const int nrows_here = LONG ? (fl ? 0 : *long_count) : m;
  for (int w = w0; w < nrows_here; w += LONG ? (int)gridDim.x * NB_WAVES : nrows_here) {
  const int r = LONG ? long_slot[w] : w;
  if (!LONG && fl) {
    if (lane == 0) count[r] = 0;
    return;
  }
  int i;
  if (rows) i = rows[r];
  else i = sorted_id[r];
  const int orow = rows ? r : i;
  int64_t o = 0;
  int len = 0;
  if constexpr (LONG) {
    o = offsets[orow];
    len = (int)(offsets[orow + 1] - o);
  }
  const Grid g = *gp;
  double xi, yi, zi, li;
  if (rows) {
    xi = pos[i];
    yi = pos[(int64_t)n + i];
    zi = pos[2 * (int64_t)n + i];
    li = lam[i];
  } else {
    const double4 pi = spos[r];
    xi = pi.x;
    yi = pi.y;
    zi = pi.z;
    li = pi.w;
  }
  const double r2 = radius2_nofma(rf_ratio, li);
  const double rad = rf_ratio * li;
  const CellRows cr = cell_rows(yi, zi, rad, box, g);
  int c = 0;  // hits so far (wavefront-uniform)
  for (int base = 0; base < cr.nrows; base += 64) {
    int s0a = 0, lena = 0, s0b = 0, lenb = 0;
    if (base + lane < cr.nrows)
      cell_row_runs(base + lane, cr, xi, yi, zi, rad, box, g, cell_start, s0a, lena, s0b, lenb);
    const int tot = lena + lenb;
    const int incl = wave_inclusive_scan(tot, lane);
    const int ncand = __shfl(incl, 63, 64);
    sh_start[wv][lane] = incl - tot;
    sh_s0a[wv][lane] = s0a;
    sh_lena[wv][lane] = lena;
    sh_s0b[wv][lane] = s0b;
    wave_lds_sync();
    const int my_start = incl - tot;  // this lane's run of cells
    for (int q0 = 0; q0 < ncand; q0 += 64 * NB_U) {
      int sl[NB_U];
      bool hit[NB_U];
      // The run of candidate q is the last non-empty run starting at or
      // before q.  For the 64 candidates Q .. Q + 63 of a window: each
      // non-empty run starting inside it marks its start with its index, a
      // maximum scan carries the marks forward, and the runs starting before
      // Q give the window's first run (non-empty runs start apart).
      int run[NB_U];
#pragma unroll
      for (int u = 0; u < NB_U; ++u) sh_mark[wv][u][lane] = -1;
      wave_lds_sync();
#pragma unroll
      for (int u = 0; u < NB_U; ++u) {
        const int Q = q0 + 64 * u;
        if (tot > 0 && my_start >= Q && my_start < Q + 64) sh_mark[wv][u][my_start - Q] = lane;
      }
      wave_lds_sync();
#pragma unroll
      for (int u = 0; u < NB_U; ++u) {
        const int Q = q0 + 64 * u;
        const uint64_t before = __ballot(tot > 0 && my_start < Q);
        const int carry = before ? 63 - (int)__clzll(before) : -1;
        run[u] = max(carry, wave_inclusive_max(sh_mark[wv][u][lane], lane));
      }
#pragma unroll
      for (int u = 0; u < NB_U; ++u) {
        const int q = q0 + 64 * u + lane;
        sl[u] = -1;
        if (q < ncand) {
          const int k = run[u];
          const int d = q - sh_start[wv][k];
          const int la = sh_lena[wv][k];
          sl[u] = d < la ? sh_s0a[wv][k] + d : sh_s0b[wv][k] + (d - la);
        }
      }
      double4 pj[NB_U];
#pragma unroll
      for (int u = 0; u < NB_U; ++u)
        pj[u] = sl[u] >= 0 ? spos[sl[u]] : make_double4(0.0, 0.0, 0.0, 0.0);
#pragma unroll
      for (int u = 0; u < NB_U; ++u) {
        const double dx = min_image(pj[u].x - xi, box.L[0], box.halfL[0], box.periodic[0]);
        const double dy = min_image(pj[u].y - yi, box.L[1], box.halfL[1], box.periodic[1]);
        const double dz = min_image(pj[u].z - zi, box.L[2], box.halfL[2], box.periodic[2]);
        hit[u] = sl[u] >= 0 && dist2_nofma(dx, dy, dz) < r2;
      }
#pragma unroll
      for (int u = 0; u < NB_U; ++u) {
        const int j = hit[u] ? sorted_id[sl[u]] : 0;
        const uint64_t mask = __ballot(hit[u]);
        const int at = c + __popcll(mask & ((1ull << lane) - 1ull));
        if (hit[u]) {
          if constexpr (LONG) {
            if (at < len) long_tmp[o + at] = j;  // the count saw the same hits
          } else if (at < NB_ROW) {
            sh_row[wv][at] = j;
          }
        }
        c += __popcll(mask);
      }
    }
    wave_lds_sync();  // the run table is rewritten for the next rows of cells
  }
  if constexpr (!LONG) {
    if (lane == 0) {
      count[orow] = c;
      if (c > NB_ROW) {
        const int q = atomicAdd(long_count, 1);
        long_slot[q] = r;
        long_row[q] = orow;
      }
    }
    if (c <= NB_ROW) {
      int32_t* dst = scratch + (int64_t)orow * NB_ROW;
      if (c <= 64) sort_lds_row<1>(sh_row[wv], dst, 0, c, lane);
      else if (c <= 128) sort_lds_row<2>(sh_row[wv], dst, 0, c, lane);
      else sort_lds_row<4>(sh_row[wv], dst, 0, c, lane);
    }
  }
  }
}

// The sorted rows of up to NB_ROW entries from the padded scratch to their
// CSR places; 16 lanes per row.
__global__ void __launch_bounds__(NB_THREADS)
    k_nb_copy(int m, const int64_t* __restrict__ offsets, const int32_t* __restrict__ scratch,
              const int32_t* __restrict__ flag, int32_t* __restrict__ idx) {
  const int64_t t = (int64_t)blockIdx.x * NB_THREADS + threadIdx.x;
  const int r = (int)(t / 16);
  if (r >= m || *flag) return;
  const int64_t o = offsets[r];
  const int len = (int)(offsets[r + 1] - o);
  if (len > NB_ROW) return;
  const int32_t* src = scratch + (int64_t)r * NB_ROW;
  for (int k = (int)(t % 16); k < len; k += 16) idx[o + k] = src[k];
}

// nnz = offsets[m] to the caller's word and the capacity check.
__global__ void k_nb_total(const int64_t* __restrict__ offsets, int m, int64_t capacity,
                           int64_t* __restrict__ nnz, int32_t* __restrict__ flag) {
  const int64_t t = offsets[m];
  *nnz = t;
  if (t > capacity) *flag |= PHB_NB_OVERFLOW;
}

// ---- transpose -------------------------------------------------------------
// The transposed row of x is T(x) = {i : x in N(i)} = A(x) + B(x):
//   A(x) = {y in N(x) : x in N(y)}, the mutual entries of row x, a sorted
//          subsequence of it;
//   B(x) = {i not in N(x) : x in N(i)}, from the one-way entries (i, x).
// With equal radii every entry is mutual; with graded lambdas the one-way
// entries are a thin shell near each sphere's edge.  Pass 1 finds, for each
// entry s = (x, y), x's place in row y (rows are sorted: a binary search):
// rev[s] = the mirrored entry (y, x), or, for a one-way entry (x joins
// B(y)), -(k + 1) with k its slot in B(y), taken from an atomic count on y.
// Pass 2 puts the one-way entries at their slots in B's part of their
// transposed rows (after A's).  Pass 3 places each transposed row's
// elements in order with the forward entry each stands for and writes t_src
// and t_pos.  Only the one-way entries use atomics, once each (the order of
// the slots they hand out is undone in pass 3).


// Pass 1, RW consecutive rows x per wavefront, a lane per entry of each: the
// rows' loads are issued together, so each lane keeps RW searches in flight
// (the passes are bound by the latency of dependent loads, not by bytes).
// The search for x in row y is a lower bound; the step that sets the upper
// end to the answer reads that entry, so a match is seen when it is read,
// and ends the search there.
constexpr int TR_RW = 4;

__global__ void __launch_bounds__(NB_THREADS)
    k_tr_mutual(int n, const int64_t* __restrict__ off, const int32_t* __restrict__ idx,
                int32_t* __restrict__ rev, int32_t* __restrict__ acnt,
                int32_t* __restrict__ bcnt) {
  const int lane = threadIdx.x & 63;
  const int x0 =
      __builtin_amdgcn_readfirstlane((xcd_block() * NB_WAVES + (threadIdx.x >> 6)) * TR_RW);
  if (x0 >= n) return;
  int64_t s0[TR_RW];
  int len[TR_RW], a[TR_RW];
  int maxlen = 0;
#pragma unroll
  for (int r = 0; r < TR_RW; ++r) {
    const int x = x0 + r;
    s0[r] = x < n ? off[x] : 0;
    len[r] = x < n ? (int)(off[x + 1] - s0[r]) : 0;
    maxlen = max(maxlen, len[r]);
    a[r] = 0;
  }
  for (int base = 0; base < maxlen; base += 64) {
    const int k = base + lane;
    int y[TR_RW], lo[TR_RW], hi[TR_RW], found[TR_RW];
#pragma unroll
    for (int r = 0; r < TR_RW; ++r) y[r] = k < len[r] ? idx[s0[r] + k] : -1;
#pragma unroll
    for (int r = 0; r < TR_RW; ++r) {
      lo[r] = y[r] >= 0 ? (int)off[y[r]] : 0;  // nnz < 2^31: offsets fit
      hi[r] = y[r] >= 0 ? (int)off[y[r] + 1] : 0;
      found[r] = -1;
    }
    for (;;) {
      bool pend = false;
#pragma unroll
      for (int r = 0; r < TR_RW; ++r) pend |= lo[r] < hi[r];
      if (!pend) break;
      // a lane with a search still open has a non-empty row, so idx[0]
      // exists for its finished searches to read
      int mid[TR_RW], v[TR_RW];
#pragma unroll
      for (int r = 0; r < TR_RW; ++r) {
        mid[r] = lo[r] + ((hi[r] - lo[r]) >> 1);
        v[r] = idx[lo[r] < hi[r] ? mid[r] : 0];
      }
#pragma unroll
      for (int r = 0; r < TR_RW; ++r) {
        if (lo[r] < hi[r]) {
          if (v[r] < x0 + r) {
            lo[r] = mid[r] + 1;
          } else if (v[r] == x0 + r) {  // keys are distinct: the answer
            found[r] = lo[r] = hi[r] = mid[r];
          } else {
            hi[r] = mid[r];
          }
        }
      }
    }
    // a one-way entry's count on y is also its slot in B(y): rev holds
    // -(slot + 1)
    int slot[TR_RW];
#pragma unroll
    for (int r = 0; r < TR_RW; ++r) {
      slot[r] = 0;
      if (y[r] >= 0 && found[r] < 0) slot[r] = atomicAdd(&bcnt[y[r]], 1);
    }
#pragma unroll
    for (int r = 0; r < TR_RW; ++r) {
      if (y[r] >= 0) rev[s0[r] + k] = found[r] >= 0 ? found[r] : -(slot[r] + 1);
      a[r] += __popcll(__ballot(found[r] >= 0));
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int r = 0; r < TR_RW; ++r)
      if (x0 + r < n) acnt[x0 + r] = a[r];
  }
}

// Row lengths |A| + |B| for the scan.
__global__ void __launch_bounds__(NB_THREADS)
    k_tr_total(int n, const int32_t* __restrict__ acnt, const int32_t* __restrict__ bcnt,
               int32_t* __restrict__ tcount) {
  const int x = blockIdx.x * NB_THREADS + threadIdx.x;
  if (x >= n) return;
  tcount[x] = acnt[x] + bcnt[x];
}

// Pass 2: one-way entry s = (i, x) into B(x) at the slot pass 1 gave it:
// key i, payload s.  TR_RW forward rows i per wavefront, a lane per entry of
// each; the offsets' reads of all the rows are in flight before the first
// store.
__global__ void __launch_bounds__(NB_THREADS)
    k_tr_oneway(int n, const int64_t* __restrict__ off, const int32_t* __restrict__ idx,
                const int32_t* __restrict__ rev, const int64_t* __restrict__ toff,
                const int32_t* __restrict__ acnt, int32_t* __restrict__ tkey,
                int32_t* __restrict__ tpay) {
  const int lane = threadIdx.x & 63;
  const int i0 =
      __builtin_amdgcn_readfirstlane((xcd_block() * NB_WAVES + (threadIdx.x >> 6)) * TR_RW);
  if (i0 >= n) return;
  int64_t s0[TR_RW];
  int len[TR_RW];
  int maxlen = 0;
#pragma unroll
  for (int r = 0; r < TR_RW; ++r) {
    const int i = i0 + r;
    s0[r] = i < n ? off[i] : 0;
    len[r] = i < n ? (int)(off[i + 1] - s0[r]) : 0;
    maxlen = max(maxlen, len[r]);
  }
  for (int base = 0; base < maxlen; base += 64) {
    const int k = base + lane;
    int x[TR_RW], cur[TR_RW];
#pragma unroll
    for (int r = 0; r < TR_RW; ++r) {
      const bool in = k < len[r];
      const int32_t rv = in ? rev[s0[r] + k] : 0;
      const int32_t xr = in ? idx[s0[r] + k] : -1;
      x[r] = rv < 0 ? xr : -1;
      cur[r] = -rv - 1;  // the slot in B(x) (one-way entries)
    }
    int64_t t[TR_RW];
#pragma unroll
    for (int r = 0; r < TR_RW; ++r) {
      const int xs = x[r] >= 0 ? x[r] : 0;
      t[r] = toff[xs] + acnt[xs];
    }
#pragma unroll
    for (int r = 0; r < TR_RW; ++r) {
      if (x[r] >= 0) {
        tkey[t[r] + cur[r]] = i0 + r;
        tpay[t[r] + cur[r]] = (int32_t)(s0[r] + k);
      }
    }
  }
}

// compare-exchange of keys (and their payloads) held in registers a
// (lower index i) and b
__device__ __forceinline__ void bitonic_regs_kv(int32_t& ka, int32_t& va, int32_t& kb,
                                                int32_t& vb, int i, int k) {
  const bool up = (i & k) == 0;
  if ((ka > kb) == up) {
    const int32_t tk = ka, tv = va;
    ka = kb; va = vb;
    kb = tk; vb = tv;
  }
}

// wave_bitonic carrying a payload per key.
template <int R>
__device__ __forceinline__ void wave_bitonic_kv(int32_t (&key)[R], int32_t (&val)[R], int m,
                                                int lane) {
  for (int k = 2; k <= m; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      if (j >= 64) {
        if constexpr (R == 2) {
          bitonic_regs_kv(key[0], val[0], key[1], val[1], lane, k);
        } else if constexpr (R == 4) {
          if (j == 64) {
            bitonic_regs_kv(key[0], val[0], key[1], val[1], lane, k);
            bitonic_regs_kv(key[2], val[2], key[3], val[3], lane + 128, k);
          } else {
            bitonic_regs_kv(key[0], val[0], key[2], val[2], lane, k);
            bitonic_regs_kv(key[1], val[1], key[3], val[3], lane + 64, k);
          }
        }
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) {
          if (64 * r < m) {
            const int32_t wk = __shfl_xor(key[r], j, 64);
            const int32_t wv = __shfl_xor(val[r], j, 64);
            const int i = lane + 64 * r;
            const bool lower = (i & j) == 0, up = (i & k) == 0;
            // keep the smaller key where the pair runs up and this is its
            // lower end (or down and upper end), else the larger
            const bool take = (lower == up) ? (wk < key[r]) : (wk > key[r]);
            if (take) {
              key[r] = wk;
              val[r] = wv;
            }
          }
        }
      }
    }
  }
}

template <int R>
__device__ __forceinline__ void sort_write_trow(const int32_t* sk, const int32_t* sp, int len,
                                                int64_t t0, int lane, int32_t* __restrict__ tsrc,
                                                int32_t* __restrict__ tpos) {
  int mm = 1;
  while (mm < len) mm <<= 1;
  int32_t k[R], v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = lane + 64 * r;
    k[r] = e < len ? sk[e] : 0x7fffffff;
    v[r] = e < len ? sp[e] : -1;
  }
  wave_bitonic_kv<R>(k, v, mm, lane);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int e = lane + 64 * r;
    if (e < len) {
      tsrc[t0 + e] = k[r];
      tpos[v[r]] = (int32_t)(t0 + e);
    }
  }
}

// Pass 3, TR_RR transposed rows x per wavefront.  A row's mutual count
// (acnt) places its one-way part, so the first 64 entries of both parts of
// every row are read together before any is used.  A row without one-way
// entries is A itself, already in order: written as it is compacted.  With
// up to 64 one-way entries, each element's place is counted (an element of
// A: its index plus the B keys below it; of B: A's keys below it, by binary
// search, plus B's); with more, the row is sorted in registers.  Keys are
// distinct, so the places are a permutation.  Rows longer than NB_ROW with
// one-way entries are left in the scratch (A's part written there too) and
// listed for k_tr_long.
constexpr int TR_RR = 2;

__global__ void __launch_bounds__(NB_THREADS)
    k_tr_rows(int n, const int64_t* __restrict__ off, const int32_t* __restrict__ idx,
              const int32_t* __restrict__ rev, const int64_t* __restrict__ toff,
              const int32_t* __restrict__ acnt, int32_t* __restrict__ tkey,
              int32_t* __restrict__ tpay, int32_t* __restrict__ tsrc,
              int32_t* __restrict__ tpos, int32_t* __restrict__ long_list,
              int32_t* __restrict__ long_count) {
  __shared__ int32_t sk[NB_WAVES][TR_RR][NB_ROW], sp[NB_WAVES][TR_RR][NB_ROW];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int x0 = __builtin_amdgcn_readfirstlane((xcd_block() * NB_WAVES + wv) * TR_RR);
  if (x0 >= n) return;
  int64_t t0[TR_RR], s0[TR_RR];
  int tl[TR_RR], len[TR_RR], c[TR_RR];
#pragma unroll
  for (int r = 0; r < TR_RR; ++r) {
    const int x = x0 + r;
    const bool ok = x < n;
    t0[r] = ok ? toff[x] : 0;
    tl[r] = ok ? (int)(toff[x + 1] - t0[r]) : 0;
    s0[r] = ok ? off[x] : 0;
    len[r] = ok ? (int)(off[x + 1] - s0[r]) : 0;
    c[r] = ok ? acnt[x] : 0;
  }
  int32_t rv[TR_RR], y[TR_RR], bk[TR_RR], bp[TR_RR];
#pragma unroll
  for (int r = 0; r < TR_RR; ++r) {
    const bool in = lane < len[r];
    rv[r] = in ? rev[s0[r] + lane] : -1;
    y[r] = in ? idx[s0[r] + lane] : 0;
    const bool inb = tl[r] <= NB_ROW && c[r] + lane < tl[r];
    bk[r] = inb ? tkey[t0[r] + c[r] + lane] : 0;
    bp[r] = inb ? tpay[t0[r] + c[r] + lane] : 0;
  }
#pragma unroll
  for (int r = 0; r < TR_RR; ++r) {
    if (x0 + r >= n) break;
    const bool direct = c[r] == tl[r];  // no one-way entries
    const bool in_lds = tl[r] <= NB_ROW;
    int32_t* K = sk[wv][r];
    int32_t* P = sp[wv][r];
    int cc = 0;  // A's elements so far, in row order
    for (int base = 0; base < len[r]; base += 64) {
      int32_t v = rv[r], yy = y[r];
      if (base > 0) {
        const int k = base + lane;
        v = k < len[r] ? rev[s0[r] + k] : -1;
        yy = k < len[r] ? idx[s0[r] + k] : 0;
      }
      const bool mutual = v >= 0;
      const uint64_t mask = __ballot(mutual);
      const int at = cc + __popcll(mask & ((1ull << lane) - 1ull));
      if (mutual && at < tl[r]) {
        if (direct) {
          tsrc[t0[r] + at] = yy;
          tpos[v] = (int32_t)(t0[r] + at);
        } else if (in_lds) {
          K[at] = yy;
          P[at] = v;
        } else {
          tkey[t0[r] + at] = yy;
          tpay[t0[r] + at] = v;
        }
      }
      cc += __popcll(mask);
    }
    if (direct) continue;
    if (!in_lds) {
      if (lane == 0) long_list[atomicAdd(long_count, 1)] = x0 + r;
      continue;
    }
    for (int k = c[r] + lane; k < tl[r]; k += 64) {
      const bool first = k < c[r] + 64;
      K[k] = first ? bk[r] : tkey[t0[r] + k];
      P[k] = first ? bp[r] : tpay[t0[r] + k];
    }
    wave_lds_sync();
    if (tl[r] - c[r] <= 64) {
      for (int k = lane; k < tl[r]; k += 64) {
        const int32_t key = K[k];
        int rank = k;
        if (k >= c[r]) {  // first element of A not below the key
          int lo = 0, hi = c[r];
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (K[mid] < key) lo = mid + 1; else hi = mid;
          }
          rank = lo;
        }
        for (int j = c[r]; j < tl[r]; ++j) rank += K[j] < key ? 1 : 0;
        tsrc[t0[r] + rank] = key;
        tpos[P[k]] = (int32_t)(t0[r] + rank);
      }
    } else if (tl[r] <= 64) {
      sort_write_trow<1>(K, P, tl[r], t0[r], lane, tsrc, tpos);
    } else if (tl[r] <= 128) {
      sort_write_trow<2>(K, P, tl[r], t0[r], lane, tsrc, tpos);
    } else {
      sort_write_trow<4>(K, P, tl[r], t0[r], lane, tsrc, tpos);
    }
  }
}

// The listed transposed rows longer than NB_ROW (rare): each element's rank
// among its row's keys (distinct) is its place.
__global__ void __launch_bounds__(64)
    k_tr_long(const int32_t* __restrict__ long_list, const int32_t* __restrict__ long_count,
              const int64_t* __restrict__ toff, const int32_t* __restrict__ tkey,
              const int32_t* __restrict__ tpay, int32_t* __restrict__ tsrc,
              int32_t* __restrict__ tpos) {
  const int nl = *long_count;
  for (int q = blockIdx.x; q < nl; q += gridDim.x) {
    const int x = long_list[q];
    const int64_t t0 = toff[x];
    const int tl = (int)(toff[x + 1] - t0);
    for (int k = threadIdx.x; k < tl; k += 64) {
      const int32_t key = tkey[t0 + k];
      int rank = 0;
      for (int u = 0; u < tl; ++u) rank += tkey[t0 + u] < key ? 1 : 0;
      tsrc[t0 + rank] = key;
      tpos[tpay[t0 + k]] = (int32_t)(t0 + rank);
    }
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

int64_t nb_max_cells(int64_t n) {
  return std::min<int64_t>(NB_MAX_CELLS, std::max<int64_t>(4096, 8 * n));
}

size_t nb_work_bytes(int64_t n, int64_t m, int64_t capacity) {
  const int64_t mc = nb_max_cells(n);
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return al(3 * NB_VALIDATE_BLOCKS * sizeof(double)) + al(sizeof(Grid)) + al(2 * sizeof(double)) +
         al((size_t)n * sizeof(int32_t)) + 2 * al((size_t)(mc + 1) * sizeof(int32_t)) +
         al((size_t)scan_tmp_elems(mc + 1) * sizeof(int32_t)) + al((size_t)n * sizeof(int32_t)) +
         al((size_t)n * sizeof(double4)) + al((size_t)std::max<int64_t>(m, 1) * sizeof(int32_t)) +
         al((size_t)scan_tmp_elems(std::max<int64_t>(m, 1)) * sizeof(int64_t)) +
         al((size_t)std::max<int64_t>(capacity, 1) * sizeof(int32_t)) +
         al((size_t)std::max<int64_t>(m, 1) * NB_ROW * sizeof(int32_t)) +
         2 * al((size_t)std::max<int64_t>(m, 1) * sizeof(int32_t)) + al(sizeof(int32_t));
}

NbWork nb_work_take(Workspace& ws, int64_t n, int64_t m, int64_t capacity) {
  const int64_t mc = nb_max_cells(n);
  NbWork w;
  w.part = ws.take<double>(3 * NB_VALIDATE_BLOCKS);
  w.grid = ws.take<Grid>(1);
  w.lrange = ws.take<double>(2);
  w.key = ws.take<int32_t>(n);
  w.ccount = ws.take<int32_t>(mc + 1);
  w.cstart = ws.take<int32_t>(mc + 1);
  w.cscan = ws.take<int32_t>(scan_tmp_elems(mc + 1));
  w.sid = ws.take<int32_t>(n);
  w.spos = ws.take<double4>(n);
  w.cnt = ws.take<int32_t>(std::max<int64_t>(m, 1));
  w.oscan = ws.take<int64_t>(scan_tmp_elems(std::max<int64_t>(m, 1)));
  w.tmp = ws.take<int32_t>(std::max<int64_t>(capacity, 1));
  w.rowbuf = ws.take<int32_t>((size_t)std::max<int64_t>(m, 1) * NB_ROW);
  w.long_slot = ws.take<int32_t>(std::max<int64_t>(m, 1));
  w.long_row = ws.take<int32_t>(std::max<int64_t>(m, 1));
  w.long_count = ws.take<int32_t>(1);
  return w;
}

__global__ void k_nb_empty(int64_t* __restrict__ offsets, int64_t* __restrict__ nnz) {
  offsets[0] = 0;
  *nnz = 0;
}

hipError_t launch_neighbor_build(hipStream_t s, int n, const double* pos, const double* lam,
                                 const Box& box, double rf_ratio, int cells_per_rf, int m,
                                 const int32_t* rows, const NbWork& w, int64_t* offsets,
                                 int32_t* idx, int64_t capacity, int64_t* nnz, int32_t* flag) {
  const int64_t mc = nb_max_cells(n);
  hipLaunchKernelGGL(k_validate, dim3(NB_VALIDATE_BLOCKS), dim3(NB_THREADS), 0, s, n, pos, lam,
                     box, w.part);
  hipLaunchKernelGGL(k_nb_setup, dim3(1), dim3(64), 0, s, w.part, NB_VALIDATE_BLOCKS, box,
                     rf_ratio, cells_per_rf, mc, 1024, w.grid, flag, w.lrange);
  hipError_t e = fill_i32(s, w.ccount, 0, mc + 1);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cell_key, dim3(grid_for(n, NB_THREADS)), dim3(NB_THREADS), 0, s, n, pos,
                     w.grid, flag, w.key, w.ccount);
  if ((e = exclusive_scan_i32_to_i32(s, w.ccount, mc, w.cstart, w.cscan)) != hipSuccess) return e;
  if ((e = fill_i32(s, w.ccount, 0, mc)) != hipSuccess) return e;  // the scatter's cursors
  hipLaunchKernelGGL(k_cell_scatter, dim3(grid_for(n, NB_THREADS)), dim3(NB_THREADS), 0, s, n, pos,
                     lam, flag, w.key, w.cstart, w.ccount, w.sid, w.spos);
  if (m == 0) {
    hipLaunchKernelGGL(k_nb_empty, dim3(1), dim3(1), 0, s, offsets, nnz);
    return hipGetLastError();
  }
  const dim3 gw(grid_for(m, NB_WAVES));
  if ((e = fill_i32(s, w.long_count, 0, 1)) != hipSuccess) return e;
  hipLaunchKernelGGL((k_nb_wave<false>), gw, dim3(NB_THREADS), 0, s, m, rows, n, pos, lam, box,
                     w.grid, rf_ratio, w.cstart, w.sid, w.spos, flag, w.cnt, w.rowbuf, nullptr,
                     nullptr, w.long_slot, w.long_row, w.long_count);
  if ((e = exclusive_scan_i32_to_i64(s, w.cnt, m, offsets, w.oscan)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_nb_total, dim3(1), dim3(1), 0, s, offsets, m, capacity, nnz, flag);
  hipLaunchKernelGGL(k_nb_copy, dim3(grid_for((int64_t)m * 16, NB_THREADS)), dim3(NB_THREADS), 0,
                     s, m, offsets, w.rowbuf, flag, idx);
  // rows longer than NB_ROW are rare: small grids stride over their list
  hipLaunchKernelGGL((k_nb_wave<true>), dim3(NB_LONG_BLOCKS), dim3(NB_THREADS), 0, s, m, rows, n,
                     pos, lam, box, w.grid, rf_ratio, w.cstart, w.sid, w.spos, flag, nullptr,
                     nullptr, offsets, w.tmp, w.long_slot, w.long_row, w.long_count);
  hipLaunchKernelGGL(k_row_sort, dim3(NB_LONG_BLOCKS * NB_WAVES), dim3(64), 0, s, w.long_row,
                     w.long_count, offsets, w.tmp, idx, flag);
  return hipGetLastError();
}

TransposeWork transpose_work_take(Workspace& ws, int64_t n, int64_t nnz) {
  TransposeWork w;
  w.acnt = ws.take<int32_t>(n);
  w.bcnt = ws.take<int32_t>(n);
  w.tcount = ws.take<int32_t>(n);
  w.scan = ws.take<int64_t>(scan_tmp_elems(n));
  w.rev = ws.take<int32_t>(std::max<int64_t>(nnz, 1));
  w.tkey = ws.take<int32_t>(std::max<int64_t>(nnz, 1));
  w.tpay = ws.take<int32_t>(std::max<int64_t>(nnz, 1));
  w.long_list = ws.take<int32_t>(std::max<int64_t>(n, 1));
  w.counts = ws.take<int32_t>(2);
  return w;
}

size_t transpose_work_bytes(int64_t n, int64_t nnz) {
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  return 3 * al((size_t)n * sizeof(int32_t)) + al((size_t)scan_tmp_elems(n) * sizeof(int64_t)) +
         3 * al((size_t)std::max<int64_t>(nnz, 1) * sizeof(int32_t)) +
         al((size_t)std::max<int64_t>(n, 1) * sizeof(int32_t)) + al(2 * sizeof(int32_t));
}

hipError_t launch_transpose(hipStream_t s, int n, const int64_t* off, const int32_t* idx,
                            int64_t* toff, int32_t* tsrc, int32_t* tpos,
                            const TransposeWork& w) {
  hipError_t e = fill_i32(s, w.bcnt, 0, n);
  if (e != hipSuccess) return e;
  if ((e = fill_i32(s, w.counts, 0, 2)) != hipSuccess) return e;
  const dim3 gw(grid_for(n, NB_WAVES * TR_RW)), gr(grid_for(n, NB_WAVES * TR_RR));
  hipLaunchKernelGGL(k_tr_mutual, gw, dim3(NB_THREADS), 0, s, n, off, idx, w.rev, w.acnt,
                     w.bcnt);
  hipLaunchKernelGGL(k_tr_total, dim3(grid_for(n, NB_THREADS)), dim3(NB_THREADS), 0, s, n,
                     w.acnt, w.bcnt, w.tcount);
  if ((e = exclusive_scan_i32_to_i64(s, w.tcount, n, toff, w.scan)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_tr_oneway, gw, dim3(NB_THREADS), 0, s, n, off, idx, w.rev, toff, w.acnt,
                     w.tkey, w.tpay);
  hipLaunchKernelGGL(k_tr_rows, gr, dim3(NB_THREADS), 0, s, n, off, idx, w.rev, toff, w.acnt,
                     w.tkey, w.tpay, tsrc, tpos, w.long_list, w.counts + 1);
  hipLaunchKernelGGL(k_tr_long, dim3(NB_LONG_BLOCKS * NB_WAVES), dim3(64), 0, s, w.long_list,
                     w.counts + 1, toff, w.tkey, w.tpay, tsrc, tpos);
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
