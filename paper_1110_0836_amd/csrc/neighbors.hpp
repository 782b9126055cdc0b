// Launchers of the neighbor-search, transpose and ordering kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device.hpp"

namespace phb {

// Uniform cell grid over the box: nc cells per axis of side L/nc.
struct Grid {
  int nc[3];
  double inv_h[3];  // nc / L
  double margin;    // slack added to every candidate range (far above rounding)
};

hipError_t launch_validate(hipStream_t s, int n, const double* pos, const double* lam,
                           const Box& box, double* part, int nblocks);
hipError_t launch_cell_sort(hipStream_t s, int n, const double* pos, const double* lam,
                            const Grid& g, int32_t* key, int32_t* cell_count,
                            int32_t* cell_start, int32_t* scan_tmp, int32_t* sorted_id,
                            double4* spos);
hipError_t launch_neighbor_count(hipStream_t s, int n, const Box& box, const Grid& g,
                                 double rf_ratio, const int32_t* cell_start,
                                 const int32_t* sorted_id, const double4* spos, int32_t* count);
hipError_t launch_neighbor_fill(hipStream_t s, int n, const Box& box, const Grid& g,
                                double rf_ratio, const int32_t* cell_start,
                                const int32_t* sorted_id, const double4* spos,
                                const int64_t* offsets, int32_t* tmp);
// The same for the particles rows[0 .. m): counts and entries per row.
hipError_t launch_neighbor_count_rows(hipStream_t s, int m, const int32_t* rows, int n,
                                      const double* pos, const double* lam, const Box& box,
                                      const Grid& g, double rf_ratio, const int32_t* cell_start,
                                      const int32_t* sorted_id, const double4* spos,
                                      int32_t* count);
hipError_t launch_neighbor_fill_rows(hipStream_t s, int m, const int32_t* rows, int n,
                                     const double* pos, const double* lam, const Box& box,
                                     const Grid& g, double rf_ratio, const int32_t* cell_start,
                                     const int32_t* sorted_id, const double4* spos,
                                     const int64_t* offsets, int32_t* tmp);
hipError_t launch_row_sort(hipStream_t s, int64_t nrows, const int64_t* off, const int32_t* in,
                           int32_t* out);
hipError_t launch_transpose(hipStream_t s, int n, int64_t nnz, const int64_t* off,
                            const int32_t* idx, int64_t* toff, int32_t* tsrc, int32_t* tpos,
                            int32_t* count, int64_t* scan_tmp, int32_t* tmp);
// perm = the particles in the order of their cells' Hilbert indices on a
// 1024^3 grid over the box of side lengths L (ties by index).  bin_count and
// bin_start hold 2^21 + 1 entries, scan_tmp scan_tmp_elems(2^21).
hipError_t launch_hilbert_order(hipStream_t s, int n, const double* pos, const double* L,
                                int32_t* key, int32_t* bin_count, int32_t* bin_start,
                                int32_t* scan_tmp, int32_t* perm);
hipError_t launch_permute(hipStream_t s, int n, int ncomp, const int32_t* perm, const double* src,
                          double* dst);

}  // namespace phb
