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
// Device scratch of one build (nb_work_bytes plans it, nb_work_take carves
// it; internal.hpp's Workspace).
struct NbWork {
  double* part;     // k_validate's per-block partials
  Grid* grid;       // the cell grid, sized on the device
  double* lrange;   // lambda min, max
  int32_t* key;
  int32_t* ccount;  // cell counts, then the scatter's cursors
  int32_t* cstart;
  int32_t* cscan;
  int32_t* sid;     // particle of each cell-sorted slot
  double4* spos;    // (x, y, z, lambda) in cell order
  int32_t* cnt;     // row lengths
  int64_t* oscan;
  int32_t* tmp;     // rows longer than the in-register sort takes, unsorted
  int32_t* rowbuf;  // sorted rows, NB_ROW entries per row
  int32_t* long_slot;   // rows longer than NB_ROW: their wavefront index,
  int32_t* long_row;    // their output row,
  int32_t* long_count;  // and how many
};
// Most cells of the grid: 8 per particle, at least 4096, at most 2^23.
constexpr int64_t NB_MAX_CELLS = int64_t(1) << 23;
constexpr int NB_VALIDATE_BLOCKS = 512;
int64_t nb_max_cells(int64_t n);
size_t nb_work_bytes(int64_t n, int64_t m, int64_t capacity);
struct Workspace;
NbWork nb_work_take(Workspace& ws, int64_t n, int64_t m, int64_t capacity);
// The whole search on the stream, without host synchronization: lists of
// all n particles (rows == null; m == n) or of rows[0 .. m) into offsets[m +
// 1] and idx (at most capacity entries), nnz = offsets[m] into *nnz and the
// status bits (PHB_NB_*) into *flag.  On invalid input the offsets are zero;
// on overflow idx is not written.
hipError_t launch_neighbor_build(hipStream_t s, int n, const double* pos, const double* lam,
                                 const Box& box, double rf_ratio, int cells_per_rf, int m,
                                 const int32_t* rows, const NbWork& w, int64_t* offsets,
                                 int32_t* idx, int64_t capacity, int64_t* nnz, int32_t* flag);
// Scratch of the transpose.
struct TransposeWork {
  int32_t* acnt;    // |A(x)|: mutual entries of row x
  int32_t* bcnt;    // |B(x)|: one-way entries into x, then cursors
  int32_t* tcount;  // transposed row lengths
  int64_t* scan;
  int32_t* rev;     // per entry: the mirrored entry, or -1
  int32_t* tkey;    // B's elements (and long rows) before their sort
  int32_t* tpay;    // the forward entry each stands for
  int32_t* long_list;  // transposed rows longer than the in-register sort takes
  int32_t* counts;     // [1]: long rows ([0] unused)
};
size_t transpose_work_bytes(int64_t n, int64_t nnz);
TransposeWork transpose_work_take(Workspace& ws, int64_t n, int64_t nnz);
// t_offsets, t_src, t_pos of the lists (off, idx) of n rows; the kernels
// read the entry count from the offsets (the scratch sizes it).
hipError_t launch_transpose(hipStream_t s, int n, const int64_t* off, const int32_t* idx,
                            int64_t* toff, int32_t* tsrc, int32_t* tpos,
                            const TransposeWork& w);
// perm = the particles in the order of their cells' Hilbert indices on a
// 1024^3 grid over the box of side lengths L (ties by index).  bin_count and
// bin_start hold 2^21 + 1 entries, scan_tmp scan_tmp_elems(2^21).
hipError_t launch_hilbert_order(hipStream_t s, int n, const double* pos, const double* L,
                                int32_t* key, int32_t* bin_count, int32_t* bin_start,
                                int32_t* scan_tmp, int32_t* perm);
hipError_t launch_permute(hipStream_t s, int n, int ncomp, const int32_t* perm, const double* src,
                          double* dst);

}  // namespace phb
