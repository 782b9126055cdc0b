// Host-side internals of libphurbas: context, workspace, launch helpers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <vector>

#include "phurbas.h"
#include "device.hpp"
#include "mhd.hpp"

struct phb_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  // Workspace arena (device memory owned by the library).
  char* arena = nullptr;
  size_t arena_cap = 0;
  size_t arena_base = 0;  // bytes held by an enclosing call (nested workspaces start here)
  // Pinned host staging for small read-backs.
  char* host = nullptr;
  size_t host_cap = 0;
  std::string last_error;
  // Tunables (see phb_tune_* in the binding).
  int cells_per_rf = 2;      // neighbor grid cells per minimum r_f
  int lanes_assemble = 4;    // lanes per particle in the moment loops (1, 2, 4)
  int lanes_apply = 4;
  int lanes_adj_y = 2;
  int lanes_gather = 4;
  int fit_fields = 4;        // FP64 fit right-hand sides: fields per lane (2, 4)
  int moments_mfma = 0;      // mixed form: FP32 moments on the matrix cores (1)
  int mixed_cond_x10 = -1;  // mixed form: FP64 path above ||A_hat^-1|| ~ 10^(x10 / 10)
  int mixed_refine = 2;     // mixed form: 1 operator-level, 0 data-level, 2 by shape
  int fp64_cut_x10 = -1;    // refinement of fits whose inverse has a row norm above
                            // 10^(x10 / 10); -1: the shape's default, 999: never
  int adj_pairs_mode = 3;  // 0: one lane per entry, 1: one wavefront per owner, 2: pipelined,
                           // 3: one block per tile of owners
  int record_order = 0;    // pair records at 0: transposed positions, 1: forward slots
  // Per-kernel timing (phb_profile): event pairs awaiting read-out and totals.
  bool capturing = false;  // a graph capture is recording the context stream
  // An allocation-free call is running: the workspace is the static scratch
  // and may not grow, and no second stream is used.
  bool no_alloc = false;
  bool prof_on = false;
  struct ProfRec {
    const char* name;
    hipEvent_t a, b;
  };
  std::vector<ProfRec> prof_pending;
  std::map<std::string, std::pair<double, int>> prof_total;
};

namespace phb {

int set_error(phb_ctx* ctx, int code, const std::string& msg);
int check_params(phb_ctx* ctx, const phb_params* p);
// Grows the context's pinned host staging buffer (ctx->host) to bytes.
int ensure_host(phb_ctx* ctx, size_t bytes);
int check_n(phb_ctx* ctx, int64_t n);
// The stabiliser coefficients of p (all zero: ideal MHD).
Stab stab_of(const phb_params* p);
int hip_check(phb_ctx* ctx, hipError_t e, const char* what);

// Carves 256-byte aligned pieces out of the context arena.  Sizes are summed
// first (plan), the arena grown once, then pieces handed out (take).
struct Workspace {
  phb_ctx* ctx;
  size_t total = 0;
  size_t cursor = 0;
  explicit Workspace(phb_ctx* c) : ctx(c), cursor(c->arena_base) {}
  void plan(size_t bytes) { total += (bytes + 255) & ~size_t(255); }
  // Grows the arena if needed (synchronizes the stream when it grows).  A
  // nested workspace (arena_base > 0) may not grow it: the enclosing call
  // must have reserved enough.
  int commit();
  template <class T>
  T* take(size_t count) {
    const size_t bytes = (count * sizeof(T) + 255) & ~size_t(255);
    T* p = reinterpret_cast<T*>(ctx->arena + cursor);
    cursor += bytes;
    return p;
  }
};

// Keeps the first `bytes` of the arena for the caller while nested calls run.
struct ArenaHold {
  phb_ctx* ctx;
  size_t saved;
  ArenaHold(phb_ctx* c, size_t bytes) : ctx(c), saved(c->arena_base) { c->arena_base += bytes; }
  ~ArenaHold() { ctx->arena_base = saved; }
};

// Brackets one kernel launch with HIP events on the context stream when
// profiling is on.
struct Prof {
  phb_ctx* ctx;
  phb_ctx::ProfRec rec{nullptr, nullptr, nullptr};
  Prof(phb_ctx* c, const char* name) : ctx(c) {
    if (!c->prof_on) return;
    rec.name = name;
    hipEventCreate(&rec.a);
    hipEventCreate(&rec.b);
    hipEventRecord(rec.a, c->stream);
  }
  ~Prof() {
    if (!rec.name) return;
    hipEventRecord(rec.b, ctx->stream);
    ctx->prof_pending.push_back(rec);
  }
};

Box make_box(const phb_params* p);

// Workspace bytes of the composite entry points (used to reserve ahead of
// nested calls).
size_t ws_bytes_neighbors(int64_t n, int64_t idx_capacity);
size_t ws_bytes_rhs(int64_t n, const phb_params* p);
size_t ws_bytes_derivs(int64_t n, const phb_params* p, bool second);

inline unsigned grid_for(int64_t work, int block) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 0x7fffffff) g = 0x7fffffff;
  return (unsigned)g;
}

// ---- launchers (stream-ordered, return the launch error) ----
hipError_t fill_i32(hipStream_t s, int32_t* p, int32_t v, int64_t n);
hipError_t fill_f64(hipStream_t s, double* p, double v, int64_t n);
// Exclusive scan of n int32 counts into out[0..n] (out[n] = total).  tmp needs
// scan_tmp_elems(n) elements of T.
int64_t scan_tmp_elems(int64_t n);
hipError_t exclusive_scan_i32_to_i64(hipStream_t s, const int32_t* in, int64_t n, int64_t* out,
                                     int64_t* tmp);
hipError_t exclusive_scan_i32_to_i32(hipStream_t s, const int32_t* in, int64_t n, int32_t* out,
                                     int32_t* tmp);

}  // namespace phb
