// Many independent particle sets evaluated together, replayed from one
// captured HIP graph, and the schedule autotuner.
//
// The sets are concatenated (SoA over the total particle count, set s owning
// particles set_offsets[s] .. set_offsets[s+1]); their neighbor lists are
// built set by set and stored as one CSR with global indices.  A particle's
// evaluation reads only its own row, so the evaluation kernels treat the
// concatenation as a single index space: every stage of the forward and
// reverse pass is one launch over all particles of all sets, whatever the
// number of sets, and the whole pass is captured once and replayed with a
// single graph launch.
//
// Capture runs on a private non-blocking stream (the context's stream may be
// the null stream, which cannot be captured); launches are ordered after the
// caller's stream by an event and the caller's stream waits for the replay.
// Nothing inside the captured region allocates, synchronizes or sets memory
// with a memset node: the workspace is sized by an eager run of the same pass
// before capture, and counters are cleared by kernels.
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "adjoint.hpp"
#include "internal.hpp"

struct phb_batch {
  int device = 0;
  phb_params p{};
  std::vector<int64_t> set_off;
  int64_t n_total = 0;
  int64_t max_set = 0;
  int64_t nnz = -1;
  double* tmp_pos = nullptr;
  int64_t* tmp_off = nullptr;
  hipStream_t stream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // Workspace the captured graph runs in, owned by the batch so that later
  // calls may regrow the context's arena without touching it.
  char* arena = nullptr;
  size_t arena_cap = 0;
  // The reverse mode's tile schedule tiles each set from its first particle,
  // as a call on that set alone does (tile starts, device, ntiles + 1).
  int32_t* tiles = nullptr;
  int64_t ntiles = 0;
};

namespace phb {
namespace {

constexpr int THREADS = 256;

__global__ void k_gather_set_pos(int ns, const double* __restrict__ pos, int64_t n_total,
                                 int64_t start, double* __restrict__ out) {
  const int i = blockIdx.x * THREADS + threadIdx.x;
  if (i >= ns) return;
#pragma unroll
  for (int a = 0; a < 3; ++a) out[(int64_t)a * ns + i] = pos[a * n_total + start + i];
}

// offsets[start + i] = base + local[i] for i <= ns.
__global__ void k_shift_offsets(int ns, const int64_t* __restrict__ local, int64_t base,
                                int64_t* __restrict__ offsets) {
  const int i = blockIdx.x * THREADS + threadIdx.x;
  if (i > ns) return;
  offsets[i] = base + local[i];
}

// idx[k] += start for k < m (the set's rows, written in place).
__global__ void k_shift_idx(int64_t m, int32_t start, int32_t* __restrict__ idx) {
  const int64_t k = (int64_t)blockIdx.x * THREADS + threadIdx.x;
  if (k < m) idx[k] += start;
}

void drop_graph(phb_batch* b) {
  if (b->exec || b->arena) hipStreamSynchronize(b->stream);
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->arena) hipFree(b->arena);
  b->exec = nullptr;
  b->graph = nullptr;
  b->arena = nullptr;
  b->arena_cap = 0;
}

// One forward (+ reverse) pass over all sets on ctx->stream.
int batch_pass(phb_ctx* ctx, phb_batch* b, const phb_batch_io* io) {
  EvalArgs a;
  int rc;
  if ((rc = eval_args(ctx, &b->p, b->n_total, io->pos, io->lambda, io->offsets, io->idx, &a)))
    return rc;
  if ((rc = eval_rhs(ctx, a, &b->p, io->q, io->rhs, io->dxdt, io->status,
                     reinterpret_cast<double*>(io->tape))))
    return rc;
  if (!io->q_bar) return PHB_OK;
  return adjoint_rhs(ctx, a, &b->p, io->t_offsets, io->t_src, io->t_pos, io->q, io->rhs_bar,
                     io->dxdt_bar, io->q_bar, io->pos_bar,
                     reinterpret_cast<const double*>(io->tape), b->nnz, true, b->tiles,
                     b->ntiles);
}

int check_io(phb_ctx* ctx, const phb_batch* b, const phb_batch_io* io) {
  if (!io || !io->pos || !io->lambda || !io->offsets || !io->idx || !io->q || !io->rhs ||
      !io->dxdt || !io->status)
    return set_error(ctx, PHB_EINVAL, "batch io: null pointer");
  if ((io->q_bar == nullptr) != (io->pos_bar == nullptr))
    return set_error(ctx, PHB_EINVAL, "batch io: q_bar and pos_bar go together");
  if (io->q_bar && (!io->rhs_bar || !io->t_offsets || !io->t_src || !io->t_pos))
    return set_error(ctx, PHB_EINVAL, "batch io: the reverse pass needs rhs_bar and the "
                                      "transposed lists");
  if (b->nnz < 0) return set_error(ctx, PHB_ESTATE, "batch neighbors not built");
  return PHB_OK;
}

}  // namespace
}  // namespace phb

using namespace phb;

extern "C" {

int phb_batch_create(phb_ctx* ctx, const phb_params* p, int32_t n_sets,
                     const int64_t* set_offsets, phb_batch** out) {
  if (!ctx || !out) return PHB_EINVAL;
  *out = nullptr;
  int rc;
  if ((rc = check_params(ctx, p))) return rc;
  if (n_sets <= 0 || !set_offsets || set_offsets[0] != 0)
    return set_error(ctx, PHB_EINVAL, "set offsets must start at 0 and n_sets be positive");
  int64_t mx = 0;
  for (int s = 0; s < n_sets; ++s) {
    const int64_t ns = set_offsets[s + 1] - set_offsets[s];
    if (ns <= 0) return set_error(ctx, PHB_EINVAL, "every set needs at least one particle");
    mx = std::max(mx, ns);
  }
  if ((rc = check_n(ctx, set_offsets[n_sets]))) return rc;
  hipSetDevice(ctx->device);
  phb_batch* b = new phb_batch();
  b->device = ctx->device;
  b->p = *p;
  b->set_off.assign(set_offsets, set_offsets + n_sets + 1);
  b->n_total = set_offsets[n_sets];
  b->max_set = mx;
  hipError_t e = hipMalloc((void**)&b->tmp_pos, (size_t)3 * mx * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&b->tmp_off, (size_t)(mx + 1) * sizeof(int64_t));
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming);
  if (e == hipSuccess) {
    std::vector<int32_t> t;
    for (int s = 0; s < n_sets; ++s) {
      const int64_t ns = set_offsets[s + 1] - set_offsets[s];
      const int64_t ts = adjoint_pair_tile();
      for (int64_t k = 0; k < ns; k += ts) t.push_back((int32_t)(set_offsets[s] + k));
    }
    t.push_back((int32_t)b->n_total);
    b->ntiles = (int64_t)t.size() - 1;
    e = hipMalloc((void**)&b->tiles, t.size() * sizeof(int32_t));
    if (e == hipSuccess)
      e = hipMemcpy(b->tiles, t.data(), t.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    phb_batch_destroy(b);
    return hip_check(ctx, e, "batch create");
  }
  *out = b;
  return PHB_OK;
}

int phb_batch_destroy(phb_batch* b) {
  if (!b) return PHB_EINVAL;
  hipSetDevice(b->device);
  if (b->stream) hipStreamSynchronize(b->stream);
  drop_graph(b);
  if (b->ev_in) hipEventDestroy(b->ev_in);
  if (b->ev_out) hipEventDestroy(b->ev_out);
  if (b->stream) hipStreamDestroy(b->stream);
  if (b->tmp_pos) hipFree(b->tmp_pos);
  if (b->tmp_off) hipFree(b->tmp_off);
  if (b->tiles) hipFree(b->tiles);
  delete b;
  return PHB_OK;
}

int phb_batch_neighbors(phb_ctx* ctx, phb_batch* b, const double* pos, const double* lambda,
                        int64_t* offsets, int32_t* idx, int64_t idx_capacity, int64_t* nnz_out) {
  if (!ctx || !b || !pos || !lambda || !offsets || !idx || !nnz_out || idx_capacity < 0)
    return PHB_EINVAL;
  hipSetDevice(ctx->device);
  drop_graph(b);  // a graph bound to the old lists must not be replayed
  b->nnz = -1;
  int64_t base = 0;
  bool short_cap = false;
  int rc;
  for (size_t s = 0; s + 1 < b->set_off.size(); ++s) {
    const int64_t start = b->set_off[s];
    const int ns = (int)(b->set_off[s + 1] - start);
    hipLaunchKernelGGL(k_gather_set_pos, dim3(grid_for(ns, THREADS)), dim3(THREADS), 0,
                       ctx->stream, ns, pos, b->n_total, start, b->tmp_pos);
    if ((rc = hip_check(ctx, hipGetLastError(), "batch gather"))) return rc;
    const int64_t cap = short_cap ? 0 : idx_capacity - base;
    int64_t got = 0;
    rc = phb_neighbors_build(ctx, &b->p, ns, b->tmp_pos, lambda + start, b->tmp_off, idx + base,
                             cap, &got);
    if (rc == PHB_ECAPACITY) {
      short_cap = true;  // keep counting what the remaining sets need
    } else if (rc) {
      return rc;
    } else if (!short_cap) {
      hipLaunchKernelGGL(k_shift_offsets, dim3(grid_for(ns + 1, THREADS)), dim3(THREADS), 0,
                         ctx->stream, ns, b->tmp_off, base, offsets + start);
      if (got > 0)
        hipLaunchKernelGGL(k_shift_idx, dim3(grid_for(got, THREADS)), dim3(THREADS), 0,
                           ctx->stream, got, (int32_t)start, idx + base);
      if ((rc = hip_check(ctx, hipGetLastError(), "batch shift"))) return rc;
    }
    base += got;
  }
  *nnz_out = base;
  if (base > PHB_NNZ_MAX)
    return set_error(ctx, PHB_EINVAL, "nnz exceeds the int32 positions of the transposed lists");
  if (short_cap)
    return set_error(ctx, PHB_ECAPACITY, "idx capacity " + std::to_string(idx_capacity) +
                                             " < " + std::to_string(base));
  if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "batch neighbors sync"))) return rc;
  b->nnz = base;
  return PHB_OK;
}

int phb_batch_run(phb_ctx* ctx, phb_batch* b, const phb_batch_io* io) {
  if (!ctx || !b) return PHB_EINVAL;
  int rc;
  if ((rc = check_io(ctx, b, io))) return rc;
  hipSetDevice(ctx->device);
  return batch_pass(ctx, b, io);
}

int phb_batch_capture(phb_ctx* ctx, phb_batch* b, const phb_batch_io* io) {
  if (!ctx || !b) return PHB_EINVAL;
  int rc;
  if ((rc = check_io(ctx, b, io))) return rc;
  if (ctx->arena_base != 0) return set_error(ctx, PHB_ESTATE, "capture inside another call");
  hipSetDevice(ctx->device);
  drop_graph(b);
  // eager pass: sizes the workspace and reports any error outside capture
  if ((rc = batch_pass(ctx, b, io))) return rc;
  if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "batch warm-up"))) return rc;
  const size_t cap = ctx->arena_cap;
  hipError_t ea = hipMalloc((void**)&b->arena, cap);
  if (ea != hipSuccess) {
    b->arena = nullptr;
    return set_error(ctx, PHB_ENOMEM, "batch workspace of " + std::to_string(cap) + " bytes");
  }
  b->arena_cap = cap;
  hipStream_t saved = ctx->stream;
  char* saved_arena = ctx->arena;
  const size_t saved_cap = ctx->arena_cap;
  const bool prof = ctx->prof_on;
  ctx->stream = b->stream;
  ctx->arena = b->arena;
  ctx->arena_cap = b->arena_cap;
  ctx->prof_on = false;
  ctx->capturing = true;
  hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    rc = batch_pass(ctx, b, io);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->stream, &g);
    if (e2 == hipSuccess) b->graph = g;
    if (!rc) e = e2;
  }
  ctx->stream = saved;
  ctx->arena = saved_arena;
  ctx->arena_cap = saved_cap;
  ctx->prof_on = prof;
  ctx->capturing = false;
  if (rc) {
    drop_graph(b);
    return rc;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    drop_graph(b);
    return hip_check(ctx, e, "batch capture");
  }
  return PHB_OK;
}

int phb_batch_launch(phb_ctx* ctx, phb_batch* b) {
  if (!ctx || !b) return PHB_EINVAL;
  if (!b->exec) return set_error(ctx, PHB_ESTATE, "no captured graph");
  hipSetDevice(ctx->device);
  hipError_t e = hipEventRecord(b->ev_in, ctx->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->ev_in, 0);
  if (e == hipSuccess) e = hipGraphLaunch(b->exec, b->stream);
  if (e == hipSuccess) e = hipEventRecord(b->ev_out, b->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(ctx->stream, b->ev_out, 0);
  return hip_check(ctx, e, "batch launch");
}

// ---------------------------------------------------------------------------
// Autotuner: coordinate descent over the schedule knobs, timing one forward
// plus reverse pass per candidate with HIP events (median of reps after one
// warm-up), on the caller's particle set.  The choice is kept on the context
// (so a later capture bakes it in) and, given a path, written to a small text
// cache keyed by n, nnz and precision.
// ---------------------------------------------------------------------------
int phb_tune(phb_ctx* ctx, const phb_params* p, int64_t n64, const double* pos,
             const double* lambda, const int64_t* offsets, const int32_t* idx,
             const int64_t* t_offsets, const int32_t* t_src, const int32_t* t_pos, int64_t nnz,
             const double* q, int32_t reps, const char* cache_path) {
  if (!ctx) return PHB_EINVAL;
  EvalArgs a;
  int rc;
  if ((rc = eval_args(ctx, p, n64, pos, lambda, offsets, idx, &a))) return rc;
  if (!t_offsets || !t_src || !t_pos || !q || nnz < 0 || reps <= 0)
    return set_error(ctx, PHB_EINVAL, "tune: bad arguments");
  hipSetDevice(ctx->device);
  struct Knob {
    const char* key;
    std::vector<int> values;
  };
  const std::vector<Knob> knobs = {
      {"lanes_moments", {1, 2, 4}}, {"lanes_apply", {1, 2, 4}},  {"lanes_adj_y", {1, 2, 4}},
      {"lanes_gather", {1, 2, 4}},  {"adj_pairs_mode", {0, 1, 2, 3}}, {"record_order", {0, 1}},
      {"fit_fields", {2, 4}}, {"moments_mfma", {0, 1}}};
  char sig[160];
  snprintf(sig, sizeof sig, "# phurbas-tune n=%lld nnz=%lld precision=%d weight=%d",
           (long long)n64, (long long)nnz, p->precision, p->weight);
  if (cache_path) {
    if (FILE* f = fopen(cache_path, "r")) {
      char line[256];
      bool match = fgets(line, sizeof line, f) && !strncmp(line, sig, strlen(sig));
      std::vector<std::pair<std::string, int>> got;
      char key[64];
      int v;
      while (match && fscanf(f, "%63s %d", key, &v) == 2) got.emplace_back(key, v);
      fclose(f);
      if (match && got.size() == knobs.size()) {
        for (auto& kv : got)
          if ((rc = phb_tune_set(ctx, kv.first.c_str(), kv.second))) return rc;
        return PHB_OK;
      }
    }
  }
  const int n = a.n;
  double *rhs = nullptr, *dxdt = nullptr, *tape = nullptr, *gbar = nullptr, *qb = nullptr,
         *pb = nullptr;
  int32_t* st = nullptr;
  hipError_t e = hipMalloc((void**)&rhs, (size_t)8 * n * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&dxdt, (size_t)3 * n * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&tape, (size_t)tape_doubles(n) * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&gbar, (size_t)8 * n * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&qb, (size_t)8 * n * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&pb, (size_t)3 * n * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void**)&st, (size_t)n * sizeof(int32_t));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = fill_f64(ctx->stream, gbar, 1.0, (int64_t)8 * n);
  rc = hip_check(ctx, e, "tune buffers");
  auto pass = [&]() -> int {
    int r = eval_rhs(ctx, a, p, q, rhs, dxdt, st, tape);
    if (!r) r = adjoint_rhs(ctx, a, p, t_offsets, t_src, t_pos, q, gbar, nullptr, qb, pb, tape, nnz);
    return r;
  };
  auto time_once = [&](double* ms) -> int {
    int r = pass();  // warm-up
    std::vector<float> t;
    for (int k = 0; !r && k < reps; ++k) {
      hipEventRecord(e0, ctx->stream);
      r = pass();
      hipEventRecord(e1, ctx->stream);
      if (!r) r = hip_check(ctx, hipEventSynchronize(e1), "tune sync");
      float x = 0.f;
      hipEventElapsedTime(&x, e0, e1);
      t.push_back(x);
    }
    if (!r) {
      std::sort(t.begin(), t.end());
      *ms = t[t.size() / 2];
    }
    return r;
  };
  const bool prof = ctx->prof_on;
  ctx->prof_on = false;
  double best = 0.0;
  if (!rc) rc = time_once(&best);
  for (size_t k = 0; !rc && k < knobs.size(); ++k) {
    int cur = 0;
    phb_tune_get(ctx, knobs[k].key, &cur);
    for (int v : knobs[k].values) {
      if (v == cur) continue;
      phb_tune_set(ctx, knobs[k].key, v);
      double ms = 0.0;
      if ((rc = time_once(&ms))) break;
      if (ms < best * 0.98) {  // a clear win only: timing noise keeps the current value
        best = ms;
        cur = v;
      }
    }
    phb_tune_set(ctx, knobs[k].key, cur);
  }
  ctx->prof_on = prof;
  hipStreamSynchronize(ctx->stream);
  if (e0) hipEventDestroy(e0);
  if (e1) hipEventDestroy(e1);
  for (void* ptr : {(void*)rhs, (void*)dxdt, (void*)tape, (void*)gbar, (void*)qb, (void*)pb,
                    (void*)st})
    if (ptr) hipFree(ptr);
  if (rc) return rc;
  if (cache_path) {
    FILE* f = fopen(cache_path, "w");
    if (!f) return set_error(ctx, PHB_EINVAL, std::string("cannot write ") + cache_path);
    fprintf(f, "%s\n", sig);
    for (auto& kb : knobs) {
      int v = 0;
      phb_tune_get(ctx, kb.key, &v);
      fprintf(f, "%s %d\n", kb.key, v);
    }
    fclose(f);
  }
  return PHB_OK;
}

}  // extern "C"
