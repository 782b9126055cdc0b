// C-ABI entry points of libphurbas (see include/phurbas.h for the contract).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "internal.hpp"
#include "mls.hpp"
#include "neighbors.hpp"
#include "adjoint.hpp"
#include "refine.hpp"

namespace phb {

int set_error(phb_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->last_error = msg;
  return code;
}

int hip_check(phb_ctx* ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return PHB_OK;
  return set_error(ctx, PHB_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

int Workspace::commit() {
  const size_t need = ctx->arena_base + total;
  if (need <= ctx->arena_cap) return PHB_OK;
  if (ctx->no_alloc)
    return set_error(ctx, PHB_ECAPACITY, "the static scratch holds " +
                                             std::to_string(ctx->arena_cap) + " bytes; " +
                                             std::to_string(need) + " needed");
  if (ctx->arena_base != 0)
    return set_error(ctx, PHB_ESTATE, "nested workspace exceeds the reserved arena");
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (ctx->capturing ||
      (hipStreamIsCapturing(ctx->stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone))
    return set_error(ctx, PHB_ESTATE, "a captured call would grow the workspace");
  hipError_t e = hipStreamSynchronize(ctx->stream);
  if (e != hipSuccess) return hip_check(ctx, e, "workspace sync");
  if (ctx->arena) hipFree(ctx->arena);
  ctx->arena = nullptr;
  ctx->arena_cap = 0;
  const size_t want = need + need / 4 + (1 << 20);
  e = hipMalloc((void**)&ctx->arena, want);
  if (e != hipSuccess) {
    ctx->arena = nullptr;
    return set_error(ctx, PHB_ENOMEM, "workspace allocation of " + std::to_string(want) +
                                          " bytes failed");
  }
  ctx->arena_cap = want;
  return PHB_OK;
}

Box make_box(const phb_params* p) {
  Box b;
  for (int a = 0; a < 3; ++a) {
    b.L[a] = p->L[a];
    b.halfL[a] = 0.5 * p->L[a];
    b.periodic[a] = p->periodic[a] ? 1 : 0;
  }
  return b;
}

int ensure_host(phb_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->host_cap) return PHB_OK;
  if (ctx->host) hipHostFree(ctx->host);
  ctx->host = nullptr;
  ctx->host_cap = 0;
  hipError_t e = hipHostMalloc((void**)&ctx->host, bytes);
  if (e != hipSuccess) return hip_check(ctx, e, "pinned host allocation");
  ctx->host_cap = bytes;
  return PHB_OK;
}

// Row lists handed in by a caller index particle arrays in the kernels: every
// entry must lie in [0, n) before any of them runs.
__global__ void k_rows_out_of_range(int m, const int32_t* __restrict__ rows, int n,
                                    int32_t* __restrict__ bad) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < m && (rows[r] < 0 || rows[r] >= n)) bad[0] = 1;
}

static int check_rows(phb_ctx* ctx, int64_t m, const int32_t* rows, int64_t n) {
  if (m <= 0) return PHB_OK;
  Workspace ws(ctx);
  ws.plan(sizeof(int32_t));
  int rc;
  if ((rc = ws.commit())) return rc;
  int32_t* bad = ws.take<int32_t>(1);
  if ((rc = hip_check(ctx, fill_i32(ctx->stream, bad, 0, 1), "row check clear"))) return rc;
  hipLaunchKernelGGL(k_rows_out_of_range, dim3(grid_for(m, 256)), dim3(256), 0, ctx->stream,
                     (int)m, rows, (int)n, bad);
  if ((rc = hip_check(ctx, hipGetLastError(), "row check"))) return rc;
  if ((rc = ensure_host(ctx, 64))) return rc;
  if ((rc = hip_check(ctx,
                      hipMemcpyAsync(ctx->host, bad, sizeof(int32_t), hipMemcpyDeviceToHost,
                                     ctx->stream),
                      "row check read-back")))
    return rc;
  if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "row check sync"))) return rc;
  if (*reinterpret_cast<int32_t*>(ctx->host))
    return set_error(ctx, PHB_EINVAL, "a row index is outside [0, n)");
  return PHB_OK;
}

int check_params(phb_ctx* ctx, const phb_params* p) {
  if (!p) return set_error(ctx, PHB_EINVAL, "params is NULL");
  for (int a = 0; a < 3; ++a)
    if (!(p->L[a] > 0.0) || !isfinite(p->L[a]))
      return set_error(ctx, PHB_EINVAL, "box length must be finite and positive");
  if (!(p->rf_ratio > 0.0) || !isfinite(p->rf_ratio))
    return set_error(ctx, PHB_EINVAL, "rf_ratio must be finite and positive");
  if (p->precision != PHB_FP64 && p->precision != PHB_MIXED)
    return set_error(ctx, PHB_EINVAL, "unknown precision");
  if (p->weight != PHB_W_POLY3 && p->weight != PHB_W_UNIT)
    return set_error(ctx, PHB_EINVAL, "unknown weight");
  if (p->fit != PHB_FIT_FULL20 && p->fit != PHB_FIT_INTERP19)
    return set_error(ctx, PHB_EINVAL, "unknown fit");
  for (double c : {p->visc_grid, p->visc_adapt, p->divb_diff})
    if (!(c >= 0.0) || !isfinite(c))
      return set_error(ctx, PHB_EINVAL, "stabiliser coefficients must be finite and >= 0");
  return PHB_OK;
}

static_assert(offsetof(phb_params, gamma) == 40 && offsetof(phb_params, visc_grid) == 72 &&
                  sizeof(phb_params) == 96,
              "phb_params layout");

Stab stab_of(const phb_params* p) {
  Stab sb;
  sb.grid = p->visc_grid;
  sb.adapt = p->visc_adapt;
  sb.divb = p->divb_diff;
  return sb;
}

int check_n(phb_ctx* ctx, int64_t n) {
  if (n <= 0 || n >= (int64_t(1) << 31) - 1)
    return set_error(ctx, PHB_EINVAL, "n must be in [1, 2^31 - 2]");
  return PHB_OK;
}

// Device-side validation of positions and lambdas; returns min/max lambda.
static constexpr int VALIDATE_BLOCKS = NB_VALIDATE_BLOCKS;
static int validate_inputs(phb_ctx* ctx, const phb_params* p, int n, const double* pos,
                           const double* lam, double* part, double* lmin, double* lmax) {
  const Box box = make_box(p);
  int rc = hip_check(ctx, launch_validate(ctx->stream, n, pos, lam, box, part, VALIDATE_BLOCKS),
                     "validate");
  if (rc) return rc;
  if ((rc = ensure_host(ctx, 3 * VALIDATE_BLOCKS * sizeof(double)))) return rc;
  rc = hip_check(ctx,
                 hipMemcpyAsync(ctx->host, part, 3 * VALIDATE_BLOCKS * sizeof(double),
                                hipMemcpyDeviceToHost, ctx->stream),
                 "validate read-back");
  if (rc) return rc;
  if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "validate sync"))) return rc;
  const double* h = reinterpret_cast<const double*>(ctx->host);
  double mn = 1e300, mx = -1e300, bad = 0.0;
  for (int b = 0; b < VALIDATE_BLOCKS; ++b) {
    mn = std::min(mn, h[3 * b]);
    mx = std::max(mx, h[3 * b + 1]);
    bad = std::max(bad, h[3 * b + 2]);
  }
  if (bad != 0.0)
    return set_error(ctx, PHB_EINVAL,
                     "a position is outside [0, L) or not finite, or a lambda is not positive");
  for (int a = 0; a < 3; ++a)
    if (p->periodic[a] && !(p->rf_ratio * mx < 0.5 * p->L[a]))
      return set_error(ctx, PHB_EINVAL, "r_f must stay below L/2 on periodic axes");
  *lmin = mn;
  *lmax = mx;
  return PHB_OK;
}

// Device words a synchronous build reads back: nnz, status, lambda range.
struct NbStat {
  int64_t nnz;
  int32_t flag, pad;
};

static void plan_neighbors(Workspace& ws, int64_t n, int64_t m, int64_t idx_capacity) {
  ws.plan(nb_work_bytes(n, m, idx_capacity));
  ws.plan(sizeof(NbStat));
}

static void plan_rhs(Workspace& ws, int64_t n, int64_t n_all, int precision, bool stab);

size_t ws_bytes_neighbors(int64_t n, int64_t idx_capacity) {
  phb_ctx dummy;
  Workspace ws(&dummy);
  plan_neighbors(ws, n, n, idx_capacity);
  return ws.total;
}

static void plan_derivs(Workspace& ws, int64_t n) {
  ws.plan((size_t)NMOM * soa_ld(n) * sizeof(double));
  ws.plan((size_t)9 * NBASIS * soa_ld(n) * sizeof(double));
  ws.plan((size_t)n * sizeof(double4));
  ws.plan((size_t)8 * n * sizeof(double));  // packed field chunk
  plan_refine(ws, n, 8);
}

size_t ws_bytes_derivs(int64_t n, const phb_params* p, bool second) {
  if (p->precision == PHB_MIXED) return mixed_derivs_bytes(n, second);
  phb_ctx dummy;
  Workspace ws(&dummy);
  plan_derivs(ws, n);
  return ws.total;
}

size_t ws_bytes_rhs(int64_t n, const phb_params* p) {
  phb_ctx dummy;
  Workspace ws(&dummy);
  plan_rhs(ws, n, n, p->precision, stab_of(p).on());
  return ws.total;
}

// n rows of n_all particles
static void plan_rhs(Workspace& ws, int64_t n, int64_t n_all, int precision, bool stab) {
  if (precision == PHB_MIXED) {  // untaped: the mixed module; taped: the data form
    phb_ctx dummy;
    Workspace wd(&dummy);
    plan_rhs(wd, n, n_all, PHB_FP64, stab);
    ws.plan(std::max(mixed_rhs_bytes(n, stab), wd.total));
    return;
  }
  ws.plan((size_t)NMOM * soa_ld(n) * sizeof(double));
  ws.plan((size_t)(stab ? 8 : 7) * NBASIS * soa_ld(n) * sizeof(double));  // B, then C
  ws.plan((size_t)n_all * sizeof(double4));
  ws.plan((size_t)n_all * 8 * sizeof(double));
  // the screened fits (7 or 8 fields; the residual sums also hold the tape's
  // 3 or 9 operator rows)
  plan_refine(ws, n, stab ? 9 : 7);
}

// The time derivatives in the form p->precision asks for.  FP64: the data
// form of the fit, C_f = A^{-1} B_f with B_f assembled from the data; the
// screened fits are refined and their outputs replace the plain solve's.
// With a tape, its AoS block receives G and C (both refined for the screened
// particles) for the reverse mode.
int eval_rhs(phb_ctx* ctx, const EvalArgs& a0, const phb_params* p, const double* q, double* rhs,
             double* dxdt, int32_t* status, double* tape) {
  const Stab sb = stab_of(p);
  // The mixed form: without a tape, FP32 assembly and its refinement (mixed
  // module).  With one, the reverse mode needs FP64 moments anyway and FP32
  // arithmetic runs no faster than FP64 here (no packed FP32), so the forward
  // is this FP64 data form; the mixed form's FP32 is then in the reverse
  // mode's pair records, half the bytes of its dominant traffic.
  if (p->precision == PHB_MIXED) {
    if (a0.rows) return set_error(ctx, PHB_ENOTIMPL, "row subsets in the mixed form");
    if (!tape) return mixed_rhs(ctx, a0, p->gamma, sb, q, rhs, dxdt, status);
  }
  EvalArgs a = a0;
  const int n = a.n;                        // rows
  const int na = a.rows ? a.n_all : n;      // particles
  const int nrows = sb.on() ? 9 : 3;
  const int nf = sb.on() ? 8 : 7;  // fields with a gradient (V, B, sigma; rho too when stabilised)
  int rc;
  Workspace ws(ctx);
  plan_rhs(ws, n, na, PHB_FP64, sb.on());
  if ((rc = ws.commit())) return rc;
  double* mom = ws.take<double>((size_t)NMOM * soa_ld(n));
  double* bc = ws.take<double>((size_t)nf * NBASIS * soa_ld(n));
  double4* geo = ws.take<double4>(na);
  double* fq = ws.take<double>((size_t)8 * na);
  const RefineBufs rb = take_refine(ws, n, sb.on() ? 9 : 7);
  double* aos = tape ? tape_aos(tape, n) : nullptr;
  a.geo = geo;
  a.fq = fq;
  { Prof pf(ctx, "k_pack");
  if ((rc = hip_check(ctx, launch_pack(ctx->stream, na, a.pos, a.lam, q, geo, fq), "pack")))
    return rc; }
  { Prof pf(ctx, nf == 8 ? "k_fit_b<8>" : "k_fit_b<7>");
  if ((rc = hip_check(ctx, launch_fit_b(ctx->stream, a, nf, ctx->fit_fields, bc), "fit right-hand sides")))
    return rc; }
  // the moments stay on chip for the factor; only the listed fits' moments
  // reach mom, for their refinement
  { Prof pf(ctx, nrows == 9 ? "k_moments_factor_fit<9>" : "k_moments_factor_fit<3>");
  if ((rc = hip_check(ctx, fill_i32(ctx->stream, rb.count, 0, 1), "clear list")) ||
      (rc = hip_check(ctx,
                      launch_moments_factor_fit(ctx->stream, a, nrows, mom, bc, aos, status,
                                                fp64_screen_cut(ctx, nrows, false), rb.list,
                                                rb.count),
                      "moments, factor and fit")))
    return rc; }
  { Prof pf(ctx, sb.on() ? "k_rows_rhs_finish<stab>" : "k_rows_rhs_finish");
  if ((rc = hip_check(ctx,
                      launch_rows_rhs_finish(ctx->stream, a, sb.on(), bc, nrows, 0, soa_ld(n),
                                             nullptr, nullptr, status, p->gamma, sb, rhs, dxdt,
                                             tape),
                      "rhs")))
    return rc; }
  // the screened fits refined on the data; their outputs (and tape records)
  // replace the plain solve's
  if ((rc = refine_fits(ctx, a, fq, sb.on() ? 0 : 1, nf, mom, rb))) return rc;
  if (aos && (rc = refine_tape(ctx, a, nrows, mom, rb, aos))) return rc;
  Prof pf(ctx, "k_rows_rhs_finish<list>");
  return hip_check(ctx,
                   launch_rows_rhs_finish(ctx->stream, a, sb.on(), rb.cbuf, NBASIS, 1, rb.ldc,
                                          rb.list, rb.count, status, p->gamma, sb, rhs, dxdt,
                                          tape),
                   "refined rhs");
}

int eval_args(phb_ctx* ctx, const phb_params* p, int64_t n64, const double* pos,
              const double* lambda, const int64_t* offsets, const int32_t* idx, EvalArgs* a) {
  int rc;
  if ((rc = check_params(ctx, p)) || (rc = check_n(ctx, n64))) return rc;
  if (!pos || !lambda || !offsets || !idx) return set_error(ctx, PHB_EINVAL, "null pointer");
  a->n = (int)n64;
  a->pos = pos;
  a->lam = lambda;
  a->off = offsets;
  a->idx = idx;
  a->box = make_box(p);
  a->rf_ratio = p->rf_ratio;
  a->wkind = p->weight;
  a->fit = p->fit;
  return PHB_OK;
}

}  // namespace phb

using namespace phb;

// ---- allocation-free variant --------------------------------------------------
// The workspace of phb_mhd_rhs_noalloc: file-scope device memory, one copy on
// every GPU the library runs on, held until the process ends.  Host code
// never passes the array's name to a kernel (on the host it stands for no
// device address): each device's address comes from hipGetSymbolAddress,
// looked up once with that device current.
static __device__ __align__(256) char scratch[PHB_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

int scratch_of(phb_ctx* ctx, char** out) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return set_error(ctx, PHB_EINVAL, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[ctx->device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) return hip_check(ctx, e, "scratch address");
    g_scratch_ptr[ctx->device] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[ctx->device];
  return PHB_OK;
}

// For the call's duration the context's workspace is the scratch (it cannot
// grow: Workspace::commit refuses), per-kernel profiling (which creates
// events) is off and no second stream is used.
struct NoAllocScope {
  phb_ctx* ctx;
  char* arena;
  size_t cap, base;
  bool prof;
  NoAllocScope(phb_ctx* c, char* sp)
      : ctx(c), arena(c->arena), cap(c->arena_cap), base(c->arena_base), prof(c->prof_on) {
    c->arena = sp;
    c->arena_cap = PHB_NOALLOC_SCRATCH_BYTES;
    c->arena_base = 0;
    c->prof_on = false;
    c->no_alloc = true;
  }
  ~NoAllocScope() {
    ctx->arena = arena;
    ctx->arena_cap = cap;
    ctx->arena_base = base;
    ctx->prof_on = prof;
    ctx->no_alloc = false;
  }
};
}  // namespace

extern "C" {

const char* phb_strerror(int code) {
  switch (code) {
    case PHB_OK: return "ok";
    case PHB_EINVAL: return "invalid argument";
    case PHB_ENOMEM: return "out of memory";
    case PHB_ECAPACITY: return "output buffer too small";
    case PHB_EHIP: return "HIP runtime error";
    case PHB_ESTATE: return "call not allowed in this state";
    case PHB_ENOTIMPL: return "not implemented";
    default: return "unknown error";
  }
}

const char* phb_last_error(phb_ctx* ctx) { return ctx ? ctx->last_error.c_str() : "no context"; }

int phb_create(phb_ctx** out, int device, void* hip_stream) {
  if (!out) return PHB_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return PHB_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return PHB_EHIP;
  phb_ctx* c = new phb_ctx();
  c->device = device;
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  // the device's address of the allocation-free entry point's scratch, looked
  // up once per device (loading the code object that holds it)
  char* sp = nullptr;
  const int rc = scratch_of(c, &sp);
  if (rc) {
    delete c;
    return rc;
  }
  *out = c;
  return PHB_OK;
}

int phb_destroy(phb_ctx* ctx) {
  if (!ctx) return PHB_EINVAL;
  hipSetDevice(ctx->device);
  hipStreamSynchronize(ctx->stream);
  if (ctx->arena) hipFree(ctx->arena);
  if (ctx->host) hipHostFree(ctx->host);
  delete ctx;
  return PHB_OK;
}

int phb_set_stream(phb_ctx* ctx, void* hip_stream) {
  if (!ctx) return PHB_EINVAL;
  ctx->stream = reinterpret_cast<hipStream_t>(hip_stream);
  return PHB_OK;
}

int phb_reserve(phb_ctx* ctx, int64_t n_max, int64_t nnz_max) {
  if (!ctx || n_max < 0 || nnz_max < 0) return PHB_EINVAL;
  // the largest workspace of the calls a capture may hold, over both
  // precisions with the stabilisers on (the larger shapes)
  phb_params p{};
  p.gamma = 5.0 / 3.0;
  p.rf_ratio = 2.3;
  p.visc_grid = p.visc_adapt = p.divb_diff = 1.0;
  size_t need = std::max(ws_bytes_neighbors(n_max, nnz_max),
                         transpose_work_bytes(n_max, nnz_max));
  for (int prec : {PHB_FP64, PHB_MIXED}) {
    p.precision = prec;
    for (int on : {0, 1}) {
      p.visc_grid = p.visc_adapt = p.divb_diff = on ? 1.0 : 0.0;
      need = std::max({need, ws_bytes_rhs(n_max, &p), ws_bytes_derivs(n_max, &p, true),
                       ws_bytes_adjoint(n_max, nnz_max, &p, true),
                       ws_bytes_adjoint(n_max, nnz_max, &p, false)});
    }
  }
  Workspace ws(ctx);
  ws.plan(need);
  return ws.commit();
}

int phb_profile(phb_ctx* ctx, int enable) {
  if (!ctx) return PHB_EINVAL;
  hipStreamSynchronize(ctx->stream);
  for (auto& r : ctx->prof_pending) {
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  ctx->prof_pending.clear();
  ctx->prof_total.clear();
  ctx->prof_on = enable != 0;
  return PHB_OK;
}

int phb_profile_read(phb_ctx* ctx, int32_t max_entries, char* names, double* total_ms,
                     int32_t* counts, int32_t* n_out) {
  if (!ctx || !n_out || max_entries < 0) return PHB_EINVAL;
  if (max_entries > 0 && (!names || !total_ms || !counts)) return PHB_EINVAL;
  int rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "profile sync");
  if (rc) return rc;
  for (auto& r : ctx->prof_pending) {
    float ms = 0.f;
    hipEventElapsedTime(&ms, r.a, r.b);
    auto& t = ctx->prof_total[r.name];
    t.first += ms;
    t.second += 1;
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  ctx->prof_pending.clear();
  int k = 0;
  for (auto& kv : ctx->prof_total) {
    if (k < max_entries) {
      strncpy(names + 64 * k, kv.first.c_str(), 63);
      names[64 * k + 63] = 0;
      total_ms[k] = kv.second.first;
      counts[k] = kv.second.second;
    }
    ++k;
  }
  *n_out = k;
  return PHB_OK;
}

static int* tune_slot(phb_ctx* ctx, const char* key) {
  if (!strcmp(key, "cells_per_rf")) return &ctx->cells_per_rf;
  if (!strcmp(key, "lanes_moments")) return &ctx->lanes_assemble;
  if (!strcmp(key, "lanes_apply")) return &ctx->lanes_apply;
  if (!strcmp(key, "lanes_adj_y")) return &ctx->lanes_adj_y;
  if (!strcmp(key, "lanes_gather")) return &ctx->lanes_gather;
  if (!strcmp(key, "mixed_cond_x10")) return &ctx->mixed_cond_x10;
  if (!strcmp(key, "mixed_refine")) return &ctx->mixed_refine;
  if (!strcmp(key, "adj_pairs_mode")) return &ctx->adj_pairs_mode;
  if (!strcmp(key, "record_order")) return &ctx->record_order;
  if (!strcmp(key, "fp64_cut_x10")) return &ctx->fp64_cut_x10;
  if (!strcmp(key, "fit_fields")) return &ctx->fit_fields;
  if (!strcmp(key, "moments_mfma")) return &ctx->moments_mfma;
  return nullptr;
}

int phb_tune_set(phb_ctx* ctx, const char* key, int value) {
  if (!ctx || !key) return PHB_EINVAL;
  int* slot = tune_slot(ctx, key);
  if (!slot) return set_error(ctx, PHB_EINVAL, std::string("unknown tuning key ") + key);
  const bool lanes = strncmp(key, "lanes_", 6) == 0;
  const bool pairs = !strcmp(key, "adj_pairs_mode");
  const bool mode = !strcmp(key, "record_order") || !strcmp(key, "moments_mfma");
  const bool cut = !strcmp(key, "mixed_cond_x10");
  const bool refine = !strcmp(key, "mixed_refine");
  const bool cut64 = !strcmp(key, "fp64_cut_x10");
  const bool fields = !strcmp(key, "fit_fields");
  if (fields ? !(value == 2 || value == 4)
      : cut64 ? !(value >= -1 && value <= 999)
      : cut ? !(value >= -1 && value <= 120)
          : refine ? !(value >= 0 && value <= 2)
          : lanes ? !(value == 1 || value == 2 || value == 4)
          : pairs ? !(value >= 0 && value <= 3)
                  : (mode ? !(value == 0 || value == 1) : !(value >= 1 && value <= 4)))
    return set_error(ctx, PHB_EINVAL, std::string("bad value for ") + key);
  *slot = value;
  return PHB_OK;
}

int phb_tune_get(phb_ctx* ctx, const char* key, int* value) {
  if (!ctx || !key || !value) return PHB_EINVAL;
  int* slot = tune_slot(ctx, key);
  if (!slot) return set_error(ctx, PHB_EINVAL, std::string("unknown tuning key ") + key);
  *value = *slot;
  return PHB_OK;
}

static_assert(TAPE_AOS == PHB_TAPE_AOS, "tape block");
int64_t phb_tape_bytes(int64_t n) {
  return tape_doubles(n) * (int64_t)sizeof(double);
}

}  // extern "C"

// Neighbor lists of all n particles (rows == nullptr) or of the m particles
// rows[0 .. m), into offsets[m + 1] and idx.  Synchronous (nnz_dev == null:
// one read-back of nnz and the status at the end, errors returned) or not
// (the status word and nnz stay on the device).
static int neighbors_build_impl(phb_ctx* ctx, const phb_params* p, int64_t n64,
                                const double* pos, const double* lambda, int64_t m64,
                                const int32_t* rows, int64_t* offsets, int32_t* idx,
                                int64_t idx_capacity, int64_t* nnz_out, bool check_rows_,
                                int64_t* nnz_dev = nullptr, int32_t* flag_dev = nullptr) {
  if (!ctx) return PHB_EINVAL;
  int rc;
  if ((rc = check_params(ctx, p)) || (rc = check_n(ctx, n64))) return rc;
  const bool sync = nnz_dev == nullptr;
  if (!pos || !lambda || !offsets || (sync ? !nnz_out : !flag_dev) || idx_capacity < 0 ||
      (idx_capacity > 0 && !idx))
    return set_error(ctx, PHB_EINVAL, "null pointer or negative capacity");
  if (rows && (m64 < 0 || m64 > n64)) return set_error(ctx, PHB_EINVAL, "bad row count");
  hipSetDevice(ctx->device);
  if (rows && check_rows_ && (rc = check_rows(ctx, m64, rows, n64))) return rc;
  const int n = (int)n64;
  const int m = rows ? (int)m64 : n;
  const Box box = make_box(p);
  Workspace ws(ctx);
  plan_neighbors(ws, n, m, idx_capacity);
  if ((rc = ws.commit())) return rc;
  const NbWork w = nb_work_take(ws, n, m, idx_capacity);
  NbStat* st = ws.take<NbStat>(1);
  int64_t* nnz_d = sync ? &st->nnz : nnz_dev;
  int32_t* flag_d = sync ? &st->flag : flag_dev;
  { Prof pf(ctx, "neighbors_build");
  if ((rc = hip_check(ctx,
                      launch_neighbor_build(ctx->stream, n, pos, lambda, box, p->rf_ratio,
                                            ctx->cells_per_rf, m, rows, w, offsets, idx,
                                            idx_capacity, nnz_d, flag_d),
                      "neighbor build")))
    return rc; }
  if (!sync) return PHB_OK;
  if ((rc = ensure_host(ctx, sizeof(NbStat)))) return rc;
  if ((rc = hip_check(ctx,
                      hipMemcpyAsync(ctx->host, st, sizeof(NbStat), hipMemcpyDeviceToHost,
                                     ctx->stream),
                      "nnz read-back")) ||
      (rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "nnz sync")))
    return rc;
  const NbStat h = *reinterpret_cast<const NbStat*>(ctx->host);
  if (h.flag & PHB_NB_INVALID)
    return set_error(ctx, PHB_EINVAL,
                     "a position is outside [0, L) or not finite, or a lambda is not positive");
  if (h.flag & PHB_NB_RADIUS)
    return set_error(ctx, PHB_EINVAL, "r_f must stay below L/2 on periodic axes");
  *nnz_out = h.nnz;
  if (h.flag & PHB_NB_OVERFLOW)
    return set_error(ctx, PHB_ECAPACITY, "idx capacity " + std::to_string(idx_capacity) +
                                             " < required " + std::to_string(h.nnz));
  return PHB_OK;
}

namespace phb {
int neighbors_rows_unchecked(phb_ctx* ctx, const phb_params* p, int64_t n, const double* pos,
                             const double* lambda, int64_t m, const int32_t* rows,
                             int64_t* offsets, int32_t* idx, int64_t idx_capacity,
                             int64_t* nnz_out) {
  return neighbors_build_impl(ctx, p, n, pos, lambda, m, rows, offsets, idx, idx_capacity,
                              nnz_out, false);
}
}  // namespace phb

extern "C" {

int phb_neighbors_build(phb_ctx* ctx, const phb_params* p, int64_t n64, const double* pos,
                        const double* lambda, int64_t* offsets, int32_t* idx,
                        int64_t idx_capacity, int64_t* nnz_out) {
  return neighbors_build_impl(ctx, p, n64, pos, lambda, n64, nullptr, offsets, idx, idx_capacity,
                              nnz_out, false);
}

int phb_neighbors_build_async(phb_ctx* ctx, const phb_params* p, int64_t n64, const double* pos,
                              const double* lambda, int64_t* offsets, int32_t* idx,
                              int64_t idx_capacity, int64_t* nnz_dev, int32_t* flag_dev) {
  if (!nnz_dev) return ctx ? set_error(ctx, PHB_EINVAL, "null nnz") : PHB_EINVAL;
  return neighbors_build_impl(ctx, p, n64, pos, lambda, n64, nullptr, offsets, idx, idx_capacity,
                              nullptr, false, nnz_dev, flag_dev);
}

int phb_neighbors_build_rows(phb_ctx* ctx, const phb_params* p, int64_t n64, const double* pos,
                             const double* lambda, int64_t m, const int32_t* rows,
                             int64_t* offsets, int32_t* idx, int64_t idx_capacity,
                             int64_t* nnz_out) {
  if (!rows) return ctx ? set_error(ctx, PHB_EINVAL, "null rows") : PHB_EINVAL;
  return neighbors_build_impl(ctx, p, n64, pos, lambda, m, rows, offsets, idx, idx_capacity,
                              nnz_out, true);
}

int phb_neighbors_transpose(phb_ctx* ctx, int64_t n64, int64_t nnz, const int64_t* offsets,
                            const int32_t* idx, int64_t* t_offsets, int32_t* t_src,
                            int32_t* t_pos) {
  if (!ctx) return PHB_EINVAL;
  int rc;
  if ((rc = check_n(ctx, n64))) return rc;
  if (nnz < 0 || !offsets || !t_offsets || (nnz > 0 && (!idx || !t_src || !t_pos)))
    return set_error(ctx, PHB_EINVAL, "null pointer or negative nnz");
  if (nnz > PHB_NNZ_MAX)
    return set_error(ctx, PHB_EINVAL, "nnz exceeds the int32 positions of the transposed lists");
  hipSetDevice(ctx->device);
  const int n = (int)n64;
  Workspace ws(ctx);
  ws.plan(transpose_work_bytes(n, nnz));
  if ((rc = ws.commit())) return rc;
  const TransposeWork w = transpose_work_take(ws, n, nnz);
  Prof pf(ctx, "neighbors_transpose");
  return hip_check(ctx,
                   launch_transpose(ctx->stream, n, offsets, idx, t_offsets, t_src, t_pos, w),
                   "transpose");
}

int phb_spatial_order(phb_ctx* ctx, const phb_params* p, int64_t n64, const double* pos,
                      const double* lambda, int32_t* perm) {
  if (!ctx) return PHB_EINVAL;
  int rc;
  if ((rc = check_params(ctx, p)) || (rc = check_n(ctx, n64))) return rc;
  if (!pos || !lambda || !perm) return set_error(ctx, PHB_EINVAL, "null pointer");
  hipSetDevice(ctx->device);
  const int n = (int)n64;
  const int64_t nbins_max = int64_t(1) << 21;  // the counting sort's bins (2^7 per axis)
  Workspace ws(ctx);
  ws.plan(3 * VALIDATE_BLOCKS * sizeof(double));
  ws.plan((size_t)n * sizeof(int32_t));
  ws.plan((size_t)(nbins_max + 1) * sizeof(int32_t));
  ws.plan((size_t)(nbins_max + 1) * sizeof(int32_t));
  ws.plan((size_t)scan_tmp_elems(nbins_max) * sizeof(int32_t));
  if ((rc = ws.commit())) return rc;
  double* part = ws.take<double>(3 * VALIDATE_BLOCKS);
  int32_t* key = ws.take<int32_t>(n);
  int32_t* bcount = ws.take<int32_t>(nbins_max + 1);
  int32_t* bstart = ws.take<int32_t>(nbins_max + 1);
  int32_t* bscan = ws.take<int32_t>(scan_tmp_elems(nbins_max));
  double lmin, lmax;
  if ((rc = validate_inputs(ctx, p, n, pos, lambda, part, &lmin, &lmax))) return rc;
  return hip_check(ctx, launch_hilbert_order(ctx->stream, n, pos, p->L, key, bcount, bstart, bscan,
                                             perm),
                   "spatial order");
}

int phb_permute(phb_ctx* ctx, int64_t n64, const int32_t* perm, int32_t ncomp, const double* src,
                double* dst) {
  if (!ctx) return PHB_EINVAL;
  int rc;
  if ((rc = check_n(ctx, n64))) return rc;
  if (!perm || !src || !dst || ncomp <= 0) return set_error(ctx, PHB_EINVAL, "bad arguments");
  hipSetDevice(ctx->device);
  return hip_check(ctx, launch_permute(ctx->stream, (int)n64, ncomp, perm, src, dst), "permute");
}


int phb_mls_derivs(phb_ctx* ctx, const phb_params* p, int64_t n64, const double* pos,
                   const double* lambda, const int64_t* offsets, const int32_t* idx, int32_t nf,
                   const double* fields, int32_t max_order, double* d1, double* d2,
                   int32_t* status) {
  if (!ctx) return PHB_EINVAL;
  EvalArgs a;
  int rc;
  if ((rc = eval_args(ctx, p, n64, pos, lambda, offsets, idx, &a))) return rc;
  if (nf <= 0 || !fields || !d1 || !status || (max_order != 1 && max_order != 2) ||
      (max_order == 2 && !d2))
    return set_error(ctx, PHB_EINVAL, "bad field arguments");
  hipSetDevice(ctx->device);
  if (p->precision == PHB_MIXED)
    return mixed_derivs(ctx, a, nf, fields, d1, max_order == 2 ? d2 : nullptr, status);
  const int n = a.n;
  const int ng = max_order == 2 ? 9 : 3;
  Workspace ws(ctx);
  plan_derivs(ws, n);
  if ((rc = ws.commit())) return rc;
  double* mom = ws.take<double>((size_t)NMOM * soa_ld(n));
  double* gop = ws.take<double>((size_t)9 * NBASIS * soa_ld(n));
  double4* geo = ws.take<double4>(n);
  double* fa = ws.take<double>((size_t)8 * n);
  const RefineBufs rb = take_refine(ws, n, 8);
  a.geo = geo;
  if ((rc = hip_check(ctx, launch_pack(ctx->stream, n, pos, lambda, nullptr, geo, nullptr),
                      "pack")))
    return rc;
  { Prof pf(ctx, "k_moments");
  if ((rc = hip_check(ctx, launch_moments(ctx->stream, a, ctx->lanes_assemble, mom), "moments")))
    return rc; }
  { Prof pf(ctx, "k_factor<9>");
  if ((rc = hip_check(ctx, fill_i32(ctx->stream, rb.count, 0, 1), "clear list")) ||
      (rc = hip_check(ctx,
                      launch_factor(ctx->stream, a, 9, mom, gop, status, ng,
                                    fp64_screen_cut(ctx, ng), rb.list, rb.count),
                      "factor")))
    return rc; }
  { Prof pf(ctx, "k_apply_derivs");
  if ((rc = hip_check(ctx,
                      launch_apply_derivs(ctx->stream, a, ctx->lanes_apply, gop, status, nf,
                                          fields, d1, max_order == 2 ? d2 : nullptr),
                      "apply derivatives")))
    return rc; }
  // the screened fits again, refined on the data, eight fields at a time
  for (int f0 = 0; f0 < nf; f0 += 8) {
    const int nfc = nf - f0 < 8 ? nf - f0 : 8;
    if ((rc = hip_check(ctx, launch_pack_chunk(ctx->stream, n, fields, f0, nfc, fa), "pack")))
      return rc;
    if ((rc = refine_fits(ctx, a, fa, 0, nfc, mom, rb))) return rc;
    if ((rc = hip_check(ctx,
                        launch_rows_derivs_finish(ctx->stream, a, ng, rb.cbuf, NBASIS, 1, rb.ldc,
                                                  rb.list, rb.count, status, nfc, f0, d1,
                                                  max_order == 2 ? d2 : nullptr),
                        "refined derivatives")))
      return rc;
  }
  return PHB_OK;
}

int phb_mhd_rhs(phb_ctx* ctx, const phb_params* p, int64_t n64, const double* pos,
                const double* lambda, const int64_t* offsets, const int32_t* idx,
                const double* q, double* rhs, double* dxdt, int32_t* status, void* tape) {
  if (!ctx) return PHB_EINVAL;
  EvalArgs a;
  int rc;
  if ((rc = eval_args(ctx, p, n64, pos, lambda, offsets, idx, &a))) return rc;
  if (!q || !rhs || !dxdt || !status) return set_error(ctx, PHB_EINVAL, "null pointer");
  hipSetDevice(ctx->device);
  return eval_rhs(ctx, a, p, q, rhs, dxdt, status, reinterpret_cast<double*>(tape));
}

int phb_mhd_rhs_noalloc(phb_ctx* ctx, const phb_params* p, int64_t n64, const double* pos,
                        const double* lambda, const int64_t* offsets, const int32_t* idx,
                        const double* q, double* rhs, double* dxdt, int32_t* status, void* tape) {
  if (!ctx) return PHB_EINVAL;
  EvalArgs a;
  int rc;
  if ((rc = eval_args(ctx, p, n64, pos, lambda, offsets, idx, &a))) return rc;
  if (!q || !rhs || !dxdt || !status) return set_error(ctx, PHB_EINVAL, "null pointer");
  if (ctx->no_alloc || ctx->arena_base != 0)
    return set_error(ctx, PHB_ESTATE, "allocation-free call inside another library call");
  const size_t need = ws_bytes_rhs(n64, p);
  if (need > PHB_NOALLOC_SCRATCH_BYTES)
    return set_error(ctx, PHB_ECAPACITY,
                     "n = " + std::to_string(n64) + " needs " + std::to_string(need) +
                         " bytes of scratch; the allocation-free call holds " +
                         std::to_string((long long)PHB_NOALLOC_SCRATCH_BYTES));
  hipSetDevice(ctx->device);
  char* sp = nullptr;
  if ((rc = scratch_of(ctx, &sp))) return rc;
  NoAllocScope scope(ctx, sp);
  return eval_rhs(ctx, a, p, q, rhs, dxdt, status, reinterpret_cast<double*>(tape));
}

int phb_mhd_rhs_rows(phb_ctx* ctx, const phb_params* p, int64_t n64, const double* pos,
                     const double* lambda, int64_t m, const int32_t* rows,
                     const int64_t* offsets, const int32_t* idx, const double* q, double* rhs,
                     double* dxdt, int32_t* status) {
  if (!ctx) return PHB_EINVAL;
  EvalArgs a;
  int rc;
  if ((rc = eval_args(ctx, p, n64, pos, lambda, offsets, idx, &a))) return rc;
  if (!rows || !q || !rhs || !dxdt || !status) return set_error(ctx, PHB_EINVAL, "null pointer");
  if (m <= 0 || m > n64) return set_error(ctx, PHB_EINVAL, "row count must be in [1, n]");
  hipSetDevice(ctx->device);
  if ((rc = check_rows(ctx, m, rows, n64))) return rc;
  a.n_all = a.n;
  a.n = (int)m;
  a.rows = rows;
  return eval_rhs(ctx, a, p, q, rhs, dxdt, status, nullptr);
}

int phb_mhd_rhs_adjoint(phb_ctx* ctx, const phb_params* p, int64_t n64, const double* pos,
                        const double* lambda, const int64_t* offsets, const int32_t* idx,
                        const int64_t* t_offsets, const int32_t* t_src, const int32_t* t_pos,
                        const double* q, const double* rhs_bar, const double* dxdt_bar,
                        double* q_bar, double* pos_bar, const void* tape) {
  if (!ctx) return PHB_EINVAL;
  EvalArgs a;
  int rc;
  if ((rc = eval_args(ctx, p, n64, pos, lambda, offsets, idx, &a))) return rc;
  if (!t_offsets || !t_src || !t_pos || !q || !rhs_bar || !q_bar || !pos_bar)
    return set_error(ctx, PHB_EINVAL, "null pointer");
  hipSetDevice(ctx->device);
  return adjoint_rhs(ctx, a, p, t_offsets, t_src, t_pos, q, rhs_bar, dxdt_bar, q_bar, pos_bar,
                     reinterpret_cast<const double*>(tape), -1);
}

int phb_mhd_rhs_adjoint_async(phb_ctx* ctx, const phb_params* p, int64_t n64, const double* pos,
                              const double* lambda, const int64_t* offsets, const int32_t* idx,
                              const int64_t* t_offsets, const int32_t* t_src,
                              const int32_t* t_pos, const double* q, const double* rhs_bar,
                              const double* dxdt_bar, double* q_bar, double* pos_bar,
                              const void* tape, int64_t nnz_bound) {
  if (!ctx) return PHB_EINVAL;
  EvalArgs a;
  int rc;
  if ((rc = eval_args(ctx, p, n64, pos, lambda, offsets, idx, &a))) return rc;
  if (!t_offsets || !t_src || !t_pos || !q || !rhs_bar || !q_bar || !pos_bar || nnz_bound < 0)
    return set_error(ctx, PHB_EINVAL, "null pointer or negative bound");
  hipSetDevice(ctx->device);
  return adjoint_rhs(ctx, a, p, t_offsets, t_src, t_pos, q, rhs_bar, dxdt_bar, q_bar, pos_bar,
                     reinterpret_cast<const double*>(tape), nnz_bound, false);
}

int phb_pc_step(phb_ctx* ctx, const phb_params* p, int64_t n64, double dt, double* pos, double* q,
                const double* lambda, int64_t* offsets, int32_t* idx, int64_t idx_capacity,
                int64_t* nnz_out, int32_t* status) {
  if (!ctx) return PHB_EINVAL;
  int rc;
  if ((rc = check_params(ctx, p)) || (rc = check_n(ctx, n64))) return rc;
  if (!pos || !q || !lambda || !offsets || !idx || !nnz_out || !status || !isfinite(dt))
    return set_error(ctx, PHB_EINVAL, "bad arguments");
  hipSetDevice(ctx->device);
  return pc_step(ctx, p, (int)n64, dt, pos, q, lambda, nullptr, offsets, idx, idx_capacity,
                 nnz_out, status, 0);
}

int phb_evolve_blocks(phb_ctx* ctx, const phb_params* p, int64_t n64, double dt_max,
                      int32_t nblocks, double cfl, int32_t kmax, double* pos, double* q,
                      const double* lambda, const int32_t* frozen, int64_t* offsets,
                      int32_t* idx, int64_t idx_capacity, int32_t* status, int32_t* level,
                      int64_t* stats) {
  if (!ctx) return PHB_EINVAL;
  int rc;
  if ((rc = check_params(ctx, p)) || (rc = check_n(ctx, n64))) return rc;
  if (!pos || !q || !lambda || !offsets || !idx || !status || !(dt_max > 0.0) ||
      !isfinite(dt_max) || nblocks < 0 || !(cfl > 0.0) || !isfinite(cfl) || kmax < 0 ||
      kmax > 30)
    return set_error(ctx, PHB_EINVAL, "bad arguments");
  if (p->precision != PHB_FP64)
    return set_error(ctx, PHB_ENOTIMPL, "individual time steps in the mixed form");
  hipSetDevice(ctx->device);
  return evolve_blocks(ctx, p, (int)n64, pos, q, lambda, frozen, dt_max, nblocks, cfl, kmax,
                       offsets, idx, idx_capacity, status, level, stats);
}

int phb_evolve(phb_ctx* ctx, const phb_params* p, int64_t n64, double dt, int32_t nsteps,
               double* pos, double* q, const double* lambda, const int32_t* frozen,
               int64_t* offsets, int32_t* idx, int64_t idx_capacity, int64_t* nnz_out,
               int32_t* status) {
  if (!ctx) return PHB_EINVAL;
  int rc;
  if ((rc = check_params(ctx, p)) || (rc = check_n(ctx, n64))) return rc;
  if (!pos || !q || !lambda || !offsets || !idx || !nnz_out || !status || !isfinite(dt) ||
      nsteps < 0)
    return set_error(ctx, PHB_EINVAL, "bad arguments");
  hipSetDevice(ctx->device);
  if (nsteps == 0) return hip_check(ctx, fill_i32(ctx->stream, status, 0, n64), "status clear");
  for (int k = 0; k < nsteps; ++k)
    if ((rc = pc_step(ctx, p, (int)n64, dt, pos, q, lambda, frozen, offsets, idx, idx_capacity,
                      nnz_out, status, k > 0)))
      return rc;
  return PHB_OK;
}

int phb_courant_dt(phb_ctx* ctx, const phb_params* p, int64_t n64, const double* q,
                   const double* lambda, const int32_t* frozen, double cfl, double* dt_out) {
  if (!ctx) return PHB_EINVAL;
  int rc;
  if ((rc = check_params(ctx, p)) || (rc = check_n(ctx, n64))) return rc;
  if (!q || !lambda || !dt_out || !(cfl > 0.0) || !isfinite(cfl))
    return set_error(ctx, PHB_EINVAL, "bad arguments");
  hipSetDevice(ctx->device);
  return courant_dt(ctx, p, (int)n64, q, lambda, frozen, cfl, dt_out);
}

}  // extern "C"
