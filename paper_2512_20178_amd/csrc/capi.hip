// C ABI of the per-rank path: argument validation, plan lifecycle, tuning,
// autotuner and HIP graph capture.  Kernels live in select/sort/spmm.hip.
#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <unordered_map>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "mvc.hpp"
#include "plan.hpp"

namespace shiro {

static thread_local std::string g_last_error;

// A roctx range around one call of the path (host side: it brackets the
// enqueue of the call's kernels; visible with rocprofv3 --marker-trace).
struct TraceRange {
  explicit TraceRange(const char* name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange&) = delete;
  TraceRange& operator=(const TraceRange&) = delete;
};

int set_error(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

// Device memory of plans and tuning buffers: hipMalloc, or the caller's
// allocator after shiro_set_allocator.  Every block remembers the allocator
// that made it, so it is returned to that one even if the hook changes.
namespace {
struct Allocator {
  shiro_alloc_fn alloc = nullptr;
  shiro_free_fn free = nullptr;
  void* ctx = nullptr;
};
struct Block {
  Allocator by;
  int64_t bytes;
};
std::mutex g_alloc_mu;
Allocator g_alloc;
std::unordered_map<void*, Block> g_blocks;
}  // namespace

int set_allocator(shiro_alloc_fn alloc, shiro_free_fn free, void* ctx) {
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_alloc = Allocator{alloc, free, ctx};
  return SHIRO_OK;
}

int dev_alloc(void** p, int64_t bytes) {
  *p = nullptr;
  if (bytes <= 0) bytes = 1;
  Allocator a;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    a = g_alloc;
  }
  if (a.alloc) {
    *p = a.alloc((size_t)bytes, a.ctx);
    if (!*p)
      return set_error(SHIRO_ERR_OOM, "device allocation of " + std::to_string(bytes) +
                                          " bytes failed (caller's allocator returned NULL)");
    if ((uintptr_t)*p % 256 != 0) {
      a.free(*p, (size_t)bytes, a.ctx);
      *p = nullptr;
      return set_error(SHIRO_ERR_UNSUPPORTED, "caller's allocator returned memory not aligned to 256 bytes");
    }
  } else {
    hipError_t e = hipMalloc(p, (size_t)bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      *p = nullptr;
      return set_error(e == hipErrorOutOfMemory ? SHIRO_ERR_OOM : SHIRO_ERR_HIP,
                       "device allocation of " + std::to_string(bytes) + " bytes failed: " +
                           hipGetErrorString(e));
    }
  }
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_blocks[*p] = Block{a, bytes};
  return SHIRO_OK;
}

void dev_free(void* p) {
  if (!p) return;
  Block b{};
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    auto it = g_blocks.find(p);
    if (it != g_blocks.end()) {
      b = it->second;
      g_blocks.erase(it);
    }
  }
  if (b.by.free) {
    // a caller's allocator may hand the block out again at once (hipFree
    // would wait for the device), so nothing of ours may still be using it
    (void)hipDeviceSynchronize();
    b.by.free(p, (size_t)b.bytes, b.by.ctx);
  } else {
    (void)hipFree(p);
  }
}

bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &st) != hipSuccess) return false;
  return st == hipStreamCaptureStatusActive;
}

void retire_buffer(shiro_plan plan, void* p) {
  if (!p) return;
  if (plan->graphs.empty()) dev_free(p);
  else plan->retired.push_back(p);
}

int ensure_scratch(shiro_plan plan, int64_t bytes) {
  if (plan->scratch_bytes >= bytes) return SHIRO_OK;
  SHIRO_HIP(hipDeviceSynchronize());  // earlier setup kernels may still use it
  retire_buffer(plan, plan->scratch);
  plan->scratch = nullptr;
  plan->scratch_bytes = 0;
  SHIRO_TRY(dev_alloc(&plan->scratch, bytes));
  plan->scratch_bytes = bytes;
  return SHIRO_OK;
}

int ensure_rows_work(shiro_plan plan, int32_t chunk, bool allocate, hipStream_t s,
                     const WorkList** out) {
  auto it = plan->rows_work.find(chunk);
  if (it == plan->rows_work.end()) {
    if (!allocate)
      return set_error(SHIRO_ERR_CAPTURING,
                       "work list for chunk " + std::to_string(chunk) + " not prepared before capture");
    WorkList wl;
    SHIRO_TRY(build_worklist(plan->row_ptr, plan->rows, plan->nnz, chunk, &wl, s));
    it = plan->rows_work.emplace(chunk, wl).first;
  }
  *out = &it->second;
  return SHIRO_OK;
}

int ensure_rb_work(shiro_plan plan, int which, int32_t chunk, bool allocate, hipStream_t s,
                   const WorkList** out) {
  auto& m = which == 0 ? plan->rb_work : plan->agg_work;
  auto it = m.find(chunk);
  if (it == m.end()) {
    if (!allocate)
      return set_error(SHIRO_ERR_CAPTURING,
                       "row-based work list for chunk " + std::to_string(chunk) + " not prepared before capture");
    WorkList wl;
    if (which == 0) SHIRO_TRY(build_worklist(plan->rb.ptr, plan->rb.R, plan->nnz, chunk, &wl, s));
    else SHIRO_TRY(build_worklist(plan->rb.agg_ptr, plan->rows, plan->rb.R, chunk, &wl, s));
    it = m.emplace(chunk, wl).first;
  }
  *out = &it->second;
  return SHIRO_OK;
}

int ensure_cols_work(shiro_plan plan, int32_t chunk, bool allocate, hipStream_t s,
                     const WorkList** out) {
  auto it = plan->cols_work.find(chunk);
  if (it == plan->cols_work.end()) {
    if (!allocate)
      return set_error(SHIRO_ERR_CAPTURING,
                       "transposed work list for chunk " + std::to_string(chunk) + " not prepared before capture");
    WorkList wl;
    SHIRO_TRY(build_worklist(plan->tr.ptr, plan->U, plan->nnz, chunk, &wl, s));
    it = plan->cols_work.emplace(chunk, wl).first;
  }
  *out = &it->second;
  return SHIRO_OK;
}

int ensure_carry(shiro_plan plan, int64_t elems, bool allocate) {
  if (plan->carry_elems >= elems) return SHIRO_OK;
  if (!allocate) return set_error(SHIRO_ERR_CAPTURING, "carry buffer not prepared before capture");
  SHIRO_HIP(hipDeviceSynchronize());
  retire_buffer(plan, plan->carry);
  plan->carry = nullptr;
  plan->carry_elems = 0;
  SHIRO_TRY(dev_alloc_n(&plan->carry, elems));
  plan->carry_elems = elems;
  return SHIRO_OK;
}

int ensure_acc32(shiro_plan plan, int64_t elems, bool allocate) {
  if (plan->acc32_elems >= elems) return SHIRO_OK;
  if (!allocate) return set_error(SHIRO_ERR_CAPTURING, "per-block accumulator not prepared before capture");
  SHIRO_HIP(hipDeviceSynchronize());
  retire_buffer(plan, plan->acc32);
  plan->acc32 = nullptr;
  plan->acc32_elems = 0;
  SHIRO_TRY(dev_alloc_n(&plan->acc32, elems));
  plan->acc32_elems = elems;
  return SHIRO_OK;
}

int ensure_tvals(shiro_plan plan, bool allocate) {
  if (plan->tvals_elems >= plan->nnz && plan->tvals) return SHIRO_OK;
  if (!allocate) return set_error(SHIRO_ERR_CAPTURING, "transposed values buffer not prepared before capture");
  SHIRO_TRY(dev_alloc_n(&plan->tvals, std::max<int64_t>(plan->nnz, 1)));
  SHIRO_TRY(dev_alloc_n(&plan->tdvals, std::max<int64_t>(plan->nnz, 1)));
  plan->tvals_elems = plan->nnz;
  return SHIRO_OK;
}

// Defaults from sweeps on MI355X (panel of a 2^24 R-MAT, N = 128): the
// nonzero walk with four nonzeros in flight per lane group and chunks of 256
// merge-path items for every kernel that has it; the sampled product keeps
// its wavefront-per-row kernel with two in flight.
shiro_tuning_t default_tuning(int kernel, int32_t, shiro_dtype) {
  const bool walk = kernel != SHIRO_KERNEL_SDDMM;
  shiro_tuning_t t;
  t.chunk = walk ? 256 : 128;
  t.lanes = 64;
  t.unroll = walk ? 4 : 2;
  t.group_rows = walk ? 2 : 0;
  t.xcd_remap = 0;
  t.wg_per_cu = walk ? 16 : 8;
  t.lds_rows = 0;
  return t;
}

int validate_tuning(int kernel, int32_t N, shiro_dtype dt, const shiro_tuning_t& t) {
  if (kernel < 0 || kernel > SHIRO_KERNEL_AGGREGATE_C)
    return set_error(SHIRO_ERR_INVALID_ARG, "tuning: unknown kernel family");
  if (t.chunk < 16 || t.chunk > (1 << 22)) return set_error(SHIRO_ERR_INVALID_ARG, "tuning: chunk outside [16, 2^22]");
  if (t.lanes != 8 && t.lanes != 16 && t.lanes != 32 && t.lanes != 64)
    return set_error(SHIRO_ERR_INVALID_ARG, "tuning: lanes must be 8, 16, 32 or 64");
  if (t.unroll != 1 && t.unroll != 2 && t.unroll != 4)
    return set_error(SHIRO_ERR_INVALID_ARG, "tuning: unroll must be 1, 2 or 4");
  if (t.group_rows < 0 || t.group_rows > 3) return set_error(SHIRO_ERR_INVALID_ARG, "tuning: group_rows must be 0, 1, 2 or 3");
  if (t.group_rows >= 2 && kernel == SHIRO_KERNEL_SDDMM)
    return set_error(SHIRO_ERR_INVALID_ARG, "tuning: the sampled product has no nonzero walk (group_rows 0 or 1)");
  if (t.xcd_remap != 0 && t.xcd_remap != 1) return set_error(SHIRO_ERR_INVALID_ARG, "tuning: xcd_remap must be 0 or 1");
  if (t.wg_per_cu < 1 || t.wg_per_cu > 32) return set_error(SHIRO_ERR_INVALID_ARG, "tuning: wg_per_cu outside [1, 32]");
  if (t.lds_rows < 0 || t.lds_rows > 128) return set_error(SHIRO_ERR_INVALID_ARG, "tuning: lds_rows outside [0, 128]");
  if (t.lds_rows > 0 && (t.group_rows != 3 || (kernel != SHIRO_KERNEL_SPMM && kernel != SHIRO_KERNEL_SPMM_T)))
    return set_error(SHIRO_ERR_INVALID_ARG, "tuning: lds_rows needs the windowed walk (group_rows 3) of spmm or spmm_t");
  if (t.lds_rows > 0 && N > 0) {
    // one workgroup holds lds_rows rows of its column tile; the fused
    // backward runs one tile of up to 64 lanes whatever t.lanes says
    const int vec16 = dt == SHIRO_F32 ? 4 : 8;
    const int vec = (N % vec16 == 0) ? vec16 : 1;
    const int64_t need = ceil_div((int64_t)N, (int64_t)vec);  // lanes a tile needs, as the launch sizes it
    int lanes = kernel == SHIRO_KERNEL_SPMM_T ? 64 : t.lanes;
    while (lanes > 8 && lanes / 2 >= need) lanes /= 2;
    const int64_t bytes = (int64_t)t.lds_rows * lanes * vec * (dt == SHIRO_F32 ? 4 : 2);
    if (bytes > 65536)
      return set_error(SHIRO_ERR_INVALID_ARG, "tuning: lds_rows rows of this width exceed 64 KB of LDS");
  }
  return SHIRO_OK;
}

shiro_tuning_t tuning_for(shiro_plan plan, int kernel, int32_t N, shiro_dtype dt) {
  auto it = plan->tuning.find(TuneKey{kernel, N, (int)dt});
  if (it != plan->tuning.end()) return it->second;
  return default_tuning(kernel, N, dt);
}

static bool env_check() {
  const char* e = std::getenv("SHIRO_CHECK");
  return e && e[0] == '1';
}

static bool valid_dt(shiro_dtype dt) { return dt == SHIRO_F32 || dt == SHIRO_BF16; }
static int64_t dt_size(shiro_dtype dt) { return dt == SHIRO_F32 ? 4 : 2; }

static void plan_free(shiro_plan plan) {
  if (!plan) return;
  (void)hipDeviceSynchronize();
  for (auto& g : plan->graphs)
    if (g) (void)hipGraphExecDestroy(g);
  dev_free(plan->row_ptr);
  dev_free(plan->col);
  dev_free(plan->vmap);
  dev_free(plan->svals);
  dev_free(plan->bits);
  dev_free(plan->bcol);
  dev_free(plan->mark_items);
  dev_free(plan->wtab);
  dev_free(plan->unique_cols);
  dev_free(plan->block_off);
  dev_free(plan->colmap);
  for (auto* m : {&plan->rows_work, &plan->cols_work, &plan->rb_work, &plan->agg_work})
    for (auto& kv : *m) {
      dev_free(kv.second.chunk_row);
      dev_free(kv.second.chunk_nz);
      dev_free(kv.second.split);
    }
  dev_free(plan->tvals);
  dev_free(plan->tdvals);
  dev_free(plan->tr.ptr);
  dev_free(plan->tr.row);
  dev_free(plan->tr.perm);
  dev_free(plan->tr.rid);
  dev_free(plan->seg.seg_row);
  dev_free(plan->seg.seg_begin);
  dev_free(plan->seg.seg_end);
  dev_free(plan->seg.seg_csr);
  dev_free(plan->rb.ptr);
  dev_free(plan->rb.col);
  dev_free(plan->rb.perm);
  dev_free(plan->rb.rid);
  dev_free(plan->rb.agg_rid);
  dev_free(plan->row_rid);
  dev_free(plan->rb.agg_ptr);
  dev_free(plan->rb.agg_idx);
  dev_free(plan->rb.ones);
  dev_free(plan->rb.iota);
  dev_free(plan->rb.vals);
  dev_free(plan->rb.block_off);
  for (auto& kv : plan->hot) {
    dev_free(kv.second.walk_idx);
    dev_free(kv.second.hot_src);
  }
  dev_free(plan->pb.ptr);
  dev_free(plan->pb.idx);
  dev_free(plan->pb.rid);
  for (auto& wl : plan->pb.work) {
    dev_free(wl.chunk_row);
    dev_free(wl.chunk_nz);
    dev_free(wl.split);
  }
  dev_free(plan->carry);
  dev_free(plan->acc32);
  dev_free(plan->scratch);
  for (void* p : plan->retired) dev_free(p);
  if (plan->h_pinned) (void)hipHostFree(plan->h_pinned);
  delete plan;
}

// ---------------------------------------------------------------------------
// autotuner
// ---------------------------------------------------------------------------
struct TuneBuffers {
  void* Bp = nullptr;
  void* Y = nullptr;
  void* dY = nullptr;
  void* dBp = nullptr;
  void* dB = nullptr;
  void* Cp = nullptr;
  float* vals = nullptr;
  float* dvals = nullptr;
  ~TuneBuffers() {
    dev_free(Bp);
    dev_free(Y);
    dev_free(dY);
    dev_free(dBp);
    dev_free(dB);
    dev_free(Cp);
    dev_free(vals);
    dev_free(dvals);
  }
};

static std::string tune_key(shiro_plan plan, int kernel, int32_t N, shiro_dtype dt) {
  hipDeviceProp_t prop;
  std::string name = "gpu";
  if (hipGetDeviceProperties(&prop, plan->device) == hipSuccess) name = prop.gcnArchName;
  for (auto& ch : name)
    if (ch == ' ' || ch == ':') ch = '_';
  std::ostringstream os;
  os << name << "|rows=" << plan->rows << "|nnz=" << plan->nnz << "|U=" << plan->U
     << "|P=" << plan->P << "|N=" << N << "|dt=" << (int)dt << "|k=" << kernel;
  return os.str();
}

static bool cache_lookup(const std::string& key, shiro_tuning_t* t) {
  const char* path = std::getenv("SHIRO_TUNE_CACHE");
  if (!path || !*path) return false;
  std::ifstream f(path);
  std::string line;
  bool found = false;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::string k;
    shiro_tuning_t c;
    if (is >> k >> c.chunk >> c.lanes >> c.unroll >> c.group_rows >> c.xcd_remap >> c.wg_per_cu) {
      if (!(is >> c.lds_rows)) c.lds_rows = 0;  // lines written before the knob existed
      if (k == key) {
        *t = c;
        found = true;  // last entry wins
      }
    }
  }
  return found;
}

static void cache_store(const std::string& key, const shiro_tuning_t& t) {
  const char* path = std::getenv("SHIRO_TUNE_CACHE");
  if (!path || !*path) return;
  std::ofstream f(path, std::ios::app);
  f << key << ' ' << t.chunk << ' ' << t.lanes << ' ' << t.unroll << ' ' << t.group_rows << ' '
    << t.xcd_remap << ' ' << t.wg_per_cu << ' ' << t.lds_rows << '\n';
}

// Median of 9 timed runs after one warm-up (the warm-up also builds any
// work list the candidate needs).
template <class F>
static int time_candidate(hipStream_t s, F&& run, float* ms_out) {
  constexpr int kReps = 9;
  hipEvent_t ev[kReps + 1];
  for (auto& e : ev) SHIRO_HIP(hipEventCreate(&e));
  int rc = run();
  if (rc == SHIRO_OK) {
    (void)hipEventRecord(ev[0], s);
    for (int rep = 0; rep < kReps && rc == SHIRO_OK; ++rep) {
      rc = run();
      (void)hipEventRecord(ev[rep + 1], s);
    }
    (void)hipEventSynchronize(ev[kReps]);
  }
  float t[kReps];
  for (int rep = 0; rep < kReps; ++rep) {
    t[rep] = 0.f;
    (void)hipEventElapsedTime(&t[rep], ev[rep], ev[rep + 1]);
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  std::sort(t, t + kReps);
  *ms_out = t[kReps / 2];
  return rc;
}

// Chunk size at which a persistent grid of wg_per_cu workgroups per CU gives
// each of its workers m chunks: merge items / (CUs * wg_per_cu * workers per
// workgroup * m).  Workers are wavefronts, or lane groups for the nonzero
// walk; the lanes a lane group uses follow from N as in the launch (the
// fused backward always asks for one tile).  0 when the items are unknown.
static int fit_chunk(shiro_plan plan, int kernel, int32_t N, shiro_dtype dt, const shiro_tuning_t& t, int m) {
  int64_t items;
  if (kernel == SHIRO_KERNEL_SPMM || kernel == SHIRO_KERNEL_SDDMM) items = plan->rows + plan->nnz;
  else if (kernel == SHIRO_KERNEL_SPMM_T) items = plan->U + plan->nnz;
  else if (!plan->rb.built) return 0;
  else if (kernel == SHIRO_KERNEL_PARTIAL_C) items = plan->rb.R + plan->nnz;
  else items = plan->rows + plan->rb.R;
  const int vec16 = dt == SHIRO_F32 ? 4 : 8;
  const int vec = (N % vec16 == 0) ? vec16 : 1;
  int lanes = kernel == SHIRO_KERNEL_SPMM_T ? 64 : t.lanes;
  const int64_t need = ceil_div((int64_t)N, (int64_t)vec);
  while (lanes > 8 && lanes / 2 >= need) lanes /= 2;
  const int64_t wpb = kWavesPerBlock * (t.group_rows >= 2 ? kWave / lanes : 1);
  const int64_t workers = (int64_t)plan->num_cus * t.wg_per_cu * wpb * m;
  const int64_t c = ceil_div(items, workers);
  return (int)std::min<int64_t>(std::max<int64_t>(c, 16), 1 << 22);
}

static int tune_one(shiro_plan plan, int kernel, int32_t N, shiro_dtype dt, TuneBuffers& b,
                    hipStream_t s) {
  const std::string key = tune_key(plan, kernel, N, dt);
  shiro_tuning_t cached;
  if (cache_lookup(key, &cached) && validate_tuning(kernel, N, dt, cached) == SHIRO_OK) {
    plan->tuning[TuneKey{kernel, N, (int)dt}] = cached;
    return SHIRO_OK;
  }
  auto run = [&](const shiro_tuning_t& t) -> int {
    if (kernel == SHIRO_KERNEL_SPMM)
      return launch_spmm(plan, t, b.vals, b.Bp, N, N, dt, b.Y, N, dt == SHIRO_F32 ? SHIRO_F32 : SHIRO_BF16, s);
    if (kernel == SHIRO_KERNEL_SPMM_T)  // the form autograd uses: dB rows overwritten, and dvals
      return launch_spmm_t(plan, t, b.vals, b.dY, N, N, dt, nullptr, 0, b.dB, N, true, b.Bp, N,
                           b.dvals, nullptr, s);
    if (kernel == SHIRO_KERNEL_PARTIAL_C)  // scratch B of n_cols x N
      return launch_partial_c(plan, t, b.vals, b.dB, N, N, dt, b.Cp, N, dt, s);
    if (kernel == SHIRO_KERNEL_AGGREGATE_C)
      return launch_aggregate_c(plan, t, b.Cp, N, N, dt, b.Y, N, dt, false, s);
    return launch_sddmm(plan, t, b.vals, b.dY, N, b.Bp, N, N, dt, b.dvals, s);
  };
  shiro_tuning_t best = default_tuning(kernel, N, dt);
  float best_ms = 1e30f;
  auto consider = [&](shiro_tuning_t t, float* ms_out = nullptr) -> int {
    float ms;
    int rc = time_candidate(s, [&] { return run(t); }, &ms);
    if (rc != SHIRO_OK) return rc;
    if (ms_out) *ms_out = ms;
    if (ms < best_ms) {
      best_ms = ms;
      best = t;
    }
    return SHIRO_OK;
  };
  // stage 1: work size and depth
  for (int chunk : {128, 256, 512, 1024, 2048})
    for (int unroll : {1, 2, 4}) {
      shiro_tuning_t t = default_tuning(kernel, N, dt);
      t.chunk = chunk;
      t.unroll = unroll;
      SHIRO_TRY(consider(t));
    }
  // stage 2: kernel form, lane width, occupancy, XCD placement around the
  // best; the best candidate of each kernel form is kept
  const shiro_tuning_t base = best;
  const bool walk = kernel != SHIRO_KERNEL_SDDMM;
  const int n_forms = walk ? 4 : 2;
  float form_ms[4] = {1e30f, 1e30f, 1e30f, 1e30f};
  shiro_tuning_t form_best[4] = {base, base, base, base};
  for (int grp = 0; grp < n_forms; ++grp)
    for (int lanes : {64, 32, 16})
      for (int wg : {2, 4, 8, 16})
        for (int xcd : {0, 1}) {
          shiro_tuning_t t = base;
          t.group_rows = grp;
          t.lanes = lanes;
          t.wg_per_cu = wg;
          t.xcd_remap = xcd;
          float ms = 1e30f;
          SHIRO_TRY(consider(t, &ms));
          if (ms < form_ms[grp]) {
            form_ms[grp] = ms;
            form_best[grp] = t;
          }
        }
  // stages 3 and 4 refine the two fastest kernel forms separately (a form
  // that loses at the first stage's depth can win at another one)
  int forms[4] = {0, 1, 2, 3};
  std::sort(forms, forms + n_forms, [&](int a, int b) { return form_ms[a] < form_ms[b]; });
  for (int f = 0; f < std::min(n_forms, 2); ++f) {
    if (form_ms[forms[f]] >= 1e30f) continue;
    shiro_tuning_t local = form_best[forms[f]];
    float local_ms = form_ms[forms[f]];
    auto refine = [&](const shiro_tuning_t& t) -> int {
      float ms = 1e30f;
      SHIRO_TRY(consider(t, &ms));
      if (ms < local_ms) {
        local_ms = ms;
        local = t;
      }
      return SHIRO_OK;
    };
    // stage 3: work size and depth again around the form's best layout, plus
    // the chunk sizes that give every worker of a full persistent grid
    // exactly one or two chunks (no tail round)
    const shiro_tuning_t base3 = local;
    std::vector<int> chunks{64, 128, 256, 512};
    for (int m : {1, 2}) {
      const int fit = fit_chunk(plan, kernel, N, dt, base3, m);
      if (fit > 0 && std::find(chunks.begin(), chunks.end(), fit) == chunks.end()) chunks.push_back(fit);
    }
    for (int chunk : chunks)
      for (int unroll : {1, 2, 4}) {
        shiro_tuning_t t = base3;
        t.chunk = chunk;
        t.unroll = unroll;
        SHIRO_TRY(refine(t));
      }
    // stage 4: occupancy and fitted chunk together around the form's best
    const shiro_tuning_t base4 = local;
    for (int wg : {2, 4, 8, 16})
      for (int m : {1, 2, 3}) {
        shiro_tuning_t t = base4;
        t.wg_per_cu = wg;
        t.chunk = fit_chunk(plan, kernel, N, dt, t, m);
        if (t.chunk > 0) SHIRO_TRY(refine(t));
      }
  }
  // stage 5: the most referenced rows of the gathered operand in LDS
  // (windowed walk of spmm and spmm_t); rows of at most 1 KB, so 64 fit
  if (best.group_rows == 3 && (kernel == SHIRO_KERNEL_SPMM || kernel == SHIRO_KERNEL_SPMM_T)) {
    const shiro_tuning_t base5 = best;
    for (int H : {16, 32, 64}) {
      shiro_tuning_t t = base5;
      t.lds_rows = H;
      SHIRO_TRY(consider(t));
    }
  }
  plan->tuning[TuneKey{kernel, N, (int)dt}] = best;
  cache_store(key, best);
  return SHIRO_OK;
}

}  // namespace shiro

using namespace shiro;

// ===========================================================================
// exported functions
// ===========================================================================
extern "C" {

SHIRO_API int shiro_version(void) { return 10000; }

SHIRO_API const char* shiro_last_error(void) { return g_last_error.c_str(); }

static int partition_impl(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t* d_row_ptr,
                          const int32_t* d_col, const uint8_t* d_keep, uint8_t keep_val, int32_t P, int32_t p,
                          uint32_t flags, shiro_stream_t stream, shiro_plan* out_plan) {
  if (!out_plan) return set_error(SHIRO_ERR_INVALID_ARG, "partition: out_plan is NULL");
  *out_plan = nullptr;
  if (n_rows < 1 || n_cols < 1 || n_rows >= (1ll << 31) || n_cols >= (1ll << 31))
    return set_error(SHIRO_ERR_INVALID_ARG, "partition: n_rows and n_cols must be in [1, 2^31)");
  if (nnz < 0) return set_error(SHIRO_ERR_INVALID_ARG, "partition: nnz < 0");
  if (!d_row_ptr) return set_error(SHIRO_ERR_INVALID_ARG, "partition: d_row_ptr is NULL");
  if (nnz > 0 && !d_col) return set_error(SHIRO_ERR_INVALID_ARG, "partition: d_col is NULL");
  if (P < 1) return set_error(SHIRO_ERR_INVALID_ARG, "partition: P < 1");
  if (p < 0 || p >= P) return set_error(SHIRO_ERR_INVALID_ARG, "partition: p outside [0, P)");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (stream_capturing(s)) return set_error(SHIRO_ERR_CAPTURING, "partition: stream is capturing");

  auto* plan = new shiro_plan_s();
  auto fail = [&](int rc) {
    plan_free(plan);
    return rc;
  };
  if (hipGetDevice(&plan->device) != hipSuccess) return fail(set_error(SHIRO_ERR_HIP, "hipGetDevice failed"));
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, plan->device) == hipSuccess && prop.multiProcessorCount > 0)
    plan->num_cus = prop.multiProcessorCount;
  plan->n_rows = n_rows;
  plan->n_cols = n_cols;
  plan->P = P;
  plan->p = p;
  plan->M = ceil_div(n_rows, P);
  plan->K = ceil_div(n_cols, P);
  plan->row_begin = std::min<int64_t>((int64_t)p * plan->M, n_rows);
  const int64_t row_end = std::min<int64_t>(plan->row_begin + plan->M, n_rows);
  plan->rows = row_end - plan->row_begin;

  if (hipHostMalloc((void**)&plan->h_pinned, (size_t)(P + 2) * 8, hipHostMallocDefault) != hipSuccess)
    return fail(set_error(SHIRO_ERR_OOM, "partition: pinned host allocation failed"));
  // panel nonzero range
  if (hipMemcpyAsync(plan->h_pinned, d_row_ptr + plan->row_begin, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(plan->h_pinned + 1, d_row_ptr + row_end, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail(set_error(SHIRO_ERR_HIP, "partition: reading row_ptr failed"));
  const int64_t nz0 = plan->h_pinned[0], nz1 = plan->h_pinned[1];
  if (nz0 < 0 || nz1 < nz0 || nz1 > nnz)
    return fail(set_error(SHIRO_ERR_BAD_CSR, "partition: row_ptr of the panel is not within [0, nnz] or decreases"));
  if (nz1 - nz0 >= (1ll << 31) - 1)
    return fail(set_error(SHIRO_ERR_UNSUPPORTED, "partition: panel has 2^31 or more nonzeros"));
  plan->nz_begin = nz0;
  plan->nnz = nz1 - nz0;
  plan->src_nnz = plan->nnz;
  plan->n_words = ceil_div(n_cols, 32);

  int rc;
  if (d_keep) {
    // keep the panel nonzeros k with d_keep[k] == keep_val, in CSR order
    const int64_t n = plan->nnz;
    if ((rc = ensure_scratch(plan, (n + 1) * 8 + 256 + scan_scratch_bytes(std::max<int64_t>(n, 1))))) return fail(rc);
    int64_t* pos = reinterpret_cast<int64_t*>(plan->scratch);
    void* scan_tmp = reinterpret_cast<char*>(plan->scratch) + ((n + 1) * 8 + 255) / 256 * 256;
    int32_t* col_tmp = nullptr;
    if ((rc = dev_alloc_n(&col_tmp, std::max<int64_t>(n, 1))) ||
        (rc = dev_alloc_n(&plan->vmap, std::max<int64_t>(n, 1))) ||
        (rc = dev_alloc_n(&plan->row_ptr, plan->rows + 1))) {
      dev_free(col_tmp);
      return fail(rc);
    }
    rc = launch_subset(d_row_ptr + plan->row_begin, plan->rows, nz0, n, d_col + nz0, d_keep, keep_val, pos,
                       col_tmp, plan->vmap, plan->row_ptr, scan_tmp, s);
    if (rc == SHIRO_OK &&
        (hipMemcpyAsync(plan->h_pinned, pos + n, 8, hipMemcpyDeviceToHost, s) != hipSuccess ||
         hipStreamSynchronize(s) != hipSuccess))
      rc = set_error(SHIRO_ERR_HIP, "partition_subset: counting the kept nonzeros failed");
    if (rc != SHIRO_OK) {
      dev_free(col_tmp);
      return fail(rc);
    }
    plan->nnz = plan->h_pinned[0];
    plan->col = col_tmp;  // first n entries hold the kept columns
    if ((rc = dev_alloc_n(&plan->svals, std::max<int64_t>(plan->nnz, 1)))) return fail(rc);
  }
  if ((!d_keep && ((rc = dev_alloc_n(&plan->row_ptr, plan->rows + 1)) ||
                   (rc = dev_alloc_n(&plan->col, std::max<int64_t>(plan->nnz, 1))))) ||
      (rc = dev_alloc_n(&plan->bits, plan->n_words)) ||
      (rc = dev_alloc_n(&plan->wtab, 2 * plan->n_words)) ||
      (rc = dev_alloc_n(&plan->unique_cols, std::max<int64_t>(std::min(plan->nnz, n_cols), 1))) ||
      (rc = dev_alloc_n(&plan->block_off, (int64_t)P + 1)) ||
      (rc = dev_alloc_n(&plan->colmap, std::max<int64_t>(plan->nnz, 1))))
    return fail(rc);
  if (!d_keep) {
    if ((rc = launch_rebase_row_ptr(d_row_ptr + plan->row_begin, plan->rows, plan->row_ptr, s))) return fail(rc);
    if (plan->nnz > 0 &&
        hipMemcpyAsync(plan->col, d_col + nz0, (size_t)plan->nnz * 4, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return fail(set_error(SHIRO_ERR_HIP, "partition: copying the panel's columns failed"));
  }
  // the selection expects an all-zero bitmap (each selection clears what it set)
  if ((rc = launch_zero_bytes(reinterpret_cast<uint8_t*>(plan->bits), plan->n_words * 4, s))) return fail(rc);

  if ((flags & SHIRO_CHECK_CSR) || env_check()) {
    if ((rc = ensure_scratch(plan, 256))) return fail(rc);
    int32_t* d_flag = reinterpret_cast<int32_t*>(plan->scratch);
    if (hipMemsetAsync(d_flag, 0, 4, s) != hipSuccess) return fail(set_error(SHIRO_ERR_HIP, "check: memset failed"));
    if ((rc = launch_check_csr(plan->row_ptr, plan->col, plan->rows, plan->nnz, n_cols, d_flag, s)))
      return fail(rc);
    int32_t* h_flag = reinterpret_cast<int32_t*>(plan->h_pinned);
    if (hipMemcpyAsync(h_flag, d_flag, 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail(set_error(SHIRO_ERR_HIP, "check: reading the flag failed"));
    if (*h_flag) {
      std::string why;
      if (*h_flag & 1) why += " row_ptr decreases;";
      if (*h_flag & 2) why += " column id outside [0, n_cols);";
      if (*h_flag & 4) why += " columns not strictly ascending inside a row;";
      return fail(set_error(SHIRO_ERR_BAD_CSR, "partition: malformed CSR:" + why));
    }
  }
  if (hipStreamSynchronize(s) != hipSuccess) return fail(set_error(SHIRO_ERR_HIP, "partition: stream failed"));
  *out_plan = plan;
  return SHIRO_OK;
}

SHIRO_API int shiro_partition(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t* d_row_ptr,
                              const int32_t* d_col, int32_t P, int32_t p, uint32_t flags,
                              shiro_stream_t stream, shiro_plan* out_plan) {
  return partition_impl(n_rows, n_cols, nnz, d_row_ptr, d_col, nullptr, 0, P, p, flags, stream, out_plan);
}

SHIRO_API int shiro_partition_subset(int64_t n_rows, int64_t n_cols, int64_t nnz, const int64_t* d_row_ptr,
                                     const int32_t* d_col, const uint8_t* d_keep, uint8_t keep_value, int32_t P,
                                     int32_t p, uint32_t flags, shiro_stream_t stream, shiro_plan* out_plan) {
  if (!d_keep) return set_error(SHIRO_ERR_INVALID_ARG, "partition_subset: d_keep is NULL");
  return partition_impl(n_rows, n_cols, nnz, d_row_ptr, d_col, d_keep, keep_value, P, p, flags, stream,
                        out_plan);
}

SHIRO_API int shiro_plan_info(shiro_plan plan, shiro_plan_info_t* h_info) {
  if (!plan || !h_info) return set_error(SHIRO_ERR_INVALID_ARG, "plan_info: NULL argument");
  h_info->n_rows = plan->n_rows;
  h_info->n_cols = plan->n_cols;
  h_info->P = plan->P;
  h_info->p = plan->p;
  h_info->M = plan->M;
  h_info->K = plan->K;
  h_info->row_begin = plan->row_begin;
  h_info->rows = plan->rows;
  h_info->nz_begin = plan->nz_begin;
  h_info->nnz = plan->nnz;
  h_info->U = plan->selected ? plan->U : -1;
  return SHIRO_OK;
}

SHIRO_API int shiro_block_nnz(shiro_plan plan, int64_t* d_block_nnz, shiro_stream_t stream) {
  if (!plan || !d_block_nnz) return set_error(SHIRO_ERR_INVALID_ARG, "block_nnz: NULL argument");
  return launch_block_nnz(plan->col, plan->nnz, plan->K, plan->P, d_block_nnz,
                          reinterpret_cast<hipStream_t>(stream));
}

SHIRO_API int shiro_select_rows(shiro_plan plan, shiro_stream_t stream, int64_t* h_U_total,
                                int64_t* h_U_per_block) {
  TraceRange range_("shiro.select_rows");
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "select_rows: plan is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (!plan->selected) {
    if (stream_capturing(s)) return set_error(SHIRO_ERR_CAPTURING, "select_rows: stream is capturing");
    SHIRO_TRY(run_select(plan, s, true));
  }
  if (h_U_total) *h_U_total = plan->U;
  if (h_U_per_block)
    for (int32_t q = 0; q < plan->P; ++q) h_U_per_block[q] = plan->h_block_off[q + 1] - plan->h_block_off[q];
  return SHIRO_OK;
}

SHIRO_API int shiro_refresh_selection(shiro_plan plan, shiro_stream_t stream) {
  TraceRange range_("shiro.select_rows(refresh)");
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "refresh_selection: plan is NULL");
  if (!plan->selected) return set_error(SHIRO_ERR_NOT_READY, "refresh_selection: call shiro_select_rows first");
  return run_select(plan, reinterpret_cast<hipStream_t>(stream), false);
}

SHIRO_API int shiro_plan_selection(shiro_plan plan, const int32_t** d_unique_cols,
                                   const int64_t** d_block_off, const int32_t** d_colmap) {
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "plan_selection: plan is NULL");
  if (!plan->selected) return set_error(SHIRO_ERR_NOT_READY, "plan_selection: call shiro_select_rows first");
  if (d_unique_cols) *d_unique_cols = plan->unique_cols;
  if (d_block_off) *d_block_off = plan->block_off;
  if (d_colmap) *d_colmap = plan->colmap;
  return SHIRO_OK;
}

SHIRO_API int shiro_copy_selection(shiro_plan plan, int32_t* d_unique_cols, int64_t* d_block_off,
                                   int32_t* d_colmap, shiro_stream_t stream) {
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "copy_selection: plan is NULL");
  if (!plan->selected) return set_error(SHIRO_ERR_NOT_READY, "copy_selection: call shiro_select_rows first");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (d_unique_cols && plan->U > 0)
    SHIRO_HIP(hipMemcpyAsync(d_unique_cols, plan->unique_cols, (size_t)plan->U * 4, hipMemcpyDeviceToDevice, s));
  if (d_block_off)
    SHIRO_HIP(hipMemcpyAsync(d_block_off, plan->block_off, (size_t)(plan->P + 1) * 8, hipMemcpyDeviceToDevice, s));
  if (d_colmap && plan->nnz > 0)
    SHIRO_HIP(hipMemcpyAsync(d_colmap, plan->colmap, (size_t)plan->nnz * 4, hipMemcpyDeviceToDevice, s));
  return SHIRO_OK;
}

SHIRO_API int shiro_pack_B(shiro_plan plan, const void* d_B, int64_t ldb, int32_t N, shiro_dtype dt,
                           void* d_Bpacked, int64_t ldp, shiro_stream_t stream) {
  TraceRange range_("shiro.pack_B");
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "pack_B: plan is NULL");
  if (!plan->selected) return set_error(SHIRO_ERR_NOT_READY, "pack_B: call shiro_select_rows first");
  if (!valid_dt(dt)) return set_error(SHIRO_ERR_UNSUPPORTED, "pack_B: unknown dtype");
  if (N < 0 || ldb < N || ldp < N) return set_error(SHIRO_ERR_INVALID_ARG, "pack_B: need N >= 0, ldb >= N, ldp >= N");
  if (N > 0 && plan->U > 0 && (!d_B || !d_Bpacked)) return set_error(SHIRO_ERR_INVALID_ARG, "pack_B: NULL matrix");
  return launch_pack(plan, d_B, ldb, N, dt, d_Bpacked, ldp, reinterpret_cast<hipStream_t>(stream));
}

SHIRO_API int shiro_spmm(shiro_plan plan, const float* d_vals, const void* d_Bpacked, int64_t ldp,
                         int32_t N, shiro_dtype in_dt, void* d_Y, int64_t ldy, shiro_dtype out_dt,
                         uint32_t mode, shiro_stream_t stream) {
  TraceRange range_("shiro.spmm");
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "spmm: plan is NULL");
  if (!plan->selected) return set_error(SHIRO_ERR_NOT_READY, "spmm: call shiro_select_rows first");
  if (!valid_dt(in_dt) || !valid_dt(out_dt)) return set_error(SHIRO_ERR_UNSUPPORTED, "spmm: unknown dtype");
  if (in_dt == SHIRO_F32 && out_dt == SHIRO_BF16)
    return set_error(SHIRO_ERR_UNSUPPORTED, "spmm: F32 input with BF16 output is not supported");
  if (N < 0 || ldp < N || ldy < N) return set_error(SHIRO_ERR_INVALID_ARG, "spmm: need N >= 0, ldp >= N, ldy >= N");
  if (mode != SHIRO_MODE_BATCHED && mode != SHIRO_MODE_PER_BLOCK) return set_error(SHIRO_ERR_INVALID_ARG, "spmm: unknown mode");
  if (N > 0 && plan->rows > 0 && !d_Y) return set_error(SHIRO_ERR_INVALID_ARG, "spmm: d_Y is NULL");
  if (N > 0 && plan->nnz > 0 && (!d_Bpacked || !d_vals)) return set_error(SHIRO_ERR_INVALID_ARG, "spmm: NULL input");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (mode == SHIRO_MODE_PER_BLOCK)
    return launch_spmm_per_block(plan, d_vals, d_Bpacked, ldp, N, in_dt, d_Y, ldy, out_dt, s);
  return launch_spmm(plan, tuning_for(plan, SHIRO_KERNEL_SPMM, N, in_dt), d_vals, d_Bpacked, ldp, N,
                     in_dt, d_Y, ldy, out_dt, s);
}

SHIRO_API int shiro_spmm_backward(shiro_plan plan, const float* d_vals, const void* d_dY, int64_t lddy,
                                  const void* d_Bpacked, int64_t ldp, int32_t N, shiro_dtype dt,
                                  void* d_dBpacked, int64_t lddbp, void* d_dB, int64_t lddb,
                                  float* d_dvals, uint32_t flags, shiro_stream_t stream) {
  TraceRange range_("shiro.spmm_backward");
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "spmm_backward: plan is NULL");
  if (flags & ~SHIRO_DB_OVERWRITE) return set_error(SHIRO_ERR_INVALID_ARG, "spmm_backward: unknown flags");
  if (!plan->selected) return set_error(SHIRO_ERR_NOT_READY, "spmm_backward: call shiro_select_rows first");
  if (!valid_dt(dt)) return set_error(SHIRO_ERR_UNSUPPORTED, "spmm_backward: unknown dtype");
  if (N < 0 || lddy < N) return set_error(SHIRO_ERR_INVALID_ARG, "spmm_backward: need N >= 0 and lddy >= N");
  if (d_dBpacked && lddbp < N) return set_error(SHIRO_ERR_INVALID_ARG, "spmm_backward: lddbp < N");
  if (d_dB && lddb < N) return set_error(SHIRO_ERR_INVALID_ARG, "spmm_backward: lddb < N");
  if (d_dvals && ldp < N) return set_error(SHIRO_ERR_INVALID_ARG, "spmm_backward: ldp < N");
  if (N > 0 && plan->nnz > 0) {
    if (!d_dY) return set_error(SHIRO_ERR_INVALID_ARG, "spmm_backward: d_dY is NULL");
    if ((d_dBpacked || d_dB) && !d_vals) return set_error(SHIRO_ERR_INVALID_ARG, "spmm_backward: d_vals is NULL");
    if (d_dvals && !d_Bpacked) return set_error(SHIRO_ERR_INVALID_ARG, "spmm_backward: d_Bpacked is NULL");
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  bool dvals_done = false;
  if (d_dBpacked || d_dB)
    SHIRO_TRY(launch_spmm_t(plan, tuning_for(plan, SHIRO_KERNEL_SPMM_T, N, dt), d_vals, d_dY, lddy, N,
                            dt, d_dBpacked, lddbp, d_dB, lddb, (flags & SHIRO_DB_OVERWRITE) != 0, d_Bpacked,
                            ldp, d_dvals, &dvals_done, s));
  if (d_dvals && !dvals_done) {
    if (N == 0) {
      // dvals of an empty product are zero
      return set_error(SHIRO_ERR_INVALID_ARG, "spmm_backward: dvals needs N >= 1");
    }
    SHIRO_TRY(launch_sddmm(plan, tuning_for(plan, SHIRO_KERNEL_SDDMM, N, dt), d_vals, d_dY, lddy,
                           d_Bpacked, ldp, N, dt, d_dvals, s));
  }
  return SHIRO_OK;
}

SHIRO_API int shiro_select_c_rows(shiro_plan plan, shiro_stream_t stream, int64_t* h_R,
                                  int64_t* h_R_per_block) {
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "select_c_rows: plan is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (stream_capturing(s)) return set_error(SHIRO_ERR_CAPTURING, "select_c_rows: stream is capturing");
  SHIRO_TRY(build_rowbased(plan, s));
  if (h_R) *h_R = plan->rb.R;
  if (h_R_per_block)
    for (int32_t q = 0; q < plan->P; ++q) h_R_per_block[q] = plan->seg.h_off[q + 1] - plan->seg.h_off[q];
  return SHIRO_OK;
}

SHIRO_API int shiro_copy_c_row_selection(shiro_plan plan, int32_t* d_rows, int64_t* d_rblock_off,
                                         shiro_stream_t stream) {
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "copy_c_row_selection: plan is NULL");
  if (!plan->rb.built) return set_error(SHIRO_ERR_NOT_READY, "copy_c_row_selection: call shiro_select_c_rows first");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (d_rows && plan->rb.R > 0)
    SHIRO_HIP(hipMemcpyAsync(d_rows, plan->seg.seg_row, (size_t)plan->rb.R * 4, hipMemcpyDeviceToDevice, s));
  if (d_rblock_off)
    SHIRO_HIP(hipMemcpyAsync(d_rblock_off, plan->rb.block_off, (size_t)(plan->P + 1) * 8,
                             hipMemcpyDeviceToDevice, s));
  return SHIRO_OK;
}

static bool valid_pair(shiro_dtype in_dt, shiro_dtype out_dt) {
  return (in_dt == SHIRO_F32 && out_dt == SHIRO_F32) || (in_dt == SHIRO_BF16 && out_dt == SHIRO_F32) ||
         (in_dt == SHIRO_BF16 && out_dt == SHIRO_BF16);
}

SHIRO_API int shiro_partial_c(shiro_plan plan, const float* d_vals, const void* d_B, int64_t ldb, int32_t N,
                              shiro_dtype in_dt, void* d_Cp, int64_t ldc, shiro_dtype out_dt,
                              shiro_stream_t stream) {
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "partial_c: plan is NULL");
  if (!plan->rb.built) return set_error(SHIRO_ERR_NOT_READY, "partial_c: call shiro_select_c_rows first");
  if (!valid_pair(in_dt, out_dt))
    return set_error(SHIRO_ERR_UNSUPPORTED, "partial_c: dtype pair not supported (F32->F32, BF16->F32, BF16->BF16)");
  if (N < 0 || ldb < N || ldc < N) return set_error(SHIRO_ERR_INVALID_ARG, "partial_c: need N >= 0, ldb >= N, ldc >= N");
  if (N > 0 && plan->rb.R > 0 && (!d_vals || !d_B || !d_Cp))
    return set_error(SHIRO_ERR_INVALID_ARG, "partial_c: NULL pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return launch_partial_c(plan, tuning_for(plan, SHIRO_KERNEL_PARTIAL_C, N, in_dt), d_vals, d_B, ldb, N, in_dt,
                          d_Cp, ldc, out_dt, s);
}

SHIRO_API int shiro_aggregate_c(shiro_plan plan, const void* d_Cp, int64_t ldc, int32_t N, shiro_dtype in_dt,
                                void* d_Y, int64_t ldy, shiro_dtype out_dt, uint32_t flags,
                                shiro_stream_t stream) {
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "aggregate_c: plan is NULL");
  if (flags & ~SHIRO_AGG_ACCUMULATE) return set_error(SHIRO_ERR_INVALID_ARG, "aggregate_c: unknown flags");
  if (!plan->rb.built) return set_error(SHIRO_ERR_NOT_READY, "aggregate_c: call shiro_select_c_rows first");
  if (!valid_pair(in_dt, out_dt))
    return set_error(SHIRO_ERR_UNSUPPORTED, "aggregate_c: dtype pair not supported (F32->F32, BF16->F32, BF16->BF16)");
  if (N < 0 || ldc < N || ldy < N) return set_error(SHIRO_ERR_INVALID_ARG, "aggregate_c: need N >= 0, ldc >= N, ldy >= N");
  if (N > 0 && plan->rows > 0 && (!d_Y || (plan->rb.R > 0 && !d_Cp)))
    return set_error(SHIRO_ERR_INVALID_ARG, "aggregate_c: NULL pointer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  return launch_aggregate_c(plan, tuning_for(plan, SHIRO_KERNEL_AGGREGATE_C, N, in_dt), d_Cp, ldc, N, in_dt, d_Y,
                            ldy, out_dt, (flags & SHIRO_AGG_ACCUMULATE) != 0, s);
}

SHIRO_API int shiro_mvc_bipartite(int64_t n_left, int64_t n_right, int64_t n_edges, const int32_t* h_left,
                                  const int32_t* h_right, const int64_t* h_w_left, const int64_t* h_w_right,
                                  uint8_t* h_cover_left, uint8_t* h_cover_right, int64_t* h_weight) {
  if (const char* why = mvc::arg_error(n_left, n_right, n_edges, h_left, h_right, h_w_left, h_w_right,
                                       h_cover_left, h_cover_right, h_weight))
    return set_error(SHIRO_ERR_INVALID_ARG, std::string("mvc_bipartite: ") + why);
  return solve_mvc(n_left, n_right, n_edges, h_left, h_right, h_w_left, h_w_right, h_cover_left,
                   h_cover_right, h_weight);
}

SHIRO_API int shiro_joint_plan(shiro_plan plan, const int64_t* h_w_row, const int64_t* h_w_col, uint8_t* h_assign,
                               int64_t* h_stats, int32_t n_threads, shiro_stream_t stream) {
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "joint_plan: plan is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (stream_capturing(s)) return set_error(SHIRO_ERR_CAPTURING, "joint_plan: stream is capturing");
  for (int64_t i = 0; h_w_row && i < plan->rows; ++i)
    if (h_w_row[i] < 0) return set_error(SHIRO_ERR_INVALID_ARG, "joint_plan: negative row cost");
  for (int64_t j = 0; h_w_col && j < plan->n_cols; ++j)
    if (h_w_col[j] < 0) return set_error(SHIRO_ERR_INVALID_ARG, "joint_plan: negative column cost");
  return joint_plan(plan, h_w_row, h_w_col, h_assign, h_stats, n_threads, s);
}

SHIRO_API int shiro_prepare(shiro_plan plan, int32_t N, shiro_dtype dt, uint32_t ops,
                            shiro_stream_t stream) {
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "prepare: plan is NULL");
  if ((ops & ~SHIRO_OP_ROW_BASED) && !plan->selected)
    return set_error(SHIRO_ERR_NOT_READY, "prepare: call shiro_select_rows first");
  if (!valid_dt(dt) || N < 1) return set_error(SHIRO_ERR_INVALID_ARG, "prepare: bad N or dtype");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (stream_capturing(s)) return set_error(SHIRO_ERR_CAPTURING, "prepare: stream is capturing");
  const WorkList* wl;
  if (ops & SHIRO_OP_SPMM) {
    const shiro_tuning_t t = tuning_for(plan, SHIRO_KERNEL_SPMM, N, dt);
    SHIRO_TRY(ensure_rows_work(plan, t.chunk, true, s, &wl));
    SHIRO_TRY(ensure_carry(plan, (int64_t)wl->W * 2 * N, true));
    SHIRO_TRY(ensure_row_rid(plan, true, s));
    const HotRows* hot;
    if (t.group_rows == 3 && t.lds_rows > 0) SHIRO_TRY(ensure_hot(plan, SHIRO_KERNEL_SPMM, t.lds_rows, true, s, &hot));
  }
  if (ops & SHIRO_OP_BACKWARD) {
    SHIRO_TRY(build_transposed(plan, s));
    SHIRO_TRY(ensure_tvals(plan, true));
    const shiro_tuning_t t = tuning_for(plan, SHIRO_KERNEL_SPMM_T, N, dt);
    SHIRO_TRY(ensure_cols_work(plan, t.chunk, true, s, &wl));
    SHIRO_TRY(ensure_carry(plan, (int64_t)wl->W * 2 * N, true));
    const HotRows* hot;
    if (t.group_rows == 3 && t.lds_rows > 0) SHIRO_TRY(ensure_hot(plan, SHIRO_KERNEL_SPMM_T, t.lds_rows, true, s, &hot));
    const shiro_tuning_t t2 = tuning_for(plan, SHIRO_KERNEL_SDDMM, N, dt);
    SHIRO_TRY(ensure_rows_work(plan, t2.chunk, true, s, &wl));
  }
  if (ops & SHIRO_OP_ROW_BASED) {
    SHIRO_TRY(build_rowbased(plan, s));
    for (int which = 0; which < 2; ++which) {
      const shiro_tuning_t t =
          tuning_for(plan, which == 0 ? SHIRO_KERNEL_PARTIAL_C : SHIRO_KERNEL_AGGREGATE_C, N, dt);
      SHIRO_TRY(ensure_rb_work(plan, which, t.chunk, true, s, &wl));
      SHIRO_TRY(ensure_carry(plan, (int64_t)wl->W * 2 * N, true));
    }
  }
  if (ops & SHIRO_OP_PER_BLOCK) {
    if (plan->vmap) return set_error(SHIRO_ERR_UNSUPPORTED, "prepare: per-block mode is not available on subset plans");
    SHIRO_TRY(build_per_block(plan, s));
    SHIRO_TRY(ensure_carry(plan, (int64_t)plan->pb.max_W * 2 * N, true));
    if (dt == SHIRO_BF16) SHIRO_TRY(ensure_acc32(plan, plan->rows * (int64_t)N, true));
  }
  SHIRO_HIP(hipStreamSynchronize(s));
  return SHIRO_OK;
}

SHIRO_API int shiro_autotune(shiro_plan plan, int32_t N, shiro_dtype dt, uint32_t ops,
                             shiro_stream_t stream) {
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "autotune: plan is NULL");
  if (!plan->selected) return set_error(SHIRO_ERR_NOT_READY, "autotune: call shiro_select_rows first");
  if (!valid_dt(dt) || N < 1) return set_error(SHIRO_ERR_INVALID_ARG, "autotune: bad N or dtype");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (stream_capturing(s)) return set_error(SHIRO_ERR_CAPTURING, "autotune: stream is capturing");
  if (plan->nnz == 0) return SHIRO_OK;
  const int64_t sz = dt_size(dt);
  TuneBuffers b;
  const int64_t U = plan->U, R = plan->rows, nnz = plan->nnz;
  // float-filled buffers are reinterpreted for bf16 only as bit patterns of
  // finite values: fill in float, then the bf16 view reads the high halves.
  SHIRO_TRY(dev_alloc(&b.Bp, U * N * 4));
  SHIRO_TRY(dev_alloc(&b.Y, R * N * 4));
  SHIRO_TRY(dev_alloc(&b.dY, R * N * 4));
  SHIRO_TRY(dev_alloc(&b.dBp, U * N * 4));
  if (ops & (SHIRO_OP_BACKWARD | SHIRO_OP_ROW_BASED)) {
    // scratch of the full B shape: dB of the backward (only the selected rows
    // are touched), B of the row-based partial rows
    SHIRO_TRY(dev_alloc(&b.dB, plan->n_cols * N * sz));
    SHIRO_TRY(launch_fill_random((float*)b.dB, plan->n_cols * N * sz / 4, 4, s));
  }
  if (ops & SHIRO_OP_ROW_BASED) {
    SHIRO_TRY(build_rowbased(plan, s));
    SHIRO_TRY(dev_alloc(&b.Cp, std::max<int64_t>(plan->rb.R, 1) * N * 4));
    SHIRO_TRY(launch_fill_random((float*)b.Cp, std::max<int64_t>(plan->rb.R, 1) * N * sz / 4, 5, s));
  }
  SHIRO_TRY(dev_alloc_n(&b.vals, plan->nz_begin + plan->src_nnz));
  SHIRO_TRY(dev_alloc_n(&b.dvals, plan->nz_begin + plan->src_nnz));
  SHIRO_TRY(launch_fill_random((float*)b.Bp, U * N * sz / 4, 1, s));
  SHIRO_TRY(launch_fill_random((float*)b.dY, R * N * sz / 4, 2, s));
  SHIRO_TRY(launch_fill_random(b.vals, plan->nz_begin + plan->src_nnz, 3, s));
  if (ops & SHIRO_OP_BACKWARD) SHIRO_TRY(build_transposed(plan, s));
  if (ops & SHIRO_OP_SPMM) SHIRO_TRY(tune_one(plan, SHIRO_KERNEL_SPMM, N, dt, b, s));
  if (ops & SHIRO_OP_BACKWARD) {
    SHIRO_TRY(tune_one(plan, SHIRO_KERNEL_SPMM_T, N, dt, b, s));
    SHIRO_TRY(tune_one(plan, SHIRO_KERNEL_SDDMM, N, dt, b, s));
  }
  if (ops & SHIRO_OP_ROW_BASED) {
    SHIRO_TRY(tune_one(plan, SHIRO_KERNEL_PARTIAL_C, N, dt, b, s));
    SHIRO_TRY(tune_one(plan, SHIRO_KERNEL_AGGREGATE_C, N, dt, b, s));
  }
  SHIRO_HIP(hipStreamSynchronize(s));
  return shiro_prepare(plan, N, dt, ops, stream);
}

SHIRO_API int shiro_get_tuning(shiro_plan plan, int32_t kernel, int32_t N, shiro_dtype dt,
                               shiro_tuning_t* h_tuning) {
  if (!plan || !h_tuning) return set_error(SHIRO_ERR_INVALID_ARG, "get_tuning: NULL argument");
  if (kernel < 0 || kernel > SHIRO_KERNEL_AGGREGATE_C)
    return set_error(SHIRO_ERR_INVALID_ARG, "get_tuning: unknown kernel family");
  *h_tuning = tuning_for(plan, kernel, N, dt);
  return SHIRO_OK;
}

SHIRO_API int shiro_set_tuning(shiro_plan plan, int32_t kernel, int32_t N, shiro_dtype dt,
                               const shiro_tuning_t* h_tuning) {
  if (!plan || !h_tuning) return set_error(SHIRO_ERR_INVALID_ARG, "set_tuning: NULL argument");
  SHIRO_TRY(validate_tuning(kernel, N, dt, *h_tuning));
  plan->tuning[TuneKey{kernel, N, (int)dt}] = *h_tuning;
  return SHIRO_OK;
}

SHIRO_API int shiro_graph_begin(shiro_plan plan, shiro_stream_t stream) {
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "graph_begin: plan is NULL");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (!s) return set_error(SHIRO_ERR_INVALID_ARG, "graph_begin: capture needs a non-default stream");
  SHIRO_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  return SHIRO_OK;
}

SHIRO_API int shiro_graph_end(shiro_plan plan, shiro_stream_t stream, int32_t* h_graph_id) {
  if (!plan || !h_graph_id) return set_error(SHIRO_ERR_INVALID_ARG, "graph_end: NULL argument");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipGraph_t g = nullptr;
  SHIRO_HIP(hipStreamEndCapture(s, &g));
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return set_error(SHIRO_ERR_HIP, std::string("graph_end: instantiate failed: ") + hipGetErrorString(e));
  plan->graphs.push_back(ex);
  *h_graph_id = (int32_t)plan->graphs.size() - 1;
  return SHIRO_OK;
}

SHIRO_API int shiro_graph_launch(shiro_plan plan, int32_t graph_id, shiro_stream_t stream) {
  if (!plan) return set_error(SHIRO_ERR_INVALID_ARG, "graph_launch: plan is NULL");
  if (graph_id < 0 || graph_id >= (int32_t)plan->graphs.size() || !plan->graphs[graph_id])
    return set_error(SHIRO_ERR_INVALID_ARG, "graph_launch: unknown graph id");
  SHIRO_HIP(hipGraphLaunch(plan->graphs[graph_id], reinterpret_cast<hipStream_t>(stream)));
  return SHIRO_OK;
}

SHIRO_API int shiro_set_allocator(shiro_alloc_fn alloc, shiro_free_fn free_fn, void* ctx) {
  if ((alloc == nullptr) != (free_fn == nullptr))
    return set_error(SHIRO_ERR_INVALID_ARG, "set_allocator: give both functions or neither");
  return set_allocator(alloc, free_fn, ctx);
}

SHIRO_API int shiro_plan_destroy(shiro_plan plan) {
  plan_free(plan);
  return SHIRO_OK;
}

}  // extern "C"
