// Library-internal plan object and the host launchers each source file
// provides.  Not part of the C ABI.
#pragma once

#include <map>
#include <tuple>
#include <vector>

#include "common.hpp"

namespace shiro {

// Merge-path work decomposition of a CSR-like pattern (ptr[0..R], nnz) into
// W chunks of `chunk` merge items (row ends + nonzeros) each.
struct WorkList {
  int32_t chunk = 0;
  int32_t W = 0;
  int32_t* chunk_row = nullptr;  // W + 1
  int32_t* chunk_nz = nullptr;   // W + 1
  // rows cut by chunk boundaries: (first chunk, last chunk, row) triples;
  // the first nsmall have at most kFixupSmall pieces, the rest more
  int32_t nsplit = 0;
  int32_t nsmall = 0;
  int32_t* split = nullptr;      // 3 * nsplit
};

// Split rows of at most this many pieces are summed by one lane group.
constexpr int32_t kFixupSmall = 8;

// Transposed pattern of the remapped panel: packed column u's nonzeros,
// rows ascending.  Built by a stable radix sort of colmap.
struct Transposed {
  bool built = false;
  int64_t* ptr = nullptr;   // U + 1
  int32_t* row = nullptr;   // nnz: panel row of each entry
  int32_t* perm = nullptr;  // nnz: CSR position of each entry (value index)
  int32_t* rid = nullptr;   // nnz: transposed row (packed column) of each entry
};

// Per-block row segments for the one-launch-per-block mode.
struct BlockSegments {
  bool built = false;
  int64_t nseg = 0;
  int32_t* seg_row = nullptr;    // nseg
  int32_t* seg_begin = nullptr;  // nseg (CSR positions)
  int32_t* seg_end = nullptr;    // nseg
  int32_t* seg_csr = nullptr;    // nseg: index of the segment in CSR (row, block) order
  std::vector<int64_t> h_off;    // P + 1 (host copy: launch sizes)
};

// Row-based scheme (Sec. 3.1): the (row, block) segments in block-major
// order are the entries of Rows(A^(p,q)) for q = 0, 1, ...  The owner's
// partial rows are an SpMM over the segments gathering B rows by global
// column id; the receiver's sum is an SpMM of the panel rows over the
// entries with unit weights, blocks ascending.
struct RowBased {
  bool built = false;
  int64_t R = 0;
  int64_t* ptr = nullptr;       // R + 1: each entry's nonzeros in the block-major copy
  int32_t* col = nullptr;       // nnz: global column id of each nonzero, block-major
  int32_t* perm = nullptr;      // nnz: CSR position of each nonzero, block-major
  int32_t* rid = nullptr;       // nnz: entry of each nonzero, block-major
  int64_t* agg_ptr = nullptr;   // rows + 1: each panel row's entries
  int32_t* agg_rid = nullptr;   // R: panel row of each entry of the sum pattern
  int32_t* agg_idx = nullptr;   // R: entry position of each (row, block) pair, blocks ascending
  float* ones = nullptr;        // R: unit weights of the sum
  int32_t* iota = nullptr;      // rows: identity row map (sum added into Y)
  float* vals = nullptr;        // nnz: values in block-major order (per call)
  int64_t* block_off = nullptr; // P + 1: first entry of each block
};

// One launch per column block (the baseline of the batched form): each
// block's own CSR over its (row, block) entries, in the row-based scheme's
// block-major order, with a work list per block.
struct PerBlock {
  bool built = false;
  int64_t* ptr = nullptr;        // R + P: block q's rebased row pointer at off[q] + q
  int32_t* idx = nullptr;        // nnz: packed row of each block-major nonzero
  int32_t* rid = nullptr;        // nnz: entry of each nonzero, counted from its block's first entry
  std::vector<WorkList> work;    // P
  std::vector<int64_t> nz_off;   // P + 1: first block-major nonzero of each block
  int32_t max_W = 0;
};

// Hot rows of a gathered operand kept in LDS by the windowed walk: the H most
// referenced rows (hot_src, by reference count, ties by index), and the
// walk's index array with every reference to them replaced by -(slot + 1).
struct HotRows {
  int32_t* walk_idx = nullptr;  // nnz
  int32_t* hot_src = nullptr;   // H
  int32_t H = 0;
};

struct TuneKey {
  int kernel, N, dt;
  bool operator<(const TuneKey& o) const {
    return std::tie(kernel, N, dt) < std::tie(o.kernel, o.N, o.dt);
  }
};

}  // namespace shiro

struct shiro_plan_s {
  int device = 0;
  int num_cus = 256;
  int64_t n_rows = 0, n_cols = 0, M = 0, K = 0;
  int32_t P = 1, p = 0;
  int64_t row_begin = 0, rows = 0, nz_begin = 0, nnz = 0;

  // pattern (library-owned copies)
  int64_t* row_ptr = nullptr;  // rows + 1, rebased to 0
  int32_t* col = nullptr;      // nnz
  // subset plans (a chosen part of the panel's nonzeros): the position of
  // each nonzero among the panel's src_nnz nonzeros, by which the caller's
  // values are read; NULL for a whole panel (src_nnz == nnz)
  int32_t* vmap = nullptr;     // nnz
  float* svals = nullptr;      // nnz: values in the subset's order (per call)
  int64_t src_nnz = 0;

  // selection
  bool selected = false;
  int64_t U = -1;
  int64_t n_words = 0;
  uint32_t* bits = nullptr;     // n_words: bit c set if column id c occurs in the panel
                                // (all zero between selections)
  int32_t* bcol = nullptr;      // nnz: the panel's column ids grouped by bins of 2^17 ids
  int32_t* mark_items = nullptr;  // 3 per chunk of bcol: bin, first, end
  int32_t n_mark_items = 0;
  bool bins_built = false;
  uint32_t* wtab = nullptr;     // 2 * n_words: (bits, exclusive prefix of popcounts) per word
  int32_t* unique_cols = nullptr;  // capacity min(nnz, n_cols)
  int64_t* block_off = nullptr;    // P + 1
  int32_t* colmap = nullptr;       // nnz
  int32_t* row_rid = nullptr;      // nnz: row of each nonzero (for the nonzero walk)
  std::vector<int64_t> h_block_off;

  // derived structures
  std::map<int32_t, shiro::WorkList> rows_work;   // keyed by chunk size (row-major pattern)
  std::map<int32_t, shiro::WorkList> cols_work;   // keyed by chunk size (transposed pattern)
  shiro::Transposed tr;
  shiro::BlockSegments seg;
  shiro::RowBased rb;
  shiro::PerBlock pb;
  std::map<int32_t, shiro::WorkList> rb_work;   // keyed by chunk size (partial C rows)
  std::map<int32_t, shiro::WorkList> agg_work;  // keyed by chunk size (sum into the panel)
  // hot-row index arrays keyed by (kernel family, H)
  std::map<std::pair<int32_t, int32_t>, shiro::HotRows> hot;

  // carry slots of split rows: 2 * W * carry_cols floats
  float* carry = nullptr;
  int64_t carry_elems = 0;

  // values and value gradients in transposed order (per backward call)
  float* tvals = nullptr;
  float* tdvals = nullptr;
  int64_t tvals_elems = 0;

  // float32 accumulator of the per-block mode when Y is bfloat16
  float* acc32 = nullptr;
  int64_t acc32_elems = 0;

  // scratch for scans and sorts
  void* scratch = nullptr;
  int64_t scratch_bytes = 0;
  int64_t* h_pinned = nullptr;  // small pinned host buffer (P + 2 int64)

  std::map<shiro::TuneKey, shiro_tuning_t> tuning;
  std::vector<hipGraphExec_t> graphs;
  // buffers replaced by larger ones after a graph was captured: a captured
  // graph may still name them, so they are freed with the plan only
  std::vector<void*> retired;
  hipGraph_t capture_graph = nullptr;
};

namespace shiro {

// ---- memory ---------------------------------------------------------------
int dev_alloc(void** p, int64_t bytes);
void dev_free(void* p);
template <typename T>
int dev_alloc_n(T** p, int64_t n) {
  return dev_alloc(reinterpret_cast<void**>(p), n * (int64_t)sizeof(T));
}
int ensure_scratch(shiro_plan plan, int64_t bytes);
// Give up a plan buffer that is being replaced: freed now, or kept until the
// plan is destroyed when a graph captured earlier may still use it.
void retire_buffer(shiro_plan plan, void* p);
bool stream_capturing(hipStream_t s);

// ---- scan.hip ---------------------------------------------------------------
// Exclusive scan of int32 counts into int64 offsets; total written to
// *d_total (nullable).  Scratch needs scan_scratch_bytes(n).
int64_t scan_scratch_bytes(int64_t n);
int exclusive_scan_i32_to_i64(const int32_t* in, int64_t n, int64_t* out, int64_t* d_total,
                              void* scratch, hipStream_t s);
int exclusive_scan_i64(const int64_t* in, int64_t n, int64_t* out, int64_t* d_total,
                       void* scratch, hipStream_t s);

// ---- select.hip -------------------------------------------------------------
int launch_rebase_row_ptr(const int64_t* src, int64_t rows, int64_t* dst, hipStream_t s);
int launch_check_csr(const int64_t* row_ptr, const int32_t* col, int64_t rows, int64_t nnz,
                     int64_t n_cols, int32_t* d_flag, hipStream_t s);
int launch_block_nnz(const int32_t* col, int64_t nnz, int64_t K, int32_t P, int64_t* out,
                     hipStream_t s);
// Selection kernels; with sync the sizes are read back and the plan marked
// selected, without it only the device arrays are rewritten.
int launch_zero_bytes(uint8_t* p, int64_t n, hipStream_t s);
int run_select(shiro_plan plan, hipStream_t s, bool sync);

// ---- sort.hip ---------------------------------------------------------------
// Stable LSD radix sort of (key, value) uint32 pairs on the low `key_bits`
// bits.  Results end in keys_out/vals_out.  Scratch: sort_scratch_bytes(n).
int64_t sort_scratch_bytes(int64_t n);
int radix_sort_pairs(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out,
                     uint32_t* vals_out, int64_t n, int key_bits, void* scratch, hipStream_t s);

// ---- spmm.hip ---------------------------------------------------------------
int build_worklist(const int64_t* ptr, int64_t R, int64_t nnz, int32_t chunk, WorkList* wl,
                   hipStream_t s);
int build_transposed(shiro_plan plan, hipStream_t s);
int build_segments(shiro_plan plan, hipStream_t s);
int build_rowbased(shiro_plan plan, hipStream_t s);
int build_per_block(shiro_plan plan, hipStream_t s);
// The panel rows' ids per nonzero (plan->row_rid), built once.
int ensure_row_rid(shiro_plan plan, bool allocate, hipStream_t s);
// Joint row-column strategy (host): minimum weighted vertex cover of one
// bipartite graph, and the per-panel plan over its off-diagonal blocks.
int solve_mvc(int64_t n_left, int64_t n_right, int64_t n_edges, const int32_t* left,
              const int32_t* right, const int64_t* w_left, const int64_t* w_right,
              uint8_t* cover_left, uint8_t* cover_right, int64_t* weight);
int joint_plan(shiro_plan plan, const int64_t* w_row, const int64_t* w_col, uint8_t* assign,
               int64_t* stats, int32_t n_threads, hipStream_t s);
// Row-based scheme: the owner's partial C rows over B (global rows), and
// their sum into the panel's rows.
int launch_partial_c(shiro_plan plan, const shiro_tuning_t& t, const float* vals, const void* B,
                     int64_t ldb, int32_t N, shiro_dtype in_dt, void* Cp, int64_t ldc,
                     shiro_dtype out_dt, hipStream_t s);
int launch_aggregate_c(shiro_plan plan, const shiro_tuning_t& t, const void* Cp, int64_t ldc,
                       int32_t N, shiro_dtype in_dt, void* Y, int64_t ldy, shiro_dtype out_dt,
                       bool accumulate, hipStream_t s);
// Subset plans: keep flags -> compacted pattern and value map; composition
// of a permutation with the value map.
int launch_subset(const int64_t* row_ptr_src, int64_t rows, int64_t nz0, int64_t nnz_panel,
                  const int32_t* col_src, const uint8_t* keep, uint8_t keep_val, int64_t* pos,
                  int32_t* col_out, int32_t* vmap, int64_t* row_ptr_out, void* scan_tmp,
                  hipStream_t s);
int launch_compose(int32_t* perm, const int32_t* vmap, int64_t n, hipStream_t s);
// which = 0: the partial rows' work list, 1: the sum's.
int ensure_rb_work(shiro_plan plan, int which, int32_t chunk, bool allocate, hipStream_t s,
                   const WorkList** out);

int launch_pack(shiro_plan plan, const void* B, int64_t ldb, int32_t N, shiro_dtype dt,
                void* Bp, int64_t ldp, hipStream_t s);
int launch_spmm(shiro_plan plan, const shiro_tuning_t& t, const float* vals, const void* X,
                int64_t ldx, int32_t N, shiro_dtype in_dt, void* Y, int64_t ldy,
                shiro_dtype out_dt, hipStream_t s);
// The batched product with its carry slots in a caller-given device area of
// carry_cap floats instead of the plan's buffer; allocates nothing: NOT_READY
// when the plan lacks the tuning's work list or row ids, WORKSPACE when the
// slots do not fit.
int launch_spmm_fixed(shiro_plan plan, const shiro_tuning_t& t, const float* vals, const void* X,
                      int64_t ldx, int32_t N, shiro_dtype in_dt, void* Y, int64_t ldy, shiro_dtype out_dt,
                      float* carry, int64_t carry_cap, hipStream_t s);
int launch_spmm_per_block(shiro_plan plan, const float* vals, const void* X, int64_t ldx,
                          int32_t N, shiro_dtype in_dt, void* Y, int64_t ldy, shiro_dtype out_dt,
                          hipStream_t s);
// A^T dY into dBpacked and/or dB.  When dvals is given and one column tile
// covers N, the value gradients are computed in the same pass (*dvals_done).
int launch_spmm_t(shiro_plan plan, const shiro_tuning_t& t, const float* vals, const void* dY,
                  int64_t lddy, int32_t N, shiro_dtype dt, void* dBp, int64_t lddbp, void* dB,
                  int64_t lddb, bool db_overwrite, const void* Bp, int64_t ldp, float* dvals,
                  bool* dvals_done, hipStream_t s);
int launch_sddmm(shiro_plan plan, const shiro_tuning_t& t, const float* vals_unused,
                 const void* dY, int64_t lddy, const void* Bp, int64_t ldp, int32_t N,
                 shiro_dtype dt, float* dvals, hipStream_t s);
int launch_fill_random(float* p, int64_t n, uint64_t seed, hipStream_t s);

// Work lists / carries needed by a tuning; allocate=false returns NOT_READY
// (or CAPTURING) instead of allocating.
int ensure_rows_work(shiro_plan plan, int32_t chunk, bool allocate, hipStream_t s,
                     const WorkList** out);
int ensure_cols_work(shiro_plan plan, int32_t chunk, bool allocate, hipStream_t s,
                     const WorkList** out);
int ensure_carry(shiro_plan plan, int64_t elems, bool allocate);
int ensure_acc32(shiro_plan plan, int64_t elems, bool allocate);
int ensure_tvals(shiro_plan plan, bool allocate);
// The hot-row arrays of kernel SHIRO_KERNEL_SPMM or _SPMM_T for H slots
// (setup: copies the index array to the host; NOT_READY/CAPTURING when
// allocate is false and they are missing).
int ensure_hot(shiro_plan plan, int kernel, int32_t H, bool allocate, hipStream_t s, const HotRows** out);

shiro_tuning_t default_tuning(int kernel, int32_t N, shiro_dtype dt);
// The tuning a plan uses for one kernel family (its own, else the default).
shiro_tuning_t tuning_for(shiro_plan plan, int kernel, int32_t N, shiro_dtype dt);
int validate_tuning(int kernel, int32_t N, shiro_dtype dt, const shiro_tuning_t& t);

}  // namespace shiro
